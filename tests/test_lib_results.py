"""Host arithmetic behind the C ABI (no GPU): per-graph results and set
totals from accumulator records (qa_results) against the oracle's estimator,
the statistical combination (qa_combine) against the paper's eq. (2), and the
pdf copies used by the pilot (qa_pdf_with, qa_pdf_tune) against the oracle's
W recursion."""
import math

import numpy as np
import pytest

import paper_1905_08007_amd as P
from oracle import mc, pdf as PD


def _records(gs, rng, bad=None):
    rec = np.zeros(len(gs), dtype=P.ACC_DTYPE)
    samples = []
    for g in range(len(gs)):
        w = rng.standard_t(4, size=int(rng.integers(50, 400))) * rng.uniform(0.1, 5) + rng.normal()
        nb = 0 if bad is None else bad[g]
        N, S1, S2 = mc.sums(list(w))
        rec[g]["n"] = N
        rec[g]["s1_hi"] = S1
        rec[g]["s2_hi"] = S2
        rec[g]["n_bad"] = nb
        rec[g]["n_flagged"] = g
        samples.append(list(w) + [0.0] * nb)   # a bad point is a drawn sample with w = 0
    return rec, samples


def test_results_match_oracle_estimate():
    gs = P.enumerate_graphs(3)
    s = P.build_forests(gs[:6], 2)
    rng = np.random.default_rng(11)
    rec, samples = _records(gs[:6], rng, bad=[0, 3, 0, 1, 0, 0])
    per, tot = P.results(s, rec)
    vs = []
    for g, w in enumerate(samples):
        N, S1, S2 = mc.sums(w)
        v, e = mc.estimate(N, S1, S2, gs[g].mult)
        vs.append((v, e))
        assert abs(per[g]["value"] - v) <= 1e-13 * max(1.0, abs(v))
        assert abs(per[g]["sigma"] - e) <= 1e-12 * e
        assert int(per[g]["n"]) == N and int(per[g]["n_bad"]) == int(rec[g]["n_bad"])
        assert abs(per[g]["sd"] - np.std(w, ddof=1)) <= 1e-12 * per[g]["sd"]
    v, e = mc.set_total(vs)
    assert abs(tot["value"] - v) <= 1e-13 * max(1.0, abs(v)) and abs(tot["sigma"] - e) <= 1e-12 * e
    assert int(tot["n_flagged"]) == sum(range(6))
    rec[2]["n"] = 1
    with pytest.raises(RuntimeError):
        P.results(s, rec)


def test_combine_reproduces_eq2():
    runs = np.zeros(2, dtype=P.RESULT_DTYPE)
    runs["value"] = [6.739, 6.905]
    runs["sigma"] = [0.132, 0.220]
    runs["n"] = [10, 20]
    out = P.combine(runs)
    ov, os_ = mc.combine([(6.739, 0.132), (6.905, 0.220)])
    assert abs(out["value"] - ov) < 1e-14 and abs(out["sigma"] - os_) < 1e-15
    assert abs(out["value"] - 6.782) < 0.0015 and abs(out["sigma"] - 0.113) < 0.0006
    assert int(out["n"]) == 30
    runs["sigma"][1] = 0.0
    with pytest.raises(RuntimeError):
        P.combine(runs)


def test_sum_results_matches_oracle_set_total():
    from test_oracle_mc import TABLE1
    rng = np.random.default_rng(5)
    parts = np.zeros(9, dtype=P.RESULT_DTYPE)
    parts["value"] = rng.normal(size=9) * 3
    parts["sigma"] = rng.uniform(0.01, 0.2, size=9)
    parts["n"] = rng.integers(10, 1000, size=9)
    out = P.sum_results(parts)
    v, e = mc.set_total(list(zip(parts["value"], parts["sigma"])))
    assert abs(out["value"] - v) <= 1e-14 * max(1.0, abs(v)) and abs(out["sigma"] - e) <= 1e-15 * e
    assert int(out["n"]) == int(parts["n"].sum())
    # Table 1: the nine Calc 1 class rows against Calc 1's total 6.739(132)
    rows = np.zeros(9, dtype=P.RESULT_DTYPE)
    rows["value"] = [TABLE1[c][1][0] for c in sorted(TABLE1)]
    rows["sigma"] = [TABLE1[c][1][1] for c in sorted(TABLE1)]
    out = P.sum_results(rows)
    assert abs(out["value"] - 6.739) < 0.005 and abs(out["sigma"] - 0.132) < 0.001
    rows["sigma"][3] = float("nan")
    with pytest.raises(RuntimeError):
        P.sum_results(rows)
    rows["sigma"][3] = -0.1
    with pytest.raises(RuntimeError):
        P.sum_results(rows)


def test_pdf_with_and_tune():
    gs = P.enumerate_graphs(2)
    s = P.build_forests(gs, 2)
    p = P.pdf_create(s)
    D1, W1 = p.tables(1)
    D = D1.copy()
    D[1:-1] += np.linspace(0.1, 0.7, len(D) - 2)
    q = p.with_graph(1, D)
    Dq, Wq = q.tables(1)
    assert np.array_equal(Dq[1:-1], D[1:-1]) and np.array_equal(Wq, PD.w_table(Dq, 6))
    for g in (0, 2, 3):   # the other graphs keep their tables
        assert np.array_equal(q.tables(g)[0], p.tables(g)[0])
    assert np.array_equal(p.tables(1)[0], D1)   # base unchanged
    bad = D.copy()
    bad[5] = -1.0
    with pytest.raises(RuntimeError):
        p.with_graph(1, bad)
    # one tuning step: a shift per set size against the size-summed gradient
    rng = np.random.default_rng(2)
    grad = rng.normal(size=64)
    grad[0] = grad[63] = 0.0
    r, th = p.tune(1, grad, 0.25, floor=0.5)
    size = np.array([bin(S).count("1") for S in range(64)])
    gc = np.array([grad[size == c].sum() for c in range(6)])
    want = np.zeros(6)
    want[1:] = -0.25 * gc[1:] / np.abs(gc[1:]).max()
    assert np.allclose(th, want, rtol=0, atol=1e-15)
    Dr, Wr = r.tables(1)
    assert np.allclose(Dr[1:-1], np.maximum(0.5, D1[1:-1] + want[size[1:-1]]), rtol=0, atol=1e-15)
    assert np.array_equal(Wr, PD.w_table(Dr, 6))
    with pytest.raises(RuntimeError):
        p.tune(1, grad, 0.25, floor=0.0)


def test_acc_merge_and_nonzero_flops():
    gs = P.enumerate_graphs(2)
    s = P.build_forests(gs, 2)
    rng = np.random.default_rng(4)
    a, sa = _records(gs, rng)
    b, sb = _records(gs, rng)
    m = P.acc_merge(a.copy(), b)
    per, _ = P.results(s, m)
    for g in range(len(gs)):
        N, S1, S2 = mc.sums(sa[g] + sb[g])
        assert int(m[g]["n"]) == N
        assert abs(m[g]["s1_hi"] + m[g]["s1_lo"] - S1) <= 1e-15 * sum(abs(x) for x in sa[g] + sb[g])
        assert abs(m[g]["s2_hi"] + m[g]["s2_lo"] - S2) <= 1e-15 * S2
        v, e = mc.estimate(N, S1, S2, gs[g].mult)
        assert abs(per[g]["value"] - v) <= 1e-13 * max(1.0, abs(v))
    with pytest.raises(RuntimeError):
        P.acc_merge(a, b[:2])
    for g in range(len(gs)):
        dense, _ = s.flops(g)
        nz = s.flops_nonzero(g)
        assert 0 < nz <= dense


def test_merged_pdf_tables_match_oracle():
    """The 3n-2-variable form's tables (qa_pdf_create_merged) against the
    oracle's merged Deg (Deg of the expanded set) and its W recursion."""
    from oracle import graphs as GR
    for n in (1, 2, 3):
        gs = P.enumerate_graphs(n)[:6]
        s = P.build_forests(gs, 2)
        p = P.pdf_create(s)
        q = p.merged()
        for i, g in enumerate(GR.enumerate_graphs(n)[:6]):
            assert q.lines(i) == 3 * n - 1 and p.lines(i) == 3 * n
            Dm, Wm = q.tables(i)
            Do = PD.merged_deg_table(g, PD.deg_table(g))
            assert np.array_equal(Dm, Do)
            assert np.array_equal(Wm, PD.w_table(Do, 3 * n - 1))
        with pytest.raises(RuntimeError):
            q.merged()


def test_production_chunks_and_class_parts():
    """Host logic of the production and class flows: the per-call share B keeps
    every call within its sample bound and is the largest such share; the
    class parts cover each class once, in enumeration order."""
    from paper_1905_08007_amd import classes as CL
    from paper_1905_08007_amd.pilot import chunk_size
    rng = np.random.default_rng(4)
    for _ in range(20):
        b = rng.integers(1, 10 ** 9, size=int(rng.integers(1, 300))).astype(np.uint64)
        cap = int(rng.integers(int(b.min()), int(b.sum()) + 1))
        B = chunk_size(b, cap)
        assert int(np.minimum(b, B).sum()) <= cap or B == 1
        if B < int(b.max()):
            assert int(np.minimum(b, B + 1).sum()) > cap
    full = P.enumerate_graphs(5)
    seen = []
    for c in CL.CLASSES:
        parts = CL.class_parts(c, max_graphs=100)
        assert all(0 < len(p) <= 100 for p in parts)
        seen += [P.graph_dict(g) for p in parts for g in p]
    assert sorted(map(str, seen)) == sorted(str(P.graph_dict(g)) for g in full)
    assert len(seen) == 3213
