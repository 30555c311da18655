"""Host-side checks of the C-ABI library (no GPU compute): it loads, exports
every symbol the header declares, and its graph / forest / term lists and
Deg / W tables are bit-identical to the oracle's; its Dirac traces equal the
oracle's (a different algorithm: spinor wiring vs Chisholm identities)."""
import os
import random
import re

import numpy as np
import pytest

import paper_1905_08007_amd as P
from oracle import graphs as GR, integrand as IN, pdf as PD
from oracle.dirac import trace as otrace

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "qedamm.h")).read()
    names = set(re.findall(r"\b(qa_[a-z_0-9]+)\s*\(", hdr))
    assert len(names) >= 18
    L = P.lib()
    for n in sorted(names):
        assert hasattr(L, n), n


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_graph_lists_match_oracle(n):
    mine = [P.graph_dict(g) for g in P.enumerate_graphs(n)]
    theirs = GR.enumerate_graphs(n)
    assert mine == [{k: g[k] for k in ("n", "x", "mate", "mult", "cls")} for g in theirs]


def test_class_filter_5loop():
    gs = P.enumerate_graphs(5, 5, 0, 0)
    assert len(gs) == 73
    assert len(P.enumerate_graphs(5)) == 3213
    # every class filter returns the class's graphs of the full list, in order
    full = [P.graph_dict(g) for g in P.enumerate_graphs(5)]
    for c in {tuple(g["cls"]) for g in full}:
        assert [P.graph_dict(g) for g in P.enumerate_graphs(5, *c)] == [g for g in full if tuple(g["cls"]) == c]


@pytest.mark.parametrize("n,count", [(2, 4), (3, 28), (4, 40)])
def test_forest_lists_match_oracle(n, count):
    gs = P.enumerate_graphs(n)[:count]
    s = P.build_forests(gs)
    v = list(s.serialize())
    pos = 0
    for g in GR.enumerate_graphs(n)[:count]:
        subs = GR.subgraphs(g)
        assert v[pos] == len(subs)
        pos += 1
        for x in subs:
            assert v[pos:pos + 4] == [x["lo"], x["hi"], 0 if x["kind"] == "V" else 1, int(x["has_x"])]
            pos += 4
        fs = GR.forests(g)
        assert v[pos] == len(fs) and v[pos + 1:pos + 1 + len(fs)] == fs
        pos += 1 + len(fs)
        ts = IN.graph_terms(g)
        assert v[pos] == len(ts)
        pos += 1
        for m, a in ts:
            assert v[pos:pos + 2] == [m, a]
            pos += 2
    assert pos == len(v)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_deg_w_tables_bit_exact(n):
    gs = P.enumerate_graphs(n)[:10]
    s = P.build_forests(gs)
    p = P.pdf_create(s)
    for i, g in enumerate(GR.enumerate_graphs(n)[:10]):
        D, W = p.tables(i)
        Do = PD.deg_table(g)
        assert np.array_equal(D, Do)
        assert np.array_equal(W, PD.w_table(Do, 3 * n))


def test_dirac_traces_match_oracle():
    rng = random.Random(9)
    for _ in range(400):
        npairs = rng.randint(0, 7)
        nps = rng.randint(0, 6)
        st = [l for l in range(1, npairs + 1) for _ in (0, 1)] + [0] * nps
        rng.shuffle(st)
        assert P.dirac_trace(st) == otrace(st), st


def test_dlogw_matches_oracle():
    from oracle import mc
    gs = P.enumerate_graphs(2)
    s = P.build_forests(gs)
    p = P.pdf_create(s)
    D, _ = p.tables(1)
    assert np.allclose(p.dlogw(1), mc.dlogW_ddeg(D, 6), rtol=1e-12, atol=1e-15)


def test_errors_are_reported():
    with pytest.raises(RuntimeError):
        P.enumerate_graphs(7)
    s = P.build_forests(P.enumerate_graphs(1))
    with pytest.raises(RuntimeError):
        P.pdf_create(s, deg=[np.zeros(8)])


def test_allocate_budgets_neyman():
    import paper_1905_08007_amd as P
    gs = P.enumerate_graphs(2)
    s = P.build_forests(gs, 2)
    ng = len(gs)
    rec = np.zeros(ng, dtype=P.ACC_DTYPE)
    rng = np.random.default_rng(7)
    sd = np.array([0.5, 2.0, 0.0, 1.0])
    for g in range(ng):
        n = 1000
        rec[g]["n"] = n
        mean = rng.normal()
        rec[g]["s1_hi"] = mean * n
        rec[g]["s2_hi"] = (sd[g] ** 2 + mean ** 2) * n
    total, floor = 100_003, 1000
    out = P.allocate_budgets(s, rec, total, floor)
    assert int(out.sum()) == total and np.all(out >= floor)
    # independent computation of the Neyman shares
    mult = np.array([g.mult for g in gs], dtype=float)
    cost = np.array([sum(s.flops(g)) for g in range(ng)])
    sdh = np.sqrt(np.maximum(0.0, rec["s2_hi"] / 1000 - (rec["s1_hi"] / 1000) ** 2))
    w = mult * sdh / np.sqrt(cost)
    share = (total - floor * ng) * w / w.sum()
    assert np.all(np.abs(out - floor - share) < 1.0 + 1e-9)
    assert out[2] == floor  # zero variance: only the floor
    # all-zero pilot: equal shares
    out0 = P.allocate_budgets(s, np.zeros(ng, dtype=P.ACC_DTYPE), 4003, 0)
    assert int(out0.sum()) == 4003 and out0.max() - out0.min() <= 1
    with pytest.raises(RuntimeError):
        P.allocate_budgets(s, rec, 10, 1000)
