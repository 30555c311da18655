"""GPU parity: the HIP path against the oracle on the same seeded inputs.

Bars: sectors and graph/forest lists bit-exact; z and log p to rounding;
per point, the precision form (FP64, and double-double where the running
error bound flags the point) within 1e-10 of the long-double oracle relative
to |f| (to the sum of |forest terms| where f vanishes); plain FP64 within its
own running error bound of the oracle; integrals within the combined Monte
Carlo sigma."""
import math

import numpy as np
import pytest

import paper_1905_08007_amd as P
from oracle import graphs as GR, integrand as IN, mc, pdf as PD
from tests import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_CACHE = {}


def setup(n, cls=None, first=None):
    key = (n, cls, first)
    if key not in _CACHE:
        gs = P.enumerate_graphs(n, *(cls or (-1, -1, -1)))
        if first:
            gs = gs[:first]
        s = P.build_forests(gs)
        p = P.pdf_create(s)
        img = P.upload(s, p)
        og = [GR.enumerate_graphs(n)[i] for i in range(len(gs))] if cls is None else None
        _CACHE[key] = (gs, s, p, img, og)
    return _CACHE[key]


def sync():
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [1, 2, 3])
def test_sample_pdf_matches_oracle(n):
    gs, s, p, img, og = setup(n)
    gi = len(gs) - 1
    seed, tag, first, count = 17, 0, 1000, 200
    z, lp, sec = P.sample_pdf(img, gi, seed, tag, first, count, want_sector=True)
    sync()
    z, lp, sec = z.cpu().numpy(), lp.cpu().numpy(), sec.cpu().numpy()
    D = PD.deg_table(og[gi])
    W = PD.w_table(D, 3 * n)
    ref = PD.sample_stream(og[gi], D, W, seed, tag, gi, first, count)
    for i, (zo, lo, order) in enumerate(ref):
        assert list(sec[:, i]) == order
        assert np.max(np.abs(z[:, i] - zo) / zo) < 1e-12
        assert abs(lp[i] - lo) < 1e-11 * max(1.0, abs(lo))


def _eval_cmp(n, gis, npts, seed, gset=None):
    gs, s, p, img, og = setup(n) if gset is None else gset
    M = 3 * n
    nres = 0
    for gi in gis:
        zs = np.concatenate([inputs.simplex_points(M, npts, seed + gi), inputs.boundary_points(M, npts // 2, seed + 100 + gi)])
        zt = torch.from_numpy(np.ascontiguousarray(zs.T)).cuda()
        f0, _, _ = P.eval_integrand(img, gi, zt, P.QA_FP64)
        fb, eb, flag = P.eval_integrand(img, gi, zt, P.QA_FP64_BOUND)
        fd, ed, _ = P.eval_integrand(img, gi, zt, P.QA_DD)
        sync()
        f0, fb, eb, flag, fd, ed = (t.cpu().numpy() for t in (f0, fb, eb, flag, fd, ed))
        final = np.where(flag.astype(bool), fd, fb)
        fin_err = np.where(flag.astype(bool), ed, eb)
        of = IN.Integrand(og[gi])
        IN.set_precision("mp")      # 60-digit reference: boundary points are ill-conditioned
        try:
            ref = [of(zz, True) for zz in zs]
        finally:
            IN.set_precision("ld")
        for i, zz in enumerate(zs):
            v, terms = ref[i]
            scale = abs(v) if v != 0 else sum(abs(t) for t in terms)
            # the precision form meets 1e-10 unless its own (double-double) bound says the
            # point is beyond double-double (a residual point, counted by the batched form)
            residual = flag[i] and ed[i] > 1e-10 * abs(fd[i])
            assert abs(final[i] - v) <= (fin_err[i] if residual else 1e-10 * scale), (gi, i, final[i], v, flag[i], eb[i], ed[i])
            assert abs(fb[i] - v) <= eb[i] + 1e-12 * abs(v), (gi, i, fb[i], v, eb[i])
            assert abs(f0[i] - fb[i]) <= eb[i] + 1e-13 * abs(v), (gi, i)
            assert abs(fd[i] - v) <= ed[i] + 1e-15 * abs(v), (gi, i, fd[i], v, ed[i])
            if residual:
                assert i >= npts, ("an interior point needed more than double-double", gi, i)
            nres += int(residual)
        # the probabilistic estimate (the batched form's flag) also covers the actual error
        fe, ee, fle = P.eval_integrand(img, gi, zt, P.QA_FP64_EST)
        sync()
        fe, ee, fle = fe.cpu().numpy(), ee.cpu().numpy(), fle.cpu().numpy()
        for i in range(len(zs)):
            v = ref[i][0]
            assert abs(fe[i] - v) <= ee[i] + 1e-12 * abs(v), (gi, i, fe[i], v, ee[i])
            assert bool(fle[i]) == (not ee[i] <= 1e-11 * abs(fe[i]))
    return nres


def test_eval_matches_oracle_1loop():
    assert _eval_cmp(1, [0], 130, 1) == 0


def test_eval_matches_oracle_2loop():
    assert _eval_cmp(2, range(4), 70, 2) == 0


def test_eval_matches_oracle_3loop():
    # residual (beyond double-double) points may appear only among the 1e-6 corner points
    _eval_cmp(3, [0, 4, 8, 14, 19, 27], 24, 3)


def test_eval_matches_oracle_4loop():
    _eval_cmp(4, [0, 100, 268], 4, 4)


@pytest.mark.parametrize("n", [2, 3])
def test_bound_covers_double_double(n):
    gs, s, p, img, og = setup(n)
    M = 3 * n
    for gi in range(min(len(gs), 6)):
        zs = np.concatenate([inputs.simplex_points(M, 64, 50 + gi), inputs.boundary_points(M, 64, 60 + gi, lam=1e-9)])
        zt = torch.from_numpy(np.ascontiguousarray(zs.T)).cuda()
        f0, _, _ = P.eval_integrand(img, gi, zt, P.QA_FP64)
        fb, eb, flag = P.eval_integrand(img, gi, zt, P.QA_FP64_BOUND)
        fd, ed, _ = P.eval_integrand(img, gi, zt, P.QA_DD)
        sync()
        f0, fb, eb, flag = f0.cpu().numpy(), fb.cpu().numpy(), eb.cpu().numpy(), flag.cpu().numpy()
        fd, ed = fd.cpu().numpy(), ed.cpu().numpy()
        assert np.all(np.abs(fb - f0) <= eb)
        assert np.all(np.abs(fb - fd) <= eb + ed)
        assert np.array_equal(flag.astype(bool), ~(eb <= 1e-11 * np.abs(fb)))
        assert np.all(ed <= eb)
        # the probabilistic estimate: covers the actual FP64 error, flags consistently
        fe, ee, fle = P.eval_integrand(img, gi, zt, P.QA_FP64_EST)
        sync()
        fe, ee, fle = fe.cpu().numpy(), ee.cpu().numpy(), fle.cpu().numpy()
        assert np.all(np.abs(fe - fd) <= ee + ed)
        assert np.all(np.abs(fe - fb) <= ee + eb)
        assert np.array_equal(fle.astype(bool), ~(ee <= 1e-11 * np.abs(fe)))


def test_accumulate_compensated():
    rng = np.random.default_rng(3)
    count = 100003
    f = rng.standard_normal(count) * 1e3
    lp = rng.standard_normal(count)
    f[17] = np.nan
    acc = P.new_acc(1)
    P.accumulate(torch.from_numpy(f).cuda(), torch.from_numpy(lp).cuda(), acc)
    sync()
    a = P.read_acc(acc)[0]
    w = f * np.exp(-lp)
    good = np.isfinite(w)
    assert int(a["n"]) == good.sum() and int(a["n_bad"]) == 1
    s1 = math.fsum(w[good])
    s2 = math.fsum(w[good] ** 2)
    assert abs(a["s1_hi"] + a["s1_lo"] - s1) <= 1e-12 * abs(s1) + 1e-9
    assert abs(a["s2_hi"] + a["s2_lo"] - s2) <= 1e-13 * s2


def _plain_integral(n, per_graph, seed, chunk=1 << 20):
    gs, s, p, img, og = setup(n)
    acc = P.new_acc(len(gs))
    for gi in range(len(gs)):
        done = 0
        while done < per_graph:
            c = min(chunk, per_graph - done)
            z, lp, _ = P.sample_pdf(img, gi, seed, 0, done, c)
            f, _, _ = P.eval_integrand(img, gi, z, P.QA_FP64)
            P.accumulate(f, lp, acc, gi)
            done += c
    sync()
    a = P.read_acc(acc)
    est = P.estimates(s, a)
    return a, est


def test_one_loop_integral_is_half():
    a, est = _plain_integral(1, 2_000_000, 1)
    v, e = est[0]
    assert abs(v - 0.5) < 4 * e, (v, e)
    assert e < 0.003


def test_two_loop_sum_matches_closed_form_and_oracle():
    import json
    import os
    a, est = _plain_integral(2, 2_000_000, 2)
    v = sum(x for x, _ in est)
    e = math.sqrt(sum(x * x for _, x in est))
    exact = -0.3441663874
    assert abs(v - exact) < 4 * e, (v, e)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_2loop.json")))
    for (x, ex), gg in zip(est, gold["graphs"]):
        comb = math.sqrt(ex * ex + gg["sigma"] ** 2)
        assert abs(x - gg["value"]) < 4.5 * comb, (x, gg["value"], comb)


def test_batched_matches_plain():
    gs, s, p, img, og = setup(2)
    budgets = [100_003, 64, 70_001, 1]
    acc = P.integrate(s, img, budgets, seed=5, tag=0, tile=512)
    sync()
    a = P.read_acc(acc)
    accp = P.new_acc(len(gs))
    for gi, b in enumerate(budgets):
        z, lp, _ = P.sample_pdf(img, gi, 5, 0, 0, b)
        f, _, _ = P.eval_integrand(img, gi, z, P.QA_FP64)
        P.accumulate(f, lp, accp, gi)
    sync()
    ap = P.read_acc(accp)
    for x, y, b in zip(a, ap, budgets):
        assert int(x["n"]) + int(x["n_bad"]) == b
        assert int(x["n"]) == int(y["n"])
        s1x, s1y = x["s1_hi"] + x["s1_lo"], y["s1_hi"] + y["s1_lo"]
        s2x, s2y = x["s2_hi"] + x["s2_lo"], y["s2_hi"] + y["s2_lo"]
        assert abs(s1x - s1y) <= 1e-9 * math.sqrt(s2y * max(1, int(y["n"]))) + 1e-300
        assert abs(s2x - s2y) <= 1e-9 * s2y + 1e-300
    # deterministic: a second run is bit-identical
    acc2 = P.integrate(s, img, budgets, seed=5, tag=0, tile=512)
    sync()
    assert P.read_acc(acc2).tobytes() == a.tobytes()


def test_variance_grad_matches_oracle():
    gs, s, p, img, og = setup(2)
    gi, seed, tag, count = 1, 4, 1, 512
    m2, g = P.variance_and_grad(s, p, img, gi, seed, tag, 0, count)
    smp = mc.graph_samples(og[gi], gi, seed, 0, count, tag=tag)
    D, _ = p.tables(gi)
    go = mc.variance_grad(smp, D, 6)
    m2o = sum(w * w for *_, w, _o in [(a, b, c, d, e) for a, b, c, d, e in smp]) / count
    assert abs(m2 - m2o) < 1e-9 * m2o
    assert np.allclose(g, go, rtol=1e-8, atol=1e-10 * np.max(np.abs(go)))


def test_variance_grad_4loop_matches_oracle():
    """The pilot's backward kernel at 4 loops (configuration of the 4-loop pilot):
    E[w^2] and its gradient over the graph's Deg table against the oracle on
    the same Philox samples (tag 1 = pilot).  FP64 integrand on the GPU, so the
    tolerance is the FP64 round-off of w^2, not the 2-loop 1e-8."""
    gs, s, p, img, og = setup(4)
    gi, seed, tag, count = 100, 4, 1, 24
    m2, g = P.variance_and_grad(s, p, img, gi, seed, tag, 0, count)
    smp = mc.graph_samples(og[gi], gi, seed, 0, count, tag=tag)
    D, _ = p.tables(gi)
    go = mc.variance_grad(smp, D, 12)
    m2o = sum(x[3] * x[3] for x in smp) / count
    assert abs(m2 - m2o) < 1e-7 * m2o
    assert np.allclose(g, go, rtol=1e-6, atol=1e-9 * np.max(np.abs(go)))


def test_edge_cases():
    gs, s, p, img, og = setup(2)
    z = torch.empty((6, 0), dtype=torch.float64, device="cuda")
    f, _, _ = P.eval_integrand(img, 0, z)
    assert f.numel() == 0
    with pytest.raises(RuntimeError):
        P.sample_pdf(img, 99, 1, 0, 0, 10)
    z1, lp1, _ = P.sample_pdf(img, 3, 8, 0, 12345, 1)
    f1, _, _ = P.eval_integrand(img, 3, z1)
    sync()
    assert np.isfinite(f1.cpu().numpy()).all()


def _golden5():
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_5loop.json")))


_FULL5 = {}


def setup5():
    """The benchmark's set: all 73 graphs of class (5,0,0)."""
    if not _FULL5:
        gs = P.enumerate_graphs(5, 5, 0, 0)
        s = P.build_forests(gs)
        p = P.pdf_create(s)
        _FULL5["v"] = (gs, s, p, P.upload(s, p))
    return _FULL5["v"]


def test_eval_5loop_matches_oracle_golden():
    gold = _golden5()
    gs, s, p, img = setup5()
    for key, gg in gold["graphs"].items():
        gi = int(key)
        zs = np.array([pt["z"] for pt in gg["points"]])
        zt = torch.from_numpy(np.ascontiguousarray(zs.T)).cuda()
        fb, eb, flag = P.eval_integrand(img, gi, zt, P.QA_FP64_BOUND)
        fd, ed, _ = P.eval_integrand(img, gi, zt, P.QA_DD)
        sync()
        fb, eb, flag, fd = (t.cpu().numpy() for t in (fb, eb, flag, fd))
        final = np.where(flag.astype(bool), fd, fb)
        for i, pt in enumerate(gg["points"]):
            v = pt["f"]
            scale = abs(v) if v != 0 else pt["terms_abs"]
            assert abs(final[i] - v) <= 1e-10 * scale, (gi, i, final[i], v, flag[i], eb[i])
            assert abs(fb[i] - v) <= eb[i] + 1e-12 * abs(v), (gi, i, fb[i], v, eb[i])
        fe, ee, _ = P.eval_integrand(img, gi, zt, P.QA_FP64_EST)
        sync()
        fe, ee = fe.cpu().numpy(), ee.cpu().numpy()
        for i, pt in enumerate(gg["points"]):
            v = pt["f"]
            assert abs(fe[i] - v) <= ee[i] + 1e-12 * abs(v), (gi, i, fe[i], v, ee[i])


def test_sample_and_eval_5loop_bench_stream():
    gold = _golden5()
    gs, s, p, img = setup5()
    for key, gg in gold["graphs"].items():
        gi = int(key)
        for pt in gg["philox"]:
            z, lp, sec = P.sample_pdf(img, gi, gold["seed"], gold["tag"], pt["sample"], 1, want_sector=True)
            fb, eb, flag = P.eval_integrand(img, gi, z, P.QA_FP64_BOUND)
            fd, _, _ = P.eval_integrand(img, gi, z, P.QA_DD)
            sync()
            assert list(sec.cpu().numpy()[:, 0]) == pt["order"]
            zz = z.cpu().numpy()[:, 0]
            assert np.max(np.abs(zz - pt["z"]) / np.array(pt["z"])) < 1e-12
            assert abs(lp.item() - pt["logp"]) < 1e-11 * max(1.0, abs(pt["logp"]))
            f = fd.item() if flag.item() else fb.item()
            # the oracle evaluated at its own z (equal to ours within ~1e-15): compare at 1e-9
            assert abs(f - pt["f"]) <= 1e-9 * abs(pt["f"]), (gi, pt["sample"], f, pt["f"])


def _check_batched_graph(img, gi, seed, tag, b, x):
    """Reproduce one graph of a single-round batched run with the plain entry
    points (same Philox points; the estimate flag; the double-double recompute
    selected against max(|w|, rms of the accurate weights)) and compare."""
    z, lp, _ = P.sample_pdf(img, gi, seed, tag, 0, b)
    fe, ee, flag = P.eval_integrand(img, gi, z, P.QA_FP64_EST)
    fd, _, _ = P.eval_integrand(img, gi, z, P.QA_DD)
    sync()
    fe, ee, flag, fd = fe.cpu().numpy(), ee.cpu().numpy(), flag.cpu().numpy().astype(bool), fd.cpu().numpy()
    ip = np.exp(-lp.cpu().numpy())
    w0 = fe * ip
    good = np.isfinite(w0)
    acc_ok = good & ~flag
    scale = math.sqrt(math.fsum(w0[acc_ok] ** 2) / max(1, good.sum()))
    need = flag & good & ~(ee * ip <= 1e-11 * np.maximum(np.abs(w0), scale))
    w = np.where(need, fd, fe) * ip
    assert int(x["n"]) == good.sum() and int(x["n_flagged"]) == int(need.sum())
    s1 = math.fsum(w[good])
    assert abs(x["s1_hi"] + x["s1_lo"] - s1) <= 1e-12 * math.fsum(np.abs(w[good]))
    # every accepted FP64 weight is within 1e-10 of the scale of the double-double one
    wd = fd * ip
    assert np.all(np.abs(w[good] - wd[good]) <= 1e-10 * np.maximum(np.abs(wd[good]), scale))


def test_batched_5loop_matches_plain():
    gs, s, p, img = setup5()
    budgets = np.zeros(len(gs), dtype=np.uint64)
    budgets[[1, 40, 72]] = [300, 128, 257]
    acc = P.integrate(s, img, budgets, seed=5, tag=0, tile=128)
    sync()
    a = P.read_acc(acc)
    for gi in (1, 40, 72):
        _check_batched_graph(img, gi, 5, 0, int(budgets[gi]), a[gi])
    assert all(int(a[g]["n"]) == 0 for g in range(len(gs)) if g not in (1, 40, 72))


def test_three_loop_pilot_budgets_batched():
    """3-loop flow: a pilot run (tag 1), Neyman budgets from its sums, the
    batched production run (tag 0) with those uneven budgets."""
    gs, s, p, img, og = setup(3)
    pilot = P.read_acc(P.integrate(s, img, [2048] * len(gs), seed=3, tag=1))
    sync()
    assert all(int(x["n"]) + int(x["n_bad"]) == 2048 for x in pilot)
    budgets = P.allocate_budgets(s, pilot, 150_000, 512)
    assert int(budgets.sum()) == 150_000 and budgets.min() >= 512 and budgets.max() > 2 * budgets.min()
    a = P.read_acc(P.integrate(s, img, budgets, seed=3, tag=0))
    sync()
    for g in range(len(gs)):
        assert int(a[g]["n"]) + int(a[g]["n_bad"]) == int(budgets[g])
    for gi in (0, 13, 27):
        _check_batched_graph(img, gi, 3, 0, int(budgets[gi]), a[gi])


def test_autotune_picks_a_candidate_and_integrates():
    gs, s, p, img, og = setup(2)
    budgets = [30_000, 20_000, 10_000, 5_000]
    tile, grid, ns = P.autotune(s, img, budgets, seed=5, tag=0, pilot=1 << 15)
    assert tile in (256, 512, 1024) and grid > 0 and grid % 4 == 0 and ns > 0
    a = P.read_acc(P.integrate(s, img, budgets, seed=5, tag=0, tile=tile, grid=grid))
    b = P.read_acc(P.integrate(s, img, budgets, seed=5, tag=0))
    sync()
    for x, y in zip(a, b):
        assert int(x["n"]) == int(y["n"]) and int(x["n_flagged"]) == int(y["n_flagged"])
        s1x, s1y = x["s1_hi"] + x["s1_lo"], y["s1_hi"] + y["s1_lo"]
        assert abs(s1x - s1y) <= 1e-12 * math.sqrt((y["s2_hi"] + y["s2_lo"]) * max(1, int(y["n"])))


def test_variance_fn_backward_matches_reweighted_finite_differences():
    """VarianceFn (torch.autograd.Function over the library's backward kernel):
    deg.grad against central finite differences of the reweighted second
    moment V(theta') = (1/N) sum w_i^2 p_theta(z_i) / p_theta'(z_i) on the same
    Philox samples (its derivative at theta' = theta is the gradient exactly)."""
    gs, s, p, img, og = setup(2)
    gi, seed, tag, count, M = 1, 6, 1, 4096, 6
    D0, W0 = p.tables(gi)
    deg = torch.tensor(D0, dtype=torch.float64, requires_grad=True)
    y = P.VarianceFn.apply(deg, (p, gi, seed, tag, 0, count))
    y.backward()
    g = deg.grad.numpy()
    m2, g2 = P.variance_gradient(p, img, gi, seed, tag, 0, count)
    # the backward kernel scatters with atomics: sums agree to rounding, not bitwise
    assert abs(float(y.detach()) - m2) <= 1e-13 * m2
    assert np.allclose(g, g2, rtol=1e-12, atol=1e-14 * np.abs(g2).max())
    z, lp, sec = P.sample_pdf(img, gi, seed, tag, 0, count, want_sector=True)
    f, _, _ = P.eval_integrand(img, gi, z, P.QA_FP64)
    sync()
    z, lp, sec, f = z.cpu().numpy(), lp.cpu().numpy(), sec.cpu().numpy().astype(np.int64), f.cpu().numpy()
    w2 = (f * np.exp(-lp)) ** 2
    assert abs(w2.mean() - m2) <= 1e-12 * m2
    full = (1 << M) - 1
    # S_l and t_l of every sample from its sector
    S = np.full(count, full)
    sets, ts = [], []
    for l in range(1, M):
        S = S ^ (1 << sec[l - 1])
        sets.append(S.copy())
        ts.append(np.log(z[sec[l - 1], np.arange(count)] / z[sec[l], np.arange(count)]))
    sets, ts = np.array(sets), np.array(ts)
    rng = np.random.default_rng(5)
    u = rng.normal(size=1 << M)
    u[0] = u[full] = 0.0

    def logp(Dt, Wt):
        return -np.log(Wt[full]) - (Dt[sets] * ts).sum(axis=0) - np.log(z).sum(axis=0)

    assert np.allclose(logp(D0, W0), lp, rtol=0, atol=1e-11 * np.abs(lp).max())
    h = 1e-5
    V = []
    for sg in (1, -1):
        Dt = D0 + sg * h * u
        Wt = p.with_graph(gi, Dt).tables(gi)[1]
        V.append(np.mean(w2 * np.exp(lp - logp(Dt, Wt))))
    fd = (V[0] - V[1]) / (2 * h)
    assert abs(fd - g @ u) <= 1e-6 * np.abs(g * u).sum(), (fd, g @ u)


def test_acc_read_and_seed_checks():
    gs, s, p, img, og = setup(2)
    acc = P.integrate(s, img, [5000, 300, 4000, 64], seed=9, tag=0)
    per, tot = P.acc_read(s, acc)
    per2, tot2 = P.results(s, P.read_acc(acc))
    assert per.tobytes() == per2.tobytes() and tot.tobytes() == tot2.tobytes()
    assert [int(r["n"]) for r in per] == [5000, 300, 4000, 64]
    with pytest.raises(RuntimeError):
        P.sample_pdf(img, 0, 1 << 32, 0, 0, 16)
    with pytest.raises(RuntimeError):
        P.integrate(s, img, [64] * 4, seed=1 << 33)
