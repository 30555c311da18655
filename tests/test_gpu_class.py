"""GPU parity at the benchmark's scale: every graph of the 5-loop class
(5,0,0), four graphs of each other 5-loop class, every graph at 1..4 loops
for the sampler, the batched form's sums
against the oracle's on the same Philox points, and the configurations'
integrals (1 and 2 loops at their full sample counts)."""
import json
import math
import os

import numpy as np
import pytest

import paper_1905_08007_amd as P
from oracle import graphs as GR, integrand as IN, pdf as PD
from oracle.philox import uniforms

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
_SETS = {}


def _set(loops, cls=(-1, -1, -1)):
    key = (loops, cls)
    if key not in _SETS:
        gs = P.enumerate_graphs(loops, *cls)
        s = P.build_forests(gs)
        p = P.pdf_create(s)
        _SETS[key] = (gs, s, p, P.upload(s, p))
    return _SETS[key]


def _gold(name):
    return json.load(open(os.path.join(HERE, "golden", name)))


@pytest.mark.parametrize("loops", [1, 2, 3, 4])
def test_sampler_every_graph(loops):
    """Sectors identical, z and log p to rounding, for every graph at n <= 4
    (the Deg / W tables themselves are pinned bit-exactly on the CPU)."""
    gs, s, p, img = _set(loops)
    M = 3 * loops
    seed, tag, first, count = 31, 0, 7, 8
    for gi in range(len(gs)):
        z, lp, sec = P.sample_pdf(img, gi, seed, tag, first, count, want_sector=True)
        torch.cuda.synchronize()
        z, lp, sec = z.cpu().numpy(), lp.cpu().numpy(), sec.cpu().numpy()
        D, W = p.tables(gi)
        for i in range(count):
            zo, lo, order = PD.sample(D, W, M, uniforms(seed, tag, gi, first + i, 2 * (M - 1)))
            assert list(sec[:, i]) == order, (loops, gi, i)
            assert np.max(np.abs(z[:, i] - zo) / zo) < 1e-12, (loops, gi, i)
            assert abs(lp[i] - lo) < 1e-11 * max(1.0, abs(lo)), (loops, gi, i)


def test_class500_every_graph_sample_and_eval():
    """All 73 graphs of class (5,0,0) at the first five points of the benchmark
    stream: sector, z, log p, and f of the precision form within 1e-10 of the
    oracle (long double, 60 digits where its terms cancel by more than 10^6);
    the probabilistic estimate covers the FP64 error."""
    gold = _gold("oracle_5loop_class.json")
    gs, s, p, img = _set(5, (5, 0, 0))
    assert len(gold["graphs"]) == len(gs) == 73
    for key, gg in gold["graphs"].items():
        gi = int(key)
        pts = gg["philox"]
        z, lp, sec = P.sample_pdf(img, gi, gold["seed"], gold["tag"], 0, len(pts), want_sector=True)
        fb, eb, flag = P.eval_integrand(img, gi, z, P.QA_FP64_BOUND)
        fd, ed, _ = P.eval_integrand(img, gi, z, P.QA_DD)
        fe, ee, _ = P.eval_integrand(img, gi, z, P.QA_FP64_EST)
        torch.cuda.synchronize()
        zc, lpc, secc = z.cpu().numpy(), lp.cpu().numpy(), sec.cpu().numpy()
        fb, eb, flag, fd, ed, fe, ee = (t.cpu().numpy() for t in (fb, eb, flag, fd, ed, fe, ee))
        for i, pt in enumerate(pts):
            assert pt["sample"] == i
            assert list(secc[:, i]) == pt["order"], (gi, i)
            assert np.max(np.abs(zc[:, i] - pt["z"]) / np.array(pt["z"])) < 1e-12, (gi, i)
            assert abs(lpc[i] - pt["logp"]) < 1e-11 * max(1.0, abs(pt["logp"])), (gi, i)
            v = pt["f"]
            scale = abs(v) if v != 0 else pt["terms_abs"]
            final = fd[i] if flag[i] else fb[i]
            # the oracle evaluated at its own z (equal to ours to ~1e-15 relative)
            assert abs(final - v) <= 1e-10 * scale + 1e-13 * pt["terms_abs"], (gi, i, final, v, flag[i])
            assert abs(fe[i] - v) <= ee[i] + 1e-10 * scale, (gi, i, fe[i], v, ee[i])


def test_class500_batched_sums_match_oracle():
    """The batched form's per-graph sums over samples 0..4 of every class
    (5,0,0) graph against the oracle's exactly rounded sums of the same
    weights: within 1e-10 of the sum of |w| (the accepted FP64 weights carry
    at most 1e-11 of the weight scale)."""
    gold = _gold("oracle_5loop_class.json")
    gs, s, p, img = _set(5, (5, 0, 0))
    budgets = np.full(len(gs), 5, dtype=np.uint64)
    a = P.read_acc(P.integrate(s, img, budgets, seed=gold["seed"], tag=gold["tag"], tile=64))
    torch.cuda.synchronize()
    for key, gg in gold["graphs"].items():
        gi = int(key)
        ws = [pt["w"] for pt in gg["philox"]]
        x = a[gi]
        assert int(x["n"]) == 5 and int(x["n_bad"]) == 0
        s1 = x["s1_hi"] + x["s1_lo"]
        s2 = x["s2_hi"] + x["s2_lo"]
        tol = 1e-10 * math.fsum(abs(w) for w in ws)
        assert abs(s1 - math.fsum(ws)) <= tol, (gi, s1, math.fsum(ws))
        assert abs(s2 - math.fsum(w * w for w in ws)) <= 2e-10 * math.fsum(w * w for w in ws), gi


def test_other_classes_sample_eval_and_sums():
    """Four graphs of each of the other eight 5-loop classes (Table 1), taken
    together as one set: the library's enumeration gives the oracle's graphs
    at the same class indices; sector, z, log p and f of the precision form
    within 1e-10 of the oracle at the first three points of the set's stream;
    the estimate covers the FP64 error; the batched sums match the oracle's."""
    gold = _gold("oracle_5loop_classes.json")
    picks = []
    by_cls = {}
    for gg in gold["graphs"]:
        c = tuple(gg["class"])
        if c not in by_cls:
            by_cls[c] = P.enumerate_graphs(5, *c)
        g = by_cls[c][gg["index"]]
        assert g.x == gg["x"] and list(g.mate)[:11] == gg["mate"] and g.mult == gg["mult"], (c, gg["index"])
        picks.append(g)
    s = P.build_forests(picks)
    img = P.upload(s, P.pdf_create(s))
    for gi, gg in enumerate(gold["graphs"]):
        pts = gg["philox"]
        z, lp, sec = P.sample_pdf(img, gi, gold["seed"], gold["tag"], 0, len(pts), want_sector=True)
        fb, eb, flag = P.eval_integrand(img, gi, z, P.QA_FP64_BOUND)
        fd, ed, _ = P.eval_integrand(img, gi, z, P.QA_DD)
        fe, ee, _ = P.eval_integrand(img, gi, z, P.QA_FP64_EST)
        torch.cuda.synchronize()
        zc, lpc, secc = z.cpu().numpy(), lp.cpu().numpy(), sec.cpu().numpy()
        fb, eb, flag, fd, ed, fe, ee = (t.cpu().numpy() for t in (fb, eb, flag, fd, ed, fe, ee))
        for i, pt in enumerate(pts):
            assert list(secc[:, i]) == pt["order"], (gi, i)
            assert np.max(np.abs(zc[:, i] - pt["z"]) / np.array(pt["z"])) < 1e-12, (gi, i)
            assert abs(lpc[i] - pt["logp"]) < 1e-11 * max(1.0, abs(pt["logp"])), (gi, i)
            v = pt["f"]
            scale = abs(v) if v != 0 else pt["terms_abs"]
            final = fd[i] if flag[i] else fb[i]
            assert abs(final - v) <= 1e-10 * scale + 1e-13 * pt["terms_abs"], (gi, i, final, v, flag[i])
            assert abs(fe[i] - v) <= ee[i] + 1e-10 * scale, (gi, i, fe[i], v, ee[i])
    n = len(gold["graphs"][0]["philox"])
    a = P.read_acc(P.integrate(s, img, np.full(len(picks), n, dtype=np.uint64), seed=gold["seed"], tag=gold["tag"],
                               tile=64))
    torch.cuda.synchronize()
    for gi, gg in enumerate(gold["graphs"]):
        ws = [pt["w"] for pt in gg["philox"]]
        x = a[gi]
        assert int(x["n"]) == n and int(x["n_bad"]) == 0
        s1 = x["s1_hi"] + x["s1_lo"]
        assert abs(s1 - math.fsum(ws)) <= 1e-10 * math.fsum(abs(w) for w in ws), (gi, s1, math.fsum(ws))


def test_class_flow_in_parts_sums_to_the_class():
    """The class-by-class flow on class (5,0,0) split into parts of at most 32
    graphs (three graph sets with their own Philox keys): the Neyman budgets
    of the parts add up to the class's samples, the class record is the sum
    of the per-graph records (value, and sigma in quadrature), and the set
    total over the classes run is that record."""
    from paper_1905_08007_amd import classes as CL
    res, total = CL.integrate_all(3, 4000, classes=[(5, 0, 0)], pilot_per_graph=1024, chunks=2, max_graphs=32)
    per, tot, sec = res[(5, 0, 0)]
    assert len(per) == 73 and sec > 0
    assert int(tot["n"]) == 73 * 4000 and int(tot["n_bad"]) == 0
    assert np.all(np.isfinite(per["value"])) and np.all(per["sigma"] > 0)
    assert abs(tot["value"] - math.fsum(per["value"])) <= 1e-12 * math.fsum(abs(per["value"]))
    assert abs(tot["sigma"] - math.sqrt(math.fsum(per["sigma"] ** 2))) <= 1e-12 * tot["sigma"]
    assert total["value"] == tot["value"] and total["sigma"] == tot["sigma"]


def test_eval_4loop_interior_many_graphs():
    """4 loops: 24 graphs spread over the set, interior points, the precision
    form within 1e-10 of the long-double oracle (whose own error there is
    below 1e-13: points whose terms cancel by more than 10^5 are skipped)."""
    from tests import inputs
    gs, s, p, img = _set(4)
    og = GR.enumerate_graphs(4)
    checked = 0
    for gi in range(0, 269, 11):
        zs = inputs.simplex_points(12, 3, 900 + gi)
        zt = torch.from_numpy(np.ascontiguousarray(zs.T)).cuda()
        fb, eb, flag = P.eval_integrand(img, gi, zt, P.QA_FP64_BOUND)
        fd, _, _ = P.eval_integrand(img, gi, zt, P.QA_DD)
        torch.cuda.synchronize()
        fb, flag, fd = fb.cpu().numpy(), flag.cpu().numpy(), fd.cpu().numpy()
        f = IN.Integrand(og[gi])
        for i, zz in enumerate(zs):
            v, terms = f(zz, True)
            tabs = sum(abs(t) for t in terms)
            if tabs > 1e5 * abs(v):
                continue
            final = fd[i] if flag[i] else fb[i]
            assert abs(final - v) <= 1e-10 * abs(v), (gi, i, final, v)
            checked += 1
    assert checked >= 48


def test_config3_batched_prefix_sums_match_oracle():
    """3-loop configuration's stream (seed 3): the batched form's per-graph sums
    over the first 256 points against the oracle's exactly rounded sums of the
    same weights, every graph."""
    gold = _gold("oracle_3loop_prefix.json")
    gs, s, p, img = _set(3)
    K = gold["samples"]
    a = P.read_acc(P.integrate(s, img, np.full(len(gs), K, dtype=np.uint64), seed=gold["seed"], tag=gold["tag"]))
    torch.cuda.synchronize()
    for gi, gg in enumerate(gold["graphs"]):
        x = a[gi]
        assert int(x["n"]) == K
        s1 = x["s1_hi"] + x["s1_lo"]
        assert abs(s1 - gg["S1"]) <= 1e-10 * gg["S1abs"], (gi, s1, gg["S1"])


def test_config1_integral_full_count():
    """Configuration 1: 10^7 Philox samples (seed 1) of the 1-loop graph; the
    paper's A_1^(2) = 0.5 within 3 sigma."""
    gs, s, p, img = _set(1)
    per, tot = P.acc_read(s, P.integrate(s, img, [10_000_000], seed=1, tag=0))
    assert int(tot["n"]) == 10_000_000
    assert abs(tot["value"] - 0.5) < 3 * tot["sigma"], (tot["value"], tot["sigma"])
    assert tot["sigma"] < 1e-3


def test_config2_integral_full_count():
    """Configuration 2: 10^8 samples (seed 2), 2.5e7 per 2-loop graph; the sum
    against the closed form (the paper's A_1^(4) without the vacuum-polarization
    graph) within 3 sigma."""
    gs, s, p, img = _set(2)
    per, tot = P.acc_read(s, P.integrate(s, img, [25_000_000] * 4, seed=2, tag=0))
    exact = 197 / 144 + math.pi ** 2 / 12 - math.pi ** 2 / 2 * math.log(2) + 0.75 * 1.2020569031595942 \
        - (119 / 36 - math.pi ** 2 / 3)
    assert abs(exact - (-0.3441663874)) < 1e-9
    assert int(tot["n"]) == 100_000_000
    assert abs(tot["value"] - exact) < 3 * tot["sigma"], (tot["value"], tot["sigma"])
