"""Accumulation of the batched form around a point whose FP64 weight is
garbage: a 4-loop graph with its exponents lowered per set size (the shape a
pilot produces) samples, rarely, points where the FP64 integrand loses all its
digits while 1/p is large, so that the FP64 weight exceeds the true one by many
orders.  The window of samples around such a point is integrated by the
batched form and its sums compared with the double-double weights of the same
points: a recomputed point's FP64 value must leave no trace in the sums (its
square can exceed the window's sum of squares by 10^20 and more, so it cannot
be added and later subtracted in double precision)."""
import math

import numpy as np
import pytest

import paper_1905_08007_amd as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# per set size |S| = 1..11: shift of the 4-loop graph's Deg(S), floored at 1/2
SHIFT = [0.0, -0.070972468, -0.026886368, -0.028261398, -0.034956102, -0.061662932, 0.0, -0.135149405, 0.0,
         -0.012225352, -0.204393742, -0.75]


def test_batched_sums_exact_around_a_garbage_fp64_weight():
    gs = P.enumerate_graphs(4)
    s = P.build_forests(gs)
    p0 = P.pdf_create(s)
    g, seed, tag, M = 207, 4, 0, 12
    D0, _ = p0.tables(g)
    pc = np.array([bin(x).count("1") for x in range(1 << M)])
    inner = (pc > 0) & (pc < M)
    D = D0.copy()
    D[inner] = np.maximum(0.5, D0[inner] + np.array(SHIFT)[pc[inner]])
    img = P.upload(s, p0.with_graph(g, D))
    # scan for the largest FP64 weight that its own error estimate calls unreliable
    best, rms2, nacc = (0.0, -1), 0.0, 0
    for first in range(0, 1 << 27, 1 << 22):
        z, lp, _ = P.sample_pdf(img, g, seed, tag, first, 1 << 22)
        f, e, _ = P.eval_integrand(img, g, z, P.QA_FP64_EST)
        ip = torch.exp(-lp)
        wf, ew = f * ip, e * ip
        ok = torch.isfinite(wf)
        good = ok & (ew < 1e-6 * wf.abs())
        rms2 += torch.sum(torch.where(good, wf * wf, torch.zeros_like(wf))).item()
        nacc += int(good.sum().item())
        score = torch.where(ok & (ew > 0.1 * wf.abs()), wf.abs(), torch.zeros_like(wf))
        i = int(torch.argmax(score).item())
        if score[i].item() > best[0]:
            best = (score[i].item(), first + i)
    rms = math.sqrt(rms2 / nacc)
    i = best[1]
    lo = max(0, i - 32)
    cnt = 64
    z, lp, _ = P.sample_pdf(img, g, seed, tag, lo, cnt)
    fd, ed, _ = P.eval_integrand(img, g, z, P.QA_DD)
    f64, _, _ = P.eval_integrand(img, g, z, P.QA_FP64)
    ip = torch.exp(-lp)
    wd, edw, wf = ((fd * ip).cpu().numpy(), (ed * ip).cpu().numpy(), (f64 * ip).cpu().numpy())
    s1d, s2d = math.fsum(wd), math.fsum(x * x for x in wd)
    # the window holds a point whose FP64 weight is garbage far beyond the weight scale
    j = i - lo
    assert abs(wf[j] - wd[j]) > 1e4 * rms and wf[j] ** 2 > 1e12 * s2d, (i, wf[j], wd[j], rms, s2d)
    budgets = np.zeros(len(gs), dtype=np.uint64)
    budgets[g] = cnt
    a = P.read_acc(P.integrate(s, img, budgets, seed, tag, first=lo, tile=64))
    torch.cuda.synchronize()
    x = a[g]
    assert int(x["n"]) == cnt and int(x["n_bad"]) == 0 and int(x["n_flagged"]) >= 1
    s1 = x["s1_hi"] + x["s1_lo"]
    s2 = x["s2_hi"] + x["s2_lo"]
    slack1 = math.fsum(edw)
    slack2 = 2.0 * math.fsum(abs(u) * v for u, v in zip(wd, edw))
    assert s2 > 0
    assert abs(s1 - s1d) <= 1e-10 * math.fsum(abs(v) for v in wd) + slack1, (s1, s1d, slack1)
    assert abs(s2 - s2d) <= 1e-9 * s2d + slack2, (s2, s2d, slack2)


def test_pilot_tune_steps_and_guard():
    """The pilot flow's sequencing on the 2-loop set: one tuned step shifts the
    exponents by one amount per set size (floored at 1/2); two steps with and
    without the guard (a move kept only where paired fresh samples confirm it)
    give finite second moments and PDFs that integrate."""
    from paper_1905_08007_amd import pilot as PL
    gs = P.enumerate_graphs(2)
    s = P.build_forests(gs)
    p0 = P.pdf_create(s)
    img0 = P.upload(s, p0)
    M = 6
    pc = np.array([bin(x).count("1") for x in range(1 << M)])
    inner = (pc > 0) & (pc < M)
    p1, _, _ = PL.tune(s, p0, img0, 2, 1 << 14, 1, 0.25)
    for g in range(len(gs)):
        D0, _ = p0.tables(g)
        D1, _ = p1.tables(g)
        assert np.all(D1[inner] >= 0.5)
        for c in range(1, M):
            sel = inner & (pc == c) & (D1 > 0.5)
            if sel.sum() > 1:
                d = D1[sel] - D0[sel]
                assert np.ptp(d) < 1e-12 and abs(d[0]) <= 0.25 + 1e-12
    for guard in (False, True):
        p2, img2, hist = PL.tune(s, p0, img0, 2, 1 << 14, 2, 0.25, guard=guard)
        assert len(hist) == 2 and all(np.all(np.isfinite(h)) and np.all(h > 0) for h in hist)
        for g in range(len(gs)):
            assert np.all(p2.tables(g)[0][inner] >= 0.5)
        per, tot, budgets = PL.production(s, img2, 2, 4e5, 1 << 12, chunks=2)
        torch.cuda.synchronize()
        assert int(tot["n"]) == 400000 and np.isfinite(tot["value"]) and tot["sigma"] > 0
