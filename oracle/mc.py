"""Monte Carlo estimator: w = f/p per sample, per-graph sums, set totals.

Oracle code (test infrastructure only).

Paper: nonadaptive Monte Carlo with the per-graph PDF of eq. (1); results are
quoted with 1-sigma errors and two independent runs are combined (section
"Preliminary numerical results").  Estimator: a_G = mult_G * mean(w),
sigma_G^2 = mult_G^2 * (mean(w^2) - mean(w)^2) / (N - 1); set value = sum of
a_G with sigma = sqrt(sum sigma_G^2); independent runs combine by inverse
variance weights.
"""
import math
import numpy as np

from . import pdf as PD
from .integrand import Integrand


def graph_samples(g, gid, seed, first, count, tag=0, deg=None):
    """Per-sample (z, log p, f, w) for graph index ``gid`` of its set."""
    M = 3 * g["n"]
    D = PD.deg_table(g) if deg is None else deg
    W = PD.w_table(D, M)
    f = Integrand(g)
    out = []
    for z, lp, order in PD.sample_stream(g, D, W, seed, tag, gid, first, count):
        fv = f(z)
        out.append((z, lp, fv, fv * math.exp(-lp), order))
    return out


def sums(ws):
    """(N, sum w, sum w^2) with exactly rounded sums."""
    return len(ws), math.fsum(ws), math.fsum(w * w for w in ws)


def estimate(N, S1, S2, mult):
    mean = S1 / N
    var = (S2 / N - mean * mean) / (N - 1) if N > 1 else float("inf")
    return mult * mean, mult * math.sqrt(max(var, 0.0))


def set_total(vals_sigmas):
    v = sum(a for a, _ in vals_sigmas)
    s = math.sqrt(sum(e * e for _, e in vals_sigmas))
    return v, s


def combine(runs):
    """Inverse-variance combination of independent (value, sigma) results."""
    wsum = sum(1.0 / (s * s) for _, s in runs)
    v = sum(a / (s * s) for a, s in runs) / wsum
    return v, 1.0 / math.sqrt(wsum)


def dlogW_ddeg(deg, M):
    """Gradient of ln W(full) with respect to every Deg(S) (reverse pass of
    the W recursion)."""
    W = PD.w_table(deg, M)
    full = (1 << M) - 1
    Wb = np.zeros(1 << M)
    Db = np.zeros(1 << M)
    Wb[full] = 1.0 / W[full]
    for s in sorted(range(1, full + 1), key=lambda t: -bin(t).count("1")):
        if Wb[s] == 0.0:
            continue
        if s != full:
            Db[s] += Wb[s] * (-W[s] / deg[s])
        if bin(s).count("1") == 1:
            continue
        scale = Wb[s] if s == full else Wb[s] / deg[s]
        t = s
        while t:
            j = t & -t
            Wb[s ^ j] += scale
            t ^= j
    return Db


def sample_tails(order, z):
    """(S_l, t_l) for l = 2..M of a sampled point."""
    M = len(order)
    S = (1 << M) - 1
    out = []
    for l in range(1, M):
        S ^= 1 << order[l - 1]
        out.append((S, math.log(z[order[l - 1]] / z[order[l]])))
    return out


def variance_grad(samples, deg, M):
    """d/dDeg(S) of E_p[w^2] = E[w^2 sum_l t_l 1{S_l = S}] + E[w^2] dlnW/dDeg(S)."""
    g = np.zeros(1 << M)
    w2 = 0.0
    for z, lp, f, w, order in samples:
        ww = w * w
        w2 += ww
        for S, t in sample_tails(order, z):
            g[S] += ww * t
    N = len(samples)
    return g / N + (w2 / N) * dlogW_ddeg(deg, M)
