"""Oracle pins for the sector PDF of eq. (1): the W recursion against brute
force over all M! sectors, the density formula re-evaluated from eq. (1),
and closed-form moments (the simplex volume and Dirichlet integrals)."""
import itertools
import math

import numpy as np

from oracle import graphs as GR, pdf as PD


def _rand_deg(M, seed):
    rng = np.random.default_rng(seed)
    D = rng.uniform(0.4, 3.0, 1 << M)
    D[0] = 0
    D[-1] = 0
    return D


def test_w_recursion_vs_all_sectors():
    M = 6
    D = _rand_deg(M, 1)
    W = PD.w_table(D, M)
    full = (1 << M) - 1
    tot = 0.0
    for perm in itertools.permutations(range(M)):
        S = full
        w = 1.0
        for l in range(1, M):
            S ^= 1 << perm[l - 1]
            w /= D[S]
        tot += w
    assert abs(W[full] - tot) <= 1e-12 * tot


def test_logp_equals_eq1():
    g = GR.enumerate_graphs(2)[3]
    M = 6
    D = PD.deg_table(g)
    W = PD.w_table(D, M)
    full = (1 << M) - 1
    for z, lp, order in PD.sample_stream(g, D, W, 11, 0, 3, 0, 50):
        # eq. (1) evaluated directly, with the sector read off by sorting z
        j = list(np.argsort(-z, kind="stable"))
        assert j == order
        S = full
        val = -math.log(W[full])
        for l in range(1, M):
            S ^= 1 << j[l - 1]
            val += D[S] * math.log(z[j[l]] / z[j[l - 1]])
        val -= sum(math.log(v) for v in z)
        assert abs(val - lp) < 1e-9 * max(1.0, abs(lp))
        assert abs(z.sum() - 1.0) < 1e-14


def test_moments_closed_form():
    g = GR.enumerate_graphs(2)[0]
    M = 6
    D = PD.deg_table(g)
    W = PD.w_table(D, M)
    a = np.array([1.0, 0.0, 2.0, 0.0, 1.0, 0.0])
    pts = PD.sample_stream(g, D, W, 5, 2, 0, 0, 20000)
    inv = np.array([math.exp(-lp) for _, lp, _ in pts])
    mom = np.array([math.prod(z ** a) * math.exp(-lp) for z, lp, _ in pts])
    vol = 1.0 / math.factorial(M - 1)
    dir_ = math.prod(math.gamma(x + 1) for x in a) / math.gamma(a.sum() + M)
    for est, exact in ((inv, vol), (mom, dir_)):
        m = est.mean()
        e = est.std() / math.sqrt(len(est))
        assert abs(m - exact) < 4.5 * e, (m, exact, e)


def test_deg_positive_and_fractional():
    g = GR.enumerate_graphs(3)[0]
    D = PD.deg_table(g)
    full = (1 << 9) - 1
    assert all(D[s] >= 0.5 for s in range(1, full))
    # single electron line: 1/2; single photon line: 1
    assert D[1] == 0.5 and D[1 << 6] == 1.0
