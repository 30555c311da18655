"""Oracle pins of the 3n-2-variable form (paper, section "The method",
footnote on reducing the variables from 3n-1 to 3n-2): the merged integrand
integrates the split of the two electron lines next to the external vertex.

- the split integral: three-point Gauss-Legendre against adaptive quadrature
  of the 3n-line integrand, and the split dependence is linear (so the
  midpoint value times s is exact), at 1-3 loops;
- 1 loop: the merged integrand is the photon's parameter (textbook form
  z/(x+y) on the 2-simplex becomes z on the 1-simplex), integral 1/2;
- the merged Deg / W tables: the W recursion against brute force over the
  sectors of the merged lines, and the expansion of line sets."""
import itertools
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import graphs as GR, integrand as IN, pdf as PD
from oracle.philox import uniforms


@pytest.mark.parametrize("n,gis", [(1, [0]), (2, [0, 1, 2, 3]), (3, [0, 7, 13, 19, 25, 27])])
def test_split_integral(n, gis):
    rng = np.random.default_rng(40 + n)
    for gi in gis:
        g = GR.enumerate_graphs(n)[gi]
        fm = IN.MergedIntegrand(g)
        f = IN.Integrand(g)
        a, b = PD.merged_lines(g)
        zm = rng.dirichlet(np.ones(3 * n - 1))
        v = fm(zm)
        ref, _ = integrate.quad(lambda t: f(PD.expand_point(g, zm, t)), 0.0, 1.0, epsabs=0, epsrel=1e-13)
        assert abs(v - zm[a] * ref) <= 1e-11 * abs(zm[a] * ref), (n, gi)
        mid = zm[a] * f(PD.expand_point(g, zm, 0.5))
        assert abs(v - mid) <= 1e-12 * max(abs(v), 1e-300), (n, gi)


def test_one_loop_merged_closed_form_and_integral():
    g = GR.enumerate_graphs(1)[0]
    fm = IN.MergedIntegrand(g)
    rng = np.random.default_rng(1)
    for _ in range(20):
        zm = rng.dirichlet(np.ones(2))
        # merged lines: 0 = {electron 0, electron 1}, 1 = photon
        assert abs(fm(zm) - zm[1]) < 1e-15
    # integral over the 1-simplex of z_photon = 1/2 (paper: A_1^(2) = 0.5)
    val, _ = integrate.quad(lambda u: fm(np.array([1 - u, u])), 0, 1)
    assert abs(val - 0.5) < 1e-12


def test_merged_tables_and_sets():
    for n in (1, 2, 3):
        for g in GR.enumerate_graphs(n)[:6]:
            a, b = PD.merged_lines(g)
            Mm = 3 * n - 1
            D = PD.deg_table(g)
            Dm = PD.merged_deg_table(g, D)
            for S in range(1, (1 << Mm) - 1):
                E = PD.expand_set(g, S)
                assert bin(E).count("1") == bin(S).count("1") + (S >> a & 1)
                assert Dm[S] == D[E]
            if Mm <= 8:
                Wm = PD.w_table(Dm, Mm)
                full = (1 << Mm) - 1
                brute = 0.0
                for perm in itertools.permutations(range(Mm)):
                    S, w = full, 1.0
                    for l in range(1, Mm):
                        S ^= 1 << perm[l - 1]
                        w /= Dm[S]
                    brute += w
                assert abs(Wm[full] - brute) <= 1e-12 * brute


def test_merged_sampler_density():
    """log p of the merged sampler re-evaluated from eq. (1) at the point."""
    g = GR.enumerate_graphs(2)[1]
    Dm = PD.merged_deg_table(g, PD.deg_table(g))
    Wm = PD.w_table(Dm, 5)
    full = (1 << 5) - 1
    for i in range(50):
        zm, lp, order = PD.sample_merged(g, Dm, Wm, uniforms(3, 0, 1, i, 8))
        S = full ^ (1 << order[0])
        acc = 0.0
        for l in range(1, 5):
            acc += Dm[S] * math.log(zm[order[l - 1]] / zm[order[l]])
            S ^= 1 << order[l]
        assert abs(lp - (-math.log(Wm[full]) - acc - np.log(zm).sum())) < 1e-10 * max(1.0, abs(lp))
