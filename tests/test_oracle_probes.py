"""Oracle pins of the graph polynomials and the subtracted integrand at
3 loops (test infrastructure):

- the contraction coefficients from the spanning-tree polynomial alone
  (Jacobi's formula: Bbar_ii = d ln U / d z_i and Bbar_ij^2 =
  -d^2 ln U / d z_i d z_j, U the brute-force spanning-tree sum), independent
  of the oracle's matrix inverse;
- finiteness toward every sector boundary (section "The method": the
  subtracted integrand of each graph is finite): for every 3-loop graph and
  every proper nonempty line set S, the decay rate kappa(S) of |f prod z| as
  the lines of S shrink (z_S -> e^-T z_S) is positive, and Deg(S) < 2 kappa(S),
  the condition for finite variance along that limit;
- mirror invariance on every graph whose forest terms use the operator L
  (nested vertex subgraphs around the external vertex), at 3 and 4 loops."""
import itertools
import math

import numpy as np
import pytest

from oracle import graphs as GR, integrand as IN, pdf as PD


def _trees(E, nv):
    out = []
    for T in itertools.combinations(range(len(E)), nv - 1):
        par = list(range(nv))

        def f(a):
            while par[a] != a:
                a = par[a]
            return a
        ok = True
        for i in T:
            a, b = f(E[i][1]), f(E[i][2])
            if a == b:
                ok = False
                break
            par[a] = b
        if ok:
            out.append(set(T))
    return out


def _poly(E, trees, z, drop=()):
    """sum over spanning trees T avoiding the edges `drop` of prod_{e not in T, e not in drop} z_e"""
    tot = 0.0
    for T in trees:
        if any(d in T for d in drop):
            continue
        tot += math.prod(z[E[i][0]] for i in range(len(E)) if i not in T and i not in drop)
    return tot


def test_bbar_from_spanning_tree_derivatives():
    rng = np.random.default_rng(8)
    checked = 0
    for g in GR.enumerate_graphs(3)[::3]:
        for m, a in IN.graph_terms(g)[:3]:
            for p in IN.term_pieces(g, m, a):
                n = g["n"]
                E = [(l, j, j + 1) for j, l in enumerate(p["lines"])]
                E += [(2 * n + c, sp[0], sp[-1] + 1) for c, sp in p["spans"]]
                nv = len(p["nodes"])
                z = rng.dirichlet(np.ones(3 * n))
                trees = _trees(E, nv)
                U = _poly(E, trees, z)
                B = IN.piece_geometry(p, z, g)["B"]
                nl = len(p["lines"])
                for i in range(nl):
                    Ui = _poly(E, trees, z, (i,))
                    assert abs(float(B[i, i]) - Ui / U) <= 1e-12 * (Ui / U), (i,)
                    for j in range(i + 1, nl):
                        Uj = _poly(E, trees, z, (j,))
                        Uij = _poly(E, trees, z, (i, j))
                        b2 = (Ui * Uj - U * Uij) / (U * U)
                        assert abs(float(B[i, j]) ** 2 - b2) <= 1e-11 * (Ui * Uj) / (U * U), (i, j)
                        checked += 1
    assert checked > 100


def _kappa(f, z0, mask, T1, T2):
    vals = []
    for T in (T1, T2):
        z = z0.copy()
        z[mask] *= math.exp(-T)
        z /= z.sum()
        vals.append(abs(f(z)) * np.prod(z))
    return -(math.log(vals[1]) - math.log(vals[0])) / (T2 - T1)


def test_finite_toward_every_boundary_3loop():
    """kappa from the slope between T = 6 and 10 in long double; where that
    reads below 1/2 (a slow approach to the limit, or long double losing the
    subtraction's cancellation), the slope between T = 12 and 20 at 60
    digits decides."""
    worst, redo = 1e9, 0
    for gi, g in enumerate(GR.enumerate_graphs(3)):
        f = IN.Integrand(g)
        D = PD.deg_table(g)
        z0 = np.random.default_rng(100 + gi).dirichlet(np.ones(9))
        for S in range(1, (1 << 9) - 1):
            mask = np.array([(S >> j) & 1 for j in range(9)], bool)
            k = _kappa(f, z0, mask, 6.0, 10.0)
            if k <= 0.5:
                redo += 1
                IN.set_precision("mp", 60)
                try:
                    k = _kappa(f, z0, mask, 12.0, 20.0)
                finally:
                    IN.set_precision("ld")
            worst = min(worst, k - D[S] / 2)
            assert k > 0.25, (gi, S, k)
            assert D[S] < 2 * k, (gi, S, D[S], k)
    assert worst > 0 and redo < 200


def _line_map_reversed(g):
    n, N = g["n"], 2 * g["n"]
    rx, rm = GR.reverse(n, g["x"], g["mate"])
    rg = {"n": n, "x": rx, "mate": rm}
    perm = {i: N - 1 - i for i in range(N)}
    rch = GR.chords(rg)
    for a, (u, v) in enumerate(GR.chords(g)):
        perm[N + a] = N + rch.index((N - v, N - u))
    return rg, perm


@pytest.mark.parametrize("n,count,least", [(3, 28, 1), (4, 6, 6)])
def test_mirror_invariance_with_L(n, count, least):
    """Graphs with an L-carrying term (an A on a vertex subgraph nested in a
    larger one around the external vertex)."""
    rng = np.random.default_rng(12)
    done = 0
    for g in GR.enumerate_graphs(n):
        subs = GR.subgraphs(g)
        with_L = any(
            any(pc["op"] == "L" for pc in IN.term_pieces(g, m, a))
            for m, a in IN.graph_terms(g) if a >= 0)
        if not with_L:
            continue
        rg, perm = _line_map_reversed(g)
        f, fr = IN.Integrand(g), IN.Integrand(rg)
        z = rng.dirichlet(np.ones(3 * n))
        zr = np.zeros_like(z)
        for i, j in perm.items():
            zr[j] = z[i]
        a, terms = f(z, True)
        assert abs(a - fr(zr)) <= 1e-11 * sum(abs(t) for t in terms)
        done += 1
        if done >= count:
            break
    assert done >= least
