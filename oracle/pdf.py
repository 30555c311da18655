"""Hepp-sector probability density of eq. (1) and its sampler.

Oracle code (test infrastructure only).

eq. (1): in the sector z_{j1} >= ... >= z_{jM},
  p(z) = C prod_{l=2..M} (z_{jl}/z_{j(l-1)})^Deg(S_l) / (z_1 ... z_M),
  S_l = {j_l, ..., j_M}.
With t_l = ln(z_{j(l-1)}/z_{jl}) the measure d^{M-1}z / prod z equals
prod dt_l, so inside a sector the t_l are independent Exp(Deg(S_l)) and the
sector has weight prod_l 1/Deg(S_l).  Summing over sectors:
  W(S) = Deg(S)^-1 sum_{j in S} W(S\\{j})  (|S| < M),  W({j}) = 1/Deg({j}),
  W(full) = sum_j W(full\\{j}),  C = 1/W(full).

Deg (section "The method"): positive numbers on proper nonempty line sets;
-omega(s) (minus the UV degree of divergence) in the plain case, with omega
applied to the I-closure of s for the infrared limit; the full definition is
not printed.  Reading used here (degrees in Feynman-parameter units, half the
momentum-space ones, which is what makes Deg fractional):
  omega_F(s) = 2 sum_{pieces P of forest F} h_P(s) - N_ph(s) - N_el(s)/2,
  Deg(s) = max(1/2, min over forests F of -omega_F(I(s))),
where h_P(s) is the number of independent loops formed by the lines of s in
the reduced graph of piece P (a forest's counterterm behaves like the product
of its pieces, whose reduced graphs can close loops that G does not), and
I(s) = s plus every photon whose electron path between its ends lies in s.
"""
from math import log, exp
import numpy as np

from . import graphs as GR
from .philox import uniforms


def line_endpoints(g):
    n = g["n"]
    ends = [(i, i + 1) for i in range(2 * n)]
    ends += list(GR.chords(g))
    return ends


def _cyclomatic(edges):
    """Independent loops of a multigraph given as (a, b) vertex pairs."""
    if not edges:
        return 0
    parent = {}

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    for a, b in edges:
        parent.setdefault(a, a)
        parent.setdefault(b, b)
    for a, b in edges:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
    comps = len({find(v) for v in parent})
    return len(edges) - len(parent) + comps


def omega(g, s):
    """Parametric UV degree of the line set s (bitmask) in G itself."""
    n = g["n"]
    ends = line_endpoints(g)
    idx = [i for i in range(3 * n) if s >> i & 1]
    nel = sum(1 for i in idx if i < 2 * n)
    nph = len(idx) - nel
    return 2 * _cyclomatic([ends[i] for i in idx]) - nph - nel / 2.0


def i_closure(g, s):
    n = g["n"]
    out = s
    for a, (u, v) in enumerate(GR.chords(g)):
        if all(s >> e & 1 for e in range(u, v)):
            out |= 1 << (2 * n + a)
    return out


def _forest_piece_edges(g):
    """For every forest: the pieces' reduced graphs as lists of (line, a, b)."""
    from .integrand import term_pieces
    n = g["n"]
    out = []
    for mask in GR.forests(g):
        st = []
        for p in term_pieces(g, mask, -1):
            E = [(l, j, j + 1) for j, l in enumerate(p["lines"])]
            E += [(2 * n + a, sp[0], sp[-1] + 1) for a, sp in p["spans"]]
            st.append(E)
        out.append(st)
    return out


def deg_table(g, delta=0.5):
    """Deg over all bitmasks 0..2^M-1 (entries 0 and full unused: 0.0)."""
    n = g["n"]
    M = 3 * n
    full = (1 << M) - 1
    structs = _forest_piece_edges(g)
    D = np.zeros(1 << M)
    for s in range(1, full):
        c = i_closure(g, s)
        nel = sum(1 for i in range(2 * n) if c >> i & 1)
        nph = bin(c).count("1") - nel
        best = None
        for st in structs:
            h = sum(_cyclomatic([(a, b) for (l, a, b) in E if c >> l & 1]) for E in st)
            v = -(2 * h - nph - nel / 2.0)
            best = v if best is None else min(best, v)
        D[s] = max(delta, best)
    return D


def w_table(deg, M):
    full = (1 << M) - 1
    W = np.zeros(1 << M)
    for s in sorted(range(1, full + 1), key=lambda t: bin(t).count("1")):
        tot = 0.0
        if bin(s).count("1") == 1:
            W[s] = 1.0 / deg[s]
            continue
        t = s
        while t:
            j = t & -t
            tot += W[s ^ j]
            t ^= j
        W[s] = tot if s == full else tot / deg[s]
    return W


def sample(deg, W, M, u):
    """One point from 2(M-1) uniforms: returns (z, log p, sector)."""
    full = (1 << M) - 1
    S = full
    order = []
    for l in range(M - 1):
        tot = 0.0
        js = [j for j in range(M) if S >> j & 1]
        ws = [W[S ^ (1 << j)] for j in js]
        for w in ws:
            tot += w
        target = u[l] * tot
        cum = 0.0
        pick = js[-1]
        for j, w in zip(js, ws):
            cum += w
            if target < cum:
                pick = j
                break
        order.append(pick)
        S ^= 1 << pick
    order.append(S.bit_length() - 1)
    lz = np.zeros(M)
    S = full ^ (1 << order[0])
    run = 0.0
    degsum = 0.0
    for l in range(1, M):
        d = deg[S]
        t = -log(u[M - 1 + l - 1]) / d
        run -= t
        degsum += d * t
        lz[order[l]] = run
        S ^= 1 << order[l]
    zmax = max(lz)
    z = np.exp(lz - zmax)
    norm = z.sum()
    z = z / norm
    logp = -log(W[full]) - degsum - float(np.sum(np.log(z)))
    return z, logp, order


def sample_stream(g, deg, W, seed, tag, graph, first, count):
    M = 3 * g["n"]
    out = []
    for i in range(first, first + count):
        u = uniforms(seed, tag, graph, i, 2 * (M - 1))
        out.append(sample(deg, W, M, u))
    return out


# ----------------------------------------------------------------------------
# 3n-2 variables (the paper's footnote on reducing 3n-1 to 3n-2): at q = 0 the
# two electron lines next to the external vertex, a = x-1 and b = x, carry
# the same momentum, so the integral over their split is done before the
# Monte Carlo: the pair becomes one "merged" line with parameter s = z_a + z_b
# and the remaining 3n-1 parameters live on a simplex of dimension 3n-2.
# Merged line j stands for original line j (j < b) or j + 1 (j >= b); merged
# line a stands for {a, b}.

def merged_lines(g):
    """(a, b) of the merged pair."""
    x = g["x"]
    return x - 1, x


def expand_set(g, Sm):
    """Original line set of a merged-line set."""
    a, b = merged_lines(g)
    low = Sm & ((1 << b) - 1)
    high = (Sm >> b) << (b + 1)
    out = low | high
    if Sm >> a & 1:
        out |= 1 << b
    return out


def merged_deg_table(g, D):
    """Deg over the merged lines: Deg'(S') = Deg(expand(S'))."""
    Mm = 3 * g["n"] - 1
    full = (1 << Mm) - 1
    Dm = np.zeros(1 << Mm)
    for S in range(1, full):
        Dm[S] = D[expand_set(g, S)]
    return Dm


def expand_point(g, zm, t=0.5):
    """Original parameters from merged ones, split t : 1-t on (a, b)."""
    a, b = merged_lines(g)
    s = zm[a]
    z = np.concatenate([zm[:b], [0.0], zm[b:]])
    z[a], z[b] = t * s, (1.0 - t) * s
    return z


def sample_merged(g, Dm, Wm, u):
    """One point of the merged form: (merged z, log p of the merged density,
    sector) from eq. (1) over the 3n-1 merged lines."""
    return sample(Dm, Wm, 3 * g["n"] - 1, u)
