"""Point-wise IR/UV-subtracted Feynman-parametric AMM integrand f_G(z).

Oracle code (test infrastructure only).

Paper, section "The method": divergences are removed point by point by a
forest-like formula of linear operators acting on the amplitudes of
UV-divergent subdiagrams; the contribution of each graph to A_1^(2n) is one
Feynman-parametric integral and A_1^(2n) is the sum of these.  The operator
definitions are not printed in the paper; the readings used here are:

  A  anomalous-magnetic-moment projection F2(0) of a vertex (q -> 0, on shell);
  U  for a self-energy Sigma(p) = a(p^2) + b(p^2) pslash:  a(m^2) + b(m^2) pslash;
     for a vertex Gamma^mu(p,p) = a gamma^mu + b p^mu + c p^mu pslash
     + d [pslash, gamma^mu]:  a(m^2) gamma^mu;
  L  on-shell F1(0) of a vertex times gamma^mu.

  f_G = sum over forests F containing G, (-1)^(|F|-1),
        sum over gamma in F that contain the external vertex:
        A on gamma; L on the elements of F strictly between gamma and G;
        (L - U) on G when gamma != G; U on every other element of F.

Arithmetic: long double (x87, unit round-off 2^-64) for the graph
polynomials, the monomial sums and the term combination, or mpmath at 60
significant digits (set_precision("mp")) for ill-conditioned points; Dirac
traces and table coefficients are exact rationals until converted.

A forest term is the product of the operator outputs of its pieces (each
element of F with its maximal sub-elements contracted), written as one
parametric integral over all lines of G (Schwinger form, common scale):

  (-4)^-n (-1)^|F\\G| prod_s U_s^-2 sum_K [t^K] prod_s P_s(t)
        (-1/2)^K Gamma(n-K) (sum_s V_s)^(K-n)

with P_s the projected Wick-contracted numerator of piece s (t counts pairs
of contracted loop momenta), U_s the determinant of its loop matrix and
V_s = m^2 sum over its electron lines z (1 - A), m = 1.  Units: (alpha/pi)^n.
"""
from fractions import Fraction
from functools import lru_cache
from math import gamma as Gamma
import numpy as np

from . import graphs as GR
from .dirac import trace_fast as trace

# ----------------------------------------------------------------------------
# structure: terms and pieces


def _inside(t, s):
    return s["lo"] <= t["lo"] and t["hi"] <= s["hi"] and (t["lo"], t["hi"]) != (s["lo"], s["hi"])


def graph_terms(g):
    """List of (mask, apos): forest mask over subgraphs and the index of the
    element carrying A (-1 for G itself)."""
    subs = GR.subgraphs(g)
    out = []
    for mask in GR.forests(g):
        out.append((mask, -1))
        for i, s in enumerate(subs):
            if mask >> i & 1 and s["has_x"]:
                out.append((mask, i))
    return out


def _build_piece(g, subs, elem, kids, op):
    """Reduced graph of segment ``elem`` with the segments ``kids`` contracted."""
    x, mate = g["x"], g["mate"]
    ch = GR.chords(g)
    photon_of = {}
    for a, (u, v) in enumerate(ch):
        photon_of[u] = a
        photon_of[v] = a
    nodes = []          # list of (kind, data)
    node_of_slot = {}
    s = elem["lo"]
    kid_at = {k["lo"]: k for k in kids}
    while s <= elem["hi"]:
        if s in kid_at:
            k = kid_at[s]
            for t in range(k["lo"], k["hi"] + 1):
                node_of_slot[t] = len(nodes)
            nodes.append(("kid", k))
            s = k["hi"] + 1
        else:
            node_of_slot[s] = len(nodes)
            nodes.append(("slot", s))
            s += 1
    lo, hi = elem["lo"], elem["hi"]
    inside = lambda t: lo <= t <= hi
    # node vertex types
    vtype = []
    pchords = []
    seen = set()
    for j, (kind, d) in enumerate(nodes):
        if kind == "slot":
            s = d
            if s == x:
                vtype.append(("ext",))
            elif inside(mate[s]):
                vtype.append(("ph", photon_of[s]))
                if photon_of[s] not in seen:
                    seen.add(photon_of[s])
                    pchords.append((photon_of[s], j, node_of_slot[mate[s]]))
            else:
                vtype.append(("ext",))
        else:
            k = d
            if k["kind"] == "S":
                vtype.append(("ins", k))
            elif k["has_x"]:
                vtype.append(("ext",))
            else:
                # the chord with exactly one end in k
                t_out = None
                for a, (u, v) in enumerate(ch):
                    iu = k["lo"] <= u <= k["hi"]
                    iv = k["lo"] <= v <= k["hi"]
                    if iu != iv:
                        t_out = (a, v if iu else u)
                a, t = t_out
                if inside(t):
                    vtype.append(("ph", a))
                    if a not in seen:
                        seen.add(a)
                        pchords.append((a, j, node_of_slot[t]))
                else:
                    vtype.append(("ext",))
    # electron lines between consecutive nodes: G line index = last slot of left node
    lines = []
    for j in range(len(nodes) - 1):
        kind, d = nodes[j]
        lines.append(d if kind == "slot" else d["hi"])
    # spans: chord (a, j1, j2) spans piece lines j1..j2-1
    spans = []
    for a, j1, j2 in pchords:
        j1, j2 = min(j1, j2), max(j1, j2)
        spans.append((a, list(range(j1, j2))))
    ext = [j for j, v in enumerate(vtype) if v[0] == "ext"]
    return {
        "elem": elem, "op": op, "nodes": nodes, "vtype": vtype, "lines": lines,
        "spans": spans, "ext": ext[0] if ext else None,
        "kids": kids, "n_lines_total": 3 * g["n"],
    }


def term_pieces(g, mask, apos):
    """Pieces of the forest term (mask, apos), ordered children first.

    Each piece gets its operator: 'A', 'LmU', 'L', 'UV' (vertex U) or 'US'
    (self-energy U, outputs the pair (a, b))."""
    subs = GR.subgraphs(g)
    n = g["n"]
    Gseg = {"lo": 0, "hi": 2 * n, "kind": "V", "has_x": True, "idx": -1}
    elems = [Gseg] + [dict(subs[i], idx=i) for i in range(len(subs)) if mask >> i & 1]
    ap = Gseg if apos < 0 else dict(subs[apos], idx=apos)
    pieces = []
    for e in elems:
        inner = [t for t in elems if _inside(t, e)]
        kids = [t for t in inner if not any(_inside(t, u) for u in inner)]
        if e["idx"] == -1:
            op = "A" if apos < 0 else "LmU"
        elif e["has_x"]:
            if e["idx"] == ap["idx"]:
                op = "A"
            elif _inside(ap, e):
                op = "L"
            else:
                op = "UV"
        else:
            op = "UV" if e["kind"] == "V" else "US"
        pieces.append(_build_piece(g, subs, e, kids, op))
    # children first: sort by segment length
    pieces.sort(key=lambda p: (p["elem"]["hi"] - p["elem"]["lo"]))
    return pieces


# ----------------------------------------------------------------------------
# projected numerators: monomials with exact coefficients

def _pairings(items):
    """All sets of disjoint pairs from ``items`` (any number of pairs)."""
    if not items:
        yield []
        return
    a, rest = items[0], items[1:]
    for m in _pairings(rest):       # a unpaired
        yield m
    for i in range(len(rest)):      # a paired with rest[i]
        b = rest[i]
        for m in _pairings(rest[:i] + rest[i + 1:]):
            yield [(a, b)] + m


def _projector(op):
    """Projector as a list of (coef, prefix symbols, ext symbol, needs_q, q symbol).

    Symbols: 0 = pslash; 'MU' = the label of the external index; 'NU' = label of
    the derivative index (Gamma_1 only).  Strings are prefix + Gamma."""
    F = Fraction
    if op == "Sa":
        return [(F(1, 4), (), None, False)]
    if op == "Sb":
        return [(F(1, 4), (0,), None, False)]
    Tg = ("MU",), "MU"
    Tp = (), 0
    Tpp = (0,), 0
    if op == "UV":
        return [(F(1, 12), Tg[0], Tg[1], False), (F(-1, 12), Tpp[0], Tpp[1], False)]
    if op == "L":
        return [(F(1, 4), Tp[0], Tp[1], False), (F(1, 4), Tpp[0], Tpp[1], False)]
    if op == "LmU":
        return [(F(3, 12), Tp[0], Tp[1], False), (F(4, 12), Tpp[0], Tpp[1], False),
                (F(-1, 12), Tg[0], Tg[1], False)]
    if op == "A":
        out = [(F(-1, 4), Tp[0], Tp[1], False), (F(-1, 3), Tpp[0], Tpp[1], False),
               (F(1, 12), Tg[0], Tg[1], False)]
        # (1/48) Tr[(p+1)(g_mu g_nu - g_nu g_mu)(p+1) Gamma_1^{mu nu}]
        for sgn, mid in ((1, ("MU", "NU")), (-1, ("NU", "MU"))):
            for left in ((0,), ()):
                for right in ((0,), ()):
                    out.append((F(sgn, 48), left + mid + right, "MU", True))
        return out
    raise ValueError(op)


@lru_cache(maxsize=None)
def _piece_monomials(sig):
    """Monomials of a piece: tuple of (k, coef, pairs, pslots, qslot).

    ``sig`` = (op, vertex factors from the last node to the first with line
    slots in between) -- see _piece_signature.  Slots are integers; a slot's
    factor is either a real line ('L', slot) or a pseudo line ('P', slot)."""
    op, seq = sig
    slots = [it[1] for it in seq if it[0] in ("L", "P")]
    real = {it[1] for it in seq if it[0] == "L"}
    proj = _projector(op)
    need_q = any(pr[3] for pr in proj)
    acc = {}
    for pairs in _pairings(slots):
        paired = {s for pr in pairs for s in pr}
        free = [s for s in slots if s not in paired]
        k = len(pairs)
        # choices for free slots: 'm' (real lines only), 'p', and at most one 'q'
        choices = [("m", "p") if s in real else ("p",) for s in free]
        qopts = [None] + (free if need_q else [])
        for qs in qopts:
            def rec(i, cur):
                if i == len(free):
                    yield dict(cur)
                    return
                s = free[i]
                if s == qs:
                    cur[s] = "q"
                    yield from rec(i + 1, cur)
                    return
                for c in choices[i]:
                    cur[s] = c
                    yield from rec(i + 1, cur)
            for ch in rec(0, {}):
                lab = {}
                nxt = [10]
                def L(key):
                    if key not in lab:
                        lab[key] = nxt[0]
                        nxt[0] += 1
                    return lab[key]
                for a, b in pairs:
                    la = L(("pair", a, b))
                    lab[("slot", a)] = la
                    lab[("slot", b)] = la
                total = Fraction(0)
                for coef, prefix, extsym, isq in proj:
                    if isq != (qs is not None):
                        continue
                    body = []
                    for it in seq:
                        if it[0] == "V":
                            v = it[1]
                            if v[0] == "ext":
                                body.append(L("MU") if extsym == "MU" else 0)
                            elif v[0] == "ph":
                                body.append(L(("ph", v[1])))
                            else:
                                raise ValueError(v)
                        else:
                            s = it[1]
                            c = ch.get(s)
                            if c is None:
                                body.append(lab[("slot", s)])
                            elif c == "m":
                                pass
                            elif c == "p":
                                body.append(0)
                            else:
                                body.append(L("NU"))
                    pre = [L(v) if isinstance(v, str) else v for v in prefix]
                    tr = trace(tuple(pre) + tuple(body))
                    if tr:
                        total += coef * tr
                if total:
                    ps = tuple(sorted(s for s, c in ch.items() if c == "p"))
                    key = (k, tuple(pairs), ps, qs)
                    acc[key] = acc.get(key, 0) + total
    return tuple((k, c, pr, ps, qs) for (k, pr, ps, qs), c in sorted(acc.items(), key=lambda t: str(t[0])) if c)


def _piece_signature(piece, variant):
    """Dirac string skeleton of a piece for one choice of self-energy outputs.

    ``variant`` maps insertion node -> 'a' | 'b'.  Returns (seq, slot_line)
    with seq from the last node to the first: ('V', vertex) for photon/ext
    vertices, ('L', slot) for lines, ('P', slot) for pseudo lines (b-insertions).
    slot_line maps slot -> piece line position that carries its momentum."""
    nodes, vt = piece["nodes"], piece["vtype"]
    nl = len(piece["lines"])
    seq = []
    slot_line = {}
    nxt = nl
    for j in range(len(nodes) - 1, -1, -1):
        v = vt[j]
        if v[0] == "ins":
            if variant[j] == "b":
                seq.append(("P", nxt))
                slot_line[nxt] = j - 1
                nxt += 1
        else:
            seq.append(("V", v))
        if j > 0:
            seq.append(("L", j - 1))
            slot_line[j - 1] = j - 1
    return tuple(seq), slot_line


# ----------------------------------------------------------------------------
# geometry at a point


LD = np.longdouble

# numeric context: dtype of arrays and the conversion of floats / rationals
_NUM = {"mode": "ld", "dtype": LD, "conv": LD}


def set_precision(mode="ld", dps=60):
    """'ld' (long double, vectorised) or 'mp' (mpmath, dps digits)."""
    if mode == "ld":
        _NUM.update(mode="ld", dtype=LD, conv=LD)
    else:
        import mpmath
        mpmath.mp.dps = dps
        _NUM.update(mode="mp", dtype=object, conv=mpmath.mpf)


def _c(x):
    """Convert a float or Fraction into the working precision."""
    conv = _NUM["conv"]
    if isinstance(x, Fraction):
        return conv(x.numerator) / conv(x.denominator)
    return conv(x)


def _spd_inverse_det(M):
    """Determinant and inverse of a small symmetric positive definite matrix
    by Gauss-Jordan elimination in long double."""
    L = M.shape[0]
    A = M.copy()
    inv = np.zeros((L, L), dtype=_NUM["dtype"])
    for i in range(L):
        inv[i, i] = _c(1)
    det = _c(1)
    for c in range(L):
        piv = A[c, c]
        det *= piv
        A[c] /= piv
        inv[c] /= piv
        for r in range(L):
            if r != c:
                fac = A[r, c]
                A[r] -= fac * A[c]
                inv[r] -= fac * inv[c]
    return det, inv


def piece_geometry(piece, z, g):
    """Loop matrix, U, flows A (momentum p) and C (momentum q), V, and the
    Wick contraction matrix Bbar of the piece's electron lines at z
    (long double)."""
    n = g["n"]
    lines = piece["lines"]
    spans = piece["spans"]
    dt = _NUM["dtype"]
    ze = np.array([_c(float(z[l])) for l in lines], dtype=dt)
    L = len(spans)
    nl = len(lines)
    eta = np.zeros((nl, L), dtype=dt)
    eta[:] = _c(0)
    M = np.zeros((L, L), dtype=dt)
    M[:] = _c(0)
    for c, (a, sp) in enumerate(spans):
        eta[sp, c] = _c(1)
        M[c, c] += _c(float(z[2 * n + a]))
    M += (eta * ze[:, None]).T @ eta
    U, Minv = _spd_inverse_det(M)
    j = eta.T @ ze
    A = _c(1) - eta @ (Minv @ j)
    ext = piece["ext"]
    if ext is not None:
        Pq = np.array([_c(-0.5) if ln < ext else _c(0.5) for ln in range(nl)], dtype=dt)
        jq = eta.T @ (ze * Pq)
        C = Pq - eta @ (Minv @ jq)
    else:
        C = np.array([_c(0)] * nl, dtype=dt)
    V = np.sum(ze * (_c(1) - A))
    B = eta @ Minv @ eta.T
    return {"U": U, "A": A, "C": C, "V": V, "B": B}


def _zeros(n):
    out = np.zeros(n, dtype=_NUM["dtype"])
    out[:] = _c(0)
    return out


def _poly_mul(a, b, n):
    out = _zeros(n)
    for i in range(n):
        if a[i] == 0:
            continue
        for j in range(n - i):
            out[i + j] += a[i] * b[j]
    return out


_PACKED = {}


def _pack(mons, slot_line):
    """Monomials as arrays: k, coef, pair line indices, p-slot lines, q line."""
    key = (id(mons), tuple(sorted(slot_line.items())), _NUM["mode"])
    if key in _PACKED:
        return _PACKED[key]
    m = len(mons)
    K = np.zeros(m, dtype=np.int64)
    coef = np.zeros(m, dtype=_NUM["dtype"])
    P1 = np.full((m, 6), -1, dtype=np.int64)
    P2 = np.full((m, 6), -1, dtype=np.int64)
    AS = np.full((m, 14), -1, dtype=np.int64)
    Q = np.full(m, -1, dtype=np.int64)
    for i, (k, c, pairs, ps, qs) in enumerate(mons):
        K[i] = k
        coef[i] = _c(c)
        for j, (a, b) in enumerate(pairs):
            P1[i, j] = slot_line[a]
            P2[i, j] = slot_line[b]
        for j, sl in enumerate(ps):
            AS[i, j] = slot_line[sl]
        if qs is not None:
            Q[i] = slot_line[qs]
    _PACKED[key] = (mons, K, coef, P1, P2, AS, Q)
    return _PACKED[key]


def _eval_monomials(mons, slot_line, geo, n):
    _, K, coef, P1, P2, AS, Q = _pack(mons, slot_line)
    A, C, B = geo["A"], geo["C"], geo["B"]
    nl = len(A)
    dt = _NUM["dtype"]
    Bp = np.zeros((nl + 1, nl + 1), dtype=dt)
    Bp[:] = _c(1)
    Bp[:nl, :nl] = B
    Ap = np.append(A, _c(1)).astype(dt)
    Cp = np.append(C, _c(1)).astype(dt)
    w = coef * np.prod(Bp[P1, P2], axis=1) * np.prod(Ap[AS], axis=1) * Cp[Q]
    keep = K < n
    out = _zeros(n)
    np.add.at(out, K[keep], w[keep])
    return out


def term_value(g, mask, apos, z, pieces=None):
    n = g["n"]
    if pieces is None:
        pieces = term_pieces(g, mask, apos)
    geos = [piece_geometry(p, z, g) for p in pieces]
    key = lambda e: (e["lo"], e["hi"])
    by_elem = {key(p["elem"]): i for i, p in enumerate(pieces)}
    out = {}
    for i, p in enumerate(pieces):           # children first
        ins = [j for j, v in enumerate(p["vtype"]) if v[0] == "ins"]
        vkids = [k for k in p["kids"] if k["kind"] == "V"]
        base = _zeros(n)
        base[0] = _c(1)
        for k in vkids:
            base = _poly_mul(base, out[key(k)], n)
        ops = ["Sa", "Sb"] if p["op"] == "US" else [p["op"]]
        res = []
        for op in ops:
            tot = _zeros(n)
            for bits in range(1 << len(ins)):
                variant = {j: ("b" if bits >> t & 1 else "a") for t, j in enumerate(ins)}
                seq, slot_line = _piece_signature(p, variant)
                mons = _piece_monomials((op, seq))
                P = _eval_monomials(mons, slot_line, geos[i], n)
                for t, j in enumerate(ins):
                    kid = p["nodes"][j][1]
                    P = _poly_mul(P, out[key(kid)][1 if bits >> t & 1 else 0], n)
                tot += P
            res.append(_poly_mul(tot, base, n))
        out[key(p["elem"])] = res if p["op"] == "US" else res[0]
    top = out[(0, 2 * n)]
    Vt = sum(gg["V"] for gg in geos)
    pref = _c(1)
    for gg in geos:
        pref /= gg["U"] ** 2
    s = _c(0)
    for K in range(n):
        s += top[K] * _c((-0.5) ** K * Gamma(n - K)) * Vt ** (K - n)
    sign = -1 if (bin(mask).count("1") + n) % 2 else 1
    return sign * pref * s / _c(4) ** n


class Integrand:
    """f_G(z) for one graph: the sum of its forest terms."""

    def __init__(self, g):
        self.g = g
        self.terms = [(m, a, term_pieces(g, m, a)) for m, a in graph_terms(g)]

    def __call__(self, z, return_terms=False):
        """f_G(z) in long double, returned as a Python float (and the forest
        terms as floats)."""
        vals = [term_value(self.g, m, a, z, pcs) for m, a, pcs in self.terms]
        tot = sum(vals, _c(0))
        if return_terms:
            return float(tot), [float(v) for v in vals]
        return float(tot)


# Gauss-Legendre nodes and weights on [0, 1], three points (exact for
# polynomials of degree <= 5 in the split)
_GL3 = ((0.5 - 0.5 * (3.0 / 5.0) ** 0.5, 5.0 / 18.0), (0.5, 8.0 / 18.0), (0.5 + 0.5 * (3.0 / 5.0) ** 0.5, 5.0 / 18.0))


class MergedIntegrand:
    """The 3n-2-variable integrand (paper's footnote on 3n-1 -> 3n-2): with
    s = z_a + z_b the parameter of the two electron lines next to the external
    vertex (a = x-1, b = x), f_m(s, rest) = s * int_0^1 f(t s, (1-t) s, rest) dt,
    the split integrated by three-point Gauss-Legendre (the integrand is a
    polynomial of low degree in t; see tests)."""

    def __init__(self, g):
        from .pdf import expand_point
        self.g = g
        self.f = Integrand(g)
        self._expand = expand_point

    def __call__(self, zm, nodes=_GL3):
        from .pdf import merged_lines
        a, _ = merged_lines(self.g)
        s = float(zm[a])
        tot = 0.0
        for t, w in nodes:
            tot += w * self.f(self._expand(self.g, np.asarray(zm, dtype=float), t))
        return s * tot
