"""Vertex graphs without lepton loops, their gauge-invariant classes, their
UV-divergent subgraphs and forests.

Oracle code (test infrastructure only).

A graph at n loops is an open electron line with 2n+1 vertex slots 0..2n.
The external photon sits at slot ``x``; the other 2n slots are paired by n
internal photons ("chords").  Lines: electron line i joins slot i and slot i+1
(i = 0..2n-1); photon line 2n+a is the a-th chord in order of its lower end.

Paper: the set is "all diagrams without lepton loops" counted with arrow
reversal identified (footnote to Table 1); the classes (k,m,n) count photons
left / right of the external photon and photons crossing it (text before
Figure 1).  Divergent subdiagrams are the objects of the subtraction
procedure (section "The method").
"""
from itertools import combinations


def _matchings(items):
    if not items:
        yield []
        return
    a = items[0]
    for i in range(1, len(items)):
        b = items[i]
        rest = items[1:i] + items[i + 1:]
        for m in _matchings(rest):
            yield [(a, b)] + m


def _has_external_self_energy(n, x, mate):
    # A prefix [0..j] (j < x) or suffix [j..2n] (j > x) closed under the photon
    # pairing is a self-energy insertion on an external electron leg.
    for j in range(0, x):
        if all(mate[s] <= j for s in range(0, j + 1)):
            return True
    for j in range(x + 1, 2 * n + 1):
        if all(mate[s] >= j for s in range(j, 2 * n + 1)):
            return True
    return False


def encode(n, x, mate):
    """Tuple key: (x, mate[0..2n]) with mate[x] = x."""
    return (x,) + tuple(mate)


def reverse(n, x, mate):
    N = 2 * n
    rm = [0] * (N + 1)
    for s in range(N + 1):
        rm[N - s] = N - mate[s]
    return N - x, rm


def enumerate_raw(n):
    """All raw graphs (x, mate) at n loops, external legs free of self-energies."""
    N = 2 * n
    out = []
    for x in range(N + 1):
        others = [s for s in range(N + 1) if s != x]
        for m in _matchings(others):
            mate = [0] * (N + 1)
            mate[x] = x
            for a, b in m:
                mate[a] = b
                mate[b] = a
            if not _has_external_self_energy(n, x, mate):
                out.append((x, mate))
    return out


def graph_class(n, x, mate):
    """(k, m, n'): photons crossing x, and max/min of photons left / right of x."""
    k = left = right = 0
    for s in range(2 * n + 1):
        if s == x or mate[s] < s:
            continue
        a, b = s, mate[s]
        if a < x < b:
            k += 1
        elif b < x:
            left += 1
        else:
            right += 1
    return (k, max(left, right), min(left, right))


def enumerate_graphs(n, cls=None):
    """Canonical representatives: list of dicts sorted by their key.

    The representative is the lexicographically smaller key of a graph and its
    reversal; ``mult`` is 1 for self-reversed graphs and 2 otherwise.
    ``cls`` filters on the (k, m, n) class (None = all).
    """
    reps = {}
    for x, mate in enumerate_raw(n):
        k1 = encode(n, x, mate)
        rx, rm = reverse(n, x, mate)
        k2 = encode(n, rx, rm)
        key = min(k1, k2)
        reps[key] = 1 if k1 == k2 else 2
    out = []
    for key in sorted(reps):
        x = key[0]
        mate = list(key[1:])
        c = graph_class(n, x, mate)
        if cls is not None and tuple(cls) != c:
            continue
        out.append({"n": n, "x": x, "mate": mate, "mult": reps[key], "cls": c})
    return out


def chords(g):
    """Chords (a, b), a < b, sorted by a: chord index = photon index."""
    n, x, mate = g["n"], g["x"], g["mate"]
    return [(s, mate[s]) for s in range(2 * n + 1) if s != x and mate[s] > s]


def subgraphs(g):
    """UV-divergent 1PI subgraphs as segments [lo, hi] != [0, 2n], sorted.

    Each entry: dict(lo, hi, kind 'V' (vertex-like) or 'S' (self-energy-like),
    has_x (the external vertex lies inside)).
    """
    n, x, mate = g["n"], g["x"], g["mate"]
    N = 2 * n
    ch = chords(g)
    out = []
    for lo in range(N + 1):
        for hi in range(lo + 1, N + 1):
            if lo == 0 and hi == N:
                continue
            ext = 0
            for a, b in ch:
                ina, inb = lo <= a <= hi, lo <= b <= hi
                if ina != inb:
                    ext += 1
            has_x = lo <= x <= hi
            ext += 1 if has_x else 0
            if ext > 1:
                continue
            # 1PI: every electron line i (slot i -> i+1) inside is spanned by an inner chord
            ok = True
            for i in range(lo, hi):
                if not any(lo <= a <= i and i + 1 <= b <= hi for a, b in ch):
                    ok = False
                    break
            if not ok:
                continue
            out.append({"lo": lo, "hi": hi, "kind": "V" if ext == 1 else "S", "has_x": has_x})
    return out


def _compatible(s, t):
    nested = (s["lo"] <= t["lo"] and t["hi"] <= s["hi"]) or (t["lo"] <= s["lo"] and s["hi"] <= t["hi"])
    disjoint = s["hi"] < t["lo"] or t["hi"] < s["lo"]
    return nested or disjoint


def forests(g):
    """Forests of proper subgraphs as sorted bitmasks (bit i = subgraph i).

    The whole graph G belongs to every forest implicitly; the empty mask is the
    forest {G}.
    """
    subs = subgraphs(g)
    k = len(subs)
    out = []
    for mask in range(1 << k):
        idx = [i for i in range(k) if mask >> i & 1]
        if all(_compatible(subs[i], subs[j]) for i, j in combinations(idx, 2)):
            out.append(mask)
    return out
