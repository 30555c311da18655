"""Dirac traces of gamma strings with contracted Lorentz indices.

Oracle code (test infrastructure only).

A string is a tuple of symbols read left to right as a matrix product:
  0      the slashed on-shell momentum p-slash, with p.p = m^2 = 1;
  L > 0  a gamma matrix whose index is contracted with the other gamma in the
         string that carries the same label L (metric g, signature +---).
Every label occurs exactly twice.  Traces are exact integers.

Method: textbook 4-dimensional contraction identities (Chisholm):
  g^a g_a = 4,
  g^a S g_a = -2 S^R                      for S a product of an odd number,
  g^a s1..sk g_a = 2 (sk s1..s(k-1) + s(k-1)..s1 sk)   for k even >= 2,
applied to an innermost-first choice of contracted pair, and p-slash p-slash = 1.
When no contracted pair is left the string is a power of p-slash.
"""
import ctypes
import os
from functools import lru_cache

_C = None


def _ctrace():
    """The plain-C port of the same recursion (oracle/_ctrace.so), if built."""
    global _C
    if _C is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_ctrace.so")
        if os.path.exists(path):
            lib = ctypes.CDLL(path)
            lib.oracle_trace.restype = ctypes.c_longlong
            lib.oracle_trace.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_int]
            _C = lib
        else:
            _C = False
    return _C or None


def trace_fast(s):
    """Same value as trace(s); uses the C port when it is built."""
    lib = _ctrace()
    if lib is None or len(s) > 60:
        return trace(s)
    arr = (ctypes.c_int * len(s))(*s)
    return int(lib.oracle_trace(arr, len(s)))


def _canon(s):
    # relabel contracted pairs by order of first appearance (memo key)
    m = {}
    out = []
    for v in s:
        if v == 0:
            out.append(0)
        else:
            if v not in m:
                m[v] = len(m) + 1
            out.append(m[v])
    return tuple(out)


def _reduce_pp(s):
    # p p = 1 for adjacent on-shell momenta (cyclic adjacency is handled by the trace)
    out = []
    for v in s:
        if v == 0 and out and out[-1] == 0:
            out.pop()
        else:
            out.append(v)
    return tuple(out)


def trace(s):
    """Exact trace of the string ``s`` (tuple of symbols)."""
    return _trace(_canon(_reduce_pp(tuple(s))))


@lru_cache(maxsize=None)
def _trace(s):
    if len(s) % 2:
        return 0
    labels = set(v for v in s if v)
    if not labels:
        return 4  # p-slash to an even power is 1
    # choose the contracted pair with the shortest inner string, preferring odd length
    pos = {}
    for i, v in enumerate(s):
        if v:
            pos.setdefault(v, []).append(i)
    best = None
    for v, (i, j) in pos.items():
        k = j - i - 1
        key = (k % 2 == 0 and k > 0, k)
        if best is None or key < best[0]:
            best = (key, i, j)
    _, i, j = best
    head, inner, tail = s[:i], s[i + 1:j], s[j + 1:]
    k = len(inner)
    if k == 0:
        return 4 * trace(head + tail)
    if k % 2 == 1:
        return -2 * trace(head + inner[::-1] + tail)
    t1 = head + (inner[-1],) + inner[:-1] + tail
    t2 = head + inner[:-1][::-1] + (inner[-1],) + tail
    return 2 * (trace(t1) + trace(t2))
