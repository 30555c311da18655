"""Oracle pins: Dirac traces against explicit 4x4 matrices (brute force over
index values), Philox4x32-10 against its published known-answer vectors."""
import itertools
import random

import numpy as np

from oracle.dirac import trace
from oracle.philox import philox4x32_10, u01


def _gammas():
    I2 = np.eye(2)
    Z = np.zeros((2, 2))
    s = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]
    g0 = np.block([[I2, Z], [Z, -I2]])
    return [g0] + [np.block([[Z, si], [-si, Z]]) for si in s]


def _brute(st, G):
    eta = [1, -1, -1, -1]
    labels = sorted(set(v for v in st if v))
    tot = 0
    for idx in itertools.product(range(4), repeat=len(labels)):
        a = dict(zip(labels, idx))
        M = np.eye(4, dtype=complex)
        sign = 1
        seen = set()
        for v in st:
            if v == 0:
                M = M @ G[0]          # p-slash with p = (1, 0, 0, 0)
            else:
                M = M @ G[a[v]]
                if v in seen:
                    sign *= eta[a[v]]
                seen.add(v)
        tot += sign * np.trace(M)
    return tot


def test_trace_vs_explicit_matrices():
    G = _gammas()
    rng = random.Random(3)
    for _ in range(150):
        npairs = rng.randint(0, 4)
        nps = rng.randint(0, 4)
        st = [l for l in range(1, npairs + 1) for _ in (0, 1)] + [0] * nps
        rng.shuffle(st)
        assert abs(trace(st) - _brute(st, G)) < 1e-9, st


def test_philox_known_answers():
    # Known-answer vectors published with the Philox generator (Salmon et al. 2011)
    assert philox4x32_10((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    assert philox4x32_10((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2) == (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)
    assert philox4x32_10((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0)) == \
        (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def test_u01_open_interval():
    assert 0.0 < u01(0, 0) < 1e-15
    assert 1.0 - 1e-15 < u01(0xFFFFFFFF, 0xFFFFFFFF) < 1.0
