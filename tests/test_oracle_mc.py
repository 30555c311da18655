"""Pins of the oracle's estimator and combination (test infrastructure).

mc.estimate is the unbiased sample mean / variance of the weights, checked
against numpy's definitions on explicit samples; mc.combine is the
inverse-variance combination, checked against the paper's own combination of
its two calculations (section "Preliminary numerical results", eq. (2):
6.739(132) and 6.905(220) give 6.782(113)) and the same for every class row
of Table 1 (value column from the Calc 1 and Calc 2 columns), within the
rounding of the printed inputs."""
import math

import numpy as np
import pytest

from oracle import mc

# Table 1 rows: (value, sigma), (Calc 1), (Calc 2)
TABLE1 = {
    (1, 4, 0): ((6.172, 0.042), (6.158, 0.049), (6.209, 0.080)),
    (2, 3, 0): ((-0.724, 0.054), (-0.746, 0.063), (-0.66, 0.10)),
    (1, 3, 1): ((0.895, 0.043), (0.854, 0.050), (1.007, 0.082)),
    (3, 2, 0): ((-0.396, 0.043), (-0.399, 0.051), (-0.390, 0.085)),
    (2, 2, 1): ((-2.160, 0.046), (-2.133, 0.053), (-2.236, 0.090)),
    (4, 1, 0): ((-1.017, 0.026), (-1.028, 0.031), (-0.984, 0.051)),
    (1, 2, 2): ((0.301, 0.025), (0.312, 0.030), (0.267, 0.050)),
    (3, 1, 1): ((2.624, 0.030), (2.628, 0.035), (2.614, 0.058)),
    (5, 0, 0): ((1.0898, 0.0080), (1.0929, 0.0094), (1.081, 0.015)),
}


def test_estimate_is_sample_mean_and_error():
    rng = np.random.default_rng(3)
    w = rng.standard_t(5, size=4001) * 3.0 + 0.7
    N, S1, S2 = mc.sums(list(w))
    for mult in (1, 2):
        v, s = mc.estimate(N, S1, S2, mult)
        assert abs(v - mult * np.mean(w)) < 1e-12 * mult * np.abs(w).max()
        assert abs(s - mult * np.std(w, ddof=1) / math.sqrt(N)) < 1e-10 * s


def test_combine_reproduces_eq2():
    v, s = mc.combine([(6.739, 0.132), (6.905, 0.220)])
    assert abs(v - 6.782) < 0.0015 and abs(s - 0.113) < 0.0006


def _half_unit(x):
    txt = repr(x)
    return 0.5 * 10.0 ** -(len(txt.split(".")[1]) if "." in txt else 0)


@pytest.mark.parametrize("cls", sorted(TABLE1))
def test_combine_reproduces_table1_rows(cls):
    """The printed value and sigma lie in the range the combination takes over
    the rounding box of the printed Calc 1 / Calc 2 inputs (each value and
    sigma within half a unit of its last printed digit), widened by half a
    unit of the printed output."""
    (val, sig), c1, c2 = TABLE1[cls]
    grid = []
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                for d in (-1, 0, 1):
                    r1 = (c1[0] + a * _half_unit(c1[0]), c1[1] + b * _half_unit(c1[1]))
                    r2 = (c2[0] + c * _half_unit(c2[0]), c2[1] + d * _half_unit(c2[1]))
                    grid.append(mc.combine([r1, r2]))
    vs = [v for v, _ in grid]
    ss = [e for _, e in grid]
    assert min(vs) - _half_unit(val) <= val <= max(vs) + _half_unit(val), (cls, min(vs), max(vs), val)
    assert min(ss) - _half_unit(sig) <= sig <= max(ss) + _half_unit(sig), (cls, min(ss), max(ss), sig)


@pytest.mark.parametrize("calc", [1, 2])
def test_set_total_adds_table1_classes_to_calc_totals(calc):
    """Table 1's nine class rows of one calculation add up to that calculation's
    total (section "Preliminary numerical results": Calc 1 6.739(132), Calc 2
    6.905(220)): mc.set_total's value lies within the summed half-units of the
    printed rows (plus half a unit of the printed total) and its sigma within
    the range the rounding box of the printed sigmas allows."""
    total = {1: (6.739, 0.132), 2: (6.905, 0.220)}[calc]
    rows = [TABLE1[c][calc] for c in sorted(TABLE1)]
    v, s = mc.set_total(rows)
    assert abs(v - total[0]) <= sum(_half_unit(a) for a, _ in rows) + _half_unit(total[0])
    lo = mc.set_total([(a, e - _half_unit(e)) for a, e in rows])[1]
    hi = mc.set_total([(a, e + _half_unit(e)) for a, e in rows])[1]
    h = _half_unit(total[1])
    assert lo - h <= total[1] <= hi + h and lo <= s <= hi
