"""GPU parity of the 3n-2-variable form (paper, section "The method",
footnote on 3n-1 -> 3n-2): the merged sampler against the oracle's (sector,
z of all lines with the merged pair split evenly, log p of the merged density
minus ln s), the merged weights against the oracle's merged integrand, and
the merged integrals at 1 and 2 loops against 0.5 and the closed form."""
import math

import numpy as np
import pytest

import paper_1905_08007_amd as P
from oracle import graphs as GR, integrand as IN, pdf as PD
from oracle.philox import uniforms

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _merged_set(n):
    gs = P.enumerate_graphs(n)
    s = P.build_forests(gs)
    q = P.pdf_create(s).merged()
    return gs, s, q, P.upload(s, q)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_merged_sampler_and_weights(n):
    gs, s, q, img = _merged_set(n)
    M, Mm = 3 * n, 3 * n - 1
    seed, tag, first, count = 21, 0, 5, 6
    for gi, g in enumerate(GR.enumerate_graphs(n)[:8]):
        z, lp, sec = P.sample_pdf(img, gi, seed, tag, first, count, want_sector=True)
        f, _, _ = P.eval_integrand(img, gi, z, P.QA_DD)
        torch.cuda.synchronize()
        z, lp, sec, f = z.cpu().numpy(), lp.cpu().numpy(), sec.cpu().numpy(), f.cpu().numpy()
        Dm, Wm = q.tables(gi)
        fm = IN.MergedIntegrand(g)
        a, b = PD.merged_lines(g)
        for i in range(count):
            zm, lpm, order = PD.sample_merged(g, Dm, Wm, uniforms(seed, tag, gi, first + i, 2 * (Mm - 1)))
            assert list(sec[:Mm, i]) == order and sec[M - 1, i] == 255
            zo = PD.expand_point(g, zm)
            assert np.max(np.abs(z[:, i] - zo) / zo) < 1e-12
            lpo = lpm - math.log(zm[a])
            assert abs(lp[i] - lpo) < 1e-11 * max(1.0, abs(lpo))
            # merged weight: f exp(-log p) = s f(s/2, s/2) / p_merged, the oracle
            # at 60 digits (near a boundary one forest term alone can lose 10
            # digits to cancellation inside its polynomials in long double)
            IN.set_precision("mp", 60)
            try:
                wo = float(fm(zm)) * math.exp(-lpm)
            finally:
                IN.set_precision("ld")
            assert abs(f[i] * math.exp(-lp[i]) - wo) <= 1e-9 * abs(wo) + 1e-300


def test_merged_integrals():
    gs, s, q, img = _merged_set(1)
    per, tot = P.acc_read(s, P.integrate(s, img, [4_000_000], seed=1, tag=0))
    assert abs(tot["value"] - 0.5) < 3 * tot["sigma"] and tot["sigma"] < 1e-3
    gs, s, q, img = _merged_set(2)
    per, tot = P.acc_read(s, P.integrate(s, img, [8_000_000] * 4, seed=2, tag=0))
    exact = 197 / 144 + math.pi ** 2 / 12 - math.pi ** 2 / 2 * math.log(2) + 0.75 * 1.2020569031595942 \
        - (119 / 36 - math.pi ** 2 / 3)
    assert abs(tot["value"] - exact) < 3 * tot["sigma"], (tot["value"], tot["sigma"])
