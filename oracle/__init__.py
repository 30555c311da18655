"""Oracle: a plain, slow CPU implementation of the per-sample hot path.

This package is TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code
with the HIP path (``paper_1905_08007_amd``): graphs, forests, Dirac traces,
graph polynomials, the Philox generator, the sector sampler and the Monte Carlo
accumulation are all written here independently, in float64 (or exact
rationals for Dirac traces), following the method of Volkov's 5-loop AMM
paper (section "The method", eq. (1), Table 1).

Modules:
  graphs    vertex graphs without lepton loops, classes (k,m,n), subgraphs, forests
  dirac     Dirac traces of gamma strings with contracted indices (Chisholm identities)
  integrand forest-formula subtracted Feynman-parametric AMM integrand f_G(z)
  philox    Philox4x32-10 counter-based generator (Salmon et al., SC'11)
  pdf       Hepp-sector PDF of eq. (1): Deg, W recursion, sampling, log p
  mc        per-graph value / variance accumulation and set combination
"""
