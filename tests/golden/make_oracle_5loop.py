"""Write tests/golden/oracle_5loop.json: oracle values of f_G at seeded points
for graphs of the 5-loop class (5,0,0).

Calls only ``oracle/`` (and the shared point generator tests/inputs.py).
Interior points in long double, near-boundary points at 60 digits.
Usage: python tests/golden/make_oracle_5loop.py
"""
import json
import os
import sys
import time
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import graphs as GR, integrand as IN, mc  # noqa: E402
from tests import inputs  # noqa: E402

GRAPHS = [1, 40, 72]          # indices in the canonical class (5,0,0) list
N_IN, N_BD = 10, 3
SEED, TAG, SAMPLES = 5, 0, [0, 1, 2, 77777]   # Philox points of the benchmark stream


def work(gi):
    g = GR.enumerate_graphs(5, (5, 0, 0))[gi]
    f = IN.Integrand(g)
    zin = inputs.simplex_points(15, N_IN, 500 + gi)
    zbd = inputs.boundary_points(15, N_BD, 600 + gi, lam=1e-3)
    t0 = time.time()
    out = []
    for z in zin:
        v, terms = f(z, True)
        out.append({"z": [float(x) for x in z], "f": v, "terms_abs": sum(abs(t) for t in terms), "prec": "ld"})
    IN.set_precision("mp")
    for z in zbd:
        v, terms = f(z, True)
        out.append({"z": [float(x) for x in z], "f": v, "terms_abs": sum(abs(t) for t in terms), "prec": "mp60"})
    IN.set_precision("ld")
    smp = []
    for i in SAMPLES:
        (z, lp, fv, w, order), = mc.graph_samples(g, gi, SEED, i, 1, tag=TAG)
        smp.append({"sample": i, "z": [float(x) for x in z], "logp": lp, "f": fv, "w": w, "order": list(order)})
    return gi, {"x": g["x"], "mate": g["mate"], "nterms": len(f.terms), "points": out, "philox": smp,
                "seconds": time.time() - t0}


def main():
    with Pool(len(GRAPHS)) as p:
        res = dict(p.map(work, GRAPHS))
    out = {"class": [5, 0, 0], "seed": SEED, "tag": TAG, "graphs": {str(k): v for k, v in sorted(res.items())}}
    with open(os.path.join(ROOT, "tests", "golden", "oracle_5loop.json"), "w") as fh:
        json.dump(out, fh)
    print({k: (v["nterms"], round(v["seconds"], 1)) for k, v in res.items()})


if __name__ == "__main__":
    main()
