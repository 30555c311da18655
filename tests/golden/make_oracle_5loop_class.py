"""Write tests/golden/oracle_5loop_class.json: for every one of the 73 graphs
of the 5-loop class (5,0,0), the oracle's first Philox points of the
benchmark stream (seed 5, tag 0, samples 0..4): z, log p, sector, f and
w = f / p.

Calls only ``oracle/``.  f is evaluated at 60 significant digits at every
point: long double is not enough where the graph polynomials themselves are
ill-conditioned (near a sector boundary one point lost ten digits in long
double with its forest terms cancelling only by 10^5), and the stored f must
carry a relative error far below the 1e-10 parity bar.
Usage: python tests/golden/make_oracle_5loop_class.py
"""
import json
import math
import os
import sys
import time
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import graphs as GR, integrand as IN, pdf as PD  # noqa: E402
from oracle.philox import uniforms  # noqa: E402

SEED, TAG, SAMPLES = 5, 0, range(5)


def work(gi):
    g = GR.enumerate_graphs(5, (5, 0, 0))[gi]
    t0 = time.time()
    D = PD.deg_table(g)
    W = PD.w_table(D, 15)
    f = IN.Integrand(g)
    out = []
    for i in SAMPLES:
        z, lp, order = PD.sample(D, W, 15, uniforms(SEED, TAG, gi, i, 28))
        IN.set_precision("mp", 60)
        try:
            v, terms = f(z, True)
        finally:
            IN.set_precision("ld")
        tabs = sum(abs(t) for t in terms)
        prec = "mp60"
        out.append({"sample": i, "z": [float(x) for x in z], "logp": lp, "order": list(order), "f": v,
                    "terms_abs": tabs, "w": v * math.exp(-lp), "prec": prec})
    return gi, {"x": g["x"], "mate": g["mate"], "mult": g["mult"], "nterms": len(f.terms), "philox": out,
                "seconds": time.time() - t0}


def main():
    with Pool(int(os.environ.get("ORACLE_PROCS", "8"))) as p:
        res = dict(p.map(work, range(73), chunksize=1))
    out = {"class": [5, 0, 0], "seed": SEED, "tag": TAG, "graphs": {str(k): v for k, v in sorted(res.items())}}
    with open(os.path.join(ROOT, "tests", "golden", "oracle_5loop_class.json"), "w") as fh:
        json.dump(out, fh)
    print({k: (v["nterms"], round(v["seconds"], 1), sum(p["prec"] == "mp60" for p in v["philox"])) for k, v in res.items()})


if __name__ == "__main__":
    main()
