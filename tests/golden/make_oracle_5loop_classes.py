"""Write tests/golden/oracle_5loop_classes.json: four graphs of each of the
eight 5-loop gauge-invariant classes other than (5,0,0) (Table 1; indices
0, N/3, 2N/3 and N-1 of the class in enumeration order), taken together as
one graph set in class order, and the oracle's first Philox points of that
set's stream (seed 5, tag 0, samples 0..2): z, log p, sector, f and w = f / p.

Calls only ``oracle/``.  f is evaluated at 60 significant digits at every
point: long double is not enough where the graph polynomials themselves are
ill-conditioned (near a sector boundary one point lost ten digits in long
double with its forest terms cancelling only by 10^5), and the stored f must
carry a relative error far below the 1e-10 parity bar.
Usage: python tests/golden/make_oracle_5loop_classes.py
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

SEED, TAG, SAMPLES = 5, 0, range(3)
CLASSES = [(1, 4, 0), (2, 3, 0), (1, 3, 1), (3, 2, 0), (2, 2, 1), (4, 1, 0), (1, 2, 2), (3, 1, 1)]


def picks():
    """(class, index in the class) of every graph of the set, in set order."""
    out = []
    for c in CLASSES:
        n = len(GR.enumerate_graphs(5, c))
        for i in sorted({0, n // 3, 2 * n // 3, n - 1}):
            out.append((c, i))
    return out


def work(arg):
    gi, (c, ci) = arg
    g = GR.enumerate_graphs(5, c)[ci]
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
    return gi, {"class": list(c), "index": ci, "x": g["x"], "mate": g["mate"], "mult": g["mult"],
                "nterms": len(f.terms), "philox": out, "seconds": time.time() - t0}


def main():
    jobs = list(enumerate(picks()))
    with Pool(int(os.environ.get("ORACLE_PROCS", "8"))) as p:
        res = dict(p.imap_unordered(work, jobs, chunksize=1))
    out = {"seed": SEED, "tag": TAG, "graphs": [res[k] for k in sorted(res)]}
    with open(os.path.join(ROOT, "tests", "golden", "oracle_5loop_classes.json"), "w") as fh:
        json.dump(out, fh)
    print([(tuple(v["class"]), v["index"], v["nterms"], round(v["seconds"], 1),
            sum(p["prec"] == "mp60" for p in v["philox"])) for v in out["graphs"]])


if __name__ == "__main__":
    main()
