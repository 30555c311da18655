"""Write tests/golden/oracle_3loop_prefix.json: for every 3-loop graph, the
oracle's weights w = f / p at the first 256 Philox points of the 3-loop
configuration's stream (seed 3, tag 0), with their exactly rounded sums.

Calls only ``oracle/``.  f in long double; a point whose forest terms cancel
by more than 10^6 is re-evaluated at 60 digits.
Usage: python tests/golden/make_oracle_3loop_prefix.py
"""
import json
import math
import os
import sys
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import graphs as GR, integrand as IN, pdf as PD  # noqa: E402
from oracle.philox import uniforms  # noqa: E402

SEED, TAG, K = 3, 0, 256


def work(gi):
    g = GR.enumerate_graphs(3)[gi]
    D = PD.deg_table(g)
    W = PD.w_table(D, 9)
    f = IN.Integrand(g)
    ws, nmp = [], 0
    for i in range(K):
        z, lp, order = PD.sample(D, W, 9, uniforms(SEED, TAG, gi, i, 16))
        v, terms = f(z, True)
        if sum(abs(t) for t in terms) > 1e6 * abs(v):
            IN.set_precision("mp")
            try:
                v, terms = f(z, True)
            finally:
                IN.set_precision("ld")
            nmp += 1
        ws.append(v * math.exp(-lp))
    return gi, {"mult": g["mult"], "S1": math.fsum(ws), "S1abs": math.fsum(abs(x) for x in ws),
                "S2": math.fsum(x * x for x in ws), "w": ws, "n_mp": nmp}


def main():
    with Pool(int(os.environ.get("ORACLE_PROCS", "8"))) as p:
        res = dict(p.map(work, range(28), chunksize=1))
    out = {"loops": 3, "seed": SEED, "tag": TAG, "samples": K, "graphs": [res[i] for i in range(28)]}
    with open(os.path.join(ROOT, "tests", "golden", "oracle_3loop_prefix.json"), "w") as fh:
        json.dump(out, fh)
    print({i: res[i]["n_mp"] for i in range(28)})


if __name__ == "__main__":
    main()
