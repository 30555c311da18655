"""Write tests/golden/tables_sha256.json: SHA-256 digests of the oracle's
subgraph / forest / term lists and its Deg and W tables (eq. (1)) for every
graph at 1..4 loops and for the 73 graphs of the 5-loop class (5,0,0).

Calls only ``oracle/``.  The lists are hashed as the int32 sequence
  nsub, (lo, hi, kind 0=vertex 1=self-energy, has_x) * nsub,
  nforest, mask * nforest, nterm, (mask, apos) * nterm
per graph, concatenated over the set; the tables as little-endian float64
arrays of 2^(3n) entries, one digest per graph.
Usage: python tests/golden/make_tables_sha.py
"""
import hashlib
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import graphs as GR, integrand as IN, pdf as PD  # noqa: E402

SETS = {"1": (1, None), "2": (2, None), "3": (3, None), "4": (4, None), "5_500": (5, (5, 0, 0))}


def forest_words(g):
    subs = GR.subgraphs(g)
    v = [len(subs)]
    for x in subs:
        v += [x["lo"], x["hi"], 0 if x["kind"] == "V" else 1, int(x["has_x"])]
    fs = GR.forests(g)
    v += [len(fs)] + fs
    ts = IN.graph_terms(g)
    v += [len(ts)]
    for m, a in ts:
        v += [m, a]
    return v


def tables(args):
    n, cls, i = args
    g = GR.enumerate_graphs(n, cls)[i]
    D = PD.deg_table(g)
    W = PD.w_table(D, 3 * n)
    h = lambda a: hashlib.sha256(np.ascontiguousarray(a, dtype="<f8").tobytes()).hexdigest()
    return h(D), h(W)


def main():
    out = {}
    with Pool(int(os.environ.get("ORACLE_PROCS", "8"))) as pool:
        for name, (n, cls) in SETS.items():
            gs = GR.enumerate_graphs(n, cls)
            words = []
            for g in gs:
                words += forest_words(g)
            dw = pool.map(tables, [(n, cls, i) for i in range(len(gs))], chunksize=1)
            out[name] = {"loops": n, "class": cls, "ngraphs": len(gs),
                         "forests": hashlib.sha256(np.asarray(words, dtype="<i4").tobytes()).hexdigest(),
                         "deg": [a for a, _ in dw], "w": [b for _, b in dw]}
            print(name, len(gs), flush=True)
    with open(os.path.join(ROOT, "tests", "golden", "tables_sha256.json"), "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main()
