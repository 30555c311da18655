"""Write tests/golden/oracle_2loop.json: the oracle's 2-loop integrals.

Calls only ``oracle/``.  Stream: seed 2, tag 2 (the oracle's own check
stream), samples [0, N) of every representative graph, in 8 processes.
Usage: python tests/golden/make_oracle_2loop.py [N]
"""
import json
import os
import sys
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import graphs as GR, mc  # noqa: E402

SEED, TAG = 2, 2
CHUNK = 20000


def work(args):
    gi, first, count = args
    g = GR.enumerate_graphs(2)[gi]
    ws = [w for _, _, _, w, _ in mc.graph_samples(g, gi, SEED, first, count, tag=TAG)]
    return gi, first, ws


def main():
    N = int(sys.argv[1]) if len(sys.argv) > 1 else 960000
    gs = GR.enumerate_graphs(2)
    jobs = [(gi, s, min(CHUNK, N - s)) for gi in range(len(gs)) for s in range(0, N, CHUNK)]
    per = {gi: {} for gi in range(len(gs))}
    with Pool(8) as p:
        for gi, first, ws in p.imap_unordered(work, jobs):
            per[gi][first] = ws
    out = {"seed": SEED, "tag": TAG, "samples_per_graph": N, "graphs": []}
    vs = []
    for gi, g in enumerate(gs):
        ws = [w for first in sorted(per[gi]) for w in per[gi][first]]
        n, s1, s2 = mc.sums(ws)
        a, e = mc.estimate(n, s1, s2, g["mult"])
        vs.append((a, e))
        out["graphs"].append({"x": g["x"], "mate": g["mate"], "mult": g["mult"], "N": n,
                              "S1": s1, "S2": s2, "value": a, "sigma": e,
                              "prefix_S1_1000": mc.sums(ws[:1000])[1]})
    out["total"], out["sigma"] = mc.set_total(vs)
    with open(os.path.join(ROOT, "tests", "golden", "oracle_2loop.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(out["total"], out["sigma"])


if __name__ == "__main__":
    main()
