"""The full 5-loop set of vertex graphs without lepton loops, class by class.

Section "Preliminary numerical results", Table 1: the 3213 integrands split
into nine gauge-invariant classes (k, m, n) (k photons with ends on opposite
sides of the external photon, m on one side, n on the other); the class
contributions add up to the whole set's A_1^(10).

Each class is integrated as one or more graph sets of at most `max_graphs`
graphs (a set's host tables and device image stay a few GiB), each with a
pilot, Neyman budgets and a chunked production (pilot.production); a class
result is the sum of its sets' totals and the set total the sum of the classes
(qa_sum_results).  The streams are independent: set j of class number c draws
from the Philox key (seed, TAG_BASE + 2 (16 c + j)) in production and from the
next tag in its pilot.  Every number is computed by the library; this module
only sequences the calls.

Usage: python -m paper_1905_08007_amd.classes --seed 7 --samples-per-graph 1e6
"""
import argparse
import json
import sys
import time

import numpy as np

# Table 1's rows in the paper's order
CLASSES = ((1, 4, 0), (2, 3, 0), (1, 3, 1), (3, 2, 0), (2, 2, 1), (4, 1, 0), (1, 2, 2), (3, 1, 1), (5, 0, 0))
TAG_BASE = 64


def class_parts(cls, max_graphs=256):
    """The class's graphs (enumeration order) split into consecutive parts."""
    from . import enumerate_graphs
    gs = enumerate_graphs(5, *cls)
    return [gs[i:i + max_graphs] for i in range(0, len(gs), max_graphs)]


def integrate_class(cls, seed, samples_per_graph, pilot_per_graph=1 << 16, chunks=4, max_graphs=256,
                    device="cuda:0", log=None):
    """One class: (per-graph result records in enumeration order, class
    result record, GPU seconds of its integrate calls)."""
    import torch
    from . import RESULT_DTYPE, build_forests, pdf_create, sum_results, upload
    from .pilot import production
    ci = CLASSES.index(tuple(cls))
    per_graph, totals = [], []
    seconds = 0.0
    for j, part in enumerate(class_parts(cls, max_graphs)):
        t0 = time.time()
        if log:
            log(f"class {tuple(cls)} part {j + 1}: building {len(part)} graphs")
        s = build_forests(part)
        img = upload(s, pdf_create(s), device=device)
        t1 = time.time()
        tag = TAG_BASE + 2 * (16 * ci + j)
        per, tot, _ = production(s, img, seed, int(samples_per_graph) * len(part), pilot_per_graph,
                                 pilot_tag=tag + 1, tag=tag, chunks=chunks, log=log)
        torch.cuda.synchronize()
        seconds += time.time() - t1
        per_graph.append(per)
        totals.append(tot)
        if log:
            log(f"class {tuple(cls)} part {j + 1}: {len(part)} graphs, setup {t1 - t0:.1f} s, "
                f"{tot['value']:.5g} +- {tot['sigma']:.3g}")
        del img, s
    return np.concatenate(per_graph).astype(RESULT_DTYPE), sum_results(np.array(totals, dtype=RESULT_DTYPE)), seconds


def integrate_all(seed, samples_per_graph, classes=CLASSES, log=None, **kw):
    """Every class in `classes`: {class: (per-graph records, class record,
    seconds)} and the sum of the class records."""
    from . import RESULT_DTYPE, sum_results
    out = {}
    for cls in classes:
        out[tuple(cls)] = integrate_class(cls, seed, samples_per_graph, log=log, **kw)
    total = sum_results(np.array([v[1] for v in out.values()], dtype=RESULT_DTYPE))
    return out, total


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--samples-per-graph", type=float, default=1e6)
    ap.add_argument("--pilot-per-graph", type=int, default=1 << 16)
    ap.add_argument("--chunks", type=int, default=4)
    ap.add_argument("--max-graphs", type=int, default=256)
    ap.add_argument("--classes", default="all", help="all, or e.g. 1,4,0;5,0,0")
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)
    classes = CLASSES if a.classes == "all" else [tuple(int(x) for x in c.split(",")) for c in a.classes.split(";")]

    def log(msg):
        print(msg, flush=True)

    res, total = integrate_all(a.seed, a.samples_per_graph, classes, log=log, pilot_per_graph=a.pilot_per_graph,
                               chunks=a.chunks, max_graphs=a.max_graphs)
    rec = {"seed": a.seed, "samples_per_graph": a.samples_per_graph, "classes": {}}
    for cls, (per, tot, sec) in res.items():
        vals = per["value"]
        rec["classes"][str(cls)] = {"value": float(tot["value"]), "sigma": float(tot["sigma"]), "n": int(tot["n"]),
                                    "graphs": len(per), "sum_abs": float(np.abs(vals).sum()),
                                    "max_abs": float(np.abs(vals).max()), "gpu_seconds": sec,
                                    "n_flagged": int(tot["n_flagged"]), "n_residual": int(tot["n_residual"]),
                                    "n_bad": int(tot["n_bad"]),
                                    "per_graph": [[float(r["value"]), float(r["sigma"])] for r in per]}
        log(f"{cls}: {tot['value']:.5f} +- {tot['sigma']:.5f}  sum|a| {np.abs(vals).sum():.1f}  "
            f"max|a| {np.abs(vals).max():.2f}  {sec:.0f} s")
    rec["total"] = {"value": float(total["value"]), "sigma": float(total["sigma"]), "n": int(total["n"])}
    log(f"total: {total['value']:.5f} +- {total['sigma']:.5f} over {int(total['n'])} samples")
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(rec, fh)
    return 0


if __name__ == "__main__":
    sys.exit(main())
