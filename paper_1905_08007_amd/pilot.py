"""Pilot-then-production flow of the differentiation form: the variance
gradient of every graph's estimator with respect to its Deg exponents
(qa_variance_gradient, backward kernel), a few exponent steps
(qa_pdf_tune), then the exponents frozen and per-graph budgets allocated from
a pilot of the frozen PDFs (qa_allocate_budgets) for a nonadaptive production
run (qa_integrate).  Every number is computed by the library; this module
only sequences the calls."""
import numpy as np


def tune(gset, pdf, img, seed, samples, steps, step_size, floor=0.5, tag=1, device="cuda:0", log=None,
         guard=False, guard_tag=6):
    """`steps` pilot steps over every graph of the set.  A step draws fresh
    samples (tag `tag`, sample range advancing by `samples` per step) from the
    current PDFs, forms each graph's gradient d E[w^2] / d Deg and moves its
    exponents by one step of at most `step_size` per set size.  With guard,
    each graph's move is kept only if E[w^2] = S2 / N measured on fresh samples
    (tag `guard_tag`, `samples` per graph, the batched form) is lower under the
    moved exponents than under the current ones.  Returns (pdf, img, history)
    with history[k] = per-graph E[w^2] measured at step k (before its move)."""
    from . import integrate, read_acc, upload, variance_gradient
    ng = len(gset)

    def second_moment(image, first):
        a = read_acc(integrate(gset, image, np.full(ng, samples, dtype=np.uint64), seed, guard_tag, first=first))
        n = (a["n"] + a["n_bad"]).astype(float)
        return (a["s2_hi"] + a["s2_lo"]) / np.maximum(n, 1.0)

    hist = []
    first = 0
    for k in range(steps):
        m2s = []
        new = pdf
        for g in range(ng):
            m2, grad = variance_gradient(pdf, img, g, seed, tag, first, samples)
            m2s.append(m2)
            new, _ = new.tune(g, grad, step_size, floor)
        hist.append(np.array(m2s))
        img_new = upload(gset, new, device=device)
        if guard:
            before, after = second_moment(img, first), second_moment(img_new, first)
            keep = after < before
            for g in np.nonzero(~keep)[0]:
                new = new.with_graph(int(g), pdf.tables(int(g))[0])
            if not keep.all():
                img_new = upload(gset, new, device=device)
            if log:
                log(f"pilot step {k + 1}/{steps}: moves kept for {int(keep.sum())} of {ng} graphs")
        if log:
            log(f"pilot step {k + 1}/{steps}: sum of per-graph E[w^2] = {np.sum(m2s):.6g}")
        pdf, img = new, img_new
        first += samples
    return pdf, img, hist


def chunk_size(budgets, max_samples):
    """The largest per-graph share B such that one call, which draws
    min(budget, B) samples of every graph, stays within max_samples."""
    b = np.asarray(budgets, dtype=np.int64)
    lo, hi = 1, max(1, int(b.max()))
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if int(np.minimum(b, mid).sum()) <= max_samples:
            lo = mid
        else:
            hi = mid - 1
    return lo


def production(gset, img, seed, total, pilot_per_graph, floor_frac=0.25, pilot_tag=1, tag=0, work=None, chunks=1,
               log=None, max_chunk_samples=0):
    """Frozen PDFs: a pilot of `pilot_per_graph` samples per graph (tag
    `pilot_tag`), Neyman budgets summing to `total` (each graph at least
    floor_frac * total / graphs), then the production integral (tag `tag`)
    in calls whose sums the library merges: `chunks` calls, or, with
    max_chunk_samples > 0, as many as keep every call within that many
    samples.  Call c draws sample indices [c B, c B + its share) of every
    graph's stream (B the largest share of one call), so the calls never
    reuse a sample.  Returns (per-graph results, set total, budgets)."""
    from . import acc_merge, allocate_budgets, integrate, read_acc, results, ACC_DTYPE
    ng = len(gset)
    pilot = read_acc(integrate(gset, img, np.full(ng, pilot_per_graph, dtype=np.uint64), seed, pilot_tag, work=work))
    budgets = allocate_budgets(gset, pilot, int(total), int(floor_frac * total / ng))
    merged = np.zeros(ng, dtype=ACC_DTYPE)
    done = np.zeros(ng, dtype=np.uint64)
    if max_chunk_samples > 0:
        B = chunk_size(budgets, int(max_chunk_samples))
        chunks = int(-(-int(budgets.max()) // B))
    else:
        B = int(-(-int(budgets.max()) // chunks))
    for c in range(chunks):
        part = np.minimum(budgets - done, np.uint64(B))
        merged = acc_merge(merged, read_acc(integrate(gset, img, part, seed, tag, work=work, first=c * B)))
        done += part
        if log:
            _, tot = results(gset, merged)
            log(f"production chunk {c + 1}/{chunks}: {tot['value']:.6g} +- {tot['sigma']:.3g} over {int(tot['n'])} samples")
    per, tot = results(gset, merged)
    return per, tot, budgets


def main(argv=None):
    """Pilot with the backward kernel -> exponent steps -> frozen production,
    for the default and the tuned exponents side by side, with an independent
    check of each PDF's per-sample spread (key tag 3).
    Usage: python -m paper_1905_08007_amd.pilot --loops 4 --seed 4 --steps 3
           python -m paper_1905_08007_amd.pilot --loops 5 --cls 5,0,0 --total 2e9"""
    import argparse
    import json
    import time
    import torch
    from . import acc_read, build_forests, enumerate_graphs, integrate, pdf_create, upload, work_bytes
    ap = argparse.ArgumentParser(description="pilot -> exponent steps -> frozen production")
    ap.add_argument("--loops", type=int, default=4)
    ap.add_argument("--cls", default="", help="gauge-invariant class k,m,n (5 loops), e.g. 5,0,0; default all graphs")
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--pilot-samples", type=int, default=1 << 20, help="per graph and step")
    ap.add_argument("--step-size", type=float, default=0.25)
    ap.add_argument("--check-samples", type=int, default=1 << 21, help="per graph, independent key")
    ap.add_argument("--total", type=float, default=1e10, help="production samples over the set")
    ap.add_argument("--chunks", type=int, default=8)
    ap.add_argument("--max-chunk-samples", type=float, default=0, help="> 0: calls of at most this many samples")
    ap.add_argument("--productions", default="tuned,default", help="which exponents get a production run")
    ap.add_argument("--guard", action="store_true", help="keep a graph's move only if fresh samples confirm it")
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    t0 = time.time()
    cls = tuple(int(x) for x in a.cls.split(",")) if a.cls else (-1, -1, -1)
    gs = enumerate_graphs(a.loops, *cls)
    s = build_forests(gs)
    p0 = pdf_create(s)
    img0 = upload(s, p0, device="cuda:0")
    ng = len(gs)
    mult = np.array([g.mult for g in gs], dtype=float)
    log(f"{a.loops} loops, {ng} graphs: set-up {time.time() - t0:.1f} s")
    work = torch.empty(work_bytes(s, np.full(ng, 1 << 25, dtype=np.uint64), 256), dtype=torch.uint8, device="cuda:0")

    def check(img, label):
        if a.check_samples <= 0:
            return None
        per, tot = acc_read(s, integrate(s, img, np.full(ng, a.check_samples, dtype=np.uint64), a.seed, 3, work=work))
        spread = float(np.sum(per["sd"] * mult))
        log(f"{label} exponents: independent check {tot['value']:.5g} +- {tot['sigma']:.4g}; "
            f"sum over graphs of mu * sd(w) = {spread:.4g}")
        return {"value": float(tot["value"]), "sigma": float(tot["sigma"]), "sum_mu_sd": spread}

    rec = {"loops": a.loops, "class": list(cls), "seed": a.seed, "check_default": check(img0, "default")}
    t1 = time.time()
    p1, img1, hist = tune(s, p0, img0, a.seed, a.pilot_samples, a.steps, a.step_size, log=log, guard=a.guard)
    rec["pilot_seconds"] = time.time() - t1
    rec["pilot_m2"] = [float(np.sum(h)) for h in hist]
    rec["check_tuned"] = check(img1, "tuned")
    for label, img in (("tuned", img1), ("default", img0)):
        if label not in a.productions.split(","):
            continue
        t2 = time.time()
        per, tot, _ = production(s, img, a.seed, a.total, 1 << 20, work=work, chunks=a.chunks, log=log,
                                 max_chunk_samples=int(a.max_chunk_samples))
        torch.cuda.synchronize()
        worst = int(np.argmax(per["sigma"]))
        rec[f"production_{label}"] = {"value": float(tot["value"]), "sigma": float(tot["sigma"]), "n": int(tot["n"]),
                                      "seconds": time.time() - t2, "largest_sigma_graph": worst,
                                      "largest_sigma": float(per["sigma"][worst])}
        log(f"production ({label} exponents, {a.total:.3g} samples): {tot['value']:.5f} +- {tot['sigma']:.5g}; "
            f"largest per-graph sigma {float(per['sigma'][worst]):.4g} (graph {worst}); {time.time() - t2:.0f} s")
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(rec, fh)
    return 0


if __name__ == "__main__":
    import sys
    sys.exit(main())
