"""Throughput of the 5-loop subtracted-integrand Monte Carlo hot path on one GPU.

Workload: the 73 representatives of the gauge-invariant class (5,0,0) of
5-loop vertex graphs without lepton loops (Table 1), batched form: one
persistent fused launch per round (Philox -> sector PDF -> graph polynomials
-> forest-formula integrand in FP64 with a probabilistic round-off estimate ->
f/p -> compensated per-tile sums), the points whose round-off matters
recomputed in double-double, deterministic reduction; a round is replayed from
two captured hipGraphs.  A step is one pass over a batch of `--samples` points
split evenly over the 73 graphs (each step uses fresh sample indices of the
same Philox stream).  Tile and grid are autotuned before the timed steps.

Prints one JSON line: metric, value (evals/s), ms_per_step, the roofline of
the fused kernel (FP64 flops of the integrand / its HIP-event time, against
the FP64 vector peak; traffic from the committed counter record while the
kernel is unchanged), the oracle timed on one host core, and the plain
per-graph FP64 path timed on the same GPU.
"""
import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
METRIC = "5-loop subtracted integrand evals/s on 1 GPU; MC σ reached per GPU-hour"
SEED = 5


def oracle_baseline(q, seconds):
    """CPU baseline: the oracle (test infrastructure) on one host core, for one
    graph of class (5,0,0): sector sampling + subtracted integrand + f/p, after
    its one-time table setup (reported separately)."""
    try:
        from oracle import graphs as GR, mc
        g = GR.enumerate_graphs(5, (5, 0, 0))[1]
        t0 = time.time()
        mc.graph_samples(g, 1, SEED, 0, 1, tag=2)        # builds the oracle's monomial tables
        setup = time.time() - t0
        n = 0
        t0 = time.time()
        while time.time() - t0 < seconds:
            mc.graph_samples(g, 1, SEED, 1 + n, 4, tag=2)
            n += 4
        dt = time.time() - t0
        q.put({"value": n / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
               "sample": f"{n} points of graph 1 of class (5,0,0) (x={g['x']}), sampling + f + f/p, "
                         f"{dt:.1f} s on one core after {setup:.1f} s one-time setup"})
    except Exception as e:  # noqa: BLE001
        q.put({"error": repr(e)})


def measured_traffic(samples_per_launch):
    """HBM-side bytes of one fused launch, from the committed FETCH_SIZE / WRITE_SIZE
    passes (profiles/k_fused_traffic.json, scaled by a plain-copy calibration), or
    None when the kernel sources changed since those counters were taken."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "k_fused_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(root, src), "rb") as fh:
                h.update(fh.read())
    except (OSError, KeyError, ValueError):
        return None
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec["bytes_per_sample"] * samples_per_launch


def plain_path(P, img, graphs, per_graph, first):
    """The plain per-graph FP64 path on the same GPU, for comparison with the
    batched form: for each graph in turn qa_sample_pdf -> qa_eval_integrand
    (FP64) -> qa_accumulate, per_graph samples each (outside the timed region
    of the batched form).  Returns its evals/s and sigma per GPU-hour."""
    import torch
    ng = len(graphs)
    acc = P.new_acc(ng)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in range(ng):
        z, lp, _ = P.sample_pdf(img, g, SEED, 0, first, per_graph)
        f, _, _ = P.eval_integrand(img, g, z, P.QA_FP64)
        P.accumulate(f, lp, acc, g)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    a = P.read_acc(acc)
    var = 0.0
    for i, gr in enumerate(graphs):
        n = float(a["n"][i])
        m = (a["s1_hi"][i] + a["s1_lo"][i]) / n
        v = ((a["s2_hi"][i] + a["s2_lo"][i]) / n - m * m) / (n - 1)
        var += gr.mult ** 2 * v
    return {"evals_per_s": per_graph * ng / dt, "sigma_per_gpu_hour": math.sqrt(var) * math.sqrt(dt / 3600.0),
            "samples_per_graph": per_graph}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--samples", type=int, default=1 << 23, help="samples per step over the 73 graphs")
    ap.add_argument("--tile", type=int, default=0, help="0 with --grid 0: autotuned")
    ap.add_argument("--grid", type=int, default=0, help="persistent waves; 0 with --tile 0: autotuned")
    ap.add_argument("--threads", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-samples", type=int, default=1 << 16,
                    help="samples per graph of the plain per-graph FP64 comparison (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (got --gpus {args.gpus}); "
              "the hot path shards by graph / sample range without communication, see DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1905_08007_amd as P

    t0 = time.time()
    graphs = P.enumerate_graphs(5, 5, 0, 0)
    gset = P.build_forests(graphs, args.threads)
    pdf = P.pdf_create(gset)
    img = P.upload(gset, pdf, device="cuda:0")
    setup_s = time.time() - t0
    ng = len(graphs)
    per = args.samples // ng
    budgets = np.full(ng, per, dtype=np.uint64)
    flops = [gset.flops(i) for i in range(ng)]
    eval_flops_step = float(sum(per * a for a, _ in flops))
    all_flops_step = float(sum(per * (a + b) for a, b in flops))

    q = None
    proc = None
    if not args.no_cpu_baseline:
        ctx = mp.get_context("spawn")
        q = ctx.Queue()
        proc = ctx.Process(target=oracle_baseline, args=(q, args.cpu_seconds))
        proc.start()

    tuned_ns = None
    if args.tile == 0 and args.grid == 0:
        # pick tile and grid on a pilot share of the budgets (outside the timed region)
        args.tile, args.grid, tuned_ns = P.autotune(gset, img, budgets, SEED, 0, pilot=1 << 20)
    elif args.tile == 0:
        args.tile = 256
    work = torch.empty(P.work_bytes(gset, budgets, args.tile), dtype=torch.uint8, device="cuda:0")
    accs = []
    step = 0
    for _ in range(args.warmup):
        P.integrate(gset, img, budgets, SEED, 0, args.tile, args.grid, work=work, first=step * per)
        step += 1
    torch.cuda.synchronize()
    fused_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        acc, ms = P.integrate(gset, img, budgets, SEED, 0, args.tile, args.grid, work=work, first=step * per,
                              timing=True)
        accs.append(acc)
        fused_ms += ms
        step += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    # per-graph sums over the timed steps
    tot = np.zeros(ng, dtype=[("n", "f8"), ("s1", "f8"), ("s2", "f8"), ("flag", "f8"), ("bad", "f8"), ("res", "f8")])
    for acc in accs:
        a = P.read_acc(acc)
        tot["n"] += a["n"]
        tot["s1"] += a["s1_hi"] + a["s1_lo"]
        tot["s2"] += a["s2_hi"] + a["s2_lo"]
        tot["flag"] += a["n_flagged"]
        tot["bad"] += a["n_bad"]
        tot["res"] += a["n_residual"]
    val, var = 0.0, 0.0
    for i, g in enumerate(graphs):
        n = tot["n"][i]
        m = tot["s1"][i] / n
        v = (tot["s2"][i] / n - m * m) / (n - 1)
        val += g.mult * m
        var += g.mult ** 2 * v
    sigma = math.sqrt(var)
    samples = float(per * ng * args.steps)
    evals_s = samples / dt
    sigma_gpu_hour = sigma * math.sqrt(dt / 3600.0)
    achieved = eval_flops_step * args.steps / (fused_ms * 1e-3) / 1e12

    plain = None
    if args.plain_samples > 0:
        plain = plain_path(P, img, graphs, args.plain_samples, first=step * per)
        # Both paths sample the same distribution; the per-sample variance of these
        # heavy-tailed weights is far better estimated by the batched run's N, so the
        # comparison at equal per-sample sigma is sigma_hour * sqrt(rate ratio).
        plain["sigma_per_gpu_hour_at_batched_variance"] = sigma_gpu_hour * math.sqrt(evals_s / plain["evals_per_s"])

    cpu = None
    if proc is not None:
        proc.join(timeout=600)
        cpu = q.get() if not q.empty() else {"error": "oracle baseline did not report"}

    out = {
        "metric": METRIC,
        "value": evals_s,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "5-loop QED vertex graphs without lepton loops, class (5,0,0), 73 graphs; batched "
                        "persistent hipGraph launch (autotuned tile and grid), FP64 with a probabilistic round-off estimate "
                        "and double-double recompute",
            "samples_per_step": int(per * ng),
            "tile": args.tile,
            "grid": args.grid,
            "autotuned": tuned_ns is not None,
            "seed": SEED,
            "sigma_per_gpu_hour": sigma_gpu_hour,
            "plain_per_graph_fp64": plain,
            "class_value": val,
            "class_sigma": sigma,
            "flagged_fraction": float(tot["flag"].sum() / max(1.0, tot["n"].sum())),
            "bad_points": int(tot["bad"].sum()),
            "residual_points": int(tot["res"].sum()),
            "host_setup_s": setup_s,
            "fused_kernel_ms_per_step": fused_ms / args.steps,
            "eval_flops_per_sample": eval_flops_step / (per * ng),
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": measured_traffic(per * ng),
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
