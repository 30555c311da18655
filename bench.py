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
the FP64 vector peak, dense and with the folds priced at their nonzero
coefficients; traffic and the counted FP64 rate from the committed counter
record while the kernel is unchanged), per-graph results with a tail check, the oracle timed on the
host's cores (after the GPU work), the plain per-graph FP64 path timed on
the same GPU, and, outside the timed region, the method's production
configuration (exponents tuned by three pilot steps, Neyman budgets) over as
many samples, for its sigma per GPU-hour.
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


def _oracle_worker(gi, seconds, q):
    """One host core: the oracle (test infrastructure) on graph gi of class
    (5,0,0): its one-time table setup, then sector sampling + subtracted
    integrand + f/p for `seconds`."""
    try:
        from oracle import graphs as GR, mc
        g = GR.enumerate_graphs(5, (5, 0, 0))[gi]
        t0 = time.time()
        mc.graph_samples(g, gi, SEED, 0, 1, tag=2)        # builds the oracle's monomial tables
        setup = time.time() - t0
        n = 0
        t0 = time.time()
        while time.time() - t0 < seconds:
            mc.graph_samples(g, gi, SEED, 1 + n, 1, tag=2)
            n += 1
        q.put((gi, n, time.time() - t0, setup))
    except Exception as e:  # noqa: BLE001
        q.put((gi, -1, repr(e), 0.0))


def oracle_baseline(seconds, cores):
    """CPU baseline: the oracle on `cores` host cores at once, one process per
    core, each on a different graph of class (5,0,0) spread evenly over the
    class (so the mix of term counts follows the class), each timed for
    `seconds` after its setup.  Rate = sum over cores of points / time."""
    ctx = mp.get_context("spawn")
    q = ctx.Queue()
    graphs = sorted({round(i * 72 / max(1, cores - 1)) for i in range(cores)})
    procs = [ctx.Process(target=_oracle_worker, args=(gi, seconds, q)) for gi in graphs]
    for pr in procs:
        pr.start()
    res = [q.get(timeout=900) for _ in procs]
    for pr in procs:
        pr.join(timeout=60)
    ok = [r for r in res if r[1] > 0]
    if not ok:
        return {"error": "oracle baseline failed: " + "; ".join(str(r[2]) for r in res)}
    rate = sum(n / dt for _, n, dt, _ in ok)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": rate, "unit": "evals/s", "cores": len(ok), "kind": "oracle",
            "sample": f"{sum(n for _, n, _, _ in ok)} points over {len(ok)} graphs of class (5,0,0) "
                      f"(indices {[gi for gi, *_ in ok]}), one process per core, about {seconds:.0f} s each after "
                      f"a one-time setup of {max(st for *_, st in ok):.0f} s; sampling + f + f/p in long double",
            "host_cores": os.cpu_count(), "cpu_model": model}


def note(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def committed_counters():
    """The committed counter record of one fused launch (profiles/k_fused_traffic.json:
    FETCH_SIZE / WRITE_SIZE scaled by a plain-copy calibration, and the FP64
    instruction counts), or None when the kernel sources changed since those
    counters were taken."""
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
    return rec


def tuned_neyman(P, gset, pdf, img, args, samples):
    """The production configuration of the method, outside the timed region:
    three pilot steps of the exponents (backward kernel, 2^20 samples per graph
    and step, key tag 1), frozen; Neyman budgets from a pilot of the frozen PDFs
    (2^20 per graph, tag 1); then one batched call over as many samples as the
    timed steps drew (tag 4), timed on its own.  Returns its class value, sigma
    and sigma per GPU-hour at that time, next to which the timed steps'
    uniform-budget figures stand (both from the same number of samples of
    heavy-tailed weights: long runs compare them better)."""
    import torch
    from paper_1905_08007_amd import pilot as PL
    ng = len(gset)
    t0 = time.perf_counter()
    _, img1, _ = PL.tune(gset, pdf, img, SEED, 1 << 20, args.tune_steps, 0.25)
    pil = P.read_acc(P.integrate(gset, img1, np.full(ng, 1 << 20, dtype=np.uint64), SEED, 1))
    budgets = P.allocate_budgets(gset, pil, int(samples), int(0.25 * samples / ng))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    acc = P.integrate(gset, img1, budgets, SEED, 4)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    per, tot = P.acc_read(gset, acc)
    return {"tune_steps": args.tune_steps, "setup_seconds": t1 - t0, "samples": int(tot["n"]),
            "seconds": dt, "class_value": float(tot["value"]), "class_sigma": float(tot["sigma"]),
            "sigma_per_gpu_hour": float(tot["sigma"]) * math.sqrt(dt / 3600.0),
            "budget_range": [int(budgets.min()), int(budgets.max())]}


def plain_path(P, gset, img, graphs, per_graph, first):
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
    per, tot = P.acc_read(gset, acc)
    return {"evals_per_s": per_graph * ng / dt, "sigma_per_gpu_hour": float(tot["sigma"]) * math.sqrt(dt / 3600.0),
            "samples_per_graph": per_graph,
            "per_graph_sigma_per_gpu_hour": [round(float(r["sigma"]) * math.sqrt(dt / 3600.0), 6) for r in per]}


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
    ap.add_argument("--cpu-cores", type=int, default=min(16, os.cpu_count() or 1),
                    help="host cores (processes) of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-steps", type=int, default=3,
                    help="pilot steps of the exponents for the tuned-PDF sigma comparison (0: skip it)")
    ap.add_argument("--plain-samples", type=int, default=1 << 16,
                    help="samples per graph of the plain per-graph FP64 comparison (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}): the hot path shards by graph set and "
              "sample range without communication, so run one process per GPU on its own share", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1905_08007_amd as P

    t0 = time.time()
    graphs = P.enumerate_graphs(5, 5, 0, 0)
    gset = P.build_forests(graphs, args.threads)
    pdf = P.pdf_create(gset)
    img = P.upload(gset, pdf, device="cuda:0")
    setup_s = time.time() - t0
    note(f"set-up {setup_s:.1f} s")
    ng = len(graphs)
    per = args.samples // ng
    budgets = np.full(ng, per, dtype=np.uint64)
    flops = [gset.flops(i) for i in range(ng)]
    eval_flops_step = float(sum(per * a for a, _ in flops))
    eval_flops_nz_step = float(sum(per * gset.flops_nonzero(i) for i in range(ng)))

    tuned_ns = None
    if args.tile == 0 and args.grid == 0:
        # pick tile and grid on a pilot share of the budgets (outside the timed region)
        args.tile, args.grid, tuned_ns = P.autotune(gset, img, budgets, SEED, 0, pilot=1 << 20)
        note(f"autotuned: tile {args.tile}, grid {args.grid}")
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
    note(f"{args.steps} timed steps: {dt:.2f} s")

    # per-graph results over the timed steps (the library merges the sums and
    # forms the estimates); tail check: each graph's per-sample sd after the
    # first step, a quarter of the steps and all of them, and the largest
    # share of its sum of w^2 that a single step holds (1/steps for light tails)
    merged = np.zeros(ng, dtype=P.ACC_DTYPE)
    marks = sorted({1, max(1, args.steps // 4), args.steps})
    sd_at, s2_steps = {}, []
    for k, acc in enumerate(accs, 1):
        a = P.read_acc(acc)
        s2_steps.append(a["s2_hi"] + a["s2_lo"])
        merged = P.acc_merge(merged, a)
        if k in marks:
            sd_at[k] = P.results(gset, merged)[0]["sd"]
    per_res, tot = P.results(gset, merged)
    s2_steps = np.array(s2_steps)
    step_share = s2_steps.max(axis=0) / np.maximum(s2_steps.sum(axis=0), 1e-300)
    val, sigma = float(tot["value"]), float(tot["sigma"])
    per_graph = [[int(r["n"]), round(float(r["mean"]), 6), round(float(r["sigma"]), 6)] +
                 [round(float(sd_at[k][i]), 2) for k in marks] + [round(float(step_share[i]), 3)]
                 for i, r in enumerate(per_res)]
    samples = float(per * ng * args.steps)
    evals_s = samples / dt
    sigma_gpu_hour = sigma * math.sqrt(dt / 3600.0)
    achieved = eval_flops_step * args.steps / (fused_ms * 1e-3) / 1e12
    counters = committed_counters()
    counted = None
    if counters is not None and "f64_flops_per_sample" in counters:
        counted = counters["f64_flops_per_sample"] * per * ng * args.steps / (fused_ms * 1e-3) / 1e12
    achieved_nz = eval_flops_nz_step * args.steps / (fused_ms * 1e-3) / 1e12

    plain = None
    if args.plain_samples > 0:
        plain = plain_path(P, gset, img, graphs, args.plain_samples, first=step * per)
        # Both paths sample the same distribution; the per-sample variance of these
        # heavy-tailed weights is far better estimated by the batched run's N, so the
        # comparison at equal per-sample sigma is sigma_hour * sqrt(rate ratio).
        plain["sigma_per_gpu_hour_at_batched_variance"] = sigma_gpu_hour * math.sqrt(evals_s / plain["evals_per_s"])
        note("plain path done")

    tuned = None
    if args.tune_steps > 0:
        tuned = tuned_neyman(P, gset, pdf, img, args, per * ng * args.steps)
        note("tuned exponents + Neyman budgets done")

    cpu = None
    if not args.no_cpu_baseline:   # after the GPU work: the oracle takes every host core it is given
        note(f"oracle on {args.cpu_cores} host cores ...")
        cpu = oracle_baseline(args.cpu_seconds, args.cpu_cores)

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
            "tuned_exponents_neyman_budgets": tuned,
            "class_value": val,
            "class_sigma": sigma,
            "flagged_fraction": float(tot["n_flagged"]) / max(1.0, float(tot["n"])),
            "bad_points": int(tot["n_bad"]),
            "residual_points": int(tot["n_residual"]),
            "host_setup_s": setup_s,
            "fused_kernel_ms_per_step": fused_ms / args.steps,
            "eval_flops_per_sample": eval_flops_step / (per * ng),
            "eval_flops_per_sample_nonzero": eval_flops_nz_step / (per * ng),
            "roofline_frac_nonzero": achieved_nz / FP64_PEAK_TFLOPS,
            "per_graph_fields": ["N", "mean w", "sigma (x mult)"] + [f"sd of w after {k} step(s)" for k in marks] +
                                ["largest one-step share of sum w^2"],
            "per_graph": per_graph,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": None if counters is None else counters["bytes_per_sample"] * per * ng,
            # FP64 arithmetic the kernel executes (rocprofv3 F64 instruction counts of the same launch,
            # FMA as 2: value and round-off-estimate folds, both geometry passes), over the same time
            "counted_achieved": counted,
            "counted_frac": None if counted is None else counted / FP64_PEAK_TFLOPS,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
