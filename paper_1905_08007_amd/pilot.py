"""Pilot-then-production flow of the differentiation form: the variance
gradient of every graph's estimator with respect to its Deg exponents
(qa_variance_gradient, backward kernel), a few exponent steps
(qa_pdf_tune), then the exponents frozen and per-graph budgets allocated from
a pilot of the frozen PDFs (qa_allocate_budgets) for a nonadaptive production
run (qa_integrate).  Every number is computed by the library; this module
only sequences the calls."""
import numpy as np


def tune(gset, pdf, img, seed, samples, steps, step_size, floor=0.5, tag=1, device="cuda:0", log=None):
    """`steps` pilot steps over every graph of the set.  A step draws fresh
    samples (tag `tag`, sample range advancing by `samples` per step) from the
    current PDFs, forms each graph's gradient d E[w^2] / d Deg and moves its
    exponents by one step of at most `step_size` per set size.  Returns
    (pdf, img, history) with history[k] = per-graph E[w^2] measured at step k
    (before that step's move)."""
    from . import upload, variance_gradient
    hist = []
    first = 0
    for k in range(steps):
        m2s = []
        new = pdf
        for g in range(len(gset)):
            m2, grad = variance_gradient(pdf, img, g, seed, tag, first, samples)
            m2s.append(m2)
            new, _ = new.tune(g, grad, step_size, floor)
        hist.append(np.array(m2s))
        if log:
            log(f"pilot step {k + 1}/{steps}: sum of per-graph E[w^2] = {np.sum(m2s):.6g}")
        pdf = new
        img = upload(gset, pdf, device=device)
        first += samples
    return pdf, img, hist


def production(gset, img, seed, total, pilot_per_graph, floor_frac=0.25, pilot_tag=1, tag=0, work=None, chunks=1,
               log=None):
    """Frozen PDFs: a pilot of `pilot_per_graph` samples per graph (tag
    `pilot_tag`), Neyman budgets summing to `total` (each graph at least
    floor_frac * total / graphs), then the production integral (tag `tag`)
    in `chunks` calls whose sums the library merges.  Chunk c draws sample
    indices [c B, c B + its share) of every graph's stream, B the largest
    share, so the chunks never reuse a sample.  Returns (per-graph results,
    set total, budgets)."""
    from . import acc_merge, allocate_budgets, integrate, read_acc, results, ACC_DTYPE
    ng = len(gset)
    pilot = read_acc(integrate(gset, img, np.full(ng, pilot_per_graph, dtype=np.uint64), seed, pilot_tag, work=work))
    budgets = allocate_budgets(gset, pilot, int(total), int(floor_frac * total / ng))
    merged = np.zeros(ng, dtype=ACC_DTYPE)
    done = np.zeros(ng, dtype=np.uint64)
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
