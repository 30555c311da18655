/*
 * qedamm.h -- C ABI of the MI355X hot path for the per-graph Monte Carlo
 * integration of the IR/UV-subtracted Feynman-parametric integrand of QED
 * vertex graphs without lepton loops (S. Volkov, 5-loop electron AMM).
 *
 * Conventions for every entry point
 *   - returns QA_OK (0) or a negative QA_E* code; qa_last_error() gives a
 *     thread-local message.  No C++ exception crosses this boundary.
 *   - "host" pointers are ordinary CPU memory owned by the caller; "device"
 *     pointers are HIP device memory owned by the caller (the library never
 *     allocates device memory in these calls, except where stated).
 *   - stream arguments are hipStream_t passed as void* (NULL = null stream);
 *     kernels are enqueued asynchronously; launch errors are returned, errors
 *     inside kernels surface at the next synchronising call.
 *   - handles (qa_set*, qa_pdf*) are immutable after creation and may be
 *     shared between threads.
 *   - seeds: the Philox key is (seed, tag), two 32-bit words; every entry
 *     point that takes a seed rejects seed >= 2^32 with QA_EINVAL.
 */
#ifndef QEDAMM_H
#define QEDAMM_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { QA_OK = 0, QA_EINVAL = -1, QA_ECAP = -2, QA_EHIP = -3, QA_ENOTSUP = -4, QA_ENOMEM = -5 };
enum { QA_FP64 = 0, QA_FP64_BOUND = 1, QA_DD = 2, QA_FP64_EST = 3 };  /* eval_integrand modes */

/* A vertex graph without lepton loops at n loops: an open electron line with
 * slots 0..2n, the external photon at slot x, mate[s] = partner slot of the
 * internal photon at s (mate[x] = x).  mult = 1 if the graph equals its
 * reversal, else 2 (arrow reversal identified, footnote to Table 1).
 * cls = (k, m, n): photons crossing x, and max / min of the photons entirely
 * left / right of x (classes of Table 1).  Lines: electron line i joins slots
 * i and i+1 (i < 2n); photon line 2n+a is the a-th photon by lower end. */
typedef struct qa_graph {
    int32_t loops;
    int32_t x;
    int8_t mate[12];
    int32_t mult;
    int32_t cls[3];
} qa_graph;

/* Per-graph Monte Carlo sums: N samples, S1 = sum of w = f/p and S2 = sum of
 * w^2, each as an unevaluated double-double (hi + lo).  Device layout. */
typedef struct qa_acc {
    uint64_t n;
    double s1_hi, s1_lo;
    double s2_hi, s2_lo;
    uint64_t n_flagged;   /* points recomputed in double-double */
    uint64_t n_bad;       /* non-finite or underflowed points, excluded */
    uint64_t n_residual;  /* recomputed points whose double-double estimate still exceeds 1e-10 of the weight scale (kept, counted) */
} qa_acc;

/* Per-graph (or set) estimate formed from the sums (host).  Every drawn
 * sample counts: a non-finite or underflowed point (n_bad) enters as w = 0,
 * so N = n + n_bad.  value = mult * S1 / N; sigma = mult * sqrt((S2/N -
 * (S1/N)^2) / (N - 1)) (section "Preliminary numerical results": per-graph
 * Monte Carlo integrals with 1-sigma errors; A_1 of a set = sum over its
 * graphs, Table 1).  mean and sd: mean and per-sample standard deviation of
 * w itself (no multiplicity).  For a set total: value = sum of the graphs'
 * values, sigma = root of the sum of their squared sigmas, counts summed,
 * mean = value and sd = sigma * sqrt(n). */
typedef struct qa_result {
    double value, sigma;
    double mean, sd;
    uint64_t n;           /* samples (good + bad) */
    uint64_t n_bad, n_flagged, n_residual;
} qa_result;

typedef struct qa_set qa_set;   /* graphs + forests + integrand tables (host) */
typedef struct qa_pdf qa_pdf;   /* Deg and W tables of eq. (1) (host) */

const char* qa_last_error(void);

/* Enumerate the canonical representatives at `loops` (1..5) loops in their
 * canonical order (ascending (x, mate[0..2n]) key, each graph the smaller key
 * of itself and its reversal).  (k, m, n) filters the class; -1 = any; m and
 * n are unordered.  Writes at most cap records to out (host); *count receives
 * the total.  QA_ECAP if cap is too small (count still set).
 * Paper: "all 3213 integrands"; Table 1 N_diag; section "The method". */
int qa_enumerate_graphs(int loops, int k, int m, int n, qa_graph* out, size_t cap, size_t* count);

/* Build the UV-divergent 1PI subgraphs, the forests, the forest-formula terms
 * and the projected-numerator coefficient tables for ng graphs (host input,
 * copied).  Section "The method": point-wise subtraction by a forest-like
 * formula of linear operators on UV-divergent subdiagrams.  nthreads <= 0:
 * use all host cores for the table build.  *out receives a new handle. */
int qa_build_forests(const qa_graph* g, size_t ng, int nthreads, qa_set** out);
void qa_set_destroy(qa_set* s);

/* Canonical byte serialisation of the subgraph and forest lists of every
 * graph (for bit-exact comparison): per graph the int32 sequence
 *   nsub, (lo, hi, kind 0=vertex 1=self-energy, has_x) * nsub,
 *   nforest, mask * nforest, nterm, (mask, apos) * nterm.
 * QA_ECAP if cap is too small; *len receives the byte length. */
int qa_forests_serialize(const qa_set* s, void* buf, size_t cap, size_t* len);

/* Statistics of the coefficient tables: monomial blocks, coefficients, terms. */
int qa_set_stats(const qa_set* s, uint64_t* nterms, uint64_t* nblocks, uint64_t* ncoef);

/* Algorithmic FP64 operation count of one plain evaluation of graph i's
 * integrand (graph polynomials of every piece, every coefficient-table block
 * with its multilinear fold, forest-term combination) plus the sector
 * sampler; an FMA counts 2.  Used for the roofline of the integrand kernel. */
int qa_graph_flops(const qa_set* s, uint32_t graph, double* eval_flops, double* sample_flops);

/* The same count with the coefficient folds priced at their nonzero
 * coefficients only (2 per nonzero coefficient instead of the dense 2^r fold;
 * the rest unchanged): the work a fold restricted to the nonzero monomials
 * would do. */
int qa_graph_flops_nonzero(const qa_set* s, uint32_t graph, double* eval_flops);

/* Per-graph budgets from a pilot (host arrays; pilot = ng qa_acc records read
 * back from the device): N_g = floor + share of (total - ng*floor) in
 * proportion to mu_g sigma_g / sqrt(c_g) (sigma_g the pilot's per-sample
 * standard deviation of w, c_g the flops of one sample from qa_graph_flops),
 * the Neyman allocation that minimises the variance of the set total at a
 * fixed cost; remainders by largest fraction (ties: lower graph index), so
 * the budgets sum to total exactly.  All weights zero (or non-finite): equal
 * shares.  QA_EINVAL if total < ng*floor.  The paper sums per-graph Monte
 * Carlo integrals (Table 1) and does not state its budgets. */
int qa_allocate_budgets(const qa_set* s, const qa_acc* pilot, uint64_t total, uint64_t floor, uint64_t* out);

/* Results from accumulator records.  qa_results: host records (ng = the
 * set's graph count); per_graph (host, ng records, nullable) and total (host,
 * nullable) receive the estimates defined at qa_result.  qa_acc_read: the
 * same from device records, copied on `stream` (the call synchronises it).
 * QA_EINVAL if a graph has fewer than 2 samples. */
int qa_results(const qa_set* s, const qa_acc* host_acc, qa_result* per_graph, qa_result* total);
int qa_acc_read(const qa_set* s, const qa_acc* dev_acc, qa_result* per_graph, qa_result* total, void* stream);

/* into[i] += from[i] for n host records: sums added as double-double,
 * counts added (runs over disjoint sample ranges of the same streams). */
int qa_acc_merge(qa_acc* into, const qa_acc* from, size_t n);

/* Statistical combination of independent results of the same quantity
 * (different generator keys): inverse-variance weighting, value =
 * sum v_i / s_i^2 / sum 1 / s_i^2, sigma = (sum 1 / s_i^2)^-1/2; counts are
 * summed, mean = value, sd = 0.  Section "Preliminary numerical results":
 * the two calculations (two generators) are statistically combined into
 * eq. (2).  QA_EINVAL if any sigma is not positive and finite. */
int qa_combine(const qa_result* runs, size_t nruns, qa_result* out);

/* Sum of results of independent integrals (the nine gauge-invariant classes
 * of Table 1 into the total of all graphs without lepton loops, or any
 * disjoint graph sets): value = sum v_i, sigma = (sum s_i^2)^1/2, counts
 * summed, mean = value, sd = sigma * sqrt(n) (as for a set total).  Section
 * "Preliminary numerical results", Table 1: the class contributions add up to
 * the whole set.  QA_EINVAL if any value or sigma is not finite or a sigma is
 * negative. */
int qa_sum_results(const qa_result* parts, size_t nparts, qa_result* out);

/* Deg and W tables of eq. (1) for every graph of the set.  deg == NULL: the
 * default Deg rule (parametric UV degree of the I-closure, minimised over the
 * reduced graphs of all forests, floored at 1/2).  Otherwise deg holds, for
 * graph i, 2^(3 n) doubles at offset sum_{j<i} 2^(3 n_j) (entries 0 and full
 * ignored, all others must be > 0).  W(S) = Deg(S)^-1 sum_j W(S\j),
 * W(full) = sum_j W(full\j). */
int qa_pdf_create(const qa_set* s, const double* deg, qa_pdf** out);
void qa_pdf_destroy(qa_pdf* p);
/* The paper's 3n-2 variables (section "The method", footnote): at q = 0 the
 * two electron lines next to the external vertex, a = x-1 and b = x, carry
 * the same momentum and the integrand is linear in their split, so the
 * integral over the split is exact at the even split: with s = z_a + z_b,
 *   int f dz = int over the 3n-1 merged parameters of s f(.., s/2, s/2, ..).
 * qa_pdf_create_merged makes, from an unmerged base pdf, the PDF of eq. (1)
 * over the 3n-1 merged lines (merged line j is line j for j < b and line
 * j+1 for j >= b; line a stands for {a, b}) with Deg'(S') = Deg(S) for the
 * original set S of S'.  An image uploaded with a merged pdf samples the
 * merged lines: qa_sample_pdf then returns z of all 3n lines (a and b at
 * s/2 each), log p of the merged density minus ln s (so that f exp(-log p)
 * is the merged weight) and sector rows 0..3n-2 (row 3n-1 = 255);
 * qa_integrate, qa_variance_grad and qa_variance_gradient use the merged
 * form throughout (gradient over the 2^(3n-1) merged sets).  QA_EINVAL if
 * base is already merged. */
int qa_pdf_create_merged(const qa_set* s, const qa_pdf* base, qa_pdf** out);
/* Lines the pdf samples for graph i: 3n, or 3n-1 for a merged pdf (its
 * tables hold 2^lines doubles). */
int qa_pdf_lines(const qa_pdf* p, uint32_t graph, int* lines);

/* Copy graph i's Deg and W tables (2^lines doubles each, qa_pdf_lines; either may be NULL). */
int qa_pdf_tables(const qa_pdf* p, uint32_t graph, double* deg, double* w);
/* Gradient of ln W(full) with respect to Deg(S) for graph i (2^(3n) doubles). */
int qa_pdf_dlogw(const qa_pdf* p, uint32_t graph, double* out);

/* A copy of base in which graph `graph` takes the Deg table deg (host,
 * 2^(3n) doubles, entries 0 and full ignored, the others > 0 and finite);
 * its W table is rebuilt.  The other graphs keep base's tables. */
int qa_pdf_with(const qa_pdf* base, uint32_t graph, const double* deg, qa_pdf** out);

/* One pilot step on graph `graph`'s exponents (the differentiation form:
 * pilot gradients move the exponents, production stays nonadaptive with the
 * frozen result).  The exponents
 * move by one shift per set size: theta_c = -step * g_c / max_c |g_c| with
 * g_c = sum over |S| = c of grad[S] (grad: host, 2^(3n) doubles, the
 * gradient d E[w^2] / d Deg(S) from qa_variance_gradient), c = 1 .. 3n-1,
 * and Deg'(S) = max(floor, Deg(S) + theta_|S|).  theta (host, 3n doubles,
 * nullable) receives the applied shifts (theta[0] unused).  *out: a new pdf
 * (base unchanged).  QA_EINVAL if floor <= 0 or grad is not finite. */
int qa_pdf_tune(const qa_pdf* base, uint32_t graph, const double* grad, double step, double floor, qa_pdf** out,
                double* theta);

/* Size of the device image holding the set's tables and the pdf tables. */
int qa_device_bytes(const qa_set* s, const qa_pdf* p, size_t* bytes);
/* Copy the image into the caller's device buffer dev (>= qa_device_bytes). */
int qa_upload(const qa_set* s, const qa_pdf* p, void* dev, size_t bytes, void* stream);

/* Draw points of graph `graph` from its sector PDF, eq. (1): Philox4x32-10
 * with key (seed, tag) and counter (block, graph, sample lo, sample hi),
 * samples first .. first+count-1.  Outputs (device): z SoA [M][count]
 * (z[l*count + i]), logp[count] = ln p(z) w.r.t. d^(M-1)z, sector (nullable)
 * SoA [M][count] bytes: j_1..j_M (z_{j1} >= ... >= z_{jM}). */
int qa_sample_pdf(const void* dev, uint32_t graph, uint64_t seed, uint32_t tag, uint64_t first,
                  uint64_t count, double* z, double* logp, uint8_t* sector, void* stream);

/* Evaluate f_G(z) for count points (device, SoA [M][count], any positive
 * scale: f is homogeneous of degree -M and is evaluated at z / sum z).
 * mode QA_FP64: f only.  QA_FP64_BOUND: also err[i] = rigorous running error
 * bound (the same evaluation on magnitudes) and flag[i] = 1 if err > 1e-11 |f|.
 * QA_FP64_EST: err[i] = probabilistic estimate of the rounding error (first-
 * order propagation of independent roundings, from the sums of squares of
 * the monomials, times a safety factor 10) and flag[i] = 1 if err > 1e-11 |f|;
 * this is the estimate the batched form flags with.  QA_DD: double-double
 * evaluation, err = its rigorous bound (when err is non-NULL an FP64
 * magnitude pass runs first to form it).  All include the conditioning of the
 * graph polynomials (computed in double-double in every mode).  err and flag
 * may be NULL for QA_FP64.  Units: (alpha/pi)^n.  Precision control: the
 * paper removes the round-off of the numerical subtraction with interval
 * arithmetic of several precisions (section "Preliminary numerical
 * results"); here an FP64 bound or estimate and a double-double recompute. */
int qa_eval_integrand(const void* dev, uint32_t graph, const double* z, uint64_t count, int mode,
                      double* f, double* err, uint8_t* flag, void* stream);

/* acc (device, one record) += the samples w = f * exp(-logp) (device arrays
 * of count doubles) with compensated (double-double) sums; non-finite w are
 * counted in n_bad and skipped. */
int qa_accumulate(const double* f, const double* logp, uint64_t count, qa_acc* acc, void* stream);

/* Batched form: all graphs of the set with per-graph budgets (host array,
 * samples per graph; graph g uses samples first .. first+budgets[g]-1 of its
 * stream), fused sample + evaluate (FP64 with the QA_FP64_EST estimate e) +
 * accumulate in a persistent launch (waves pull tiles of `tile` samples from
 * a queue).  A point is recomputed in double-double when e / p exceeds
 * 1e-11 max(|w|, S_g), S_g the rms weight of graph g over the accurate
 * weights seen so far in the call (earlier rounds, and this round's points
 * with e <= 1e-11 |f|): the round-off of the accepted points stays below
 * 1e-11 of the weight scale.  A point's weight enters the sums once: FP64
 * when accepted, double-double when recomputed (a recomputed weight that is
 * not finite counts in n_bad, as w = 0).  acc.n_flagged counts the
 * recomputed points,
 * n_residual those whose double-double estimate still exceeds 1e-10 of that
 * scale.  Deterministic per-tile partials are reduced into acc (device, ng
 * records, overwritten).  The
 * work is split into rounds of at most 2^25 samples; one round is captured as
 * a hipGraph and replayed.  work (device) >= qa_work_bytes (same budgets and
 * tile; about 116 bytes per sample of a round plus 0.6 GB of per-wave
 * buffers).  tile = multiple of 64
 * (0 = 256); grid = persistent waves (0 = 16 per CU, max 4096; rounded up to
 * a multiple of 4: the fused pass runs workgroups of 4 waves).
 * fused_ms (host, nullable): receives the summed duration of the fused
 * kernel over all rounds, from HIP events on `stream`. */
int qa_work_bytes(const qa_set* s, const uint64_t* budgets, uint32_t tile, size_t* bytes);
int qa_integrate(const qa_set* s, const void* dev, const uint64_t* budgets, uint64_t first, uint64_t seed,
                 uint32_t tag, uint32_t tile, uint32_t grid, void* work, size_t work_bytes, qa_acc* acc,
                 double* fused_ms, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops or harnesses that forbid hipMalloc): the batched form of
 * qa_integrate with no work argument and no allocation of any kind.  Its work
 * memory is a library-owned device array of 384 MiB per GPU, reserved when
 * the library's code object is loaded on that GPU and held until the process
 * ends; its address is looked up once per GPU (hipGetSymbolAddress).  The
 * call enqueues only kernel launches on `stream` (budgets travel in kernel
 * arguments; counters and acc are cleared by kernels; no private stream,
 * hipGraph or event), so it may itself be captured into a graph.  Meaning,
 * inputs and outputs as qa_integrate (same points, sums and recompute rule;
 * no fused-kernel timing), except: rounds hold at most 2^19 samples, and grid
 * (0 = 16 waves per CU) is lowered to the largest multiple of 4 whose
 * per-wave buffers fit the array next to a round's records.  With one round
 * and the same tile and grid the sums are bit-identical to qa_integrate's.
 * QA_ECAP if not even 4 waves fit (a set of thousands of graphs).  Every call
 * on a GPU uses that GPU's one array, which keeps the last call's contents:
 * calls that overlap on one GPU (two streams or threads) race and must be
 * serialised by the caller. */
int qa_integrate_noalloc(const qa_set* s, const void* dev, const uint64_t* budgets, uint64_t first, uint64_t seed,
                         uint32_t tag, uint32_t tile, uint32_t grid, qa_acc* acc, void* stream);

/* Autotuner of the batched form: for each candidate tile (256, 512, 1024
 * samples; a fused workgroup of 256 lanes takes tile/256 samples per lane)
 * and grid (16, 12 and 8 persistent waves per CU), runs qa_integrate twice on
 * a pilot share of the budgets (about `pilot` samples in total, at least one
 * per graph with a nonzero budget; 0 = 2^20) and times the fused kernel.
 * Returns the fastest (tile, grid) and its time per sample in ns (nullable).
 * work / work_bytes as for qa_integrate (candidates that do not fit are
 * skipped; QA_ECAP if none fits); acc (device, ng records) is overwritten
 * with pilot sums.  The pilot draws samples 0.. of the same streams. */
int qa_autotune(const qa_set* s, const void* dev, const uint64_t* budgets, uint64_t seed, uint32_t tag,
                uint64_t pilot, void* work, size_t work_bytes, qa_acc* acc, uint32_t* tile,
                uint32_t* grid, double* ns_per_sample, void* stream);

/* Variance gradient (pilot runs): for graph `graph`, samples first..first+
 * count-1 of stream (seed, tag): grad (device, 2^M doubles, accumulated +=)
 * receives sum_i w_i^2 sum_l t_l [S_l = S]; w2sum (device, 1 double) += sum
 * w_i^2.  d Var / d Deg(S) = grad[S]/N + (w2sum/N) dlnW/dDeg(S). */
int qa_variance_grad(const void* dev, uint32_t graph, uint64_t seed, uint32_t tag, uint64_t first,
                     uint64_t count, double* grad, double* w2sum, void* stream);

/* The full pilot gradient of graph `graph`: runs qa_variance_grad on
 * samples first..first+count-1 into work (device, 2^(3n)+1 doubles, cleared
 * here), copies the sums back (synchronising `stream`) and forms
 *   grad[S] = d E_p[w^2] / d Deg(S) = (1/N) sum_i w_i^2 t_l(i) [S_l(i) = S]
 *             + E_p[w^2] d ln W(full) / d Deg(S)
 * (host, 2^(3n) doubles) and *m2 = E_p[w^2] (nullable), with p the pdf that
 * the image on dev was uploaded from: QA_EINVAL if p's Deg table of the
 * graph differs from the image's. */
int qa_variance_gradient(const qa_pdf* p, const void* dev, uint32_t graph, uint64_t seed, uint32_t tag, uint64_t first,
                         uint64_t count, double* work, double* grad, double* m2, void* stream);

/* Debug / test hook: exact Dirac trace of a symbol string (0 = on-shell
 * p-slash with p.p = 1; 0 < L < 32 = gamma contracted with the other L;
 * at most 60 symbols; QA_EINVAL otherwise). */
int qa_dirac_trace(const int32_t* sym, int len, double* out);

#ifdef __cplusplus
}
#endif
#endif
