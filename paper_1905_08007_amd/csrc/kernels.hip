// HIP kernels of the hot path (gfx950) and the C-ABI entry points that launch them.
#include <hip/hip_runtime.h>

#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/qedamm.h"
#include "eval.h"
#include "host.h"

std::shared_ptr<const std::vector<uint8_t>> qa_image(const qa_set* s, const qa_pdf* p);
int qa_fail(int code, const std::string& msg);
size_t qa_set_size(const qa_set* s);
const qa::GraphTables& qa_graph_tables(const qa_set* s, size_t i);

#define HIPCHK(x)                                                                  \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) return qa_fail(QA_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al. 2011) and the uniform double mapping

__device__ __forceinline__ uint4 philox(uint4 c, uint2 k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
        k.x += 0x9E3779B9u;
        k.y += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ double u01(uint32_t a, uint32_t b) {
    const uint64_t k = (uint64_t)(a >> 6) * 67108864ull + (b >> 6);
    return (double)(2 * k + 1) * 0x1p-53;
}

struct Stream {
    uint2 key;
    uint32_t graph;
    uint64_t sample;
    __device__ void pair(int blk, double& u0, double& u1) const {
        uint4 x = philox(make_uint4((uint32_t)blk, graph, (uint32_t)sample, (uint32_t)(sample >> 32)), key);
        u0 = u01(x.x, x.y);
        u1 = u01(x.z, x.w);
    }
};

// ---------------------------------------------------------------------------
// sector-tree sampling from eq. (1): choose j_1..j_M with P(j | S) =
// W(S\j) / sum_j' W(S\j'), then t_l ~ Exp(Deg(S_l)) and ln z_{j_l} = -sum t.
// Writes z (normalised) through zv, returns log p; order[l] = j_(l+1).
__device__ __forceinline__ bool sample_lines(const QA_RO double* D, const QA_RO double* W, int M, const Stream& st,
                             LV<double> zv, double& logp, uint8_t* order, double* tl) {
    const uint32_t full = (1u << M) - 1;
    uint32_t S = full;
    double u0 = 0.0, u1 = 0.0;
    int ublk = -1;
    auto uni = [&](int i) {
        if ((i >> 1) != ublk) { ublk = i >> 1; st.pair(ublk, u0, u1); }
        return (i & 1) ? u1 : u0;
    };
#pragma unroll
    for (int l = 0; l < QA_MAXM - 1; ++l) {
        if (l >= M - 1) break;
        double ws[QA_MAXM];
        double tot = 0.0;
#pragma unroll
        for (int j = 0; j < QA_MAXM; ++j) {
            ws[j] = 0.0;
            if (j < M && (S >> j & 1)) { ws[j] = W[S ^ (1u << j)]; tot += ws[j]; }
        }
        const double target = uni(l) * tot;
        double cum = 0.0;
        int pick = -1, last = 0;
#pragma unroll
        for (int j = 0; j < QA_MAXM; ++j) {
            if (j < M && (S >> j & 1)) {
                last = j;
                if (pick < 0) {
                    cum += ws[j];
                    if (target < cum) pick = j;
                }
            }
        }
        if (pick < 0) pick = last;
        order[l] = (uint8_t)pick;
        S ^= 1u << pick;
    }
    order[M - 1] = (uint8_t)__builtin_ctz(S);
    S = full ^ (1u << order[0]);
    double run = 0.0, degsum = 0.0, lzsum = 0.0;
    zv[order[0]] = 0.0;
#pragma unroll
    for (int l = 1; l < QA_MAXM; ++l) {
        if (l >= M) break;
        const double d = D[S];
        const double t = -log(uni(M - 1 + l - 1)) / d;
        tl[l] = t;
        run -= t;
        degsum += d * t;
        lzsum += run;
        zv[order[l]] = run;
        S ^= 1u << order[l];
    }
    double norm = 0.0;
    for (int i = 0; i < M; ++i) { const double e = exp(zv[i]); zv[i] = e; norm += e; }
    const double inv = 1.0 / norm;
    bool ok = true;
    for (int i = 0; i < M; ++i) { zv[i] *= inv; ok &= zv[i] > 0.0; }
    logp = -log(W[full]) - degsum - (lzsum - M * log(norm));
    return ok && isfinite(logp);
}

// A point of graph G: all M lines from eq. (1), or in the merged form (the
// paper's 3n-2 variables, mb >= 0) the M - 1 merged lines, whose merged
// parameter s is split evenly over its two lines a = mb - 1, b = mb (the
// integrand is linear in the split, so s f(s/2, s/2, ...) is the exact split
// integral); logp then carries -ln s, so that f exp(-logp) is the merged
// weight.  order and tl are over the sampled lines.
__device__ __forceinline__ bool sample_point(const QA_RO double* D, const QA_RO double* W, int M, int mb,
                                             const Stream& st, LV<double> zv, double& logp, uint8_t* order,
                                             double* tl) {
    if (mb < 0) return sample_lines(D, W, M, st, zv, logp, order, tl);
    bool ok = sample_lines(D, W, M - 1, st, zv, logp, order, tl);
    const double sm = zv[mb - 1];
#pragma unroll
    for (int i = QA_MAXM - 1; i > 0; --i)
        if (i > mb && i < M) zv[i] = zv[i - 1];
    zv[mb - 1] = 0.5 * sm;
    zv[mb] = 0.5 * sm;
    logp -= log(sm);
    return ok && isfinite(logp);
}

__device__ __forceinline__ const QA_RO DevGraph& dev_graph(const QA_RO uint8_t* img, uint32_t g) {
    const QA_RO DevHeader* h = reinterpret_cast<const QA_RO DevHeader*>(img);
    return reinterpret_cast<const QA_RO DevGraph*>(img + h->graphs_off)[g];
}

__global__ void __launch_bounds__(256) k_sample(const uint8_t* __restrict__ img_, uint32_t graph, uint2 key,
                                                uint64_t first, uint64_t count, double* __restrict__ z,
                                                double* __restrict__ logp, uint8_t* __restrict__ sector) {
    const QA_RO uint8_t* img = (const QA_RO uint8_t*)img_;
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const QA_RO DevGraph& G = dev_graph(img, graph);
    const QA_RO double* D = reinterpret_cast<const QA_RO double*>(img + G.deg_off);
    const QA_RO double* W = reinterpret_cast<const QA_RO double*>(img + G.w_off);
    Stream st{key, graph, first + i};
    uint8_t order[QA_MAXM];
    double tl[QA_MAXM];
    double lp;
    sample_point(D, W, G.M, G.mb, st, LV<double>{z + i, (int)count}, lp, order, tl);
    logp[i] = lp;
    const int Ms = G.mb >= 0 ? G.M - 1 : G.M;
    if (sector)
        for (int l = 0; l < G.M; ++l) sector[(uint64_t)l * count + i] = l < Ms ? order[l] : 0xff;
}

// ---------------------------------------------------------------------------
// evaluation kernels: one point per lane, per-lane scratch in LDS laid out
// [element][lane]: geometry variables (QA_NVAR of the geometry type) then the
// piece-result polynomials (npoly * QA_MAXN of the evaluation type).

template <class T> __device__ __forceinline__ void lane_views(char* lds, int npoly, VV<typename GeoOf<T>::type>& vars,
                                                             LV<T>& polys) {
    using S = typename GeoOf<T>::type;
    const int lane = threadIdx.x, nt = blockDim.x;
    S* vbase = reinterpret_cast<S*>(lds);
    T* pbase = reinterpret_cast<T*>(lds + sizeof(S) * QA_NVAR * nt);
    vars = vv(vbase + lane, nt);
    polys = LV<T>{pbase + lane, nt};
    (void)npoly;
}

template <class T> __host__ __device__ size_t lds_bytes_dev(int npoly, int nt) {
    using S = typename GeoOf<T>::type;
    return (sizeof(S) * QA_NVAR + sizeof(T) * QA_MAXN * npoly) * nt;
}
template <class T> size_t lds_bytes(int npoly, int nt) { return lds_bytes_dev<T>(npoly, nt); }

// Running error bounds.  The graph polynomials are computed in double-double;
// their relative error is <= 16 * cond * 2^-104 (cond: their conditioning from
// eval_point).  The coefficient tables are exact integers.  The FP64
// evaluation then differs from the exact value by at most
//   u * mag * (128 + 16 * cond * 2^-51),
// where mag is the same computation on magnitudes and 128 exceeds the number
// of roundings along any product / sum path; the double-double evaluation by
//   2^-104 * mag * (256 + 16 * cond) + u |f| (final rounding to double).
constexpr double QA_U = 0x1p-53;
__device__ __forceinline__ double bound_of(double mag, double cond) { return mag * QA_U * (128.0 + 16.0 * cond * 0x1p-51); }
__device__ __forceinline__ double bound_dd(double mag, double cond, double f) {
    return mag * 0x1p-104 * (256.0 + 16.0 * cond) + fabs(f) * QA_U;
}

// Flag estimates.  est_of: the ER estimate u sqrt(q) of the FP64 rounding
// error with a safety factor of 10 (the observed ratio of the actual error to
// u sqrt(q) stays below 2), plus the error of the double-double geometry
// (relative 16 cond 2^-104 per value, through up to 16 factors).  est_dd: the
// same scale for the double-double evaluation, plus its final rounding.
__device__ __forceinline__ double est_of(double q, double cond) { return QA_U * sqrt(q) * (10.0 + cond * 0x1p-43); }
__device__ __forceinline__ double est_dd(double q, double cond, double f) {
    return 0x1p-104 * sqrt(q) * (40.0 + 256.0 * cond) + QA_U * fabs(f);
}

__global__ void __launch_bounds__(64) k_eval_fp64(const uint8_t* __restrict__ img_, uint32_t graph,
                                                  const double* __restrict__ z, uint64_t count, double* __restrict__ f) {
    const QA_RO uint8_t* img = (const QA_RO uint8_t*)img_;
    extern __shared__ char lds[];
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const QA_RO DevGraph& G = dev_graph(img, graph);
    VV<double> vars;
    LV<double> polys;
    lane_views<double>(lds, G.npoly, vars, polys);
    double cond;
    f[i] = eval_point<double>(img, G, CLV<double>{z + i, (int)count}, vars, polys, cond);
}

__global__ void __launch_bounds__(64) k_eval_bound(const uint8_t* __restrict__ img_, uint32_t graph,
                                                   const double* __restrict__ z, uint64_t count, double* __restrict__ f,
                                                   double* __restrict__ err, uint8_t* __restrict__ flag) {
    const QA_RO uint8_t* img = (const QA_RO uint8_t*)img_;
    extern __shared__ char lds[];
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const QA_RO DevGraph& G = dev_graph(img, graph);
    VV<double> vars;
    LV<EB> polys;
    lane_views<EB>(lds, G.npoly, vars, polys);
    double cond;
    EB r = eval_point<EB>(img, G, CLV<double>{z + i, (int)count}, vars, polys, cond);
    const double e = bound_of(r.a, cond);
    f[i] = r.v;
    if (err) err[i] = e;
    if (flag) flag[i] = !(e <= 1e-11 * fabs(r.v));
}

__global__ void __launch_bounds__(64) k_eval_est(const uint8_t* __restrict__ img_, uint32_t graph,
                                                 const double* __restrict__ z, uint64_t count, double* __restrict__ f,
                                                 double* __restrict__ err, uint8_t* __restrict__ flag) {
    const QA_RO uint8_t* img = (const QA_RO uint8_t*)img_;
    extern __shared__ char lds[];
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const QA_RO DevGraph& G = dev_graph(img, graph);
    VV<double> vars;
    LV<ER> polys;
    lane_views<ER>(lds, G.npoly, vars, polys);
    double cond;
    ER r = eval_point<ER>(img, G, CLV<double>{z + i, (int)count}, vars, polys, cond);
    const double e = est_of(r.q, cond);
    f[i] = r.v;
    if (err) err[i] = e;
    if (flag) flag[i] = !(e <= 1e-11 * fabs(r.v));
}

__global__ void __launch_bounds__(64) k_eval_dd(const uint8_t* __restrict__ img_, uint32_t graph,
                                                const double* __restrict__ z, uint64_t count, double* __restrict__ f,
                                                double* __restrict__ err) {
    const QA_RO uint8_t* img = (const QA_RO uint8_t*)img_;
    extern __shared__ char lds[];
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const QA_RO DevGraph& G = dev_graph(img, graph);
    double cond = 1.0, cond_dd;
    double mag = 0.0;
    if (err) {   // magnitude pass for the bound
        VV<double> v1;
        LV<EB> p1;
        lane_views<EB>(lds, G.npoly, v1, p1);
        mag = eval_point<EB>(img, G, CLV<double>{z + i, (int)count}, v1, p1, cond).a;
    }
    VV<DD> vars;
    LV<DD> polys;
    lane_views<DD>(lds, G.npoly, vars, polys);
    DD r = eval_point<DD>(img, G, CLV<double>{z + i, (int)count}, vars, polys, cond_dd);
    f[i] = r.hi + r.lo;
    if (err) err[i] = bound_dd(mag, fmax(cond, cond_dd), r.hi + r.lo);
}

// ---------------------------------------------------------------------------
// compensated sums

__device__ __forceinline__ DD dd_add(DD a, DD b) { return a + b; }

__device__ DD wave_sum_dd(DD v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        DD o{__shfl_xor(v.hi, off), __shfl_xor(v.lo, off)};
        v = v + o;
    }
    return v;
}
__device__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

// single block, fixed order: deterministic for a given count
__global__ void __launch_bounds__(1024) k_accumulate(const double* __restrict__ f, const double* __restrict__ logp,
                                                     uint64_t count, qa_acc* acc) {
    __shared__ double sh[4][16];
    __shared__ uint64_t sn[2][16];
    DD s1{0, 0}, s2{0, 0};
    uint64_t n = 0, bad = 0;
    for (uint64_t i = threadIdx.x; i < count; i += blockDim.x) {
        const double w = f[i] * exp(-logp[i]);
        if (!isfinite(w)) { ++bad; continue; }
        s1 = s1 + dd(w);
        s2 = s2 + two_prod(w, w);
        ++n;
    }
    s1 = wave_sum_dd(s1);
    s2 = wave_sum_dd(s2);
    n = wave_sum_u64(n);
    bad = wave_sum_u64(bad);
    const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
    if (ln == 0) { sh[0][wv] = s1.hi; sh[1][wv] = s1.lo; sh[2][wv] = s2.hi; sh[3][wv] = s2.lo; sn[0][wv] = n; sn[1][wv] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        DD a1{acc->s1_hi, acc->s1_lo}, a2{acc->s2_hi, acc->s2_lo};
        uint64_t an = acc->n, ab = acc->n_bad;
        for (int w = 0; w < (int)(blockDim.x / 64); ++w) {
            a1 = a1 + DD{sh[0][w], sh[1][w]};
            a2 = a2 + DD{sh[2][w], sh[3][w]};
            an += sn[0][w];
            ab += sn[1][w];
        }
        acc->s1_hi = a1.hi; acc->s1_lo = a1.lo;
        acc->s2_hi = a2.hi; acc->s2_lo = a2.lo;
        acc->n = an;
        acc->n_bad = ab;
    }
}

// ---------------------------------------------------------------------------
// batched form: persistent waves over tiles (graph, sample range)

struct Partial {
    double s1_hi, s1_lo, s2_hi, s2_lo;   // over the points that passed the relative test, then (k_select)
                                         // plus the candidates kept in FP64
    double s2g;              // sum of w^2 over points that passed the relative test
    uint64_t n, nflag, nbad;
};
struct FlagEntry {
    uint64_t sample;
    double w;         // FP64 weight f / p
    double estw;      // FP64 error estimate of w
    double q, cond;   // ER variance and geometry conditioning of the FP64 pass
    double ip;        // 1 / p
    DD c1, c2;        // double-double pass: w and w^2 of the recomputed value
    uint32_t graph;
    uint8_t fixed;    // recomputed in double-double
    uint8_t residual; // double-double estimate still above 1e-10 of the scale
    uint8_t bad;      // double-double w or w^2 not finite: the point counts as w = 0 (n_bad)
    uint8_t pad;
};
static_assert(sizeof(DD) == sizeof(ER), "the DD pass reuses the piece-result buffer of the fused pass");
struct Work {
    uint32_t* counter;       // [0..7] tile queues (one per XCD), [8] round, [9] selected entries, [10] fix chunks,
                             // [11] slices, [12..13] Philox key (seed, tag), [14..15] first sample (lo, hi)
    uint64_t* gtile0;        // per graph: first global tile index (ng + 1 entries)
    uint64_t* budget;        // per graph samples
    Partial* partial;        // per round-tile
    uint32_t* nflag;         // per round-tile: candidate entries
    FlagEntry* flags;        // per round-tile * tile
    double* scale;           // per graph: rms of the accurate weights so far
    uint32_t* nsel;          // per round-tile: entries selected for double-double
    uint32_t* seloff;        // per round-tile: offset of its selected entries
    uint32_t* sel;           // selected entry indices (t * tile + e), tile order
    DD* fpart;               // double-double pass: partial f per (selected entry, slice)
    double* fcond;           // double-double pass: geometry conditioning per selected entry
    uint32_t grid;           // persistent waves of the double-double pass
    double* zbuf;            // per persistent wave: QA_MAXM * 64
    ER* pbuf;                // per persistent wave: piece results [QA_MAXPOLY * QA_MAXN][64] (ER, or DD in the DD pass)
    double* vbuf;            // per persistent wave of the fused pass: contraction matrix [QA_VAR_A][64]
    uint32_t tile, per_round, ng;
    uint64_t ntiles;
};

constexpr uint32_t kQueues = 8;   // one tile queue per XCD (L2 domain)
enum { kCRound = 8, kCSel = 9, kCFix = 10, kCSlices = 11, kCKey = 12, kCFirst = 14 };

// the call's Philox key and first sample index live in the work buffer, so
// that a captured round does not depend on them and is replayed across calls
__device__ __forceinline__ uint2 call_key(const Work& w) {
    return make_uint2(__builtin_amdgcn_readfirstlane(w.counter[kCKey]), __builtin_amdgcn_readfirstlane(w.counter[kCKey + 1]));
}
__device__ __forceinline__ uint64_t call_first(const Work& w) {
    return (uint64_t)__builtin_amdgcn_readfirstlane(w.counter[kCFirst]) |
           ((uint64_t)__builtin_amdgcn_readfirstlane(w.counter[kCFirst + 1]) << 32);
}

// first round-tile and number of tiles of the current round
__device__ __forceinline__ uint32_t round_len(const Work& w, uint64_t& t0) {
    t0 = (uint64_t)w.counter[kCRound] * w.per_round;
    const uint64_t left = w.ntiles - t0;
    return (uint32_t)(left < w.per_round ? left : w.per_round);
}

__device__ __forceinline__ void tile_of(const Work& w, uint64_t first, uint64_t gt, uint32_t& g, uint64_t& s0,
                                        uint32_t& cnt) {
    uint32_t lo = 0, hi = w.ng;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) / 2;
        if (w.gtile0[mid] <= gt) lo = mid; else hi = mid;
    }
    g = lo;
    const uint64_t off = (gt - w.gtile0[lo]) * w.tile;
    const uint64_t rem = w.budget[lo] - off;
    cnt = (uint32_t)(rem < w.tile ? rem : w.tile);
    s0 = first + off;
}

// round-tile range [a, b) of graph g in the current round
__device__ __forceinline__ bool round_tiles(const Work& w, uint32_t g, uint64_t& a, uint64_t& b, uint64_t& t0) {
    const uint32_t nr = round_len(w, t0);
    const uint64_t t1 = t0 + nr;
    a = w.gtile0[g] > t0 ? w.gtile0[g] : t0;
    b = w.gtile0[g + 1] < t1 ? w.gtile0[g + 1] : t1;
    return a < b;
}

__global__ void k_reset(Work w) {
    if (blockIdx.x == 0 && threadIdx.x < kQueues) w.counter[threadIdx.x] = 0;
}
__global__ void k_next_round(Work w) {
    if (threadIdx.x == 0 && blockIdx.x == 0) w.counter[kCRound] += 1;
}

// Fused pass: sample, evaluate in FP64 with the ER estimate, accumulate w and
// w^2 per tile, and list the points whose estimate exceeds 1e-11 |f|
// (candidates for the double-double pass).  A workgroup of kFusedWaves waves
// (one per SIMD of a CU) takes a tile at a time, so that its waves walk the
// same coefficient tables together and share the CU's scalar cache.  LDS
// holds the flows A, C of the geometry (20 doubles per lane, read about twice
// as often as the contraction matrix); the contraction matrix and the piece
// results live in per-wave global buffers.  Four waves per SIMD.
constexpr int kFusedWaves = 4;
constexpr int kFusedThreads = 64 * kFusedWaves;
constexpr int kFusedOcc = 4;   // waves per SIMD the fused pass is compiled for
__global__ void __launch_bounds__(kFusedThreads, kFusedOcc) k_fused(const uint8_t* __restrict__ img_, Work w) {
    const QA_RO uint8_t* img = (const QA_RO uint8_t*)img_;
    const uint2 key = call_key(w);
    const uint64_t first = call_first(w);
    // LDS: the flows A, C of the workgroup's lanes, [20][256] doubles.  Between
    // evaluations (after a barrier) its first bytes carry the workgroup's
    // exchange: tile index, candidate counts, per-wave sums.
    extern __shared__ char lds[];
    uint32_t* sh_u = reinterpret_cast<uint32_t*>(lds);          // [0] tile, [1..4] counts
    double* sh_s = reinterpret_cast<double*>(lds) + 8;            // [4][5] sums
    uint64_t* sh_n = reinterpret_cast<uint64_t*>(lds) + 32;       // [4][2] counts
    const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
    const uint64_t gw = (uint64_t)blockIdx.x * kFusedWaves + wv;
    VV<double> vars{w.vbuf + gw * (QA_VAR_A * 64) + lane, 64, reinterpret_cast<double*>(lds) + tid, kFusedThreads};
    LV<ER> polys{w.pbuf + gw * (QA_MAXPOLY * QA_MAXN * 64) + lane, 64};
    double* zb = w.zbuf + gw * QA_MAXM * 64;
    uint64_t rt0;
    const uint32_t nr = round_len(w, rt0);
    // The round's tiles (graph-major) are split into kQueues contiguous ranges.
    // Workgroups are dispatched to the XCDs round-robin, so the workgroups of
    // one XCD share a range, and with it the coefficient tables in their L2; a
    // workgroup whose range is drained helps the following ones.
    const uint32_t x0 = blockIdx.x % kQueues;
    for (uint32_t k = 0; k < kQueues; ++k) {
      const uint32_t x = (x0 + k) % kQueues;
      const uint32_t qlo = (uint32_t)((uint64_t)nr * x / kQueues), qhi = (uint32_t)((uint64_t)nr * (x + 1) / kQueues);
      for (;;) {
        if (tid == 0) sh_u[0] = atomicAdd(w.counter + x, 1u);
        __syncthreads();
        uint32_t t = __builtin_amdgcn_readfirstlane(sh_u[0]);   // workgroup-uniform: scalar loads
        __syncthreads();
        if (t >= qhi - qlo) break;
        t += qlo;
        const uint64_t gt = rt0 + t;
        uint32_t g, cnt;
        uint64_t s0;
        tile_of(w, first, gt, g, s0, cnt);
        const QA_RO DevGraph& G = dev_graph(img, g);
        const QA_RO double* D = reinterpret_cast<const QA_RO double*>(img + G.deg_off);
        const QA_RO double* W = reinterpret_cast<const QA_RO double*>(img + G.w_off);
        DD s1{0, 0}, s2{0, 0};
        double s2g = 0.0;
        uint64_t n = 0, bad = 0;
        uint32_t nfl = 0;
        for (uint32_t base = 0; base < cnt; base += kFusedThreads) {
            const uint32_t j = base + tid;
            const bool act = j < cnt;
            double wv_ = 0.0, ew = 0.0, qv = 0.0, cnd = 1.0, ipv = 0.0;
            bool flagged = false, good = false;
            if (act) {
                Stream st{key, g, s0 + j};
                uint8_t order[QA_MAXM];
                double tl[QA_MAXM];
                double lp;
                LV<double> zv{zb + lane, 64};
                bool ok = sample_point(D, W, G.M, G.mb, st, zv, lp, order, tl);
                if (ok) {
                    double cond;
                    ER r = eval_point<ER>(img, G, CLV<double>{zb + lane, 64}, vars, polys, cond);
                    const double e = est_of(r.q, cond);
                    const double ip = exp(-lp);
                    qv = r.q;
                    cnd = cond;
                    wv_ = r.v * ip;
                    ew = e * ip;
                    ipv = ip;
                    good = isfinite(wv_);
                    flagged = good && !(e <= 1e-11 * fabs(r.v));
                }
            }
            if (act && good) {
                // a candidate enters the sums later, once: in FP64 if it is kept
                // (k_select), in double-double if it is recomputed (k_reduce);
                // its FP64 value may be off by many orders
                if (!flagged) {
                    s1 = s1 + dd(wv_);
                    s2 = s2 + two_prod(wv_, wv_);
                    s2g += wv_ * wv_;
                }
                ++n;
            } else if (act) {
                ++bad;
            }
            // candidate list: positions in wave order, then lane order
            const uint64_t mask = __ballot(flagged);
            __syncthreads();   // every wave is done with the variables
            if (lane == 0) sh_u[1 + wv] = (uint32_t)__popcll(mask);
            __syncthreads();
            uint32_t off = nfl, tot = 0;
            for (int v = 0; v < kFusedWaves; ++v) {
                if (v < wv) off += sh_u[1 + v];
                tot += sh_u[1 + v];
            }
            if (flagged) {
                const uint32_t pos = off + __popcll(mask & ((1ull << lane) - 1));
                FlagEntry& fe = w.flags[(uint64_t)t * w.tile + pos];
                fe.sample = s0 + j;
                fe.w = wv_;
                fe.estw = ew;
                fe.q = qv;
                fe.cond = cnd;
                fe.ip = ipv;
                fe.c1 = DD{0.0, 0.0};
                fe.c2 = DD{0.0, 0.0};
                fe.graph = g;
                fe.fixed = 0;
                fe.residual = 0;
                fe.bad = 0;
            }
            nfl += tot;
            __syncthreads();
        }
        s1 = wave_sum_dd(s1);
        s2 = wave_sum_dd(s2);
        s2g = wave_sum_f64(s2g);
        n = wave_sum_u64(n);
        bad = wave_sum_u64(bad);
        if (lane == 0) {
            double* q = sh_s + 5 * wv;
            q[0] = s1.hi; q[1] = s1.lo; q[2] = s2.hi; q[3] = s2.lo; q[4] = s2g;
            sh_n[2 * wv] = n; sh_n[2 * wv + 1] = bad;
        }
        __syncthreads();
        if (tid == 0) {
            // waves combined in a fixed order
            DD a1{0, 0}, a2{0, 0};
            double ag = 0.0;
            uint64_t an = 0, ab = 0;
            for (int v = 0; v < kFusedWaves; ++v) {
                const double* q = sh_s + 5 * v;
                a1 = a1 + DD{q[0], q[1]};
                a2 = a2 + DD{q[2], q[3]};
                ag += q[4];
                an += sh_n[2 * v];
                ab += sh_n[2 * v + 1];
            }
            Partial pr{};
            pr.s1_hi = a1.hi; pr.s1_lo = a1.lo; pr.s2_hi = a2.hi; pr.s2_lo = a2.lo;
            pr.s2g = ag;
            pr.n = an; pr.nflag = nfl; pr.nbad = ab;
            w.partial[t] = pr;
            w.nflag[t] = nfl;
        }
        __syncthreads();
      }
    }
}

// Per graph: the scale of its weights, sqrt(sum w^2 / N) over the accurate
// weights of earlier rounds and the points of this round that passed the
// relative test (a lower bound of the rms weight).
__global__ void __launch_bounds__(64) k_scale(Work w, const qa_acc* __restrict__ acc) {
    const uint32_t g = blockIdx.x, lane = threadIdx.x;
    uint64_t a, b, t0;
    if (g >= w.ng || !round_tiles(w, g, a, b, t0)) return;
    double s2 = 0.0;
    uint64_t n = 0;
    for (uint64_t gt = a + lane; gt < b; gt += 64) {
        s2 += w.partial[gt - t0].s2g;
        n += w.partial[gt - t0].n;
    }
    s2 = wave_sum_f64(s2);
    n = wave_sum_u64(n);
    if (lane == 0) {
        s2 += acc[g].s2_hi + acc[g].s2_lo;
        n += acc[g].n;
        w.scale[g] = n ? sqrt(s2 / (double)n) : 0.0;
    }
}

// A candidate is recomputed in double-double when its error estimate on w
// exceeds 1e-11 of max(|w|, scale of its graph).
__device__ __forceinline__ bool needs_dd(const FlagEntry& fe, const double* scale) {
    return !(fe.estw <= 1e-11 * fmax(fabs(fe.w), scale[fe.graph]));
}

__global__ void __launch_bounds__(64) k_select(Work w) {
    const int lane = threadIdx.x;
    uint64_t rt0;
    const uint32_t nr = round_len(w, rt0);
    for (uint32_t t = blockIdx.x; t < nr; t += gridDim.x) {
        const uint32_t nf = w.nflag[t];
        uint32_t cnt = 0;
        DD k1{0.0, 0.0}, k2{0.0, 0.0};
        for (uint32_t b = 0; b < nf; b += 64) {
            const uint32_t e = b + lane;
            bool need = false;
            if (e < nf) {
                FlagEntry& fe = w.flags[(uint64_t)t * w.tile + e];
                need = needs_dd(fe, w.scale);
                fe.fixed = need;
                if (!need) {
                    k1 = k1 + dd(fe.w);
                    k2 = k2 + two_prod(fe.w, fe.w);
                }
            }
            cnt += __popcll(__ballot(need));
        }
        if (nf) {
            k1 = wave_sum_dd(k1);
            k2 = wave_sum_dd(k2);
            if (lane == 0) {
                Partial& pr = w.partial[t];
                const DD a1 = DD{pr.s1_hi, pr.s1_lo} + k1, a2 = DD{pr.s2_hi, pr.s2_lo} + k2;
                pr.s1_hi = a1.hi; pr.s1_lo = a1.lo;
                pr.s2_hi = a2.hi; pr.s2_lo = a2.lo;
            }
        }
        if (lane == 0) w.nsel[t] = cnt;
    }
}

// exclusive prefix sum of nsel over the round's tiles (one block of 1024)
__global__ void __launch_bounds__(1024) k_scan(Work w) {
    __shared__ uint32_t wsum[16];
    const uint32_t tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    uint64_t rt0;
    const uint32_t nr = round_len(w, rt0);
    const uint32_t per = (nr + 1023) / 1024;
    const uint32_t t0 = tid * per < nr ? tid * per : nr, t1 = t0 + per < nr ? t0 + per : nr;
    uint32_t loc = 0;
    for (uint32_t t = t0; t < t1; ++t) loc += w.nsel[t];
    uint32_t inc = loc;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(inc, d);
        if ((int)lane >= d) inc += o;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int i = 0; i < 16; ++i) {
            const uint32_t v = wsum[i];
            wsum[i] = run;
            run += v;
        }
    }
    __syncthreads();
    uint32_t off = wsum[wave] + inc - loc;
    for (uint32_t t = t0; t < t1; ++t) {
        w.seloff[t] = off;
        off += w.nsel[t];
    }
    if (tid == 1023) {
        // the double-double pass splits each chunk of 64 entries into slices so
        // that chunks x slices fills its waves
        const uint32_t nchunks = (off + 63) / 64;
        uint32_t ns = nchunks ? w.grid / nchunks : 1;
        ns = ns < 1 ? 1 : (ns > 64 ? 64 : ns);
        w.counter[kCSel] = off;
        w.counter[kCFix] = 0;
        w.counter[kCSlices] = ns;
    }
}

__global__ void __launch_bounds__(64) k_compact(Work w) {
    const int lane = threadIdx.x;
    uint64_t rt0;
    const uint32_t nr = round_len(w, rt0);
    for (uint32_t t = blockIdx.x; t < nr; t += gridDim.x) {
        const uint32_t nf = w.nflag[t];
        uint32_t pos = w.seloff[t];
        for (uint32_t b = 0; b < nf; b += 64) {
            const uint32_t e = b + lane;
            const bool need = e < nf && w.flags[(uint64_t)t * w.tile + e].fixed;
            const uint64_t mask = __ballot(need);
            if (need) w.sel[pos + __popcll(mask & ((1ull << lane) - 1))] = t * w.tile + e;
            pos += __popcll(mask);
        }
    }
}

// Double-double recompute of the selected entries: persistent waves take
// items (chunk of 64 consecutive entries in graph-major order, slice of the
// whole-graph coefficient tables); a chunk that spans graphs is processed one
// graph at a time.  Each item writes its partial f; k_fix_combine adds the
// slices in order.
__global__ void __launch_bounds__(64) k_fix_dd(const uint8_t* __restrict__ img_, Work w) {
    const QA_RO uint8_t* img = (const QA_RO uint8_t*)img_;
    const uint2 key = call_key(w);
    // LDS holds the flows A, C (20 double-doubles per lane, 20 KB per wave); the
    // contraction matrix and the piece results use the per-wave global buffers
    // of the fused pass (which does not run concurrently), so that eight waves
    // fit on a CU.
    extern __shared__ char lds[];
    const int lane = threadIdx.x;
    const uint64_t gw = blockIdx.x;
    VV<DD> vars{reinterpret_cast<DD*>(w.vbuf) + gw * (QA_VAR_A * 64) + lane, 64, reinterpret_cast<DD*>(lds) + lane, 64};
    LV<DD> polys{reinterpret_cast<DD*>(w.pbuf) + gw * (QA_MAXPOLY * QA_MAXN * 64) + lane, 64};
    double* zb = w.zbuf + gw * QA_MAXM * 64;
    const uint32_t total = w.counter[kCSel], ns = w.counter[kCSlices];
    const uint32_t items = (total + 63) / 64 * ns;
    for (;;) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(w.counter + kCFix, 1u);
        it = __builtin_amdgcn_readfirstlane(__shfl(it, 0));
        if (it >= items) break;
        const uint32_t c = it / ns, j = it % ns;
        const uint32_t idx = c * 64 + lane;
        const bool act = idx < total;
        const FlagEntry* fe = act ? &w.flags[w.sel[idx]] : nullptr;
        const uint32_t mine = act ? fe->graph : 0xffffffffu;
        bool done = !act;
        for (;;) {
            const uint32_t g = __builtin_amdgcn_readfirstlane(wave_min_u32(done ? 0xffffffffu : mine));
            if (g == 0xffffffffu) break;
            if (!done && mine == g) {
                const QA_RO DevGraph& G = dev_graph(img, g);
                const QA_RO double* D = reinterpret_cast<const QA_RO double*>(img + G.deg_off);
                const QA_RO double* W = reinterpret_cast<const QA_RO double*>(img + G.w_off);
                Stream st{key, g, fe->sample};
                uint8_t order[QA_MAXM];
                double tl[QA_MAXM], lp, cond;
                LV<double> zv{zb + lane, 64};
                sample_point(D, W, G.M, G.mb, st, zv, lp, order, tl);
                const DD r = eval_point<DD>(img, G, CLV<double>{zb + lane, 64}, vars, polys, cond, (int)j, (int)ns);
                w.fpart[(uint64_t)idx * ns + j] = r;
                if (j == 0) w.fcond[idx] = cond;
                done = true;
            }
        }
    }
}

// per selected entry: f = sum of its slices (in order), its double-double w
// and w^2 (k_reduce adds them: the entry's FP64 value never entered the sums,
// so no correction has to cancel a possibly huge FP64 w) and the residual test
__global__ void __launch_bounds__(256) k_fix_combine(Work w) {
    const uint32_t total = w.counter[kCSel], ns = w.counter[kCSlices];
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        FlagEntry& fe = w.flags[w.sel[e]];
        DD r{0.0, 0.0};
        for (uint32_t j = 0; j < ns; ++j) r = r + w.fpart[(uint64_t)e * ns + j];
        const double fdd = r.hi + r.lo, ip = fe.ip;
        fe.residual = !(est_dd(fe.q, fmax(w.fcond[e], fe.cond), fdd) * ip <=
                        1e-10 * fmax(fabs(fdd) * ip, w.scale[fe.graph]));
        const DD wd = r * ip;
        const DD w2 = wd * wd;
        // as in the fused pass, a weight that is not finite counts as a drawn
        // sample with w = 0 (moved from n to n_bad in k_reduce)
        fe.bad = !(isfinite(wd.hi) && isfinite(wd.lo) && isfinite(w2.hi) && isfinite(w2.lo));
        fe.c1 = fe.bad ? DD{0.0, 0.0} : wd;
        fe.c2 = fe.bad ? DD{0.0, 0.0} : w2;
    }
}

// per graph (one wave): the round's partials and the corrections of its
// selected entries -> acc, in a fixed order
__global__ void __launch_bounds__(64) k_reduce(Work w, qa_acc* acc) {
    const uint32_t g = blockIdx.x, lane = threadIdx.x;
    uint64_t a, b, t0;
    if (g >= w.ng || !round_tiles(w, g, a, b, t0)) return;
    DD s1{0.0, 0.0}, s2{0.0, 0.0};
    uint64_t n = 0, nb = 0, nr = 0, nfb = 0;
    for (uint64_t gt = a + lane; gt < b; gt += 64) {
        const Partial& p = w.partial[gt - t0];
        s1 = s1 + DD{p.s1_hi, p.s1_lo};
        s2 = s2 + DD{p.s2_hi, p.s2_lo};
        n += p.n;
        nb += p.nbad;
    }
    // the selected entries of graph g are contiguous in sel (tile order)
    const uint32_t e0 = w.seloff[a - t0], e1 = w.seloff[b - 1 - t0] + w.nsel[b - 1 - t0];
    for (uint32_t e = e0 + lane; e < e1; e += 64) {
        const FlagEntry& fe = w.flags[w.sel[e]];
        s1 = s1 + fe.c1;
        s2 = s2 + fe.c2;
        nr += fe.residual;
        nfb += fe.bad;
    }
    s1 = wave_sum_dd(s1);
    s2 = wave_sum_dd(s2);
    n = wave_sum_u64(n);
    nb = wave_sum_u64(nb);
    nr = wave_sum_u64(nr);
    nfb = wave_sum_u64(nfb);
    if (lane == 0) {
        s1 = DD{acc[g].s1_hi, acc[g].s1_lo} + s1;
        s2 = DD{acc[g].s2_hi, acc[g].s2_lo} + s2;
        acc[g].s1_hi = s1.hi; acc[g].s1_lo = s1.lo;
        acc[g].s2_hi = s2.hi; acc[g].s2_lo = s2.lo;
        acc[g].n += n - nfb;   // recomputed points whose weight is not finite count as bad
        acc[g].n_flagged += e1 - e0;
        acc[g].n_bad += nb + nfb;
        acc[g].n_residual += nr;
    }
}

// ---------------------------------------------------------------------------
// variance gradient: grad[S_l] += w^2 t_l, w2sum += w^2

__global__ void __launch_bounds__(64) k_vargrad(const uint8_t* __restrict__ img_, uint32_t graph, uint2 key,
                                                uint64_t first, uint64_t count, double* grad, double* w2sum) {
    const QA_RO uint8_t* img = (const QA_RO uint8_t*)img_;
    extern __shared__ char lds[];
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const QA_RO DevGraph& G = dev_graph(img, graph);
    VV<double> vars;
    LV<double> polys;
    lane_views<double>(lds, G.npoly, vars, polys);
    // z after the polynomial region
    double* zb = reinterpret_cast<double*>(lds + lds_bytes_dev<double>(G.npoly, blockDim.x));
    double w2 = 0.0;
    if (i < count) {
        const QA_RO double* D = reinterpret_cast<const QA_RO double*>(img + G.deg_off);
        const QA_RO double* W = reinterpret_cast<const QA_RO double*>(img + G.w_off);
        Stream st{key, graph, first + i};
        uint8_t order[QA_MAXM];
        double tl[QA_MAXM], lp, cond;
        LV<double> zv{zb + threadIdx.x, (int)blockDim.x};
        if (sample_point(D, W, G.M, G.mb, st, zv, lp, order, tl)) {
            const double f = eval_point<double>(img, G, CLV<double>{zb + threadIdx.x, (int)blockDim.x}, vars, polys, cond);
            const double w = f * exp(-lp);
            if (isfinite(w)) {
                w2 = w * w;
                const int Ms = G.mb >= 0 ? G.M - 1 : G.M;
                uint32_t S = (1u << Ms) - 1;
                for (int l = 1; l < Ms; ++l) {
                    S ^= 1u << order[l - 1];
                    atomicAdd(grad + S, w2 * tl[l]);
                }
            }
        }
    }
    // one atomic per wave for the w^2 sum
    double s = w2;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (threadIdx.x == 0) atomicAdd(w2sum, s);
}

// ---------------------------------------------------------------------------
// C ABI launchers

// allow more than the default 64 KB of dynamic LDS where a launch needs it
template <class K> static int lds_attr(K kernel, size_t bytes) {
    if (bytes > 160 * 1024) return qa_fail(QA_ENOTSUP, "LDS requirement exceeds 160 KB");
    if (bytes > 64 * 1024)
        HIPCHK(hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return QA_OK;
}

static const DevGraph* host_graph(const std::vector<uint8_t>& img, uint32_t g) {
    const DevHeader* h = reinterpret_cast<const DevHeader*>(img.data());
    if (g >= h->ngraphs) return nullptr;
    return reinterpret_cast<const DevGraph*>(img.data() + h->graphs_off) + g;
}

// the host copy of the last image uploaded to each device buffer
#include <map>
#include <mutex>
static std::mutex g_up_mu;
static std::map<const void*, std::shared_ptr<const std::vector<uint8_t>>> g_uploaded;

static std::shared_ptr<const std::vector<uint8_t>> image_of(const void* dev) {
    std::lock_guard<std::mutex> l(g_up_mu);
    auto it = g_uploaded.find(dev);
    return it == g_uploaded.end() ? nullptr : it->second;
}

extern "C" int qa_upload(const qa_set* s, const qa_pdf* p, void* dev, size_t bytes, void* stream) {
    auto img = qa_image(s, p);
    if (!img) return QA_EINVAL;
    if (!dev || bytes < img->size()) return qa_fail(QA_ECAP, "device buffer too small");
    HIPCHK(hipMemcpyAsync(dev, img->data(), img->size(), hipMemcpyHostToDevice, (hipStream_t)stream));
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    std::lock_guard<std::mutex> l(g_up_mu);
    g_uploaded[dev] = img;
    return QA_OK;
}

extern "C" int qa_sample_pdf(const void* dev, uint32_t graph, uint64_t seed, uint32_t tag, uint64_t first,
                             uint64_t count, double* z, double* logp, uint8_t* sector, void* stream) {
    auto img = image_of(dev);
    if (!img) return qa_fail(QA_EINVAL, "device image not uploaded by qa_upload");
    if (!host_graph(*img, graph)) return qa_fail(QA_EINVAL, "graph index out of range");
    if (count == 0) return QA_OK;
    if (!z || !logp) return qa_fail(QA_EINVAL, "NULL output");
    if (count > (1ull << 31)) return qa_fail(QA_EINVAL, "count too large for one call");
    if (seed >> 32) return qa_fail(QA_EINVAL, "seed must be below 2^32 (32-bit Philox key word)");
    const uint2 key = make_uint2((uint32_t)seed, tag);
    dim3 grid((unsigned)((count + 255) / 256));
    hipLaunchKernelGGL(k_sample, grid, dim3(256), 0, (hipStream_t)stream, (const uint8_t*)dev, graph, key, first,
                       count, z, logp, sector);
    HIPCHK(hipGetLastError());
    return QA_OK;
}

extern "C" int qa_eval_integrand(const void* dev, uint32_t graph, const double* z, uint64_t count, int mode, double* f,
                                 double* err, uint8_t* flag, void* stream) {
    auto img = image_of(dev);
    if (!img) return qa_fail(QA_EINVAL, "device image not uploaded by qa_upload");
    const DevGraph* G = host_graph(*img, graph);
    if (!G) return qa_fail(QA_EINVAL, "graph index out of range");
    if (count == 0) return QA_OK;
    if (!z || !f) return qa_fail(QA_EINVAL, "NULL argument");
    if (count > (1ull << 31)) return qa_fail(QA_EINVAL, "count too large for one call");
    dim3 grid((unsigned)((count + 63) / 64)), block(64);
    const uint8_t* d = (const uint8_t*)dev;
    hipStream_t st = (hipStream_t)stream;
    int rc = QA_OK;
    if (mode == QA_FP64) rc = lds_attr(k_eval_fp64, lds_bytes<double>(G->npoly, 64));
    else if (mode == QA_FP64_BOUND) rc = lds_attr(k_eval_bound, lds_bytes<EB>(G->npoly, 64));
    else if (mode == QA_DD) rc = lds_attr(k_eval_dd, lds_bytes<DD>(G->npoly, 64));
    else if (mode == QA_FP64_EST) rc = lds_attr(k_eval_est, lds_bytes<ER>(G->npoly, 64));
    if (rc != QA_OK) return rc;
    if (mode == QA_FP64) {
        hipLaunchKernelGGL(k_eval_fp64, grid, block, lds_bytes<double>(G->npoly, 64), st, d, graph, z, count, f);
    } else if (mode == QA_FP64_BOUND) {
        hipLaunchKernelGGL(k_eval_bound, grid, block, lds_bytes<EB>(G->npoly, 64), st, d, graph, z, count, f, err, flag);
    } else if (mode == QA_FP64_EST) {
        hipLaunchKernelGGL(k_eval_est, grid, block, lds_bytes<ER>(G->npoly, 64), st, d, graph, z, count, f, err, flag);
    } else if (mode == QA_DD) {
        hipLaunchKernelGGL(k_eval_dd, grid, block, lds_bytes<DD>(G->npoly, 64), st, d, graph, z, count, f, err);
    } else {
        return qa_fail(QA_EINVAL, "bad mode");
    }
    HIPCHK(hipGetLastError());
    return QA_OK;
}

extern "C" int qa_accumulate(const double* f, const double* logp, uint64_t count, qa_acc* acc, void* stream) {
    if (count == 0) return QA_OK;
    if (!f || !logp || !acc) return qa_fail(QA_EINVAL, "NULL argument");
    hipLaunchKernelGGL(k_accumulate, dim3(1), dim3(1024), 0, (hipStream_t)stream, f, logp, count, acc);
    HIPCHK(hipGetLastError());
    return QA_OK;
}

// work buffer layout for qa_integrate
struct WorkLayout {
    size_t counter, gtile0, budget, partial, nflag, flags, scale, nsel, seloff, sel, fpart, fcond, zbuf, pbuf, vbuf, total;
};
static WorkLayout work_layout(size_t ng, uint32_t tile, uint32_t per_round, uint32_t grid) {
    WorkLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = (o + bytes + 255) / 256 * 256; return r; };
    L.counter = take(64);
    L.gtile0 = take(8 * (ng + 1));
    L.budget = take(8 * ng);
    L.partial = take(sizeof(Partial) * per_round);
    L.nflag = take(4 * per_round);
    L.flags = take(sizeof(FlagEntry) * (size_t)per_round * tile);
    L.scale = take(8 * ng);
    L.nsel = take(4 * per_round);
    L.seloff = take(4 * per_round);
    L.sel = take(4 * (size_t)per_round * tile);
    // partial results: at most max(64 * grid, entries) (slices only when chunks < waves)
    const size_t nfp = std::max<size_t>((size_t)per_round * tile, 64 * (size_t)grid);
    L.fpart = take(sizeof(DD) * nfp);
    L.fcond = take(8 * (size_t)per_round * tile);
    L.zbuf = take(8ull * QA_MAXM * 64 * grid);
    L.pbuf = take(sizeof(ER) * QA_MAXPOLY * QA_MAXN * 64 * (size_t)grid);
    L.vbuf = take(sizeof(DD) * QA_VAR_A * 64 * (size_t)grid);   // double in the fused pass, DD in the DD pass
    L.total = o;
    return L;
}

// a round holds at most this many samples (flag storage: 68 B per sample)
static const uint64_t kRoundSamples = 1ull << 25;
static const uint32_t kDefaultTile = 256;

static uint32_t tiles_per_round(uint64_t ntiles, uint32_t tile) {
    const uint64_t cap = std::max<uint64_t>(1, kRoundSamples / tile);
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(ntiles, cap));
}
static uint64_t count_tiles(const uint64_t* budgets, size_t ng, uint32_t tile) {
    uint64_t t = 0;
    for (size_t g = 0; g < ng; ++g) t += (budgets[g] + tile - 1) / tile;
    return t;
}

static const uint32_t kMaxWaves = 4096;   // persistent waves of a batched launch (16 per CU on 256 CUs)

static uint32_t default_grid() {
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
    }
    return (uint32_t)ncu * 4 * kFusedOcc;
}

extern "C" int qa_work_bytes(const qa_set* s, const uint64_t* budgets, uint32_t tile, size_t* bytes) {
    if (!s || !bytes || !budgets) return qa_fail(QA_EINVAL, "NULL argument");
    if (tile == 0) tile = kDefaultTile;
    if (tile % 64) return qa_fail(QA_EINVAL, "tile must be a multiple of 64");
    const size_t ng = qa_set_size(s);
    // enough persistent waves for any grid up to 8 per CU on 256 CUs
    *bytes = work_layout(ng, tile, tiles_per_round(count_tiles(budgets, ng, tile), tile), kMaxWaves).total;
    return QA_OK;
}

// pointers of the work buffer's regions
static void set_work(Work& w, char* wb, const WorkLayout& L) {
    w.counter = (uint32_t*)(wb + L.counter);
    w.gtile0 = (uint64_t*)(wb + L.gtile0);
    w.budget = (uint64_t*)(wb + L.budget);
    w.partial = (Partial*)(wb + L.partial);
    w.nflag = (uint32_t*)(wb + L.nflag);
    w.flags = (FlagEntry*)(wb + L.flags);
    w.scale = (double*)(wb + L.scale);
    w.nsel = (uint32_t*)(wb + L.nsel);
    w.seloff = (uint32_t*)(wb + L.seloff);
    w.sel = (uint32_t*)(wb + L.sel);
    w.fpart = (DD*)(wb + L.fpart);
    w.fcond = (double*)(wb + L.fcond);
    w.zbuf = (double*)(wb + L.zbuf);
    w.pbuf = (ER*)(wb + L.pbuf);
    w.vbuf = (double*)(wb + L.vbuf);
}

// A round as two instantiated graphs: (reset queue, fused pass) and (weight
// scales, selection and compaction of the candidates, double-double pass,
// reduce, advance round).  The graphs depend only on the image, the work and
// acc buffers and the layout (set size, tile, grid, tiles per round, tile
// count): the call's key and first sample are read from the work buffer.  A
// small cache keeps the instantiated graphs of recent plans, so that repeated
// calls (steps of a run) replay them without capture or instantiation.
struct RoundGraphs {
    const void* dev;
    const void* work;
    const void* acc;
    size_t ng;
    uint32_t tile, grid, per_round;
    uint64_t ntiles;
    hipGraphExec_t ea, eb;
    uint64_t used;
};
static std::mutex g_graph_mu;
static std::vector<RoundGraphs> g_graphs;
static uint64_t g_graph_clock = 0;
constexpr size_t kGraphCache = 8;

static void destroy_round_graphs(RoundGraphs& r) {
    if (r.ea) hipGraphExecDestroy(r.ea);
    if (r.eb) hipGraphExecDestroy(r.eb);
    r.ea = r.eb = nullptr;
}

static int capture_round(const void* dev, const Work& w, qa_acc* acc, size_t ng, uint32_t grid, RoundGraphs& out) {
    const size_t lds_fp = sizeof(double) * (QA_NVAR - QA_VAR_A) * kFusedThreads,
                 lds_dd = sizeof(DD) * (QA_NVAR - QA_VAR_A) * 64;
    if (int rc = lds_attr(k_fused, lds_fp)) return rc;
    if (int rc = lds_attr(k_fix_dd, lds_dd)) return rc;
    hipStream_t cs;   // capture needs a stream other than the null stream
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t ga = nullptr, gb = nullptr;
    hipError_t ce = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (ce == hipSuccess) {
        hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, cs, w);
        hipLaunchKernelGGL(k_fused, dim3(grid / kFusedWaves), dim3(kFusedThreads), lds_fp, cs, (const uint8_t*)dev, w);
        ce = hipStreamEndCapture(cs, &ga);
    }
    if (ce == hipSuccess) ce = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (ce == hipSuccess) {
        const dim3 gng((unsigned)ng);
        hipLaunchKernelGGL(k_scale, gng, dim3(64), 0, cs, w, acc);
        hipLaunchKernelGGL(k_select, dim3(grid), dim3(64), 0, cs, w);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, cs, w);
        hipLaunchKernelGGL(k_compact, dim3(grid), dim3(64), 0, cs, w);
        hipLaunchKernelGGL(k_fix_dd, dim3(grid), dim3(64), lds_dd, cs, (const uint8_t*)dev, w);
        hipLaunchKernelGGL(k_fix_combine, dim3(512), dim3(256), 0, cs, w);
        hipLaunchKernelGGL(k_reduce, gng, dim3(64), 0, cs, w, acc);
        hipLaunchKernelGGL(k_next_round, dim3(1), dim3(64), 0, cs, w);
        ce = hipStreamEndCapture(cs, &gb);
    }
    if (ce == hipSuccess) ce = hipGraphInstantiate(&out.ea, ga, nullptr, nullptr, 0);
    if (ce == hipSuccess) ce = hipGraphInstantiate(&out.eb, gb, nullptr, nullptr, 0);
    if (ga) hipGraphDestroy(ga);
    if (gb) hipGraphDestroy(gb);
    hipStreamDestroy(cs);
    if (ce != hipSuccess) {
        destroy_round_graphs(out);
        return qa_fail(QA_EHIP, std::string("graph capture: ") + hipGetErrorString(ce));
    }
    return QA_OK;
}

extern "C" int qa_integrate(const qa_set* s, const void* dev, const uint64_t* budgets, uint64_t first, uint64_t seed,
                            uint32_t tag, uint32_t tile, uint32_t grid, void* work, size_t work_bytes, qa_acc* acc,
                            double* fused_ms, void* stream) {
    auto img = image_of(dev);
    if (!img) return qa_fail(QA_EINVAL, "device image not uploaded by qa_upload");
    if (!s || !budgets || !work || !acc) return qa_fail(QA_EINVAL, "NULL argument");
    if (seed >> 32) return qa_fail(QA_EINVAL, "seed must be below 2^32 (32-bit Philox key word)");
    const size_t ng = qa_set_size(s);
    if (reinterpret_cast<const DevHeader*>(img->data())->ngraphs != ng) return qa_fail(QA_EINVAL, "set / image mismatch");
    if (tile == 0) tile = kDefaultTile;
    if (tile % 64) return qa_fail(QA_EINVAL, "tile must be a multiple of 64");
    if (grid == 0) grid = default_grid();
    if (grid > kMaxWaves) return qa_fail(QA_EINVAL, "grid too large (max 4096 waves)");
    grid = (grid + kFusedWaves - 1) / kFusedWaves * kFusedWaves;   // the fused pass runs workgroups of 4 waves
    for (size_t g = 0; g < ng; ++g)
        if (host_graph(*img, (uint32_t)g)->npoly > QA_MAXPOLY) return qa_fail(QA_ENOTSUP, "too many piece-result slots");
    std::vector<uint64_t> g0(ng + 1, 0);
    for (size_t g = 0; g < ng; ++g) g0[g + 1] = g0[g] + (budgets[g] + tile - 1) / tile;
    const uint64_t ntiles = g0[ng];
    const uint32_t per_round = tiles_per_round(ntiles, tile);
    WorkLayout L = work_layout(ng, tile, per_round, grid);
    if (work_bytes < L.total) return qa_fail(QA_ECAP, "work buffer too small");
    hipStream_t st = (hipStream_t)stream;
    char* wb = (char*)work;
    uint32_t hdr[16] = {};
    hdr[kCKey] = (uint32_t)seed;
    hdr[kCKey + 1] = tag;
    hdr[kCFirst] = (uint32_t)first;
    hdr[kCFirst + 1] = (uint32_t)(first >> 32);
    HIPCHK(hipMemcpyAsync(wb + L.counter, hdr, sizeof hdr, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(wb + L.gtile0, g0.data(), 8 * (ng + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(wb + L.budget, budgets, 8 * ng, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(acc, 0, sizeof(qa_acc) * ng, st));
    HIPCHK(hipStreamSynchronize(st));
    if (ntiles == 0) return QA_OK;
    Work w{};
    set_work(w, wb, L);
    w.grid = grid;
    w.tile = tile;
    w.per_round = per_round;
    w.ng = (uint32_t)ng;
    w.ntiles = ntiles;
    hipGraphExec_t ea = nullptr, eb = nullptr;
    {
        std::lock_guard<std::mutex> l(g_graph_mu);
        RoundGraphs* hit = nullptr;
        for (auto& r : g_graphs)
            if (r.dev == dev && r.work == work && r.acc == acc && r.ng == ng && r.tile == tile && r.grid == grid &&
                r.per_round == per_round && r.ntiles == ntiles)
                hit = &r;
        if (!hit) {
            RoundGraphs r{dev, work, acc, ng, tile, grid, per_round, ntiles, nullptr, nullptr, 0};
            if (int rc = capture_round(dev, w, acc, ng, grid, r)) return rc;
            if (g_graphs.size() >= kGraphCache) {
                auto old = std::min_element(g_graphs.begin(), g_graphs.end(),
                                            [](const RoundGraphs& a, const RoundGraphs& b) { return a.used < b.used; });
                destroy_round_graphs(*old);
                g_graphs.erase(old);
            }
            g_graphs.push_back(r);
            hit = &g_graphs.back();
        }
        hit->used = ++g_graph_clock;
        ea = hit->ea;
        eb = hit->eb;
        // replays of one cached plan from two threads would race on its buffers anyway
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        if (fused_ms) {
            *fused_ms = 0.0;
            if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess)
                return qa_fail(QA_EHIP, "hipEventCreate failed");
        }
        const uint64_t rounds = (ntiles + per_round - 1) / per_round;
        int rc = QA_OK;
        for (uint64_t r = 0; r < rounds && rc == QA_OK; ++r) {
            hipError_t e = hipSuccess;
            if (ev0) e = hipEventRecord(ev0, st);
            if (e == hipSuccess) e = hipGraphLaunch(ea, st);
            if (e == hipSuccess && ev1) e = hipEventRecord(ev1, st);
            if (e == hipSuccess) e = hipGraphLaunch(eb, st);
            if (e == hipSuccess && ev1) {
                e = hipEventSynchronize(ev1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
                *fused_ms += ms;
            }
            if (e != hipSuccess) rc = qa_fail(QA_EHIP, std::string("round launch: ") + hipGetErrorString(e));
        }
        hipError_t e = hipStreamSynchronize(st);
        if (ev0) hipEventDestroy(ev0);
        if (ev1) hipEventDestroy(ev1);
        if (rc != QA_OK) return rc;
        if (e != hipSuccess) return qa_fail(QA_EHIP, std::string("integrate: ") + hipGetErrorString(e));
    }
    return QA_OK;
}

// ---------------------------------------------------------------------------
// Batched form without allocation: the work memory is the library's own
// device array `scratch` (one per GPU, reserved when the code object is
// loaded on that GPU, held until the process ends); budgets travel in kernel
// arguments and every buffer that must start at zero is cleared by a kernel,
// so the call enqueues only kernel launches on the caller's stream.

constexpr size_t kScratchBytes = 384ull << 20;
constexpr uint64_t kNoAllocRoundSamples = 1ull << 19;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];

// device address of this GPU's `scratch` (the array's name in host code is a
// host-side stand-in, not a device address)
static int scratch_address(void** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return qa_fail(QA_ENOTSUP, "device index beyond 63");
    std::lock_guard<std::mutex> l(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return qa_fail(QA_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return QA_OK;
}

constexpr int kBudgetChunk = 48;
struct BudgetChunk {
    uint32_t off, cnt;
    uint64_t b[kBudgetChunk];
};
__global__ void k_put_budgets(Work w, BudgetChunk c) {
    const uint32_t i = threadIdx.x;
    if (i < c.cnt) w.budget[c.off + i] = c.b[i];
}
// counters to zero, the call's key and first sample, the graphs' first tiles
// (prefix over the budgets) and acc cleared: one wave
__global__ void k_setup(Work w, qa_acc* acc, uint32_t seed, uint32_t tag, uint64_t first) {
    const uint32_t lane = threadIdx.x;
    if (lane < 16) {
        uint32_t v = 0;
        if (lane == kCKey) v = seed;
        if (lane == kCKey + 1) v = tag;
        if (lane == kCFirst) v = (uint32_t)first;
        if (lane == kCFirst + 1) v = (uint32_t)(first >> 32);
        w.counter[lane] = v;
    }
    for (uint32_t g = lane; g < w.ng; g += 64) acc[g] = qa_acc{};
    if (lane == 0) {
        uint64_t t = 0;
        for (uint32_t g = 0; g < w.ng; ++g) {
            w.gtile0[g] = t;
            t += (w.budget[g] + w.tile - 1) / w.tile;
        }
        w.gtile0[w.ng] = t;
    }
}


// rounds of at most kNoAllocRoundSamples samples; the largest grid (a multiple
// of the fused workgroup, at most the requested one) whose work fits scratch
static int noalloc_plan(size_t ng, const uint64_t* budgets, uint32_t tile, uint32_t grid, uint64_t& ntiles,
                        uint32_t& per_round, uint32_t& grid_out, WorkLayout& L) {
    ntiles = 0;
    for (size_t g = 0; g < ng; ++g) ntiles += (budgets[g] + tile - 1) / tile;
    per_round = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(ntiles, std::max<uint64_t>(1, kNoAllocRoundSamples / tile)));
    const size_t fixed = work_layout(ng, tile, per_round, 0).total;
    const size_t per_wave = (work_layout(ng, tile, per_round, 64 * kFusedWaves).total - fixed) / 64;
    if (fixed + per_wave > kScratchBytes) return qa_fail(QA_ECAP, "set does not fit the no-allocation scratch");
    if (grid == 0) grid = default_grid();
    grid = std::min<uint32_t>(grid, (uint32_t)std::min<size_t>(kMaxWaves, (kScratchBytes - fixed) / per_wave * kFusedWaves));
    grid = grid / kFusedWaves * kFusedWaves;
    while (grid > 0 && work_layout(ng, tile, per_round, grid).total > kScratchBytes) grid -= kFusedWaves;
    if (grid == 0) return qa_fail(QA_ECAP, "no persistent wave fits the no-allocation scratch");
    grid_out = grid;
    L = work_layout(ng, tile, per_round, grid);
    return QA_OK;
}

extern "C" int qa_integrate_noalloc(const qa_set* s, const void* dev, const uint64_t* budgets, uint64_t first,
                                    uint64_t seed, uint32_t tag, uint32_t tile, uint32_t grid, qa_acc* acc,
                                    void* stream) {
    auto img = image_of(dev);
    if (!img) return qa_fail(QA_EINVAL, "device image not uploaded by qa_upload");
    if (!s || !budgets || !acc) return qa_fail(QA_EINVAL, "NULL argument");
    if (seed >> 32) return qa_fail(QA_EINVAL, "seed must be below 2^32 (32-bit Philox key word)");
    const size_t ng = qa_set_size(s);
    if (ng == 0) return qa_fail(QA_EINVAL, "empty set");
    if (reinterpret_cast<const DevHeader*>(img->data())->ngraphs != ng) return qa_fail(QA_EINVAL, "set / image mismatch");
    if (tile == 0) tile = kDefaultTile;
    if (tile % 64) return qa_fail(QA_EINVAL, "tile must be a multiple of 64");
    if (grid > kMaxWaves) return qa_fail(QA_EINVAL, "grid too large (max 4096 waves)");
    for (size_t g = 0; g < ng; ++g)
        if (host_graph(*img, (uint32_t)g)->npoly > QA_MAXPOLY) return qa_fail(QA_ENOTSUP, "too many piece-result slots");
    uint64_t ntiles = 0;
    uint32_t per_round = 0;
    WorkLayout L{};
    if (int rc = noalloc_plan(ng, budgets, tile, grid, ntiles, per_round, grid, L)) return rc;
    void* base = nullptr;
    if (int rc = scratch_address(&base)) return rc;
    hipStream_t st = (hipStream_t)stream;
    Work w{};
    set_work(w, (char*)base, L);
    w.grid = grid;
    w.tile = tile;
    w.per_round = per_round;
    w.ng = (uint32_t)ng;
    w.ntiles = ntiles;
    for (size_t off = 0; off < ng; off += kBudgetChunk) {
        BudgetChunk c{};
        c.off = (uint32_t)off;
        c.cnt = (uint32_t)std::min<size_t>(kBudgetChunk, ng - off);
        for (uint32_t i = 0; i < c.cnt; ++i) c.b[i] = budgets[off + i];
        hipLaunchKernelGGL(k_put_budgets, dim3(1), dim3(64), 0, st, w, c);
    }
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(64), 0, st, w, acc, (uint32_t)seed, tag, first);
    HIPCHK(hipGetLastError());
    if (ntiles == 0) return QA_OK;
    const size_t lds_fp = sizeof(double) * (QA_NVAR - QA_VAR_A) * kFusedThreads,
                 lds_dd = sizeof(DD) * (QA_NVAR - QA_VAR_A) * 64;
    if (int rc = lds_attr(k_fused, lds_fp)) return rc;
    if (int rc = lds_attr(k_fix_dd, lds_dd)) return rc;
    const uint64_t rounds = (ntiles + per_round - 1) / per_round;
    const dim3 gng((unsigned)ng);
    for (uint64_t r = 0; r < rounds; ++r) {
        hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, w);
        hipLaunchKernelGGL(k_fused, dim3(grid / kFusedWaves), dim3(kFusedThreads), lds_fp, st, (const uint8_t*)dev, w);
        hipLaunchKernelGGL(k_scale, gng, dim3(64), 0, st, w, acc);
        hipLaunchKernelGGL(k_select, dim3(grid), dim3(64), 0, st, w);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, w);
        hipLaunchKernelGGL(k_compact, dim3(grid), dim3(64), 0, st, w);
        hipLaunchKernelGGL(k_fix_dd, dim3(grid), dim3(64), lds_dd, st, (const uint8_t*)dev, w);
        hipLaunchKernelGGL(k_fix_combine, dim3(512), dim3(256), 0, st, w);
        hipLaunchKernelGGL(k_reduce, gng, dim3(64), 0, st, w, acc);
        hipLaunchKernelGGL(k_next_round, dim3(1), dim3(64), 0, st, w);
        HIPCHK(hipGetLastError());
    }
    return QA_OK;
}

// Autotuner of the batched form: times the fused pass on a pilot share of the
// budgets for each candidate (tile, grid) and returns the fastest per sample.
// A fused workgroup of 256 lanes takes tile / 256 samples per lane (the
// samples per thread); grid is the number of persistent waves.
extern "C" int qa_autotune(const qa_set* s, const void* dev, const uint64_t* budgets, uint64_t seed, uint32_t tag,
                           uint64_t pilot, void* work, size_t work_bytes, qa_acc* acc, uint32_t* tile_out,
                           uint32_t* grid_out, double* ns_per_sample, void* stream) {
    if (!s || !dev || !budgets || !work || !acc || !tile_out || !grid_out) return qa_fail(QA_EINVAL, "NULL argument");
    if (seed >> 32) return qa_fail(QA_EINVAL, "seed must be below 2^32 (32-bit Philox key word)");
    const size_t ng = qa_set_size(s);
    double total = 0.0;
    for (size_t g = 0; g < ng; ++g) total += (double)budgets[g];
    if (total <= 0.0) return qa_fail(QA_EINVAL, "all budgets are zero");
    if (pilot == 0) pilot = 1ull << 20;
    std::vector<uint64_t> pb(ng, 0);
    uint64_t ptot = 0;
    for (size_t g = 0; g < ng; ++g) {
        if (budgets[g] == 0) continue;
        pb[g] = std::max<uint64_t>(1, (uint64_t)((double)budgets[g] * (double)pilot / total));
        ptot += pb[g];
    }
    const uint32_t full = default_grid(), cu4 = full / kFusedOcc;   // 4 waves per CU = one per SIMD
    const uint32_t tiles[3] = {256, 512, 1024};
    const uint32_t grids[3] = {full, std::min<uint32_t>(kMaxWaves, 3 * cu4), 2 * cu4};
    double best = 1e300;
    uint32_t bt = 0, bg = 0;
    for (uint32_t tile : tiles) {
        const size_t need = work_layout(ng, tile, tiles_per_round(count_tiles(pb.data(), ng, tile), tile), kMaxWaves).total;
        if (need > work_bytes) continue;
        for (uint32_t grid : grids) {
            double ms = 0.0;
            for (int rep = 0; rep < 2; ++rep) {   // the first run warms caches and instantiates the graphs
                if (int rc = qa_integrate(s, dev, pb.data(), 0, seed, tag, tile, grid, work, work_bytes, acc, &ms, stream))
                    return rc;
            }
            const double t = ms * 1e6 / (double)ptot;
            if (t < best) {
                best = t;
                bt = tile;
                bg = grid;
            }
        }
    }
    if (bt == 0) return qa_fail(QA_ECAP, "work buffer too small for the pilot");
    *tile_out = bt;
    *grid_out = bg;
    if (ns_per_sample) *ns_per_sample = best;
    return QA_OK;
}

extern "C" int qa_variance_grad(const void* dev, uint32_t graph, uint64_t seed, uint32_t tag, uint64_t first,
                                uint64_t count, double* grad, double* w2sum, void* stream) {
    auto img = image_of(dev);
    if (!img) return qa_fail(QA_EINVAL, "device image not uploaded by qa_upload");
    const DevGraph* G = host_graph(*img, graph);
    if (!G) return qa_fail(QA_EINVAL, "graph index out of range");
    if (count == 0) return QA_OK;
    if (!grad || !w2sum) return qa_fail(QA_EINVAL, "NULL argument");
    if (count > (1ull << 31)) return qa_fail(QA_EINVAL, "count too large for one call");
    if (seed >> 32) return qa_fail(QA_EINVAL, "seed must be below 2^32 (32-bit Philox key word)");
    const unsigned nb = (unsigned)((count + 63) / 64);
    if (int rc = lds_attr(k_vargrad, lds_bytes<double>(G->npoly, 64) + 8 * QA_MAXM * 64)) return rc;
    hipLaunchKernelGGL(k_vargrad, dim3(nb), dim3(64), lds_bytes<double>(G->npoly, 64) + 8 * QA_MAXM * 64,
                       (hipStream_t)stream, (const uint8_t*)dev, graph, make_uint2((uint32_t)seed, tag), first, count,
                       grad, w2sum);
    HIPCHK(hipGetLastError());
    return QA_OK;
}

// ---------------------------------------------------------------------------
// results and the assembled pilot gradient (device copies + host arithmetic)

const std::vector<double>* qa_pdf_deg(const qa_pdf* p, uint32_t graph);
std::vector<double> qa_pdf_dlogw_vec(const qa_pdf* p, uint32_t graph);

extern "C" int qa_acc_read(const qa_set* s, const qa_acc* dev_acc, qa_result* per_graph, qa_result* total,
                           void* stream) {
    if (!s || !dev_acc) return qa_fail(QA_EINVAL, "NULL argument");
    std::vector<qa_acc> h(qa_set_size(s));
    if (h.empty()) return qa_fail(QA_EINVAL, "empty set");
    HIPCHK(hipMemcpyAsync(h.data(), dev_acc, sizeof(qa_acc) * h.size(), hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    return qa_results(s, h.data(), per_graph, total);
}

extern "C" int qa_variance_gradient(const qa_pdf* p, const void* dev, uint32_t graph, uint64_t seed, uint32_t tag,
                                    uint64_t first, uint64_t count, double* work, double* grad, double* m2,
                                    void* stream) {
    auto img = image_of(dev);
    if (!img) return qa_fail(QA_EINVAL, "device image not uploaded by qa_upload");
    const DevGraph* G = host_graph(*img, graph);
    if (!G) return qa_fail(QA_EINVAL, "graph index out of range");
    const std::vector<double>* D = qa_pdf_deg(p, graph);
    const int Ms = G->mb >= 0 ? G->M - 1 : G->M;
    if (!D || D->size() != (size_t(1) << Ms)) return qa_fail(QA_EINVAL, "pdf does not match the image");
    if (std::memcmp(D->data(), img->data() + G->deg_off, 8 * D->size()) != 0)
        return qa_fail(QA_EINVAL, "the image on dev was not uploaded from this pdf");
    if (!work || !grad) return qa_fail(QA_EINVAL, "NULL argument");
    if (count < 1) return qa_fail(QA_EINVAL, "count must be positive");
    const size_t nS = size_t(1) << Ms;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemsetAsync(work, 0, 8 * (nS + 1), st));
    if (int rc = qa_variance_grad(dev, graph, seed, tag, first, count, work, work + nS, stream)) return rc;
    std::vector<double> h(nS + 1);
    HIPCHK(hipMemcpyAsync(h.data(), work, 8 * (nS + 1), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double N = (double)count, mom2 = h[nS] / N;
    const std::vector<double> dl = qa_pdf_dlogw_vec(p, graph);
    for (size_t S = 0; S < nS; ++S) grad[S] = h[S] / N + mom2 * dl[S];
    grad[0] = 0.0;
    grad[nS - 1] = 0.0;
    if (m2) *m2 = mom2;
    return QA_OK;
}
