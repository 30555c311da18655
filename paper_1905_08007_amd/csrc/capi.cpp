// C ABI: handles, error reporting and packing of the device image.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>

#include "../../include/qedamm.h"
#include "host.h"

using namespace qa;

static thread_local std::string g_err;
static int fail(int code, const std::string& msg) { g_err = msg; return code; }
int qa_fail(int code, const std::string& msg) { return fail(code, msg); }
extern "C" const char* qa_last_error(void) { return g_err.c_str(); }

struct qa_set {
    std::vector<GraphTables> graphs;
};
struct qa_pdf {
    std::vector<int> M;                        // sampled lines per graph (3n, or 3n - 1 in the merged form)
    std::vector<int> mb;                       // merged form: line b of the merged pair, else -1
    std::vector<std::vector<double>> deg, w;
};

static Graph from_c(const qa_graph& c) {
    Graph g{};
    g.n = c.loops; g.x = c.x; g.mult = c.mult;
    for (int i = 0; i < 12; ++i) g.mate[i] = c.mate[i];
    for (int i = 0; i < 3; ++i) g.cls[i] = c.cls[i];
    return g;
}

extern "C" int qa_enumerate_graphs(int loops, int k, int m, int n, qa_graph* out, size_t cap, size_t* count) {
    try {
        if (loops < 1 || loops > QA_MAXN) return fail(QA_EINVAL, "loops must be 1..5");
        if (!count) return fail(QA_EINVAL, "count is NULL");
        auto all = enumerate(loops);
        size_t c = 0;
        for (auto& g : all) {
            if (k >= 0 && g.cls[0] != k) continue;
            if (m >= 0 || n >= 0) {
                int mm = std::max(m, n), nn = std::min(m, n);
                if (m < 0 || n < 0) { if (g.cls[1] != mm && g.cls[2] != mm) continue; }
                else if (g.cls[1] != mm || g.cls[2] != nn) continue;
            }
            if (c < cap && out) {
                qa_graph& o = out[c];
                std::memset(&o, 0, sizeof o);
                o.loops = g.n; o.x = g.x; o.mult = g.mult;
                for (int s = 0; s <= 2 * g.n; ++s) o.mate[s] = (int8_t)g.mate[s];
                for (int i = 0; i < 3; ++i) o.cls[i] = g.cls[i];
            }
            ++c;
        }
        *count = c;
        if (c > cap) return fail(QA_ECAP, "output capacity too small");
        return QA_OK;
    } catch (std::exception& e) { return fail(QA_EINVAL, e.what()); }
}

// structure of one graph (fast); the tables are filled by build_tables
static void build_structure(GraphTables& T) {
    const Graph& g = T.g;
    T.subs = subgraphs(g);
    T.forests = forests(T.subs);
    T.terms = terms(T.subs);
    for (auto& tm : T.terms) {
        auto pcs = term_pieces(g, T.subs, tm.first, tm.second);
        std::vector<std::vector<Table>> tabs;
        for (auto& p : pcs) {
            int nins = 0;
            for (auto& nd : p.nodes) nins += nd.vtype == 2;
            int nop = p.op == QA_OP_US ? 2 : 1;
            tabs.push_back(std::vector<Table>((size_t)nop << nins));
        }
        T.pieces.push_back(std::move(pcs));
        T.tabs.push_back(std::move(tabs));
    }
}

extern "C" int qa_build_forests(const qa_graph* gs, size_t ng, int nthreads, qa_set** out) {
    try {
        if (!gs || !out) return fail(QA_EINVAL, "NULL argument");
        auto* s = new qa_set;
        s->graphs.resize(ng);
        for (size_t i = 0; i < ng; ++i) {
            if (gs[i].loops < 1 || gs[i].loops > QA_MAXN) { delete s; return fail(QA_EINVAL, "bad loops"); }
            s->graphs[i].g = from_c(gs[i]);
            build_structure(s->graphs[i]);
        }
        // jobs: slices of coefficient tables (large tables split by block
        // index mod nparts), largest first; slices are merged in block order
        struct Job { size_t g, t, p, v; int part, nparts; size_t cost; };
        std::vector<Job> jobs;
        for (size_t gi = 0; gi < ng; ++gi) {
            auto& T = s->graphs[gi];
            for (size_t ti = 0; ti < T.terms.size(); ++ti)
                for (size_t pi = 0; pi < T.pieces[ti].size(); ++pi) {
                    const size_t nl = T.pieces[ti][pi].lines.size();
                    const int np = nl >= 9 ? 32 : (nl >= 7 ? 4 : 1);
                    for (size_t v = 0; v < T.tabs[ti][pi].size(); ++v)
                        for (int part = 0; part < np; ++part) jobs.push_back({gi, ti, pi, v, part, np, nl});
                }
        }
        std::stable_sort(jobs.begin(), jobs.end(), [](const Job& a, const Job& b) { return a.cost > b.cost; });
        std::vector<Table> slices(jobs.size());
        int nt = nthreads > 0 ? nthreads : (int)std::thread::hardware_concurrency();
        nt = std::max(1, std::min<int>(nt, (int)jobs.size()));
        std::atomic<size_t> next{0};
        std::string err;
        std::mutex mu;
        std::vector<std::thread> th;
        for (int t = 0; t < nt; ++t)
            th.emplace_back([&] {
                for (size_t i; (i = next++) < jobs.size();) {
                    const Job& j = jobs[i];
                    auto& T = s->graphs[j.g];
                    const Piece& pc = T.pieces[j.t][j.p];
                    const size_t nvar = T.tabs[j.t][j.p].size();
                    const int nop = pc.op == QA_OP_US ? 2 : 1;
                    const size_t per = nvar / nop;
                    try { slices[i] = build_table(pc, (int)(j.v / per), (uint32_t)(j.v % per), T.g.n, j.part, j.nparts); }
                    catch (std::exception& e) { std::lock_guard<std::mutex> l(mu); err = e.what(); }
                }
            });
        for (auto& t : th) t.join();
        // merge slices: blocks are interleaved by index mod nparts within each k
        std::map<std::array<size_t, 4>, std::vector<size_t>> parts;
        for (size_t i = 0; i < jobs.size(); ++i) parts[{jobs[i].g, jobs[i].t, jobs[i].p, jobs[i].v}].push_back(i);
        for (auto& kv : parts) {
            auto& idx = kv.second;
            std::sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return jobs[a].part < jobs[b].part; });
            Table merged = slices[idx[0]];
            merged.blocks.clear();
            std::vector<size_t> pos(idx.size(), 0);
            for (int k = 0; k <= QA_MAXN; ++k) {
                // round-robin over slices, blocks of this k, restores enumeration order of the kept blocks
                std::vector<std::vector<const Block*>> per(idx.size());
                for (size_t q = 0; q < idx.size(); ++q)
                    for (auto& b : slices[idx[q]].blocks) if (b.k == k) per[q].push_back(&b);
                size_t maxlen = 0;
                for (auto& v : per) maxlen = std::max(maxlen, v.size());
                for (size_t r = 0; r < maxlen; ++r)
                    for (size_t q = 0; q < idx.size(); ++q)
                        if (r < per[q].size()) merged.blocks.push_back(*per[q][r]);
            }
            s->graphs[kv.first[0]].tabs[kv.first[1]][kv.first[2]][kv.first[3]] = std::move(merged);
        }
        if (!err.empty()) { delete s; return fail(QA_EINVAL, err); }
        *out = s;
        return QA_OK;
    } catch (std::exception& e) { return fail(QA_ENOMEM, e.what()); }
}

void qa_image_forget(const void* s, const void* p);
extern "C" void qa_set_destroy(qa_set* s) {
    qa_image_forget(s, nullptr);
    delete s;
}

extern "C" int qa_forests_serialize(const qa_set* s, void* buf, size_t cap, size_t* len) {
    if (!s || !len) return fail(QA_EINVAL, "NULL argument");
    std::vector<int32_t> v;
    for (auto& T : s->graphs) {
        v.push_back((int32_t)T.subs.size());
        for (auto& x : T.subs) { v.push_back(x.lo); v.push_back(x.hi); v.push_back(x.kind); v.push_back(x.has_x); }
        v.push_back((int32_t)T.forests.size());
        for (auto f : T.forests) v.push_back((int32_t)f);
        v.push_back((int32_t)T.terms.size());
        for (auto& t : T.terms) { v.push_back((int32_t)t.first); v.push_back(t.second); }
    }
    *len = v.size() * 4;
    if (!buf || cap < *len) return fail(QA_ECAP, "buffer too small");
    std::memcpy(buf, v.data(), *len);
    return QA_OK;
}

extern "C" int qa_set_stats(const qa_set* s, uint64_t* nterms, uint64_t* nblocks, uint64_t* ncoef) {
    if (!s) return fail(QA_EINVAL, "NULL set");
    uint64_t a = 0, b = 0, c = 0;
    for (auto& T : s->graphs) {
        a += T.terms.size();
        for (auto& tv : T.tabs) for (auto& pv : tv) for (auto& tb : pv) {
            b += tb.blocks.size();
            for (auto& bl : tb.blocks) c += bl.coef.size();
        }
    }
    if (nterms) *nterms = a;
    if (nblocks) *nblocks = b;
    if (ncoef) *ncoef = c;
    return QA_OK;
}

// FP64 operations of geometry_L for a piece (mirrors its loops)
static double geometry_flops(const Piece& p) {
    const int L = (int)p.chords.size(), nl = (int)p.lines.size();
    auto span = [&](int c, int i) { return i >= p.chords[c][1] && i < p.chords[c][2]; };
    double f = 0;
    for (int c = 0; c < L; ++c)
        for (int d = c; d < L; ++d) {
            for (int i = 0; i < nl; ++i) f += span(c, i) && span(d, i);
            f += (c == d);
        }
    for (int c = 0; c < L; ++c) { for (int d = 0; d <= c; ++d) f += 2 * d + 1; }   // Cholesky (sqrt / div as 1)
    f += 2 * L;                                                                      // U
    for (int c = 0; c < L; ++c) { f += 1; for (int d = 0; d < c; ++d) f += 2 * (c - d) + 1; }
    for (int c = 0; c < L; ++c) for (int d = c; d < L; ++d) f += 2 * (L - d);         // M^-1
    for (int c = 0; c < L; ++c) for (int i = 0; i < nl; ++i) f += 2 * span(c, i);     // jq
    f += 4.0 * L * L;                                                                 // y, yq
    for (int i = 0; i < nl; ++i) {
        int ns = 0;
        for (int c = 0; c < L; ++c) ns += span(c, i);
        f += 2 * ns + 3 + (double)L * ns;                                              // A, C, V, Y
        for (int j = i; j < nl; ++j) { for (int d = 0; d < L; ++d) f += span(d, j); }
    }
    return f;
}

static double table_flops(const Table& t, int n) {
    double f = n;  // scale
    for (auto& b : t.blocks) {
        f += b.k > 1 ? b.k - 1 : 0;
        f += 2.0 * ((1 << b.r) - 1);
        if (t.has_q) f += b.r * (2.0 * ((1 << (b.r > 0 ? b.r - 1 : 0)) - 1) + 2);
        f += 2;
    }
    return f;
}

extern "C" int qa_graph_flops(const qa_set* s, uint32_t graph, double* eval_flops, double* sample_flops) {
    if (!s || graph >= s->graphs.size()) return fail(QA_EINVAL, "bad graph index");
    const auto& T = s->graphs[graph];
    const int n = T.g.n, M = 3 * n;
    double f = 0;
    for (size_t ti = 0; ti < T.terms.size(); ++ti) {
        for (size_t pi = 0; pi < T.pieces[ti].size(); ++pi) {
            const Piece& p = T.pieces[ti][pi];
            f += geometry_flops(p) + 4;  // + U^-2, V sum
            int nins = 0, nv = 0;
            for (auto& nd : p.nodes) { nins += nd.vtype == 2; nv += nd.kid >= 0 && nd.vtype != 2; }
            for (auto& tb : T.tabs[ti][pi]) f += table_flops(tb, n) + nins * n * (n + 1.0) + n;
            f += nv * n * (n + 1.0);
        }
        f += 6.0 * n + 4;  // K sum, prefactors
    }
    if (eval_flops) *eval_flops = f;
    if (sample_flops) *sample_flops = 1.5 * M * M + 50.0 * M;  // sector tree adds, log/exp as ~20 each
    return QA_OK;
}

extern "C" int qa_graph_flops_nonzero(const qa_set* s, uint32_t graph, double* eval_flops) {
    if (!s || graph >= s->graphs.size() || !eval_flops) return fail(QA_EINVAL, "bad argument");
    double dense = 0.0;
    if (int rc = qa_graph_flops(s, graph, &dense, nullptr)) return rc;
    const auto& T = s->graphs[graph];
    double fold_dense = 0.0, fold_nz = 0.0;
    for (auto& tv : T.tabs)
        for (auto& pv : tv)
            for (auto& tb : pv)
                for (auto& b : tb.blocks) {
                    fold_dense += 2.0 * ((1 << b.r) - 1);
                    if (tb.has_q) fold_dense += b.r * (2.0 * ((1 << (b.r > 0 ? b.r - 1 : 0)) - 1) + 2);
                    for (double x : b.coef) fold_nz += 2.0 * (x != 0.0);
                }
    *eval_flops = dense - fold_dense + fold_nz;
    return QA_OK;
}

// Budgets across graphs from a pilot (Neyman allocation: the variance of the
// set total, sum mu_g^2 sigma_g^2 / N_g, is smallest at a fixed cost sum c_g N_g
// when N_g is proportional to mu_g sigma_g / sqrt(c_g)); every graph gets at
// least `floor` samples and the remainder is split by largest remainders.
extern "C" int qa_allocate_budgets(const qa_set* s, const qa_acc* pilot, uint64_t total, uint64_t floor,
                                   uint64_t* out) {
    if (!s || !pilot || !out) return fail(QA_EINVAL, "NULL argument");
    const size_t ng = s->graphs.size();
    if (ng == 0) return QA_OK;
    if (floor > total / ng) return fail(QA_EINVAL, "total below floor * graphs");
    std::vector<double> wt(ng, 0.0);
    double sw = 0.0;
    for (size_t g = 0; g < ng; ++g) {
        const qa_acc& a = pilot[g];
        double sd = 0.0;
        if (a.n >= 2) {
            const double n = (double)a.n, m = (a.s1_hi + a.s1_lo) / n, m2 = (a.s2_hi + a.s2_lo) / n;
            sd = std::sqrt(std::max(0.0, m2 - m * m));
        }
        double fe = 0.0, fs = 0.0;
        qa_graph_flops(s, (uint32_t)g, &fe, &fs);
        wt[g] = s->graphs[g].g.mult * sd / std::sqrt(std::max(1.0, fe + fs));
        sw += wt[g];
    }
    const uint64_t rest = total - floor * ng;
    if (!(sw > 0.0) || !std::isfinite(sw)) {
        for (size_t g = 0; g < ng; ++g) wt[g] = 1.0;
        sw = (double)ng;
    }
    std::vector<std::pair<double, size_t>> rem(ng);
    uint64_t given = 0;
    for (size_t g = 0; g < ng; ++g) {
        const double share = (double)rest * wt[g] / sw;
        const uint64_t base = (uint64_t)std::floor(share);
        out[g] = floor + base;
        given += base;
        rem[g] = {share - (double)base, g};
    }
    // largest remainders first; ties by graph index
    std::stable_sort(rem.begin(), rem.end(), [](const std::pair<double, size_t>& a, const std::pair<double, size_t>& b) {
        return a.first > b.first;
    });
    for (size_t i = 0; given < rest && i < ng; ++i, ++given) out[rem[i].second] += 1;
    return QA_OK;
}

// ---------------------------------------------------------------------------
// estimates: per-graph value and sigma from the sums, set totals, and the
// inverse-variance combination of independent runs

extern "C" int qa_results(const qa_set* s, const qa_acc* acc, qa_result* per_graph, qa_result* total) {
    if (!s || !acc) return fail(QA_EINVAL, "NULL argument");
    const size_t ng = s->graphs.size();
    qa_result tot{};
    double var_tot = 0.0;
    for (size_t g = 0; g < ng; ++g) {
        const qa_acc& a = acc[g];
        const uint64_t N = a.n + a.n_bad;   // a bad point is a drawn sample with w = 0
        if (N < 2) return fail(QA_EINVAL, "graph " + std::to_string(g) + " has fewer than 2 samples");
        const double n = (double)N, mu = (double)s->graphs[g].g.mult;
        const double m1 = (a.s1_hi + a.s1_lo) / n, m2 = (a.s2_hi + a.s2_lo) / n;
        const double var_w = std::max(0.0, m2 - m1 * m1);
        qa_result r{};
        r.mean = m1;
        r.sd = std::sqrt(var_w * n / (n - 1.0));
        r.value = mu * m1;
        r.sigma = mu * std::sqrt(var_w / (n - 1.0));
        r.n = N; r.n_bad = a.n_bad; r.n_flagged = a.n_flagged; r.n_residual = a.n_residual;
        if (per_graph) per_graph[g] = r;
        tot.value += r.value;
        var_tot += r.sigma * r.sigma;
        tot.n += r.n; tot.n_bad += r.n_bad; tot.n_flagged += r.n_flagged; tot.n_residual += r.n_residual;
    }
    tot.sigma = std::sqrt(var_tot);
    tot.mean = tot.value;
    tot.sd = tot.sigma * std::sqrt((double)tot.n);
    if (total) *total = tot;
    return QA_OK;
}

static void dd_add_into(double& hi, double& lo, double bhi, double blo) {
    // two-sum of the high parts, then the low parts (double-double addition)
    const double s = hi + bhi, bb = s - hi, e = (hi - (s - bb)) + (bhi - bb) + lo + blo;
    hi = s + e;
    lo = e - (hi - s);
}

extern "C" int qa_acc_merge(qa_acc* into, const qa_acc* from, size_t n) {
    if (!into || !from) return fail(QA_EINVAL, "NULL argument");
    for (size_t i = 0; i < n; ++i) {
        dd_add_into(into[i].s1_hi, into[i].s1_lo, from[i].s1_hi, from[i].s1_lo);
        dd_add_into(into[i].s2_hi, into[i].s2_lo, from[i].s2_hi, from[i].s2_lo);
        into[i].n += from[i].n;
        into[i].n_flagged += from[i].n_flagged;
        into[i].n_bad += from[i].n_bad;
        into[i].n_residual += from[i].n_residual;
    }
    return QA_OK;
}

extern "C" int qa_combine(const qa_result* runs, size_t nruns, qa_result* out) {
    if (!runs || !out || nruns == 0) return fail(QA_EINVAL, "NULL or empty argument");
    double sw = 0.0, swv = 0.0;
    qa_result r{};
    for (size_t i = 0; i < nruns; ++i) {
        const double s = runs[i].sigma;
        if (!(s > 0.0) || !std::isfinite(s) || !std::isfinite(runs[i].value))
            return fail(QA_EINVAL, "run " + std::to_string(i) + ": sigma must be positive and finite");
        const double w = 1.0 / (s * s);
        sw += w;
        swv += w * runs[i].value;
        r.n += runs[i].n; r.n_bad += runs[i].n_bad; r.n_flagged += runs[i].n_flagged; r.n_residual += runs[i].n_residual;
    }
    r.value = swv / sw;
    r.sigma = 1.0 / std::sqrt(sw);
    r.mean = r.value;
    r.sd = 0.0;
    *out = r;
    return QA_OK;
}

extern "C" int qa_sum_results(const qa_result* parts, size_t nparts, qa_result* out) {
    if (!parts || !out || nparts == 0) return fail(QA_EINVAL, "NULL or empty argument");
    double var = 0.0;
    qa_result r{};
    for (size_t i = 0; i < nparts; ++i) {
        const double s = parts[i].sigma;
        if (!(s >= 0.0) || !std::isfinite(s) || !std::isfinite(parts[i].value))
            return fail(QA_EINVAL, "part " + std::to_string(i) + ": value and sigma must be finite, sigma >= 0");
        r.value += parts[i].value;
        var += s * s;
        r.n += parts[i].n; r.n_bad += parts[i].n_bad; r.n_flagged += parts[i].n_flagged; r.n_residual += parts[i].n_residual;
    }
    r.sigma = std::sqrt(var);
    r.mean = r.value;
    r.sd = r.sigma * std::sqrt((double)r.n);
    *out = r;
    return QA_OK;
}

extern "C" int qa_pdf_create(const qa_set* s, const double* deg, qa_pdf** out) {
    try {
        if (!s || !out) return fail(QA_EINVAL, "NULL argument");
        const size_t ng = s->graphs.size();
        std::vector<size_t> off(ng + 1, 0);
        for (size_t g = 0; g < ng; ++g) off[g + 1] = off[g] + (size_t(1) << (3 * s->graphs[g].g.n));
        if (deg)
            for (size_t g = 0; g < ng; ++g)
                for (size_t x = off[g] + 1; x + 1 < off[g + 1]; ++x)
                    if (!(deg[x] > 0.0) || !std::isfinite(deg[x])) return fail(QA_EINVAL, "Deg entries must be positive");
        auto* p = new qa_pdf;
        p->M.resize(ng);
        p->mb.assign(ng, -1);
        p->deg.resize(ng);
        p->w.resize(ng);
        // graphs are independent: one per host thread at a time
        std::atomic<size_t> next{0};
        std::string err;
        std::mutex mu;
        auto work = [&] {
            for (size_t g; (g = next++) < ng;) {
                try {
                    const int M = 3 * s->graphs[g].g.n;
                    std::vector<double> D;
                    if (deg) {
                        D.assign(deg + off[g], deg + off[g + 1]);
                        D[0] = 0.0; D[(size_t(1) << M) - 1] = 0.0;
                    } else D = default_deg(s->graphs[g].g);
                    p->M[g] = M;
                    p->w[g] = w_table(D, M);
                    p->deg[g] = std::move(D);
                } catch (std::exception& e) { std::lock_guard<std::mutex> l(mu); err = e.what(); }
            }
        };
        const int nt = std::max(1, std::min<int>((int)std::thread::hardware_concurrency(), (int)ng));
        std::vector<std::thread> th;
        for (int t = 1; t < nt; ++t) th.emplace_back(work);
        work();
        for (auto& t : th) t.join();
        if (!err.empty()) { delete p; return fail(QA_ENOMEM, err); }
        *out = p;
        return QA_OK;
    } catch (std::exception& e) { return fail(QA_ENOMEM, e.what()); }
}

void qa_image_forget(const void* s, const void* p);
// 3n-2 variables: Deg'(S') = Deg(expand(S')) over the merged lines (line j
// stands for j (j < b) or j + 1 (j >= b); line a = b - 1 stands for {a, b})
static uint32_t expand_merged(uint32_t Sm, int b) {
    const uint32_t low = Sm & ((1u << b) - 1), high = (Sm >> b) << (b + 1);
    return low | high | (((Sm >> (b - 1)) & 1u) << b);
}

extern "C" int qa_pdf_create_merged(const qa_set* s, const qa_pdf* base, qa_pdf** out) {
    try {
        if (!s || !base || !out) return fail(QA_EINVAL, "NULL argument");
        if (base->M.size() != s->graphs.size()) return fail(QA_EINVAL, "set / pdf mismatch");
        auto* p = new qa_pdf;
        for (size_t gi = 0; gi < s->graphs.size(); ++gi) {
            const Graph& g = s->graphs[gi].g;
            const int M = 3 * g.n, Mm = M - 1, b = g.x;
            if (base->mb[gi] >= 0 || base->M[gi] != M) { delete p; return fail(QA_EINVAL, "base pdf is already merged"); }
            if (b < 1 || b > 2 * g.n - 1) { delete p; return fail(QA_EINVAL, "external vertex without two internal electron lines"); }
            std::vector<double> D(size_t(1) << Mm, 0.0);
            for (uint32_t S = 1; S + 1 < (1u << Mm); ++S) D[S] = base->deg[gi][expand_merged(S, b)];
            p->M.push_back(Mm);
            p->mb.push_back(b);
            p->w.push_back(w_table(D, Mm));
            p->deg.push_back(std::move(D));
        }
        *out = p;
        return QA_OK;
    } catch (std::exception& e) { return fail(QA_ENOMEM, e.what()); }
}

extern "C" int qa_pdf_lines(const qa_pdf* p, uint32_t graph, int* lines) {
    if (!p || graph >= p->M.size() || !lines) return fail(QA_EINVAL, "bad argument");
    *lines = p->M[graph];
    return QA_OK;
}

extern "C" void qa_pdf_destroy(qa_pdf* p) {
    qa_image_forget(nullptr, p);
    delete p;
}

extern "C" int qa_pdf_with(const qa_pdf* base, uint32_t graph, const double* deg, qa_pdf** out) {
    try {
        if (!base || !deg || !out) return fail(QA_EINVAL, "NULL argument");
        if (graph >= base->M.size()) return fail(QA_EINVAL, "bad graph index");
        const int M = base->M[graph];
        std::vector<double> D(deg, deg + (size_t(1) << M));
        for (uint32_t x = 1; x + 1 < (1u << M); ++x)
            if (!(D[x] > 0.0) || !std::isfinite(D[x])) return fail(QA_EINVAL, "Deg entries must be positive and finite");
        D[0] = 0.0; D[(1u << M) - 1] = 0.0;
        auto* p = new qa_pdf(*base);
        p->w[graph] = w_table(D, M);
        p->deg[graph] = std::move(D);
        *out = p;
        return QA_OK;
    } catch (std::exception& e) { return fail(QA_ENOMEM, e.what()); }
}

// One pilot step: a shift per set size, against the size-summed gradient,
// normalised so that the largest shift is `step`.
extern "C" int qa_pdf_tune(const qa_pdf* base, uint32_t graph, const double* grad, double step, double floor,
                           qa_pdf** out, double* theta) {
    if (!base || !grad || !out) return fail(QA_EINVAL, "NULL argument");
    if (graph >= base->M.size()) return fail(QA_EINVAL, "bad graph index");
    if (!(floor > 0.0) || !std::isfinite(step)) return fail(QA_EINVAL, "floor must be positive, step finite");
    const int M = base->M[graph];
    const uint32_t full = (1u << M) - 1;
    std::vector<double> gc(M, 0.0);
    for (uint32_t S = 1; S < full; ++S) {
        if (!std::isfinite(grad[S])) return fail(QA_EINVAL, "gradient is not finite");
        gc[__builtin_popcount(S)] += grad[S];
    }
    double gmax = 0.0;
    for (int c = 1; c < M; ++c) gmax = std::max(gmax, std::fabs(gc[c]));
    std::vector<double> th(M, 0.0);
    if (gmax > 0.0)
        for (int c = 1; c < M; ++c) th[c] = -step * gc[c] / gmax;
    std::vector<double> D = base->deg[graph];
    for (uint32_t S = 1; S < full; ++S) D[S] = std::max(floor, D[S] + th[__builtin_popcount(S)]);
    if (theta) for (int c = 0; c < M; ++c) theta[c] = th[c];
    return qa_pdf_with(base, graph, D.data(), out);
}

// helpers for the device-side entry points (kernels.hip)
const std::vector<double>* qa_pdf_deg(const qa_pdf* p, uint32_t graph) {
    return (p && graph < p->M.size()) ? &p->deg[graph] : nullptr;
}
std::vector<double> qa_pdf_dlogw_vec(const qa_pdf* p, uint32_t graph) { return dlogw(p->deg[graph], p->M[graph]); }


extern "C" int qa_pdf_tables(const qa_pdf* p, uint32_t graph, double* deg, double* w) {
    if (!p || graph >= p->M.size()) return fail(QA_EINVAL, "bad graph index");
    size_t n = size_t(1) << p->M[graph];
    if (deg) std::memcpy(deg, p->deg[graph].data(), n * 8);
    if (w) std::memcpy(w, p->w[graph].data(), n * 8);
    return QA_OK;
}

extern "C" int qa_pdf_dlogw(const qa_pdf* p, uint32_t graph, double* out) {
    if (!p || graph >= p->M.size() || !out) return fail(QA_EINVAL, "bad argument");
    auto d = dlogw(p->deg[graph], p->M[graph]);
    std::memcpy(out, d.data(), d.size() * 8);
    return QA_OK;
}

// ---------------------------------------------------------------------------
// device image

namespace {
struct Packer {
    std::vector<uint8_t> buf;
    uint64_t alloc(size_t bytes, size_t align = 16) {
        size_t off = (buf.size() + align - 1) / align * align;
        buf.resize(off + bytes, 0);
        return off;
    }
    template <class T> T* at(uint64_t off) { return reinterpret_cast<T*>(buf.data() + off); }
};
}  // namespace

static int pack(const qa_set* s, const qa_pdf* p, std::vector<uint8_t>& out) {
    if (!s || !p || p->M.size() != s->graphs.size()) return fail(QA_EINVAL, "set / pdf mismatch");
    Packer P;
    uint64_t h = P.alloc(sizeof(DevHeader), 256);
    uint64_t goff = P.alloc(sizeof(DevGraph) * s->graphs.size(), 256);
    {
        auto* hd = P.at<DevHeader>(h);
        hd->magic = 0x51454441u; hd->version = 1; hd->ngraphs = (uint32_t)s->graphs.size(); hd->graphs_off = goff;
    }
    for (size_t gi = 0; gi < s->graphs.size(); ++gi) {
        const auto& T = s->graphs[gi];
        const int M = 3 * T.g.n, Ms = p->M[gi];
        if (Ms != (p->mb[gi] >= 0 ? M - 1 : M)) return fail(QA_EINVAL, "pdf does not match the set's graphs");
        uint64_t doff = P.alloc(8u << Ms, 256);
        std::memcpy(P.buf.data() + doff, p->deg[gi].data(), 8u << Ms);
        uint64_t woff = P.alloc(8u << Ms, 256);
        std::memcpy(P.buf.data() + woff, p->w[gi].data(), 8u << Ms);
        uint64_t toff = P.alloc(sizeof(DevTerm) * T.terms.size(), 64);
        int npoly_max = 0;
        for (size_t ti = 0; ti < T.terms.size(); ++ti) {
            const auto& pcs = T.pieces[ti];
            uint64_t poff = P.alloc(sizeof(DevPiece) * pcs.size(), 64);
            {
                auto* dt = P.at<DevTerm>(toff + ti * sizeof(DevTerm));
                int nf = __builtin_popcount(T.terms[ti].first);
                dt->sign = ((nf + T.g.n) % 2) ? -1 : 1;
                dt->npieces = (int)pcs.size();
                dt->pieces_off = poff;
            }
            // result slots: free list
            std::vector<int> slot_of(pcs.size(), -1);
            std::vector<int> busy(QA_MAXPOLY, 0);
            auto grab = [&](int w) {
                for (int s0 = 0; s0 + w <= QA_MAXPOLY; ++s0) {
                    bool ok = true;
                    for (int q = 0; q < w; ++q) ok &= !busy[s0 + q];
                    if (ok) { for (int q = 0; q < w; ++q) busy[s0 + q] = 1; return s0; }
                }
                throw std::runtime_error("too many live polynomials");
            };
            for (size_t pi = 0; pi < pcs.size(); ++pi) {
                const Piece& pc = pcs[pi];
                DevPiece dp{};
                dp.op = pc.op;
                dp.nlines = (int)pc.lines.size();
                dp.nchords = (int)pc.chords.size();
                dp.ext = pc.ext;
                if (dp.nlines > QA_MAXL || dp.nchords > QA_MAXC) throw std::runtime_error("piece too large");
                for (int i = 0; i < dp.nlines; ++i) dp.line_id[i] = pc.lines[i];
                for (int c = 0; c < dp.nchords; ++c) {
                    dp.chord_photon[c] = 2 * T.g.n + pc.chords[c][0];
                    dp.chord_lo[c] = pc.chords[c][1];
                    dp.chord_hi[c] = pc.chords[c][2];
                }
                auto piece_of = [&](int sub) {
                    for (size_t q = 0; q < pcs.size(); ++q) if (pcs[q].elem == sub) return (int)q;
                    throw std::runtime_error("child piece missing");
                };
                dp.nins = 0; dp.nvkids = 0;
                for (auto& nd : pc.nodes) {
                    if (nd.kid < 0) continue;
                    int q = piece_of(nd.kid);
                    if (nd.vtype == 2) dp.ins_slot[dp.nins++] = slot_of[q];
                    else dp.vkid_slot[dp.nvkids++] = slot_of[q];
                }
                // children's results are consumed here: free them, then grab ours
                for (auto& nd : pc.nodes) {
                    if (nd.kid < 0) continue;
                    int q = piece_of(nd.kid);
                    int w = pcs[q].op == QA_OP_US ? 2 : 1;
                    for (int z = 0; z < w; ++z) busy[slot_of[q] + z] = 0;
                }
                slot_of[pi] = grab(pc.op == QA_OP_US ? 2 : 1);
                dp.out_slot = slot_of[pi];
                for (int z = 0; z < QA_MAXPOLY; ++z) if (busy[z]) npoly_max = std::max(npoly_max, z + 1);
                const auto& tv = T.tabs[ti][pi];
                dp.ntab = (int)tv.size();
                uint64_t taboff = P.alloc(sizeof(DevTable) * tv.size(), 64);
                dp.tab_off = taboff;
                std::memcpy(P.buf.data() + poff + pi * sizeof(DevPiece), &dp, sizeof dp);
                for (size_t k = 0; k < tv.size(); ++k) {
                    const Table& tb = tv[k];
                    uint64_t hoff = P.alloc(sizeof(DevBlock) * std::max<size_t>(1, tb.blocks.size()), 64);
                    size_t ncoef = 0;
                    for (auto& b : tb.blocks) ncoef += b.coef.size();
                    uint64_t coff = P.alloc(sizeof(qa_coef) * std::max<size_t>(1, ncoef), 256);
                    DevTable dtb{};
                    dtb.nblocks = (int)tb.blocks.size();
                    for (int k = 0, bi = 0; k <= QA_MAXN; ++k) {
                        while (bi < dtb.nblocks && tb.blocks[bi].k < k) ++bi;
                        dtb.kstart[k] = bi;
                    }
                    for (size_t bi = 1; bi < tb.blocks.size(); ++bi)
                        if (tb.blocks[bi].k == tb.blocks[bi - 1].k && tb.blocks[bi].r != tb.blocks[bi - 1].r)
                            throw std::runtime_error("blocks of one k must share r");
                    dtb.has_q = tb.has_q;
                    dtb.denom = 1.0 / tb.scale;
                    dtb.hdr_off = hoff;
                    dtb.coef_off = coff;
                    std::memcpy(P.buf.data() + taboff + k * sizeof(DevTable), &dtb, sizeof dtb);
                    size_t c = 0;
                    // identical coefficient arrays within a table are stored once (a
                    // repeat then hits the scalar cache instead of streaming again)
                    std::map<std::vector<float>, uint32_t> seen;
                    for (size_t bi = 0; bi < tb.blocks.size(); ++bi) {
                        const Block& b = tb.blocks[bi];
                        DevBlock db{};
                        db.k = (uint8_t)b.k; db.r = (uint8_t)b.r; db.coef = (uint32_t)c;
                        auto ins = seen.emplace(b.coef, (uint32_t)c);
                        const bool repeat = !ins.second;
                        if (repeat) db.coef = ins.first->second;
                        double cmax = 0.0;
                        for (double x : b.coef) cmax = std::max(cmax, std::fabs(x));
                        int ce = 0;
                        while (std::ldexp(1.0, ce) < cmax) ++ce;
                        if (ce > 255) throw std::runtime_error("coefficient too large for the block exponent");
                        db.cexp = (uint8_t)ce;
                        std::memcpy(db.bidx, b.bidx, QA_MAXK);
                        std::memcpy(db.aidx, b.aidx, QA_MAXR);
                        for (int i = 0; i < QA_MAXR; ++i)
                            if (i < b.r && b.cidx[i] != b.aidx[i] + (QA_VAR_C - QA_VAR_A))
                                throw std::runtime_error("free slot with A and C of different lines");
                        std::memcpy(P.buf.data() + hoff + bi * sizeof(DevBlock), &db, sizeof db);
                        if (repeat) continue;
                        for (size_t j = 0; j < b.coef.size(); ++j) {
                            const qa_coef v = (qa_coef)b.coef[j];
                            if ((double)v != b.coef[j]) throw std::runtime_error("coefficient not exact in the table format");
                            std::memcpy(P.buf.data() + coff + sizeof(qa_coef) * (c + j), &v, sizeof v);
                        }
                        c += b.coef.size();
                    }
                }
            }
        }
        DevGraph dg{};
        dg.n = T.g.n; dg.M = M; dg.mult = T.g.mult; dg.nterms = (int)T.terms.size();
        dg.deg_off = doff; dg.w_off = woff; dg.terms_off = toff; dg.npoly = std::max(1, npoly_max);
        dg.mb = p->mb[gi];
        std::memcpy(P.buf.data() + goff + gi * sizeof(DevGraph), &dg, sizeof dg);
    }
    out.swap(P.buf);
    return QA_OK;
}

// image cache: the packed bytes for (set, pdf).  Entries are dropped when
// either handle is destroyed (a new handle may reuse the address); an image
// that was uploaded stays alive as long as a device buffer refers to it.
static std::mutex g_pack_mu;
static std::map<std::pair<const void*, const void*>, std::shared_ptr<const std::vector<uint8_t>>> g_images;

std::shared_ptr<const std::vector<uint8_t>> qa_image(const qa_set* s, const qa_pdf* p) {
    std::lock_guard<std::mutex> l(g_pack_mu);
    auto key = std::make_pair((const void*)s, (const void*)p);
    auto it = g_images.find(key);
    if (it != g_images.end()) return it->second;
    auto img = std::make_shared<std::vector<uint8_t>>();
    if (pack(s, p, *img) != QA_OK) return nullptr;
    return g_images[key] = img;
}

void qa_image_forget(const void* s, const void* p) {
    std::lock_guard<std::mutex> l(g_pack_mu);
    for (auto it = g_images.begin(); it != g_images.end();) {
        if (it->first.first == s || it->first.second == p) it = g_images.erase(it); else ++it;
    }
}

extern "C" int qa_device_bytes(const qa_set* s, const qa_pdf* p, size_t* bytes) {
    try {
        if (!bytes) return fail(QA_EINVAL, "NULL bytes");
        auto img = qa_image(s, p);
        if (!img) return QA_EINVAL;
        *bytes = img->size();
        return QA_OK;
    } catch (std::exception& e) { return fail(QA_EINVAL, e.what()); }
}

extern "C" int qa_dirac_trace(const int32_t* sym, int len, double* out) {
    try {
        if (!sym || !out || len < 0 || len > 60) return fail(QA_EINVAL, "bad string");
        *out = (double)dirac_trace(sym, len);
        return QA_OK;
    } catch (std::exception& e) { return fail(QA_EINVAL, e.what()); }
}

// graph / pdf accessors for the launch code
const GraphTables& qa_graph_tables(const qa_set* s, size_t i) { return s->graphs[i]; }
size_t qa_set_size(const qa_set* s) { return s->graphs.size(); }
