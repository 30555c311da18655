// Host side of the hot path: graph enumeration, UV-divergent subgraphs and
// forests, forest-formula terms and their pieces, Deg / W tables of eq. (1),
// exact Dirac traces (two-component spinor wiring) and the projected-numerator
// coefficient tables that the HIP kernels evaluate.
#include "host.h"

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <numeric>
#include <stdexcept>
#include <thread>

namespace qa {

// ---------------------------------------------------------------------------
// graphs

static void matchings(std::vector<int>& items, std::vector<int>& mate, std::vector<std::vector<int>>& out) {
    if (items.empty()) { out.push_back(mate); return; }
    int a = items[0];
    for (size_t i = 1; i < items.size(); ++i) {
        int b = items[i];
        std::vector<int> rest;
        for (size_t j = 1; j < items.size(); ++j) if (j != i) rest.push_back(items[j]);
        mate[a] = b; mate[b] = a;
        matchings(rest, mate, out);
    }
}

static bool external_leg_se(int n, int x, const std::vector<int>& mate) {
    for (int j = 0; j < x; ++j) {
        bool closed = true;
        for (int s = 0; s <= j && closed; ++s) closed = mate[s] <= j;
        if (closed) return true;
    }
    for (int j = x + 1; j <= 2 * n; ++j) {
        bool closed = true;
        for (int s = j; s <= 2 * n && closed; ++s) closed = mate[s] >= j;
        if (closed) return true;
    }
    return false;
}

std::vector<Graph> enumerate(int n) {
    std::map<std::vector<int>, int> reps;  // key (x, mate...) -> mult
    const int N = 2 * n;
    for (int x = 0; x <= N; ++x) {
        std::vector<int> others;
        for (int s = 0; s <= N; ++s) if (s != x) others.push_back(s);
        std::vector<int> mate(N + 1, 0);
        std::vector<std::vector<int>> all;
        matchings(others, mate, all);
        for (auto& m : all) {
            m[x] = x;
            if (external_leg_se(n, x, m)) continue;
            std::vector<int> k1{x}; k1.insert(k1.end(), m.begin(), m.end());
            std::vector<int> k2{N - x};
            std::vector<int> rm(N + 1);
            for (int s = 0; s <= N; ++s) rm[N - s] = N - m[s];
            k2.insert(k2.end(), rm.begin(), rm.end());
            auto key = std::min(k1, k2);
            reps[key] = (k1 == k2) ? 1 : 2;
        }
    }
    std::vector<Graph> out;
    for (auto& kv : reps) {
        Graph g{};
        g.n = n;
        g.x = kv.first[0];
        for (int s = 0; s <= N; ++s) g.mate[s] = kv.first[1 + s];
        g.mult = kv.second;
        int k = 0, l = 0, r = 0;
        for (int s = 0; s <= N; ++s) {
            if (s == g.x || g.mate[s] < s) continue;
            int a = s, b = g.mate[s];
            if (a < g.x && g.x < b) ++k; else if (b < g.x) ++l; else ++r;
        }
        g.cls[0] = k; g.cls[1] = std::max(l, r); g.cls[2] = std::min(l, r);
        out.push_back(g);
    }
    return out;
}

std::vector<std::pair<int, int>> chords(const Graph& g) {
    std::vector<std::pair<int, int>> c;
    for (int s = 0; s <= 2 * g.n; ++s)
        if (s != g.x && g.mate[s] > s) c.push_back({s, g.mate[s]});
    return c;
}

std::vector<Sub> subgraphs(const Graph& g) {
    const int N = 2 * g.n;
    auto ch = chords(g);
    std::vector<Sub> out;
    for (int lo = 0; lo <= N; ++lo)
        for (int hi = lo + 1; hi <= N; ++hi) {
            if (lo == 0 && hi == N) continue;
            int ext = 0;
            for (auto& c : ch) ext += ((lo <= c.first && c.first <= hi) != (lo <= c.second && c.second <= hi));
            bool hx = lo <= g.x && g.x <= hi;
            ext += hx;
            if (ext > 1) continue;
            bool ok = true;
            for (int i = lo; i < hi && ok; ++i) {
                bool spanned = false;
                for (auto& c : ch) spanned |= (lo <= c.first && c.first <= i && i + 1 <= c.second && c.second <= hi);
                ok = spanned;
            }
            if (!ok) continue;
            out.push_back(Sub{lo, hi, ext == 1 ? 0 : 1, hx});
        }
    return out;
}

static bool compatible(const Sub& a, const Sub& b) {
    bool nested = (a.lo <= b.lo && b.hi <= a.hi) || (b.lo <= a.lo && a.hi <= b.hi);
    return nested || a.hi < b.lo || b.hi < a.lo;
}

std::vector<uint32_t> forests(const std::vector<Sub>& subs) {
    std::vector<uint32_t> out;
    const int k = (int)subs.size();
    for (uint32_t mask = 0; mask < (1u << k); ++mask) {
        bool ok = true;
        for (int i = 0; i < k && ok; ++i)
            if (mask >> i & 1)
                for (int j = i + 1; j < k && ok; ++j)
                    if (mask >> j & 1) ok = compatible(subs[i], subs[j]);
        if (ok) out.push_back(mask);
    }
    return out;
}

// ---------------------------------------------------------------------------
// terms and pieces

static bool strictly_inside(const Sub& t, const Sub& s) {
    return s.lo <= t.lo && t.hi <= s.hi && !(t.lo == s.lo && t.hi == s.hi);
}

std::vector<std::pair<uint32_t, int>> terms(const std::vector<Sub>& subs) {
    std::vector<std::pair<uint32_t, int>> out;
    for (uint32_t mask : forests(subs)) {
        out.push_back({mask, -1});
        for (int i = 0; i < (int)subs.size(); ++i)
            if ((mask >> i & 1) && subs[i].has_x) out.push_back({mask, i});
    }
    return out;
}

// Reduced graph of element e (index -1 = G) with its maximal sub-elements of
// the forest contracted; op is assigned by the caller.
static Piece make_piece(const Graph& g, const std::vector<Sub>& subs, int e, uint32_t mask) {
    Sub E = e < 0 ? Sub{0, 2 * g.n, 0, true} : subs[e];
    std::vector<int> inner;
    for (int i = 0; i < (int)subs.size(); ++i)
        if ((mask >> i & 1) && i != e && strictly_inside(subs[i], E)) inner.push_back(i);
    std::vector<int> kids;
    for (int i : inner) {
        bool maximal = true;
        for (int j : inner) if (j != i && strictly_inside(subs[i], subs[j])) maximal = false;
        if (maximal) kids.push_back(i);
    }
    auto ch = chords(g);
    std::vector<int> photon_of(2 * g.n + 1, -1);
    for (int a = 0; a < (int)ch.size(); ++a) { photon_of[ch[a].first] = a; photon_of[ch[a].second] = a; }
    Piece p;
    p.elem = e; p.lo = E.lo; p.hi = E.hi; p.kids = kids;
    std::vector<int> node_of(2 * g.n + 1, -1);
    for (int s = E.lo; s <= E.hi;) {
        int kid = -1;
        for (int k : kids) if (subs[k].lo == s) kid = k;
        Piece::Node nd{};
        if (kid >= 0) {
            for (int t = subs[kid].lo; t <= subs[kid].hi; ++t) node_of[t] = (int)p.nodes.size();
            nd.kid = kid; nd.slot = -1;
            p.nodes.push_back(nd);
            s = subs[kid].hi + 1;
        } else {
            node_of[s] = (int)p.nodes.size();
            nd.kid = -1; nd.slot = s;
            p.nodes.push_back(nd);
            ++s;
        }
    }
    auto inside = [&](int t) { return E.lo <= t && t <= E.hi; };
    std::vector<int> seen;
    for (int j = 0; j < (int)p.nodes.size(); ++j) {
        auto& nd = p.nodes[j];
        int partner = -1, ph = -1;
        if (nd.kid < 0) {
            int s = nd.slot;
            if (s == g.x) { nd.vtype = 1; continue; }
            ph = photon_of[s]; partner = g.mate[s];
        } else {
            const Sub& k = subs[nd.kid];
            if (k.kind == 1) { nd.vtype = 2; continue; }
            if (k.has_x) { nd.vtype = 1; continue; }
            for (int a = 0; a < (int)ch.size(); ++a) {
                bool iu = k.lo <= ch[a].first && ch[a].first <= k.hi;
                bool iv = k.lo <= ch[a].second && ch[a].second <= k.hi;
                if (iu != iv) { ph = a; partner = iu ? ch[a].second : ch[a].first; }
            }
        }
        if (!inside(partner)) { nd.vtype = 1; continue; }
        nd.vtype = 0; nd.photon = ph;
        if (std::find(seen.begin(), seen.end(), ph) == seen.end()) {
            seen.push_back(ph);
            int j2 = node_of[partner];
            p.chords.push_back({ph, std::min(j, j2), std::max(j, j2)});
        }
    }
    for (int j = 0; j + 1 < (int)p.nodes.size(); ++j) {
        auto& nd = p.nodes[j];
        p.lines.push_back(nd.kid < 0 ? nd.slot : subs[nd.kid].hi);
    }
    p.ext = -1;
    for (int j = 0; j < (int)p.nodes.size(); ++j) if (p.nodes[j].vtype == 1) p.ext = j;
    return p;
}

std::vector<Piece> term_pieces(const Graph& g, const std::vector<Sub>& subs, uint32_t mask, int apos) {
    std::vector<int> elems{-1};
    for (int i = 0; i < (int)subs.size(); ++i) if (mask >> i & 1) elems.push_back(i);
    std::vector<Piece> out;
    for (int e : elems) {
        Piece p = make_piece(g, subs, e, mask);
        if (e < 0) p.op = apos < 0 ? QA_OP_A : QA_OP_LMU;
        else if (subs[e].has_x) {
            if (e == apos) p.op = QA_OP_A;
            else if (apos >= 0 && strictly_inside(subs[apos], subs[e])) p.op = QA_OP_L;
            else p.op = QA_OP_UV;
        } else p.op = subs[e].kind == 0 ? QA_OP_UV : QA_OP_US;
        out.push_back(std::move(p));
    }
    std::stable_sort(out.begin(), out.end(), [](const Piece& a, const Piece& b) {
        return (a.hi - a.lo) < (b.hi - b.lo);
    });
    return out;
}

// ---------------------------------------------------------------------------
// Deg and W

// cyclomatic number (edges - vertices + components) of the edges of a piece
// whose line ids are in the set c; the piece's nodes are numbered 0..nodes-1
struct PieceEdges {
    int ne = 0;
    int id[2 * QA_MAXL], a[2 * QA_MAXL], b[2 * QA_MAXL];
};

static int cyclomatic(const PieceEdges& E, uint32_t c) {
    int par[2 * QA_MAXL + 2];
    uint32_t touched = 0;
    int edges = 0, merges = 0;
    for (int e = 0; e < E.ne; ++e) {
        if (!(c >> E.id[e] & 1)) continue;
        ++edges;
        int x = E.a[e], y = E.b[e];
        if (!(touched >> x & 1)) { touched |= 1u << x; par[x] = x; }
        if (!(touched >> y & 1)) { touched |= 1u << y; par[y] = y; }
        while (par[x] != x) x = par[x] = par[par[x]];
        while (par[y] != y) y = par[y] = par[par[y]];
        if (x != y) { par[x] = y; ++merges; }
    }
    // vertices - components = merges
    return edges - merges;
}

std::vector<double> default_deg(const Graph& g) {
    const int n = g.n, M = 3 * n;
    const uint32_t full = (1u << M) - 1;
    auto subs = subgraphs(g);
    auto ch = chords(g);
    // reduced-graph edge lists of every forest: (line id, node a, node b)
    std::vector<std::vector<PieceEdges>> structs;
    for (uint32_t mask : forests(subs)) {
        std::vector<PieceEdges> st;
        for (auto& p : term_pieces(g, subs, mask, -1)) {
            PieceEdges E;
            auto add = [&](int id, int a, int b) {
                if (E.ne == 2 * QA_MAXL || a >= 2 * QA_MAXL + 2 || b >= 2 * QA_MAXL + 2)
                    throw std::runtime_error("default_deg: piece too large");
                E.id[E.ne] = id; E.a[E.ne] = a; E.b[E.ne] = b; ++E.ne;
            };
            for (int j = 0; j < (int)p.lines.size(); ++j) add(p.lines[j], j, j + 1);
            for (auto& c : p.chords) add(2 * n + c[0], c[1], c[2]);
            st.push_back(E);
        }
        structs.push_back(st);
    }
    std::vector<double> D(size_t(1) << M, 0.0);
    for (uint32_t s = 1; s < full; ++s) {
        uint32_t c = s;
        for (int a = 0; a < (int)ch.size(); ++a) {
            bool all = true;
            for (int e = ch[a].first; e < ch[a].second; ++e) all &= (c >> e & 1) != 0;
            if (all) c |= 1u << (2 * n + a);
        }
        int nel = 0, nph = 0;
        for (int i = 0; i < M; ++i) if (c >> i & 1) (i < 2 * n ? nel : nph)++;
        double best = 1e300;
        for (auto& st : structs) {
            int h = 0;
            for (auto& E : st) h += cyclomatic(E, c);
            best = std::min(best, -(2.0 * h - nph - 0.5 * nel));
        }
        D[s] = std::max(0.5, best);
    }
    return D;
}

std::vector<double> w_table(const std::vector<double>& D, int M) {
    const uint32_t full = (1u << M) - 1;
    std::vector<double> W(size_t(1) << M, 0.0);
    for (uint32_t s = 1; s <= full; ++s) {
        if (__builtin_popcount(s) == 1) { W[s] = 1.0 / D[s]; continue; }
        double tot = 0.0;
        for (uint32_t t = s; t; t &= t - 1) tot += W[s ^ (t & (0u - t))];
        W[s] = (s == full) ? tot : tot / D[s];
    }
    return W;
}

std::vector<double> dlogw(const std::vector<double>& D, int M) {
    auto W = w_table(D, M);
    const uint32_t full = (1u << M) - 1;
    std::vector<double> Wb(W.size(), 0.0), Db(W.size(), 0.0);
    Wb[full] = 1.0 / W[full];
    for (uint32_t s = full; s >= 1; --s) {
        if (Wb[s] != 0.0) {
            if (s != full) Db[s] += Wb[s] * (-W[s] / D[s]);
            if (__builtin_popcount(s) > 1) {
                double sc = (s == full) ? Wb[s] : Wb[s] / D[s];
                for (uint32_t t = s; t; t &= t - 1) Wb[s ^ (t & (0u - t))] += sc;
            }
        }
        if (s == 1) break;
    }
    return Db;
}

// ---------------------------------------------------------------------------
// Dirac traces by two-component spinor wiring.
//
// Chiral representation, rest frame p = (1, 0, 0, 0): every symbol (gamma or
// p-slash) flips chirality, so the 2x2 block of symbol i is sigma^mu or
// sigmabar^mu according to the parity of i, and p-slash is the identity.  A
// contracted pair (i, j) of opposite kinds (odd j - i) is
//   sigma^mu_{a_i b_i} sigmabar_mu{}_{a_j b_j} = 2 delta_{a_i b_j} delta_{a_j b_i},
// and of equal kinds (even j - i)
//   sigma^mu_{a_i b_i} sigma_mu{}_{a_j b_j}   = 2 eps_{a_i a_j} eps_{b_i b_j}.
// With matrix products linking b_i to a_{i+1}, the index network is a union
// of cycles; a cycle carrying q eps-links traversed with net sign s
// contributes tr(s eps^q) = 0 (q odd) or 2 s (-1)^(q/2).  Both chiralities
// give the same value, so Tr = 2 * 2^pairs * prod over cycles.

// labels of contracted pairs: 1..kMaxLabel-1 (photons, Wick pairs, projector indices)
constexpr int kMaxLabel = 32;

long long dirac_trace(const int* sym, int L) {
    if (L == 0) return 4;
    if (L % 2) return 0;
    if (L > 62) throw std::runtime_error("dirac_trace: string too long");
    int first[kMaxLabel];
    for (int l = 0; l < kMaxLabel; ++l) first[l] = -1;
    uint8_t partner[128];
    int8_t eps[128];   // 0: delta link; +1 / -1: eps link traversed forward / backward from this node
    int nch = 0;
    for (int i = 0; i < L; ++i) {
        const int s = sym[i];
        if (s <= 0) {
            partner[2 * i] = (uint8_t)(2 * i + 1); partner[2 * i + 1] = (uint8_t)(2 * i);
            eps[2 * i] = eps[2 * i + 1] = 0;
            continue;
        }
        if (s >= kMaxLabel) throw std::runtime_error("dirac_trace: label too large");
        if (first[s] < 0) { first[s] = i; continue; }
        const int a = first[s], b = i;
        first[s] = -2;
        ++nch;
        if ((b - a) % 2) {
            partner[2 * a] = (uint8_t)(2 * b + 1); partner[2 * b + 1] = (uint8_t)(2 * a);
            partner[2 * b] = (uint8_t)(2 * a + 1); partner[2 * a + 1] = (uint8_t)(2 * b);
            eps[2 * a] = eps[2 * b + 1] = eps[2 * b] = eps[2 * a + 1] = 0;
        } else {
            partner[2 * a] = (uint8_t)(2 * b); partner[2 * b] = (uint8_t)(2 * a);
            partner[2 * a + 1] = (uint8_t)(2 * b + 1); partner[2 * b + 1] = (uint8_t)(2 * a + 1);
            eps[2 * a] = 1; eps[2 * b] = -1;
            eps[2 * a + 1] = 1; eps[2 * b + 1] = -1;
        }
    }
    for (int l = 0; l < kMaxLabel; ++l)
        if (first[l] >= 0) throw std::runtime_error("dirac_trace: unpaired label");
    uint8_t chain[128];
    for (int i = 0; i < L; ++i) {
        const int b = 2 * i + 1, a = 2 * ((i + 1) % L);
        chain[b] = (uint8_t)a; chain[a] = (uint8_t)b;
    }
    uint64_t vis0 = 0, vis1 = 0;
    long long val = 1;
    for (int v = 0; v < 2 * L; ++v) {
        const bool seen = v < 64 ? (vis0 >> v & 1) : (vis1 >> (v - 64) & 1);
        if (seen) continue;
        int q = 0, sg = 1;
        int u = v;
        do {
            if (u < 64) vis0 |= 1ull << u; else vis1 |= 1ull << (u - 64);
            const int w = chain[u];
            if (w < 64) vis0 |= 1ull << w; else vis1 |= 1ull << (w - 64);
            if (eps[w]) { ++q; sg *= eps[w]; }
            u = partner[w];
        } while (u != v);
        if (q % 2) return 0;
        val *= 2 * sg * ((q / 2) % 2 ? -1 : 1);
    }
    return 2 * val * (1LL << nch);
}

}  // namespace qa
