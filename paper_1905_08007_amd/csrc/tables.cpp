// Projected-numerator coefficient tables.
//
// The Wick-contracted numerator of a piece is a sum over sets of disjoint
// pairs of its momentum slots (electron lines, plus one pseudo line per
// b-output self-energy insertion, which carries the momentum of the line
// before it); each pair contributes the contraction coefficient Bbar of the
// two lines and a contracted gamma pair; every unpaired slot carries m = 1 or
// A pslash (its share of the external momentum), and for the magnetic
// projection at most one unpaired slot carries C qslash (the q-derivative).
// For each pairing ("block") the table stores, for every choice of the
// unpaired slots, the exact projected trace times a common denominator.
#include <cstdio>
#include <stdexcept>
#include <string>

#include "host.h"

namespace qa {

namespace {

struct ProjTerm {
    int num;          // coefficient times the common denominator
    int prefix[4];
    int nprefix;
    int ext;          // symbol at the external vertex: 0 = pslash, MU label
    bool q;           // Gamma_1 term (one slot carries the derivative gamma)
};

constexpr int LAB_MU = 11, LAB_NU = 12, LAB_PAIR0 = 6;

std::vector<ProjTerm> projector(int op, int opvar, int& denom) {
    std::vector<ProjTerm> t;
    if (op == QA_OP_US) {
        denom = 4;
        if (opvar == 0) t.push_back({1, {}, 0, 0, false});
        else t.push_back({1, {0}, 1, 0, false});
        return t;
    }
    denom = 48;
    ProjTerm Tg{0, {LAB_MU}, 1, LAB_MU, false}, Tp{0, {}, 0, 0, false}, Tpp{0, {0}, 1, 0, false};
    auto add = [&](ProjTerm x, int num) { x.num = num; t.push_back(x); };
    switch (op) {
        case QA_OP_UV: add(Tg, 4); add(Tpp, -4); break;                       // (Tg - Tpp)/12
        case QA_OP_L: add(Tp, 12); add(Tpp, 12); break;                       // (Tp + Tpp)/4
        case QA_OP_LMU: add(Tp, 12); add(Tpp, 16); add(Tg, -4); break;        // (3Tp + 4Tpp - Tg)/12
        case QA_OP_A: {
            add(Tp, -12); add(Tpp, -16); add(Tg, 4);                            // -Tp/4 - Tpp/3 + Tg/12
            // (1/48) Tr[(p+1)(g_mu g_nu - g_nu g_mu)(p+1) Gamma_1]
            for (int sg = 0; sg < 2; ++sg)
                for (int l = 0; l < 2; ++l)
                    for (int r = 0; r < 2; ++r) {
                        ProjTerm x{};
                        x.num = sg ? -1 : 1;
                        x.nprefix = 0;
                        if (l) x.prefix[x.nprefix++] = 0;
                        x.prefix[x.nprefix++] = sg ? LAB_NU : LAB_MU;
                        x.prefix[x.nprefix++] = sg ? LAB_MU : LAB_NU;
                        if (r) x.prefix[x.nprefix++] = 0;
                        x.ext = LAB_MU;
                        x.q = true;
                        t.push_back(x);
                    }
            break;
        }
        default: throw std::runtime_error("projector: bad op");
    }
    return t;
}

void pairings_rec(const std::vector<int>& slots, size_t i, std::vector<int>& used,
                  std::vector<std::pair<int, int>>& cur, std::vector<std::vector<std::pair<int, int>>>& out) {
    while (i < slots.size() && used[i]) ++i;
    if (i == slots.size()) { out.push_back(cur); return; }
    used[i] = 1;
    pairings_rec(slots, i + 1, used, cur, out);                  // slot i unpaired
    for (size_t j = i + 1; j < slots.size(); ++j) {
        if (used[j]) continue;
        used[j] = 1;
        cur.push_back({slots[i], slots[j]});
        pairings_rec(slots, i + 1, used, cur, out);
        cur.pop_back();
        used[j] = 0;
    }
    used[i] = 0;
}

// Trace after the p-slash p-slash = 1 reduction (adjacent, and cyclic at the
// ends).  The spinor-wiring trace is linear in the string length, cheaper than
// any lookup keyed by the string.
long long reduced_trace(const std::vector<int>& in) {
    int red[64];
    int n = 0;
    for (int v : in) {
        if (v == 0 && n > 0 && red[n - 1] == 0) { --n; continue; }
        if (n == 64) throw std::runtime_error("trace: string too long");
        red[n++] = v;
    }
    int lo = 0;
    while (n - lo >= 2 && red[lo] == 0 && red[n - 1] == 0) { ++lo; --n; }
    if ((n - lo) % 2) return 0;
    return dirac_trace(red + lo, n - lo);
}

// coefficients are integers over the table's common denominator; float holds
// them exactly below 2^24, which every table here satisfies
float exact_float(double v) {
    const float f = (float)v;
    if ((double)f != v) throw std::runtime_error("coefficient not exact in float");
    return f;
}

}  // namespace

Table build_table(const Piece& p, int opvar, uint32_t variant, int nloops, int part, int nparts) {
    const int nl = (int)p.lines.size();
    // slots: lines 0..nl-1, then pseudo lines of b-insertions
    std::vector<int> slot_line;
    for (int i = 0; i < nl; ++i) slot_line.push_back(i);
    std::vector<int> pseudo_at(p.nodes.size(), -1);
    int t = 0;
    for (int j = 0; j < (int)p.nodes.size(); ++j) {
        if (p.nodes[j].vtype != 2) continue;
        if (variant >> t & 1) {
            pseudo_at[j] = (int)slot_line.size();
            slot_line.push_back(j - 1);   // momentum of the line entering the insertion
        }
        ++t;
    }
    const int ns = (int)slot_line.size();
    std::vector<int> photon_label(QA_MAXC + 1, 0);
    int denom = 1;
    auto proj = projector(p.op, opvar, denom);
    Table tab;
    tab.scale = 1.0 / denom;
    tab.has_q = p.op == QA_OP_A;

    std::vector<int> slots(ns);
    for (int i = 0; i < ns; ++i) slots[i] = i;
    std::vector<std::vector<std::pair<int, int>>> prs;
    std::vector<int> used(ns, 0);
    std::vector<std::pair<int, int>> cur;
    pairings_rec(slots, 0, used, cur, prs);

    // photon labels 1..5 by order of the piece's chords
    std::vector<int> plab(64, 0);
    for (int c = 0; c < (int)p.chords.size(); ++c) plab[p.chords[c][0]] = 1 + c;

    auto tri = [](int a, int b) { if (a > b) std::swap(a, b); return b * (b + 1) / 2 + a; };

    long long ord = -1;
    for (int kk = 0; kk < nloops; ++kk) {
        for (auto& pr : prs) {
            const int k = (int)pr.size();
            if (k != kk) continue;
            ++ord;
            if (ord % nparts != part) continue;
            std::vector<int> label(ns, 0);       // pair label of paired slots
            for (int q = 0; q < k; ++q) { label[pr[q].first] = LAB_PAIR0 + q; label[pr[q].second] = LAB_PAIR0 + q; }
            std::vector<int> freeS;
            for (int s = 0; s < ns; ++s) if (!label[s]) freeS.push_back(s);
            const int r = (int)freeS.size();
            if (r > QA_MAXR) throw std::runtime_error("too many free slots");
            Block b{};
            b.k = k; b.r = r;
            for (int q = 0; q < k; ++q) b.bidx[q] = (uint8_t)tri(slot_line[pr[q].first], slot_line[pr[q].second]);
            for (int i = 0; i < r; ++i) {
                b.aidx[i] = (uint8_t)(QA_VAR_A + slot_line[freeS[i]]);
                b.cidx[i] = (uint8_t)(QA_VAR_C + slot_line[freeS[i]]);
            }
            const size_t n0 = size_t(1) << r;
            const size_t n1 = tab.has_q && r > 0 ? size_t(r) << (r - 1) : 0;
            b.coef.assign(n0 + n1, 0.0f);
            // choice per slot: -1 m (scalar), 0 pslash, LAB_NU derivative gamma, or the pair label
            // the string after the projector's prefix is the same for every
            // projector term but for the symbol at the external vertex
            std::vector<int> sym, body;
            sym.reserve(64);
            body.reserve(64);
            auto eval = [&](const std::vector<int>& choice, bool qterm) -> double {
                body.clear();
                int ext_at = -1;
                for (int j = (int)p.nodes.size() - 1; j >= 0; --j) {
                    const auto& nd = p.nodes[j];
                    if (nd.vtype == 0) body.push_back(plab[nd.photon]);
                    else if (nd.vtype == 1) { ext_at = (int)body.size(); body.push_back(0); }
                    else if (pseudo_at[j] >= 0) {
                        int c = choice[pseudo_at[j]];
                        if (c >= 0) body.push_back(c);
                    }
                    if (j > 0) {
                        int c = choice[j - 1];
                        if (c >= 0) body.push_back(c);
                    }
                }
                long long acc = 0;
                for (auto& pt : proj) {
                    if (pt.q != qterm) continue;
                    if (ext_at >= 0) body[ext_at] = pt.ext;
                    sym.assign(pt.prefix, pt.prefix + pt.nprefix);
                    sym.insert(sym.end(), body.begin(), body.end());
                    acc += (long long)pt.num * reduced_trace(sym);
                }
                return (double)acc;
            };
            std::vector<int> choice(ns, -1);
            for (int s = 0; s < ns; ++s) if (label[s]) choice[s] = label[s];
            bool any = false;
            for (size_t mask = 0; mask < n0; ++mask) {
                bool ok = true;
                for (int i = 0; i < r; ++i) {
                    int s = freeS[i];
                    bool ps = mask >> i & 1;
                    if (!ps && s >= nl) ok = false;      // pseudo lines carry pslash only
                    choice[s] = ps ? 0 : -1;
                }
                if (!ok) continue;
                double v = eval(choice, false);
                b.coef[mask] = exact_float(v);
                any |= v != 0.0;
            }
            if (tab.has_q) {
                for (int jq = 0; jq < r; ++jq) {
                    for (size_t mask = 0; mask < (size_t(1) << (r - 1)); ++mask) {
                        bool ok = true;
                        int bit = 0;
                        for (int i = 0; i < r; ++i) {
                            int s = freeS[i];
                            if (i == jq) { choice[s] = LAB_NU; continue; }
                            bool ps = mask >> bit & 1;
                            ++bit;
                            if (!ps && s >= nl) ok = false;
                            choice[s] = ps ? 0 : -1;
                        }
                        if (!ok) continue;
                        double v = eval(choice, true);
                        b.coef[n0 + (size_t(jq) << (r - 1)) + mask] = exact_float(v);
                        any |= v != 0.0;
                    }
                }
            }
            if (any) tab.blocks.push_back(std::move(b));
        }
    }
    return tab;
}

}  // namespace qa
