// Internal host-side structures of the hot-path library.
#pragma once
#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "qa_dev.h"

namespace qa {

struct Graph {
    int n, x;
    int mate[12];
    int mult;
    int cls[3];
};

struct Sub {
    int lo, hi;
    int kind;      // 0 vertex-like, 1 self-energy-like
    bool has_x;
};

struct Piece {
    struct Node {
        int slot;    // original slot, or -1 for a contracted child
        int kid;     // subgraph index of the contracted child, or -1
        int vtype;   // 0 photon vertex, 1 external vertex, 2 self-energy insertion
        int photon;
    };
    int op = 0;
    int elem = -1, lo = 0, hi = 0;
    std::vector<int> kids;
    std::vector<Node> nodes;
    std::vector<int> lines;                    // G electron line ids between consecutive nodes
    std::vector<std::array<int, 3>> chords;    // photon id, node lo, node hi (span = lines lo..hi-1)
    int ext = -1;
};

std::vector<Graph> enumerate(int n);
std::vector<std::pair<int, int>> chords(const Graph& g);
std::vector<Sub> subgraphs(const Graph& g);
std::vector<uint32_t> forests(const std::vector<Sub>& subs);
std::vector<std::pair<uint32_t, int>> terms(const std::vector<Sub>& subs);
std::vector<Piece> term_pieces(const Graph& g, const std::vector<Sub>& subs, uint32_t mask, int apos);
std::vector<double> default_deg(const Graph& g);
std::vector<double> w_table(const std::vector<double>& D, int M);
std::vector<double> dlogw(const std::vector<double>& D, int M);
long long dirac_trace(const int* sym, int L);

// coefficient tables of one piece / operator output / self-energy variant
struct Block {
    int k, r;
    uint8_t bidx[QA_MAXK], aidx[QA_MAXR], cidx[QA_MAXR];
    std::vector<float> coef;    // 2^r (Gamma_0) then r * 2^(r-1) (Gamma_1) when has_q; integers
                                // below 2^24, exact in float (checked when the table is built)
};
struct Table {
    bool has_q = false;
    double scale = 1.0;
    std::vector<Block> blocks;  // sorted by k
};
// part / nparts: build only the blocks whose index is part mod nparts
Table build_table(const Piece& p, int opvar, uint32_t variant, int nloops, int part = 0, int nparts = 1);

struct GraphTables {
    Graph g;
    std::vector<Sub> subs;
    std::vector<uint32_t> forests;
    std::vector<std::pair<uint32_t, int>> terms;
    std::vector<std::vector<Piece>> pieces;          // per term
    std::vector<std::vector<std::vector<Table>>> tabs;  // per term, per piece, per (opvar, variant)
};

}  // namespace qa
