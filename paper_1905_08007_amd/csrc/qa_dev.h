// Device image format shared by the host table builder and the HIP kernels.
#pragma once
#include <stdint.h>

#define QA_MAXN 5          // loops
#define QA_MAXM 15         // lines = 3n
#define QA_MAXL 10         // electron lines of a piece
#define QA_MAXC 5          // chords (loops) of a piece
#define QA_MAXR 12         // free slots of a pairing block
#define QA_MAXK 5          // pairs of a block
#define QA_NVAR 75         // per-lane variables: Bbar[55] A[10] C[10]
#define QA_VAR_A 55
#define QA_VAR_C 65
#define QA_MAXPOLY 16      // live piece-result polynomials per term

// The device image is read-only for every kernel: device code reads it
// through the constant address space, so that wave-uniform reads become
// scalar loads even in kernels that also store to global memory.
#if defined(__HIP_DEVICE_COMPILE__)
#define QA_RO __attribute__((address_space(4)))
#else
#define QA_RO
#endif

enum { QA_OP_A = 0, QA_OP_LMU = 1, QA_OP_L = 2, QA_OP_UV = 3, QA_OP_US = 4 };

struct DevHeader {
    uint32_t magic, version, ngraphs, pad;
    uint64_t graphs_off;
};

struct DevGraph {
    int32_t n, M, mult, nterms;
    uint64_t deg_off, w_off;    // double[2^Ms], Ms = M (mb < 0) or M - 1 (merged form)
    uint64_t terms_off;         // DevTerm[nterms]
    int32_t npoly;              // LDS polynomial slots used by any term
    int32_t mb;                 // merged form: line b = x of the merged pair (a = b - 1, b); -1: all M lines sampled
};

struct DevTerm {
    int32_t sign;               // (-1)^(|F|-1) * (-1)^n
    int32_t npieces;            // children first; the last piece is the whole graph
    uint64_t pieces_off;        // DevPiece[npieces]
};

struct DevPiece {
    int32_t op;
    int32_t nlines, nchords, ext;          // ext: node index (lines before it carry -q/2) or -1
    int32_t line_id[QA_MAXL];
    int32_t chord_photon[QA_MAXC], chord_lo[QA_MAXC], chord_hi[QA_MAXC];
    int32_t nins, ins_slot[4];             // result slots of the self-energy children (a at s, b at s+1)
    int32_t nvkids, vkid_slot[8];          // result slots of the vertex children
    int32_t out_slot;                      // result slot(s) of this piece
    int32_t ntab;                          // (op == US ? 2 : 1) << nins; index = opvar * 2^nins + variant
    uint64_t tab_off;                      // DevTable[ntab]
};

// Coefficient tables hold integers (numerators over the table's common
// denominator) of at most 24 bits, so float stores them exactly and halves
// the scalar-load stream of the evaluators; the packer checks exactness.
typedef float qa_coef;

struct DevTable {
    int32_t nblocks;
    int32_t has_q;                         // Gamma_1 part present (A projector)
    int32_t kstart[QA_MAXN + 1];           // blocks with k pairs: [kstart[k], kstart[k+1])
    int32_t pad;
    double denom;                          // common denominator of the integer coefficients
    uint64_t hdr_off;                      // DevBlock[nblocks], sorted by k
    uint64_t coef_off;                     // qa_coef coefficients, blocks back to back
};

struct DevBlock {
    uint8_t k, r, cexp, pad1;              // cexp: 2^cexp >= max |coefficient| of the block
    uint32_t coef;                         // offset (in coefficients) from the table's coef_off
    uint8_t bidx[QA_MAXK];                 // variable indices of the k pair factors
    uint8_t aidx[QA_MAXR];                 // variable indices of A for the r free slots; the
                                           // slot's C is at aidx + (QA_VAR_C - QA_VAR_A)
    uint8_t pad2[7];                       // 32 bytes: one scalar load
};
