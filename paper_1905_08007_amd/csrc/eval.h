// Integrand evaluator core: graph polynomials of each piece, projected
// numerator tables, forest-term combination.  Templated on the number type.
#pragma once
#include "numeric.h"
#include "qa_dev.h"
#include <stddef.h>
#include <type_traits>

// lane view of per-lane scratch laid out [element][lane]
template <class T> struct LV {
    T* p;
    int stride;
    QA_HD T& operator[](int i) const { return p[i * stride]; }
};
template <class T> struct CLV {
    const T* p;
    int stride;
    QA_HD const T& operator[](int i) const { return p[i * stride]; }
};

// Per-lane geometry variables of the current piece in two regions, each laid
// out [element][lane]: the contraction matrix Bbar (indices < QA_VAR_A) and the
// flows A, C (indices QA_VAR_A ..).  The flows are read about twice as often;
// the fused pass keeps them in LDS and Bbar in global memory.
template <class T> struct VV {
    T* pb;
    int sb;
    T* pa;
    int sa;
    QA_HD T& bb(int i) const { return pb[i * sb]; }
    QA_HD T& ac(int i) const { return pa[(i - QA_VAR_A) * sa]; }
};
template <class T> QA_HD VV<T> vv(T* p, int stride) { return VV<T>{p, stride, p + QA_VAR_A * stride, stride}; }

QA_HD int tri_idx(int a, int b) { return a <= b ? b * (b + 1) / 2 + a : a * (a + 1) / 2 + b; }

// store a geometry output; in the comparing pass measure |double - dd| / (u |dd|)
template <class S, class T, bool Cmp> QA_HD void geo_out(S& dst, const T& x, double& cond);
template <> QA_HD void geo_out<double, double, false>(double& dst, const double& x, double&) { dst = x; }
template <> QA_HD void geo_out<DD, double, false>(DD& dst, const double& x, double&) { dst = dd(x); }
template <> QA_HD void geo_out<double, DD, true>(double& dst, const DD& x, double& cond) {
    const double v = x.hi + x.lo;
    cond = fmax(cond, fabs(dst - v) / (0x1p-53 * fabs(v)));
    dst = v;
}
template <> QA_HD void geo_out<DD, DD, true>(DD& dst, const DD& x, double& cond) {
    const double v = x.hi + x.lo;
    cond = fmax(cond, fabs(dst.hi - v) / (0x1p-53 * fabs(v)));
    dst = x;
}
template <class T, bool Cmp> QA_HD void geo_scalar(DD& dst, const T& x, double& cond);
template <> QA_HD void geo_scalar<double, false>(DD& dst, const double& x, double&) { dst = dd(x); }
template <> QA_HD void geo_scalar<DD, true>(DD& dst, const DD& x, double& cond) {
    const double v = x.hi + x.lo;
    cond = fmax(cond, fabs(dst.hi - v) / (0x1p-53 * fabs(v)));
    dst = x;
}

// ---------------------------------------------------------------------------
// graph polynomials of a piece: loop matrix M (chord basis), U = det M,
// Wick contraction matrix Bbar_ij = eta_i^T M^-1 eta_j, flows A (external p
// from the first to the last node) and C (q entering at the external node,
// -1/2 leaving at each end), V = sum_i z_i (1 - A_i).
// Computed in T (double or double-double); results stored as S (double or
// double-double).  With Cmp = true (T = DD) each output is compared with the
// value already stored by a plain-double pass: cond receives the largest
// discrepancy in units of the double round-off, i.e. an estimate of the
// polynomials' conditioning (the double-double error is about cond * 2^-104).
template <class S, class T, int L, bool Cmp>
QA_HD void geometry_L(const QA_RO DevPiece& pc, CLV<double> z, VV<S> vars, DD& Uo, DD& Vo, double& cond) {
    T U, V;
    const int nl = pc.nlines;
    T zl[QA_MAXL];
#pragma unroll
    for (int i = 0; i < QA_MAXL; ++i) zl[i] = from_d<T>(i < nl ? z[pc.line_id[i]] : 0.0);
    bool in[QA_MAXL][L];
#pragma unroll
    for (int i = 0; i < QA_MAXL; ++i)
#pragma unroll
        for (int c = 0; c < L; ++c) in[i][c] = i >= pc.chord_lo[c] && i < pc.chord_hi[c];
    T Mx[L][L];
    T jv[L];
#pragma unroll
    for (int c = 0; c < L; ++c) {
#pragma unroll
        for (int d = c; d < L; ++d) {
            T s = from_d<T>(0.0);
#pragma unroll
            for (int i = 0; i < QA_MAXL; ++i)
                if (in[i][c] && in[i][d]) s += zl[i];
            if (c == d) { jv[c] = s; s += from_d<T>(z[pc.chord_photon[c]]); }
            Mx[c][d] = s;
            Mx[d][c] = s;
        }
    }
    // Cholesky M = R R^T (R lower triangular), positive definite for z > 0
    T R[L][L];
    double dmin = 1e300, dmax = 0.0;
#pragma unroll
    for (int c = 0; c < L; ++c) {
#pragma unroll
        for (int d = 0; d <= c; ++d) {
            T s = Mx[c][d];
#pragma unroll
            for (int e = 0; e < d; ++e) s = s - R[c][e] * R[d][e];
            if (c == d) {
                dmax = fmax(dmax, val(Mx[c][c]));
                dmin = fmin(dmin, val(s));
                R[c][c] = sqrt_(s);
            } else {
                R[c][d] = s / R[d][d];
            }
        }
    }
    (void)dmax;
    (void)dmin;
    U = from_d<T>(1.0);
#pragma unroll
    for (int c = 0; c < L; ++c) U = U * (R[c][c] * R[c][c]);
    // inverse of R, then M^-1 = R^-T R^-1
    T Ri[L][L];
#pragma unroll
    for (int c = 0; c < L; ++c) {
        Ri[c][c] = from_d<T>(1.0) / R[c][c];
#pragma unroll
        for (int d = 0; d < c; ++d) {
            T s = from_d<T>(0.0);
#pragma unroll
            for (int e = d; e < c; ++e) s = s + R[c][e] * Ri[e][d];
            Ri[c][d] = -(s / R[c][c]);
        }
    }
    T Mi[L][L];
#pragma unroll
    for (int c = 0; c < L; ++c)
#pragma unroll
        for (int d = c; d < L; ++d) {
            T s = from_d<T>(0.0);
#pragma unroll
            for (int e = d; e < L; ++e) s = s + Ri[e][c] * Ri[e][d];
            Mi[c][d] = s;
            Mi[d][c] = s;
        }

    // flows
    T y[L], yq[L], jq[L];
    const bool hq = pc.ext >= 0;
#pragma unroll
    for (int c = 0; c < L; ++c) {
        T s = from_d<T>(0.0);
#pragma unroll
        for (int i = 0; i < QA_MAXL; ++i)
            if (in[i][c]) s += zl[i] * (i < pc.ext ? -0.5 : 0.5);
        jq[c] = s;
    }
#pragma unroll
    for (int c = 0; c < L; ++c) {
        T s = from_d<T>(0.0), sq = from_d<T>(0.0);
#pragma unroll
        for (int d = 0; d < L; ++d) {
            s = s + Mi[c][d] * jv[d];
            sq = sq + Mi[c][d] * jq[d];
        }
        y[c] = s;
        yq[c] = sq;
    }
    V = from_d<T>(0.0);
    T Y[QA_MAXL][L];
#pragma unroll
    for (int i = 0; i < QA_MAXL; ++i) {
        if (i < nl) {
        T a = from_d<T>(1.0), cq = from_d<T>(hq ? (i < pc.ext ? -0.5 : 0.5) : 0.0);
#pragma unroll
        for (int c = 0; c < L; ++c)
            if (in[i][c]) { a = a - y[c]; cq = cq - yq[c]; }
        if (!hq) cq = from_d<T>(0.0);
        geo_out<S, T, Cmp>(vars.ac(QA_VAR_A + i), a, cond);
        geo_out<S, T, Cmp>(vars.ac(QA_VAR_C + i), cq, cond);
        V = V + zl[i] * (from_d<T>(1.0) - a);
#pragma unroll
        for (int d = 0; d < L; ++d) {
            T s = from_d<T>(0.0);
#pragma unroll
            for (int c = 0; c < L; ++c)
                if (in[i][c]) s = s + Mi[c][d];
            Y[i][d] = s;
        }
        }
    }
#pragma unroll
    for (int i = 0; i < QA_MAXL; ++i) {
#pragma unroll
        for (int j = i; j < QA_MAXL; ++j) {
            if (j < nl) {
                T s = from_d<T>(0.0);
#pragma unroll
                for (int d = 0; d < L; ++d)
                    if (in[j][d]) s = s + Y[i][d];
                geo_out<S, T, Cmp>(vars.bb(tri_idx(i, j)), s, cond);
            }
        }
    }
    geo_scalar<T, Cmp>(Uo, U, cond);
    geo_scalar<T, Cmp>(Vo, V, cond);
}

// plain-double pass, then the double-double pass comparing against it
template <class S, int L>
QA_HD void geometry_2(const QA_RO DevPiece& pc, CLV<double> z, VV<S> vars, DD& U, DD& V, double& cond) {
    geometry_L<S, double, L, false>(pc, z, vars, U, V, cond);
    geometry_L<S, DD, L, true>(pc, z, vars, U, V, cond);
}

template <class S>
QA_HD void geometry(const QA_RO DevPiece& pc, CLV<double> z, VV<S> vars, DD& U, DD& V, double& cond) {
    cond = 1.0;
    switch (pc.nchords) {
        case 1: geometry_2<S, 1>(pc, z, vars, U, V, cond); break;
        case 2: geometry_2<S, 2>(pc, z, vars, U, V, cond); break;
        case 3: geometry_2<S, 3>(pc, z, vars, U, V, cond); break;
        case 4: geometry_2<S, 4>(pc, z, vars, U, V, cond); break;
        default: geometry_2<S, 5>(pc, z, vars, U, V, cond); break;
    }
}

// ---------------------------------------------------------------------------
// A block header held in scalar registers: the 32-byte record is read as eight
// wave-uniform words and its byte fields are extracted with scalar shifts
// (a per-lane byte load would stall each block on vector-memory latency).
QA_HD uint32_t uni(uint32_t x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_readfirstlane(x);
#else
    return x;
#endif
}
struct BH {
    uint32_t w[8];
    QA_HD int byte(int o) const { return (int)((w[o >> 2] >> (8 * (o & 3))) & 0xffu); }
    QA_HD int k() const { return byte(0); }
    QA_HD int r() const { return byte(1); }
    QA_HD int cexp() const { return byte(2); }
    QA_HD uint32_t coef() const { return w[1]; }
    QA_HD int bidx(int q) const { return byte(8 + q); }
    QA_HD int aidx(int i) const { return byte(13 + i); }
    QA_HD int cidx(int i) const { return byte(13 + i) + (QA_VAR_C - QA_VAR_A); }
};
static_assert(sizeof(DevBlock) == 32 && offsetof(DevBlock, coef) == 4 && offsetof(DevBlock, bidx) == 8 &&
                  offsetof(DevBlock, aidx) == 13,
              "block header layout");
QA_HD BH load_bh(const QA_RO DevBlock& b) {
    const QA_RO uint32_t* p = reinterpret_cast<const QA_RO uint32_t*>(&b);
    BH h;
#pragma unroll
    for (int i = 0; i < 8; ++i) h.w[i] = uni(p[i]);
    return h;
}

// ---------------------------------------------------------------------------
// multilinear fold: sum_s c[s] prod_{bit i of s} A[map(i)], r <= QA_MAXR, where
// map skips the compile-time index J (J = QA_MAXR: no skip).  Used with the
// free-slot values A of a block; the q-derivative part folds the other slots.
template <int J> QA_HD constexpr int amap(int i) { return i + (i >= J ? 1 : 0); }

// With Abs the leaves are |c[s]| (used with squared slot values for the
// rounding-error estimate).
template <class T, int R, int J, bool Abs = false> struct Fold {
    QA_HD static T run(const QA_RO qa_coef* c, const T* A) {
        return Fold<T, R - 1, J, Abs>::run(c, A) + A[amap<J>(R - 1)] * Fold<T, R - 1, J, Abs>::run(c + (1 << (R - 1)), A);
    }
};
template <class T, int J, bool Abs> struct Fold<T, 0, J, Abs> {
    QA_HD static T run(const QA_RO qa_coef* c, const T*) {
        const double v = (double)c[0];
        return from_d<T>(Abs ? fabs(v) : v);
    }
};

template <class T, int J, bool Abs = false> QA_HD T fold(const QA_RO qa_coef* c, const T* A, int r) {
    switch (r) {
        case 0: return Fold<T, 0, J, Abs>::run(c, A);
        case 1: return Fold<T, 1, J, Abs>::run(c, A);
        case 2: return Fold<T, 2, J, Abs>::run(c, A);
        case 3: return Fold<T, 3, J, Abs>::run(c, A);
        case 4: return Fold<T, 4, J, Abs>::run(c, A);
        default: break;
    }
    // 16-coefficient leaves combined by a carry chain over the high bits
    T acc[QA_MAXR - 4];
    T v = from_d<T>(0.0);
    const int nleaves = 1 << (r - 4);
    for (int leaf = 0; leaf < nleaves; ++leaf) {
        v = Fold<T, 4, J, Abs>::run(c + 16 * leaf, A);
        int b = leaf;
        bool stored = false;
#pragma unroll
        for (int l = 0; l < QA_MAXR - 4; ++l) {
            if (stored || 4 + l >= r) break;
            if ((b & 1) == 0) { acc[l] = v; stored = true; }
            else { v = acc[l] + A[amap<J>(4 + l)] * v; b >>= 1; }
        }
    }
    return v;
}

// sum over the free slot j carrying the q-derivative: C_j * fold(others)
template <class T, class S, int J> struct QTerms {
    QA_HD static void run(T& s, const QA_RO qa_coef* c, const T* A, int r, VV<S> vars, const BH& b) {
        if (J >= r) return;
        const int half = 1 << (r - 1);
        s = s + lift_to<T>(vars.ac(b.cidx(J))) * fold<T, J>(c + (1 << r) + J * half, A, r - 1);
        QTerms<T, S, J + 1>::run(s, c, A, r, vars, b);
    }
};
template <class T, class S> struct QTerms<T, S, QA_MAXR> {
    QA_HD static void run(T&, const QA_RO qa_coef*, const T*, int, VV<S>, const BH&) {}
};

// one block: w * (Gamma_0 fold + Gamma_1 folds)
template <class T, class S>
QA_HD T eval_block(const BH& b, const QA_RO qa_coef* c, VV<S> vars, bool has_q) {
    const int k = b.k(), r = b.r();
    T w = from_d<T>(1.0);
#pragma unroll
    for (int q = 0; q < QA_MAXK; ++q)
        if (q < k) w = w * lift_to<T>(vars.bb(b.bidx(q)));
    T A[QA_MAXR + 1];
#pragma unroll
    for (int i = 0; i < QA_MAXR; ++i) A[i] = i < r ? lift_to<T>(vars.ac(b.aidx(i))) : from_d<T>(0.0);
    A[QA_MAXR] = from_d<T>(0.0);
    T s = fold<T, QA_MAXR>(c, A, r);
    if (has_q) QTerms<T, S, 0>::run(s, c, A, r, vars, b);
    return w * s;
}

// statically sized block (R free slots, R <= QA_STATIC_R): fully unrolled folds
#define QA_STATIC_R 8
template <class T, class S, int R, int J> struct QStatic {
    QA_HD static void run(T& s, const QA_RO qa_coef* c, const T* A, VV<S> vars, const BH& b) {
        s = s + lift_to<T>(vars.ac(b.cidx(J))) * Fold<T, R - 1, J>::run(c + (1 << R) + J * (1 << (R - 1)), A);
        QStatic<T, S, R, J + 1>::run(s, c, A, vars, b);
    }
};
template <class T, class S, int R> struct QStatic<T, S, R, R> {
    QA_HD static void run(T&, const QA_RO qa_coef*, const T*, VV<S>, const BH&) {}
};

template <class T, class S, int R>
QA_HD T block_static(const BH& b, const QA_RO qa_coef* c, VV<S> vars, bool has_q) {
    const int k = b.k();
    T w = from_d<T>(1.0);
#pragma unroll
    for (int q = 0; q < QA_MAXK; ++q)
        if (q < k) w = w * lift_to<T>(vars.bb(b.bidx(q)));
    T A[R + 1];
#pragma unroll
    for (int i = 0; i < R; ++i) A[i] = lift_to<T>(vars.ac(b.aidx(i)));
    A[R] = from_d<T>(0.0);
    T s = Fold<T, R, QA_MAXR>::run(c, A);
    if (has_q) QStatic<T, S, R, 0>::run(s, c, A, vars, b);
    return w * s;
}

// The value fold (leaves c) and the square fold (leaves |c|, slot values
// squared) in one pass, so that each coefficient is converted once and feeds
// both (|.| is a free source modifier of the FMA).
template <int R, int J> struct Fold2 {
    QA_HD static void run(const QA_RO qa_coef* c, const double* A, const double* A2, double& v, double& q) {
        double v0, q0, v1, q1;
        Fold2<R - 1, J>::run(c, A, A2, v0, q0);
        Fold2<R - 1, J>::run(c + (1 << (R - 1)), A, A2, v1, q1);
        v = v0 + A[amap<J>(R - 1)] * v1;
        q = q0 + A2[amap<J>(R - 1)] * q1;
    }
};
template <int J> struct Fold2<0, J> {
    QA_HD static void run(const QA_RO qa_coef* c, const double*, const double*, double& v, double& q) {
        const double x = (double)c[0];
        v = x;
        q = fabs(x);
    }
};
template <int J> QA_HD void fold2(const QA_RO qa_coef* c, const double* A, const double* A2, int r, double& v, double& q) {
    switch (r) {
        case 0: Fold2<0, J>::run(c, A, A2, v, q); return;
        case 1: Fold2<1, J>::run(c, A, A2, v, q); return;
        case 2: Fold2<2, J>::run(c, A, A2, v, q); return;
        case 3: Fold2<3, J>::run(c, A, A2, v, q); return;
        case 4: Fold2<4, J>::run(c, A, A2, v, q); return;
        default: break;
    }
    // 16-coefficient leaves combined by a carry chain over the high bits
    double av[QA_MAXR - 4], aq[QA_MAXR - 4];
    const int nleaves = 1 << (r - 4);
    for (int leaf = 0; leaf < nleaves; ++leaf) {
        Fold2<4, J>::run(c + 16 * leaf, A, A2, v, q);
        int b = leaf;
        bool stored = false;
#pragma unroll
        for (int l = 0; l < QA_MAXR - 4; ++l) {
            if (stored || 4 + l >= r) break;
            if ((b & 1) == 0) {
                av[l] = v;
                aq[l] = q;
                stored = true;
            } else {
                v = av[l] + A[amap<J>(4 + l)] * v;
                q = aq[l] + A2[amap<J>(4 + l)] * q;
                b >>= 1;
            }
        }
    }
}

// sum over the free slot j carrying the q-derivative, value and square folds
template <class S, int J> struct QTermsQ {
    QA_HD static void run(double& s, double& sq, const QA_RO qa_coef* c, const double* A, const double* A2, int r, VV<S> vars,
                          const BH& b) {
        if (J >= r) return;
        const QA_RO qa_coef* cc = c + (1 << r) + J * (1 << (r - 1));
        const double cj = vars.ac(b.cidx(J));
        double fv, fq;
        fold2<J>(cc, A, A2, r - 1, fv, fq);
        s = s + cj * fv;
        sq = sq + (cj * cj) * fq;
        QTermsQ<S, J + 1>::run(s, sq, c, A, A2, r, vars, b);
    }
};
template <class S> struct QTermsQ<S, QA_MAXR> {
    QA_HD static void run(double&, double&, const QA_RO qa_coef*, const double*, const double*, int, VV<S>, const BH&) {}
};

// Block in EQ: the value, and q = 2^cexp * w^2 * sum_s |c_s| m_s^2 >= the sum
// of squares of the block's monomials (m_s: product of the slot values of s;
// 2^cexp >= max |c|).  Both folds share the coefficient loads.
template <class S>
QA_HD EQ eval_block_q(const BH& b, const QA_RO qa_coef* c, VV<S> vars, bool has_q) {
    const int k = b.k(), r = b.r();
    double w = 1.0;
#pragma unroll
    for (int q = 0; q < QA_MAXK; ++q)
        if (q < k) w = w * vars.bb(b.bidx(q));
    double A[QA_MAXR + 1], A2[QA_MAXR + 1];
#pragma unroll
    for (int i = 0; i < QA_MAXR; ++i) {
        A[i] = i < r ? vars.ac(b.aidx(i)) : 0.0;
        A2[i] = A[i] * A[i];
    }
    A[QA_MAXR] = A2[QA_MAXR] = 0.0;
    double s, sq;
    fold2<QA_MAXR>(c, A, A2, r, s, sq);
    if (has_q) QTermsQ<S, 0>::run(s, sq, c, A, A2, r, vars, b);
    return EQ{w * s, ldexp(w * w * sq, b.cexp())};
}

template <class S, int R, int J> struct QStaticQ {
    QA_HD static void run(double& s, double& sq, const QA_RO qa_coef* c, const double* A, const double* A2, VV<S> vars,
                          const BH& b) {
        const double cj = vars.ac(b.cidx(J));
        const QA_RO qa_coef* cc = c + (1 << R) + J * (1 << (R - 1));
        double fv, fq;
        Fold2<R - 1, J>::run(cc, A, A2, fv, fq);
        s = s + cj * fv;
        sq = sq + (cj * cj) * fq;
        QStaticQ<S, R, J + 1>::run(s, sq, c, A, A2, vars, b);
    }
};
template <class S, int R> struct QStaticQ<S, R, R> {
    QA_HD static void run(double&, double&, const QA_RO qa_coef*, const double*, const double*, VV<S>, const BH&) {}
};

template <class S, int R>
QA_HD EQ block_static_q(const BH& b, const QA_RO qa_coef* c, VV<S> vars, bool has_q) {
    const int k = b.k();
    double w = 1.0;
#pragma unroll
    for (int q = 0; q < QA_MAXK; ++q)
        if (q < k) w = w * vars.bb(b.bidx(q));
    double A[R + 1], A2[R + 1];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        A[i] = vars.ac(b.aidx(i));
        A2[i] = A[i] * A[i];
    }
    A[R] = A2[R] = 0.0;
    double s, sq;
    Fold2<R, QA_MAXR>::run(c, A, A2, s, sq);
    if (has_q) QStaticQ<S, R, 0>::run(s, sq, c, A, A2, vars, b);
    return EQ{w * s, ldexp(w * w * sq, b.cexp())};
}
template <class T, class S, int R>
QA_HD T block_any(const BH& b, const QA_RO qa_coef* c, VV<S> vars, bool has_q) {
    if constexpr (std::is_same<T, EQ>::value) return block_static_q<S, R>(b, c, vars, has_q);
    else return block_static<T, S, R>(b, c, vars, has_q);
}

// blocks [b0, b1) all with R free slots, two at a time for instruction-level
// parallelism.  A block's value passes through at most 2 (k + R) + 3 roundings
// (k + R lifted geometry values, the R-level fold, the k-pair product, the
// final product), which acc_add uses for the ER estimate.
template <class T, class S, int R, class AT>
QA_HD void group_static(const QA_RO DevBlock* blocks, int b0, int b1, const QA_RO qa_coef* coefs, VV<S> vars, bool hq, AT& acc) {
    int bi = b0;
    if (bi + 1 < b1) {
        // software pipeline: the next pair's headers are loaded (clamped to the
        // last pair, always in range) before this pair is evaluated, so their
        // latency overlaps this pair's coefficient loads
        BH x = load_bh(blocks[bi]);
        BH y = load_bh(blocks[bi + 1]);
        for (;;) {
            const int nb = bi + 2;
            const int pf = nb + 1 < b1 ? nb : b1 - 2;
            const BH xn = load_bh(blocks[pf]);
            const BH yn = load_bh(blocks[pf + 1]);
            const T vx = block_any<T, S, R>(x, coefs + x.coef(), vars, hq);
            const T vy = block_any<T, S, R>(y, coefs + y.coef(), vars, hq);
            acc_add(acc, vx, 2 * (x.k() + R) + 3);
            acc_add(acc, vy, 2 * (y.k() + R) + 3);
            bi = nb;
            if (bi + 1 >= b1) break;
            x = xn;
            y = yn;
        }
    }
    if (bi < b1) {
        const BH x = load_bh(blocks[bi]);
        acc_add(acc, block_any<T, S, R>(x, coefs + x.coef(), vars, hq), 2 * (x.k() + R) + 3);
    }
}

// Evaluate one coefficient table: poly[k] = (1/denom) * sum over blocks with k
// pairs.  All blocks with the same k have the same number of free slots r.
template <class T, class S>
QA_HD void eval_table(const QA_RO uint8_t* img, const QA_RO DevTable& tb, VV<S> vars, int n, T* poly,
                      int slice = 0, int nslices = 1) {
    using AT = typename Acc<T>::type;
    using BT = typename BlockOf<T>::type;
    const QA_RO DevBlock* blocks = reinterpret_cast<const QA_RO DevBlock*>(img + tb.hdr_off);
    const QA_RO qa_coef* coefs = reinterpret_cast<const QA_RO qa_coef*>(img + tb.coef_off);
    const bool hq = tb.has_q != 0;
#pragma unroll
    for (int k = 0; k < QA_MAXN; ++k) {
        AT acc = acc_zero((AT*)nullptr);
        // slice `slice` of nslices: a contiguous share of each k-range
        const int k0 = tb.kstart[k], k1 = tb.kstart[k + 1];
        const int b0 = k0 + (k1 - k0) * slice / nslices, b1 = k0 + (k1 - k0) * (slice + 1) / nslices;
        if (k < n && b0 < b1) {
            // the double-double path (flagged points only) uses the compact generic loop
            const int rsel = std::is_same<T, DD>::value ? -1 : load_bh(blocks[b0]).r();
            switch (rsel) {
                case 0: group_static<BT, S, 0>(blocks, b0, b1, coefs, vars, hq, acc); break;
                case 1: group_static<BT, S, 1>(blocks, b0, b1, coefs, vars, hq, acc); break;
                case 2: group_static<BT, S, 2>(blocks, b0, b1, coefs, vars, hq, acc); break;
                case 3: group_static<BT, S, 3>(blocks, b0, b1, coefs, vars, hq, acc); break;
                case 4: group_static<BT, S, 4>(blocks, b0, b1, coefs, vars, hq, acc); break;
                case 5: group_static<BT, S, 5>(blocks, b0, b1, coefs, vars, hq, acc); break;
                case 6: group_static<BT, S, 6>(blocks, b0, b1, coefs, vars, hq, acc); break;
                case 8: group_static<BT, S, 8>(blocks, b0, b1, coefs, vars, hq, acc); break;
                default:
                    for (int bi = b0; bi < b1; ++bi) {
                        const BH b = load_bh(blocks[bi]);
                        if constexpr (std::is_same<BT, EQ>::value)
                            acc_add(acc, eval_block_q<S>(b, coefs + b.coef(), vars, hq), 2 * (b.k() + b.r()) + 3);
                        else
                            acc_add(acc, eval_block<BT, S>(b, coefs + b.coef(), vars, hq), 2 * (b.k() + b.r()) + 3);
                    }
            }
        }
        poly[k] = div_den(acc_get(acc), tb.denom);
    }
}

template <class T> QA_HD void poly_mul(T* a, const T* b, int n) {
    T out[QA_MAXN];
#pragma unroll
    for (int i = 0; i < QA_MAXN; ++i) {
        T s = from_d<T>(0.0);
#pragma unroll
        for (int j = 0; j <= i; ++j) s = s + a[j] * b[i - j];
        out[i] = s;
    }
#pragma unroll
    for (int i = 0; i < QA_MAXN; ++i) a[i] = i < n ? out[i] : from_d<T>(0.0);
}

// coefficient (-1/2)^K Gamma(n-K) of the K-pair term
QA_HD double kcoef(int n, int K) {
    double g = 1.0;
    for (int i = 2; i < n - K; ++i) g *= i;
    double h = 1.0;
    for (int i = 0; i < K; ++i) h *= -0.5;
    return g * h;
}

// f_G(z) at one point.  z: the M line parameters, used as given (f is
// homogeneous of degree -M).  f is linear in the coefficient table of the
// last (whole-graph) piece of each term: with nslices > 1 only the share
// `slice` of those tables' blocks is summed, and the nslices partial results
// add up to f (the double-double pass splits a point over several waves).
// Returns f (for EB with its magnitude, for ER with its rounding-error
// variance estimate); cond_out = worst conditioning of the graph
// polynomials seen (loop-matrix pivot ratio, cancellation ratios of flows and
// contraction coefficients), which bounds their relative error in units of
// the double-double round-off.
template <class T>
QA_HD T eval_point(const QA_RO uint8_t* img, const QA_RO DevGraph& G, CLV<double> z,
                   VV<typename GeoOf<T>::type> vars, LV<T> polys, double& cond_out, int slice = 0,
                   int nslices = 1) {
    using S = typename GeoOf<T>::type;
    const int n = G.n;
    const QA_RO DevTerm* terms = reinterpret_cast<const QA_RO DevTerm*>(img + G.terms_off);
    T f = from_d<T>(0.0);
    double cond_max = 1.0;
    double scale_n = 1.0;
    for (int i = 0; i < n; ++i) scale_n *= 0.25;
    for (int ti = 0; ti < G.nterms; ++ti) {
        const QA_RO DevTerm& tm = terms[ti];
        const QA_RO DevPiece* pcs = reinterpret_cast<const QA_RO DevPiece*>(img + tm.pieces_off);
        T pref = from_d<T>(1.0);
        T Vt = from_d<T>(0.0);
        T top[QA_MAXN];
        for (int pi = 0; pi < tm.npieces; ++pi) {
            const QA_RO DevPiece& pc = pcs[pi];
            DD Ud, Vd;
            double cond;
            geometry<S>(pc, z, vars, Ud, Vd, cond);
            S Us, Vs;
            store_geo(Us, Ud);
            store_geo(Vs, Vd);
            T U = lift_to<T>(Us), V = lift_to<T>(Vs);
            cond_max = fmax(cond_max, cond);
            pref = pref * (from_d<T>(1.0) / (U * U));
            Vt = Vt + V;
            const int nins = pc.nins;
            const int nop = pc.op == QA_OP_US ? 2 : 1;
            const QA_RO DevTable* tabs = reinterpret_cast<const QA_RO DevTable*>(img + pc.tab_off);
            T res[2][QA_MAXN];
#pragma unroll
            for (int opv = 0; opv < 2; ++opv) {
                if (opv >= nop) break;
                T acc[QA_MAXN];
#pragma unroll
                for (int k = 0; k < QA_MAXN; ++k) acc[k] = from_d<T>(0.0);
                for (int var = 0; var < (1 << nins); ++var) {
                    T P[QA_MAXN];
                    if (pi + 1 == tm.npieces)
                        eval_table<T, S>(img, tabs[(opv << nins) + var], vars, n, P, slice, nslices);
                    else
                        eval_table<T, S>(img, tabs[(opv << nins) + var], vars, n, P);
                    for (int t = 0; t < nins; ++t) {
                        T ch[QA_MAXN];
                        const int s = pc.ins_slot[t] + ((var >> t) & 1);
#pragma unroll
                        for (int k = 0; k < QA_MAXN; ++k) ch[k] = polys[s * QA_MAXN + k];
                        poly_mul(P, ch, n);
                    }
#pragma unroll
                    for (int k = 0; k < QA_MAXN; ++k) acc[k] = acc[k] + P[k];
                }
                for (int t = 0; t < pc.nvkids; ++t) {
                    T ch[QA_MAXN];
#pragma unroll
                    for (int k = 0; k < QA_MAXN; ++k) ch[k] = polys[pc.vkid_slot[t] * QA_MAXN + k];
                    poly_mul(acc, ch, n);
                }
#pragma unroll
                for (int k = 0; k < QA_MAXN; ++k) res[opv][k] = acc[k];
            }
            if (pi + 1 == tm.npieces) {
#pragma unroll
                for (int k = 0; k < QA_MAXN; ++k) top[k] = res[0][k];
            } else {
#pragma unroll
                for (int opv = 0; opv < 2; ++opv)
                    if (opv < nop)
#pragma unroll
                        for (int k = 0; k < QA_MAXN; ++k) polys[(pc.out_slot + opv) * QA_MAXN + k] = res[opv][k];
            }
        }
        // sum_K top[K] (-1/2)^K Gamma(n-K) Vt^(K-n)
        T iv = from_d<T>(1.0) / Vt;
        T ivp = from_d<T>(1.0);
        for (int i = 0; i < n; ++i) ivp = ivp * iv;
        T s = from_d<T>(0.0);
        for (int K = 0; K < n; ++K) {
            T t = top[K] * kcoef(n, K);
            s = s + t * ivp;
            ivp = ivp * Vt;
        }
        f = f + s * pref * (tm.sign * scale_n);
    }
    cond_out = cond_max;
    return f;
}
