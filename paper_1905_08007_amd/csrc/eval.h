// Integrand evaluator core: graph polynomials of each piece, projected
// numerator tables, forest-term combination.  Templated on the number type.
#pragma once
#include "numeric.h"
#include "qa_dev.h"

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

QA_HD int tri_idx(int a, int b) { return a <= b ? b * (b + 1) / 2 + a : a * (a + 1) / 2 + b; }

// ---------------------------------------------------------------------------
// graph polynomials of a piece: loop matrix M (chord basis), U = det M,
// Wick contraction matrix Bbar_ij = eta_i^T M^-1 eta_j, flows A (external p
// from the first to the last node) and C (q entering at the external node,
// -1/2 leaving at each end), V = sum_i z_i (1 - A_i).
// computed in double-double (T = DD); results stored as S (double or DD)
template <class S, int L>
QA_HD void geometry_L(const DevPiece& pc, CLV<double> z, LV<S> vars, DD& U, DD& V, double& cond) {
    using T = DD;
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
    cond = dmax / dmin;
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
        for (int d = 0; d < L; ++d) { s = s + Mi[c][d] * jv[d]; sq = sq + Mi[c][d] * jq[d]; }
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
        store_geo(vars[QA_VAR_A + i], a);
        store_geo(vars[QA_VAR_C + i], cq);
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
                store_geo(vars[tri_idx(i, j)], s);
            }
        }
    }
}

template <class S>
QA_HD void geometry(const DevPiece& pc, CLV<double> z, LV<S> vars, DD& U, DD& V, double& cond) {
    switch (pc.nchords) {
        case 1: geometry_L<S, 1>(pc, z, vars, U, V, cond); break;
        case 2: geometry_L<S, 2>(pc, z, vars, U, V, cond); break;
        case 3: geometry_L<S, 3>(pc, z, vars, U, V, cond); break;
        case 4: geometry_L<S, 4>(pc, z, vars, U, V, cond); break;
        default: geometry_L<S, 5>(pc, z, vars, U, V, cond); break;
    }
}

// ---------------------------------------------------------------------------
// multilinear fold: sum_s c[s] prod_{bit i of s} A[i], r <= QA_MAXR
template <class T, int R> struct Fold {
    QA_HD static T run(const double* c, const T* A) {
        return Fold<T, R - 1>::run(c, A) + A[R - 1] * Fold<T, R - 1>::run(c + (1 << (R - 1)), A);
    }
};
template <class T> struct Fold<T, 0> {
    QA_HD static T run(const double* c, const T*) { return from_d<T>(c[0]); }
};

template <class T> QA_HD T fold(const double* c, const T* A, int r) {
    switch (r) {
        case 0: return Fold<T, 0>::run(c, A);
        case 1: return Fold<T, 1>::run(c, A);
        case 2: return Fold<T, 2>::run(c, A);
        case 3: return Fold<T, 3>::run(c, A);
        case 4: return Fold<T, 4>::run(c, A);
        default: break;
    }
    // 16-coefficient leaves combined by a carry chain over the high bits
    T acc[QA_MAXR - 4];
    T v = from_d<T>(0.0);
    const int nleaves = 1 << (r - 4);
    for (int leaf = 0; leaf < nleaves; ++leaf) {
        v = Fold<T, 4>::run(c + 16 * leaf, A);
        int b = leaf;
        bool stored = false;
#pragma unroll
        for (int l = 0; l < QA_MAXR - 4; ++l) {
            if (stored || 4 + l >= r) break;
            if ((b & 1) == 0) { acc[l] = v; stored = true; }
            else { v = acc[l] + A[4 + l] * v; b >>= 1; }
        }
    }
    return v;
}

// Evaluate one coefficient table: poly[k] = scale * sum over blocks with k pairs
template <class T, class S>
QA_HD void eval_table(const uint8_t* __restrict__ img, const DevTable& tb, LV<S> vars, int n, T* poly) {
    using AT = typename Acc<T>::type;
    AT acc[QA_MAXN];
#pragma unroll
    for (int k = 0; k < QA_MAXN; ++k) acc[k] = acc_zero((AT*)nullptr);
    const DevBlock* blocks = reinterpret_cast<const DevBlock*>(img + tb.hdr_off);
    const double* coefs = reinterpret_cast<const double*>(img + tb.coef_off);
    for (int bi = 0; bi < tb.nblocks; ++bi) {
        const DevBlock& b = blocks[bi];
        const int k = b.k, r = b.r;
        if (k >= n) break;
        T w = from_d<T>(1.0);
#pragma unroll
        for (int q = 0; q < QA_MAXK; ++q)
            if (q < k) w = w * lift_to<T>(vars[b.bidx[q]]);
        T A[QA_MAXR];
#pragma unroll
        for (int i = 0; i < QA_MAXR; ++i) A[i] = i < r ? lift_to<T>(vars[b.aidx[i]]) : from_d<T>(0.0);
        const double* c = coefs + b.coef;
        T s = fold(c, A, r);
        if (tb.has_q) {
            const int half = r > 0 ? 1 << (r - 1) : 0;
#pragma unroll
            for (int j = 0; j < QA_MAXR; ++j) {
                if (j >= r) break;
                T Ap[QA_MAXR];
#pragma unroll
                for (int i = 0; i < QA_MAXR - 1; ++i) Ap[i] = i < j ? A[i] : A[i + 1];
                Ap[QA_MAXR - 1] = from_d<T>(0.0);
                s = s + lift_to<T>(vars[b.cidx[j]]) * fold(c + (1 << r) + j * half, Ap, r - 1);
            }
        }
        T ws = w * s;
#pragma unroll
        for (int kk = 0; kk < QA_MAXN; ++kk)
            if (kk == k) acc_add(acc[kk], ws);
    }
#pragma unroll
    for (int k = 0; k < QA_MAXN; ++k) poly[k] = div_den(acc_get(acc[k]), tb.denom);
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

// f_G(z) at one point.  z: the M line parameters (any positive scale; they
// are used as given, so callers normalise to sum 1).  Returns f; for EB the
// magnitude carries the rounding-error scale; cond_out = worst loop-matrix
// conditioning seen.
template <class T>
QA_HD T eval_point(const uint8_t* __restrict__ img, const DevGraph& G, CLV<double> z,
                   LV<typename GeoOf<T>::type> vars, LV<T> polys, double& cond_out) {
    using S = typename GeoOf<T>::type;
    const int n = G.n;
    const DevTerm* terms = reinterpret_cast<const DevTerm*>(img + G.terms_off);
    T f = from_d<T>(0.0);
    double cond_max = 1.0;
    double scale_n = 1.0;
    for (int i = 0; i < n; ++i) scale_n *= 0.25;
    for (int ti = 0; ti < G.nterms; ++ti) {
        const DevTerm& tm = terms[ti];
        const DevPiece* pcs = reinterpret_cast<const DevPiece*>(img + tm.pieces_off);
        T pref = from_d<T>(1.0);
        T Vt = from_d<T>(0.0);
        T top[QA_MAXN];
        for (int pi = 0; pi < tm.npieces; ++pi) {
            const DevPiece& pc = pcs[pi];
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
            const DevTable* tabs = reinterpret_cast<const DevTable*>(img + pc.tab_off);
            T res[2][QA_MAXN];
#pragma unroll
            for (int opv = 0; opv < 2; ++opv) {
                if (opv >= nop) break;
                T acc[QA_MAXN];
#pragma unroll
                for (int k = 0; k < QA_MAXN; ++k) acc[k] = from_d<T>(0.0);
                for (int var = 0; var < (1 << nins); ++var) {
                    T P[QA_MAXN];
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
