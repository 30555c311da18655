/* Oracle code (test infrastructure only).
 *
 * Dirac trace of a gamma string with contracted indices by the textbook
 * 4-dimensional Chisholm identities, the same recursion as oracle/dirac.py
 * (innermost-first pair, odd inner length preferred), in plain C for speed.
 * Symbols: 0 = on-shell p-slash with p.p = 1; L > 0 = gamma contracted with
 * the other occurrence of L.
 */
#include <string.h>

static long long tr(const int* s, int n);

static int reduce_pp(const int* in, int n, int* out) {
    int m = 0;
    for (int i = 0; i < n; ++i) {
        if (in[i] == 0 && m > 0 && out[m - 1] == 0) { --m; continue; }
        out[m++] = in[i];
    }
    return m;
}

static long long tr(const int* s0, int n0) {
    int s[64];
    int n = reduce_pp(s0, n0, s);
    if (n % 2) return 0;
    int bi = -1, bj = -1, bk = 1 << 30, beven = 1;
    for (int i = 0; i < n; ++i) {
        if (s[i] <= 0) continue;
        for (int j = i + 1; j < n; ++j) {
            if (s[j] == s[i]) {
                int k = j - i - 1;
                int ev = (k % 2 == 0 && k > 0);
                if (bi < 0 || ev < beven || (ev == beven && k < bk)) { bi = i; bj = j; bk = k; beven = ev; }
                break;
            }
        }
    }
    if (bi < 0) return 4;
    int t[64], m = 0;
    int k = bj - bi - 1;
    if (k == 0) {
        for (int i = 0; i < n; ++i) if (i != bi && i != bj) t[m++] = s[i];
        return 4 * tr(t, m);
    }
    if (k % 2) {
        for (int i = 0; i < bi; ++i) t[m++] = s[i];
        for (int i = bj - 1; i > bi; --i) t[m++] = s[i];
        for (int i = bj + 1; i < n; ++i) t[m++] = s[i];
        return -2 * tr(t, m);
    }
    /* 2 (s_k s_1 .. s_(k-1) + s_(k-1) .. s_1 s_k) */
    int u[64], mu = 0;
    for (int i = 0; i < bi; ++i) { t[m++] = s[i]; u[mu++] = s[i]; }
    t[m++] = s[bj - 1];
    for (int i = bi + 1; i < bj - 1; ++i) t[m++] = s[i];
    for (int i = bj - 2; i > bi; --i) u[mu++] = s[i];
    u[mu++] = s[bj - 1];
    for (int i = bj + 1; i < n; ++i) { t[m++] = s[i]; u[mu++] = s[i]; }
    return 2 * (tr(t, m) + tr(u, mu));
}

long long oracle_trace(const int* s, int n) {
    if (n > 60) return 0x7fffffffffffffffLL;
    return tr(s, n);
}
