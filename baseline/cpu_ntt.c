/*
 * Single-threaded CPU NTT convolution for the Toeplitz extractor: the timing
 * baseline for a plain CPU implementation of the paper's route (convolution
 * theorem, section "The number-theoretic transform and the convolution
 * theorem"; the Toeplitz matrix as a convolution, section "Toeplitz").
 *
 * Only the benchmark times it; a CPU test checks it against the oracle. It
 * shares no code with the GPU library or with the oracle.
 *
 * Field: p = 2^64 - 2^32 + 1 (2^64 = 2^32 - 1 and 2^96 = -1 mod p), the prime of
 * the single large-transform configuration; 7 generates the multiplicative
 * group. Iterative radix-2 decimation-in-time transform on bit-reversed input.
 *
 *   z_i = XOR_{j<n} s_{i-j+n-1} x_j,  i < m,  s_k = y_k (linear order) or
 *   y_{(k+m) mod N} (the paper's order), N = n + m - 1.
 * With L >= N the cyclic convolution c = x (*) s has c_{i+n-1} = that sum for
 * i < m (its indices i+n-1-j stay in [0, N)), so z_i = c_{i+n-1} mod 2.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
static const uint64_t P = 0xFFFFFFFF00000001ull;
static const uint64_t EPS = 0xFFFFFFFFull; /* 2^64 mod p */

static inline uint64_t canon(uint64_t a) { return a >= P ? a - P : a; }
static inline uint64_t add(uint64_t a, uint64_t b) { /* a, b < p */
    uint64_t s = a + b;
    return (s < a || s >= P) ? s - P : s;
}
static inline uint64_t sub(uint64_t a, uint64_t b) { /* a, b < p */
    return a >= b ? a - b : a - b + P;
}
/* a * b mod p: t = hi 2^64 + lo, hi = h1 2^32 + h0, t = lo + h0 (2^32 - 1) - h1 */
static inline uint64_t mul(uint64_t a, uint64_t b) {
    u128 t = (u128)a * b;
    uint64_t lo = (uint64_t)t, hi = (uint64_t)(t >> 64);
    uint64_t h0 = hi & EPS, h1 = hi >> 32;
    uint64_t r = lo - h1;
    if (lo < h1) r -= EPS; /* the borrowed 2^64 is worth EPS */
    uint64_t u = r + h0 * EPS;
    if (u < r) u += EPS; /* the carried 2^64 is worth EPS */
    return canon(u);
}
static uint64_t power(uint64_t a, uint64_t e) {
    uint64_t r = 1;
    while (e) {
        if (e & 1) r = mul(r, a);
        a = mul(a, a);
        e >>= 1;
    }
    return r;
}

static void transform(uint64_t *a, int lg, int inverse) {
    const uint64_t L = (uint64_t)1 << lg;
    for (uint64_t i = 1, j = 0; i < L; ++i) { /* bit-reversal permutation */
        uint64_t bit = L >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            uint64_t t = a[i];
            a[i] = a[j];
            a[j] = t;
        }
    }
    uint64_t *w = (uint64_t *)malloc((L / 2 + 1) * sizeof(uint64_t));
    for (int s = 1; s <= lg; ++s) {
        const uint64_t len = (uint64_t)1 << s, half = len / 2;
        uint64_t root = power(7, (P - 1) >> s); /* order exactly 2^s */
        if (inverse) root = power(root, P - 2);
        w[0] = 1;
        for (uint64_t k = 1; k < half; ++k) w[k] = mul(w[k - 1], root);
        for (uint64_t blk = 0; blk < L; blk += len)
            for (uint64_t k = 0; k < half; ++k) {
                uint64_t u = a[blk + k], v = mul(a[blk + k + half], w[k]);
                a[blk + k] = add(u, v);
                a[blk + k + half] = sub(u, v);
            }
    }
    free(w);
    if (inverse) {
        const uint64_t linv = power(L % P, P - 2);
        for (uint64_t i = 0; i < L; ++i) a[i] = mul(a[i], linv);
    }
}

static inline int bit(const uint64_t *b, uint64_t i) { return (int)((b[i >> 6] >> (i & 63)) & 1u); }

/* z gets ceil(m/64) words (tail bits 0). Returns 0, or -1 if memory runs out. */
int cpu_ntt_toeplitz(const uint64_t *x, uint64_t n, const uint64_t *y, uint64_t m, int linear, uint64_t *z) {
    const uint64_t N = n + m - 1;
    int lg = 0;
    while (((uint64_t)1 << lg) < N) ++lg;
    const uint64_t L = (uint64_t)1 << lg;
    uint64_t *A = (uint64_t *)calloc(L, sizeof(uint64_t));
    uint64_t *B = (uint64_t *)calloc(L, sizeof(uint64_t));
    if (!A || !B) {
        free(A);
        free(B);
        return -1;
    }
    for (uint64_t j = 0; j < n; ++j) A[j] = (uint64_t)bit(x, j);
    for (uint64_t k = 0; k < N; ++k) B[k] = (uint64_t)bit(y, linear ? k : (k + m) % N);
    transform(A, lg, 0);
    transform(B, lg, 0);
    for (uint64_t i = 0; i < L; ++i) A[i] = mul(A[i], B[i]);
    transform(A, lg, 1);
    memset(z, 0, ((m + 63) / 64) * sizeof(uint64_t));
    for (uint64_t i = 0; i < m; ++i)
        if (A[i + n - 1] & 1u) z[i >> 6] |= (uint64_t)1 << (i & 63);
    free(A);
    free(B);
    return 0;
}
