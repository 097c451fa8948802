/*
 * Oracle for the Toeplitz, Circulant and Dodis et al. extractors, and for the
 * Von Neumann extractor.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, calls or
 * reads this file; only the tests, the smoke check and the CPU baseline of the
 * benchmark use it. It shares no code with the GPU path.
 *
 * Every function computes the extractor straight from its definition as a
 * matrix-vector product over GF(2) (AND, then XOR-accumulate). There is no
 * transform, no field other than GF(2), and no blocking beyond packing 64
 * bits into a word.
 *
 *   Toeplitz, paper seed order (Sec. "Toeplitz", eq. toep):
 *       z_i = XOR_{j<n} y_{(i-j) mod N} & x_j,            N = n + m - 1, i < m
 *   Toeplitz, linear seed order (the workload's own statement):
 *       z_i = XOR_{j<n} s_{i-j+n-1} & x_j
 *   Circulant (Def. of Circulant, eq. circ-matrix): x' = [x, 0] of length n,
 *       z_i = XOR_{j<n} x'_{(j-i) mod n} & y_j
 *   Dodis et al. (Sec. "Dodis and Circulant implementation", the full matrix
 *   and the R(x) convolution form):
 *       z_i = XOR_{j<n} x_{(j-i) mod n} & y_j
 *
 *   Von Neumann (Sec. "Von Neumann", the definition of output bit j, and
 *   Alg. 3): for the pairs (x_{2j}, x_{2j+1}), j < floor(n/2), in order of j,
 *       emit x_{2j} when x_{2j} != x_{2j+1}, nothing otherwise.
 *
 * Bit layout: bit i of a string is (w[i >> 6] >> (i & 63)) & 1.
 * Preconditions (lengths, primality, degenerate inputs) are checked by the
 * Python wrapper; these routines only compute.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline int bit(const uint64_t *a, uint64_t i) { return (int)((a[i >> 6] >> (i & 63)) & 1u); }
static inline void put(uint64_t *a, uint64_t i, int v) {
    if (v) a[i >> 6] |= (uint64_t)1 << (i & 63);
    else a[i >> 6] &= ~((uint64_t)1 << (i & 63));
}

/* ------------------------------------------------------------ bit by bit */

void oracle_toeplitz_bits(const uint64_t *x, uint64_t n, const uint64_t *y, uint64_t m,
                          int linear, uint64_t *z) {
    uint64_t N = n + m - 1;
    for (uint64_t i = 0; i < m; ++i) {
        int acc = 0;
        for (uint64_t j = 0; j < n; ++j) {
            uint64_t k = linear ? (i + n - 1 - j) : ((i + N - j) % N);
            acc ^= bit(y, k) & bit(x, j);
        }
        put(z, i, acc);
    }
}

/* a is the n-bit generator of the circulant rows: row i, column j holds a_{(j-i) mod n} */
static void circ_rows_bits(const uint64_t *a, const uint64_t *y, uint64_t n, uint64_t m, uint64_t *z) {
    for (uint64_t i = 0; i < m; ++i) {
        int acc = 0;
        for (uint64_t j = 0; j < n; ++j) acc ^= bit(a, (j + n - i) % n) & bit(y, j);
        put(z, i, acc);
    }
}

void oracle_dodis_bits(const uint64_t *x, const uint64_t *y, uint64_t n, uint64_t m, uint64_t *z) {
    circ_rows_bits(x, y, n, m, z);
}

/* x has n_in bits; the circulant generator is x' = [x, 0] of length n = n_in + 1 */
void oracle_circulant_bits(const uint64_t *x, uint64_t n_in, const uint64_t *y, uint64_t m, uint64_t *z) {
    uint64_t n = n_in + 1;
    uint64_t *xp = (uint64_t *)calloc((n + 63) / 64 + 1, 8);
    for (uint64_t j = 0; j < n_in; ++j) put(xp, j, bit(x, j));
    circ_rows_bits(xp, y, n, m, z);
    free(xp);
}

/* ------------------------------------------------------------ packed rows
 * The same sums, 64 terms at a time: a row of the matrix is a contiguous
 * window of some bit string, so each output bit is the parity of
 * popcount(window AND vector). Rows i0 .. i0+cnt-1 are computed; bit r of
 * out (packed) receives z_{i0+r}. */

/* word w (w = 0, 1, ...) of the bit string a read from bit offset off */
static inline uint64_t window_word(const uint64_t *a, uint64_t off, uint64_t w) {
    uint64_t q = (off >> 6) + w, b = off & 63;
    return b ? ((a[q] >> b) | (a[q + 1] << (64 - b))) : a[q];
}

static int parity_window_and(const uint64_t *a, uint64_t off, const uint64_t *v, uint64_t len) {
    uint64_t words = len >> 6, rem = len & 63;
    uint64_t acc = 0;
    for (uint64_t w = 0; w < words; ++w) acc ^= window_word(a, off, w) & v[w];
    if (rem) acc ^= window_word(a, off, words) & v[words] & (((uint64_t)1 << rem) - 1);
    return __builtin_parityll(acc);
}

/* bit order of one word reversed: bit b moves to bit 63 - b (swap halves, then
 * quarters, ... down to single bits) */
static uint64_t rev64(uint64_t v) {
    v = (v >> 32) | (v << 32);
    v = ((v >> 16) & 0x0000FFFF0000FFFFull) | ((v & 0x0000FFFF0000FFFFull) << 16);
    v = ((v >> 8) & 0x00FF00FF00FF00FFull) | ((v & 0x00FF00FF00FF00FFull) << 8);
    v = ((v >> 4) & 0x0F0F0F0F0F0F0F0Full) | ((v & 0x0F0F0F0F0F0F0F0Full) << 4);
    v = ((v >> 2) & 0x3333333333333333ull) | ((v & 0x3333333333333333ull) << 2);
    v = ((v >> 1) & 0x5555555555555555ull) | ((v & 0x5555555555555555ull) << 1);
    return v;
}

/* reversed copy: r_k = a_{len-1-k}; the input's bits beyond len must be zero.
 * With W words and pad = 64W - len, the reversal of all 64W bits has word i equal
 * to rev64(a[W-1-i]) and bit k + pad equal to a_{len-1-k}; shifting it down by pad
 * bits gives r. One spare zero word at the end for window reads. */
static uint64_t *reversed(const uint64_t *a, uint64_t len) {
    uint64_t W = (len + 63) / 64, pad = 64 * W - len;
    uint64_t *full = (uint64_t *)calloc(W + 2, 8);
    uint64_t *r = (uint64_t *)calloc(W + 2, 8);
    for (uint64_t i = 0; i < W; ++i) full[i] = rev64(a[W - 1 - i]);
    for (uint64_t i = 0; i < W; ++i)
        r[i] = pad ? ((full[i] >> pad) | (full[i + 1] << (64 - pad))) : full[i];
    free(full);
    return r;
}

/* two periods a || a of an len-bit string (input bits beyond len zero): the second
 * copy is a shifted up by len bits. A spare zero word at the end. */
static uint64_t *doubled(const uint64_t *a, uint64_t len) {
    uint64_t W = (len + 63) / 64, q = len >> 6, b = len & 63;
    uint64_t *d = (uint64_t *)calloc((2 * len + 63) / 64 + 2, 8);
    for (uint64_t i = 0; i < W; ++i) {
        d[i] |= a[i];
        d[q + i] |= a[i] << b;
        if (b) d[q + i + 1] |= a[i] >> (64 - b);
    }
    return d;
}

/* Linear order: with r the reversed seed (r_k = s_{N-1-k}), s_{i-j+n-1} = r_{(m-1-i)+j},
 * so row i is the n-bit window of r at offset m-1-i.
 * Paper order: with e = y || y, y_{(i-j) mod N} = e_{N+i-j} (0 < N+i-j < 2N), and with
 * re the reversal of e (re_k = e_{2N-1-k}), e_{N+i-j} = re_{(N-1-i)+j}: the window of re
 * at offset N-1-i. */
void oracle_toeplitz_rows(const uint64_t *x, uint64_t n, const uint64_t *y, uint64_t m, int linear,
                          uint64_t i0, uint64_t cnt, uint64_t *out) {
    uint64_t N = n + m - 1;
    uint64_t *r;
    if (linear) {
        r = reversed(y, N);
    } else {
        uint64_t *e = doubled(y, N);
        r = reversed(e, 2 * N);
        free(e);
    }
    memset(out, 0, ((cnt + 63) / 64) * 8);
    for (uint64_t t = 0; t < cnt; ++t) {
        uint64_t i = i0 + t;
        uint64_t off = linear ? (m - 1 - i) : (N - 1 - i);
        put(out, t, parity_window_and(r, off, x, n));
    }
    free(r);
}

/* Circulant / Dodis rows: with e = a || a, a_{(j-i) mod n} = e_{n+j-i}: row i is the
 * n-bit window of e at offset n-i (for i = 0 the window at offset n is a itself). */
static void circ_rows_packed(const uint64_t *a, const uint64_t *y, uint64_t n, uint64_t i0, uint64_t cnt,
                             uint64_t *out) {
    uint64_t *e = doubled(a, n);
    memset(out, 0, ((cnt + 63) / 64) * 8);
    for (uint64_t t = 0; t < cnt; ++t) {
        uint64_t i = i0 + t;
        put(out, t, parity_window_and(e, n - i, y, n));
    }
    free(e);
}

void oracle_dodis_rows(const uint64_t *x, const uint64_t *y, uint64_t n, uint64_t i0, uint64_t cnt, uint64_t *out) {
    circ_rows_packed(x, y, n, i0, cnt, out);
}

void oracle_circulant_rows(const uint64_t *x, uint64_t n_in, const uint64_t *y, uint64_t i0, uint64_t cnt,
                           uint64_t *out) {
    uint64_t n = n_in + 1;
    uint64_t *xp = (uint64_t *)calloc((n + 63) / 64 + 1, 8);
    for (uint64_t j = 0; j < n_in; ++j) put(xp, j, bit(x, j));
    circ_rows_packed(xp, y, n, i0, cnt, out);
    free(xp);
}

/* ------------------------------------------------------------ Von Neumann
 * Pair by pair, as the definition reads: the output is appended to while the
 * pairs are walked in order. Returns the number of output bits m; out must have
 * room for floor(n/2) bits and is written only at bits < m. */
uint64_t oracle_von_neumann_bits(const uint64_t *x, uint64_t n, uint64_t *out) {
    uint64_t m = 0;
    for (uint64_t j = 0; j < n / 2; ++j) {
        int a = bit(x, 2 * j), b = bit(x, 2 * j + 1);
        if (a != b) put(out, m++, a);
    }
    return m;
}
