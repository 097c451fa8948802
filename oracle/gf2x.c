/*
 * Whole-output checks of the convolution extractors as polynomial products
 * over GF(2) — TEST INFRASTRUCTURE ONLY. Nothing in the product library links,
 * calls or reads this file; only the tests, the smoke check and the CPU leg of
 * the benchmark use it. It shares no code with the GPU path: no transform, no
 * prime field, no table or constant of the GPU kernels.
 *
 * Over GF(2) each extractor is a polynomial product (the convolution form of
 * the section "Toeplitz implementation", Alg. 2, and of the Dodis et al. /
 * Circulant route, Alg. 1, with XOR in place of the integer sum):
 *
 *   Toeplitz, linear seed order: z_i = XOR_{j<n} x_j s_{i-j+n-1}, i < m. With
 *     X(t) = sum_j x_j t^j and S(t) = sum_{k<N} s_k t^k (N = n+m-1), z_i is the
 *     coefficient of t^(n-1+i) in X(t) S(t). (The paper's order is the same
 *     with s_k = y_{(k+m) mod N}; the caller rotates the seed.)
 *   Dodis et al. and Circulant: z_i = XOR_{j<n} a_{(j-i) mod n} y_j with the
 *     generator a (x, or x' = [x, 0] for Circulant). With b_k = a_{(-k) mod n},
 *     z_i = XOR_j b_{(i-j) mod n} y_j is the cyclic convolution of b and y:
 *     the coefficient of t^i plus that of t^(i+n) in B(t) Y(t).
 *
 * Products: Karatsuba's identity a b = a0 b0 + t^h ((a0+a1)(b0+b1) + a0 b0 +
 * a1 b1) + t^(2h) a1 b1 (a = a0 + t^h a1; + is XOR) down to a few 64-bit words,
 * then schoolbook over 64 x 64-bit carry-less products (the PCLMULQDQ
 * instruction where the CPU has it, else a shift-and-XOR loop). The top
 * levels of the recursion run their three products on separate threads.
 *
 * Bit layout: bit i of a string is (w[i >> 6] >> (i & 63)) & 1; every routine
 * reads exactly ceil(len/64) words of an input and ignores its bits >= len.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;

/* ------------------------------------------------------------ 64 x 64 carry-less product */

static void clmul_soft(u64 a, u64 b, u64 *lo, u64 *hi) {
    u64 l = 0, h = 0;
    for (int i = 0; i < 64; ++i)
        if ((b >> i) & 1) {
            l ^= a << i;
            if (i) h ^= a >> (64 - i);
        }
    *lo = l;
    *hi = h;
}

#if defined(__x86_64__)
#include <immintrin.h>
__attribute__((target("pclmul,sse4.1"))) static void clmul_hw(u64 a, u64 b, u64 *lo, u64 *hi) {
    __m128i r = _mm_clmulepi64_si128(_mm_set_epi64x(0, (long long)a), _mm_set_epi64x(0, (long long)b), 0x00);
    *lo = (u64)_mm_cvtsi128_si64(r);
    *hi = (u64)_mm_extract_epi64(r, 1);
}
/* schoolbook a (na words) x b (nb words) into r (na + nb words), one output word
 * pair at a time: r[k], r[k+1] ^= XOR_i a_i b_(k-i) */
__attribute__((target("pclmul,sse4.1"))) static void school_hw(const u64 *a, size_t na, const u64 *b, size_t nb,
                                                                u64 *r) {
    memset(r, 0, (na + nb) * 8);
    for (size_t k = 0; k + 1 < na + nb; ++k) {
        __m128i acc = _mm_setzero_si128();
        const size_t i0 = k + 1 > nb ? k + 1 - nb : 0, i1 = k < na - 1 ? k : na - 1;
        for (size_t i = i0; i <= i1; ++i)
            acc = _mm_xor_si128(acc, _mm_clmulepi64_si128(_mm_set_epi64x(0, (long long)a[i]),
                                                          _mm_set_epi64x(0, (long long)b[k - i]), 0x00));
        r[k] ^= (u64)_mm_cvtsi128_si64(acc);
        r[k + 1] ^= (u64)_mm_extract_epi64(acc, 1);
    }
}
static int have_pclmul(void) {
    __builtin_cpu_init();
    return __builtin_cpu_supports("pclmul") && __builtin_cpu_supports("sse4.1");
}
#else
static void clmul_hw(u64 a, u64 b, u64 *lo, u64 *hi) { clmul_soft(a, b, lo, hi); }
static void school_hw(const u64 *a, size_t na, const u64 *b, size_t nb, u64 *r) { (void)a, (void)na, (void)b, (void)nb, (void)r; }
static int have_pclmul(void) { return 0; }
#endif

static int g_hw = -1;  /* 1: PCLMULQDQ, 0: software; -1: not probed yet */
static int g_force_soft = 0;

static int use_hw(void) {
    if (g_hw < 0) g_hw = have_pclmul();
    return g_hw && !g_force_soft;
}

/* testing aid: 1 forces the shift-and-XOR product (to pin it against the
 * instruction); returns whether the instruction is available */
int gf2_force_software(int on) {
    g_force_soft = on != 0;
    if (g_hw < 0) g_hw = have_pclmul();
    return g_hw;
}

void gf2_clmul64(u64 a, u64 b, u64 *lo, u64 *hi) {
    if (use_hw()) clmul_hw(a, b, lo, hi);
    else clmul_soft(a, b, lo, hi);
}

static void school(const u64 *a, size_t na, const u64 *b, size_t nb, u64 *r) {
    if (use_hw()) {
        school_hw(a, na, b, nb, r);
        return;
    }
    memset(r, 0, (na + nb) * 8);
    for (size_t i = 0; i < na; ++i)
        for (size_t j = 0; j < nb; ++j) {
            u64 lo, hi;
            clmul_soft(a[i], b[j], &lo, &hi);
            r[i + j] ^= lo;
            r[i + j + 1] ^= hi;
        }
}

/* ------------------------------------------------------------ Karatsuba */

#define KARA_BASE 32 /* words: schoolbook at or below this size (fastest measured) */

static void xor_into(u64 *d, const u64 *s, size_t n) {
    for (size_t i = 0; i < n; ++i) d[i] ^= s[i];
}

/* scratch words kara() needs for n-word operands */
static size_t kara_scratch(size_t n) {
    if (n <= KARA_BASE) return 0;
    const size_t h = (n + 1) / 2;
    return 4 * h + kara_scratch(h);
}

/* r (2n words) = a b for a, b of n words each. a = a0 + t^(64h) a1 with a0 the low
 * h = ceil(n/2) words and a1 the high n - h words (likewise b). */
static void kara(const u64 *a, const u64 *b, size_t n, u64 *r, u64 *scr) {
    if (n <= KARA_BASE) {
        school(a, n, b, n, r);
        return;
    }
    const size_t h = (n + 1) / 2, l = n - h;
    u64 *sa = scr, *sb = scr + h, *p1 = scr + 2 * h, *rest = scr + 4 * h;
    kara(a, b, h, r, rest);                   /* a0 b0 -> r[0, 2h) */
    kara(a + h, b + h, l, r + 2 * h, rest);   /* a1 b1 -> r[2h, 2n) */
    memcpy(sa, a, h * 8);
    memcpy(sb, b, h * 8);
    xor_into(sa, a + h, l);
    xor_into(sb, b + h, l);
    kara(sa, sb, h, p1, rest);                /* (a0 + a1)(b0 + b1) */
    xor_into(p1, r, 2 * h);                   /* minus a0 b0 */
    xor_into(p1, r + 2 * h, 2 * l);           /* minus a1 b1 */
    xor_into(r + h, p1, 2 * h);               /* the middle term at t^(64h) */
}

/* The same product with the recursion's top `depth` levels on threads. */
struct kjob {
    const u64 *a, *b;
    size_t n;
    u64 *r;
    int depth;
    int rc;
};

static int kara_par(const u64 *a, const u64 *b, size_t n, u64 *r, int depth);

static void *kara_thread(void *p) {
    struct kjob *j = (struct kjob *)p;
    j->rc = kara_par(j->a, j->b, j->n, j->r, j->depth);
    return NULL;
}

static int kara_par(const u64 *a, const u64 *b, size_t n, u64 *r, int depth) {
    if (depth <= 0 || n < 4096) {
        u64 *scr = (u64 *)malloc((kara_scratch(n) + 1) * 8);
        if (!scr) return -1;
        kara(a, b, n, r, scr);
        free(scr);
        return 0;
    }
    const size_t h = (n + 1) / 2, l = n - h;
    u64 *sa = (u64 *)malloc(h * 8), *sb = (u64 *)malloc(h * 8), *p1 = (u64 *)malloc(2 * h * 8);
    if (!sa || !sb || !p1) {
        free(sa), free(sb), free(p1);
        return -1;
    }
    memcpy(sa, a, h * 8);
    memcpy(sb, b, h * 8);
    xor_into(sa, a + h, l);
    xor_into(sb, b + h, l);
    struct kjob j0 = {a, b, h, r, depth - 1, 0}, j2 = {a + h, b + h, l, r + 2 * h, depth - 1, 0};
    pthread_t t0, t2;
    const int s0 = pthread_create(&t0, NULL, kara_thread, &j0);
    const int s2 = pthread_create(&t2, NULL, kara_thread, &j2);
    int rc = kara_par(sa, sb, h, p1, depth - 1);
    if (s0 == 0) pthread_join(t0, NULL);
    else kara_thread(&j0);
    if (s2 == 0) pthread_join(t2, NULL);
    else kara_thread(&j2);
    if (rc == 0 && j0.rc == 0 && j2.rc == 0) {
        xor_into(p1, r, 2 * h);
        xor_into(p1, r + 2 * h, 2 * l);
        xor_into(r + h, p1, 2 * h);
    } else {
        rc = -1;
    }
    free(sa), free(sb), free(p1);
    return rc;
}

static int g_depth = 3; /* 3^3 = 27 leaf products on threads */

void gf2_set_threads_depth(int depth) { g_depth = depth < 0 ? 0 : depth; }

/* r (na + nb words) = a b for any word counts: the longer operand in pieces of
 * the shorter one's length, each piece's product added at its offset. Returns 0,
 * or -1 when memory runs out. */
int gf2_mul(const u64 *a, size_t na, const u64 *b, size_t nb, u64 *r) {
    if (na < nb) {
        const u64 *t = a;
        a = b;
        b = t;
        size_t tn = na;
        na = nb;
        nb = tn;
    }
    memset(r, 0, (na + nb) * 8);
    if (nb == 0) return 0;
    u64 *piece = (u64 *)calloc(nb, 8), *prod = (u64 *)malloc(2 * nb * 8);
    if (!piece || !prod) {
        free(piece), free(prod);
        return -1;
    }
    int rc = 0;
    for (size_t off = 0; off < na && rc == 0; off += nb) {
        const size_t k = na - off < nb ? na - off : nb;
        const u64 *src = a + off;
        if (k < nb) {
            memset(piece, 0, nb * 8);
            memcpy(piece, a + off, k * 8);
            src = piece;
        }
        rc = kara_par(src, b, nb, prod, g_depth);
        /* the piece's product has k + nb words; the rest are zero */
        xor_into(r + off, prod, k + nb);
    }
    free(piece), free(prod);
    return rc;
}

/* ------------------------------------------------------------ bit strings */

/* copy of len bits of a starting at bit `from` into out (ceil(len/64) words,
 * tail bits zero); a must have a readable word past its last bit used */
static void bits_range(const u64 *a, u64 from, u64 len, u64 *out) {
    const u64 W = (len + 63) >> 6, q = from >> 6, s = from & 63;
    for (u64 w = 0; w < W; ++w) out[w] = s ? ((a[q + w] >> s) | (a[q + w + 1] << (64 - s))) : a[q + w];
    if (len & 63) out[W - 1] &= ((u64)1 << (len & 63)) - 1;
}

static u64 *masked_copy(const u64 *a, u64 len, u64 extra_words) {
    const u64 W = (len + 63) >> 6;
    u64 *c = (u64 *)calloc(W + extra_words + 1, 8);
    if (!c) return NULL;
    memcpy(c, a, W * 8);
    if (len & 63) c[W - 1] &= ((u64)1 << (len & 63)) - 1;
    return c;
}

/* Toeplitz, linear seed order, the share of input positions [j0, j0 + w):
 * z ^= XOR_{j0 <= j < j0+w} x_j s_{i-j+n-1} (i < m; z has ceil(m/64) words). With
 * x' = x_j0 .. x_(j0+w-1) and the seed window s' = s_t0 .. s_(t0+w+m-2),
 * t0 = n - j0 - w, that share is z_i = XOR_j' x'_j' s'_(w-1+i-j'): the
 * coefficients t^(w-1) .. t^(w-2+m) of X'(t) S'(t). The whole output is the
 * share of [0, n). x and s need one readable word past their last bit.
 * Returns 0 or -1 (out of memory). */
int gf2_toeplitz_block(const u64 *x, u64 n, const u64 *s, u64 m, u64 j0, u64 w, u64 *z) {
    if (w == 0 || j0 + w > n) return -1;
    const u64 sw = w + m - 1, nx = (w + 63) >> 6, ns = (sw + 63) >> 6, mw = (m + 63) >> 6;
    u64 *xc = (u64 *)calloc(nx + 1, 8), *sc = (u64 *)calloc(ns + 1, 8), *prod = (u64 *)calloc(nx + ns + 2, 8),
        *part = (u64 *)calloc(mw + 1, 8);
    int rc = -1;
    if (xc && sc && prod && part) {
        bits_range(x, j0, w, xc);
        bits_range(s, n - j0 - w, sw, sc);
        rc = gf2_mul(xc, nx, sc, ns, prod);
        if (rc == 0) {
            bits_range(prod, w - 1, m, part);
            for (u64 i = 0; i < mw; ++i) z[i] ^= part[i];
        }
    }
    free(xc), free(sc), free(prod), free(part);
    return rc;
}

/* the whole Toeplitz output (linear order): the share of every input position */
int gf2_toeplitz_linear(const u64 *x, u64 n, const u64 *s, u64 m, u64 *z) {
    memset(z, 0, ((m + 63) >> 6) * 8);
    return gf2_toeplitz_block(x, n, s, m, 0, n, z);
}

/* dst bits [pos, pos + len) ^= the first len bits of src (src tail bits zero) */
static void xor_bits_at(u64 *dst, u64 pos, const u64 *src, u64 len) {
    const u64 W = (len + 63) >> 6, q = pos >> 6, s = pos & 63;
    for (u64 w = 0; w < W; ++w) {
        dst[q + w] ^= src[w] << s;
        if (s) dst[q + w + 1] ^= src[w] >> (64 - s);
    }
}

/* bit order of one word reversed (bit b to bit 63 - b) */
static u64 rev64(u64 v) {
    u64 r = 0;
    for (int b = 0; b < 64; ++b) r |= ((v >> b) & 1u) << (63 - b);
    return r;
}

/* out_k = a_{from + len - 1 - k}, k < len (ceil(len/64) words + 1 spare) */
static int rev_range(const u64 *a, u64 from, u64 len, u64 *out) {
    const u64 W = (len + 63) >> 6, pad = 64 * W - len;
    u64 *w = (u64 *)calloc(W + 1, 8), *full = (u64 *)calloc(W + 1, 8);
    if (!w || !full) {
        free(w), free(full);
        return -1;
    }
    bits_range(a, from, len, w);
    /* the reversal of all 64 W bits puts a_{from+len-1-k} at bit k + pad */
    for (u64 i = 0; i < W; ++i) full[i] = rev64(w[W - 1 - i]);
    bits_range(full, pad, len, out);
    free(w), free(full);
    return 0;
}

/* The seed of the paper's order as the linear-order string: s_k = y_{(k + m) mod N}
 * (the rotation that maps eq. (toep) onto the linear order): s[0, N - r) = y[r, N)
 * and s[N - r, N) = y[0, r) with r = m mod N. s: ceil(N/64) words. */
int gf2_paper_to_linear(const u64 *y, u64 N, u64 m, u64 *s) {
    const u64 r = m % N, W = (N + 63) >> 6;
    u64 *yc = masked_copy(y, N, 1), *head = (u64 *)calloc(((r + 63) >> 6) + 1, 8), *t = (u64 *)calloc(W + 2, 8);
    if (!yc || !head || !t) {
        free(yc), free(head), free(t);
        return -1;
    }
    bits_range(yc, r, N - r, t);
    if (r) {
        bits_range(yc, 0, r, head);
        xor_bits_at(t, N - r, head, r);
    }
    memcpy(s, t, W * 8);
    free(yc), free(head), free(t);
    return 0;
}

/* Dodis et al. / Circulant rows i < m of the circulant generated by a (n bits):
 * z_i = XOR_j a_{(j-i) mod n} y_j, from the cyclic convolution of
 * b_k = a_{(-k) mod n} and y. Returns 0 or -1 (out of memory). */
int gf2_circulant_rows(const u64 *a, u64 n, const u64 *y, u64 m, u64 *z) {
    const u64 W = (n + 63) >> 6;
    u64 *ac = masked_copy(a, n, 0), *b = (u64 *)calloc(W + 1, 8), *yc = masked_copy(y, n, 0),
        *prod = (u64 *)calloc(2 * W + 2, 8);
    int rc = -1;
    if (ac && b && yc && prod) {
        /* b_0 = a_0 and b_k = a_{n-k}: bits 1.. of b are a_1 .. a_{n-1} reversed */
        b[0] = ac[0] & 1u;
        rc = 0;
        if (n > 1) {
            u64 *rv = (u64 *)calloc(W + 2, 8);
            rc = rv ? rev_range(ac, 1, n - 1, rv) : -1;
            if (rc == 0) xor_bits_at(b, 1, rv, n - 1);
            free(rv);
        }
        if (rc == 0) rc = gf2_mul(b, W, yc, W, prod);
        if (rc == 0) {
            const u64 mw = (m + 63) >> 6;
            u64 *hi = (u64 *)calloc(mw + 1, 8);
            if (!hi) {
                rc = -1;
            } else {
                bits_range(prod, 0, m, z);   /* coefficients i < m */
                bits_range(prod, n, m, hi);  /* coefficients i + n (zero beyond 2n - 2) */
                for (u64 w = 0; w < mw; ++w) z[w] ^= hi[w];
                free(hi);
            }
        }
    }
    free(ac), free(b), free(yc), free(prod);
    return rc;
}
