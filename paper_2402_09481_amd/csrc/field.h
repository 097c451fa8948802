// Prime fields for the number-theoretic transform (NTT definition and
// convolution theorem, section "The number-theoretic transform and the
// convolution theorem").
//
// The extractors only need the exact integer cyclic convolution of two 0/1
// vectors; each coefficient is at most n < p, so any prime p > n whose
// multiplicative group has an element of order L (the transform length)
// gives the same integers, hence the same bits after mod 2.
//
//   FBB: p = 15 * 2^27 + 1 (< 2^31), 32-bit words, L <= 2^27. Values are kept
//        canonical in [0, p); products use Montgomery multiplication with
//        R = 2^32, and twiddle tables hold Montgomery forms w*R mod p, so that
//        mont(a, w*R) = a*w mod p.
//   FGL: p = 2^64 - 2^32 + 1, 64-bit words, L <= 2^32. Values are any 64-bit
//        representative (< 2^64) of their class; only canon() returns the
//        representative in [0, p). 2^64 = 2^32 - 1 (mod p) and 2^96 = -1 (mod p)
//        give a multiply-free reduction of 128-bit products.
//
// Both fields use one fixed primitive root of unity w_max of order 2^LGMAX;
// every transform of length L uses w_L = w_max^(2^LGMAX / L), so that all
// sub-transforms of a multi-pass transform agree on their roots.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ext {

// ------------------------------------------------------------ 15 * 2^27 + 1
struct FBB {
    using T = uint32_t;
    static constexpr uint32_t P = 0x78000001u;
    static constexpr uint32_t PINV = 2281701377u;  // P^-1 mod 2^32
    static constexpr int LGMAX = 27;
    static constexpr uint32_t WMAX = 440564289u;   // 31^15: order 2^27 (31 generates the group)
    static constexpr uint32_t R_MOD_P = 268435454u; // 2^32 mod P (Montgomery form of 1)
    static constexpr int WORD_BITS = 32;

    __host__ __device__ static constexpr uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }
    // a, b in [0, P): result in [0, P). If s >= P, s - P < s; otherwise s - P wraps above s.
    __device__ static inline uint32_t add(uint32_t a, uint32_t b) {
        uint32_t s = a + b;
        return umin(s, s - P);
    }
    __device__ static inline uint32_t sub(uint32_t a, uint32_t b) {
        uint32_t d = a - b;
        return umin(d, d + P);
    }
    // Montgomery product a*b*2^-32 mod P for a, b < P (signed variant):
    // with t = a*b = hi*2^32 + lo and q = lo*P^-1 mod 2^32, q*P = lo (mod 2^32), so
    // (t - q*P) / 2^32 = hi - mulhi(q, P), which lies in (-P, P).
    __device__ static inline uint32_t mont(uint32_t a, uint32_t b) {
        uint32_t lo = a * b;
        uint32_t hi = __umulhi(a, b);
        uint32_t q = lo * PINV;
        uint32_t r = hi - __umulhi(q, P);
        return umin(r, r + P);
    }
    // multiply data by a twiddle stored in Montgomery form
    __device__ static inline uint32_t mul_tw(uint32_t a, uint32_t tw) { return mont(a, tw); }
    // product of two Montgomery-form twiddles, in Montgomery form
    __device__ static inline uint32_t tw_combine(uint32_t hi, uint32_t lo) { return mont(hi, lo); }
    __device__ static inline uint32_t canon(uint32_t a) { return a; }
    __device__ static inline uint32_t from_bit(uint32_t b) { return b; }

    // host/compile-time helpers
    __host__ __device__ static constexpr uint32_t mulmod(uint32_t a, uint32_t b) {
        return (uint32_t)((uint64_t)a * b % P);
    }
    __host__ __device__ static constexpr uint32_t powmod(uint32_t a, uint64_t e) {
        uint32_t r = 1;
        while (e) {
            if (e & 1) r = mulmod(r, a);
            a = mulmod(a, a);
            e >>= 1;
        }
        return r;
    }
    __host__ __device__ static constexpr uint32_t to_tw(uint32_t w) {  // Montgomery form
        return (uint32_t)(((uint64_t)w << 32) % P);
    }
};

// ------------------------------------------------------------ Goldilocks 2^64 - 2^32 + 1
struct FGL {
    using T = uint64_t;
    static constexpr uint64_t P = 0xFFFFFFFF00000001ull;
    static constexpr uint64_t EPS = 0xFFFFFFFFull;  // 2^64 mod P
    static constexpr int LGMAX = 32;
    // order 2^32, chosen (as a power of 7^((P-1)/2^32), 7 generating the group) so
    // that WMAX^(2^26) = 8: the 64th roots of unity are then powers of 2.
    static constexpr uint64_t WMAX = 5980198667562970375ull;
    static constexpr int WORD_BITS = 64;

    // a + b for any 64-bit representatives: each wrap past 2^64 is worth EPS; the
    // first correction can wrap once more, the second cannot.
    __device__ static inline uint64_t add(uint64_t a, uint64_t b) {
        uint64_t s, s2;
        bool c = __builtin_add_overflow(a, b, &s);
        bool c2 = __builtin_add_overflow(s, c ? EPS : 0ull, &s2);
        return s2 + (c2 ? EPS : 0ull);
    }
    __device__ static inline uint64_t sub(uint64_t a, uint64_t b) {
        uint64_t d, d2;
        bool c = __builtin_sub_overflow(a, b, &d);
        bool c2 = __builtin_sub_overflow(d, c ? EPS : 0ull, &d2);
        return d2 - (c2 ? EPS : 0ull);
    }
    // 128-bit x = x3*2^96 + x2*2^64 + (x1:x0)  ->  (x1:x0) - x3 + x2*(2^32 - 1)  (mod P)
    __device__ static inline uint64_t reduce128(uint64_t hi, uint64_t lo) {
        uint64_t x3 = hi >> 32, x2 = hi & EPS;
        uint64_t t0;
        if (__builtin_sub_overflow(lo, x3, &t0)) t0 -= EPS;  // t0 >= 2^64 - 2^32 + 1 here: no second wrap
        uint64_t t1 = (x2 << 32) - x2;                      // x2 * EPS < 2^64
        uint64_t r;
        bool c = __builtin_add_overflow(t0, t1, &r);        // r <= 2^64 - 2^33 after a wrap
        return r + (c ? EPS : 0ull);
    }
    __device__ static inline uint64_t mul(uint64_t a, uint64_t b) {
        return reduce128(__umul64hi(a, b), a * b);
    }
    __device__ static inline uint64_t mont(uint64_t a, uint64_t b) { return mul(a, b); }
    __device__ static inline uint64_t mul_tw(uint64_t a, uint64_t tw) { return mul(a, tw); }
    __device__ static inline uint64_t tw_combine(uint64_t hi, uint64_t lo) { return mul(hi, lo); }
    __device__ static inline uint64_t canon(uint64_t a) { return a >= P ? a - P : a; }
    __device__ static inline uint64_t from_bit(uint32_t b) { return b; }

    __host__ __device__ static constexpr uint64_t mulmod(uint64_t a, uint64_t b) {
        return (uint64_t)((unsigned __int128)a * b % P);
    }
    __host__ __device__ static constexpr uint64_t powmod(uint64_t a, uint64_t e) {
        uint64_t r = 1;
        while (e) {
            if (e & 1) r = mulmod(r, a);
            a = mulmod(a, a);
            e >>= 1;
        }
        return r;
    }
    __host__ __device__ static constexpr uint64_t to_tw(uint64_t w) { return w; }
};

// Compile-time table of the RAD-th roots of unity w_RAD^k (k < RAD) in twiddle form.
template <class F, int RAD>
struct RootsOf {
    typename F::T w[RAD];
    constexpr RootsOf() : w() {
        typename F::T r = F::powmod(F::WMAX, (uint64_t(1) << F::LGMAX) / RAD);
        typename F::T acc = 1;
        for (int k = 0; k < RAD; ++k) {
            w[k] = F::to_tw(acc);
            acc = F::mulmod(acc, r);
        }
    }
};

}  // namespace ext
