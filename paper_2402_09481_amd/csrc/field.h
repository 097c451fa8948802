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
//   FP0: p = 3 * 2^30 + 1 (> 2^31, < 2^32), 32-bit words, L <= 2^30. As FBB
//        (canonical values, Montgomery products with R = 2^32, Montgomery-form
//        twiddles), but a + b of two canonical values can pass 2^32, so add
//        and sub use the carry / borrow instead of the unsigned-min trick.
//   FGL: p = 2^64 - 2^32 + 1, 64-bit words, L <= 2^32. Values are any 64-bit
//        representative (< 2^64) of their class; only canon() returns the
//        representative in [0, p). 2^64 = 2^32 - 1 (mod p) and 2^96 = -1 (mod p)
//        give a multiply-free reduction of 128-bit products.
//   FLZ: p = 7 * 2^26 + 1 (< 2^29), 32-bit words, L <= 2^26. Small enough that
//        values can be kept lazily in [0, 4p) (4p < 2^31): a butterfly reduces
//        its first operand to [0, 2p) with one compare-subtract, its second comes
//        out of a product in [0, 2p) (or is reduced the same way), and the sum
//        and the difference plus 2p need no reduction (Harvey's butterfly).
//        Products by known constants (the in-register roots and the in-pass
//        twiddles) are Shoup products: with w' = floor(w 2^32 / p), x w -
//        mulhi(x, w') p lies in [0, 2p) for any x < 2^32. Products of two
//        variables (the pointwise product) and the twiddles between passes
//        (Montgomery-form tables) use Montgomery products, whose result lies
//        in [0, 3p). Only canon() returns the representative in [0, p).
//
// Besides the values' type T every field names TW, the type of the in-pass
// (Stockham) twiddle table entries: T itself, or for FLZ the pair w | w' << 32.
// as_a / as_b prepare a butterfly's first / second operand for add and sub;
// CONST_PRODUCT_REDUCED says that mul_root and mul_tw already return operands
// in that form.
//
// Every field uses one fixed primitive root of unity w_max of order 2^LGMAX;
// every transform of length L uses w_L = w_max^(2^LGMAX / L), so that all
// sub-transforms of a multi-pass transform agree on their roots.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ext {

// ------------------------------------------------------------ 15 * 2^27 + 1
struct FBB {
    using T = uint32_t;
    using TW = uint32_t;
    static constexpr uint32_t P = 0x78000001u;
    static constexpr uint32_t PINV = 2281701377u;  // P^-1 mod 2^32
    static constexpr int LGMAX = 27;
    static constexpr uint32_t WMAX = 440564289u;   // 31^15: order 2^27 (31 generates the group)
    static constexpr uint32_t R_MOD_P = 268435454u; // 2^32 mod P (Montgomery form of 1)
    static constexpr int WORD_BITS = 32;
    static constexpr bool CONST_PRODUCT_REDUCED = false;  // see FLZ

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
    // multiply data by a twiddle stored in Montgomery form (in-pass and between passes)
    __device__ static inline uint32_t mul_tw(uint32_t a, uint32_t tw) { return mont(a, tw); }
    __device__ static inline uint32_t mul_ip(uint32_t a, uint32_t tw) { return mont(a, tw); }
    // product of two Montgomery-form twiddles, in Montgomery form
    __device__ static inline uint32_t tw_combine(uint32_t hi, uint32_t lo) { return mont(hi, lo); }
    __device__ static inline uint32_t canon(uint32_t a) { return a; }
    __device__ static inline uint32_t from_bit(uint32_t b) { return b; }
    __device__ static inline uint32_t as_a(uint32_t v) { return v; }
    __device__ static inline uint32_t as_b(uint32_t v) { return v; }
    // x * w_RAD^K with the root's Montgomery form as a compile-time constant
    template <int RAD, int K>
    __device__ static inline uint32_t mul_root(uint32_t x);

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
    __host__ __device__ static constexpr uint32_t to_stk(uint32_t w) { return to_tw(w); }
};

// ------------------------------------------------------------ 3 * 2^30 + 1
struct FP0 {
    using T = uint32_t;
    using TW = uint32_t;
    static constexpr uint32_t P = 0xC0000001u;
    static constexpr uint32_t PINV = 1073741825u;  // P^-1 mod 2^32
    static constexpr int LGMAX = 30;
    static constexpr uint32_t WMAX = 125u;         // 5^3: order 2^30 (5 generates the group)
    static constexpr uint32_t R_MOD_P = 1073741823u; // 2^32 mod P (Montgomery form of 1)
    static constexpr int WORD_BITS = 32;
    static constexpr bool CONST_PRODUCT_REDUCED = false;  // see FLZ

    // a, b in [0, P): a + b < 2P may carry out of 32 bits; the result is
    // a + b - P when it carried or reached P (no borrow in s - P), else a + b.
    __device__ static inline uint32_t add(uint32_t a, uint32_t b) {
        uint32_t s, t;
        const bool c = __builtin_add_overflow(a, b, &s);
        const bool below = __builtin_sub_overflow(s, P, &t);
        return (c || !below) ? t : s;
    }
    // the borrow of a - b selects the correction (written out, so that operands
    // known to be high halves of products are not compared as 64-bit values)
    __device__ static inline uint32_t sub(uint32_t a, uint32_t b) {
        uint32_t d;
        const bool borrow = __builtin_sub_overflow(a, b, &d);
        return borrow ? d + P : d;
    }
    // Montgomery product a*b*2^-32 mod P for a, b < P (signed variant, as FBB):
    // hi - mulhi(q, P) lies in (-P, P) since hi = (a b) >> 32 < P.
    __device__ static inline uint32_t mont(uint32_t a, uint32_t b) {
        const uint32_t lo = a * b;
        const uint32_t hi = __umulhi(a, b);
        const uint32_t q = lo * PINV;
        const uint32_t m = __umulhi(q, P);
        return sub(hi, m);
    }
    __device__ static inline uint32_t mul_tw(uint32_t a, uint32_t tw) { return mont(a, tw); }
    __device__ static inline uint32_t mul_ip(uint32_t a, uint32_t tw) { return mont(a, tw); }
    __device__ static inline uint32_t tw_combine(uint32_t hi, uint32_t lo) { return mont(hi, lo); }
    __device__ static inline uint32_t canon(uint32_t a) { return a; }
    __device__ static inline uint32_t from_bit(uint32_t b) { return b; }
    __device__ static inline uint32_t as_a(uint32_t v) { return v; }
    __device__ static inline uint32_t as_b(uint32_t v) { return v; }
    template <int RAD, int K>
    __device__ static inline uint32_t mul_root(uint32_t x);

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
    __host__ __device__ static constexpr uint32_t to_stk(uint32_t w) { return to_tw(w); }
};

// ------------------------------------------------------------ Goldilocks 2^64 - 2^32 + 1
struct FGL {
    using T = uint64_t;
    using TW = uint64_t;
    static constexpr uint64_t P = 0xFFFFFFFF00000001ull;
    static constexpr uint64_t EPS = 0xFFFFFFFFull;  // 2^64 mod P
    static constexpr int LGMAX = 32;
    // order 2^32, chosen (as a power of 7^((P-1)/2^32), 7 generating the group) so
    // that WMAX^(2^26) = 8: the 64th roots of unity are then powers of 2, and
    // w_RAD^k = 2^(192 k / RAD) for RAD <= 64 (2^96 = -1, so 2 has order 192).
    static constexpr uint64_t WMAX = 5980198667562970375ull;
    static constexpr int WORD_BITS = 64;
    static constexpr bool CONST_PRODUCT_REDUCED = false;  // see FLZ

    // representative in [0, P): subtracting P is adding EPS mod 2^64
    __device__ static inline uint64_t canon(uint64_t a) { return a + (a >= P ? EPS : 0ull); }
    // a + b for any a < 2^64 and b < P: a single wrap past 2^64 (worth EPS) leaves
    // a + b - 2^64 < P, so adding EPS cannot wrap again.
    __device__ static inline uint64_t add(uint64_t a, uint64_t b) {
        uint64_t s = a + b;
        return s + (s < b ? EPS : 0ull);
    }
    // a - b for any a < 2^64 and b < P, on 32-bit halves so that the borrow of
    // the high half selects the correction: after a borrow a - b + 2^64 > EPS, so
    // adding P = 2^64 - EPS (low half + 1, high half - 1) cannot wrap again.
    __device__ static inline uint64_t sub(uint64_t a, uint64_t b) {
        unsigned b0, b1, k, k2;
        const uint32_t d0 = __builtin_subc((uint32_t)a, (uint32_t)b, 0u, &b0);
        const uint32_t d1 = __builtin_subc((uint32_t)(a >> 32), (uint32_t)(b >> 32), b0, &b1);
        const uint32_t e0 = __builtin_addc(d0, 0u, b1, &k);
        const uint32_t e1 = __builtin_addc(d1, b1 ? 0xFFFFFFFFu : 0u, k, &k2);
        return ((uint64_t)e1 << 32) | e0;
    }
    // 128-bit x = x3*2^96 + x2*2^64 + lo (any limbs). With 2^64 = EPS and
    // 2^96 = -1: x3*2^96 + x2*2^64 = x2*EPS - x3 = (x2 - 1)*EPS + ~x3 + [x2 == 0],
    // where (x2 - 1 mod 2^32)*EPS + ~x3 <= EPS^2 is one multiply-add and the
    // [x2 == 0] term is the borrow of x2 - 1, fed in as the carry of the next add.
    // A wrap of lo + v past 2^64 is worth EPS; after it the sum is at most
    // EPS^2 + EPS, so adding EPS cannot wrap again.
    __device__ static inline uint64_t reduce(uint32_t x3, uint32_t x2, uint64_t lo) {
        unsigned bz, c0, c1, k, k2;
        const uint32_t x2m1 = __builtin_subc(x2, 1u, 0u, &bz);
        const uint64_t v = (uint64_t)x2m1 * EPS + (uint64_t)(uint32_t)~x3;
        const uint32_t r0 = __builtin_addc((uint32_t)lo, (uint32_t)v, bz, &c0);
        uint32_t r1 = __builtin_addc((uint32_t)(lo >> 32), (uint32_t)(v >> 32), c0, &c1);
#if defined(__HIP_DEVICE_COMPILE__)
        // keep r1 in a register: otherwise r1 + k is refolded into a three-input
        // add that needs c0 as a value (two more instructions); emits no code
        asm("" : "+v"(r1));
#endif
        const uint32_t s0 = __builtin_addc(r0, c1 ? 0xFFFFFFFFu : 0u, 0u, &k);
        const uint32_t s1 = __builtin_addc(r1, 0u, k, &k2);
        return ((uint64_t)s1 << 32) | s0;
    }
    __device__ static inline uint64_t reduce128(uint64_t hi, uint64_t lo) {
        return reduce((uint32_t)(hi >> 32), (uint32_t)hi, lo);
    }
    // a * b mod P (result < 2^64, not necessarily canonical); schoolbook on 32-bit
    // halves with 32x32+64 multiply-adds. The two high halves of the middle
    // products are summed into a 33-bit addend of the top product (no overflow:
    // (2^32-1)^2 + 2^33 - 2 < 2^64), so the top product is already limbs x3:x2.
    __device__ static inline uint64_t mul(uint64_t a, uint64_t b) {
        const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
        const uint64_t t00 = (uint64_t)a0 * b0;
        const uint64_t t10 = (uint64_t)a1 * b0 + (t00 >> 32);
        const uint64_t t01 = (uint64_t)a0 * b1 + (uint32_t)t10;
        unsigned c;
        const uint32_t s = __builtin_addc((uint32_t)(t10 >> 32), (uint32_t)(t01 >> 32), 0u, &c);
        const uint64_t t11 = (uint64_t)a1 * b1 + (((uint64_t)c << 32) | s);
        const uint64_t lo = (t01 << 32) | (uint32_t)t00;
        return reduce((uint32_t)(t11 >> 32), (uint32_t)t11, lo);
    }
    // x * 2^S mod P for a compile-time S (not necessarily canonical).
    template <int S>
    __device__ static inline uint64_t mul_pow2(uint64_t x) {
        constexpr int s = ((S % 192) + 192) % 192;
        if constexpr (s == 0) {
            return x;
        } else if constexpr (s >= 96) {  // 2^96 = -1
            return P - canon(mul_pow2<s - 96>(x));
        } else if constexpr (s < 32) {
            // x 2^s = hi*2^64 + lo with hi < 2^32: lo + hi*EPS
            uint64_t r;
            bool c = __builtin_add_overflow(x << s, (uint64_t)(uint32_t)(x >> (64 - s)) * EPS, &r);
            return r + (c ? EPS : 0ull);  // r < 2^63 after a wrap
        } else if constexpr (s == 32) {
            // x 2^32 = x1*2^64 + x0*2^32: (x0 << 32) + x1*EPS
            uint64_t r;
            bool c = __builtin_add_overflow(x << 32, (uint64_t)(uint32_t)(x >> 32) * EPS, &r);
            return r + (c ? EPS : 0ull);
        } else if constexpr (s < 64) {
            return reduce128(x >> (64 - s), x << s);
        } else if constexpr (s == 64) {
            return reduce128(x, 0ull);
        } else {
            // 64 < s < 96, k = s - 64: x 2^k = h 2^64 + y (h < 2^32), so
            // x 2^s = h 2^128 + y 2^64 with 2^128 = -2^32; -h 2^32 is taken as
            // P - h 2^32 = (~h) 2^32 + 1, the low word beside limbs y = x3:x2.
            constexpr int k = s - 64;
            const uint64_t y = x << k;
            const uint32_t h = (uint32_t)(x >> (64 - k));
            return reduce128(y, ((uint64_t)(uint32_t)~h << 32) | 1u);
        }
    }
    // x * w_RAD^K (the compile-time roots of the in-register DFTs)
    template <int RAD, int K>
    __device__ static inline uint64_t mul_root(uint64_t x) {
        return mul_pow2<(192 / RAD) * K>(x);
    }
    __device__ static inline uint64_t mont(uint64_t a, uint64_t b) { return mul(a, b); }
    __device__ static inline uint64_t mul_tw(uint64_t a, uint64_t tw) { return mul(a, tw); }
    __device__ static inline uint64_t mul_ip(uint64_t a, uint64_t tw) { return mul(a, tw); }
    __device__ static inline uint64_t tw_combine(uint64_t hi, uint64_t lo) { return mul(hi, lo); }
    __device__ static inline uint64_t from_bit(uint32_t b) { return b; }
    // operands prepared for add/sub: the first may be any representative, the
    // second must be canonical
    __device__ static inline uint64_t as_a(uint64_t v) { return v; }
    __device__ static inline uint64_t as_b(uint64_t v) { return canon(v); }

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
    __host__ __device__ static constexpr uint64_t to_stk(uint64_t w) { return w; }
};

// ------------------------------------------------------------ 7 * 2^26 + 1, lazy
struct FLZ {
    using T = uint32_t;
    using TW = uint64_t;  // Shoup pair: w | w' << 32, w' = floor(w 2^32 / P)
    static constexpr uint32_t P = 469762049u;     // 7 * 2^26 + 1
    static constexpr uint32_t P2 = 2 * P;
    static constexpr uint32_t PINV = 3825205249u; // P^-1 mod 2^32
    static constexpr int LGMAX = 26;
    static constexpr uint32_t WMAX = 2187u;       // 3^7: order 2^26 (3 generates the group)
    static constexpr uint32_t R_MOD_P = 67108855u; // 2^32 mod P (Montgomery form of 1)
    static constexpr int WORD_BITS = 32;
    // the products by known constants (mul_root, mul_tw) return butterfly operands
    // as they are: their Shoup results lie in [0, 2P), so as_a / as_b are not needed
    static constexpr bool CONST_PRODUCT_REDUCED = true;

    __host__ __device__ static constexpr uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }
    // [0, 4P) -> [0, 2P): if v >= 2P, v - 2P < v; otherwise v - 2P wraps above v
    __device__ static inline uint32_t red2(uint32_t v) { return umin(v, v - P2); }
    __device__ static inline uint32_t as_a(uint32_t v) { return red2(v); }
    __device__ static inline uint32_t as_b(uint32_t v) { return red2(v); }
    // a, b in [0, 2P): a + b and a - b + 2P lie in [0, 4P)
    __device__ static inline uint32_t add(uint32_t a, uint32_t b) { return a + b; }
    __device__ static inline uint32_t sub(uint32_t a, uint32_t b) { return a - b + P2; }
    // Shoup product x w for x < 2^32, w < P, wq = floor(w 2^32 / P): with
    // q = floor(x wq / 2^32), x w - q P lies in [0, 2P); computed mod 2^32
    __device__ static inline uint32_t shoup(uint32_t x, uint32_t w, uint32_t wq) {
        const uint32_t q = __umulhi(x, wq);
        return x * w - q * P;
    }
    __device__ static inline uint32_t mul_tw(uint32_t a, uint64_t tw) {
        return shoup(a, (uint32_t)tw, (uint32_t)(tw >> 32));
    }
    // Montgomery product a b 2^-32 for a, b < 4P: a b < 16 P^2, so its high half
    // is below 16 P^2 / 2^32 < 2P; hi - mulhi(q, P) lies in (-P, 2P), and + P puts
    // it in (0, 3P)
    __device__ static inline uint32_t mont(uint32_t a, uint32_t b) {
        const uint32_t lo = a * b;
        const uint32_t hi = __umulhi(a, b);
        const uint32_t q = lo * PINV;
        return hi - __umulhi(q, P) + P;
    }
    // between passes: twiddles in Montgomery form
    __device__ static inline uint32_t mul_ip(uint32_t a, uint32_t tw) { return mont(a, tw); }
    __device__ static inline uint32_t tw_combine(uint32_t hi, uint32_t lo) { return mont(hi, lo); }
    __device__ static inline uint32_t canon(uint32_t a) {
        const uint32_t b = red2(a);
        return umin(b, b - P);
    }
    __device__ static inline uint32_t from_bit(uint32_t b) { return b; }
    template <int RAD, int K>
    __device__ static inline uint32_t mul_root(uint32_t x);

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
    __host__ __device__ static constexpr uint32_t shoup_q(uint32_t w) { return (uint32_t)(((uint64_t)w << 32) / P); }
    __host__ __device__ static constexpr uint64_t to_stk(uint32_t w) {
        return (uint64_t)w | ((uint64_t)shoup_q(w) << 32);
    }
};

template <int RAD, int K>
__device__ inline uint32_t FBB::mul_root(uint32_t x) {
    constexpr uint32_t w = FBB::powmod(FBB::powmod(FBB::WMAX, (uint64_t(1) << FBB::LGMAX) / RAD), K);
    return mont(x, FBB::to_tw(w));
}

template <int RAD, int K>
__device__ inline uint32_t FP0::mul_root(uint32_t x) {
    constexpr uint32_t w = FP0::powmod(FP0::powmod(FP0::WMAX, (uint64_t(1) << FP0::LGMAX) / RAD), K);
    return mont(x, FP0::to_tw(w));
}

static_assert((uint32_t)(FLZ::P * FLZ::PINV) == 1u, "PINV is the inverse of P mod 2^32");
static_assert((uint64_t(1) << 32) % FLZ::P == FLZ::R_MOD_P, "R mod P");
static_assert(uint64_t(4) * FLZ::P < (uint64_t(1) << 31), "lazy values below 4P fit 31 bits");
static_assert(FLZ::powmod(FLZ::WMAX, uint64_t(1) << 25) == FLZ::P - 1, "w_max has order 2^26");

template <int RAD, int K>
__device__ inline uint32_t FLZ::mul_root(uint32_t x) {
    constexpr uint32_t w = FLZ::powmod(FLZ::powmod(FLZ::WMAX, (uint64_t(1) << FLZ::LGMAX) / RAD), K);
    return shoup(x, w, FLZ::shoup_q(w));
}

}  // namespace ext
