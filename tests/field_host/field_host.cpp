// The kernels' own field routines (csrc/field.h), compiled for the CPU and
// exported over arrays, so that tests/test_field_host.py can check every routine
// against exact integer arithmetic. Test infrastructure only.
#include <stddef.h>
#include <stdint.h>
#include "../../paper_2402_09481_amd/csrc/field.h"

using namespace ext;

template <int S>
static uint64_t gl_pow2_dispatch(uint64_t x, int s) {
    if constexpr (S < 192) {
        if (s == S) return FGL::mul_pow2<S>(x);
        return gl_pow2_dispatch<S + 1>(x, s);
    } else {
        return 0;
    }
}

template <int RAD, int K>
static uint32_t lz_root_dispatch(uint32_t x, int k) {
    if constexpr (K < RAD) {
        if (k == K) return FLZ::mul_root<RAD, K>(x);
        return lz_root_dispatch<RAD, K + 1>(x, k);
    } else {
        return 0;
    }
}

extern "C" {
// op: 0 mul, 1 add (b made canonical first, as every call site does), 2 sub (same),
// 3 canon, 4 x * 2^s for s = b (0 <= s < 192), 5 reduce(x3 = a >> 32, x2 = a, lo = b)
void fgl_op(int op, const uint64_t *a, const uint64_t *b, uint64_t *out, size_t n) {
    for (size_t i = 0; i < n; ++i) {
        switch (op) {
            case 0: out[i] = FGL::mul(a[i], b[i]); break;
            case 1: out[i] = FGL::add(a[i], FGL::as_b(b[i])); break;
            case 2: out[i] = FGL::sub(a[i], FGL::as_b(b[i])); break;
            case 3: out[i] = FGL::canon(a[i]); break;
            case 4: out[i] = gl_pow2_dispatch<0>(a[i], (int)b[i]); break;
            default: out[i] = FGL::reduce((uint32_t)(a[i] >> 32), (uint32_t)a[i], b[i]); break;
        }
    }
}
// 32-bit fields: field 0 = 15*2^27+1, 1 = 3*2^30+1; op: 0 mont, 1 add, 2 sub
void f32_op(int field, int op, const uint32_t *a, const uint32_t *b, uint32_t *out, size_t n) {
    for (size_t i = 0; i < n; ++i) {
        if (field == 0)
            out[i] = op == 0 ? FBB::mont(a[i], b[i]) : op == 1 ? FBB::add(a[i], b[i]) : FBB::sub(a[i], b[i]);
        else
            out[i] = op == 0 ? FP0::mont(a[i], b[i]) : op == 1 ? FP0::add(a[i], b[i]) : FP0::sub(a[i], b[i]);
    }
}
// lazy field 7*2^26+1 (values in [0, 4P)): op 0 mont, 1 butterfly sum
// add(as_a(a), as_b(b)), 2 butterfly difference sub(as_a(a), as_b(b)), 3 canon,
// 4 Shoup product by the in-pass twiddle pair of b (b < P), 5-8 mul_root<RAD, b>
// for RAD = 2, 4, 8, 16
void flz_op(int op, const uint32_t *a, const uint32_t *b, uint32_t *out, size_t n) {
    for (size_t i = 0; i < n; ++i) {
        switch (op) {
            case 0: out[i] = FLZ::mont(a[i], b[i]); break;
            case 1: out[i] = FLZ::add(FLZ::as_a(a[i]), FLZ::as_b(b[i])); break;
            case 2: out[i] = FLZ::sub(FLZ::as_a(a[i]), FLZ::as_b(b[i])); break;
            case 3: out[i] = FLZ::canon(a[i]); break;
            case 4: out[i] = FLZ::mul_tw(a[i], FLZ::to_stk(b[i])); break;
            // butterflies whose second operand is a constant product as it comes
            // (no as_b: CONST_PRODUCT_REDUCED); the constant is 3^7 (w_max)
            case 9: out[i] = FLZ::add(FLZ::as_a(a[i]), FLZ::mul_tw(b[i], FLZ::to_stk(FLZ::WMAX))); break;
            case 10: out[i] = FLZ::sub(FLZ::as_a(a[i]), FLZ::mul_tw(b[i], FLZ::to_stk(FLZ::WMAX))); break;
            // a first operand that is itself a constant product (no as_a)
            case 11: out[i] = FLZ::add(FLZ::mul_tw(a[i], FLZ::to_stk(FLZ::WMAX)), FLZ::as_b(b[i])); break;
            case 12: out[i] = FLZ::sub(FLZ::mul_tw(a[i], FLZ::to_stk(FLZ::WMAX)), FLZ::as_b(b[i])); break;
            case 5: out[i] = lz_root_dispatch<2, 0>(a[i], (int)b[i]); break;
            case 6: out[i] = lz_root_dispatch<4, 0>(a[i], (int)b[i]); break;
            case 7: out[i] = lz_root_dispatch<8, 0>(a[i], (int)b[i]); break;
            default: out[i] = lz_root_dispatch<16, 0>(a[i], (int)b[i]); break;
        }
    }
}
}
