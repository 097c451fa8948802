// Transform kernels for the convolution extractors.
//
// The extractor output is the mod-2 reduction of an exact integer cyclic
// convolution of two 0/1 vectors (Alg. 1 / Alg. 2), computed with the
// convolution theorem: NTT(u * v) = NTT(u) . NTT(v) (section "The
// number-theoretic transform and the convolution theorem").
//
// A transform of length L = R_1 R_2 ... R_k is done in k passes (the
// "four-step" factorisation applied recursively). Pass i transforms, for each
// block of size M_{i-1} = R_i ... R_k, the columns of that block viewed as an
// R_i x M_i row-major matrix, then multiplies entry (row k_i, column c) by
// w_{M_{i-1}}^(c k_i). The spectrum ends up in digit-reversed order, which is
// harmless: the pointwise product is order-agnostic, and the inverse runs the
// passes backwards (twiddles w^-(c k_i) applied before each column
// transform), returning the convolution in natural order.
//
// Inside a pass each column (or row) of length R = 2^lgr is transformed by
// radix-16 Stockham steps (the first forward step takes the leftover radix
// 2, 4 or 8), exchanging data through LDS between steps. Step with radix r
// and span Ns: group j reads elements j + t R/r (t < r), multiplies element
// t by w_{Ns r}^(t (j mod Ns)), does an r-point DFT in registers and writes
// output t to ((j - j mod Ns) r + j mod Ns) + t Ns. The output is in natural
// order. The last step's output positions are the first step's input
// positions of the same radix, so consecutive steps of opposite direction
// can hand data over in registers.
//
// Passes:
//   strided    S_FWD_BITS: embed packed bits (first pass of a forward transform)
//              S_FWD: column transform, then twiddle, in place
//              S_INV: twiddle^-1, then inverse column transform, in place
//              S_INV_PARITY: as S_INV, then canonical residue mod 2, packed
//              (the last inverse pass also applies L^-1 and computes only the
//              rows that hold output coefficients)
//   contiguous C_FWD: row transform (last level of a forward transform)
//              C_FUSED: row transform of one operand, times the other operand's
//              spectrum (S), inverse row transform (last forward level, the
//              pointwise product, first inverse level)
//              C_PROD, C_FUSED2: the two-piece schedule's second-piece product
//              and its first piece's fused pass with that product added
//   small      whole extraction of one job in one workgroup (L <= 2^14)
#include <algorithm>
#include <cstring>
#include <tuple>
#include <type_traits>
#include <utility>

#include "field.h"
#include "kernels.h"

// The file is compiled once per part (NTT_PART = 0..9) so that the template
// instantiations build in parallel; without NTT_PART everything is built.
#ifndef NTT_PART
#define NTT_PART -1
#endif
#define NTT_HAS(k) (NTT_PART < 0 || NTT_PART == (k))

namespace ext {

// ------------------------------------------------------------------ launching

extern thread_local GraphRecorder *t_graph_recorder;

// Launches kern on stream s, or adds it to the recording graph of this thread.
// The arguments are converted to the kernel's parameter types first; both paths
// pass pointers to those values (a graph node copies them when it is added).
template <typename... P, typename... A>
static hipError_t launch_k(void (*kern)(P...), dim3 grid, dim3 block, size_t shmem, hipStream_t s, A &&...args) {
    static_assert(sizeof...(P) == sizeof...(A), "argument count");
    std::tuple<std::decay_t<P>...> vals(std::forward<A>(args)...);
    void *ptrs[sizeof...(P) > 0 ? sizeof...(P) : 1];
    std::apply([&](auto &...v) {
        int i = 0;
        ((ptrs[i++] = (void *)&v), ...);
    }, vals);
    if (GraphRecorder *r = t_graph_recorder) {
        if (r->err != hipSuccess) return r->err;
        hipKernelNodeParams kp = {};
        kp.func = (void *)kern;
        kp.gridDim = grid;
        kp.blockDim = block;
        kp.sharedMemBytes = (unsigned)shmem;
        kp.kernelParams = ptrs;
        kp.extra = nullptr;
        hipGraphNode_t node = nullptr;
        r->err = hipGraphAddKernelNode(&node, r->graph, r->last ? &r->last : nullptr, r->last ? 1 : 0, &kp);
        if (r->err == hipSuccess) r->last = node;
        return r->err;
    }
    return hipLaunchKernel((const void *)kern, grid, block, ptrs, shmem, s);
}

// ------------------------------------------------------------------ helpers

// The Dodis degenerate-input check's result, from the flags of its parts (see
// degen_part): x has no one bit or no zero bit among its first degen_n bits.
constexpr uint32_t DEGEN_PARTS_MAX = 31;
__device__ inline bool degenerate(const JobDev &J) {
    if (!J.degen_n) return false;
    const uint32_t parts = J.flags[0] < DEGEN_PARTS_MAX ? J.flags[0] : DEGEN_PARTS_MAX;
    uint32_t one_ = 0, zero_ = 0;
    for (uint32_t g = 0; g < parts; ++g) {
        one_ |= J.flags[2 + 2 * g];
        zero_ |= J.flags[3 + 2 * g];
    }
    return one_ == 0 || zero_ == 0;
}


__host__ __device__ inline uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

// An unsigned integer of C bits (one row segment of a strided tile as bits).
template <int C>
using UnitOf = typename std::conditional<C == 8, uint8_t, typename std::conditional<C == 16, uint16_t, uint32_t>::type>::type;

// Loads and stores through the global address space. A pointer read from a job
// descriptor is otherwise a flat access, which also counts against the LDS wait
// counter, so that every barrier (which waits for LDS) would wait for it too.
template <class T>
__device__ inline T gload(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ inline void gstore(T *p, T v) {
    *(__attribute__((address_space(1))) T *)p = v;
}

__host__ __device__ inline uint32_t getbit(const uint64_t *b, uint64_t i) {
    return (uint32_t)(b[i >> 6] >> (i & 63)) & 1u;
}

__host__ __device__ inline uint64_t mod_small(uint64_t v, uint64_t P) {
    while (v >= P) v -= P;  // v < 3P at every call site
    return v;
}

__host__ __device__ inline uint32_t emb_bit(const Emb &e, uint64_t i, uint64_t L) {
    if (e.mode == EMB_PREFIX) return i < e.len ? getbit(e.bits, i) : 0u;
    if (e.mode == EMB_SEED) {
        uint64_t k = i + e.a;
        if (k >= L) k -= L;
        if (k >= e.N) return 0u;
        return getbit(e.bits, mod_small(k + e.rot, e.P));
    }
    if (i >= e.a) return 0u;
    const uint64_t j = e.N - 1 - i;
    return j < e.len ? getbit(e.bits, j) : 0u;
}

// emb_bit for transforms of at most 2^16 (the single-workgroup path), where
// every position, length and offset of a job fits 32 bits: the index maps as
// 32-bit selects rather than branches (jobs side by side in one wave may differ),
// one load through the global address space per bit. The input's map is PREFIX
// or REV, the seed's is SEED, as for every job the library builds.
__device__ inline uint32_t bit_at32(const uint64_t *b, uint32_t idx, bool ok) {
    idx = ok ? idx : 0u;
    const uint32_t bit = (uint32_t)(gload(b + (idx >> 6)) >> (idx & 63)) & 1u;
    return ok ? bit : 0u;
}
__device__ inline uint32_t emb_bit32_input(const Emb &e, uint32_t i) {
    const bool rev = e.mode == EMB_REV;
    const uint32_t idx = rev ? (uint32_t)e.N - 1u - i : i;
    return bit_at32(e.bits, idx, (!rev || i < (uint32_t)e.a) && idx < (uint32_t)e.len);
}
__device__ inline uint32_t emb_bit32_seed(const Emb &e, uint32_t i, uint32_t L) {
    uint32_t k = i + (uint32_t)e.a;
    k = k >= L ? k - L : k;
    const uint32_t P = (uint32_t)e.P;
    uint32_t v = k + (uint32_t)e.rot;  // < 3P
    v = v >= P ? v - P : v;
    v = v >= P ? v - P : v;
    return bit_at32(e.bits, v, k < (uint32_t)e.N);
}

template <int N>
__host__ __device__ constexpr int bitrev(int i) {
    int r = 0;
    for (int b = 1; b < N; b <<= 1) {
        r = (r << 1) | (i & 1);
        i >>= 1;
    }
    return r;
}

// In-register RAD-point DFT, forward (w_RAD^(t k)) or inverse (w_RAD^-(t k)).
// Iterative radix-2 decimation in time on bit-reversed input; the roots are
// compile-time (for the 64-bit field they are powers of 2, applied by shifts).
// TWD: inputs t >= 1 come straight out of the Stockham twiddle product (where
// the field's constant products return reduced operands, the first layer then
// prepares only input t = 0, at u[0]).
template <class F, int RAD, int LEN, int K, bool TWD = false>
__device__ inline void dft_layer_k(typename F::T *u) {
    if constexpr (K < LEN / 2) {
        constexpr bool RED_IN = F::CONST_PRODUCT_REDUCED && TWD && LEN == 2;
#pragma unroll
        for (int s = 0; s < RAD; s += LEN) {
            typename F::T a = (RED_IN && s + K != 0) ? u[s + K] : F::as_a(u[s + K]);
            typename F::T b = u[s + K + LEN / 2];
            if constexpr (K == 0)
                b = RED_IN ? b : F::as_b(b);
            else if constexpr (F::CONST_PRODUCT_REDUCED)
                b = F::template mul_root<LEN, K>(b);
            else
                b = F::as_b(F::template mul_root<LEN, K>(b));
            u[s + K] = F::add(a, b);
            u[s + K + LEN / 2] = F::sub(a, b);
        }
        dft_layer_k<F, RAD, LEN, K + 1, TWD>(u);
    }
}

template <class F, int RAD, int LEN, bool TWD = false>
__device__ inline void dft_layers(typename F::T *u) {
    if constexpr (LEN <= RAD) {
        dft_layer_k<F, RAD, LEN, 0, TWD && LEN == 2>(u);
        dft_layers<F, RAD, LEN * 2, false>(u);
    }
}

template <class F, int RAD, bool TWD = false>
__device__ inline void dft_reg(typename F::T *v, bool inv) {
    using T = typename F::T;
    T u[RAD];
#pragma unroll
    for (int i = 0; i < RAD; ++i) u[bitrev<RAD>(i)] = v[i];
    dft_layers<F, RAD, 2, TWD>(u);
    // inverse DFT = forward DFT with outputs k and RAD - k exchanged
#pragma unroll
    for (int k = 0; k < RAD; ++k) v[k] = u[inv ? ((RAD - k) & (RAD - 1)) : k];
}

// ------------------------------------------------------------------ tile geometry

// Radix of step s of a 2^lgr-point transform done in radix-16 Stockham steps
// plus one leftover radix RF. A step of radix r multiplies (r-1)/r of its
// values by twiddles, except the first step, which has none; so RF is best
// anywhere but first (9 levels: 16*2*16 takes 1/2 + 15/16 twiddle products per
// value where 2*16*16 takes 15/16 + 15/16). ORDER 1: RF second in both
// directions; ORDER 2: RF second in the forward and last in the inverse (the
// fused pass: as cheap, and fewer registers); ORDER 0: RF first in the forward
// and last in the inverse. With two steps the forward order is always RF, 16
// and the inverse 16, RF, so that a fused pass hands the forward's last
// radix-16 layout to the inverse's first step. Every order gives the same
// transform in the same (natural) order.
__host__ __device__ constexpr int step_radix(int lgr, int order, int s, bool inv) {
    const int rf = (lgr % 4) ? (1 << (lgr % 4)) : 16, nsteps = (lgr + 3) / 4;
    if (nsteps >= 3 && (order == 1 || (order == 2 && !inv))) return s == 1 ? rf : 16;
    if (nsteps >= 2) return inv ? (s == nsteps - 1 ? rf : 16) : (s == 0 ? rf : 16);
    return rf;
}
__host__ __device__ constexpr int step_span(int lgr, int order, int s, bool inv) {
    int ns = 1;
    for (int i = 0; i < s; ++i) ns *= step_radix(lgr, order, i, inv);
    return ns;
}
// Stockham twiddles kept in LDS beside a tile. The block of step s ((radix - 1)
// span words, laid out as the global block; step 0 has none) is local for every
// step of a strided tile, and for the steps of a contiguous tile whose block
// has at most CTW_MAX words (the large blocks of its last steps stay global, so
// that the tile's workgroups per CU do not drop). A strided kernel runs one
// direction; a contiguous tile holds the forward blocks, then the inverse ones.
constexpr int CTW_MAX = 512;
__host__ __device__ constexpr int step_block_words(int lgr, int order, int s, bool inv) {
    return (step_radix(lgr, order, s, inv) - 1) * step_span(lgr, order, s, inv);
}
__host__ __device__ constexpr bool step_twiddle_local(int lgr, int order, bool strided, int s, bool inv) {
    return s >= 1 && s < (lgr + 3) / 4 && (strided || step_block_words(lgr, order, s, inv) <= CTW_MAX);
}
__host__ __device__ constexpr int step_twiddle_dir_words(int lgr, int order, bool strided, bool inv) {
    int o = 0;
    for (int i = 1; i < (lgr + 3) / 4; ++i)
        if (step_twiddle_local(lgr, order, strided, i, inv)) o += step_block_words(lgr, order, i, inv);
    return o;
}
__host__ __device__ constexpr int step_twiddle_off(int lgr, int order, bool strided, int s, bool inv) {
    int o = (strided || !inv) ? 0 : step_twiddle_dir_words(lgr, order, strided, false);
    for (int i = 1; i < s; ++i)
        if (step_twiddle_local(lgr, order, strided, i, inv)) o += step_block_words(lgr, order, i, inv);
    return o;
}
__host__ __device__ constexpr int step_twiddle_words(int lgr, int order, bool strided) {
    const int f = step_twiddle_dir_words(lgr, order, strided, false);
    const int i = step_twiddle_dir_words(lgr, order, strided, true);
    return strided ? (f > i ? f : i) : f + i;
}

// Where the Stockham twiddles of a column or row transform are read from LDS
// (the blocks that step_twiddle_local admits) rather than from the global
// blocks in every step: every strided pass; the contiguous passes without the
// pointwise product and inverse (C_FWD, C_PROD). Measured against global loads
// (the 64-bit field's issued one step early): 64-bit strided passes 5-9%
// faster with half the registers, 32-bit strided passes 8-10% faster, the
// 64-bit row pass 9% faster; the fused row pass 2% slower, so it keeps the
// global loads.
__host__ __device__ constexpr bool lds_twiddles(bool strided, int cmode) {
    return strided || cmode == C_FWD || cmode == C_PROD || cmode == C_PROD_ADD;
}
// The row passes that fuse the product with the transforms around it (C_FUSED,
// C_FUSED2) take the twiddle blocks of both directions from LDS as well in the
// lazy field, whose twiddles are Shoup pairs of two registers each: from global
// memory a step's fifteen pairs are loaded ahead of its butterflies and keep the
// pass above the register count at which more of its workgroups fit a CU.
template <class F>
__host__ __device__ constexpr bool fused_lds_twiddles() {
    return std::is_same<F, FLZ>::value;
}
// SMODE: the pass mode (StridedMode for strided tiles, ContigMode otherwise).
template <class F, int LGR, bool STRIDED, int ORDER = 1, int SMODE = S_FWD_BITS>
struct Tile {
    using T = typename F::T;
    static constexpr int R = 1 << LGR;
    // strided tiles: C adjacent columns give 128-byte row segments in HBM
    static constexpr int C = STRIDED ? strided_cols(F::WORD_BITS, SMODE) : (R >= 2048 ? 1 : 2048 / R);
    static constexpr int NT0 = C * R / 16;
    static constexpr int NT = NT0 > 1024 ? 1024 : NT0;
    static constexpr int EPT = C * R / NT;
    static constexpr int RF = (LGR % 4) ? (1 << (LGR % 4)) : 16;
    static constexpr int NSTEPS = (LGR + 3) / 4;
    static_assert(EPT >= 16 && EPT % 16 == 0, "tile too small");
    static_assert(NT % 64 == 0 || NT < 64, "whole waves");

    __host__ __device__ static constexpr int radix(int s, bool inv) { return step_radix(LGR, ORDER, s, inv); }
    __host__ __device__ static constexpr int span(int s, bool inv) { return step_span(LGR, ORDER, s, inv); }
    __host__ __device__ static constexpr bool stw_local(int s, bool inv) {
        return step_twiddle_local(LGR, ORDER, STRIDED, s, inv);
    }
    __host__ __device__ static constexpr int stw_off(int s, bool inv) {
        return step_twiddle_off(LGR, ORDER, STRIDED, s, inv);
    }
    // the step with radix rad and span ns: whether its block is in LDS, and where
    __host__ __device__ static constexpr bool stw_has(int rad, int ns, bool inv) {
        for (int i = 1; i < NSTEPS; ++i)
            if (radix(i, inv) == rad && span(i, inv) == ns) return stw_local(i, inv);
        return false;
    }
    __host__ __device__ static constexpr int stw_block(int rad, int ns, bool inv) {
        for (int i = 1; i < NSTEPS; ++i)
            if (radix(i, inv) == rad && span(i, inv) == ns) return stw_off(i, inv);
        return 0;
    }
    static constexpr bool FUSED_ROW = !STRIDED && (SMODE == C_FUSED || SMODE == C_FUSED2);
    static constexpr bool LT = lds_twiddles(STRIDED, SMODE) || (FUSED_ROW && fused_lds_twiddles<F>());
    // (a contiguous tile with LDS twiddles holds the forward blocks, and the
    // inverse ones after them if it runs both directions)
    static constexpr int STW_WORDS = !LT       ? 0
                                     : STRIDED ? step_twiddle_words(LGR, ORDER, true)
                                     : FUSED_ROW ? step_twiddle_words(LGR, ORDER, false)
                                                 : step_twiddle_dir_words(LGR, ORDER, false, false);
    static_assert(!LT || NSTEPS >= 2, "the LDS twiddles are first read after the first step's barrier");

    // 64-bit strided tiles exchange values between steps through LDS in two 32-bit
    // halves, so that the tile takes half the LDS and twice the workgroups fit a CU
    // (256 rows and more: the smaller tiles would spill at that occupancy)
    static constexpr bool HALFX = STRIDED && sizeof(T) == 8 && LGR >= 8;
    // contiguous tiles pad one word per 16 so that power-of-two strides spread over banks
    static constexpr int RP = STRIDED ? R : R + R / 16;
    static constexpr int TILE_WORDS = STRIDED ? (HALFX ? C * R / 2 : C * R) : C * RP;
    static constexpr int LDS_WORDS = TILE_WORDS + STW_WORDS;
    // Waves per SIMD that strided kernels promise the register allocator: as
    // many as the LDS admits (160 KiB per CU, 4 SIMDs), at most 8. A register
    // count above that would leave LDS idle and halve the resident workgroups
    // (the bit-reading first pass of 32-bit fields needed 72 registers for 64).
    static constexpr int LDS_BYTES = TILE_WORDS * (int)sizeof(T) + STW_WORDS * (int)sizeof(typename F::TW);
    static constexpr int WG_BY_LDS = (160 * 1024) / LDS_BYTES;
    static constexpr int WPE0 = WG_BY_LDS * (NT / 64) / 4;
    static constexpr int WAVES_PER_SIMD = WPE0 < 1 ? 1 : (WPE0 > 8 ? 8 : WPE0);
    __device__ static inline int lidx(int c, int r) { return STRIDED ? r * C + c : c * RP + r + (r >> 4); }
    template <int RAD>
    __device__ static inline void coords(int q, int &c, int &j) {
        int g = (int)threadIdx.x + q * NT;
        if (STRIDED) {
            c = g % C;
            j = g / C;
        } else {
            j = g % (R / RAD);
            c = g / (R / RAD);
        }
    }
};

// Stockham step compute on registers v (EPT values = EPT/RAD groups of RAD).
// Twiddles from the global blocks, or (LT) from the tile's LDS copy stw.
template <class F, class Tl, int RAD, int NS, bool INV, bool LT = false>
__device__ inline void step_compute(typename F::T *v, const Tables &tb, const typename F::TW *stw = nullptr) {
    using TW = typename F::TW;
    static_assert(NS * RAD <= (1 << TWIN_LG) && RAD <= 16, "step beyond the Stockham twiddle blocks");
    const TW *tw = (const TW *)tb.stk + stk_offset(RAD, NS, INV);
    if constexpr (LT) {
        if constexpr (Tl::stw_has(RAD, NS, INV)) tw = stw + Tl::stw_block(RAD, NS, INV);
    }
    constexpr int GPT = Tl::EPT / RAD;
#pragma unroll
    for (int q = 0; q < GPT; ++q) {
        int c, j;
        Tl::template coords<RAD>(q, c, j);
        (void)c;
        if constexpr (NS > 1) {
            const int jm = j & (NS - 1);
#pragma unroll
            for (int t = 1; t < RAD; ++t) v[q * RAD + t] = F::mul_tw(v[q * RAD + t], tw[(t - 1) * NS + jm]);
        }
        dft_reg<F, RAD, (NS > 1)>(&v[q * RAD], INV);
    }
}

template <class Tl, class = void>
struct HasHalfx : std::false_type {};
template <class Tl>
struct HasHalfx<Tl, std::void_t<decltype(Tl::HALFX)>> : std::integral_constant<bool, Tl::HALFX> {};
template <class Tl>
__host__ __device__ constexpr bool tile_halfx() {
    return HasHalfx<Tl>::value;
}

template <class F, class Tl, int RAD>
__device__ inline void step_load_lds(typename F::T *v, const typename F::T *lds) {
    constexpr int GPT = Tl::EPT / RAD;
#pragma unroll
    for (int q = 0; q < GPT; ++q) {
        int c, j;
        Tl::template coords<RAD>(q, c, j);
#pragma unroll
        for (int t = 0; t < RAD; ++t) v[q * RAD + t] = lds[Tl::lidx(c, j + t * (Tl::R / RAD))];
    }
}

template <class F, class Tl, int RAD>
__device__ inline void step_store_lds(const typename F::T *v, typename F::T *lds, int Ns) {
    constexpr int GPT = Tl::EPT / RAD;
#pragma unroll
    for (int q = 0; q < GPT; ++q) {
        int c, j;
        Tl::template coords<RAD>(q, c, j);
        int jm = j & (Ns - 1);
        int d = (j - jm) * RAD + jm;
#pragma unroll
        for (int t = 0; t < RAD; ++t) lds[Tl::lidx(c, d + t * Ns)] = v[q * RAD + t];
    }
}

// The exchange between a step of radix RAD and span NS and the next step (radix
// RADN) in two rounds of 32-bit halves through an LDS tile of C R 32-bit words:
// low halves out in the old layout and in to the new, then the high halves.
template <class F, class Tl, int RAD, int NS, int RADN>
__device__ inline void exchange_halves(typename F::T *v, typename F::T *lds) {
    static_assert(sizeof(typename F::T) == 8, "64-bit values");
    uint32_t *l = (uint32_t *)lds;
    uint32_t part[Tl::EPT];
    __syncthreads();  // every read of the previous layout is done
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (h) __syncthreads();  // the low halves are read
#pragma unroll
        for (int q = 0; q < Tl::EPT / RAD; ++q) {
            int c, j;
            Tl::template coords<RAD>(q, c, j);
            const int jm = j & (NS - 1), d = (j - jm) * RAD + jm;
#pragma unroll
            for (int t = 0; t < RAD; ++t) l[Tl::lidx(c, d + t * NS)] = (uint32_t)(v[q * RAD + t] >> (32 * h));
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Tl::EPT / RADN; ++q) {
            int c, j;
            Tl::template coords<RADN>(q, c, j);
#pragma unroll
            for (int t = 0; t < RADN; ++t) {
                const uint32_t w = l[Tl::lidx(c, j + t * (Tl::R / RADN))];
                if (h == 0)
                    part[q * RADN + t] = w;
                else
                    v[q * RADN + t] = ((uint64_t)w << 32) | part[q * RADN + t];
            }
        }
    }
}

// Run steps [s0, s1) of a transform whose inputs for step s0 are already in
// registers; the outputs of step s1-1 stay in registers (positions of the
// last-step layout if s1 == NSTEPS). LDS exchanges in between. A thread with
// active = false (uniform in its wave) only takes part in the barriers.
template <class F, class Tl, bool INV, int S, bool LT = false>
__device__ inline void run_steps_from(typename F::T *v, typename F::T *lds, const Tables &tb,
                                      const typename F::TW *stw = nullptr, bool active = true) {
    if constexpr (S < Tl::NSTEPS) {
        constexpr int RAD = Tl::radix(S, INV);
        constexpr int NS = Tl::span(S, INV);
        if (active) {
            if constexpr (S > 0 && !tile_halfx<Tl>()) {
                // inputs of this step come from LDS, written by the previous step
                step_load_lds<F, Tl, RAD>(v, lds);
            }
            step_compute<F, Tl, RAD, NS, INV, LT>(v, tb, stw);
        }
        if constexpr (S + 1 < Tl::NSTEPS) {
            if constexpr (tile_halfx<Tl>()) {
                exchange_halves<F, Tl, RAD, NS, Tl::radix(S + 1, INV)>(v, lds);
            } else {
                __syncthreads();  // every read of the previous layout is done
                if (active) step_store_lds<F, Tl, RAD>(v, lds, NS);
                __syncthreads();
            }
            run_steps_from<F, Tl, INV, S + 1, LT>(v, lds, tb, stw, active);
        }
    }
}

template <class Tl, bool INV>
struct Ends {
    static constexpr int RAD_FIRST = Tl::radix(0, INV);
    static constexpr int RAD_LAST = Tl::radix(Tl::NSTEPS - 1, INV);
};

// ------------------------------------------------------------------ strided pass

// Workgroups are dealt to the 8 XCDs (each with its own L2 and address
// translation cache) round-robin by index. Tile = this remap of the index gives
// every XCD one contiguous run of tiles, so neighbouring column groups (the same
// rows, the same memory pages) are read through the same L2. A bijection when
// the grid is a multiple of 8, the identity otherwise.
__device__ inline uint64_t xcd_tile(uint64_t b, uint64_t nb) {
    constexpr uint64_t XCDS = 8;
    if (nb % XCDS) return b;
    return (b % XCDS) * (nb / XCDS) + b / XCDS;
}

struct KArgs {
    const JobDev *jobs;
    JobDev one;
    Tables tb;
    uint64_t S, Mprev;
    int which;  // array read and written (0: A, 1: B; -1: both, A for blockIdx.z = 0, B for 1)
};

// A strided pass: one workgroup per tile of C adjacent columns of R rows. The
// Stockham twiddles of the column transform are staged in LDS beside the tile.
// TQ (the last inverse pass only): the last step's outputs t < TQ of each group
// are the rows that hold needed coefficients (0: all); the arithmetic of the
// others is dropped at compile time.
template <class F, int LGR, int MODE, int TQ = 0>
__global__ void __launch_bounds__((Tile<F, LGR, true, 1, MODE>::NT))
__attribute__((amdgpu_waves_per_eu(Tile<F, LGR, true, 1, MODE>::WAVES_PER_SIMD))) k_strided(KArgs a) {
    using Tl = Tile<F, LGR, true, 1, MODE>;
    using T = typename F::T;
    constexpr int R = Tl::R, C = Tl::C, EPT = Tl::EPT, NT = Tl::NT;
    constexpr bool INV = (MODE == S_INV || MODE == S_INV_PARITY);
    constexpr bool FWD = !INV;
    constexpr bool BITS = MODE == S_FWD_BITS;
    constexpr int RF = Ends<Tl, INV>::RAD_FIRST, GF = EPT / RF;
    constexpr int RL = Ends<Tl, INV>::RAD_LAST, GL = EPT / RL;
    static_assert(Tl::LT, "strided tiles keep their twiddles in LDS");
    // The bit-reading pass with a radix-16 first step: that step's first two
    // butterfly layers are 4-point DFTs of four input bits (inputs t, t+4, t+8,
    // t+12), read from a 16 x 4 table built here by the same arithmetic.
    constexpr bool LUT = BITS && RF == 16;
    using Unit = UnitOf<C>;
    using TW = typename F::TW;
    __shared__ T lds[Tl::TILE_WORDS];
    __shared__ TW stw[Tl::STW_WORDS > 0 ? Tl::STW_WORDS : 1];
    __shared__ T lut[LUT ? 64 : 1];

    const JobDev &J = a.jobs ? a.jobs[blockIdx.y] : a.one;
    const int which = a.which < 0 ? (int)blockIdx.z : a.which;
    T *data = (T *)(which ? J.B : J.A);
    const T *thi = (const T *)a.tb.hi, *tlo = (const T *)a.tb.lo;
    const uint64_t colTiles = a.S / C;
    // (measured: the remap helps the value passes and slows the bit-reading first
    // forward pass)
    const uint64_t tile = (MODE == S_FWD || MODE == S_INV) ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint64_t blk = tile / colTiles, ct = tile - blk * colTiles;
    const uint64_t base = blk * a.Mprev + ct * C;
    const int shift = F::LGMAX - (63 - __builtin_clzll(a.Mprev));  // 2^LGMAX / Mprev = 2^shift
    const uint64_t emask = (uint64_t(1) << F::LGMAX) - 1;

    // the twiddle blocks of steps 1.., first read in step 1, after the barrier
    // that follows step 0
    for (int s = 1; s < Tl::NSTEPS; ++s) {
        const int rad = Tl::radix(s, INV), ns = Tl::span(s, INV);
        const TW *src = (const TW *)a.tb.stk + stk_offset(rad, ns, INV);
        for (int i = threadIdx.x; i < (rad - 1) * ns; i += NT) stw[Tl::stw_off(s, INV) + i] = gload(src + i);
    }

    if constexpr (LUT) {
        // entry (idx, k): output k of the first two layers when input 4 i is bit i
        // of idx and the other inputs are zero (every group of four takes the same
        // table)
        if (threadIdx.x < 64) {
            T u[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) u[i] = F::from_bit(0u);
#pragma unroll
            for (int i = 0; i < 4; ++i) u[bitrev<16>(4 * i)] = F::from_bit((threadIdx.x >> (2 + i)) & 1u);
            dft_layer_k<F, 16, 2, 0>(u);
            dft_layer_k<F, 16, 4, 0>(u);
            const int k = threadIdx.x & 3;
            lut[threadIdx.x] = k == 0 ? u[0] : k == 1 ? u[1] : k == 2 ? u[2] : u[3];
        }
    }

    T v[EPT];
    uint32_t bt[LUT ? EPT : 1];  // the input bits of the table path
#pragma unroll
    for (int q = 0; q < GF; ++q) {
        int c, j;
        Tl::template coords<RF>(q, c, j);
        // inverse: twiddle w^-(col r) for rows r = j + t R/RF, a geometric
        // sequence in t: two table twiddles per group, then products
        T wt = T(), st = T();
        if constexpr (INV) {
            const uint64_t col = ct * C + c;
            const uint64_t ew = (uint64_t(0) - ((col * (uint64_t)j) << shift)) & emask;
            const uint64_t es = (uint64_t(0) - ((col * (uint64_t)(R / RF)) << shift)) & emask;
            wt = F::tw_combine(gload(thi + (ew >> 16)), gload(tlo + (ew & 0xFFFF)));
            st = F::tw_combine(gload(thi + (es >> 16)), gload(tlo + (es & 0xFFFF)));
            // the last inverse pass also applies the pointwise constant K (L^-1
            // and Montgomery factors): one product per group at the start of
            // its twiddle sequence instead of one per value in the fused pass
            if constexpr (MODE == S_INV_PARITY) wt = F::tw_combine(wt, (T)J.K);
        }
        // element index of row r = j + t R/RF, column c: a running sum (one
        // 64-bit add per element instead of a 32x64-bit product)
        const uint64_t rstep = (uint64_t)(R / RF) * a.S;
        uint64_t gi = base + (uint64_t)j * a.S + c;
#pragma unroll
        for (int t = 0; t < RF; ++t, gi += rstep) {
            T x;
            if constexpr (BITS) {
                // a row segment of the tile is C adjacent bits starting at a
                // multiple of C: one C-bit unit, the same address for every lane
                // of the row. The embedding lays the units out tile-major (unit of
                // row r of column tile ct at ct R + r), so a tile's rows are
                // consecutive units and a wave's loads fall in one cache line.
                const Unit *ub = (const Unit *)J.eb[which] + ct * R;
                const uint32_t bit = (uint32_t)(gload(ub + j + t * (R / RF)) >> c) & 1u;
                if constexpr (LUT) bt[q * RF + t] = bit;
                x = F::from_bit(bit);
            } else {
                x = gload(data + gi);
            }
            if constexpr (INV) {
                x = F::mul_ip(x, wt);
                if (t + 1 < RF) wt = F::tw_combine(wt, st);
            }
            v[q * RF + t] = x;
        }
    }
    if constexpr (LUT) {
        // step 0 (radix 16, no twiddles): table lookups, then the last two layers
        __syncthreads();  // the table
#pragma unroll
        for (int q = 0; q < GF; ++q) {
            T u[16];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const uint32_t *b = &bt[q * 16 + bitrev<4>(g)];
                const uint32_t idx = b[0] | (b[4] << 1) | (b[8] << 2) | (b[12] << 3);
#pragma unroll
                for (int k = 0; k < 4; ++k) u[4 * g + k] = lut[4 * idx + k];
            }
            dft_layer_k<F, 16, 8, 0>(u);
            dft_layer_k<F, 16, 16, 0>(u);
#pragma unroll
            for (int k = 0; k < 16; ++k) v[q * 16 + k] = u[k];
        }
        static_assert(Tl::NSTEPS >= 2 && Tl::span(0, false) == 1, "step 0 is followed by an exchange");
        if constexpr (Tl::HALFX) {
            exchange_halves<F, Tl, 16, 1, Tl::radix(1, false)>(v, lds);
        } else {
            __syncthreads();
            step_store_lds<F, Tl, 16>(v, lds, 1);
            __syncthreads();
        }
        run_steps_from<F, Tl, false, 1, true>(v, lds, a.tb, stw);
    } else {
        run_steps_from<F, Tl, INV, 0, true>(v, lds, a.tb, stw);
    }
    // the last inverse pass of the 32-bit fields writes z itself unless the job
    // folds (z_i = c_i ^ c_(i+n), which needs the whole parity string first)
    constexpr bool DIRECT = MODE == S_INV_PARITY && C == 32;
    const bool direct = DIRECT && J.nfold == 0;
    const uint64_t zbits = DIRECT ? ((J.m + 63) >> 6) << 6 : 0;
    const bool degen = direct && degenerate(J);
    if (direct && blockIdx.x == 0 && threadIdx.x == 0 && J.status) *J.status = degen ? -3 : 0;
#pragma unroll
    for (int q = 0; q < GL; ++q) {
        int c, j;
        Tl::template coords<RL>(q, c, j);
        // forward: twiddle w^(col r), the same geometric sequence in t
        T wt = T(), st = T();
        if constexpr (FWD) {
            const uint64_t col = ct * C + c;
            const uint64_t ew = ((col * (uint64_t)j) << shift) & emask;
            const uint64_t es = ((col * (uint64_t)(R / RL)) << shift) & emask;
            wt = F::tw_combine(gload(thi + (ew >> 16)), gload(tlo + (ew & 0xFFFF)));
            st = F::tw_combine(gload(thi + (es >> 16)), gload(tlo + (es & 0xFFFF)));
        }
        const uint64_t rstep = (uint64_t)(R / RL) * a.S;
        uint64_t gi = base + (uint64_t)j * a.S + c;
#pragma unroll
        for (int t = 0; t < (TQ ? TQ : RL); ++t, gi += rstep) {
            const int r = j + t * (R / RL);
            T x = v[q * RL + t];
            if constexpr (FWD) {
                gstore(data + gi, F::mul_ip(x, wt));
                if (t + 1 < RL) wt = F::tw_combine(wt, st);
            } else if constexpr (MODE == S_INV) {
                gstore(data + gi, x);
            } else {
                // level 0 of the inverse: gi is the coefficient index; the C lanes
                // of a row hold C consecutive coefficients. With 32 columns and no
                // fold, that row unit's parities go straight into z (bits gi ..
                // gi + 31, a 32-bit-aligned word of z; bits past m cleared, zero
                // for a degenerate Dodis input). Otherwise they go out tile-major
                // (unit (ct, r) at ct*R + r, contiguous per workgroup) and a
                // transpose kernel turns that into packed natural order.
                uint32_t bit = (uint32_t)(F::canon(x) & 1u);
                uint64_t mask = __ballot(bit);
                const int lane = (int)(threadIdx.x & 63);
                if (c == 0) {
                    const Unit u = (Unit)(mask >> (lane & ~(C - 1)));
                    if (DIRECT && direct) {
                        if (gi < zbits) {
                            uint32_t w = (uint32_t)u;
                            if (degen || gi >= J.m) w = 0u;
                            else if (J.m - gi < 32) w &= (1u << (uint32_t)(J.m - gi)) - 1u;
                            gstore((uint32_t *)J.z + (gi >> 5), w);
                        }
                    } else {
                        gstore((Unit *)J.eb[0] + ct * R + r, u);
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ contiguous pass

// Waves per SIMD that the lazy field's row passes promise the register
// allocator (1: no promise). A workgroup of 2^13 rows puts two waves on each
// SIMD, so that above 80 registers two of them fit a CU where the LDS admits
// four; the counts below are the highest each pass reaches without spilling, and
// each was measured faster on the 4096-block batched workload (the fused passes
// of 2^13 rows 12-19% faster). The other fields' passes keep the allocator's own
// choice: the same promises made the two-piece product pass over 3*2^30+1
// slower.
template <class F, int LGR, int MODE>
constexpr int contig_waves_per_eu() {
    if (!std::is_same<F, FLZ>::value) return 1;
    if ((MODE == C_FUSED || MODE == C_FUSED2) && LGR >= 13) return 6;
    if (MODE == C_FUSED2 && (LGR == 11 || LGR == 12)) return 5;
    if (MODE == C_FWD && LGR == 12) return 8;
    return 1;
}

template <class F, int LGR, int MODE>
__global__ void __launch_bounds__((Tile<F, LGR, false>::NT))
__attribute__((amdgpu_waves_per_eu(contig_waves_per_eu<F, LGR, MODE>()))) k_contig(KArgs a) {
    using Tl = Tile<F, LGR, false, (MODE == C_FWD ? 1 : 2), MODE>;
    using T = typename F::T;
    constexpr int R = Tl::R, C = Tl::C, EPT = Tl::EPT;
    constexpr bool FUSED = (MODE == C_FUSED || MODE == C_FUSED2);
    using TW = typename F::TW;
    __shared__ T lds[C * Tl::RP];
    __shared__ TW stw[Tl::STW_WORDS > 0 ? Tl::STW_WORDS : 1];
    // the small Stockham twiddle blocks of the forward transform (and of the
    // inverse one in a fused pass), first read in step 1, after the barrier that
    // follows step 0
    if constexpr (Tl::LT) {
#pragma unroll
        for (int d = 0; d < (FUSED ? 2 : 1); ++d) {
            const bool inv = d == 1;
#pragma unroll
            for (int s = 1; s < Tl::NSTEPS; ++s) {
                if (!Tl::stw_local(s, inv)) continue;
                const int rad = Tl::radix(s, inv), ns = Tl::span(s, inv);
                const TW *src = (const TW *)a.tb.stk + stk_offset(rad, ns, inv);
                for (int i = threadIdx.x; i < (rad - 1) * ns; i += Tl::NT) stw[Tl::stw_off(s, inv) + i] = gload(src + i);
            }
        }
    }

    const JobDev &J = a.jobs ? a.jobs[blockIdx.y] : a.one;
    T *data = (T *)(a.which ? J.B : J.A);
    const T *spec = (const T *)J.S;
    const uint64_t base = (uint64_t)blockIdx.x * C * R;

    T v[EPT];
    {
        constexpr int RAD = Ends<Tl, false>::RAD_FIRST;
        constexpr int GPT = EPT / RAD;
#pragma unroll
        for (int q = 0; q < GPT; ++q) {
            int c, j;
            Tl::template coords<RAD>(q, c, j);
#pragma unroll
            for (int t = 0; t < RAD; ++t) v[q * RAD + t] = gload(data + base + (uint64_t)c * R + j + t * (R / RAD));
        }
    }
    constexpr int RADL = Ends<Tl, false>::RAD_LAST;
    constexpr int GPTL = EPT / RADL;
    // C_PROD, C_PROD_ADD: the spectrum operand's values are loaded before the
    // transform, so that their latency overlaps it (its registers are free under
    // the LDS limit)
    constexpr bool PROD = (MODE == C_PROD || MODE == C_PROD_ADD);
    T sv[PROD ? EPT : 1];
    if constexpr (PROD) {
#pragma unroll
        for (int q = 0; q < GPTL; ++q) {
            int c, j;
            Tl::template coords<RADL>(q, c, j);
#pragma unroll
            for (int t = 0; t < RADL; ++t) sv[q * RADL + t] = gload(spec + base + (uint64_t)c * R + j + t * (R / RADL));
        }
    }
    run_steps_from<F, Tl, false, 0, Tl::LT>(v, lds, a.tb, stw);
    if constexpr (MODE == C_FUSED || MODE == C_FUSED2) {
        static_assert(Ends<Tl, true>::RAD_FIRST == RADL, "register hand-over needs equal radices");
        // (the constant K is applied by the last inverse pass)
        const T *prod2 = (const T *)J.S2;
#pragma unroll
        for (int q = 0; q < GPTL; ++q) {
            int c, j;
            Tl::template coords<RADL>(q, c, j);
#pragma unroll
            for (int t = 0; t < RADL; ++t) {
                const uint64_t gi = base + (uint64_t)c * R + j + t * (R / RADL);
                T prod = F::mont(v[q * RADL + t], gload(spec + gi));
                if constexpr (MODE == C_FUSED2) prod = F::add(F::as_a(prod), F::as_b(gload(prod2 + gi)));
                v[q * RADL + t] = prod;
            }
        }
        __syncthreads();  // LDS is reused by the inverse steps
        run_steps_from<F, Tl, true, 0, Tl::LT>(v, lds, a.tb, stw);
        constexpr int RADI = Ends<Tl, true>::RAD_LAST;
#pragma unroll
        for (int q = 0; q < EPT / RADI; ++q) {
            int c, j;
            Tl::template coords<RADI>(q, c, j);
#pragma unroll
            for (int t = 0; t < RADI; ++t) gstore(data + base + (uint64_t)c * R + j + t * (R / RADI), v[q * RADI + t]);
        }
    } else {
#pragma unroll
        for (int q = 0; q < GPTL; ++q) {
            int c, j;
            Tl::template coords<RADL>(q, c, j);
#pragma unroll
            for (int t = 0; t < RADL; ++t) {
                const uint64_t gi = base + (uint64_t)c * R + j + t * (R / RADL);
                if constexpr (MODE == C_PROD)
                    gstore(data + gi, F::mont(v[q * RADL + t], sv[q * RADL + t]));
                else if constexpr (MODE == C_PROD_ADD)
                    gstore(data + gi, F::add(F::mont(v[q * RADL + t], sv[q * RADL + t]),
                                             F::as_b(gload((const T *)J.S2 + gi))));
                else
                    gstore(data + gi, v[q * RADL + t]);
            }
        }
    }
}

// ------------------------------------------------------------------ small: whole job in one thread group

// A job of length L = 2^LG is done by a group of NT = L/16 threads (16 values each)
// with L (+ padding) words of LDS. Groups are NT-aligned blocks of a workgroup,
// so a thread's index within its group is threadIdx.x & (NT - 1).
template <int LG>
struct SmallTile {
    static constexpr int R = 1 << LG;
    static constexpr int C = 1;
    static constexpr int NT = R / 16;  // a partial wave for L < 2^10
    static constexpr int EPT = R / NT;
    static constexpr int RF = (LG % 4) ? (1 << (LG % 4)) : 16;
    static constexpr int NSTEPS = (LG + 3) / 4;
    static constexpr int LDS_WORDS = R + R / 16;
    __device__ static inline int lid() { return (int)(threadIdx.x & (NT - 1)); }
    __device__ static inline int lidx(int c, int r) { return r + (r >> 4); }
    template <int RAD>
    __device__ static inline void coords(int q, int &c, int &j) {
        c = 0;
        j = lid() + q * NT;
    }
    // the leftover radix second in the forward transforms and last in the
    // inverse (the order of the fused contiguous pass, see Tile::radix)
    __host__ __device__ static constexpr int radix(int s, bool inv) {
        if (NSTEPS >= 3 && !inv) return s == 1 ? RF : 16;
        return inv ? (s == NSTEPS - 1 ? RF : 16) : (s == 0 ? RF : 16);
    }
    __host__ __device__ static constexpr int span(int s, bool inv) {
        int ns = 1;
        for (int i = 0; i < s; ++i) ns *= radix(i, inv);
        return ns;
    }
};

// The whole extraction of job J by one thread group: both forward transforms,
// the pointwise product, the inverse, parity, fold, pack, and the Dodis
// degenerate-input check. Every thread of the workgroup must call this (it
// contains workgroup barriers); `write` = false runs the arithmetic without
// writing any output (idle groups of a persistent workgroup). Field FLZ
// (7 * 2^26 + 1, lazy values).
template <int LG>
__device__ inline void small_body(const JobDev &J, bool write, uint32_t *lds, uint32_t *red, const Tables &tb) {
    using F = FLZ;
    using Tl = SmallTile<LG>;
    using T = uint32_t;
    constexpr int R = Tl::R, EPT = Tl::EPT, NT = Tl::NT;
    constexpr int RAD0 = Ends<Tl, false>::RAD_FIRST;
    const int lt = Tl::lid();

    static_assert(LG <= 16, "32-bit embedding positions");
    // both operands' bits are read first, so that the seed's loads are in flight
    // during the input's transform
    T va[EPT], vb[EPT];
    const uint32_t L32 = (uint32_t)J.L;
#pragma unroll
    for (int q = 0; q < EPT / RAD0; ++q) {
        int c, j;
        Tl::template coords<RAD0>(q, c, j);
#pragma unroll
        for (int t = 0; t < RAD0; ++t) {
            va[q * RAD0 + t] = emb_bit32_input(J.ex, (uint32_t)(j + t * (R / RAD0)));
            vb[q * RAD0 + t] = emb_bit32_seed(J.ey, (uint32_t)(j + t * (R / RAD0)), L32);
        }
    }
    run_steps_from<F, Tl, false, 0>(va, lds, tb);
    __syncthreads();
    run_steps_from<F, Tl, false, 0>(vb, lds, tb);
    const T K = (T)J.K;
#pragma unroll
    for (int i = 0; i < EPT; ++i) vb[i] = F::mont(F::mont(vb[i], va[i]), K);
    __syncthreads();
    run_steps_from<F, Tl, true, 0>(vb, lds, tb);
    constexpr int RADI = Ends<Tl, true>::RAD_LAST;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < EPT / RADI; ++q) {
        int c, j;
        Tl::template coords<RADI>(q, c, j);
#pragma unroll
        for (int t = 0; t < RADI; ++t) lds[Tl::lidx(0, j + t * (R / RADI))] = F::canon(vb[q * RADI + t]);
    }
    if (lt < 2) red[lt] = 0;
    __syncthreads();
    if (J.degen_n) {
        const uint64_t nw = (J.degen_n + 63) >> 6;
        uint32_t one_ = 0, zero_ = 0;
        for (uint64_t w = lt; w < nw; w += NT) {
            uint64_t x = J.ex.bits[w];
            uint64_t mk = (w + 1 < nw || (J.degen_n & 63) == 0) ? ~0ull : ((1ull << (J.degen_n & 63)) - 1);
            one_ |= (x & mk) != 0;
            zero_ |= (~x & mk) != 0;
        }
        if (one_) atomicOr(&red[0], 1u);
        if (zero_) atomicOr(&red[1], 1u);
    }
    __syncthreads();
    const bool degen = J.degen_n && (red[0] == 0 || red[1] == 0);
    if (write) {
        const uint64_t m = J.m, nfold = J.nfold;
        uint64_t *const z = J.z;
        const uint64_t nwm = (m + 63) >> 6;
        if constexpr (NT >= 64) {
            // a group of whole waves: word w is one ballot of coefficients 64 w ..
            const int lane = lt & 63;
            for (uint64_t w = (uint64_t)(lt >> 6); w < nwm; w += NT / 64) {
                const uint64_t i = w * 64 + lane;
                uint32_t bit = 0;
                if (!degen && i < m) {
                    bit = lds[Tl::lidx(0, (int)i)] & 1u;
                    if (nfold) bit ^= lds[Tl::lidx(0, (int)(i + nfold))] & 1u;
                }
                const uint64_t word = __ballot(bit);
                if (lane == 0) z[w] = word;
            }
        } else {
            for (uint64_t w = lt; w < nwm; w += NT) {
                uint64_t word = 0;
                if (!degen) {
                    for (int b = 0; b < 64; ++b) {
                        const uint64_t i = w * 64 + b;
                        if (i >= m) break;
                        uint32_t bit = lds[Tl::lidx(0, (int)i)] & 1u;
                        if (nfold) bit ^= lds[Tl::lidx(0, (int)(i + nfold))] & 1u;
                        word |= (uint64_t)bit << b;
                    }
                }
                z[w] = word;
            }
        }
        if (lt == 0 && J.status) *J.status = degen ? -3 : 0;
    }
}

// One job per workgroup.
template <int LG>
__global__ void __launch_bounds__(SmallTile<LG>::NT) k_small(const JobDev *jobs, JobDev one, Tables tb) {
    __shared__ uint32_t lds[SmallTile<LG>::LDS_WORDS];
    __shared__ uint32_t red[2];
    const JobDev &J = jobs ? jobs[blockIdx.x] : one;
    small_body<LG>(J, true, lds, red, tb);
}

// A single job with its two forward transforms side by side (single calls of
// 2^10 to 2^13, where the one workgroup is the whole launch): threads [0, NT)
// transform the input and [NT, 2 NT) the seed, each group in its own tile of
// LDS_WORDS. The input's group then leaves its spectrum in its tile (positions
// of the last forward step), the seed's group multiplies by it and runs the
// inverse in its own tile while the input's group only keeps the barriers, and
// both groups pack the parity from the seed group's tile. The same arithmetic as
// small_body, in the same order for each value.
template <int LG>
__global__ void __launch_bounds__(2 * SmallTile<LG>::NT) k_small_pair(JobDev J, Tables tb) {
    using F = FLZ;
    using Tl = SmallTile<LG>;
    using T = uint32_t;
    constexpr int R = Tl::R, EPT = Tl::EPT, NT = Tl::NT, W = Tl::LDS_WORDS;
    static_assert(NT >= 64 && 2 * NT <= 1024, "groups of whole waves in one workgroup");
    __shared__ uint32_t lds[2 * W];
    __shared__ uint32_t red[2];
    const int g = __builtin_amdgcn_readfirstlane((int)threadIdx.x / NT);  // uniform in a wave
    uint32_t *const tile = lds + g * W;
    constexpr int RAD0 = Ends<Tl, false>::RAD_FIRST;
    constexpr int RADL = Ends<Tl, false>::RAD_LAST;
    constexpr int RADI = Ends<Tl, true>::RAD_LAST;
    const uint32_t L32 = (uint32_t)J.L;

    T v[EPT];
#pragma unroll
    for (int q = 0; q < EPT / RAD0; ++q) {
        int c, j;
        Tl::template coords<RAD0>(q, c, j);
#pragma unroll
        for (int t = 0; t < RAD0; ++t) {
            const uint32_t i = (uint32_t)(j + t * (R / RAD0));
            v[q * RAD0 + t] = g == 0 ? emb_bit32_input(J.ex, i) : emb_bit32_seed(J.ey, i, L32);
        }
    }
    run_steps_from<F, Tl, false, 0>(v, tile, tb);
    __syncthreads();  // every read of the tiles by the last forward step is done
    if (g == 0) {
#pragma unroll
        for (int q = 0; q < EPT / RADL; ++q) {
            int c, j;
            Tl::template coords<RADL>(q, c, j);
#pragma unroll
            for (int t = 0; t < RADL; ++t) tile[Tl::lidx(0, j + t * (R / RADL))] = v[q * RADL + t];
        }
    }
    __syncthreads();
    if (g == 1) {
        const T K = (T)J.K;
#pragma unroll
        for (int q = 0; q < EPT / RADL; ++q) {
            int c, j;
            Tl::template coords<RADL>(q, c, j);
#pragma unroll
            for (int t = 0; t < RADL; ++t) {
                const T a = lds[Tl::lidx(0, j + t * (R / RADL))];  // the input's tile
                v[q * RADL + t] = F::mont(F::mont(v[q * RADL + t], a), K);
            }
        }
    }
    run_steps_from<F, Tl, true, 0>(v, tile, tb, nullptr, g == 1);
    __syncthreads();
    if (g == 1) {
#pragma unroll
        for (int q = 0; q < EPT / RADI; ++q) {
            int c, j;
            Tl::template coords<RADI>(q, c, j);
#pragma unroll
            for (int t = 0; t < RADI; ++t) tile[Tl::lidx(0, j + t * (R / RADI))] = F::canon(v[q * RADI + t]);
        }
    }
    if (threadIdx.x < 2) red[threadIdx.x] = 0;
    __syncthreads();
    if (J.degen_n) {
        const uint64_t nw = (J.degen_n + 63) >> 6;
        uint32_t one_ = 0, zero_ = 0;
        for (uint64_t w = threadIdx.x; w < nw; w += 2 * NT) {
            uint64_t x = J.ex.bits[w];
            uint64_t mk = (w + 1 < nw || (J.degen_n & 63) == 0) ? ~0ull : ((1ull << (J.degen_n & 63)) - 1);
            one_ |= (x & mk) != 0;
            zero_ |= (~x & mk) != 0;
        }
        if (one_) atomicOr(&red[0], 1u);
        if (zero_) atomicOr(&red[1], 1u);
    }
    __syncthreads();
    const bool degen = J.degen_n && (red[0] == 0 || red[1] == 0);
    const uint32_t *const out = lds + W;  // the seed group's tile
    const uint64_t m = J.m, nfold = J.nfold;
    const uint64_t nwm = (m + 63) >> 6;
    const int lane = (int)threadIdx.x & 63;
    for (uint64_t w = threadIdx.x >> 6; w < nwm; w += 2 * NT / 64) {
        const uint64_t i = w * 64 + lane;
        uint32_t bit = 0;
        if (!degen && i < m) {
            bit = out[Tl::lidx(0, (int)i)] & 1u;
            if (nfold) bit ^= out[Tl::lidx(0, (int)(i + nfold))] & 1u;
        }
        const uint64_t word = __ballot(bit);
        if (lane == 0) J.z[w] = word;
    }
    if (threadIdx.x == 0 && J.status) *J.status = degen ? -3 : 0;
}

#if NTT_HAS(4)
// ------------------------------------------------------------------ embedding of the packed inputs

// cnt (<= 64) bits of b starting at bit `start`, as the low bits of a word
__host__ __device__ inline uint64_t bits_at(const uint64_t *b, uint64_t start, int cnt) {
    const uint64_t q = start >> 6;
    const int o = (int)(start & 63);
    uint64_t w = b[q] >> o;
    if (o && o + cnt > 64) w |= b[q + 1] << (64 - o);
    return cnt == 64 ? w : (w & ((uint64_t(1) << cnt) - 1));
}

// Word w of the L-bit coefficient string of embedding e: bit t is emb_bit(e, 64w + t),
// assembled from runs of consecutive source bits.
__host__ __device__ inline uint64_t embed_word(const Emb &e, uint64_t L, uint64_t w) {
    const uint64_t i0 = w * 64;
    uint64_t out = 0;
    if (e.mode == EMB_PREFIX) {
        if (i0 >= e.len) return 0;
        const int cnt = (int)umin64(64, e.len - i0);
        return bits_at(e.bits, i0, cnt);
    }
    if (e.mode == EMB_SEED) {
        int pos = 0;
        while (pos < 64) {
            uint64_t k = i0 + pos + e.a;
            if (k >= L) k -= L;
            if (k >= e.N) {  // zeros until k wraps at L
                pos += (int)umin64(64 - pos, L - k);
                continue;
            }
            const uint64_t src = mod_small(k + e.rot, e.P);
            const int run = (int)umin64(64 - pos, umin64(e.N - k, e.P - src));
            out |= bits_at(e.bits, src, run) << pos;
            pos += run;
        }
        return out;
    }
    // REV: position i < a holds b'_{N-1-i}, b'_j = j < len ? b_j : 0
    for (int t = 0; t < 64;) {
        const uint64_t i = i0 + t;
        if (i >= e.a) break;
        const uint64_t j = e.N - 1 - i;  // positions i.. read j, j-1, ..
        if (j >= e.len) {                // sources beyond len are zero: skip to j = len - 1
            t += (int)umin64(j - e.len + 1, (uint64_t)(64 - t));
            continue;
        }
        const int run = (int)umin64(umin64(64 - t, j + 1), e.a - i);
        const uint64_t rev = __builtin_bitreverse64(bits_at(e.bits, j - run + 1, run)) >> (64 - run);
        out |= rev << t;
        t += run;
    }
    return out;
}

// Dodis degenerate-input check (section "Dodis et al.": x must not be all zeros
// or all ones), split over the first `parts` (<= DEGEN_PARTS_MAX) workgroups of
// the embedding's check slice. Part g scans words [g c, (g+1) c) of the first
// degen_n bits of x (c = ceil(words / parts)) and writes flags[2 + 2g] = the
// part has a one bit, flags[3 + 2g] = it has a zero bit; part 0 also writes
// flags[0] = parts. Every part's slots are written on every launch, so the flags
// need no clearing. degenerate() reduces them (the job's 256-byte flag region
// holds 64 words).
__device__ inline void degen_part(const JobDev &J, uint32_t g, uint32_t parts) {
    __shared__ uint32_t red[2];
    if (threadIdx.x < 2) red[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t nw = (J.degen_n + 63) >> 6, chunk = (nw + parts - 1) / parts;
    const uint64_t w0 = (uint64_t)g * chunk, w1 = umin64(nw, w0 + chunk);
    const uint64_t tail = (J.degen_n & 63) ? ((1ull << (J.degen_n & 63)) - 1) : ~0ull;
    uint32_t one_ = 0, zero_ = 0;
#pragma unroll 4
    for (uint64_t w = w0 + threadIdx.x; w < w1; w += 256) {
        const uint64_t x = gload(J.ex.bits + w);
        const uint64_t mk = w + 1 < nw ? ~0ull : tail;
        one_ |= (x & mk) != 0;
        zero_ |= (~x & mk) != 0;
    }
    if (one_) atomicOr(&red[0], 1u);
    if (zero_) atomicOr(&red[1], 1u);
    __syncthreads();
    if (threadIdx.x < 2) J.flags[2 + 2 * g + threadIdx.x] = red[threadIdx.x];
    if (g == 0 && threadIdx.x == 0) J.flags[0] = parts;
}

// The embedded L-bit coefficient strings, in the unit layout the first strided
// level reads: the transform viewed as R = 2^lgr0 rows of S = L / R coefficients,
// the C-bit unit of row r and column tile ct (coefficients r S + ct C ..) at unit
// index ct R + r. A workgroup takes 64 rows by up to 16 words of each row: it
// assembles the words (coalesced along the rows' words) in LDS, then writes each
// column tile's 64 row units as one contiguous run.
// blockIdx.z = 0, 1: the embedding of x, y; z = 2 (launched for shapes with the
// degenerate check): the check, by the slice's first DEGEN_PARTS_MAX workgroups.
template <int C>
__global__ void __launch_bounds__(256) k_embed(const JobDev *jobs, JobDev one, uint32_t lgr0, uint32_t row_groups) {
    using Unit = UnitOf<C>;
    constexpr int UPW = 64 / C;  // units per word
    const JobDev &J = jobs ? jobs[blockIdx.y] : one;
    if (blockIdx.z == 2) {
        const uint32_t parts = umin64(gridDim.x, DEGEN_PARTS_MAX);
        if (blockIdx.x < parts && J.degen_n) degen_part(J, blockIdx.x, parts);
        return;
    }
    __shared__ uint64_t tl[64][17];
    // (the descriptor is read once: the stores could alias it)
    const uint64_t L = J.L, R = uint64_t(1) << lgr0, wpr = (L >> lgr0) >> 6;  // words per row
    const int which = blockIdx.z;
    const Emb e = which ? J.ey : J.ex;
    Unit *const dst = (Unit *)J.eb[which];
    const uint64_t rg = blockIdx.x % row_groups, kg = blockIdx.x / row_groups;
    const uint64_t r0 = rg * 64, k0 = kg * 16;
    const int nk = (int)umin64(16, wpr - k0);
    for (int i = threadIdx.x; i < 64 * 16; i += 256) {
        const int rr = i >> 4, kk = i & 15;
        if (kk < nk) tl[rr][kk] = embed_word(e, L, (r0 + rr) * wpr + k0 + kk);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * nk * UPW; i += 256) {
        const int rr = i & 63, uu = i >> 6;  // 64 consecutive rows of one column tile
        const Unit u = (Unit)(tl[rr][uu / UPW] >> ((uu % UPW) * C));
        gstore(dst + (k0 * UPW + uu) * R + r0 + rr, u);
    }
}

// ------------------------------------------------------------------ persistent batch of small jobs

// Work items are taken from *counter until all are done. Item k of class c covers
// jobs first_job + (k - first_item) * JPW .. + JPW - 1, JPW = 2^(14 - LG): a
// 1024-thread workgroup runs JPW jobs of length 2^LG side by side, one per
// 2^(LG-4)-thread group, with 2^14 words of LDS in total. Every workgroup exits
// once the counter passes the last item.
__device__ inline void small_item(int lg, const JobDev *jobs, uint64_t first, uint64_t count, uint32_t *lds,
                                  uint32_t *red, const Tables &tb) {
    switch (lg) {
#define CASE(LG)                                                                                        \
    case LG: {                                                                                          \
        constexpr int NT = SmallTile<LG>::NT;                                                           \
        const uint64_t g = threadIdx.x / NT;                                                            \
        const bool valid = g < count;                                                                   \
        small_body<LG>(jobs[first + (valid ? g : 0)], valid, lds + g * SmallTile<LG>::LDS_WORDS, red + 2 * g, tb); \
        break;                                                                                          \
    }
        CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11) CASE(12) CASE(13) CASE(14)
#undef CASE
    }
}

__global__ void __launch_bounds__(1024) k_small_persist(const JobDev *jobs, SmallClasses cls, uint32_t *counter,
                                                        Tables tb) {
    __shared__ uint32_t lds[(1 << 14) + (1 << 10)];
    __shared__ uint32_t red[2 * 256];
    __shared__ uint32_t item_s;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t item = item_s;
        __syncthreads();
        if (item >= cls.total_items) break;
        int c = 0;
        while (c + 1 < cls.n && item >= cls.first_item[c + 1]) ++c;
        const int lg = cls.lg[c];
        const uint64_t jpw = uint64_t(1) << (14 - lg);
        const uint64_t first = cls.first_job[c] + (uint64_t)(item - cls.first_item[c]) * jpw;
        const uint64_t end = cls.first_job[c] + cls.njobs[c];
        small_item(lg, jobs, first, end - first < jpw ? end - first : jpw, lds, red, tb);
        __syncthreads();  // LDS reuse by the next item
    }
}

__global__ void k_zero_u32(uint32_t *p) { *p = 0u; }

// The allocation-free entry point's workspace: one copy on every GPU the library
// runs on, for the life of the process. Host code uses the address that
// noalloc_scratch_address returns, never this name (on the host it is only a
// stand-in for the symbol).
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch_address(void **ptr) {
    *ptr = nullptr;
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

// ------------------------------------------------------------------ pack, degenerate check

__global__ void __launch_bounds__(256) k_pack(const JobDev *jobs, JobDev one) {
    const JobDev &J = jobs ? jobs[blockIdx.y] : one;
    const uint64_t nwm = (J.m + 63) >> 6;
    const uint64_t w = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    const bool degen = degenerate(J);
    if (w < nwm) {
        uint64_t word = J.pb[w];
        if (J.nfold) {
            const uint64_t off = J.nfold + w * 64;
            const uint64_t q = off >> 6, b = off & 63;
            word ^= b ? ((J.pb[q] >> b) | (J.pb[q + 1] << (64 - b))) : J.pb[q];
        }
        const uint64_t rem = J.m - w * 64;
        if (rem < 64) word &= (1ull << rem) - 1;
        J.z[w] = degen ? 0ull : word;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && J.status) *J.status = degen ? -3 : 0;
}

// Tile-major parity units (unit u of row r at u*R + r, C bits each, in J.eb[0]) to
// packed natural order in J.pb (bit r*S + u*C + c). 64 x 64 units per workgroup
// through LDS, coalesced on both sides.
// PACK: write z itself (the job's first ceil(m/64) words, bits past m cleared,
// zero for a degenerate Dodis input, and the status word) instead of pb, for
// shapes without the wrap-around fold; k_pack is then not needed.
template <int C, bool PACK>
__global__ void __launch_bounds__(256) k_ptrans(const JobDev *jobs, JobDev one, uint64_t R, uint64_t S) {
    using Unit = UnitOf<C>;
    constexpr int UPW = 64 / C;  // units per word
    __shared__ Unit tl[64][65];
    const JobDev &J = jobs ? jobs[blockIdx.z] : one;
    const Unit *U = (const Unit *)J.eb[0];
    const uint64_t units = S / C;
    const uint64_t r0 = (uint64_t)blockIdx.x * 64, u0 = (uint64_t)blockIdx.y * 64;
    for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
        const int uu = idx >> 6, rr = idx & 63;
        const uint64_t u = u0 + uu, r = r0 + rr;
        tl[rr][uu] = (u < units && r < R) ? U[u * R + r] : (Unit)0;
    }
    __syncthreads();
    constexpr int WPR = 64 / UPW;  // words per tile row
    const uint64_t nwm = (J.m + 63) >> 6;
    const bool degen = PACK && degenerate(J);
    for (int idx = threadIdx.x; idx < 64 * WPR; idx += 256) {
        const int rr = idx / WPR, wk = idx % WPR;
        const uint64_t r = r0 + rr, u = u0 + (uint64_t)wk * UPW;
        if (r < R && u < units) {
            uint64_t word = 0;
#pragma unroll
            for (int k = 0; k < UPW; ++k) word |= (uint64_t)tl[rr][wk * UPW + k] << (k * C);
            const uint64_t wi = r * (S / 64) + u / UPW;
            if constexpr (PACK) {
                if (wi < nwm) {
                    const uint64_t rem = J.m - wi * 64;
                    if (rem < 64) word &= (1ull << rem) - 1;
                    J.z[wi] = degen ? 0ull : word;
                }
            } else {
                J.pb[wi] = word;
            }
        }
    }
    if (PACK && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && J.status) *J.status = degen ? -3 : 0;
}


#endif

// ------------------------------------------------------------------ launchers

static KArgs make_args(const PassLaunch &p, const Tables &t) {
    KArgs ka;
    ka.jobs = p.jobs;
    if (p.one) ka.one = *p.one;
    else std::memset(&ka.one, 0, sizeof(ka.one));
    ka.tb = t;
    ka.S = p.S;
    ka.Mprev = p.Mprev;
    ka.which = p.which;
    return ka;
}

template <class F, int LGR>
static hipError_t strided_one(const PassLaunch &p, const KArgs &ka0, hipStream_t s) {
    const KArgs &ka = ka0;
#define L1(M, Q)                                                                                        \
    e = launch_k(k_strided<F, LGR, M, Q>, dim3((unsigned)p.tiles, p.njobs, p.which < 0 ? 2u : 1u), \
                 dim3(Tile<F, LGR, true, 1, M>::NT), 0, s, ka)
    // last inverse pass: rows j + t R/RL of group j come out of its last step's
    // output t, so the first out_rows rows need t < ceil(out_rows RL / R)
    constexpr int RL = Ends<Tile<F, LGR, true, 1, S_INV_PARITY>, true>::RAD_LAST;
    const uint64_t R = uint64_t(1) << LGR;
    const uint64_t tq = p.out_rows ? (p.out_rows * RL + R - 1) / R : (uint64_t)RL;
    hipError_t e = hipSuccess;
    switch (p.mode) {
        case S_FWD_BITS: L1(S_FWD_BITS, 0); break;
        case S_FWD: L1(S_FWD, 0); break;
        case S_INV: L1(S_INV, 0); break;
        default:
            if (tq <= RL / 4)
                L1(S_INV_PARITY, RL / 4);
            else if (tq <= RL / 2)
                L1(S_INV_PARITY, RL / 2);
            else
                L1(S_INV_PARITY, 0);
            break;
    }
#undef L1
    return e;
}

template <class F, int LGR>
static hipError_t contig_one(const PassLaunch &p, const KArgs &ka, hipStream_t s) {
    using Tl = Tile<F, LGR, false>;
    dim3 grid((unsigned)p.tiles, p.njobs), block(Tl::NT);
    if (p.mode == C_FUSED2 || p.mode == C_PROD || p.mode == C_PROD_ADD) {
        // piece schedules: two pieces over 3*2^30+1 or 7*2^26+1, any number over
        // the 64-bit field
        if constexpr (std::is_same<F, FP0>::value || std::is_same<F, FGL>::value || std::is_same<F, FLZ>::value) {
            if (p.mode == C_FUSED2)
                return launch_k(k_contig<F, LGR, C_FUSED2>, grid, block, 0, s, ka);
            else if (p.mode == C_PROD)
                return launch_k(k_contig<F, LGR, C_PROD>, grid, block, 0, s, ka);
            else if constexpr (std::is_same<F, FGL>::value)
                return launch_k(k_contig<F, LGR, C_PROD_ADD>, grid, block, 0, s, ka);
            else
                return hipErrorInvalidValue;
        } else {
            return hipErrorInvalidValue;
        }
    } else if (p.mode == C_FUSED) {
        return launch_k(k_contig<F, LGR, C_FUSED>, grid, block, 0, s, ka);
    }
    return launch_k(k_contig<F, LGR, C_FWD>, grid, block, 0, s, ka);
}

constexpr int BB_STRIDED_MAX = 10, BB_CONTIG_MAX = 14, GL_STRIDED_MAX = 10, GL_CONTIG_MAX = 13;
constexpr int SMALL_MAX = 14;

hipError_t launch_strided_bb(const PassLaunch &p, const Tables &t, hipStream_t s);
hipError_t launch_strided_gl(const PassLaunch &p, const Tables &t, hipStream_t s);
hipError_t launch_strided_p0(const PassLaunch &p, const Tables &t, hipStream_t s);
hipError_t launch_contig_bb(const PassLaunch &p, const Tables &t, hipStream_t s);
hipError_t launch_contig_gl(const PassLaunch &p, const Tables &t, hipStream_t s);
hipError_t launch_contig_gl_hi(const PassLaunch &p, const Tables &t, hipStream_t s);  // rows of 2^11..2^13
hipError_t launch_strided_lz(const PassLaunch &p, const Tables &t, hipStream_t s);
hipError_t launch_contig_lz(const PassLaunch &p, const Tables &t, hipStream_t s);
hipError_t launch_contig_p0(const PassLaunch &p, const Tables &t, hipStream_t s);

#if NTT_HAS(0)
hipError_t launch_strided_bb(const PassLaunch &p, const Tables &t, hipStream_t s) {
    KArgs ka = make_args(p, t);
    switch (p.lgr) {
        case 7: return strided_one<FBB, 7>(p, ka, s);
        case 8: return strided_one<FBB, 8>(p, ka, s);
        case 9: return strided_one<FBB, 9>(p, ka, s);
        case 10: return strided_one<FBB, 10>(p, ka, s);
    }
    return hipErrorInvalidValue;
}
#endif

#if NTT_HAS(1)
hipError_t launch_strided_gl(const PassLaunch &p, const Tables &t, hipStream_t s) {
    KArgs ka = make_args(p, t);
    switch (p.lgr) {
        case 7: return strided_one<FGL, 7>(p, ka, s);
        case 8: return strided_one<FGL, 8>(p, ka, s);
        case 9: return strided_one<FGL, 9>(p, ka, s);
        case 10: return strided_one<FGL, 10>(p, ka, s);
    }
    return hipErrorInvalidValue;
}
#endif

#if NTT_HAS(2)
hipError_t launch_contig_bb(const PassLaunch &p, const Tables &t, hipStream_t s) {
    KArgs ka = make_args(p, t);
    switch (p.lgr) {
        case 7: return contig_one<FBB, 7>(p, ka, s);
        case 8: return contig_one<FBB, 8>(p, ka, s);
        case 9: return contig_one<FBB, 9>(p, ka, s);
        case 10: return contig_one<FBB, 10>(p, ka, s);
        case 11: return contig_one<FBB, 11>(p, ka, s);
        case 12: return contig_one<FBB, 12>(p, ka, s);
        case 13: return contig_one<FBB, 13>(p, ka, s);
        case 14: return contig_one<FBB, 14>(p, ka, s);
    }
    return hipErrorInvalidValue;
}
#endif

#if NTT_HAS(3)
hipError_t launch_contig_gl(const PassLaunch &p, const Tables &t, hipStream_t s) {
    if (p.lgr >= 11) return launch_contig_gl_hi(p, t, s);
    KArgs ka = make_args(p, t);
    switch (p.lgr) {
        case 7: return contig_one<FGL, 7>(p, ka, s);
        case 8: return contig_one<FGL, 8>(p, ka, s);
        case 9: return contig_one<FGL, 9>(p, ka, s);
        case 10: return contig_one<FGL, 10>(p, ka, s);
    }
    return hipErrorInvalidValue;
}
#endif

#if NTT_HAS(7)
hipError_t launch_contig_gl_hi(const PassLaunch &p, const Tables &t, hipStream_t s) {
    KArgs ka = make_args(p, t);
    switch (p.lgr) {
        case 11: return contig_one<FGL, 11>(p, ka, s);
        case 12: return contig_one<FGL, 12>(p, ka, s);
        case 13: return contig_one<FGL, 13>(p, ka, s);
    }
    return hipErrorInvalidValue;
}
#endif

#if NTT_HAS(8)
hipError_t launch_strided_lz(const PassLaunch &p, const Tables &t, hipStream_t s) {
    KArgs ka = make_args(p, t);
    switch (p.lgr) {
        case 7: return strided_one<FLZ, 7>(p, ka, s);
        case 8: return strided_one<FLZ, 8>(p, ka, s);
        case 9: return strided_one<FLZ, 9>(p, ka, s);
        case 10: return strided_one<FLZ, 10>(p, ka, s);
    }
    return hipErrorInvalidValue;
}
#endif

#if NTT_HAS(9)
hipError_t launch_contig_lz(const PassLaunch &p, const Tables &t, hipStream_t s) {
    KArgs ka = make_args(p, t);
    switch (p.lgr) {
        case 7: return contig_one<FLZ, 7>(p, ka, s);
        case 8: return contig_one<FLZ, 8>(p, ka, s);
        case 9: return contig_one<FLZ, 9>(p, ka, s);
        case 10: return contig_one<FLZ, 10>(p, ka, s);
        case 11: return contig_one<FLZ, 11>(p, ka, s);
        case 12: return contig_one<FLZ, 12>(p, ka, s);
        case 13: return contig_one<FLZ, 13>(p, ka, s);
        case 14: return contig_one<FLZ, 14>(p, ka, s);
    }
    return hipErrorInvalidValue;
}
#endif

#if NTT_HAS(5)
hipError_t launch_strided_p0(const PassLaunch &p, const Tables &t, hipStream_t s) {
    KArgs ka = make_args(p, t);
    switch (p.lgr) {
        case 7: return strided_one<FP0, 7>(p, ka, s);
        case 8: return strided_one<FP0, 8>(p, ka, s);
        case 9: return strided_one<FP0, 9>(p, ka, s);
        case 10: return strided_one<FP0, 10>(p, ka, s);
    }
    return hipErrorInvalidValue;
}
#endif

#if NTT_HAS(6)
hipError_t launch_contig_p0(const PassLaunch &p, const Tables &t, hipStream_t s) {
    KArgs ka = make_args(p, t);
    switch (p.lgr) {
        case 7: return contig_one<FP0, 7>(p, ka, s);
        case 8: return contig_one<FP0, 8>(p, ka, s);
        case 9: return contig_one<FP0, 9>(p, ka, s);
        case 10: return contig_one<FP0, 10>(p, ka, s);
        case 11: return contig_one<FP0, 11>(p, ka, s);
        case 12: return contig_one<FP0, 12>(p, ka, s);
        case 13: return contig_one<FP0, 13>(p, ka, s);
        case 14: return contig_one<FP0, 14>(p, ka, s);
    }
    return hipErrorInvalidValue;
}
#endif

#if NTT_HAS(4)
thread_local GraphRecorder *t_graph_recorder = nullptr;
void set_graph_recorder(GraphRecorder *rec) { t_graph_recorder = rec; }

// the 32-bit fields share tile sizes
int max_strided_lg(int field) { return field == FIELD_GL ? GL_STRIDED_MAX : BB_STRIDED_MAX; }
int max_contig_lg(int field) { return field == FIELD_GL ? GL_CONTIG_MAX : BB_CONTIG_MAX; }
int max_small_lg() { return SMALL_MAX; }

template <class F, int M>
static Geometry geo_s_mode(int lgr) {
    switch (lgr) {
#define G(L) case L: return Geometry{Tile<F, L, true, 1, M>::C, Tile<F, L, true, 1, M>::NT};
        G(7) G(8) G(9) G(10)
#undef G
    }
    return Geometry{0, 0};
}
template <class F>
static Geometry geo_s(int lgr, int mode) {
    switch (mode) {
        case S_FWD_BITS: return geo_s_mode<F, S_FWD_BITS>(lgr);
        case S_FWD: return geo_s_mode<F, S_FWD>(lgr);
        case S_INV: return geo_s_mode<F, S_INV>(lgr);
        case S_INV_PARITY: return geo_s_mode<F, S_INV_PARITY>(lgr);
    }
    return Geometry{0, 0};
}
template <class F>
static Geometry geo_c(int lgr) {
    switch (lgr) {
#define G(L) case L: return Geometry{Tile<F, L, false>::C, Tile<F, L, false>::NT};
        G(7) G(8) G(9) G(10) G(11) G(12) G(13) G(14)
#undef G
    }
    return Geometry{0, 0};
}
Geometry strided_geometry(int field, int lgr, int mode) {
    return field == FIELD_GL   ? geo_s<FGL>(lgr, mode)
           : field == FIELD_P0 ? geo_s<FP0>(lgr, mode)
           : field == FIELD_LZ ? geo_s<FLZ>(lgr, mode)
                               : geo_s<FBB>(lgr, mode);
}
Geometry contig_geometry(int field, int lgr) {
    return field == FIELD_GL   ? geo_c<FGL>(lgr)
           : field == FIELD_P0 ? geo_c<FP0>(lgr)
           : field == FIELD_LZ ? geo_c<FLZ>(lgr)
                               : geo_c<FBB>(lgr);
}

hipError_t launch_strided(const PassLaunch &p, const Tables &t, hipStream_t s) {
    switch (p.field) {
        case FIELD_BB: return launch_strided_bb(p, t, s);
        case FIELD_GL: return launch_strided_gl(p, t, s);
        case FIELD_P0: return launch_strided_p0(p, t, s);
        case FIELD_LZ: return launch_strided_lz(p, t, s);
    }
    return hipErrorInvalidValue;
}
hipError_t launch_contig(const PassLaunch &p, const Tables &t, hipStream_t s) {
    switch (p.field) {
        case FIELD_BB: return launch_contig_bb(p, t, s);
        case FIELD_GL: return launch_contig_gl(p, t, s);
        case FIELD_P0: return launch_contig_p0(p, t, s);
        case FIELD_LZ: return launch_contig_lz(p, t, s);
    }
    return hipErrorInvalidValue;
}

template <int LG>
static hipError_t small_one(uint32_t njobs, const JobDev *jobs, const JobDev *one, const Tables &t, hipStream_t s) {
    JobDev o;
    if (one) o = *one;
    else std::memset(&o, 0, sizeof(o));
    if constexpr (LG >= 10 && LG <= 13) {
        if (!jobs && one && njobs == 1) return launch_k(k_small_pair<LG>, dim3(1), dim3(2 * SmallTile<LG>::NT), 0, s, o, t);
    }
    return launch_k(k_small<LG>, dim3(njobs), dim3(SmallTile<LG>::NT), 0, s, jobs, o, t);
}

hipError_t launch_small(int lg, uint32_t njobs, const JobDev *jobs, const JobDev *one, const Tables &t,
                        hipStream_t s) {
    switch (lg) {
        case 6: return small_one<6>(njobs, jobs, one, t, s);
        case 7: return small_one<7>(njobs, jobs, one, t, s);
        case 8: return small_one<8>(njobs, jobs, one, t, s);
        case 9: return small_one<9>(njobs, jobs, one, t, s);
        case 10: return small_one<10>(njobs, jobs, one, t, s);
        case 11: return small_one<11>(njobs, jobs, one, t, s);
        case 12: return small_one<12>(njobs, jobs, one, t, s);
        case 13: return small_one<13>(njobs, jobs, one, t, s);
        case 14: return small_one<14>(njobs, jobs, one, t, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_small_batch(const SmallClasses &cls, const JobDev *jobs, uint32_t *counter, unsigned workgroups,
                              const Tables &t, hipStream_t s) {
    hipError_t e = launch_k(k_zero_u32, dim3(1), dim3(1), 0, s, counter);
    if (e != hipSuccess) return e;
    return launch_k(k_small_persist, dim3(workgroups), dim3(1024), 0, s, jobs, cls, counter, t);
}

hipError_t launch_pack(uint32_t njobs, uint64_t max_words, const JobDev *jobs, const JobDev *one, hipStream_t s) {
    JobDev o;
    if (one) o = *one;
    else std::memset(&o, 0, sizeof(o));
    unsigned gx = (unsigned)((max_words + 255) / 256);
    if (gx == 0) gx = 1;
    return launch_k(k_pack, dim3(gx, njobs), dim3(256), 0, s, jobs, o);
}

hipError_t launch_embed(uint32_t njobs, uint64_t L, int lgr0, int C, const JobDev *jobs, const JobDev *one,
                        bool degen, hipStream_t s) {
    JobDev o;
    if (one) o = *one;
    else std::memset(&o, 0, sizeof(o));
    const uint64_t R = uint64_t(1) << lgr0, wpr = (L >> lgr0) >> 6;
    if (R % 64 || wpr == 0) return hipErrorInvalidValue;
    const uint64_t row_groups = R / 64, word_groups = (wpr + 15) / 16;
    const dim3 grid((unsigned)(row_groups * word_groups), njobs, degen ? 3 : 2);
    if (C == 16) return launch_k(k_embed<16>, grid, dim3(256), 0, s, jobs, o, (uint32_t)lgr0, (uint32_t)row_groups);
    if (C == 32) return launch_k(k_embed<32>, grid, dim3(256), 0, s, jobs, o, (uint32_t)lgr0, (uint32_t)row_groups);
    return hipErrorInvalidValue;
}

hipError_t launch_ptrans(int field, uint64_t R, uint64_t S, uint64_t rows, uint32_t njobs, const JobDev *jobs,
                         const JobDev *one, bool pack, hipStream_t s) {
    JobDev o;
    if (one) o = *one;
    else std::memset(&o, 0, sizeof(o));
    const int C = strided_cols(field == FIELD_GL ? 64 : 32, S_INV_PARITY);  // columns of the parity pass
    rows = (rows == 0 || rows > R) ? R : rows;
    dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((S / C + 63) / 64), njobs);
    if (C == 16) {
        if (pack) return launch_k(k_ptrans<16, true>, grid, dim3(256), 0, s, jobs, o, R, S);
        return launch_k(k_ptrans<16, false>, grid, dim3(256), 0, s, jobs, o, R, S);
    }
    if (pack) return launch_k(k_ptrans<32, true>, grid, dim3(256), 0, s, jobs, o, R, S);
    return launch_k(k_ptrans<32, false>, grid, dim3(256), 0, s, jobs, o, R, S);
}

#endif

}  // namespace ext
