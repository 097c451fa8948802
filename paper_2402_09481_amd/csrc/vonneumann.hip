// Von Neumann extractor on gfx950 (section "Von Neumann": output bit j is
// x_{2j} when x_{2j} != x_{2j+1} and nothing otherwise; Alg. 3 walks the pairs
// in order and appends).
//
// The output is a stream compaction of the input's pairs, done in one pass
// over the input:
//
//   k_vn_zero  clears the tile states and the tile ticket counter.
//   k_vn_main  one workgroup per tile of VN_TILE_W input words, in the order
//              of a ticket counter. The tile is loaded coalesced and its
//              aggregate (its count of differing pairs) published at once; its
//              output offset comes from a decoupled look-back over the states
//              of the tiles before it (aggregate, then inclusive prefix, one
//              64-bit word each), whose first poll goes out with the aggregate
//              and is answered while the tile is compressed. The tile is staged
//              in LDS, each thread takes VN_WPT consecutive words and compresses
//              each (per byte a 256-entry table: the bits kept from its four
//              pairs), and the per-thread counts are scanned to assemble the
//              tile's bits in LDS at tile-local positions. They are written out
//              shifted onto the output's 64-bit word grid: words wholly inside
//              the tile's range straight to z, the first and last partial words
//              to side arrays.
//   k_vn_fix   one thread per tile: the partial words. The tile holding a word's
//              first output bit ORs in the parts of the tiles that follow it
//              inside that word and stores it; the last thread writes the output
//              length and the status.
//
// Every wait in the look-back is bounded: past VN_SPIN_LIMIT polls a tile
// publishes an error state (which the tiles after it pass on) and the status
// reports EXT_EDEVICE instead of hanging.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/extractor.h"
#include "kernels.h"

namespace ext {
namespace {

#ifndef VN_WORDS_PER_THREAD
#define VN_WORDS_PER_THREAD 8
#endif
// Tiles of 8192 words (1024 threads x 8 words; 73 KiB of LDS, two workgroups
// per CU): measured against 4096-word tiles of 256 x 16, 0.444 -> 0.424 ms at
// n = 2^33 and 0.049 -> 0.036 ms at n = 5*10^8 (half the workgroups to launch
// and look back over, twice the waves per CU).
constexpr int VN_NT = 1024;
constexpr int VN_WPT = VN_WORDS_PER_THREAD;       // consecutive input words per thread
constexpr int VN_TILE_W = VN_NT * VN_WPT;         // words per tile
constexpr int VN_RAW = VN_TILE_W + VN_NT;         // padded LDS words (one pad word per thread's run)
constexpr int VN_OBUF = VN_TILE_W / 2 + 2;        // output words of one tile, on the global grid
static_assert(VN_OBUF <= VN_RAW, "output buffer aliases the input tile");
static_assert(VN_WPT >= 2 && VN_WPT <= 32, "words per thread");
static_assert(VN_NT >= 256 && VN_NT <= 1024 && VN_NT % 64 == 0, "the byte table is filled by the first 256 threads");

constexpr uint64_t ST_AGG = 1ull << 62, ST_PREFIX = 2ull << 62, ST_ERR = 3ull << 62;
constexpr uint64_t ST_VAL = (1ull << 62) - 1;
constexpr uint32_t VN_SPIN_LIMIT = 1u << 22;
constexpr int VN_LB = 4;  // look-back states polled per lane per round trip

__device__ __forceinline__ uint64_t load_state(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_state(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Byte b holds four pairs (bits 2j, 2j+1, j < 4): the kept bits, packed.
__device__ __forceinline__ uint32_t byte_entry(uint32_t b) {
    uint32_t out = 0, k = 0;
    for (int j = 0; j < 4; ++j) {
        uint32_t a = (b >> (2 * j)) & 1u, c = (b >> (2 * j + 1)) & 1u;
        if (a != c) out |= a << k++;
    }
    return out;
}

// One input word: the kept bits (<= 32, packed from bit 0) and their count.
__device__ __forceinline__ uint32_t vn_word(uint64_t v, const uint8_t *tab, uint32_t &cnt) {
    const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    const uint32_t dlo = (lo ^ (lo >> 1)) & 0x55555555u, dhi = (hi ^ (hi >> 1)) & 0x55555555u;
    uint32_t out = tab[lo & 255u];
    out |= (uint32_t)tab[(lo >> 8) & 255u] << __popc(dlo & 0xffu);
    out |= (uint32_t)tab[(lo >> 16) & 255u] << __popc(dlo & 0xffffu);
    out |= (uint32_t)tab[lo >> 24] << __popc(dlo & 0xffffffu);
    const uint32_t a = __popc(dlo);
    out |= (uint32_t)tab[hi & 255u] << a;
    out |= (uint32_t)tab[(hi >> 8) & 255u] << (a + __popc(dhi & 0xffu));
    out |= (uint32_t)tab[(hi >> 16) & 255u] << (a + __popc(dhi & 0xffffu));
    out |= (uint32_t)tab[hi >> 24] << (a + __popc(dhi & 0xffffffu));
    cnt = a + __popc(dhi);
    return out;
}

__device__ __forceinline__ int raw_index(int w) { return w + w / VN_WPT; }

__global__ void k_vn_zero(VnWork w, uint64_t T) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < T) w.state[i] = 0;
    if (i < 2) w.counter[i] = 0;
}

// Input words of tile t in the coalesced order (word k * VN_NT + tid of the tile
// in pre[k]). The loads are the same instructions for every tile, from addresses
// clamped into x (tiles at or past T read word 0): no branch, so a wave's later
// waits can count exactly which loads are still in flight. Words past the pairs
// are zeroed before the tile is used (mask_tile).
__device__ __forceinline__ void load_tile(const uint64_t *__restrict__ x, uint64_t nwords, uint32_t t, uint32_t T,
                                          int tid, uint64_t (&pre)[VN_WPT]) {
    const uint64_t base = (uint64_t)t * VN_TILE_W;
#pragma unroll
    for (int k = 0; k < VN_WPT; ++k) {
        const uint64_t gi = base + k * VN_NT + tid;
        const uint64_t idx = t < T ? (gi < nwords ? gi : nwords - 1) : 0;
        pre[k] = x[idx];
    }
}

// Zero the words of pre past the pairs (only the tile holding the last input
// word has any).
__device__ __forceinline__ void mask_tile(uint64_t (&pre)[VN_WPT], uint64_t nwords, uint64_t last_mask, uint32_t t,
                                          int tid) {
    const uint64_t base = (uint64_t)t * VN_TILE_W;
    if (base + VN_TILE_W < nwords) return;
#pragma unroll
    for (int k = 0; k < VN_WPT; ++k) {
        const uint64_t gi = base + k * VN_NT + tid;
        if (gi >= nwords) pre[k] = 0;
        if (gi == nwords - 1) pre[k] &= last_mask;
    }
}

// Pairs of a word whose bits differ.
__device__ __forceinline__ uint32_t pairs_differing(uint64_t v) {
    return (uint32_t)__popcll((v ^ (v >> 1)) & 0x5555555555555555ull);
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Look-back state of the control wave. A poll reads VN_LB states per lane:
// lane l, slot k holds tile j - 64 k with j = t - 1 - l for the first window,
// so one round trip covers the 64 VN_LB nearest tiles; tiles before tile 0
// count as a zero prefix.
struct LookBack {
    uint64_t s[VN_LB];
    int64_t j;
    uint64_t excl;
    uint32_t spins;
    bool err;
};

enum LbStep { LB_DONE, LB_WAIT, LB_NEXT };

__device__ __forceinline__ void lb_load(LookBack &b, const VnWork &w) {
#pragma unroll
    for (int k = 0; k < VN_LB; ++k) b.s[k] = b.j - 64 * k >= 0 ? load_state(&w.state[b.j - 64 * k]) : ST_PREFIX;
}

// Re-read the states that were not yet published.
__device__ __forceinline__ void lb_repoll(LookBack &b, const VnWork &w) {
#pragma unroll
    for (int k = 0; k < VN_LB; ++k)
        if ((b.s[k] >> 62) == 0) b.s[k] = load_state(&w.state[b.j - 64 * k]);
}

// One look at the current window: DONE when the exclusive prefix is known (or
// on error), WAIT when a nearer tile has published nothing yet, NEXT when the
// whole window holds aggregates only (their sum is taken and the window moves
// back; its states are requested).
__device__ __forceinline__ LbStep lb_step(LookBack &b, int lane, const VnWork &w) {
    uint32_t d = 64 * VN_LB;  // distance (lane + 64 k) of the nearest tile with a prefix
#pragma unroll
    for (int k = VN_LB - 1; k >= 0; --k) {
        const uint64_t pm = __ballot((b.s[k] >> 62) == 2);
        if (pm) d = 64 * k + (__ffsll((unsigned long long)pm) - 1);
    }
    bool waiting = false;
#pragma unroll
    for (int k = 0; k < VN_LB; ++k) waiting |= __ballot((b.s[k] >> 62) == 0 && (uint32_t)(lane + 64 * k) < d) != 0;
    if (waiting) {
        if (++b.spins > VN_SPIN_LIMIT) {
            b.err = true;
            return LB_DONE;
        }
        return LB_WAIT;
    }
    uint64_t part = 0;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < VN_LB; ++k) {
        if ((uint32_t)(lane + 64 * k) <= d) {  // d = window size: the whole window
            part += b.s[k] & ST_VAL;
            bad |= (b.s[k] >> 62) == 3;
        }
    }
    if (__ballot(bad) != 0) {
        b.err = true;
        return LB_DONE;
    }
    b.excl += wave_sum(part);
    if (d < 64 * VN_LB) return LB_DONE;
    b.j -= 64 * VN_LB;
    lb_load(b, w);
    return LB_NEXT;
}

// One workgroup per tile. The tile index comes from a ticket counter, so every
// tile before this one belongs to a workgroup that is already running: the
// look-back waits only on work that is under way. The tile's aggregate is
// published as soon as the tile is loaded and the first look-back poll goes out
// with it; the look-back is finished (by wave 0) after the words are
// compressed, and the bits are assembled at tile-local positions and shifted
// onto the output's word grid as they are written.
__global__ __launch_bounds__(VN_NT) void k_vn_main(const uint64_t *__restrict__ x, uint64_t nwords, uint64_t last_mask,
                                                   uint64_t *__restrict__ z, uint64_t zcap, VnWork w, uint32_t T) {
    __shared__ uint64_t raw[VN_RAW];
    __shared__ uint8_t tab[256];
    __shared__ uint32_t wsum[VN_NT / 64];
    __shared__ uint32_t wagg[VN_NT / 64];
    __shared__ uint32_t sh_ticket;
    __shared__ uint64_t sh_excl;
    uint64_t *obuf = raw;  // tile-local output words, once every thread holds its input words
    constexpr int NW = VN_NT / 64;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform in a wave: scalar branches
    if (tid == 0) sh_ticket = atomicAdd(w.counter, 1u);
    if (tid < 256) tab[tid] = (uint8_t)byte_entry((uint32_t)tid);
    __syncthreads();
    const uint32_t t = sh_ticket;

    // load the tile (coalesced), count its differing pairs (a sum, so the order
    // of the words does not matter) and stage it in LDS
    {
        uint64_t pre[VN_WPT];
        load_tile(x, nwords, t, T, tid, pre);
        mask_tile(pre, nwords, last_mask, t, tid);
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < VN_WPT; ++k) {
            c += pairs_differing(pre[k]);
            raw[raw_index(k * VN_NT + tid)] = pre[k];
        }
        c = wave_sum32(c);
        if (lane == 0) wagg[wave] = c;
    }
    __syncthreads();
    uint32_t agg = 0;
#pragma unroll
    for (int v = 0; v < NW; ++v) agg += wagg[v];

    // wave 0: publish the aggregate and send the first poll
    LookBack b;
    if (wave == 0) {
        b.excl = 0;
        b.spins = 0;
        b.err = false;
        if (lane == 0) store_state(&w.state[t], (t == 0 ? ST_PREFIX : ST_AGG) | agg);
        if (t != 0) {
            b.j = (int64_t)t - 1 - lane;
            lb_load(b, w);
        }
    }

    // this thread's VN_WPT consecutive words
    uint32_t out[VN_WPT], cnt[VN_WPT];
    uint32_t total = 0;
#pragma unroll
    for (int i = 0; i < VN_WPT; ++i) {
        out[i] = vn_word(raw[tid * (VN_WPT + 1) + i], tab, cnt[i]);
        // materialise the packed word here, so its eight table values are not
        // kept live until the assembly below
        asm volatile("" : "+v"(out[i]), "+v"(cnt[i]));
        total += cnt[i];
    }
    // workgroup scan of the per-thread counts
    uint32_t incl = total;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();  // raw is free; the wave sums are visible
    uint32_t before = 0;
#pragma unroll
    for (int v = 0; v < NW; ++v) before += v < wave ? wsum[v] : 0u;
    const uint32_t pos0 = before + incl - total;  // this thread's first bit within the tile
    for (int i = tid; i < VN_OBUF; i += VN_NT) obuf[i] = 0;

    // wave 0: finish the look-back
    if (wave == 0) {
        if (t != 0) {
            for (;;) {
                const LbStep r = lb_step(b, lane, w);
                if (r == LB_DONE) break;
                if (r == LB_WAIT) {
                    __builtin_amdgcn_s_sleep(2);
                    lb_repoll(b, w);
                }
            }
            if (lane == 0) {
                store_state(&w.state[t], (b.err ? ST_ERR : ST_PREFIX) | ((b.excl + agg) & ST_VAL));
                if (b.err) atomicOr(&w.counter[1], 1u);
            }
        }
        if (lane == 0) sh_excl = b.excl;
    }
    __syncthreads();

    // this thread's bits at tile-local positions (local word q = tile bits 64 q ..)
    {
        uint32_t wi = pos0 >> 6, sh = pos0 & 63;
        uint64_t cur = 0;
#pragma unroll
        for (int i = 0; i < VN_WPT; ++i) {
            cur |= (uint64_t)out[i] << sh;
            if (sh + cnt[i] >= 64) {  // then sh >= 32: the carry shift is in [1, 32]
                atomicOr((unsigned long long *)&obuf[wi < VN_OBUF ? wi : VN_OBUF - 1], (unsigned long long)cur);
                ++wi;
                cur = (uint64_t)out[i] >> (64 - sh);
            }
            sh = (sh + cnt[i]) & 63;
        }
        if (sh) atomicOr((unsigned long long *)&obuf[wi < VN_OBUF ? wi : VN_OBUF - 1], (unsigned long long)cur);
    }
    __syncthreads();

    // the tile's bits start at global bit E: shift them onto the 64-bit word grid
    const uint64_t E = sh_excl;
    if (agg != 0) {
        const uint64_t g0 = E >> 6;
        const uint32_t sft = (uint32_t)(E & 63);
        const uint32_t nq = (uint32_t)((sft + agg + 63) >> 6);
        const bool head = sft != 0, tail = ((E + agg) & 63) != 0;
        for (uint32_t q = tid; q < nq && q < VN_OBUF; q += VN_NT) {
            uint64_t v = obuf[q];
            if (sft) v = (v << sft) | (q ? obuf[q - 1] >> (64 - sft) : 0);
            const bool first = q == 0 && head, last = q == nq - 1 && tail;
            if (first) w.pf[t] = v;
            if (last) w.pl[t] = v;
            if (!first && !last && g0 + q < zcap) z[g0 + q] = v;
        }
    }
}

__global__ void k_vn_fix(VnWork w, uint64_t T, uint64_t *__restrict__ z, uint64_t zcap, uint64_t *m_out,
                         int32_t *status) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const uint64_t incl = w.state[t] & ST_VAL;
    const uint64_t E = t ? (w.state[t - 1] & ST_VAL) : 0;
    if (t == T - 1) {
        if (m_out) *m_out = incl;
        if (status) *status = w.counter[1] ? EXT_EDEVICE : (incl ? EXT_OK : EXT_EDEGENERATE);
    }
    if (incl <= E || (incl & 63) == 0) return;  // empty tile, or its range ends on a word boundary
    const uint64_t ql = (incl - 1) >> 6;
    if ((ql << 6) < E) return;  // the word's first bit belongs to an earlier tile
    uint64_t v = w.pl[t];
    const uint64_t end = (ql << 6) + 64;
    for (uint64_t u = t + 1; u < T; ++u) {
        const uint64_t Eu = w.state[u - 1] & ST_VAL;
        if (Eu >= end) break;
        const uint64_t iu = w.state[u] & ST_VAL;
        if (iu == Eu) continue;
        v |= w.pf[u];
        if (iu >= end) break;
    }
    if (ql < zcap) z[ql] = v;
}

}  // namespace

uint64_t vn_tiles(uint64_t n) {
    const uint64_t nwords = ((n & ~1ull) + 63) >> 6;
    return nwords ? (nwords + VN_TILE_W - 1) / VN_TILE_W : 0;
}

size_t vn_workspace_bytes(uint64_t n) {
    const uint64_t T = vn_tiles(n);
    return (size_t)(3 * T * 8 + 256);
}

VnWork vn_work(char *ws, uint64_t n) {
    const uint64_t T = vn_tiles(n);
    VnWork w;
    w.state = (uint64_t *)ws;
    w.pf = w.state + T;
    w.pl = w.pf + T;
    w.counter = (uint32_t *)(w.pl + T);
    return w;
}

hipError_t launch_vn_zero(const VnWork &w, uint64_t n, hipStream_t s) {
    const uint64_t T = vn_tiles(n);
    const uint64_t items = T > 2 ? T : 2;
    hipLaunchKernelGGL(k_vn_zero, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s, w, T);
    return hipGetLastError();
}

hipError_t launch_vn_main(const uint64_t *x, uint64_t n, uint64_t *z, uint64_t zcap, const VnWork &w, hipStream_t s) {
    const uint64_t T = vn_tiles(n);
    const uint64_t nb = n & ~1ull;  // bits that form pairs
    const uint64_t nwords = (nb + 63) >> 6;
    const uint64_t last_mask = (nb & 63) ? ((1ull << (nb & 63)) - 1) : ~0ull;
    hipLaunchKernelGGL(k_vn_main, dim3((unsigned)T), dim3(VN_NT), 0, s, x, nwords, last_mask, z, zcap, w, (uint32_t)T);
    return hipGetLastError();
}

hipError_t launch_vn_fix(const VnWork &w, uint64_t n, uint64_t *z, uint64_t zcap, uint64_t *m_out, int32_t *status,
                         hipStream_t s) {
    const uint64_t T = vn_tiles(n);
    hipLaunchKernelGGL(k_vn_fix, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, w, T, z, zcap, m_out, status);
    return hipGetLastError();
}

}  // namespace ext
