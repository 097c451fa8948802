// Von Neumann extractor on gfx950 (section "Von Neumann": output bit j is
// x_{2j} when x_{2j} != x_{2j+1} and nothing otherwise; Alg. 3 walks the pairs
// in order and appends).
//
// The output is a stream compaction of the input's pairs. One pass over the
// input, bound by HBM:
//
//   k_vn_zero  clears the tile states and the tile ticket counter.
//   k_vn_main  one workgroup per tile of VN_TILE_W input words. A workgroup
//              takes its tile index from a ticket counter (so every tile with a
//              smaller index is already running), loads the tile coalesced into
//              LDS, gives each thread VN_WPT consecutive words, compresses every
//              word (per byte a 256-entry table: the bits kept from its four
//              pairs), scans the per-thread counts, and finds the tile's output
//              offset by a decoupled look-back over the states of the tiles
//              before it (aggregate, then inclusive prefix, published as one
//              64-bit word each). The tile's bits are assembled in LDS on the
//              global 64-bit word grid; words wholly inside the tile's range go
//              straight to z, the first and last partial words to side arrays.
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

constexpr int VN_NT = 256;
constexpr int VN_WPT = 16;
constexpr int VN_TILE_W = VN_NT * VN_WPT;         // words per tile
constexpr int VN_RAW = VN_TILE_W + VN_TILE_W / 16; // padded LDS words (one pad per 16)
constexpr int VN_OBUF = VN_TILE_W / 2 + 2;        // output words of one tile, on the global grid
static_assert(VN_OBUF <= VN_RAW, "output buffer aliases the input tile");

constexpr uint64_t ST_AGG = 1ull << 62, ST_PREFIX = 2ull << 62, ST_ERR = 3ull << 62;
constexpr uint64_t ST_VAL = (1ull << 62) - 1;
constexpr uint32_t VN_SPIN_LIMIT = 1u << 22;

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

__device__ __forceinline__ int raw_index(int w) { return w + (w >> 4); }

__global__ void k_vn_zero(VnWork w, uint64_t T) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < T) w.state[i] = 0;
    if (i < 2) w.counter[i] = 0;
}

__global__ __launch_bounds__(VN_NT) void k_vn_main(const uint64_t *__restrict__ x, uint64_t nwords, uint64_t last_mask,
                                                   uint64_t *__restrict__ z, uint64_t zcap, VnWork w) {
    __shared__ uint64_t raw[VN_RAW];
    __shared__ uint8_t tab[256];
    __shared__ uint32_t wsum[VN_NT / 64];
    __shared__ uint32_t sh_tile;
    __shared__ uint64_t sh_excl;
    uint64_t *obuf = raw;  // reused once every thread holds its words

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) sh_tile = atomicAdd(w.counter, 1u);
    tab[tid] = (uint8_t)byte_entry((uint32_t)tid);
    __syncthreads();
    const uint64_t tile = sh_tile;
    const uint64_t base = tile * VN_TILE_W;

    // coalesced load of the tile (words past the pairs read as 0)
#pragma unroll
    for (int k = 0; k < VN_WPT; ++k) {
        const int li = k * VN_NT + tid;
        const uint64_t gi = base + li;
        uint64_t v = 0;
        if (gi < nwords) {
            v = x[gi];
            if (gi == nwords - 1) v &= last_mask;
        }
        raw[raw_index(li)] = v;
    }
    __syncthreads();

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
    __syncthreads();  // raw is free from here on
    for (int i = tid; i < VN_OBUF; i += VN_NT) obuf[i] = 0;

    // workgroup scan of the per-thread counts
    uint32_t incl = total;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0, agg = 0;
#pragma unroll
    for (int v = 0; v < VN_NT / 64; ++v) {
        before += v < wave ? wsum[v] : 0u;
        agg += wsum[v];
    }
    const uint32_t texcl = before + incl - total;

    // decoupled look-back (wave 0)
    if (wave == 0) {
        uint64_t excl = 0;
        bool err = false;
        if (tile == 0) {
            if (lane == 0) store_state(&w.state[0], ST_PREFIX | agg);
        } else {
            if (lane == 0) store_state(&w.state[tile], ST_AGG | agg);
            int64_t j = (int64_t)tile - 1 - lane;
            uint32_t spins = 0;
            for (;;) {
                uint64_t s = j >= 0 ? load_state(&w.state[j]) : ST_PREFIX;
                while (__ballot((s >> 62) == 0) != 0) {
                    if (++spins > VN_SPIN_LIMIT) {
                        err = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                    if ((s >> 62) == 0) s = load_state(&w.state[j]);
                }
                if (err || __ballot((s >> 62) == 3) != 0) {
                    err = true;
                    break;
                }
                const uint64_t pm = __ballot((s >> 62) == 2);
                if (pm) {
                    const int first = __ffsll((unsigned long long)pm) - 1;  // nearest tile with a prefix
                    excl += wave_sum(lane <= first ? (s & ST_VAL) : 0);
                    break;
                }
                excl += wave_sum(s & ST_VAL);
                j -= 64;
            }
            if (lane == 0) {
                store_state(&w.state[tile], (err ? ST_ERR : ST_PREFIX) | ((excl + agg) & ST_VAL));
                if (err) atomicOr(&w.counter[1], 1u);
            }
        }
        if (lane == 0) sh_excl = excl;
    }
    __syncthreads();
    const uint64_t E = sh_excl;

    // this thread's bits, on the global 64-bit grid (local word 0 = global word E / 64)
    {
        uint64_t pos = (E & 63) + texcl;
        uint32_t wi = (uint32_t)(pos >> 6), sh = (uint32_t)(pos & 63);
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

    if (agg == 0) return;
    const uint64_t g0 = E >> 6;
    const uint32_t nq = (uint32_t)(((E & 63) + agg + 63) >> 6);
    const bool head = (E & 63) != 0, tail = ((E + agg) & 63) != 0;
    for (uint32_t q = tid; q < nq && q < VN_OBUF; q += VN_NT) {
        const uint64_t v = obuf[q];
        const bool first = q == 0 && head, last = q == nq - 1 && tail;
        if (first) w.pf[tile] = v;
        if (last) w.pl[tile] = v;
        if (!first && !last && g0 + q < zcap) z[g0 + q] = v;
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
    hipLaunchKernelGGL(k_vn_main, dim3((unsigned)T), dim3(VN_NT), 0, s, x, nwords, last_mask, z, zcap, w);
    return hipGetLastError();
}

hipError_t launch_vn_fix(const VnWork &w, uint64_t n, uint64_t *z, uint64_t zcap, uint64_t *m_out, int32_t *status,
                         hipStream_t s) {
    const uint64_t T = vn_tiles(n);
    hipLaunchKernelGGL(k_vn_fix, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, w, T, z, zcap, m_out, status);
    return hipGetLastError();
}

}  // namespace ext
