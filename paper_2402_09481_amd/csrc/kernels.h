// Device-side job descriptors and the host-side launch interface of the
// transform kernels. Shared by the kernel translation unit (ntt.hip) and the
// C-ABI / planner (abi.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ext {

// Embedding of a packed bit string into coefficient vector position i of a
// length-L cyclic convolution, written as index maps:
//   PREFIX  (Toeplitz input x): i < len ? b_i : 0
//   SEED    (seed): k = (i + a) mod L; k < N ? b_{(k + rot) mod P} : 0. With
//           a = n - 1 the seed string s_k lands at (k - n + 1) mod L, so output i
//           of the cyclic convolution is z_i = XOR_j s_{i-j+n-1} x_j (linear
//           order, Toeplitz: P = N, rot = 0); rot = m gives the paper's order of
//           eq. toep (Alg. 2's placement v'[i] = y_i for i < m, v'[L-n+1+t] =
//           y_{m+t}). Dodis/Circulant use P = n, rot = 0: s_k = y_{k mod n}.
//   REV     (Dodis/Circulant input): i < a ? b'_{N-1-i} : 0 with
//           b'_j = (j < len ? b_j : 0): the input reversed (Circulant: x' = [x, 0],
//           len = N - 1); a = N for the whole input, a < N for the first piece of
//           the two-piece schedule (its positions a.. belong to the second piece).
// The input's map is always PREFIX or REV and the seed's SEED (the
// single-workgroup path relies on it).
// Dodis(x, y)_i = XOR_j x_{(j-i) mod n} y_j equals the linear-order Toeplitz
// extractor of rev(x) with the seed y || y_{0..m-2}: both sides are
// XOR_{j'} x_{j'} y_{(i+j') mod n}. That needs a transform of length n + m - 1
// instead of the 2n - 1 (plus a wrap-around fold) of the R(x) * y form of Alg. 1.
enum EmbMode : uint32_t { EMB_PREFIX = 0, EMB_SEED = 1, EMB_REV = 2 };

struct Emb {
    const uint64_t *bits;
    uint64_t len;
    uint64_t a;
    uint64_t N;
    uint64_t rot;
    uint64_t P;  // period of the seed string (SEED)
    uint32_t mode;
    uint32_t pad_;
};

// One extraction as the kernels see it.
struct JobDev {
    void *A;           // L words: the input transform, then its spectrum
    void *B;           // L words: the seed transform, then the product, then the convolution
    void *S;           // spectrum operand of the fused pass: A, or a cached seed spectrum
    const void *S2;    // two-piece schedule: the second piece's product spectrum (C_FUSED2 adds it)
    uint64_t *pb;      // packed parity of coefficients [0, out_len) (+1 spare word)
    uint64_t *eb[2];   // the two embedded coefficient vectors as L-bit strings (multi-pass only)
    uint32_t *flags;   // degenerate check: flags[0] = parts, flags[2 + 2g] / [3 + 2g] = part g saw a one / zero bit
    uint64_t *z;       // caller's output, ceil(m/64) words
    int32_t *status;   // caller's status word or nullptr
    Emb ex, ey;        // embeddings of the input (into A) and the seed (into B)
    uint64_t L;        // transform length
    uint64_t m;        // output bits
    uint64_t nfold;    // 0, or n for a wrap-around fold z_i = c_i ^ c_{i+n} (unused by the built-in shapes)
    uint64_t out_len;  // coefficients whose parity is needed: m or m + n
    uint64_t degen_n;  // bits of x checked for all-0/all-1 (Dodis), 0 = no check
    uint64_t K;        // pointwise constant: folds L^-1 (and Montgomery factors); applied by
                       // the single-workgroup pass or the last inverse strided pass
};

struct Tables {
    const void *lo;   // w_max^j, j < 2^16 (twiddle form)
    const void *hi;   // w_max^(j 2^16), j < 2^(LGMAX-16)
    const void *stk;  // Stockham step twiddles (twiddle form), blocks at stk_offset()
};

// In-pass (Stockham) steps span at most 2^TWIN_LG values.
constexpr int TWIN_LG = 14;

// Stockham step twiddles. A step of radix RAD and span NS multiplies value t
// (1 <= t < RAD) of group jm (jm < NS) by w_(NS RAD)^(t jm), or its inverse. The
// block of (RAD, NS, direction) holds these at [(t - 1) NS + jm]: for one t the
// lanes of a wave (consecutive jm) read consecutive words, where indexing one
// table of w_(2^TWIN_LG) by t jm 2^TWIN_LG / (NS RAD) spread a wave's load over
// up to 64 cache lines. Blocks for RAD in {2, 4, 8, 16} and NS = 1, 2, 4, ...
// with NS RAD <= 2^TWIN_LG; radix RAD's blocks take (RAD - 1)(2^(TWIN_LG+1)/RAD - 1)
// words; all forward blocks, then all inverse blocks.
__host__ __device__ constexpr uint64_t stk_rad_words(int rad) {
    return (uint64_t)(rad - 1) * ((uint64_t(2) << TWIN_LG) / rad - 1);
}
__host__ __device__ constexpr uint64_t stk_rad_base(int rad) {
    return rad <= 2 ? 0 : stk_rad_base(rad / 2) + stk_rad_words(rad / 2);
}
constexpr uint64_t STK_DIR_WORDS = stk_rad_base(32);
__host__ __device__ constexpr uint64_t stk_offset(int rad, int ns, bool inv) {
    return (inv ? STK_DIR_WORDS : 0) + stk_rad_base(rad) + (uint64_t)(rad - 1) * (uint64_t)(ns - 1);
}

// Field selector for the launchers.
enum FieldId : int { FIELD_BB = 0, FIELD_GL = 1, FIELD_P0 = 2, FIELD_LZ = 3 };
constexpr int NFIELDS = 4;

// Tile geometry (host copy of the kernels' compile-time choices).
struct Geometry {
    int C;   // columns (strided) or rows (contiguous) per workgroup
    int NT;  // threads per workgroup
};
Geometry strided_geometry(int field, int lgr, int mode);
Geometry contig_geometry(int field, int lgr);
int max_strided_lg(int field);
int max_contig_lg(int field);
int max_small_lg();

// Strided pass over columns: the array viewed as (L / Mprev) blocks of R x S
// (row-major, R = 2^lgr rows at stride S), each column transformed.
enum StridedMode : int { S_FWD_BITS = 0, S_FWD = 1, S_INV = 2, S_INV_PARITY = 3 };
// Columns of a strided tile: C adjacent columns make each row segment 128 bytes
// (32 for 32-bit words, 16 for 64-bit words). (Measured: 8 columns of 64-bit
// words, 64-byte segments and four 32 KiB workgroups per CU, made the value
// passes faster and the passes beside them slower by as much.)
constexpr int strided_cols(int word_bits, int mode) {
    return (void)mode, word_bits == 32 ? 32 : 16;
}
// Contiguous pass over rows of R = 2^lgr consecutive words (last level).
// C_FUSED: the seed's last forward level, the product with the input spectrum S
// and the first inverse level (the factor L^-1, K, is applied by the last
// inverse pass, S_INV_PARITY). Piece schedules (the defining sum split over
// input positions, the pieces' products added in the transform domain): C_PROD
// is the last piece's seed last forward level times its input spectrum S,
// written back (the piece's product spectrum); C_PROD_ADD the same plus the
// product sum S2 of the later pieces; C_FUSED2 is C_FUSED of the first piece
// with the sum S2 added before the inverse.
enum ContigMode : int { C_FWD = 0, C_FUSED = 1, C_FUSED2 = 2, C_PROD = 3, C_PROD_ADD = 4 };

struct PassLaunch {
    int field, lgr, mode;
    int which;            // 0: array A, 1: array B (ignored by C_FUSED, which reads A and B); strided
                          // passes also -1: both arrays in one launch (blockIdx.z selects)
    uint64_t S, Mprev;    // strided only
    uint64_t tiles;       // workgroups per job
    uint64_t out_rows = 0;  // S_INV_PARITY: rows of the level-0 column transform that hold
                            // needed coefficients (the first out_rows rows; 0 or R: all)
    uint32_t njobs;
    const JobDev *jobs;   // device array of njobs, or nullptr to use `one`
    const JobDev *one;    // host copy for single-job launches (passed by value)
};

// Graph recording without stream capture. While a thread has set a recorder,
// every launcher below adds its kernel to rec->graph as a node that depends on
// the previous one (rec->last), in launch order, instead of launching it on the
// stream; the first failure is kept in rec->err. Stream capture is not used for
// batch graphs because, on this runtime, a capture in progress makes
// device-wide calls of other host threads fail (and is invalidated by them).
struct GraphRecorder {
    hipGraph_t graph = nullptr;
    hipGraphNode_t last = nullptr;
    hipError_t err = hipSuccess;
};
void set_graph_recorder(GraphRecorder *rec);  // this thread; nullptr ends recording

hipError_t launch_strided(const PassLaunch &p, const Tables &t, hipStream_t s);
hipError_t launch_contig(const PassLaunch &p, const Tables &t, hipStream_t s);
// Whole extraction in one workgroup (field FLZ, L = 2^lg <= 2^14).
hipError_t launch_small(int lg, uint32_t njobs, const JobDev *jobs, const JobDev *one, const Tables &t,
                        hipStream_t s);
// Size classes of a persistent small-job launch (jobs sorted by class).
struct SmallClasses {
    int n;                    // number of classes (<= 9: lengths 2^6 .. 2^14)
    int lg[9];
    uint32_t first_job[9];    // index of the class's first job in the descriptor array
    uint32_t njobs[9];
    uint32_t first_item[9];   // work items of earlier classes
    uint32_t total_items;
};
// All single-workgroup jobs of a batch in one persistent launch (after zeroing *counter).
hipError_t launch_small_batch(const SmallClasses &cls, const JobDev *jobs, uint32_t *counter, unsigned workgroups,
                              const Tables &t, hipStream_t s);
// Packed parity -> z (fold, mask, degenerate check result, status).
hipError_t launch_pack(uint32_t njobs, uint64_t max_words, const JobDev *jobs, const JobDev *one, hipStream_t s);
// Lay out both inputs as L-bit coefficient strings (eb[0], eb[1]) in the unit
// layout of the first strided level (2^lgr0 rows, C-bit units, tile-major); with
// degen, also the Dodis degenerate-input check (flags). Every job has length L.
hipError_t launch_embed(uint32_t njobs, uint64_t L, int lgr0, int C, const JobDev *jobs, const JobDev *one,
                        bool degen, hipStream_t s);
// Tile-major parity units of the last inverse pass -> packed natural order, rows
// [0, rows) of R (the rows that hold needed coefficients): into pb, or with pack
// straight into z (tail bits cleared, degenerate check applied, status written;
// shapes without the wrap-around fold).
hipError_t launch_ptrans(int field, uint64_t R, uint64_t S, uint64_t rows, uint32_t njobs, const JobDev *jobs,
                         const JobDev *one, bool pack, hipStream_t s);

// Fixed device workspace of the allocation-free Toeplitz entry point: one array
// per GPU for the life of the process (ntt.hip). noalloc_scratch_address looks
// up the calling thread's current device's copy (hipGetSymbolAddress) and must
// be called with that device current; kernels take the returned address, never
// the array's host-side name.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(40) << 20;  // = EXT_NOALLOC_SCRATCH_BYTES
hipError_t noalloc_scratch_address(void **ptr);

// Von Neumann compaction (vonneumann.hip). Workspace of one call: the
// look-back state of every tile (flag in bits 62-63, value below), the partial
// first and last output word of every tile, counter[0] = tile ticket,
// counter[1] = error flag.
struct VnWork {
    uint64_t *state;
    uint64_t *pf;
    uint64_t *pl;
    uint32_t *counter;
};
uint64_t vn_tiles(uint64_t n);
size_t vn_workspace_bytes(uint64_t n);
VnWork vn_work(char *ws, uint64_t n);
hipError_t launch_vn_zero(const VnWork &w, uint64_t n, hipStream_t s);
hipError_t launch_vn_main(const uint64_t *x, uint64_t n, uint64_t *z, uint64_t zcap, const VnWork &w, hipStream_t s);
hipError_t launch_vn_fix(const VnWork &w, uint64_t n, uint64_t *z, uint64_t zcap, uint64_t *m_out, int32_t *status,
                         hipStream_t s);

}  // namespace ext
