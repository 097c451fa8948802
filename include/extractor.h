/*
 * extractor.h — C-ABI of the MI355X convolution-extractor library
 * (Toeplitz, Circulant and Dodis et al. randomness extractors, computed
 * exactly as an integer convolution by a number-theoretic transform modulo an
 * NTT-friendly prime, reduced mod 2 and truncated).
 *
 * Paper: "Cryptomite: a versatile and user-friendly library of randomness
 * extractors", arXiv 2402.09481.
 *
 * Conventions shared by every call
 * --------------------------------
 * Bit strings are packed little-endian uint64 words: bit i is
 * (w[i >> 6] >> (i & 63)) & 1. Input bits beyond a string's length are
 * ignored; output bits of z beyond m are written as 0.
 *
 * x, y, z are DEVICE pointers, owned by the caller, on the context's device.
 * Inputs are read-only. z must not overlap x or y (EXT_EINVAL otherwise).
 *
 * Every extraction call is stream-ordered and asynchronous: it validates its
 * arguments on the host, synchronously, then enqueues GPU work on `stream`
 * (a hipStream_t, NULL = the default stream) and returns. z is valid once
 * that stream has reached the end of the enqueued work. With EXT_SYNC the
 * call waits for the stream itself and returns the device-side status.
 *
 * Return values: 0 = enqueued (or done, with EXT_SYNC); a negative EXT_E*
 * code otherwise. On any host-side error nothing is enqueued and z is not
 * touched. The one data-dependent check (Dodis et al.: x must not be all
 * zeros or all ones) runs on the device: z is zero-filled and the code
 * EXT_EDEGENERATE is written to *status (if status is not NULL; a device or
 * host-pinned int32) — and returned, with EXT_SYNC.
 *
 * The library keeps device workspace in a stream-ordered pool bounded by the
 * context's HBM budget; a call whose workspace does not fit returns
 * EXT_ENOMEM without enqueuing anything. Calls on one context may be made from
 * several host threads and on several streams (graph-mode batch calls,
 * EXT_GRAPH, take their host-side steps one call at a time per context).
 */
#ifndef PAPER_2402_09481_AMD_EXTRACTOR_H
#define PAPER_2402_09481_AMD_EXTRACTOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------- */
#define EXT_OK 0
#define EXT_EINVAL (-1)      /* null pointer, size out of range, z overlapping x or y, bad flags */
#define EXT_ENOTNA (-2)      /* length must be a prime with 2 as a primitive root */
#define EXT_EDEGENERATE (-3) /* Dodis et al.: x is all zeros or all ones */
#define EXT_ENOMEM (-4)      /* workspace does not fit the context's HBM budget */
#define EXT_ETOOLARGE (-5)   /* the transform length would exceed 2^32 (Von Neumann: n beyond EXT_VN_MAX_BITS) */
#define EXT_EDEVICE (-6)     /* a HIP runtime call failed (Von Neumann: also a device-side wait that ran out) */
#define EXT_ESCRATCH (-7)    /* extract_toeplitz_noalloc: the shape's workspace exceeds EXT_NOALLOC_SCRATCH_BYTES */

/* ---- flags ---------------------------------------------------------- */
/* Toeplitz seed order. PAPER (default): the matrix of eq. (toep) in the
 * section "Toeplitz", entry (i, j) = y_{(i-j) mod (n+m-1)}. LINEAR:
 * z_i = XOR_j s_{i-j+n-1} x_j. The two are one seed rotation apart:
 * s_k = y_{(k+m) mod (n+m-1)}. */
#define EXT_SEED_PAPER 0u
#define EXT_SEED_LINEAR 1u
/* Wait for the stream and return the device status. */
#define EXT_SYNC 2u
/* extract_batch only: record the batch's launch sequence as a HIP graph on
 * first use of a batch signature (the multiset of transform sizes) and replay it
 * afterwards. Worth it when the same signature repeats; without the flag the
 * grouped launches are enqueued directly. The graph is built node by node, not
 * by stream capture, so other host threads may use the device meanwhile. */
#define EXT_GRAPH 4u
/* Single calls: keep the seed's transform in HBM and reuse it. A strong seeded
 * extractor may use one seed for many input blocks (the theorem on extractors
 * with near-perfect seeds used t times); the cache is keyed by the seed pointer and the
 * shape (kind, n, m, seed order), so the caller must not change the seed bits
 * at that address while they are cached (ext_seed_cache_clear drops them).
 * A hit skips one of the three transforms. Sizes that run in one workgroup
 * and the piece schedules (see EXT_SINGLE_TRANSFORM) ignore the flag. */
#define EXT_SEED_CACHED 8u
/* Single calls: compute the extraction as one transform even where the
 * two-piece schedule applies. By default an extraction whose single transform
 * would need the 64-bit field (n + m - 1 > 2^30; for Dodis and Circulant n is
 * the circulant length) while halves of the input fit transforms of at most
 * 2^30 runs as two pieces over 3*2^30+1: the sum over input positions that
 * defines z_i (Toeplitz directly, Dodis and Circulant in their Toeplitz form
 * over the reversed input) split at a = ceil(n/2) rounded up to whole words,
 * each part extracted with its own seed window, the two products added in the
 * transform domain before one inverse — same bits, 32-bit arithmetic. In the
 * same way an extraction whose single transform is 2^27 (over 15*2^27+1) runs
 * as two pieces over 7*2^26+1 when the halves fit transforms of 2^26. This flag
 * keeps the one transform of nextpow2(n+m-1) (over 2^64 - 2^32 + 1 beyond 2^30).
 * Shapes longer than one transform of 2^32 (n + m - 1 > 2^32, such as the
 * paper's QRNG example with n = 6.5e9) always run as k pieces over the 64-bit
 * field: the same split into k balanced, word-aligned pieces of input positions,
 * each piece's transforms of 2^31 (2^32 when m leaves pieces under 2^29), the k
 * products summed in the transform domain (every coefficient of the whole sum is
 * at most n < 2^64 - 2^32 + 1) before one inverse. Four arrays of transform
 * length words; m must be at most 2^32 - 64. */
#define EXT_SINGLE_TRANSFORM 16u

typedef struct ext_ctx ext_ctx;

/* Create a context on HIP device `hip_device`: uploads the twiddle tables of
 * both fields and sets up the workspace pool, capped at hbm_budget_bytes
 * (0 = 90% of the device's free memory). tune_path: a tuning table written by
 * ext_tune_save (or NULL for the built-in plans); a missing or malformed file
 * is ignored. Returns EXT_OK and *out, or an error code and *out = NULL. */
int ext_create(ext_ctx **out, int hip_device, size_t hbm_budget_bytes, const char *tune_path);

/* Synchronise the device, free all device memory of the context. NULL is a no-op. */
void ext_destroy(ext_ctx *ctx);

/* Toeplitz extractor (section "Toeplitz", eq. toeplitz-ext and eq. toep;
 * embedding into a circulant, eq. toeplitz-embed and Alg. 2).
 *   x: n bits (the weak input), y: n+m-1 bits (the seed), z: m bits.
 *   Requires 1 <= m <= n. z_i = XOR_{j<n} toep(y)[i][j] x_j over GF(2).
 *   flags: EXT_SEED_PAPER | EXT_SEED_LINEAR, optionally | EXT_SYNC,
 *   EXT_SEED_CACHED, EXT_SINGLE_TRANSFORM. */
int extract_toeplitz(ext_ctx *ctx, const uint64_t *x, uint64_t n, const uint64_t *y, uint64_t m,
                     uint64_t *z, uint32_t flags, int32_t *status, void *stream);

/* Circulant extractor (Definition of Circulant, eq. circ-matrix; computed by
 * the Dodis et al. route on x' = [x, 0], section "Dodis (and Circulant)
 * implementation").
 *   x: n_in bits; n = n_in + 1 must be a prime with primitive root 2
 *   (EXT_ENOTNA otherwise); y: n bits; z: m bits, 1 <= m <= n - 1.
 *   z_i = XOR_{j<n} x'_{(j-i) mod n} y_j.
 *   flags: optionally EXT_SYNC, EXT_SEED_CACHED, EXT_SINGLE_TRANSFORM. */
int extract_circulant(ext_ctx *ctx, const uint64_t *x, uint64_t n_in, const uint64_t *y, uint64_t m,
                      uint64_t *z, uint32_t flags, int32_t *status, void *stream);

/* Dodis et al. two-source extractor (section "Dodis et al.", eq. DodisOUT with
 * cyclic-shift matrices; convolution form Dodis(x,y)_i = (R(x) * y)_i with
 * indices mod n, Alg. 1).
 *   x, y: n bits each; n prime with primitive root 2 (EXT_ENOTNA otherwise);
 *   1 <= m <= n; x must be neither all zeros nor all ones (device check,
 *   EXT_EDEGENERATE via status). z_i = XOR_{j<n} x_{(j-i) mod n} y_j.
 *   flags: optionally EXT_SYNC, EXT_SEED_CACHED, EXT_SINGLE_TRANSFORM. */
int extract_dodis(ext_ctx *ctx, const uint64_t *x, const uint64_t *y, uint64_t n, uint64_t m, uint64_t *z,
                  uint32_t flags, int32_t *status, void *stream);

/* The Toeplitz extractor (as extract_toeplitz) for callers that cannot
 * allocate memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation. It calls no hipMalloc, hipFree, hipHostMalloc or other
 * allocating routine: its workspace is a fixed array of EXT_NOALLOC_SCRATCH_BYTES
 * in device memory, one per GPU, held from the first ext_create on that GPU until
 * the process ends. The caller still passes x, y and z (device pointers).
 *   Shapes whose workspace does not fit the array return EXT_ESCRATCH (transforms
 *   up to 2^22, i.e. n + m - 1 <= 2^22, fit; up to 2^14 need none). flags:
 *   EXT_SEED_PAPER | EXT_SEED_LINEAR, optionally | EXT_SYNC (without a status
 *   pointer the status word is kept in the array). Launches are not traced.
 *   Every call on one GPU uses that GPU's one array: calls that overlap in time on
 *   one GPU (other streams, other threads, other contexts) race and give wrong
 *   results; order them (one stream, or events). Each call writes every part of
 *   the array it reads, so no call depends on what an earlier call left. */
#define EXT_NOALLOC_SCRATCH_BYTES (((size_t)40) << 20)
int extract_toeplitz_noalloc(ext_ctx *ctx, const uint64_t *x, uint64_t n, const uint64_t *y, uint64_t m,
                             uint64_t *z, uint32_t flags, int32_t *status, void *stream);

/* Von Neumann extractor (section "Von Neumann": for every pair
 * (x_{2j}, x_{2j+1}), j < floor(n/2), in order of j, output x_{2j} when the two
 * bits differ and nothing when they are equal; Alg. 3).
 *   x: n bits, 2 <= n <= EXT_VN_MAX_BITS (EXT_EINVAL below, EXT_ETOOLARGE
 *   above); a trailing odd bit belongs to no pair.
 *   z: z_words >= ceil(floor(n/2) / 64) words (the longest possible output;
 *   EXT_EINVAL otherwise). Words of z below ceil(m/64) are written, the bits
 *   of the last one beyond m as 0; later words are not touched.
 *   m_out: device or host-pinned uint64 (not NULL), receives the output length
 *   m, which depends on the data (about p(1-p)n for i.i.d. bits of bias p).
 *   When no pair differs (Alg. 3's error case) m = 0 and the status is
 *   EXT_EDEGENERATE; written to *status (device or host-pinned, nullable) and
 *   returned with EXT_SYNC. flags: EXT_SYNC only. */
#define EXT_VN_MAX_BITS (((uint64_t)1) << 40)
int extract_von_neumann(ext_ctx *ctx, const uint64_t *x, uint64_t n, uint64_t *z, uint64_t z_words, uint64_t *m_out,
                        uint32_t flags, int32_t *status, void *stream);

/* ---- batched entry point -------------------------------------------- */
#define EXT_KIND_TOEPLITZ 0
#define EXT_KIND_CIRCULANT 1
#define EXT_KIND_DODIS 2
/* ext_workspace_bytes only (extract_batch rejects it): the Von Neumann call */
#define EXT_KIND_VON_NEUMANN 3

typedef struct ext_job {
    int32_t kind;          /* EXT_KIND_* */
    uint32_t flags;        /* EXT_SEED_*, EXT_SINGLE_TRANSFORM (EXT_SYNC is ignored per job) */
    uint64_t n;            /* input length as for the single calls (Circulant: n_in) */
    uint64_t m;            /* output bits */
    const uint64_t *x;     /* device */
    const uint64_t *y;     /* device */
    uint64_t *z;           /* device */
    int32_t *status;       /* device or pinned, nullable: device-side status */
    int32_t err;           /* out: host-side validation result for this job */
    int32_t reserved;
} ext_job;

/* Run many independent extractions (the paper's many privacy-amplification
 * blocks, section "Cryptomite for privacy amplification in QKD") as a few
 * grouped launches: jobs are grouped by transform size; all single-workgroup
 * sizes (transform length <= 2^14) run in one persistent launch that takes
 * jobs from a work counter, larger sizes as batched multi-pass launches, one
 * set per size class. Jobs whose single call would run a piece schedule (see
 * EXT_SINGLE_TRANSFORM) run it in the batch too, their pieces' launches grouped
 * like the others'. With EXT_GRAPH the launch sequence of a batch signature
 * is recorded once as a HIP graph and replayed. `jobs` is a host array of
 * `count` entries. Each job is validated on the host first and gets job.err;
 * invalid jobs are skipped (their z untouched). Returns EXT_OK if every job
 * was enqueued, the first failing job's code if some were skipped, or a
 * context-level error (EXT_ENOMEM, EXT_EDEVICE) with nothing enqueued.
 * flags: EXT_SYNC, EXT_GRAPH. */
int extract_batch(ext_ctx *ctx, ext_job *jobs, size_t count, uint32_t flags, void *stream);

/* The same jobs, one extraction call sequence per job (no grouping, no
 * graph) — the comparison point for extract_batch. */
int extract_batch_unbatched(ext_ctx *ctx, ext_job *jobs, size_t count, uint32_t flags, void *stream);

/* ---- sizes, memory, utilities --------------------------------------- */

/* Device workspace bytes one extraction of this shape takes from the pool
 * (0 if the shape is invalid). kind: EXT_KIND_*; n as for the calls (m is
 * ignored for EXT_KIND_VON_NEUMANN). */
size_t ext_workspace_bytes(int32_t kind, uint64_t n, uint64_t m);

/* Transform length L and field (32 or 64 = word bits) chosen for a shape by
 * default (for a piece schedule: the length of each piece's transforms);
 * 0 on error. */
uint64_t ext_plan_length(int32_t kind, uint64_t n, uint64_t m, int32_t *word_bits);

/* Pool accounting: budget, bytes currently leased by in-flight calls, bytes
 * held by the pool (leased + cached). Any pointer may be NULL. */
int ext_mem_stats(ext_ctx *ctx, size_t *budget, size_t *in_use, size_t *reserved);

/* Release cached (not leased) workspace back to the device. */
int ext_trim(ext_ctx *ctx);

/* Forget every cached seed transform (waits for calls still using them) and
 * report bytes / entries held before, if the pointers are not NULL. */
int ext_seed_cache_clear(ext_ctx *ctx, size_t *bytes, size_t *entries);

/* ---- tuning -------------------------------------------------------------
 * A plan for transform length 2^lg in the field with word_bits (32 or 64):
 * nlev = 0 runs each job in one workgroup (32-bit field, lg <= 14); nlev >= 2
 * gives the log2 sizes of the passes, lgr[0..nlev-2] the strided ones and
 * lgr[nlev-1] the contiguous one (sum = lg, each within the compiled tile
 * sizes). ext_tune_set overrides the built-in plan for later calls (nlev < 0
 * removes the override); EXT_EINVAL for an unsupported plan. ext_tune_get
 * reports the plan in use. These plans serve batches (extract_batch), and single
 * calls whose size class has no single-call plan.
 * ext_tune_set_single / ext_tune_get_single: the plan of single extraction
 * calls (extract_toeplitz, extract_circulant, extract_dodis and the
 * allocation-free variant, each piece of a piece schedule included) for one
 * size class. One job leaves most of the GPU idle, and fewer, larger workgroups
 * can finish it sooner than the plan that is fastest for many jobs at once.
 * nlev < 0 removes it (the class falls back to the ext_tune_set plan);
 * ext_tune_get_single reports the plan a single call uses. ext_tune_save
 * writes every override as a text line "<word_bits> <lg> <nlev> <lgr...>",
 * single-call ones as "single <word_bits> <lg> <nlev> <lgr...>"; the tuning
 * file given to ext_create takes both. */
int ext_tune_set(ext_ctx *ctx, int word_bits, int lg, int nlev, const int *lgr);
int ext_tune_get(ext_ctx *ctx, int word_bits, int lg, int *nlev, int *lgr /* 4 entries */);
int ext_tune_set_single(ext_ctx *ctx, int word_bits, int lg, int nlev, const int *lgr);
int ext_tune_get_single(ext_ctx *ctx, int word_bits, int lg, int *nlev, int *lgr /* 4 entries */);
int ext_tune_save(ext_ctx *ctx, const char *path);

/* Primes with 2 as a primitive root (footnote of the Circulant definition;
 * utilities next_na_set / closest_na_set):
 * ext_is_na_prime: 1 if n is prime and 2 generates (Z/nZ)*, else 0.
 * ext_next_na: smallest such prime >= v (0 if beyond 2^63).
 * ext_closest_na: the nearest one to v; the smaller on a tie. */
int ext_is_na_prime(uint64_t n);
uint64_t ext_next_na(uint64_t v);
uint64_t ext_closest_na(uint64_t v);

/* ---- tracing ----------------------------------------------------------
 * With profiling on, every kernel launch an extraction call enqueues (not the
 * graph-replayed batches) is bracketed by HIP events on the call's stream.
 * ext_profile_read waits for those events and writes one line per launch,
 * "<kernel label> <milliseconds>\n", into buf (NUL-terminated, truncated to
 * cap), then forgets them. Returns the number of launches or a negative code. */
int ext_profile(ext_ctx *ctx, int enable);
int ext_profile_read(ext_ctx *ctx, char *buf, size_t cap);

/* Static text for an EXT_E* code. */
const char *ext_strerror(int code);

/* Library version string. */
const char *ext_version(void);

#ifdef __cplusplus
}
#endif
#endif
