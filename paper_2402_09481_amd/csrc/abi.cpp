// C-ABI of the extractor library: argument validation, planning, the
// stream-ordered workspace pool, launch sequences, batching with HIP graphs,
// and the prime utilities. See include/extractor.h for the contract.
#include "../../include/extractor.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "field.h"
#include "kernels.h"

using namespace ext;

namespace {

// ------------------------------------------------------------------ primes with primitive root 2

typedef unsigned __int128 u128;

uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }
uint64_t powmod64(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod64(r, a, m);
        a = mulmod64(a, a, m);
        e >>= 1;
    }
    return r;
}

// Deterministic Miller-Rabin for 64-bit integers (the first 12 primes as bases suffice).
bool is_prime64(uint64_t n) {
    if (n < 2) return false;
    static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t p : small) {
        if (n % p == 0) return n == p;
    }
    uint64_t d = n - 1;
    int s = 0;
    while (!(d & 1)) {
        d >>= 1;
        ++s;
    }
    for (uint64_t a : small) {
        uint64_t x = powmod64(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; ++r) {
            x = mulmod64(x, x, n);
            if (x == n - 1) {
                comp = false;
                break;
            }
        }
        if (comp) return false;
    }
    return true;
}

uint64_t gcd64(uint64_t a, uint64_t b) {
    while (b) {
        uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Pollard's rho (Brent's cycle detection) for a composite n.
uint64_t rho(uint64_t n) {
    if (n % 2 == 0) return 2;
    for (uint64_t c = 1;; ++c) {
        uint64_t y = 2, x = 2, g = 1, q = 1, ys = 2;
        uint64_t r = 1;
        const uint64_t mstep = 128;
        auto f = [&](uint64_t v) { return (mulmod64(v, v, n) + c) % n; };
        do {
            x = y;
            for (uint64_t i = 0; i < r; ++i) y = f(y);
            uint64_t k = 0;
            do {
                ys = y;
                for (uint64_t i = 0; i < std::min(mstep, r - k); ++i) {
                    y = f(y);
                    q = mulmod64(q, x > y ? x - y : y - x, n);
                }
                g = gcd64(q, n);
                k += mstep;
            } while (k < r && g == 1);
            r <<= 1;
        } while (g == 1);
        if (g == n) {
            do {
                ys = f(ys);
                g = gcd64(x > ys ? x - ys : ys - x, n);
            } while (g == 1);
        }
        if (g != n) return g;
    }
}

void factor_into(uint64_t n, std::vector<uint64_t> &out) {
    if (n == 1) return;
    for (uint64_t p = 2; p < 1000 && p * p <= n; ++p) {
        if (n % p == 0) {
            out.push_back(p);
            while (n % p == 0) n /= p;
        }
    }
    if (n == 1) return;
    if (is_prime64(n)) {
        out.push_back(n);
        return;
    }
    uint64_t d = rho(n);
    factor_into(d, out);
    factor_into(n / d, out);
}

bool is_na(uint64_t n) {
    if (n < 3 || !is_prime64(n)) return false;
    std::vector<uint64_t> fs;
    factor_into(n - 1, fs);
    std::sort(fs.begin(), fs.end());
    fs.erase(std::unique(fs.begin(), fs.end()), fs.end());
    for (uint64_t q : fs)
        if (powmod64(2, (n - 1) / q, n) == 1) return false;
    return true;
}

// ------------------------------------------------------------------ fields on the host

template <class F>
std::vector<typename F::T> table_pow(typename F::T base, size_t count) {
    std::vector<typename F::T> t(count);
    typename F::T acc = 1;
    for (size_t j = 0; j < count; ++j) {
        t[j] = F::to_tw(acc);
        acc = F::mulmod(acc, base);
    }
    return t;
}

// The Stockham step blocks (kernels.h, stk_offset) gathered from the powers of
// w_(2^TWIN_LG): entry (t, jm) of the block (rad, ns, inverse) is w_(ns rad)^(+-t jm)
// = w_(2^TWIN_LG)^(+-t jm 2^TWIN_LG / (ns rad)).
template <class F>
std::vector<typename F::TW> stockham_tables() {
    // plain powers of w_(2^TWIN_LG); entries are stored in the field's in-pass form
    std::vector<typename F::T> in(size_t(1) << TWIN_LG);
    {
        const typename F::T base = F::powmod(F::WMAX, uint64_t(1) << (F::LGMAX - TWIN_LG));
        typename F::T acc = 1;
        for (auto &v : in) {
            v = acc;
            acc = F::mulmod(acc, base);
        }
    }
    std::vector<typename F::TW> out(2 * STK_DIR_WORDS);
    const int mask = (1 << TWIN_LG) - 1;
    for (int inv = 0; inv < 2; ++inv)
        for (int rad = 2; rad <= 16; rad *= 2)
            for (int ns = 1; ns * rad <= (1 << TWIN_LG); ns *= 2) {
                const int scale = (1 << TWIN_LG) / (ns * rad);
                for (int t = 1; t < rad; ++t)
                    for (int jm = 0; jm < ns; ++jm) {
                        const int e = t * jm * scale;
                        out[stk_offset(rad, ns, inv != 0) + (uint64_t)(t - 1) * ns + jm] =
                            F::to_stk(in[inv ? (-e) & mask : e]);
                    }
            }
    return out;
}

int ceil_log2(uint64_t v) {
    int l = 0;
    while ((uint64_t(1) << l) < v) ++l;
    return l;
}

// ------------------------------------------------------------------ plan

struct Plan {
    int field = FIELD_BB;
    int lg = 0;
    bool small = false;
    int nlev = 0;
    int lgr[4] = {0, 0, 0, 0};
    int pieces = 1;      // >= 2: a piece schedule, the defining sum split over input
    uint64_t split = 0;  // positions in pieces of `split` bits (a multiple of 64)
};

constexpr int MIN_LEVEL_LG = 7;
constexpr int MIN_LG = 6;

// Level sizes: the last (contiguous) level takes up to its cap, strided levels
// are balanced and kept at or below the preferred size (LDS tile <= 64 KiB).
bool split_levels(int field, int lg, Plan &p) {
    const int cap_c = max_contig_lg(field), cap_s = max_strided_lg(field);
    const int pref_s = 9;  // strided tiles of 2^9 rows fit 64 KiB of LDS in both fields
    for (int k = 2; k <= 4; ++k) {
        if (lg < MIN_LEVEL_LG * k) return false;
        if (lg > cap_c + (k - 1) * cap_s) continue;
        int c = std::max(lg - (k - 1) * pref_s, (lg + k - 1) / k);
        c = std::min(c, cap_c);
        c = std::max(c, MIN_LEVEL_LG);
        int rem = lg - c;
        int ns = k - 1;
        if (rem > ns * cap_s || rem < ns * MIN_LEVEL_LG) continue;
        p.nlev = k;
        for (int i = 0; i < ns; ++i) {
            int share = rem / (ns - i) + ((rem % (ns - i)) ? 1 : 0);
            share = std::min(share, cap_s);
            p.lgr[i] = share;
            rem -= share;
        }
        if (rem != 0) continue;
        p.lgr[k - 1] = c;
        return true;
    }
    return false;
}

// The field of a plan: 15*2^27+1 up to its 2^27, then 3*2^30+1 (32-bit words
// as well) up to 2^30, then Goldilocks; below them all, 7*2^26+1 (lazy values) up
// to its 2^26. Every coefficient is at most the input length n <= L, below every
// prime used for that length.
// force: 0 = automatic, 1 = 15*2^27+1, 2 = Goldilocks, 3 = 3*2^30+1, 5 = 7*2^26+1
// (testing aids; 4 is the two-piece schedule, see plan_shape)
int make_plan(uint64_t Lmin, int force, Plan &p) {
    p = Plan();
    p.lg = std::max(MIN_LG, ceil_log2(Lmin));
    if (p.lg > 32) return EXT_ETOOLARGE;
    p.field = p.lg <= FLZ::LGMAX   ? FIELD_LZ
              : p.lg <= FBB::LGMAX ? FIELD_BB
              : p.lg <= FP0::LGMAX ? FIELD_P0
                                   : FIELD_GL;
    if (force == 1) {
        if (p.lg > FBB::LGMAX) return EXT_ETOOLARGE;
        p.field = FIELD_BB;
        p.lg = std::max(p.lg, 2 * MIN_LEVEL_LG);  // (one workgroup per job is the lazy field's)
    } else if (force == 5) {
        if (p.lg > FLZ::LGMAX) return EXT_ETOOLARGE;
        p.field = FIELD_LZ;
    } else if (force == 2) {
        p.field = FIELD_GL;
        p.lg = std::max(p.lg, 2 * MIN_LEVEL_LG);
    } else if (force == 3) {
        if (p.lg > FP0::LGMAX) return EXT_ETOOLARGE;
        p.field = FIELD_P0;
        p.lg = std::max(p.lg, 2 * MIN_LEVEL_LG);
    }
    if (p.field == FIELD_LZ && p.lg <= max_small_lg()) {
        p.small = true;
        return EXT_OK;
    }
    return split_levels(p.field, p.lg, p) ? EXT_OK : EXT_ETOOLARGE;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout {
    size_t a = 0, b = 0, a2 = 0, b2 = 0, pb = 0, eb0 = 0, eb1 = 0, flags = 0, total = 0;
};

// A and B (L words each; the two-piece schedule has a second pair A2, B2), the
// packed parity and the two embedded inputs (L bits each, plus a spare word),
// and the degenerate-check flags.
Layout workspace_layout(const Plan &p) {
    Layout l;
    if (p.small) return l;
    const size_t L = size_t(1) << p.lg;
    const size_t w = p.field == FIELD_GL ? 8 : 4;
    const size_t bits = align256((L / 64 + 2) * 8);
    const size_t arr = align256(L * w);
    l.a = 0;
    l.b = arr;
    size_t off = 2 * arr;
    if (p.pieces >= 2) {
        l.a2 = off;
        l.b2 = off + arr;
        off += 2 * arr;
    }
    l.pb = off;
    l.eb0 = l.pb + bits;
    l.eb1 = l.eb0 + bits;
    l.flags = l.eb1 + bits;
    l.total = l.flags + 256;
    return l;
}

// ------------------------------------------------------------------ job description

struct Shape {
    int kind;
    uint64_t n, m;     // as passed by the caller
    uint64_t nfold;    // 0 or the circulant length
    uint64_t Lmin;
    uint64_t out_len;
};

int shape_of(int kind, uint64_t n, uint64_t m, Shape &s) {
    s.kind = kind;
    s.n = n;
    s.m = m;
    if (kind == EXT_KIND_TOEPLITZ) {
        if (n < 1 || m < 1 || m > n) return EXT_EINVAL;
        if (n > (uint64_t(1) << 40)) return EXT_ETOOLARGE;
        s.nfold = 0;
        s.Lmin = n + m - 1;
        s.out_len = m;
    } else if (kind == EXT_KIND_CIRCULANT) {
        // computed as the linear-order Toeplitz extractor of rev([x, 0]) with the
        // seed y || y_{0..m-2} (length (n+1) + m - 1)
        if (n < 1 || m < 1 || m > n) return EXT_EINVAL;
        if (n > (uint64_t(1) << 40)) return EXT_ETOOLARGE;
        s.nfold = 0;
        s.Lmin = (n + 1) + m - 1;
        s.out_len = m;
    } else if (kind == EXT_KIND_DODIS) {
        // computed as the linear-order Toeplitz extractor of rev(x) with y || y_{0..m-2}
        if (n < 1 || m < 1 || m > n) return EXT_EINVAL;
        if (n > (uint64_t(1) << 40)) return EXT_ETOOLARGE;
        s.nfold = 0;
        s.Lmin = n + m - 1;
        s.out_len = m;
    } else {
        return EXT_EINVAL;
    }
    // beyond one transform of 2^32 the single calls run a piece schedule over the
    // 64-bit field (plan_shape); m itself must leave room in a transform of 2^32
    if (s.m > (uint64_t(1) << 32) - 64) return EXT_ETOOLARGE;
    return EXT_OK;
}

// is_na with a memo of recent answers: a batch or a serving loop checks the same
// few thousand lengths on every call (Miller-Rabin plus factoring n - 1, a few
// microseconds each)
bool is_na_cached(uint64_t n) {
    static std::mutex mu;
    static std::unordered_map<uint64_t, bool> memo;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = memo.find(n);
        if (it != memo.end()) return it->second;
    }
    const bool r = is_na(n);
    std::lock_guard<std::mutex> g(mu);
    if (memo.size() >= (size_t(1) << 16)) memo.clear();
    memo[n] = r;
    return r;
}

int check_primes(const Shape &s) {
    if (s.kind == EXT_KIND_CIRCULANT && !is_na_cached(s.n + 1)) return EXT_ENOTNA;
    if (s.kind == EXT_KIND_DODIS && !is_na_cached(s.n)) return EXT_ENOTNA;
    return EXT_OK;
}

bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes) {
    uintptr_t x0 = (uintptr_t)a, x1 = x0 + abytes, y0 = (uintptr_t)b, y1 = y0 + bbytes;
    return x0 < y1 && y0 < x1;
}

uint64_t words(uint64_t bits) { return (bits + 63) >> 6; }

// the length of the sum over j: Toeplitz and Dodis n, Circulant n_in + 1
uint64_t conv_n(const Shape &s) { return s.kind == EXT_KIND_CIRCULANT ? s.n + 1 : s.n; }

uint64_t seed_bits(const Shape &s) {
    if (s.kind == EXT_KIND_TOEPLITZ) return s.n + s.m - 1;
    if (s.kind == EXT_KIND_CIRCULANT) return s.n + 1;
    return s.n;
}

int validate(const Shape &s, const uint64_t *x, const uint64_t *y, const uint64_t *z, uint32_t flags) {
    if (!x || !y || !z) return EXT_EINVAL;
    if (flags & ~(EXT_SEED_LINEAR | EXT_SYNC | EXT_SEED_CACHED | EXT_SINGLE_TRANSFORM)) return EXT_EINVAL;
    const size_t zb = words(s.m) * 8;
    if (overlaps(z, zb, x, words(s.n) * 8) || overlaps(z, zb, y, words(seed_bits(s)) * 8)) return EXT_EINVAL;
    return check_primes(s);
}

// Pointwise constant: the 32-bit fields fold L^-1 and two Montgomery factors
// (mont(mont(u, v), K) = u v L^-1), Goldilocks just L^-1.
template <class F>
uint64_t mont_K(int lg) {
    const uint32_t Linv = F::powmod(F::powmod(2, lg), F::P - 2);
    return F::mulmod(F::mulmod(Linv, F::R_MOD_P), F::R_MOD_P);
}
uint64_t pointwise_K(const Plan &p) {
    if (p.field == FIELD_BB) return mont_K<FBB>(p.lg);
    if (p.field == FIELD_LZ) return mont_K<FLZ>(p.lg);
    if (p.field == FIELD_P0) return mont_K<FP0>(p.lg);
    return FGL::powmod(FGL::powmod(2, p.lg), FGL::P - 2);
}

// piece: 0 for a single transform; for a piece schedule, the piece (0 .. pieces-1).
// Piece q takes the input positions [q a, min((q+1) a, n)) of the defining sum
// (a = p.split) and runs on array pair q mod 2; its product spectrum goes to its
// B array, and S2 of piece q points at piece q+1's B (the sum of the later pieces'
// products, which its last pass adds).
JobDev make_jobdev(const Shape &s, const Plan &p, const uint64_t *x, const uint64_t *y, uint64_t *z, int32_t *status,
                   uint32_t flags, char *ws, int piece = 0) {
    JobDev j;
    std::memset(&j, 0, sizeof(j));
    const Layout l = workspace_layout(p);
    const bool odd = (piece & 1) != 0;
    if (ws) {
        j.A = ws + (odd ? l.a2 : l.a);
        j.B = ws + (odd ? l.b2 : l.b);
        j.pb = (uint64_t *)(ws + l.pb);
        j.S = j.A;
        if (p.pieces >= 2 && piece + 1 < p.pieces) j.S2 = ws + (odd ? l.b : l.b2);
        j.eb[0] = (uint64_t *)(ws + l.eb0);
        j.eb[1] = (uint64_t *)(ws + l.eb1);
        j.flags = (uint32_t *)(ws + l.flags);
    }
    j.z = z;
    j.status = status;
    j.L = uint64_t(1) << p.lg;
    j.m = s.m;
    j.nfold = s.nfold;
    j.out_len = s.out_len;
    j.K = pointwise_K(p);
    if (p.pieces >= 2) {
        // z_i = sum_j s_(i-j+n-1) x'_j (Toeplitz: x' = x, s the seed in the linear
        // order; Dodis and Circulant: x' = rev of the circulant generator, s_k =
        // y_(k mod n)). The share of positions [j0, j0 + w) is the Toeplitz extraction
        // of x'_j0 .. x'_(j0+w-1) with the seed window s_t0 .. s_(t0+w+m-2),
        // t0 = n - j0 - w (each index i - j + n - 1 = t0 + (w - 1 + i - (j - j0))).
        const uint64_t n = conv_n(s), a = p.split;
        const uint64_t j0 = (uint64_t)piece * a, w = std::min<uint64_t>(a, n - j0), t0 = n - j0 - w;
        const uint64_t Np = w + s.m - 1;
        if (s.kind == EXT_KIND_TOEPLITZ) {
            const uint64_t N = s.n + s.m - 1;
            const uint64_t rot = ((flags & EXT_SEED_LINEAR) ? t0 : t0 + s.m) % N;  // s_k = y_((k+m) mod N)
            j.ex = Emb{x + j0 / 64, w, 0, 0, 0, 0, EMB_PREFIX, 0};
            j.ey = Emb{y, Np, w - 1, Np, rot, N, EMB_SEED, 0};
            j.degen_n = 0;
        } else {
            // x'_(j0+i) = generator bit n-1-j0-i: the reversed embedding of the
            // generator's first n - j0 positions, w of them
            j.ex = Emb{x, s.n, w, n - j0, 0, 0, EMB_REV, 0};
            j.ey = Emb{y, n, w - 1, Np, t0 % n, n, EMB_SEED, 0};
            j.degen_n = (s.kind == EXT_KIND_DODIS && piece == 0) ? s.n : 0;
        }
    } else if (s.kind == EXT_KIND_TOEPLITZ) {
        const uint64_t N = s.n + s.m - 1;
        j.ex = Emb{x, s.n, 0, 0, 0, 0, EMB_PREFIX, 0};
        const uint64_t rot = (flags & EXT_SEED_LINEAR) ? 0 : (s.m % N);
        j.ey = Emb{y, N, s.n - 1, N, rot, N, EMB_SEED, 0};
        j.degen_n = 0;
    } else {
        // circulant length n (Circulant: n_in + 1 with x' = [x, 0]); x reversed, the
        // seed repeated with period n, output z_i = XOR_j s_{i-j+n-1} rev(x')_j
        const uint64_t n = s.kind == EXT_KIND_CIRCULANT ? s.n + 1 : s.n;
        const uint64_t N = n + s.m - 1;
        j.ex = Emb{x, s.n, n, n, 0, 0, EMB_REV, 0};
        j.ey = Emb{y, n, n - 1, N, 0, n, EMB_SEED, 0};
        j.degen_n = s.kind == EXT_KIND_DODIS ? s.n : 0;
    }
    return j;
}

// ------------------------------------------------------------------ stream-ordered workspace pool

struct Block {
    char *ptr;
    size_t size;
    hipEvent_t ev;       // recorded after the last use
    hipStream_t stream;  // stream of the last use
    bool used;           // ev valid
};

}  // namespace

struct ext_ctx {
    int device = 0;
    size_t budget = 0;
    size_t reserved = 0;  // pool bytes (cached + leased) and tables
    size_t leased = 0;
    std::vector<Block> free_blocks;
    std::mutex mu;
    Tables tb[NFIELDS];
    void *tb_mem[NFIELDS][3] = {};
    int force_field = 0;
    uint64_t piece_bits = 0;  // testing aid: piece schedule for every sum longer than this
    // smallest single transform (log2) replaced by two pieces of half its length, for
    // single calls and batch members (SPLIT_MIN_LG, BATCH_SPLIT_MIN_LG unless a
    // testing aid sets them)
    int split_min_lg = 0, batch_split_min_lg = 0;  // (set by ext_create)
    void *scratch = nullptr;  // this device's allocation-free workspace (noalloc_scratch_address)
    std::map<int, Plan> tuned;  // key: field * 64 + lg
    // plans for single extraction calls where they differ (the GPU mostly idle
    // during one job: fewer, larger workgroups can be faster); same key
    std::map<int, Plan> tuned_single;
    // pinned status words for EXT_SYNC calls without a status pointer
    std::vector<int32_t *> pinned_status;
    // batch graph cache
    // Descriptors are staged in two pinned buffers used in turn, so that the host
    // fills one while the copy of the previous replay may still read the other;
    // done[k] is recorded after the copy from staging k. The device copy desc_dev
    // is overwritten only after the previous replay has finished (its stream waits
    // for `replayed`, recorded after each replay, on the device).
    struct GraphEntry {
        hipGraphExec_t exec = nullptr;
        JobDev *desc_dev = nullptr;
        JobDev *desc_host[2] = {nullptr, nullptr};  // pinned
        size_t ndesc = 0;
        hipEvent_t done[2] = {nullptr, nullptr};
        bool used[2] = {false, false};
        int next = 0;
        hipEvent_t replayed = nullptr;
        bool ever = false;
    };
    std::map<std::string, GraphEntry> graphs;
    // held by a graph-mode batch call from its cache lookup until its replay is
    // enqueued: entries and their staging are used by one call at a time, and
    // eviction never meets an entry in use
    std::mutex graph_mu;
    // transformed-seed cache
    struct SeedEntry {
        char *ptr = nullptr;
        size_t bytes = 0;
        hipEvent_t ready = nullptr;  // the seed transform is complete
        hipEvent_t used = nullptr;   // the last call that read it is complete
        uint64_t tick = 0;
        int busy = 0;                // calls between lookup and recording `used`
        bool recorded = false;       // `ready` is recorded (before that, other calls must not wait on it)
    };
    std::map<std::string, SeedEntry> seeds;
    size_t seed_bytes = 0;
    int seed_clearing = 0;  // clears in progress: calls run without the cache meanwhile
    uint64_t seed_tick = 0;
    // tracing
    bool profile = false;
    struct Mark {
        std::string label;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
};

namespace {

// The field a tuning entry refers to: 32-bit words are 15*2^27+1 up to its
// 2^27 and 3*2^30+1 above; -1 if no field has that length.
int tune_field(int word_bits, int lg) {
    if (word_bits == 64) return lg <= FGL::LGMAX ? FIELD_GL : -1;
    return lg <= FLZ::LGMAX ? FIELD_LZ : lg <= FBB::LGMAX ? FIELD_BB : lg <= FP0::LGMAX ? FIELD_P0 : -1;
}

bool valid_plan(const Plan &p) {
    if (p.small) return p.field == FIELD_LZ && p.lg >= MIN_LG && p.lg <= max_small_lg() && p.nlev == 0;
    if (p.nlev < 2 || p.nlev > 4) return false;
    int sum = 0;
    for (int i = 0; i < p.nlev; ++i) {
        const int cap = i + 1 < p.nlev ? max_strided_lg(p.field) : max_contig_lg(p.field);
        if (p.lgr[i] < MIN_LEVEL_LG || p.lgr[i] > cap) return false;
        sum += p.lgr[i];
    }
    return sum == p.lg;
}

// The built-in plan, or the context's tuned one for the same field and length
// (also in a context that forces a field: a tuned plan of that field applies, so
// that every plan of every field can be run and checked). A single extraction
// call (single) takes the single-call plan of its size class where there is one.
int plan_in_field(ext_ctx *c, uint64_t Lmin, int force, Plan &p, bool single = false) {
    int rc = make_plan(Lmin, force, p);
    if (rc != EXT_OK || !c) return rc;
    const int key = p.field * 64 + p.lg;
    std::lock_guard<std::mutex> g(c->mu);
    if (single) {
        auto it = c->tuned_single.find(key);
        if (it != c->tuned_single.end()) {
            p = it->second;
            return EXT_OK;
        }
    }
    auto it = c->tuned.find(key);
    if (it != c->tuned.end()) p = it->second;
    return EXT_OK;
}

int plan_for(ext_ctx *c, uint64_t Lmin, Plan &p, bool single = false) {
    return plan_in_field(c, Lmin, c ? c->force_field : 0, p, single);
}

// Two-piece schedule for shapes beyond one transform of 3*2^30+1, and for shapes
// whose one transform of 2^27 would run over 15*2^27+1 while their pieces fit the
// lazy field 7*2^26+1 (transforms of at most 2^26). The extraction
// is a sum over input positions j (Toeplitz: z_i = sum_j s_(i-j+n-1) x_j; Dodis and
// Circulant: the same with rev(x') and the periodic seed, n the circulant length);
// it is split at a = ceil(n/2) rounded up to whole words, and each part is a
// Toeplitz extraction of its a_p input positions with its own seed window of
// a_p + m - 1 bits, so both run as transforms of length nextpow2(a + m - 1) over
// 3*2^30+1 or 7*2^26+1 (every coefficient of the two convolutions together is at
// most n, below either prime where it is used). Their products are added in the
// transform domain before one inverse.
constexpr uint64_t TWO_PIECE_MIN_N = 128;
uint64_t two_piece_split(uint64_t n) { return ((n + 1) / 2 + 63) & ~uint64_t(63); }

// The plan for a shape: a single transform (plan_for), or the two-piece
// schedule for a shape whose single transform would need the 64-bit field while
// each piece fits 3*2^30+1, or 15*2^27+1 while each piece fits 7*2^26+1 (unless
// the caller asks for one transform).
// Forced-field contexts keep single transforms, except force 4 (testing aid: two
// pieces whenever n allows).
// Piece schedule over the 64-bit field, for shapes beyond one transform of 2^32
// (or, as a testing aid, any shape whose sum is longer than the context's
// piece_bits): the sum over input positions in k balanced pieces of a bits
// (a multiple of 64), each piece a Toeplitz extraction run as transforms of
// nextpow2(a + m - 1) <= 2^32 (2^31 unless the output leaves pieces under 2^29),
// the k products added in the transform domain (every coefficient of the whole
// sum is at most n < 2^64 - 2^32 + 1) before one inverse.
int plan_pieces_gl(ext_ctx *c, const Shape &s, uint64_t forced_bits, Plan &p, bool single) {
    const uint64_t n = conv_n(s);
    uint64_t a;
    if (forced_bits) {
        a = (forced_bits + 63) & ~uint64_t(63);
    } else {
        const int lg = (uint64_t(1) << 31) >= s.m + (uint64_t(1) << 29) ? 31 : 32;
        const uint64_t amax = ((uint64_t(1) << lg) - s.m + 1) & ~uint64_t(63);
        if (amax < 64) return EXT_ETOOLARGE;
        const uint64_t k = (n + amax - 1) / amax;
        a = (((n + k - 1) / k) + 63) & ~uint64_t(63);
    }
    const int rc = plan_in_field(c, a + s.m - 1, 2, p, single);
    if (rc != EXT_OK) return rc;
    p.split = a;
    p.pieces = (int)((n + a - 1) / a);
    if (p.pieces < 2) {
        p.pieces = 1;
        p.split = 0;
    }
    return EXT_OK;
}

// Smallest single transform (log2) that the halving below replaces, for single
// calls and for batch members, whose extra launches are shared by their class
// (measured: a single call of 2^25 went 0.48 -> 0.42 ms and one of 2^24 0.23 ->
// 0.24 ms; the 4096-block batch 54.7 -> 47.7 ms with batch members from 2^17).
constexpr int SPLIT_MIN_LG = 25, BATCH_SPLIT_MIN_LG = 17;

int plan_shape(ext_ctx *c, const Shape &s, Plan &p, uint32_t flags = 0, bool batch = false) {
    const int force = c ? c->force_field : 0;
    const uint64_t n = conv_n(s);
    const uint64_t piece_bits = c ? c->piece_bits : 0;
    if (s.Lmin > (uint64_t(1) << 32) || (piece_bits && n > piece_bits)) return plan_pieces_gl(c, s, piece_bits, p, !batch);
    const bool can_split = !(flags & EXT_SINGLE_TRANSFORM) && n >= TWO_PIECE_MIN_N &&
                           two_piece_split(n) + s.m - 1 <= (uint64_t(1) << FP0::LGMAX);
    if (force == 4) {
        if (!can_split) return make_plan(s.Lmin, 3, p);
        const int rc = make_plan(two_piece_split(n) + s.m - 1, 3, p);
        p.pieces = 2;
        p.split = two_piece_split(n);
        return rc;
    }
    const int rc = plan_for(c, s.Lmin, p, !batch);
    if (rc != EXT_OK || force || !can_split) return rc;
    // one transform over the 64-bit field: two pieces over 3*2^30+1 where the halves
    // fit; one transform of 2^27 over 15*2^27+1: two pieces of at most 2^26 over the
    // lazy 7*2^26+1 where the halves fit (fewer values, and cheaper ones)
    const uint64_t half = two_piece_split(n) + s.m - 1;
    const bool cheaper_field =
        p.field == FIELD_GL || (p.field == FIELD_BB && half <= (uint64_t(1) << FLZ::LGMAX));
    // a single transform that rounds up past twice the halves: two pieces of half
    // its length, five transforms of L/2 against three of L (a sixth fewer values);
    // not with a cached seed spectrum, which saves a whole transform of L
    const int min_lg = batch ? (c ? c->batch_split_min_lg : BATCH_SPLIT_MIN_LG) : (c ? c->split_min_lg : SPLIT_MIN_LG);
    const bool halving = !(flags & EXT_SEED_CACHED) && !p.small && p.lg >= min_lg && ceil_log2(half) < p.lg;
    if (!cheaper_field && !halving) return rc;
    Plan q;
    if (plan_for(c, half, q, !batch) != EXT_OK || !(q.field == FIELD_P0 || q.field == FIELD_LZ) || q.small) return rc;
    q.pieces = 2;
    q.split = two_piece_split(n);
    p = q;
    return EXT_OK;
}

}  // namespace

namespace {

struct Lease {
    char *ptr = nullptr;
    size_t size = 0;
};

// Take a block of at least `size` bytes usable on `stream`.
int pool_acquire(ext_ctx *c, size_t size, hipStream_t stream, Lease &out) {
    out = Lease();
    if (size == 0) return EXT_OK;
    size = align256(size);
    std::lock_guard<std::mutex> g(c->mu);
    int best = -1;
    for (size_t i = 0; i < c->free_blocks.size(); ++i) {
        Block &b = c->free_blocks[i];
        if (b.size < size || b.size > 2 * size + (size_t(64) << 20)) continue;
        if (b.used && b.stream != stream && hipEventQuery(b.ev) != hipSuccess) continue;
        if (best < 0 || b.size < c->free_blocks[best].size) best = (int)i;
    }
    if (best < 0) {
        // any idle block of a usable size, or room in the budget
        if (c->reserved + size > c->budget) {
            // release idle cached blocks until the new one fits
            for (size_t i = 0; i < c->free_blocks.size() && c->reserved + size > c->budget;) {
                Block &b = c->free_blocks[i];
                if (!b.used || hipEventQuery(b.ev) == hipSuccess) {
                    if (b.used) hipEventDestroy(b.ev);
                    hipFree(b.ptr);
                    c->reserved -= b.size;
                    c->free_blocks.erase(c->free_blocks.begin() + i);
                } else {
                    ++i;
                }
            }
            if (c->reserved + size > c->budget) return EXT_ENOMEM;
        }
        void *p = nullptr;
        if (hipMalloc(&p, size) != hipSuccess) {
            (void)hipGetLastError();
            return EXT_ENOMEM;
        }
        c->reserved += size;
        c->leased += size;
        out.ptr = (char *)p;
        out.size = size;
        return EXT_OK;
    }
    Block b = c->free_blocks[best];
    c->free_blocks.erase(c->free_blocks.begin() + best);
    if (b.used) {
        if (b.stream != stream) hipStreamWaitEvent(stream, b.ev, 0);
        hipEventDestroy(b.ev);
    }
    c->leased += b.size;
    out.ptr = b.ptr;
    out.size = b.size;
    return EXT_OK;
}

void pool_release(ext_ctx *c, Lease &l, hipStream_t stream) {
    if (!l.ptr) return;
    Block b;
    b.ptr = l.ptr;
    b.size = l.size;
    b.stream = stream;
    b.used = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) == hipSuccess;
    if (b.used) hipEventRecord(b.ev, stream);
    std::lock_guard<std::mutex> g(c->mu);
    c->leased -= l.size;
    c->free_blocks.push_back(b);
    l = Lease();
}

// ------------------------------------------------------------------ launch sequences

// Brackets one launch with timing events when tracing is on.
struct Tracer {
    ext_ctx *c;
    hipStream_t s;
    bool on;
    hipEvent_t a = nullptr;
    Tracer(ext_ctx *c_, hipStream_t s_, bool quiet) : c(c_), s(s_), on(c_->profile && !quiet) {}
    void begin() {
        if (!on) return;
        if (hipEventCreate(&a) != hipSuccess) {
            a = nullptr;
            return;
        }
        hipEventRecord(a, s);
    }
    // (labels are built only when tracing is on: `if (tr.on) tr.end(...)`, so
    // that an untraced launch sequence makes no host allocation)
    void end(const std::string &label) {
        if (!on || !a) return;
        hipEvent_t b = nullptr;
        if (hipEventCreate(&b) != hipSuccess) return;
        hipEventRecord(b, s);
        std::lock_guard<std::mutex> g(c->mu);
        c->marks.push_back(ext_ctx::Mark{label, a, b});
        a = nullptr;
    }
};

// "<kind>[<field>,lgr=<log2 transform size>,mode=<pass mode>,arr=<0: input, 1: seed>]"
// field: u32 = 15*2^27+1, p0 = 3*2^30+1 (32-bit words), u64 = Goldilocks
const char *field_tag(int field) {
    return field == FIELD_BB ? "u32" : field == FIELD_P0 ? "p0" : field == FIELD_LZ ? "lz" : "u64";
}
std::string pass_label(const char *what, int field, int lgr, int mode, int which = 0) {
    char b[112];
    snprintf(b, sizeof b, "%s[%s,lgr=%d,mode=%d,arr=%d]", what, field_tag(field), lgr, mode, which);
    return b;
}

// Enqueue the whole extraction for njobs jobs sharing one plan. jobs_dev: device
// descriptors (batched launches) or nullptr with `one` for a single job.
// COLD: both transforms, product, inverse, parity. SEED_ONLY: the seed's full
// forward transform into B (a seed-cache entry). WARM: the input's transform
// fused with the cached seed spectrum S, inverse in A, parity.
// FWD_BOTH: the second piece of the two-piece schedule: both operands' forward
// transforms, the seed's last level multiplied by the input's spectrum (the
// piece's product, left in B); TWO: the first piece, whose fused pass adds the
// second piece's product.
enum Phase { PH_COLD = 0, PH_SEED_ONLY = 1, PH_WARM = 2, PH_FWD_BOTH = 3, PH_TWO = 4, PH_FWD_ACC = 5 };

// The launches of one extraction phase for njobs jobs (descriptors jobs_dev, or
// the single job `one`). quiet: no tracing events (graph recording and the
// allocation-free entry point).

hipError_t enqueue(ext_ctx *c, const Plan &p, uint32_t njobs, const JobDev *jobs_dev, const JobDev *one,
                   uint64_t max_m, bool any_degen, hipStream_t s, bool quiet = false, Phase ph = PH_COLD) {
    const Tables &tb = c->tb[p.field];
    Tracer tr(c, s, quiet);
    if (p.small) {
        tr.begin();
        hipError_t e = launch_small(p.lg, njobs, jobs_dev, one, tb, s);
        if (tr.on) tr.end(pass_label("small", p.field, p.lg, 0));
        return e;
    }
    const uint64_t L = uint64_t(1) << p.lg;
    hipError_t e;
    tr.begin();
    e = launch_embed(njobs, L, p.lgr[0], strided_geometry(p.field, p.lgr[0], S_FWD_BITS).C, jobs_dev, one, any_degen,
                     s);
    if (tr.on) tr.end("embed");
    if (e != hipSuccess) return e;
    // the operands transformed here: both (-1), or only the seed (SEED_ONLY) or only
    // the input (WARM); the fused pass runs on `fused`
    const int only = ph == PH_SEED_ONLY ? 1 : ph == PH_WARM ? 0 : -1;
    const int fused = ph == PH_WARM ? 0 : 1;
    // strided forward levels: both operands in one launch per level (blockIdx.z
    // selects the array; they are independent until the fused pass)
    uint64_t Mprev = L;
    for (int i = 0; i + 1 < p.nlev; ++i) {
        PassLaunch pl;
        pl.field = p.field;
        pl.lgr = p.lgr[i];
        pl.mode = i == 0 ? S_FWD_BITS : S_FWD;
        const Geometry g = strided_geometry(p.field, p.lgr[i], pl.mode);
        pl.which = only;
        pl.Mprev = Mprev;
        pl.S = Mprev >> p.lgr[i];
        pl.tiles = (L / Mprev) * (pl.S / g.C);
        pl.njobs = njobs;
        pl.jobs = jobs_dev;
        pl.one = one;
        tr.begin();
        e = launch_strided(pl, tb, s);
        if (tr.on) tr.end(pass_label("strided", p.field, pl.lgr, pl.mode, only < 0 ? 2 : only));
        if (e != hipSuccess) return e;
        Mprev = pl.S;
    }
    // the last forward level: the input's first (its spectrum is an operand of the
    // seed's fused pass)
    for (int which = 0; which < 2; ++which) {
        if (only >= 0 && which != only) continue;
        const int lc = p.lgr[p.nlev - 1];
        const Geometry g = contig_geometry(p.field, lc);
        PassLaunch pl;
        pl.field = p.field;
        pl.lgr = lc;
        const bool fwd_only = ph == PH_SEED_ONLY || ph == PH_FWD_BOTH || ph == PH_FWD_ACC;
        pl.mode = (ph == PH_FWD_BOTH && which == 1)   ? C_PROD
                  : (ph == PH_FWD_ACC && which == 1)  ? C_PROD_ADD
                  : (fwd_only || ((ph == PH_COLD || ph == PH_TWO) && which == 0)) ? C_FWD
                  : ph == PH_TWO                      ? C_FUSED2
                                                      : C_FUSED;
        pl.which = which;
        pl.S = 0;
        pl.Mprev = 0;
        pl.tiles = L >> lc;
        pl.tiles /= (uint64_t)g.C;
        pl.njobs = njobs;
        pl.jobs = jobs_dev;
        pl.one = one;
        tr.begin();
        e = launch_contig(pl, tb, s);
        if (tr.on) tr.end(pass_label("contig", p.field, pl.lgr, pl.mode, which));
        if (e != hipSuccess) return e;
    }
    if (ph == PH_SEED_ONLY || ph == PH_FWD_BOTH || ph == PH_FWD_ACC) return hipSuccess;
    // inverse: strided levels backwards; level 0 writes packed parity. The output
    // length out_len is m for every shape built here (batch descriptors included);
    // a single job's own out_len is honoured as well.
    const uint64_t max_out = one ? std::max<uint64_t>(max_m, one->out_len) : max_m;
    uint64_t out_rows = 0;
    uint64_t mp[4] = {0, 0, 0, 0};  // the block size M before level i (nlev <= 4)
    uint64_t M = L;
    for (int i = 0; i < p.nlev; ++i) {
        mp[i] = M;
        M >>= p.lgr[i];
    }
    for (int i = p.nlev - 2; i >= 0; --i) {
        PassLaunch pl;
        pl.field = p.field;
        pl.lgr = p.lgr[i];
        pl.mode = i == 0 ? S_INV_PARITY : S_INV;
        const Geometry g = strided_geometry(p.field, p.lgr[i], pl.mode);
        pl.which = fused;
        pl.Mprev = mp[i];
        pl.S = mp[i] >> p.lgr[i];
        pl.tiles = (L / mp[i]) * (pl.S / g.C);
        // level 0: coefficient r S + c sits in row r, and only the coefficients below
        // the output length are read back
        pl.out_rows = std::min<uint64_t>((max_out + pl.S - 1) / pl.S, uint64_t(1) << p.lgr[i]);
        if (i == 0) out_rows = pl.out_rows;
        pl.njobs = njobs;
        pl.jobs = jobs_dev;
        pl.one = one;
        tr.begin();
        e = launch_strided(pl, tb, s);
        if (tr.on) tr.end(pass_label("strided", p.field, pl.lgr, pl.mode, fused));
        if (e != hipSuccess) return e;
    }
    // the 32-bit fields' last inverse pass has written z; for the 64-bit field the
    // parity transpose writes z itself (the degenerate check ran with the
    // embedding), unless a job folds (z_i = c_i ^ c_(i+n), which reads the packed
    // parity string): batch descriptors never fold
    const bool fold = one && one->nfold;
    if (!fold && p.field != FIELD_GL) return hipSuccess;
    tr.begin();
    e = launch_ptrans(p.field, uint64_t(1) << p.lgr[0], L >> p.lgr[0], out_rows, njobs, jobs_dev, one, !fold, s);
    if (tr.on) tr.end(fold ? "ptrans" : "ptrans_pack");
    if (e != hipSuccess || !fold) return e;
    tr.begin();
    e = launch_pack(njobs, words(max_m), jobs_dev, one, s);
    if (tr.on) tr.end("pack");
    return e;
}

int32_t *take_pinned_status(ext_ctx *c) {
    std::lock_guard<std::mutex> g(c->mu);
    if (!c->pinned_status.empty()) {
        int32_t *p = c->pinned_status.back();
        c->pinned_status.pop_back();
        return p;
    }
    int32_t *p = nullptr;
    if (hipHostMalloc((void **)&p, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) return nullptr;
    return p;
}

void give_pinned_status(ext_ctx *c, int32_t *p) {
    std::lock_guard<std::mutex> g(c->mu);
    c->pinned_status.push_back(p);
}

void seed_free(ext_ctx::SeedEntry &se) {
    hipEventSynchronize(se.used);
    hipEventDestroy(se.ready);
    hipEventDestroy(se.used);
    hipFree(se.ptr);
}

// The cached spectrum of this call's seed, computing it (on stream s, into a new
// entry) on a miss. Entries are evicted least recently used, once the calls that
// read them are done, to keep the cache within a quarter of the budget. Returns
// nullptr (and leaves e = hipSuccess) when no entry can be made: the caller then
// runs the cold path.
ext_ctx::SeedEntry *seed_entry(ext_ctx *c, const Shape &sh, const Plan &p, const uint64_t *y, uint32_t flags,
                               hipStream_t s, const JobDev &jd, hipError_t &e) {
    // (the pass split is part of the key: the spectrum's order in memory follows
    // the plan, and the plan of a size class can change between calls)
    char key[192];
    snprintf(key, sizeof key, "%p:%d:%llu:%llu:%u:%d:%d:%d.%d.%d.%d.%d", (const void *)y, sh.kind,
             (unsigned long long)sh.n, (unsigned long long)sh.m, flags & EXT_SEED_LINEAR, p.field, p.lg, p.nlev,
             p.lgr[0], p.lgr[1], p.lgr[2], p.lgr[3]);
    const size_t bytes = (size_t(1) << p.lg) * (p.field == FIELD_GL ? 8 : 4);
    std::unique_lock<std::mutex> g(c->mu);
    if (c->seed_clearing) return nullptr;
    auto it = c->seeds.find(key);
    if (it != c->seeds.end()) {
        // an entry whose transform another call is still enqueueing: waiting on
        // its unrecorded event would not wait, so this call runs without the cache
        if (!it->second.recorded) return nullptr;
        it->second.tick = ++c->seed_tick;
        it->second.busy++;
        ext_ctx::SeedEntry *se = &it->second;
        g.unlock();
        e = hipStreamWaitEvent(s, se->ready, 0);
        return se;
    }
    const size_t cap = c->budget / 4;
    while (c->seed_bytes + bytes > cap) {
        auto victim = c->seeds.end();
        for (auto jt = c->seeds.begin(); jt != c->seeds.end(); ++jt)
            if (!jt->second.busy && (victim == c->seeds.end() || jt->second.tick < victim->second.tick)) victim = jt;
        if (victim == c->seeds.end()) break;
        c->seed_bytes -= victim->second.bytes;
        c->reserved -= victim->second.bytes;
        seed_free(victim->second);
        c->seeds.erase(victim);
    }
    if (c->seed_bytes + bytes > cap || c->reserved + bytes > c->budget) return nullptr;
    ext_ctx::SeedEntry se;
    if (hipMalloc((void **)&se.ptr, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (hipEventCreateWithFlags(&se.ready, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&se.used, hipEventDisableTiming) != hipSuccess) {
        hipFree(se.ptr);
        e = hipErrorOutOfMemory;
        return nullptr;
    }
    se.bytes = bytes;
    se.tick = ++c->seed_tick;
    se.busy = 1;
    c->seed_bytes += bytes;
    c->reserved += bytes;
    ext_ctx::SeedEntry *ent = &(c->seeds[key] = se);
    g.unlock();
    JobDev sj = jd;
    sj.B = ent->ptr;  // the seed's full transform lands in the entry
    e = enqueue(c, p, 1, nullptr, &sj, sh.m, false, s, false, PH_SEED_ONLY);
    if (e == hipSuccess) e = hipEventRecord(ent->ready, s);
    if (e == hipSuccess) e = hipEventRecord(ent->used, s);
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> g2(c->mu);
        ent->recorded = true;
    }
    return ent;
}

int extract_one(ext_ctx *c, int kind, const uint64_t *x, uint64_t n, const uint64_t *y, uint64_t m, uint64_t *z,
                uint32_t flags, int32_t *status, hipStream_t s) {
    if (!c) return EXT_EINVAL;
    Shape sh;
    int rc = shape_of(kind, n, m, sh);
    if (rc) return rc;
    if ((rc = validate(sh, x, y, z, flags)) != EXT_OK) return rc;
    Plan p;
    if ((rc = plan_shape(c, sh, p, flags)) != EXT_OK) return rc;
    if (hipSetDevice(c->device) != hipSuccess) return EXT_EDEVICE;
    const Layout lay = workspace_layout(p);
    Lease lease;
    if ((rc = pool_acquire(c, lay.total, s, lease)) != EXT_OK) return rc;
    int32_t *st = status;
    int32_t *mine = nullptr;
    if ((flags & EXT_SYNC) && !st) {
        mine = take_pinned_status(c);
        if (!mine) {
            pool_release(c, lease, s);
            return EXT_EDEVICE;
        }
        *mine = 0;
        st = mine;
    }
    JobDev jd = make_jobdev(sh, p, x, y, z, st, flags, lease.ptr);
    hipError_t e = hipSuccess;
    // (the two-piece schedule does not use the seed cache)
    ext_ctx::SeedEntry *se = (flags & EXT_SEED_CACHED) && !p.small && p.pieces == 1
                                 ? seed_entry(c, sh, p, y, flags, s, jd, e)
                                 : nullptr;
    if (se && e != hipSuccess) {
        std::lock_guard<std::mutex> g(c->mu);
        se->busy--;
    }
    if (e == hipSuccess) {
        if (se) {
            jd.S = se->ptr;
            e = enqueue(c, p, 1, nullptr, &jd, sh.m, jd.degen_n != 0, s, false, PH_WARM);
            if (e == hipSuccess) e = hipEventRecord(se->used, s);
            std::lock_guard<std::mutex> g(c->mu);
            se->busy--;
        } else if (p.pieces >= 2) {
            // the last piece's product, then each earlier piece's product plus the sum
            // so far, then the first piece fused with that sum, one inverse, parity
            for (int q = p.pieces - 1; q >= 1 && e == hipSuccess; --q) {
                const JobDev jq = make_jobdev(sh, p, x, y, z, st, flags, lease.ptr, q);
                e = enqueue(c, p, 1, nullptr, &jq, sh.m, false, s, false,
                            q == p.pieces - 1 ? PH_FWD_BOTH : PH_FWD_ACC);
            }
            if (e == hipSuccess) e = enqueue(c, p, 1, nullptr, &jd, sh.m, jd.degen_n != 0, s, false, PH_TWO);
        } else {
            e = enqueue(c, p, 1, nullptr, &jd, sh.m, jd.degen_n != 0, s);
        }
    }
    pool_release(c, lease, s);
    if (e != hipSuccess) {
        if (mine) give_pinned_status(c, mine);
        return EXT_EDEVICE;
    }
    if (flags & EXT_SYNC) {
        if (hipStreamSynchronize(s) != hipSuccess) rc = EXT_EDEVICE;
        else {
            int32_t v = 0;
            if (mine) v = *mine;
            else if (hipMemcpy(&v, st, sizeof(v), hipMemcpyDefault) != hipSuccess) v = EXT_EDEVICE;
            rc = v;
        }
        if (mine) give_pinned_status(c, mine);
    }
    return rc;
}

}  // namespace

namespace {
void pinned_release_all(ext_ctx *c);

void graph_entry_free(ext_ctx::GraphEntry &ge) {
    if (ge.exec) hipGraphExecDestroy(ge.exec);
    if (ge.desc_dev) hipFree(ge.desc_dev);
    for (int k = 0; k < 2; ++k) {
        if (ge.desc_host[k]) hipHostFree(ge.desc_host[k]);
        if (ge.done[k]) hipEventDestroy(ge.done[k]);
    }
    if (ge.replayed) hipEventDestroy(ge.replayed);
}

bool graph_entry_idle(ext_ctx::GraphEntry &ge) {
    for (int k = 0; k < 2; ++k)
        if (ge.used[k] && hipEventQuery(ge.done[k]) != hipSuccess) return false;
    return !ge.ever || hipEventQuery(ge.replayed) == hipSuccess;
}

// The address of each device's allocation-free workspace, looked up once per
// device (with that device current) and kept for the life of the process.
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch;

hipError_t scratch_for_device(int device, void **out) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch.find(device);
    if (it != g_scratch.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void *p = nullptr;
    const hipError_t e = noalloc_scratch_address(&p);  // the caller made `device` current
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return e != hipSuccess ? e : hipErrorInvalidSymbol;
    }
    g_scratch[device] = p;
    *out = p;
    return hipSuccess;
}
}  // namespace

// ================================================================== C-ABI

extern "C" {

const char *ext_version(void) { return "paper_2402_09481_amd 0.1 (gfx950)"; }

const char *ext_strerror(int code) {
    switch (code) {
        case EXT_OK: return "ok";
        case EXT_EINVAL: return "invalid argument (null pointer, size out of range, overlapping output, bad flags)";
        case EXT_ENOTNA: return "length must be a prime with 2 as a primitive root";
        case EXT_EDEGENERATE: return "Dodis et al.: the input is all zeros or all ones";
        case EXT_ENOMEM: return "workspace exceeds the context's HBM budget";
        case EXT_ETOOLARGE: return "transform length would exceed 2^32";
        case EXT_EDEVICE: return "HIP runtime error";
        case EXT_ESCRATCH: return "workspace exceeds the allocation-free entry point's fixed scratch";
    }
    return "unknown error code";
}

int ext_is_na_prime(uint64_t n) { return is_na(n) ? 1 : 0; }

uint64_t ext_next_na(uint64_t v) {
    for (uint64_t c = std::max<uint64_t>(v, 3); c < (uint64_t(1) << 63); ++c)
        if (is_na(c)) return c;
    return 0;
}

uint64_t ext_closest_na(uint64_t v) {
    uint64_t up = ext_next_na(v);
    uint64_t lo = 0;
    for (uint64_t c = v; c >= 3; --c)
        if (is_na(c)) {
            lo = c;
            break;
        }
    if (lo == 0) return up;
    if (up == 0) return lo;
    return (v - lo) <= (up - v) ? lo : up;
}

size_t ext_workspace_bytes(int32_t kind, uint64_t n, uint64_t m) {
    Shape s;
    Plan p;
    if (kind == EXT_KIND_VON_NEUMANN) return (n >= 2 && n <= EXT_VN_MAX_BITS) ? align256(vn_workspace_bytes(n)) : 0;
    if (shape_of(kind, n, m, s) != EXT_OK) return 0;
    if (plan_shape(nullptr, s, p) != EXT_OK) return 0;
    return workspace_layout(p).total;
}

uint64_t ext_plan_length(int32_t kind, uint64_t n, uint64_t m, int32_t *word_bits) {
    Shape s;
    Plan p;
    if (shape_of(kind, n, m, s) != EXT_OK) return 0;
    if (plan_shape(nullptr, s, p) != EXT_OK) return 0;
    if (word_bits) *word_bits = p.field == FIELD_GL ? 64 : 32;
    return uint64_t(1) << p.lg;
}

int ext_create(ext_ctx **out, int hip_device, size_t hbm_budget_bytes, const char *tune_path) {
    if (!out) return EXT_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return EXT_EDEVICE;
    if (hipSetDevice(hip_device) != hipSuccess) return EXT_EDEVICE;
    ext_ctx *c = new ext_ctx();
    c->device = hip_device;
    if (scratch_for_device(hip_device, &c->scratch) != hipSuccess) {
        delete c;
        return EXT_EDEVICE;
    }
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) {
        delete c;
        return EXT_EDEVICE;
    }
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)freeb);
    const char *ff = getenv("EXT_FORCE_FIELD");  // testing aid: "bb", "gl" or "p0"
    if (ff && !strcmp(ff, "gl")) c->force_field = 2;
    if (ff && !strcmp(ff, "bb")) c->force_field = 1;
    if (ff && !strcmp(ff, "p0")) c->force_field = 3;
    if (ff && !strcmp(ff, "lz")) c->force_field = 5;
    if (ff && !strcmp(ff, "p0x2")) c->force_field = 4;  // two-piece schedule wherever it can run
    // testing aid: the 64-bit piece schedule with pieces of this many input bits
    if (const char *pb = getenv("EXT_PIECE_BITS")) c->piece_bits = strtoull(pb, nullptr, 10);
    // testing aids: the transform sizes from which the halving applies
    c->split_min_lg = SPLIT_MIN_LG;
    c->batch_split_min_lg = BATCH_SPLIT_MIN_LG;
    if (const char *v = getenv("EXT_SPLIT_MIN_LG")) c->split_min_lg = atoi(v);
    if (const char *v = getenv("EXT_BATCH_SPLIT_MIN_LG")) c->batch_split_min_lg = atoi(v);
    // twiddle tables
    auto upload = [&](int f, int k, const void *src, size_t bytes) -> bool {
        void *d = nullptr;
        if (hipMalloc(&d, bytes) != hipSuccess) return false;
        if (hipMemcpy(d, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return false;
        c->tb_mem[f][k] = d;
        c->reserved += bytes;
        return true;
    };
    bool ok = true;
    {
        using F = FBB;
        auto lo = table_pow<F>(F::WMAX, size_t(1) << 16);
        auto hi = table_pow<F>(F::powmod(F::WMAX, uint64_t(1) << 16), size_t(1) << (F::LGMAX - 16));
        auto stk = stockham_tables<F>();
        ok = ok && upload(FIELD_BB, 0, lo.data(), lo.size() * 4) && upload(FIELD_BB, 1, hi.data(), hi.size() * 4) &&
             upload(FIELD_BB, 2, stk.data(), stk.size() * 4);
    }
    {
        using F = FGL;
        auto lo = table_pow<F>(F::WMAX, size_t(1) << 16);
        auto hi = table_pow<F>(F::powmod(F::WMAX, uint64_t(1) << 16), size_t(1) << (F::LGMAX - 16));
        auto stk = stockham_tables<F>();
        ok = ok && upload(FIELD_GL, 0, lo.data(), lo.size() * 8) && upload(FIELD_GL, 1, hi.data(), hi.size() * 8) &&
             upload(FIELD_GL, 2, stk.data(), stk.size() * 8);
    }
    {
        using F = FP0;
        auto lo = table_pow<F>(F::WMAX, size_t(1) << 16);
        auto hi = table_pow<F>(F::powmod(F::WMAX, uint64_t(1) << 16), size_t(1) << (F::LGMAX - 16));
        auto stk = stockham_tables<F>();
        ok = ok && upload(FIELD_P0, 0, lo.data(), lo.size() * 4) && upload(FIELD_P0, 1, hi.data(), hi.size() * 4) &&
             upload(FIELD_P0, 2, stk.data(), stk.size() * 4);
    }
    {
        using F = FLZ;  // between passes Montgomery form; in-pass Shoup pairs (8 bytes)
        auto lo = table_pow<F>(F::WMAX, size_t(1) << 16);
        auto hi = table_pow<F>(F::powmod(F::WMAX, uint64_t(1) << 16), size_t(1) << (F::LGMAX - 16));
        auto stk = stockham_tables<F>();
        ok = ok && upload(FIELD_LZ, 0, lo.data(), lo.size() * 4) && upload(FIELD_LZ, 1, hi.data(), hi.size() * 4) &&
             upload(FIELD_LZ, 2, stk.data(), stk.size() * 8);
    }
    if (!ok) {
        ext_destroy(c);
        return EXT_EDEVICE;
    }
    for (int f = 0; f < NFIELDS; ++f) c->tb[f] = Tables{c->tb_mem[f][0], c->tb_mem[f][1], c->tb_mem[f][2]};
    if (tune_path) {
        // lines "<word_bits> <lg> <nlev> <lgr...>", and "single <word_bits> <lg> <nlev>
        // <lgr...>" for single-call plans; anything unparsable or unsupported is skipped
        if (FILE *f = fopen(tune_path, "r")) {
            char line[256];
            while (fgets(line, sizeof line, f)) {
                if (line[0] == '#') continue;
                const bool single = strncmp(line, "single ", 7) == 0;
                int wb, lg, nlev, r[4] = {0, 0, 0, 0};
                int k = sscanf(line + (single ? 7 : 0), "%d %d %d %d %d %d %d", &wb, &lg, &nlev, &r[0], &r[1], &r[2],
                               &r[3]);
                if (k >= 3 && k == 3 + std::max(nlev, 0)) {
                    if (single)
                        ext_tune_set_single(c, wb, lg, nlev, r);
                    else
                        ext_tune_set(c, wb, lg, nlev, r);
                }
            }
            fclose(f);
        }
    }
    *out = c;
    return EXT_OK;
}

void ext_destroy(ext_ctx *c) {
    if (!c) return;
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    for (auto &b : c->free_blocks) {
        if (b.used) hipEventDestroy(b.ev);
        hipFree(b.ptr);
    }
    for (auto &kv : c->graphs) graph_entry_free(kv.second);
    for (int f = 0; f < NFIELDS; ++f)
        for (int k = 0; k < 3; ++k)
            if (c->tb_mem[f][k]) hipFree(c->tb_mem[f][k]);
    for (auto p : c->pinned_status) hipHostFree(p);
    pinned_release_all(c);
    for (auto &kv : c->seeds) seed_free(kv.second);
    for (auto &mk : c->marks) {
        hipEventDestroy(mk.a);
        hipEventDestroy(mk.b);
    }
    delete c;
}

namespace {

int tune_set_in(ext_ctx *c, bool single, int word_bits, int lg, int nlev, const int *lgr) {
    if (!c || (word_bits != 32 && word_bits != 64) || lg < MIN_LG || lg > 32) return EXT_EINVAL;
    const int field = tune_field(word_bits, lg);
    if (field < 0) return EXT_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    std::map<int, Plan> &table = single ? c->tuned_single : c->tuned;
    if (nlev < 0) {
        table.erase(field * 64 + lg);
        return EXT_OK;
    }
    Plan p;
    p.field = field;
    p.lg = lg;
    p.small = nlev == 0;
    p.nlev = nlev;
    for (int i = 0; i < nlev && i < 4; ++i) {
        if (!lgr) return EXT_EINVAL;
        p.lgr[i] = lgr[i];
    }
    if (!valid_plan(p)) return EXT_EINVAL;
    table[field * 64 + lg] = p;
    return EXT_OK;
}

int tune_get_in(ext_ctx *c, bool single, int word_bits, int lg, int *nlev, int *lgr) {
    if (!c || (word_bits != 32 && word_bits != 64) || lg < MIN_LG || lg > 32) return EXT_EINVAL;
    const int field = tune_field(word_bits, lg);
    if (field < 0) return EXT_EINVAL;
    Plan p;
    {
        // a single call's plan: its own where there is one, else the batch plan
        std::lock_guard<std::mutex> g(c->mu);
        const int key = field * 64 + lg;
        auto its = c->tuned_single.find(key);
        auto itb = c->tuned.find(key);
        if (single && its != c->tuned_single.end())
            p = its->second;
        else if (itb != c->tuned.end())
            p = itb->second;
    }
    if (p.lg == 0) {
        const int rc = make_plan(uint64_t(1) << lg,
                                 field == FIELD_GL ? 2 : field == FIELD_P0 ? 3 : field == FIELD_LZ ? 5 : 1, p);
        if (rc != EXT_OK) return rc;
    }
    if (nlev) *nlev = p.small ? 0 : p.nlev;
    if (lgr)
        for (int i = 0; i < 4; ++i) lgr[i] = p.lgr[i];
    return EXT_OK;
}

}  // namespace

int ext_tune_set(ext_ctx *c, int word_bits, int lg, int nlev, const int *lgr) {
    return tune_set_in(c, false, word_bits, lg, nlev, lgr);
}
int ext_tune_get(ext_ctx *c, int word_bits, int lg, int *nlev, int *lgr) {
    return tune_get_in(c, false, word_bits, lg, nlev, lgr);
}
int ext_tune_set_single(ext_ctx *c, int word_bits, int lg, int nlev, const int *lgr) {
    return tune_set_in(c, true, word_bits, lg, nlev, lgr);
}
int ext_tune_get_single(ext_ctx *c, int word_bits, int lg, int *nlev, int *lgr) {
    return tune_get_in(c, true, word_bits, lg, nlev, lgr);
}

int ext_tune_save(ext_ctx *c, const char *path) {
    if (!c || !path) return EXT_EINVAL;
    FILE *f = fopen(path, "w");
    if (!f) return EXT_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    fprintf(f, "# word_bits lg nlev lgr...  (nlev 0: one workgroup per job)\n");
    fprintf(f, "# single word_bits lg nlev lgr...  (plans of single extraction calls where they differ)\n");
    for (int t = 0; t < 2; ++t)
        for (auto &kv : t ? c->tuned_single : c->tuned) {
            const Plan &p = kv.second;
            fprintf(f, "%s%d %d %d", t ? "single " : "", p.field == FIELD_GL ? 64 : 32, p.lg, p.small ? 0 : p.nlev);
            for (int i = 0; i < (p.small ? 0 : p.nlev); ++i) fprintf(f, " %d", p.lgr[i]);
            fprintf(f, "\n");
        }
    fclose(f);
    return EXT_OK;
}

int ext_seed_cache_clear(ext_ctx *c, size_t *bytes, size_t *entries) {
    if (!c) return EXT_EINVAL;
    std::unique_lock<std::mutex> g(c->mu);
    // new calls run without the cache until the clear is done; calls that hold an
    // entry (between its lookup and the event that marks their last read of it)
    // finish with it first
    ++c->seed_clearing;
    for (;;) {
        bool busy = false;
        for (auto &kv : c->seeds) busy |= kv.second.busy > 0;
        if (!busy) break;
        g.unlock();
        std::this_thread::yield();
        g.lock();
    }
    --c->seed_clearing;
    if (bytes) *bytes = c->seed_bytes;
    if (entries) *entries = c->seeds.size();
    for (auto &kv : c->seeds) seed_free(kv.second);
    c->reserved -= c->seed_bytes;
    c->seed_bytes = 0;
    c->seeds.clear();
    return EXT_OK;
}

int ext_mem_stats(ext_ctx *c, size_t *budget, size_t *in_use, size_t *reserved) {
    if (!c) return EXT_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (budget) *budget = c->budget;
    if (in_use) *in_use = c->leased;
    if (reserved) *reserved = c->reserved;
    return EXT_OK;
}

int ext_trim(ext_ctx *c) {
    if (!c) return EXT_EINVAL;
    hipSetDevice(c->device);
    std::lock_guard<std::mutex> g(c->mu);
    for (size_t i = 0; i < c->free_blocks.size();) {
        Block &b = c->free_blocks[i];
        if (!b.used || hipEventQuery(b.ev) == hipSuccess) {
            if (b.used) hipEventDestroy(b.ev);
            hipFree(b.ptr);
            c->reserved -= b.size;
            c->free_blocks.erase(c->free_blocks.begin() + i);
        } else {
            ++i;
        }
    }
    return EXT_OK;
}

int extract_toeplitz(ext_ctx *ctx, const uint64_t *x, uint64_t n, const uint64_t *y, uint64_t m, uint64_t *z,
                     uint32_t flags, int32_t *status, void *stream) {
    return extract_one(ctx, EXT_KIND_TOEPLITZ, x, n, y, m, z, flags, status, (hipStream_t)stream);
}

int extract_circulant(ext_ctx *ctx, const uint64_t *x, uint64_t n_in, const uint64_t *y, uint64_t m, uint64_t *z,
                      uint32_t flags, int32_t *status, void *stream) {
    if (flags & EXT_SEED_LINEAR) return EXT_EINVAL;
    return extract_one(ctx, EXT_KIND_CIRCULANT, x, n_in, y, m, z, flags, status, (hipStream_t)stream);
}

int extract_dodis(ext_ctx *ctx, const uint64_t *x, const uint64_t *y, uint64_t n, uint64_t m, uint64_t *z,
                  uint32_t flags, int32_t *status, void *stream) {
    if (flags & EXT_SEED_LINEAR) return EXT_EINVAL;
    return extract_one(ctx, EXT_KIND_DODIS, x, n, y, m, z, flags, status, (hipStream_t)stream);
}

int extract_toeplitz_noalloc(ext_ctx *c, const uint64_t *x, uint64_t n, const uint64_t *y, uint64_t m, uint64_t *z,
                             uint32_t flags, int32_t *status, void *stream) {
    if (!c || !c->scratch) return EXT_EINVAL;
    if (flags & ~(EXT_SEED_LINEAR | EXT_SYNC)) return EXT_EINVAL;
    Shape sh;
    int rc = shape_of(EXT_KIND_TOEPLITZ, n, m, sh);
    if (rc) return rc;
    if ((rc = validate(sh, x, y, z, flags)) != EXT_OK) return rc;
    Plan p;
    if ((rc = plan_for(c, sh.Lmin, p, true)) != EXT_OK) return rc;
    // the last 256 bytes of the scratch hold the status word of EXT_SYNC calls
    // without one of their own
    const size_t status_off = NOALLOC_SCRATCH_BYTES - 256;
    if (workspace_layout(p).total > status_off) return EXT_ESCRATCH;
    if (hipSetDevice(c->device) != hipSuccess) return EXT_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)c->scratch;
    int32_t *st = status;
    const bool own_status = (flags & EXT_SYNC) && !st;
    if (own_status) st = (int32_t *)(ws + status_off);
    JobDev jd = make_jobdev(sh, p, x, y, z, st, flags, p.small ? nullptr : ws);
    // every workspace region is written before it is read (embedded bits, both
    // arrays, the parity string), so nothing needs clearing; launches are not
    // traced (tracing creates events)
    if (enqueue(c, p, 1, nullptr, &jd, sh.m, false, s, /*quiet=*/true) != hipSuccess) return EXT_EDEVICE;
    if (!(flags & EXT_SYNC)) return EXT_OK;
    if (hipStreamSynchronize(s) != hipSuccess) return EXT_EDEVICE;
    int32_t v = 0;
    if (hipMemcpy(&v, st, sizeof(v), own_status ? hipMemcpyDeviceToHost : hipMemcpyDefault) != hipSuccess)
        return EXT_EDEVICE;
    return v;
}

int extract_von_neumann(ext_ctx *c, const uint64_t *x, uint64_t n, uint64_t *z, uint64_t z_words, uint64_t *m_out,
                        uint32_t flags, int32_t *status, void *stream) {
    if (!c || !x || !z || !m_out) return EXT_EINVAL;
    if (flags & ~EXT_SYNC) return EXT_EINVAL;
    if (n < 2) return EXT_EINVAL;
    if (n > EXT_VN_MAX_BITS) return EXT_ETOOLARGE;
    if (z_words < words(n / 2) || z_words > (uint64_t(1) << 58)) return EXT_EINVAL;
    const size_t zb = z_words * 8;
    if (overlaps(z, zb, x, words(n) * 8) || overlaps(z, zb, m_out, 8) || (status && overlaps(z, zb, status, 4)))
        return EXT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(c->device) != hipSuccess) return EXT_EDEVICE;
    Lease lease;
    int rc = pool_acquire(c, vn_workspace_bytes(n), s, lease);
    if (rc != EXT_OK) return rc;
    int32_t *st = status;
    int32_t *mine = nullptr;
    if ((flags & EXT_SYNC) && !st) {
        if (!(mine = take_pinned_status(c))) {
            pool_release(c, lease, s);
            return EXT_EDEVICE;
        }
        *mine = 0;
        st = mine;
    }
    const VnWork w = vn_work(lease.ptr, n);
    Tracer tr(c, s, false);
    tr.begin();
    hipError_t e = launch_vn_zero(w, n, s);
    tr.end("vn_zero");
    if (e == hipSuccess) {
        tr.begin();
        e = launch_vn_main(x, n, z, z_words, w, s);
        tr.end("vn_main");
    }
    if (e == hipSuccess) {
        tr.begin();
        e = launch_vn_fix(w, n, z, z_words, m_out, st, s);
        tr.end("vn_fix");
    }
    pool_release(c, lease, s);
    if (e != hipSuccess) {
        if (mine) give_pinned_status(c, mine);
        return EXT_EDEVICE;
    }
    rc = EXT_OK;
    if (flags & EXT_SYNC) {
        if (hipStreamSynchronize(s) != hipSuccess) rc = EXT_EDEVICE;
        else {
            int32_t v = 0;
            if (mine) v = *mine;
            else if (hipMemcpy(&v, st, sizeof(v), hipMemcpyDefault) != hipSuccess) v = EXT_EDEVICE;
            rc = v;
        }
        if (mine) give_pinned_status(c, mine);
    }
    return rc;
}

int extract_batch_unbatched(ext_ctx *ctx, ext_job *jobs, size_t count, uint32_t flags, void *stream) {
    if (!ctx || (!jobs && count)) return EXT_EINVAL;
    int first = EXT_OK;
    for (size_t i = 0; i < count; ++i) {
        ext_job &j = jobs[i];
        // the job checks of extract_batch (the seed order is a Toeplitz option)
        if ((j.flags & ~(EXT_SEED_LINEAR | EXT_SYNC | EXT_SINGLE_TRANSFORM)) ||
            (j.kind != EXT_KIND_TOEPLITZ && (j.flags & EXT_SEED_LINEAR)))
            j.err = EXT_EINVAL;
        else
            j.err = extract_one(ctx, j.kind, j.x, j.n, j.y, j.m, j.z, j.flags & (EXT_SEED_LINEAR | EXT_SINGLE_TRANSFORM),
                                j.status, (hipStream_t)stream);
        if (j.err && first == EXT_OK) first = j.err;
    }
    if ((flags & EXT_SYNC) && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return EXT_EDEVICE;
    return first;
}

int extract_batch(ext_ctx *ctx, ext_job *jobs, size_t count, uint32_t flags, void *stream);

int ext_profile(ext_ctx *c, int enable) {
    if (!c) return EXT_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    c->profile = enable != 0;
    return EXT_OK;
}

int ext_profile_read(ext_ctx *c, char *buf, size_t cap) {
    if (!c) return EXT_EINVAL;
    std::vector<ext_ctx::Mark> marks;
    {
        std::lock_guard<std::mutex> g(c->mu);
        marks.swap(c->marks);
    }
    std::string out;
    int n = 0;
    int rc = EXT_OK;
    for (auto &mk : marks) {
        float ms = 0.f;
        if (hipEventSynchronize(mk.b) != hipSuccess || hipEventElapsedTime(&ms, mk.a, mk.b) != hipSuccess) rc = EXT_EDEVICE;
        char line[160];
        snprintf(line, sizeof line, "%s %.6f\n", mk.label.c_str(), ms);
        out += line;
        hipEventDestroy(mk.a);
        hipEventDestroy(mk.b);
        ++n;
    }
    if (buf && cap) {
        size_t k = std::min(cap - 1, out.size());
        memcpy(buf, out.data(), k);
        buf[k] = 0;
    }
    return rc == EXT_OK ? n : rc;
}

}  // extern "C"

// ------------------------------------------------------------------ batching

namespace {

struct Member {
    size_t job;
    Shape shape;
    Plan plan;
};

// (a piece schedule's split is per job: it lives in the job's descriptors, so
// jobs of different splits share launches; the piece count does not)
std::string plan_key(const Plan &p) {
    char b[64];
    snprintf(b, sizeof b, "%d:%d:%d:%d.%d.%d.%d:%d", p.field, p.lg, p.small ? 1 : 0, p.lgr[0], p.lgr[1], p.lgr[2],
             p.lgr[3], p.pieces);
    return b;
}

// Launch layout of a batch: single-workgroup jobs first (sorted by size, one
// persistent launch), then chunks of one multi-pass size class each. A chunk's
// jobs get consecutive workspaces; chunks run one after another in stream
// order and share one workspace region, capped so that a chunk fits it. A chunk
// of a piece schedule (k pieces) has k descriptors per job: piece q of its
// jobs at first_desc + q n, in the jobs' order.
struct BatchLayout {
    std::vector<const Member *> order;
    SmallClasses cls{};
    size_t n_small = 0;
    size_t ndesc = 0;
    struct Chunk {
        Plan plan;
        size_t first_member, first_desc, n;
        uint64_t max_m;
        bool any_degen;
        size_t ws_each;
    };
    std::vector<Chunk> chunks;
    size_t max_ws = 0;
    std::string sig;
};

void layout_batch(ext_ctx *c, const std::vector<Member> &members, BatchLayout &bl) {
    std::vector<const Member *> small;
    std::map<std::string, std::vector<const Member *>> large;
    for (auto &mb : members) {
        if (mb.plan.small)
            small.push_back(&mb);
        else
            large[plan_key(mb.plan)].push_back(&mb);
    }
    std::stable_sort(small.begin(), small.end(),
                     [](const Member *a, const Member *b) { return a->plan.lg > b->plan.lg; });
    bl.n_small = small.size();
    uint32_t item = 0;
    for (size_t i = 0; i < small.size();) {
        const int lg = small[i]->plan.lg;
        size_t j = i;
        while (j < small.size() && small[j]->plan.lg == lg) ++j;
        const int k = bl.cls.n++;
        bl.cls.lg[k] = lg;
        bl.cls.first_job[k] = (uint32_t)i;
        bl.cls.njobs[k] = (uint32_t)(j - i);
        bl.cls.first_item[k] = item;
        const size_t jpw = size_t(1) << (14 - lg);
        item += (uint32_t)((j - i + jpw - 1) / jpw);
        char b[32];
        snprintf(b, sizeof b, "s%d#%zu|", lg, j - i);
        bl.sig += b;
        i = j;
    }
    bl.cls.total_items = item;
    bl.order = small;
    bl.ndesc = small.size();
    const size_t cap = std::max<size_t>(size_t(1) << 30, std::min<size_t>(c->budget / 4, size_t(16) << 30));
    for (auto &kv : large) {
        const Plan &p = kv.second.front()->plan;
        const size_t each = workspace_layout(p).total;
        size_t per_chunk = std::max<size_t>(1, cap / each);
        per_chunk = std::min<size_t>(per_chunk, 65535);
        for (size_t s0 = 0; s0 < kv.second.size(); s0 += per_chunk) {
            BatchLayout::Chunk ch;
            ch.plan = p;
            ch.first_member = bl.order.size();
            ch.first_desc = bl.ndesc;
            ch.n = std::min(per_chunk, kv.second.size() - s0);
            bl.ndesc += ch.n * (size_t)std::max(1, p.pieces);
            ch.max_m = 0;
            ch.any_degen = false;
            ch.ws_each = each;
            for (size_t k = 0; k < ch.n; ++k) {
                const Member *mb = kv.second[s0 + k];
                bl.order.push_back(mb);
                ch.max_m = std::max(ch.max_m, mb->shape.m);
                ch.any_degen |= mb->shape.kind == EXT_KIND_DODIS;
            }
            bl.max_ws = std::max(bl.max_ws, each * ch.n);
            bl.chunks.push_back(ch);
            char b[96];
            snprintf(b, sizeof b, "%s#%zu:%llu:%d|", kv.first.c_str(), ch.n, (unsigned long long)ch.max_m,
                     ch.any_degen ? 1 : 0);
            bl.sig += b;
        }
    }
}

void fill_descs(const BatchLayout &bl, const ext_job *jobs, char *ws, JobDev *out) {
    for (size_t i = 0; i < bl.n_small; ++i) {
        const Member &mb = *bl.order[i];
        const ext_job &j = jobs[mb.job];
        out[i] = make_jobdev(mb.shape, mb.plan, j.x, j.y, j.z, j.status, j.flags & EXT_SEED_LINEAR, nullptr);
    }
    for (auto &ch : bl.chunks)
        for (int q = 0; q < std::max(1, ch.plan.pieces); ++q)
            for (size_t k = 0; k < ch.n; ++k) {
                const Member &mb = *bl.order[ch.first_member + k];
                const ext_job &j = jobs[mb.job];
                out[ch.first_desc + (size_t)q * ch.n + k] = make_jobdev(
                    mb.shape, mb.plan, j.x, j.y, j.z, j.status, j.flags & EXT_SEED_LINEAR, ws + k * ch.ws_each, q);
            }
}

hipError_t enqueue_batch(ext_ctx *c, const BatchLayout &bl, JobDev *desc_dev, uint32_t *counter, hipStream_t s,
                         bool quiet) {
    hipError_t e = hipSuccess;
    if (bl.cls.total_items) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) cus = 256;
        const unsigned wgs = std::min<unsigned>(bl.cls.total_items, (unsigned)(2 * cus));
        Tracer tr(c, s, quiet);
        tr.begin();
        e = launch_small_batch(bl.cls, desc_dev, counter, wgs, c->tb[FIELD_LZ], s);
        tr.end("small_persist");
        if (e != hipSuccess) return e;
    }
    for (auto &ch : bl.chunks) {
        const int k = ch.plan.pieces;
        if (k >= 2) {
            // the last piece's product, each earlier piece's product plus the sum so
            // far, then the first piece fused with that sum, one inverse, parity
            for (int q = k - 1; q >= 1 && e == hipSuccess; --q)
                e = enqueue(c, ch.plan, (uint32_t)ch.n, desc_dev + ch.first_desc + (size_t)q * ch.n, nullptr, ch.max_m,
                            false, s, quiet, q == k - 1 ? PH_FWD_BOTH : PH_FWD_ACC);
            if (e == hipSuccess)
                e = enqueue(c, ch.plan, (uint32_t)ch.n, desc_dev + ch.first_desc, nullptr, ch.max_m, ch.any_degen, s,
                            quiet, PH_TWO);
        } else {
            e = enqueue(c, ch.plan, (uint32_t)ch.n, desc_dev + ch.first_desc, nullptr, ch.max_m, ch.any_degen, s,
                        quiet);
        }
        if (e != hipSuccess) return e;
    }
    return e;
}

// Pinned staging for descriptor uploads, recycled once the copy that read it is done.
struct Pinned {
    char *ptr;
    size_t size;
    hipEvent_t ev;
};

}  // namespace

struct ext_pinned_ring {
    std::vector<Pinned> items;
};

namespace {
std::mutex g_ring_mu;
std::map<ext_ctx *, ext_pinned_ring> g_rings;

char *pinned_take(ext_ctx *c, size_t bytes, Pinned &out) {
    std::lock_guard<std::mutex> g(g_ring_mu);
    auto &ring = g_rings[c].items;
    for (size_t i = 0; i < ring.size(); ++i) {
        if (ring[i].size >= bytes && hipEventQuery(ring[i].ev) == hipSuccess) {
            out = ring[i];
            ring.erase(ring.begin() + i);
            return out.ptr;
        }
    }
    out.size = std::max<size_t>(bytes, 4096);
    if (hipHostMalloc((void **)&out.ptr, out.size, hipHostMallocDefault) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&out.ev, hipEventDisableTiming) != hipSuccess) {
        hipHostFree(out.ptr);
        return nullptr;
    }
    return out.ptr;
}

void pinned_give(ext_ctx *c, Pinned &p, hipStream_t s) {
    hipEventRecord(p.ev, s);
    std::lock_guard<std::mutex> g(g_ring_mu);
    auto &ring = g_rings[c].items;
    ring.push_back(p);
    if (ring.size() > 64) {  // keep the ring bounded: drop the oldest idle buffer
        for (size_t i = 0; i < ring.size(); ++i)
            if (hipEventQuery(ring[i].ev) == hipSuccess) {
                hipEventDestroy(ring[i].ev);
                hipHostFree(ring[i].ptr);
                ring.erase(ring.begin() + i);
                break;
            }
    }
}

void pinned_release_all(ext_ctx *c) {
    std::lock_guard<std::mutex> g(g_ring_mu);
    auto it = g_rings.find(c);
    if (it == g_rings.end()) return;
    for (auto &p : it->second.items) {
        hipEventDestroy(p.ev);
        hipHostFree(p.ptr);
    }
    g_rings.erase(it);
}

constexpr size_t GRAPH_CACHE_MAX = 32;

}  // namespace

extern "C" int extract_batch(ext_ctx *c, ext_job *jobs, size_t count, uint32_t flags, void *stream_) {
    if (!c || (!jobs && count)) return EXT_EINVAL;
    if (flags & ~(EXT_SYNC | EXT_GRAPH)) return EXT_EINVAL;
    hipStream_t stream = (hipStream_t)stream_;
    if (hipSetDevice(c->device) != hipSuccess) return EXT_EDEVICE;
    int first = EXT_OK;
    std::vector<Member> members;
    members.reserve(count);
    for (size_t i = 0; i < count; ++i) {
        ext_job &j = jobs[i];
        Member mb;
        mb.job = i;
        int rc = shape_of(j.kind, j.n, j.m, mb.shape);
        if (rc == EXT_OK && (j.flags & ~(EXT_SEED_LINEAR | EXT_SYNC | EXT_SINGLE_TRANSFORM))) rc = EXT_EINVAL;
        if (rc == EXT_OK && j.kind != EXT_KIND_TOEPLITZ && (j.flags & EXT_SEED_LINEAR)) rc = EXT_EINVAL;
        if (rc == EXT_OK) rc = validate(mb.shape, j.x, j.y, j.z, j.flags & EXT_SEED_LINEAR);
        if (rc == EXT_OK) rc = plan_shape(c, mb.shape, mb.plan, j.flags, true);  // piece schedules included
        j.err = rc;
        if (rc != EXT_OK) {
            if (first == EXT_OK) first = rc;
            continue;
        }
        members.push_back(mb);
    }
    if (members.empty()) return first;
    BatchLayout bl;
    layout_batch(c, members, bl);
    const size_t ndesc = bl.ndesc;
    const size_t desc_bytes = align256(ndesc * sizeof(JobDev));
    hipError_t e = hipSuccess;
    if (flags & EXT_GRAPH) {
        std::lock_guard<std::mutex> graph_lock(c->graph_mu);
        Lease lease;
        int rc = pool_acquire(c, bl.max_ws, stream, lease);
        if (rc != EXT_OK) return rc;
        ext_ctx::GraphEntry *ge;
        {
            std::lock_guard<std::mutex> g(c->mu);
            if (c->graphs.size() >= GRAPH_CACHE_MAX && !c->graphs.count(bl.sig)) {
                // bounded cache: evict an entry whose last replay is done
                for (auto it = c->graphs.begin(); it != c->graphs.end(); ++it) {
                    if (graph_entry_idle(it->second)) {
                        graph_entry_free(it->second);
                        c->graphs.erase(it);
                        break;
                    }
                }
            }
            ge = &c->graphs[bl.sig];
        }
        if (!ge->desc_dev) {
            ge->ndesc = ndesc;
            bool ok = hipMalloc((void **)&ge->desc_dev, desc_bytes + 256) == hipSuccess &&
                      hipEventCreateWithFlags(&ge->replayed, hipEventDisableTiming) == hipSuccess;
            for (int k = 0; k < 2 && ok; ++k)
                ok = hipHostMalloc((void **)&ge->desc_host[k], desc_bytes, hipHostMallocDefault) == hipSuccess &&
                     hipEventCreateWithFlags(&ge->done[k], hipEventDisableTiming) == hipSuccess;
            if (!ok) {
                pool_release(c, lease, stream);
                return EXT_EDEVICE;
            }
        }
        uint32_t *counter = (uint32_t *)((char *)ge->desc_dev + desc_bytes);
        // this staging buffer may still be read by the copy of the replay before last
        const int k = ge->next;
        ge->next ^= 1;
        if (ge->used[k]) hipEventSynchronize(ge->done[k]);
        fill_descs(bl, jobs, lease.ptr, ge->desc_host[k]);
        if (ge->ever) e = hipStreamWaitEvent(stream, ge->replayed, 0);  // the last replay read desc_dev
        if (e == hipSuccess)
            e = hipMemcpyAsync(ge->desc_dev, ge->desc_host[k], ndesc * sizeof(JobDev), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipEventRecord(ge->done[k], stream);
        ge->used[k] = true;
        if (e == hipSuccess && !ge->exec) {
            // the launch sequence is recorded as the kernel nodes of a new graph
            // (no stream capture: other host threads stay unaffected)
            hipGraph_t graph = nullptr;
            e = hipGraphCreate(&graph, 0);
            if (e == hipSuccess) {
                GraphRecorder rec;
                rec.graph = graph;
                set_graph_recorder(&rec);
                e = enqueue_batch(c, bl, ge->desc_dev, counter, stream, true);
                set_graph_recorder(nullptr);
                if (e == hipSuccess) e = rec.err;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&ge->exec, graph, nullptr, nullptr, 0);
            if (graph) hipGraphDestroy(graph);
            if (e != hipSuccess) ge->exec = nullptr;
        }
        if (e == hipSuccess) e = hipGraphLaunch(ge->exec, stream);
        if (e == hipSuccess) e = hipEventRecord(ge->replayed, stream);
        ge->ever = true;
        pool_release(c, lease, stream);
    } else {
        // descriptors and the work counter live at the front of the leased workspace
        Lease lease;
        int rc = pool_acquire(c, desc_bytes + 256 + bl.max_ws, stream, lease);
        if (rc != EXT_OK) return rc;
        Pinned pin;
        JobDev *host = (JobDev *)pinned_take(c, ndesc * sizeof(JobDev), pin);
        if (!host) {
            pool_release(c, lease, stream);
            return EXT_EDEVICE;
        }
        JobDev *desc_dev = (JobDev *)lease.ptr;
        uint32_t *counter = (uint32_t *)(lease.ptr + desc_bytes);
        fill_descs(bl, jobs, lease.ptr + desc_bytes + 256, host);
        e = hipMemcpyAsync(desc_dev, host, ndesc * sizeof(JobDev), hipMemcpyHostToDevice, stream);
        pinned_give(c, pin, stream);
        if (e == hipSuccess) e = enqueue_batch(c, bl, desc_dev, counter, stream, false);
        pool_release(c, lease, stream);
    }
    if (e != hipSuccess) return EXT_EDEVICE;
    if ((flags & EXT_SYNC) && hipStreamSynchronize(stream) != hipSuccess) return EXT_EDEVICE;
    return first;
}
