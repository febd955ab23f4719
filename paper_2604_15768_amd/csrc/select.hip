// Reverse index and top-K selection (paper section 2.2: the reverse index from
// every coupled configuration to the unique set, and the selection of the
// candidates with the largest inferred amplitudes; section 4.3, stages 2-3).
//
// Reverse index.  The paper builds it by searching each original
// configuration in the unique set.  Two kinds of index give that answer (the
// position of the key in the sorted set, or -1):
//   hash   the unique set loaded into an open-addressing table in HBM (key ->
//          position, linear probing, load factor <= 1/2): a lookup costs about
//          one random sector read instead of ~log2|U| dependent reads; the table
//          takes 32-64 bytes per set key.
//   sorted the paper's search of the sorted set itself, for sets whose table
//          would not fit next to them: the index holds every 256th set key (1/256
//          of the set's bytes, small enough to stay in the last-level cache); a
//          lookup finds its 256-key block by searching a top level of those
//          samples held in LDS and then the samples, and searches the block.
//
// Top-K.  Entries are ranked by |psi| descending, equal magnitudes by key
// ascending.  Each entry's rank value is a composite of (64 + 64W) bits: the
// magnitude bits of psi (sign cleared), then the complemented key words, most
// significant first; larger composite = better rank, and composites are
// distinct when keys are.  An MSD radix select over 8-bit digits pins the K-th
// largest composite T (histogram of the surviving entries' next digit, pick
// the digit holding the K-th, keep only that digit's entries); every entry with
// composite >= T is selected, and a stable compaction writes them in input order.
#include <algorithm>

#include "sci_internal.hpp"

namespace sci {

constexpr int kSelThreads = 256;

// ---------------------------------------------------------------------------
// reverse index: hash table
// ---------------------------------------------------------------------------

// slot: key words, then position + 1 (0 = empty); W=1 16 bytes, W=2 32 bytes
template <int W>
struct SlotCfg {
    static constexpr int WORDS = (W == 1) ? 2 : 4;
    static constexpr int IDX = W;  // word holding position + 1
};

// header (int64 words): [0] hash slot count (power of two; 0 for the sorted kind),
// [1] W, [2] kind tag (kSortedTag for the sorted kind), sorted kind only: [3] set
// size, [4] set address, [5] sample stride, [6] sample count
constexpr size_t kIndexHeader = 256;
constexpr int64_t kSortedTag = 0x534F525445444958ll;  // "SORTEDIX"
constexpr int64_t kSortedStride = 256;                 // every 256th set key is a sample
constexpr int kTopLevel = 2048;                        // samples' top level held in LDS

// SplitMix64 output mixer (Steele, Lea, Flood, "Fast splittable pseudorandom
// number generators", 2014), applied to the folded key words.
template <int W>
__device__ __forceinline__ uint64_t slot_hash(const Key<W> &k) {
    uint64_t x = k.w[0];
    if (W == 2) x ^= (k.w[W - 1] << 32 | k.w[W - 1] >> 32) * 0xD6E8FEB86659FD93ull;
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBull;
    x ^= x >> 31;
    return x;
}

static int64_t index_slots(int64_t set_bound) {
    int64_t t = 64;
    while (t < 2 * set_bound) t <<= 1;
    return t;
}

__global__ void index_clear_kernel(uint64_t *tab, int64_t words, int64_t *hdr, int64_t T, int W) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) tab[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        hdr[0] = T;
        hdr[1] = W;
        hdr[2] = 0;
    }
}

template <int W>
__global__ void index_insert_kernel(const uint64_t *set, const int64_t *n_set, int64_t bound, uint64_t *tab,
                                    int64_t T, uint32_t *flags) {
    using S = SlotCfg<W>;
    const int64_t n_all = *n_set;
    if (n_all > bound && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flags, SCI_FLAG_OVERFLOW);
    const int64_t n = n_all < bound ? n_all : bound;
    const uint64_t mask = (uint64_t)T - 1;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const Key<W> k = load_key<W>(set, i);
        uint64_t h = slot_hash<W>(k) & mask;
        // the set's keys are distinct: claiming any empty slot is enough (T >= 2n, so one
        // exists and the walk ends within T probes)
        for (int64_t probe = 0; probe < T; ++probe) {
            uint64_t *slot = tab + h * S::WORDS;
            if (atomicCAS((unsigned long long *)(slot + S::IDX), 0ull, (unsigned long long)(i + 1)) == 0ull) {
#pragma unroll
                for (int j = 0; j < W; ++j) slot[j] = k.w[j];
                break;
            }
            h = (h + 1) & mask;
        }
    }
}

template <int W>
__device__ __forceinline__ void load_slot(const uint64_t *slot, Key<W> &k, uint64_t &idx1) {
    if (W == 1) {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(slot);
        k.w[0] = v.x;
        idx1 = v.y;
    } else {
        const ulonglong2 a = *reinterpret_cast<const ulonglong2 *>(slot);
        const ulonglong2 b = *reinterpret_cast<const ulonglong2 *>(slot + 2);
        k.w[0] = a.x;
        k.w[W - 1] = a.y;
        idx1 = b.x;
    }
}

// tmax: the most slots the caller's buffer can hold.  A header that is not one
// sci_index_build wrote for this W and size gives -1 everywhere.
template <int W>
__global__ void index_lookup_kernel(const uint64_t *tab, const int64_t *hdr, int64_t tmax, const uint64_t *cand,
                                    int64_t n, int64_t *idx) {
    using S = SlotCfg<W>;
    if (hdr[2] == kSortedTag) return;  // a sorted index: index_lookup_sorted_kernel answers
    int64_t T = hdr[0];
    if (T < 64 || (T & (T - 1)) != 0 || T > tmax || hdr[1] != W) T = 0;
    const uint64_t mask = (uint64_t)T - 1;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const Key<W> k = load_key<W>(cand, i);
        uint64_t h = slot_hash<W>(k) & mask;
        int64_t r = -1;
        // at least half the slots of a built table are empty, so the walk stops at one
        // long before the T-probe bound
        for (int64_t probe = 0; probe < T; ++probe) {
            Key<W> s;
            uint64_t id1;
            load_slot<W>(tab + h * S::WORDS, s, id1);
            if (id1 == 0) break;
            if (key_eq<W>(s, k)) {
                r = (int64_t)id1 - 1;
                break;
            }
            h = (h + 1) & mask;
        }
        idx[i] = r;
    }
}

// ---------------------------------------------------------------------------
// reverse index: search of the sorted set (samples of every kSortedStride-th key)
// ---------------------------------------------------------------------------

static int64_t sorted_samples(int64_t set_bound) { return ceil_div(std::max<int64_t>(set_bound, 0), kSortedStride); }

template <int W>
__global__ void index_sample_kernel(const uint64_t *set, const int64_t *n_set, int64_t bound, uint64_t *samples,
                                    int64_t *hdr, uint32_t *flags) {
    const int64_t n_all = *n_set;
    const int64_t n = n_all < bound ? n_all : bound;
    const int64_t m = ceil_div_dev(n, kSortedStride);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += stride)
        store_key<W>(samples, t, load_key<W>(set, t * kSortedStride));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (n_all > bound) atomicOr(flags, SCI_FLAG_OVERFLOW);
        hdr[0] = 0;
        hdr[1] = W;
        hdr[2] = kSortedTag;
        hdr[3] = n;
        hdr[4] = (int64_t)(uintptr_t)set;
        hdr[5] = kSortedStride;
        hdr[6] = m;
    }
}

// number of keys in a[lo, hi) that are <= k (a ascending), by binary search
template <int W>
__device__ __forceinline__ int64_t count_le(const uint64_t *a, int64_t lo, int64_t hi, const Key<W> &k) {
    const int64_t base = lo;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (key_less<W>(k, load_key<W>(a, mid))) hi = mid;
        else lo = mid + 1;
    }
    return lo - base;
}

// max_samples: the most samples the caller's buffer can hold.  A header that is not a
// sorted index for this W and buffer size gives -1 everywhere.
template <int W>
__global__ __launch_bounds__(256) void index_lookup_sorted_kernel(const int64_t *hdr, int64_t max_samples,
                                                                  const uint64_t *samples, const uint64_t *cand,
                                                                  int64_t n, int64_t *idx) {
    __shared__ Key<W> top[kTopLevel];
    if (hdr[2] != kSortedTag) return;  // a hash index: index_lookup_kernel answers
    const int64_t n_set = hdr[3], m = hdr[6];
    const uint64_t *set = (const uint64_t *)(uintptr_t)hdr[4];
    const bool valid = hdr[1] == W && hdr[5] == kSortedStride && m >= 0 && m <= max_samples && n_set >= 0 &&
                       m == ceil_div_dev(n_set, kSortedStride) && (n_set == 0 || set != nullptr);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (!valid || m == 0) {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) idx[i] = -1;
        return;
    }
    // top level: every R-th sample, at most kTopLevel of them
    const int64_t R = ceil_div_dev(m, kTopLevel);
    const int nt = (int)ceil_div_dev(m, R);
    for (int t = threadIdx.x; t < nt; t += blockDim.x) top[t] = load_key<W>(samples, (int64_t)t * R);
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const Key<W> k = load_key<W>(cand, i);
        // top entries <= k
        int lo = 0, hi = nt;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (key_less<W>(k, top[mid])) hi = mid;
            else lo = mid + 1;
        }
        int64_t r = -1;
        if (lo > 0) {  // else k is below the first set key
            // the last sample <= k lies in the top entry's block of R samples
            const int64_t s0 = (int64_t)(lo - 1) * R;
            const int64_t s1 = s0 + R < m ? s0 + R : m;
            const int64_t t = s0 + count_le<W>(samples, s0, s1, k) - 1;  // >= s0: samples[s0] <= k
            // and the key, if present, in that sample's block of set keys
            const int64_t b0 = t * kSortedStride;
            const int64_t b1 = b0 + kSortedStride < n_set ? b0 + kSortedStride : n_set;
            const int64_t c = count_le<W>(set, b0, b1, k);  // >= 1: set[b0] = samples[t] <= k
            if (key_eq<W>(load_key<W>(set, b0 + c - 1), k)) r = b0 + c - 1;
        }
        idx[i] = r;
    }
}

// ---------------------------------------------------------------------------
// top-K: radix select on the composite rank value
// ---------------------------------------------------------------------------

struct SelState {
    uint64_t prefix[3];  // pinned composite digits so far (word W = magnitude, words W-1..0 = ~key)
    int64_t k_rem;       // entries still to take among the survivors
    int64_t n_in;        // survivors the current pass reads
    int64_t n_surv;      // survivors the current pass writes
    int32_t digits;      // digits pinned
    int32_t done;        // threshold complete
    unsigned long long hist[256];
};

template <int W>
__device__ __forceinline__ void composite(const uint64_t *keys, const double *psi, int64_t i, uint64_t c[3]) {
    const Key<W> k = load_key<W>(keys, i);
    c[W] = (uint64_t)__double_as_longlong(psi[i]) & 0x7FFFFFFFFFFFFFFFull;
#pragma unroll
    for (int j = 0; j < W; ++j) c[j] = ~k.w[j];
}

// digit p (p = 0 most significant) of a composite of W+1 words
template <int W>
__device__ __forceinline__ uint32_t comp_digit(const uint64_t c[3], int p) {
    const int word = W - (p >> 3);
    const int shift = 8 * (7 - (p & 7));
    return (uint32_t)(c[word] >> shift) & 0xffu;
}

// composite's first p digits equal the pinned prefix
template <int W>
__device__ __forceinline__ bool prefix_match(const uint64_t c[3], const SelState &s, int p) {
    for (int q = W; q >= 0 && p > 0; --q) {
        const int take = p < 8 ? p : 8;
        const uint64_t m = take == 8 ? ~0ull : ~0ull << (64 - 8 * take);
        if ((c[q] & m) != (s.prefix[q] & m)) return false;
        p -= take;
    }
    return true;
}

// histogram of digit p over the survivors (all entries for p = 0)
template <int W>
__global__ __launch_bounds__(kSelThreads) void sel_hist_kernel(const uint64_t *keys, const double *psi, int64_t n,
                                                               const int64_t *surv, SelState *st, int p) {
    __shared__ uint32_t h[256];
    if (st->done) return;
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t m = p == 0 ? n : st->n_surv;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += stride) {
        const int64_t i = p == 0 ? t : surv[t];
        uint64_t c[3];
        composite<W>(keys, psi, i, c);
        atomicAdd(&h[comp_digit<W>(c, p)], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&st->hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// one thread: the digit holding the k_rem-th largest survivor
template <int W>
__global__ void sel_pick_kernel(SelState *st, int p) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || st->done) return;
    unsigned long long above = 0;
    int d = 255;
    for (; d > 0; --d) {
        if (above + st->hist[d] >= (unsigned long long)st->k_rem) break;
        above += st->hist[d];
    }
    const int64_t in_bin = (int64_t)st->hist[d];
    st->k_rem -= (int64_t)above;
    const int word = W - (p >> 3);
    st->prefix[word] |= (uint64_t)d << (8 * (7 - (p & 7)));
    st->digits = p + 1;
    st->n_in = st->n_surv;
    st->n_surv = 0;
    if (st->k_rem == in_bin || p + 1 == 8 * (W + 1)) st->done = 1;  // the whole bin is taken: threshold found
    for (int j = 0; j < 256; ++j) st->hist[j] = 0;
}

// survivors of digit p: entries whose first p+1 digits equal the new prefix
template <int W>
__global__ __launch_bounds__(kSelThreads) void sel_compact_kernel(const uint64_t *keys, const double *psi, int64_t n,
                                                                  const int64_t *surv_in, int64_t *surv_out,
                                                                  SelState *st, int p) {
    __shared__ long long s_base;
    __shared__ int s_cnt;
    if (st->done) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t m = p == 0 ? n : st->n_in;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < m; t0 += stride) {
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        const int64_t t = t0 + threadIdx.x;
        bool keep = false;
        int64_t i = 0;
        if (t < m) {
            i = p == 0 ? t : surv_in[t];
            uint64_t c[3];
            composite<W>(keys, psi, i, c);
            keep = prefix_match<W>(c, *st, p + 1);
        }
        const uint64_t bal = __ballot(keep);
        int wbase = 0;
        if (lane == 0 && bal) wbase = atomicAdd(&s_cnt, __popcll(bal));
        wbase = __shfl(wbase, 0);
        __syncthreads();
        if (threadIdx.x == 0 && s_cnt)
            s_base = (long long)atomicAdd((unsigned long long *)&st->n_surv, (unsigned long long)s_cnt);
        __syncthreads();
        if (keep) surv_out[s_base + wbase + __popcll(bal & lanemask_lt())] = i;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// final stable compaction of the entries with composite >= threshold
// ---------------------------------------------------------------------------

constexpr int kSelTile = kSelThreads * 8;

template <int W>
__device__ __forceinline__ bool selected(const uint64_t *keys, const double *psi, int64_t i, const SelState &s) {
    uint64_t c[3];
    composite<W>(keys, psi, i, c);
    // composite >= threshold: the threshold is the prefix followed by zero digits
    for (int q = W; q >= 0; --q) {
        if (c[q] != s.prefix[q]) return c[q] > s.prefix[q];
    }
    return true;
}

template <int W>
__global__ __launch_bounds__(kSelThreads) void sel_count_kernel(const uint64_t *keys, const double *psi, int64_t n,
                                                                const SelState *st, int64_t *counts) {
    __shared__ int s_c;
    if (threadIdx.x == 0) s_c = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSelTile;
    int c = 0;
    for (int u = 0; u < kSelTile / kSelThreads; ++u) {
        const int64_t i = base + u * kSelThreads + threadIdx.x;
        if (i < n && selected<W>(keys, psi, i, *st)) ++c;
    }
    if (c) atomicAdd(&s_c, c);
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = s_c;
}

template <int W>
__global__ __launch_bounds__(kSelThreads) void sel_write_kernel(const uint64_t *keys, const double *psi, int64_t n,
                                                                const SelState *st, const int64_t *offs,
                                                                uint64_t *out_keys, double *out_psi, int64_t cap) {
    __shared__ int s_w[kSelThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t base = (int64_t)blockIdx.x * kSelTile;
    int64_t run = offs[blockIdx.x];
    for (int u = 0; u < kSelTile / kSelThreads; ++u) {
        const int64_t i = base + u * kSelThreads + threadIdx.x;
        const bool keep = i < n && selected<W>(keys, psi, i, *st);
        const uint64_t bal = __ballot(keep);
        if (lane == 0) s_w[w] = __popcll(bal);
        __syncthreads();
        int before = 0, tot = 0;
        for (int q = 0; q < kSelThreads / kWave; ++q) {
            before += q < w ? s_w[q] : 0;
            tot += s_w[q];
        }
        if (keep) {
            const int64_t o = run + before + __popcll(bal & lanemask_lt());
            if (o < cap) {
                store_key<W>(out_keys, o, load_key<W>(keys, i));
                if (out_psi) out_psi[o] = psi[i];
            }
        }
        run += tot;
        __syncthreads();
    }
}

__global__ void sel_finish_kernel(const int64_t *total, int64_t cap, int64_t *n_out, uint32_t *flags) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *n_out = *total;
        if (*total > cap) atomicOr(flags, SCI_FLAG_OVERFLOW);
    }
}

__global__ void sel_init_kernel(SelState *st, int64_t k) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->prefix[0] = st->prefix[1] = st->prefix[2] = 0;
        st->k_rem = k;
        st->n_in = 0;
        st->n_surv = 0;
        st->digits = 0;
        st->done = 0;
    }
    for (int j = threadIdx.x; j < 256; j += blockDim.x) st->hist[j] = 0;
}

struct SelLayout {
    size_t state, survA, survB, counts, sums, scal, total;
};

static SelLayout sel_layout(int64_t n) {
    SelLayout L{};
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += (b + 255) / 256 * 256;
        return o;
    };
    const int64_t nn = n > 1 ? n : 1;
    const int64_t tiles = ceil_div(nn, kSelTile);
    L.state = take(sizeof(SelState));
    L.survA = take((size_t)nn * 8);
    L.survB = take((size_t)nn * 8);
    L.counts = take((size_t)(tiles + 1) * 8);
    L.sums = take((size_t)device_scan_sums(tiles + 1) * 8);
    L.scal = take(64);
    L.total = off;
    return L;
}

template <int W>
static int32_t topk_impl(const uint64_t *keys, const double *psi, int64_t n, int64_t k, uint64_t *out_keys,
                         double *out_psi, int64_t *n_out, int64_t cap, char *ws, uint32_t *flags, hipStream_t st) {
    const SelLayout L = sel_layout(n);
    SelState *S = (SelState *)(ws + L.state);
    int64_t *surv[2] = {(int64_t *)(ws + L.survA), (int64_t *)(ws + L.survB)};
    int64_t *counts = (int64_t *)(ws + L.counts);
    int64_t *scal = (int64_t *)(ws + L.scal);
    const int64_t kk = k < n ? k : n;
    if (kk == 0) return launch_set_i64(n_out, 0, st) == hipSuccess ? SCI_OK : fail(SCI_EHIP, "sci_topk: launch");
    SCI_LAUNCH(sel_init_kernel, dim3(1), dim3(256), 0, st, S, kk);
    const int P = 8 * (W + 1);
    const unsigned g0 = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, ceil_div(n, kSelThreads)));
    for (int p = 0; p < P; ++p) {
        SCI_LAUNCH((sel_hist_kernel<W>), dim3(p == 0 ? g0 : 1024), dim3(kSelThreads), 0, st, keys, psi, n,
                   (const int64_t *)surv[(p + 1) & 1], S, p);
        SCI_LAUNCH((sel_pick_kernel<W>), dim3(1), dim3(64), 0, st, S, p);
        // survivors of pass p feed pass p+1; the input list of pass p is surv[(p+1)&1]
        SCI_LAUNCH((sel_compact_kernel<W>), dim3(p == 0 ? g0 : 1024), dim3(kSelThreads), 0, st, keys, psi, n,
                   (const int64_t *)surv[(p + 1) & 1], surv[p & 1], S, p);
    }
    const int64_t tiles = ceil_div(n, kSelTile);
    SCI_LAUNCH((sel_count_kernel<W>), dim3((unsigned)tiles), dim3(kSelThreads), 0, st, keys, psi, n,
               (const SelState *)S, counts);
    SCI_HIP_TRY(launch_set_i64(counts + tiles, 0, st));
    SCI_HIP_TRY(device_scan(counts, nullptr, tiles + 1, (int64_t *)(ws + L.sums), scal, st));
    SCI_LAUNCH((sel_write_kernel<W>), dim3((unsigned)tiles), dim3(kSelThreads), 0, st, keys, psi, n,
               (const SelState *)S, (const int64_t *)counts, out_keys, out_psi, cap);
    SCI_LAUNCH(sel_finish_kernel, dim3(1), dim3(64), 0, st, (const int64_t *)scal, cap, n_out, flags);
    SCI_HIP_TRY(hipGetLastError());
    return SCI_OK;
}

}  // namespace sci

using namespace sci;

extern "C" size_t sci_index_bytes(int32_t n_words, int64_t set_bound) {
    if (n_words < 1 || n_words > SCI_MAX_WORDS || set_bound < 0) return 0;
    const int words = n_words == 1 ? SlotCfg<1>::WORDS : SlotCfg<2>::WORDS;
    return kIndexHeader + (size_t)index_slots(set_bound) * words * 8;
}

extern "C" size_t sci_index_bytes_sorted(int32_t n_words, int64_t set_bound) {
    if (n_words < 1 || n_words > SCI_MAX_WORDS || set_bound < 0) return 0;
    return kIndexHeader + (size_t)std::max<int64_t>(sorted_samples(set_bound), 1) * n_words * 8;
}

extern "C" int32_t sci_index_build(int32_t n_words, const uint64_t *set, const int64_t *n_set, int64_t set_bound,
                                   void *index, size_t index_bytes, uint32_t *dev_flags, sci_stream_t stream) {
    set_error("");
    if (n_words < 1 || n_words > SCI_MAX_WORDS)
        return fail(n_words < 1 ? SCI_EINVAL : SCI_EUNSUPPORTED, "sci_index_build: n_words=%d", n_words);
    if (set_bound < 0) return fail(SCI_EINVAL, "sci_index_build: negative set_bound");
    if (!n_set || !index || !dev_flags || (set_bound > 0 && !set))
        return fail(SCI_EINVAL, "sci_index_build: NULL pointer argument");
    const size_t need = sci_index_bytes(n_words, set_bound);
    const size_t need_sorted = sci_index_bytes_sorted(n_words, set_bound);
    if (index_bytes < need_sorted)
        return fail(SCI_ECAPACITY, "sci_index_build: index %zu < %zu bytes (sorted kind; %zu for a hash table)",
                    index_bytes, need_sorted, need);
    hipStream_t st = (hipStream_t)stream;
    if (index_bytes < need) {
        // room for the samples but not for a table: the sorted kind
        int64_t *hdr = (int64_t *)index;
        uint64_t *samples = (uint64_t *)((char *)index + kIndexHeader);
        const unsigned g = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, ceil_div(sorted_samples(set_bound), 256)));
        if (n_words == 1)
            SCI_LAUNCH(index_sample_kernel<1>, dim3(g), dim3(256), 0, st, set, n_set, set_bound, samples, hdr, dev_flags);
        else
            SCI_LAUNCH(index_sample_kernel<2>, dim3(g), dim3(256), 0, st, set, n_set, set_bound, samples, hdr, dev_flags);
        SCI_HIP_TRY(hipGetLastError());
        return SCI_OK;
    }
    const int64_t T = index_slots(set_bound);
    const int words = n_words == 1 ? SlotCfg<1>::WORDS : SlotCfg<2>::WORDS;
    int64_t *hdr = (int64_t *)index;
    uint64_t *tab = (uint64_t *)((char *)index + kIndexHeader);
    SCI_LAUNCH(index_clear_kernel, dim3(4096), dim3(256), 0, st, tab, T * words, hdr, T, (int)n_words);
    if (n_words == 1)
        SCI_LAUNCH(index_insert_kernel<1>, dim3(4096), dim3(256), 0, st, set, n_set, set_bound, tab, T, dev_flags);
    else
        SCI_LAUNCH(index_insert_kernel<2>, dim3(4096), dim3(256), 0, st, set, n_set, set_bound, tab, T, dev_flags);
    SCI_HIP_TRY(hipGetLastError());
    return SCI_OK;
}

extern "C" int32_t sci_index_lookup(int32_t n_words, const void *index, size_t index_bytes, const uint64_t *cand,
                                    int64_t n_cand, int64_t *idx, sci_stream_t stream) {
    set_error("");
    if (n_words < 1 || n_words > SCI_MAX_WORDS)
        return fail(n_words < 1 ? SCI_EINVAL : SCI_EUNSUPPORTED, "sci_index_lookup: n_words=%d", n_words);
    if (n_cand < 0) return fail(SCI_EINVAL, "sci_index_lookup: negative n_cand");
    if (!index || (n_cand > 0 && (!cand || !idx))) return fail(SCI_EINVAL, "sci_index_lookup: NULL pointer argument");
    if (index_bytes < sci_index_bytes_sorted(n_words, 0))
        return fail(SCI_ECAPACITY, "sci_index_lookup: index buffer of %zu bytes holds no index", index_bytes);
    if (n_cand == 0) return SCI_OK;
    hipStream_t st = (hipStream_t)stream;
    const int64_t *hdr = (const int64_t *)index;
    const uint64_t *tab = (const uint64_t *)((const char *)index + kIndexHeader);
    const int words = n_words == 1 ? SlotCfg<1>::WORDS : SlotCfg<2>::WORDS;
    // the most hash slots / samples the buffer holds (what a valid header can claim)
    int64_t tmax = 0;
    if (index_bytes >= sci_index_bytes(n_words, 0)) {
        tmax = 64;
        while (kIndexHeader + (size_t)(2 * tmax) * words * 8 <= index_bytes) tmax <<= 1;
    }
    const int64_t smax = (int64_t)((index_bytes - kIndexHeader) / ((size_t)n_words * 8));
    // the index kind is in the device header: both kernels are enqueued and the one that
    // does not match it returns at once
    const unsigned g = (unsigned)std::min<int64_t>(1 << 16, ceil_div(n_cand, 256));
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    // the sorted kernel loads its top level once per workgroup: a small persistent grid
    const unsigned gs = (unsigned)std::min<int64_t>((int64_t)std::max(n_cu, 1) * 8, ceil_div(n_cand, 256));
    if (n_words == 1) {
        SCI_LAUNCH(index_lookup_kernel<1>, dim3(g), dim3(256), 0, st, tab, hdr, tmax, cand, n_cand, idx);
        SCI_LAUNCH(index_lookup_sorted_kernel<1>, dim3(gs), dim3(256), 0, st, hdr, smax, tab, cand, n_cand, idx);
    } else {
        SCI_LAUNCH(index_lookup_kernel<2>, dim3(g), dim3(256), 0, st, tab, hdr, tmax, cand, n_cand, idx);
        SCI_LAUNCH(index_lookup_sorted_kernel<2>, dim3(gs), dim3(256), 0, st, hdr, smax, tab, cand, n_cand, idx);
    }
    SCI_HIP_TRY(hipGetLastError());
    return SCI_OK;
}

extern "C" size_t sci_topk_workspace_bytes(int64_t n) {
    if (n < 0) return 0;
    return sel_layout(n).total;
}

extern "C" int32_t sci_topk(int32_t n_words, const uint64_t *keys, const double *psi, int64_t n, int64_t k,
                            uint64_t *out_keys, double *out_psi, int64_t *n_out, int64_t capacity, void *workspace,
                            size_t workspace_bytes, uint32_t *dev_flags, sci_stream_t stream) {
    set_error("");
    if (n_words < 1 || n_words > SCI_MAX_WORDS)
        return fail(n_words < 1 ? SCI_EINVAL : SCI_EUNSUPPORTED, "sci_topk: n_words=%d", n_words);
    if (n < 0 || k < 0 || capacity < 0) return fail(SCI_EINVAL, "sci_topk: negative size");
    if (!n_out || !dev_flags || !workspace || (n > 0 && (!keys || !psi)) || (k > 0 && n > 0 && !out_keys))
        return fail(SCI_EINVAL, "sci_topk: NULL pointer argument");
    const int64_t kk = k < n ? k : n;
    if (capacity < kk) return fail(SCI_ECAPACITY, "sci_topk: capacity %lld < %lld", (long long)capacity, (long long)kk);
    if (workspace_bytes < sel_layout(n).total)
        return fail(SCI_ECAPACITY, "sci_topk: workspace %zu < %zu bytes", workspace_bytes, sel_layout(n).total);
    hipStream_t st = (hipStream_t)stream;
    if (n_words == 1)
        return topk_impl<1>(keys, psi, n, k, out_keys, out_psi, n_out, capacity, (char *)workspace, dev_flags, st);
    return topk_impl<2>(keys, psi, n, k, out_keys, out_psi, n_out, capacity, (char *)workspace, dev_flags, st);
}
