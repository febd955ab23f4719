// Global de-duplication on one GPU (paper section 4.1), merged into a running
// set.
//
// The paper's three steps map onto one device as follows:
//   step 1 (local sort + regular sampling)  -> regular-stride samples of the
//          candidates, sorted in LDS (or by one workgroup over global memory
//          when there are more samples than fit), give splitters at equal
//          sample ranks;
//   step 2 (splitters + binary search)       -> every key finds its bucket by
//          binary search over the splitters held in LDS;
//   step 3 (all-to-all + local merge/unique) -> a histogram/scan/scatter pass
//          moves each key into its bucket's contiguous range; two such levels
//          leave buckets small enough for one LDS-local radix sort each,
//          followed by run-length unique.  Buckets cover disjoint, ascending
//          key ranges, so the concatenated unique runs are globally sorted and
//          equal keys can never straddle two buckets.
// The sorted unique run is then merged with the running set by merge path,
// keeping one copy of keys present in both and optionally emitting the keys
// that were not in the set ("novel").
//
// Sort vs. hash (paper section 4.1.2): no hash table and no global atomics on
// keys; the only atomics are LDS counters.  A bucket larger than the LDS
// capacity (skewed or heavily repeated keys) is sorted by its workgroup with
// the same radix ranking over global memory, so every size is handled.
#include <algorithm>

#include "sci_internal.hpp"

namespace sci {

constexpr int kDThreads = 256;
constexpr int kDWaves = kDThreads / kWave;

template <int W>
struct DCfg {
    static constexpr int CAP = (W == 1) ? 4096 : 2048;     // LDS sort capacity (keys)
    static constexpr int K = CAP / kDThreads;              // keys per thread
    static constexpr int CH = CAP / kDWaves;               // keys per wave
    static constexpr int TARGET = CAP / 2;                 // mean final bucket size
    static constexpr int F1 = 4096;                        // level-1 fan-out bound
    static constexpr int F2 = (W == 1) ? 512 : 256;        // level-2 fan-out bound
    static constexpr int OVS2 = CAP / F2;                  // level-2 oversampling (8)
    static constexpr int M1 = 65536;                       // level-1 sample bound
    static constexpr int64_t TILE1 = 131072;               // keys per level-1 tile
    static constexpr int64_t TILE2 = 16384;                // keys per level-2 tile
};

// ---------------------------------------------------------------------------
// small block-wide helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = threadIdx.x & (kWave - 1);
    return lane ? ((~0ull) >> (64 - lane)) : 0ull;
}

// exclusive scan of one int64 per thread across the block; returns the prefix, *total the sum
__device__ int64_t block_excl_scan_i64(int64_t v, int64_t *total, int64_t *s_wave /*[kDWaves]*/) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int64_t x = v;
    for (int o = 1; o < kWave; o <<= 1) {
        const int64_t u = __shfl_up(x, o);
        if (lane >= o) x += u;
    }
    __syncthreads();
    if (lane == kWave - 1) s_wave[w] = x;
    __syncthreads();
    int64_t pre = 0, tot = 0;
    for (int i = 0; i < kDWaves; ++i) {
        if (i < w) pre += s_wave[i];
        tot += s_wave[i];
    }
    *total = tot;
    return pre + x - v;
}

template <int W>
__device__ __forceinline__ uint32_t digit_of(const Key<W> &k, int shift) {
    return (uint32_t)(k.w[shift >> 6] >> (shift & 63)) & 0xffu;
}

// number of low bits in which keys may differ, given the OR of (key ^ key0)
template <int W>
__device__ __forceinline__ int varying_bits(const uint64_t *orx) {
    for (int j = W - 1; j >= 0; --j)
        if (orx[j]) return 64 * j + 64 - __clzll((long long)orx[j]);
    return 0;
}

// Rank 64 digits of one wave: *rank = position among same-digit lanes below,
// return = number of active lanes with the same digit.
__device__ __forceinline__ int wave_match_rank(uint32_t d, bool valid, int *rank) {
    const uint64_t act = __ballot(valid);
    uint64_t same = act;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(valid && bit);
        same &= bit ? bal : ~bal;
    }
    *rank = __popcll(same & lanemask_lt());
    return __popcll(same);
}

struct RadixLds {
    uint32_t cnt[kDWaves][256];
    int64_t wsum[kDWaves];
    uint64_t orx[2];
};

// Turn per-wave digit counts into output offsets: cnt[w][d] <- base(d) + sum_{w'<w} cnt[w'][d].
// Optionally also returns per-digit totals in dtot (nullable).
__device__ void radix_offsets(RadixLds &R, uint32_t *dtot) {
    const int t = threadIdx.x;  // one digit per thread (kDThreads == 256)
    uint32_t run = 0;
    for (int w = 0; w < kDWaves; ++w) {
        const uint32_t c = R.cnt[w][t];
        R.cnt[w][t] = run;
        run += c;
    }
    if (dtot) dtot[t] = run;
    int64_t total;
    const int64_t base = block_excl_scan_i64((int64_t)run, &total, R.wsum);
    for (int w = 0; w < kDWaves; ++w) R.cnt[w][t] += (uint32_t)base;
}

// Stable LSD radix sort (8-bit digits over bits [0, nbits)) of m <= CAP keys in LDS.
// Returns the buffer holding the result (buf or tmp).
template <int W>
__device__ Key<W> *lds_radix_sort(Key<W> *buf, Key<W> *tmp, int m, int nbits, RadixLds &R) {
    using C = DCfg<W>;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int shift = 0; shift < nbits; shift += 8) {
        for (int d = lane; d < 256; d += kWave) R.cnt[w][d] = 0;
        Key<W> kr[C::K];
        uint32_t meta[C::K];  // local rank | digit << 16
#pragma unroll
        for (int k = 0; k < C::K; ++k) {
            const int pos = w * C::CH + k * kWave + lane;
            const bool valid = pos < m;
            Key<W> key;
            if (valid) key = buf[pos];
            else {
#pragma unroll
                for (int j = 0; j < W; ++j) key.w[j] = 0;
            }
            const uint32_t d = valid ? digit_of<W>(key, shift) : 0u;
            int rk;
            const int tot = wave_match_rank(d, valid, &rk);
            uint32_t base = 0;
            if (valid) base = R.cnt[w][d];
            if (valid && rk == 0) R.cnt[w][d] = base + (uint32_t)tot;
            kr[k] = key;
            meta[k] = (base + (uint32_t)rk) | (d << 16);
        }
        __syncthreads();
        radix_offsets(R, nullptr);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < C::K; ++k) {
            const int pos = w * C::CH + k * kWave + lane;
            if (pos < m) {
                const uint32_t d = meta[k] >> 16;
                tmp[R.cnt[w][d] + (meta[k] & 0xffffu)] = kr[k];
            }
        }
        __syncthreads();
        Key<W> *sw = buf;
        buf = tmp;
        tmp = sw;
    }
    return buf;
}

// block-wide OR of (key ^ ref) over keys[0..m) read through `get`
template <int W, typename Get>
__device__ int block_varying_bits(int64_t m, const Key<W> &ref, Get get, RadixLds &R) {
    if (threadIdx.x == 0) R.orx[0] = R.orx[1] = 0;
    __syncthreads();
    uint64_t acc[W];
#pragma unroll
    for (int j = 0; j < W; ++j) acc[j] = 0;
    for (int64_t i = threadIdx.x; i < m; i += kDThreads) {
        const Key<W> k = get(i);
#pragma unroll
        for (int j = 0; j < W; ++j) acc[j] |= k.w[j] ^ ref.w[j];
    }
#pragma unroll
    for (int j = 0; j < W; ++j)
        if (acc[j]) atomicOr((unsigned long long *)&R.orx[j], (unsigned long long)acc[j]);
    __syncthreads();
    uint64_t o[W];
#pragma unroll
    for (int j = 0; j < W; ++j) o[j] = R.orx[j];
    __syncthreads();
    return varying_bits<W>(o);
}

// Stable LSD radix sort of m keys in global memory by one workgroup.
// X holds the input (may be const-casted only if never written: the first pass
// reads X and writes Y).  Returns 0 if the result is in X, 1 if in Y.
template <int W>
__device__ int global_radix_sort(const uint64_t *X0, uint64_t *X, uint64_t *Y, int64_t m, RadixLds &R,
                                 uint32_t *gbase /*[256] LDS*/, uint32_t *dtot /*[256] LDS*/) {
    using C = DCfg<W>;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const Key<W> ref = load_key<W>(X0, 0);
    const int nbits = block_varying_bits<W>(m, ref, [&](int64_t i) { return load_key<W>(X0, i); }, R);
    const uint64_t *src = X0;
    uint64_t *dst = Y;
    int where = 0;  // 0: data in X0/X, 1: data in Y
    for (int shift = 0; shift < nbits; shift += 8) {
        // sweep 1: digit totals
        gbase[threadIdx.x] = 0;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < m; i += kDThreads)
            atomicAdd(&gbase[digit_of<W>(load_key<W>(src, i), shift)], 1u);
        __syncthreads();
        {
            int64_t total;
            const uint32_t c = gbase[threadIdx.x];
            const int64_t ex = block_excl_scan_i64((int64_t)c, &total, R.wsum);
            __syncthreads();
            gbase[threadIdx.x] = (uint32_t)ex;
        }
        __syncthreads();
        // sweep 2: stable scatter tile by tile
        for (int64_t t0 = 0; t0 < m; t0 += C::CAP) {
            for (int d = lane; d < 256; d += kWave) R.cnt[w][d] = 0;
            Key<W> kr[C::K];
            uint32_t meta[C::K];
#pragma unroll
            for (int k = 0; k < C::K; ++k) {
                const int64_t pos = t0 + w * C::CH + k * kWave + lane;
                const bool valid = pos < m;
                Key<W> key;
                if (valid) key = load_key<W>(src, pos);
                else {
#pragma unroll
                    for (int j = 0; j < W; ++j) key.w[j] = 0;
                }
                const uint32_t d = valid ? digit_of<W>(key, shift) : 0u;
                int rk;
                const int tot = wave_match_rank(d, valid, &rk);
                uint32_t base = 0;
                if (valid) base = R.cnt[w][d];
                if (valid && rk == 0) R.cnt[w][d] = base + (uint32_t)tot;
                kr[k] = key;
                meta[k] = (base + (uint32_t)rk) | (d << 16);
            }
            __syncthreads();
            // within-tile offsets relative to each digit's running global base
            {
                const int t = threadIdx.x;
                uint32_t run = 0;
                for (int ww = 0; ww < kDWaves; ++ww) {
                    const uint32_t c = R.cnt[ww][t];
                    R.cnt[ww][t] = run + gbase[t];
                    run += c;
                }
                dtot[t] = run;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < C::K; ++k) {
                const int64_t pos = t0 + w * C::CH + k * kWave + lane;
                if (pos < m) {
                    const uint32_t d = meta[k] >> 16;
                    store_key<W>(dst, (int64_t)R.cnt[w][d] + (meta[k] & 0xffffu), kr[k]);
                }
            }
            __syncthreads();
            gbase[threadIdx.x] += dtot[threadIdx.x];
            __syncthreads();
        }
        // the data now lives in dst
        if (where == 0) {
            src = Y;
            dst = X;
            where = 1;
        } else {
            src = X;
            dst = Y;
            where = 0;
        }
        __threadfence();  // make this pass's stores visible (and drop stale L1 lines) before the next pass
        __syncthreads();
    }
    return where;
}

// ---------------------------------------------------------------------------
// level planning, sampling and splitters
// ---------------------------------------------------------------------------

struct LevelArgs {
    const uint64_t *in;      // keys of this level
    uint64_t *out;           // partitioned keys
    uint16_t *ids;           // bucket id per key
    const int64_t *seg_in;   // [S_in + 1]
    int64_t *seg_out;        // [S_in * F + 1]
    int S_in;
    int F;                   // fan-out bound of this level
    int64_t tile;            // keys per tile
    int target;              // mean bucket size aimed at
    int ovs;                 // samples per bucket
    int max_samples;
    int32_t *fan;            // [S_in] chosen fan-out
    uint64_t *spl;           // [S_in][F-1][W] splitters
    int64_t *tile_base;      // [S_in + 1]
    int64_t *cbase;          // [S_in + 1]
    int64_t *counts;         // [cbase[S_in]] per (segment, bucket, tile)
    int64_t max_tiles;       // grid bound
    uint64_t *sample_buf;    // level-1 only: [max_samples][W] + scratch of the same size
};

__device__ __forceinline__ int64_t seg_size(const int64_t *seg, int s) { return seg[s + 1] - seg[s]; }

// One workgroup per input segment: choose the fan-out, draw regular-stride
// samples, sort them, pick splitters at equal sample ranks.
template <int W>
__global__ __launch_bounds__(kDThreads) void splitter_kernel(LevelArgs a) {
    using C = DCfg<W>;
    __shared__ Key<W> s_buf[C::CAP];
    __shared__ Key<W> s_tmp[C::CAP];
    __shared__ RadixLds R;
    __shared__ uint32_t gbase[256], dtot[256];
    const int s = blockIdx.x;
    const int64_t start = a.seg_in[s], size = seg_size(a.seg_in, s);
    int f = (int)std::min<int64_t>((int64_t)a.F, std::max<int64_t>(1, ceil_div_dev(size, a.target)));
    if (size <= 0) f = 1;
    if (threadIdx.x == 0) a.fan[s] = f;
    if (f == 1) return;
    const int64_t M = std::min<int64_t>(size, std::min<int64_t>((int64_t)a.ovs * f, a.max_samples));
    uint64_t *sp = a.spl + (int64_t)s * (a.F - 1) * W;
    if (M <= C::CAP) {
        for (int64_t k = threadIdx.x; k < M; k += kDThreads) {
            const int64_t pos = start + (k * size + size / 2) / M;  // regular stride
            s_buf[k] = load_key<W>(a.in, pos);
        }
        __syncthreads();
        const Key<W> ref = s_buf[0];
        __syncthreads();
        const int nbits = block_varying_bits<W>(M, ref, [&](int64_t i) { return s_buf[i]; }, R);
        Key<W> *res = lds_radix_sort<W>(s_buf, s_tmp, (int)M, nbits, R);
        for (int j = threadIdx.x; j < f - 1; j += kDThreads) {
            const int64_t r = ((int64_t)(j + 1) * M) / f;
            store_key<W>(sp, j, res[r]);
        }
    } else {
        uint64_t *X = a.sample_buf, *Y = a.sample_buf + (int64_t)a.max_samples * W;
        for (int64_t k = threadIdx.x; k < M; k += kDThreads) {
            const int64_t pos = start + (k * size + size / 2) / M;
            store_key<W>(X, k, load_key<W>(a.in, pos));
        }
        __threadfence();
        __syncthreads();
        const int where = global_radix_sort<W>(X, X, Y, M, R, gbase, dtot);
        const uint64_t *res = where ? Y : X;
        for (int j = threadIdx.x; j < f - 1; j += kDThreads) {
            const int64_t r = ((int64_t)(j + 1) * M) / f;
            store_key<W>(sp, j, load_key<W>(res, r));
        }
    }
}

// Single workgroup: tiles and counter bases per segment (exclusive scans).
__global__ __launch_bounds__(kDThreads) void plan_kernel(LevelArgs a) {
    __shared__ int64_t wsum[kDWaves];
    int64_t tile_run = 0, c_run = 0;
    for (int s0 = 0; s0 < a.S_in; s0 += kDThreads) {
        const int s = s0 + threadIdx.x;
        int64_t t = 0, c = 0;
        if (s < a.S_in) {
            const int64_t size = seg_size(a.seg_in, s);
            t = size > 0 ? ceil_div_dev(size, a.tile) : 0;
            c = t * (int64_t)a.fan[s];
        }
        int64_t tt, ct;
        const int64_t te = block_excl_scan_i64(t, &tt, wsum);
        __syncthreads();
        const int64_t ce = block_excl_scan_i64(c, &ct, wsum);
        if (s < a.S_in) {
            a.tile_base[s] = tile_run + te;
            a.cbase[s] = c_run + ce;
        }
        tile_run += tt;
        c_run += ct;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.tile_base[a.S_in] = tile_run;
        a.cbase[a.S_in] = c_run;
    }
}

__device__ __forceinline__ int find_segment(const int64_t *base, int S, int64_t g) {
    // largest s with base[s] <= g (base is non-decreasing, base[0] = 0)
    int lo = 0, hi = S;  // answer in [0, S)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <int W>
__device__ __forceinline__ int bucket_of(const Key<W> &k, const Key<W> *spl, int nspl) {
    // number of splitters strictly below k (lower bound)
    int lo = 0, hi = nspl;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (key_less<W>(spl[mid], k)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Histogram pass: bucket id of every key (kept for the scatter pass) and the
// per-(segment, bucket, tile) counts.
template <int W, int FMAX>
__global__ __launch_bounds__(kDThreads) void hist_kernel(LevelArgs a) {
    __shared__ Key<W> s_spl[FMAX - 1];
    __shared__ uint32_t s_cnt[FMAX];
    const int64_t g = blockIdx.x;
    if (g >= a.tile_base[a.S_in]) return;
    const int s = find_segment(a.tile_base, a.S_in, g);
    const int64_t t = g - a.tile_base[s];
    const int64_t T = a.tile_base[s + 1] - a.tile_base[s];
    const int f = a.fan[s];
    const int64_t start = a.seg_in[s] + t * a.tile;
    const int64_t end = std::min<int64_t>(start + a.tile, a.seg_in[s + 1]);
    const uint64_t *sp = a.spl + (int64_t)s * (a.F - 1) * W;
    for (int j = threadIdx.x; j < f - 1; j += kDThreads) s_spl[j] = load_key<W>(sp, j);
    for (int j = threadIdx.x; j < f; j += kDThreads) s_cnt[j] = 0;
    __syncthreads();
    for (int64_t i = start + threadIdx.x; i < end; i += kDThreads) {
        const int b = (f > 1) ? bucket_of<W>(load_key<W>(a.in, i), s_spl, f - 1) : 0;
        a.ids[i] = (uint16_t)b;
        atomicAdd(&s_cnt[b], 1u);
    }
    __syncthreads();
    int64_t *cp = a.counts + a.cbase[s];
    for (int j = threadIdx.x; j < f; j += kDThreads) cp[(int64_t)j * T + t] = s_cnt[j];
}

// Scatter pass: each key to its bucket's range (order inside a bucket is free).
template <int W, int FMAX>
__global__ __launch_bounds__(kDThreads) void scatter_kernel(LevelArgs a) {
    __shared__ unsigned long long s_run[FMAX];
    const int64_t g = blockIdx.x;
    if (g >= a.tile_base[a.S_in]) return;
    const int s = find_segment(a.tile_base, a.S_in, g);
    const int64_t t = g - a.tile_base[s];
    const int64_t T = a.tile_base[s + 1] - a.tile_base[s];
    const int f = a.fan[s];
    const int64_t start = a.seg_in[s] + t * a.tile;
    const int64_t end = std::min<int64_t>(start + a.tile, a.seg_in[s + 1]);
    const int64_t *cp = a.counts + a.cbase[s];
    for (int j = threadIdx.x; j < f; j += kDThreads) s_run[j] = (unsigned long long)cp[(int64_t)j * T + t];
    __syncthreads();
    for (int64_t i = start + threadIdx.x; i < end; i += kDThreads) {
        const int b = a.ids[i];
        const unsigned long long pos = atomicAdd(&s_run[b], 1ull);
        store_key<W>(a.out, (int64_t)pos, load_key<W>(a.in, i));
    }
}

// Output segments of this level: slot (s, b) for b < F.
__global__ void next_segments_kernel(LevelArgs a, int64_t n_total) {
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n_slots = (int64_t)a.S_in * a.F;
    if (slot > n_slots) return;
    if (slot == n_slots) {
        a.seg_out[n_slots] = n_total;
        return;
    }
    const int s = (int)(slot / a.F), b = (int)(slot % a.F);
    const int64_t T = a.tile_base[s + 1] - a.tile_base[s];
    const int f = a.fan[s];
    int64_t v;
    if (T == 0) v = a.seg_in[s];
    else if (b < f) v = a.counts[a.cbase[s] + (int64_t)b * T];
    else v = a.seg_in[s + 1];
    a.seg_out[slot] = v;
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan of int64 (reduce, scan the block sums, apply)
// ---------------------------------------------------------------------------
constexpr int kScanPer = kDThreads * 16;

__global__ __launch_bounds__(kDThreads) void scan_reduce_kernel(const int64_t *x, const int64_t *n_dev, int64_t n_host,
                                                                int64_t *sums) {
    __shared__ int64_t wsum[kDWaves];
    const int64_t n = n_dev ? *n_dev : n_host;
    const int64_t base = (int64_t)blockIdx.x * kScanPer;
    int64_t v = 0;
    if (base < n) {
        for (int k = 0; k < 16; ++k) {
            const int64_t i = base + (int64_t)k * kDThreads + threadIdx.x;
            if (i < n) v += x[i];
        }
    }
    int64_t tot;
    block_excl_scan_i64(v, &tot, wsum);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kDThreads) void scan_sums_kernel(int64_t *sums, int64_t nb, int64_t *total_out) {
    __shared__ int64_t wsum[kDWaves];
    int64_t run = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kDThreads) {
        const int64_t b = b0 + threadIdx.x;
        const int64_t v = b < nb ? sums[b] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan_i64(v, &tot, wsum);
        if (b < nb) sums[b] = run + ex;
        run += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total_out) *total_out = run;
}

__global__ __launch_bounds__(kDThreads) void scan_apply_kernel(int64_t *x, const int64_t *n_dev, int64_t n_host,
                                                               const int64_t *sums) {
    __shared__ int64_t wsum[kDWaves];
    const int64_t n = n_dev ? *n_dev : n_host;
    const int64_t base = (int64_t)blockIdx.x * kScanPer;
    if (base >= n) return;
    // each thread owns 16 consecutive elements
    const int64_t mine = base + (int64_t)threadIdx.x * 16;
    int64_t v[16];
    int64_t loc = 0;
    for (int k = 0; k < 16; ++k) {
        const int64_t i = mine + k;
        v[k] = (i < n) ? x[i] : 0;
        loc += v[k];
    }
    int64_t tot;
    int64_t ex = block_excl_scan_i64(loc, &tot, wsum) + sums[blockIdx.x];
    for (int k = 0; k < 16; ++k) {
        const int64_t i = mine + k;
        if (i < n) x[i] = ex;
        ex += v[k];
    }
}

// ---------------------------------------------------------------------------
// final buckets: LDS radix sort + run-length unique
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kDThreads) void bucket_sort_unique_kernel(const uint64_t *src, uint64_t *dst,
                                                                       uint64_t *scratch, const int64_t *seg,
                                                                       int64_t *ucount) {
    using C = DCfg<W>;
    __shared__ Key<W> s_buf[C::CAP];
    __shared__ Key<W> s_tmp[C::CAP];
    __shared__ RadixLds R;
    __shared__ uint32_t gbase[256], dtot[256];
    const int64_t s = blockIdx.x;
    const int64_t start = seg[s], size = seg[s + 1] - seg[s];
    if (size <= 0) {
        if (threadIdx.x == 0) ucount[s] = 0;
        return;
    }
    int64_t nu_total = 0;
    if (size <= C::CAP) {
        const int m = (int)size;
        for (int i = threadIdx.x; i < m; i += kDThreads) s_buf[i] = load_key<W>(src, start + i);
        __syncthreads();
        const Key<W> ref = s_buf[0];
        const int nbits = block_varying_bits<W>(m, ref, [&](int64_t i) { return s_buf[i]; }, R);
        const Key<W> *res = lds_radix_sort<W>(s_buf, s_tmp, m, nbits, R);
        // run-length unique, in order: K consecutive keys per thread
        int64_t run = 0;
        for (int i0 = 0; i0 < m; i0 += kDThreads) {
            const int i = i0 + threadIdx.x;
            const bool keep = i < m && (i == 0 || !key_eq<W>(res[i], res[i - 1]));
            int64_t tot;
            const int64_t ex = block_excl_scan_i64(keep ? 1 : 0, &tot, R.wsum);
            if (keep) store_key<W>(dst, start + run + ex, res[i]);
            run += tot;
            __syncthreads();
        }
        nu_total = run;
    } else {
        // oversized bucket: radix sort over global memory (src range -> dst/src ping-pong)
        uint64_t *X = const_cast<uint64_t *>(src) + start * W;  // src is level output: writable
        uint64_t *Y = dst + start * W;
        const int where = global_radix_sort<W>(X, X, Y, size, R, gbase, dtot);
        const uint64_t *res = where ? Y : X;
        // unique into dst range (in place when res == Y: reads stay ahead of writes per tile)
        int64_t run = 0;
        for (int64_t i0 = 0; i0 < size; i0 += kDThreads) {
            const int64_t i = i0 + threadIdx.x;
            Key<W> cur, prev;
            bool keep = false;
            if (i < size) {
                cur = load_key<W>(res, i);
                keep = (i == 0);
                if (i > 0) {
                    prev = load_key<W>(res, i - 1);
                    keep = !key_eq<W>(cur, prev);
                }
            }
            __syncthreads();
            int64_t tot;
            const int64_t ex = block_excl_scan_i64(keep ? 1 : 0, &tot, R.wsum);
            if (keep) store_key<W>(dst, start + run + ex, cur);
            run += tot;
            __threadfence();
            __syncthreads();
        }
        nu_total = run;
        (void)scratch;
    }
    if (threadIdx.x == 0) ucount[s] = nu_total;
}

// copy each bucket's unique run to its place in the contiguous sorted run
template <int W>
__global__ __launch_bounds__(kDThreads) void compact_runs_kernel(const uint64_t *runs, const int64_t *seg,
                                                                 const int64_t *uoff, uint64_t *out) {
    const int64_t s = blockIdx.x;
    const int64_t start = seg[s];
    const int64_t n = uoff[s + 1] - uoff[s];
    const int64_t o = uoff[s];
    for (int64_t i = threadIdx.x; i < n; i += kDThreads) store_key<W>(out, o + i, load_key<W>(runs, start + i));
}

// ---------------------------------------------------------------------------
// merge path: run R (sorted unique) with set S (sorted unique)
// ---------------------------------------------------------------------------
constexpr int kMergeBlocks = 2048;
constexpr int kMergePer = 8;  // outputs per thread per round

struct MergeArgs {
    const uint64_t *A;      // run
    const int64_t *nA;
    const uint64_t *B;      // set_in (nullable when empty)
    const int64_t *nB;      // nullable: 0
    uint64_t *out;
    int64_t *n_out;
    int64_t out_cap;
    uint64_t *novel;        // nullable
    int64_t *n_novel;
    int64_t novel_cap;
    int64_t *blk;           // [2][kMergeBlocks] unique / novel counts, scanned in place
    uint32_t *flags;
};

template <int W>
__device__ __forceinline__ int64_t merge_path(const uint64_t *A, int64_t nA, const uint64_t *B, int64_t nB,
                                              int64_t k) {
    int64_t lo = k > nB ? k - nB : 0, hi = k < nA ? k : nA;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (key_less<W>(load_key<W>(A, mid), load_key<W>(B, k - mid - 1))) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// PASS 0: count unique / novel per block; PASS 1: write.
template <int W, int PASS>
__global__ __launch_bounds__(kDThreads) void merge_kernel(MergeArgs a) {
    __shared__ int64_t wsum[kDWaves];
    const int64_t nA = *a.nA, nB = a.nB ? *a.nB : 0;
    const int64_t total = nA + nB;
    const int64_t per = ceil_div_dev(total, (int64_t)kMergeBlocks);
    const int64_t b0 = (int64_t)blockIdx.x * per;
    const int64_t b1 = std::min<int64_t>(b0 + per, total);
    int64_t cu = 0, cn = 0;
    int64_t base_u = 0, base_n = 0;
    if (PASS == 1) {
        base_u = a.blk[blockIdx.x];
        base_n = a.blk[kMergeBlocks + blockIdx.x];
    }
    const int64_t step = (int64_t)kDThreads * kMergePer;
    for (int64_t c0 = b0; c0 < b1; c0 += step) {
        const int64_t p0 = c0 + (int64_t)threadIdx.x * kMergePer;
        const int64_t p1 = std::min<int64_t>(p0 + kMergePer, b1);
        int64_t i = 0, j = 0;
        uint32_t fa = 0, fd = 0;  // per output: from A, duplicate
        Key<W> vals[kMergePer];
        int cnt = 0;
        if (p0 < p1) {
            i = merge_path<W>(a.A, nA, a.B, nB, p0);
            j = p0 - i;
            for (int64_t p = p0; p < p1; ++p, ++cnt) {
                bool takeA;
                if (i >= nA) takeA = false;
                else if (j >= nB) takeA = true;
                else takeA = key_less<W>(load_key<W>(a.A, i), load_key<W>(a.B, j));
                if (takeA) {
                    const Key<W> x = load_key<W>(a.A, i);
                    const bool dup = (j > 0) && key_eq<W>(load_key<W>(a.B, j - 1), x);
                    vals[cnt] = x;
                    fa |= 1u << cnt;
                    if (dup) fd |= 1u << cnt;
                    ++i;
                } else {
                    vals[cnt] = load_key<W>(a.B, j);
                    ++j;
                }
            }
        }
        int lu = 0, ln = 0;
        for (int q = 0; q < cnt; ++q) {
            const bool dup = (fd >> q) & 1u, fromA = (fa >> q) & 1u;
            lu += !dup;
            ln += fromA && !dup;
        }
        int64_t tu, tn;
        const int64_t eu = block_excl_scan_i64(lu, &tu, wsum);
        __syncthreads();
        const int64_t en = block_excl_scan_i64(ln, &tn, wsum);
        __syncthreads();
        if (PASS == 1) {
            int64_t ou = base_u + cu + eu, on = base_n + cn + en;
            for (int q = 0; q < cnt; ++q) {
                const bool dup = (fd >> q) & 1u, fromA = (fa >> q) & 1u;
                if (dup) continue;
                if (ou < a.out_cap) store_key<W>(a.out, ou, vals[q]);
                ++ou;
                if (fromA && a.novel) {
                    if (on < a.novel_cap) store_key<W>(a.novel, on, vals[q]);
                    ++on;
                }
            }
        }
        cu += tu;
        cn += tn;
    }
    if (PASS == 0 && threadIdx.x == 0) {
        a.blk[blockIdx.x] = cu;
        a.blk[kMergeBlocks + blockIdx.x] = cn;
    }
}

__global__ __launch_bounds__(kDThreads) void merge_scan_kernel(MergeArgs a) {
    __shared__ int64_t wsum[kDWaves];
    for (int part = 0; part < 2; ++part) {
        int64_t *x = a.blk + part * kMergeBlocks;
        int64_t run = 0;
        for (int b0 = 0; b0 < kMergeBlocks; b0 += kDThreads) {
            const int b = b0 + threadIdx.x;
            const int64_t v = x[b];
            int64_t tot;
            const int64_t ex = block_excl_scan_i64(v, &tot, wsum);
            x[b] = run + ex;
            run += tot;
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (part == 0) {
                *a.n_out = run;
                if (run > a.out_cap) atomicOr(a.flags, SCI_FLAG_OVERFLOW);
            } else if (a.n_novel) {
                *a.n_novel = run;
                if (a.novel && run > a.novel_cap) atomicOr(a.flags, SCI_FLAG_OVERFLOW);
            }
        }
        __syncthreads();
    }
}

// checks that set_in is strictly ascending
template <int W>
__global__ void check_sorted_kernel(const uint64_t *S, const int64_t *nS, uint32_t *flags) {
    const int64_t n = *nS;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i + 1 < n; i += (int64_t)gridDim.x * blockDim.x)
        if (!key_less<W>(load_key<W>(S, i), load_key<W>(S, i + 1))) {
            atomicOr(flags, SCI_FLAG_UNSORTED);
            return;
        }
}

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------
struct WsLayout {
    size_t bufA, bufB, ids, segA, segB, fan, spl, tile_base, cbase, counts, sums, samples, ucount, blk, scal;
    size_t total;
    int64_t max_counts, max_sums, n_final_slots;
};

static size_t al256(size_t b) { return (b + 255) / 256 * 256; }

template <int W>
static WsLayout ws_layout(int64_t n) {
    using C = DCfg<W>;
    WsLayout L{};
    const int64_t nn = std::max<int64_t>(n, 1);
    const int64_t S1 = C::F1, S2 = (int64_t)C::F1 * C::F2;
    const int64_t tiles1 = ceil_div(nn, C::TILE1) + 1;
    const int64_t tiles2 = ceil_div(nn, C::TILE2) + S1;
    L.max_counts = std::max<int64_t>(tiles1 * C::F1, tiles2 * C::F2) + 1;
    L.n_final_slots = S2;
    L.max_sums = ceil_div(std::max<int64_t>(L.max_counts, S2 + 1), kScanPer) + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += al256(bytes);
        return o;
    };
    L.bufA = take((size_t)nn * W * 8);
    L.bufB = take((size_t)nn * W * 8);
    L.ids = take((size_t)nn * 2);
    L.segA = take((size_t)(S2 + 1) * 8);
    L.segB = take((size_t)(S2 + 1) * 8);
    L.fan = take((size_t)S1 * 4);
    L.spl = take((size_t)S1 * (C::F2 > C::F1 ? C::F2 : C::F1) * W * 8);
    L.tile_base = take((size_t)(S1 + 1) * 8);
    L.cbase = take((size_t)(S1 + 1) * 8);
    L.counts = take((size_t)std::max<int64_t>(L.max_counts, S2 + 1) * 8);
    L.sums = take((size_t)L.max_sums * 8);
    L.samples = take((size_t)C::M1 * 2 * W * 8);
    L.ucount = take((size_t)(S2 + 1) * 8);
    L.blk = take((size_t)2 * kMergeBlocks * 8);
    L.scal = take(64);
    L.total = off;
    return L;
}

static hipError_t device_scan(int64_t *x, const int64_t *n_dev, int64_t n_bound, int64_t *sums, int64_t *total_out,
                              hipStream_t st) {
    const int64_t nb = std::max<int64_t>(1, ceil_div(n_bound, kScanPer));
    SCI_LAUNCH(scan_reduce_kernel, dim3((unsigned)nb), dim3(kDThreads), 0, st, (const int64_t *)x, n_dev,
                       n_bound, sums);
    SCI_LAUNCH(scan_sums_kernel, dim3(1), dim3(kDThreads), 0, st, sums, nb, total_out);
    SCI_LAUNCH(scan_apply_kernel, dim3((unsigned)nb), dim3(kDThreads), 0, st, x, n_dev, n_bound,
                       (const int64_t *)sums);
    return hipGetLastError();
}

__global__ void init_level0_kernel(int64_t *seg, int64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        seg[0] = 0;
        seg[1] = n;
    }
}

template <int W>
static int32_t dedup_impl(const uint64_t *cand, int64_t n, const uint64_t *set_in, const int64_t *n_set_in,
                          uint64_t *set_out, int64_t *n_set_out, int64_t set_cap, uint64_t *novel,
                          int64_t *n_novel, int64_t novel_cap, char *ws, uint32_t *flags, hipStream_t st) {
    using C = DCfg<W>;
    const WsLayout L = ws_layout<W>(n);
    uint64_t *bufA = (uint64_t *)(ws + L.bufA);
    uint64_t *bufB = (uint64_t *)(ws + L.bufB);
    uint16_t *ids = (uint16_t *)(ws + L.ids);
    int64_t *segA = (int64_t *)(ws + L.segA);
    int64_t *segB = (int64_t *)(ws + L.segB);
    int64_t *counts = (int64_t *)(ws + L.counts);
    int64_t *sums = (int64_t *)(ws + L.sums);
    int64_t *ucount = (int64_t *)(ws + L.ucount);
    int64_t *scal = (int64_t *)(ws + L.scal);  // [0]: |run|, [1]: counts total
    int64_t *nrun = scal;

    const uint64_t *run = nullptr;  // sorted unique candidates
    if (n > 0) {
        const uint64_t *cur = cand;
        const int64_t *seg_cur = segA;
        int S_cur = 1;
        SCI_LAUNCH(init_level0_kernel, dim3(1), dim3(64), 0, st, segA, n);
        uint64_t *sort_src;
        const int64_t *final_seg;
        int64_t n_final;
        if (n <= C::CAP) {
            sort_src = const_cast<uint64_t *>(cand);  // read only: size <= CAP never writes src
            final_seg = segA;
            n_final = 1;
        } else {
            // level 1: one segment -> up to F1 buckets; level 2: each -> up to F2 buckets
            for (int lvl = 0; lvl < 2; ++lvl) {
                LevelArgs a{};
                a.in = cur;
                a.out = (lvl == 0) ? bufA : bufB;
                a.ids = ids;
                a.seg_in = seg_cur;
                a.seg_out = (lvl == 0) ? segB : segA;
                a.S_in = S_cur;
                a.F = (lvl == 0) ? C::F1 : C::F2;
                a.tile = (lvl == 0) ? C::TILE1 : C::TILE2;
                if (lvl == 0) {
                    // level-1 buckets sized so level 2 splits each into about F2/2 final buckets
                    a.target = (int)std::min<int64_t>((int64_t)C::TARGET * (C::F2 / 2), 1ll << 30);
                    a.ovs = 16;
                    a.max_samples = C::M1;
                } else {
                    a.target = C::TARGET;
                    a.ovs = C::OVS2;
                    a.max_samples = C::CAP;
                }
                a.fan = (int32_t *)(ws + L.fan);
                a.spl = (uint64_t *)(ws + L.spl);
                a.tile_base = (int64_t *)(ws + L.tile_base);
                a.cbase = (int64_t *)(ws + L.cbase);
                a.counts = counts;
                a.sample_buf = (uint64_t *)(ws + L.samples);
                const int64_t tiles_bound = ceil_div(n, a.tile) + S_cur;
                a.max_tiles = tiles_bound;
                SCI_LAUNCH(splitter_kernel<W>, dim3(S_cur), dim3(kDThreads), 0, st, a);
                SCI_LAUNCH(plan_kernel, dim3(1), dim3(kDThreads), 0, st, a);
                if (lvl == 0) {
                    SCI_LAUNCH((hist_kernel<W, C::F1>), dim3((unsigned)tiles_bound), dim3(kDThreads), 0, st, a);
                } else {
                    SCI_LAUNCH((hist_kernel<W, C::F2>), dim3((unsigned)tiles_bound), dim3(kDThreads), 0, st, a);
                }
                SCI_HIP_TRY(hipGetLastError());
                // exclusive scan of all counters -> absolute output offsets
                const int64_t cbound = tiles_bound * (int64_t)a.F;
                SCI_HIP_TRY(device_scan(counts, a.cbase + S_cur, cbound, sums, scal + 1, st));
                if (lvl == 0) {
                    SCI_LAUNCH((scatter_kernel<W, C::F1>), dim3((unsigned)tiles_bound), dim3(kDThreads), 0, st, a);
                } else {
                    SCI_LAUNCH((scatter_kernel<W, C::F2>), dim3((unsigned)tiles_bound), dim3(kDThreads), 0, st, a);
                }
                const int64_t slots = (int64_t)S_cur * a.F;
                SCI_LAUNCH(next_segments_kernel, dim3((unsigned)ceil_div(slots + 1, 256)), dim3(256), 0, st, a, n);
                SCI_HIP_TRY(hipGetLastError());
                cur = a.out;
                seg_cur = a.seg_out;
                S_cur = (int)slots;
            }
            sort_src = bufB;
            final_seg = segA;  // level-2 output segments
            n_final = S_cur;
        }
        // sorted unique runs per final bucket, written into bufA at the bucket offsets
        SCI_LAUNCH(bucket_sort_unique_kernel<W>, dim3((unsigned)n_final), dim3(kDThreads), 0, st,
                           (const uint64_t *)sort_src, bufA, bufB, final_seg, ucount);
        SCI_HIP_TRY(hipGetLastError());
        SCI_HIP_TRY(launch_set_i64(ucount + n_final, 0, st));
        SCI_HIP_TRY(device_scan(ucount, nullptr, n_final + 1, sums, nrun, st));
        uint64_t *dest = bufB;  // free once the buckets are sorted
        SCI_LAUNCH(compact_runs_kernel<W>, dim3((unsigned)n_final), dim3(kDThreads), 0, st,
                           (const uint64_t *)bufA, final_seg, (const int64_t *)ucount, dest);
        SCI_HIP_TRY(hipGetLastError());
        run = dest;
    } else {
        SCI_HIP_TRY(launch_set_i64(nrun, 0, st));
        run = (uint64_t *)(ws + L.bufA);
    }

    // merge the run into the set
    if (set_in && n_set_in)
        SCI_LAUNCH(check_sorted_kernel<W>, dim3(1024), dim3(256), 0, st, set_in, n_set_in, flags);
    MergeArgs m{};
    m.A = run;
    m.nA = nrun;
    m.B = set_in;
    m.nB = (set_in && n_set_in) ? n_set_in : nullptr;
    m.out = set_out;
    m.n_out = n_set_out;
    m.out_cap = set_cap;
    m.novel = novel;
    m.n_novel = n_novel;
    m.novel_cap = novel_cap;
    m.blk = (int64_t *)(ws + L.blk);
    m.flags = flags;
    SCI_LAUNCH((merge_kernel<W, 0>), dim3(kMergeBlocks), dim3(kDThreads), 0, st, m);
    SCI_LAUNCH(merge_scan_kernel, dim3(1), dim3(kDThreads), 0, st, m);
    SCI_LAUNCH((merge_kernel<W, 1>), dim3(kMergeBlocks), dim3(kDThreads), 0, st, m);
    SCI_HIP_TRY(hipGetLastError());
    return SCI_OK;
}

}  // namespace sci

using namespace sci;

extern "C" size_t sci_dedup_workspace_bytes(int32_t n_words, int64_t n_cand) {
    if (n_cand < 0) return 0;
    if (n_words == 1) return ws_layout<1>(n_cand).total;
    if (n_words == 2) return ws_layout<2>(n_cand).total;
    return 0;
}

extern "C" int32_t sci_dedup_merge(int32_t n_words, const uint64_t *cand, int64_t n_cand, const uint64_t *set_in,
                                   const int64_t *n_set_in, uint64_t *set_out, int64_t *n_set_out,
                                   int64_t set_capacity, uint64_t *novel, int64_t *n_novel, int64_t novel_capacity,
                                   void *workspace, size_t workspace_bytes, uint32_t *dev_flags,
                                   sci_stream_t stream) {
    set_error("");
    if (n_words < 1 || n_words > SCI_MAX_WORDS)
        return fail(n_words < 1 ? SCI_EINVAL : SCI_EUNSUPPORTED, "sci_dedup_merge: n_words=%d", n_words);
    if (n_cand < 0 || set_capacity < 0 || novel_capacity < 0)
        return fail(SCI_EINVAL, "sci_dedup_merge: negative size");
    if ((n_cand > 0 && !cand) || !set_out || !n_set_out || !dev_flags || !workspace)
        return fail(SCI_EINVAL, "sci_dedup_merge: NULL pointer argument");
    if (set_in && !n_set_in) return fail(SCI_EINVAL, "sci_dedup_merge: set_in without n_set_in");
    if (novel && !n_novel) return fail(SCI_EINVAL, "sci_dedup_merge: novel without n_novel");
    if (set_out == set_in || (const uint64_t *)set_out == cand)
        return fail(SCI_EINVAL, "sci_dedup_merge: set_out aliases an input");
    if (n_cand >= (1ll << 32))
        return fail(SCI_EUNSUPPORTED, "sci_dedup_merge: %lld candidates exceed one call", (long long)n_cand);
    const size_t need = sci_dedup_workspace_bytes(n_words, n_cand);
    if (workspace_bytes < need)
        return fail(SCI_ECAPACITY, "sci_dedup_merge: workspace %zu < %zu bytes", workspace_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    if (n_words == 1)
        return dedup_impl<1>(cand, n_cand, set_in, n_set_in, set_out, n_set_out, set_capacity, novel, n_novel,
                             novel_capacity, (char *)workspace, dev_flags, st);
    return dedup_impl<2>(cand, n_cand, set_in, n_set_in, set_out, n_set_out, set_capacity, novel, n_novel,
                         novel_capacity, (char *)workspace, dev_flags, st);
}
