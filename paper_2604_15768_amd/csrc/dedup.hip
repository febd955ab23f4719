// Global de-duplication on one GPU (paper section 4.1), merged into a running
// set.
//
// The paper's three steps map onto one device as follows:
//   step 1 (local sort + regular sampling)  -> one sample per equal stratum of
//          the candidates (hashed offset inside the stratum), sorted in LDS (more
//          samples than fit: runs sorted by separate workgroups, then each sample
//          ranked in their merged order), gives splitters at equal sample ranks;
//   step 2 (splitters + binary search)       -> every key finds its bucket by
//          binary search over the splitters held in LDS;
//   step 3 (all-to-all + local merge/unique) -> a histogram/scan/scatter pass
//          moves each key into its bucket's contiguous range; two such levels
//          leave buckets small enough for one LDS-local radix sort each,
//          followed by run-length unique.  Buckets cover disjoint, ascending
//          key ranges, so the concatenated unique runs are globally sorted and
//          equal keys can never straddle two buckets.
// Each unique run then drops the keys the running set already holds in its
// range (found while the run is in LDS), and what is left ("novel", optionally
// emitted) is inserted among the set keys: every set key moves by the number of
// run keys below it, so the merge reads the run and the set range once.
//
// Sort vs. hash (paper section 4.1.2): no hash table and no global atomics on
// keys; the only atomics are LDS counters.  A bucket larger than the LDS
// capacity (heavily repeated keys) streams through LDS against one hash table
// when its distinct keys fit, else is sorted by its workgroup with the same
// radix ranking over global memory, so every size is handled.
#include <algorithm>

#include "sci_internal.hpp"

namespace sci {

constexpr int kDThreads = 256;
constexpr int kDWaves = kDThreads / kWave;

template <int W>
struct DCfg {
    static constexpr int CAP = (W == 1) ? 3072 : 1536;     // LDS sort capacity (keys)
    static constexpr int K = CAP / kDThreads;              // keys per thread
    static constexpr int CH = CAP / kDWaves;               // keys per wave
    // mean final bucket size (tail past CAP is rare); two-word keys get fewer level-2
    // samples per bucket, a wider spread, so their mean stays further below CAP
    static constexpr int TARGET = (W == 1) ? CAP * 3 / 8 : CAP / 4;
    static constexpr int F1 = 4096;                        // level-1 fan-out bound
    // level-2 fan-out bound: 1,024 for two-word keys, whose streamed pool chunks of 2^31
    // candidates then keep final buckets of about 512 keys
    static constexpr int F2 = (W == 1) ? 512 : 1024;
    // level-2 splitters: one workgroup per level-1 bucket sorts its samples in LDS, up
    // to SCAP at once (the whole of a CU's LDS for two-word keys); two-word keys sort
    // two such runs (MS2 samples in all), 8 per final bucket against 12 for one word
    static constexpr int SCAP = (W == 1) ? 6144 : 4096;
    static constexpr int MS2 = (W == 1) ? SCAP : 2 * SCAP;  // level-2 sample bound
    static constexpr int OVS2 = MS2 / F2;                  // 12 W=1, 8 W=2
    static constexpr int M1 = 65536;                       // level-1 sample bound
    static constexpr int64_t TILE1 = 131072;               // keys per level-1 tile
    static constexpr int64_t TILE2 = 16384;                // keys per level-2 tile
};

// ---------------------------------------------------------------------------
// small block-wide helpers
// ---------------------------------------------------------------------------

// exclusive scan of one int64 per thread across the block; returns the prefix, *total the sum
template <int NW = kDWaves>
__device__ int64_t block_excl_scan_i64(int64_t v, int64_t *total, int64_t *s_wave /*[NW]*/) {
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
    for (int i = 0; i < NW; ++i) {
        if (i < w) pre += s_wave[i];
        tot += s_wave[i];
    }
    *total = tot;
    return pre + x - v;
}

template <int W>
__device__ __forceinline__ uint32_t digit_of(const Key<W> &k, int shift) {
    // the 8 bits from `shift` up, which may straddle two words; words are selected
    // with static indices (a runtime index would put the key in scratch)
    const int q = shift >> 6, r = shift & 63;
    uint64_t lo = k.w[0], hi = 0;
#pragma unroll
    for (int j = 1; j < W; ++j) {
        if (q == j) lo = k.w[j];
        if (q + 1 == j) hi = k.w[j];
    }
    uint64_t v = lo >> r;
    if (r > 56) v |= hi << (64 - r);
    return (uint32_t)v & 0xffu;
}

// number of low bits in which keys may differ, given the OR of (key ^ key0)
template <int W>
__device__ __forceinline__ int varying_bits(const uint64_t *orx) {
    for (int j = W - 1; j >= 0; --j)
        if (orx[j]) return 64 * j + 64 - __clzll((long long)orx[j]);
    return 0;
}

// position of the lowest bit that varies (0 when none does)
template <int W>
__device__ __forceinline__ int lowest_varying_bit(const uint64_t *orx) {
    for (int j = 0; j < W; ++j)
        if (orx[j]) return 64 * j + __ffsll((unsigned long long)orx[j]) - 1;
    return 0;
}

// Rank one digit per lane within the wave among the lanes holding the same digit.
// Only the digit bits in `vmask` can differ (the others agree across the whole
// unit), so only those are balloted; the loop over them is wave-uniform.  Invalid
// lanes carry digit 0 and are left out of `same` from the start.
__device__ __forceinline__ int wave_match_rank_bits(uint32_t d, bool valid, uint32_t vmask, int *rank) {
    uint64_t same = __ballot(valid);
    for (uint32_t m = vmask; m; m &= m - 1u) {
        const int b = __builtin_ctz(m);
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
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

// Stable LSD radix sort (8-bit digits over bits [0, nbits)) of m <= MAXM keys in LDS.
// Returns the buffer holding the result (buf or tmp).
template <int W, int MAXM = DCfg<W>::CAP>
__device__ Key<W> *lds_radix_sort(Key<W> *buf, Key<W> *tmp, int m, int nbits, const Key<W> &orkey, RadixLds &R) {
    constexpr int kK = MAXM / kDThreads;   // keys per thread
    constexpr int kCH = MAXM / kDWaves;    // keys per wave
    static_assert(MAXM % kDThreads == 0 && MAXM < 65536, "radix sort capacity");
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int shift = 0; shift < nbits; shift += 8) {
        const uint32_t vm = digit_of<W>(orkey, shift);  // bits of this window that vary
        if (vm == 0u) continue;                         // an identity pass

        for (int d = lane; d < 256; d += kWave) R.cnt[w][d] = 0;
        Key<W> kr[kK];
        uint32_t meta[kK];  // local rank | digit << 16
#pragma unroll
        for (int k = 0; k < kK; ++k) {
            const int pos = w * kCH + k * kWave + lane;
            const bool valid = pos < m;
            Key<W> key;
            if (valid) key = buf[pos];
            else {
#pragma unroll
                for (int j = 0; j < W; ++j) key.w[j] = 0;
            }
            const uint32_t d = valid ? digit_of<W>(key, shift) : 0u;
            int rk;
            const int tot = wave_match_rank_bits(d, valid, vm, &rk);
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
        for (int k = 0; k < kK; ++k) {
            const int pos = w * kCH + k * kWave + lane;
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
__device__ int block_varying_bits(int64_t m, const Key<W> &ref, Get get, RadixLds &R, Key<W> *orkey) {
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
    for (int j = 0; j < W; ++j) orkey->w[j] = o[j] = R.orx[j];
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
    Key<W> orkey;
    const int nbits = block_varying_bits<W>(m, ref, [&](int64_t i) { return load_key<W>(X0, i); }, R, &orkey);
    const uint64_t *src = X0;
    uint64_t *dst = Y;
    int where = 0;  // 0: data in X0/X, 1: data in Y
    for (int shift = 0; shift < nbits; shift += 8) {
        const uint32_t vm = digit_of<W>(orkey, shift);  // bits of this window that vary
        if (vm == 0u) continue;                         // an identity pass
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
                const int tot = wave_match_rank_bits(d, valid, vm, &rk);
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
    uint64_t *sample_buf;    // level-1 only: [max_samples][W] sorted sample runs
};

__device__ __forceinline__ int64_t seg_size(const int64_t *seg, int s) { return seg[s + 1] - seg[s]; }

// Position of sample k of M from the segment [start, start + size): one sample in
// each of M equal strata, at a hashed offset inside it (SplitMix64 finaliser of k).
// A fixed offset would make the sample stride a fixed number of keys, and the
// generated candidates are laid out with periods (excitations per source, blocks
// of single excitations) that such a stride can keep hitting at the same phase:
// whole classes of keys then go unsampled and their buckets grow far past the
// target.  Hashed offsets keep the stratification and break that resonance.
__device__ __forceinline__ int64_t sample_pos(int64_t start, int64_t size, int64_t k, int64_t M) {
    uint64_t x = (uint64_t)k + 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    const int64_t r = (int64_t)__umul64hi(x, (uint64_t)size);  // uniform in [0, size)
    return start + (k * size + r) / M;                         // in stratum k
}

// One workgroup per input segment: choose the fan-out, draw one sample per
// stratum, sort them, pick splitters at equal sample ranks.  Above one LDS load
// of samples (two-word keys at level 2), the first half of the strata is sorted
// and set aside while the second half is sorted, then loaded beside it; the
// sample of merged rank r is found by a merge-path search over the two runs,
// which gives the keys one sort of all samples would give.
template <int W>
__global__ __launch_bounds__(kDThreads) void splitter_kernel(LevelArgs a) {
    using C = DCfg<W>;
    __shared__ Key<W> s_buf[C::SCAP];
    __shared__ Key<W> s_tmp[C::SCAP];
    __shared__ RadixLds R;
    const int s = blockIdx.x;
    const int64_t start = a.seg_in[s], size = seg_size(a.seg_in, s);
    int f = (int)std::min<int64_t>((int64_t)a.F, std::max<int64_t>(1, ceil_div_dev(size, a.target)));
    if (size <= 0) f = 1;
    if (threadIdx.x == 0) a.fan[s] = f;
    if (f == 1) return;
    const int64_t M = std::min<int64_t>(size, std::min<int64_t>((int64_t)a.ovs * f, a.max_samples));
    if (M > 2 * C::SCAP) return;  // cannot happen: the host sorts larger samples in runs
    uint64_t *sp = a.spl + (int64_t)s * (a.F - 1) * W;
    // one run, or two of M/2 and M - M/2 samples; the first of two waits in this
    // segment's part of the level's output (at least M keys, written only by the
    // scatter pass that follows) while the second is sorted
    const int n_runs = M > C::SCAP ? 2 : 1;
    const int nA = n_runs == 2 ? (int)(M / 2) : 0, nB = (int)(M - nA);
    uint64_t *stage = a.out + start * W;
    const Key<W> *B = nullptr;
    for (int run = 0; run < n_runs; ++run) {
        const int k0 = run == n_runs - 1 ? nA : 0, m = run == n_runs - 1 ? nB : nA;
        for (int k = threadIdx.x; k < m; k += kDThreads)
            s_buf[k] = load_key<W>(a.in, sample_pos(start, size, k0 + k, M));
        __syncthreads();
        const Key<W> ref = s_buf[0];
        __syncthreads();
        Key<W> orkey;
        const int nbits = block_varying_bits<W>(m, ref, [&](int64_t i) { return s_buf[i]; }, R, &orkey);
        B = lds_radix_sort<W, C::SCAP>(s_buf, s_tmp, m, nbits, orkey, R);
        if (run < n_runs - 1) {
            for (int i = threadIdx.x; i < m; i += kDThreads) store_key<W>(stage, i, B[i]);
            __syncthreads();  // both LDS buffers are reused by the next run
        }
    }
    Key<W> *A = (B == s_buf) ? s_tmp : s_buf;
    for (int i = threadIdx.x; i < nA; i += kDThreads) A[i] = load_key<W>(stage, i);
    __syncthreads();
    for (int j = threadIdx.x; j < f - 1; j += kDThreads) {
        const int r = (int)(((int64_t)(j + 1) * M) / f);  // 0 < r < M
        // i = keys of A among the first r of the merge (equal keys: A first); with one
        // run A is empty and the pick is B[r]
        int lo = r > nB ? r - nB : 0, hi = r < nA ? r : nA;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (!key_less<W>(B[r - mid - 1], A[mid])) lo = mid + 1;
            else hi = mid;
        }
        const int i = lo, jb = r - lo;
        const bool takeA = i < nA && (jb >= nB || !key_less<W>(B[jb], A[i]));
        store_key<W>(sp, j, takeA ? A[i] : B[jb]);
    }
}

// Splitters of one segment from more samples than one LDS sort holds (level 1).
// Workgroup g sorts samples [g CAP, (g+1) CAP) in LDS and stores the sorted run
// (section 4.1 step 1, local sort); sample_rank_kernel then places every sample in
// the merged order of all runs, and those at splitter ranks are the splitters
// (step 2).  They are the keys one sort of all samples would give.
template <int W>
__global__ __launch_bounds__(kDThreads) void sample_runs_kernel(LevelArgs a, int64_t n, int64_t M, int f) {
    using C = DCfg<W>;
    __shared__ Key<W> s_buf[C::CAP];
    __shared__ Key<W> s_tmp[C::CAP];
    __shared__ RadixLds R;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.fan[0] = f;
    const int64_t k0 = (int64_t)blockIdx.x * C::CAP;
    const int m = (int)std::min<int64_t>(C::CAP, M - k0);
    for (int k = threadIdx.x; k < m; k += kDThreads) s_buf[k] = load_key<W>(a.in, sample_pos(0, n, k0 + k, M));
    __syncthreads();
    const Key<W> ref = s_buf[0];
    __syncthreads();
    Key<W> orkey;
    const int nbits = block_varying_bits<W>(m, ref, [&](int64_t i) { return s_buf[i]; }, R, &orkey);
    Key<W> *res = lds_radix_sort<W>(s_buf, s_tmp, m, nbits, orkey, R);
    for (int k = threadIdx.x; k < m; k += kDThreads) store_key<W>(a.sample_buf, k0 + k, res[k]);
}

// One thread per sample: its rank in the stable merge of the sorted runs (keys of
// earlier runs first among equals) is its index in its own run plus, in every other
// run, the keys that come before it.  Ranks are distinct, so each splitter rank
// (j+1) M / f has exactly one writer.
template <int W>
__global__ __launch_bounds__(kDThreads) void sample_rank_kernel(LevelArgs a, int64_t M, int f) {
    using C = DCfg<W>;
    const int64_t k = (int64_t)blockIdx.x * kDThreads + threadIdx.x;
    if (k >= M) return;
    const int n_runs = (int)ceil_div_dev(M, C::CAP);
    const int g = (int)(k / C::CAP);
    const Key<W> x = load_key<W>(a.sample_buf, k);
    int64_t rank = k - (int64_t)g * C::CAP;
    for (int h = 0; h < n_runs; ++h) {
        if (h == g) continue;
        const int64_t b0 = (int64_t)h * C::CAP;
        int lo = 0, len = (int)std::min<int64_t>(C::CAP, M - b0);
        while (len > 0) {
            const int half = len >> 1;
            const Key<W> y = load_key<W>(a.sample_buf, b0 + lo + half);
            // before x: keys below it, and in earlier runs also keys equal to it
            const bool before = (h < g) ? !key_less<W>(x, y) : key_less<W>(y, x);
            if (before) {
                lo += half + 1;
                len -= half + 1;
            } else {
                len = half;
            }
        }
        rank += lo;
    }
    // M >= f, so at most one splitter index c has floor((c+1) M / f) == rank
    const int64_t j = (rank * f) / M;
    for (int64_t c = j - 1; c <= j; ++c) {
        if (c >= 0 && c < f - 1 && ((c + 1) * M) / f == rank) store_key<W>(a.spl, c, x);
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

// Lanes of one wave whose values in `b` are equal and adjacent form runs (keys in
// generation order often share a bucket).  Returns the run's length at its first
// lane (0 elsewhere) and that lane's index in *head.  Valid lanes form a prefix.
__device__ __forceinline__ int wave_run(int b, bool valid, int *head) {
    const int lane = threadIdx.x & (kWave - 1);
    const int prev = __shfl_up(b, 1);
    const bool is_head = valid && (lane == 0 || prev != b);
    const uint64_t heads = __ballot(is_head);
    const int nvalid = __popcll(__ballot(valid));
    const uint64_t upto = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull);
    *head = 63 - __clzll((long long)(heads & upto));
    if (!is_head) return 0;
    const uint64_t later = heads & ~upto;
    const int next = later ? __ffsll((long long)later) - 1 : nvalid;
    return next - lane;
}

// Histogram pass: bucket id of every key (kept for the scatter pass) and the
// per-(segment, bucket, tile) counts.
// 1,024-thread workgroups: the LDS of a tile (its splitters and counters) serves four
// times the waves of a 256-thread one, which hide the latency of the conflicting
// splitter reads (level 1: 10.6 -> 9.7 ms on the medium workload).
constexpr int kHThreads = 1024;

template <int W, int FMAX>
__global__ __launch_bounds__(kHThreads) void hist_kernel(LevelArgs a) {
    constexpr int kH = kHThreads;
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
    constexpr int kSteps = __builtin_ctz(FMAX);
    // Splitters padded to FMAX-1 with the all-ones key, which no key is above, form a
    // perfect binary search tree stored level by level (node j at s_spl[j-1], children
    // 2j and 2j+1): sorted splitter i sits at depth d = kSteps-1-ctz(i+1), position
    // (i+1) >> (ctz(i+1)+1) in that level.  The lanes of a wave then read one
    // contiguous level per step instead of entries a power of two apart (which fall
    // into the same LDS bank), and every search takes exactly log2(FMAX) steps.
    // Two-word keys: when every splitter of the segment has the same top word X (most
    // level-2 segments: a level-1 bucket inside one top word), the tree holds only the
    // low words, half the LDS reads per step; keys with another top word have every
    // splitter above them (top word below X) or below them (above X).
    bool one_top = false;
    uint64_t X = 0;
    if constexpr (W == 2) {
        if (f > 2) {
            X = sp[1];
            one_top = sp[(int64_t)(f - 2) * W + 1] == X;
        }
    }
    uint64_t *s_low = reinterpret_cast<uint64_t *>(s_spl);  // [FMAX - 1] when one_top
    for (int i = threadIdx.x; i < FMAX - 1; i += kH) {
        const int z = __builtin_ctz((unsigned)(i + 1));
        const int j = (1 << (kSteps - 1 - z)) + ((i + 1) >> (z + 1));
        if (one_top) {
            s_low[j - 1] = i < f - 1 ? sp[(int64_t)i * W] : ~0ull;
        } else if (i < f - 1) {
            s_spl[j - 1] = load_key<W>(sp, i);
        } else {
#pragma unroll
            for (int q = 0; q < W; ++q) s_spl[j - 1].w[q] = ~0ull;
        }
    }
    for (int j = threadIdx.x; j < f; j += kH) s_cnt[j] = 0;
    __syncthreads();
    for (int64_t i0 = start; i0 < end; i0 += 4 * kH) {
        Key<W> k[4];
        int pos[4];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + u * kH + threadIdx.x;
            ok[u] = i < end;
            if (ok[u]) k[u] = load_key<W>(a.in, i);
            else {
#pragma unroll
                for (int j = 0; j < W; ++j) k[u].w[j] = 0;
            }
            pos[u] = 0;
        }
        // branch-free descent: going right at a node means the node is below the key,
        // so the leaf reached, less FMAX, is the number of splitters below the key
#pragma unroll
        for (int u = 0; u < 4; ++u) pos[u] = 1;
        if (one_top) {  // workgroup-uniform
#pragma unroll
            for (int st = 0; st < kSteps; ++st) {
#pragma unroll
                for (int u = 0; u < 4; ++u) pos[u] = 2 * pos[u] + (s_low[pos[u] - 1] < k[u].w[0] ? 1 : 0);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                pos[u] -= FMAX;
                if (k[u].w[W - 1] != X) pos[u] = k[u].w[W - 1] < X ? 0 : f - 1;
            }
        } else {
#pragma unroll
            for (int st = 0; st < kSteps; ++st) {
#pragma unroll
                for (int u = 0; u < 4; ++u) pos[u] = 2 * pos[u] + (key_less<W>(s_spl[pos[u] - 1], k[u]) ? 1 : 0);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) pos[u] -= FMAX;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + u * kH + threadIdx.x;
            int head;
            const int len = wave_run(pos[u], ok[u], &head);
            if (!ok[u]) continue;
            a.ids[i] = (uint16_t)pos[u];
            if (len) atomicAdd(&s_cnt[pos[u]], (uint32_t)len);
        }
    }
    __syncthreads();
    int64_t *cp = a.counts + a.cbase[s];
    for (int j = threadIdx.x; j < f; j += kH) cp[(int64_t)j * T + t] = s_cnt[j];
}

// Scatter pass: each key to its bucket's range (order inside a bucket is free).
// The scatter pass runs one 1,024-thread workgroup per CU: the open output runs
// stay one per bucket per workgroup while twice as many loads are in flight as with
// 512 threads (level-2 scatter 16.4 -> 15.3 ms on the medium workload), and one
// workgroup per CU rather than two halves the partial lines held open in L2
// (both levels together 31-34 -> 28.4 ms).
constexpr int kSThreads = 1024;

template <int W, int FMAX>
__global__ __launch_bounds__(kSThreads) void scatter_kernel(LevelArgs a) {
    constexpr int kT = kSThreads;
    // each bucket's output cursor for this tile: positions are below n < 2^32 (the entry
    // point refuses larger inputs), so 32 bits hold them and the LDS stays small
    __shared__ uint32_t s_cur[FMAX];
    // a small persistent grid walks the tiles: every workgroup keeps one open output
    // run per bucket, and fewer runs in flight at once merge better in the caches.
    // A bucket's runs of consecutive tiles are adjacent in the output and share their
    // boundary lines, so each round of gridDim tiles is dealt out XCD by XCD: those
    // lines are then written through one L2 instead of two.
    const int64_t n_tiles = a.tile_base[a.S_in];
    for (int64_t g = xcd_local_block(blockIdx.x, gridDim.x); g < n_tiles; g += gridDim.x) {
        __syncthreads();  // the previous tile's cursors are no longer read
        const int s = find_segment(a.tile_base, a.S_in, g);
        const int64_t t = g - a.tile_base[s];
        const int64_t T = a.tile_base[s + 1] - a.tile_base[s];
        const int f = a.fan[s];
        const int64_t start = a.seg_in[s] + t * a.tile;
        const int64_t end = std::min<int64_t>(start + a.tile, a.seg_in[s + 1]);
        const int64_t *cp = a.counts + a.cbase[s];
        for (int j = threadIdx.x; j < f; j += kT) s_cur[j] = (uint32_t)cp[(int64_t)j * T + t];
        __syncthreads();
        // sixteen keys per thread in flight: with one workgroup per CU the loads, not
        // the stores, set the pace (levels 1+2: 31.0 -> 27.3 ms against eight)
        constexpr int U = 16;
        for (int64_t i0 = start; i0 < end; i0 += (int64_t)U * kT) {
            Key<W> k[U];
            int b[U];
    #pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = i0 + u * kT + threadIdx.x;
                b[u] = -1;
                if (i < end) {
                    b[u] = a.ids[i];
                    k[u] = load_key<W>(a.in, i);
                }
            }
    #pragma unroll
            for (int u = 0; u < U; ++u) {
                if (b[u] >= 0) {
                    const uint32_t pos = atomicAdd(&s_cur[b[u]], 1u);
                    store_key<W>(a.out, (int64_t)pos, k[u]);
                }
            }
        }
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
// final buckets: LDS radix sort + run-length unique, and the union counts
// against the running set's keys that fall in each bucket's key range
// ---------------------------------------------------------------------------

struct BucketArgs {
    const uint64_t *src;      // partitioned candidates (writable workspace unless single bucket)
    uint64_t *dst;            // each unit's sorted unique keys absent from the set, at the unit's offset
    const int64_t *seg;       // [n_slots + 1] final bucket offsets
    int64_t n_slots;          // bound on the number of units
    const int32_t *ufirst;    // [n_units] first slot of each unit (consecutive buckets of one level-1 bucket)
    const int32_t *uend;      // [n_units] one past its last slot
    const int64_t *n_units;   // device count
    int two_level;            // 0: one bucket covering every key
    const int32_t *fan1;      // [1] level-1 fan-out
    const uint64_t *spl1;     // [F1-1][W]
    const int32_t *fan2;      // [F1] level-2 fan-out per level-1 bucket
    const uint64_t *spl2;     // [F1][F2-1][W]
    int F2;
    const uint64_t *B;        // running set (nullable)
    const int64_t *nB;        // nullable
    int64_t *nuniq;           // [n_units] unique candidates per unit that the set does not hold
    int64_t *bstart;          // [n_units] first set element in the unit's key range
    int64_t *bcount;          // [n_units] set elements in the range
    int64_t *ucount;          // [n_units + 1] union size per unit (scanned later)
    int64_t *ncount;          // [n_units + 1] novel size per unit (scanned later)
    int64_t *n_big;           // device count of oversized units (single buckets above CAP)
    int64_t *big;             // [n_units] their unit indices
    int64_t *n_big2;          // those with more distinct keys than LDS holds
    int64_t *big2;            // [n_units] their unit indices (sorted over global memory)
};

__device__ __forceinline__ void unit_span(const BucketArgs &a, int64_t u, int64_t &start, int64_t &size) {
    start = a.seg[a.ufirst[u]];
    size = a.seg[a.uend[u]] - start;
}

// number of set elements <= k (upper bound) in B[0..n)
template <int W>
__device__ int64_t upper_bound_set(const uint64_t *B, int64_t n, const Key<W> &k) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (key_less<W>(k, load_key<W>(B, mid))) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

template <int W>
__device__ bool contains_set(const uint64_t *B, int64_t lo, int64_t hi, const Key<W> &k) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const Key<W> m = load_key<W>(B, mid);
        if (key_less<W>(m, k)) lo = mid + 1;
        else if (key_less<W>(k, m)) hi = mid;
        else return true;
    }
    return false;
}

// Key range (lo, hi] of final slot s; returns false for slots that are not buckets.
template <int W>
__device__ bool slot_range(const BucketArgs &a, int64_t s, Key<W> &lo, bool &has_lo, Key<W> &hi, bool &has_hi) {
    has_lo = has_hi = false;
    if (!a.two_level) return s == 0;
    const int b1 = (int)(s / a.F2), b2 = (int)(s % a.F2);
    const int f1 = a.fan1[0];
    if (b1 >= f1) return false;
    const int f2 = a.fan2[b1];
    if (b2 >= f2) return false;
    const uint64_t *s2 = a.spl2 + (int64_t)b1 * (a.F2 - 1) * W;
    if (b2 > 0) {
        lo = load_key<W>(s2, b2 - 1);
        has_lo = true;
    } else if (b1 > 0) {
        lo = load_key<W>(a.spl1, b1 - 1);
        has_lo = true;
    }
    if (b2 < f2 - 1) {
        hi = load_key<W>(s2, b2);
        has_hi = true;
    } else if (b1 < f1 - 1) {
        hi = load_key<W>(a.spl1, b1);
        has_hi = true;
    }
    return true;
}

// one thread per unit: the set elements whose keys fall in the unit's range, the
// lower bound of its first bucket to the upper bound of its last
template <int W>
__global__ void set_range_kernel(BucketArgs a) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= *a.n_units) return;
    const int64_t nB = (a.B && a.nB) ? *a.nB : 0;
    Key<W> lo, hi, tmp;
    bool hl, hh, t0;
    int64_t bl = 0, bh = 0;
    if (nB > 0 && slot_range<W>(a, a.ufirst[u], lo, hl, tmp, t0) && slot_range<W>(a, a.uend[u] - 1, tmp, t0, hi, hh)) {
        bl = hl ? upper_bound_set<W>(a.B, nB, lo) : 0;
        bh = hh ? upper_bound_set<W>(a.B, nB, hi) : nB;
        if (bh < bl) bh = bl;
    }
    a.bstart[u] = bl;
    a.bcount[u] = bh - bl;
}

// Units: consecutive final buckets of one level-1 bucket, greedily grouped while the
// total stays within CAP keys (a bucket above CAP is a unit of its own).  Pass 0
// counts each level-1 bucket's units, pass 1 (after a scan) writes them.
template <int W, int PASS>
__global__ void pack_units_kernel(BucketArgs a, int S1, int64_t *ucnt, int64_t *n_units1) {
    using C = DCfg<W>;
    const int s1 = blockIdx.x * blockDim.x + threadIdx.x;
    if (s1 > S1) return;
    if (s1 == S1) {  // the scan's tail element, and the counts' zero tails
        if (PASS == 0) ucnt[S1] = 0;
        else {
            const int64_t nu = ucnt[S1];
            *n_units1 = nu + 1;
            a.ucount[nu] = 0;
            a.ncount[nu] = 0;
        }
        return;
    }
    const int f2 = s1 < a.fan1[0] ? a.fan2[s1] : 0;
    const int32_t s0 = s1 * a.F2;
    int64_t k = PASS == 0 ? 0 : ucnt[s1];
    const int64_t k0 = k;
    int32_t first = s0;
    int64_t fill = 0;
    for (int b = 0; b < f2; ++b) {
        const int64_t sz = a.seg[s0 + b + 1] - a.seg[s0 + b];
        if (b > first - s0 && fill + sz > C::CAP) {
            if (PASS == 1) {
                const_cast<int32_t *>(a.ufirst)[k] = first;
                const_cast<int32_t *>(a.uend)[k] = s0 + b;
            }
            ++k;
            first = s0 + b;
            fill = 0;
        }
        fill += sz;
    }
    if (f2 > 0) {
        if (PASS == 1) {
            const_cast<int32_t *>(a.ufirst)[k] = first;
            const_cast<int32_t *>(a.uend)[k] = s0 + f2;
        }
        ++k;
    }
    if (PASS == 0) ucnt[s1] = k - k0;
}

// one bucket covering every key: one unit
__global__ void single_unit_kernel(BucketArgs a, int64_t *n_units1) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const_cast<int32_t *>(a.ufirst)[0] = 0;
        const_cast<int32_t *>(a.uend)[0] = 1;
        const_cast<int64_t *>(a.n_units)[0] = 1;
        *n_units1 = 2;
        a.ucount[1] = 0;
        a.ncount[1] = 0;
    }
}

struct BucketLds {
    RadixLds R;
    int64_t brange[2];
    uint32_t gbase[256], dtot[256];
    int64_t red[kDWaves];
};

// Multiplicative hash of a key to log2(T) bits (keys of one bucket differ mostly in low bits).
template <int W>
__device__ __forceinline__ uint32_t key_hash(const Key<W> &k, int log_t) {
    uint64_t x = k.w[0];
#pragma unroll
    for (int j = 1; j < W; ++j) x ^= k.w[j] * 0x9E3779B97F4A7C15ull;
    const uint32_t y = (uint32_t)x ^ (uint32_t)(x >> 32) * 0x85EBCA6Bu;
    return (y * 0x9E3779B1u) >> (32 - log_t);
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
    for (int o = 1; o < kWave; o <<= 1) v |= __shfl_xor(v, o);
    return v;
}

// Wave-level exclusive scan of 256 digit totals held 4 per lane; returns the
// prefix of digit 4*lane+j in pre[j].
__device__ __forceinline__ void wave_scan256(const uint32_t tot[4], uint32_t pre[4]) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t s = tot[0] + tot[1] + tot[2] + tot[3];
    uint32_t x = s;
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    uint32_t run = x - s;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        pre[j] = run;
        run += tot[j];
    }
}

// The bucket kernel runs 512-thread workgroups, three per CU for one-word keys and
// four for two-word keys (what LDS allows), and the extra waves hide LDS and memory
// latency.
constexpr int kBThreads = 512;
constexpr int kBWaves = kBThreads / kWave;

// One stable LSD pass of the 512-thread unit sort on the 8-bit digit at `shift`, of
// which the bits in `vmask` vary in the unit.  Stability inside a wave rests on LDS
// atomics of one instruction to one address being served in lane order (checked on
// gfx950: every wave of 131,072 probes with 1, 4, 32 and 256 distinct addresses
// received lane-ordered counts).  This wave's keys are
// cur[base_pos + k*64 + lane] for k < rounds, positions below `limit`; each key goes
// to nxt at (keys of smaller digits) + (keys of its digit in lower waves or earlier
// in this wave).  Keys and ranks stay in registers between the two sweeps.
template <int W, int KB>
__device__ __forceinline__ void unit_radix_pass(const Key<W> *cur, Key<W> *nxt, int shift, uint32_t vmask,
                                                int base_pos, int rounds, int limit, uint16_t (*s_cnt)[256]) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    constexpr int kBK = KB;
    // digits with few varying bits take a ballot per bit; more take one LDS atomic
    // per key (fewer instructions, and the counts then spread over enough words that
    // same-word serialisation stays short)
    const bool many = __popc(vmask) > 3;
    *reinterpret_cast<uint64_t *>(&s_cnt[w][4 * lane]) = 0ull;
    // keys and their ranks stay in registers until the scatter below
    Key<W> kr[kBK];
    uint32_t rr[kBK];
#pragma unroll
    for (int k = 0; k < kBK; ++k) {
        if (k >= rounds) break;  // wave-uniform
        const int pos = base_pos + k * kWave + lane;
        const bool valid = pos < limit;
        if (valid) kr[k] = cur[pos];
        const uint32_t d = valid ? digit_of<W>(kr[k], shift) : 0u;
        if (many) {
            // one LDS add per key on the 32-bit word holding the digit's 16-bit count: the
            // lanes of one instruction that hit the same word are served in lane order, so
            // the count returned is this key's rank among equal digits before it
            uint32_t old = 0;
            if (valid) old = atomicAdd(reinterpret_cast<uint32_t *>(&s_cnt[w][d & ~1u]), (d & 1u) ? 0x10000u : 1u);
            rr[k] = (d & 1u) ? (old >> 16) : (old & 0xffffu);
        } else {
            int rk;
            const int tot = wave_match_rank_bits(d, valid, vmask, &rk);
            uint32_t base = 0;
            if (valid) base = s_cnt[w][d];
            if (valid && rk == 0) s_cnt[w][d] = (uint16_t)(base + (uint32_t)tot);
            rr[k] = base + (uint32_t)rk;
        }
    }
    __syncthreads();
    // this wave's output offset per digit: all keys of smaller digits, plus
    // keys of this digit held by lower waves (each wave computes its own row)
    // (each lane holds digits 4*lane .. 4*lane+3: one 8-byte LDS read per wave row)
    // the four 16-bit fields add without carries: no digit count exceeds the unit's keys
    static_assert(kBK * kBThreads < 65536, "digit counts must fit 16 bits");
    uint64_t tot4 = 0, low4 = 0;
#pragma unroll
    for (int ww = 0; ww < kBWaves; ++ww) {
        const uint64_t c4 = *reinterpret_cast<const uint64_t *>(&s_cnt[ww][4 * lane]);
        tot4 += c4;
        low4 += (ww < w) ? c4 : 0ull;
    }
    uint32_t tot[4], pre[4], low[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        tot[j] = (uint32_t)(tot4 >> (16 * j)) & 0xffffu;
        low[j] = (uint32_t)(low4 >> (16 * j)) & 0xffffu;
    }
    wave_scan256(tot, pre);
    __syncthreads();  // every wave has read the counts before rows are overwritten
    {
        uint64_t o4 = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) o4 |= (uint64_t)((pre[j] + low[j]) & 0xffffu) << (16 * j);
        *reinterpret_cast<uint64_t *>(&s_cnt[w][4 * lane]) = o4;
    }
#pragma unroll
    for (int k = 0; k < kBK; ++k) {
        if (k >= rounds) break;
        const int pos = base_pos + k * kWave + lane;
        if (pos < limit) nxt[s_cnt[w][digit_of<W>(kr[k], shift)] + rr[k]] = kr[k];
    }
    __syncthreads();
}

// v of lane (this lane ^ j): j = 1 and 2 stay inside each group of four lanes and take a
// DPP quad permutation (a vector move, no LDS round trip); wider strides a lane shuffle
__device__ __forceinline__ uint32_t lane_xor_u32(uint32_t v, int j) {
    if (j == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);  // lanes 1,0,3,2
    if (j == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);  // lanes 2,3,0,1
    return (uint32_t)__shfl_xor((int)v, j);
}

__device__ __forceinline__ uint64_t lane_xor_u64(uint64_t v, int j) {
    const uint32_t lo = lane_xor_u32((uint32_t)v, j), hi = lane_xor_u32((uint32_t)(v >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

// a < b where an invalid key counts as larger than every valid one
template <int W>
__device__ __forceinline__ bool less_valid(const Key<W> &a, bool av, const Key<W> &b, bool bv) {
    return av && (!bv || key_less<W>(a, b));
}

// Sort of at most one key per thread of a workgroup (u <= kBThreads distinct keys):
// thread t holds key t (valid iff t < u).  Each wave sorts its 64 keys in registers
// with a bitonic network (partners exchanged across lanes, no barrier); the sorted
// runs of 64 are then merged pairwise in buf, each key moving to its index in its own
// run plus its rank in the partner run (keys are distinct, so ranks never tie).  The
// sorted keys end in buf[0, u).
template <int W>
__device__ __forceinline__ void small_unit_sort(Key<W> key, bool valid, int u, Key<W> *buf) {
    const int lane = threadIdx.x & (kWave - 1);
    // a wave holding no key (all of its positions at or above u) skips the network
    if ((int)(threadIdx.x & ~(kWave - 1)) < u) {  // wave-uniform
#pragma unroll
        for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                Key<W> p;
#pragma unroll
                for (int q = 0; q < W; ++q) p.w[q] = lane_xor_u64(key.w[q], j);
                const bool pv = lane_xor_u32((uint32_t)valid, j) != 0u;
                // ascending blocks of k lanes alternate with descending ones (the last
                // is the whole wave, ascending); the lower lane of a pair keeps the
                // smaller key of an ascending block
                const bool keep_min = ((lane & k) == 0) == ((lane & j) == 0);
                const bool take = keep_min ? less_valid<W>(p, pv, key, valid) : less_valid<W>(key, valid, p, pv);
                if (take) {
                    key = p;
                    valid = pv;
                }
            }
        }
    }
    int pos = threadIdx.x;  // valid keys of each wave now lead its 64 positions
    if (valid) buf[pos] = key;
    __syncthreads();
    for (int L = kWave; L < u; L <<= 1) {  // workgroup-uniform
        int np = pos;
        if (valid) {
            const int r = pos / L;
            const int ps = (r ^ 1) * L;
            int lo = ps, hi = ps + L < u ? ps + L : u;
            if (lo > hi) lo = hi;  // no partner run
            const int p0 = lo;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (key_less<W>(buf[mid], key)) lo = mid + 1;
                else hi = mid;
            }
            np = (r & ~1) * L + (pos - r * L) + (lo - p0);
        }
        __syncthreads();  // every search of this round has read buf
        if (valid) buf[np] = key;
        pos = np;
        __syncthreads();
    }
}

// The sorted unique run of unit s (cur[0..u) in LDS), less the keys the running set
// already holds in the unit's range, to its place in dst, and the unit's counts:
// the run that emit merges is then disjoint from the set keys it is merged with.
// A short set range is streamed once and each of its keys searched among the unique
// keys in LDS (a hit marks that key in `dup`, one bit per key, LDS the caller no
// longer needs); a long one is searched per unique key instead, whichever moves
// fewer bytes.
template <int W>
__device__ __forceinline__ void finish_unit(const BucketArgs &a, int64_t s, const Key<W> *cur, int u, int64_t start,
                                            int64_t bl, int64_t bh, uint32_t *dup, int64_t *s_wsum) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t nb = bh - bl;
    if (nb > 0) {
        const bool stream_set = nb <= 56 * (int64_t)u;
        for (int i = threadIdx.x; i < (u + 31) / 32; i += kBThreads) dup[i] = 0u;
        __syncthreads();
        if (stream_set) {
            // each thread takes G consecutive set keys: one search for the first, then
            // the position advances along the run (it never decreases)
            constexpr int G = 8;
            for (int64_t jt = bl; jt < bh; jt += (int64_t)G * kBThreads) {
                const int64_t jb = jt + (int64_t)threadIdx.x * G;
                if (jb >= bh) continue;
                Key<W> kb[G];
#pragma unroll
                for (int g = 0; g < G; ++g)
                    if (jb + g < bh) kb[g] = load_key<W>(a.B, jb + g);
                int lo = 0, hi = u;  // first unique key not below kb[0]
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (key_less<W>(cur[mid], kb[0])) lo = mid + 1;
                    else hi = mid;
                }
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    if (jb + g >= bh) break;
                    if (g) while (lo < u && key_less<W>(cur[lo], kb[g])) ++lo;
                    if (lo < u && key_eq<W>(cur[lo], kb[g])) atomicOr(&dup[lo >> 5], 1u << (lo & 31));
                }
            }
        } else {
            for (int i = threadIdx.x; i < u; i += kBThreads)
                if (contains_set<W>(a.B, bl, bh, cur[i])) atomicOr(&dup[i >> 5], 1u << (i & 31));
        }
        __syncthreads();
    }
    // each wave compacts one contiguous slice of the run, in order
    const int span = ((u + kBWaves * kWave - 1) / (kBWaves * kWave)) * kWave;
    const int lo = w * span < u ? w * span : u, hi = lo + span < u ? lo + span : u;
    int keep_n = 0;
    for (int i0 = lo; i0 < hi; i0 += kWave) {
        const int i = i0 + lane;
        const bool keep = i < hi && (nb == 0 || !((dup[i >> 5] >> (i & 31)) & 1u));
        keep_n += __popcll(__ballot(keep));
    }
    if (lane == 0) s_wsum[w] = keep_n;
    __syncthreads();
    int64_t base = 0, total = 0;
#pragma unroll
    for (int ww = 0; ww < kBWaves; ++ww) {
        base += ww < w ? s_wsum[ww] : 0;
        total += s_wsum[ww];
    }
    for (int i0 = lo; i0 < hi; i0 += kWave) {
        const int i = i0 + lane;
        const bool keep = i < hi && (nb == 0 || !((dup[i >> 5] >> (i & 31)) & 1u));
        const uint64_t bal = __ballot(keep);
        if (keep) store_key<W>(a.dst, start + base + __popcll(bal & lanemask_lt()), cur[i]);
        base += __popcll(bal);
    }
    if (threadIdx.x == 0) {
        a.nuniq[s] = total;
        a.ucount[s] = total + nb;
        a.ncount[s] = total;
    }
}

// LDS holds 24 KB of keys per workgroup (3,072 one-word or 1,536 two-word keys) and a
// hash table of 16-bit slots (16 / 8 KB): four workgroups per CU for two-word keys,
// three for one-word keys.  The radix passes sort in place: each pass holds its keys in
// registers from before its first barrier, so it writes back into the buffer it read.
// A unit left with at most one novel key per thread (most units once the set holds the
// earlier chunks' keys) skips them: each wave sorts its keys in registers and three
// merge rounds at most finish the run (8 barriers at most instead of 3 per radix pass).  Two-word
// workgroups are held to 64 VGPRs, so that four of them (eight waves per SIMD) fit a CU.
//
// The running set's keys of the unit's range are looked up in the unit's hash table
// before anything is sorted: a short range is streamed through the table (its first
// loads issued together with the unit's own keys), a long one is searched per
// distinct key.  Only the keys the set does not hold are compacted, sorted and
// written, so the run handed to emit is disjoint from the set and the sort skips
// every key the set already holds.
template <int W>
__global__ __launch_bounds__(kBThreads) __attribute__((amdgpu_waves_per_eu(W == 2 ? 8 : 6, 8)))
void bucket_kernel(BucketArgs a) {
    using C = DCfg<W>;
    constexpr int kBK = (C::CAP + kBThreads - 1) / kBThreads;  // keys per thread at capacity
    constexpr int kSP = 2;                                      // set keys per thread loaded up front
    // table slots: the smallest power of two at least twice the capacity (load at most 1/2)
    constexpr int kLogTab = 32 - __builtin_clz(2u * C::CAP - 1u);
    __shared__ Key<W> s_k0[C::CAP];          // candidate keys, then each wave's novel keys, sorted in place
    __shared__ uint32_t s_tab[(1 << kLogTab) / 2];  // hash table, two 16-bit slots per word
    __shared__ __align__(8) uint16_t s_cnt[kBWaves][256];  // per-wave digit counts, then output offsets
    __shared__ uint32_t s_dup[C::CAP / 32];  // bit i: the key at position i is a set key
    __shared__ uint64_t s_or[2];
    __shared__ int s_u[kBWaves];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t s = blockIdx.x;  // unit
    if (s >= *a.n_units) return;
    int64_t start, size;
    unit_span(a, s, start, size);
    const int64_t bl = a.bstart[s], bh = bl + a.bcount[s];
    const int64_t nb = bh - bl;

    if (size > C::CAP) {
        // sorted by bucket_big_kernel
        if (threadIdx.x == 0) {
            const unsigned long long slot = atomicAdd((unsigned long long *)a.n_big, 1ull);
            a.big[slot] = s;
        }
        return;
    }
    if (size > 0) {
        const int m = (int)size;
        // each wave owns a contiguous slice of CHm positions
        const int Km = (m + kBThreads - 1) / kBThreads;
        const int CHm = Km * kWave;
        const int my0 = w * CHm;
        // this lane's keys stay in registers (positions my0 + k*64 + lane, the order of
        // the hashing and compaction below); LDS holds them for the probes' comparisons
        Key<W> kk[kBK];
#pragma unroll
        for (int k = 0; k < kBK; ++k) {
            const int i = my0 + k * kWave + lane;
            if (k < Km && i < m) kk[k] = load_key<W>(a.src, start + i);
        }
        // a set range up to 56 keys per unit key is streamed through the hash table;
        // its first kSP x 512 keys are in flight with the unit's own
        const bool stream_set = nb > 0 && nb <= 56 * (int64_t)m;
        Key<W> sk[kSP];
        if (stream_set) {
#pragma unroll
            for (int p = 0; p < kSP; ++p) {
                const int64_t j = bl + p * kBThreads + threadIdx.x;
                if (j < bh) sk[p] = load_key<W>(a.B, j);
            }
        }
#pragma unroll
        for (int k = 0; k < kBK; ++k) {
            const int i = my0 + k * kWave + lane;
            if (k < Km && i < m) s_k0[i] = kk[k];
        }
        // hash table of 16-bit key indices (0xffff = empty), two slots per 32-bit word
        int log_t = 4;
        while ((1 << log_t) < 2 * m) ++log_t;
        const uint32_t tmask = (1u << log_t) - 1u;
        uint32_t *tab = s_tab;
        for (int i = threadIdx.x; i < (1 << log_t) / 2; i += kBThreads) tab[i] = 0xffffffffu;
        for (int i = threadIdx.x; i < C::CAP / 32; i += kBThreads) s_dup[i] = 0u;
        if (threadIdx.x == 0) s_or[0] = s_or[1] = 0;
        __syncthreads();
        const Key<W> ref = s_k0[0];
        // bit k of `fresh`: this lane's key of round k is the first occurrence of its value
        uint32_t fresh = 0;
#pragma unroll
        for (int k = 0; k < kBK; ++k) {
            if (k >= Km) break;  // wave-uniform
            const int i = my0 + k * kWave + lane;
            if (i >= m) continue;
            const Key<W> key = kk[k];
            uint32_t h = key_hash<W>(key, log_t);
            while (true) {
                const uint32_t cur = tab[h >> 1];
                const uint32_t v = (h & 1u) ? (cur >> 16) : (cur & 0xffffu);
                if (v == 0xffffu) {
                    const uint32_t want = (h & 1u) ? ((cur & 0xffffu) | ((uint32_t)i << 16))
                                                   : ((cur & 0xffff0000u) | (uint32_t)i);
                    if (atomicCAS(&tab[h >> 1], cur, want) == cur) {
                        fresh |= 1u << k;
                        break;
                    }
                    continue;  // the word changed: look at this slot again
                }
                if (key_eq<W>(s_k0[v], key)) break;  // seen before
                h = (h + 1u) & tmask;
            }
        }
        __syncthreads();  // the table is complete (and read-only from here)
        if (nb > 0) {
            if (stream_set) {
                // a set key found in the table marks the unit key that holds the slot; the
                // table is at most half full, so every walk reaches an empty slot
                auto mark = [&](const Key<W> &key) {
                    uint32_t h = key_hash<W>(key, log_t);
                    while (true) {
                        const uint32_t cur = tab[h >> 1];
                        const uint32_t v = (h & 1u) ? (cur >> 16) : (cur & 0xffffu);
                        if (v == 0xffffu) return;
                        if (key_eq<W>(s_k0[v], key)) {
                            atomicOr(&s_dup[v >> 5], 1u << (v & 31));
                            return;
                        }
                        h = (h + 1u) & tmask;
                    }
                };
#pragma unroll
                for (int p = 0; p < kSP; ++p)
                    if (bl + p * kBThreads + threadIdx.x < bh) mark(sk[p]);
                for (int64_t j0 = bl + kSP * kBThreads; j0 < bh; j0 += kSP * kBThreads) {
#pragma unroll
                    for (int p = 0; p < kSP; ++p) {
                        const int64_t j = j0 + p * kBThreads + threadIdx.x;
                        if (j < bh) sk[p] = load_key<W>(a.B, j);
                    }
#pragma unroll
                    for (int p = 0; p < kSP; ++p)
                        if (j0 + p * kBThreads + threadIdx.x < bh) mark(sk[p]);
                }
            } else {
#pragma unroll
                for (int k = 0; k < kBK; ++k) {
                    if (k >= Km) break;  // wave-uniform
                    const int i = my0 + k * kWave + lane;
                    if (((fresh >> k) & 1u) && contains_set<W>(a.B, bl, bh, kk[k]))
                        atomicOr(&s_dup[i >> 5], 1u << (i & 31));
                }
            }
            __syncthreads();
        }
        // each wave compacts its novel keys (first occurrences the set does not hold)
        // to the front of its own slice
        int uw = 0;
        uint64_t acc[W];
#pragma unroll
        for (int j = 0; j < W; ++j) acc[j] = 0;
#pragma unroll
        for (int k = 0; k < kBK; ++k) {
            if (k >= Km) break;  // wave-uniform
            const int i = my0 + k * kWave + lane;
            const bool keep = (i < m) && ((fresh >> k) & 1u) && !((s_dup[i >> 5] >> (i & 31)) & 1u);
            Key<W> key;
            if (keep) {
                key = kk[k];
#pragma unroll
                for (int j = 0; j < W; ++j) acc[j] |= key.w[j] ^ ref.w[j];
            }
            const uint64_t bal = __ballot(keep);
            if (keep) s_k0[my0 + uw + __popcll(bal & lanemask_lt())] = key;
            uw += __popcll(bal);
        }
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const uint64_t o = wave_or64(acc[j]);
            if (lane == 0 && o) atomicOr((unsigned long long *)&s_or[j], (unsigned long long)o);
        }
        if (lane == 0) s_u[w] = uw;
        __syncthreads();
        uint64_t orx[W];
#pragma unroll
        for (int j = 0; j < W; ++j) orx[j] = s_or[j];
        const int nbits = varying_bits<W>(orx);
        const int lo_bit = lowest_varying_bit<W>(orx);
        Key<W> orkey;
#pragma unroll
        for (int j = 0; j < W; ++j) orkey.w[j] = orx[j];
        int u = 0;
#pragma unroll
        for (int ww = 0; ww < kBWaves; ++ww) u += s_u[ww];

        if (u > 1 && u <= kBThreads) {  // workgroup-uniform
            // one novel key per thread: thread t takes the t-th key of the waves' slices
            int src = -1;
            {
                int pre = 0;
#pragma unroll
                for (int ww = 0; ww < kBWaves; ++ww) {
                    const int c = s_u[ww];
                    if (threadIdx.x >= pre && threadIdx.x < pre + c) src = ww * CHm + ((int)threadIdx.x - pre);
                    pre += c;
                }
            }
            const bool valid = src >= 0;
            bool low_only = false;
            if constexpr (W == 2) low_only = orx[1] == 0ull;  // every novel key has ref's top word
            if (low_only) {
                Key<1> *s_lw = reinterpret_cast<Key<1> *>(s_k0);
                Key<1> lk;
                lk.w[0] = valid ? s_k0[src].w[0] : 0ull;
                __syncthreads();  // every source read before the 8-byte view is written
                small_unit_sort<1>(lk, valid, u, s_lw);
                for (int i = threadIdx.x; i < u; i += kBThreads) {
                    Key<W> k = ref;
                    k.w[0] = s_lw[i].w[0];
                    store_key<W>(a.dst, start + i, k);
                }
            } else {
                Key<W> k = ref;
                if (valid) k = s_k0[src];
                __syncthreads();  // every source read before buf is written
                small_unit_sort<W>(k, valid, u, s_k0);
                for (int i = threadIdx.x; i < u; i += kBThreads) store_key<W>(a.dst, start + i, s_k0[i]);
            }
            if (threadIdx.x == 0) {
                a.nuniq[s] = u;
                a.ucount[s] = u + nb;
                a.ncount[s] = u;
            }
            return;
        }
        // stable LSD radix sort of the u novel keys, in place in LDS.  The first pass
        // reads every wave's own slice (any starting order is fine); later passes
        // read the contiguous result of the previous pass.
        const int Kd = (u + kBThreads - 1) / kBThreads;
        const int CHd0 = Kd * kWave;
        if constexpr (W == 2) {
            if (orx[1] == 0ull) {  // workgroup-uniform
                // Every novel key has the top word of `ref` (most units lie in one top
                // word): the low words are sorted alone, half the LDS bytes per pass, and
                // the top word is put back as the run is written.  Each wave's keys move
                // to the same positions of an 8-byte view, read before any is written.
                Key<1> *s_lw = reinterpret_cast<Key<1> *>(s_k0);
                uint64_t lw[kBK];
#pragma unroll
                for (int k = 0; k < kBK; ++k)
                    if (k * kWave + lane < uw) lw[k] = s_k0[my0 + k * kWave + lane].w[0];
                __syncthreads();
#pragma unroll
                for (int k = 0; k < kBK; ++k)
                    if (k * kWave + lane < uw) s_lw[my0 + k * kWave + lane].w[0] = lw[k];
                __syncthreads();
                Key<1> orlow;
                orlow.w[0] = orx[0];
                bool first1 = true;
                for (int shift = lo_bit; shift < nbits; shift += 8) {
                    const uint32_t vm = digit_of<1>(orlow, shift);
                    if (vm == 0u) continue;  // workgroup-uniform
                    const int base_pos = first1 ? my0 : w * CHd0;
                    const int rounds = first1 ? (uw + kWave - 1) / kWave : Kd;
                    const int limit = first1 ? my0 + uw : u;
                    unit_radix_pass<1, kBK>(s_lw, s_lw, shift, vm, base_pos, rounds, limit, s_cnt);
                    first1 = false;
                }
                if (first1) {
                    // no pass ran: at most one novel key
                    if (threadIdx.x == 0) {
                        for (int ww = 0; ww < kBWaves; ++ww)
                            if (s_u[ww] > 0) {
                                s_lw[0] = s_lw[ww * CHm];
                                break;
                            }
                    }
                    __syncthreads();
                }
                for (int i = threadIdx.x; i < u; i += kBThreads) {
                    Key<W> k;
                    k.w[0] = s_lw[i].w[0];
                    k.w[1] = ref.w[1];
                    store_key<W>(a.dst, start + i, k);
                }
                if (threadIdx.x == 0) {
                    a.nuniq[s] = u;
                    a.ucount[s] = u + nb;
                    a.ncount[s] = u;
                }
                return;
            }
        }
        const int CHd = Kd * kWave;
        bool first = true;
        // digits cover only the bits that vary among the novel keys; a window in which
        // no key differs would be an identity pass and is skipped
        for (int shift = lo_bit; shift < nbits; shift += 8) {
            const uint32_t vm = digit_of<W>(orkey, shift);  // varying bits of this window
            if (vm == 0u) continue;                         // workgroup-uniform
            const int base_pos = first ? my0 : w * CHd;
            const int rounds = first ? (uw + kWave - 1) / kWave : Kd;  // the first pass reads only this wave's keys
            const int limit = first ? my0 + uw : u;
            unit_radix_pass<W, kBK>(s_k0, s_k0, shift, vm, base_pos, rounds, limit, s_cnt);
            first = false;
        }
        if (first) {
            // no pass ran: at most one novel key (distinct keys differ somewhere)
            if (threadIdx.x == 0) {
                for (int ww = 0; ww < kBWaves; ++ww)
                    if (s_u[ww] > 0) {
                        s_k0[0] = s_k0[ww * CHm];
                        break;
                    }
            }
            __syncthreads();
        }
        for (int i = threadIdx.x; i < u; i += kBThreads) store_key<W>(a.dst, start + i, s_k0[i]);
        if (threadIdx.x == 0) {
            a.nuniq[s] = u;
            a.ucount[s] = u + nb;
            a.ncount[s] = u;
        }
        return;
    }
    if (threadIdx.x == 0) {  // an empty unit: its range holds only set keys
        a.nuniq[s] = 0;
        a.ucount[s] = nb;
        a.ncount[s] = 0;
    }
}

// Oversized units, mostly a few keys repeated many times: the keys stream through
// LDS in CAP-key chunks against one unit-wide hash table, and first occurrences
// collect in LDS.  When the distinct keys fit they are sorted there as in
// bucket_kernel; otherwise the unit moves on to bucket_big_kernel.
template <int W>
__global__ __launch_bounds__(kBThreads) void bucket_stream_kernel(BucketArgs a) {
    using C = DCfg<W>;
    constexpr int kBK = (C::CAP + kBThreads - 1) / kBThreads;
    // at least 4 CAP slots (a power of two): load at most 1/2
    constexpr int kLogT = 32 - __builtin_clz(4u * C::CAP - 1u);
    constexpr uint32_t kTSlots = 1u << kLogT;
    constexpr uint32_t kTMask = kTSlots - 1u;
    __shared__ Key<W> s_in[C::CAP];     // the current chunk; radix ping-pong at the end
    __shared__ Key<W> s_uq[C::CAP];     // distinct keys so far
    __shared__ uint32_t s_tab[kTSlots / 2];  // 16-bit slots: index < CAP in s_uq, CAP + i in s_in
    __shared__ __align__(8) uint16_t s_cnt[kBWaves][256];
    __shared__ uint64_t s_or[2];
    __shared__ int s_nu, s_over;
    __shared__ int64_t s_wsum[kBWaves];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t n_big = *a.n_big;
    for (int64_t t = blockIdx.x; t < n_big; t += gridDim.x) {
        const int64_t s = a.big[t];
        int64_t start, size;
        unit_span(a, s, start, size);
        const int64_t bl = a.bstart[s], bh = bl + a.bcount[s];
        const Key<W> ref = load_key<W>(a.src, start);
        for (int i = threadIdx.x; i < (int)(kTSlots / 2); i += kBThreads) s_tab[i] = 0xffffffffu;
        if (threadIdx.x == 0) {
            s_nu = 0;
            s_over = 0;
            s_or[0] = s_or[1] = 0;
        }
        uint64_t acc[W];
#pragma unroll
        for (int j = 0; j < W; ++j) acc[j] = 0;
        __syncthreads();
        for (int64_t c0 = 0; c0 < size; c0 += C::CAP) {
            const int m = (int)std::min<int64_t>(C::CAP, size - c0);
            Key<W> kk[kBK];
#pragma unroll
            for (int k = 0; k < kBK; ++k) {
                const int i = k * kBThreads + threadIdx.x;
                if (i < m) kk[k] = load_key<W>(a.src, start + c0 + i);
            }
#pragma unroll
            for (int k = 0; k < kBK; ++k) {
                const int i = k * kBThreads + threadIdx.x;
                if (i < m) s_in[i] = kk[k];
            }
            __syncthreads();
            uint32_t fresh = 0, slot[kBK];
#pragma unroll
            for (int k = 0; k < kBK; ++k) {
                const int i = k * kBThreads + threadIdx.x;
                if (i >= m) continue;
                uint32_t h = key_hash<W>(kk[k], kLogT);
                // At most 2 CAP keys (CAP distinct so far, CAP in this chunk) occupy the
                // kTSlots >= 4 CAP slots, and each failed exchange follows another lane's
                // insertion: the walk ends within kTSlots visits plus 2 CAP retries.
                for (int probe = 0; probe < (int)kTSlots + 2 * C::CAP; ++probe) {
                    const uint32_t cur = s_tab[h >> 1];
                    const uint32_t v = (h & 1u) ? (cur >> 16) : (cur & 0xffffu);
                    if (v == 0xffffu) {
                        const uint32_t idx = (uint32_t)(C::CAP + i);
                        const uint32_t want = (h & 1u) ? ((cur & 0xffffu) | (idx << 16)) : ((cur & 0xffff0000u) | idx);
                        if (atomicCAS(&s_tab[h >> 1], cur, want) == cur) {
                            fresh |= 1u << k;
                            slot[k] = h;
                            break;
                        }
                        continue;  // the word changed: look at this slot again
                    }
                    const Key<W> other = v < (uint32_t)C::CAP ? s_uq[v] : s_in[v - C::CAP];
                    if (key_eq<W>(other, kk[k])) break;  // seen before
                    h = (h + 1u) & kTMask;
                }
            }
            __syncthreads();
            // this chunk's first occurrences join the distinct keys (one LDS atomic per wave and round)
#pragma unroll
            for (int k = 0; k < kBK; ++k) {
                const bool keep = (fresh >> k) & 1u;
                const uint64_t bal = __ballot(keep);
                if (bal == 0ull) continue;
                int base = 0;
                if (lane == 0) base = atomicAdd(&s_nu, __popcll(bal));
                base = __shfl(base, 0);
                if (keep) {
                    const int pos = base + __popcll(bal & lanemask_lt());
                    if (pos < C::CAP) {
                        s_uq[pos] = kk[k];
                        // the slot now names s_uq[pos] instead of s_in[i]; the word's other
                        // slot may change meanwhile, so flip just this slot's bits
                        const uint32_t h = slot[k];
                        const uint32_t flip = (uint32_t)(C::CAP + k * kBThreads + threadIdx.x) ^ (uint32_t)pos;
                        atomicXor(&s_tab[h >> 1], (h & 1u) ? (flip << 16) : flip);
#pragma unroll
                        for (int j = 0; j < W; ++j) acc[j] |= kk[k].w[j] ^ ref.w[j];
                    } else {
                        s_over = 1;
                    }
                }
            }
            __syncthreads();
            if (s_over) break;  // workgroup-uniform after the barrier
        }
        if (s_over) {
            if (threadIdx.x == 0) {
                const unsigned long long q = atomicAdd((unsigned long long *)a.n_big2, 1ull);
                a.big2[q] = s;
            }
            __syncthreads();
            continue;
        }
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const uint64_t o = wave_or64(acc[j]);
            if (lane == 0 && o) atomicOr((unsigned long long *)&s_or[j], (unsigned long long)o);
        }
        __syncthreads();
        uint64_t orx[W];
        Key<W> orkey;
#pragma unroll
        for (int j = 0; j < W; ++j) orkey.w[j] = orx[j] = s_or[j];
        const int nbits = varying_bits<W>(orx);
        const int lo_bit = lowest_varying_bit<W>(orx);
        const int u = s_nu;
        Key<W> *cur = s_uq, *nxt = s_in;
        const int Kd = (u + kBThreads - 1) / kBThreads;
        for (int shift = lo_bit; shift < nbits; shift += 8) {
            const uint32_t vm = digit_of<W>(orkey, shift);
            if (vm == 0u) continue;
            unit_radix_pass<W, kBK>(cur, nxt, shift, vm, w * Kd * kWave, Kd, u, s_cnt);
            Key<W> *tmp = cur;
            cur = nxt;
            nxt = tmp;
        }
        finish_unit<W>(a, s, cur, u, start, bl, bh, reinterpret_cast<uint32_t *>(nxt), s_wsum);
        __syncthreads();  // LDS is reused by the next unit
    }
}

// Oversized units with more distinct keys than LDS holds (the streaming kernel
// above passes them on): one workgroup per listed unit sorts over global memory
// with the same radix ranking, then run-length unique; fixed grid, units taken in
// grid-stride order from the device list.
template <int W>
__global__ __launch_bounds__(kDThreads) void bucket_big_kernel(BucketArgs a) {
    using C = DCfg<W>;
    __shared__ BucketLds L;
    // a unit of up to SCAP keys (the splitter kernel's LDS sort) is sorted in LDS, a
    // larger one over global memory
    __shared__ Key<W> s_buf[C::SCAP];
    __shared__ Key<W> s_tmp[C::SCAP];
    const int64_t n_big = *a.n_big2;
    for (int64_t t = blockIdx.x; t < n_big; t += gridDim.x) {
        const int64_t s = a.big2[t];
        int64_t start, size;
        unit_span(a, s, start, size);
        const int64_t bl = a.bstart[s], bh = bl + a.bcount[s];
        const bool in_lds = size <= C::SCAP;
        const uint64_t *res = nullptr;
        const Key<W> *lres = nullptr;
        if (in_lds) {
            const int m = (int)size;
            for (int i = threadIdx.x; i < m; i += kDThreads) s_buf[i] = load_key<W>(a.src, start + i);
            __syncthreads();
            const Key<W> ref = s_buf[0];
            __syncthreads();
            Key<W> orkey;
            const int nbits = block_varying_bits<W>(m, ref, [&](int64_t i) { return s_buf[i]; }, L.R, &orkey);
            lres = lds_radix_sort<W, C::SCAP>(s_buf, s_tmp, m, nbits, orkey, L.R);
        } else {
            uint64_t *X = const_cast<uint64_t *>(a.src) + start * W;
            uint64_t *Y = a.dst + start * W;
            const int where = global_radix_sort<W>(X, X, Y, size, L.R, L.gbase, L.dtot);
            res = where ? Y : X;
        }
        auto key_at = [&](int64_t i) { return in_lds ? lres[i] : load_key<W>(res, i); };
        // first occurrences the running set does not hold, compacted in order
        int64_t run = 0;
        for (int64_t i0 = 0; i0 < size; i0 += kDThreads) {
            const int64_t i = i0 + threadIdx.x;
            Key<W> cur;
            bool keep = false;
            if (i < size) {
                cur = key_at(i);
                keep = (i == 0) || !key_eq<W>(cur, key_at(i - 1));
            }
            __syncthreads();  // every read of this round precedes the writes (in place when res == dst)
            if (keep && bh > bl && contains_set<W>(a.B, bl, bh, cur)) keep = false;
            int64_t tot;
            const int64_t ex = block_excl_scan_i64(keep ? 1 : 0, &tot, L.R.wsum);
            if (keep) store_key<W>(a.dst, start + run + ex, cur);
            run += tot;
            __threadfence();
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            a.nuniq[s] = run;
            a.ucount[s] = run + (bh - bl);
            a.ncount[s] = run;
        }
        __threadfence();
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// emit: per bucket, merge its unique run with the set elements of its range
// into set_out at the scanned union offset; novel keys at the novel offset
// ---------------------------------------------------------------------------
constexpr int kMergePer = 2;                     // merged positions per thread per window
constexpr int kEmitStep = kDThreads * kMergePer;  // outputs per staged merge window

struct EmitArgs {
    const uint64_t *runs;     // unit runs, disjoint from the set (at their first bucket's seg offset)
    const int64_t *seg;
    const int32_t *ufirst;
    const int64_t *n_units;
    const int64_t *nuniq, *bstart, *bcount;
    const int64_t *uoff, *noff;  // scanned ucount / ncount
    const uint64_t *B;
    uint64_t *out;
    int64_t out_cap;
    uint64_t *novel;          // nullable
    int64_t novel_cap;
};

// Run keys among the first k outputs of merge(A, B) (ties: B first), searched by one
// wave: each round probes 64 evenly spaced split points and keeps the interval
// between the last that is still too low and the first that is not.
template <int W>
__device__ int64_t wave_merge_path(const uint64_t *A, int64_t nA, const uint64_t *B, int64_t nB, int64_t k) {
    const int lane = threadIdx.x & (kWave - 1);
    int64_t lo = k > nB ? k - nB : 0, hi = k < nA ? k : nA;  // answer in [lo, hi]
    while (hi > lo) {
        const int64_t span = hi - lo;
        const int64_t x = lo + (span * lane) / kWave;  // probes cover [lo, hi) once span <= 64
        const bool p = key_less<W>(load_key<W>(A, x), load_key<W>(B, k - x - 1));
        const int t = __popcll(__ballot(p));  // the true probes form a prefix of the lanes
        if (t == 0) return lo;
        const int64_t last_true = lo + (span * (t - 1)) / kWave;
        const int64_t first_false = t < kWave ? lo + (span * t) / kWave : hi;
        lo = last_true + 1;
        hi = first_false;
    }
    return lo;
}

template <int W>
__global__ __launch_bounds__(kDThreads) __attribute__((amdgpu_waves_per_eu(6, 8)))
void emit_kernel(EmitArgs a) {
    __shared__ int64_t wsum[kDWaves];
    const int64_t s = blockIdx.x;  // unit
    if (s >= *a.n_units) return;
    const uint64_t *A = a.runs + a.seg[a.ufirst[s]] * W;
    const int64_t nA = a.nuniq[s];
    const uint64_t *Bs = a.B ? a.B + a.bstart[s] * W : nullptr;
    const int64_t nBs = a.bcount[s];
    const int64_t total = nA + nBs;
    if (total == 0) return;
    int64_t ou = a.uoff[s], on = a.noff[s];
    if (nBs == 0) {
        // common case: the run is the union and all of it is novel
        constexpr int U = 8;
        for (int64_t i0 = 0; i0 < nA; i0 += (int64_t)U * kDThreads) {
            Key<W> k[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = i0 + u * kDThreads + threadIdx.x;
                if (i < nA) k[u] = load_key<W>(A, i);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = i0 + u * kDThreads + threadIdx.x;
                if (i < nA) {
                    if (ou + i < a.out_cap) store_key<W>(a.out, ou + i, k[u]);
                    if (a.novel && on + i < a.novel_cap) store_key<W>(a.novel, on + i, k[u]);
                }
            }
        }
        return;
    }
    // general case.  The run holds no key of the set (the bucket kernels drop those),
    // so the union is the merge of two disjoint sorted lists.
    constexpr int kCutBatch = 64;
    constexpr int kRunCap = DCfg<W>::CAP / 2;
    constexpr size_t kWinBytes = (2 * kEmitStep + 1) * sizeof(Key<W>) + kCutBatch * 8;
    constexpr size_t kInsBytes = kRunCap * (sizeof(Key<W>) + 4);
    __shared__ __align__(16) char s_raw[kWinBytes > kInsBytes ? kWinBytes : kInsBytes];
    if (nA <= kRunCap && nBs < (1ll << 31)) {
        // The run sits in LDS (up to CAP/2 keys: the LDS stays small enough for six
        // workgroups per CU, which hide more of the memory latency this kernel waits
        // on).  Set key j goes to position j + r_j, r_j = run keys below it; run keys
        // between set keys j-1 and j (indices r_{j-1} .. r_j - 1) go to i + j, i.e.
        // below run key i lie sC[i] set keys.  Reads the run and the set range once,
        // writes the union once.
        Key<W> *sR = reinterpret_cast<Key<W> *>(s_raw);
        int32_t *sC = reinterpret_cast<int32_t *>(sR + kRunCap);
        const int nAi = (int)nA, nBi = (int)nBs, lane = threadIdx.x & (kWave - 1);
        constexpr int G = 4;
        Key<W> kb[G];
        {   // the first block of set keys is in flight while the run is staged
            const int jb = (int)threadIdx.x * G;
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (jb + g < nBi) kb[g] = load_key<W>(Bs, jb + g);
        }
        for (int i = threadIdx.x; i < nAi; i += kDThreads) {
            const Key<W> k = load_key<W>(A, i);
            sR[i] = k;
            sC[i] = nBi;
            if (a.novel && on + i < a.novel_cap) store_key<W>(a.novel, on + i, k);
        }
        __syncthreads();
        auto below = [&](const Key<W> &key) {  // run keys below `key`
            int lo = 0, hi = nAi;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (key_less<W>(sR[mid], key)) lo = mid + 1;
                else hi = mid;
            }
            return lo;
        };
        // each thread takes G consecutive set keys: one search for the first, then the
        // count advances along the run (r_j never decreases with j); G = 4 measured
        // against 2 and 8 (large workload 22.7 / 21.7 / 28.1 ms per chunk)
        for (int jt = 0; jt < nBi; jt += G * kDThreads) {
            const int jb = jt + (int)threadIdx.x * G;
            if (jt > 0) {
#pragma unroll
                for (int g = 0; g < G; ++g)
                    if (jb + g < nBi) kb[g] = load_key<W>(Bs, jb + g);
            }
            int r[G];
            r[0] = jb < nBi ? below(kb[0]) : nAi;
#pragma unroll
            for (int g = 1; g < G; ++g) {
                int x = r[g - 1];
                if (jb + g < nBi)
                    while (x < nAi && key_less<W>(sR[x], kb[g])) ++x;
                r[g] = x;
            }
            // run keys below the set key just before this thread's first one: the previous
            // lane's last count, searched afresh by the first lane of a wave
            int rp = __shfl_up(r[G - 1], 1);
            if (lane == 0) rp = (jb < nBi && jb > 0) ? below(load_key<W>(Bs, jb - 1)) : 0;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int j = jb + g;
                if (j >= nBi) break;
                if (ou + j + r[g] < a.out_cap) store_key<W>(a.out, ou + j + r[g], kb[g]);
                for (int i = (g ? r[g - 1] : rp); i < r[g]; ++i) sC[i] = j;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nAi; i += kDThreads)
            if (ou + i + sC[i] < a.out_cap) store_key<W>(a.out, ou + i + sC[i], sR[i]);
        return;
    }
    // a run above LDS (an oversized unit): one window of kEmitStep outputs per round
    // with both inputs staged in LDS.  Only window ends inside the merge need a split
    // search over global memory; the four waves find those of up to kCutBatch windows
    // at once before the windows are merged.
    Key<W> *sA = reinterpret_cast<Key<W> *>(s_raw);          // [kEmitStep]
    Key<W> *sB = sA + kEmitStep;                              // [kEmitStep + 1], sB[0]: the set key before the window
    int64_t *s_cut = reinterpret_cast<int64_t *>(sB + kEmitStep + 1);  // [kCutBatch]
    const int wv = threadIdx.x / kWave;
    const int64_t n_win = ceil_div_dev(total, kEmitStep);
    int64_t i0 = 0;  // run keys consumed by earlier windows
    for (int64_t w0 = 0; w0 < n_win; w0 += kCutBatch) {
        const int nw = (int)(n_win - w0 < kCutBatch ? n_win - w0 : kCutBatch);
        for (int q = wv; q < nw; q += kDWaves) {
            const int64_t c1 = (w0 + q + 1) * kEmitStep < total ? (w0 + q + 1) * kEmitStep : total;
            const int64_t cut = (c1 == total) ? nA : wave_merge_path<W>(A, nA, Bs, nBs, c1);
            if ((threadIdx.x & (kWave - 1)) == 0) s_cut[q] = cut;
        }
        __syncthreads();
        for (int qw = 0; qw < nw; ++qw) {
            const int64_t c0 = (w0 + qw) * kEmitStep;
            const int64_t c1 = c0 + kEmitStep < total ? c0 + kEmitStep : total;
            // A split search returns a cut in [max(0, c1 - nBs), min(c1, nA)] for any data,
            // and for sorted inputs consecutive cuts differ by 0..win.  Clamping to that
            // step keeps na, nb in [0, win] (the LDS window) and every load in range
            // even when an unsorted set (flagged by the order check) breaks monotony;
            // for sorted inputs it changes nothing.
            const int64_t win64 = c1 - c0;
            int64_t i1 = s_cut[qw];
            i1 = i1 < i0 ? i0 : (i1 > i0 + win64 ? i0 + win64 : i1);
            const int64_t j0 = c0 - i0;
            const int na = (int)(i1 - i0), nb = (int)((c1 - i1) - j0);
            for (int t = threadIdx.x; t < na; t += kDThreads) sA[t] = load_key<W>(A, i0 + t);
            for (int t = threadIdx.x; t <= nb; t += kDThreads)
                if (t > 0 || j0 > 0) sB[t] = load_key<W>(Bs, j0 - 1 + t);
            __syncthreads();
            const int p0 = threadIdx.x * kMergePer;
            const int win = (int)(c1 - c0);
            const int cnt = p0 < win ? (win - p0 < kMergePer ? win - p0 : kMergePer) : 0;
            Key<W> vals[kMergePer];
            uint32_t fa = 0, fd = 0;
            if (cnt > 0) {
                // run keys among this window's first p0 outputs (ties: set key first)
                int lo = p0 > nb ? p0 - nb : 0, hi = p0 < na ? p0 : na;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (key_less<W>(sA[mid], sB[p0 - mid])) lo = mid + 1;
                    else hi = mid;
                }
                int i = lo, j = p0 - lo;
    #pragma unroll
                for (int q = 0; q < kMergePer; ++q) {
                    if (q < cnt) {
                        const bool takeA = i < na && (j >= nb || key_less<W>(sA[i], sB[1 + j]));
                        if (takeA) {
                            const Key<W> x = sA[i];
                            vals[q] = x;
                            fa |= 1u << q;
                            // equal to the set key emitted just before it: already in the union
                            if (j0 + j > 0 && key_eq<W>(sB[j], x)) fd |= 1u << q;
                            ++i;
                        } else {
                            vals[q] = sB[1 + j];
                            ++j;
                        }
                    }
                }
            }
            int lu = 0, ln = 0;
    #pragma unroll
            for (int q = 0; q < kMergePer; ++q) {
                const bool dup = (fd >> q) & 1u, fromA = (fa >> q) & 1u;
                lu += (q < cnt) && !dup;
                ln += (q < cnt) && fromA && !dup;
            }
            int64_t tu, tn;
            const int64_t eu = block_excl_scan_i64(lu, &tu, wsum);
            const int64_t en = block_excl_scan_i64(ln, &tn, wsum);
            int64_t pu = ou + eu, pn = on + en;
    #pragma unroll
            for (int q = 0; q < kMergePer; ++q) {
                const bool dup = (fd >> q) & 1u, fromA = (fa >> q) & 1u;
                if (q >= cnt || dup) continue;
                if (pu < a.out_cap) store_key<W>(a.out, pu, vals[q]);
                ++pu;
                if (fromA) {
                    if (a.novel && pn < a.novel_cap) store_key<W>(a.novel, pn, vals[q]);
                    ++pn;
                }
            }
            ou += tu;
            on += tn;
            i0 = i1;
            __syncthreads();  // the next window overwrites sA / sB (and the next batch s_cut)
        }
    }
}

// empty candidate list: the union is the set itself
template <int W>
__global__ void copy_keys_kernel(const uint64_t *B, const int64_t *nB, uint64_t *out, int64_t cap) {
    const int64_t n = nB ? *nB : 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n && i < cap;
         i += (int64_t)gridDim.x * blockDim.x)
        store_key<W>(out, i, load_key<W>(B, i));
}

__global__ void finish_counts_kernel(const int64_t *total_u, const int64_t *total_n, int64_t *n_out, int64_t out_cap,
                                     int64_t *n_novel, int64_t novel_cap, int novel_given, uint32_t *flags) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t u = *total_u;
    *n_out = u;
    if (u > out_cap) atomicOr(flags, SCI_FLAG_OVERFLOW);
    if (n_novel) {
        *n_novel = *total_n;
        if (novel_given && *total_n > novel_cap) atomicOr(flags, SCI_FLAG_OVERFLOW);
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
    size_t bufA, bufB, ids, segA, segB, fan1, fan2, spl1, spl2, tile_base, cbase, counts, sums, samples;
    size_t nuniq, bstart, bcount, ucount, ncount, big, big2, ufirst, uend, ucnt, scal;
    size_t total;
    int64_t max_counts, max_sums, n_final_slots;
};

static size_t al256(size_t b) { return (b + 255) / 256 * 256; }

template <int W>
static WsLayout ws_layout(int64_t n, bool cand_scratch = false) {
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
    L.bufB = cand_scratch ? 0 : take((size_t)nn * W * 8);
    L.ids = take((size_t)nn * 2);
    L.segA = take((size_t)(S2 + 1) * 8);
    L.segB = take((size_t)(S2 + 1) * 8);
    L.fan1 = take(64);
    L.fan2 = take((size_t)S1 * 4);
    L.spl1 = take((size_t)C::F1 * W * 8);
    L.spl2 = take((size_t)S1 * C::F2 * W * 8);
    L.tile_base = take((size_t)(S1 + 1) * 8);
    L.cbase = take((size_t)(S1 + 1) * 8);
    L.counts = take((size_t)L.max_counts * 8);
    L.sums = take((size_t)L.max_sums * 8);
    L.samples = take((size_t)C::M1 * W * 8);
    L.nuniq = take((size_t)S2 * 8);
    L.bstart = take((size_t)S2 * 8);
    L.bcount = take((size_t)S2 * 8);
    L.ucount = take((size_t)(S2 + 1) * 8);
    L.ncount = take((size_t)(S2 + 1) * 8);
    L.big = take((size_t)S2 * 8);
    L.big2 = take((size_t)S2 * 8);
    L.ufirst = take((size_t)(S2 + 1) * 4);
    L.uend = take((size_t)(S2 + 1) * 4);
    L.ucnt = take((size_t)(S1 + 2) * 8);
    L.scal = take(64);
    L.total = off;
    return L;
}

int64_t device_scan_sums(int64_t n_bound) { return ceil_div(std::max<int64_t>(n_bound, 1), kScanPer) + 1; }

hipError_t device_scan(int64_t *x, const int64_t *n_dev, int64_t n_bound, int64_t *sums, int64_t *total_out,
                       hipStream_t st) {
    const int64_t nb = std::max<int64_t>(1, ceil_div(n_bound, kScanPer));
    SCI_LAUNCH(scan_reduce_kernel, dim3((unsigned)nb), dim3(kDThreads), 0, st, (const int64_t *)x, n_dev, n_bound, sums);
    SCI_LAUNCH(scan_sums_kernel, dim3(1), dim3(kDThreads), 0, st, sums, nb, total_out);
    SCI_LAUNCH(scan_apply_kernel, dim3((unsigned)nb), dim3(kDThreads), 0, st, x, n_dev, n_bound, (const int64_t *)sums);
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
                          int64_t *n_novel, int64_t novel_cap, char *ws, uint32_t *flags, hipStream_t st,
                          bool check_set, bool cand_scratch, hipEvent_t after_split) {
    using C = DCfg<W>;
    bool split_marked = false;
    auto mark_split = [&]() -> hipError_t {
        if (!after_split || split_marked) return hipSuccess;
        split_marked = true;
        return hipEventRecord(after_split, st);
    };
    const WsLayout L = ws_layout<W>(n, cand_scratch);
    uint64_t *bufA = (uint64_t *)(ws + L.bufA);
    // the second level writes over the candidates when they may be overwritten
    uint64_t *bufB = cand_scratch ? const_cast<uint64_t *>(cand) : (uint64_t *)(ws + L.bufB);
    int64_t *segA = (int64_t *)(ws + L.segA);
    int64_t *segB = (int64_t *)(ws + L.segB);
    int64_t *counts = (int64_t *)(ws + L.counts);
    int64_t *sums = (int64_t *)(ws + L.sums);
    // [0] union total, [1] novel total, [2] level counters, [3] oversized units, [4] units, [5] units + 1
    int64_t *scal = (int64_t *)(ws + L.scal);
    int dev = 0, n_cu_i = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&n_cu_i, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t n_cu = std::max(n_cu_i, 1);
    const bool have_set = set_in && n_set_in;

    if (have_set && check_set)
        SCI_LAUNCH(check_sorted_kernel<W>, dim3(1024), dim3(256), 0, st, set_in, n_set_in, flags);
    if (n == 0) {
        SCI_LAUNCH(copy_keys_kernel<W>, dim3(4096), dim3(256), 0, st, set_in, have_set ? n_set_in : nullptr, set_out,
                   set_cap);
        if (have_set) {
            SCI_HIP_TRY(launch_set_i64(scal + 1, 0, st));
            SCI_LAUNCH(finish_counts_kernel, dim3(1), dim3(64), 0, st, n_set_in, (const int64_t *)(scal + 1),
                       n_set_out, set_cap, n_novel, novel_cap, novel ? 1 : 0, flags);
        } else {
            SCI_HIP_TRY(launch_set_i64(n_set_out, 0, st));
            if (n_novel) SCI_HIP_TRY(launch_set_i64(n_novel, 0, st));
        }
        SCI_HIP_TRY(mark_split());
        return SCI_OK;
    }

    BucketArgs b{};
    b.ufirst = (const int32_t *)(ws + L.ufirst);
    b.uend = (const int32_t *)(ws + L.uend);
    b.n_units = scal + 4;
    b.ucount = (int64_t *)(ws + L.ucount);
    b.ncount = (int64_t *)(ws + L.ncount);
    b.fan1 = (const int32_t *)(ws + L.fan1);
    b.fan2 = (const int32_t *)(ws + L.fan2);
    b.F2 = C::F2;
    SCI_LAUNCH(init_level0_kernel, dim3(1), dim3(64), 0, st, segA, n);
    if (n <= C::CAP) {
        b.src = cand;  // one bucket: read only
        b.seg = segA;
        b.n_slots = 1;
        b.two_level = 0;
        SCI_LAUNCH(single_unit_kernel, dim3(1), dim3(64), 0, st, b, scal + 5);
    } else {
        const uint64_t *cur = cand;
        const int64_t *seg_cur = segA;
        int S_cur = 1;
        for (int lvl = 0; lvl < 2; ++lvl) {
            LevelArgs a{};
            a.in = cur;
            a.out = (lvl == 0) ? bufA : bufB;
            a.ids = (uint16_t *)(ws + L.ids);
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
                a.fan = (int32_t *)(ws + L.fan1);
                a.spl = (uint64_t *)(ws + L.spl1);
            } else {
                a.target = C::TARGET;
                a.ovs = C::OVS2;
                a.max_samples = C::MS2;
                a.fan = (int32_t *)(ws + L.fan2);
                a.spl = (uint64_t *)(ws + L.spl2);
            }
            a.tile_base = (int64_t *)(ws + L.tile_base);
            a.cbase = (int64_t *)(ws + L.cbase);
            a.counts = counts;
            a.sample_buf = (uint64_t *)(ws + L.samples);
            const int64_t tiles_bound = ceil_div(n, a.tile) + S_cur;
            a.max_tiles = tiles_bound;
            // the fan-out and sample count of the single level-1 segment are known here
            int64_t n_smp = 0;
            int fan0 = 1;
            if (lvl == 0) {
                fan0 = (int)std::min<int64_t>((int64_t)a.F, std::max<int64_t>(1, ceil_div_dev(n, a.target)));
                n_smp = std::min<int64_t>(n, std::min<int64_t>((int64_t)a.ovs * fan0, a.max_samples));
            }
            if (lvl == 0 && fan0 > 1 && n_smp > C::CAP) {
                SCI_LAUNCH(sample_runs_kernel<W>, dim3((unsigned)ceil_div(n_smp, C::CAP)), dim3(kDThreads), 0, st, a,
                           n, n_smp, fan0);
                SCI_LAUNCH(sample_rank_kernel<W>, dim3((unsigned)ceil_div(n_smp, kDThreads)), dim3(kDThreads), 0, st,
                           a, n_smp, fan0);
            } else {
                SCI_LAUNCH(splitter_kernel<W>, dim3(S_cur), dim3(kDThreads), 0, st, a);
            }
            if (lvl == 0) SCI_HIP_TRY(mark_split());
            SCI_LAUNCH(plan_kernel, dim3(1), dim3(kDThreads), 0, st, a);
            if (lvl == 0) {
                SCI_LAUNCH((hist_kernel<W, C::F1>), dim3((unsigned)tiles_bound), dim3(kHThreads), 0, st, a);
            } else {
                SCI_LAUNCH((hist_kernel<W, C::F2>), dim3((unsigned)tiles_bound), dim3(kHThreads), 0, st, a);
            }
            SCI_HIP_TRY(hipGetLastError());
            // exclusive scan of all counters -> absolute output offsets
            const int64_t cbound = tiles_bound * (int64_t)a.F;
            SCI_HIP_TRY(device_scan(counts, a.cbase + S_cur, cbound, sums, scal + 2, st));
            if (lvl == 0) {
                SCI_LAUNCH((scatter_kernel<W, C::F1>), dim3((unsigned)std::min<int64_t>(tiles_bound, n_cu)),
                           dim3(kSThreads), 0, st, a);
            } else {
                SCI_LAUNCH((scatter_kernel<W, C::F2>), dim3((unsigned)std::min<int64_t>(tiles_bound, n_cu)),
                           dim3(kSThreads), 0, st, a);
            }
            const int64_t slots = (int64_t)S_cur * a.F;
            SCI_LAUNCH(next_segments_kernel, dim3((unsigned)ceil_div(slots + 1, 256)), dim3(256), 0, st, a, n);
            SCI_HIP_TRY(hipGetLastError());
            cur = a.out;
            seg_cur = a.seg_out;
            S_cur = (int)slots;
        }
        b.src = bufB;
        b.seg = segA;  // level-2 output segments
        b.n_slots = S_cur;
        b.two_level = 1;
        // group consecutive buckets into units of at most CAP keys
        int64_t *ucnt = (int64_t *)(ws + L.ucnt);
        const unsigned pg = (unsigned)ceil_div(C::F1 + 1, 256);
        SCI_LAUNCH((pack_units_kernel<W, 0>), dim3(pg), dim3(256), 0, st, b, (int)C::F1, ucnt, scal + 5);
        SCI_HIP_TRY(device_scan(ucnt, nullptr, C::F1 + 1, sums, scal + 4, st));
        SCI_LAUNCH((pack_units_kernel<W, 1>), dim3(pg), dim3(256), 0, st, b, (int)C::F1, ucnt, scal + 5);
    }
    b.dst = bufA;
    b.spl1 = (const uint64_t *)(ws + L.spl1);
    b.spl2 = (const uint64_t *)(ws + L.spl2);
    b.B = have_set ? set_in : nullptr;
    b.nB = have_set ? n_set_in : nullptr;
    b.nuniq = (int64_t *)(ws + L.nuniq);
    b.bstart = (int64_t *)(ws + L.bstart);
    b.bcount = (int64_t *)(ws + L.bcount);
    SCI_LAUNCH(set_range_kernel<W>, dim3((unsigned)ceil_div(b.n_slots, 256)), dim3(256), 0, st, b);
    b.n_big = scal + 3;
    b.big = (int64_t *)(ws + L.big);
    b.n_big2 = scal + 6;
    b.big2 = (int64_t *)(ws + L.big2);
    SCI_HIP_TRY(launch_set_i64(b.n_big, 0, st));
    SCI_HIP_TRY(launch_set_i64(b.n_big2, 0, st));
    SCI_LAUNCH(bucket_kernel<W>, dim3((unsigned)b.n_slots), dim3(kBThreads), 0, st, b);
    SCI_LAUNCH(bucket_stream_kernel<W>, dim3((unsigned)n_cu), dim3(kBThreads), 0, st, b);
    SCI_LAUNCH(bucket_big_kernel<W>, dim3(4096), dim3(kDThreads), 0, st, b);
    SCI_HIP_TRY(hipGetLastError());
    SCI_HIP_TRY(device_scan(b.ucount, scal + 5, b.n_slots + 1, sums, scal + 0, st));
    SCI_HIP_TRY(device_scan(b.ncount, scal + 5, b.n_slots + 1, sums, scal + 1, st));
    EmitArgs e{};
    e.runs = bufA;
    e.seg = b.seg;
    e.ufirst = b.ufirst;
    e.n_units = b.n_units;
    e.nuniq = b.nuniq;
    e.bstart = b.bstart;
    e.bcount = b.bcount;
    e.uoff = b.ucount;
    e.noff = b.ncount;
    e.B = b.B;
    e.out = set_out;
    e.out_cap = set_cap;
    e.novel = novel;
    e.novel_cap = novel_cap;
    SCI_LAUNCH(emit_kernel<W>, dim3((unsigned)b.n_slots), dim3(kDThreads), 0, st, e);
    SCI_LAUNCH(finish_counts_kernel, dim3(1), dim3(64), 0, st, (const int64_t *)(scal + 0),
               (const int64_t *)(scal + 1), n_set_out, set_cap, n_novel, novel_cap, novel ? 1 : 0, flags);
    SCI_HIP_TRY(hipGetLastError());
    SCI_HIP_TRY(mark_split());
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

namespace sci {

// Workspace of one dedup call; with cand_scratch the candidate buffer itself takes the
// second partition level's output (the streaming loop's pool chunk, free once the
// first level has read it), so one key buffer fewer is needed.
size_t dedup_ws_bytes(int32_t n_words, int64_t n_cand, bool cand_scratch) {
    if (n_cand < 0) return 0;
    if (n_words == 1) return ws_layout<1>(n_cand, cand_scratch).total;
    if (n_words == 2) return ws_layout<2>(n_cand, cand_scratch).total;
    return 0;
}

// sci_dedup_merge with the strict-order check of set_in optional (callers that pass a
// set this library produced skip the extra pass over it) and, for callers that own
// the candidate buffer, its reuse as scratch.
int32_t dedup_merge_checked(int32_t n_words, const uint64_t *cand, int64_t n_cand, const uint64_t *set_in,
                            const int64_t *n_set_in, uint64_t *set_out, int64_t *n_set_out, int64_t set_capacity,
                            uint64_t *novel, int64_t *n_novel, int64_t novel_capacity, void *workspace,
                            size_t workspace_bytes, uint32_t *dev_flags, hipStream_t st, bool check_set_in,
                            bool cand_scratch, hipEvent_t after_split) {
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
    const size_t need = dedup_ws_bytes(n_words, n_cand, cand_scratch);
    if (workspace_bytes < need)
        return fail(SCI_ECAPACITY, "sci_dedup_merge: workspace %zu < %zu bytes", workspace_bytes, need);
    if (n_words == 1)
        return dedup_impl<1>(cand, n_cand, set_in, n_set_in, set_out, n_set_out, set_capacity, novel, n_novel,
                             novel_capacity, (char *)workspace, dev_flags, st, check_set_in, cand_scratch,
                             after_split);
    return dedup_impl<2>(cand, n_cand, set_in, n_set_in, set_out, n_set_out, set_capacity, novel, n_novel,
                         novel_capacity, (char *)workspace, dev_flags, st, check_set_in, cand_scratch, after_split);
}

}  // namespace sci

extern "C" int32_t sci_dedup_merge(int32_t n_words, const uint64_t *cand, int64_t n_cand, const uint64_t *set_in,
                                   const int64_t *n_set_in, uint64_t *set_out, int64_t *n_set_out,
                                   int64_t set_capacity, uint64_t *novel, int64_t *n_novel, int64_t novel_capacity,
                                   void *workspace, size_t workspace_bytes, uint32_t *dev_flags,
                                   sci_stream_t stream) {
    return sci::dedup_merge_checked(n_words, cand, n_cand, set_in, n_set_in, set_out, n_set_out, set_capacity, novel,
                                    n_novel, novel_capacity, workspace, workspace_bytes, dev_flags,
                                    (hipStream_t)stream, true);
}
