// Internal definitions shared by the HIP translation units of libsci.
// Device code targets gfx950 (CDNA4): 64-lane wavefronts, 160 KiB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <new>
#include <stdexcept>
#include <string>

#include "sci.h"

namespace sci {

constexpr int kWave = 64;

// Workgroups are dispatched to the 8 XCDs of the chip in turn, and each XCD has its
// own L2.  Workgroup b (on XCD b % 8) of n gets index x*q + min(x, r) + b/8, with
// q, r = n / 8, n % 8: every XCD takes one contiguous range of [0, n).  The map is a
// bijection on [0, n) whatever the dispatch order.
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_local_block(int64_t b, int64_t n) {
    const int64_t x = b % kXcds, q = n / kXcds, r = n % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

// ---------------------------------------------------------------------------
// Hamiltonian handle: integrals and the tables the kernels read, all device.
// ---------------------------------------------------------------------------
struct HamDev {
    int n_orb, n_alpha, n_beta, W;
    int v_alpha, v_beta;
    int64_t n_coupled;
    // class boundaries of the per-source rank space:
    //   [0,c1) alpha singles, [c1,c2) beta singles, [c2,c3) alpha-alpha,
    //   [c3,c4) beta-beta, [c4,n_coupled) alpha-beta
    int64_t c1, c2, c3, c4;
    const double *h1;    // [n][n]
    const double *eri;   // [n][n][n][n] chemists' (pq|rs)
    const double *vdir;  // [p][q][a][b] = (ap|bq)
    const double *vanti; // [p][q][a][b] = (ap|bq) - (aq|bp)
    const double *jmat;  // [p][q] = (pp|qq)
    const double *kmat;  // [p][q] = (pq|qp)
    const double *jtpq;  // [t][p][q] = (tp|qq): the Coulomb sum of a single t <- p is a row over q
    const double *ktpq;  // [t][p][q] = (tq|qp): its exchange sum, also a row over q
    // [s][t][p]: the single t <- p (spin s) on the reference determinant (the lowest
    // n_alpha alpha and n_beta beta orbitals), h_tp + sum_{Q occ} [(tp|qq) - d_s (tq|qp)]
    const double *fref;
    // lexicographic pairs (i<j) of m items as i | j<<8, for m = n_alpha,
    // n_beta, v_alpha, v_beta (index 0..3)
    const uint16_t *pairs[4];
};

}  // namespace sci

struct sci_ham_s {
    sci::HamDev dev;
    void *block;  // single device allocation holding every table
};

namespace sci {

// enqueue *p = v with a one-thread kernel (no memset node, so graph-safe)
hipError_t launch_set_i64(int64_t *p, int64_t v, hipStream_t st);
hipError_t launch_set_u32(uint32_t *p, uint32_t v, hipStream_t st);

// optional per-launch timing (sci_profile_enable): events around each launch
struct ProfScope {
    ProfScope(const char *name, hipStream_t st);
    ~ProfScope();
    hipStream_t st;
    int slot;
};

// every kernel launch of the library goes through this (timing when enabled)
#define SCI_LAUNCH(kern, grid, block, shm, st, ...)                 \
    do {                                                            \
        ::sci::ProfScope sci_prof_scope_(#kern, (st));              \
        hipLaunchKernelGGL(kern, grid, block, shm, st, __VA_ARGS__); \
    } while (0)

// thread-local last-error text
void set_error(const char *fmt, ...);
int32_t fail(int32_t status, const char *fmt, ...);

// Runs the body of a C entry point that allocates host memory: no C++ exception
// crosses the C ABI.  An exhausted or oversized host allocation (std::bad_alloc,
// std::length_error) and anything else thrown become SCI_ENOMEM with the entry
// point's name in the last-error text.  The body cleans up what it owns (RAII).
template <typename F>
int32_t guarded(const char *where, F &&body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return fail(SCI_ENOMEM, "%s: host allocation failed", where);
    } catch (const std::length_error &) {
        return fail(SCI_ENOMEM, "%s: host allocation too large", where);
    } catch (...) {
        return fail(SCI_ENOMEM, "%s: unexpected host exception", where);
    }
}

#define SCI_HIP_TRY(expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return ::sci::fail(SCI_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

// ---------------------------------------------------------------------------
// multi-word keys
// ---------------------------------------------------------------------------
template <int W>
struct Key {
    uint64_t w[W];
};

template <int W>
__device__ __forceinline__ bool key_less(const Key<W> &a, const Key<W> &b) {
#pragma unroll
    for (int i = W - 1; i >= 0; --i) {
        if (a.w[i] != b.w[i]) return a.w[i] < b.w[i];
    }
    return false;
}

template <int W>
__device__ __forceinline__ bool key_eq(const Key<W> &a, const Key<W> &b) {
    bool e = true;
#pragma unroll
    for (int i = 0; i < W; ++i) e = e && (a.w[i] == b.w[i]);
    return e;
}

template <int W>
__device__ __forceinline__ Key<W> load_key(const uint64_t *p, int64_t i) {
    Key<W> k;
    if constexpr (W == 2) {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(p + 2 * i);
        k.w[0] = v.x;
        k.w[1] = v.y;
    } else {
#pragma unroll
        for (int j = 0; j < W; ++j) k.w[j] = p[W * i + j];
    }
    return k;
}

template <int W>
__device__ __forceinline__ void store_key(uint64_t *p, int64_t i, const Key<W> &k) {
    if constexpr (W == 2) {
        ulonglong2 v;
        v.x = k.w[0];
        v.y = k.w[1];
        *reinterpret_cast<ulonglong2 *>(p + 2 * i) = v;
    } else {
#pragma unroll
        for (int j = 0; j < W; ++j) p[W * i + j] = k.w[j];
    }
}

template <int W>
__device__ __forceinline__ void key_flip(Key<W> &k, int bit) {
    if constexpr (W == 1) {
        k.w[0] ^= 1ull << bit;
    } else {
#pragma unroll
        for (int j = 0; j < W; ++j) k.w[j] ^= ((bit >> 6) == j) ? (1ull << (bit & 63)) : 0ull;
    }
}

template <int W>
__device__ __forceinline__ int key_popc(const Key<W> &k) {
    int c = 0;
#pragma unroll
    for (int j = 0; j < W; ++j) c += __popcll(k.w[j]);
    return c;
}

// number of set bits of k strictly below bit position `bit`
template <int W>
__device__ __forceinline__ int key_popc_below(const Key<W> &k, int bit) {
    int c = 0;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const int lo = 64 * j;
        uint64_t m;
        if (bit >= lo + 64) m = ~0ull;
        else if (bit <= lo) m = 0ull;
        else m = (1ull << (bit - lo)) - 1ull;
        c += __popcll(k.w[j] & m);
    }
    return c;
}

// popcounts of the alpha (bits [0,n)) and beta (bits [n,2n)) blocks
template <int W>
__device__ __forceinline__ void spin_popc(const Key<W> &k, int n, int &na, int &nb) {
    const int below_n = key_popc_below<W>(k, n);
    const int below_2n = key_popc_below<W>(k, 2 * n);
    na = below_n;
    nb = below_2n - below_n;
}

// ---------------------------------------------------------------------------
// fast exact division for 0 <= x < 2^24 by a positive divisor < 2^24
// ---------------------------------------------------------------------------
struct FastDiv {
    uint32_t d;
    float rcp;
};

inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d ? d : 1;
    f.rcp = 1.0f / (float)f.d;
    return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t x, const FastDiv &f, uint32_t &rem) {
    // float estimate is within one of the true quotient for x, d < 2^24
    int q = (int)((float)x * f.rcp);
    int r = (int)x - q * (int)f.d;
    if (r < 0) { q -= 1; r += (int)f.d; }
    if (r >= (int)f.d) { q += 1; r -= (int)f.d; }
    rem = (uint32_t)r;
    return (uint32_t)q;
}

inline int64_t comb2(int64_t x) { return x * (x - 1) / 2; }

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// lanes below this one in the wavefront
__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = threadIdx.x & (kWave - 1);
    return lane ? ((~0ull) >> (64 - lane)) : 0ull;
}

// Device-wide exclusive scan of int64 x[0..n), n = *n_dev when n_dev is given, else
// n_bound; sums holds device_scan_sums(n_bound) entries; *total_out (nullable) gets the sum.
hipError_t device_scan(int64_t *x, const int64_t *n_dev, int64_t n_bound, int64_t *sums, int64_t *total_out,
                       hipStream_t st);
int64_t device_scan_sums(int64_t n_bound);

// sci_dedup_merge, with the strict-order check of set_in optional; with cand_scratch
// the candidate buffer is overwritten (the caller owns it); after_split, when given,
// is recorded on st once the first partition level's splitters are chosen (or, on
// paths without them, before the call returns)
int32_t dedup_merge_checked(int32_t n_words, const uint64_t *cand, int64_t n_cand, const uint64_t *set_in,
                            const int64_t *n_set_in, uint64_t *set_out, int64_t *n_set_out, int64_t set_capacity,
                            uint64_t *novel, int64_t *n_novel, int64_t novel_capacity, void *workspace,
                            size_t workspace_bytes, uint32_t *dev_flags, hipStream_t st, bool check_set_in,
                            bool cand_scratch = false, hipEvent_t after_split = nullptr);
size_t dedup_ws_bytes(int32_t n_words, int64_t n_cand, bool cand_scratch);
__host__ __device__ inline int64_t ceil_div_dev(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace sci
