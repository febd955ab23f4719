// Coupled-configuration generation (paper section 4.2, Algorithm 1; Eq. 4).
//
// One workgroup takes one (source, rank chunk) tile.  The source determinant
// is decoded once into LDS: occupied / empty orbital lists per spin, the count
// of occupied orbitals below every orbital (for fermionic signs), and the
// lexicographic pair lists used to unrank double excitations.  Every lane
// then maps its rank to (class, p, q, a, b), flips bits of the source to form
// the new key, reads one integral-table entry for a double (or sums the
// occupied-orbital terms for a single), applies the sign and writes key and
// H_ij with unit-stride stores (one wave writes 64 consecutive entries).
//
// Unlike the paper's padded virtual-thread space (Eqs. 6-7), ranks cover only
// valid excitations, so dense mode needs no compaction and its output order is
// fixed.  Screened mode (eps >= 0) keeps |H| > eps and compacts with a wave
// ballot and one atomic per workgroup iteration (the paper's block-wide
// compaction with a single atomicAdd per block).
#include "sci_internal.hpp"

namespace sci {

constexpr int kGenThreads = 256;
constexpr int kMaxPairs = 64 * 63 / 2;

struct GenArgs {
    // system
    int n, na, nb, va, vb;
    int c1, c2, c3, c4, nc;
    const double *h1, *eri, *vdir, *vanti;
    const uint16_t *pairs[4];
    // tiles
    const uint64_t *dets;
    int64_t src_first;
    int chunk, chunks_per_src;
    int64_t exc_begin, exc_end;
    // outputs
    uint64_t *keys;
    double *hij;
    int32_t *src_out;
    int64_t capacity;
    unsigned long long *n_out;
    uint32_t *flags;
    double eps;
    // fast division
    FastDiv d_va, d_vb, d_nb, d_vab, d_pva, d_pvb;
};

struct GenLds {
    uint8_t occ[2][64];
    uint8_t vir[2][64];
    uint8_t below[2][64];  // occupied orbitals of the same spin strictly below p
    uint16_t pocc[2][kMaxPairs];
    uint16_t pvir[2][kMaxPairs];
    int bad;
    int wave_tot[kGenThreads / kWave];
    unsigned long long slab;
};

__device__ __forceinline__ void copy_pairs(uint16_t *dst, const uint16_t *src, int m, int tid) {
    const int total = m * (m - 1) / 2;
    for (int t = tid; t < total; t += kGenThreads) dst[t] = src[t];
}

template <int W>
__device__ __forceinline__ void gen_one(const GenArgs &a, const GenLds &L, const Key<W> &src, int r,
                                        Key<W> &key, double &h) {
    const int n = a.n;
    key = src;
    if (r < a.c2) {
        // single excitation p -> a within one spin
        const int sg = r < a.c1 ? 0 : 1;
        const uint32_t x = (uint32_t)(sg ? r - a.c1 : r);
        uint32_t ia;
        const uint32_t ip = fdiv(x, sg ? a.d_vb : a.d_va, ia);
        const int p = L.occ[sg][ip];
        const int t = L.vir[sg][ia];
        const int off = sg * n;
        key_flip<W>(key, p + off);
        key_flip<W>(key, t + off);
        const int par = L.below[sg][p] + L.below[sg][t] - (p < t ? 1 : 0);
        // h_ap + sum over occupied Q != P of [(ap|qq) - delta_spin (aq|qp)], Q ascending
        double v = a.h1[t * n + p];
        const int nocc0 = a.na, nocc1 = a.nb;
        for (int s2 = 0; s2 < 2; ++s2) {
            const int cnt = s2 ? nocc1 : nocc0;
            for (int k = 0; k < cnt; ++k) {
                const int q = L.occ[s2][k];
                if (s2 == sg && q == p) continue;
                const double j = a.eri[((int64_t)(t * n + p) * n + q) * n + q];
                const double kx = (s2 == sg) ? a.eri[((int64_t)(t * n + q) * n + q) * n + p] : 0.0;
                v += j - kx;
            }
        }
        h = (par & 1) ? -v : v;
    } else if (r < a.c4) {
        // same-spin double p<q -> a<b
        const int sg = r < a.c3 ? 0 : 1;
        const uint32_t x = (uint32_t)(r - (sg ? a.c3 : a.c2));
        uint32_t tv;
        const uint32_t o = fdiv(x, sg ? a.d_pvb : a.d_pva, tv);
        const uint16_t po = L.pocc[sg][o];
        const uint16_t pv = L.pvir[sg][tv];
        const int p = L.occ[sg][po & 0xff], q = L.occ[sg][po >> 8];
        const int ta = L.vir[sg][pv & 0xff], tb = L.vir[sg][pv >> 8];
        const int off = sg * n;
        key_flip<W>(key, p + off);
        key_flip<W>(key, q + off);
        key_flip<W>(key, ta + off);
        key_flip<W>(key, tb + off);
        const int par = L.below[sg][p] + L.below[sg][q] - 1 + L.below[sg][tb] - (p < tb) - (q < tb) +
                        L.below[sg][ta] - (p < ta) - (q < ta);
        const double v = a.vanti[((int64_t)(p * n + q) * n + ta) * n + tb];
        h = (par & 1) ? -v : v;
    } else {
        // alpha-beta double p(alpha) q(beta) -> a(alpha) b(beta)
        const uint32_t x = (uint32_t)(r - a.c4);
        uint32_t t;
        const uint32_t o = fdiv(x, a.d_vab, t);
        uint32_t iq, ib;
        const uint32_t ip = fdiv(o, a.d_nb, iq);
        const uint32_t ia = fdiv(t, a.d_vb, ib);
        const int p = L.occ[0][ip], q = L.occ[1][iq];
        const int ta = L.vir[0][ia], tb = L.vir[1][ib];
        key_flip<W>(key, p);
        key_flip<W>(key, ta);
        key_flip<W>(key, q + n);
        key_flip<W>(key, tb + n);
        const int par = L.below[0][p] + L.below[0][ta] - (p < ta) + L.below[1][q] + L.below[1][tb] - (q < tb);
        const double v = a.vdir[((int64_t)(p * n + q) * n + ta) * n + tb];
        h = (par & 1) ? -v : v;
    }
}

template <int W, bool DENSE>
__global__ __launch_bounds__(kGenThreads) void gen_kernel(GenArgs a) {
    __shared__ GenLds L;
    const int tid = threadIdx.x;
    const int64_t src = a.src_first + blockIdx.x / a.chunks_per_src;
    const int chunk_id = blockIdx.x % a.chunks_per_src;
    const int64_t flat0 = src * a.nc;
    int64_t lo = flat0 + (int64_t)chunk_id * a.chunk;
    int64_t hi = lo + a.chunk;
    if (hi > flat0 + a.nc) hi = flat0 + a.nc;
    if (lo < a.exc_begin) lo = a.exc_begin;
    if (hi > a.exc_end) hi = a.exc_end;
    if (lo >= hi) return;  // uniform per workgroup

    const Key<W> s = load_key<W>(a.dets, src);
    const int n = a.n;
    if (tid == 0) {
        int na, nb;
        spin_popc<W>(s, n, na, nb);
        const int tot = key_popc<W>(s);
        L.bad = (na != a.na || nb != a.nb || tot != na + nb) ? 1 : 0;
    }
    if (tid < 2 * n) {
        const int sg = tid >= n ? 1 : 0;
        const int p = tid - sg * n;
        const int k = tid;
        const int below_all = key_popc_below<W>(s, k);
        const int below_same = sg ? below_all - key_popc_below<W>(s, n) : below_all;
        const bool occ = (s.w[k >> 6] >> (k & 63)) & 1ull;
        L.below[sg][p] = (uint8_t)below_same;
        if (occ) {
            if (below_same < 64) L.occ[sg][below_same] = (uint8_t)p;
        } else {
            const int e = p - below_same;
            if (e >= 0 && e < 64) L.vir[sg][e] = (uint8_t)p;
        }
    }
    copy_pairs(L.pocc[0], a.pairs[0], a.na, tid);
    copy_pairs(L.pocc[1], a.pairs[1], a.nb, tid);
    copy_pairs(L.pvir[0], a.pairs[2], a.va, tid);
    copy_pairs(L.pvir[1], a.pairs[3], a.vb, tid);
    __syncthreads();

    const bool bad = L.bad != 0;
    if (bad && tid == 0) atomicOr(a.flags, SCI_FLAG_BAD_DET);
    const int r_lo = (int)(lo - flat0), r_hi = (int)(hi - flat0);

    if constexpr (DENSE) {
        for (int r = r_lo + tid; r < r_hi; r += kGenThreads) {
            Key<W> key;
            double h;
            if (!bad) {
                gen_one<W>(a, L, s, r, key, h);
            } else {
#pragma unroll
                for (int j = 0; j < W; ++j) key.w[j] = 0;
                h = 0.0;
            }
            const int64_t o = flat0 + r - a.exc_begin;
            store_key<W>(a.keys, o, key);
            a.hij[o] = h;
            if (a.src_out) a.src_out[o] = (int32_t)src;
        }
    } else {
        if (bad) return;
        const int lane = tid & (kWave - 1), wid = tid / kWave;
        // iterate with a uniform trip count so every lane reaches the barriers
        for (int base = r_lo; base < r_hi; base += kGenThreads) {
            const int r = base + tid;
            Key<W> key;
            double h = 0.0;
            bool keep = false;
            if (r < r_hi) {
                gen_one<W>(a, L, s, r, key, h);
                keep = fabs(h) > a.eps;
            }
            const unsigned long long m = __ballot(keep);
            const int before = __popcll(m & ((1ull << lane) - 1ull));
            if (lane == 0) L.wave_tot[wid] = __popcll(m);
            __syncthreads();
            if (tid == 0) {
                int tot = 0;
                for (int w = 0; w < kGenThreads / kWave; ++w) {
                    const int c = L.wave_tot[w];
                    L.wave_tot[w] = tot;
                    tot += c;
                }
                L.slab = tot ? atomicAdd(a.n_out, (unsigned long long)tot) : 0ull;
                if (tot && (int64_t)(L.slab + tot) > a.capacity) atomicOr(a.flags, SCI_FLAG_OVERFLOW);
            }
            __syncthreads();
            if (keep) {
                const int64_t o = (int64_t)L.slab + L.wave_tot[wid] + before;
                if (o < a.capacity) {
                    store_key<W>(a.keys, o, key);
                    a.hij[o] = h;
                    a.src_out[o] = (int32_t)src;
                }
            }
            __syncthreads();
        }
    }
}

}  // namespace sci

using namespace sci;

extern "C" int32_t sci_gen_coupled(sci_ham_t ham, const uint64_t *dets, int64_t n_dets,
                                   int64_t exc_begin, int64_t exc_end, double eps,
                                   uint64_t *out_keys, double *out_hij, int32_t *out_src,
                                   int64_t capacity, int64_t *n_out, uint32_t *dev_flags,
                                   sci_stream_t stream) {
    set_error("");
    if (!ham) return fail(SCI_EINVAL, "sci_gen_coupled: NULL handle");
    const HamDev &d = ham->dev;
    if (n_dets < 0) return fail(SCI_EINVAL, "sci_gen_coupled: n_dets < 0");
    const int64_t total = n_dets * d.n_coupled;
    if (exc_begin < 0 || exc_end < exc_begin || exc_end > total)
        return fail(SCI_EINVAL, "sci_gen_coupled: range [%lld,%lld) outside [0,%lld)",
                    (long long)exc_begin, (long long)exc_end, (long long)total);
    if (!dev_flags) return fail(SCI_EINVAL, "sci_gen_coupled: dev_flags is NULL");
    const bool dense = eps < 0.0;
    if (!dense && (!out_src || !n_out))
        return fail(SCI_EINVAL, "sci_gen_coupled: screened mode needs out_src and n_out");
    if (capacity < 0) return fail(SCI_EINVAL, "sci_gen_coupled: capacity < 0");
    if (dense && capacity < exc_end - exc_begin)
        return fail(SCI_ECAPACITY, "sci_gen_coupled: capacity %lld < %lld entries", (long long)capacity,
                    (long long)(exc_end - exc_begin));
    if (d.W > SCI_MAX_WORDS) return fail(SCI_EUNSUPPORTED, "sci_gen_coupled: W=%d", d.W);
    if (d.n_coupled >= (1ll << 24))
        return fail(SCI_EUNSUPPORTED, "sci_gen_coupled: %lld excitations per source", (long long)d.n_coupled);
    hipStream_t st = (hipStream_t)stream;
    // n_out: dense count is known here; screened count starts at zero
    if (n_out) SCI_HIP_TRY(launch_set_i64(n_out, dense ? exc_end - exc_begin : 0, st));
    if (exc_end == exc_begin) return SCI_OK;
    if (!dets || !out_keys || !out_hij) return fail(SCI_EINVAL, "sci_gen_coupled: NULL buffer");

    GenArgs a;
    a.n = d.n_orb;
    a.na = d.n_alpha;
    a.nb = d.n_beta;
    a.va = d.v_alpha;
    a.vb = d.v_beta;
    a.c1 = (int)d.c1;
    a.c2 = (int)d.c2;
    a.c3 = (int)d.c3;
    a.c4 = (int)d.c4;
    a.nc = (int)d.n_coupled;
    a.h1 = d.h1;
    a.eri = d.eri;
    a.vdir = d.vdir;
    a.vanti = d.vanti;
    for (int t = 0; t < 4; ++t) a.pairs[t] = d.pairs[t];
    a.dets = dets;
    a.src_first = exc_begin / d.n_coupled;
    const int64_t src_last = (exc_end - 1) / d.n_coupled;
    const int64_t n_src = src_last - a.src_first + 1;
    // split each source into near-equal chunks of at most 8192 ranks, rounded to the workgroup size
    const int64_t chunks = ceil_div(d.n_coupled, 8192);
    a.chunk = (int)(ceil_div(ceil_div(d.n_coupled, chunks), kGenThreads) * kGenThreads);
    a.chunks_per_src = (int)ceil_div(d.n_coupled, a.chunk);
    a.exc_begin = exc_begin;
    a.exc_end = exc_end;
    a.keys = out_keys;
    a.hij = out_hij;
    a.src_out = out_src;
    a.capacity = capacity;
    a.n_out = (unsigned long long *)n_out;
    a.flags = dev_flags;
    a.eps = eps;
    a.d_va = make_fastdiv((uint32_t)d.v_alpha);
    a.d_vb = make_fastdiv((uint32_t)d.v_beta);
    a.d_nb = make_fastdiv((uint32_t)d.n_beta);
    a.d_vab = make_fastdiv((uint32_t)(d.v_alpha * d.v_beta));
    a.d_pva = make_fastdiv((uint32_t)comb2(d.v_alpha));
    a.d_pvb = make_fastdiv((uint32_t)comb2(d.v_beta));

    const int64_t grid = n_src * a.chunks_per_src;
    if (grid > 0x7fffffffll) return fail(SCI_EUNSUPPORTED, "sci_gen_coupled: range too large for one launch");
    dim3 g((unsigned)grid), b(kGenThreads);
    if (d.W == 1) {
        if (dense) SCI_LAUNCH((gen_kernel<1, true>), g, b, 0, st, a);
        else SCI_LAUNCH((gen_kernel<1, false>), g, b, 0, st, a);
    } else {
        if (dense) SCI_LAUNCH((gen_kernel<2, true>), g, b, 0, st, a);
        else SCI_LAUNCH((gen_kernel<2, false>), g, b, 0, st, a);
    }
    SCI_HIP_TRY(hipGetLastError());
    return SCI_OK;
}
