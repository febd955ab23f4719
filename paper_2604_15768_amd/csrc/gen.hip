// Coupled-configuration generation (paper section 4.2, Algorithm 1; Eq. 4).
//
// One workgroup per source determinant.  The source is decoded once into LDS:
// occupied / empty orbital lists per spin, the count of occupied orbitals below
// every orbital (for fermionic signs), and the lexicographic pair lists used to
// unrank same-spin doubles.  Its excitations are processed in rows that share
// their holes; each wave takes whole rows, so the row's partial key, integral
// row and per-particle sign bits are wave-uniform, and lanes step through the
// particles of the row with unit-stride stores (one wave writes 64 consecutive
// entries).
//
// Unlike the paper's padded virtual-thread space (Eqs. 6-7), ranks cover only
// valid excitations, so dense mode needs no compaction and its output order is
// fixed.  Screened mode (eps >= 0) keeps |H| > eps and compacts with a wave
// ballot and one atomic per wave iteration (the paper compacts per block with
// one atomicAdd per block).
#include <algorithm>
#include <vector>

#include "sci_internal.hpp"

namespace sci {

constexpr int kGenThreads = 256;
constexpr int kMaxPairs = 64 * 63 / 2;
constexpr int kUnroll = 4;  // row positions per lane per loop trip (loads issued before stores)

struct GenArgs {
    // system
    int W;
    int n, na, nb, va, vb;
    int c1, c2, c3, c4, nc;
    const double *h1, *eri, *vdir, *vanti, *jtpq, *ktpq;
    const uint16_t *pairs[4];
    // tiles
    const uint64_t *dets;
    int64_t src_first;
    int pva, pvb;  // C(v_alpha, 2), C(v_beta, 2)
    int64_t exc_begin, exc_end;
    // outputs
    uint64_t *keys;
    double *hij;
    int32_t *src_out;
    int64_t capacity;
    unsigned long long *n_out;
    uint32_t *flags;
    double eps;
};

constexpr int kMaxSingles = 512;  // per spin; larger systems compute singles per lane

struct GenLds {
    double sval[2][kMaxSingles];  // single-excitation elements (unsigned) of the source, [ip * v + ia]
    uint8_t occ[2][64];
    uint8_t vir[2][64];
    uint8_t below[2][64];  // occupied orbitals of the same spin strictly below p
    uint16_t pocc[2][kMaxPairs];
    uint16_t pvir[2][kMaxPairs];
    int bad;
};

__device__ __forceinline__ void copy_pairs(uint16_t *dst, const uint16_t *src, int m, int tid) {
    const int total = m * (m - 1) / 2;
    for (int t = tid; t < total; t += kGenThreads) dst[t] = src[t];
}

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | (uint64_t)uni((uint32_t)x);
}

template <int W>
__device__ __forceinline__ Key<W> uni_key(const Key<W> &k) {
    Key<W> r;
#pragma unroll
    for (int j = 0; j < W; ++j) r.w[j] = uni64(k.w[j]);
    return r;
}

// Screened output is staged per wave: kept entries collect in LDS and leave with one
// atomic on the output counter per kStage entries, not one per wave-wide batch (the
// counter is a single address every workgroup of the launch updates).
constexpr int kStage = 512;

template <int W>
struct GenStage {
    Key<W> key[kGenThreads / kWave][kStage];
    double hij[kGenThreads / kWave][kStage];
    int fill[kGenThreads / kWave];  // entries left in each wave's stage at the end of a source
    unsigned long long base;        // their output range, reserved once per workgroup
};

// LDS written by some lanes of a wave is read by others: order the accesses
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Write this wave's staged entries (all of one source) at a reserved output range.
template <int W>
__device__ __forceinline__ void flush_stage(const GenArgs &a, GenStage<W> *st, int &fill, int64_t src) {
    if (fill == 0) return;  // wave-uniform
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    wave_lds_sync();
    unsigned long long base = 0;
    if (lane == 0) {
        base = atomicAdd(a.n_out, (unsigned long long)fill);
        if ((int64_t)(base + fill) > a.capacity) atomicOr(a.flags, SCI_FLAG_OVERFLOW);
    }
    base = __shfl(base, 0);
    for (int i = lane; i < fill; i += kWave) {
        const int64_t o = (int64_t)base + i;
        if (o < a.capacity) {
            store_key<W>(a.keys, o, st->key[w][i]);
            a.hij[o] = st->hij[w][i];
            a.src_out[o] = (int32_t)src;
        }
    }
    wave_lds_sync();  // every lane has read the stage before it is refilled
    fill = 0;
}

// Write one output slot (dense) or stage it for compaction (screened); called by
// whole waves.
template <int W, bool DENSE>
__device__ __forceinline__ void emit(const GenArgs &a, int64_t o_dense, bool valid, const Key<W> &key, double h,
                                     int64_t src, GenStage<W> *st, int &fill) {
    if constexpr (DENSE) {
        if (valid) {
            store_key<W>(a.keys, o_dense, key);
            a.hij[o_dense] = h;
            if (a.src_out) a.src_out[o_dense] = (int32_t)src;
        }
    } else {
        const bool keep = valid && fabs(h) > a.eps;
        const unsigned long long m = __ballot(keep);
        if (m == 0ull) return;
        const int c = __popcll(m);
        if (fill + c > kStage) flush_stage<W>(a, st, fill, src);
        if (keep) {
            const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
            const int i = fill + __popcll(m & ((1ull << lane) - 1ull));
            st->key[w][i] = key;
            st->hij[w][i] = h;
        }
        fill += c;
    }
}

// One workgroup per source.  The source's excitations are organised in rows
// that share their holes: a single row per occupied orbital p (singles), per
// occupied pair p<q (same-spin doubles) and per (p alpha, q beta) (mixed
// doubles).  Waves take rows round-robin; inside a row every hole-dependent
// quantity (row key, integral row base, per-particle sign bits gathered with a
// ballot) is wave-uniform and lanes walk the particle index without division.
template <int W, bool DENSE>
__device__ __forceinline__ void gen_source(const GenArgs &a, const int64_t src, GenLds &L, GenStage<W> *st) {
    int fill = 0;  // screened entries staged by this wave
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    const int64_t flat0 = src * a.nc;
    const int64_t lo = (a.exc_begin > flat0 ? a.exc_begin : flat0) - flat0;
    const int64_t hi = (a.exc_end < flat0 + a.nc ? a.exc_end : flat0 + a.nc) - flat0;
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
        uint64_t word = s.w[0];
#pragma unroll
        for (int j = 1; j < W; ++j) word = ((k >> 6) == j) ? s.w[j] : word;
        const bool occ = (word >> (k & 63)) & 1ull;
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
    const int64_t obase = flat0 - a.exc_begin;  // output index of rank 0 of this source
    const bool lds_singles = a.na * a.va <= kMaxSingles && a.nb * a.vb <= kMaxSingles;
    if (lds_singles && !L.bad) {
        // every single element of the source at once: h_ap + sum_{Q occ, Q != P} [(ap|qq) - d_spin (aq|qp)]
        const int s0 = a.na * a.va, s_tot = s0 + a.nb * a.vb;
        for (int e = tid; e < s_tot; e += kGenThreads) {
            const int sg = e < s0 ? 0 : 1;
            const int el = sg ? e - s0 : e;
            const int vs = sg ? a.vb : a.va;
            const int ip = el / vs, ia = el - ip * vs;
            const int p = L.occ[sg][ip], t = L.vir[sg][ia];
            double v = a.h1[t * n + p];
            for (int s2 = 0; s2 < 2; ++s2) {
                const int cnt = s2 ? a.nb : a.na;
                const double *jr = a.jtpq + (int64_t)(t * n + p) * n;  // (tp|qq) over q
                const double *kr = a.ktpq + (int64_t)(t * n + p) * n;  // (tq|qp) over q
                for (int k = 0; k < cnt; ++k) {
                    const int q = L.occ[s2][k];
                    if (s2 == sg && q == p) continue;
                    const double j = jr[q];
                    const double kx = (s2 == sg) ? kr[q] : 0.0;
                    v += j - kx;
                }
            }
            L.sval[sg][el] = v;
        }
        __syncthreads();
    }

    if (L.bad) {
        if (tid == 0) atomicOr(a.flags, SCI_FLAG_BAD_DET);
        if constexpr (DENSE) {
            for (int64_t r = lo + tid; r < hi; r += kGenThreads) {
                Key<W> z;
#pragma unroll
                for (int j = 0; j < W; ++j) z.w[j] = 0;
                store_key<W>(a.keys, obase + r, z);
                a.hij[obase + r] = 0.0;
                if (a.src_out) a.src_out[obase + r] = (int32_t)src;
            }
        }
        return;
    }

    const int Pa = a.na * (a.na - 1) / 2, Pb = a.nb * (a.nb - 1) / 2;
    const int g1 = a.na, g2 = g1 + a.nb, g3 = g2 + Pa, g4 = g3 + Pb, n_rows = g4 + a.na * a.nb;
    for (int g = wave; g < n_rows; g += kGenThreads / kWave) {
        if (g < g2) {
            // single excitations p -> a of one spin
            const int sg = g < g1 ? 0 : 1;
            const int ip = sg ? g - g1 : g;
            const int R = sg ? a.vb : a.va;
            const int64_t rb = sg ? (int64_t)a.c1 + (int64_t)ip * R : (int64_t)ip * R;
            const int64_t t0 = lo > rb ? lo - rb : 0, t1 = hi - rb < R ? hi - rb : R;
            if (t0 >= t1) continue;
            const int off = sg * n;
            const int p = (int)uni(L.occ[sg][ip]);
            Key<W> rk = s;
            key_flip<W>(rk, p + off);
            rk = uni_key<W>(rk);
            const int nocc0 = a.na, nocc1 = a.nb;
            for (int64_t t = t0 + lane; t - lane < t1; t += kWave) {
                const bool valid = t < t1;
                Key<W> key = rk;
                double h = 0.0;
                if (valid && lds_singles) {
                    const int ta = L.vir[sg][t];
                    key_flip<W>(key, ta + off);
                    const int par = L.below[sg][p] + L.below[sg][ta] - (p < ta ? 1 : 0);
                    const double v = L.sval[sg][ip * R + (int)t];
                    h = (par & 1) ? -v : v;
                } else if (valid) {
                    const int ta = L.vir[sg][t];
                    key_flip<W>(key, ta + off);
                    const int par = L.below[sg][p] + L.below[sg][ta] - (p < ta ? 1 : 0);
                    // h_ap + sum over occupied Q != P of [(ap|qq) - delta_spin (aq|qp)], Q ascending
                    double v = a.h1[ta * n + p];
                    for (int s2 = 0; s2 < 2; ++s2) {
                        const int cnt = s2 ? nocc1 : nocc0;
                        for (int k = 0; k < cnt; ++k) {
                            const int q = L.occ[s2][k];
                            if (s2 == sg && q == p) continue;
                            const double j = a.jtpq[(int64_t)(ta * n + p) * n + q];
                            const double kx = (s2 == sg) ? a.ktpq[(int64_t)(ta * n + p) * n + q] : 0.0;
                            v += j - kx;
                        }
                    }
                    h = (par & 1) ? -v : v;
                }
                emit<W, DENSE>(a, obase + rb + t, valid, key, h, src, st, fill);
            }
        } else if (g < g4) {
            // same-spin doubles p<q -> a<b
            const int sg = g < g3 ? 0 : 1;
            const int o = sg ? g - g3 : g - g2;
            const int R = sg ? a.pvb : a.pva;
            const int64_t rb = (int64_t)(sg ? a.c3 : a.c2) + (int64_t)o * R;
            const int64_t t0 = lo > rb ? lo - rb : 0, t1 = hi - rb < R ? hi - rb : R;
            if (t0 >= t1) continue;
            const int off = sg * n;
            const uint32_t po = uni(L.pocc[sg][o]);
            const int p = (int)uni(L.occ[sg][po & 0xff]), q = (int)uni(L.occ[sg][po >> 8]);
            const int vs = sg ? a.vb : a.va;
            // parity bit of each particle: below(v) - [p<v] - [q<v]
            int fb = 0;
            if (lane < vs) {
                const int v = L.vir[sg][lane];
                fb = (L.below[sg][v] - (p < v) - (q < v)) & 1;
            }
            const uint64_t F = __ballot(fb != 0);
            const uint32_t par0 = (uint32_t)(L.below[sg][p] + L.below[sg][q] - 1) & 1u;
            Key<W> rk = s;
            key_flip<W>(rk, p + off);
            key_flip<W>(rk, q + off);
            rk = uni_key<W>(rk);
            const double *row = a.vanti + (int64_t)(p * n + q) * n * n;
            for (int64_t t = t0 + lane; t - lane < t1; t += kUnroll * kWave) {
                int ta[kUnroll], tb[kUnroll];
                uint32_t par[kUnroll];
                double v[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int64_t tu = t + u * kWave;
                    ta[u] = tb[u] = 0;
                    par[u] = 0;
                    v[u] = 0.0;
                    if (tu < t1) {
                        const uint32_t pv = L.pvir[sg][tu];
                        const int ia = pv & 0xff, ib = pv >> 8;
                        ta[u] = L.vir[sg][ia];
                        tb[u] = L.vir[sg][ib];
                        par[u] = par0 ^ ((uint32_t)((F >> ia) ^ (F >> ib)) & 1u);
                        v[u] = row[ta[u] * n + tb[u]];
                    }
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int64_t tu = t + u * kWave;
                    if (tu - lane >= t1) break;  // uniform: the wave's first position is past the row
                    Key<W> key = rk;
                    key_flip<W>(key, ta[u] + off);
                    key_flip<W>(key, tb[u] + off);
                    emit<W, DENSE>(a, obase + rb + tu, tu < t1, key, par[u] ? -v[u] : v[u], src, st, fill);
                }
            }
        } else {
            // alpha-beta doubles p(alpha) q(beta) -> a(alpha) b(beta)
            const int o = g - g4;
            const int ip = o / a.nb, iq = o - ip * a.nb;
            const int R = a.va * a.vb;
            const int64_t rb = (int64_t)a.c4 + (int64_t)o * R;
            const int64_t t0 = lo > rb ? lo - rb : 0, t1 = hi - rb < R ? hi - rb : R;
            if (t0 >= t1) continue;
            const int p = (int)uni(L.occ[0][ip]), q = (int)uni(L.occ[1][iq]);
            int fa = 0, fb = 0;
            if (lane < a.va) {
                const int v = L.vir[0][lane];
                fa = (L.below[0][v] - (p < v)) & 1;
            }
            if (lane < a.vb) {
                const int v = L.vir[1][lane];
                fb = (L.below[1][v] - (q < v)) & 1;
            }
            const uint64_t Fa = __ballot(fa != 0), Fb = __ballot(fb != 0);
            const uint32_t par0 = (uint32_t)(L.below[0][p] + L.below[1][q]) & 1u;
            Key<W> rk = s;
            key_flip<W>(rk, p);
            key_flip<W>(rk, q + n);
            rk = uni_key<W>(rk);
            const double *row = a.vdir + (int64_t)(p * n + q) * n * n;
            // particle pair of the first lane's position, then fixed strides of one wave
            const int64_t tf = t0 + lane;
            int ia = (int)tf / a.vb, ib = (int)tf - ((int)tf / a.vb) * a.vb;
            const int dia = kWave / a.vb, dib = kWave - dia * a.vb;
            for (int64_t t = tf; t - lane < t1; t += kUnroll * kWave) {
                int ta[kUnroll], tb[kUnroll];
                uint32_t par[kUnroll];
                double v[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int64_t tu = t + u * kWave;
                    ta[u] = tb[u] = 0;
                    par[u] = 0;
                    v[u] = 0.0;
                    if (tu < t1) {
                        ta[u] = L.vir[0][ia];
                        tb[u] = L.vir[1][ib];
                        par[u] = par0 ^ ((uint32_t)((Fa >> ia) ^ (Fb >> ib)) & 1u);
                        v[u] = row[ta[u] * n + tb[u]];
                    }
                    ib += dib;
                    ia += dia;
                    if (ib >= a.vb) {
                        ib -= a.vb;
                        ++ia;
                    }
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int64_t tu = t + u * kWave;
                    if (tu - lane >= t1) break;  // uniform: the wave's first position is past the row
                    Key<W> key = rk;
                    key_flip<W>(key, ta[u]);
                    key_flip<W>(key, tb[u] + n);
                    emit<W, DENSE>(a, obase + rb + tu, tu < t1, key, par[u] ? -v[u] : v[u], src, st, fill);
                }
            }
        }
    }
    if constexpr (!DENSE) {
        // what the waves still hold leaves with one reservation for the workgroup
        const int w = tid / kWave;
        if (lane == 0) st->fill[w] = fill;
        __syncthreads();
        if (tid == 0) {
            unsigned long long tot = 0;
            for (int x = 0; x < kGenThreads / kWave; ++x) tot += (unsigned long long)st->fill[x];
            st->base = tot ? atomicAdd(a.n_out, tot) : 0ull;
            if (tot && (int64_t)(st->base + tot) > a.capacity) atomicOr(a.flags, SCI_FLAG_OVERFLOW);
        }
        __syncthreads();
        unsigned long long b0 = st->base;
        for (int x = 0; x < w; ++x) b0 += (unsigned long long)st->fill[x];
        for (int i = lane; i < fill; i += kWave) {
            const int64_t o = (int64_t)b0 + i;
            if (o < a.capacity) {
                store_key<W>(a.keys, o, st->key[w][i]);
                a.hij[o] = st->hij[w][i];
                a.src_out[o] = (int32_t)src;
            }
        }
    }
}

// Sources are taken XCD by XCD (xcd_local_block): neighbouring sources (sorted keys
// share most integral rows) meet in one L2.
template <int W, bool DENSE>
__global__ __launch_bounds__(kGenThreads) void gen_kernel(GenArgs a) {
    __shared__ GenLds L;
    const int64_t src = a.src_first + xcd_local_block(blockIdx.x, gridDim.x);
    if constexpr (DENSE) {
        gen_source<W, true>(a, src, L, nullptr);
    } else {
        __shared__ GenStage<W> st;
        gen_source<W, false>(a, src, L, &st);
    }
}

// A tile: n_src consecutive sources of one system of a batch.
struct GenTile {
    int32_t item;
    int32_t n_src;
    int64_t src0;
};

// Many systems of one key width in one launch: a persistent grid takes tiles
// from a device counter (tiles are ordered largest first); each tile's system
// arguments come from the batch's device table through scalar loads.
template <int W>
__global__ __launch_bounds__(kGenThreads) void gen_batched_kernel(const GenArgs *__restrict__ items,
                                                                  const GenTile *__restrict__ tiles, int64_t n_tiles,
                                                                  unsigned long long *next) {
    __shared__ GenLds L;
    __shared__ long long s_t;
    while (true) {
        __syncthreads();  // the previous source is done with LDS and s_t
        if (threadIdx.x == 0) s_t = (long long)atomicAdd(next, 1ull);
        __syncthreads();
        // the tile index is the same in every lane: say so, so the tile and its system's
        // arguments are read with scalar loads
        const uint64_t tu = (uint64_t)s_t;
        const int64_t t = (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(tu >> 32)) << 32) |
                                    (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)tu));
        if (t >= n_tiles) break;
        const GenTile tile = tiles[t];
        const GenArgs &a = items[tile.item];
        for (int j = 0; j < tile.n_src; ++j) {
            if (j > 0) __syncthreads();
            gen_source<W, true>(a, tile.src0 + j, L, nullptr);
        }
    }
}

static GenArgs make_gen_args(const HamDev &d, const uint64_t *dets, int64_t exc_begin, int64_t exc_end,
                             uint64_t *out_keys, double *out_hij, int32_t *out_src, int64_t capacity,
                             unsigned long long *n_out, uint32_t *dev_flags, double eps) {
    GenArgs a;
    a.W = d.W;
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
    a.jtpq = d.jtpq;
    a.ktpq = d.ktpq;
    for (int t = 0; t < 4; ++t) a.pairs[t] = d.pairs[t];
    a.dets = dets;
    a.src_first = exc_begin / d.n_coupled;
    a.pva = (int)comb2(d.v_alpha);
    a.pvb = (int)comb2(d.v_beta);
    a.exc_begin = exc_begin;
    a.exc_end = exc_end;
    a.keys = out_keys;
    a.hij = out_hij;
    a.src_out = out_src;
    a.capacity = capacity;
    a.n_out = n_out;
    a.flags = dev_flags;
    a.eps = eps;
    return a;
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
    if (exc_end > exc_begin && (!dets || !out_keys || !out_hij))
        return fail(SCI_EINVAL, "sci_gen_coupled: NULL buffer");
    hipStream_t st = (hipStream_t)stream;
    // n_out: dense count is known here; screened count starts at zero
    if (n_out) SCI_HIP_TRY(launch_set_i64(n_out, dense ? exc_end - exc_begin : 0, st));
    if (exc_end == exc_begin) return SCI_OK;

    GenArgs a = make_gen_args(d, dets, exc_begin, exc_end, out_keys, out_hij, out_src, capacity,
                              (unsigned long long *)n_out, dev_flags, eps);
    const int64_t n_src = (exc_end - 1) / d.n_coupled - a.src_first + 1;
    const int64_t grid = n_src;
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

// ---------------------------------------------------------------------------
// batches of systems (one persistent launch)
// ---------------------------------------------------------------------------

struct sci_gen_batch_s {
    std::vector<GenArgs> items;
    GenArgs *d_items = nullptr;
    GenTile *d_tiles = nullptr;        // W=1 tiles, then W=2 tiles
    unsigned long long *d_next = nullptr;  // one work counter per key width
    int64_t n_tiles[2] = {0, 0}, tile_alloc = 0;
    int64_t tile_candidates = 0;
    int grid[2] = {0, 0};
};

namespace sci {

// tiles of about tile_cand candidates (at least one source) of the systems of key
// width W, largest first
static void build_tiles(const std::vector<GenArgs> &items, int W, int64_t tile_cand, std::vector<GenTile> &tiles) {
    tiles.clear();
    for (size_t i = 0; i < items.size(); ++i) {
        const GenArgs &a = items[i];
        if (a.W != W || a.exc_end <= a.exc_begin) continue;
        const int64_t s0 = a.src_first, s1 = (a.exc_end - 1) / a.nc;
        const int64_t per = std::min<int64_t>(std::max<int64_t>(1, tile_cand / a.nc), 1 << 20);
        for (int64_t src = s0; src <= s1; src += per)
            tiles.push_back(GenTile{(int32_t)i, (int32_t)std::min<int64_t>(per, s1 - src + 1), src});
    }
    std::stable_sort(tiles.begin(), tiles.end(), [&](const GenTile &x, const GenTile &y) {
        return (int64_t)x.n_src * items[x.item].nc > (int64_t)y.n_src * items[y.item].nc;
    });
}

static int32_t upload_tiles(sci_gen_batch_s *b, int64_t tile_cand) {
    // host lists first (these may throw); the batch changes only once they exist
    std::vector<GenTile> tiles, t2;
    build_tiles(b->items, 1, tile_cand, tiles);
    build_tiles(b->items, 2, tile_cand, t2);
    const int64_t n1 = (int64_t)tiles.size(), n2 = (int64_t)t2.size();
    tiles.insert(tiles.end(), t2.begin(), t2.end());
    const int64_t nt = (int64_t)tiles.size();
    if (nt > b->tile_alloc) {
        if (b->d_tiles) (void)hipFree(b->d_tiles);
        b->d_tiles = nullptr;
        b->tile_alloc = 0;
        b->n_tiles[0] = b->n_tiles[1] = 0;
        SCI_HIP_TRY(hipMalloc((void **)&b->d_tiles, (size_t)std::max<int64_t>(nt, 1) * sizeof(GenTile)));
        b->tile_alloc = std::max<int64_t>(nt, 1);
    }
    if (nt) SCI_HIP_TRY(hipMemcpy(b->d_tiles, tiles.data(), (size_t)nt * sizeof(GenTile), hipMemcpyHostToDevice));
    b->n_tiles[0] = n1;
    b->n_tiles[1] = n2;
    b->tile_candidates = tile_cand;
    return SCI_OK;
}

static int32_t launch_batch(sci_gen_batch_s *b, hipStream_t st) {
    if (b->n_tiles[0] > 0) {
        SCI_HIP_TRY(launch_set_i64((int64_t *)b->d_next, 0, st));
        SCI_LAUNCH(gen_batched_kernel<1>, dim3((unsigned)b->grid[0]), dim3(kGenThreads), 0, st,
                   (const GenArgs *)b->d_items, (const GenTile *)b->d_tiles, b->n_tiles[0], b->d_next);
    }
    if (b->n_tiles[1] > 0) {
        SCI_HIP_TRY(launch_set_i64((int64_t *)(b->d_next + 1), 0, st));
        SCI_LAUNCH(gen_batched_kernel<2>, dim3((unsigned)b->grid[1]), dim3(kGenThreads), 0, st,
                   (const GenArgs *)b->d_items, (const GenTile *)(b->d_tiles + b->n_tiles[0]), b->n_tiles[1],
                   b->d_next + 1);
    }
    SCI_HIP_TRY(hipGetLastError());
    return SCI_OK;
}

}  // namespace sci

extern "C" int32_t sci_gen_batch_destroy(sci_gen_batch_t b) {
    if (!b) return SCI_OK;
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_next) (void)hipFree(b->d_next);
    delete b;
    return SCI_OK;
}

static int32_t gen_batch_create_impl(const sci_gen_item *items, int32_t n_items, int64_t tile_candidates,
                                     uint32_t *dev_flags, sci_gen_batch_t *out);

extern "C" int32_t sci_gen_batch_create(const sci_gen_item *items, int32_t n_items, int64_t tile_candidates,
                                        uint32_t *dev_flags, sci_gen_batch_t *out) {
    set_error("");
    return guarded("sci_gen_batch_create",
                   [&] { return gen_batch_create_impl(items, n_items, tile_candidates, dev_flags, out); });
}

static int32_t gen_batch_create_impl(const sci_gen_item *items, int32_t n_items, int64_t tile_candidates,
                                     uint32_t *dev_flags, sci_gen_batch_t *out) {
    if (!out) return fail(SCI_EINVAL, "sci_gen_batch_create: NULL output handle");
    *out = nullptr;
    if (n_items < 0 || (n_items > 0 && !items)) return fail(SCI_EINVAL, "sci_gen_batch_create: bad item list");
    if (tile_candidates < 1) return fail(SCI_EINVAL, "sci_gen_batch_create: tile_candidates must be >= 1");
    if (!dev_flags) return fail(SCI_EINVAL, "sci_gen_batch_create: dev_flags is NULL");
    std::vector<GenArgs> args;
    args.reserve((size_t)n_items);
    for (int32_t i = 0; i < n_items; ++i) {
        const sci_gen_item &it = items[i];
        if (!it.ham) return fail(SCI_EINVAL, "sci_gen_batch_create: item %d has no handle", i);
        const HamDev &d = it.ham->dev;
        const int64_t total = it.n_dets * d.n_coupled;
        if (it.n_dets < 0 || it.exc_begin < 0 || it.exc_end < it.exc_begin || it.exc_end > total)
            return fail(SCI_EINVAL, "sci_gen_batch_create: item %d range [%lld,%lld) outside [0,%lld)", i,
                        (long long)it.exc_begin, (long long)it.exc_end, (long long)total);
        if (d.W > SCI_MAX_WORDS || d.n_coupled >= (1ll << 24))
            return fail(SCI_EUNSUPPORTED, "sci_gen_batch_create: item %d exceeds the kernel's limits", i);
        if (it.exc_end > it.exc_begin && (!it.dets || !it.out_keys || !it.out_hij))
            return fail(SCI_EINVAL, "sci_gen_batch_create: item %d has a NULL buffer", i);
        args.push_back(make_gen_args(d, it.dets, it.exc_begin, it.exc_end, it.out_keys, it.out_hij, nullptr,
                                     it.exc_end - it.exc_begin, nullptr, dev_flags, -1.0));
    }
    sci_gen_batch_s *b = new (std::nothrow) sci_gen_batch_s;
    if (!b) return fail(SCI_ENOMEM, "sci_gen_batch_create: host allocation failed");
    b->items = std::move(args);
    auto bail = [&](int32_t st) {
        sci_gen_batch_destroy(b);
        return st;
    };
    if (hipMalloc((void **)&b->d_items, std::max<size_t>(b->items.size(), 1) * sizeof(GenArgs)) != hipSuccess ||
        hipMalloc((void **)&b->d_next, 256) != hipSuccess)
        return bail(fail(SCI_ENOMEM, "sci_gen_batch_create: device allocation failed"));
    if (!b->items.empty() &&
        hipMemcpy(b->d_items, b->items.data(), b->items.size() * sizeof(GenArgs), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(SCI_EHIP, "sci_gen_batch_create: upload failed"));
    int32_t st;
    try {
        st = upload_tiles(b, tile_candidates);
    } catch (...) {
        return bail(fail(SCI_ENOMEM, "sci_gen_batch_create: host allocation failed"));
    }
    if (st != SCI_OK) return bail(st);
    int dev = 0, n_cu = 256, per1 = 1, per2 = 1;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per1, gen_batched_kernel<1>, kGenThreads, 0) != hipSuccess ||
        per1 < 1)
        per1 = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per2, gen_batched_kernel<2>, kGenThreads, 0) != hipSuccess ||
        per2 < 1)
        per2 = 1;
    b->grid[0] = std::max(1, n_cu) * per1;
    b->grid[1] = std::max(1, n_cu) * per2;
    *out = b;
    return SCI_OK;
}

extern "C" int32_t sci_gen_coupled_batched(sci_gen_batch_t batch, sci_stream_t stream) {
    set_error("");
    if (!batch) return fail(SCI_EINVAL, "sci_gen_coupled_batched: NULL handle");
    return launch_batch(batch, (hipStream_t)stream);
}

static int32_t gen_batch_autotune_impl(sci_gen_batch_t batch, sci_stream_t stream, int64_t *tile_candidates);

extern "C" int32_t sci_gen_batch_autotune(sci_gen_batch_t batch, sci_stream_t stream, int64_t *tile_candidates) {
    set_error("");
    return guarded("sci_gen_batch_autotune", [&] { return gen_batch_autotune_impl(batch, stream, tile_candidates); });
}

// The tile list is rebuilt for each size tried (host vectors: a throw leaves the
// batch with its previous, still valid, tile list; the events are released by RAII).
static int32_t gen_batch_autotune_impl(sci_gen_batch_t batch, sci_stream_t stream, int64_t *tile_candidates) {
    if (!batch) return fail(SCI_EINVAL, "sci_gen_batch_autotune: NULL handle");
    hipStream_t st = (hipStream_t)stream;
    static const int64_t kTry[] = {1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22};
    struct Events {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } ev;
    SCI_HIP_TRY(hipEventCreate(&ev.e0));
    SCI_HIP_TRY(hipEventCreate(&ev.e1));
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
    int64_t best = batch->tile_candidates;
    float best_ms = -1.0f;
    int32_t rc = SCI_OK;
    for (int64_t tc : kTry) {
        if ((rc = upload_tiles(batch, tc)) != SCI_OK) break;
        if ((rc = launch_batch(batch, st)) != SCI_OK) break;  // warm
        if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(SCI_EHIP, "sci_gen_batch_autotune: event"); break; }
        if ((rc = launch_batch(batch, st)) != SCI_OK) break;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rc = fail(SCI_EHIP, "sci_gen_batch_autotune: event");
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (best_ms < 0.0f || ms < best_ms) {
            best_ms = ms;
            best = tc;
        }
    }
    if (rc != SCI_OK) return rc;
    if ((rc = upload_tiles(batch, best)) != SCI_OK) return rc;
    if (tile_candidates) *tile_candidates = best;
    return SCI_OK;
}
