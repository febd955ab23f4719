// Selected-space variational energy (paper Eq. 1 with the sums of Eqs. 3/5
// restricted to the selected set S), matrix-free, and its adjoint.
//
//   (H psi)_i = H_ii psi_i + sum_{j in S, j != i} H_ij psi_j
//   E = psi.(H psi) / psi.psi,   g_i = 2((H psi)_i - E psi_i) / psi.psi
//
// Membership of j in C_i is decided one of two ways, picked per shape:
//   pair screening  H_ij can be non-zero only when D_i XOR D_j has two or four
//       set bits (at most two electrons moved, paper section 2.1).  A workgroup
//       owns 256 rows (one per lane) and streams every determinant of S through
//       LDS in tiles; all lanes read the same LDS entry at a time (broadcast), so
//       the screening is one XOR + popcount per pair: |S|^2 tests.
//   enumeration     C_i is generated (every single and double of D_i) and each
//       determinant searched in the sorted S (the paper's search of configurations
//       in a sorted set, section 4.3): |S| N_c searches, a win when N_c is small
//       against |S|.
// For a connected pair the lane rebuilds the excitation from the XOR bits and
// reads the same integral tables the generation kernel uses; H_ij is never
// stored.  Row sums run in a fixed order (ascending j for pair screening, the
// excitation order for enumeration), block sums in a fixed tree, so repeated
// calls are bit-identical.
#include <algorithm>
#include <mutex>
#include <vector>

#include "sci_internal.hpp"

namespace sci {

constexpr int kRowThreads = 256;
constexpr int kColTile = 1024;
constexpr int kRedThreads = 256;

struct EnergyArgs {
    int n, na, nb;
    const double *h1, *eri, *vdir, *vanti, *jmat, *kmat, *jtpq, *ktpq;
    const double *fref;             // [s][t][p] single elements on the reference determinant
    uint64_t ref[SCI_MAX_WORDS];    // the reference: alpha 0..na-1, beta 0..nb-1
    const uint64_t *sel;
    int64_t n_sel;
    const double *psi;
    double *hpsi;      // [n_sel]
    double *partial;   // [2][n_blocks]
    double *partial_rows;  // [n_col][n_sel] off-diagonal partial row sums
    double *scalars;   // [2]: numerator, denominator
    double *energy;    // [1]
    double *grad;      // nullable [n_sel]
    uint32_t *flags;
    // enumeration only: empty orbitals per spin and the lexicographic pairs (i | j << 8)
    // of v_alpha and v_beta items
    int va, vb;
    const uint16_t *vpairs[2];
};

template <int W>
__device__ __forceinline__ int lowest_bit(const Key<W> &k) {
#pragma unroll
    for (int j = 0; j < W; ++j)
        if (k.w[j]) return 64 * j + __ffsll((unsigned long long)k.w[j]) - 1;
    return -1;
}

// static word indexing keeps the key in registers (a runtime index would put it in scratch)
template <int W>
__device__ __forceinline__ void clear_bit(Key<W> &k, int b) {
    const uint64_t m = ~(1ull << (b & 63));
#pragma unroll
    for (int j = 0; j < W; ++j)
        if ((b >> 6) == j) k.w[j] &= m;
}

// <bra|H|ket> for bra = ket with one or two electrons moved (x = bra ^ ket, pc = popcount(x))
template <int W>
__device__ double offdiag_elem(const EnergyArgs &a, const Key<W> &bra, const Key<W> &ket, const Key<W> &x,
                               int pc) {
    const int n = a.n;
    Key<W> holes, parts;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        holes.w[j] = ket.w[j] & x.w[j];
        parts.w[j] = bra.w[j] & x.w[j];
    }
    // malformed input (unequal popcounts, bits at or above 2n, spin changes) contributes nothing;
    // the caller flags such determinants
    if (key_popc<W>(holes) * 2 != pc || key_popc<W>(parts) * 2 != pc) return 0.0;
    if (pc == 2) {
        const int P = lowest_bit<W>(holes), A = lowest_bit<W>(parts);
        if (P >= 2 * n || A >= 2 * n || (P >= n) != (A >= n)) return 0.0;
        const int sg = P >= n ? 1 : 0;
        const int p = P - sg * n, t = A - sg * n;
        const int par = key_popc_below<W>(ket, P) + key_popc_below<W>(ket, A) - (P < A ? 1 : 0);
        double v = a.h1[t * n + p];
        const double *jr = a.jtpq + (int64_t)(t * n + p) * n;  // (tp|qq) over q
        const double *kr = a.ktpq + (int64_t)(t * n + p) * n;  // (tq|qp) over q
        // The sum over the ket's occupied spin orbitals Q may include Q = P, whose term
        // (tp|pp) - (tp|pp) is exactly zero.  It is the reference's sum (a table entry)
        // corrected by the spin orbitals in which the ket and the reference differ,
        // when those are fewer than the ket's electrons.
        Key<W> gain, loss;
#pragma unroll
        for (int j = 0; j < W; ++j) {
            gain.w[j] = ket.w[j] & ~a.ref[j];
            loss.w[j] = a.ref[j] & ~ket.w[j];
        }
        if (2 * key_popc<W>(gain) < a.na + a.nb) {
            v = a.fref[((int64_t)sg * n + t) * n + p];
            while (true) {
                const int Q = lowest_bit<W>(gain);
                if (Q < 0 || Q >= 2 * n) break;
                clear_bit<W>(gain, Q);
                const int s2 = Q >= n ? 1 : 0;
                const int q = Q - s2 * n;
                v += jr[q] - ((s2 == sg) ? kr[q] : 0.0);
            }
            while (true) {
                const int Q = lowest_bit<W>(loss);
                if (Q < 0) break;
                clear_bit<W>(loss, Q);
                const int s2 = Q >= n ? 1 : 0;
                const int q = Q - s2 * n;
                v -= jr[q] - ((s2 == sg) ? kr[q] : 0.0);
            }
            return (par & 1) ? -v : v;
        }
        // occupied spin orbitals of the ket in ascending order (alpha block, then beta)
        Key<W> occ = ket;
        while (true) {
            const int Q = lowest_bit<W>(occ);
            if (Q < 0 || Q >= 2 * n) break;
            clear_bit<W>(occ, Q);
            if (Q == P) continue;
            const int s2 = Q >= n ? 1 : 0;
            const int q = Q - s2 * n;
            const double jv = jr[q];
            const double kv = (s2 == sg) ? kr[q] : 0.0;
            v += jv - kv;
        }
        return (par & 1) ? -v : v;
    }
    // pc == 4: holes P<Q, particles A<B
    const int P = lowest_bit<W>(holes);
    clear_bit<W>(holes, P);
    const int Q = lowest_bit<W>(holes);
    const int A = lowest_bit<W>(parts);
    clear_bit<W>(parts, A);
    const int B = lowest_bit<W>(parts);
    if (Q >= 2 * n || B >= 2 * n) return 0.0;
    if ((P >= n) != (A >= n) || (Q >= n) != (B >= n)) return 0.0;  // spin of each pair conserved
    const int par = key_popc_below<W>(ket, P) + key_popc_below<W>(ket, Q) - 1 + key_popc_below<W>(ket, B) -
                    (P < B) - (Q < B) + key_popc_below<W>(ket, A) - (P < A) - (Q < A);
    const int sp = P >= n, sq = Q >= n;
    const int p = P - sp * n, q = Q - sq * n;
    const int ta = A - (A >= n) * n, tb = B - (B >= n) * n;
    const int64_t idx = ((int64_t)(p * n + q) * n + ta) * n + tb;
    const double v = (sp == sq) ? a.vanti[idx] : a.vdir[idx];
    return (par & 1) ? -v : v;
}

template <int W>
__device__ double diag_elem(const EnergyArgs &a, const Key<W> &d) {
    const int n = a.n;
    double e1 = 0.0, e2 = 0.0;
    Key<W> occ = d;
    // ignore bits at or above 2n (such determinants are flagged by the caller)
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const int lo = 64 * j;
        if (2 * n <= lo) occ.w[j] = 0;
        else if (2 * n < lo + 64) occ.w[j] &= (1ull << (2 * n - lo)) - 1ull;
    }
    while (true) {
        const int P = lowest_bit<W>(occ);
        if (P < 0) break;
        clear_bit<W>(occ, P);
        const int sp = P >= n, p = P - sp * n;
        e1 += a.h1[p * n + p];
        Key<W> rest = occ;  // spin orbitals above P
        while (true) {
            const int Q = lowest_bit<W>(rest);
            if (Q < 0) break;
            clear_bit<W>(rest, Q);
            const int sq = Q >= n, q = Q - sq * n;
            e2 += a.jmat[p * n + q] - ((sp == sq) ? a.kmat[p * n + q] : 0.0);
        }
    }
    return e1 + e2;
}

// Off-diagonal part of (H psi)_i for the rows of blockIdx.x against the
// columns of column block blockIdx.y; the partial sum goes to
// partial_rows[blockIdx.y][i] (combined in a fixed order by hpsi_finish_kernel).
//
// Screening is a dense contraction.  With each determinant read as a 0/1 vector
// over the 2n spin orbitals, D_i XOR D_j has 2N - 2 <D_i, D_j> set bits when both
// hold N electrons, so the pair is connected (two or four bits) exactly when the
// overlap is N - 1 or N - 2.  Each wave computes the overlaps of its 64 rows with 32
// columns at a time by 8-bit matrix-core products (32 x 32 x 32 per instruction,
// the bits expanded to bytes), accumulating from 2 - N so that a connected pair
// reads 0 or 1.  Connected pairs wait in a per-wave LDS queue and are evaluated
// 64 at a time with every lane busy (one entry per lane, the row's determinant
// fetched from its owner lane, the excitation rebuilt from the exact XOR).  The
// pairs of one row and one group of 32 columns are consecutive in the queue, in
// ascending column order; the row lane records each such segment and adds its
// entries in queue order, so every row still sums its terms in ascending j.
constexpr int kQueue = 2 * kWave;
constexpr int kSlots = 8;  // queue segments per row lane before the queue is flushed

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// bits [32c + 16g, 32c + 16g + 16) of a key, bit b to byte b (0 or 1) of the result
template <int W, int C>
__device__ __forceinline__ v4i key_bytes16(const Key<W> &k, int g) {
    const uint32_t x = (uint32_t)(k.w[C / 2] >> (32 * (C % 2) + 16 * g)) & 0xffffu;
    v4i r;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        // nibble bits 0..3 land on bits 0, 8, 16, 24: the four shifted copies occupy
        // disjoint bit ranges, so the product has no carries
        r[d] = (int)((((x >> (4 * d)) & 15u) * 0x00204081u) & 0x01010101u);
    }
    return r;
}

template <int W>
__device__ __forceinline__ void flush_queue(const EnergyArgs &a, const Key<W> &di, int n_q, const uint32_t *q_ent,
                                           double *q_val, const uint16_t *q_seg, int mine, const Key<W> *tile_keys,
                                           const double *tile_psi, double &acc) {
    const int lane = threadIdx.x & (kWave - 1);
    for (int base = 0; base < n_q; base += kWave) {
        const int k = base + lane;
        const uint32_t e = k < n_q ? q_ent[k] : 0u;
        const int r = (int)(e >> 16);
        Key<W> bra;
#pragma unroll
        for (int j = 0; j < W; ++j) bra.w[j] = __shfl(di.w[j], r);
        if (k < n_q) {
            const int t = (int)(e & 0x3ffu);
            const Key<W> ket = tile_keys[t];
            Key<W> x;
#pragma unroll
            for (int j = 0; j < W; ++j) x.w[j] = bra.w[j] ^ ket.w[j];
            // the overlap test is exact for determinants of N electrons; others (flagged)
            // can pass it without being connected and contribute nothing
            const int pc = key_popc<W>(x);
            q_val[k] = (pc == 2 || pc == 4) ? offdiag_elem<W>(a, bra, ket, x, pc) * tile_psi[t] : 0.0;
        }
    }
    __builtin_amdgcn_wave_barrier();
    for (int j = 0; j < mine; ++j) {
        const uint32_t sg = q_seg[lane * kSlots + j];
        const int k0 = (int)(sg & 0xffu), k1 = k0 + (int)(sg >> 8);
        for (int k = k0; k < k1; ++k) acc += q_val[k];
    }
    __builtin_amdgcn_wave_barrier();
}

template <int W>
struct HpsiLds {
    Key<W> tile_keys[kColTile];
    double tile_psi[kColTile];
    uint32_t ent[kRowThreads / kWave][kQueue];  // (row lane << 16) | column
    double val[kRowThreads / kWave][kQueue];
    uint16_t seg[kRowThreads / kWave][kWave * kSlots];  // each row lane's queue segments: start | count << 8
};

// rows [rb*256, rb*256+256) against column block cb of n_col
template <int W>
__device__ __forceinline__ void hpsi_tile(const EnergyArgs &a, int64_t rb, int cb, int n_col, HpsiLds<W> &S) {
    Key<W> *tile_keys = S.tile_keys;
    double *tile_psi = S.tile_psi;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), w = tid / kWave, g = lane >> 5;
    const int64_t i = rb * kRowThreads + tid;
    const bool active = i < a.n_sel;
    Key<W> di;
#pragma unroll
    for (int j = 0; j < W; ++j) di.w[j] = 0;
    double acc = 0.0;
    if (active) {
        di = load_key<W>(a.sel, i);
        if (cb == 0) {
            int na, nb;
            spin_popc<W>(di, a.n, na, nb);
            if (na != a.na || nb != a.nb || key_popc<W>(di) != na + nb) atomicOr(a.flags, SCI_FLAG_BAD_DET);
            if (i + 1 < a.n_sel && !key_less<W>(di, load_key<W>(a.sel, i + 1)))
                atomicOr(a.flags, SCI_FLAG_UNSORTED);
        }
    }
    const uint64_t act = __ballot(active);
    // 32-bit chunks of the key that hold spin orbitals (2n bits)
    constexpr int kCh = 2 * W;
    const int nch = (2 * a.n + 31) / 32 < kCh ? (2 * a.n + 31) / 32 : kCh;
    const int bias = 2 - (a.na + a.nb);
    // matrix-core operands of this wave's rows: half h holds rows 32h .. 32h+31, lane
    // l the row 32h + l%32 and bytes 16 (l/32) .. +15 of each chunk.  They are rebuilt
    // after every queue flush, so their registers are free while the queue is evaluated.
    v4i fa[2][kCh];
    auto build_rows = [&]() {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            Key<W> rk;
#pragma unroll
            for (int j = 0; j < W; ++j) rk.w[j] = __shfl(di.w[j], 32 * h + (lane & 31));
#pragma unroll
            for (int c = 0; c < kCh; ++c) {
                if (c == 0) fa[h][c] = key_bytes16<W, 0>(rk, g);
                if (c == 1) fa[h][c] = key_bytes16<W, 1>(rk, g);
                if constexpr (kCh > 2) {
                    if (c == 2) fa[h][c] = key_bytes16<W, (kCh > 2 ? 2 : 0)>(rk, g);
                    if (c == 3) fa[h][c] = key_bytes16<W, (kCh > 2 ? 3 : 0)>(rk, g);
                }
            }
        }
    };
    build_rows();
    uint32_t *q_ent = S.ent[w];
    double *q_val = S.val[w];
    uint16_t *q_seg = S.seg[w];
    const int64_t per = ceil_div_dev(ceil_div_dev(a.n_sel, (int64_t)n_col), (int64_t)kColTile) * kColTile;
    const int64_t c0 = (int64_t)cb * per;
    const int64_t c1 = min<int64_t>(c0 + per, a.n_sel);
    for (int64_t j0 = c0; j0 < c1; j0 += kColTile) {
        const int cnt = (int)min<int64_t>(kColTile, c1 - j0);
        __syncthreads();
        {
            constexpr int U = kColTile / kRowThreads;
            Key<W> kt[U];
            double pt[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = u * kRowThreads + tid;
                if (t < cnt) {
                    kt[u] = load_key<W>(a.sel, j0 + t);
                    pt[u] = a.psi[j0 + t];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = u * kRowThreads + tid;
                if (t < cnt) {
                    tile_keys[t] = kt[u];
                    tile_psi[t] = pt[u];
                }
            }
        }
        __syncthreads();
        int n_q = 0;   // wave-uniform
        int mine = 0;  // this row lane's queue segments
        for (int t0 = 0; t0 < cnt; t0 += 32) {
            const int t = t0 + (lane & 31);
            const bool tv = t < cnt;
            const Key<W> ck = tile_keys[tv ? t : 0];
            // Columns are the first operand and rows the second: accumulator r of product h
            // holds row 32h + l%32 against column t0 + 8(r/4) + 4(l/32) + r%4.  Each lane
            // gathers, per product, its 16 columns' tests into a mask at their column bits.
            // The two products run one after the other through the same accumulators.
            uint32_t mh[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                v16i ov;
#pragma unroll
                for (int r = 0; r < 16; ++r) ov[r] = bias;
#pragma unroll
                for (int c = 0; c < kCh; ++c) {
                    if (c >= nch) break;
                    v4i fb;
                    if (c == 0) fb = key_bytes16<W, 0>(ck, g);
                    if (c == 1) fb = key_bytes16<W, 1>(ck, g);
                    if constexpr (kCh > 2) {
                        if (c == 2) fb = key_bytes16<W, (kCh > 2 ? 2 : 0)>(ck, g);
                        if (c == 3) fb = key_bytes16<W, (kCh > 2 ? 3 : 0)>(ck, g);
                    }
                    ov = __builtin_amdgcn_mfma_i32_32x32x32_i8(fb, fa[h][c], ov, 0, 0, 0);
                }
                uint32_t m = 0u;
#pragma unroll
                for (int r = 0; r < 16; ++r) m |= ((uint32_t)ov[r] < 2u ? 1u : 0u) << (8 * (r >> 2) + (r & 3));
                mh[h] = m << (4 * g);
            }
            const uint32_t m0 = mh[0], m1 = mh[1];
            // this lane's row l = 32g + l%32 is in its product g (its 16 columns) and in
            // product g of lane l^32 (the other 16): each lane keeps one mask, sends the other
            uint32_t M = (g ? m1 : m0) | (uint32_t)__shfl_xor((int)(g ? m0 : m1), 32);
            M &= cnt - t0 >= 32 ? 0xffffffffu : ((1u << (cnt - t0)) - 1u);  // columns inside the tile
            if (!active) M = 0u;
            // the group's entries in row order, each row's in column order: row lane l
            // owns entries [excl, incl) of the group
            const int cr = __popc(M);
            int incl = cr;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const int y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            const int excl = incl - cr;
            const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
            for (int done = 0; done < total;) {
                // entries [done, done + take) of the group fit the queue now
                const int take = min(kQueue - n_q, total - done);
                const int s0 = max(excl, done), s1 = min(incl, done + take);
                if (s1 > s0) {
                    uint32_t mm = M;
                    for (int e = excl; e < s1; ++e) {
                        const int bit = __builtin_ctz(mm);
                        mm &= mm - 1u;
                        if (e >= s0) q_ent[n_q + e - done] = ((uint32_t)lane << 16) | (uint32_t)(t0 + bit);
                    }
                    q_seg[lane * kSlots + mine++] = (uint16_t)((n_q + s0 - done) | ((s1 - s0) << 8));
                }
                n_q += take;
                done += take;
                if (done < total || n_q >= kWave || __ballot(mine >= kSlots) != 0ull) {
                    __builtin_amdgcn_wave_barrier();
                    flush_queue<W>(a, di, n_q, q_ent, q_val, q_seg, mine, tile_keys, tile_psi, acc);
                    n_q = 0;
                    mine = 0;
                    build_rows();
                }
            }
        }
        if (n_q > 0) {
            __builtin_amdgcn_wave_barrier();
            flush_queue<W>(a, di, n_q, q_ent, q_val, q_seg, mine, tile_keys, tile_psi, acc);
        }
    }
    if (active) a.partial_rows[(int64_t)cb * a.n_sel + i] = acc;
}

template <int W>
__global__ __launch_bounds__(kRowThreads) void hpsi_kernel(EnergyArgs a) {
    __shared__ HpsiLds<W> S;
    hpsi_tile<W>(a, blockIdx.x, blockIdx.y, gridDim.y, S);
}

// ---------------------------------------------------------------------------
// off-diagonal row sums by enumeration of C_i and search in the sorted S
// ---------------------------------------------------------------------------

constexpr int kEnumThreads = 256;
constexpr int kEnumTop = 1024;  // every R-th key of S held in LDS (all of S when it fits)

// Position of k in the ascending S[0, n), or -1: the top level (top[t] = S[t R]) is
// searched in LDS, then the R-key block it names in S.
template <int W>
__device__ __forceinline__ int64_t find_sorted(const uint64_t *S, int64_t n, const Key<W> *top, int nt, int64_t R,
                                               const Key<W> &k) {
    int lo = 0, hi = nt;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (key_less<W>(k, top[mid])) hi = mid;
        else lo = mid + 1;
    }
    if (lo == 0) return -1;  // below S[0]
    int64_t b = (int64_t)(lo - 1) * R, e = b + R < n ? b + R : n;
    while (b < e) {
        const int64_t mid = b + ((e - b) >> 1);
        const Key<W> m = load_key<W>(S, mid);
        if (key_less<W>(m, k)) b = mid + 1;
        else if (key_less<W>(k, m)) e = mid;
        else return mid;
    }
    return -1;
}

struct EnumLds {
    uint8_t occ[2][64];
    uint8_t vir[2][64];
    int bad;
    double wsum[kEnumThreads / kWave];
};

// A persistent grid over the rows: per row i, every excitation of D_i (rows of
// excitations sharing their holes, lanes over the particles) is searched in S; a
// member j adds <D_i|H|D_j> psi_j.  The row's sum goes to partial_rows[0][i].
template <int W>
__global__ __launch_bounds__(kEnumThreads) void hpsi_enum_kernel(EnergyArgs a) {
    __shared__ Key<W> top[kEnumTop];
    __shared__ EnumLds L;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int64_t nS = a.n_sel;
    const int64_t R = ceil_div_dev(nS, kEnumTop);
    const int nt = (int)ceil_div_dev(nS, R);
    for (int t = tid; t < nt; t += kEnumThreads) top[t] = load_key<W>(a.sel, (int64_t)t * R);
    const int n = a.n;
    const int pa = a.na * (a.na - 1) / 2, pb = a.nb * (a.nb - 1) / 2;
    const int g1 = a.na, g2 = g1 + a.nb, g3 = g2 + pa, g4 = g3 + pb, n_rows = g4 + a.na * a.nb;
    const int pva = a.va * (a.va - 1) / 2, pvb = a.vb * (a.vb - 1) / 2;
    for (int64_t i = blockIdx.x; i < nS; i += gridDim.x) {
        __syncthreads();  // the previous row is done with L (and top is loaded)
        const Key<W> di = load_key<W>(a.sel, i);
        if (tid == 0) {
            int na, nb;
            spin_popc<W>(di, n, na, nb);
            L.bad = (na != a.na || nb != a.nb || key_popc<W>(di) != na + nb) ? 1 : 0;
            if (L.bad) atomicOr(a.flags, SCI_FLAG_BAD_DET);
            if (i + 1 < nS && !key_less<W>(di, load_key<W>(a.sel, i + 1))) atomicOr(a.flags, SCI_FLAG_UNSORTED);
        }
        if (tid < 2 * n) {
            const int sg = tid >= n ? 1 : 0;
            const int p = tid - sg * n;
            const int below = key_popc_below<W>(di, tid) - (sg ? key_popc_below<W>(di, n) : 0);
            uint64_t word = di.w[0];
#pragma unroll
            for (int j = 1; j < W; ++j) word = ((tid >> 6) == j) ? di.w[j] : word;
            if ((word >> (tid & 63)) & 1ull) {
                if (below < 64) L.occ[sg][below] = (uint8_t)p;
            } else if (p - below >= 0 && p - below < 64) {
                L.vir[sg][p - below] = (uint8_t)p;
            }
        }
        __syncthreads();
        double acc = 0.0;
        if (!L.bad) {
            for (int g = wave; g < n_rows; g += kEnumThreads / kWave) {
                Key<W> rk = di;
                int R_len, sg = 0, kind;  // kind 0 single, 1 same-spin double, 2 mixed double
                if (g < g2) {
                    sg = g < g1 ? 0 : 1;
                    key_flip<W>(rk, L.occ[sg][sg ? g - g1 : g] + sg * n);
                    R_len = sg ? a.vb : a.va;
                    kind = 0;
                } else if (g < g4) {
                    sg = g < g3 ? 0 : 1;
                    // hole pair o of this spin, lexicographic: o -> (x < y)
                    int o = sg ? g - g3 : g - g2, x = 0, m = sg ? a.nb : a.na;
                    while (o >= m - 1 - x) {
                        o -= m - 1 - x;
                        ++x;
                    }
                    key_flip<W>(rk, L.occ[sg][x] + sg * n);
                    key_flip<W>(rk, L.occ[sg][x + 1 + o] + sg * n);
                    R_len = sg ? pvb : pva;
                    kind = 1;
                } else {
                    const int o = g - g4, ip = o / a.nb, iq = o - ip * a.nb;
                    key_flip<W>(rk, L.occ[0][ip]);
                    key_flip<W>(rk, L.occ[1][iq] + n);
                    R_len = a.va * a.vb;
                    kind = 2;
                }
                for (int t = lane; t < R_len; t += kWave) {
                    Key<W> key = rk;
                    if (kind == 0) {
                        key_flip<W>(key, L.vir[sg][t] + sg * n);
                    } else if (kind == 1) {
                        const uint32_t pv = a.vpairs[sg][t];
                        key_flip<W>(key, L.vir[sg][pv & 0xff] + sg * n);
                        key_flip<W>(key, L.vir[sg][pv >> 8] + sg * n);
                    } else {
                        const int ia = t / a.vb, ib = t - ia * a.vb;
                        key_flip<W>(key, L.vir[0][ia]);
                        key_flip<W>(key, L.vir[1][ib] + n);
                    }
                    const int64_t j = find_sorted<W>(a.sel, nS, top, nt, R, key);
                    if (j >= 0) {
                        Key<W> x;
#pragma unroll
                        for (int q = 0; q < W; ++q) x.w[q] = di.w[q] ^ key.w[q];
                        acc += offdiag_elem<W>(a, di, key, x, kind == 0 ? 2 : 4) * a.psi[j];
                    }
                }
            }
        }
        // fixed-order block sum: a butterfly inside each wave, then the waves in order
        for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) L.wsum[wave] = acc;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < kEnumThreads / kWave; ++w) t += L.wsum[w];
            a.partial_rows[i] = t;
        }
    }
}

// (H psi)_i = H_ii psi_i + the column-block partial sums in block order
template <int W>
__device__ __forceinline__ void hpsi_finish_rows(const EnergyArgs &a, int64_t rb, int n_col) {
    const int64_t i = rb * kRowThreads + threadIdx.x;
    if (i >= a.n_sel) return;
    double acc = 0.0;
    for (int c = 0; c < n_col; ++c) acc += a.partial_rows[(int64_t)c * a.n_sel + i];
    const Key<W> di = load_key<W>(a.sel, i);
    a.hpsi[i] = diag_elem<W>(a, di) * a.psi[i] + acc;
}

template <int W>
__global__ __launch_bounds__(kRowThreads) void hpsi_finish_kernel(EnergyArgs a, int n_col) {
    hpsi_finish_rows<W>(a, blockIdx.x, n_col);
}

// per-block partial sums of psi_i*(H psi)_i and psi_i^2, fixed tree order
__device__ __forceinline__ void reduce_partial_block(const EnergyArgs &a, int64_t blk, double *s_num, double *s_den) {
    const int tid = threadIdx.x;
    const int64_t per_block = (int64_t)kRedThreads * 8;
    const int64_t base = blk * per_block;
    double num = 0.0, den = 0.0;
    for (int k = 0; k < 8; ++k) {
        const int64_t i = base + (int64_t)k * kRedThreads + tid;
        if (i < a.n_sel) {
            const double p = a.psi[i];
            num += p * a.hpsi[i];
            den += p * p;
        }
    }
    s_num[tid] = num;
    s_den[tid] = den;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (tid < s) {
            s_num[tid] += s_num[tid + s];
            s_den[tid] += s_den[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        a.partial[2 * blk] = s_num[0];
        a.partial[2 * blk + 1] = s_den[0];
    }
}

__global__ __launch_bounds__(kRedThreads) void reduce_partial_kernel(EnergyArgs a) {
    __shared__ double s_num[kRedThreads], s_den[kRedThreads];
    reduce_partial_block(a, blockIdx.x, s_num, s_den);
}

__device__ __forceinline__ void reduce_final_all(const EnergyArgs &a, int n_blocks, double *s_num, double *s_den) {
    const int tid = threadIdx.x;
    double num = 0.0, den = 0.0;
    for (int b = tid; b < n_blocks; b += kRedThreads) {
        num += a.partial[2 * b];
        den += a.partial[2 * b + 1];
    }
    s_num[tid] = num;
    s_den[tid] = den;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (tid < s) {
            s_num[tid] += s_num[tid + s];
            s_den[tid] += s_den[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        a.scalars[0] = s_num[0];
        a.scalars[1] = s_den[0];
        a.energy[0] = s_num[0] / s_den[0];
    }
}

__global__ __launch_bounds__(kRedThreads) void reduce_final_kernel(EnergyArgs a, int n_blocks) {
    __shared__ double s_num[kRedThreads], s_den[kRedThreads];
    reduce_final_all(a, n_blocks, s_num, s_den);
}

__device__ __forceinline__ void grad_rows(const EnergyArgs &a, int64_t i) {
    if (i >= a.n_sel) return;
    const double e = a.energy[0], den = a.scalars[1];
    a.grad[i] = 2.0 * (a.hpsi[i] - e * a.psi[i]) / den;
}

__global__ void grad_kernel(EnergyArgs a) { grad_rows(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x); }

static int64_t reduce_blocks(int64_t n_sel) { return std::max<int64_t>(1, ceil_div(n_sel, (int64_t)kRedThreads * 8)); }

constexpr int kColSplit = 8;  // column blocks per row block (more workgroups in flight)

static int col_split(int64_t n_sel) { return n_sel >= (int64_t)kColSplit * kColTile ? kColSplit : 1; }

constexpr size_t al256c(size_t b) { return (b + 255) / 256 * 256; }

// workspace layout of one energy call: H psi (when the caller keeps none), per-block
// partial sums, the two scalars, the column-block partial row sums
constexpr size_t energy_ws(int64_t n_sel) {
    return al256c((size_t)n_sel * 8) +
           al256c((size_t)(n_sel > (int64_t)kRedThreads * 8 ? (n_sel + kRedThreads * 8 - 1) / (kRedThreads * 8) : 1) * 16) +
           al256c(16) + al256c((size_t)(n_sel >= (int64_t)kColSplit * kColTile ? kColSplit : 1) * (size_t)n_sel * 8);
}

static EnergyArgs energy_args(const HamDev &d, const uint64_t *sel, int64_t n_sel, const double *psi, double *energy,
                              double *h_psi, double *grad, char *ws, uint32_t *dev_flags) {
    EnergyArgs a;
    a.va = d.v_alpha;
    a.vb = d.v_beta;
    a.vpairs[0] = d.pairs[2];
    a.vpairs[1] = d.pairs[3];
    a.n = d.n_orb;
    a.na = d.n_alpha;
    a.nb = d.n_beta;
    a.h1 = d.h1;
    a.eri = d.eri;
    a.vdir = d.vdir;
    a.vanti = d.vanti;
    a.jmat = d.jmat;
    a.kmat = d.kmat;
    a.jtpq = d.jtpq;
    a.ktpq = d.ktpq;
    a.fref = d.fref;
    for (int j = 0; j < SCI_MAX_WORDS; ++j) a.ref[j] = 0;
    for (int k = 0; k < d.n_alpha; ++k) a.ref[k >> 6] |= 1ull << (k & 63);
    for (int k = d.n_orb; k < d.n_orb + d.n_beta; ++k) a.ref[k >> 6] |= 1ull << (k & 63);
    a.sel = sel;
    a.n_sel = n_sel;
    a.psi = psi;
    a.hpsi = h_psi ? h_psi : (double *)ws;
    const size_t o1 = al256c((size_t)n_sel * 8);
    const size_t o2 = o1 + al256c((size_t)reduce_blocks(n_sel) * 16);
    a.partial = (double *)(ws + o1);
    a.scalars = (double *)(ws + o2);
    a.partial_rows = (double *)(ws + o2 + al256c(16));
    a.energy = energy;
    a.grad = grad;
    a.flags = dev_flags;
    return a;
}

// Membership by enumeration when |S| exceeds N_c by this factor.  Pair screening
// tests |S|^2 pairs (measured 3.6e12 tests/s at |S| = 1e5, 8e10/s at |S| = 1.7e4
// where too few row blocks fill the chip); enumeration builds |S| N_c determinants
// and searches each in S (2-5e10/s).  Measured: |S| = 17,000, N_c = 804: 0.61 ms
// enumeration vs 3.4 ms pairs; |S| = 1e5, N_c = 25,137 and |S| = 2e5, N_c = 361,250:
// pairs (2.8 ms, 70 ms) far ahead.
constexpr int64_t kEnumRatio = 8;

static int pick_method(const HamDev &d, int64_t n_sel, int32_t method) {
    if (method == SCI_ENERGY_PAIRS || method == SCI_ENERGY_ENUM) return method;
    return d.n_coupled * kEnumRatio < n_sel ? SCI_ENERGY_ENUM : SCI_ENERGY_PAIRS;
}

// Every kernel of one energy evaluation, in order, on `st`.  `timed` launches go through
// the per-launch profiler (which may create events); the allocation-free entry point
// launches untimed.
static int32_t energy_launch(int W, const EnergyArgs &a, hipStream_t st, bool timed, int method) {
#define SCI_ELAUNCH(kern, ...)                          \
    do {                                                \
        if (timed) SCI_LAUNCH(kern, __VA_ARGS__);       \
        else hipLaunchKernelGGL(kern, __VA_ARGS__);     \
    } while (0)
    const int64_t n_sel = a.n_sel;
    const int64_t row_blocks = ceil_div(n_sel, kRowThreads);
    if (method == SCI_ENERGY_ENUM) {
        int dev = 0, n_cu = 256;
        if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        const unsigned g = (unsigned)std::min<int64_t>(n_sel, (int64_t)std::max(n_cu, 1) * 8);
        if (W == 1) {
            SCI_ELAUNCH(hpsi_enum_kernel<1>, dim3(g), dim3(kEnumThreads), 0, st, a);
            SCI_ELAUNCH(hpsi_finish_kernel<1>, dim3((unsigned)row_blocks), dim3(kRowThreads), 0, st, a, 1);
        } else {
            SCI_ELAUNCH(hpsi_enum_kernel<2>, dim3(g), dim3(kEnumThreads), 0, st, a);
            SCI_ELAUNCH(hpsi_finish_kernel<2>, dim3((unsigned)row_blocks), dim3(kRowThreads), 0, st, a, 1);
        }
    } else {
        const int nc = col_split(n_sel);
        if (W == 1) {
            SCI_ELAUNCH(hpsi_kernel<1>, dim3((unsigned)row_blocks, nc), dim3(kRowThreads), 0, st, a);
            SCI_ELAUNCH(hpsi_finish_kernel<1>, dim3((unsigned)row_blocks), dim3(kRowThreads), 0, st, a, nc);
        } else {
            SCI_ELAUNCH(hpsi_kernel<2>, dim3((unsigned)row_blocks, nc), dim3(kRowThreads), 0, st, a);
            SCI_ELAUNCH(hpsi_finish_kernel<2>, dim3((unsigned)row_blocks), dim3(kRowThreads), 0, st, a, nc);
        }
    }
    SCI_HIP_TRY(hipGetLastError());
    const int64_t nb = reduce_blocks(n_sel);
    SCI_ELAUNCH(reduce_partial_kernel, dim3((unsigned)nb), dim3(kRedThreads), 0, st, a);
    SCI_HIP_TRY(hipGetLastError());
    SCI_ELAUNCH(reduce_final_kernel, dim3(1), dim3(kRedThreads), 0, st, a, (int)nb);
    SCI_HIP_TRY(hipGetLastError());
    if (a.grad) {
        SCI_ELAUNCH(grad_kernel, dim3((unsigned)ceil_div(n_sel, 256)), dim3(256), 0, st, a);
        SCI_HIP_TRY(hipGetLastError());
    }
#undef SCI_ELAUNCH
    return SCI_OK;
}

// argument checks shared by the energy entry points (everything but the workspace)
static int32_t energy_check(const char *where, sci_ham_t ham, const uint64_t *sel, int64_t n_sel, const double *psi,
                            const double *energy, const uint32_t *dev_flags) {
    if (!ham) return fail(SCI_EINVAL, "%s: NULL handle", where);
    if (n_sel < 1) return fail(SCI_EINVAL, "%s: n_sel must be >= 1", where);
    if (!sel || !psi || !energy || !dev_flags) return fail(SCI_EINVAL, "%s: NULL pointer argument", where);
    if (ham->dev.W > SCI_MAX_WORDS) return fail(SCI_EUNSUPPORTED, "%s: W=%d", where, ham->dev.W);
    return SCI_OK;
}

}  // namespace sci

using namespace sci;

extern "C" size_t sci_energy_workspace_bytes(int64_t n_sel) {
    if (n_sel < 0) return 0;
    return energy_ws(n_sel);
}

extern "C" int32_t sci_energy_method(sci_ham_t ham, int64_t n_sel) {
    if (!ham || n_sel < 1) return -1;
    return pick_method(ham->dev, n_sel, SCI_ENERGY_AUTO);
}

extern "C" int32_t sci_energy_ex(sci_ham_t ham, const uint64_t *sel, int64_t n_sel, const double *psi,
                                 double *energy, double *h_psi, double *grad, int32_t method, void *workspace,
                                 size_t workspace_bytes, uint32_t *dev_flags, sci_stream_t stream) {
    set_error("");
    int32_t rc = energy_check("sci_energy", ham, sel, n_sel, psi, energy, dev_flags);
    if (rc != SCI_OK) return rc;
    if (method < SCI_ENERGY_AUTO || method > SCI_ENERGY_ENUM)
        return fail(SCI_EINVAL, "sci_energy: unknown method %d", method);
    if (!workspace) return fail(SCI_EINVAL, "sci_energy: NULL pointer argument");
    if (workspace_bytes < energy_ws(n_sel))
        return fail(SCI_ECAPACITY, "sci_energy: workspace %zu < %zu bytes", workspace_bytes, energy_ws(n_sel));
    const EnergyArgs a = energy_args(ham->dev, sel, n_sel, psi, energy, h_psi, grad, (char *)workspace, dev_flags);
    return energy_launch(ham->dev.W, a, (hipStream_t)stream, true, pick_method(ham->dev, n_sel, method));
}

extern "C" int32_t sci_energy(sci_ham_t ham, const uint64_t *sel, int64_t n_sel, const double *psi,
                              double *energy, double *h_psi, double *grad, void *workspace,
                              size_t workspace_bytes, uint32_t *dev_flags, sci_stream_t stream) {
    return sci_energy_ex(ham, sel, n_sel, psi, energy, h_psi, grad, SCI_ENERGY_AUTO, workspace, workspace_bytes,
                         dev_flags, stream);
}

// ---------------------------------------------------------------------------
// allocation-free variant: the workspace lives in a file-scope device array
// ---------------------------------------------------------------------------

namespace sci {

constexpr int64_t kNoAllocMaxSel = 1 << 18;
constexpr size_t kNoAllocBytes = energy_ws(kNoAllocMaxSel);

// One copy per device, held until the process ends.  In host code `scratch` names
// a host-side stand-in, never the device memory: kernels get the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch, looked up on the first call per device.
static int32_t scratch_address(char **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(SCI_EHIP, "sci_energy_noalloc: no usable current device (%d)", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SCI_EHIP, "sci_energy_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = (char *)p;
    }
    *out = g_scratch_ptr[dev];
    return SCI_OK;
}

}  // namespace sci

extern "C" int64_t sci_energy_noalloc_max_sel(void) { return kNoAllocMaxSel; }

extern "C" int32_t sci_energy_noalloc(sci_ham_t ham, const uint64_t *sel, int64_t n_sel, const double *psi,
                                      double *energy, double *h_psi, double *grad, uint32_t *dev_flags,
                                      sci_stream_t stream) {
    set_error("");
    int32_t rc = energy_check("sci_energy_noalloc", ham, sel, n_sel, psi, energy, dev_flags);
    if (rc != SCI_OK) return rc;
    if (n_sel > kNoAllocMaxSel)
        return fail(SCI_ECAPACITY, "sci_energy_noalloc: n_sel=%lld exceeds the scratch limit of %lld determinants",
                    (long long)n_sel, (long long)kNoAllocMaxSel);
    char *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc != SCI_OK) return rc;
    // every scratch word the kernels read is written earlier in the same call, so
    // nothing needs clearing; launches bypass the per-launch profiler (it creates events)
    const EnergyArgs a = energy_args(ham->dev, sel, n_sel, psi, energy, h_psi, grad, ws, dev_flags);
    return energy_launch(ham->dev.W, a, (hipStream_t)stream, false, pick_method(ham->dev, n_sel, SCI_ENERGY_AUTO));
}

// ---------------------------------------------------------------------------
// batches of systems: the same per-block work as sci_energy, over tile lists
// that cover every system, so each system's results are bit-identical to its
// own sci_energy call
// ---------------------------------------------------------------------------

namespace sci {

struct EnergyTile {
    int32_t item;
    int32_t cb;  // column block (H psi tiles)
    int64_t rb;  // row block of 256 (H psi, finish, gradient) or reduction block
};

template <int W>
__global__ __launch_bounds__(kRowThreads) void hpsi_batched_kernel(const EnergyArgs *__restrict__ items,
                                                                   const int32_t *__restrict__ ncol,
                                                                   const EnergyTile *__restrict__ tiles) {
    __shared__ HpsiLds<W> S;
    const EnergyTile t = tiles[blockIdx.x];
    hpsi_tile<W>(items[t.item], t.rb, t.cb, ncol[t.item], S);
}

template <int W>
__global__ __launch_bounds__(kRowThreads) void hpsi_finish_batched_kernel(const EnergyArgs *__restrict__ items,
                                                                          const int32_t *__restrict__ ncol,
                                                                          const EnergyTile *__restrict__ rows) {
    const EnergyTile t = rows[blockIdx.x];
    hpsi_finish_rows<W>(items[t.item], t.rb, ncol[t.item]);
}

__global__ __launch_bounds__(kRedThreads) void reduce_partial_batched_kernel(const EnergyArgs *__restrict__ items,
                                                                             const EnergyTile *__restrict__ blocks) {
    __shared__ double s_num[kRedThreads], s_den[kRedThreads];
    const EnergyTile t = blocks[blockIdx.x];
    reduce_partial_block(items[t.item], t.rb, s_num, s_den);
}

__global__ __launch_bounds__(kRedThreads) void reduce_final_batched_kernel(const EnergyArgs *__restrict__ items,
                                                                           const int32_t *__restrict__ n_blocks) {
    __shared__ double s_num[kRedThreads], s_den[kRedThreads];
    reduce_final_all(items[blockIdx.x], n_blocks[blockIdx.x], s_num, s_den);
}

__global__ __launch_bounds__(kRowThreads) void grad_batched_kernel(const EnergyArgs *__restrict__ items,
                                                                   const EnergyTile *__restrict__ rows) {
    const EnergyTile t = rows[blockIdx.x];
    const EnergyArgs &a = items[t.item];
    if (a.grad) grad_rows(a, t.rb * kRowThreads + threadIdx.x);
}

}  // namespace sci

struct sci_energy_batch_s {
    int n_items = 0;
    EnergyArgs *d_items = nullptr;
    int32_t *d_ncol = nullptr, *d_nblk = nullptr;
    EnergyTile *d_tiles = nullptr;  // H psi tiles (W=1, W=2), row tiles (W=1, W=2), reduction blocks
    int64_t n_hpsi[2] = {0, 0}, n_rows[2] = {0, 0}, n_red = 0;
    char *d_ws = nullptr;
};

extern "C" int32_t sci_energy_batch_destroy(sci_energy_batch_t b) {
    if (!b) return SCI_OK;
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_ncol) (void)hipFree(b->d_ncol);
    if (b->d_nblk) (void)hipFree(b->d_nblk);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_ws) (void)hipFree(b->d_ws);
    delete b;
    return SCI_OK;
}

static int32_t energy_batch_create_impl(const sci_energy_item *items, int32_t n_items, uint32_t *dev_flags,
                                        sci_energy_batch_t *out);

extern "C" int32_t sci_energy_batch_create(const sci_energy_item *items, int32_t n_items, uint32_t *dev_flags,
                                           sci_energy_batch_t *out) {
    set_error("");
    return guarded("sci_energy_batch_create", [&] { return energy_batch_create_impl(items, n_items, dev_flags, out); });
}

// Host vectors are built before anything is allocated on the device, so a throw
// from them leaves nothing behind.
static int32_t energy_batch_create_impl(const sci_energy_item *items, int32_t n_items, uint32_t *dev_flags,
                                        sci_energy_batch_t *out) {
    if (!out) return fail(SCI_EINVAL, "sci_energy_batch_create: NULL output handle");
    *out = nullptr;
    if (n_items < 1 || !items) return fail(SCI_EINVAL, "sci_energy_batch_create: empty item list");
    if (!dev_flags) return fail(SCI_EINVAL, "sci_energy_batch_create: dev_flags is NULL");
    std::vector<EnergyArgs> args((size_t)n_items);
    std::vector<int32_t> ncol((size_t)n_items), nblk((size_t)n_items);
    std::vector<size_t> ws_off((size_t)n_items);
    std::vector<EnergyTile> hp[2], rows[2], red;
    size_t ws = 0;
    for (int32_t i = 0; i < n_items; ++i) {
        const sci_energy_item &it = items[i];
        if (!it.ham) return fail(SCI_EINVAL, "sci_energy_batch_create: item %d has no handle", i);
        if (it.n_sel < 1) return fail(SCI_EINVAL, "sci_energy_batch_create: item %d has n_sel < 1", i);
        if (!it.sel || !it.psi || !it.energy) return fail(SCI_EINVAL, "sci_energy_batch_create: item %d NULL buffer", i);
        const HamDev &d = it.ham->dev;
        if (d.W > SCI_MAX_WORDS) return fail(SCI_EUNSUPPORTED, "sci_energy_batch_create: item %d W=%d", i, d.W);
        ws_off[(size_t)i] = ws;
        ws += energy_ws(it.n_sel);
        ncol[(size_t)i] = col_split(it.n_sel);
        nblk[(size_t)i] = (int32_t)reduce_blocks(it.n_sel);
        const int w = d.W - 1;
        const int64_t row_blocks = ceil_div(it.n_sel, kRowThreads);
        for (int64_t rb = 0; rb < row_blocks; ++rb) {
            for (int cb = 0; cb < ncol[(size_t)i]; ++cb) hp[w].push_back(EnergyTile{i, cb, rb});
            rows[w].push_back(EnergyTile{i, 0, rb});
        }
        for (int64_t k = 0; k < nblk[(size_t)i]; ++k) red.push_back(EnergyTile{i, 0, k});
    }
    std::vector<EnergyTile> tiles;
    for (int w = 0; w < 2; ++w) tiles.insert(tiles.end(), hp[w].begin(), hp[w].end());
    for (int w = 0; w < 2; ++w) tiles.insert(tiles.end(), rows[w].begin(), rows[w].end());
    tiles.insert(tiles.end(), red.begin(), red.end());

    sci_energy_batch_s *b = new (std::nothrow) sci_energy_batch_s;
    if (!b) return fail(SCI_ENOMEM, "sci_energy_batch_create: host allocation failed");
    b->n_items = n_items;
    b->n_hpsi[0] = (int64_t)hp[0].size();
    b->n_hpsi[1] = (int64_t)hp[1].size();
    b->n_rows[0] = (int64_t)rows[0].size();
    b->n_rows[1] = (int64_t)rows[1].size();
    b->n_red = (int64_t)red.size();
    auto bail = [&](int32_t st) {
        sci_energy_batch_destroy(b);
        return st;
    };
    if (hipMalloc((void **)&b->d_items, args.size() * sizeof(EnergyArgs)) != hipSuccess ||
        hipMalloc((void **)&b->d_ncol, ncol.size() * 4) != hipSuccess ||
        hipMalloc((void **)&b->d_nblk, nblk.size() * 4) != hipSuccess ||
        hipMalloc((void **)&b->d_tiles, tiles.size() * sizeof(EnergyTile)) != hipSuccess ||
        hipMalloc((void **)&b->d_ws, std::max<size_t>(ws, 256)) != hipSuccess)
        return bail(fail(SCI_ENOMEM, "sci_energy_batch_create: device allocation failed"));
    for (int32_t i = 0; i < n_items; ++i) {
        const sci_energy_item &it = items[i];
        const HamDev &d = it.ham->dev;
        const int64_t n_sel = it.n_sel;
        args[(size_t)i] = energy_args(d, it.sel, n_sel, it.psi, it.energy, it.h_psi, it.grad,
                                      b->d_ws + ws_off[(size_t)i], dev_flags);
    }
    if (hipMemcpy(b->d_items, args.data(), args.size() * sizeof(EnergyArgs), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_ncol, ncol.data(), ncol.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_nblk, nblk.data(), nblk.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_tiles, tiles.data(), tiles.size() * sizeof(EnergyTile), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(SCI_EHIP, "sci_energy_batch_create: upload failed"));
    *out = b;
    return SCI_OK;
}

extern "C" int32_t sci_energy_batched(sci_energy_batch_t b, sci_stream_t stream) {
    set_error("");
    if (!b) return fail(SCI_EINVAL, "sci_energy_batched: NULL handle");
    hipStream_t st = (hipStream_t)stream;
    const EnergyArgs *it = b->d_items;
    const EnergyTile *hp1 = b->d_tiles, *hp2 = hp1 + b->n_hpsi[0];
    const EnergyTile *r1 = hp2 + b->n_hpsi[1], *r2 = r1 + b->n_rows[0], *red = r2 + b->n_rows[1];
    if (b->n_hpsi[0]) SCI_LAUNCH(hpsi_batched_kernel<1>, dim3((unsigned)b->n_hpsi[0]), dim3(kRowThreads), 0, st, it, b->d_ncol, hp1);
    if (b->n_hpsi[1]) SCI_LAUNCH(hpsi_batched_kernel<2>, dim3((unsigned)b->n_hpsi[1]), dim3(kRowThreads), 0, st, it, b->d_ncol, hp2);
    if (b->n_rows[0]) SCI_LAUNCH(hpsi_finish_batched_kernel<1>, dim3((unsigned)b->n_rows[0]), dim3(kRowThreads), 0, st, it, b->d_ncol, r1);
    if (b->n_rows[1]) SCI_LAUNCH(hpsi_finish_batched_kernel<2>, dim3((unsigned)b->n_rows[1]), dim3(kRowThreads), 0, st, it, b->d_ncol, r2);
    SCI_LAUNCH(reduce_partial_batched_kernel, dim3((unsigned)b->n_red), dim3(kRedThreads), 0, st, it, red);
    SCI_LAUNCH(reduce_final_batched_kernel, dim3((unsigned)b->n_items), dim3(kRedThreads), 0, st, it, b->d_nblk);
    const int64_t nr = b->n_rows[0] + b->n_rows[1];
    SCI_LAUNCH(grad_batched_kernel, dim3((unsigned)nr), dim3(kRowThreads), 0, st, it, r1);
    SCI_HIP_TRY(hipGetLastError());
    return SCI_OK;
}
