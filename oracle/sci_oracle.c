/*
 * CPU oracle for the NNQS-SCI hot path.  TEST INFRASTRUCTURE ONLY: it is
 * called by the tests, the smoke check and the CPU-baseline leg of the
 * benchmark, never by the product path.  It shares no code with the HIP
 * library; the only common ground is the determinant encoding below and the
 * seeded input files.
 *
 * What it computes (paper section 2.1, Eqs. 1-5, and sections 4.1-4.2):
 *   - the Hamiltonian  H = sum_PQ h_PQ a+_P a_Q
 *                        + 1/2 sum_PQRS <PQ|RS> a+_P a+_Q a_S a_R
 *     over spin orbitals, with h_PQ = h_pq d(sP,sQ) and
 *     <PQ|RS> = (pr|qs) d(sP,sR) d(sQ,sS) (chemists' (pq|rs), real, 8-fold
 *     symmetric).  The paper never writes the operator; this is the standard
 *     second-quantised form of the Hermitian H of Eq. 1.
 *   - the coupled set C_i of Eq. 4: determinants reached from D_i by moving
 *     one or two occupied positions (spin conserving), with H_ji.
 *   - global de-duplication: the sorted set union of section 4.1.
 *   - the Rayleigh quotient of Eq. 1 restricted to the selected space, and its
 *     exact gradient 2(H psi - E psi)/(psi.psi).
 *
 * Encoding: spin orbital k = p + sigma*n_orb (alpha block, then beta block);
 * bit k lives in word k>>6 at bit k&63; keys compare as unsigned integers
 * with word W-1 most significant.
 *
 * Phase convention: |D> = a+_{k1} a+_{k2} ... a+_{kN} |0> with k1 < k2 < ...;
 * a_k and a+_k pick up (-1)^(number of occupied spin orbitals below k).
 *
 * Two tiers:
 *   literal  : every term of H applied by explicit a / a+ operators (the
 *              definition; cost (2 n_orb)^4 per determinant, tiny systems).
 *   Slater-Condon : one term per excitation, still applied by explicit
 *              operators, matrix element by the Slater-Condon rules.  Pinned
 *              to the literal tier by the tests.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_MAXW 4

typedef struct {
    int n_orb, n_alpha, n_beta, W;
    const double *h;    /* [n][n] */
    const double *eri;  /* [n][n][n][n], (pq|rs) */
} ora_ham;

/* ------------------------------------------------------------------------ */
/* bits and operators                                                         */
/* ------------------------------------------------------------------------ */

static int bit_get(const uint64_t *d, int k) { return (int)((d[k >> 6] >> (k & 63)) & 1u); }
static void bit_flip(uint64_t *d, int k) { d[k >> 6] ^= (uint64_t)1 << (k & 63); }

static int count_below(const uint64_t *d, int W, int k)
{
    int c = 0;
    for (int j = 0; j < k; ++j) c += bit_get(d, j);
    (void)W;
    return c;
}

/* a_k |d> : returns 0 if orbital k is empty, else the sign; d is updated */
static int annihilate(uint64_t *d, int W, int k)
{
    if (!bit_get(d, k)) return 0;
    int s = (count_below(d, W, k) & 1) ? -1 : 1;
    bit_flip(d, k);
    return s;
}

/* a+_k |d> */
static int create(uint64_t *d, int W, int k)
{
    if (bit_get(d, k)) return 0;
    int s = (count_below(d, W, k) & 1) ? -1 : 1;
    bit_flip(d, k);
    return s;
}

static int key_cmp(const uint64_t *a, const uint64_t *b, int W)
{
    for (int w = W - 1; w >= 0; --w) {
        if (a[w] < b[w]) return -1;
        if (a[w] > b[w]) return 1;
    }
    return 0;
}

static int spin_of(const ora_ham *H, int k) { return k >= H->n_orb; }
static int spatial_of(const ora_ham *H, int k) { return k >= H->n_orb ? k - H->n_orb : k; }

static double h_so(const ora_ham *H, int P, int Q)
{
    if (spin_of(H, P) != spin_of(H, Q)) return 0.0;
    int n = H->n_orb;
    return H->h[spatial_of(H, P) * n + spatial_of(H, Q)];
}

static double chem(const ora_ham *H, int p, int q, int r, int s)
{
    int n = H->n_orb;
    return H->eri[(((size_t)p * n + q) * n + r) * n + s];
}

/* physicists' <PQ|RS> over spin orbitals */
static double phys_so(const ora_ham *H, int P, int Q, int R, int S)
{
    if (spin_of(H, P) != spin_of(H, R)) return 0.0;
    if (spin_of(H, Q) != spin_of(H, S)) return 0.0;
    return chem(H, spatial_of(H, P), spatial_of(H, R), spatial_of(H, Q), spatial_of(H, S));
}

/* ------------------------------------------------------------------------ */
/* validation                                                                */
/* ------------------------------------------------------------------------ */

static int det_valid(const ora_ham *H, const uint64_t *d)
{
    int na = 0, nb = 0, n = H->n_orb;
    for (int k = 0; k < 64 * H->W; ++k) {
        if (!bit_get(d, k)) continue;
        if (k < n) na++;
        else if (k < 2 * n) nb++;
        else return 0;
    }
    return na == H->n_alpha && nb == H->n_beta;
}

/* ------------------------------------------------------------------------ */
/* literal tier                                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t key[ORA_MAXW];
    int64_t order;
    double val;
} term_rec;

static int W_sort;
static int term_cmp(const void *a, const void *b)
{
    const term_rec *x = (const term_rec *)a, *y = (const term_rec *)b;
    int c = key_cmp(x->key, y->key, W_sort);
    if (c) return c;
    return (x->order > y->order) - (x->order < y->order);
}

static void push_term(term_rec **buf, int64_t *len, int64_t *cap, const uint64_t *key, int W, double v)
{
    if (*len == *cap) {
        *cap = *cap ? 2 * *cap : 4096;
        *buf = (term_rec *)realloc(*buf, (size_t)*cap * sizeof(term_rec));
    }
    term_rec *t = &(*buf)[*len];
    memset(t->key, 0, sizeof t->key);
    memcpy(t->key, key, (size_t)W * sizeof(uint64_t));
    t->order = *len;
    t->val = v;
    (*len)++;
}

/*
 * H|det> by applying every one- and two-body term with explicit operators.
 * Writes each determinant reached by at least one term (the diagonal
 * included), ascending, with the summed coefficient <det'|H|det>.
 * Returns the count, or -1 if the buffer is too small, -2 if det is invalid.
 */
int64_t ora_literal_row(int n_orb, int n_alpha, int n_beta, int W,
                        const double *h, const double *eri, const uint64_t *det,
                        uint64_t *out_keys, double *out_val, int64_t cap)
{
    ora_ham H = {n_orb, n_alpha, n_beta, W, h, eri};
    if (W < 1 || W > ORA_MAXW || 2 * n_orb > 64 * W) return -2;
    if (!det_valid(&H, det)) return -2;
    int M = 2 * n_orb;
    term_rec *buf = NULL;
    int64_t len = 0, bcap = 0;
    uint64_t d[ORA_MAXW], e[ORA_MAXW];

    /* one-body: h_PQ a+_P a_Q */
    for (int P = 0; P < M; ++P)
        for (int Q = 0; Q < M; ++Q) {
            if (spin_of(&H, P) != spin_of(&H, Q)) continue; /* spin-forbidden term */
            double c = h_so(&H, P, Q);
            memcpy(d, det, (size_t)W * 8);
            int s = annihilate(d, W, Q);
            if (!s) continue;
            int s2 = create(d, W, P);
            if (!s2) continue;
            push_term(&buf, &len, &bcap, d, W, c * s * s2);
        }
    /* two-body: 1/2 <PQ|RS> a+_P a+_Q a_S a_R */
    for (int R = 0; R < M; ++R) {
        memcpy(d, det, (size_t)W * 8);
        int sr = annihilate(d, W, R);
        if (!sr) continue;
        for (int S = 0; S < M; ++S) {
            uint64_t d1[ORA_MAXW];
            memcpy(d1, d, (size_t)W * 8);
            int ss = annihilate(d1, W, S);
            if (!ss) continue;
            for (int Q = 0; Q < M; ++Q) {
                uint64_t d2[ORA_MAXW];
                memcpy(d2, d1, (size_t)W * 8);
                int sq = create(d2, W, Q);
                if (!sq) continue;
                for (int P = 0; P < M; ++P) {
                    if (spin_of(&H, P) != spin_of(&H, R) || spin_of(&H, Q) != spin_of(&H, S))
                        continue; /* spin-forbidden term */
                    memcpy(e, d2, (size_t)W * 8);
                    int sp = create(e, W, P);
                    if (!sp) continue;
                    double c = 0.5 * phys_so(&H, P, Q, R, S);
                    push_term(&buf, &len, &bcap, e, W, c * sr * ss * sq * sp);
                }
            }
        }
    }
    W_sort = W;
    qsort(buf, (size_t)len, sizeof(term_rec), term_cmp);
    int64_t n_out = 0;
    for (int64_t i = 0; i < len;) {
        int64_t j = i;
        double acc = 0.0;
        while (j < len && key_cmp(buf[j].key, buf[i].key, W) == 0) acc += buf[j++].val;
        if (n_out < cap) {
            memcpy(out_keys + n_out * W, buf[i].key, (size_t)W * 8);
            out_val[n_out] = acc;
        }
        n_out++;
        i = j;
    }
    free(buf);
    return n_out <= cap ? n_out : -1;
}

/* ------------------------------------------------------------------------ */
/* Slater-Condon tier                                                         */
/* ------------------------------------------------------------------------ */

static int64_t comb2(int64_t x) { return x * (x - 1) / 2; }

int64_t ora_n_coupled(int n_orb, int n_alpha, int n_beta)
{
    int64_t va = n_orb - n_alpha, vb = n_orb - n_beta;
    return (int64_t)n_alpha * va + (int64_t)n_beta * vb
         + comb2(n_alpha) * comb2(va) + comb2(n_beta) * comb2(vb)
         + (int64_t)n_alpha * va * n_beta * vb;
}

/* <D|H|D> = sum_P h_pp + 1/2 sum_{P != Q} [<PQ|PQ> - <PQ|QP>] */
static double diag_elem(const ora_ham *H, const uint64_t *det)
{
    int M = 2 * H->n_orb;
    double e1 = 0.0, e2 = 0.0;
    for (int P = 0; P < M; ++P) {
        if (!bit_get(det, P)) continue;
        e1 += h_so(H, P, P);
        for (int Q = 0; Q < M; ++Q) {
            if (Q == P || !bit_get(det, Q)) continue;
            e2 += phys_so(H, P, Q, P, Q) - phys_so(H, P, Q, Q, P);
        }
    }
    return e1 + 0.5 * e2;
}

double ora_diag(int n_orb, int n_alpha, int n_beta, int W,
                const double *h, const double *eri, const uint64_t *det)
{
    ora_ham H = {n_orb, n_alpha, n_beta, W, h, eri};
    if (!det_valid(&H, det)) return NAN;
    return diag_elem(&H, det);
}

/* single P -> A: D' = a+_A a_P D,
   H = s [ h_PA' + sum_{Q in occ(D), Q != P} (<AQ|PQ> - <AQ|QP>) ]          */
static double single_elem(const ora_ham *H, const uint64_t *det, int P, int A, uint64_t *out, int *ok)
{
    int W = H->W, M = 2 * H->n_orb;
    memcpy(out, det, (size_t)W * 8);
    int s = annihilate(out, W, P);
    s *= create(out, W, A);
    *ok = (s != 0);
    if (!s) return 0.0;
    double v = h_so(H, A, P);
    for (int Q = 0; Q < M; ++Q) {
        if (Q == P || !bit_get(det, Q)) continue;
        v += phys_so(H, A, Q, P, Q) - phys_so(H, A, Q, Q, P);
    }
    return s * v;
}

/* double P<Q -> A<B: D' = a+_A a+_B a_Q a_P D, H = s (<AB|PQ> - <AB|QP>) */
static double double_elem(const ora_ham *H, const uint64_t *det, int P, int Q, int A, int B,
                          uint64_t *out, int *ok)
{
    int W = H->W;
    memcpy(out, det, (size_t)W * 8);
    int s = annihilate(out, W, P);
    s *= annihilate(out, W, Q);
    s *= create(out, W, B);
    s *= create(out, W, A);
    *ok = (s != 0);
    if (!s) return 0.0;
    return s * (phys_so(H, A, B, P, Q) - phys_so(H, A, B, Q, P));
}

/*
 * All coupled determinants of one source in the canonical order:
 *   alpha singles (p asc, then a asc), beta singles,
 *   alpha-alpha doubles ((p<q) lexicographic, then (a<b) lexicographic),
 *   beta-beta doubles, alpha-beta doubles (p, q, a, b lexicographic),
 * where p,a are alpha (or the spin of the class) and q,b beta for the mixed class.
 * Returns the number written (== ora_n_coupled) or -1.
 */
static int64_t gen_one(const ora_ham *H, const uint64_t *det, uint64_t *keys, double *hij)
{
    int n = H->n_orb, W = H->W;
    int occ[2][128], vir[2][128], no[2] = {0, 0}, nv[2] = {0, 0};
    for (int sg = 0; sg < 2; ++sg)
        for (int p = 0; p < n; ++p) {
            int k = p + sg * n;
            if (bit_get(det, k)) occ[sg][no[sg]++] = k;
            else vir[sg][nv[sg]++] = k;
        }
    int64_t r = 0;
    int ok;
    for (int sg = 0; sg < 2; ++sg)
        for (int i = 0; i < no[sg]; ++i)
            for (int a = 0; a < nv[sg]; ++a) {
                hij[r] = single_elem(H, det, occ[sg][i], vir[sg][a], keys + r * W, &ok);
                if (!ok) return -1;
                r++;
            }
    for (int sg = 0; sg < 2; ++sg)
        for (int i = 0; i < no[sg]; ++i)
            for (int j = i + 1; j < no[sg]; ++j)
                for (int a = 0; a < nv[sg]; ++a)
                    for (int b = a + 1; b < nv[sg]; ++b) {
                        hij[r] = double_elem(H, det, occ[sg][i], occ[sg][j], vir[sg][a], vir[sg][b],
                                             keys + r * W, &ok);
                        if (!ok) return -1;
                        r++;
                    }
    for (int i = 0; i < no[0]; ++i)
        for (int j = 0; j < no[1]; ++j)
            for (int a = 0; a < nv[0]; ++a)
                for (int b = 0; b < nv[1]; ++b) {
                    hij[r] = double_elem(H, det, occ[0][i], occ[1][j], vir[0][a], vir[1][b],
                                         keys + r * W, &ok);
                    if (!ok) return -1;
                    r++;
                }
    return r;
}

/*
 * Coupled generation for n_dets sources.  eps < 0: dense output, entry
 * i*N_coupled + r for source i and rank r (out_src may be NULL).  eps >= 0:
 * only |H| > eps kept, source-major then rank order, out_src filled.
 * Returns the number of entries written, -1 on capacity overflow, -2 on an
 * invalid determinant.
 */
int64_t ora_gen_coupled(int n_orb, int n_alpha, int n_beta, int W,
                        const double *h, const double *eri,
                        const uint64_t *dets, int64_t n_dets, double eps,
                        uint64_t *out_keys, double *out_hij, int32_t *out_src, int64_t cap)
{
    ora_ham H = {n_orb, n_alpha, n_beta, W, h, eri};
    if (W < 1 || W > ORA_MAXW || 2 * n_orb > 64 * W || n_orb > 128) return -2;
    int64_t nc = ora_n_coupled(n_orb, n_alpha, n_beta);
    for (int64_t i = 0; i < n_dets; ++i)
        if (!det_valid(&H, dets + i * W)) return -2;
    if (eps < 0) {
        if (cap < nc * n_dets) return -1;
        int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
        for (int64_t i = 0; i < n_dets; ++i) {
            int64_t got = gen_one(&H, dets + i * W, out_keys + i * nc * W, out_hij + i * nc);
            if (got != nc) bad = 1;
            if (out_src)
                for (int64_t r = 0; r < nc; ++r) out_src[i * nc + r] = (int32_t)i;
        }
        return bad ? -2 : nc * n_dets;
    }
    uint64_t *kb = (uint64_t *)malloc((size_t)nc * W * 8);
    double *hb = (double *)malloc((size_t)nc * 8);
    int64_t n_out = 0;
    for (int64_t i = 0; i < n_dets; ++i) {
        gen_one(&H, dets + i * W, kb, hb);
        for (int64_t r = 0; r < nc; ++r) {
            if (!(fabs(hb[r]) > eps)) continue;
            if (n_out < cap) {
                memcpy(out_keys + n_out * W, kb + r * W, (size_t)W * 8);
                out_hij[n_out] = hb[r];
                if (out_src) out_src[n_out] = (int32_t)i;
            }
            n_out++;
        }
    }
    free(kb);
    free(hb);
    return n_out <= cap ? n_out : -1;
}

/* ------------------------------------------------------------------------ */
/* de-duplication: sorted set union                                           */
/* ------------------------------------------------------------------------ */

static int W_keys;
static int key_qcmp(const void *a, const void *b)
{
    return key_cmp((const uint64_t *)a, (const uint64_t *)b, W_keys);
}

/*
 * out = sorted(set(cand) | set(set_in)); novel = sorted(set(cand) - set(set_in)).
 * set_in must be strictly ascending.  Returns |out|, -1 if set_in is not
 * strictly ascending, -3 on capacity overflow.
 */
int64_t ora_dedup_merge(int W, const uint64_t *cand, int64_t n_cand,
                        const uint64_t *set_in, int64_t n_set,
                        uint64_t *out, int64_t out_cap,
                        uint64_t *novel, int64_t novel_cap, int64_t *n_novel)
{
    for (int64_t i = 1; i < n_set; ++i)
        if (key_cmp(set_in + (i - 1) * W, set_in + i * W, W) >= 0) return -1;
    uint64_t *c = (uint64_t *)malloc((size_t)(n_cand ? n_cand : 1) * W * 8);
    memcpy(c, cand, (size_t)n_cand * W * 8);
    W_keys = W;
    qsort(c, (size_t)n_cand, (size_t)W * 8, key_qcmp);
    int64_t nu = 0;
    for (int64_t i = 0; i < n_cand; ++i)
        if (nu == 0 || key_cmp(c + (nu - 1) * W, c + i * W, W) != 0) {
            memmove(c + nu * W, c + i * W, (size_t)W * 8);
            nu++;
        }
    int64_t a = 0, b = 0, no = 0, nn = 0;
    int overflow = 0;
    while (a < nu || b < n_set) {
        const uint64_t *take;
        int from_c = 0;
        if (b >= n_set) { take = c + a * W; a++; from_c = 1; }
        else if (a >= nu) { take = set_in + b * W; b++; }
        else {
            int k = key_cmp(c + a * W, set_in + b * W, W);
            if (k < 0) { take = c + a * W; a++; from_c = 1; }
            else if (k > 0) { take = set_in + b * W; b++; }
            else { take = set_in + b * W; a++; b++; }
        }
        if (no < out_cap) memcpy(out + no * W, take, (size_t)W * 8);
        else overflow = 1;
        no++;
        if (from_c && novel) {
            if (nn < novel_cap) memcpy(novel + nn * W, take, (size_t)W * 8);
            else overflow = 1;
            nn++;
        }
    }
    if (n_novel) *n_novel = nn;
    free(c);
    return overflow ? -3 : no;
}

/* ------------------------------------------------------------------------ */
/* energy over the selected space                                             */
/* ------------------------------------------------------------------------ */

static int64_t find_key(const uint64_t *sel, int64_t n, int W, const uint64_t *key)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int c = key_cmp(sel + mid * W, key, W);
        if (c == 0) return mid;
        if (c < 0) lo = mid + 1;
        else hi = mid;
    }
    return -1;
}

/*
 * (H psi)_i = H_ii psi_i + sum_{j in C_i, j in S} H_ij psi_j
 * E = psi.(H psi) / psi.psi,  grad = 2 (H psi - E psi) / psi.psi.
 * Sums in long double.  sel must be strictly ascending.  Returns 0, or -1
 * (unsorted), -2 (invalid determinant).
 */
int ora_energy(int n_orb, int n_alpha, int n_beta, int W,
               const double *h, const double *eri,
               const uint64_t *sel, int64_t n_sel, const double *psi,
               double *energy, double *h_psi, double *grad)
{
    ora_ham H = {n_orb, n_alpha, n_beta, W, h, eri};
    for (int64_t i = 1; i < n_sel; ++i)
        if (key_cmp(sel + (i - 1) * W, sel + i * W, W) >= 0) return -1;
    for (int64_t i = 0; i < n_sel; ++i)
        if (!det_valid(&H, sel + i * W)) return -2;
    int64_t nc = ora_n_coupled(n_orb, n_alpha, n_beta);
    long double *hp = (long double *)malloc((size_t)(n_sel ? n_sel : 1) * sizeof(long double));
#pragma omp parallel
    {
        uint64_t *kb = (uint64_t *)malloc((size_t)nc * W * 8);
        double *hb = (double *)malloc((size_t)nc * 8);
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n_sel; ++i) {
            const uint64_t *d = sel + i * W;
            long double acc = (long double)diag_elem(&H, d) * psi[i];
            gen_one(&H, d, kb, hb);
            for (int64_t r = 0; r < nc; ++r) {
                int64_t j = find_key(sel, n_sel, W, kb + r * W);
                if (j >= 0) acc += (long double)hb[r] * psi[j];
            }
            hp[i] = acc;
        }
        free(kb);
        free(hb);
    }
    long double num = 0.0L, den = 0.0L;
    for (int64_t i = 0; i < n_sel; ++i) {
        num += (long double)psi[i] * hp[i];
        den += (long double)psi[i] * psi[i];
    }
    long double e = num / den;
    if (energy) *energy = (double)e;
    for (int64_t i = 0; i < n_sel; ++i) {
        if (h_psi) h_psi[i] = (double)hp[i];
        if (grad) grad[i] = (double)(2.0L * (hp[i] - e * psi[i]) / den);
    }
    free(hp);
    return 0;
}

/* (H psi)_i for the listed rows only (each row independent). */
int ora_hpsi_rows(int n_orb, int n_alpha, int n_beta, int W,
                  const double *h, const double *eri,
                  const uint64_t *sel, int64_t n_sel, const double *psi,
                  const int64_t *rows, int64_t n_rows, double *out)
{
    ora_ham H = {n_orb, n_alpha, n_beta, W, h, eri};
    for (int64_t i = 1; i < n_sel; ++i)
        if (key_cmp(sel + (i - 1) * W, sel + i * W, W) >= 0) return -1;
    int64_t nc = ora_n_coupled(n_orb, n_alpha, n_beta);
    int bad = 0;
#pragma omp parallel reduction(| : bad)
    {
        uint64_t *kb = (uint64_t *)malloc((size_t)nc * W * 8);
        double *hb = (double *)malloc((size_t)nc * 8);
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < n_rows; ++t) {
            int64_t i = rows[t];
            if (i < 0 || i >= n_sel || !det_valid(&H, sel + i * W)) { bad = 1; continue; }
            const uint64_t *d = sel + i * W;
            long double acc = (long double)diag_elem(&H, d) * psi[i];
            gen_one(&H, d, kb, hb);
            for (int64_t r = 0; r < nc; ++r) {
                int64_t j = find_key(sel, n_sel, W, kb + r * W);
                if (j >= 0) acc += (long double)hb[r] * psi[j];
            }
            out[t] = (double)acc;
        }
        free(kb);
        free(hb);
    }
    return bad ? -2 : 0;
}

/*
 * Dense <b_i|H|b_j> on a strictly ascending basis (column-major by source j:
 * out[j*n + i]).  Column j holds H_jj and every coupled determinant of b_j
 * that lies in the basis.  Returns 0, -1 (unsorted), -2 (invalid determinant).
 */
int ora_dense_h(int n_orb, int n_alpha, int n_beta, int W,
                const double *h, const double *eri,
                const uint64_t *basis, int64_t n, double *out)
{
    ora_ham H = {n_orb, n_alpha, n_beta, W, h, eri};
    for (int64_t i = 1; i < n; ++i)
        if (key_cmp(basis + (i - 1) * W, basis + i * W, W) >= 0) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (!det_valid(&H, basis + i * W)) return -2;
    int64_t nc = ora_n_coupled(n_orb, n_alpha, n_beta);
    memset(out, 0, (size_t)n * n * sizeof(double));
#pragma omp parallel
    {
        uint64_t *kb = (uint64_t *)malloc((size_t)(nc ? nc : 1) * W * 8);
        double *hb = (double *)malloc((size_t)(nc ? nc : 1) * 8);
#pragma omp for schedule(dynamic, 4)
        for (int64_t j = 0; j < n; ++j) {
            const uint64_t *d = basis + j * W;
            out[j * n + j] = diag_elem(&H, d);
            gen_one(&H, d, kb, hb);
            for (int64_t r = 0; r < nc; ++r) {
                int64_t i = find_key(basis, n, W, kb + r * W);
                if (i >= 0) out[j * n + i] = hb[r];
            }
        }
        free(kb);
        free(hb);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* reverse index and selection                                               */
/* ------------------------------------------------------------------------ */

/*
 * Reverse index (paper section 2.2, energy evaluation; section 4.3 stage 3:
 * each original configuration is searched in the unique set):
 * idx[i] = position of cand[i] in the strictly ascending set u, or -1 when
 * cand[i] is not in u.  Returns 0, or -1 if u is not strictly ascending.
 */
int ora_inverse_map(int W, const uint64_t *u, int64_t n_u, const uint64_t *cand, int64_t n, int64_t *idx)
{
    for (int64_t i = 1; i < n_u; ++i)
        if (key_cmp(u + (i - 1) * W, u + i * W, W) >= 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) idx[i] = find_key(u, n_u, W, cand + i * W);
    return 0;
}

/*
 * Selection of the K most important candidates (paper section 2.2,
 * wavefunction optimisation: top-K by inferred amplitude; section 4.3 stage 2):
 * rank entries by |psi| descending, equal magnitudes by key ascending, and mark
 * the first min(K, n) in mask.  With distinct keys the ranking is a total
 * order, so the selection is unique.  NaN amplitudes are outside the contract.
 * Returns the number marked, or -1 if two keys are equal.
 */
static int tk_W;
static const uint64_t *tk_keys;
static const double *tk_psi;
static int tk_cmp(const void *a, const void *b)
{
    const int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    const double x = fabs(tk_psi[i]), y = fabs(tk_psi[j]);
    if (x > y) return -1;
    if (x < y) return 1;
    return key_cmp(tk_keys + i * tk_W, tk_keys + j * tk_W, tk_W);
}

int64_t ora_topk(int W, const uint64_t *keys, const double *psi, int64_t n, int64_t K, uint8_t *mask)
{
    int64_t *order = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) order[i] = i;
    tk_W = W;
    tk_keys = keys;
    tk_psi = psi;
    qsort(order, (size_t)n, sizeof(int64_t), tk_cmp);
    int dup = 0;
    for (int64_t r = 1; r < n; ++r)
        if (key_cmp(keys + order[r - 1] * W, keys + order[r] * W, W) == 0) dup = 1;
    const int64_t k = K < n ? K : n;
    memset(mask, 0, (size_t)n);
    for (int64_t r = 0; r < k; ++r) mask[order[r]] = 1;
    free(order);
    return dup ? -1 : k;
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
