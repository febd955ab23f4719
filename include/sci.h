/*
 * sci.h — C ABI of the MI355X (gfx950) hot path of NNQS-SCI:
 * exact coupled-configuration generation, on-device de-duplication, and the
 * selected-space variational energy (arXiv 2604.15768).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Determinant ("key"): occupation bitstring over 2*n_orb spin orbitals packed
 *   into W = ceil(2*n_orb/64) little-endian uint64 words.  Spin orbital
 *   k = p + sigma*n_orb (sigma 0 = alpha, 1 = beta) is bit k&63 of word k>>6.
 *   Keys compare as unsigned W*64-bit integers, word W-1 most significant.
 *   An array of n keys is n*W contiguous uint64 ("[n][W]").
 * Phase convention: |D> = a+_{k1} a+_{k2} ... |0> with k1 < k2 < ...; the
 *   fermionic sign of an operator on spin orbital k is (-1)^(occupied spin
 *   orbitals below k).
 * Integrals: h1 is [n][n] (symmetric), eri is [n][n][n][n] in chemists'
 *   notation (pq|rs), real and 8-fold symmetric.  Everything floating point is
 *   IEEE double (FP64).
 * Memory: "device" pointers are HIP device memory owned by the caller (the
 *   library never frees or retains them past the enqueued work); "host"
 *   pointers are ordinary host memory read before the call returns.
 * Streams: every compute call enqueues on `stream` (a hipStream_t; NULL means
 *   the null stream) and returns without synchronising.  Results, device
 *   counters and device flags are valid once the stream has reached that point.
 * Errors: each call returns a status (sci_status).  Argument errors that the
 *   host can see are reported before anything is enqueued; the thread-local
 *   text of the last error is available from sci_last_error().  Conditions
 *   only the device can see set bits in *dev_flags (a caller-owned device
 *   uint32 that the library only ORs into; the caller clears it).  No C++
 *   exception leaves any entry point: a failed host allocation inside the
 *   library is returned as SCI_ENOMEM.
 */
#ifndef SCI_H
#define SCI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sci_ham_s *sci_ham_t; /* opaque Hamiltonian handle */
typedef void *sci_stream_t;          /* a hipStream_t */

typedef enum {
    SCI_OK = 0,
    SCI_EINVAL = 1,       /* bad argument (null pointer, size, shape)        */
    SCI_ECAPACITY = 2,    /* an output buffer is too small (host-visible)    */
    SCI_ENOMEM = 3,       /* the library could not allocate its own tables   */
    SCI_EHIP = 4,         /* a HIP runtime call failed                       */
    SCI_EUNSUPPORTED = 5  /* size outside what the library supports          */
} sci_status;

/* bits of *dev_flags */
#define SCI_FLAG_OVERFLOW 0x1u /* device-side count exceeded a capacity      */
#define SCI_FLAG_BAD_DET 0x2u  /* a determinant has wrong popcounts / bits   */
#define SCI_FLAG_UNSORTED 0x4u /* a set that must be strictly ascending isn't */

/* Largest sizes the library supports. */
#define SCI_MAX_WORDS 2
#define SCI_MAX_ORB 64

/* Human-readable name of a status code (static string). */
const char *sci_status_string(int32_t status);
/* Text of the last error raised on the calling thread ("" if none). */
const char *sci_last_error(void);

/* W = ceil(2*n_orb/64). */
int32_t sci_words(int32_t n_orb);

/*
 * Size of every coupled set C_i (paper Eq. 4: determinants reached by moving
 * one or two occupied positions, spin conserving, D_i itself excluded):
 *   n_a*v_a + n_b*v_b + C(n_a,2)C(v_a,2) + C(n_b,2)C(v_b,2) + n_a v_a n_b v_b,
 * v = n_orb - n.  Returns -1 for invalid sizes.
 */
int64_t sci_n_coupled(int32_t n_orb, int32_t n_alpha, int32_t n_beta);

/*
 * Upload a Hamiltonian and build the device tables the kernels read
 * (paper section 4.2, the single/double excitation tables; here the
 * integral slices V_pq[a][b] = (ap|bq) and their antisymmetrised same-spin
 * form).  h1_host, eri_host: host arrays as above.  On success *out owns one
 * device allocation of about (3*n_orb^4 + 2*n_orb^3 + 5*n_orb^2)*8 bytes
 * (the ERI, the two n^4 slice tables, the n^3 Coulomb/exchange row tables,
 * h1, J, K, the reference determinant's single-excitation elements per spin;
 * plus small pair lists) until sci_ham_destroy: 311 MB for n_orb=60.
 * The handle is immutable and may be used from several streams at once.
 * Synchronous and stream-free (unlike the compute calls): the integrals are
 * copied with blocking copies, the tables are built on the null stream, and
 * the call returns once that stream has finished, so the handle is ready for
 * any stream.  The host arrays may be freed on return.
 * Errors: SCI_EINVAL (null pointers, n_alpha/n_beta outside [0, n_orb]),
 * SCI_EUNSUPPORTED (n_orb > SCI_MAX_ORB), SCI_ENOMEM (device or host
 * allocation), SCI_EHIP.
 */
int32_t sci_ham_create(int32_t n_orb, int32_t n_alpha, int32_t n_beta,
                       const double *h1_host, const double *eri_host, sci_ham_t *out);

/* Free a handle (NULL is allowed).  The caller ensures no enqueued work still uses it. */
int32_t sci_ham_destroy(sci_ham_t ham);

/*
 * Coupled-configuration generation (paper section 4.2, Algorithm 1; Eq. 4).
 *
 * Flat excitation index f = i*N_c + r for source i in [0, n_dets) and rank
 * r in [0, N_c), N_c = sci_n_coupled(...).  Ranks follow a fixed order per
 * source: alpha singles (p asc, a asc), beta singles, alpha-alpha doubles
 * ((p<q) lexicographic, then (a<b) lexicographic), beta-beta doubles,
 * alpha-beta doubles ((p, q, a, b) lexicographic), with p,q occupied and a,b
 * empty in the source.  The call covers f in [exc_begin, exc_end).
 *
 * For each f: key = the determinant D' reached, hij = <D'|H|D_i> (FP64,
 * Slater-Condon rules with the exact fermionic sign).
 *
 * dets      device [n_dets][W], each with n_alpha alpha and n_beta beta bits
 *           and no bit at or above 2*n_orb (else SCI_FLAG_BAD_DET is set and
 *           that source's outputs are zero).
 * eps < 0   dense mode: entry f is written at index f - exc_begin of
 *           out_keys ([capacity][W]) / out_hij ([capacity]); out_src (nullable)
 *           receives i.  Requires capacity >= exc_end - exc_begin
 *           (SCI_ECAPACITY otherwise).  Output is deterministic.
 * eps >= 0  screened mode: only |hij| > eps is kept, compacted in an
 *           unspecified order; out_src is required.  *n_out (device int64,
 *           required here, nullable in dense mode) is set to the number kept;
 *           if it exceeds capacity, SCI_FLAG_OVERFLOW is set and only the first
 *           `capacity` slots are written.
 * Errors: SCI_EINVAL (null handle/pointers, W mismatch, bad range),
 *         SCI_ECAPACITY, SCI_EHIP.
 */
int32_t sci_gen_coupled(sci_ham_t ham, const uint64_t *dets, int64_t n_dets,
                        int64_t exc_begin, int64_t exc_end, double eps,
                        uint64_t *out_keys, double *out_hij, int32_t *out_src,
                        int64_t capacity, int64_t *n_out, uint32_t *dev_flags,
                        sci_stream_t stream);

/*
 * Batched generation (several systems, one persistent launch; paper section
 * 4.2: the grid-stride virtual-thread loop over all work, here over the
 * sources of every system of the batch).
 *
 * sci_gen_item describes one system's dense-mode call, exactly as
 * sci_gen_coupled with eps < 0: the excitation range [exc_begin, exc_end) of
 * dets (device [n_dets][W]) is written to out_keys (device
 * [exc_end - exc_begin][W]) and out_hij (device [exc_end - exc_begin]).
 * Items may mix key widths and may alias nothing they write.
 *
 * sci_gen_batch_create: validates every item (as sci_gen_coupled would) and
 * uploads the item table and a tile list (runs of consecutive sources of
 * about tile_candidates candidates, largest first) to device memory owned by
 * the handle; device-detected conditions set bits in dev_flags.  Synchronous.
 * sci_gen_coupled_batched: one launch over every tile of the batch on
 * `stream`: it allocates nothing and never synchronises, so it can be
 * captured in a graph.  One launch of a given batch at a time.
 * sci_gen_batch_autotune: times the batch with several tile sizes, keeps the
 * fastest and returns it in *tile_candidates (nullable).  Synchronous; it
 * writes the outputs (with their correct values).
 * Errors: SCI_EINVAL, SCI_EUNSUPPORTED, SCI_ENOMEM, SCI_EHIP.
 */
typedef struct sci_gen_item {
    sci_ham_t ham;
    const uint64_t *dets;
    int64_t n_dets;
    int64_t exc_begin, exc_end;
    uint64_t *out_keys;
    double *out_hij;
} sci_gen_item;
typedef struct sci_gen_batch_s *sci_gen_batch_t;

int32_t sci_gen_batch_create(const sci_gen_item *items, int32_t n_items, int64_t tile_candidates,
                             uint32_t *dev_flags, sci_gen_batch_t *out);
int32_t sci_gen_batch_destroy(sci_gen_batch_t batch);
int32_t sci_gen_coupled_batched(sci_gen_batch_t batch, sci_stream_t stream);
int32_t sci_gen_batch_autotune(sci_gen_batch_t batch, sci_stream_t stream, int64_t *tile_candidates);

/*
 * Workspace bytes sci_dedup_merge needs for n_cand candidates of W words.
 */
size_t sci_dedup_workspace_bytes(int32_t n_words, int64_t n_cand);

/*
 * Global de-duplication and merge into a running set (paper section 4.1:
 * sort, regular-sampling partition, local unique, merge).
 *
 * cand        device [n_cand][W], any order, duplicates allowed.
 * set_in      device [*n_set_in][W], strictly ascending (the running set,
 *             e.g. the selected space); n_set_in is a device int64.
 * set_out     device [set_capacity][W]: receives sorted(set(cand) | set_in);
 *             *n_set_out (device int64) its size.  Must not alias set_in or cand.
 * novel       nullable device [novel_capacity][W]: sorted(set(cand) - set_in),
 *             size in *n_novel (device int64; required when novel is given).
 * workspace   device, at least sci_dedup_workspace_bytes(W, n_cand) bytes.
 * If the union (or the novel set) does not fit, SCI_FLAG_OVERFLOW is set,
 * the required size is still written to *n_set_out / *n_novel, and the
 * contents of set_out / novel are unspecified; set_in is never modified.
 * Errors: SCI_EINVAL, SCI_ECAPACITY (workspace too small), SCI_EHIP.
 */
int32_t sci_dedup_merge(int32_t n_words, const uint64_t *cand, int64_t n_cand,
                        const uint64_t *set_in, const int64_t *n_set_in,
                        uint64_t *set_out, int64_t *n_set_out, int64_t set_capacity,
                        uint64_t *novel, int64_t *n_novel, int64_t novel_capacity,
                        void *workspace, size_t workspace_bytes,
                        uint32_t *dev_flags, sci_stream_t stream);

/*
 * Workspace bytes sci_energy needs for n_sel determinants.
 */
size_t sci_energy_workspace_bytes(int64_t n_sel);

/*
 * Variational energy over the selected space (paper Eq. 1, with the sums of
 * Eqs. 3 and 5 restricted to j in S), matrix-free:
 *   (H psi)_i = H_ii psi_i + sum_{j in S, j != i} H_ij psi_j,
 *   E = psi.(H psi) / psi.psi,   grad_i = dE/dpsi_i = 2((H psi)_i - E psi_i)/psi.psi.
 * H_ij is recomputed from the integrals, never stored.
 *
 * sel      device [n_sel][W], strictly ascending (else SCI_FLAG_UNSORTED),
 *          each with the handle's popcounts (else SCI_FLAG_BAD_DET).
 * psi      device [n_sel] FP64 real amplitudes (not necessarily normalised).
 * energy   device double [1] (required).
 * h_psi    nullable device [n_sel]; grad nullable device [n_sel].
 * workspace device, at least sci_energy_workspace_bytes(n_sel) bytes.
 * The reduction order is fixed, so repeated calls give identical bits.
 * Errors: SCI_EINVAL, SCI_ECAPACITY (workspace), SCI_EHIP.
 */
int32_t sci_energy(sci_ham_t ham, const uint64_t *sel, int64_t n_sel, const double *psi,
                   double *energy, double *h_psi, double *grad,
                   void *workspace, size_t workspace_bytes,
                   uint32_t *dev_flags, sci_stream_t stream);

/*
 * How membership j in C_i is decided (both give H psi within rounding; each
 * method's results repeat bit for bit):
 *   SCI_ENERGY_PAIRS  pair screening: every (i, j) of S x S tested by one XOR +
 *                     popcount (D_i and D_j differ in at most two electrons).
 *   SCI_ENERGY_ENUM   enumeration + search (paper section 4.3: configurations
 *                     searched in a sorted set): C_i generated for every i (the
 *                     excitation order of sci_gen_coupled), each determinant
 *                     searched in the sorted S.  |S| N_c searches against |S|^2
 *                     tests: the faster one when N_c is small against |S|.
 *   SCI_ENERGY_AUTO   the method a cost model picks for this shape:
 *                     enumeration when N_c * 8 < n_sel, else pair screening
 *                     (sci_energy always uses it; sci_energy_method reports it).
 * sci_energy_ex is sci_energy with the method given; sci_energy_method returns
 * the method SCI_ENERGY_AUTO picks for n_sel determinants of this handle (-1 for
 * invalid arguments).
 */
#define SCI_ENERGY_AUTO 0
#define SCI_ENERGY_PAIRS 1
#define SCI_ENERGY_ENUM 2
int32_t sci_energy_ex(sci_ham_t ham, const uint64_t *sel, int64_t n_sel, const double *psi,
                      double *energy, double *h_psi, double *grad, int32_t method,
                      void *workspace, size_t workspace_bytes,
                      uint32_t *dev_flags, sci_stream_t stream);
int32_t sci_energy_method(sci_ham_t ham, int64_t n_sel);

/*
 * Batched energy (several systems; the per-block work of sci_energy over tile
 * lists covering every system, a handful of launches in all).  Each item is
 * one sci_energy call (sel strictly ascending, psi, energy required; h_psi and
 * grad nullable), and each system's results are bit-identical to that call.
 * sci_energy_batch_create validates the items, uploads the tile lists and
 * allocates each system's workspace (owned by the handle); synchronous.
 * sci_energy_batched enqueues the work on `stream`; it allocates nothing and
 * never synchronises.  One launch of a given batch at a time.
 * Errors: SCI_EINVAL, SCI_EUNSUPPORTED, SCI_ENOMEM, SCI_EHIP.
 */
typedef struct sci_energy_item {
    sci_ham_t ham;
    const uint64_t *sel;
    int64_t n_sel;
    const double *psi;
    double *energy;
    double *h_psi;
    double *grad;
} sci_energy_item;
typedef struct sci_energy_batch_s *sci_energy_batch_t;

int32_t sci_energy_batch_create(const sci_energy_item *items, int32_t n_items, uint32_t *dev_flags,
                                sci_energy_batch_t *out);
int32_t sci_energy_batch_destroy(sci_energy_batch_t batch);
int32_t sci_energy_batched(sci_energy_batch_t batch, sci_stream_t stream);

/*
 * sci_energy for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments and results as sci_energy (method SCI_ENERGY_AUTO, bit-identical
 * output) without the workspace: the library keeps its own scratch, one
 * file-scope device array per GPU of sci_energy_workspace_bytes(
 * sci_energy_noalloc_max_sel()) bytes (about 19 MB), held until the process
 * ends.  Calls no hipMalloc/hipFree; the first call on a device looks up that
 * device's scratch address (hipGetSymbolAddress) and keeps it.
 *
 * n_sel at most sci_energy_noalloc_max_sel() (2^18 = 262,144), else
 * SCI_ECAPACITY before anything is enqueued.  Every call on one GPU shares that
 * GPU's scratch, so calls whose work overlaps on one GPU (different streams,
 * or host threads without ordering) race and give undefined results; calls
 * ordered on one stream are safe.  Errors: as sci_energy, plus SCI_ECAPACITY.
 */
int64_t sci_energy_noalloc_max_sel(void);
int32_t sci_energy_noalloc(sci_ham_t ham, const uint64_t *sel, int64_t n_sel, const double *psi,
                           double *energy, double *h_psi, double *grad,
                           uint32_t *dev_flags, sci_stream_t stream);

/*
 * Streaming generation + de-duplication through a device pool (paper
 * section 4.3: mini-batches of bounded size, reduced as they are produced;
 * section 4.1: every batch is merged into the running unique set).
 *
 * The flat excitation range [exc_begin, exc_end) of `dets` (as in
 * sci_gen_coupled) is cut into chunks of at most `chunk` candidates.  Chunk k
 * is generated (dense mode) into pool buffer k%2 on `gen_stream`; the keys are
 * de-duplicated and merged into the running set on `dedup_stream`, while chunk
 * k+1 is generated into the other buffer (its generation starts once the dedup
 * of chunk k has chosen its first-level splitters and the dedup of chunk k-1
 * has released the buffer).  `chunk` is below 2^32 (one sci_dedup_merge call
 * per chunk; SCI_EUNSUPPORTED otherwise).  The running set starts as set_in
 * (strictly ascending, device count n_set_in) and alternates between set_a and
 * set_b (each set_capacity keys); *final_is_b (host) tells which one holds the
 * result, *n_set_out (device int64) its size.  H_ij values are produced into
 * the pool and not kept.  Both streams may be the same stream.
 *
 * workspace   device, at least sci_stream_workspace_bytes(ham, chunk) bytes
 *             (two pool chunks of keys + H_ij, and the dedup workspace).
 * On overflow of set_capacity, SCI_FLAG_OVERFLOW is set and the running set
 * keeps only the first set_capacity keys of the sorted union; later chunks
 * merge into that truncated set (never reading past set_capacity keys), so the
 * final set is incomplete and *n_set_out is then a lower bound on the size the
 * complete union needs.  The call only enqueues work; the result is ready when
 * dedup_stream reaches the end of it.
 * Errors: SCI_EINVAL, SCI_ECAPACITY (workspace), SCI_EHIP.
 */
size_t sci_stream_workspace_bytes(sci_ham_t ham, int64_t chunk);
int32_t sci_stream_dedup(sci_ham_t ham, const uint64_t *dets, int64_t n_dets,
                         int64_t exc_begin, int64_t exc_end, int64_t chunk,
                         const uint64_t *set_in, const int64_t *n_set_in,
                         uint64_t *set_a, uint64_t *set_b, int64_t set_capacity,
                         int64_t *n_set_out, int32_t *final_is_b,
                         void *workspace, size_t workspace_bytes, uint32_t *dev_flags,
                         sci_stream_t gen_stream, sci_stream_t dedup_stream);

/*
 * Reverse index (paper section 2.2: every coupled configuration mapped to its
 * entry in the unique set; section 4.3 stage 3: each original configuration
 * searched in the unique set).  Two kinds of index return the same answer:
 *
 *   hash    an open-addressing table of 2^ceil(log2(2*set_bound)) slots of 16
 *           bytes (W=1) or 32 bytes (W=2), at least 64 slots, after a 256-byte
 *           header: sci_index_bytes(n_words, set_bound) bytes.  One lookup reads
 *           about one slot.  Independent of the set once built.
 *   sorted  the paper's search of the sorted set: a 256-byte header and every
 *           256th set key (1/256 of the set's bytes):
 *           sci_index_bytes_sorted(n_words, set_bound) bytes.  A lookup searches
 *           a top level of those samples in LDS, then the samples, then one
 *           256-key block of the set itself, so the set must stay in place and
 *           unchanged while the index is used.  For sets whose table would not
 *           fit beside them (3.06e9 two-word keys: a 275 GB table, a 191 MB
 *           sorted index).
 *
 * sci_index_build: index the strictly ascending set (device [*n_set][W], count
 * on the device) into `index` (device, caller-owned).  The kind follows from the
 * buffer: index_bytes >= sci_index_bytes(n_words, set_bound) builds the hash
 * kind, else index_bytes >= sci_index_bytes_sorted(...) the sorted kind, else
 * SCI_ECAPACITY.  If *n_set > set_bound, SCI_FLAG_OVERFLOW is set and only the
 * first set_bound keys are indexed.  The set must stay unchanged while the index
 * is used.
 *
 * sci_index_lookup: idx[i] (device int64) = position of cand[i] in the set,
 * or -1 when the key is not in it, for i < n_cand; cand is device
 * [n_cand][W], any order.  Deterministic (positions, not probe order).  The
 * kind is read from the index's device header (the kernels of both kinds are
 * enqueued; the one that does not match returns at once).  An index buffer that
 * sci_index_build did not fill for this n_words and a size that fits in
 * index_bytes gives -1 for every candidate.
 * Errors: SCI_EINVAL, SCI_EUNSUPPORTED (n_words), SCI_ECAPACITY (index too
 * small), SCI_EHIP.
 */
size_t sci_index_bytes(int32_t n_words, int64_t set_bound);
size_t sci_index_bytes_sorted(int32_t n_words, int64_t set_bound);
int32_t sci_index_build(int32_t n_words, const uint64_t *set, const int64_t *n_set, int64_t set_bound,
                        void *index, size_t index_bytes, uint32_t *dev_flags, sci_stream_t stream);
int32_t sci_index_lookup(int32_t n_words, const void *index, size_t index_bytes,
                         const uint64_t *cand, int64_t n_cand, int64_t *idx, sci_stream_t stream);

/*
 * Top-K selection (paper section 2.2: the candidates with the largest
 * inferred amplitudes are added to S; section 4.3 stage 2).
 *
 * Ranks the n entries (keys device [n][W], distinct; psi device [n] FP64) by
 * |psi| descending, equal magnitudes by key ascending, and writes the first
 * min(k, n) of that ranking, in input order, to out_keys ([capacity][W]) and
 * out_psi (nullable, [capacity]); *n_out (device int64) gets their number.
 * The selection is unique and bit-exact for distinct keys; with repeated keys
 * more entries may tie (SCI_FLAG_OVERFLOW if they exceed capacity).  NaN
 * amplitudes are outside the contract.  Merging the result into S is a call
 * of sci_dedup_merge.
 * workspace: device, at least sci_topk_workspace_bytes(n) bytes.
 * Errors: SCI_EINVAL, SCI_EUNSUPPORTED (n_words), SCI_ECAPACITY (capacity <
 * min(k, n), or workspace), SCI_EHIP.
 */
size_t sci_topk_workspace_bytes(int64_t n);
int32_t sci_topk(int32_t n_words, const uint64_t *keys, const double *psi, int64_t n, int64_t k,
                 uint64_t *out_keys, double *out_psi, int64_t *n_out, int64_t capacity,
                 void *workspace, size_t workspace_bytes, uint32_t *dev_flags, sci_stream_t stream);

/*
 * Per-kernel timing, for profiling and roofline reports (not part of the
 * method).  While enabled (process-wide), every kernel the library launches
 * is bracketed by two HIP events recorded on that kernel's stream.
 * sci_profile_read waits for the recorded events, copies up to `cap`
 * (static kernel name, milliseconds) pairs in launch order into names/ms,
 * clears the record and returns the number of records that were held (which
 * may exceed cap).  Returns -1 on a HIP error.  Synchronous.
 */
int32_t sci_profile_enable(int32_t on);
int32_t sci_profile_read(const char **names, float *ms, int32_t cap);

#ifdef __cplusplus
}
#endif

#endif /* SCI_H */
