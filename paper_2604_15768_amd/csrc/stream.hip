// Pool streaming: chunked generation feeding de-duplication (paper section
// 4.3, mini-batch execution; section 4.1, merge into the unique set).
//
// Two pool buffers hold consecutive chunks of candidates.  Generation of chunk
// k+1 (gen stream) overlaps the de-duplication and merge of chunk k (dedup
// stream); events order each buffer's reuse.  The dedup of a chunk writes its
// second partition level back into the chunk's own pool buffer (consumed by the
// first level), so the dedup workspace holds one key buffer.  Set sizes never
// leave the device, so the loop needs no host synchronisation.
#include <vector>

#include "sci_internal.hpp"

namespace sci {

struct StreamLayout {
    size_t keys[2], hij[2], dedup, n_gen, n_run, total;
};

static size_t al256s(size_t b) { return (b + 255) / 256 * 256; }

static StreamLayout stream_layout(int W, int64_t chunk) {
    StreamLayout L{};
    size_t off = 0;
    for (int b = 0; b < 2; ++b) {
        L.keys[b] = off;
        off += al256s((size_t)chunk * W * 8);
        L.hij[b] = off;
        off += al256s((size_t)chunk * 8);
    }
    L.n_gen = off;
    off += 256;
    L.n_run = off;
    off += 256;
    L.dedup = off;
    off += dedup_ws_bytes(W, chunk, true);
    L.total = off;
    return L;
}

// events of one call, released on every return path (destroying an event with
// work still pending on it is allowed; the release happens when it completes)
struct StreamEvents {
    hipEvent_t ready[2] = {nullptr, nullptr}, filled[2] = {nullptr, nullptr}, split = nullptr;
    ~StreamEvents() {
        for (int b = 0; b < 2; ++b) {
            if (ready[b]) (void)hipEventDestroy(ready[b]);
            if (filled[b]) (void)hipEventDestroy(filled[b]);
        }
        if (split) (void)hipEventDestroy(split);
    }
};

// After a merge that overflowed, *n_set_out holds the size the union needs, but
// the set buffer holds only the first `cap` keys: the next chunk reads that many.
__global__ void clamp_count_kernel(const int64_t *n, int64_t cap, int64_t *kept) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t v = *n;
        *kept = v < cap ? v : cap;
    }
}

}  // namespace sci

using namespace sci;

extern "C" size_t sci_stream_workspace_bytes(sci_ham_t ham, int64_t chunk) {
    if (!ham || chunk < 1) return 0;
    return stream_layout(ham->dev.W, chunk).total;
}

extern "C" int32_t sci_stream_dedup(sci_ham_t ham, const uint64_t *dets, int64_t n_dets, int64_t exc_begin,
                                    int64_t exc_end, int64_t chunk, const uint64_t *set_in, const int64_t *n_set_in,
                                    uint64_t *set_a, uint64_t *set_b, int64_t set_capacity, int64_t *n_set_out,
                                    int32_t *final_is_b, void *workspace, size_t workspace_bytes,
                                    uint32_t *dev_flags, sci_stream_t gen_stream, sci_stream_t dedup_stream) {
    set_error("");
    if (!ham) return fail(SCI_EINVAL, "sci_stream_dedup: NULL handle");
    const int W = ham->dev.W;
    if (chunk < 1) return fail(SCI_EINVAL, "sci_stream_dedup: chunk must be >= 1");
    if (chunk >= (1ll << 32))
        return fail(SCI_EUNSUPPORTED, "sci_stream_dedup: chunk %lld exceeds one dedup call (2^32 - 1)",
                    (long long)chunk);
    if (!set_a || !set_b || set_a == set_b || !n_set_out || !final_is_b || !workspace || !dev_flags)
        return fail(SCI_EINVAL, "sci_stream_dedup: NULL or aliased argument");
    if (set_in && !n_set_in) return fail(SCI_EINVAL, "sci_stream_dedup: set_in without n_set_in");
    if (set_in == set_a || set_in == set_b) return fail(SCI_EINVAL, "sci_stream_dedup: set_in aliases an output set");
    if (n_dets < 0 || exc_begin < 0 || exc_end < exc_begin || exc_end > n_dets * ham->dev.n_coupled)
        return fail(SCI_EINVAL, "sci_stream_dedup: bad excitation range");
    const StreamLayout L = stream_layout(W, chunk);
    if (workspace_bytes < L.total)
        return fail(SCI_ECAPACITY, "sci_stream_dedup: workspace %zu < %zu bytes", workspace_bytes, L.total);
    hipStream_t sg = (hipStream_t)gen_stream, sd = (hipStream_t)dedup_stream;
    char *ws = (char *)workspace;
    const int64_t n_chunks = exc_end > exc_begin ? ceil_div(exc_end - exc_begin, chunk) : 0;

    // ready[b]: buffer b consumed by the dedup stream; filled[b]: buffer b generated
    StreamEvents ev;
    hipEvent_t *ready = ev.ready, *filled = ev.filled;
    for (int b = 0; b < 2; ++b) {
        SCI_HIP_TRY(hipEventCreateWithFlags(&ready[b], hipEventDisableTiming));
        SCI_HIP_TRY(hipEventCreateWithFlags(&filled[b], hipEventDisableTiming));
    }
    SCI_HIP_TRY(hipEventCreateWithFlags(&ev.split, hipEventDisableTiming));

    const uint64_t *cur_set = set_in;
    const int64_t *cur_n = set_in ? n_set_in : nullptr;
    int out_b = 0;  // next output set: 0 -> set_a, 1 -> set_b
    int32_t st = SCI_OK;
    if (n_chunks == 0) {
        // nothing to generate: the result is the input set
        st = sci_dedup_merge(W, nullptr, 0, cur_set, cur_n, set_a, n_set_out, set_capacity, nullptr, nullptr, 0,
                             ws + L.dedup, workspace_bytes - L.dedup, dev_flags, dedup_stream);
        *final_is_b = 0;
        return st;
    }
    // the dedup stream must not start before work already queued on the gen stream (inputs)
    SCI_HIP_TRY(hipEventRecord(filled[1], sg));
    SCI_HIP_TRY(hipStreamWaitEvent(sd, filled[1], 0));
    for (int64_t k = 0; k < n_chunks; ++k) {
        const int b = (int)(k & 1);
        const int64_t e0 = exc_begin + k * chunk;
        const int64_t e1 = e0 + chunk < exc_end ? e0 + chunk : exc_end;
        if (k >= 2) SCI_HIP_TRY(hipStreamWaitEvent(sg, ready[b], 0));  // buffer b free again
        // the next chunk is generated once the previous chunk's dedup has chosen its first
        // splitters: its small, latency-bound sample sort then does not queue behind
        // a full-chip generation launch, which overlaps the partition passes instead
        if (k >= 1) SCI_HIP_TRY(hipStreamWaitEvent(sg, ev.split, 0));
        st = sci_gen_coupled(ham, dets, n_dets, e0, e1, -1.0, (uint64_t *)(ws + L.keys[b]), (double *)(ws + L.hij[b]),
                             nullptr, chunk, (int64_t *)(ws + L.n_gen), dev_flags, gen_stream);
        if (st != SCI_OK) break;
        SCI_HIP_TRY(hipEventRecord(filled[b], sg));
        SCI_HIP_TRY(hipStreamWaitEvent(sd, filled[b], 0));
        uint64_t *dst = out_b ? set_b : set_a;
        // the set written by the previous chunk is read now, with its kept count; only the
        // caller's set_in needs the order check
        st = dedup_merge_checked(W, (const uint64_t *)(ws + L.keys[b]), e1 - e0, cur_set, cur_n, dst, n_set_out,
                                 set_capacity, nullptr, nullptr, 0, ws + L.dedup, workspace_bytes - L.dedup,
                                 dev_flags, sd, /*check_set_in=*/k == 0, /*cand_scratch=*/true, ev.split);
        if (st != SCI_OK) break;
        SCI_HIP_TRY(hipEventRecord(ready[b], sd));
        int64_t *n_run = (int64_t *)(ws + L.n_run);
        SCI_LAUNCH(clamp_count_kernel, dim3(1), dim3(64), 0, sd, (const int64_t *)n_set_out, set_capacity, n_run);
        SCI_HIP_TRY(hipGetLastError());
        cur_set = dst;
        cur_n = n_run;
        out_b ^= 1;
    }
    *final_is_b = out_b ^ 1;
    return st;
}
