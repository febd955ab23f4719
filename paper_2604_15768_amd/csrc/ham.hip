// Hamiltonian handle: upload of h1 and (pq|rs), and the device tables the
// generation and energy kernels read (paper section 4.2: integrals are
// pre-arranged per source/target orbitals so a kernel reads one entry per
// excitation).  Also the ABI's error plumbing and size helpers.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <mutex>
#include <cstring>
#include <new>
#include <vector>

#include "sci_internal.hpp"

namespace sci {

static thread_local char g_last_error[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
}

int32_t fail(int32_t status, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return status;
}

// vdir[p][q][a][b] = (ap|bq); vanti[p][q][a][b] = (ap|bq) - (aq|bp);
// jtpq[t][p][q] = (tp|qq), ktpq[t][p][q] = (tq|qp).
// One thread per output element; grid covers n^4 exactly (bounds-checked).
__global__ void build_tables_kernel(const double *__restrict__ eri, double *__restrict__ vdir,
                                    double *__restrict__ vanti, double *__restrict__ jmat,
                                    double *__restrict__ kmat, double *__restrict__ jtpq,
                                    double *__restrict__ ktpq, int n) {
    const int64_t n2 = (int64_t)n * n;
    const int64_t total = n2 * n2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < total) {
        const int b = (int)(t % n);
        const int a = (int)((t / n) % n);
        const int q = (int)((t / n2) % n);
        const int p = (int)(t / (n2 * n));
        const double d = eri[((int64_t)(a * n + p) * n + b) * n + q];  // (ap|bq)
        const double x = eri[((int64_t)(a * n + q) * n + b) * n + p];  // (aq|bp)
        vdir[t] = d;
        vanti[t] = d - x;
    }
    if (t < n2 * n) {
        const int q = (int)(t % n);
        const int p = (int)((t / n) % n);
        const int tt = (int)(t / n2);
        jtpq[t] = eri[((int64_t)(tt * n + p) * n + q) * n + q];  // (tp|qq)
        ktpq[t] = eri[((int64_t)(tt * n + q) * n + q) * n + p];  // (tq|qp)
    }
    if (t < n2) {
        const int p = (int)(t / n), q = (int)(t % n);
        jmat[t] = eri[((int64_t)(p * n + p) * n + q) * n + q];  // (pp|qq)
        kmat[t] = eri[((int64_t)(p * n + q) * n + q) * n + p];  // (pq|qp)
    }
}

// fref[s][t][p] = h_tp + sum over the reference's occupied spin orbitals Q of
// (tp|qq) - [Q has spin s] (tq|qp), in the order alpha block then beta block.  The
// reference holds alpha orbitals 0..n_alpha-1 and beta orbitals 0..n_beta-1.  For
// any determinant D the single t <- p element is fref plus the same terms over the
// spin orbitals D has and the reference lacks, minus those over the ones it lacks.
__global__ void build_fref_kernel(const double *__restrict__ h1, const double *__restrict__ jtpq,
                                  const double *__restrict__ ktpq, double *__restrict__ fref, int n, int na,
                                  int nb) {
    const int64_t n2 = (int64_t)n * n;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * n2) return;
    const int s = (int)(t / n2);
    const int64_t tp = t - s * n2;  // (orbital t) * n + p
    const double *jr = jtpq + tp * n, *kr = ktpq + tp * n;
    double v = h1[tp];
    for (int q = 0; q < na; ++q) v += jr[q] - (s == 0 ? kr[q] : 0.0);
    for (int q = 0; q < nb; ++q) v += jr[q] - (s == 1 ? kr[q] : 0.0);
    fref[t] = v;
}

// ---------------------------------------------------------------------------
// per-launch timing
// ---------------------------------------------------------------------------
namespace {
struct ProfRec {
    const char *name;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
std::atomic<int> g_prof_on{0};
std::vector<ProfRec> g_prof;      // records of the current window
std::vector<hipEvent_t> g_events; // pool of created events
size_t g_next_event = 0;

// An event from the pool (nullptr when none can be had: that launch goes untimed).
hipEvent_t take_event() noexcept {
    if (g_next_event == g_events.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        try {
            g_events.push_back(e);
        } catch (...) {
            (void)hipEventDestroy(e);
            return nullptr;
        }
    }
    return g_events[g_next_event++];
}
}  // namespace

// Timing is best effort: when the record cannot grow, the launch goes untimed and
// nothing is thrown (this runs inside every entry point that launches a kernel).
ProfScope::ProfScope(const char *name, hipStream_t s) : st(s), slot(-1) {
    if (!g_prof_on.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    ProfRec r{name, take_event(), take_event()};
    if (!r.a || !r.b) return;
    try {
        g_prof.reserve(g_prof.size() + 1);
    } catch (...) {
        return;
    }
    if (hipEventRecord(r.a, st) != hipSuccess) return;
    slot = (int)g_prof.size();
    g_prof.push_back(r);  // capacity reserved above: cannot throw
}

ProfScope::~ProfScope() {
    if (slot < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    (void)hipEventRecord(g_prof[slot].b, st);
}

__global__ void set_i64_kernel(int64_t *p, int64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void set_u32_kernel(uint32_t *p, uint32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

hipError_t launch_set_i64(int64_t *p, int64_t v, hipStream_t st) {
    SCI_LAUNCH(set_i64_kernel, dim3(1), dim3(64), 0, st, p, v);
    return hipGetLastError();
}

hipError_t launch_set_u32(uint32_t *p, uint32_t v, hipStream_t st) {
    SCI_LAUNCH(set_u32_kernel, dim3(1), dim3(64), 0, st, p, v);
    return hipGetLastError();
}

}  // namespace sci

using namespace sci;

extern "C" {

const char *sci_status_string(int32_t status) {
    switch (status) {
        case SCI_OK: return "SCI_OK";
        case SCI_EINVAL: return "SCI_EINVAL";
        case SCI_ECAPACITY: return "SCI_ECAPACITY";
        case SCI_ENOMEM: return "SCI_ENOMEM";
        case SCI_EHIP: return "SCI_EHIP";
        case SCI_EUNSUPPORTED: return "SCI_EUNSUPPORTED";
        default: return "SCI_UNKNOWN";
    }
}

const char *sci_last_error(void) { return g_last_error; }

int32_t sci_words(int32_t n_orb) {
    if (n_orb < 0) return -1;
    return (2 * n_orb + 63) / 64;
}

int64_t sci_n_coupled(int32_t n_orb, int32_t n_alpha, int32_t n_beta) {
    if (n_orb < 0 || n_alpha < 0 || n_beta < 0 || n_alpha > n_orb || n_beta > n_orb) return -1;
    const int64_t va = n_orb - n_alpha, vb = n_orb - n_beta;
    return (int64_t)n_alpha * va + (int64_t)n_beta * vb + comb2(n_alpha) * comb2(va) +
           comb2(n_beta) * comb2(vb) + (int64_t)n_alpha * va * n_beta * vb;
}

static int32_t ham_create_impl(int32_t n_orb, int32_t n_alpha, int32_t n_beta, const double *h1_host,
                               const double *eri_host, sci_ham_t *out);

int32_t sci_ham_create(int32_t n_orb, int32_t n_alpha, int32_t n_beta, const double *h1_host,
                       const double *eri_host, sci_ham_t *out) {
    set_error("");
    return guarded("sci_ham_create", [&] { return ham_create_impl(n_orb, n_alpha, n_beta, h1_host, eri_host, out); });
}

static int32_t ham_create_impl(int32_t n_orb, int32_t n_alpha, int32_t n_beta, const double *h1_host,
                               const double *eri_host, sci_ham_t *out) {
    if (!out) return fail(SCI_EINVAL, "sci_ham_create: out is NULL");
    *out = nullptr;
    if (!h1_host || !eri_host) return fail(SCI_EINVAL, "sci_ham_create: NULL integrals");
    if (n_orb < 1 || n_alpha < 0 || n_beta < 0 || n_alpha > n_orb || n_beta > n_orb)
        return fail(SCI_EINVAL, "sci_ham_create: bad sizes n_orb=%d n_alpha=%d n_beta=%d", n_orb,
                    n_alpha, n_beta);
    if (n_orb > SCI_MAX_ORB)
        return fail(SCI_EUNSUPPORTED, "sci_ham_create: n_orb=%d exceeds %d", n_orb, SCI_MAX_ORB);

    const int64_t n = n_orb, n2 = n * n, n4 = n2 * n2;
    // layout of the single device block (each table 256-byte aligned)
    auto align = [](int64_t b) { return (b + 255) / 256 * 256; };
    const int64_t off_h1 = 0;
    const int64_t off_eri = off_h1 + align(n2 * 8);
    const int64_t off_vdir = off_eri + align(n4 * 8);
    const int64_t off_vanti = off_vdir + align(n4 * 8);
    const int64_t off_j = off_vanti + align(n4 * 8);
    const int64_t off_k = off_j + align(n2 * 8);
    const int64_t off_jt = off_k + align(n2 * 8);
    const int64_t off_kt = off_jt + align(n2 * n * 8);
    const int64_t off_fref = off_kt + align(n2 * n * 8);
    const int pair_m[4] = {n_alpha, n_beta, n_orb - n_alpha, n_orb - n_beta};
    int64_t off_pairs[4];
    int64_t cursor = off_fref + align(2 * n2 * 8);
    for (int t = 0; t < 4; ++t) {
        off_pairs[t] = cursor;
        cursor += align(std::max<int64_t>(1, comb2(pair_m[t])) * 2);
    }
    const int64_t total = cursor;

    // pair tables on the host first: if their allocation throws, nothing is held yet
    std::vector<uint16_t> tabs[4];
    for (int t = 0; t < 4; ++t) {
        const int m = pair_m[t];
        tabs[t].reserve((size_t)std::max<int64_t>(0, comb2(m)));
        for (int i = 0; i < m; ++i)
            for (int j = i + 1; j < m; ++j) tabs[t].push_back((uint16_t)(i | (j << 8)));
    }
    sci_ham_s *h = new (std::nothrow) sci_ham_s;
    if (!h) return fail(SCI_ENOMEM, "sci_ham_create: host allocation failed");

    void *block = nullptr;
    if (hipMalloc(&block, (size_t)total) != hipSuccess) {
        delete h;
        return fail(SCI_ENOMEM, "sci_ham_create: hipMalloc(%lld) failed", (long long)total);
    }
    char *base = (char *)block;
    auto cleanup = [&](int32_t st) {
        (void)hipFree(block);
        delete h;
        return st;
    };
    if (hipMemcpy(base + off_h1, h1_host, (size_t)(n2 * 8), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(base + off_eri, eri_host, (size_t)(n4 * 8), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(SCI_EHIP, "sci_ham_create: upload failed"));
    for (int t = 0; t < 4; ++t) {
        const std::vector<uint16_t> &tab = tabs[t];
        if (!tab.empty() &&
            hipMemcpy(base + off_pairs[t], tab.data(), tab.size() * 2, hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(SCI_EHIP, "sci_ham_create: pair table upload failed"));
    }

    const int threads = 256;
    const int64_t blocks = ceil_div(n4, threads);
    SCI_LAUNCH(build_tables_kernel, dim3((unsigned)blocks), dim3(threads), 0, 0,
                       (const double *)(base + off_eri), (double *)(base + off_vdir),
                       (double *)(base + off_vanti), (double *)(base + off_j),
                       (double *)(base + off_k), (double *)(base + off_jt), (double *)(base + off_kt), (int)n);
    SCI_LAUNCH(build_fref_kernel, dim3((unsigned)ceil_div(2 * n2, threads)), dim3(threads), 0, 0,
               (const double *)(base + off_h1), (const double *)(base + off_jt), (const double *)(base + off_kt),
               (double *)(base + off_fref), (int)n, n_alpha, n_beta);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(nullptr) != hipSuccess)
        return cleanup(fail(SCI_EHIP, "sci_ham_create: table build failed"));

    HamDev &d = h->dev;
    d.n_orb = n_orb;
    d.n_alpha = n_alpha;
    d.n_beta = n_beta;
    d.W = (2 * n_orb + 63) / 64;
    d.v_alpha = n_orb - n_alpha;
    d.v_beta = n_orb - n_beta;
    d.c1 = (int64_t)n_alpha * d.v_alpha;
    d.c2 = d.c1 + (int64_t)n_beta * d.v_beta;
    d.c3 = d.c2 + comb2(n_alpha) * comb2(d.v_alpha);
    d.c4 = d.c3 + comb2(n_beta) * comb2(d.v_beta);
    d.n_coupled = d.c4 + (int64_t)n_alpha * d.v_alpha * n_beta * d.v_beta;
    d.h1 = (const double *)(base + off_h1);
    d.eri = (const double *)(base + off_eri);
    d.vdir = (const double *)(base + off_vdir);
    d.vanti = (const double *)(base + off_vanti);
    d.jmat = (const double *)(base + off_j);
    d.kmat = (const double *)(base + off_k);
    d.jtpq = (const double *)(base + off_jt);
    d.ktpq = (const double *)(base + off_kt);
    d.fref = (const double *)(base + off_fref);
    for (int t = 0; t < 4; ++t) d.pairs[t] = (const uint16_t *)(base + off_pairs[t]);
    h->block = block;
    *out = h;
    return SCI_OK;
}

int32_t sci_profile_enable(int32_t on) {
    g_prof_on.store(on ? 1 : 0);
    return SCI_OK;
}

int32_t sci_profile_read(const char **names, float *ms, int32_t cap) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    const int32_t n = (int32_t)g_prof.size();
    int32_t rc = n;
    for (int32_t i = 0; i < n; ++i) {
        float t = 0.0f;
        if (hipEventSynchronize(g_prof[i].b) != hipSuccess ||
            hipEventElapsedTime(&t, g_prof[i].a, g_prof[i].b) != hipSuccess)
            rc = -1;
        if (i < cap) {
            if (names) names[i] = g_prof[i].name;
            if (ms) ms[i] = t;
        }
    }
    g_prof.clear();
    g_next_event = 0;
    return rc;
}

int32_t sci_ham_destroy(sci_ham_t ham) {
    if (!ham) return SCI_OK;
    (void)hipFree(ham->block);
    delete ham;
    return SCI_OK;
}

}  // extern "C"
