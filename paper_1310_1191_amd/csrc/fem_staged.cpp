// fem_staged.cpp -- meshes held in host memory: integration in element chunks whose host-to-
// device copies, kernels and device-to-host copies overlap on several streams. This is the
// end-to-end view of the paper's experiments (section 5.4, Tables 6 and 7: input transfer, kernel
// and output transfer timed separately), with the transfers hidden behind the kernels where the copy engines allow.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <mutex>
#include <vector>

#include "fem.h"

namespace fem {

namespace {

struct Slot {
    void *geom = nullptr, *elem = nullptr, *A = nullptr, *b = nullptr;
    hipStream_t stream = nullptr;
};

// Device staging reused across calls (grown on demand, released by fem_finalize).
struct Pool {
    std::vector<Slot> slots;
    size_t geom_bytes = 0, elem_bytes = 0, A_bytes = 0, b_bytes = 0;
    double *field = nullptr;   // 175 doubles
    int32_t *status = nullptr; // 2 counters
};
Pool g_pool;
std::mutex g_pool_mutex;

void release_locked()
{
    for (Slot &s : g_pool.slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        (void)hipFree(s.geom);
        (void)hipFree(s.elem);
        (void)hipFree(s.A);
        (void)hipFree(s.b);
        if (s.stream) (void)hipStreamDestroy(s.stream);
    }
    g_pool.slots.clear();
    (void)hipFree(g_pool.field);
    (void)hipFree(g_pool.status);
    g_pool = Pool();
}

int ensure_locked(int nslots, size_t gb, size_t eb, size_t ab, size_t bb)
{
    if ((int)g_pool.slots.size() == nslots && g_pool.geom_bytes >= gb && g_pool.elem_bytes >= eb &&
        g_pool.A_bytes >= ab && g_pool.b_bytes >= bb)
        return FEM_OK;
    release_locked();
    if (hipMalloc(&g_pool.field, 175 * sizeof(double)) != hipSuccess ||
        hipMalloc(&g_pool.status, 2 * sizeof(int32_t)) != hipSuccess) {
        release_locked();
        return FEM_ENOMEM;
    }
    g_pool.slots.resize(nslots);
    for (Slot &s : g_pool.slots) {
        if (hipMalloc(&s.geom, gb) != hipSuccess || hipMalloc(&s.elem, eb) != hipSuccess ||
            hipMalloc(&s.A, ab) != hipSuccess || hipMalloc(&s.b, bb) != hipSuccess) {
            release_locked();
            return FEM_ENOMEM;
        }
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) {
            release_locked();
            return FEM_EHIP;
        }
    }
    g_pool.geom_bytes = gb;
    g_pool.elem_bytes = eb;
    g_pool.A_bytes = ab;
    g_pool.b_bytes = bb;
    return FEM_OK;
}

}  // namespace

void staged_release()
{
    std::lock_guard<std::mutex> lock(g_pool_mutex);
    release_locked();
}

}  // namespace fem

using namespace fem;

extern "C" int fem_integrate_staged(int64_t nel, int p, const double *geom, const fem_coeffs *coeffs,
                                    void *out_A, void *out_b, int64_t chunk, int nstreams,
                                    fem_staged_stats *stats)
{
    if (nel < 0 || !coeffs || chunk <= 0 || nstreams < 1 || nstreams > FEM_STAGED_MAX_STREAMS)
        return FEM_EINVAL;
    if (coeffs->precision < FEM_FP64 || coeffs->precision > FEM_SPLIT_FP16) return FEM_EINVAL;
    const int mode = coeffs->mode;
    if (mode != FEM_COEF_ELEMENT && mode != FEM_COEF_FIELD && mode != FEM_COEF_ELASTIC)
        return FEM_EINVAL;
    if (p < 1 || p > 7) return FEM_EDEGREE;
    if (coeffs->degree || coeffs->a_off || coeffs->b_off || coeffs->jac) return FEM_EINVAL;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (nel == 0) return FEM_OK;
    if (!geom || !coeffs->elem || !out_A || (mode == FEM_COEF_FIELD && !coeffs->field))
        return FEM_EINVAL;

    const int64_t n1 = p + 1, ns = n1 * n1 * n1;
    const int64_t blocks = mode == FEM_COEF_ELASTIC ? 9 : 1, comps = mode == FEM_COEF_ELASTIC ? 3 : 1;
    const int64_t rec = mode == FEM_COEF_ELEMENT ? 14 : (mode == FEM_COEF_FIELD ? 10 : 5);
    const int64_t ob = coeffs->precision == FEM_FP64 ? 8 : 4;
    const int64_t a_per = blocks * ns * ns * ob, b_per = comps * ns * ob;
    const int64_t ce = chunk < nel ? chunk : nel;
    const int64_t nchunks = (nel + ce - 1) / ce;
    const int nslots = (int)(nstreams < nchunks ? nstreams : nchunks);

    std::lock_guard<std::mutex> lock(g_pool_mutex);
    int rc = ensure_locked(nslots, size_t(ce) * 192, size_t(ce * rec) * 8, size_t(ce * a_per),
                           size_t(ce * b_per));
    if (rc != FEM_OK) return rc;
    if (mode == FEM_COEF_FIELD &&
        hipMemcpy(g_pool.field, coeffs->field, 175 * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return FEM_EHIP;
    if (hipMemset(g_pool.status, 0, 2 * sizeof(int32_t)) != hipSuccess) return FEM_EHIP;

    std::vector<hipEvent_t> ev(size_t(nchunks) * 4, nullptr);
    auto cleanup = [&]() {
        for (Slot &s : g_pool.slots) (void)hipStreamSynchronize(s.stream);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    for (hipEvent_t &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            cleanup();
            return FEM_EHIP;
        }

    const auto t0 = std::chrono::steady_clock::now();
    const char *gh = reinterpret_cast<const char *>(geom);
    const char *eh = reinterpret_cast<const char *>(coeffs->elem);
    char *Ah = static_cast<char *>(out_A);
    char *bh = static_cast<char *>(out_b);
    bool ok = true;
    int irc = FEM_OK;
    for (int64_t c = 0; c < nchunks && ok; ++c) {
        Slot &sl = g_pool.slots[size_t(c % nslots)];
        const int64_t e0 = c * ce, n = (nel - e0) < ce ? (nel - e0) : ce;
        hipEvent_t *e = &ev[size_t(c) * 4];
        fem_coeffs cc = *coeffs;
        cc.elem = static_cast<const double *>(sl.elem);
        cc.field = mode == FEM_COEF_FIELD ? g_pool.field : nullptr;
        cc.status = g_pool.status;
        cc.workspace = nullptr;
        cc.workspace_bytes = 0;
        ok = hipEventRecord(e[0], sl.stream) == hipSuccess &&
             hipMemcpyAsync(sl.geom, gh + e0 * 192, size_t(n) * 192, hipMemcpyHostToDevice, sl.stream) == hipSuccess &&
             hipMemcpyAsync(sl.elem, eh + e0 * rec * 8, size_t(n * rec) * 8, hipMemcpyHostToDevice, sl.stream) == hipSuccess &&
             hipEventRecord(e[1], sl.stream) == hipSuccess &&
             (irc = fem_integrate(n, p, static_cast<const double *>(sl.geom), &cc, sl.A, bh ? sl.b : nullptr, sl.stream)) == FEM_OK &&
             hipEventRecord(e[2], sl.stream) == hipSuccess &&
             hipMemcpyAsync(Ah + e0 * a_per, sl.A, size_t(n * a_per), hipMemcpyDeviceToHost, sl.stream) == hipSuccess &&
             (!bh || hipMemcpyAsync(bh + e0 * b_per, sl.b, size_t(n * b_per), hipMemcpyDeviceToHost, sl.stream) == hipSuccess) &&
             hipEventRecord(e[3], sl.stream) == hipSuccess;
    }
    for (Slot &s : g_pool.slots)
        if (hipStreamSynchronize(s.stream) != hipSuccess) ok = false;
    const auto t1 = std::chrono::steady_clock::now();
    if (!ok) {
        cleanup();
        return irc != FEM_OK ? irc : FEM_EHIP;
    }
    if (coeffs->status) {
        int32_t st[2] = {0, 0};
        if (hipMemcpy(st, g_pool.status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) {
            cleanup();
            return FEM_EHIP;
        }
        coeffs->status[0] += st[0];
        coeffs->status[1] += st[1];
    }
    if (stats) {
        stats->total_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        stats->chunks = nchunks;
        stats->h2d_bytes = nel * (192 + rec * 8);
        stats->d2h_bytes = nel * (a_per + (bh ? b_per : 0));
        for (int64_t c = 0; c < nchunks; ++c) {
            float a = 0, k = 0, d = 0;
            hipEvent_t *e = &ev[size_t(c) * 4];
            (void)hipEventElapsedTime(&a, e[0], e[1]);
            (void)hipEventElapsedTime(&k, e[1], e[2]);
            (void)hipEventElapsedTime(&d, e[2], e[3]);
            stats->h2d_ms += a;
            stats->kernel_ms += k;
            stats->d2h_ms += d;
        }
    }
    cleanup();
    return FEM_OK;
}
