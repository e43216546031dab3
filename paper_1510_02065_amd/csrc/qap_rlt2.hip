// Host side of the qap_rlt2 library: handle state, launch schedule of one
// dual-ascent iteration (Algorithm 1 of arXiv 1510.02065), HIP-graph replay,
// and the C ABI declared in include/qap_rlt2.h.
#include "qap_rlt2.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lap_kernels.hpp"
#include "rlt2_kernels.hpp"

namespace {

thread_local std::string g_last_error;

qap_status fail(qap_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

#define QAP_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(QAP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int seg_for(int n)
{
    if (n <= 8) return 8;
    if (n <= 16) return 16;
    if (n <= 32) return 32;
    return 64;
}

inline unsigned grid_for(int64_t work, int threads) { return (unsigned)((work + threads - 1) / threads); }

// ---- launch helpers (one wave per workgroup for the assignment kernels) ----

template <typename T, int SEG>
hipError_t launch_family_seg(hipStream_t st, T* blocks, int64_t bstride, int n, int64_t nblocks,
                             T* parent, double* values)
{
    if (nblocks <= 0) return hipSuccess;
    constexpr int LPW = 64 / SEG;
    const size_t lds = LPW * qap::SegLds<T, SEG>::bytes(n);
    const unsigned grid = (unsigned)((nblocks + LPW - 1) / LPW);
    hipLaunchKernelGGL((qap::k_lap_family<T, SEG>), dim3(grid), dim3(64), lds, st, blocks, bstride, n,
                       nblocks, parent, values);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_family(hipStream_t st, T* blocks, int64_t bstride, int n, int64_t nblocks, T* parent,
                         double* values)
{
    switch (seg_for(n)) {
    case 8: return launch_family_seg<T, 8>(st, blocks, bstride, n, nblocks, parent, values);
    case 16: return launch_family_seg<T, 16>(st, blocks, bstride, n, nblocks, parent, values);
    case 32: return launch_family_seg<T, 32>(st, blocks, bstride, n, nblocks, parent, values);
    default: return launch_family_seg<T, 64>(st, blocks, bstride, n, nblocks, parent, values);
    }
}

template <typename T, int SEG>
hipError_t launch_B_seg(hipStream_t st, T* B, int n, double* lb, double* trace, long long* counter,
                        long long cap, double* values)
{
    constexpr int LPW = 64 / SEG;
    const size_t lds = LPW * qap::SegLds<T, SEG>::bytes(n);
    hipLaunchKernelGGL((qap::k_lap_B<T, SEG>), dim3(1), dim3(64), lds, st, B, n, lb, trace, counter, cap,
                       values);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_B(hipStream_t st, T* B, int n, double* lb, double* trace, long long* counter,
                    long long cap, double* values)
{
    switch (seg_for(n)) {
    case 8: return launch_B_seg<T, 8>(st, B, n, lb, trace, counter, cap, values);
    case 16: return launch_B_seg<T, 16>(st, B, n, lb, trace, counter, cap, values);
    case 32: return launch_B_seg<T, 32>(st, B, n, lb, trace, counter, cap, values);
    default: return launch_B_seg<T, 64>(st, B, n, lb, trace, counter, cap, values);
    }
}

template <typename T, int SEG>
hipError_t launch_batch_seg(hipStream_t st, int batch, const int32_t* n, const int64_t* mo,
                            const int64_t* vo, T* cost, double* value, T* duals, int32_t* assign, int wr)
{
    if (batch <= 0) return hipSuccess;
    constexpr int LPW = 64 / SEG;
    const size_t lds = LPW * qap::SegLds<T, SEG>::bytes(SEG);
    const unsigned grid = (unsigned)((batch + LPW - 1) / LPW);
    hipLaunchKernelGGL((qap::k_lap_batch<T, SEG>), dim3(grid), dim3(64), lds, st, batch, n, mo, vo, cost,
                       value, duals, assign, wr);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch(hipStream_t st, int seg, int batch, const int32_t* n, const int64_t* mo,
                        const int64_t* vo, T* cost, double* value, T* duals, int32_t* assign, int wr)
{
    switch (seg) {
    case 8: return launch_batch_seg<T, 8>(st, batch, n, mo, vo, cost, value, duals, assign, wr);
    case 16: return launch_batch_seg<T, 16>(st, batch, n, mo, vo, cost, value, duals, assign, wr);
    case 32: return launch_batch_seg<T, 32>(st, batch, n, mo, vo, cost, value, duals, assign, wr);
    default: return launch_batch_seg<T, 64>(st, batch, n, mo, vo, cost, value, duals, assign, wr);
    }
}

constexpr long long kTraceCap = 1024;

}  // namespace

// ============================================================================
// Handle
// ============================================================================

struct qap_rlt2 {
    int N = 0;
    int precision = QAP_FP64;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int trace_level = 1;
    int use_graph = 1;
    size_t elem = 8;       // bytes per reduced cost
    int64_t nB = 0, nC = 0, nblkD = 0, ldD = 0, ngroups = 0;
    void* dB = nullptr;
    void* dC = nullptr;
    void* dD = nullptr;
    void* dCC = nullptr;
    double* dLB = nullptr;      // [LB, LB']
    double* dValD = nullptr;    // per-block values of the last step 4
    double* dValC = nullptr;    // per-block values of the last step 6
    double* dValB = nullptr;
    double* dTrace = nullptr;   // kTraceCap x (LB, LB')
    long long* dCounter = nullptr;
    int* dTri = nullptr;
    double* dCt = nullptr;      // certification: c~ per C entry
    double* dBt = nullptr;      // certification: b~ per B entry
    double* dCert = nullptr;    // certification result
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<double> tLB, tLBp;
    int64_t iterations = 0;
    bool broken = false;
};

namespace {

template <typename T>
hipError_t enqueue_step(qap_rlt2* h, int step)
{
    const int N = h->N;
    T* B = static_cast<T*>(h->dB);
    T* C = static_cast<T*>(h->dC);
    T* D = static_cast<T*>(h->dD);
    T* CC = static_cast<T*>(h->dCC);
    hipStream_t st = h->stream;
    const bool vals = h->trace_level >= 2;
    switch (step) {
    case 3: {   // steps 1-3
        hipLaunchKernelGGL((qap::k_spread_prep<T>), dim3(grid_for(h->nC, 256)), dim3(256), 0, st, C, B, CC, N);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int ntri = N * (N - 1) * (N - 2) / 6;
        const int wpt = (N * (N - 1) * (N - 2) + 255) / 256;
        const unsigned grid = (unsigned)(8 * ((ntri + 7) / 8) * wpt);
        hipLaunchKernelGGL((qap::k_sweep<T>), dim3(grid), dim3(256), 0, st, D, CC, B, h->dTri, N, h->ldD, ntri,
                           wpt);
        return hipGetLastError();
    }
    case 4:
        return launch_family<T>(st, D, h->ldD, N - 2, h->nblkD, C, vals ? h->dValD : nullptr);
    case 5:
        hipLaunchKernelGGL((qap::k_transfer_C<T>), dim3(grid_for(h->nC, 256)), dim3(256), 0, st, C, N);
        return hipGetLastError();
    case 6:
        return launch_family<T>(st, C, (int64_t)(N - 1) * (N - 1), N - 1, h->nB, B, vals ? h->dValC : nullptr);
    case 7:
        return launch_B<T>(st, B, N, h->dLB, h->trace_level >= 1 ? h->dTrace : nullptr,
                           h->trace_level >= 1 ? h->dCounter : nullptr, kTraceCap, vals ? h->dValB : nullptr);
    default:
        return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t enqueue_certify(qap_rlt2* h)
{
    const int N = h->N, n2 = N - 2;
    hipStream_t st = h->stream;
    hipLaunchKernelGGL((qap::k_cert_D<T>), dim3(grid_for(h->nblkD, 4)), dim3(256), 0, st,
                       static_cast<const T*>(h->dD), h->ldD, n2 * n2, h->nblkD, static_cast<const T*>(h->dC),
                       h->dCt, N);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((qap::k_cert_C<T>), dim3(grid_for(h->nB, 4)), dim3(256), 0, st, h->dCt,
                       static_cast<const T*>(h->dB), h->dBt, N);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(qap::k_cert_final, dim3(1), dim3(64), 0, st, h->dBt, N, h->dLB, h->dCert);
    return hipGetLastError();
}

hipError_t enqueue_step_any(qap_rlt2* h, int step)
{
    return h->precision == QAP_FP64 ? enqueue_step<double>(h, step) : enqueue_step<float>(h, step);
}

hipError_t enqueue_iteration(qap_rlt2* h)
{
    for (int s : {3, 4, 5, 6, 7}) {
        hipError_t e = enqueue_step_any(h, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Copy the trace entries written since the counter was last reset, then reset.
qap_status drain_trace(qap_rlt2* h)
{
    long long cnt = 0;
    QAP_HIP(hipMemcpyAsync(&cnt, h->dCounter, sizeof(cnt), hipMemcpyDeviceToHost, h->stream));
    QAP_HIP(hipStreamSynchronize(h->stream));
    cnt = std::min(cnt, kTraceCap);
    if (cnt > 0) {
        std::vector<double> buf(2 * (size_t)cnt);
        QAP_HIP(hipMemcpyAsync(buf.data(), h->dTrace, buf.size() * sizeof(double), hipMemcpyDeviceToHost,
                               h->stream));
        QAP_HIP(hipStreamSynchronize(h->stream));
        for (long long t = 0; t < cnt; ++t) {
            h->tLB.push_back(buf[2 * t]);
            h->tLBp.push_back(buf[2 * t + 1]);
        }
    }
    const long long zero = 0;
    QAP_HIP(hipMemcpyAsync(h->dCounter, &zero, sizeof(zero), hipMemcpyHostToDevice, h->stream));
    QAP_HIP(hipStreamSynchronize(h->stream));
    return QAP_OK;
}

void release(qap_rlt2* h)
{
    if (!h) return;
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    void* ptrs[] = {h->dB, h->dC, h->dD, h->dCC, h->dLB, h->dValD, h->dValC, h->dValB, h->dTrace,
                    h->dCounter, h->dTri, h->dCt, h->dBt, h->dCert};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
}

qap_status check_handle(qap_rlt2* h)
{
    if (!h) return fail(QAP_EINVAL, "null handle");
    if (h->broken) return fail(QAP_ESTATE, "handle unusable after an earlier device failure");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return fail(QAP_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    return QAP_OK;
}

qap_status mark_broken(qap_rlt2* h, hipError_t e, const char* what)
{
    h->broken = true;
    return fail(QAP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

extern "C" {

qap_status qap_rlt2_default_opts(qap_rlt2_opts* o)
{
    if (!o) return fail(QAP_EINVAL, "null opts");
    o->precision = QAP_FP64;
    o->device = -1;
    o->stream = nullptr;
    o->trace_level = 1;
    o->use_graph = 1;
    return QAP_OK;
}

qap_status qap_rlt2_create(int N, const double* F, const double* D, qap_rlt2** out)
{
    return qap_rlt2_create_ex(N, F, D, nullptr, 0.0, nullptr, out);
}

qap_status qap_rlt2_create_ex(int N, const double* F, const double* Dm, const double* B0, double constant,
                              const qap_rlt2_opts* opts, qap_rlt2** out)
{
    g_last_error.clear();
    if (!out) return fail(QAP_EINVAL, "null output handle pointer");
    *out = nullptr;
    if (N < 3 || N > QAP_RLT2_MAX_N) return fail(QAP_EINVAL, "N must be in [3, 64]");
    if (!F || !Dm) return fail(QAP_EINVAL, "null F or D");
    for (int x = 0; x < N * N; ++x)
        if (!std::isfinite(F[x]) || !std::isfinite(Dm[x]) || (B0 && !std::isfinite(B0[x])))
            return fail(QAP_EINVAL, "non-finite entry in F, D or B0");
    if (!std::isfinite(constant)) return fail(QAP_EINVAL, "non-finite constant");
    qap_rlt2_opts o;
    qap_rlt2_default_opts(&o);
    if (opts) o = *opts;
    if (o.precision != QAP_FP64 && o.precision != QAP_FP32_CERTIFIED)
        return fail(QAP_EINVAL, "unknown precision");

    qap_rlt2* h = new (std::nothrow) qap_rlt2();
    if (!h) return fail(QAP_ENOMEM, "host allocation failed");
    h->N = N;
    h->precision = o.precision;
    h->trace_level = std::max(0, std::min(2, o.trace_level));
    h->use_graph = o.use_graph ? 1 : 0;
    h->elem = o.precision == QAP_FP64 ? sizeof(double) : sizeof(float);

    auto bail = [&](qap_status st) {
        release(h);
        delete h;
        return st;
    };
#define CK(call)                                                                                    \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return bail(fail(e_ == hipErrorOutOfMemory ? QAP_ENOMEM : QAP_EDEVICE,                   \
                             std::string(#call) + ": " + hipGetErrorString(e_)));                   \
    } while (0)

    if (o.device >= 0) {
        CK(hipSetDevice(o.device));
        h->device = o.device;
    } else {
        CK(hipGetDevice(&h->device));
    }
    if (o.stream) {
        h->stream = static_cast<hipStream_t>(o.stream);
    } else {
        CK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
        h->own_stream = true;
    }

    const int n1 = N - 1, n2 = N - 2;
    h->nB = (int64_t)N * N;
    h->nC = h->nB * n1 * n1;
    h->nblkD = h->nC;
    const int64_t blk = (int64_t)n2 * n2;
    const int64_t align_elems = 128 / (int64_t)h->elem;
    h->ldD = (blk + align_elems - 1) / align_elems * align_elems;
    h->ngroups = (int64_t)N * (N - 1) * (N - 2) / 6 * ((int64_t)N * n1 * n2);

    const size_t bytesD = (size_t)h->nblkD * h->ldD * h->elem;
    size_t freeb = 0, totalb = 0;
    CK(hipMemGetInfo(&freeb, &totalb));
    if (bytesD + (size_t)h->nC * h->elem * 2 > freeb)
        return bail(fail(QAP_ENOMEM, "reduced-cost array does not fit in free device memory"));

    CK(hipMalloc(&h->dB, h->nB * h->elem));
    CK(hipMalloc(&h->dC, h->nC * h->elem));
    CK(hipMalloc(&h->dCC, h->nC * h->elem));
    CK(hipMalloc(&h->dD, bytesD));
    CK(hipMalloc(&h->dLB, 2 * sizeof(double)));
    CK(hipMalloc(&h->dTrace, 2 * kTraceCap * sizeof(double)));
    CK(hipMalloc(&h->dCounter, sizeof(long long)));
    CK(hipMalloc(&h->dCt, h->nC * sizeof(double)));
    CK(hipMalloc(&h->dBt, h->nB * sizeof(double)));
    CK(hipMalloc(&h->dCert, sizeof(double)));
    if (h->trace_level >= 2) {
        CK(hipMalloc(&h->dValD, h->nblkD * sizeof(double)));
        CK(hipMalloc(&h->dValC, h->nB * sizeof(double)));
        CK(hipMalloc(&h->dValB, sizeof(double)));
    }
    std::vector<int> tri;
    for (int i = 0; i < N; ++i)
        for (int k = i + 1; k < N; ++k)
            for (int p = k + 1; p < N; ++p) {
                tri.push_back(i);
                tri.push_back(k);
                tri.push_back(p);
            }
    CK(hipMalloc(&h->dTri, tri.size() * sizeof(int)));
    CK(hipMemcpyAsync(h->dTri, tri.data(), tri.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));

    double* dF = nullptr;
    double* dDm = nullptr;
    double* dB0 = nullptr;
    CK(hipMalloc(&dF, h->nB * sizeof(double)));
    CK(hipMalloc(&dDm, h->nB * sizeof(double)));
    if (B0) CK(hipMalloc(&dB0, h->nB * sizeof(double)));
    CK(hipMemcpyAsync(dF, F, h->nB * sizeof(double), hipMemcpyHostToDevice, h->stream));
    CK(hipMemcpyAsync(dDm, Dm, h->nB * sizeof(double), hipMemcpyHostToDevice, h->stream));
    if (B0) CK(hipMemcpyAsync(dB0, B0, h->nB * sizeof(double), hipMemcpyHostToDevice, h->stream));
    const double lb0[2] = {constant, 0.0};
    CK(hipMemcpyAsync(h->dLB, lb0, sizeof(lb0), hipMemcpyHostToDevice, h->stream));
    const long long zero = 0;
    CK(hipMemcpyAsync(h->dCounter, &zero, sizeof(zero), hipMemcpyHostToDevice, h->stream));
    CK(hipMemsetAsync(h->dD, 0, bytesD, h->stream));

    if (h->precision == QAP_FP64) {
        hipLaunchKernelGGL((qap::k_init<double>), dim3(grid_for(h->nC, 256)), dim3(256), 0, h->stream, dF, dDm,
                           dB0, static_cast<double*>(h->dB), static_cast<double*>(h->dC), N);
    } else {
        hipLaunchKernelGGL((qap::k_init<float>), dim3(grid_for(h->nC, 256)), dim3(256), 0, h->stream, dF, dDm,
                           dB0, static_cast<float*>(h->dB), static_cast<float*>(h->dC), N);
    }
    CK(hipGetLastError());
    // Iteration 0: C -> B, then B -> LB.
    CK(enqueue_step_any(h, 6));
    CK(enqueue_step_any(h, 7));
    CK(hipStreamSynchronize(h->stream));
    (void)hipFree(dF);
    (void)hipFree(dDm);
    if (dB0) (void)hipFree(dB0);
    qap_status st = drain_trace(h);
    if (st != QAP_OK) return bail(st);
#undef CK
    *out = h;
    return QAP_OK;
}

qap_status qap_rlt2_ascend(qap_rlt2* h, int iters, double* bound)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (iters < 0) return fail(QAP_EINVAL, "iters must be >= 0");
    int left = iters;
    while (left > 0) {
        const int chunk = (int)std::min<long long>(left, kTraceCap);
        if (h->use_graph) {
            if (!h->graph_exec) {
                hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) return mark_broken(h, e, "hipStreamBeginCapture");
                hipError_t el = enqueue_iteration(h);
                e = hipStreamEndCapture(h->stream, &h->graph);
                if (el != hipSuccess) return mark_broken(h, el, "kernel launch during capture");
                if (e != hipSuccess) return mark_broken(h, e, "hipStreamEndCapture");
                e = hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0);
                if (e != hipSuccess) return mark_broken(h, e, "hipGraphInstantiate");
            }
            for (int t = 0; t < chunk; ++t) {
                hipError_t e = hipGraphLaunch(h->graph_exec, h->stream);
                if (e != hipSuccess) return mark_broken(h, e, "hipGraphLaunch");
            }
        } else {
            for (int t = 0; t < chunk; ++t) {
                hipError_t e = enqueue_iteration(h);
                if (e != hipSuccess) return mark_broken(h, e, "kernel launch");
            }
        }
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return mark_broken(h, e, "hipStreamSynchronize");
        h->iterations += chunk;
        st = drain_trace(h);
        if (st != QAP_OK) {
            h->broken = true;
            return st;
        }
        left -= chunk;
    }
    if (bound) {
        if (h->precision == QAP_FP64) {
            double lb[2];
            hipError_t e = hipMemcpy(lb, h->dLB, sizeof(lb), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return mark_broken(h, e, "hipMemcpy");
            *bound = lb[0];
        } else {
            return qap_rlt2_certify(h, bound);
        }
    }
    return QAP_OK;
}

qap_status qap_rlt2_step(qap_rlt2* h, int step)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (step != 3 && step != 4 && step != 5 && step != 6 && step != 7)
        return fail(QAP_EINVAL, "step must be 3 (steps 1-3), 4, 5, 6 or 7 (steps 7-8)");
    hipError_t e = enqueue_step_any(h, step);
    if (e != hipSuccess) return mark_broken(h, e, "kernel launch");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return mark_broken(h, e, "hipStreamSynchronize");
    if (step == 7) {
        h->iterations += 1;
        st = drain_trace(h);
        if (st != QAP_OK) return st;
    }
    return QAP_OK;
}

qap_status qap_rlt2_certify(qap_rlt2* h, double* certified)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (!certified) return fail(QAP_EINVAL, "null output");
    hipError_t e = h->precision == QAP_FP64 ? enqueue_certify<double>(h) : enqueue_certify<float>(h);
    if (e != hipSuccess) return mark_broken(h, e, "certification launch");
    e = hipMemcpyAsync(certified, h->dCert, sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return mark_broken(h, e, "hipMemcpyAsync");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return mark_broken(h, e, "hipStreamSynchronize");
    return QAP_OK;
}

qap_status qap_rlt2_bound(qap_rlt2* h, double* lb, int64_t* iterations)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (lb) {
        double v[2];
        hipError_t e = hipMemcpy(v, h->dLB, sizeof(v), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return mark_broken(h, e, "hipMemcpy");
        *lb = v[0];
    }
    if (iterations) *iterations = h->iterations;
    return QAP_OK;
}

qap_status qap_rlt2_trace(qap_rlt2* h, int64_t capacity, int64_t* count, double* lb, double* lbprime)
{
    if (!h) return fail(QAP_EINVAL, "null handle");
    if (capacity < 0) return fail(QAP_EINVAL, "negative capacity");
    const int64_t n = (int64_t)h->tLB.size();
    if (count) *count = n;
    const int64_t m = std::min(n, capacity);
    if (lb) std::copy(h->tLB.begin(), h->tLB.begin() + m, lb);
    if (lbprime) std::copy(h->tLBp.begin(), h->tLBp.begin() + m, lbprime);
    return QAP_OK;
}

qap_status qap_rlt2_lap_values(qap_rlt2* h, double* sD, double* sC, double* sB)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (h->trace_level < 2) return fail(QAP_EINVAL, "per-assignment values need trace_level 2");
    if (sD) QAP_HIP(hipMemcpy(sD, h->dValD, h->nblkD * sizeof(double), hipMemcpyDeviceToHost));
    if (sC) QAP_HIP(hipMemcpy(sC, h->dValC, h->nB * sizeof(double), hipMemcpyDeviceToHost));
    if (sB) QAP_HIP(hipMemcpy(sB, h->dValB, sizeof(double), hipMemcpyDeviceToHost));
    return QAP_OK;
}

qap_status qap_rlt2_read_state(qap_rlt2* h, double* lb, double* B, double* C, double* D)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    QAP_HIP(hipStreamSynchronize(h->stream));
    if (lb) {
        double v[2];
        QAP_HIP(hipMemcpy(v, h->dLB, sizeof(v), hipMemcpyDeviceToHost));
        *lb = v[0];
    }
    const int n2 = h->N - 2;
    const int64_t blk = (int64_t)n2 * n2;
    auto widen = [&](void* dst, const void* src, int64_t count, size_t src_pitch, int64_t rows) -> hipError_t {
        if (h->precision == QAP_FP64) {
            return hipMemcpy2D(dst, count * sizeof(double), src, src_pitch, count * sizeof(double), rows,
                               hipMemcpyDeviceToHost);
        }
        std::vector<float> tmp((size_t)count * rows);
        hipError_t e = hipMemcpy2D(tmp.data(), count * sizeof(float), src, src_pitch, count * sizeof(float), rows,
                                   hipMemcpyDeviceToHost);
        if (e != hipSuccess) return e;
        double* d = static_cast<double*>(dst);
        for (size_t x = 0; x < tmp.size(); ++x) d[x] = (double)tmp[x];
        return hipSuccess;
    };
    if (B) QAP_HIP(widen(B, h->dB, h->nB, h->nB * h->elem, 1));
    if (C) QAP_HIP(widen(C, h->dC, h->nC, h->nC * h->elem, 1));
    if (D) QAP_HIP(widen(D, h->dD, blk, h->ldD * h->elem, h->nblkD));
    return QAP_OK;
}

void qap_rlt2_destroy(qap_rlt2* h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    release(h);
    delete h;
}

qap_status qap_lap_solve(int batch, const int32_t* n, const int64_t* mat_off, const int64_t* vec_off, void* cost,
                         int dtype, double* value, void* duals, int32_t* assign, int flags, void* stream)
{
    g_last_error.clear();
    if (batch < 0) return fail(QAP_EINVAL, "negative batch");
    if (batch == 0) return QAP_OK;
    if (!n || !mat_off || !cost || !value) return fail(QAP_EINVAL, "null n, mat_off, cost or value");
    if ((duals || assign) && !vec_off) return fail(QAP_EINVAL, "vec_off needed for duals or assign");
    if (dtype != QAP_FP64 && dtype != QAP_FP32_CERTIFIED) return fail(QAP_EINVAL, "unknown dtype");
    const bool f32 = dtype == QAP_FP32_CERTIFIED;
    const size_t es = f32 ? sizeof(float) : sizeof(double);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int wr = (flags & QAP_LAP_RESIDUAL) ? 1 : 0;
    if (flags & QAP_LAP_DEVICE) {
        if (f32)
            QAP_HIP(launch_batch<float>(st, 64, batch, n, mat_off, vec_off, static_cast<float*>(cost), value,
                                        static_cast<float*>(duals), assign, wr));
        else
            QAP_HIP(launch_batch<double>(st, 64, batch, n, mat_off, vec_off, static_cast<double*>(cost), value,
                                         static_cast<double*>(duals), assign, wr));
        return QAP_OK;
    }
    // Host pointers: validate, stage, solve, copy back.
    int maxn = 0;
    int64_t mat_end = 0, vec_end = 0;
    for (int b = 0; b < batch; ++b) {
        if (n[b] < 0 || n[b] > QAP_RLT2_MAX_N) return fail(QAP_EINVAL, "n[b] must be in [0, 64]");
        if (mat_off[b] < 0) return fail(QAP_EINVAL, "negative mat_off");
        maxn = std::max(maxn, (int)n[b]);
        mat_end = std::max(mat_end, mat_off[b] + (int64_t)n[b] * n[b]);
        for (int64_t e = 0; e < (int64_t)n[b] * n[b]; ++e) {
            const double x = f32 ? (double)static_cast<const float*>(cost)[mat_off[b] + e]
                                 : static_cast<const double*>(cost)[mat_off[b] + e];
            if (!std::isfinite(x)) return fail(QAP_EINVAL, "non-finite cost entry");
        }
        if (vec_off) {
            if (vec_off[b] < 0) return fail(QAP_EINVAL, "negative vec_off");
            vec_end = std::max(vec_end, vec_off[b] + (int64_t)n[b]);
        }
    }
    const int seg = seg_for(std::max(maxn, 1));
    int32_t* dn = nullptr;
    int64_t *dmo = nullptr, *dvo = nullptr;
    void *dcost = nullptr, *ddual = nullptr;
    double* dval = nullptr;
    int32_t* dassign = nullptr;
    qap_status result = QAP_OK;
    auto cleanup = [&]() {
        for (void* p : {(void*)dn, (void*)dmo, (void*)dvo, (void*)dcost, (void*)dval, (void*)ddual, (void*)dassign})
            if (p) (void)hipFree(p);
    };
#define CK2(call)                                                                                    \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            result = fail(e_ == hipErrorOutOfMemory ? QAP_ENOMEM : QAP_EDEVICE,                      \
                          std::string(#call) + ": " + hipGetErrorString(e_));                        \
            cleanup();                                                                               \
            return result;                                                                           \
        }                                                                                            \
    } while (0)
    CK2(hipMalloc(&dn, batch * sizeof(int32_t)));
    CK2(hipMalloc(&dmo, batch * sizeof(int64_t)));
    CK2(hipMalloc(&dcost, std::max<int64_t>(mat_end, 1) * es));
    CK2(hipMalloc(&dval, batch * sizeof(double)));
    CK2(hipMemcpyAsync(dn, n, batch * sizeof(int32_t), hipMemcpyHostToDevice, st));
    CK2(hipMemcpyAsync(dmo, mat_off, batch * sizeof(int64_t), hipMemcpyHostToDevice, st));
    CK2(hipMemcpyAsync(dcost, cost, mat_end * es, hipMemcpyHostToDevice, st));
    if (vec_off) {
        CK2(hipMalloc(&dvo, batch * sizeof(int64_t)));
        CK2(hipMemcpyAsync(dvo, vec_off, batch * sizeof(int64_t), hipMemcpyHostToDevice, st));
    }
    if (duals) CK2(hipMalloc(&ddual, std::max<int64_t>(4 * vec_end, 1) * es));
    if (assign) CK2(hipMalloc(&dassign, std::max<int64_t>(vec_end, 1) * sizeof(int32_t)));
    if (f32)
        CK2(launch_batch<float>(st, seg, batch, dn, dmo, dvo, static_cast<float*>(dcost), dval,
                                static_cast<float*>(ddual), dassign, wr));
    else
        CK2(launch_batch<double>(st, seg, batch, dn, dmo, dvo, static_cast<double*>(dcost), dval,
                                 static_cast<double*>(ddual), dassign, wr));
    CK2(hipMemcpyAsync(value, dval, batch * sizeof(double), hipMemcpyDeviceToHost, st));
    if (wr) CK2(hipMemcpyAsync(cost, dcost, mat_end * es, hipMemcpyDeviceToHost, st));
    if (duals) CK2(hipMemcpyAsync(duals, ddual, 4 * vec_end * es, hipMemcpyDeviceToHost, st));
    if (assign) CK2(hipMemcpyAsync(assign, dassign, vec_end * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CK2(hipStreamSynchronize(st));
#undef CK2
    cleanup();
    return QAP_OK;
}

const char* qap_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
