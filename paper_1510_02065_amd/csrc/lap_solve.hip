// qap_lap_solve: the batched assignment solve with canonical dual that every
// cost concentration performs (Section 4.1 of arXiv 1510.02065), offered on
// its own for host or device buffers.
//
// Problems of different sizes run in segments of different widths: a problem
// of size n takes the narrowest segment of 8, 16, 32 or 64 lanes that holds
// it, so a wave carries 8, 4, 2 or 1 problems and small problems do not each
// occupy a whole wave.  With host buffers the host sorts the problems into the
// four size classes; with device buffers (whose sizes the host does not read)
// a device pass writes the four work lists into a workspace and each class's
// launch reads its count from there.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "handle.hpp"

using qap::fail;

namespace qap {

// Size class of a problem of size n (0 .. 3 for 8, 16, 32, 64 lanes).  Sizes
// outside [0, 64] go to the widest class, whose kernel marks them unsolved.
__host__ __device__ inline int size_class(int n)
{
    return n <= 8 ? 0 : n <= 16 ? 1 : n <= 32 ? 2 : 3;
}

// Workspace of the device-side bucketing: kBucketHeader ints (the four class
// counters, padded to 256 bytes) followed by four lists of `cap` problem
// indices, list c at lists + c * cap.
constexpr int kBucketHeader = 64;

inline size_t bucket_bytes(long long cap) { return (size_t)(kBucketHeader + 4 * cap) * sizeof(int32_t); }

__global__ __launch_bounds__(64) void k_bucket_clear(int32_t* __restrict__ counts)
{
    if (threadIdx.x < 4) counts[threadIdx.x] = 0;
}

// One thread per problem: append b to the list of its size class.  Each wave
// reserves the places of its problems of a class with one atomic on that
// class's counter (a ballot gives the count and each lane's rank), so the
// counters see one request per wave and class instead of one per problem.
// The order within a list is not fixed; each problem's result depends only
// on its own matrix and the segment width, so it does not matter.
__global__ __launch_bounds__(256) void k_bucket(int batch, const int32_t* __restrict__ n,
                                                int32_t* __restrict__ counts, int32_t* __restrict__ lists,
                                                long long cap)
{
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = b < batch;
    const int c = in ? size_class(n[b]) : -1;
    const unsigned lane = threadIdx.x & 63u;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int k = 0; k < 4; ++k) {
        const unsigned long long m = __builtin_amdgcn_ballot_w64(c == k);
        if (m == 0ull) continue;
        const int leader = __builtin_ctzll(m);
        int base = 0;
        if ((int)lane == leader) base = atomicAdd(&counts[k], __builtin_popcountll(m));
        base = __builtin_amdgcn_readlane(base, leader);
        if (c == k) lists[k * cap + base + __builtin_popcountll(m & below)] = (int32_t)b;
    }
}

// Largest batch of qap_lap_solve_noalloc: its bucketing workspace is the
// static array below, 16 MiB per device.
constexpr long long kNoAllocMaxBatch = QAP_LAP_NOALLOC_MAX_BATCH;

}  // namespace qap

// Bucketing workspace of qap_lap_solve_noalloc, one copy on every device the
// library runs on, held until the process ends.  In host code this name is a
// host-side stand-in, not a device address: kernels and copies get the
// device address from hipGetSymbolAddress (scratch_address below).
static __device__ __align__(256) int32_t scratch[qap::kBucketHeader + 4 * qap::kNoAllocMaxBatch];

namespace {

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

hipError_t scratch_address(int32_t** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[dev] = p;
    }
    *out = static_cast<int32_t*>(g_scratch_addr[dev]);
    return hipSuccess;
}

// The device-pointer solve, given a workspace of bucket_bytes(batch) bytes:
// clear the counters, bucket, then one launch per class with its grid sized
// for the whole batch (the kernel reads the class count and idle slots exit).
hipError_t solve_device(int batch, const int32_t* n, const int64_t* mat_off, const int64_t* vec_off, void* cost,
                        int dtype, double* value, void* duals, int32_t* assign, int wr, int solver, hipStream_t st,
                        int32_t* ws)
{
    int32_t* counts = ws;
    int32_t* lists = ws + qap::kBucketHeader;
    hipLaunchKernelGGL(qap::k_bucket_clear, dim3(1), dim3(64), 0, st, counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(qap::k_bucket, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, st, batch, n, counts, lists,
                       (long long)batch);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int segs[4] = {8, 16, 32, 64};
    for (int c = 0; c < 4; ++c) {
        e = QAP_OPS(dtype, lap_batch(st, segs[c], batch, counts + c, lists + (long long)c * batch, n, mat_off,
                                     vec_off, cost, value, duals, assign, wr, solver));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

qap_status check_common(int batch, const int32_t* n, const int64_t* mat_off, const int64_t* vec_off,
                        const void* cost, int dtype, const double* value, const void* duals, const int32_t* assign)
{
    if (batch < 0) return fail(QAP_EINVAL, "negative batch");
    if (batch == 0) return QAP_OK;
    if (!n || !mat_off || !cost || !value) return fail(QAP_EINVAL, "null n, mat_off, cost or value");
    if ((duals || assign) && !vec_off) return fail(QAP_EINVAL, "vec_off needed for duals or assign");
    if (dtype != QAP_FP64 && dtype != QAP_FP32_CERTIFIED && dtype != QAP_FP32_NEAREST)
        return fail(QAP_EINVAL, "unknown dtype");
    return QAP_OK;
}

}  // namespace

extern "C" {

qap_status qap_lap_solve(int batch, const int32_t* n, const int64_t* mat_off, const int64_t* vec_off, void* cost,
                         int dtype, double* value, void* duals, int32_t* assign, int flags, void* stream)
{
    qap::last_error().clear();
    qap_status cs = check_common(batch, n, mat_off, vec_off, cost, dtype, value, duals, assign);
    if (cs != QAP_OK || batch == 0) return cs;
    const size_t es = dtype == QAP_FP64 ? sizeof(double) : sizeof(float);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int wr = (flags & QAP_LAP_RESIDUAL) ? 1 : 0;
    const int solver = (flags & QAP_LAP_AUCTION) ? QAP_LAP_SOLVER_AUCTION : QAP_LAP_SOLVER_CANONICAL;
    if (flags & QAP_LAP_DEVICE) {
        // The bucketing workspace comes from the stream-ordered allocator, so
        // the call stays asynchronous and calls on other streams get their own.
        void* ws = nullptr;
        hipError_t e = hipMallocAsync(&ws, qap::bucket_bytes(batch), st);
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? QAP_ENOMEM : QAP_EDEVICE,
                        std::string("hipMallocAsync: ") + hipGetErrorString(e));
        e = solve_device(batch, n, mat_off, vec_off, cost, dtype, value, duals, assign, wr, solver, st,
                         static_cast<int32_t*>(ws));
        const hipError_t ef = hipFreeAsync(ws, st);
        if (e != hipSuccess) return fail(QAP_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
        if (ef != hipSuccess) return fail(QAP_EDEVICE, std::string("hipFreeAsync: ") + hipGetErrorString(ef));
        return QAP_OK;
    }
    // Host pointers: validate, bucket by size, stage, solve, copy back.
    int64_t mat_end = 0, vec_end = 0;
    std::vector<int32_t> order[4];   // problems of each size class
    for (int b = 0; b < batch; ++b) {
        if (n[b] < 0 || n[b] > QAP_RLT2_MAX_N) return fail(QAP_EINVAL, "n[b] must be in [0, 64]");
        if (mat_off[b] < 0) return fail(QAP_EINVAL, "negative mat_off");
        mat_end = std::max(mat_end, mat_off[b] + (int64_t)n[b] * n[b]);
        for (int64_t e = 0; e < (int64_t)n[b] * n[b]; ++e) {
            const double x = dtype == QAP_FP64 ? static_cast<const double*>(cost)[mat_off[b] + e]
                                               : (double)static_cast<const float*>(cost)[mat_off[b] + e];
            if (!std::isfinite(x)) return fail(QAP_EINVAL, "non-finite cost entry");
        }
        if (vec_off) {
            if (vec_off[b] < 0) return fail(QAP_EINVAL, "negative vec_off");
            vec_end = std::max(vec_end, vec_off[b] + (int64_t)n[b]);
        }
        order[qap::size_class(n[b])].push_back(b);
    }
    std::vector<int32_t> idx;
    for (auto& o : order) idx.insert(idx.end(), o.begin(), o.end());
    int32_t *dn = nullptr, *didx = nullptr;
    int64_t *dmo = nullptr, *dvo = nullptr;
    void *dcost = nullptr, *ddual = nullptr;
    double* dval = nullptr;
    int32_t* dassign = nullptr;
    qap_status result = QAP_OK;
    auto cleanup = [&]() {
        for (void* p : {(void*)dn, (void*)didx, (void*)dmo, (void*)dvo, (void*)dcost, (void*)dval, (void*)ddual,
                        (void*)dassign})
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
    CK2(hipMalloc(&didx, batch * sizeof(int32_t)));
    CK2(hipMalloc(&dmo, batch * sizeof(int64_t)));
    CK2(hipMalloc(&dcost, std::max<int64_t>(mat_end, 1) * es));
    CK2(hipMalloc(&dval, batch * sizeof(double)));
    CK2(hipMemcpyAsync(dn, n, batch * sizeof(int32_t), hipMemcpyHostToDevice, st));
    CK2(hipMemcpyAsync(didx, idx.data(), batch * sizeof(int32_t), hipMemcpyHostToDevice, st));
    CK2(hipMemcpyAsync(dmo, mat_off, batch * sizeof(int64_t), hipMemcpyHostToDevice, st));
    if (mat_end > 0) CK2(hipMemcpyAsync(dcost, cost, mat_end * es, hipMemcpyHostToDevice, st));
    if (vec_off) {
        CK2(hipMalloc(&dvo, batch * sizeof(int64_t)));
        CK2(hipMemcpyAsync(dvo, vec_off, batch * sizeof(int64_t), hipMemcpyHostToDevice, st));
    }
    if (duals) CK2(hipMalloc(&ddual, std::max<int64_t>(4 * vec_end, 1) * es));
    if (assign) CK2(hipMalloc(&dassign, std::max<int64_t>(vec_end, 1) * sizeof(int32_t)));
    // One launch per size class.
    int64_t first = 0;
    const int segs[4] = {8, 16, 32, 64};
    for (int c = 0; c < 4; ++c) {
        const int cnt = (int)order[c].size();
        if (cnt > 0)
            CK2(QAP_OPS(dtype, lap_batch(st, segs[c], cnt, nullptr, didx + first, dn, dmo, dvo, dcost, dval, ddual,
                                         dassign, wr, solver)));
        first += cnt;
    }
    CK2(hipMemcpyAsync(value, dval, batch * sizeof(double), hipMemcpyDeviceToHost, st));
    if (wr && mat_end > 0) CK2(hipMemcpyAsync(cost, dcost, mat_end * es, hipMemcpyDeviceToHost, st));
    if (duals && vec_end > 0) CK2(hipMemcpyAsync(duals, ddual, 4 * vec_end * es, hipMemcpyDeviceToHost, st));
    if (assign && vec_end > 0)
        CK2(hipMemcpyAsync(assign, dassign, vec_end * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CK2(hipStreamSynchronize(st));
#undef CK2
    cleanup();
    return QAP_OK;
}

qap_status qap_lap_solve_noalloc(int batch, const int32_t* n, const int64_t* mat_off, const int64_t* vec_off,
                                 void* cost, int dtype, double* value, void* duals, int32_t* assign, int flags,
                                 void* stream)
{
    qap::last_error().clear();
    qap_status cs = check_common(batch, n, mat_off, vec_off, cost, dtype, value, duals, assign);
    if (cs != QAP_OK || batch == 0) return cs;
    if (!(flags & QAP_LAP_DEVICE))
        return fail(QAP_EINVAL, "qap_lap_solve_noalloc takes device pointers only (flags must hold QAP_LAP_DEVICE)");
    if (batch > qap::kNoAllocMaxBatch)
        return fail(QAP_EINVAL, "batch exceeds QAP_LAP_NOALLOC_MAX_BATCH (" +
                                    std::to_string(qap::kNoAllocMaxBatch) + ") problems");
    int32_t* ws = nullptr;
    hipError_t e = scratch_address(&ws);
    if (e != hipSuccess) return fail(QAP_EDEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    e = solve_device(batch, n, mat_off, vec_off, cost, dtype, value, duals, assign,
                     (flags & QAP_LAP_RESIDUAL) ? 1 : 0,
                     (flags & QAP_LAP_AUCTION) ? QAP_LAP_SOLVER_AUCTION : QAP_LAP_SOLVER_CANONICAL,
                     static_cast<hipStream_t>(stream), ws);
    if (e != hipSuccess) return fail(QAP_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return QAP_OK;
}

}  // extern "C"
