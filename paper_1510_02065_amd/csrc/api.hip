// C ABI of the qap_rlt2 library (include/qap_rlt2.h): handles for one or many
// instances, the schedule of one dual-ascent iteration (Algorithm 1 of
// arXiv 1510.02065), HIP-graph replay, state I/O and snapshots, the stop rule,
// children of branch-and-bound nodes, strong branching and the batched
// assignment solve.  The kernels are launched by the per-precision code in
// ops_impl.hpp; nothing here runs on the device itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "handle.hpp"

namespace qap {
std::string& last_error()
{
    thread_local std::string msg;
    return msg;
}
}  // namespace qap

using qap::fail;

namespace {

// ---- autotuner cache ---------------------------------------------------------

std::string tune_key(const qap_rlt2* h, int famk, const qap::ClassHost& c)
{
    char buf[128];
    snprintf(buf, sizeof(buf), "gfx950 prec=%d fam=%d seg=%d nmax=%d", h->precision, famk, c.seg, c.nmax);
    return buf;
}

std::map<std::string, std::pair<int, int>> read_tune_file(const std::string& path)
{
    std::map<std::string, std::pair<int, int>> m;
    FILE* f = fopen(path.c_str(), "r");
    if (!f) return m;
    char line[256];
    while (fgets(line, sizeof(line), f)) {
        char* bar = strchr(line, '|');
        if (!bar) continue;
        *bar = 0;
        int seg = 0, k = 0;
        if (sscanf(bar + 1, "%d %d", &seg, &k) == 2) m[line] = {seg, k};
    }
    fclose(f);
    return m;
}

void load_tune_cache(qap_rlt2* h)
{
    if (h->tune_cache.empty()) return;
    const auto m = read_tune_file(h->tune_cache);
    int hits = 0, need = 0;
    for (int famk = 0; famk < 2; ++famk)
        for (qap::ClassHost& c : h->fam[famk]) {
            if (c.total <= 0) continue;
            ++need;
            auto it = m.find(tune_key(h, famk, c));
            if (it != m.end() && qap::slot_cfg_allowed(it->second.first, it->second.second) &&
                it->second.first * it->second.second >= c.nmax) {
                c.seg_run = it->second.first;
                c.k_run = it->second.second;
                ++hits;
            }
        }
    if (need > 0 && hits == need) h->tuned = true;
}

void save_tune_cache(const qap_rlt2* h)
{
    if (h->tune_cache.empty()) return;
    auto m = read_tune_file(h->tune_cache);
    for (int famk = 0; famk < 2; ++famk)
        for (const qap::ClassHost& c : h->fam[famk])
            if (c.total > 0) m[tune_key(h, famk, c)] = {c.seg_run, c.k_run};
    if (FILE* f = fopen(h->tune_cache.c_str(), "w")) {
        for (auto& kv : m) fprintf(f, "%s|%d %d\n", kv.first.c_str(), kv.second.first, kv.second.second);
        fclose(f);
    }
}

// ---- iteration schedule ------------------------------------------------------

hipError_t enqueue_step_any(qap_rlt2* h, int step) { return QAP_OPS(h->precision, enqueue_step(h, step)); }

hipError_t enqueue_iteration(qap_rlt2* h)
{
    if (h->overlap) {
        hipError_t e = QAP_OPS(h->precision, enqueue_sweep_concentrate_overlapped(h));
        for (int s : {5, 6, 7})
            if (e == hipSuccess) e = enqueue_step_any(h, s);
        return e;
    }
    for (int s : {3, 4, 5, 6, 7}) {
        hipError_t e = enqueue_step_any(h, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// First iteration of a handle with autotuning: run the steps one by one and
// tune each concentration family on its live data just before it runs.
hipError_t tuned_first_iteration(qap_rlt2* h)
{
    hipError_t e;
    if (h->lap_solver == QAP_LAP_SOLVER_AUCTION) {   // one column per lane: nothing to tune
        h->tuned = true;
        return enqueue_iteration(h);
    }
    if ((e = enqueue_step_any(h, 3)) != hipSuccess) return e;
    if (h->level == 2 && (e = QAP_OPS(h->precision, tune_family(h, qap::kFamD))) != hipSuccess) return e;
    if ((e = enqueue_step_any(h, 4)) != hipSuccess) return e;
    if ((e = enqueue_step_any(h, 5)) != hipSuccess) return e;
    if ((e = QAP_OPS(h->precision, tune_family(h, qap::kFamC))) != hipSuccess) return e;
    if ((e = enqueue_step_any(h, 6)) != hipSuccess) return e;
    if ((e = enqueue_step_any(h, 7)) != hipSuccess) return e;
    h->tuned = true;
    save_tune_cache(h);
    return hipSuccess;
}

// Copy the trace entries written since the counters were last reset, add the
// iteration counts, then reset the counters.  `counts_iteration0`: the
// entries come from iteration 0 (recorded in the trace, not counted).
qap_status drain_trace(qap_rlt2* h, bool counts_iteration0 = false)
{
    std::vector<long long> cnt(h->K);
    QAP_HIP(hipMemcpyAsync(cnt.data(), h->dCounter, h->K * sizeof(long long), hipMemcpyDeviceToHost, h->stream));
    QAP_HIP(hipStreamSynchronize(h->stream));
    long long mx = 0;
    for (long long c : cnt) mx = std::max(mx, std::min(c, qap::kTraceCap));
    if (mx > 0 && h->trace_level >= 1) {
        std::vector<double> buf((size_t)h->K * qap::kTraceCap * 2);
        QAP_HIP(hipMemcpyAsync(buf.data(), h->dTrace, buf.size() * sizeof(double), hipMemcpyDeviceToHost,
                               h->stream));
        QAP_HIP(hipStreamSynchronize(h->stream));
        for (int k = 0; k < h->K; ++k) {
            const long long c = std::min(cnt[k], qap::kTraceCap);
            for (long long t = 0; t < c; ++t) {
                h->tLB[k].push_back(buf[((size_t)k * qap::kTraceCap + t) * 2]);
                h->tLBp[k].push_back(buf[((size_t)k * qap::kTraceCap + t) * 2 + 1]);
            }
        }
    }
    if (!counts_iteration0)
        for (int k = 0; k < h->K; ++k) h->itk[k] += cnt[k];
    QAP_HIP(hipMemsetAsync(h->dCounter, 0, h->K * sizeof(long long), h->stream));
    QAP_HIP(hipStreamSynchronize(h->stream));
    return QAP_OK;
}

void release(qap_rlt2* h)
{
    if (!h) return;
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    void* ptrs[] = {h->dB,     h->dC,     h->dD,     h->dCC,   h->dLB,   h->dValD,  h->dValC,  h->dValB,
                    h->dTrace, h->dCounter, h->dTri, h->dAct,  h->dStop, h->dSigma, h->dCt,    h->dBt,
                    h->dCert,  h->dInst,  h->dPreB,  h->dPreC, h->dPreWG};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (auto& f : h->fam)
        for (auto& c : f) {
            if (c.d_ids) (void)hipFree(c.d_ids);
            if (c.d_pre) (void)hipFree(c.d_pre);
        }
    for (auto& c : h->sweep_cls) {
        if (c.d_ids) (void)hipFree(c.d_ids);
        if (c.d_pre) (void)hipFree(c.d_pre);
    }
    for (auto& c : h->famD_size) {
        if (c.d_ids) (void)hipFree(c.d_ids);
        if (c.d_pre) (void)hipFree(c.d_pre);
    }
    for (hipEvent_t ev : h->ev_size)
        if (ev) (void)hipEventDestroy(ev);
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    if (h->stream2) (void)hipStreamDestroy(h->stream2);
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

template <typename X>
hipError_t upload(X** dst, const std::vector<X>& v, hipStream_t st)
{
    hipError_t e = hipMalloc(dst, std::max<size_t>(v.size(), 1) * sizeof(X));
    if (e != hipSuccess) return e;
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice, st);
}

// Layout and device memory of a handle with `count` instances of sizes Ns
// (no values yet: D is zero, B, C and LB uninitialised).
qap_status make_handle(int count, const int32_t* Ns, const qap_rlt2_opts& o, qap_rlt2** out)
{
    *out = nullptr;
    if (count < 1) return fail(QAP_EINVAL, "count must be >= 1");
    for (int k = 0; k < count; ++k)
        if (Ns[k] < 3 || Ns[k] > QAP_RLT2_MAX_N) return fail(QAP_EINVAL, "N must be in [3, 64]");
    if (o.precision != QAP_FP64 && o.precision != QAP_FP32_CERTIFIED && o.precision != QAP_FP32_NEAREST)
        return fail(QAP_EINVAL, "unknown precision");
    if (o.level != 1 && o.level != 2) return fail(QAP_EINVAL, "level must be 1 or 2");
    if (o.lap_solver != QAP_LAP_SOLVER_CANONICAL && o.lap_solver != QAP_LAP_SOLVER_AUCTION)
        return fail(QAP_EINVAL, "unknown lap_solver");
    if (!std::isfinite(o.K) || !std::isfinite(o.UB)) return fail(QAP_EINVAL, "non-finite K or UB");

    qap_rlt2* h = new (std::nothrow) qap_rlt2();
    if (!h) return fail(QAP_ENOMEM, "host allocation failed");
    h->K = count;
    h->precision = o.precision;
    h->level = o.level;
    h->trace_level = std::max(0, std::min(2, o.trace_level));
    h->use_graph = o.use_graph ? 1 : 0;
    h->autotune = o.autotune ? 1 : 0;
    h->lap_solver = o.lap_solver;
    if (o.tune_cache) h->tune_cache = o.tune_cache;
    h->dmode = o.complementary ? qap::kHalfStore : qap::kAllBlocks;
    h->elem = o.precision == QAP_FP64 ? sizeof(double) : sizeof(float);
    h->stopK = o.K;
    h->stopUB = o.UB;
    h->tLB.resize(count);
    h->tLBp.resize(count);
    h->itk.assign(count, 0);

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
    {
        int lim = 0;
        if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) == hipSuccess && lim > 0)
            h->lds_limit = (size_t)lim;
        if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess && lim > 0)
            h->num_cu = lim;
    }
    // Packed layout of all instances, and the steps 1-3 kernel: one
    // workgroup per facility triple when the largest instance's triple fits
    // in LDS, else location cubes; k_sweep when every block is stored.
    const long long align_elems = 128 / (long long)h->elem;
    for (int k = 0; k < count; ++k) h->Nmax = std::max(h->Nmax, (int)Ns[k]);
    if (h->dmode == qap::kAllBlocks)
        h->sweep_kind = 0;
    else
        h->sweep_kind = QAP_OPS(h->precision, sweep_lds(h->Nmax)) <= h->lds_limit ? 2 : 1;
    h->inst.resize(count);
    for (int k = 0; k < count; ++k) {
        const int N = Ns[k], n1 = N - 1, n2 = N - 2;
        qap::Inst& I = h->inst[k];
        I.N = N;
        I.ntri = N * (N - 1) * (N - 2) / 6;
        I.wpt = h->sweep_kind == 0 ? (N * n1 * n2 + 255) / 256 : h->sweep_kind == 1 ? qap::kSweepParts : 1;
        I.pad_ = 0;
        I.offB = h->totalB;
        I.offC = h->totalC;
        I.offD = h->totalD;
        I.ldD = ((long long)n2 * n2 + align_elems - 1) / align_elems * align_elems;
        I.wg0 = h->totalWG;
        I.tri0 = (long long)h->tri.size();
        if (h->level == 2)   // facility triples of the sweep
            for (int i = 0; i < N; ++i)
                for (int kk = i + 1; kk < N; ++kk)
                    for (int p = kk + 1; p < N; ++p) {
                        h->tri.push_back(i);
                        h->tri.push_back(kk);
                        h->tri.push_back(p);
                    }
        h->preB.push_back(h->totalB);
        h->preC.push_back(h->totalC);
        h->preWG.push_back(h->totalWG);
        const long long nC = (long long)N * N * n1 * n1;
        h->totalB += (long long)N * N;
        h->totalC += nC;
        if (h->level == 2) {
            if (h->dmode == qap::kAllBlocks)
                h->totalD += nC * I.ldD;
            else   // pair-major, one block per pair, unpadded; instances start 128-byte aligned
                h->totalD += ((nC / 2) * n2 * n2 + align_elems - 1) / align_elems * align_elems;
        }
        h->totalWG += h->sweep_kind == 2 ? (long long)I.ntri : 8LL * ((I.ntri + 7) / 8) * I.wpt;
    }
    // One sweep launch per instance size when a batch mixes sizes.
    if (h->sweep_kind == 2 && h->level == 2) {
        h->sweep_nt = QAP_OPS(h->precision, triple_threads(h->Nmax));
        std::vector<int> sizes(Ns, Ns + count);
        std::sort(sizes.begin(), sizes.end(), std::greater<int>());
        sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
        if (sizes.size() > 1) {
            for (int N : sizes) {
                qap::SweepClass c;
                c.N = N;
                c.nt = QAP_OPS(h->precision, triple_threads(N));
                for (int k = 0; k < count; ++k)
                    if ((int)Ns[k] == N) {
                        c.ids.push_back(k);
                        c.pre.push_back(c.ntri);
                        c.ntri += h->inst[k].ntri;
                    }
                h->sweep_cls.push_back(std::move(c));
            }
        }
    }
    // Segment-size classes of the three families.
    for (int f = 0; f < 3; ++f) {
        if (f == 0 && h->level == 1) continue;
        for (int k = 0; k < count; ++k) {
            const int N = Ns[k];
            const int n = (f == 0) ? N - 2 : (f == 1) ? N - 1 : N;
            const int seg = qap::seg_for(n);
            const int ci = seg == 8 ? 0 : seg == 16 ? 1 : seg == 32 ? 2 : 3;
            qap::ClassHost& c = h->fam[f][ci];
            c.seg = seg;
            c.nmax = std::max(c.nmax, n);
            c.ids.push_back(k);
            c.pre.push_back(c.total);
            const long long nblk = (long long)N * N * (N - 1) * (N - 1);
            c.total += (f == 0) ? (h->dmode == qap::kAllBlocks ? nblk : nblk / 2) : (f == 1) ? (long long)N * N : 1;
        }
    }
    // Default configuration of every class: the most problems per wave that
    // fit (families D and C).  The B family (one problem per instance) is
    // latency-bound: one column per lane, the smallest segment that holds it.
    for (qap::ClassHost& c : h->fam[2]) {
        if (c.total <= 0) continue;
        const int seg = qap::seg_for(c.nmax);
        if (qap::slot_lds_prec(h->precision, seg, 1, c.nmax) <= h->lds_limit) {
            c.seg_run = seg;
            c.k_run = 1;
        }
    }
    for (auto& f : h->fam)
        for (qap::ClassHost& c : f) {
            if (c.total <= 0 || c.seg_run != 0) continue;
            for (int seg : {8, 16, 32, 64}) {
                const int k = (c.nmax + seg - 1) / seg;
                if (!qap::slot_cfg_allowed(seg, k)) continue;
                if (qap::slot_lds_prec(h->precision, seg, k, c.nmax) > h->lds_limit) continue;
                c.seg_run = seg;
                c.k_run = k;
                break;
            }
            if (c.seg_run == 0) return bail(fail(QAP_EINVAL, "problem size needs more LDS than a workgroup has"));
        }

    // The overlapped schedule: the D family split by instance size, in the
    // sweep classes' order, a second stream and the events between them.
    if (o.overlap && h->level == 2 && h->dmode == qap::kHalfStore && h->sweep_cls.size() > 1) {
        for (const qap::SweepClass& sc : h->sweep_cls) {
            qap::ClassHost c;
            c.nmax = sc.N - 2;
            c.seg = qap::seg_for(c.nmax);
            for (int k : sc.ids) {
                const long long N = h->inst[k].N;
                c.ids.push_back(k);
                c.pre.push_back(c.total);
                c.total += N * N * (N - 1) * (N - 1) / 2;
            }
            h->famD_size.push_back(std::move(c));
        }
        CK(hipStreamCreateWithFlags(&h->stream2, hipStreamNonBlocking));
        h->ev_size.assign(h->sweep_cls.size(), nullptr);
        for (hipEvent_t& ev : h->ev_size) CK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        CK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
        CK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
        h->overlap = true;
    }

    const size_t bytesD = (size_t)h->totalD * h->elem;
    size_t freeb = 0, totalb = 0;
    CK(hipMemGetInfo(&freeb, &totalb));
    const size_t ccbytes = h->level == 2 ? (size_t)h->totalC * h->elem : 0;
    if (bytesD + ccbytes + (size_t)h->totalC * (h->elem + 8) > freeb)
        return bail(fail(QAP_ENOMEM, "reduced-cost arrays do not fit in free device memory"));

    CK(hipMalloc(&h->dB, h->totalB * h->elem));
    CK(hipMalloc(&h->dC, h->totalC * h->elem));
    if (h->level == 2) {
        CK(hipMalloc(&h->dCC, h->totalC * h->elem));
        CK(hipMalloc(&h->dD, std::max<size_t>(bytesD, 1)));
    }
    CK(hipMalloc(&h->dLB, 2 * count * sizeof(double)));
    CK(hipMalloc(&h->dTrace, 2 * qap::kTraceCap * count * sizeof(double)));
    CK(hipMalloc(&h->dCounter, count * sizeof(long long)));
    CK(hipMalloc(&h->dAct, count * sizeof(int)));
    CK(hipMalloc(&h->dStop, 2 * sizeof(double)));
    CK(hipMalloc(&h->dSigma, h->totalB * sizeof(int32_t)));
    CK(hipMalloc(&h->dCert, count * sizeof(double)));
    if (h->trace_level >= 2) {
        CK(hipMalloc(&h->dValD, h->totalC * sizeof(double)));
        CK(hipMalloc(&h->dValC, h->totalB * sizeof(double)));
        CK(hipMalloc(&h->dValB, count * sizeof(double)));
    }
    CK(upload(&h->dTri, h->tri, h->stream));
    CK(upload(&h->dInst, h->inst, h->stream));
    CK(upload(&h->dPreB, h->preB, h->stream));
    CK(upload(&h->dPreC, h->preC, h->stream));
    CK(upload(&h->dPreWG, h->preWG, h->stream));
    for (auto& c : h->sweep_cls) {
        CK(upload(&c.d_ids, c.ids, h->stream));
        CK(upload(&c.d_pre, c.pre, h->stream));
    }
    for (auto& f : h->fam)
        for (auto& c : f) {
            if (c.ids.empty()) continue;
            CK(upload(&c.d_ids, c.ids, h->stream));
            CK(upload(&c.d_pre, c.pre, h->stream));
        }
    for (auto& c : h->famD_size) {
        CK(upload(&c.d_ids, c.ids, h->stream));
        CK(upload(&c.d_pre, c.pre, h->stream));
    }
    if (h->autotune) load_tune_cache(h);
    const std::vector<int> ones(count, 1);
    const double stop[2] = {h->stopK, h->stopUB};
    CK(hipMemcpyAsync(h->dAct, ones.data(), count * sizeof(int), hipMemcpyHostToDevice, h->stream));
    CK(hipMemcpyAsync(h->dStop, stop, sizeof(stop), hipMemcpyHostToDevice, h->stream));
    CK(hipMemsetAsync(h->dCounter, 0, count * sizeof(long long), h->stream));
    CK(hipMemsetAsync(h->dSigma, 0, h->totalB * sizeof(int32_t), h->stream));
    if (h->level == 2) CK(hipMemsetAsync(h->dD, 0, std::max<size_t>(bytesD, 1), h->stream));
    CK(hipStreamSynchronize(h->stream));
#undef CK
    *out = h;
    return QAP_OK;
}

void destroy_handle(qap_rlt2* h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    release(h);
    delete h;
}

// Move the trace entries of iterations run by qap_rlt2_step to the host.
qap_status flush_steps(qap_rlt2* h)
{
    if (h->pending == 0) return QAP_OK;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return mark_broken(h, e, "hipStreamSynchronize");
    qap_status st = drain_trace(h);
    if (st != QAP_OK) {
        h->broken = true;
        return st;
    }
    h->pending = 0;
    return QAP_OK;
}

bool any_active(qap_rlt2* h, hipError_t* err)
{
    std::vector<int> act(h->K);
    *err = hipMemcpyAsync(act.data(), h->dAct, h->K * sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (*err == hipSuccess) *err = hipStreamSynchronize(h->stream);
    if (*err != hipSuccess) return false;
    for (int a : act)
        if (a) return true;
    return false;
}

// Round an FP64 host value as the FP32 modes write it into the state.
float host_round(double x, int precision)
{
    float f = (float)x;
    if (precision == QAP_FP32_CERTIFIED && (double)f > x) f = std::nextafter(f, -std::numeric_limits<float>::infinity());
    return f;
}

// The device copy of one handle's values that a snapshot holds.
struct SnapPart {
    void* dev;
    size_t bytes;
};

std::vector<SnapPart> snap_parts(qap_rlt2* h)
{
    return {{h->dB, (size_t)h->totalB * h->elem},
            {h->dC, (size_t)h->totalC * h->elem},
            {h->dD, h->level == 2 ? (size_t)h->totalD * h->elem : 0},
            {h->dLB, 2 * (size_t)h->K * sizeof(double)},
            {h->dAct, (size_t)h->K * sizeof(int)},
            {h->dStop, 2 * sizeof(double)},
            {h->dSigma, (size_t)h->totalB * sizeof(int32_t)}};
}

constexpr char kSnapMagic[8] = {'Q', 'A', 'P', 'R', 'L', 'T', '2', 'S'};
constexpr uint32_t kSnapVersion = 1;

// Little serialisation helpers over a byte vector / cursor.
template <typename X>
void put(std::vector<char>& v, const X& x)
{
    const char* p = reinterpret_cast<const char*>(&x);
    v.insert(v.end(), p, p + sizeof(X));
}
template <typename X>
bool get(const char*& p, const char* end, X& x)
{
    if ((size_t)(end - p) < sizeof(X)) return false;
    memcpy(&x, p, sizeof(X));
    p += sizeof(X);
    return true;
}

// Header of a snapshot: the layout it must be restored into.
std::vector<char> snap_header(const qap_rlt2* h)
{
    std::vector<char> v(kSnapMagic, kSnapMagic + 8);
    put(v, kSnapVersion);
    put(v, (int32_t)h->K);
    put(v, (int32_t)h->precision);
    put(v, (int32_t)h->level);
    put(v, (int32_t)h->dmode);
    put(v, (int64_t)h->totalB);
    put(v, (int64_t)h->totalC);
    put(v, (int64_t)h->totalD);
    for (const auto& I : h->inst) put(v, (int32_t)I.N);
    return v;
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
    o->autotune = 1;
    o->tune_cache = nullptr;
    o->complementary = 1;
    o->K = 0.0;
    o->UB = 0.0;
    o->level = 2;
    o->lap_solver = QAP_LAP_SOLVER_CANONICAL;
    o->overlap = 1;
    return QAP_OK;
}

qap_status qap_rlt2_create(int N, const double* F, const double* D, qap_rlt2** out)
{
    return qap_rlt2_create_ex(N, F, D, nullptr, 0.0, nullptr, out);
}

qap_status qap_rlt2_create_ex(int N, const double* F, const double* Dm, const double* B0, double constant,
                              const qap_rlt2_opts* opts, qap_rlt2** out)
{
    const int32_t n32 = N;
    const double* Fs[1] = {F};
    const double* Ds[1] = {Dm};
    const double* Bs[1] = {B0};
    return qap_rlt2_batch_create(1, &n32, Fs, Ds, Bs, &constant, opts, out);
}

qap_status qap_rlt2_batch_create(int count, const int32_t* Ns, const double* const* Fs, const double* const* Ds,
                                 const double* const* B0s, const double* constants, const qap_rlt2_opts* opts,
                                 qap_rlt2** out)
{
    qap::last_error().clear();
    if (!out) return fail(QAP_EINVAL, "null output handle pointer");
    *out = nullptr;
    if (count < 1) return fail(QAP_EINVAL, "count must be >= 1");
    if (!Ns || !Fs || !Ds) return fail(QAP_EINVAL, "null N, F or D array");
    for (int k = 0; k < count; ++k) {
        const int N = Ns[k];
        if (N < 3 || N > QAP_RLT2_MAX_N) return fail(QAP_EINVAL, "N must be in [3, 64]");
        if (!Fs[k] || !Ds[k]) return fail(QAP_EINVAL, "null F or D");
        const double* B0 = B0s ? B0s[k] : nullptr;
        for (int x = 0; x < N * N; ++x)
            if (!std::isfinite(Fs[k][x]) || !std::isfinite(Ds[k][x]) || (B0 && !std::isfinite(B0[x])))
                return fail(QAP_EINVAL, "non-finite entry in F, D or B0");
        if (constants && !std::isfinite(constants[k])) return fail(QAP_EINVAL, "non-finite constant");
    }
    qap_rlt2_opts o;
    qap_rlt2_default_opts(&o);
    if (opts) o = *opts;
    qap_rlt2* h = nullptr;
    qap_status st = make_handle(count, Ns, o, &h);
    if (st != QAP_OK) return st;
    auto bail = [&](qap_status s) {
        destroy_handle(h);
        return s;
    };
#define CK(call)                                                                                    \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return bail(fail(e_ == hipErrorOutOfMemory ? QAP_ENOMEM : QAP_EDEVICE,                   \
                             std::string(#call) + ": " + hipGetErrorString(e_)));                   \
    } while (0)
    std::vector<double> lb0(2 * count, 0.0);
    for (int k = 0; k < count; ++k) lb0[2 * k] = constants ? constants[k] : 0.0;
    CK(hipMemcpyAsync(h->dLB, lb0.data(), lb0.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));

    // Initial dual of every instance.
    double* dF = nullptr;
    double* dDm = nullptr;
    double* dB0 = nullptr;
    const size_t nbmax = (size_t)h->Nmax * h->Nmax * sizeof(double);
    auto free_staging = [&]() {
        (void)hipFree(dF);
        (void)hipFree(dDm);
        (void)hipFree(dB0);
    };
    hipError_t e = hipMalloc(&dF, nbmax);
    if (e == hipSuccess) e = hipMalloc(&dDm, nbmax);
    if (e == hipSuccess) e = hipMalloc(&dB0, nbmax);
    for (int k = 0; k < count && e == hipSuccess; ++k) {
        const int N = Ns[k];
        const size_t nb = (size_t)N * N * sizeof(double);
        const double* B0 = B0s ? B0s[k] : nullptr;
        e = hipMemcpyAsync(dF, Fs[k], nb, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(dDm, Ds[k], nb, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess && B0) e = hipMemcpyAsync(dB0, B0, nb, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = QAP_OPS(h->precision, init_instance(h, k, dF, dDm, B0 ? dB0 : nullptr));
        // The staging buffers are reused by the next instance.
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    }
    free_staging();
    CK(e);
    // Iteration 0: C -> B, then B -> LB.
    CK(enqueue_step_any(h, 6));
    CK(enqueue_step_any(h, 7));
    CK(hipStreamSynchronize(h->stream));
    st = drain_trace(h, true);
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
    if ((st = flush_steps(h)) != QAP_OK) return st;
    int left = iters;
    const bool stop_rule = h->stopUB > 0.0;
    if (left > 0 && stop_rule) {
        hipError_t e = hipSuccess;
        if (!any_active(h, &e)) {
            if (e != hipSuccess) return mark_broken(h, e, "reading the stop flags");
            left = 0;
        }
    }
    if (left > 0 && h->autotune && !h->tuned) {
        hipError_t e = tuned_first_iteration(h);
        if (e != hipSuccess) return mark_broken(h, e, "autotuned first iteration");
        e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return mark_broken(h, e, "hipStreamSynchronize");
        st = drain_trace(h);
        if (st != QAP_OK) {
            h->broken = true;
            return st;
        }
        --left;
    }
    while (left > 0) {
        // With the stop rule on, iterations go in small chunks so that the
        // call returns soon after every instance has stopped.
        const int chunk = (int)std::min<long long>(left, stop_rule ? 8 : qap::kTraceCap);
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
        st = drain_trace(h);
        if (st != QAP_OK) {
            h->broken = true;
            return st;
        }
        left -= chunk;
        if (left > 0 && stop_rule && !any_active(h, &e)) {
            if (e != hipSuccess) return mark_broken(h, e, "reading the stop flags");
            break;
        }
    }
    if (bound) {
        if (h->precision == QAP_FP64) {
            double lb[2];
            hipError_t e = hipStreamSynchronize(h->stream);
            if (e == hipSuccess) e = hipMemcpy(lb, h->dLB, sizeof(lb), hipMemcpyDeviceToHost);
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
    if (step == 7) {
        // The trace entry stays on the device until a call reads the trace
        // or the device buffer is full.
        if (++h->pending >= qap::kTraceCap) return flush_steps(h);
    }
    return QAP_OK;
}

qap_status qap_rlt2_batch_bounds(qap_rlt2* h, double* lb, double* certified)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (certified) {
        hipError_t e = hipSuccess;
        if (!h->dCt) e = hipMalloc(&h->dCt, h->totalC * sizeof(double));
        if (e == hipSuccess && !h->dBt) e = hipMalloc(&h->dBt, h->totalB * sizeof(double));
        if (e != hipSuccess) return fail(QAP_ENOMEM, std::string("certification buffers: ") + hipGetErrorString(e));
        e = QAP_OPS(h->precision, certify(h));
        if (e != hipSuccess) return mark_broken(h, e, "certification launch");
        e = hipMemcpyAsync(certified, h->dCert, h->K * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        if (e != hipSuccess) return mark_broken(h, e, "hipMemcpyAsync");
    }
    if (lb) {
        std::vector<double> v(2 * h->K);
        hipError_t e = hipMemcpyAsync(v.data(), h->dLB, v.size() * sizeof(double), hipMemcpyDeviceToHost,
                                      h->stream);
        if (e != hipSuccess) return mark_broken(h, e, "hipMemcpyAsync");
        e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return mark_broken(h, e, "hipStreamSynchronize");
        for (int k = 0; k < h->K; ++k) lb[k] = v[2 * k];
    }
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return mark_broken(h, e, "hipStreamSynchronize");
    return QAP_OK;
}

qap_status qap_rlt2_certify(qap_rlt2* h, double* certified)
{
    if (!certified) return fail(QAP_EINVAL, "null output");
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    std::vector<double> c(h->K);
    st = qap_rlt2_batch_bounds(h, nullptr, c.data());
    if (st == QAP_OK) *certified = c[0];
    return st;
}

qap_status qap_rlt2_count(qap_rlt2* h, int* count)
{
    if (!h || !count) return fail(QAP_EINVAL, "null argument");
    *count = h->K;
    return QAP_OK;
}

qap_status qap_rlt2_bound(qap_rlt2* h, double* lb, int64_t* iterations)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if ((st = flush_steps(h)) != QAP_OK) return st;
    if (lb) {
        double v[2];
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e == hipSuccess) e = hipMemcpy(v, h->dLB, sizeof(v), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return mark_broken(h, e, "hipMemcpy");
        *lb = v[0];
    }
    if (iterations) *iterations = h->itk[0];
    return QAP_OK;
}

qap_status qap_rlt2_set_stop(qap_rlt2* h, double K, double UB)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (!std::isfinite(K) || !std::isfinite(UB)) return fail(QAP_EINVAL, "non-finite K or UB");
    h->stopK = K;
    h->stopUB = UB;
    const double stop[2] = {K, UB};
    QAP_HIP(hipMemcpyAsync(h->dStop, stop, sizeof(stop), hipMemcpyHostToDevice, h->stream));
    QAP_HIP(hipStreamSynchronize(h->stream));
    return QAP_OK;
}

qap_status qap_rlt2_batch_status(qap_rlt2* h, int* active, int64_t* iterations)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if ((st = flush_steps(h)) != QAP_OK) return st;
    if (active) {
        QAP_HIP(hipMemcpyAsync(active, h->dAct, h->K * sizeof(int), hipMemcpyDeviceToHost, h->stream));
        QAP_HIP(hipStreamSynchronize(h->stream));
    }
    if (iterations) std::copy(h->itk.begin(), h->itk.end(), iterations);
    return QAP_OK;
}

qap_status qap_rlt2_instance_assignment(qap_rlt2* h, int k, int32_t* perm)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (k < 0 || k >= h->K) return fail(QAP_EINVAL, "instance index out of range");
    if (!perm) return fail(QAP_EINVAL, "null perm");
    const qap::Inst& I = h->inst[k];
    QAP_HIP(hipStreamSynchronize(h->stream));
    QAP_HIP(hipMemcpy(perm, h->dSigma + I.offB, I.N * sizeof(int32_t), hipMemcpyDeviceToHost));
    return QAP_OK;
}

qap_status qap_rlt2_instance_trace(qap_rlt2* h, int k, int64_t capacity, int64_t* count, double* lb,
                                   double* lbprime)
{
    if (!h) return fail(QAP_EINVAL, "null handle");
    if (!h->broken && h->pending > 0) {
        qap_status st = flush_steps(h);
        if (st != QAP_OK) return st;
    }
    if (k < 0 || k >= h->K) return fail(QAP_EINVAL, "instance index out of range");
    if (capacity < 0) return fail(QAP_EINVAL, "negative capacity");
    const int64_t n = (int64_t)h->tLB[k].size();
    if (count) *count = n;
    const int64_t m = std::min(n, capacity);
    if (lb) std::copy(h->tLB[k].begin(), h->tLB[k].begin() + m, lb);
    if (lbprime) std::copy(h->tLBp[k].begin(), h->tLBp[k].begin() + m, lbprime);
    return QAP_OK;
}

qap_status qap_rlt2_trace(qap_rlt2* h, int64_t capacity, int64_t* count, double* lb, double* lbprime)
{
    return qap_rlt2_instance_trace(h, 0, capacity, count, lb, lbprime);
}

qap_status qap_rlt2_instance_lap_values(qap_rlt2* h, int k, double* sD, double* sC, double* sB)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (k < 0 || k >= h->K) return fail(QAP_EINVAL, "instance index out of range");
    if (h->trace_level < 2) return fail(QAP_EINVAL, "per-assignment values need trace_level 2");
    const qap::Inst& I = h->inst[k];
    const long long nC = (long long)I.N * I.N * (I.N - 1) * (I.N - 1);
    QAP_HIP(hipStreamSynchronize(h->stream));
    if (sD) QAP_HIP(hipMemcpy(sD, h->dValD + I.offC, nC * sizeof(double), hipMemcpyDeviceToHost));
    if (sC) QAP_HIP(hipMemcpy(sC, h->dValC + I.offB, (size_t)I.N * I.N * sizeof(double), hipMemcpyDeviceToHost));
    if (sB) QAP_HIP(hipMemcpy(sB, h->dValB + k, sizeof(double), hipMemcpyDeviceToHost));
    return QAP_OK;
}

qap_status qap_rlt2_lap_values(qap_rlt2* h, double* sD, double* sC, double* sB)
{
    return qap_rlt2_instance_lap_values(h, 0, sD, sC, sB);
}

qap_status qap_rlt2_instance_state(qap_rlt2* h, int k, double* lb, double* B, double* C, double* D)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (k < 0 || k >= h->K) return fail(QAP_EINVAL, "instance index out of range");
    QAP_HIP(hipStreamSynchronize(h->stream));
    const qap::Inst& I = h->inst[k];
    const int N = I.N, n2 = N - 2;
    if (lb) {
        double v[2];
        QAP_HIP(hipMemcpy(v, h->dLB + 2 * k, sizeof(v), hipMemcpyDeviceToHost));
        *lb = v[0];
    }
    const long long blk = (long long)n2 * n2;
    const long long nC = (long long)N * N * (N - 1) * (N - 1);
    auto widen = [&](void* dst, const void* src, long long count, size_t src_pitch, long long rows) -> hipError_t {
        if (h->precision == QAP_FP64)
            return hipMemcpy2D(dst, count * sizeof(double), src, src_pitch, count * sizeof(double), rows,
                               hipMemcpyDeviceToHost);
        std::vector<float> tmp((size_t)count * rows);
        hipError_t e = hipMemcpy2D(tmp.data(), count * sizeof(float), src, src_pitch, count * sizeof(float), rows,
                                   hipMemcpyDeviceToHost);
        if (e != hipSuccess) return e;
        double* d = static_cast<double*>(dst);
        for (size_t x = 0; x < tmp.size(); ++x) d[x] = (double)tmp[x];
        return hipSuccess;
    };
    const char* b = static_cast<const char*>(h->dB) + I.offB * h->elem;
    const char* c = static_cast<const char*>(h->dC) + I.offC * h->elem;
    if (B) QAP_HIP(widen(B, b, (long long)N * N, (size_t)N * N * h->elem, 1));
    if (C) QAP_HIP(widen(C, c, nC, (size_t)nC * h->elem, 1));
    if (D && h->level == 2) {
        const char* d = static_cast<const char*>(h->dD) + I.offD * h->elem;
        if (h->dmode == qap::kAllBlocks) {
            QAP_HIP(widen(D, d, blk, I.ldD * h->elem, nC));
        } else {
            // One stored block per complementary pair, pair-major: copy each
            // row to both blocks of the pair.
            const long long total = (nC / 2) * blk;
            std::vector<double> half((size_t)total);
            QAP_HIP(widen(half.data(), d, total, (size_t)total * h->elem, 1));
            const long long ld = (long long)N * (N - 1) * n2;
            for (long long hb = 0; hb < nC / 2; ++hb) {
                long long beta = 0, twin = 0, base = 0;
                qap::pair_block(N, hb, &beta, &twin, &base);
                for (int r = 0; r < n2; ++r) {
                    const double* src = half.data() + base + r * ld;
                    std::copy(src, src + n2, D + beta * blk + r * n2);
                    std::copy(src, src + n2, D + twin * blk + r * n2);
                }
            }
        }
    }
    return QAP_OK;
}

qap_status qap_rlt2_read_state(qap_rlt2* h, double* lb, double* B, double* C, double* D)
{
    return qap_rlt2_instance_state(h, 0, lb, B, C, D);
}

qap_status qap_rlt2_load_state(qap_rlt2* h, int k, const double* lb, const double* B, const double* C,
                               const double* D)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (k < 0 || k >= h->K) return fail(QAP_EINVAL, "instance index out of range");
    if ((st = flush_steps(h)) != QAP_OK) return st;
    const qap::Inst& I = h->inst[k];
    const int N = I.N, n2 = N - 2;
    const long long blk = (long long)n2 * n2;
    const long long nC = (long long)N * N * (N - 1) * (N - 1);
    auto check = [](const double* a, long long n) {
        for (long long x = 0; x < n; ++x)
            if (!std::isfinite(a[x])) return false;
        return true;
    };
    if ((lb && !std::isfinite(*lb)) || (B && !check(B, (long long)N * N)) || (C && !check(C, nC)) ||
        (D && h->level == 2 && !check(D, nC * blk)))
        return fail(QAP_EINVAL, "non-finite entry in the state");
    // Host array -> device, rounded as the handle's mode writes its state.
    auto narrow = [&](void* dst, const double* src, long long count) -> hipError_t {
        if (h->precision == QAP_FP64)
            return hipMemcpy(dst, src, count * sizeof(double), hipMemcpyHostToDevice);
        std::vector<float> tmp((size_t)count);
        for (long long x = 0; x < count; ++x) tmp[x] = host_round(src[x], h->precision);
        return hipMemcpy(dst, tmp.data(), count * sizeof(float), hipMemcpyHostToDevice);
    };
    QAP_HIP(hipStreamSynchronize(h->stream));
    if (lb) QAP_HIP(hipMemcpy(h->dLB + 2 * k, lb, sizeof(double), hipMemcpyHostToDevice));
    if (B) QAP_HIP(narrow(static_cast<char*>(h->dB) + I.offB * h->elem, B, (long long)N * N));
    if (C) QAP_HIP(narrow(static_cast<char*>(h->dC) + I.offC * h->elem, C, nC));
    if (D && h->level == 2) {
        char* d = static_cast<char*>(h->dD) + I.offD * h->elem;
        if (h->dmode == qap::kAllBlocks) {
            std::vector<double> pad((size_t)(nC * I.ldD), 0.0);
            for (long long b = 0; b < nC; ++b) std::copy(D + b * blk, D + (b + 1) * blk, pad.begin() + b * I.ldD);
            QAP_HIP(narrow(d, pad.data(), nC * I.ldD));
        } else {
            const long long total = (nC / 2) * blk;
            const long long ld = (long long)N * (N - 1) * n2;
            std::vector<double> half((size_t)total);
            for (long long hb = 0; hb < nC / 2; ++hb) {
                long long beta = 0, twin = 0, base = 0;
                qap::pair_block(N, hb, &beta, &twin, &base);
                for (int r = 0; r < n2; ++r)
                    std::copy(D + beta * blk + r * n2, D + beta * blk + (r + 1) * n2, half.begin() + base + r * ld);
            }
            QAP_HIP(narrow(d, half.data(), total));
        }
    }
    return QAP_OK;
}

qap_status qap_rlt2_snapshot(qap_rlt2* h, void* buf, uint64_t capacity, uint64_t* size)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (!size) return fail(QAP_EINVAL, "null size");
    if ((st = flush_steps(h)) != QAP_OK) return st;
    std::vector<char> v = snap_header(h);
    size_t need = v.size();
    for (const SnapPart& p : snap_parts(h)) need += p.bytes;
    // host part: tuned choices, iteration counts and traces
    std::vector<char> tail;
    put(tail, (int32_t)h->tuned);
    for (auto& f : h->fam)
        for (auto& c : f) {
            put(tail, (int32_t)c.seg_run);
            put(tail, (int32_t)c.k_run);
        }
    for (int k = 0; k < h->K; ++k) {
        put(tail, (int64_t)h->itk[k]);
        put(tail, (int64_t)h->tLB[k].size());
        for (size_t t = 0; t < h->tLB[k].size(); ++t) {
            put(tail, h->tLB[k][t]);
            put(tail, h->tLBp[k][t]);
        }
    }
    need += tail.size();
    *size = need;
    if (!buf) return QAP_OK;
    if (capacity < need) return fail(QAP_EINVAL, "snapshot buffer too small");
    char* p = static_cast<char*>(buf);
    memcpy(p, v.data(), v.size());
    p += v.size();
    QAP_HIP(hipStreamSynchronize(h->stream));
    for (const SnapPart& s : snap_parts(h)) {
        if (s.bytes) QAP_HIP(hipMemcpy(p, s.dev, s.bytes, hipMemcpyDeviceToHost));
        p += s.bytes;
    }
    memcpy(p, tail.data(), tail.size());
    return QAP_OK;
}

qap_status qap_rlt2_restore(qap_rlt2* h, const void* buf, uint64_t size)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (!buf) return fail(QAP_EINVAL, "null buffer");
    if ((st = flush_steps(h)) != QAP_OK) return st;
    const std::vector<char> hdr = snap_header(h);
    if (size < hdr.size() || memcmp(buf, hdr.data(), hdr.size()) != 0)
        return fail(QAP_EINVAL, "snapshot does not match this handle's instances, precision, level or storage");
    const char* p = static_cast<const char*>(buf) + hdr.size();
    const char* end = static_cast<const char*>(buf) + size;
    const auto parts = snap_parts(h);
    size_t dev_bytes = 0;
    for (const SnapPart& s : parts) dev_bytes += s.bytes;
    if ((size_t)(end - p) < dev_bytes) return fail(QAP_EINVAL, "truncated snapshot");
    // Parse the host part before touching the device.
    const char* q = p + dev_bytes;
    int32_t tuned = 0;
    if (!get(q, end, tuned)) return fail(QAP_EINVAL, "truncated snapshot");
    int32_t cfg[3][4][2];
    for (int f = 0; f < 3; ++f)
        for (int c = 0; c < 4; ++c)
            if (!get(q, end, cfg[f][c][0]) || !get(q, end, cfg[f][c][1]))
                return fail(QAP_EINVAL, "truncated snapshot");
    std::vector<int64_t> itk(h->K);
    std::vector<std::vector<double>> tl(h->K), tp(h->K);
    for (int k = 0; k < h->K; ++k) {
        int64_t n = 0;
        if (!get(q, end, itk[k]) || !get(q, end, n) || n < 0 || (uint64_t)n > (uint64_t)(end - q) / 16)
            return fail(QAP_EINVAL, "truncated snapshot");
        tl[k].resize(n);
        tp[k].resize(n);
        for (int64_t t = 0; t < n; ++t) {
            get(q, end, tl[k][t]);
            get(q, end, tp[k][t]);
        }
    }
    for (int f = 0; f < 3; ++f)
        for (int c = 0; c < 4; ++c) {
            qap::ClassHost& ch = h->fam[f][c];
            if (ch.total <= 0) continue;
            const int sg = cfg[f][c][0], kk = cfg[f][c][1];
            if (!qap::slot_cfg_allowed(sg, kk) || sg * kk < ch.nmax ||
                qap::slot_lds_prec(h->precision, sg, kk, ch.nmax) > h->lds_limit)
                return fail(QAP_EINVAL, "snapshot holds a kernel configuration this device cannot run");
        }
    QAP_HIP(hipStreamSynchronize(h->stream));
    for (const SnapPart& s : parts) {
        if (s.bytes) QAP_HIP(hipMemcpy(s.dev, p, s.bytes, hipMemcpyHostToDevice));
        p += s.bytes;
    }
    QAP_HIP(hipMemsetAsync(h->dCounter, 0, h->K * sizeof(long long), h->stream));
    QAP_HIP(hipStreamSynchronize(h->stream));
    h->tuned = tuned != 0;
    bool changed = false;
    for (int f = 0; f < 3; ++f)
        for (int c = 0; c < 4; ++c) {
            qap::ClassHost& ch = h->fam[f][c];
            if (ch.total <= 0) continue;
            changed = changed || ch.seg_run != cfg[f][c][0] || ch.k_run != cfg[f][c][1];
            ch.seg_run = cfg[f][c][0];
            ch.k_run = cfg[f][c][1];
        }
    if (changed && h->graph_exec) {   // the captured launches used the old choices
        (void)hipGraphExecDestroy(h->graph_exec);
        (void)hipGraphDestroy(h->graph);
        h->graph_exec = nullptr;
        h->graph = nullptr;
    }
    h->itk = itk;
    h->tLB = tl;
    h->tLBp = tp;
    h->stopK = 0.0;
    h->stopUB = 0.0;
    double stop[2];
    QAP_HIP(hipMemcpy(stop, h->dStop, sizeof(stop), hipMemcpyDeviceToHost));
    h->stopK = stop[0];
    h->stopUB = stop[1];
    return QAP_OK;
}

void qap_rlt2_destroy(qap_rlt2* h) { destroy_handle(h); }

qap_status qap_rlt2_children(qap_rlt2* h, int k, int count, const int32_t* fac, const int32_t* loc, int level,
                             qap_rlt2** out)
{
    qap::last_error().clear();
    if (!out) return fail(QAP_EINVAL, "null output handle pointer");
    *out = nullptr;
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (k < 0 || k >= h->K) return fail(QAP_EINVAL, "instance index out of range");
    if (count < 1 || !fac || !loc) return fail(QAP_EINVAL, "need count >= 1 and fac, loc");
    if (level != 1 && level != 2) return fail(QAP_EINVAL, "level must be 1 or 2");
    if (level == 2 && h->level != 2) return fail(QAP_EINVAL, "level-2 children need a level-2 parent");
    const int N = h->inst[k].N;
    if (N - 1 < 3) return fail(QAP_EINVAL, "children need N - 1 >= 3");
    std::vector<int> fix(2 * count);
    for (int c = 0; c < count; ++c) {
        if (fac[c] < 0 || fac[c] >= N || loc[c] < 0 || loc[c] >= N)
            return fail(QAP_EINVAL, "fixed facility or location out of range");
        fix[2 * c] = fac[c];
        fix[2 * c + 1] = loc[c];
    }
    if ((st = flush_steps(h)) != QAP_OK) return st;
    qap_rlt2_opts o;
    qap_rlt2_default_opts(&o);
    o.precision = h->precision;
    o.device = h->device;
    o.stream = h->own_stream ? nullptr : h->stream;
    o.trace_level = h->trace_level;
    o.use_graph = h->use_graph;
    o.autotune = h->autotune;
    o.tune_cache = h->tune_cache.empty() ? nullptr : h->tune_cache.c_str();
    o.complementary = h->dmode == qap::kHalfStore ? 1 : 0;
    o.K = h->stopK;
    o.UB = h->stopUB;
    o.level = level;
    o.lap_solver = h->lap_solver;
    o.overlap = h->overlap ? 1 : 0;
    std::vector<int32_t> Ns(count, N - 1);
    qap_rlt2* c = nullptr;
    if ((st = make_handle(count, Ns.data(), o, &c)) != QAP_OK) return st;
    int* dfix = nullptr;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipMalloc(&dfix, fix.size() * sizeof(int));
    if (e == hipSuccess) e = hipMemcpyAsync(dfix, fix.data(), fix.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = QAP_OPS(c->precision, inherit(h, k, c, dfix));
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    std::vector<double> lb(2 * count);
    if (e == hipSuccess) e = hipMemcpy(lb.data(), c->dLB, lb.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (dfix) (void)hipFree(dfix);
    if (e != hipSuccess) {
        destroy_handle(c);
        return fail(e == hipErrorOutOfMemory ? QAP_ENOMEM : QAP_EDEVICE,
                    std::string("building the children: ") + hipGetErrorString(e));
    }
    // The inherited bound is each child's trace entry 0; the stop rule
    // applies to it as it does to iteration 0 of a new instance.
    std::vector<int> act(count, 1);
    for (int x = 0; x < count; ++x) {
        c->tLB[x].push_back(lb[2 * x]);
        c->tLBp[x].push_back(0.0);
        if (c->stopUB > 0.0 && lb[2 * x] >= c->stopUB) act[x] = 0;
    }
    e = hipMemcpy(c->dAct, act.data(), count * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        destroy_handle(c);
        return fail(QAP_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    *out = c;
    return QAP_OK;
}

qap_status qap_rlt2_strong_branch(qap_rlt2* h, int k, int iters, double* bounds, int* kind, int* index)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (k < 0 || k >= h->K) return fail(QAP_EINVAL, "instance index out of range");
    if (iters < 0) return fail(QAP_EINVAL, "iters must be >= 0");
    const int N = h->inst[k].N;
    std::vector<int32_t> fac(N * N), loc(N * N);
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            fac[a * N + b] = a;
            loc[a * N + b] = b;
        }
    qap_rlt2* c = nullptr;
    // The evaluation runs without the stop rule: every child's bound is
    // wanted, also above the incumbent (its row or column may still win).
    const double K0 = h->stopK, UB0 = h->stopUB;
    h->stopK = 0.0;
    h->stopUB = 0.0;
    st = qap_rlt2_children(h, k, N * N, fac.data(), loc.data(), 1, &c);
    h->stopK = K0;
    h->stopUB = UB0;
    if (st != QAP_OK) return st;
    std::vector<double> lb(N * N), cert(N * N);
    st = qap_rlt2_ascend(c, iters, nullptr);
    if (st == QAP_OK)
        st = qap_rlt2_batch_bounds(c, lb.data(), h->precision == QAP_FP64 ? nullptr : cert.data());
    destroy_handle(c);
    if (st != QAP_OK) return st;
    const std::vector<double>& v = h->precision == QAP_FP64 ? lb : cert;
    if (bounds) std::copy(v.begin(), v.end(), bounds);
    int best_kind = 0, best_index = 0;
    double best_min = -std::numeric_limits<double>::infinity(), best_sum = -std::numeric_limits<double>::infinity();
    for (int kd = 0; kd < 2; ++kd)
        for (int x = 0; x < N; ++x) {
            double mn = std::numeric_limits<double>::infinity(), sm = 0.0;
            for (int y = 0; y < N; ++y) {
                const double b = kd == 0 ? v[x * N + y] : v[y * N + x];
                mn = std::min(mn, b);
                sm += b;
            }
            if (mn > best_min || (mn == best_min && sm > best_sum)) {
                best_min = mn;
                best_sum = sm;
                best_kind = kd;
                best_index = x;
            }
        }
    if (kind) *kind = best_kind;
    if (index) *index = best_index;
    return QAP_OK;
}

qap_status qap_subproblem(int N, const double* F, const double* D, int m, const int32_t* fac, const int32_t* loc,
                          double* Fsub, double* Dsub, double* B0sub, double* constant)
{
    qap::last_error().clear();
    if (N < 1 || N > 4096) return fail(QAP_EINVAL, "N out of range");
    if (m < 0 || m > N) return fail(QAP_EINVAL, "m out of range");
    if (!F || !D || (m > 0 && (!fac || !loc)) || !Fsub || !Dsub || !B0sub || !constant)
        return fail(QAP_EINVAL, "null argument");
    std::vector<char> fixf(N, 0), fixl(N, 0);
    for (int t = 0; t < m; ++t) {
        if (fac[t] < 0 || fac[t] >= N || loc[t] < 0 || loc[t] >= N) return fail(QAP_EINVAL, "index out of range");
        if (fixf[fac[t]] || fixl[loc[t]]) return fail(QAP_EINVAL, "repeated facility or location");
        fixf[fac[t]] = 1;
        fixl[loc[t]] = 1;
    }
    std::vector<int> fr, lr;
    for (int i = 0; i < N; ++i) {
        if (!fixf[i]) fr.push_back(i);
        if (!fixl[i]) lr.push_back(i);
    }
    const int M = N - m;
    for (int a = 0; a < M; ++a)
        for (int b = 0; b < M; ++b) {
            Fsub[a * M + b] = F[fr[a] * N + fr[b]];
            Dsub[a * M + b] = D[lr[a] * N + lr[b]];
        }
    // Linear cost of free facility fr[a] at free location lr[b]: its flows to
    // and from every fixed facility times the matching distances.
    for (int a = 0; a < M; ++a)
        for (int b = 0; b < M; ++b) {
            double s = 0.0;
            const int i = fr[a], j = lr[b];
            for (int t = 0; t < m; ++t) {
                s += F[i * N + fac[t]] * D[j * N + loc[t]];
                s += F[fac[t] * N + i] * D[loc[t] * N + j];
            }
            B0sub[a * M + b] = s;
        }
    // Cost among the fixed facilities themselves (diagonal terms included).
    double c = 0.0;
    for (int t = 0; t < m; ++t)
        for (int u = 0; u < m; ++u) c += F[fac[t] * N + fac[u]] * D[loc[t] * N + loc[u]];
    *constant = c;
    return QAP_OK;
}

const char* qap_last_error(void) { return qap::last_error().c_str(); }

}  // extern "C"
