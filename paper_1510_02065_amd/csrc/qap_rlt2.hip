// Host side of the qap_rlt2 library: handle state for one or many instances,
// the launch schedule of one dual-ascent iteration (Algorithm 1 of
// arXiv 1510.02065), HIP-graph replay, and the C ABI of include/qap_rlt2.h.
#include "qap_rlt2.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
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

inline unsigned grid_for(long long work, int threads) { return (unsigned)((work + threads - 1) / threads); }

constexpr long long kTraceCap = 1024;

// Instances of one family that share a segment size.
struct ClassHost {
    int seg = 0;       // size bucket: next power of two >= n (8 at least)
    int seg_run = 0;   // lanes per problem, chosen by the tuner
    int k_run = 0;     // columns per lane (seg_run * k_run >= nmax)
    int wpb = 1;
    int nmax = 0;
    std::vector<int> ids;
    std::vector<long long> pre;
    long long total = 0;
    int* d_ids = nullptr;
    long long* d_pre = nullptr;
    qap::FamilyClass dev() const { return qap::FamilyClass{d_ids, d_pre, (int)ids.size(), total}; }
};

// Instances of one size in a batch: the per-triple cost sweep of steps 1-3
// runs one launch per size, with the workgroup width and LDS for that size,
// so a CU holds as many of the small instances' workgroups as fit.
struct SweepClass {
    int N = 0;
    std::vector<int> ids;          // instances of this size
    std::vector<long long> pre;    // first workgroup (triple) of each, within the launch
    long long ntri = 0;            // triples of the launch
    int nt = 0;                    // threads of a per-triple workgroup (0: persistent kernel)
    bool zero_b = false;           // this launch also clears B
    int* d_ids = nullptr;
    long long* d_pre = nullptr;
};

}  // namespace

// ============================================================================
// Handle
// ============================================================================

struct qap_rlt2 {
    int K = 0;
    int precision = QAP_FP64;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int trace_level = 1;
    int use_graph = 1;
    int autotune = 1;
    long long pending = 0;   // iterations of qap_rlt2_step whose trace entries are still on the device
    int dmode = qap::kHalfStore;   // D storage and enumeration (kAllBlocks or kHalfStore)
    int Nmax = 0;                  // largest instance
    int sweep_kind = 0;            // steps 1-3: 0 k_sweep, 1 k_sweep_cube, 2 k_sweep_triple
    bool tuned = false;
    size_t lds_limit = 65536;   // dynamic LDS a workgroup may request
    int num_cu = 256;           // compute units of the device
    std::string tune_cache;
    size_t elem = 8;   // bytes per reduced cost
    std::vector<qap::Inst> inst;
    long long totalB = 0, totalC = 0, totalD = 0, totalWG = 0;
    std::vector<long long> preB, preC, preWG;
    ClassHost fam[3][4];   // [D, C, B][segment class]
    std::vector<SweepClass> sweep_cls;   // empty: one sweep launch over every instance
    int sweep_nt = 0;                    // that launch: threads of a per-triple workgroup (0: persistent)
    qap::Inst* dInst = nullptr;
    long long *dPreB = nullptr, *dPreC = nullptr, *dPreWG = nullptr;
    void* dB = nullptr;
    void* dC = nullptr;
    void* dD = nullptr;
    void* dCC = nullptr;
    double* dLB = nullptr;      // [LB, LB'] per instance
    double* dValD = nullptr;    // per-block values of the last step 4 (packed like C)
    double* dValC = nullptr;    // per-block values of the last step 6 (packed like B)
    double* dValB = nullptr;    // per-instance value of the last step 7
    double* dTrace = nullptr;   // K x kTraceCap x (LB, LB')
    long long* dCounter = nullptr;
    int* dTri = nullptr;
    double* dCt = nullptr;      // certification: c~ (packed like C)
    double* dBt = nullptr;      // certification: b~ (packed like B)
    double* dCert = nullptr;    // certification result per instance
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<std::vector<double>> tLB, tLBp;
    int64_t iterations = 0;
    bool broken = false;
};

namespace {

// ---- launches ---------------------------------------------------------------

hipError_t enqueue_step_any(qap_rlt2* h, int step);

// (lanes per problem, columns per lane) configurations of the concentration
// kernels; for a problem size n the candidates are (SEG, ceil(n/SEG)).
bool slot_cfg_allowed(int seg, int k)
{
    switch (seg) {
    case 8: return (k >= 1 && k <= 6) || k == 8;
    case 16: return k >= 1 && k <= 4;
    case 32: return k >= 1 && k <= 2;
    case 64: return k == 1;
    default: return false;
    }
}

template <typename T, int SEG, int K>
size_t slot_lds(int nmax) { return (size_t)(64 / SEG) * qap::SlotLds<T, SEG, K>::bytes(nmax); }

template <typename T>
size_t slot_lds_any(int seg, int k, int nmax)
{
#define QAP_CFG(SG, KK) \
    if (seg == SG && k == KK) return slot_lds<T, SG, KK>(nmax);
    QAP_CFG(8, 1) QAP_CFG(8, 2) QAP_CFG(8, 3) QAP_CFG(8, 4) QAP_CFG(8, 5) QAP_CFG(8, 6) QAP_CFG(8, 8)
    QAP_CFG(16, 1) QAP_CFG(16, 2) QAP_CFG(16, 3) QAP_CFG(16, 4) QAP_CFG(32, 1) QAP_CFG(32, 2) QAP_CFG(64, 1)
#undef QAP_CFG
    return (size_t)-1;
}

template <typename T, int SEG, int K>
hipError_t launch_family_sk(qap_rlt2* h, int famk, const ClassHost& c, qap::FamilyClass fc, double* values,
                            int mode)
{
    if (fc.total <= 0) return hipSuccess;
    constexpr int LPW = 64 / SEG;
    const size_t lds = slot_lds<T, SEG, K>(c.nmax);
    if (lds > h->lds_limit) return hipErrorInvalidConfiguration;   // not launched
    const unsigned grid = (unsigned)((fc.total + LPW - 1) / LPW);
    T* D = static_cast<T*>(h->dD);
    T* C = static_cast<T*>(h->dC);
    T* B = static_cast<T*>(h->dB);
    if (famk == qap::kFamD)
        hipLaunchKernelGGL((qap::k_lap_family_s<T, SEG, K, qap::kFamD>), dim3(grid), dim3(64), lds, h->stream, D, C,
                           B, h->dInst, fc, c.nmax, values, mode);
    else
        hipLaunchKernelGGL((qap::k_lap_family_s<T, SEG, K, qap::kFamC>), dim3(grid), dim3(64), lds, h->stream, D, C,
                           B, h->dInst, fc, c.nmax, values, qap::kAllBlocks);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_family_class(qap_rlt2* h, int famk, const ClassHost& c, qap::FamilyClass fc, int seg, int k,
                               double* values, int mode)
{
#define QAP_CFG(SG, KK) \
    if (seg == SG && k == KK) return launch_family_sk<T, SG, KK>(h, famk, c, fc, values, mode);
    QAP_CFG(8, 1) QAP_CFG(8, 2) QAP_CFG(8, 3) QAP_CFG(8, 4) QAP_CFG(8, 5) QAP_CFG(8, 6) QAP_CFG(8, 8)
    QAP_CFG(16, 1) QAP_CFG(16, 2) QAP_CFG(16, 3) QAP_CFG(16, 4) QAP_CFG(32, 1) QAP_CFG(32, 2) QAP_CFG(64, 1)
#undef QAP_CFG
    return hipErrorInvalidConfiguration;
}

template <typename T>
hipError_t launch_family(qap_rlt2* h, int famk, double* values)
{
    for (const ClassHost& c : h->fam[famk]) {
        if (c.total <= 0) continue;
        hipError_t e = launch_family_class<T>(h, famk, c, c.dev(), c.seg_run, c.k_run, values, h->dmode);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---- autotuner ----------------------------------------------------------------
// For each class of a family, time every (lanes per problem, columns per
// lane) candidate on the first min(total, kTuneItems) problems of the class,
// each run starting from the same saved copy of the blocks and parents those
// problems touch, and keep the fastest.  The choice does not change the
// algorithm's decisions (ties go to the lowest column either way); it changes
// only the order of the final sums, by rounding.
constexpr long long kTuneItems = 16384;

std::string tune_key(const qap_rlt2* h, int famk, const ClassHost& c)
{
    char buf[128];
    snprintf(buf, sizeof(buf), "gfx950 prec=%d fam=%d seg=%d nmax=%d", h->precision, famk, c.seg, c.nmax);
    return buf;
}

void load_tune_cache(qap_rlt2* h)
{
    if (h->tune_cache.empty()) return;
    FILE* f = fopen(h->tune_cache.c_str(), "r");
    if (!f) return;
    std::map<std::string, std::pair<int, int>> m;
    char line[256];
    while (fgets(line, sizeof(line), f)) {
        char* bar = strchr(line, '|');
        if (!bar) continue;
        *bar = 0;
        int seg = 0, wpb = 0;
        if (sscanf(bar + 1, "%d %d", &seg, &wpb) == 2) m[line] = {seg, wpb};
    }
    fclose(f);
    int hits = 0, need = 0;
    for (int famk = 0; famk < 2; ++famk)
        for (ClassHost& c : h->fam[famk]) {
            if (c.total <= 0) continue;
            ++need;
            auto it = m.find(tune_key(h, famk, c));
            if (it != m.end() && slot_cfg_allowed(it->second.first, it->second.second) &&
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
    std::map<std::string, std::pair<int, int>> m;
    if (FILE* f = fopen(h->tune_cache.c_str(), "r")) {
        char line[256];
        while (fgets(line, sizeof(line), f)) {
            char* bar = strchr(line, '|');
            if (!bar) continue;
            *bar = 0;
            int seg = 0, wpb = 0;
            if (sscanf(bar + 1, "%d %d", &seg, &wpb) == 2) m[line] = {seg, wpb};
        }
        fclose(f);
    }
    for (int famk = 0; famk < 2; ++famk)
        for (const ClassHost& c : h->fam[famk])
            if (c.total > 0) m[tune_key(h, famk, c)] = {c.seg_run, c.k_run};
    if (FILE* f = fopen(h->tune_cache.c_str(), "w")) {
        for (auto& kv : m) fprintf(f, "%s|%d %d\n", kv.first.c_str(), kv.second.first, kv.second.second);
        fclose(f);
    }
}

template <typename T>
hipError_t tune_family(qap_rlt2* h, int famk)
{
    hipError_t e = hipSuccess;
    for (ClassHost& c : h->fam[famk]) {
        if (c.total <= 0) continue;
        const long long X = std::min(c.total, kTuneItems);
        // Element ranges touched by the first X problems: blocks and parents.
        int kk = 0;
        while (kk + 1 < (int)c.pre.size() && c.pre[kk + 1] <= X - 1) ++kk;
        const qap::Inst& I0 = h->inst[c.ids[0]];
        const qap::Inst& IL = h->inst[c.ids[kk]];
        const long long bl = X - 1 - c.pre[kk];
        long long blk0, blk1, par0, par1;
        char* blkbase;
        char* parbase;
        // Tuning runs on stored half blocks write only the parent c_beta, and
        // the parents of the first X half blocks lie at or below the last one's.
        const int mode = h->dmode == qap::kAllBlocks ? qap::kAllBlocks : qap::kHalfStoreTune;
        if (famk == qap::kFamD) {
            blk0 = I0.offD;
            par0 = I0.offC;
            if (mode == qap::kAllBlocks) {
                blk1 = IL.offD + (bl + 1) * IL.ldD;
                par1 = IL.offC + bl + 1;
            } else {
                // Stored blocks 0..bl lie in the first bl / (N(N-1)) + 1 facility
                // pairs of the pair-major layout; their parents c_beta anywhere
                // below the largest beta among them.
                const long long NL = (long long)IL.N * (IL.N - 1), n2 = IL.N - 2;
                blk1 = IL.offD + (bl / NL + 1) * n2 * NL * n2;
                long long pmax = 0;
                for (long long hb = 0; hb <= bl; ++hb) {
                    long long beta = 0, twin = 0, base = 0;
                    qap::pair_block(IL.N, hb, &beta, &twin, &base);
                    pmax = std::max(pmax, beta);
                }
                par1 = IL.offC + pmax + 1;
            }
            blkbase = static_cast<char*>(h->dD);
            parbase = static_cast<char*>(h->dC);
        } else {
            blk0 = I0.offC;
            blk1 = IL.offC + (bl + 1) * (long long)(IL.N - 1) * (IL.N - 1);
            par0 = I0.offB;
            par1 = IL.offB + bl + 1;
            blkbase = static_cast<char*>(h->dC);
            parbase = static_cast<char*>(h->dB);
        }
        const size_t bbytes = (size_t)(blk1 - blk0) * h->elem, pbytes = (size_t)(par1 - par0) * h->elem;
        void* sblk = nullptr;
        void* spar = nullptr;
        if ((e = hipMalloc(&sblk, bbytes)) != hipSuccess) return e;
        if ((e = hipMalloc(&spar, pbytes)) != hipSuccess) {
            (void)hipFree(sblk);
            return e;
        }
        char* b0 = blkbase + blk0 * h->elem;
        char* p0 = parbase + par0 * h->elem;
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        auto cleanup = [&]() {
            if (ev0) (void)hipEventDestroy(ev0);
            if (ev1) (void)hipEventDestroy(ev1);
            (void)hipFree(sblk);
            (void)hipFree(spar);
        };
        if ((e = hipMemcpyAsync(sblk, b0, bbytes, hipMemcpyDeviceToDevice, h->stream)) != hipSuccess ||
            (e = hipMemcpyAsync(spar, p0, pbytes, hipMemcpyDeviceToDevice, h->stream)) != hipSuccess ||
            (e = hipEventCreate(&ev0)) != hipSuccess || (e = hipEventCreate(&ev1)) != hipSuccess) {
            cleanup();
            return e;
        }
        qap::FamilyClass fc = c.dev();
        fc.total = X;
        float best = 1e30f;
        int best_seg = c.seg_run, best_k = c.k_run;
        for (int seg : {8, 16, 32, 64}) {
            const int k = (c.nmax + seg - 1) / seg;
            if (!slot_cfg_allowed(seg, k)) continue;
            if (slot_lds_any<T>(seg, k, c.nmax) > h->lds_limit) continue;
            float ms = 0.f;
            for (int rep = 0; rep < 2; ++rep) {
                if ((e = hipMemcpyAsync(b0, sblk, bbytes, hipMemcpyDeviceToDevice, h->stream)) != hipSuccess ||
                    (e = hipMemcpyAsync(p0, spar, pbytes, hipMemcpyDeviceToDevice, h->stream)) != hipSuccess ||
                    (e = hipEventRecord(ev0, h->stream)) != hipSuccess ||
                    (e = launch_family_class<T>(h, famk, c, fc, seg, k, nullptr, mode)) != hipSuccess ||
                    (e = hipEventRecord(ev1, h->stream)) != hipSuccess ||
                    (e = hipEventSynchronize(ev1)) != hipSuccess ||
                    (e = hipEventElapsedTime(&ms, ev0, ev1)) != hipSuccess) {
                    cleanup();
                    return e;
                }
            }
            if (ms < best) {
                best = ms;
                best_seg = seg;
                best_k = k;
            }
        }
        c.seg_run = best_seg;
        c.k_run = best_k;
        e = hipMemcpyAsync(b0, sblk, bbytes, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(p0, spar, pbytes, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        cleanup();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// First iteration of a handle with autotuning: run the steps one by one and
// tune each concentration family on its live data just before it runs.
hipError_t tuned_first_iteration(qap_rlt2* h)
{
    const bool f64 = h->precision == QAP_FP64;
    hipError_t e;
    if ((e = enqueue_step_any(h, 3)) != hipSuccess) return e;
    if ((e = f64 ? tune_family<double>(h, qap::kFamD) : tune_family<float>(h, qap::kFamD)) != hipSuccess) return e;
    if ((e = enqueue_step_any(h, 4)) != hipSuccess) return e;
    if ((e = enqueue_step_any(h, 5)) != hipSuccess) return e;
    if ((e = f64 ? tune_family<double>(h, qap::kFamC) : tune_family<float>(h, qap::kFamC)) != hipSuccess) return e;
    if ((e = enqueue_step_any(h, 6)) != hipSuccess) return e;
    if ((e = enqueue_step_any(h, 7)) != hipSuccess) return e;
    h->tuned = true;
    save_tune_cache(h);
    return hipSuccess;
}

template <typename T, int SEG, int K>
hipError_t launch_B_sk(qap_rlt2* h, const ClassHost& c)
{
    constexpr int LPW = 64 / SEG;
    const size_t lds = slot_lds<T, SEG, K>(c.nmax);
    if (lds > h->lds_limit) return hipErrorInvalidConfiguration;
    const unsigned grid = (unsigned)((c.total + LPW - 1) / LPW);
    const bool tr = h->trace_level >= 1;
    hipLaunchKernelGGL((qap::k_lap_B_s<T, SEG, K>), dim3(grid), dim3(64), lds, h->stream, static_cast<T*>(h->dB),
                       h->dInst, c.dev(), c.nmax, h->dLB, tr ? h->dTrace : nullptr, tr ? h->dCounter : nullptr,
                       kTraceCap, h->trace_level >= 2 ? h->dValB : nullptr);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_B(qap_rlt2* h)
{
    for (const ClassHost& c : h->fam[2]) {
        if (c.total <= 0) continue;
        hipError_t e = hipErrorInvalidConfiguration;
#define QAP_CFG(SG, KK) \
    else if (c.seg_run == SG && c.k_run == KK) e = launch_B_sk<T, SG, KK>(h, c);
        if (false) {
        }
        QAP_CFG(8, 1) QAP_CFG(8, 2) QAP_CFG(8, 3) QAP_CFG(8, 4) QAP_CFG(8, 5) QAP_CFG(8, 6) QAP_CFG(8, 8)
        QAP_CFG(16, 1) QAP_CFG(16, 2) QAP_CFG(16, 3) QAP_CFG(16, 4) QAP_CFG(32, 1) QAP_CFG(32, 2) QAP_CFG(64, 1)
#undef QAP_CFG
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, int SEG>
hipError_t launch_batch_seg(hipStream_t st, int batch, const int32_t* n, const int64_t* mo,
                            const int64_t* vo, T* cost, double* value, T* duals, int32_t* assign, int wr)
{
    if (batch <= 0) return hipSuccess;
    constexpr int LPW = 64 / SEG;
    const size_t lds = LPW * qap::SlotLds<T, SEG, 1>::bytes(SEG);
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

// Workgroups of k_sweep_triple<T, NT> a CU holds at size N (its registers
// and its LDS); 0 when the triple does not fit NT threads.
template <typename T, int NT>
int triple_per_cu(int N)
{
    const size_t lds = qap::sweep_triple_lds<T, NT>(N);
    if (lds == (size_t)-1) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, qap::k_sweep_triple<T, NT>, NT, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

// Threads of a per-triple workgroup for size N, or 0 for the persistent
// kernel (a CU holds one triple's workgroup at most): of the two workgroup
// sizes with two or more workgroups per CU, the one with more resident waves,
// the smaller on a tie.
template <typename T>
int triple_threads(int N)
{
    const int small = triple_per_cu<T, qap::kTripleThreadsSmall>(N);
    const int large = triple_per_cu<T, qap::kTripleThreads>(N);
    const long long ws = small >= 2 ? (long long)small * qap::kTripleThreadsSmall : 0;
    const long long wl = large >= 2 ? (long long)large * qap::kTripleThreads : 0;
    if (ws == 0 && wl == 0) return 0;
    return wl > ws ? qap::kTripleThreads : qap::kTripleThreadsSmall;
}

int triple_threads_any(const qap_rlt2* h, int N)
{
    return h->precision == QAP_FP64 ? triple_threads<double>(N) : triple_threads<float>(N);
}

// Steps 1-3 over `ntri` triples of the instances ids[0..K) (all instances
// when ids is null), whose triples start at workgroups pre[0..K), laid out in
// LDS for size N.  When a CU holds only one triple's workgroup, one persistent
// workgroup per CU walks the triples and overlaps each triple's start with the
// previous one's tiles; when it holds two or more (nt > 0), one workgroup of
// nt threads per triple lets the hardware overlap them.  The launch clears
// B[0..zeroB); a per-triple launch clears one entry per thread, so zeroB <=
// ntri * nt there.
template <typename T>
hipError_t launch_triple(qap_rlt2* h, const long long* pre, const int* ids, int K, long long ntri, int N, int nt,
                         long long zeroB)
{
    T* B = static_cast<T*>(h->dB);
    T* D = static_cast<T*>(h->dD);
    const T* CC = static_cast<const T*>(h->dCC);
    if (nt > 0) {
        if (zeroB > ntri * nt) return hipErrorInvalidConfiguration;
        if (nt == qap::kTripleThreadsSmall) {
            const size_t lds = qap::sweep_triple_lds<T, qap::kTripleThreadsSmall>(N);
            if (lds == (size_t)-1) return hipErrorInvalidConfiguration;
            hipLaunchKernelGGL((qap::k_sweep_triple<T, qap::kTripleThreadsSmall>), dim3((unsigned)ntri),
                               dim3(qap::kTripleThreadsSmall), lds, h->stream, D, CC, B, h->dTri, h->dInst, pre, ids,
                               K, zeroB);
        } else {
            const size_t lds = qap::sweep_triple_lds<T>(N);
            hipLaunchKernelGGL((qap::k_sweep_triple<T, qap::kTripleThreads>), dim3((unsigned)ntri),
                               dim3(qap::kTripleThreads), lds, h->stream, D, CC, B, h->dTri, h->dInst, pre, ids, K,
                               zeroB);
        }
    } else {
        const size_t lds = qap::sweep_triple_lds<T>(N);
        const long long grid = std::min<long long>(ntri, h->num_cu);
        hipLaunchKernelGGL((qap::k_sweep_triple_p<T>), dim3((unsigned)grid), dim3(qap::kTripleThreads), lds,
                           h->stream, D, CC, B, h->dTri, h->dInst, pre, ids, K, zeroB, ntri, N);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t enqueue_step(qap_rlt2* h, int step)
{
    T* B = static_cast<T*>(h->dB);
    T* C = static_cast<T*>(h->dC);
    T* D = static_cast<T*>(h->dD);
    T* CC = static_cast<T*>(h->dCC);
    hipStream_t st = h->stream;
    const bool vals = h->trace_level >= 2;
    switch (step) {
    case 3: {   // steps 1-3
        hipLaunchKernelGGL((qap::k_spread_prep<T>), dim3(grid_for(h->totalC, 256)), dim3(256), 0, st, C, B, CC,
                           h->dInst, h->dPreC, h->K, h->totalC);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (h->dmode == qap::kAllBlocks) {
            hipLaunchKernelGGL((qap::k_sweep<T>), dim3((unsigned)h->totalWG), dim3(256), 0, st, D, CC, B,
                               h->dTri, h->dInst, h->dPreWG, h->K, h->totalB);
            return hipGetLastError();
        }
        if (h->sweep_kind == 2) {
            if (h->sweep_cls.empty())
                return launch_triple<T>(h, h->dPreWG, nullptr, h->K, h->totalWG, h->Nmax, h->sweep_nt, h->totalB);
            for (const SweepClass& c : h->sweep_cls) {
                e = launch_triple<T>(h, c.d_pre, c.d_ids, (int)c.ids.size(), c.ntri, c.N, c.nt,
                                     c.zero_b ? h->totalB : 0);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        }
        const size_t lds = (size_t)6 * h->Nmax * h->Nmax * sizeof(T);
        if (lds <= h->lds_limit)
            hipLaunchKernelGGL((qap::k_sweep_cube<T, true>), dim3((unsigned)h->totalWG), dim3(256), lds, st, D, CC,
                               B, h->dTri, h->dInst, h->dPreWG, h->K, h->totalB, h->Nmax);
        else
            hipLaunchKernelGGL((qap::k_sweep_cube<T, false>), dim3((unsigned)h->totalWG), dim3(256), 0, st, D, CC,
                               B, h->dTri, h->dInst, h->dPreWG, h->K, h->totalB, h->Nmax);
        return hipGetLastError();
    }
    case 4:
        return launch_family<T>(h, qap::kFamD, vals ? h->dValD : nullptr);
    case 5:
        hipLaunchKernelGGL((qap::k_transfer_C<T>), dim3(grid_for(h->totalC, 256)), dim3(256), 0, st, C, h->dInst,
                           h->dPreC, h->K, h->totalC);
        return hipGetLastError();
    case 6:
        return launch_family<T>(h, qap::kFamC, vals ? h->dValC : nullptr);
    case 7:
        return launch_B<T>(h);
    default:
        return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t enqueue_certify(qap_rlt2* h)
{
    hipStream_t st = h->stream;
    if (h->dmode == qap::kAllBlocks)
        hipLaunchKernelGGL((qap::k_cert_D<T, false>), dim3(grid_for(h->totalC, 4)), dim3(256), 0, st,
                           static_cast<const T*>(h->dD), static_cast<const T*>(h->dC), h->dCt, h->dInst, h->dPreC,
                           h->K, h->totalC);
    else
        hipLaunchKernelGGL((qap::k_cert_D<T, true>), dim3(grid_for(h->totalC / 2, 4)), dim3(256), 0, st,
                           static_cast<const T*>(h->dD), static_cast<const T*>(h->dC), h->dCt, h->dInst, h->dPreC,
                           h->K, h->totalC);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((qap::k_cert_C<T>), dim3(grid_for(h->totalB, 4)), dim3(256), 0, st, h->dCt,
                       static_cast<const T*>(h->dB), h->dBt, h->dInst, h->dPreB, h->K, h->totalB);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(qap::k_cert_final, dim3(h->K), dim3(64), 0, st, h->dBt, h->dLB, h->dCert, h->dInst);
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

// Copy the trace entries written since the counters were last reset, then
// reset them.
qap_status drain_trace(qap_rlt2* h)
{
    std::vector<long long> cnt(h->K);
    QAP_HIP(hipMemcpyAsync(cnt.data(), h->dCounter, h->K * sizeof(long long), hipMemcpyDeviceToHost, h->stream));
    QAP_HIP(hipStreamSynchronize(h->stream));
    long long mx = 0;
    for (long long c : cnt) mx = std::max(mx, std::min(c, kTraceCap));
    if (mx > 0) {
        std::vector<double> buf((size_t)h->K * kTraceCap * 2);
        QAP_HIP(hipMemcpyAsync(buf.data(), h->dTrace, buf.size() * sizeof(double), hipMemcpyDeviceToHost,
                               h->stream));
        QAP_HIP(hipStreamSynchronize(h->stream));
        for (int k = 0; k < h->K; ++k) {
            const long long c = std::min(cnt[k], kTraceCap);
            for (long long t = 0; t < c; ++t) {
                h->tLB[k].push_back(buf[((size_t)k * kTraceCap + t) * 2]);
                h->tLBp[k].push_back(buf[((size_t)k * kTraceCap + t) * 2 + 1]);
            }
        }
    }
    QAP_HIP(hipMemsetAsync(h->dCounter, 0, h->K * sizeof(long long), h->stream));
    QAP_HIP(hipStreamSynchronize(h->stream));
    return QAP_OK;
}

void release(qap_rlt2* h)
{
    if (!h) return;
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    void* ptrs[] = {h->dB,     h->dC,     h->dD,     h->dCC,   h->dLB,       h->dValD, h->dValC,
                    h->dValB,  h->dTrace, h->dCounter, h->dTri, h->dCt,    h->dBt,   h->dCert,
                    h->dInst,  h->dPreB,  h->dPreC,  h->dPreWG};
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
    g_last_error.clear();
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
    if (o.precision != QAP_FP64 && o.precision != QAP_FP32_CERTIFIED)
        return fail(QAP_EINVAL, "unknown precision");

    qap_rlt2* h = new (std::nothrow) qap_rlt2();
    if (!h) return fail(QAP_ENOMEM, "host allocation failed");
    h->K = count;
    h->precision = o.precision;
    h->trace_level = std::max(0, std::min(2, o.trace_level));
    h->use_graph = o.use_graph ? 1 : 0;
    h->autotune = o.autotune ? 1 : 0;
    if (o.tune_cache) h->tune_cache = o.tune_cache;
    h->dmode = o.complementary ? qap::kHalfStore : qap::kAllBlocks;
    h->elem = o.precision == QAP_FP64 ? sizeof(double) : sizeof(float);
    h->tLB.resize(count);
    h->tLBp.resize(count);

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

    // LDS a workgroup may request.
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
    else {
        const size_t need = h->precision == QAP_FP64 ? qap::sweep_triple_lds<double>(h->Nmax)
                                                     : qap::sweep_triple_lds<float>(h->Nmax);
        h->sweep_kind = need <= h->lds_limit ? 2 : 1;
    }
    std::vector<int> tri;
    h->inst.resize(count);
    for (int k = 0; k < count; ++k) {
        const int N = Ns[k], n1 = N - 1, n2 = N - 2;
        qap::Inst& I = h->inst[k];
        I.N = N;
        I.ntri = N * (N - 1) * (N - 2) / 6;
        // sweep workgroups per facility triple: kSweepParts (one stored block
        // per pair), or one per 256 groups (every block)
        I.wpt = h->sweep_kind == 0 ? (N * n1 * n2 + 255) / 256 : h->sweep_kind == 1 ? qap::kSweepParts : 1;
        I.pad_ = 0;
        I.offB = h->totalB;
        I.offC = h->totalC;
        I.offD = h->totalD;
        I.ldD = ((long long)n2 * n2 + align_elems - 1) / align_elems * align_elems;
        I.wg0 = h->totalWG;
        I.tri0 = (long long)tri.size();
        for (int i = 0; i < N; ++i)
            for (int kk = i + 1; kk < N; ++kk)
                for (int p = kk + 1; p < N; ++p) {
                    tri.push_back(i);
                    tri.push_back(kk);
                    tri.push_back(p);
                }
        h->preB.push_back(h->totalB);
        h->preC.push_back(h->totalC);
        h->preWG.push_back(h->totalWG);
        const long long nC = (long long)N * N * n1 * n1;
        h->totalB += (long long)N * N;
        h->totalC += nC;
        if (h->dmode == qap::kAllBlocks)
            h->totalD += nC * I.ldD;
        else   // pair-major, one block per pair, unpadded; instances start 128-byte aligned
            h->totalD += ((nC / 2) * n2 * n2 + align_elems - 1) / align_elems * align_elems;
        h->totalWG += h->sweep_kind == 2 ? (long long)I.ntri : 8LL * ((I.ntri + 7) / 8) * I.wpt;
    }
    // One sweep launch per instance size when a batch mixes sizes; the launch
    // of the largest size that can clear B does so.
    if (h->sweep_kind == 2) {
        h->sweep_nt = triple_threads_any(h, h->Nmax);
        if (h->totalB > h->totalWG * h->sweep_nt) h->sweep_nt = 0;
        std::vector<int> sizes(Ns, Ns + count);
        std::sort(sizes.begin(), sizes.end(), std::greater<int>());
        sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
        if (sizes.size() > 1) {
            for (int N : sizes) {
                SweepClass c;
                c.N = N;
                c.nt = triple_threads_any(h, N);
                for (int k = 0; k < count; ++k)
                    if ((int)Ns[k] == N) {
                        c.ids.push_back(k);
                        c.pre.push_back(c.ntri);
                        c.ntri += h->inst[k].ntri;
                    }
                h->sweep_cls.push_back(std::move(c));
            }
            bool placed = false;
            for (SweepClass& c : h->sweep_cls) {
                if (c.nt == 0 || c.ntri * c.nt >= h->totalB) {
                    c.zero_b = placed = true;
                    break;
                }
            }
            if (!placed) h->sweep_cls.clear();
        }
    }
    // Segment-size classes of the three families.
    for (int f = 0; f < 3; ++f) {
        for (int k = 0; k < count; ++k) {
            const int N = Ns[k];
            const int n = (f == 0) ? N - 2 : (f == 1) ? N - 1 : N;
            const int seg = seg_for(n);
            const int ci = seg == 8 ? 0 : seg == 16 ? 1 : seg == 32 ? 2 : 3;
            ClassHost& c = h->fam[f][ci];
            c.seg = seg;
            c.nmax = std::max(c.nmax, n);
            c.ids.push_back(k);
            c.pre.push_back(c.total);
            const long long nblk = (long long)N * N * (N - 1) * (N - 1);
            c.total += (f == 0) ? (h->dmode == qap::kAllBlocks ? nblk : nblk / 2) : (f == 1) ? (long long)N * N : 1;
        }
    }

    // LDS a workgroup may request, and the default configuration of every
    // class: the most problems per wave that fit (families D and C).
    // The B family (one problem per instance) is latency-bound: one column per
    // lane, the smallest segment that holds the problem.
    for (ClassHost& c : h->fam[2]) {
        if (c.total <= 0) continue;
        const int seg = c.nmax <= 8 ? 8 : c.nmax <= 16 ? 16 : c.nmax <= 32 ? 32 : 64;
        const size_t need = h->precision == QAP_FP64 ? slot_lds_any<double>(seg, 1, c.nmax)
                                                     : slot_lds_any<float>(seg, 1, c.nmax);
        if (need <= h->lds_limit) {
            c.seg_run = seg;
            c.k_run = 1;
        }
    }
    for (auto& f : h->fam)
        for (ClassHost& c : f) {
            if (c.total <= 0 || c.seg_run != 0) continue;
            for (int seg : {8, 16, 32, 64}) {
                const int k = (c.nmax + seg - 1) / seg;
                if (!slot_cfg_allowed(seg, k)) continue;
                const size_t need = h->precision == QAP_FP64 ? slot_lds_any<double>(seg, k, c.nmax)
                                                             : slot_lds_any<float>(seg, k, c.nmax);
                if (need > h->lds_limit) continue;
                c.seg_run = seg;
                c.k_run = k;
                break;
            }
            if (c.seg_run == 0) return bail(fail(QAP_EINVAL, "problem size needs more LDS than a workgroup has"));
        }

    const size_t bytesD = (size_t)h->totalD * h->elem;
    size_t freeb = 0, totalb = 0;
    CK(hipMemGetInfo(&freeb, &totalb));
    if (bytesD + (size_t)h->totalC * (2 * h->elem + 8) > freeb)
        return bail(fail(QAP_ENOMEM, "reduced-cost arrays do not fit in free device memory"));

    CK(hipMalloc(&h->dB, h->totalB * h->elem));
    CK(hipMalloc(&h->dC, h->totalC * h->elem));
    CK(hipMalloc(&h->dCC, h->totalC * h->elem));
    CK(hipMalloc(&h->dD, bytesD));
    CK(hipMalloc(&h->dLB, 2 * count * sizeof(double)));
    CK(hipMalloc(&h->dTrace, 2 * kTraceCap * count * sizeof(double)));
    CK(hipMalloc(&h->dCounter, count * sizeof(long long)));
    CK(hipMalloc(&h->dCt, h->totalC * sizeof(double)));
    CK(hipMalloc(&h->dBt, h->totalB * sizeof(double)));
    CK(hipMalloc(&h->dCert, count * sizeof(double)));
    if (h->trace_level >= 2) {
        CK(hipMalloc(&h->dValD, h->totalC * sizeof(double)));
        CK(hipMalloc(&h->dValC, h->totalB * sizeof(double)));
        CK(hipMalloc(&h->dValB, count * sizeof(double)));
    }
    CK(upload(&h->dTri, tri, h->stream));
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
    if (h->autotune) load_tune_cache(h);
    std::vector<double> lb0(2 * count, 0.0);
    for (int k = 0; k < count; ++k) lb0[2 * k] = constants ? constants[k] : 0.0;
    CK(hipMemcpyAsync(h->dLB, lb0.data(), lb0.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
    CK(hipMemsetAsync(h->dCounter, 0, count * sizeof(long long), h->stream));
    CK(hipMemsetAsync(h->dD, 0, bytesD, h->stream));

    // Initial dual of every instance.
    int Nmax = 0;
    for (int k = 0; k < count; ++k) Nmax = std::max(Nmax, (int)Ns[k]);
    double* dF = nullptr;
    double* dDm = nullptr;
    double* dB0 = nullptr;
    CK(hipMalloc(&dF, (size_t)Nmax * Nmax * sizeof(double)));
    CK(hipMalloc(&dDm, (size_t)Nmax * Nmax * sizeof(double)));
    CK(hipMalloc(&dB0, (size_t)Nmax * Nmax * sizeof(double)));
    for (int k = 0; k < count; ++k) {
        const int N = Ns[k];
        const size_t nb = (size_t)N * N * sizeof(double);
        const double* B0 = B0s ? B0s[k] : nullptr;
        CK(hipMemcpyAsync(dF, Fs[k], nb, hipMemcpyHostToDevice, h->stream));
        CK(hipMemcpyAsync(dDm, Ds[k], nb, hipMemcpyHostToDevice, h->stream));
        if (B0) CK(hipMemcpyAsync(dB0, B0, nb, hipMemcpyHostToDevice, h->stream));
        const qap::Inst& I = h->inst[k];
        const long long nC = (long long)N * N * (N - 1) * (N - 1);
        if (h->precision == QAP_FP64)
            hipLaunchKernelGGL((qap::k_init<double>), dim3(grid_for(nC, 256)), dim3(256), 0, h->stream, dF, dDm,
                               B0 ? dB0 : nullptr, static_cast<double*>(h->dB) + I.offB,
                               static_cast<double*>(h->dC) + I.offC, N);
        else
            hipLaunchKernelGGL((qap::k_init<float>), dim3(grid_for(nC, 256)), dim3(256), 0, h->stream, dF, dDm,
                               B0 ? dB0 : nullptr, static_cast<float*>(h->dB) + I.offB,
                               static_cast<float*>(h->dC) + I.offC, N);
        CK(hipGetLastError());
        // The staging buffers are reused by the next instance.
        CK(hipStreamSynchronize(h->stream));
    }
    (void)hipFree(dF);
    (void)hipFree(dDm);
    (void)hipFree(dB0);
    // Iteration 0: C -> B, then B -> LB.
    CK(enqueue_step_any(h, 6));
    CK(enqueue_step_any(h, 7));
    CK(hipStreamSynchronize(h->stream));
    qap_status st = drain_trace(h);
    if (st != QAP_OK) return bail(st);
#undef CK
    *out = h;
    return QAP_OK;
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

qap_status qap_rlt2_ascend(qap_rlt2* h, int iters, double* bound)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (iters < 0) return fail(QAP_EINVAL, "iters must be >= 0");
    if ((st = flush_steps(h)) != QAP_OK) return st;
    int left = iters;
    if (left > 0 && h->autotune && !h->tuned) {
        hipError_t e = tuned_first_iteration(h);
        if (e != hipSuccess) return mark_broken(h, e, "autotuned first iteration");
        e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return mark_broken(h, e, "hipStreamSynchronize");
        h->iterations += 1;
        st = drain_trace(h);
        if (st != QAP_OK) {
            h->broken = true;
            return st;
        }
        --left;
    }
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
        h->iterations += 1;
        // The trace entry stays on the device until a call reads the trace
        // or the device buffer is full.
        if (++h->pending >= kTraceCap) return flush_steps(h);
    }
    return QAP_OK;
}

qap_status qap_rlt2_batch_bounds(qap_rlt2* h, double* lb, double* certified)
{
    qap_status st = check_handle(h);
    if (st != QAP_OK) return st;
    if (certified) {
        hipError_t e = h->precision == QAP_FP64 ? enqueue_certify<double>(h) : enqueue_certify<float>(h);
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
    if (lb) {
        double v[2];
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e == hipSuccess) e = hipMemcpy(v, h->dLB, sizeof(v), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return mark_broken(h, e, "hipMemcpy");
        *lb = v[0];
    }
    if (iterations) *iterations = h->iterations;
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
    const char* d = static_cast<const char*>(h->dD) + I.offD * h->elem;
    if (B) QAP_HIP(widen(B, b, (long long)N * N, (size_t)N * N * h->elem, 1));
    if (C) QAP_HIP(widen(C, c, nC, (size_t)nC * h->elem, 1));
    if (D) {
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

void qap_rlt2_destroy(qap_rlt2* h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    release(h);
    delete h;
}

qap_status qap_subproblem(int N, const double* F, const double* D, int m, const int32_t* fac, const int32_t* loc,
                          double* Fsub, double* Dsub, double* B0sub, double* constant)
{
    g_last_error.clear();
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
