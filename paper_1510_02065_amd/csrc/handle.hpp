// Internal host-side state of a qap_rlt2 handle, shared by the C ABI
// (api.hip) and the per-precision launch code (ops_*.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "inherit_kernels.hpp"
#include "qap_rlt2.h"

namespace qap {

// Thread-local message of the last failure (qap_last_error).
std::string& last_error();

inline qap_status fail(qap_status st, const std::string& msg)
{
    last_error() = msg;
    return st;
}

#define QAP_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::qap::fail(QAP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline int seg_for(int n)
{
    if (n <= 8) return 8;
    if (n <= 16) return 16;
    if (n <= 32) return 32;
    return 64;
}

inline unsigned grid_for(long long work, int threads) { return (unsigned)((work + threads - 1) / threads); }

// Per-instance trace entries kept on the device between host reads.
constexpr long long kTraceCap = 1024;

// (lanes per problem, columns per lane) configurations of the concentration
// kernels; for a problem size n the candidates are (SEG, ceil(n/SEG)).
inline bool slot_cfg_allowed(int seg, int k)
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
size_t slot_lds(int nmax) { return (size_t)(64 / SEG) * SlotLds<T, SEG, K>::bytes(nmax); }

// LDS of a one-wave workgroup of the (seg, k) configuration at size nmax.
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

inline size_t slot_lds_prec(int precision, int seg, int k, int nmax)
{
    return precision == kPrecF64 ? slot_lds_any<double>(seg, k, nmax) : slot_lds_any<float>(seg, k, nmax);
}

// Instances of one family that share a segment size.
struct ClassHost {
    int seg = 0;       // size bucket: next power of two >= n (8 at least)
    int seg_run = 0;   // lanes per problem, chosen by the tuner
    int k_run = 0;     // columns per lane (seg_run * k_run >= nmax)
    int nmax = 0;
    std::vector<int> ids;
    std::vector<long long> pre;
    long long total = 0;
    int* d_ids = nullptr;
    long long* d_pre = nullptr;
    FamilyClass dev() const { return FamilyClass{d_ids, d_pre, (int)ids.size(), total}; }
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
    int* d_ids = nullptr;
    long long* d_pre = nullptr;
};

}  // namespace qap

struct qap_rlt2 {
    int K = 0;
    int precision = QAP_FP64;
    int level = 2;                 // 2: RLT2 (B, C, D); 1: RLT1 (B, C only)
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int trace_level = 1;
    int use_graph = 1;
    int autotune = 1;
    int lap_solver = QAP_LAP_SOLVER_CANONICAL;   // qap_lap_solver of the concentrations
    long long pending = 0;   // iterations of qap_rlt2_step whose trace entries are still on the device
    int dmode = qap::kHalfStore;   // D storage and enumeration (kAllBlocks or kHalfStore)
    int Nmax = 0;                  // largest instance
    int sweep_kind = 0;            // steps 1-3: 0 k_sweep, 1 k_sweep_cube, 2 k_sweep_triple
    bool tuned = false;
    size_t lds_limit = 65536;   // dynamic LDS a workgroup may request
    int num_cu = 256;           // compute units of the device
    std::string tune_cache;
    size_t elem = 8;   // bytes per reduced cost
    double stopK = 0.0, stopUB = 0.0;   // stop rule of Algorithm 1 (UB <= 0: off)
    std::vector<qap::Inst> inst;
    long long totalB = 0, totalC = 0, totalD = 0, totalWG = 0;
    std::vector<long long> preB, preC, preWG;
    qap::ClassHost fam[3][4];   // [D, C, B][segment class]
    std::vector<qap::SweepClass> sweep_cls;   // empty: one sweep launch over every instance
    int sweep_nt = 0;                         // that launch: threads of a per-triple workgroup (0: persistent)
    // Overlapped steps 1-4 of a batch of mixed sizes (qap_rlt2_ascend): the
    // sweep of each size runs on `stream`, and the D->C concentration of that
    // size on `stream2` as soon as its sweep is done, so one size's
    // assignment problems run beside the next size's sweep.
    bool overlap = false;
    hipStream_t stream2 = nullptr;
    std::vector<qap::ClassHost> famD_size;    // D family of each sweep class's instances (same order)
    std::vector<hipEvent_t> ev_size;          // one per sweep class: its sweep is done
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::vector<int> tri;                     // facility triples of every instance
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
    int* dAct = nullptr;        // per-instance flag: the dual ascent still runs
    double* dStop = nullptr;    // (K, UB) of the stop rule
    int32_t* dSigma = nullptr;  // assignment of the last B problem (packed like B)
    double* dCt = nullptr;      // certification: c~ (packed like C), allocated by the first certification
    double* dBt = nullptr;      // certification: b~ (packed like B)
    double* dCert = nullptr;    // certification result per instance
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<std::vector<double>> tLB, tLBp;
    std::vector<int64_t> itk;       // loop iterations each instance has run
    bool broken = false;
};

namespace qap {

// Launch code of one precision mode (ops_impl.hpp, instantiated in
// ops_f64.hip, ops_f32d.hip and ops_f32n.hip).
template <int PM>
struct Ops {
    // One step of an iteration: 3 (steps 1-3, or step 1 at level 1), 4, 5,
    // 6, 7 (steps 7-8).
    static hipError_t enqueue_step(qap_rlt2* h, int step);
    // Autotune family famk (kFamD or kFamC) on its live data.
    static hipError_t tune_family(qap_rlt2* h, int famk);
    // FP64 certification cascade into h->dCert.
    static hipError_t certify(qap_rlt2* h);
    // Initial dual of instance k from device copies of F, D and B0 (nullable).
    static hipError_t init_instance(qap_rlt2* h, int k, const double* dF, const double* dDm, const double* dB0);
    // Threads of a per-triple sweep workgroup at size N (0: persistent kernel).
    static int triple_threads(int N);
    // LDS of a per-triple sweep workgroup at size N ((size_t)-1: does not fit).
    static size_t sweep_lds(int N);
    // Batched assignment problems (qap_lap_solve) with `seg` lanes per
    // problem: slot s < count (count = *dcount if dcount is not null, the
    // grid sized for `count`) solves problem idx[s] (s if idx is null), by
    // the canonical dual or the auction (solver, a qap_lap_solver value).
    static hipError_t lap_batch(hipStream_t st, int seg, int count, const int* dcount, const int32_t* idx,
                                const int32_t* n, const int64_t* mo, const int64_t* vo, void* cost, double* value,
                                void* duals, int32_t* assign, int wr, int solver);
    // Children of parent instance pk of handle ph (fixings fix[2c], fix[2c+1]
    // in device memory) into handle ch, whose instances are those children.
    static hipError_t inherit(qap_rlt2* ph, int pk, qap_rlt2* ch, const int* dfix);
    // Steps 1-4 with each size's concentration overlapped with the next
    // size's sweep (h->overlap).
    static hipError_t enqueue_sweep_concentrate_overlapped(qap_rlt2* h);
};

extern template struct Ops<kPrecF64>;
extern template struct Ops<kPrecF32Down>;
extern template struct Ops<kPrecF32Near>;

// Dispatch to Ops<precision>.
#define QAP_OPS(prec, call)                                     \
    ((prec) == ::qap::kPrecF64       ? ::qap::Ops<::qap::kPrecF64>::call      \
     : (prec) == ::qap::kPrecF32Down ? ::qap::Ops<::qap::kPrecF32Down>::call  \
                                     : ::qap::Ops<::qap::kPrecF32Near>::call)

}  // namespace qap
