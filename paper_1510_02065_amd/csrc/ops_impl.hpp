// Launch code of one precision mode: the kernels of one dual-ascent iteration
// (Algorithm 1 of arXiv 1510.02065), the autotuner's timed runs, the
// certification cascade, the initial dual, the batched assignment solve and
// the children of a branch-and-bound node.  Included by ops_f64.hip,
// ops_f32d.hip and ops_f32n.hip, each of which instantiates Ops<PM> for one
// mode, so the three modes compile in parallel.
#pragma once
#include "handle.hpp"

namespace qap {

namespace {

template <int PM, int SEG, int K, bool AUC = false>
hipError_t launch_family_sk(qap_rlt2* h, int famk, const ClassHost& c, FamilyClass fc, double* values, int mode)
{
    using T = StoreT<PM>;
    if (fc.total <= 0) return hipSuccess;
    constexpr int LPW = 64 / SEG;
    const size_t lds = slot_lds<T, SEG, K>(c.nmax);
    if (lds > h->lds_limit) return hipErrorInvalidConfiguration;   // not launched
    const unsigned grid = (unsigned)((fc.total + LPW - 1) / LPW);
    T* D = static_cast<T*>(h->dD);
    T* C = static_cast<T*>(h->dC);
    T* B = static_cast<T*>(h->dB);
    if (famk == kFamD)
        hipLaunchKernelGGL((k_lap_family_s<PM, SEG, K, kFamD, AUC>), dim3(grid), dim3(64), lds, h->stream, D, C,
                           B, h->dInst, fc, c.nmax, values, mode, h->dAct);
    else
        hipLaunchKernelGGL((k_lap_family_s<PM, SEG, K, kFamC, AUC>), dim3(grid), dim3(64), lds, h->stream, D, C,
                           B, h->dInst, fc, c.nmax, values, kAllBlocks, h->dAct);
    return hipGetLastError();
}

template <int PM>
hipError_t launch_family_class(qap_rlt2* h, int famk, const ClassHost& c, FamilyClass fc, int seg, int k,
                               double* values, int mode)
{
#define QAP_CFG(SG, KK) \
    if (seg == SG && k == KK) return launch_family_sk<PM, SG, KK>(h, famk, c, fc, values, mode);
    QAP_CFG(8, 1) QAP_CFG(8, 2) QAP_CFG(8, 3) QAP_CFG(8, 4) QAP_CFG(8, 5) QAP_CFG(8, 6) QAP_CFG(8, 8)
    QAP_CFG(16, 1) QAP_CFG(16, 2) QAP_CFG(16, 3) QAP_CFG(16, 4) QAP_CFG(32, 1) QAP_CFG(32, 2) QAP_CFG(64, 1)
#undef QAP_CFG
    return hipErrorInvalidConfiguration;
}

// The auction solver's launch for a size class: one column per lane, in the
// class's own segment width.
template <int PM>
hipError_t launch_family_auction(qap_rlt2* h, int famk, const ClassHost& c, double* values, int mode)
{
    switch (c.seg) {
    case 8: return launch_family_sk<PM, 8, 1, true>(h, famk, c, c.dev(), values, mode);
    case 16: return launch_family_sk<PM, 16, 1, true>(h, famk, c, c.dev(), values, mode);
    case 32: return launch_family_sk<PM, 32, 1, true>(h, famk, c, c.dev(), values, mode);
    default: return launch_family_sk<PM, 64, 1, true>(h, famk, c, c.dev(), values, mode);
    }
}

template <int PM>
hipError_t launch_family(qap_rlt2* h, int famk, double* values)
{
    for (const ClassHost& c : h->fam[famk]) {
        if (c.total <= 0) continue;
        hipError_t e = h->lap_solver == QAP_LAP_SOLVER_AUCTION
                           ? launch_family_auction<PM>(h, famk, c, values, h->dmode)
                           : launch_family_class<PM>(h, famk, c, c.dev(), c.seg_run, c.k_run, values, h->dmode);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int PM, int SEG, int K, bool AUC = false>
hipError_t launch_B_sk(qap_rlt2* h, const ClassHost& c)
{
    using T = StoreT<PM>;
    constexpr int LPW = 64 / SEG;
    const size_t lds = slot_lds<T, SEG, K>(c.nmax);
    if (lds > h->lds_limit) return hipErrorInvalidConfiguration;
    const unsigned grid = (unsigned)((c.total + LPW - 1) / LPW);
    const bool tr = h->trace_level >= 1;
    hipLaunchKernelGGL((k_lap_B_s<PM, SEG, K, AUC>), dim3(grid), dim3(64), lds, h->stream, static_cast<T*>(h->dB),
                       h->dInst, c.dev(), c.nmax, h->dLB, tr ? h->dTrace : nullptr, h->dCounter, kTraceCap,
                       h->trace_level >= 2 ? h->dValB : nullptr, h->dSigma, h->dAct, h->dStop);
    return hipGetLastError();
}

template <int PM>
hipError_t launch_B(qap_rlt2* h)
{
    for (const ClassHost& c : h->fam[2]) {
        if (c.total <= 0) continue;
        hipError_t e = hipErrorInvalidConfiguration;
#define QAP_CFG(SG, KK) \
    else if (c.seg_run == SG && c.k_run == KK) e = launch_B_sk<PM, SG, KK>(h, c);
        if (h->lap_solver == QAP_LAP_SOLVER_AUCTION) {
            e = c.seg == 8    ? launch_B_sk<PM, 8, 1, true>(h, c)
                : c.seg == 16 ? launch_B_sk<PM, 16, 1, true>(h, c)
                : c.seg == 32 ? launch_B_sk<PM, 32, 1, true>(h, c)
                              : launch_B_sk<PM, 64, 1, true>(h, c);
        }
        QAP_CFG(8, 1) QAP_CFG(8, 2) QAP_CFG(8, 3) QAP_CFG(8, 4) QAP_CFG(8, 5) QAP_CFG(8, 6) QAP_CFG(8, 8)
        QAP_CFG(16, 1) QAP_CFG(16, 2) QAP_CFG(16, 3) QAP_CFG(16, 4) QAP_CFG(32, 1) QAP_CFG(32, 2) QAP_CFG(64, 1)
#undef QAP_CFG
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int PM, int SEG, bool AUC>
hipError_t launch_batch_seg(hipStream_t st, int count, const int* dcount, const int32_t* idx, const int32_t* n,
                            const int64_t* mo, const int64_t* vo, StoreT<PM>* cost, double* value,
                            StoreT<PM>* duals, int32_t* assign, int wr)
{
    using T = StoreT<PM>;
    if (count <= 0) return hipSuccess;
    constexpr int LPW = 64 / SEG;
    const size_t lds = LPW * SlotLds<T, SEG, 1>::bytes(SEG);
    const unsigned grid = (unsigned)((count + LPW - 1) / LPW);
    hipLaunchKernelGGL((k_lap_batch<PM, SEG, AUC>), dim3(grid), dim3(64), lds, st, count, dcount, idx, n, mo, vo, cost,
                       value, duals, assign, wr);
    return hipGetLastError();
}

// Workgroups of k_sweep_triple<PM, NT> a CU holds at size N (its registers
// and its LDS); 0 when the triple does not fit NT threads.
template <int PM, int NT>
int triple_per_cu(int N)
{
    const size_t lds = sweep_triple_lds<StoreT<PM>, NT>(N);
    if (lds == (size_t)-1) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sweep_triple<PM, NT>, NT, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

// Steps 1-3 over `ntri` triples of the instances ids[0..K) (all instances
// when ids is null), whose triples start at workgroups pre[0..K), laid out in
// LDS for size N.  When a CU holds only one triple's workgroup, one persistent
// workgroup per CU walks the triples and overlaps each triple's start with the
// previous one's tiles; when it holds two or more (nt > 0), one workgroup of
// nt threads per triple lets the hardware overlap them.  The workgroup that
// takes an instance's first triple clears its B.
template <int PM>
hipError_t launch_triple(qap_rlt2* h, const long long* pre, const int* ids, int K, long long ntri, int N, int nt)
{
    using T = StoreT<PM>;
    T* B = static_cast<T*>(h->dB);
    T* D = static_cast<T*>(h->dD);
    const T* CC = static_cast<const T*>(h->dCC);
    if (nt > 0) {
        if (nt == kTripleThreadsSmall) {
            const size_t lds = sweep_triple_lds<T, kTripleThreadsSmall>(N);
            if (lds == (size_t)-1) return hipErrorInvalidConfiguration;
            hipLaunchKernelGGL((k_sweep_triple<PM, kTripleThreadsSmall>), dim3((unsigned)ntri),
                               dim3(kTripleThreadsSmall), lds, h->stream, D, CC, B, h->dTri, h->dInst, pre, ids, K,
                               h->dAct);
        } else {
            const size_t lds = sweep_triple_lds<T>(N);
            hipLaunchKernelGGL((k_sweep_triple<PM, kTripleThreads>), dim3((unsigned)ntri), dim3(kTripleThreads), lds,
                               h->stream, D, CC, B, h->dTri, h->dInst, pre, ids, K, h->dAct);
        }
    } else {
        const size_t lds = sweep_triple_lds<T>(N);
        const long long grid = std::min<long long>(ntri, h->num_cu);
        hipLaunchKernelGGL((k_sweep_triple_p<PM>), dim3((unsigned)grid), dim3(kTripleThreads), lds, h->stream, D, CC,
                           B, h->dTri, h->dInst, pre, ids, K, ntri, N, h->dAct);
    }
    return hipGetLastError();
}

}  // namespace

template <int PM>
int Ops<PM>::triple_threads(int N)
{
    // The smaller workgroup when a CU holds two or more of them, else the larger
    // one when a CU holds two or more, else 0 (persistent).  Smaller
    // workgroups keep more triples in flight per CU, each waiting at its own
    // barriers: on the 256-node batch in certified FP32 the 512-thread sweeps
    // took 5.7 ms per iteration where the 1024-thread ones, holding more
    // waves, took 8.7 ms.
    if (triple_per_cu<PM, kTripleThreadsSmall>(N) >= 2) return kTripleThreadsSmall;
    if (triple_per_cu<PM, kTripleThreads>(N) >= 2) return kTripleThreads;
    return 0;
}

template <int PM>
size_t Ops<PM>::sweep_lds(int N)
{
    return sweep_triple_lds<StoreT<PM>>(N);
}

template <int PM>
hipError_t Ops<PM>::enqueue_step(qap_rlt2* h, int step)
{
    using T = StoreT<PM>;
    T* B = static_cast<T*>(h->dB);
    T* C = static_cast<T*>(h->dC);
    T* D = static_cast<T*>(h->dD);
    T* CC = static_cast<T*>(h->dCC);
    hipStream_t st = h->stream;
    const bool vals = h->trace_level >= 2;
    switch (step) {
    case 3: {   // steps 1-3 (level 1: step 1)
        if (h->level == 1) {
            hipLaunchKernelGGL((k_spread_B<PM>), dim3(grid_for(h->totalC, 256)), dim3(256), 0, st, C, B, h->dInst,
                               h->dPreC, h->K, h->totalC, h->dAct);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_clear_B<PM>), dim3(grid_for(h->totalB, 256)), dim3(256), 0, st, B, h->dPreB, h->K,
                               h->totalB, h->dAct);
            return hipGetLastError();
        }
        hipLaunchKernelGGL((k_spread_prep<PM>), dim3(grid_for(h->totalC, 256)), dim3(256), 0, st, C, B, CC,
                           h->dInst, h->dPreC, h->K, h->totalC, h->dAct);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (h->dmode == kAllBlocks) {
            hipLaunchKernelGGL((k_sweep<PM>), dim3((unsigned)h->totalWG), dim3(256), 0, st, D, CC, B, h->dTri,
                               h->dInst, h->dPreWG, h->K, h->dAct);
            return hipGetLastError();
        }
        if (h->sweep_kind == 2) {
            if (h->sweep_cls.empty())
                return launch_triple<PM>(h, h->dPreWG, nullptr, h->K, h->totalWG, h->Nmax, h->sweep_nt);
            for (const SweepClass& c : h->sweep_cls) {
                e = launch_triple<PM>(h, c.d_pre, c.d_ids, (int)c.ids.size(), c.ntri, c.N, c.nt);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        }
        const size_t lds = (size_t)6 * h->Nmax * h->Nmax * sizeof(T);
        if (lds <= h->lds_limit)
            hipLaunchKernelGGL((k_sweep_cube<PM, true>), dim3((unsigned)h->totalWG), dim3(256), lds, st, D, CC, B,
                               h->dTri, h->dInst, h->dPreWG, h->K, h->Nmax, h->dAct);
        else
            hipLaunchKernelGGL((k_sweep_cube<PM, false>), dim3((unsigned)h->totalWG), dim3(256), 0, st, D, CC, B,
                               h->dTri, h->dInst, h->dPreWG, h->K, h->Nmax, h->dAct);
        return hipGetLastError();
    }
    case 4:
        if (h->level == 1) return hipSuccess;
        return launch_family<PM>(h, kFamD, vals ? h->dValD : nullptr);
    case 5:
        hipLaunchKernelGGL((k_transfer_C<PM>), dim3(grid_for(h->totalC, 256)), dim3(256), 0, st, C, h->dInst,
                           h->dPreC, h->K, h->totalC, h->dAct);
        return hipGetLastError();
    case 6:
        return launch_family<PM>(h, kFamC, vals ? h->dValC : nullptr);
    case 7:
        return launch_B<PM>(h);
    default:
        return hipErrorInvalidValue;
    }
}

template <int PM>
hipError_t Ops<PM>::enqueue_sweep_concentrate_overlapped(qap_rlt2* h)
{
    using T = StoreT<PM>;
    hipStream_t A = h->stream, Bs = h->stream2;
    hipLaunchKernelGGL((k_spread_prep<PM>), dim3(grid_for(h->totalC, 256)), dim3(256), 0, A, static_cast<T*>(h->dC),
                       static_cast<T*>(h->dB), static_cast<T*>(h->dCC), h->dInst, h->dPreC, h->K, h->totalC,
                       h->dAct);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(h->ev_fork, A)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(Bs, h->ev_fork, 0)) != hipSuccess) return e;
    for (size_t i = 0; i < h->sweep_cls.size() && e == hipSuccess; ++i) {
        const SweepClass& c = h->sweep_cls[i];
        e = launch_triple<PM>(h, c.d_pre, c.d_ids, (int)c.ids.size(), c.ntri, c.N, c.nt);
        if (e == hipSuccess) e = hipEventRecord(h->ev_size[i], A);
        if (e == hipSuccess) e = hipStreamWaitEvent(Bs, h->ev_size[i], 0);
        if (e != hipSuccess) break;
        // The concentration of this size, on the second stream, with the
        // configuration tuned for its segment-size class.
        const ClassHost& d = h->famD_size[i];
        const ClassHost& bucket = h->fam[kFamD][d.seg == 8 ? 0 : d.seg == 16 ? 1 : d.seg == 32 ? 2 : 3];
        double* vals = h->trace_level >= 2 ? h->dValD : nullptr;
        h->stream = Bs;
        e = h->lap_solver == QAP_LAP_SOLVER_AUCTION
                ? launch_family_auction<PM>(h, kFamD, d, vals, h->dmode)
                : launch_family_class<PM>(h, kFamD, d, d.dev(), bucket.seg_run, bucket.k_run, vals, h->dmode);
        h->stream = A;
    }
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(h->ev_join, Bs)) != hipSuccess) return e;
    return hipStreamWaitEvent(A, h->ev_join, 0);
}

template <int PM>
hipError_t Ops<PM>::certify(qap_rlt2* h)
{
    using T = StoreT<PM>;
    hipStream_t st = h->stream;
    if (h->level == 1)
        hipLaunchKernelGGL((k_cert_noD<T>), dim3(grid_for(h->totalC, 256)), dim3(256), 0, st,
                           static_cast<const T*>(h->dC), h->dCt, h->totalC);
    else if (h->dmode == kAllBlocks)
        hipLaunchKernelGGL((k_cert_D<T, false>), dim3(grid_for(h->totalC, 4)), dim3(256), 0, st,
                           static_cast<const T*>(h->dD), static_cast<const T*>(h->dC), h->dCt, h->dInst, h->dPreC,
                           h->K, h->totalC);
    else
        hipLaunchKernelGGL((k_cert_D<T, true>), dim3(grid_for(h->totalC / 2, 4)), dim3(256), 0, st,
                           static_cast<const T*>(h->dD), static_cast<const T*>(h->dC), h->dCt, h->dInst, h->dPreC,
                           h->K, h->totalC);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_cert_C<T>), dim3(grid_for(h->totalB, 4)), dim3(256), 0, st, h->dCt,
                       static_cast<const T*>(h->dB), h->dBt, h->dInst, h->dPreB, h->K, h->totalB);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cert_final<>, dim3(h->K), dim3(64), 0, st, h->dBt, h->dLB, h->dCert, h->dInst);
    return hipGetLastError();
}

template <int PM>
hipError_t Ops<PM>::init_instance(qap_rlt2* h, int k, const double* dF, const double* dDm, const double* dB0)
{
    using T = StoreT<PM>;
    const Inst& I = h->inst[k];
    const int N = I.N;
    const long long nC = (long long)N * N * (N - 1) * (N - 1);
    hipLaunchKernelGGL((k_init<PM>), dim3(grid_for(nC, 256)), dim3(256), 0, h->stream, dF, dDm, dB0,
                       static_cast<T*>(h->dB) + I.offB, static_cast<T*>(h->dC) + I.offC, N);
    return hipGetLastError();
}

template <int PM>
hipError_t Ops<PM>::lap_batch(hipStream_t st, int seg, int count, const int* dcount, const int32_t* idx,
                              const int32_t* n, const int64_t* mo, const int64_t* vo, void* cost, double* value,
                              void* duals, int32_t* assign, int wr, int solver)
{
    using T = StoreT<PM>;
    T* c = static_cast<T*>(cost);
    T* d = static_cast<T*>(duals);
#define QAP_SEG(SG)                                                                                            \
    return solver == QAP_LAP_SOLVER_AUCTION                                                                    \
               ? launch_batch_seg<PM, SG, true>(st, count, dcount, idx, n, mo, vo, c, value, d, assign, wr)  \
               : launch_batch_seg<PM, SG, false>(st, count, dcount, idx, n, mo, vo, c, value, d, assign, wr)
    switch (seg) {
    case 8: QAP_SEG(8);
    case 16: QAP_SEG(16);
    case 32: QAP_SEG(32);
    default: QAP_SEG(64);
    }
#undef QAP_SEG
}

template <int PM>
hipError_t Ops<PM>::inherit(qap_rlt2* ph, int pk, qap_rlt2* ch, const int* dfix)
{
    using T = StoreT<PM>;
    const Inst& P = ph->inst[pk];
    ChildSrc<T> src;
    src.B = static_cast<const T*>(ph->dB) + P.offB;
    src.C = static_cast<const T*>(ph->dC) + P.offC;
    src.D = ph->level == 2 ? static_cast<const T*>(ph->dD) + P.offD : nullptr;
    src.lb = ph->dLB + 2 * pk;
    src.N = P.N;
    src.mode = ph->dmode;
    src.ldD = P.ldD;
    src.fix = dfix;
    const int K = ch->K, M = P.N - 1;
    hipStream_t st = ch->stream;
    hipLaunchKernelGGL((k_child_B<PM>), dim3(grid_for((long long)K * M * M, 256)), dim3(256), 0, st, src,
                       static_cast<T*>(ch->dB), ch->dLB, ch->dInst, K);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long perC = (long long)M * M * (M - 1) * (M - 1);
    hipLaunchKernelGGL((k_child_C<PM>), dim3(grid_for(K * perC, 256)), dim3(256), 0, st, src,
                       static_cast<T*>(ch->dC), ch->dInst, K);
    e = hipGetLastError();
    if (e != hipSuccess || ch->level == 1) return e;
    const Inst& I0 = ch->inst[0];
    const long long perD = ch->dmode == kAllBlocks ? perC * I0.ldD : (perC / 2) * (M - 2) * (M - 2);
    // Children of one size are packed with 128-byte aligned starts; the kernel
    // indexes each child's entries from its own offD.
    hipLaunchKernelGGL((k_child_D<PM>), dim3(grid_for(K * perD, 256)), dim3(256), 0, st, src,
                       static_cast<T*>(ch->dD), ch->dInst, K, perD, ch->dmode);
    return hipGetLastError();
}

// ---- autotuner ----------------------------------------------------------------
// For each class of a family, time every (lanes per problem, columns per
// lane) candidate on the first min(total, kTuneItems) problems of the class,
// each run starting from the same saved copy of the blocks and parents those
// problems touch, and keep the fastest.  The choice does not change the
// algorithm's decisions (ties go to the lowest column either way); it changes
// only the order of the final sums, by rounding.
constexpr long long kTuneItems = 16384;

template <int PM>
hipError_t Ops<PM>::tune_family(qap_rlt2* h, int famk)
{
    using T = StoreT<PM>;
    hipError_t e = hipSuccess;
    for (ClassHost& c : h->fam[famk]) {
        if (c.total <= 0) continue;
        const long long X = std::min(c.total, kTuneItems);
        // Element ranges touched by the first X problems: blocks and parents.
        int kk = 0;
        while (kk + 1 < (int)c.pre.size() && c.pre[kk + 1] <= X - 1) ++kk;
        const Inst& I0 = h->inst[c.ids[0]];
        const Inst& IL = h->inst[c.ids[kk]];
        const long long bl = X - 1 - c.pre[kk];
        long long blk0, blk1, par0, par1;
        char* blkbase;
        char* parbase;
        // Tuning runs on stored half blocks write only the parent c_beta, and
        // the parents of the first X half blocks lie at or below the last one's.
        const int mode = h->dmode == kAllBlocks ? kAllBlocks : kHalfStoreTune;
        if (famk == kFamD) {
            blk0 = I0.offD;
            par0 = I0.offC;
            if (mode == kAllBlocks) {
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
                    pair_block(IL.N, hb, &beta, &twin, &base);
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
        FamilyClass fc = c.dev();
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
                    (e = launch_family_class<PM>(h, famk, c, fc, seg, k, nullptr, mode)) != hipSuccess ||
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

}  // namespace qap
