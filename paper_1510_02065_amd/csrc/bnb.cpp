// Branch and bound of Section 6 of arXiv 1510.02065 on one GPU, and the
// upper-bound heuristic of Algorithm 1.  Host code over the library's public
// C ABI only: every node's dual ascent runs in the HIP kernels behind
// qap_rlt2_*.
//
// Search: depth first.  The children of a node (one more assignment fixed,
// over a whole row or column of the node's assignment matrix) are created
// together in one batch handle that inherits the node's reduced costs
// (qap_rlt2_children) and advanced together; children whose bound reaches the
// incumbent are discarded, the others are explored best bound first.  The
// branch is chosen by strong branching (qap_rlt2_strong_branch) or, without
// it, is the node's lowest free facility.  Small nodes are enumerated on the
// host.  Every node's B-level assignment is a permutation; its objective,
// improved by pairwise-exchange descent, updates the incumbent, and the stop
// rule of every live handle follows the incumbent.
//
// Checkpoints (Section 7 runs long searches through interruptions): the
// incumbent, the counters and the fixed assignments of every open node, in
// exploration order, written to a file atomically.  A resumed run re-creates
// the open nodes from their subproblems (qap_subproblem), so their dual ascent
// restarts at the Gilmore-Lawler bound instead of the inherited state.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <numeric>
#include <string>
#include <vector>

#include "qap_rlt2.h"

namespace qap {
std::string& last_error();   // api.hip: the message behind qap_last_error
}

namespace {

qap_status bnb_fail(qap_status st, const std::string& msg)
{
    qap::last_error() = msg;
    return st;
}

bool is_perm(int N, const int32_t* p)
{
    std::vector<char> seen(N, 0);
    for (int i = 0; i < N; ++i) {
        if (p[i] < 0 || p[i] >= N || seen[p[i]]) return false;
        seen[p[i]] = 1;
    }
    return true;
}

double objective(int N, const double* F, const double* D, const double* B0, double constant, const int32_t* p)
{
    double s = 0.0;
    for (int i = 0; i < N; ++i) {
        const double* Fi = F + (size_t)i * N;
        const double* Dp = D + (size_t)p[i] * N;
        for (int k = 0; k < N; ++k) s += Fi[k] * Dp[p[k]];
    }
    if (B0)
        for (int i = 0; i < N; ++i) s += B0[(size_t)i * N + p[i]];
    return s + constant;
}

// Objective change when facilities r and s exchange locations.
double swap_delta(int N, const double* F, const double* D, const double* B0, const int32_t* p, int r, int s)
{
    const int pr = p[r], ps = p[s];
    double d = 0.0;
    for (int k = 0; k < N; ++k) {
        if (k == r || k == s) continue;
        const int pk = p[k];
        d += (F[r * N + k] - F[s * N + k]) * (D[ps * N + pk] - D[pr * N + pk]);
        d += (F[k * N + r] - F[k * N + s]) * (D[pk * N + ps] - D[pk * N + pr]);
    }
    d += F[r * N + r] * (D[ps * N + ps] - D[pr * N + pr]) + F[s * N + s] * (D[pr * N + pr] - D[ps * N + ps]);
    d += F[r * N + s] * (D[ps * N + pr] - D[pr * N + ps]) + F[s * N + r] * (D[pr * N + ps] - D[ps * N + pr]);
    if (B0) d += B0[r * N + ps] + B0[s * N + pr] - B0[r * N + pr] - B0[s * N + ps];
    return d;
}

// Best-improvement pairwise-exchange descent; returns the objective.
double local_search(int N, const double* F, const double* D, const double* B0, double constant, int32_t* p)
{
    double v = objective(N, F, D, B0, constant, p);
    const double tol = 1e-12 * std::max(1.0, std::fabs(v));
    for (int round = 0; round < 100 * N * N; ++round) {
        double best = -tol;
        int br = -1, bs = -1;
        for (int r = 0; r < N; ++r)
            for (int s = r + 1; s < N; ++s) {
                const double d = swap_delta(N, F, D, B0, p, r, s);
                if (d < best) {
                    best = d;
                    br = r;
                    bs = s;
                }
            }
        if (br < 0) break;
        std::swap(p[br], p[bs]);
        v = objective(N, F, D, B0, constant, p);   // recomputed: no drift from summed deltas
    }
    return v;
}

// A node of the tree: its fixed assignments in the original indices.
struct Node {
    std::vector<int32_t> fac, loc;
};

// Free facilities and locations of a node, ascending (instance indices).
void free_lists(int N, const Node& nd, std::vector<int>& ff, std::vector<int>& fl)
{
    std::vector<char> a(N, 0), b(N, 0);
    for (size_t t = 0; t < nd.fac.size(); ++t) {
        a[nd.fac[t]] = 1;
        b[nd.loc[t]] = 1;
    }
    ff.clear();
    fl.clear();
    for (int i = 0; i < N; ++i) {
        if (!a[i]) ff.push_back(i);
        if (!b[i]) fl.push_back(i);
    }
}

// Handles whose instances are explored in `order`.
struct Frame {
    qap_rlt2* h = nullptr;
    std::vector<Node> nodes;     // instance x of h is nodes[x]
    std::vector<double> bound;   // bound of instance x after its dual ascent
    std::vector<int> order;      // instances still to explore, best bound first
    size_t next = 0;
};

struct Search {
    int N;
    const double* F;
    const double* D;
    const qap_bnb_params* p;
    bool integral = true;
    double ub = std::numeric_limits<double>::infinity();
    std::vector<int32_t> best;
    int64_t nodes = 0, pruned = 0, leaves = 0;
    double root_bound = -std::numeric_limits<double>::infinity();
    std::vector<Frame> stack;

    // A node is discarded once its bound reaches this value: with integral
    // data every objective is an integer, so a bound above UB - 1 suffices;
    // delta allows for the rounding of the bound itself.
    double threshold() const
    {
        if (!std::isfinite(ub)) return 0.0;   // no incumbent: the stop rule stays off
        const double delta = (p->precision == QAP_FP32_NEAREST ? 1e-5 : 1e-9) * std::max(1.0, std::fabs(ub));
        return integral ? ub - 1.0 + delta : ub + delta;
    }
    bool prunable(double b) const { return std::isfinite(ub) && b >= threshold(); }

    qap_status offer(const int32_t* perm)
    {
        std::vector<int32_t> q(perm, perm + N);
        const double v = local_search(N, F, D, nullptr, 0.0, q.data());
        if (v < ub) {
            ub = v;
            best = q;
            const double t = threshold();
            for (Frame& f : stack) {
                qap_status st = qap_rlt2_set_stop(f.h, p->K, t);
                if (st != QAP_OK) return st;
            }
        }
        return QAP_OK;
    }

    // Incumbent candidates from the B-level assignment of each instance.
    qap_status harvest(qap_rlt2* h, const std::vector<Node>& nds)
    {
        std::vector<int> ff, fl;
        std::vector<int32_t> loc(N), full(N);
        for (size_t x = 0; x < nds.size(); ++x) {
            free_lists(N, nds[x], ff, fl);
            qap_status st = qap_rlt2_instance_assignment(h, (int)x, loc.data());
            if (st != QAP_OK) return st;
            const int M = (int)ff.size();
            if (!is_perm(M, loc.data())) continue;   // not yet a solved B problem
            for (size_t t = 0; t < nds[x].fac.size(); ++t) full[nds[x].fac[t]] = nds[x].loc[t];
            for (int a = 0; a < M; ++a) full[ff[a]] = fl[loc[a]];
            if ((st = offer(full.data())) != QAP_OK) return st;
        }
        return QAP_OK;
    }

    // Advance a new frame's handle, read its bounds and order its survivors.
    qap_status settle(Frame& f, int iters)
    {
        qap_status st = qap_rlt2_ascend(f.h, iters, nullptr);
        if (st != QAP_OK) return st;
        const int K = (int)f.nodes.size();
        std::vector<double> lb(K), cert(K);
        st = qap_rlt2_batch_bounds(f.h, lb.data(), p->precision == QAP_FP64 ? nullptr : cert.data());
        if (st != QAP_OK) return st;
        f.bound = p->precision == QAP_FP64 ? lb : cert;
        nodes += K;
        if ((st = harvest(f.h, f.nodes)) != QAP_OK) return st;
        f.order.clear();
        for (int x = 0; x < K; ++x) {
            if (prunable(f.bound[x]))
                ++pruned;
            else
                f.order.push_back(x);
        }
        std::stable_sort(f.order.begin(), f.order.end(), [&](int a, int b) { return f.bound[a] < f.bound[b]; });
        f.next = 0;
        return QAP_OK;
    }

    // Enumerate every completion of a small node on the host.
    void enumerate(const Node& nd)
    {
        std::vector<int> ff, fl;
        free_lists(N, nd, ff, fl);
        std::vector<int32_t> perm(N);
        for (size_t t = 0; t < nd.fac.size(); ++t) perm[nd.fac[t]] = nd.loc[t];
        std::vector<int> order(fl);
        do {
            for (size_t a = 0; a < ff.size(); ++a) perm[ff[a]] = order[a];
            const double v = objective(N, F, D, nullptr, 0.0, perm.data());
            if (v < ub) {
                ub = v;
                best = perm;
            }
        } while (std::next_permutation(order.begin(), order.end()));
        ++leaves;
        const double t = threshold();
        for (Frame& f : stack) (void)qap_rlt2_set_stop(f.h, p->K, t);
    }

    // Children of instance x of frame fi, pushed as a new frame.
    qap_status expand(size_t fi, int x)
    {
        Frame& f = stack[fi];
        const Node& nd = f.nodes[x];
        std::vector<int> ff, fl;
        free_lists(N, nd, ff, fl);
        const int M = (int)ff.size();
        int kind = 0, index = 0;
        if (p->strong_iters >= 0) {
            qap_status st = qap_rlt2_strong_branch(f.h, x, p->strong_iters, nullptr, &kind, &index);
            if (st != QAP_OK) return st;
        }
        std::vector<int32_t> fac(M), loc(M);
        Frame c;
        for (int y = 0; y < M; ++y) {
            fac[y] = kind == 0 ? index : y;
            loc[y] = kind == 0 ? y : index;
            Node ch = nd;
            ch.fac.push_back(ff[fac[y]]);
            ch.loc.push_back(fl[loc[y]]);
            c.nodes.push_back(ch);
        }
        qap_status st = qap_rlt2_children(f.h, x, M, fac.data(), loc.data(), 2, &c.h);
        if (st != QAP_OK) return st;
        stack.push_back(std::move(c));
        st = qap_rlt2_set_stop(stack.back().h, p->K, threshold());
        if (st == QAP_OK) st = settle(stack.back(), p->iters);
        return st;
    }

    void pop()
    {
        qap_rlt2_destroy(stack.back().h);
        stack.pop_back();
    }

    ~Search()
    {
        while (!stack.empty()) pop();
    }

    // Open nodes in exploration order (the top frame's next node first).
    std::vector<Node> open_nodes() const
    {
        std::vector<Node> out;
        for (size_t fi = stack.size(); fi-- > 0;) {
            const Frame& f = stack[fi];
            for (size_t y = f.next; y < f.order.size(); ++y) out.push_back(f.nodes[f.order[y]]);
        }
        return out;
    }

    qap_status checkpoint() const
    {
        if (!p->checkpoint) return QAP_OK;
        const std::string path = p->checkpoint, tmp = path + ".tmp";
        FILE* fp = fopen(tmp.c_str(), "wb");
        if (!fp) return bnb_fail(QAP_EINVAL, "cannot write checkpoint " + tmp);
        const std::vector<Node> open = open_nodes();
        const int64_t nopen = (int64_t)open.size();
        bool ok = fwrite("QAPBNB01", 1, 8, fp) == 8;
        auto w = [&](const void* d, size_t n) { ok = ok && fwrite(d, 1, n, fp) == n; };
        w(&N, sizeof(N));
        w(F, sizeof(double) * N * N);
        w(D, sizeof(double) * N * N);
        const int has = std::isfinite(ub) ? 1 : 0;
        w(&has, sizeof(has));
        w(&ub, sizeof(ub));
        std::vector<int32_t> b = best;
        b.resize(N, 0);
        w(b.data(), sizeof(int32_t) * N);
        w(&nodes, sizeof(nodes));
        w(&pruned, sizeof(pruned));
        w(&leaves, sizeof(leaves));
        w(&root_bound, sizeof(root_bound));
        w(&nopen, sizeof(nopen));
        for (const Node& nd : open) {
            const int32_t m = (int32_t)nd.fac.size();
            w(&m, sizeof(m));
            w(nd.fac.data(), sizeof(int32_t) * m);
            w(nd.loc.data(), sizeof(int32_t) * m);
        }
        ok = (fclose(fp) == 0) && ok;
        if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0)
            return bnb_fail(QAP_EINVAL, "writing checkpoint " + path + " failed");
        return QAP_OK;
    }

    // Re-create the open nodes of a checkpoint as one frame.
    qap_status resume()
    {
        FILE* fp = fopen(p->checkpoint, "rb");
        if (!fp) return bnb_fail(QAP_EINVAL, std::string("cannot read checkpoint ") + p->checkpoint);
        bool ok = true;
        auto r = [&](void* d, size_t n) { ok = ok && fread(d, 1, n, fp) == n; };
        char magic[8];
        r(magic, 8);
        int n0 = 0;
        r(&n0, sizeof(n0));
        if (!ok || memcmp(magic, "QAPBNB01", 8) != 0 || n0 != N) {
            fclose(fp);
            return bnb_fail(QAP_EINVAL, "checkpoint is not for this instance");
        }
        std::vector<double> F0(N * N), D0(N * N);
        r(F0.data(), sizeof(double) * N * N);
        r(D0.data(), sizeof(double) * N * N);
        if (!ok || memcmp(F0.data(), F, sizeof(double) * N * N) != 0 ||
            memcmp(D0.data(), D, sizeof(double) * N * N) != 0) {
            fclose(fp);
            return bnb_fail(QAP_EINVAL, "checkpoint is not for this instance");
        }
        int has = 0;
        double u = 0.0;
        r(&has, sizeof(has));
        r(&u, sizeof(u));
        std::vector<int32_t> b(N);
        r(b.data(), sizeof(int32_t) * N);
        r(&nodes, sizeof(nodes));
        r(&pruned, sizeof(pruned));
        r(&leaves, sizeof(leaves));
        r(&root_bound, sizeof(root_bound));
        int64_t nopen = 0;
        r(&nopen, sizeof(nopen));
        std::vector<Node> open;
        for (int64_t t = 0; ok && t < nopen; ++t) {
            int32_t m = 0;
            r(&m, sizeof(m));
            if (!ok || m < 0 || m > N) {
                ok = false;
                break;
            }
            Node nd;
            nd.fac.resize(m);
            nd.loc.resize(m);
            r(nd.fac.data(), sizeof(int32_t) * m);
            r(nd.loc.data(), sizeof(int32_t) * m);
            open.push_back(nd);
        }
        fclose(fp);
        if (!ok) return bnb_fail(QAP_EINVAL, "truncated checkpoint");
        if (has) {
            if (!is_perm(N, b.data())) return bnb_fail(QAP_EINVAL, "checkpoint incumbent is not a permutation");
            ub = u;
            best = b;
        }
        if (open.empty()) return QAP_OK;
        // Nodes of the frame, as subproblems of the instance.
        std::vector<int32_t> Ns;
        std::vector<std::vector<double>> Fs, Ds, Bs;
        std::vector<double> consts;
        for (const Node& nd : open) {
            const int m = (int)nd.fac.size(), M = N - m;
            if (M < 3) return bnb_fail(QAP_EINVAL, "checkpoint holds a node below 3 free facilities");
            std::vector<double> Fm(M * M), Dm(M * M), Bm(M * M);
            double c = 0.0;
            qap_status st = qap_subproblem(N, F, D, m, nd.fac.data(), nd.loc.data(), Fm.data(), Dm.data(), Bm.data(),
                                           &c);
            if (st != QAP_OK) return st;
            Ns.push_back(M);
            Fs.push_back(Fm);
            Ds.push_back(Dm);
            Bs.push_back(Bm);
            consts.push_back(c);
        }
        std::vector<const double*> fp_, dp_, bp_;
        for (size_t x = 0; x < open.size(); ++x) {
            fp_.push_back(Fs[x].data());
            dp_.push_back(Ds[x].data());
            bp_.push_back(Bs[x].data());
        }
        qap_rlt2_opts o = opts();
        Frame f;
        f.nodes = open;
        qap_status st = qap_rlt2_batch_create((int)open.size(), Ns.data(), fp_.data(), dp_.data(), bp_.data(),
                                              consts.data(), &o, &f.h);
        if (st != QAP_OK) return st;
        stack.push_back(std::move(f));
        st = settle(stack.back(), p->iters);
        if (st != QAP_OK) return st;
        // settle() counted these nodes again; they were counted when created.
        nodes -= (int64_t)open.size();
        // Keep the checkpoint's exploration order rather than bound order.
        Frame& top = stack.back();
        std::vector<int> keep;
        for (int x = 0; x < (int)open.size(); ++x)
            if (!prunable(top.bound[x])) keep.push_back(x);
        top.order = keep;
        return QAP_OK;
    }

    qap_rlt2_opts opts() const
    {
        qap_rlt2_opts o;
        qap_rlt2_default_opts(&o);
        o.precision = p->precision;
        o.device = p->device;
        o.stream = p->stream;
        o.trace_level = 0;
        o.use_graph = 0;   // few iterations per handle: plain launches
        o.autotune = 0;
        o.K = p->K;
        o.UB = threshold();
        return o;
    }
};

}  // namespace

extern "C" {

qap_status qap_objective(int N, const double* F, const double* D, const double* B0, double constant,
                         const int32_t* perm, double* value)
{
    if (N < 1 || !F || !D || !perm || !value) return bnb_fail(QAP_EINVAL, "bad argument");
    if (!is_perm(N, perm)) return bnb_fail(QAP_EINVAL, "perm is not a permutation");
    *value = objective(N, F, D, B0, constant, perm);
    return QAP_OK;
}

qap_status qap_ub_local_search(int N, const double* F, const double* D, const double* B0, double constant,
                               int32_t* perm, double* value)
{
    if (N < 1 || !F || !D || !perm) return bnb_fail(QAP_EINVAL, "bad argument");
    if (!is_perm(N, perm)) return bnb_fail(QAP_EINVAL, "perm is not a permutation");
    const double v = local_search(N, F, D, B0, constant, perm);
    if (value) *value = v;
    return QAP_OK;
}

qap_status qap_bnb_default_params(qap_bnb_params* p)
{
    if (!p) return bnb_fail(QAP_EINVAL, "null params");
    p->precision = QAP_FP64;
    p->device = -1;
    p->stream = nullptr;
    p->root_iters = 50;
    p->iters = 10;
    p->K = 0.0;
    p->UB = 0.0;
    p->strong_iters = 2;
    p->leaf_size = 5;
    p->max_nodes = 0;
    p->checkpoint = nullptr;
    p->checkpoint_every = 64;
    p->resume = 0;
    return QAP_OK;
}

qap_status qap_bnb_solve(int N, const double* F, const double* D, const qap_bnb_params* prm, qap_bnb_result* r)
{
    if (N < 3 || N > QAP_RLT2_MAX_N || !F || !D || !r) return bnb_fail(QAP_EINVAL, "bad argument");
    qap_bnb_params p;
    qap_bnb_default_params(&p);
    if (prm) p = *prm;
    if (p.leaf_size < 3 || p.leaf_size > 9) return bnb_fail(QAP_EINVAL, "leaf_size must be in [3, 9]");
    if (p.iters < 0 || p.root_iters < 0 || p.checkpoint_every < 1) return bnb_fail(QAP_EINVAL, "bad iteration counts");
    if (p.resume && !p.checkpoint) return bnb_fail(QAP_EINVAL, "resume needs a checkpoint path");
    for (int x = 0; x < N * N; ++x)
        if (!std::isfinite(F[x]) || !std::isfinite(D[x])) return bnb_fail(QAP_EINVAL, "non-finite F or D");
    Search s;
    s.N = N;
    s.F = F;
    s.D = D;
    s.p = &p;
    for (int x = 0; x < N * N; ++x)
        s.integral = s.integral && F[x] == std::floor(F[x]) && D[x] == std::floor(D[x]);
    // Incumbent: the caller's UB, and the heuristic from the identity.
    std::vector<int32_t> id(N);
    std::iota(id.begin(), id.end(), 0);
    qap_status st = s.offer(id.data());
    if (st != QAP_OK) return st;
    if (p.UB > 0.0 && p.UB < s.ub) s.ub = p.UB;
    int64_t last_ck = 0;
    if (p.resume) {
        if ((st = s.resume()) != QAP_OK) return st;
        last_ck = s.nodes;
    } else {
        // Root node.
        Frame f;
        f.nodes.push_back(Node());
        qap_rlt2_opts o = s.opts();
        if ((st = qap_rlt2_create_ex(N, F, D, nullptr, 0.0, &o, &f.h)) != QAP_OK) return st;
        s.stack.push_back(std::move(f));
        if ((st = s.settle(s.stack.back(), p.root_iters)) != QAP_OK) return st;
        s.root_bound = s.stack.back().bound[0];
    }
    bool complete = true;
    while (!s.stack.empty()) {
        Frame& f = s.stack.back();
        if (f.next >= f.order.size()) {
            s.pop();
            continue;
        }
        if (p.max_nodes > 0 && s.nodes >= p.max_nodes) {
            complete = false;
            break;
        }
        if (p.checkpoint && s.nodes - last_ck >= p.checkpoint_every) {
            if ((st = s.checkpoint()) != QAP_OK) return st;
            last_ck = s.nodes;
        }
        const int x = f.order[f.next++];
        if (s.prunable(f.bound[x])) {
            ++s.pruned;
            continue;
        }
        const int M = N - (int)f.nodes[x].fac.size();
        if (M <= p.leaf_size) {
            s.enumerate(f.nodes[x]);
            continue;
        }
        if ((st = s.expand(s.stack.size() - 1, x)) != QAP_OK) return st;
    }
    if (!complete && p.checkpoint && (st = s.checkpoint()) != QAP_OK) return st;
    if (complete && p.checkpoint) std::remove(p.checkpoint);
    r->value = s.ub;
    std::fill(r->perm, r->perm + QAP_RLT2_MAX_N, -1);
    for (int i = 0; i < N && i < (int)s.best.size(); ++i) r->perm[i] = s.best[i];
    r->root_bound = s.root_bound;
    r->nodes = s.nodes;
    r->pruned = s.pruned;
    r->leaves = s.leaves;
    r->complete = complete ? 1 : 0;
    return QAP_OK;
}

}  // extern "C"
