// Mixed-robot scheduler: several groups of IK problems (different robots,
// shapes and kernel variants) solved together.
//
//  * Each group runs persistent LM launches: a fixed grid whose wavefronts
//    pop work items (64 problems per item for the per-lane kernel, one for
//    the wave kernel) from a device queue.
//  * A launch runs at most k iterations per problem; the problem state stays
//    in HBM (resumable kernels).  Between launches a compaction kernel packs
//    the unfinished problems into the next active list, so problems that
//    exited early stop occupying lanes.
//  * The whole chain (all rounds of all groups) is captured once into a
//    hipGraph with one branch per group and replayed; groups run
//    concurrently on the device.
//  * k and the persistent grid size come from an autotuner that times the
//    candidates and keeps the best per batch signature.
// Per-problem results do not depend on k, the grid or the group order: a
// resumed problem rebuilds exactly the values it would have kept.
#include <stdio.h>
#include <string.h>

#include <map>
#include <string>
#include <vector>

#include "pk_ctx.hpp"
#include "pk_device.hpp"

namespace pk {
namespace {

__global__ void sched_fill_kernel(int64_t count, int32_t v, int32_t *p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// Unfinished problems of the current list -> next list.
__global__ void compact_kernel(int64_t N, const int32_t *__restrict__ cur,
                               const int32_t *__restrict__ n_cur,
                               const int32_t *__restrict__ st_state, int32_t *next,
                               int32_t *n_next)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nc = n_cur ? (int64_t)*n_cur : N;
    if (i >= nc) return;
    const int32_t p = cur ? cur[i] : (int32_t)i;
    if (!(st_state[p] & PK_ST_DONE)) next[atomicAdd(n_next, 1)] = p;
}

inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

struct GroupPlan {
    const RobotEntry *rb;
    SolveParams P;
    int variant;
    pk_ik_outputs out;
    // workspace
    int32_t *lists[2];
    int32_t *counters;   // [0..1] list sizes, [2] queue head
};

struct GraphEntry {
    std::string key;
    hipGraphExec_t exec = nullptr;
    std::vector<hipStream_t> streams;
};

struct SchedCache {
    std::vector<GraphEntry> graphs;
    std::map<std::string, pk_sched_options> tuned;
    std::vector<void *> bufs;
    size_t bytes = 0;
    void *buf = nullptr;
    std::vector<hipStream_t> streams;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins;
};

std::map<pk_ctx *, SchedCache> g_sched;

int cu_count(pk_ctx *ctx)
{
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, ctx->device) != hipSuccess) return 256;
    return pr.multiProcessorCount;
}

std::string signature(int n_groups, const pk_ik_group *g, const pk_lm_options *o)
{
    char buf[128];
    std::string s;
    for (int i = 0; i < n_groups; ++i) {
        snprintf(buf, sizeof buf, "r%d:T%lld:K%d;", g[i].robot_id, (long long)g[i].problem.n_targets,
                 g[i].problem.K);
        s += buf;
    }
    snprintf(buf, sizeof buf, "it%d:ee%d:v%d", o->max_iters, o->early_exit, o->variant);
    return s + buf;
}

// Enqueues the chain of every group on its own stream (forked from / joined
// into `main`).  Valid both eagerly and under stream capture.
hipError_t enqueue(pk_ctx *ctx, SchedCache &C, std::vector<GroupPlan> &plans, int k, int bpc,
                   hipStream_t main)
{
    const int G = (int)plans.size();
    while ((int)C.streams.size() < G) {
        hipStream_t s;
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        C.streams.push_back(s);
        hipEvent_t ev;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return e;
        C.joins.push_back(ev);
    }
    if (!C.fork) {
        hipError_t e = hipEventCreateWithFlags(&C.fork, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(C.fork, main);
    if (e != hipSuccess) return e;
    const int cus = cu_count(ctx);
    for (int g = 0; g < G; ++g) {
        hipStream_t s = C.streams[g];
        if ((e = hipStreamWaitEvent(s, C.fork, 0)) != hipSuccess) return e;
        GroupPlan &pl = plans[g];
        const int max_it = pl.P.max_iters;
        const int kk = (k <= 0 || k > max_it) ? (max_it > 0 ? max_it : 1) : k;
        const int rounds = max_it > 0 ? (max_it + kk - 1) / kk : 1;
        const int64_t N = pl.P.N;
        for (int r = 0; r < rounds; ++r) {
            SolveParams P = pl.P;
            P.iter_budget = kk;
            P.resume = r > 0;
            const int cur = r & 1;
            P.active = r > 0 ? pl.lists[cur] : nullptr;
            P.n_active = r > 0 ? pl.counters + cur : nullptr;
            P.queue_head = pl.counters + 2;
            hipLaunchKernelGGL(sched_fill_kernel, dim3(1), dim3(64), 0, s, (int64_t)1, 0, pl.counters + 2);
            const int pblocks = bpc * cus;
            e = launch_lm(*pl.rb, P, pl.variant, s, pblocks);
            if (e != hipSuccess) return e;
            if (r + 1 < rounds) {
                const int nxt = cur ^ 1;
                hipLaunchKernelGGL(sched_fill_kernel, dim3(1), dim3(64), 0, s, (int64_t)1, 0, pl.counters + nxt);
                hipLaunchKernelGGL(compact_kernel, dim3(nb(N, 256)), dim3(256), 0, s, N,
                                   r > 0 ? pl.lists[cur] : (const int32_t *)nullptr,
                                   r > 0 ? pl.counters + cur : (const int32_t *)nullptr, pl.P.st_state,
                                   pl.lists[nxt], pl.counters + nxt);
            }
        }
        if (pl.out.best_index || pl.out.best_joints || pl.out.target_success) {
            e = launch_best_of_k(pl.P, pl.rb->host.nv, pl.out.best_index, pl.out.best_joints,
                                 pl.out.target_success, s);
            if (e != hipSuccess) return e;
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipEventRecord(C.joins[g], s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(main, C.joins[g], 0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

int build_plans(pk_ctx *ctx, SchedCache &C, int n_groups, const pk_ik_group *groups,
                const pk_lm_options *opt, const pk_sched_options &sch, std::vector<GroupPlan> &plans)
{
    // workspace sizing: per problem lambda, state, iters, accepts, itt,
    // pose_cost, cost, status and two lists (4-byte words) + counters.
    size_t words = 0;
    for (int g = 0; g < n_groups; ++g) {
        const pk_ik_problem &pr = groups[g].problem;
        words += (size_t)pr.n_targets * pr.K * 10 + 64;
    }
    if (words * 4 > C.bytes) {
        if (C.buf) (void)hipFree(C.buf);
        C.buf = nullptr;
        C.bytes = 0;
        for (auto &ge : C.graphs)
            if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
        C.graphs.clear();
        if (hipMalloc(&C.buf, words * 4) != hipSuccess)
            return fail(ctx, PK_ENOMEM, "pk_ik_solve_mixed: workspace of %zu bytes", words * 4);
        C.bytes = words * 4;
    }
    int32_t *w = (int32_t *)C.buf;
    plans.clear();
    for (int g = 0; g < n_groups; ++g) {
        const pk_ik_group &gr = groups[g];
        const RobotEntry *rb = robot_of(ctx, gr.robot_id);
        if (!rb) return fail(ctx, PK_ENOTFOUND, "pk_ik_solve_mixed: group %d: unknown robot %d", g, gr.robot_id);
        const pk_ik_problem &pr = gr.problem;
        if (pr.n_targets <= 0 || pr.K < 1) return fail(ctx, PK_EINVAL, "pk_ik_solve_mixed: group %d is empty", g);
        const int64_t N = pr.n_targets * pr.K;
        if (N >= (int64_t)1 << 31) return fail(ctx, PK_EUNSUPPORTED, "pk_ik_solve_mixed: group %d too large", g);
        if (!pr.targets || !pr.seeds || !gr.out.joints)
            return fail(ctx, PK_EINVAL, "pk_ik_solve_mixed: group %d: NULL targets/seeds/joints", g);
        if (gr.out.trace_iters != 0) return fail(ctx, PK_EINVAL, "pk_ik_solve_mixed: traces are not supported");
        GroupPlan pl;
        pl.rb = rb;
        pl.out = gr.out;
        pk_lm_options og = *opt;
        if (sch.variant[g] != PK_VARIANT_AUTO) og.variant = sch.variant[g];
        int rc = prepare_solve(ctx, *rb, &gr.weights, &og, pl.P, pl.variant);
        if (rc) return rc;
        SolveParams &P = pl.P;
        P.K = pr.K;
        P.N = N;
        P.T = pr.n_targets;
        P.targets = pr.targets;
        P.seeds = pr.seeds;
        P.joints = gr.out.joints;
        P.pos_err = gr.out.pos_err;
        P.rot_err = gr.out.rot_err;
        P.st_lambda = (float *)w;           w += N;
        P.st_state = w;                     w += N;
        P.iters = gr.out.iters ? gr.out.iters : w;                    w += N;
        P.accepts = gr.out.accepts ? gr.out.accepts : w;              w += N;
        P.iters_to_tol = gr.out.iters_to_tol ? gr.out.iters_to_tol : w; w += N;
        P.pose_cost = (float *)w;           w += N;
        P.cost = gr.out.cost ? gr.out.cost : (float *)w;              w += N;
        P.status = gr.out.status ? gr.out.status : w;                 w += N;
        pl.lists[0] = w;                    w += N;
        pl.lists[1] = w;                    w += N;
        pl.counters = w;                    w += 64;
        plans.push_back(pl);
    }
    return PK_OK;
}

int run(pk_ctx *ctx, int n_groups, const pk_ik_group *groups, const pk_lm_options *opt,
        const pk_sched_options &sch, hipStream_t stream)
{
    SchedCache &C = g_sched[ctx];
    std::vector<GroupPlan> plans;
    int rc = build_plans(ctx, C, n_groups, groups, opt, sch, plans);
    if (rc) return rc;
    const int k = sch.iters_per_launch, bpc = sch.blocks_per_cu > 0 ? sch.blocks_per_cu : 4;
    if (!sch.use_graph) {
        PK_HIP(ctx, enqueue(ctx, C, plans, k, bpc, stream));
        return PK_OK;
    }
    // Graph cache keyed by every pointer, size and option baked into the chain.
    char kb[256];
    std::string key;
    for (int g = 0; g < n_groups; ++g) {
        const pk_ik_outputs &go = groups[g].out;
        snprintf(kb, sizeof kb, "%p.%p.%p.%p.%p.%p.%p.%p.%p.%p.%p.%p.%p.%p|", groups[g].problem.targets,
                 groups[g].problem.seeds, (void *)go.joints, (void *)go.status, (void *)go.cost,
                 (void *)go.iters, (void *)go.accepts, (void *)go.pos_err, (void *)go.rot_err,
                 (void *)go.iters_to_tol, (void *)go.best_index, (void *)go.best_joints,
                 (void *)go.target_success, (void *)groups[g].weights.q_rest);
        key += kb;
        snprintf(kb, sizeof kb, "%g,%g,%g,%g;", groups[g].weights.w_pos, groups[g].weights.w_rot,
                 groups[g].weights.w_limit, groups[g].weights.w_rest);
        key += kb;
    }
    snprintf(kb, sizeof kb, "k%d.b%d.", k, bpc);
    key += kb;
    for (int g = 0; g < n_groups; ++g) {
        snprintf(kb, sizeof kb, "v%d.", plans[g].variant);
        key += kb;
    }
    key += signature(n_groups, groups, opt);
    snprintf(kb, sizeof kb, "|%g,%g,%g,%g,%g,%g,%g,%g,%g", opt->lambda0, opt->nu_up, opt->nu_down,
             opt->lambda_min, opt->lambda_max, opt->tol_pos, opt->tol_rot, opt->damping_floor,
             opt->pivot_rel);
    key += kb;
    for (auto &ge : C.graphs)
        if (ge.key == key) {
            PK_HIP(ctx, hipGraphLaunch(ge.exec, stream));
            return PK_OK;
        }
    hipStream_t cap;
    PK_HIP(ctx, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e1 = enqueue(ctx, C, plans, k, bpc, cap);
        hipError_t e2 = hipStreamEndCapture(cap, &graph);
        e = e1 != hipSuccess ? e1 : e2;
    }
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(ctx, PK_EHIP, "pk_ik_solve_mixed: graph capture failed: %s", hipGetErrorString(e));
    }
    GraphEntry ge;
    ge.key = key;
    e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(ctx, PK_EHIP, "pk_ik_solve_mixed: instantiate: %s", hipGetErrorString(e));
    if (C.graphs.size() >= 8) {
        (void)hipGraphExecDestroy(C.graphs.front().exec);
        C.graphs.erase(C.graphs.begin());
    }
    C.graphs.push_back(ge);
    PK_HIP(ctx, hipGraphLaunch(ge.exec, stream));
    return PK_OK;
}

}  // namespace

int sched_run(pk_ctx *ctx, int n_groups, const pk_ik_group *groups, const pk_lm_options *opt,
              const pk_sched_options &sch, hipStream_t stream)
{
    return run(ctx, n_groups, groups, opt, sch, stream);
}

void sched_free(pk_ctx *ctx)
{
    auto it = g_sched.find(ctx);
    if (it == g_sched.end()) return;
    SchedCache &C = it->second;
    for (auto &ge : C.graphs)
        if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
    for (auto s : C.streams) (void)hipStreamDestroy(s);
    for (auto e : C.joins) (void)hipEventDestroy(e);
    if (C.fork) (void)hipEventDestroy(C.fork);
    if (C.buf) (void)hipFree(C.buf);
    g_sched.erase(it);
}

}  // namespace pk

using namespace pk;

extern "C" {

int pk_ik_solve_mixed(pk_ctx *ctx, int32_t n_groups, const pk_ik_group *groups,
                      const pk_lm_options *opt, const pk_sched_options *sched, void *stream)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_ik_solve_mixed: ctx is NULL");
    if (n_groups < 1 || n_groups > PK_MAX_GROUPS || !groups || !opt)
        return fail(ctx, PK_EINVAL, "pk_ik_solve_mixed: need 1..16 groups and options");
    PK_HIP(ctx, hipSetDevice(ctx->device));
    pk_sched_options s = {};
    s.use_graph = 1;
    if (sched) s = *sched;
    if (s.iters_per_launch == 0 && s.blocks_per_cu == 0) {
        auto &C = g_sched[ctx];
        auto it = C.tuned.find(signature(n_groups, groups, opt));
        if (it != C.tuned.end()) {
            const int ug = s.use_graph;
            s = it->second;
            s.use_graph = ug;
        }
    }
    if (s.iters_per_launch < 0 || s.blocks_per_cu < 0)
        return fail(ctx, PK_EINVAL, "pk_ik_solve_mixed: negative schedule option");
    return run(ctx, n_groups, groups, opt, s, (hipStream_t)stream);
}

int pk_autotune_mixed(pk_ctx *ctx, int32_t n_groups, const pk_ik_group *groups,
                      const pk_lm_options *opt, pk_sched_options *best, float *best_ms, void *stream)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_autotune_mixed: ctx is NULL");
    if (!best || n_groups < 1 || n_groups > PK_MAX_GROUPS || !groups || !opt)
        return fail(ctx, PK_EINVAL, "pk_autotune_mixed: bad arguments");
    PK_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const int ks[] = {5, 10, 25, 0};
    const int bs[] = {2, 4, 8};
    // Lanes per problem: both mappings for groups the per-lane kernel
    // supports (all combinations up to 4 such groups, else each one flipped
    // on its own), the wave mapping for the others.
    std::vector<int> flex;
    for (int g = 0; g < n_groups; ++g) {
        const RobotEntry *rb = robot_of(ctx, groups[g].robot_id);
        if (!rb) return fail(ctx, PK_ENOTFOUND, "pk_autotune_mixed: group %d: unknown robot", g);
        const RobotC &H = rb->host;
        if (H.chains > 0 && H.prismatic == 0 && H.n_mimic == 0 &&
            lane_variant_available(H.chains, H.chain_len, H.e[0].kind))
            flex.push_back(g);
    }
    std::vector<std::vector<int>> vsets;
    auto base = [&]() {
        std::vector<int> v(PK_MAX_GROUPS, PK_VARIANT_AUTO);
        for (int g = 0; g < n_groups; ++g) v[g] = PK_VARIANT_WAVE;
        for (int g : flex) v[g] = PK_VARIANT_LANE;
        return v;
    };
    if (flex.size() <= 4) {
        for (unsigned mask = 0; mask < (1u << flex.size()); ++mask) {
            std::vector<int> v = base();
            for (size_t i = 0; i < flex.size(); ++i)
                if (mask >> i & 1u) v[flex[i]] = PK_VARIANT_WAVE;
            vsets.push_back(v);
        }
    } else {
        vsets.push_back(base());
        for (int g : flex) {
            std::vector<int> v = base();
            v[g] = PK_VARIANT_WAVE;
            vsets.push_back(v);
        }
    }
    hipEvent_t a, b;
    PK_HIP(ctx, hipEventCreate(&a));
    PK_HIP(ctx, hipEventCreate(&b));
    float bestt = 1e30f;
    pk_sched_options bo = {};
    bo.blocks_per_cu = 4;
    bo.use_graph = 1;
    for (const auto &vs : vsets)
        for (int k : ks)
            for (int bpc : bs) {
                pk_sched_options s = {};
                s.iters_per_launch = k;
                s.blocks_per_cu = bpc;
                s.use_graph = 1;
                for (int g = 0; g < PK_MAX_GROUPS; ++g) s.variant[g] = vs[g];
                int rc = run(ctx, n_groups, groups, opt, s, st);   // capture + warm-up
                if (rc) return rc;
                PK_HIP(ctx, hipEventRecord(a, st));
                for (int r = 0; r < 3; ++r) {
                    rc = run(ctx, n_groups, groups, opt, s, st);
                    if (rc) return rc;
                }
                PK_HIP(ctx, hipEventRecord(b, st));
                PK_HIP(ctx, hipEventSynchronize(b));
                float ms = 0.f;
                PK_HIP(ctx, hipEventElapsedTime(&ms, a, b));
                ms /= 3.f;
                if (ms < bestt) {
                    bestt = ms;
                    bo = s;
                }
            }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    g_sched[ctx].tuned[signature(n_groups, groups, opt)] = bo;
    *best = bo;
    if (best_ms) *best_ms = bestt;
    return PK_OK;
}

}  // extern "C"
