// Mixed-robot scheduler: several groups of IK problems (different robots,
// shapes and device paths) solved in ONE persistent launch per round.
//
//  * A round runs every unfinished problem of every group for at most k more
//    LM iterations.  A plan kernel turns the groups' active-list sizes into
//    work items (64 problems for a per-lane path, one for a per-wavefront
//    path), the persistent kernel's wavefronts pop items from one device
//    queue and branch to the item's device path (lm_mixed.hip), and a
//    compaction kernel packs the problems still unfinished into the next
//    round's active lists, so problems that exited early stop taking lanes.
//  * Problem state stays in HBM between rounds (resumable kernels).
//  * The chain of rounds plus the per-group best-of-K is captured once into a
//    hipGraph per (buffers, options, schedule) and replayed.
//  * k, the persistent grid (wavefronts per CU), the workgroup size and the
//    lanes per problem of each group come from an autotuner that times the
//    candidates; its table is keyed by the batch's robot classes (variables
//    n, EEs m, EE kind), the options and the GPU architecture, and is stored
//    as JSON (pk_autotune_save / pk_autotune_load, and the file named by
//    PK_AUTOTUNE_TABLE, read at pk_create and written after tuning).
// Per-problem results do not depend on k, the grid, the workgroup size or
// the queue order: a resumed problem rebuilds exactly the values it would
// have kept.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "pk_ctx.hpp"
#include "pk_device.hpp"
#include "sched_table.hpp"

namespace pk {
namespace {

inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

struct GroupPlan {
    const RobotEntry *rb;
    SolveParams P;
    int variant;
    int path;
    pk_ik_outputs out;
    // workspace
    int32_t *lists[2];
    int32_t *counters;   // [0..1] list sizes
};

struct TableEntry {
    std::string key;                 // buffers, weights, options, paths
    MixedArgs base;                  // the batch for the single launch (per-round fields unset)
    int32_t *dev = nullptr;          // item_end [PK_MIX_GROUPS], then the queue head
    int lds_floats = 0;              // per wavefront, largest over the batch's paths
    int max_n = 0;
    bool single_ok = false;          // every group has a path in the single launch
};

struct GraphEntry {
    std::string key;                 // table key + '#' + schedule
    hipGraphExec_t exec = nullptr;
};

struct Tuned {
    pk_sched_options s;
    float ms;
};

struct SchedCache {
    std::vector<TableEntry> tables;
    std::vector<GraphEntry> graphs;
    std::map<std::string, Tuned> tuned;
    size_t bytes = 0;
    void *buf = nullptr;
    // per-group mode: one stream per group, forked from and joined into the caller's
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

size_t lds_per_block(pk_ctx *ctx)
{
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, ctx->device) != hipSuccess) return 65536;
    return pr.sharedMemPerBlock;
}

std::string arch_name(pk_ctx *ctx)
{
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, ctx->device) != hipSuccess) return "unknown";
    std::string a = pr.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// Robot class of a group: variables, EEs and EE kind.
std::string robot_class(const RobotC &H)
{
    int pose = 0;
    for (int k = 0; k < H.m; ++k) pose += H.e[k].kind == PK_EE_POSE;
    const char *kind = pose == H.m ? "pose" : (pose == 0 ? "position" : "mixed");
    char buf[64];
    snprintf(buf, sizeof buf, "n%d_m%d_%s", H.nv, H.m, kind);
    return buf;
}

// Autotune table key: the groups' classes in order, the options that shape
// the run, and the architecture.
std::string tune_key(pk_ctx *ctx, int n_groups, const pk_ik_group *g, const pk_lm_options *o)
{
    std::string s;
    for (int i = 0; i < n_groups; ++i) {
        const RobotEntry *rb = robot_of(ctx, g[i].robot_id);
        if (i) s += "+";
        s += rb ? robot_class(rb->host) : std::string("unknown");
    }
    char buf[96];
    snprintf(buf, sizeof buf, "|it%d|ee%d|v%d|%s", o->max_iters, o->early_exit ? 1 : 0, o->variant,
             arch_name(ctx).c_str());
    return s + buf;
}

// The device path of a group's robot under a lanes-per-problem variant in
// the single launch (MIX_WAVE_64_8: the robot has no path there; the batch
// then runs in per-group mode).
int path_of(const RobotC &H, int variant)
{
    if (variant == PK_VARIANT_LANE) {
        if (H.chains == 1 && H.chain_len == 7 && H.e[0].kind == PK_EE_POSE) return MIX_LANE_ARM;
        if (H.chains == 4 && H.chain_len == 4 && H.e[0].kind == PK_EE_POSITION) return MIX_LANE_HAND;
        return MIX_WAVE_64_8;
    }
    if (H.max_depth + 1 > 16 || H.m > 4) return MIX_WAVE_64_8;
    if (variant == PK_VARIANT_WAVE && path_variant_available(H)) return MIX_PATH_16_4;
    return MIX_WAVE_16_4;
}

void drop_graphs(SchedCache &C)
{
    for (auto &ge : C.graphs)
        if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
    C.graphs.clear();
}

void drop_tables(SchedCache &C)
{
    drop_graphs(C);
    for (auto &te : C.tables)
        if (te.dev) (void)hipFree(te.dev);
    C.tables.clear();
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
        // tables and graphs hold pointers into the old workspace
        drop_tables(C);
        if (C.buf) (void)hipFree(C.buf);
        C.buf = nullptr;
        C.bytes = 0;
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
        og.target_exit = 0;   // resumed, compacted problems: not honoured here
        if (sch.variant[g] != PK_VARIANT_AUTO) og.variant = sch.variant[g];
        int rc = prepare_solve(ctx, *rb, &gr.weights, &og, pl.P, pl.variant);
        if (rc) return rc;
        pl.path = path_of(rb->host, pl.variant);
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

// Key of everything a batch's device table and graph bake in, except the
// schedule.
std::string data_key(int n_groups, const pk_ik_group *groups, const pk_lm_options *opt,
                     const std::vector<GroupPlan> &plans)
{
    char kb[320];
    std::string key;
    for (int g = 0; g < n_groups; ++g) {
        const pk_ik_outputs &go = groups[g].out;
        snprintf(kb, sizeof kb, "r%d:T%lld:K%d:%p.%p.%p.%p.%p.%p.%p.%p.%p.%p.%p.%p.%p.%p|", groups[g].robot_id,
                 (long long)groups[g].problem.n_targets, groups[g].problem.K, groups[g].problem.targets,
                 groups[g].problem.seeds, (void *)go.joints, (void *)go.status, (void *)go.cost,
                 (void *)go.iters, (void *)go.accepts, (void *)go.pos_err, (void *)go.rot_err,
                 (void *)go.iters_to_tol, (void *)go.best_index, (void *)go.best_joints,
                 (void *)go.target_success, (void *)groups[g].weights.q_rest);
        key += kb;
        snprintf(kb, sizeof kb, "%g,%g,%g,%g,p%d;", groups[g].weights.w_pos, groups[g].weights.w_rot,
                 groups[g].weights.w_limit, groups[g].weights.w_rest, plans[g].path);
        key += kb;
    }
    snprintf(kb, sizeof kb, "|%d,%d,%g,%g,%g,%g,%g,%g,%g,%g,%g", opt->max_iters, opt->early_exit,
             opt->lambda0, opt->nu_up, opt->nu_down, opt->lambda_min, opt->lambda_max, opt->tol_pos,
             opt->tol_rot, opt->damping_floor, opt->pivot_rel);
    return key + kb;
}

// The batch's single-launch description (built once per key) and its small
// device buffers.  Wave paths go first in the queue: their items are the
// longest.
int table_for(pk_ctx *ctx, SchedCache &C, const std::string &key, const std::vector<GroupPlan> &plans,
              TableEntry **out)
{
    for (auto &te : C.tables)
        if (te.key == key) {
            *out = &te;
            return PK_OK;
        }
    TableEntry te;
    te.key = key;
    memset(&te.base, 0, sizeof te.base);
    te.single_ok = (int)plans.size() <= PK_MIX_GROUPS;
    for (const GroupPlan &pl : plans) te.single_ok = te.single_ok && pl.path != MIX_WAVE_64_8;
    if (te.single_ok) {
        te.base.n_groups = (int)plans.size();
        int slot = 0;
        for (int pass = 0; pass < 2; ++pass)
            for (const GroupPlan &pl : plans) {
                const bool wave = pl.path == MIX_WAVE_16_4 || pl.path == MIX_PATH_16_4;
                if (wave != (pass == 0)) continue;
                MixedGroup &G = te.base.g[slot++];
                G.rb = pl.rb->dev;
                G.qr = pl.P.q_rest ? pl.P.q_rest : pl.rb->dev->mid;
                G.P = pl.P;
                G.P.queue_head = nullptr;
                G.list[0] = pl.lists[0];
                G.list[1] = pl.lists[1];
                G.count = pl.counters;
                G.path = pl.path;
                G.per_item = wave ? 1 : 64;
                te.lds_floats = std::max(te.lds_floats, mixed_lds_floats(pl.path));
                te.max_n = std::max(te.max_n, (int)pl.P.N);
            }
        if (hipMalloc(&te.dev, 256) != hipSuccess)
            return fail(ctx, PK_ENOMEM, "pk_ik_solve_mixed: queue buffers");
    }
    if (C.tables.size() >= 8) {
        // the oldest entry goes, with the graphs built on it
        const std::string old = C.tables.front().key + "#";
        for (size_t i = 0; i < C.graphs.size();)
            if (C.graphs[i].key.compare(0, old.size(), old) == 0) {
                (void)hipGraphExecDestroy(C.graphs[i].exec);
                C.graphs.erase(C.graphs.begin() + i);
            } else {
                ++i;
            }
        if (C.tables.front().dev) (void)hipFree(C.tables.front().dev);
        C.tables.erase(C.tables.begin());
    }
    C.tables.push_back(te);
    *out = &C.tables.back();
    return PK_OK;
}

// Iterations per launch and the number of rounds for a budget of max_it.
void rounds_of(int max_it, int k, int &kk, int &rounds)
{
    kk = (k <= 0 || k > max_it) ? (max_it > 0 ? max_it : 1) : k;
    rounds = max_it > 0 ? (max_it + kk - 1) / kk : 1;
}

// Single mode: the whole chain on one stream, rounds of (plan, one
// persistent launch over every group, compaction), then best-of-K per
// group.  Valid eagerly and under capture.
hipError_t enqueue_single(pk_ctx *ctx, const TableEntry &te, std::vector<GroupPlan> &plans, int k,
                          int wpc, int wg, hipStream_t s)
{
    int kk, rounds;
    rounds_of(plans[0].P.max_iters, k, kk, rounds);
    const int waves = wpc * cu_count(ctx);
    for (int r = 0; r < rounds; ++r) {
        MixedArgs a = te.base;
        a.round = r;
        const int cur = r & 1;
        for (int g = 0; g < a.n_groups; ++g) {
            MixedGroup &G = a.g[g];
            G.P.iter_budget = kk;
            G.P.resume = r > 0;
            G.P.active = r > 0 ? G.list[cur] : nullptr;
            G.P.n_active = r > 0 ? G.count + cur : nullptr;
        }
        hipError_t e = launch_mixed_round(a, te.dev, te.dev + PK_MIX_GROUPS, te.max_n, r + 1 == rounds,
                                          waves, wg, te.lds_floats, s);
        if (e != hipSuccess) return e;
    }
    for (GroupPlan &pl : plans)
        if (pl.out.best_index || pl.out.best_joints || pl.out.target_success) {
            hipError_t e = launch_best_of_k(pl.P, pl.rb->host.nv, pl.out.best_index, pl.out.best_joints,
                                            pl.out.target_success, s);
            if (e != hipSuccess) return e;
        }
    return hipGetLastError();
}

__global__ void sched_fill_kernel(int64_t count, int32_t v, int32_t *p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// Unfinished problems of the current list -> next list (per-group mode).
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

// Per-group mode: each group's chain of persistent launches (its own robot's
// kernel, its own queue) on its own stream, forked from and joined into
// `main`, so the groups run concurrently.  Valid eagerly and under capture.
hipError_t enqueue_per_group(pk_ctx *ctx, SchedCache &C, std::vector<GroupPlan> &plans, int k, int wpc,
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
    // Groups solved one problem per wavefront go first: they run longest, and
    // launched after the per-lane groups they found the CUs taken (mixed84k:
    // 1.14 against 1.41 ms at 8 wavefronts per CU).  Each group keeps its own
    // stream, so the order changes no result.
    std::vector<int> order;
    for (int pass = 0; pass < 2; ++pass)
        for (int g = 0; g < G; ++g)
            if ((plans[g].variant != PK_VARIANT_LANE) == (pass == 0)) order.push_back(g);
    for (int g : order) {
        hipStream_t s = C.streams[g];
        if ((e = hipStreamWaitEvent(s, C.fork, 0)) != hipSuccess) return e;
        GroupPlan &pl = plans[g];
        int kk, rounds;
        rounds_of(pl.P.max_iters, k, kk, rounds);
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
            e = launch_lm(*pl.rb, P, pl.variant, s, wpc * cus);
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

hipError_t enqueue(pk_ctx *ctx, SchedCache &C, const TableEntry &te, std::vector<GroupPlan> &plans,
                   const pk_sched_options &sch, int wpc, int wg, hipStream_t s)
{
    if (sch.mode == PK_SCHED_PER_GROUP) return enqueue_per_group(ctx, C, plans, sch.iters_per_launch, wpc, s);
    return enqueue_single(ctx, te, plans, sch.iters_per_launch, wpc, wg, s);
}

int run(pk_ctx *ctx, int n_groups, const pk_ik_group *groups, const pk_lm_options *opt,
        const pk_sched_options &sch, hipStream_t stream)
{
    SchedCache &C = g_sched[ctx];
    std::vector<GroupPlan> plans;
    int rc = build_plans(ctx, C, n_groups, groups, opt, sch, plans);
    if (rc) return rc;
    for (int g = 1; g < n_groups; ++g)
        if (plans[g].P.max_iters != plans[0].P.max_iters)
            return fail(ctx, PK_EINVAL, "pk_ik_solve_mixed: groups differ in max_iters");
    const int k = sch.iters_per_launch;
    const int wpc = sch.waves_per_cu > 0 ? sch.waves_per_cu : 4;
    const int wg = sch.workgroup_size > 0 ? sch.workgroup_size : 64;
    if (sch.mode != PK_SCHED_SINGLE && sch.mode != PK_SCHED_PER_GROUP)
        return fail(ctx, PK_EINVAL, "pk_ik_solve_mixed: unknown mode %d", sch.mode);
    if (wg != 64 && wg != 128 && wg != 256)
        return fail(ctx, PK_EINVAL, "pk_ik_solve_mixed: workgroup size %d (64, 128 or 256)", wg);
    const std::string dkey = data_key(n_groups, groups, opt, plans);
    TableEntry *te = nullptr;
    rc = table_for(ctx, C, dkey, plans, &te);
    if (rc) return rc;
    if (sch.mode == PK_SCHED_SINGLE) {
        if (!te->single_ok)
            return fail(ctx, PK_EUNSUPPORTED, "pk_ik_solve_mixed: the single launch serves at most %d "
                        "groups of robots with at most 16 tree levels and 4 EEs (use per-group mode)",
                        PK_MIX_GROUPS);
        if ((size_t)(wg / 64) * te->lds_floats * sizeof(float) > lds_per_block(ctx))
            return fail(ctx, PK_EUNSUPPORTED, "pk_ik_solve_mixed: %d-thread workgroups need %zu bytes of LDS",
                        wg, (size_t)(wg / 64) * te->lds_floats * sizeof(float));
    }
    if (!sch.use_graph) {
        PK_HIP(ctx, enqueue(ctx, C, *te, plans, sch, wpc, wg, stream));
        return PK_OK;
    }
    char kb[64];
    snprintf(kb, sizeof kb, "#m%d.k%d.w%d.g%d", sch.mode, k, wpc, wg);
    const std::string key = dkey + kb;
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
        hipError_t e1 = enqueue(ctx, C, *te, plans, sch, wpc, wg, cap);
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
    if (C.graphs.size() >= 16) {
        (void)hipGraphExecDestroy(C.graphs.front().exec);
        C.graphs.erase(C.graphs.begin());
    }
    C.graphs.push_back(ge);
    PK_HIP(ctx, hipGraphLaunch(ge.exec, stream));
    return PK_OK;
}

// ------------------------------------------------------------ JSON table
// One entry per line:
//   {"key": "...", "mode": 0, "k": 25, "waves_per_cu": 8, "workgroup_size": 64,
//    "variants": [1, 1, 2], "ms": 2.35}

int save_table(pk_ctx *ctx, const SchedCache &C, const char *path)
{
    FILE *f = fopen(path, "w");
    if (!f) return fail(ctx, PK_EINVAL, "pk_autotune_save: cannot write %s", path);
    fprintf(f, "{\"format\": \"pkmi-autotune-1\", \"entries\": [\n");
    size_t i = 0;
    for (const auto &kv : C.tuned) {
        const pk_sched_options &s = kv.second.s;
        const int ng = (int)std::count(kv.first.begin(), kv.first.begin() + kv.first.find('|'), '+') + 1;
        fprintf(f, "{\"key\": \"%s\", \"mode\": %d, \"k\": %d, \"waves_per_cu\": %d, "
                   "\"workgroup_size\": %d, \"variants\": [", kv.first.c_str(), s.mode, s.iters_per_launch,
                s.waves_per_cu, s.workgroup_size);
        for (int g = 0; g < ng && g < PK_MAX_GROUPS; ++g) fprintf(f, "%s%d", g ? ", " : "", s.variant[g]);
        fprintf(f, "], \"ms\": %.5f}%s\n", kv.second.ms, ++i < C.tuned.size() ? "," : "");
    }
    fprintf(f, "]}\n");
    const bool ok = fclose(f) == 0;
    return ok ? PK_OK : fail(ctx, PK_EINVAL, "pk_autotune_save: error writing %s", path);
}

// Integer after "\"name\": " in line, or def.
int json_int(const std::string &line, const char *name, int def)
{
    const std::string pat = std::string("\"") + name + "\": ";
    const size_t at = line.find(pat);
    return at == std::string::npos ? def : atoi(line.c_str() + at + pat.size());
}

int load_table(pk_ctx *ctx, SchedCache &C, const char *path)
{
    FILE *f = fopen(path, "r");
    if (!f) return fail(ctx, PK_ENOTFOUND, "pk_autotune_load: cannot read %s", path);
    char buf[4096];
    int n = 0;
    while (fgets(buf, sizeof buf, f)) {
        const std::string line = buf;
        const std::string kp = "\"key\": \"";
        const size_t a = line.find(kp);
        if (a == std::string::npos) continue;
        const size_t b = line.find('"', a + kp.size());
        if (b == std::string::npos) continue;
        Tuned t;
        memset(&t.s, 0, sizeof t.s);
        t.s.mode = json_int(line, "mode", PK_SCHED_SINGLE);
        t.s.iters_per_launch = json_int(line, "k", 0);
        t.s.waves_per_cu = json_int(line, "waves_per_cu", 4);
        t.s.workgroup_size = json_int(line, "workgroup_size", 64);
        t.s.use_graph = 1;
        const size_t v = line.find("\"variants\": [");
        if (v != std::string::npos) {
            const char *c = line.c_str() + v + 13;
            for (int g = 0; g < PK_MAX_GROUPS && *c && *c != ']'; ++g) {
                t.s.variant[g] = (int32_t)strtol(c, (char **)&c, 10);
                while (*c == ',' || *c == ' ') ++c;
            }
        }
        const size_t m = line.find("\"ms\": ");
        t.ms = m == std::string::npos ? 0.f : (float)atof(line.c_str() + m + 6);
        C.tuned[line.substr(a + kp.size(), b - a - kp.size())] = t;
        ++n;
    }
    fclose(f);
    return n;
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
    drop_tables(C);
    for (auto s : C.streams) (void)hipStreamDestroy(s);
    for (auto e : C.joins) (void)hipEventDestroy(e);
    if (C.fork) (void)hipEventDestroy(C.fork);
    if (C.buf) (void)hipFree(C.buf);
    g_sched.erase(it);
}

void sched_load_env(pk_ctx *ctx)
{
    const char *path = getenv("PK_AUTOTUNE_TABLE");
    if (path && *path) {
        const std::string err = ctx->err;
        (void)load_table(ctx, g_sched[ctx], path);   // a missing file is not an error here
        ctx->err = err;
    }
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
    if (s.iters_per_launch == 0 && s.waves_per_cu == 0) {
        for (int g = 0; g < n_groups; ++g)
            if (!robot_of(ctx, groups[g].robot_id))
                return fail(ctx, PK_ENOTFOUND, "pk_ik_solve_mixed: group %d: unknown robot", g);
        auto &C = g_sched[ctx];
        auto it = C.tuned.find(tune_key(ctx, n_groups, groups, opt));
        if (it != C.tuned.end()) {
            const int ug = s.use_graph;
            s = it->second.s;
            s.use_graph = ug;
        }
    }
    if (s.iters_per_launch < 0 || s.waves_per_cu < 0 || s.workgroup_size < 0)
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
    const int ks[] = {1, 2, 5, 10, 25, 0};
    const int ws[] = {2, 4, 8, 16};   // 16: four wavefronts per SIMD (the path-pair tree kernel)
    const int wgs[] = {64, 128, 256};
    // Lanes per problem: both mappings for groups the per-lane kernel
    // supports (all combinations up to 4 such groups, else each one flipped
    // on its own), the wave mapping for the others.
    std::vector<int> flex;
    for (int g = 0; g < n_groups; ++g) {
        const RobotEntry *rb = robot_of(ctx, groups[g].robot_id);
        if (!rb) return fail(ctx, PK_ENOTFOUND, "pk_autotune_mixed: group %d: unknown robot", g);
        const RobotC &H = rb->host;
        if (H.chains > 0 && H.n_mimic == 0 && (H.prismatic == 0 || H.chains == 1) &&
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
    bo.waves_per_cu = 4;
    bo.workgroup_size = 64;
    bo.use_graph = 1;
    const size_t lds_max = lds_per_block(ctx);
    for (const auto &vs : vsets) {
        // per-wavefront LDS of this variant set in the single launch (workgroups
        // that do not fit are skipped), and whether it serves the batch at all
        int ldsf = 0;
        bool single = n_groups <= PK_MIX_GROUPS;
        for (int g = 0; g < n_groups; ++g) {
            const int path = path_of(robot_of(ctx, groups[g].robot_id)->host,
                                     vs[g] == PK_VARIANT_WAVE ? PK_VARIANT_WAVE : PK_VARIANT_LANE);
            single = single && path != MIX_WAVE_64_8;
            if (path != MIX_WAVE_64_8) ldsf = std::max(ldsf, mixed_lds_floats(path));
        }
        for (int mode : {PK_SCHED_SINGLE, PK_SCHED_PER_GROUP})
        for (int k : ks)
            for (int wpc : ws)
                for (int wg : wgs) {
                    if (mode == PK_SCHED_SINGLE && (!single || (size_t)(wg / 64) * ldsf * sizeof(float) > lds_max))
                        continue;
                    if (mode == PK_SCHED_PER_GROUP && wg != 64) continue;   // its kernels run 64-thread blocks
                    pk_sched_options s = {};
                    s.mode = mode;
                    s.iters_per_launch = k;
                    s.waves_per_cu = wpc;
                    s.workgroup_size = wg;
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
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    SchedCache &C = g_sched[ctx];
    C.tuned[tune_key(ctx, n_groups, groups, opt)] = Tuned{bo, bestt};
    *best = bo;
    if (best_ms) *best_ms = bestt;
    const char *path = getenv("PK_AUTOTUNE_TABLE");
    if (path && *path) {
        int rc = save_table(ctx, C, path);
        if (rc) return rc;
    }
    return PK_OK;
}

int pk_autotune_save(pk_ctx *ctx, const char *path)
{
    if (!ctx || !path) return fail(ctx, PK_EINVAL, "pk_autotune_save: NULL argument");
    return save_table(ctx, g_sched[ctx], path);
}

int pk_autotune_load(pk_ctx *ctx, const char *path, int32_t *entries)
{
    if (!ctx || !path) return fail(ctx, PK_EINVAL, "pk_autotune_load: NULL argument");
    const int n = load_table(ctx, g_sched[ctx], path);
    if (n < 0) return n;
    if (entries) *entries = n;
    return PK_OK;
}

int pk_autotune_lookup(pk_ctx *ctx, int32_t n_groups, const pk_ik_group *groups,
                       const pk_lm_options *opt, pk_sched_options *found, float *ms)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_autotune_lookup: ctx is NULL");
    if (n_groups < 1 || n_groups > PK_MAX_GROUPS || !groups || !opt || !found)
        return fail(ctx, PK_EINVAL, "pk_autotune_lookup: bad arguments");
    for (int g = 0; g < n_groups; ++g)
        if (!robot_of(ctx, groups[g].robot_id))
            return fail(ctx, PK_ENOTFOUND, "pk_autotune_lookup: group %d: unknown robot", g);
    auto &C = g_sched[ctx];
    auto it = C.tuned.find(tune_key(ctx, n_groups, groups, opt));
    if (it == C.tuned.end()) return fail(ctx, PK_ENOTFOUND, "pk_autotune_lookup: no entry");
    *found = it->second.s;
    if (ms) *ms = it->second.ms;
    return PK_OK;
}

}  // extern "C"
