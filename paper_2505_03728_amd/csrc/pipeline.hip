// Learned seeds + LM refinement, a restart of the unsolved targets' problems
// from their refined joints, and a random-seed LM fallback on the targets
// still unsolved.  Everything stays on the device: each later pass's
// problems are compacted into an active list that a persistent LM launch
// (wavefronts popping items from a device queue) reads, so the host never
// synchronises and a pass costs what its listed problems cost.
#include <string.h>

#include <algorithm>

#include "pk_ctx.hpp"
#include "pk_device.hpp"

namespace pk {
namespace {

__global__ void fill_i32_kernel(int64_t count, int32_t v, int32_t *p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// Targets not solved (success[t] == 0) -> active problem list of a later
// pass (Kf problems per target, problem t * Kf + k).
__global__ void fallback_list_kernel(int64_t T, int Kf, const int32_t *__restrict__ success,
                                     int32_t *count_t, int32_t *count_p, int32_t *active)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T || success[t]) return;
    const int pos = atomicAdd(count_t, 1);
    atomicAdd(count_p, Kf);
    for (int k = 0; k < Kf; ++k) active[(int64_t)pos * Kf + k] = (int32_t)(t * Kf + k);
}

// Fallback stage [c0, c1) of every target's Kf random seeds.  Stage 0 lists
// the targets the earlier passes left unsolved; a later stage lists those
// that ran the previous stage [cp, c0) and got no converged problem from it.
// done[t] counts the target's fallback seeds run so far.
__global__ void fallback_stage_kernel(int64_t T, int Kf, int cp, int c0, int c1,
                                      const int32_t *__restrict__ success,
                                      const int32_t *__restrict__ status, int32_t *done,
                                      int32_t *count_t, int32_t *count_p, int32_t *count_stage,
                                      int32_t *active)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    if (c0 == 0) {
        if (success[t]) {
            done[t] = 0;
            return;
        }
    } else {
        if (done[t] != c0) return;
        for (int k = cp; k < c0; ++k)
            if ((status[t * Kf + k] & 0xff) == PK_CONVERGED) return;
    }
    done[t] = c1;
    const int w = c1 - c0;
    const int pos = atomicAdd(count_stage, w);
    if (count_t) atomicAdd(count_t, 1);
    atomicAdd(count_p, w);
    for (int k = 0; k < w; ++k) active[pos + k] = (int32_t)(t * Kf + c0 + k);
}

struct MergeArgs {
    int64_t T;
    int K, Kf, n, refine_its;
    const int32_t *best_a, *succ_a, *succ_r, *itt_a;
    const float *joints_a;
    const int32_t *status_b, *itt_b, *done_b;
    const float *cost_b, *pcost_b, *joints_b;
    float *best_joints;
    int32_t *success, *source, *itt;
};

__global__ void merge_kernel(MergeArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.T) return;
    const int64_t NA = a.T * a.K, NB = a.T * a.Kf;
    int src = -1, it = -1;
    // pass A (learned seeds), or its restart: best_a / itt_a then hold the
    // restart's values for the targets that were restarted
    const bool restarted = a.succ_r && !a.succ_a[t];
    if (a.succ_a[t] || (restarted && a.succ_r[t])) {
        src = restarted ? 2 : 0;
        const int b = a.best_a[t];
        for (int j = 0; j < a.n; ++j) a.best_joints[(int64_t)j * a.T + t] = a.joints_a[(int64_t)j * NA + t * a.K + b];
        for (int k = 0; k < a.K; ++k) {
            const int v = a.itt_a[t * a.K + k];
            if (v >= 0 && (it < 0 || v < it)) it = v;
        }
        if (restarted) it += a.refine_its;
    } else if (a.Kf > 0) {
        // the fallback seeds this target ran (every stage up to its first
        // converged problem)
        const int kr = a.done_b[t];
        bool any;
        const int b = best_of_k_pick(a.status_b, a.cost_b, a.pcost_b, t * a.Kf, kr, any);
        for (int j = 0; j < a.n; ++j) a.best_joints[(int64_t)j * a.T + t] = a.joints_b[(int64_t)j * NB + t * a.Kf + b];
        if (any) {
            src = 1;
            for (int k = 0; k < kr; ++k) {
                const int v = a.itt_b[t * a.Kf + k];
                if (v >= 0 && (it < 0 || v < it)) it = v;
            }
        }
    } else {
        const int b = a.best_a[t];
        for (int j = 0; j < a.n; ++j) a.best_joints[(int64_t)j * a.T + t] = a.joints_a[(int64_t)j * NA + t * a.K + b];
    }
    if (a.success) a.success[t] = src >= 0 ? 1 : 0;
    if (a.source) a.source[t] = src;
    if (a.itt) a.itt[t] = it;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace
}  // namespace pk

using namespace pk;

extern "C" int pk_ik_solve_seeded(pk_ctx *ctx, int32_t robot_id, int64_t T, const float *targets,
                                  const pk_cost_weights *w, const pk_seeded_options *o,
                                  const pk_seeded_outputs *out, void *stream)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_ik_solve_seeded: ctx is NULL");
    RobotEntry *rb = robot_of(ctx, robot_id);
    if (!rb) return fail(ctx, PK_ENOTFOUND, "pk_ik_solve_seeded: unknown robot %d", robot_id);
    if (!w || !o || !out) return fail(ctx, PK_EINVAL, "pk_ik_solve_seeded: NULL argument");
    if (T < 0) return fail(ctx, PK_EINVAL, "pk_ik_solve_seeded: T < 0");
    if (T == 0) return PK_OK;
    if (!targets || !out->best_joints) return fail(ctx, PK_EINVAL, "pk_ik_solve_seeded: NULL targets/best_joints");
    if (o->fallback_K < 0 || (o->fallback_K > 0 && !o->fallback_seeds))
        return fail(ctx, PK_EINVAL, "pk_ik_solve_seeded: fallback seeds missing");
    if (o->fallback_chunk < 0) return fail(ctx, PK_EINVAL, "pk_ik_solve_seeded: fallback_chunk < 0");
    hipStream_t s = (hipStream_t)stream;
    PK_HIP(ctx, hipSetDevice(ctx->device));
    SolveParams PA, PB;
    int va = 0, vb = 0;
    int rc = prepare_solve(ctx, *rb, w, &o->refine, PA, va);
    if (rc) return rc;
    rc = prepare_solve(ctx, *rb, w, &o->fallback, PB, vb);
    if (rc) return rc;
    // Seeds from the network (also validates the seeder / robot pairing).
    int32_t K = 0, srobot = -1;
    {
        // probe K and robot without launching
        rc = seeder_infer_into(ctx, o->seeder_id, targets, 0, nullptr, s, &K, &srobot);
        if (rc) return rc;
    }
    if (srobot != robot_id) return fail(ctx, PK_EINVAL, "pk_ik_solve_seeded: seeder belongs to robot %d", srobot);
    const int n = rb->host.nv, Kf = o->fallback_K;
    const int Kc = o->fallback_chunk > 0 && o->fallback_chunk < Kf ? o->fallback_chunk : Kf;
    const int64_t NA = T * K, NB = T * Kf;
    if (NA >= (int64_t)1 << 31 || NB >= (int64_t)1 << 31)
        return fail(ctx, PK_EUNSUPPORTED, "pk_ik_solve_seeded: too many problems");
    const int R = o->restart_iters;
    if (R < 0) return fail(ctx, PK_EINVAL, "pk_ik_solve_seeded: restart_iters < 0");
    const int wpc = o->persist_waves_per_cu > 0 ? o->persist_waves_per_cu : 8;
    hipDeviceProp_t prop;
    PK_HIP(ctx, hipGetDeviceProperties(&prop, ctx->device));
    const int persist = wpc * prop.multiProcessorCount;
    const int64_t NS = std::max(NA, NB);   // resumable-state words of the persistent passes
    // Workspace layout (4-byte words).
    const size_t words = (size_t)NA * (2 * n + 6) + 4 * T + 16 + (size_t)NB * (n + 6) + 2 * (size_t)NS;
    if (words * 4 > ctx->ws2_bytes) {
        if (ctx->ws2) (void)hipFree(ctx->ws2);
        ctx->ws2 = nullptr;
        ctx->ws2_bytes = 0;
        if (hipMalloc(&ctx->ws2, words * 4) != hipSuccess)
            return fail(ctx, PK_ENOMEM, "pk_ik_solve_seeded: workspace of %zu bytes", words * 4);
        ctx->ws2_bytes = words * 4;
    }
    float *f = (float *)ctx->ws2;
    float *seeds_a = f;                 f += (size_t)NA * n;
    float *joints_a = f;                f += (size_t)NA * n;
    float *cost_a = f;                  f += NA;
    float *pcost_a = f;                 f += NA;
    int32_t *status_a = (int32_t *)f;   f += NA;
    int32_t *itt_a = (int32_t *)f;      f += NA;
    int32_t *spare_a = (int32_t *)f;    f += NA;
    int32_t *best_a = (int32_t *)f;     f += T;
    int32_t *succ_a = (int32_t *)f;     f += T;
    int32_t *succ_r = (int32_t *)f;     f += T;
    int32_t *list_r = (int32_t *)f;     f += NA;
    int32_t *done_b = (int32_t *)f;     f += T;
    // [0..1] fallback targets and problems, [2..3] restart list, [4] queue
    // head, [5] problems of the current fallback stage
    int32_t *counters = (int32_t *)f;   f += 16;
    float *st_lambda = f;               f += NS;
    int32_t *st_state = (int32_t *)f;   f += NS;
    float *joints_b = f;                f += (size_t)NB * n;
    float *cost_b = f;                  f += NB;
    float *pcost_b = f;                 f += NB;
    int32_t *status_b = (int32_t *)f;   f += NB;
    int32_t *itt_b = (int32_t *)f;      f += NB;
    int32_t *active = (int32_t *)f;     f += NB;
    (void)spare_a;

    rc = seeder_infer_into(ctx, o->seeder_id, targets, T, seeds_a, s, nullptr, nullptr);
    if (rc) return rc;
    // Pass A: LM from the learned seeds.
    PA.K = K; PA.N = NA; PA.T = T;
    PA.targets = targets; PA.seeds = seeds_a;
    PA.joints = joints_a; PA.cost = cost_a; PA.pose_cost = pcost_a; PA.status = status_a;
    PA.iters = out->refine_iters; PA.accepts = out->refine_accepts; PA.iters_to_tol = itt_a;
    if (o->refine_iters_per_launch > 0) {
        // Persistent, compacted schedule (same per-problem results).
        pk_ik_group g;
        memset(&g, 0, sizeof g);
        g.robot_id = robot_id;
        g.problem.n_targets = T;
        g.problem.K = K;
        g.problem.targets = targets;
        g.problem.seeds = seeds_a;
        g.weights = *w;
        g.out.joints = joints_a;
        g.out.cost = cost_a;
        g.out.iters = out->refine_iters;
        g.out.accepts = out->refine_accepts;
        g.out.status = status_a;
        g.out.iters_to_tol = itt_a;
        g.out.best_index = best_a;
        g.out.target_success = succ_a;
        pk_sched_options so;
        memset(&so, 0, sizeof so);
        so.iters_per_launch = o->refine_iters_per_launch;
        so.waves_per_cu = o->refine_blocks_per_cu > 0 ? o->refine_blocks_per_cu : 4;
        so.workgroup_size = 64;
        so.use_graph = 1;
        rc = sched_run(ctx, 1, &g, &o->refine, so, s);
        if (rc) return rc;
    } else if (va == PK_VARIANT_LANE && 64 % K == 0) {
        const BestOut B{best_a, nullptr, succ_a};   // best-of-K in the same launch
        PK_HIP(ctx, launch_lm(*rb, PA, va, s, 0, &B));
    } else {
        PK_HIP(ctx, launch_lm(*rb, PA, va, s));
        PK_HIP(ctx, launch_best_of_k(PA, n, best_a, nullptr, succ_a, s));
    }
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, (int64_t)16, 0, counters);
    // Pass A': the K problems of each unsolved target again from their
    // refined joints (lambda back at lambda0), in place, then best-of-K again.
    const int32_t *succ_now = succ_a;
    if (R > 0) {
        if (out->restart_iters)
            hipLaunchKernelGGL(fill_i32_kernel, dim3(nblk(NA, 256)), dim3(256), 0, s, NA, 0, out->restart_iters);
        if (out->restart_accepts)
            hipLaunchKernelGGL(fill_i32_kernel, dim3(nblk(NA, 256)), dim3(256), 0, s, NA, 0, out->restart_accepts);
        hipLaunchKernelGGL(fallback_list_kernel, dim3(nblk(T, 256)), dim3(256), 0, s, T, K, succ_a,
                           counters + 2, counters + 3, list_r);
        SolveParams PR = PA;
        PR.max_iters = R;
        PR.seeds = joints_a;            // each problem reads its joints before writing them
        PR.iters = out->restart_iters; PR.accepts = out->restart_accepts;
        PR.active = list_r; PR.n_active = counters + 3;
        PR.st_lambda = st_lambda; PR.st_state = st_state;
        PR.resume = 0; PR.iter_budget = R;
        PR.queue_head = counters + 4;
        PK_HIP(ctx, launch_lm(*rb, PR, va, s, persist));
        PK_HIP(ctx, launch_best_of_k(PA, n, best_a, nullptr, succ_r, s));
        succ_now = succ_r;
    }
    // Pass B: random seeds on the targets still unsolved.
    if (Kf > 0) {
        if (out->fallback_iters)
            hipLaunchKernelGGL(fill_i32_kernel, dim3(nblk(NB, 256)), dim3(256), 0, s, NB, 0, out->fallback_iters);
        if (out->fallback_accepts)
            hipLaunchKernelGGL(fill_i32_kernel, dim3(nblk(NB, 256)), dim3(256), 0, s, NB, 0, out->fallback_accepts);
        PB.K = Kf; PB.N = NB; PB.T = T;
        PB.targets = targets; PB.seeds = o->fallback_seeds;
        PB.joints = joints_b; PB.cost = cost_b; PB.pose_cost = pcost_b; PB.status = status_b;
        PB.iters = out->fallback_iters; PB.accepts = out->fallback_accepts; PB.iters_to_tol = itt_b;
        PB.active = active; PB.n_active = counters + 5;
        PB.st_lambda = st_lambda; PB.st_state = st_state;
        PB.resume = 0; PB.iter_budget = PB.max_iters;
        PB.queue_head = counters + 4;
        for (int cp = 0, c0 = 0; c0 < Kf; cp = c0, c0 += Kc) {
            const int c1 = std::min(Kf, c0 + Kc);
            hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, (int64_t)2, 0, counters + 4);
            hipLaunchKernelGGL(fallback_stage_kernel, dim3(nblk(T, 256)), dim3(256), 0, s, T, Kf, cp, c0,
                               c1, succ_now, status_b, done_b, c0 == 0 ? counters : nullptr, counters + 1,
                               counters + 5, active);
            PK_HIP(ctx, hipGetLastError());
            PK_HIP(ctx, launch_lm(*rb, PB, vb, s, persist));
        }
    }
    MergeArgs m;
    m.T = T; m.K = K; m.Kf = Kf; m.n = n; m.refine_its = o->refine.max_iters;
    m.best_a = best_a; m.succ_a = succ_a; m.succ_r = R > 0 ? succ_r : nullptr; m.itt_a = itt_a;
    m.joints_a = joints_a;
    m.status_b = status_b; m.itt_b = itt_b; m.done_b = done_b; m.cost_b = cost_b; m.pcost_b = pcost_b; m.joints_b = joints_b;
    m.best_joints = out->best_joints; m.success = out->target_success; m.source = out->source;
    m.itt = out->iters_to_tol;
    hipLaunchKernelGGL(merge_kernel, dim3(nblk(T, 256)), dim3(256), 0, s, m);
    PK_HIP(ctx, hipGetLastError());
    if (out->n_fallback)
        PK_HIP(ctx, hipMemcpyAsync(out->n_fallback, counters, 4, hipMemcpyDeviceToDevice, s));
    if (out->n_restart)
        PK_HIP(ctx, hipMemcpyAsync(out->n_restart, counters + 2, 4, hipMemcpyDeviceToDevice, s));
    if (out->n_fallback_problems)
        PK_HIP(ctx, hipMemcpyAsync(out->n_fallback_problems, counters + 1, 4, hipMemcpyDeviceToDevice, s));
    return PK_OK;
}
