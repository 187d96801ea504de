// IK-Beam (Sec. V-C, runtime analysis): a beam search over the batched LM
// solver.  Per target, every seed runs a short LM stage; the survivors (one
// wavefront ranks a target's seeds) restart LM from their joints; the first
// survivor result in the same order is returned.  Four launches on one
// stream, no host synchronisation: LM, rank-and-gather, LM, pick.
#include <string.h>

#include <type_traits>

#include "pk_ctx.hpp"
#include "pk_device.hpp"

namespace pk {
namespace {

constexpr int BEAM_MAX_SEEDS = 64;   // one wavefront ranks one target's seeds
constexpr int BEAM_TARGETS_PER_BLOCK = 4;

// Survivor order: within tolerance first; then total cost (within) or
// pose-only cost (not), a NaN after every number; then the lower index.
PK_DEV bool beam_before(bool conv_a, float va, int ka, bool conv_b, float vb, int kb)
{
    if (conv_a != conv_b) return conv_a;
    const bool na = va != va, nb = vb != vb;
    if (na != nb) return nb;
    if (!na && va != vb) return va < vb;
    return ka < kb;
}

PK_DEV float beam_value(const int32_t *status, const float *cost, const float *pcost, int64_t p,
                        bool &conv)
{
    conv = (status[p] & 0xff) == PK_CONVERGED;
    return conv ? cost[p] : pcost[p];
}

// One wavefront per target: lane k holds seed k, counts the seeds ordered
// before it (its rank) and, if the rank is below `keep`, writes its index to
// kept[t][rank] and its joints to the stage-1 seeds.  Ranks are distinct
// because the order is total.
__global__ __launch_bounds__(256) void beam_rank_kernel(int64_t T, int K, int keep, int n,
                                                        const int32_t *__restrict__ status,
                                                        const float *__restrict__ cost,
                                                        const float *__restrict__ pcost,
                                                        const float *__restrict__ joints,
                                                        int32_t *__restrict__ kept,
                                                        float *__restrict__ seeds1)
{
    __shared__ float sv[BEAM_TARGETS_PER_BLOCK][BEAM_MAX_SEEDS];
    __shared__ int sc[BEAM_TARGETS_PER_BLOCK][BEAM_MAX_SEEDS];
    const int w = threadIdx.x >> 6, k = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * BEAM_TARGETS_PER_BLOCK + w;
    const bool live = t < T && k < K;
    bool conv = false;
    float v = 0.f;
    if (live) v = beam_value(status, cost, pcost, t * K + k, conv);
    sv[w][k] = v;
    sc[w][k] = conv ? 1 : 0;
    __syncthreads();
    if (!live) return;
    int rank = 0;
    for (int u = 0; u < K; ++u)
        if (u != k && beam_before(sc[w][u] != 0, sv[w][u], u, conv, v, k)) ++rank;
    if (rank >= keep) return;
    const int64_t N0 = T * K, N1 = T * keep, dst = t * keep + rank;
    kept[dst] = k;
    for (int j = 0; j < n; ++j) seeds1[(int64_t)j * N1 + dst] = joints[(int64_t)j * N0 + t * K + k];
}

struct PickArgs {
    int64_t T;
    int keep, n, m;
    const int32_t *kept, *status;
    const float *cost, *pcost, *joints, *pos_err, *rot_err;
    float *best_joints, *best_pos, *best_rot, *best_cost;
    int32_t *best_index, *success;
};

// Per target: the first of its `keep` stage-1 results in the survivor order.
__global__ __launch_bounds__(256) void beam_pick_kernel(PickArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.T) return;
    const int64_t N1 = a.T * a.keep, base = t * a.keep;
    int b = 0;
    bool cb;
    float vb = beam_value(a.status, a.cost, a.pcost, base, cb);
    for (int r = 1; r < a.keep; ++r) {
        bool c;
        const float v = beam_value(a.status, a.cost, a.pcost, base + r, c);
        if (beam_before(c, v, r, cb, vb, b)) {
            b = r;
            cb = c;
            vb = v;
        }
    }
    const int64_t p = base + b;
    for (int j = 0; j < a.n; ++j) a.best_joints[(int64_t)j * a.T + t] = a.joints[(int64_t)j * N1 + p];
    if (a.best_index) a.best_index[t] = a.kept[p];
    if (a.success) a.success[t] = cb ? 1 : 0;
    if (a.best_cost) a.best_cost[t] = a.cost[p];
    for (int e = 0; e < a.m; ++e) {
        if (a.best_pos) a.best_pos[(int64_t)e * a.T + t] = a.pos_err[(int64_t)e * N1 + p];
        if (a.best_rot) a.best_rot[(int64_t)e * a.T + t] = a.rot_err[(int64_t)e * N1 + p];
    }
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace
}  // namespace pk

using namespace pk;

extern "C" int pk_ik_beam(pk_ctx *ctx, int32_t robot_id, int64_t T, const float *targets,
                          const float *seeds, const pk_cost_weights *w, const pk_lm_options *opt,
                          const pk_beam_schedule *sch, const pk_beam_outputs *out, void *stream)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_ik_beam: ctx is NULL");
    RobotEntry *rb = robot_of(ctx, robot_id);
    if (!rb) return fail(ctx, PK_ENOTFOUND, "pk_ik_beam: unknown robot %d", robot_id);
    if (!w || !opt || !sch || !out) return fail(ctx, PK_EINVAL, "pk_ik_beam: NULL argument");
    const int K = sch->n_seeds, keep = sch->keep;
    if (K < 1 || K > BEAM_MAX_SEEDS || keep < 1 || keep > K || sch->iters0 < 0 || sch->iters1 < 0)
        return fail(ctx, PK_EINVAL, "pk_ik_beam: schedule n_seeds=%d keep=%d iters0=%d iters1=%d "
                    "(need 1 <= keep <= n_seeds <= %d, iterations >= 0)", K, keep, sch->iters0,
                    sch->iters1, BEAM_MAX_SEEDS);
    if (T < 0) return fail(ctx, PK_EINVAL, "pk_ik_beam: T < 0");
    if (T == 0) return PK_OK;
    if (!targets || !seeds || !out->best_joints)
        return fail(ctx, PK_EINVAL, "pk_ik_beam: NULL targets/seeds/best_joints");
    const int64_t N0 = T * K, N1 = T * keep;
    if (N0 >= (int64_t)1 << 31) return fail(ctx, PK_EUNSUPPORTED, "pk_ik_beam: %lld problems, limit 2^31 - 1", (long long)N0);
    pk_lm_options o0 = *opt, o1 = *opt;
    o0.max_iters = sch->iters0;
    o1.max_iters = sch->iters1;
    o0.target_exit = o1.target_exit = 0;   // the beam ranks every seed's cost
    SolveParams P0, P1;
    int v0 = 0, v1 = 0;
    int rc = prepare_solve(ctx, *rb, w, &o0, P0, v0);
    if (rc) return rc;
    rc = prepare_solve(ctx, *rb, w, &o1, P1, v1);
    if (rc) return rc;
    const int n = rb->host.nv, m = rb->host.m;
    PK_HIP(ctx, hipSetDevice(ctx->device));

    // Workspace (4-byte words) for whatever the caller did not provide.
    size_t words = 0;
    auto need = [&](bool given, size_t count) { if (!given) words += count; };
    need(out->stage0_joints, (size_t)N0 * n);
    need(out->stage0_cost, N0);
    need(out->stage0_pose_cost, N0);
    need(out->stage0_status, N0);
    need(out->kept, N1);
    need(false, (size_t)N1 * n);                 // stage-1 seeds
    need(out->stage1_joints, (size_t)N1 * n);
    need(out->stage1_cost, N1);
    need(out->stage1_pose_cost, N1);
    need(out->stage1_status, N1);
    need(false, (size_t)N1 * m * 2);             // stage-1 errors
    if (words * 4 > ctx->ws3_bytes) {
        if (ctx->ws3) (void)hipFree(ctx->ws3);
        ctx->ws3 = nullptr;
        ctx->ws3_bytes = 0;
        if (hipMalloc(&ctx->ws3, words * 4) != hipSuccess)
            return fail(ctx, PK_ENOMEM, "pk_ik_beam: workspace of %zu bytes", words * 4);
        ctx->ws3_bytes = words * 4;
    }
    float *f = (float *)ctx->ws3;
    auto take = [&](auto *given, size_t count) {
        using Tp = std::remove_pointer_t<decltype(given)>;
        if (given) return given;
        Tp *p = (Tp *)f;
        f += count;
        return p;
    };
    float *joints0 = take(out->stage0_joints, (size_t)N0 * n);
    float *cost0 = take(out->stage0_cost, N0);
    float *pcost0 = take(out->stage0_pose_cost, N0);
    int32_t *status0 = take(out->stage0_status, N0);
    int32_t *kept = take(out->kept, N1);
    float *seeds1 = take((float *)nullptr, (size_t)N1 * n);
    float *joints1 = take(out->stage1_joints, (size_t)N1 * n);
    float *cost1 = take(out->stage1_cost, N1);
    float *pcost1 = take(out->stage1_pose_cost, N1);
    int32_t *status1 = take(out->stage1_status, N1);
    float *pos1 = take((float *)nullptr, (size_t)N1 * m);
    float *rot1 = take((float *)nullptr, (size_t)N1 * m);

    hipStream_t s = (hipStream_t)stream;
    // Stage 0: every seed.
    P0.K = K; P0.N = N0; P0.T = T;
    P0.targets = targets; P0.seeds = seeds;
    P0.joints = joints0; P0.cost = cost0; P0.pose_cost = pcost0; P0.status = status0;
    PK_HIP(ctx, launch_lm(*rb, P0, v0, s));
    // Survivors -> stage-1 seeds.
    hipLaunchKernelGGL(beam_rank_kernel, dim3(nblk(T, BEAM_TARGETS_PER_BLOCK)),
                       dim3(64 * BEAM_TARGETS_PER_BLOCK), 0, s, T, K, keep, n,
                       (const int32_t *)status0, (const float *)cost0, (const float *)pcost0,
                       (const float *)joints0, kept, seeds1);
    PK_HIP(ctx, hipGetLastError());
    // Stage 1: the survivors, LM started afresh.
    P1.K = keep; P1.N = N1; P1.T = T;
    P1.targets = targets; P1.seeds = seeds1;
    P1.joints = joints1; P1.cost = cost1; P1.pose_cost = pcost1; P1.status = status1;
    P1.pos_err = pos1; P1.rot_err = rot1;
    PK_HIP(ctx, launch_lm(*rb, P1, v1, s));
    PickArgs a;
    a.T = T; a.keep = keep; a.n = n; a.m = m;
    a.kept = kept; a.status = status1; a.cost = cost1; a.pcost = pcost1; a.joints = joints1;
    a.pos_err = pos1; a.rot_err = rot1;
    a.best_joints = out->best_joints; a.best_pos = out->pos_err; a.best_rot = out->rot_err;
    a.best_cost = out->cost; a.best_index = out->best_index; a.success = out->target_success;
    hipLaunchKernelGGL(beam_pick_kernel, dim3(nblk(T, 256)), dim3(256), 0, s, a);
    PK_HIP(ctx, hipGetLastError());
    return PK_OK;
}
