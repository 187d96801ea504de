// Batched forward kinematics, residual/Jacobian (parity entry points) and
// the best-of-K selection.  One problem per thread, any tree up to
// PK_MAX_JOINTS joints; frames live in per-thread arrays.  The per-joint and
// per-EE arithmetic is the same device code the LM kernels run.
#include <math.h>

#include "pk_device.hpp"

namespace pk {
namespace {

// Value of joint j for problem p (SoA q over the variables): its variable,
// or a mimic joint's rule on its driver's.
PK_DEV float joint_value(const RobotC *__restrict__ rb, const float *q, int64_t N, int64_t p, int j)
{
    const JointC &J = rb->j[j];
    if (J.mimic_src < 0) return q[(int64_t)J.var * N + p];
    return J.mimic_a * q[(int64_t)rb->j[J.mimic_src].var * N + p] + J.mimic_b;
}

// FK of every joint of problem p (SoA q): O[j], pos[j].
PK_DEV void fk_all(const RobotC *__restrict__ rb, const float *q, int64_t N, int64_t p,
                   float (*O)[9], float (*pos)[3])
{
    const int n = rb->n;
    for (int j = 0; j < n; ++j) {
        const int par = rb->j[j].parent;
        float Ob[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f}, pb[3] = {0.f, 0.f, 0.f};
        const float *Op = par < 0 ? Ob : O[par];
        const float *pp = par < 0 ? pb : pos[par];
        const float qj = joint_value(rb, q, N, p, j);
        const bool pri = rb->j[j].type == PK_JOINT_PRISMATIC;
        float s = 0.f, c = 1.f;
        if (!pri) joint_sincos(qj, s, c);
        joint_step(Op, pp, rb->j[j].G, rb->j[j].t, s, c, O[j], pos[j]);
        if (pri) joint_slide(O[j], qj, pos[j]);
    }
}

__global__ __launch_bounds__(64) void fk_kernel(const RobotC *__restrict__ rb, int64_t N,
                                                const float *__restrict__ q, float *ee_pose,
                                                float *joint_frames)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    float O[PK_MAX_JOINTS][9], pos[PK_MAX_JOINTS][3];
    fk_all(rb, q, N, p, O, pos);
    const int n = rb->n, m = rb->m;
    if (joint_frames) {
        for (int j = 0; j < n; ++j) {
            const int v = rb->j[j].var;   // frames of the variables' joints
            if (v < 0) continue;
            float R[9];
            mm3(O[j], rb->j[j].Ut, R);   // paper frame R_j = O_j U_j^T
            for (int u = 0; u < 9; ++u) joint_frames[((int64_t)v * 12 + u) * N + p] = R[u];
            for (int u = 0; u < 3; ++u) joint_frames[((int64_t)v * 12 + 9 + u) * N + p] = pos[j][u];
        }
    }
    for (int k = 0; k < m; ++k) {
        const int e = rb->e[k].joint;
        float R[9], pe[3], w, x, y, z;
        ee_frame(O[e], pos[e], rb->e[k].G, rb->e[k].t, R, pe);
        rot_to_quat(R, w, x, y, z);
        const float v[7] = {pe[0], pe[1], pe[2], w, x, y, z};
        for (int u = 0; u < 7; ++u) ee_pose[((int64_t)k * 7 + u) * N + p] = v[u];
    }
}

__global__ __launch_bounds__(64) void resjac_kernel(const RobotC *__restrict__ rb, int64_t N,
                                                    int32_t K, const float *__restrict__ targets,
                                                    const float *__restrict__ q, SolveParams P,
                                                    float *r, float *J)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t T = N / K, t = p / K;
    float O[PK_MAX_JOINTS][9], pos[PK_MAX_JOINTS][3];
    fk_all(rb, q, N, p, O, pos);
    // Columns per variable; a mimic joint's column adds into its driver's.
    const int n = rb->n, m = rb->m, nv = rb->nv;
    const int rows = rb->pose_rows + 2 * nv;
    if (J)
        for (int row = 0; row < rows; ++row)
            for (int v = 0; v < nv; ++v) J[((int64_t)row * nv + v) * N + p] = 0.f;
    for (int k = 0; k < m; ++k) {
        const EEC &E = rb->e[k];
        float Re[9], pe[3], d[3], tp[7];
        ee_frame(O[E.joint], pos[E.joint], E.G, E.t, Re, pe);
        const int W = E.kind == PK_EE_POSE ? 7 : 3;
        for (int u = 0; u < W; ++u) tp[u] = targets[(int64_t)(E.tgt_off + u) * T + t];
        for (int u = 0; u < 3; ++u) d[u] = pe[u] - tp[u];
        const int row0 = E.row_off;
        if (E.kind == PK_EE_POSE) {
            float Rt[9], M[9], Nb[9];
            quat_to_rot(tp[3], tp[4], tp[5], tp[6], Rt);
            PoseLog lg = pose_log(Rt, Re, d);
            for (int u = 0; u < 3; ++u) {
                r[(int64_t)(row0 + u) * N + p] = P.w_pos * lg.rho[u];
                r[(int64_t)(row0 + 3 + u) * N + p] = P.w_rot * lg.phi[u];
            }
            if (J) {
                jr_inv_blocks(lg, Re, M, Nb);
                for (int j = 0; j < n; ++j) {
                    if (!((rb->anc[k] >> j) & 1ull)) continue;
                    const int ms = rb->j[j].mimic_src;
                    const int c = ms < 0 ? rb->j[j].var : rb->j[ms].var;
                    const float f = ms < 0 ? 1.f : rb->j[j].mimic_a;
                    const float om[3] = {O[j][2], O[j][5], O[j][8]};
                    float v[3], wv[3];
                    joint_twist(rb->j[j].type == PK_JOINT_PRISMATIC, om, pos[j], pe, v, wv);
                    for (int u = 0; u < 3; ++u) {
                        float mv = M[3 * u] * v[0] + M[3 * u + 1] * v[1] + M[3 * u + 2] * v[2];
                        float nw = Nb[3 * u] * wv[0] + Nb[3 * u + 1] * wv[1] + Nb[3 * u + 2] * wv[2];
                        float mw = M[3 * u] * wv[0] + M[3 * u + 1] * wv[1] + M[3 * u + 2] * wv[2];
                        J[((int64_t)(row0 + u) * nv + c) * N + p] += f * (P.w_pos * (mv + nw));
                        J[((int64_t)(row0 + 3 + u) * nv + c) * N + p] += f * (P.w_rot * mw);
                    }
                }
            }
        } else {
            for (int u = 0; u < 3; ++u) r[(int64_t)(row0 + u) * N + p] = P.w_pos * d[u];
            if (J) {
                for (int j = 0; j < n; ++j) {
                    if (!((rb->anc[k] >> j) & 1ull)) continue;
                    const int ms = rb->j[j].mimic_src;
                    const int c = ms < 0 ? rb->j[j].var : rb->j[ms].var;
                    const float f = ms < 0 ? 1.f : rb->j[j].mimic_a;
                    const float om[3] = {O[j][2], O[j][5], O[j][8]};
                    float v[3], wv[3];
                    joint_twist(rb->j[j].type == PK_JOINT_PRISMATIC, om, pos[j], pe, v, wv);
                    for (int u = 0; u < 3; ++u) J[((int64_t)(row0 + u) * nv + c) * N + p] += f * (P.w_pos * v[u]);
                }
            }
        }
    }
    // limit and rest rows, one per variable
    const int lr = rb->pose_rows, rr = lr + nv;
    for (int j = 0; j < n; ++j) {
        const int v = rb->j[j].var;
        if (v < 0) continue;
        const float qj = q[(int64_t)v * N + p];
        const float qrj = P.q_rest ? P.q_rest[v] : rb->j[j].mid;
        const float over = qj - rb->j[j].hi, under = rb->j[j].lo - qj;
        r[(int64_t)(lr + v) * N + p] = P.w_limit * (fmaxf(over, 0.f) + fmaxf(under, 0.f));
        r[(int64_t)(rr + v) * N + p] = P.w_rest * (qj - qrj);
        if (J) {
            J[((int64_t)(lr + v) * nv + v) * N + p] =
                over > 0.f ? P.w_limit : (under > 0.f ? -P.w_limit : 0.f);
            J[((int64_t)(rr + v) * nv + v) * N + p] = P.w_rest;
        }
    }
}

// Best of K per target (rule: lowest total cost among converged seeds, else
// lowest pose-only cost; ties to the lower index).
__global__ __launch_bounds__(256) void best_of_k_kernel(int64_t T, int32_t K, int n, int64_t N,
                                                        const int32_t *__restrict__ status,
                                                        const float *__restrict__ cost,
                                                        const float *__restrict__ pcost,
                                                        const float *__restrict__ joints,
                                                        int32_t *best_index, float *best_joints,
                                                        int32_t *success)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    bool any;
    const int b = best_of_k_pick(status, cost, pcost, t * K, K, any);
    if (best_index) best_index[t] = b;
    if (success) success[t] = any ? 1 : 0;
    if (best_joints)
        for (int j = 0; j < n; ++j) best_joints[(int64_t)j * T + t] = joints[(int64_t)j * N + t * K + b];
}

}  // namespace

hipError_t launch_fk(const RobotC *rb, int64_t N, const float *q, float *ee_pose,
                     float *joint_frames, hipStream_t s)
{
    const int block = 64;
    hipLaunchKernelGGL(fk_kernel, dim3((unsigned)((N + block - 1) / block)), dim3(block), 0, s,
                       rb, N, q, ee_pose, joint_frames);
    return hipGetLastError();
}

hipError_t launch_residual_jacobian(const RobotC *rb, int64_t N, int32_t K, const float *targets,
                                    const float *q, const SolveParams &P, float *r, float *J,
                                    hipStream_t s)
{
    const int block = 64;
    hipLaunchKernelGGL(resjac_kernel, dim3((unsigned)((N + block - 1) / block)), dim3(block), 0, s,
                       rb, N, K, targets, q, P, r, J);
    return hipGetLastError();
}

hipError_t launch_best_of_k(const SolveParams &P, int n, int32_t *best_index, float *best_joints,
                            int32_t *success, hipStream_t s)
{
    const int block = 256;
    hipLaunchKernelGGL(best_of_k_kernel, dim3((unsigned)((P.T + block - 1) / block)), dim3(block), 0,
                       s, P.T, P.K, n, P.N, P.status, P.cost, P.pose_cost, P.joints, best_index,
                       best_joints, success);
    return hipGetLastError();
}

}  // namespace pk
