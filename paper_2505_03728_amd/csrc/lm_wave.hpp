// Wave-per-problem Levenberg-Marquardt IK kernel for any revolute tree
// (up to 64 joints, 8 EEs): one problem per 64-lane wavefront, lane j owns
// joint j.
//
//  * FK runs level by level over tree depth; a lane reads its parent's frame
//    with a lane shuffle.
//  * Lane k < m evaluates EE k (pose log, errors, right-Jacobian-inverse
//    blocks); those values are broadcast to all lanes with readlane.
//  * Lane j forms its Jacobian column for every EE it is an ancestor of,
//    then row j of J^T J from the other lanes' columns (readlane).
//  * Right-looking Cholesky with the rows in registers; column k is
//    broadcast with readlane.  The forward solve works on the rows; L is
//    transposed through LDS once for the backward solve.
//  * Decisions (accept/reject, lambda, pivot test, early exit) are uniform
//    across the wave, so the whole LM loop runs without divergence.
//
// Method: Sec. III-A (LM on the sum of squared weighted residuals, limits as
// penalties), Sec. III-B (FK), Sec. III-C (joint pose, limit and rest costs).
#pragma once

#include <math.h>

#include "pk_device.hpp"

namespace pk {
namespace wave {

PK_DEV float bcast(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

PK_DEV double bcast(double v, int lane)
{
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

PK_DEV float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

PK_DEV float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

template <int MMAX>
struct Eval {
    float col[MMAX][6];   // this lane's Jacobian column for each EE (0 if not an ancestor)
    float g;              // (J^T r)_j
    float dl;             // limit-row derivative of joint j
    float cost, pcost;    // uniform
    float perr, rerr;     // EE lane values
    bool meets;           // uniform
};

// Per-lane constants of the joint and EE owned by this lane.
struct LaneConst {
    float G[9], t[3], lo, hi, qr;
    int parent, depth;
    float eG[9], et[3];
    int ee_joint, ee_kind;
    float tp[3], tR[9];   // this lane's EE target
};

template <int MMAX>
PK_DEV void evaluate(const RobotC *__restrict__ rb, const SolveParams &P, const LaneConst &C,
                     int lane, int n, int m, int max_depth, float q, Eval<MMAX> &E)
{
    const bool isj = lane < n, ise = lane < m;
    float s = 0.f, c = 1.f;
    if (isj) joint_sincos(q, s, c);
    // FK, one tree level at a time.
    float O[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f}, pos[3] = {0.f, 0.f, 0.f};
    const int src = C.parent < 0 ? 0 : C.parent;
    for (int d = 0; d <= max_depth; ++d) {
        float Op[9], pp[3];
#pragma unroll
        for (int u = 0; u < 9; ++u) Op[u] = __shfl(O[u], src, 64);
#pragma unroll
        for (int u = 0; u < 3; ++u) pp[u] = __shfl(pos[u], src, 64);
        if (C.depth == d) {
            if (C.parent < 0) {
#pragma unroll
                for (int u = 0; u < 9; ++u) Op[u] = (u % 4 == 0) ? 1.f : 0.f;
                pp[0] = pp[1] = pp[2] = 0.f;
            }
            joint_step(Op, pp, C.G, C.t, s, c, O, pos);
        }
    }
    // EE lanes: frame of the EE joint, residual, errors, J_r^-1 blocks.
    float Oe[9], pj[3];
    const int esrc = ise ? C.ee_joint : 0;
#pragma unroll
    for (int u = 0; u < 9; ++u) Oe[u] = __shfl(O[u], esrc, 64);
#pragma unroll
    for (int u = 0; u < 3; ++u) pj[u] = __shfl(pos[u], esrc, 64);
    float r[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, M[9], Nb[9], pe[3];
    float ecost = 0.f;
    E.perr = 0.f;
    E.rerr = 0.f;
    if (ise) {
        float Re[9], d[3];
        ee_frame(Oe, pj, C.eG, C.et, Re, pe);
#pragma unroll
        for (int u = 0; u < 3; ++u) d[u] = pe[u] - C.tp[u];
        E.perr = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (C.ee_kind == PK_EE_POSE) {
            PoseLog lg = pose_log(C.tR, Re, d);
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                r[u] = P.w_pos * lg.rho[u];
                r[3 + u] = P.w_rot * lg.phi[u];
            }
            E.rerr = lg.theta;
            jr_inv_blocks(lg, Re, M, Nb);
        } else {
#pragma unroll
            for (int u = 0; u < 3; ++u) r[u] = P.w_pos * d[u];
#pragma unroll
            for (int u = 0; u < 9; ++u) M[u] = Nb[u] = 0.f;
        }
#pragma unroll
        for (int u = 0; u < 6; ++u) ecost += r[u] * r[u];
    }
    // Joint lanes: limit and rest rows.
    float jcost = 0.f, rl = 0.f, rr = 0.f;
    E.dl = 0.f;
    if (isj) {
        const float over = q - C.hi, under = C.lo - q;
        rl = P.w_limit * (fmaxf(over, 0.f) + fmaxf(under, 0.f));
        rr = P.w_rest * (q - C.qr);
        E.dl = over > 0.f ? P.w_limit : (under > 0.f ? -P.w_limit : 0.f);
        jcost = rl * rl + rr * rr;
    }
    E.pcost = wave_sum(ecost);
    E.cost = wave_sum(ecost + jcost);
    bool ok = true;
    if (ise) ok = E.perr <= P.tol_pos && (C.ee_kind != PK_EE_POSE || E.rerr <= P.tol_rot);
    E.meets = __all(ok);
    // Jacobian columns of this lane's joint, one per EE.
    const float om[3] = {O[2], O[5], O[8]};
    float g = E.dl * rl + P.w_rest * rr;
#pragma unroll
    for (int k = 0; k < MMAX; ++k) {
#pragma unroll
        for (int u = 0; u < 6; ++u) E.col[k][u] = 0.f;
        if (k < m) {
            const int kind = rb->e[k].kind;
            const bool anc = isj && ((rb->anc[k] >> lane) & 1ull);
            float bpe[3], bM[9], bN[9], br[6];
#pragma unroll
            for (int u = 0; u < 3; ++u) bpe[u] = bcast(pe[u], k);
#pragma unroll
            for (int u = 0; u < 6; ++u) br[u] = bcast(r[u], k);
            float lev[3] = {bpe[0] - pos[0], bpe[1] - pos[1], bpe[2] - pos[2]}, v[3];
            cross(om, lev, v);
            if (kind == PK_EE_POSE) {
#pragma unroll
                for (int u = 0; u < 9; ++u) {
                    bM[u] = bcast(M[u], k);
                    bN[u] = bcast(Nb[u], k);
                }
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    float mv = bM[3 * u] * v[0] + bM[3 * u + 1] * v[1] + bM[3 * u + 2] * v[2];
                    float nw = bN[3 * u] * om[0] + bN[3 * u + 1] * om[1] + bN[3 * u + 2] * om[2];
                    float mw = bM[3 * u] * om[0] + bM[3 * u + 1] * om[1] + bM[3 * u + 2] * om[2];
                    E.col[k][u] = anc ? P.w_pos * (mv + nw) : 0.f;
                    E.col[k][3 + u] = anc ? P.w_rot * mw : 0.f;
                }
            } else {
#pragma unroll
                for (int u = 0; u < 3; ++u) E.col[k][u] = anc ? P.w_pos * v[u] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < 6; ++u) g += E.col[k][u] * br[u];
        }
    }
    E.g = isj ? g : 0.f;
}

// Form row `lane` of A + lambda diag(max(A_jj, floor)) in precision T from
// the Jacobian columns, factor it (rows in registers), and solve for
// delta = -(L L^T)^-1 g.  Returns false if a pivot is not above
// pivot_rel * max diagonal (thresh_rel > 0) or not positive (thresh_rel = 0).
template <int NMAX, int MMAX, typename T>
PK_DEV bool damped_solve(const RobotC *__restrict__ rb, const SolveParams &P, const Eval<MMAX> &E,
                         int lane, int n, int m, float lam, float thresh_rel, T *lds, float &delta)
{
    const bool isj = lane < n;
    T a[NMAX];
    // own diagonal of J^T J (+ limit/rest rows) and the damping term
    T diag = 0;
#pragma unroll
    for (int k = 0; k < MMAX; ++k)
#pragma unroll
        for (int u = 0; u < 6; ++u) diag += (T)E.col[k][u] * (T)E.col[k][u];
    diag += (T)E.dl * (T)E.dl + (T)P.w_rest * (T)P.w_rest;
    const T D = diag > (T)P.damping_floor ? diag : (T)P.damping_floor;
    const T dampd = isj ? diag + (T)lam * D : (T)0;
#pragma unroll
    for (int c = 0; c < NMAX; ++c) {
        T s = 0;
        if (c < n) {
#pragma unroll
            for (int k = 0; k < MMAX; ++k) {
                if (k < m && ((rb->anc[k] >> c) & 1ull)) {
#pragma unroll
                    for (int u = 0; u < 6; ++u) s += (T)E.col[k][u] * (T)bcast(E.col[k][u], c);
                }
            }
        }
        a[c] = (lane == c) ? dampd : s;
    }
    T thresh = 0;
    if (thresh_rel > 0.f) thresh = (T)thresh_rel * (T)wave_max((float)dampd);
    bool ok = true;
    // Right-looking Cholesky; lane i holds row i.
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
        if (k < n) {
            T d = bcast(a[k], k);
            if (!(d > thresh) || !(d < (T)INFINITY)) {
                ok = false;
                d = 1;
            }
            const T lkk = sqrt(d), inv = (T)1 / lkk;
            if (lane > k) a[k] *= inv;
            if (lane == k) a[k] = lkk;
#pragma unroll
            for (int j = k + 1; j < NMAX; ++j) {
                if (j < n) {
                    const T ljk = bcast(a[k], j);
                    if (lane >= j) a[j] -= a[k] * ljk;
                }
            }
        }
    }
    // Forward: L y = -g (lane i ends with y_i).
    T b = isj ? -(T)E.g : (T)0;
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
        if (k < n) {
            const T yk = bcast(b, k) / bcast(a[k], k);
            if (lane > k) b -= a[k] * yk;
            if (lane == k) b = yk;
        }
    }
    // Transpose L through LDS: lane k then holds column k (lt[i] = L_ik).
    if (isj) {
#pragma unroll
        for (int c = 0; c < NMAX; ++c) lds[lane * (NMAX + 1) + c] = a[c];
    }
    __syncthreads();
    T lt[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; ++i) lt[i] = (i < n && isj) ? lds[i * (NMAX + 1) + lane] : (T)0;
    __syncthreads();
    // Backward: L^T x = y.
#pragma unroll
    for (int i = NMAX - 1; i >= 0; --i) {
        if (i < n) {
            const T xi = bcast(b, i) / bcast(lt[i], i);
            if (lane < i) b -= lt[i] * xi;
            if (lane == i) b = xi;
        }
    }
    delta = isj ? (float)b : 0.f;
    return ok;
}

// One LM problem (active index wi) on this wavefront; resumable like the
// per-lane kernel (state in HBM, at most P.iter_budget iterations per launch).
template <int NMAX, int MMAX>
PK_DEV void wave_problem(const RobotC *__restrict__ rb, const SolveParams &P, double *lds_raw,
                         int64_t wi)
{
    const int lane = threadIdx.x;
    const int64_t p = P.active ? (int64_t)P.active[wi] : wi;
    const int64_t N = P.N, T = P.T, t = p / P.K;
    const int n = rb->n, m = rb->m, max_depth = rb->max_depth;
    const bool isj = lane < n, ise = lane < m;
    const bool resumable = P.st_state != nullptr, resume = resumable && P.resume;

    LaneConst C;
    const int jl = isj ? lane : 0, el = ise ? lane : 0;
#pragma unroll
    for (int u = 0; u < 9; ++u) C.G[u] = rb->j[jl].G[u];
#pragma unroll
    for (int u = 0; u < 3; ++u) C.t[u] = rb->j[jl].t[u];
    C.lo = rb->j[jl].lo;
    C.hi = rb->j[jl].hi;
    C.qr = P.q_rest ? P.q_rest[jl] : rb->j[jl].mid;
    C.parent = rb->j[jl].parent;
    C.depth = isj ? rb->j[jl].depth : -1;
#pragma unroll
    for (int u = 0; u < 9; ++u) C.eG[u] = rb->e[el].G[u];
#pragma unroll
    for (int u = 0; u < 3; ++u) C.et[u] = rb->e[el].t[u];
    C.ee_joint = rb->e[el].joint;
    C.ee_kind = rb->e[el].kind;
    bool fin = true;
    float q = 0.f;
    if (isj) {
        q = (resume ? P.joints : P.seeds)[(int64_t)lane * N + p];
        fin = isfinite(q);
    }
    if (ise) {
        const int off = rb->e[el].tgt_off;
        const int W = C.ee_kind == PK_EE_POSE ? 7 : 3;
        float v[7] = {0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f};
        for (int u = 0; u < W; ++u) {
            v[u] = P.targets[(int64_t)(off + u) * T + t];
            fin = fin && isfinite(v[u]);
        }
#pragma unroll
        for (int u = 0; u < 3; ++u) C.tp[u] = v[u];
        quat_to_rot(v[3], v[4], v[5], v[6], C.tR);
    }
    const bool finite = __all(fin);
    if (!finite) {
        if (isj) {
            P.joints[(int64_t)lane * N + p] = q;
            for (int it = 0; it < P.trace_iters; ++it)
                P.trace_q[((int64_t)it * n + lane) * N + p] = q;
        }
        if (ise) {
            if (P.pos_err) P.pos_err[(int64_t)lane * N + p] = NAN;
            if (P.rot_err) P.rot_err[(int64_t)lane * N + p] = NAN;
        }
        if (lane == 0) {
            if (P.cost) P.cost[p] = NAN;
            P.pose_cost[p] = NAN;
            if (P.iters) P.iters[p] = 0;
            if (P.accepts) P.accepts[p] = 0;
            if (P.status) P.status[p] = PK_NONFINITE;
            if (P.iters_to_tol) P.iters_to_tol[p] = -1;
            if (resumable) P.st_state[p] = PK_ST_DONE;
            for (int it = 0; it < P.trace_iters; ++it) P.trace_acc[(int64_t)it * N + p] = 0;
        }
        return;
    }

    Eval<MMAX> E, Et;
    evaluate<MMAX>(rb, P, C, lane, n, m, max_depth, q, E);
    int iters, accepts, itt, flags;
    bool done, stalled;
    float lam;
    if (resume) {
        const int st = P.st_state[p];
        iters = P.iters[p];
        accepts = P.accepts[p];
        itt = P.iters_to_tol[p];
        flags = st & 0xffff;
        stalled = (st & PK_ST_STALLED) != 0;
        done = (st & PK_ST_DONE) != 0;
        lam = P.st_lambda[p];
    } else {
        iters = accepts = flags = 0;
        itt = E.meets ? 0 : -1;
        stalled = false;
        done = P.early_exit && itt == 0;
        lam = P.lambda0;
    }
    const int iter_end = resumable ? min(P.max_iters, iters + P.iter_budget) : P.max_iters;
    while (!done && iters < iter_end) {
        float delta;
        bool ok = damped_solve<NMAX, MMAX, float>(rb, P, E, lane, n, m, lam, P.pivot_rel,
                                                  (float *)lds_raw, delta);
        if (!ok) {
            flags |= PK_FLAG_FP64;
            ok = damped_solve<NMAX, MMAX, double>(rb, P, E, lane, n, m, lam, 0.f, lds_raw, delta);
        }
        float ct = INFINITY;
        const float qt = q + delta;
        if (ok) {
            evaluate<MMAX>(rb, P, C, lane, n, m, max_depth, qt, Et);
            ct = Et.cost;
        }
        ++iters;
        const bool acc = ct < E.cost;
        if (acc) {
            q = qt;
            E = Et;
            lam = fmaxf(lam / P.nu_down, P.lambda_min);
            ++accepts;
            if (E.meets) {
                if (itt < 0) itt = iters;
                if (P.early_exit) done = true;
            }
        } else {
            if (lam >= P.lambda_max) {
                stalled = true;
                done = true;
            }
            lam = fminf(lam * P.nu_up, P.lambda_max);
        }
        if (iters - 1 < P.trace_iters) {
            if (isj) P.trace_q[((int64_t)(iters - 1) * n + lane) * N + p] = q;
            if (lane == 0) P.trace_acc[(int64_t)(iters - 1) * N + p] = acc ? 1 : 0;
        }
    }
    const bool finished = done || iters >= P.max_iters;
    if (finished)
        for (int it = iters; it < P.trace_iters; ++it) {
            if (isj) P.trace_q[((int64_t)it * n + lane) * N + p] = q;
            if (lane == 0) P.trace_acc[(int64_t)it * N + p] = 0;
        }
    if (isj) P.joints[(int64_t)lane * N + p] = q;
    if (ise) {
        if (P.pos_err) P.pos_err[(int64_t)lane * N + p] = E.perr;
        if (P.rot_err) P.rot_err[(int64_t)lane * N + p] = E.rerr;
    }
    if (lane == 0) {
        if (P.cost) P.cost[p] = E.cost;
        P.pose_cost[p] = E.pcost;
        if (P.iters) P.iters[p] = iters;
        if (P.accepts) P.accepts[p] = accepts;
        if (P.status)
            P.status[p] = (E.meets ? PK_CONVERGED : (stalled ? PK_STALLED : PK_MAX_ITERS)) | flags;
        if (P.iters_to_tol) P.iters_to_tol[p] = itt;
        if (resumable) {
            P.st_lambda[p] = lam;
            P.st_state[p] = flags | (stalled ? PK_ST_STALLED : 0) | (finished ? PK_ST_DONE : 0);
        }
    }
}

PK_DEV int64_t pop_item_wave(int32_t *head)
{
    int v = 0;
    if (threadIdx.x == 0) v = atomicAdd(head, 1);
    return (int64_t)__shfl(v, 0, 64);
}

template <int NMAX, int MMAX>
__global__ __launch_bounds__(64) void lm_wave_kernel(const RobotC *__restrict__ rb, SolveParams P)
{
    __shared__ double lds_raw[NMAX * (NMAX + 1)];
    const int64_t nact = P.n_active ? (int64_t)*P.n_active : P.N;
    int64_t wi = P.queue_head ? pop_item_wave(P.queue_head) : (int64_t)blockIdx.x;
    while (wi < nact) {
        wave_problem<NMAX, MMAX>(rb, P, lds_raw, wi);
        if (!P.queue_head) break;
        __syncthreads();
        wi = pop_item_wave(P.queue_head);
    }
}

template <int NMAX, int MMAX>
hipError_t launch_wave(const RobotC *rb, const SolveParams &P, int persist_blocks, hipStream_t s)
{
    int64_t grid = P.N;
    if (P.queue_head && persist_blocks > 0 && persist_blocks < grid) grid = persist_blocks;
    hipLaunchKernelGGL((lm_wave_kernel<NMAX, MMAX>), dim3((unsigned)grid), dim3(64), 0, s, rb, P);
    return hipGetLastError();
}

}  // namespace wave
}  // namespace pk
