// Per-lane Levenberg-Marquardt IK kernel: one problem per lane, the whole LM
// state (q, lambda, J^T J, J^T r, the Cholesky factor) in registers.
//
// Robot shape: a "star" of C serial chains of L revolute joints hanging off
// the base, one EE at each chain tip (a serial arm is C = 1).  Because a
// chain's joints only move its own EE, J^T J is block diagonal with C dense
// L x L blocks; each block is factored on its own.  Robot constants are
// uniform across the launch and are read with scalar loads.
//
// Method: Sec. III-A (LM over the sum of squared weighted residuals, limits
// as penalties) and Sec. III-C (joint pose cost log(T_target^-1 T_ee), joint
// limit cost, joint regularisation cost).
#include <math.h>

#include "pk_device.hpp"

namespace pk {
namespace {

template <int C, int L, int KIND>
struct Star {
    static constexpr int N = C * L;
    static constexpr int NA = L * (L + 1) / 2;   // packed lower triangle of one block
    static constexpr int ROWS = KIND == PK_EE_POSE ? 6 : 3;
};

PK_DEV constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Per-lane slice of the block's LDS: slot i of this lane lives at
// base[i * BLOCK] (lane-contiguous, conflict-free).
constexpr int BLOCK = 64;

struct LaneLds {
    float *base;
    PK_DEV float &operator[](int slot) const { return base[slot * BLOCK]; }
};

// LDS slots: [targets | A blocks | g].  Targets per EE: p (3) and, for pose
// EEs, the target rotation (9).
template <int C, int L, int KIND>
struct Slots {
    static constexpr int TGW = KIND == PK_EE_POSE ? 12 : 3;
    static constexpr int TG = 0;
    static constexpr int A = C * TGW;
    static constexpr int G = A + C * Star<C, L, KIND>::NA;
    static constexpr int TOTAL = G + C * L;
};

// FK along chain c at q; optionally keeps each joint's world axis and origin.
template <int C, int L, bool KEEP>
PK_DEV void chain_fk(const RobotC *__restrict__ rb, int c, const float *q, float (*om)[3],
                     float (*pj)[3], float *Re, float *pe)
{
    float O[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
    float p[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const int j = c * L + i;
        float s, co, On[9], pn[3];
        joint_sincos(q[j], s, co);
        joint_step(O, p, rb->j[j].G, rb->j[j].t, s, co, On, pn);
#pragma unroll
        for (int u = 0; u < 9; ++u) O[u] = On[u];
#pragma unroll
        for (int u = 0; u < 3; ++u) p[u] = pn[u];
        if (KEEP) {
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                om[i][u] = O[3 * u + 2];
                pj[i][u] = p[u];
            }
        }
    }
    ee_frame(O, p, rb->e[c].G, rb->e[c].t, Re, pe);
}

// Weighted EE residual rows of chain c (pose: [w_pos rho; w_rot phi]).
template <int KIND>
PK_DEV void ee_residual(const SolveParams &P, const LaneLds &S, int tg_slot, const float *Re,
                        const float *pe, float *r, float &perr, float &rerr, PoseLog *lg)
{
    float d[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) d[u] = pe[u] - S[tg_slot + u];
    perr = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if constexpr (KIND == PK_EE_POSE) {
        float Rt[9];
#pragma unroll
        for (int u = 0; u < 9; ++u) Rt[u] = S[tg_slot + 3 + u];
        *lg = pose_log(Rt, Re, d);
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            r[u] = P.w_pos * lg->rho[u];
            r[3 + u] = P.w_rot * lg->phi[u];
        }
        rerr = lg->theta;
    } else {
#pragma unroll
        for (int u = 0; u < 3; ++u) r[u] = P.w_pos * d[u];
        rerr = 0.f;
    }
}

// Cost and per-EE errors at q (no Jacobian).
template <int C, int L, int KIND>
PK_DEV void eval_cost(const RobotC *__restrict__ rb, const SolveParams &P,
                      const float *__restrict__ qr, const LaneLds &S, const float *q, float &cost,
                      float &pcost, float *perr, float *rerr)
{
    using SL = Slots<C, L, KIND>;
    constexpr int ROWS = Star<C, L, KIND>::ROWS;
    float cp = 0.f, cj = 0.f;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float Re[9], pe[3], r[ROWS];
        PoseLog lg;
        chain_fk<C, L, false>(rb, c, q, nullptr, nullptr, Re, pe);
        ee_residual<KIND>(P, S, SL::TG + c * SL::TGW, Re, pe, r, perr[c], rerr[c], &lg);
#pragma unroll
        for (int u = 0; u < ROWS; ++u) cp += r[u] * r[u];
    }
#pragma unroll
    for (int j = 0; j < C * L; ++j) {
        const float over = q[j] - rb->j[j].hi, under = rb->j[j].lo - q[j];
        const float rl = P.w_limit * (fmaxf(over, 0.f) + fmaxf(under, 0.f));
        const float rr = P.w_rest * (q[j] - qr[j]);
        cj += rl * rl + rr * rr;
    }
    pcost = cp;
    cost = cp + cj;
}

// Normal equations at q: for each chain, the packed J_c^T J_c (+ limit and
// rest diagonal) and J^T r, handed to sink.a(c, idx, v) / sink.g(j, v).
template <int C, int L, int KIND, typename AT, typename Sink>
PK_DEV void eval_normal_chain(const RobotC *__restrict__ rb, const SolveParams &P,
                              const float *__restrict__ qr, const LaneLds &S, const float *q,
                              int c, Sink &sink)
{
    using SL = Slots<C, L, KIND>;
    constexpr int ROWS = Star<C, L, KIND>::ROWS;
    {
        float om[L][3], pj[L][3], Re[9], pe[3], r[ROWS], pe_err, re_err, M[9], Nb[9];
        PoseLog lg;
        chain_fk<C, L, true>(rb, c, q, om, pj, Re, pe);
        ee_residual<KIND>(P, S, SL::TG + c * SL::TGW, Re, pe, r, pe_err, re_err, &lg);
        if constexpr (KIND == PK_EE_POSE) jr_inv_blocks(lg, Re, M, Nb);
        float col[L][ROWS];
#pragma unroll
        for (int i = 0; i < L; ++i) {
            float lev[3] = {pe[0] - pj[i][0], pe[1] - pj[i][1], pe[2] - pj[i][2]}, v[3];
            cross(om[i], lev, v);
            if constexpr (KIND == PK_EE_POSE) {
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    float mv = M[3 * u] * v[0] + M[3 * u + 1] * v[1] + M[3 * u + 2] * v[2];
                    float nw = Nb[3 * u] * om[i][0] + Nb[3 * u + 1] * om[i][1] + Nb[3 * u + 2] * om[i][2];
                    float mw = M[3 * u] * om[i][0] + M[3 * u + 1] * om[i][1] + M[3 * u + 2] * om[i][2];
                    col[i][u] = P.w_pos * (mv + nw);
                    col[i][3 + u] = P.w_rot * mw;
                }
            } else {
#pragma unroll
                for (int u = 0; u < 3; ++u) col[i][u] = P.w_pos * v[u];
            }
        }
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const int j = c * L + i;
            const float over = q[j] - rb->j[j].hi, under = rb->j[j].lo - q[j];
            const float rl = P.w_limit * (fmaxf(over, 0.f) + fmaxf(under, 0.f));
            const float rr = P.w_rest * (q[j] - qr[j]);
            const float dl = over > 0.f ? P.w_limit : (under > 0.f ? -P.w_limit : 0.f);
#pragma unroll
            for (int k = 0; k <= i; ++k) {
                AT s = 0;
#pragma unroll
                for (int u = 0; u < ROWS; ++u) s += (AT)col[i][u] * (AT)col[k][u];
                if (k == i) s += (AT)dl * (AT)dl + (AT)P.w_rest * (AT)P.w_rest;
                sink.a(c, tri(i, k), s);
            }
            AT s = (AT)dl * (AT)rl + (AT)P.w_rest * (AT)rr;
#pragma unroll
            for (int u = 0; u < ROWS; ++u) s += (AT)col[i][u] * (AT)r[u];
            sink.g(j, s);
        }
    }
}

template <int C, int L, int KIND, typename AT, typename Sink>
PK_DEV void eval_normal(const RobotC *__restrict__ rb, const SolveParams &P,
                        const float *__restrict__ qr, const LaneLds &S, const float *q, Sink &sink)
{
#pragma unroll
    for (int c = 0; c < C; ++c) eval_normal_chain<C, L, KIND, AT>(rb, P, qr, S, q, c, sink);
}

template <int C, int L, int KIND>
struct LdsSink {
    LaneLds S;
    PK_DEV void a(int c, int idx, float v) { S[Slots<C, L, KIND>::A + c * Star<C, L, KIND>::NA + idx] = v; }
    PK_DEV void g(int j, float v) { S[Slots<C, L, KIND>::G + j] = v; }
};

// One chain's block in FP64 registers.
template <int C, int L, int KIND>
struct RegSink64 {
    double A[Star<C, L, KIND>::NA];
    double G[L];
    PK_DEV void a(int, int idx, double v) { A[idx] = v; }
    PK_DEV void g(int j, double v) { G[j % L] = v; }
};

// Damped Cholesky of one packed block: Lf = chol(A + lam diag(max(A_ii, floor))).
// Lf may alias A (in-place).  The diagonal slots of Lf hold 1 / L_ii.  Returns false if a pivot is not
// above `thresh` (or not finite).
template <int L, typename T>
PK_DEV bool chol_damped(const T *A, T lam, T floor_, T thresh, T *Lf)
{
    bool ok = true;
#pragma unroll
    for (int i = 0; i < L * (L + 1) / 2; ++i) Lf[i] = A[i];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        T a = A[tri(i, i)];
        Lf[tri(i, i)] += lam * (a > floor_ ? a : floor_);
    }
#pragma unroll
    for (int k = 0; k < L; ++k) {
        T d = Lf[tri(k, k)];
#pragma unroll
        for (int l = 0; l < k; ++l) d -= Lf[tri(k, l)] * Lf[tri(k, l)];
        if (!(d > thresh) || !(d < (T)INFINITY)) {
            ok = false;
            d = 1;
        }
        const T inv = rsqrt_t(d);
        Lf[tri(k, k)] = inv;
#pragma unroll
        for (int i = k + 1; i < L; ++i) {
            T s = Lf[tri(i, k)];
#pragma unroll
            for (int l = 0; l < k; ++l) s -= Lf[tri(i, l)] * Lf[tri(k, l)];
            Lf[tri(i, k)] = s * inv;
        }
    }
    return ok;
}

// x = -(L L^T)^-1 g for one block.
template <int L, typename T>
PK_DEV void chol_solve_neg(const T *Lf, const T *g, T *x)
{
    T y[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        T s = -g[i];
#pragma unroll
        for (int l = 0; l < i; ++l) s -= Lf[tri(i, l)] * y[l];
        y[i] = s * Lf[tri(i, i)];
    }
#pragma unroll
    for (int i = L - 1; i >= 0; --i) {
        T s = y[i];
#pragma unroll
        for (int l = i + 1; l < L; ++l) s -= Lf[tri(l, i)] * x[l];
        x[i] = s * Lf[tri(i, i)];
    }
}

// FP64 re-solve: J (FP32) is formed again at q, J^T J and J^T r are
// accumulated, damped and factored in FP64.  False if FP64 also fails.
template <int C, int L, int KIND>
PK_DEV bool step_fp64(const RobotC *__restrict__ rb, const SolveParams &P,
                      const float *__restrict__ qr, const LaneLds &S, const float *q, float lam,
                      float *delta)
{
    bool ok = true;
    // Blocks are independent: one chain at a time, factored in place.
#pragma unroll
    for (int c = 0; c < C; ++c) {
        RegSink64<C, L, KIND> sk;
        eval_normal_chain<C, L, KIND, double>(rb, P, qr, S, q, c, sk);
        double x[L];
        ok &= chol_damped<L, double>(sk.A, (double)lam, (double)P.damping_floor, 0.0, sk.A);
        chol_solve_neg<L, double>(sk.A, sk.G, x);
#pragma unroll
        for (int i = 0; i < L; ++i) delta[c * L + i] = (float)x[i];
    }
    return ok;
}

template <int C, int L, int KIND>
PK_DEV bool meets_tol(const SolveParams &P, const float *perr, const float *rerr)
{
    bool ok = true;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        ok &= perr[c] <= P.tol_pos;
        if (KIND == PK_EE_POSE) ok &= rerr[c] <= P.tol_rot;
    }
    return ok;
}

template <int C, int L, int KIND>
PK_DEV void write_trace(const SolveParams &P, int it, int64_t p, const float *q, bool acc)
{
    using S = Star<C, L, KIND>;
    if (it < P.trace_iters) {
#pragma unroll
        for (int j = 0; j < S::N; ++j) P.trace_q[((int64_t)it * S::N + j) * P.N + p] = q[j];
        P.trace_acc[(int64_t)it * P.N + p] = acc ? 1 : 0;
    }
}

template <int C, int L, int KIND>
__global__ __launch_bounds__(BLOCK) void lm_lane_kernel(const RobotC *__restrict__ rb,
                                                        const float *__restrict__ qr, SolveParams P)
{
    using St = Star<C, L, KIND>;
    using SL = Slots<C, L, KIND>;
    __shared__ float smem[SL::TOTAL * BLOCK];
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p >= P.N) return;
    const int64_t N = P.N, T = P.T, t = p / P.K;
    const LaneLds S{smem + threadIdx.x};

    float q[St::N];
    bool finite = true;
#pragma unroll
    for (int j = 0; j < St::N; ++j) {
        q[j] = P.seeds[j * N + p];
        finite &= isfinite(q[j]);
    }
    const int W = KIND == PK_EE_POSE ? 7 : 3;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float v[W];
#pragma unroll
        for (int u = 0; u < W; ++u) {
            v[u] = P.targets[(int64_t)(c * W + u) * T + t];
            finite &= isfinite(v[u]);
        }
        const int base = SL::TG + c * SL::TGW;
#pragma unroll
        for (int u = 0; u < 3; ++u) S[base + u] = v[u];
        if constexpr (KIND == PK_EE_POSE) {
            float R[9];
            quat_to_rot(v[3], v[4], v[5], v[6], R);
#pragma unroll
            for (int u = 0; u < 9; ++u) S[base + 3 + u] = R[u];
        }
    }

    if (!finite) {
#pragma unroll
        for (int j = 0; j < St::N; ++j) P.joints[j * N + p] = q[j];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (P.pos_err) P.pos_err[c * N + p] = NAN;
            if (P.rot_err) P.rot_err[c * N + p] = NAN;
        }
        if (P.cost) P.cost[p] = NAN;
        P.pose_cost[p] = NAN;
        if (P.iters) P.iters[p] = 0;
        if (P.accepts) P.accepts[p] = 0;
        if (P.status) P.status[p] = PK_NONFINITE;
        if (P.iters_to_tol) P.iters_to_tol[p] = -1;
        for (int it = 0; it < P.trace_iters; ++it) write_trace<C, L, KIND>(P, it, p, q, false);
        return;
    }

    float cost, pcost, perr[C], rerr[C];
    eval_cost<C, L, KIND>(rb, P, qr, S, q, cost, pcost, perr, rerr);
    int iters = 0, accepts = 0, itt = -1, flags = 0;
    if (meets_tol<C, L, KIND>(P, perr, rerr)) itt = 0;
    bool done = P.early_exit && itt == 0, stalled = false, need_j = true;
    float lam = P.lambda0;
    LdsSink<C, L, KIND> sink{S};

    for (int it = 0; it < P.max_iters; ++it) {
        // keep LDS-resident state out of registers across iterations
        __asm__ volatile("" ::: "memory");
        if (done) {
            write_trace<C, L, KIND>(P, it, p, q, false);
            continue;
        }
        if (need_j) {
            // J^T J and J^T r at the current point (after an accept) -> LDS.
            eval_normal<C, L, KIND, float>(rb, P, qr, S, q, sink);
            need_j = false;
        }
        // Damped normal equations, FP32 Cholesky with the pivot test.
        float dmax = 0.f;
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const float a = S[SL::A + c * St::NA + tri(i, i)];
                dmax = fmaxf(dmax, a + lam * fmaxf(a, P.damping_floor));
            }
        const float thresh = P.pivot_rel * dmax;
        float delta[St::N];
        bool ok = true;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            float Ac[St::NA], gc[L], x[L];
#pragma unroll
            for (int i = 0; i < St::NA; ++i) Ac[i] = S[SL::A + c * St::NA + i];
#pragma unroll
            for (int i = 0; i < L; ++i) gc[i] = S[SL::G + c * L + i];
            ok &= chol_damped<L, float>(Ac, lam, P.damping_floor, thresh, Ac);   // in place
            chol_solve_neg<L, float>(Ac, gc, x);
#pragma unroll
            for (int i = 0; i < L; ++i) delta[c * L + i] = x[i];
        }
        if (!ok) {
            flags |= PK_FLAG_FP64;
            ok = step_fp64<C, L, KIND>(rb, P, qr, S, q, lam, delta);
        }
        float ct = INFINITY, pct = 0.f, pe_t[C], re_t[C], qt[St::N];
        if (ok) {
#pragma unroll
            for (int j = 0; j < St::N; ++j) qt[j] = q[j] + delta[j];
            eval_cost<C, L, KIND>(rb, P, qr, S, qt, ct, pct, pe_t, re_t);
        }
        ++iters;
        const bool acc = ct < cost;
        if (acc) {
#pragma unroll
            for (int j = 0; j < St::N; ++j) q[j] = qt[j];
            cost = ct;
            pcost = pct;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                perr[c] = pe_t[c];
                rerr[c] = re_t[c];
            }
            lam = fmaxf(lam / P.nu_down, P.lambda_min);
            ++accepts;
            need_j = true;
            if (meets_tol<C, L, KIND>(P, perr, rerr)) {
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
        write_trace<C, L, KIND>(P, it, p, q, acc);
    }

    const bool conv = meets_tol<C, L, KIND>(P, perr, rerr);
#pragma unroll
    for (int j = 0; j < St::N; ++j) P.joints[j * N + p] = q[j];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if (P.pos_err) P.pos_err[c * N + p] = perr[c];
        if (P.rot_err) P.rot_err[c * N + p] = rerr[c];
    }
    if (P.cost) P.cost[p] = cost;
    P.pose_cost[p] = pcost;
    if (P.iters) P.iters[p] = iters;
    if (P.accepts) P.accepts[p] = accepts;
    if (P.status)
        P.status[p] = (conv ? PK_CONVERGED : (stalled ? PK_STALLED : PK_MAX_ITERS)) | flags;
    if (P.iters_to_tol) P.iters_to_tol[p] = itt;
}

template <int C, int L, int KIND>
hipError_t launch_star(const RobotC *rb, const SolveParams &P, hipStream_t s)
{
    const int block = BLOCK;
    const int64_t grid = (P.N + block - 1) / block;
    // rest pose: caller's array, else the robot's mid-range table
    const float *qr = P.q_rest ? P.q_rest : rb->mid;
    hipLaunchKernelGGL((lm_lane_kernel<C, L, KIND>), dim3((unsigned)grid), dim3(block), 0, s, rb, qr,
                       P);
    return hipGetLastError();
}

}  // namespace

bool lane_variant_available(int chains, int chain_len, int kind)
{
    return (chains == 1 && chain_len == 7 && kind == PK_EE_POSE) ||
           (chains == 4 && chain_len == 4 && kind == PK_EE_POSITION);
}

hipError_t launch_lm_lane(const RobotC *dev_robot, const RobotC &h, const SolveParams &P,
                          hipStream_t s)
{
    const int kind = h.e[0].kind;
    if (h.chains == 1 && h.chain_len == 7 && kind == PK_EE_POSE)
        return launch_star<1, 7, PK_EE_POSE>(dev_robot, P, s);
    if (h.chains == 4 && h.chain_len == 4 && kind == PK_EE_POSITION)
        return launch_star<4, 4, PK_EE_POSITION>(dev_robot, P, s);
    return hipErrorInvalidValue;
}

}  // namespace pk
