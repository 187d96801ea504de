// Per-lane Levenberg-Marquardt IK kernel: one problem per lane, the whole LM
// state (q, lambda, J^T J, J^T r, the Cholesky factor) in registers.
//
// Robot shape: a "star" of C serial chains of L joints (revolute, or
// prismatic on a single chain) hanging off the base, one EE at each chain tip
// (a serial arm is C = 1).  Because a
// chain's joints only move its own EE, J^T J is block diagonal with C dense
// L x L blocks; each block is factored on its own.  Robot constants are
// uniform across the launch and are read with scalar loads.
//
// Method: Sec. III-A (LM over the sum of squared weighted residuals, limits
// as penalties) and Sec. III-C (joint pose cost log(T_target^-1 T_ee), joint
// limit cost, joint regularisation cost).
#pragma once

#include <math.h>

#include "pk_device.hpp"

namespace pk {
namespace lane {

// The kernels' KIND template argument: the EE kind (PK_EE_POSE or
// PK_EE_POSITION) plus LANE_PRISMATIC when the robot has prismatic joints
// (robots without them compile the revolute-only code).
constexpr int LANE_PRISMATIC = 4;
constexpr int ee_of(int kind) { return kind & 3; }
constexpr bool pris_of(int kind) { return (kind & LANE_PRISMATIC) != 0; }


template <int C, int L, int KIND>
struct Star {
    static constexpr int N = C * L;
    static constexpr int NA = L * (L + 1) / 2;   // packed lower triangle of one block
    static constexpr int ROWS = ee_of(KIND) == PK_EE_POSE ? 6 : 3;
};

PK_DEV constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Per-lane slice of the block's LDS: slot i of this lane lives at
// base[i * BLOCK] (lane-contiguous, conflict-free).
constexpr int BLOCK = 64;

struct LaneLds {
    float *base;
    PK_DEV float &operator[](int slot) const { return base[slot * BLOCK]; }
};

// LDS slots: [targets | Jacobian columns | residual rows | diagonal terms].
// Targets per EE: p (3) and, for pose EEs, the target rotation (9).  The
// Jacobian of the current point (weighted rows, ROWS per EE, chain-major),
// the EE residual rows, and per joint the limit/rest contributions to the
// diagonal (dl^2 + w_rest^2) and to J^T r (dl rl + w_rest rr).
template <int C, int L, int KIND>
struct Slots {
    static constexpr int ROWS = Star<C, L, KIND>::ROWS;
    static constexpr int TGW = ee_of(KIND) == PK_EE_POSE ? 12 : 3;
    static constexpr int TG = 0;
    static constexpr int COL = C * TGW;
    static constexpr int RES = COL + C * L * ROWS;
    static constexpr int DG = RES + C * ROWS;
    static constexpr int GX = DG + C * L;
    // Single chains keep only the FP32 normal equations of the current point:
    // packed J^T J (+ diagonal terms) then J^T r after the targets, formed
    // once per taken point and reused by rejected steps (their rare FP64
    // re-solve rebuilds the Jacobian in registers, so no column slots).
    static constexpr int AG = COL;
    static constexpr int TOTAL = C == 1 ? AG + Star<C, L, KIND>::NA + L : GX + C * L;
};

// FK along chain c at q; optionally keeps each joint's world axis and origin.
// A prismatic joint (a robot constant, so the branch is uniform) does not
// rotate its frame and slides its origin by q along its axis.
template <int C, int L, bool KEEP, int KIND = PK_EE_POSE>
PK_DEV void chain_fk(const RobotC *__restrict__ rb, int c, const float *q, float (*om)[3],
                     float (*pj)[3], float *Re, float *pe)
{
    float O[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
    float p[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const int j = c * L + i;
        float s = 0.f, co = 1.f, On[9], pn[3];
        const bool pris = pris_of(KIND) && rb->j[j].type == PK_JOINT_PRISMATIC;
        if (!pris) joint_sincos(q[j], s, co);
        joint_step(O, p, rb->j[j].G, rb->j[j].t, s, co, On, pn);
        if (pris) joint_slide(On, q[j], pn);
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
    if constexpr (ee_of(KIND) == PK_EE_POSE) {
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
        chain_fk<C, L, false, KIND>(rb, c, q, nullptr, nullptr, Re, pe);
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

// Weighted Jacobian column of a joint with world axis w and origin pj, for
// the single EE at pe (M, Nb: the EE's right-Jacobian-inverse blocks, pose
// EEs only): a revolute joint moves the EE with twist (w x (pe - pj), w), a
// prismatic one with (w, 0).
template <int KIND>
PK_DEV void jac_column(const SolveParams &P, const float *M, const float *Nb, const float *w,
                       const float *pj, const float *pe, bool pris, float *col)
{
    float v[3], wv[3];
    if constexpr (pris_of(KIND)) {
        // the joint type as a 0/1 factor (a uniform condition per column
        // used in selects had doubled the kernel's register allocation)
        const float rv = pris ? 0.f : 1.f, pv = 1.f - rv;
        const float lev[3] = {pe[0] - pj[0], pe[1] - pj[1], pe[2] - pj[2]};
        float vr[3];
        cross(w, lev, vr);
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            v[u] = rv * vr[u] + pv * w[u];
            wv[u] = rv * w[u];
        }
    } else {
        joint_twist(false, w, pj, pe, v, wv);
    }
    if constexpr (ee_of(KIND) == PK_EE_POSE) {
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            float mv = M[3 * u] * v[0] + M[3 * u + 1] * v[1] + M[3 * u + 2] * v[2];
            float nw = Nb[3 * u] * wv[0] + Nb[3 * u + 1] * wv[1] + Nb[3 * u + 2] * wv[2];
            float mw = M[3 * u] * wv[0] + M[3 * u + 1] * wv[1] + M[3 * u + 2] * wv[2];
            col[u] = P.w_pos * (mv + nw);
            col[3 + u] = P.w_rot * mw;
        }
    } else {
#pragma unroll
        for (int u = 0; u < 3; ++u) col[u] = P.w_pos * v[u];
    }
}

// Normal equations at q: for each chain, the packed J_c^T J_c (+ limit and
// rest diagonal) and J^T r, handed to sink.a(c, idx, v) / sink.g(j, v).
// Jacobian of chain c at q (weighted EE rows and the limit/rest diagonal
// terms) -> LDS.
template <int C, int L, int KIND>
PK_DEV void eval_jacobian_chain(const RobotC *__restrict__ rb, const SolveParams &P,
                                const float *__restrict__ qr, const LaneLds &S, const float *q, int c)
{
    using SL = Slots<C, L, KIND>;
    constexpr int ROWS = SL::ROWS;
    float om[L][3], pj[L][3], Re[9], pe[3], r[ROWS], pe_err, re_err, M[9], Nb[9];
    PoseLog lg;
    chain_fk<C, L, true, KIND>(rb, c, q, om, pj, Re, pe);
    ee_residual<KIND>(P, S, SL::TG + c * SL::TGW, Re, pe, r, pe_err, re_err, &lg);
    if constexpr (ee_of(KIND) == PK_EE_POSE) jr_inv_blocks(lg, Re, M, Nb);
#pragma unroll
    for (int u = 0; u < ROWS; ++u) S[SL::RES + c * ROWS + u] = r[u];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const int j = c * L + i;
        const int base = SL::COL + (c * L + i) * ROWS;
        float col[ROWS];
        jac_column<KIND>(P, M, Nb, om[i], pj[i], pe, rb->j[j].type == PK_JOINT_PRISMATIC, col);
#pragma unroll
        for (int u = 0; u < ROWS; ++u) S[base + u] = col[u];
        const float over = q[j] - rb->j[j].hi, under = rb->j[j].lo - q[j];
        const float rl = P.w_limit * (fmaxf(over, 0.f) + fmaxf(under, 0.f));
        const float rr = P.w_rest * (q[j] - qr[j]);
        const float dl = over > 0.f ? P.w_limit : (under > 0.f ? -P.w_limit : 0.f);
        S[SL::DG + j] = dl * dl + P.w_rest * P.w_rest;
        S[SL::GX + j] = dl * rl + P.w_rest * rr;
    }
}

// Limit and rest terms of joint i at q: its share of the normal matrix's
// diagonal (dl^2 + w_rest^2) and of J^T r (dl rl + w_rest rr).
PK_DEV void joint_terms(const RobotC *__restrict__ rb, const SolveParams &P, const float *__restrict__ qr,
                        const float *q, int i, float &dg, float &gx)
{
    const float over = q[i] - rb->j[i].hi, under = rb->j[i].lo - q[i];
    const float rl = P.w_limit * (fmaxf(over, 0.f) + fmaxf(under, 0.f));
    const float rr = P.w_rest * (q[i] - qr[i]);
    const float dl = over > 0.f ? P.w_limit : (under > 0.f ? -P.w_limit : 0.f);
    dg = dl * dl + P.w_rest * P.w_rest;
    gx = dl * rl + P.w_rest * rr;
}

// Single chain: FP32 J^T J (+ diagonal terms) and J^T r at q straight from
// the columns as they are formed (the sums of form_normal, in its order;
// the columns never go through LDS), into the cached normal equations (AG).
template <int L, int KIND>
PK_DEV void normal1(const RobotC *__restrict__ rb, const SolveParams &P, const float *__restrict__ qr,
                    const LaneLds &S, const float *q, const float (*om)[3], const float (*pj)[3],
                    const float *Re, const float *pe, const float *r, const PoseLog &lg)
{
    using SL = Slots<1, L, KIND>;
    constexpr int ROWS = SL::ROWS, NA = Star<1, L, KIND>::NA;
    float M[9], Nb[9];
    if constexpr (ee_of(KIND) == PK_EE_POSE) jr_inv_blocks(lg, Re, M, Nb);
    float col[L][ROWS];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        float dg, gx;
        jac_column<KIND>(P, M, Nb, om[i], pj[i], pe, rb->j[i].type == PK_JOINT_PRISMATIC, col[i]);
        joint_terms(rb, P, qr, q, i, dg, gx);
#pragma unroll
        for (int k = 0; k <= i; ++k) {
            float a = 0.f;
#pragma unroll
            for (int u = 0; u < ROWS; ++u) a += col[i][u] * col[k][u];
            if (k == i) a += dg;
            S[SL::AG + tri(i, k)] = a;
        }
        float b = gx;
#pragma unroll
        for (int u = 0; u < ROWS; ++u) b += col[i][u] * r[u];
        S[SL::AG + NA + i] = b;
    }
}

template <int C, int L, int KIND, typename T>
PK_DEV void form_normal(const LaneLds &S, int c, T *A, T *g);

// Single-chain robots: cost and errors at q and, when the point is taken
// (the start point, or a trial with cost below `cur`), its Jacobian and
// normal equations from the same forward kinematics, so an accepted trial is
// not evaluated a second time.  Returns whether it was taken.
template <int L, int KIND>
PK_DEV bool eval_point1(const RobotC *__restrict__ rb, const SolveParams &P, const float *__restrict__ qr,
                        const LaneLds &S, const float *q, bool first, float cur, float &cost, float &pcost,
                        float *perr, float *rerr)
{
    using SL = Slots<1, L, KIND>;
    constexpr int ROWS = SL::ROWS;
    float om[L][3], pj[L][3], Re[9], pe[3], r[ROWS];
    PoseLog lg;
    chain_fk<1, L, true, KIND>(rb, 0, q, om, pj, Re, pe);
    ee_residual<KIND>(P, S, SL::TG, Re, pe, r, perr[0], rerr[0], &lg);
    float cp = 0.f, cj = 0.f;
#pragma unroll
    for (int u = 0; u < ROWS; ++u) cp += r[u] * r[u];
#pragma unroll
    for (int j = 0; j < L; ++j) {
        const float over = q[j] - rb->j[j].hi, under = rb->j[j].lo - q[j];
        const float rl = P.w_limit * (fmaxf(over, 0.f) + fmaxf(under, 0.f));
        const float rr = P.w_rest * (q[j] - qr[j]);
        cj += rl * rl + rr * rr;
    }
    pcost = cp;
    cost = cp + cj;
    const bool take = first || cost < cur;
    if (take) normal1<L, KIND>(rb, P, qr, S, q, om, pj, Re, pe, r, lg);
    return take;
}

// Packed block c of J^T J (+ diagonal terms) and J^T r in precision T, from
// the FP32 columns in LDS.
template <int C, int L, int KIND, typename T>
PK_DEV void form_normal(const LaneLds &S, int c, T *A, T *g)
{
    using SL = Slots<C, L, KIND>;
    constexpr int ROWS = SL::ROWS;
    float col[L][ROWS], r[ROWS];
#pragma unroll
    for (int i = 0; i < L; ++i)
#pragma unroll
        for (int u = 0; u < ROWS; ++u) col[i][u] = S[SL::COL + (c * L + i) * ROWS + u];
#pragma unroll
    for (int u = 0; u < ROWS; ++u) r[u] = S[SL::RES + c * ROWS + u];
#pragma unroll
    for (int i = 0; i < L; ++i) {
#pragma unroll
        for (int k = 0; k <= i; ++k) {
            T s = 0;
#pragma unroll
            for (int u = 0; u < ROWS; ++u) s += (T)col[i][u] * (T)col[k][u];
            if (k == i) s += (T)S[SL::DG + c * L + i];
            A[tri(i, k)] = s;
        }
        T s = (T)S[SL::GX + c * L + i];
#pragma unroll
        for (int u = 0; u < ROWS; ++u) s += (T)col[i][u] * (T)r[u];
        g[i] = s;
    }
}

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

// FP64 re-solve: J^T J and J^T r are formed again from the FP32 Jacobian in
// LDS, damped and factored in FP64, one chain at a time.  False if FP64 also
// fails.
template <int C, int L, int KIND>
PK_DEV bool step_fp64(const SolveParams &P, const LaneLds &S, float lam, float *delta)
{
    bool ok = true;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        double A[Star<C, L, KIND>::NA], g[L], x[L];
        form_normal<C, L, KIND, double>(S, c, A, g);
        ok &= chol_damped<L, double>(A, (double)lam, (double)P.damping_floor, 0.0, A);
        chol_solve_neg<L, double>(A, g, x);
#pragma unroll
        for (int i = 0; i < L; ++i) delta[c * L + i] = (float)x[i];
    }
    return ok;
}

// Single chain, FP64 re-solve: the Jacobian at q is formed again in
// registers (the same FP32 columns the cached normal equations came from),
// J^T J and J^T r accumulated in FP64 with each product's columns recomputed
// (a rare path: register use, not work, is what it must keep low), damped
// and factored in FP64.  The FP32 cache in LDS is left as it was.
template <int L, int KIND>
PK_DEV bool step_fp64_1(const RobotC *__restrict__ rb, const SolveParams &P, const float *__restrict__ qr,
                        const LaneLds &S, const float *q, float lam, float *delta)
{
    using SL = Slots<1, L, KIND>;
    constexpr int ROWS = SL::ROWS;
    float om[L][3], pj[L][3], Re[9], pe[3], r[ROWS], pe_err, re_err, M[9], Nb[9];
    PoseLog lg;
    chain_fk<1, L, true, KIND>(rb, 0, q, om, pj, Re, pe);
    ee_residual<KIND>(P, S, SL::TG, Re, pe, r, pe_err, re_err, &lg);
    if constexpr (ee_of(KIND) == PK_EE_POSE) jr_inv_blocks(lg, Re, M, Nb);
    double A[Star<1, L, KIND>::NA], g[L], x[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        float ci[ROWS], dg, gx;
        jac_column<KIND>(P, M, Nb, om[i], pj[i], pe, rb->j[i].type == PK_JOINT_PRISMATIC, ci);
        joint_terms(rb, P, qr, q, i, dg, gx);
#pragma unroll
        for (int k = 0; k <= i; ++k) {
            float ck[ROWS];
            jac_column<KIND>(P, M, Nb, om[k], pj[k], pe, rb->j[k].type == PK_JOINT_PRISMATIC, ck);
            double a = 0;
#pragma unroll
            for (int u = 0; u < ROWS; ++u) a += (double)ci[u] * (double)ck[u];
            if (k == i) a += (double)dg;
            A[tri(i, k)] = a;
        }
        double b = (double)gx;
#pragma unroll
        for (int u = 0; u < ROWS; ++u) b += (double)ci[u] * (double)r[u];
        g[i] = b;
    }
    const bool ok = chol_damped<L, double>(A, (double)lam, (double)P.damping_floor, 0.0, A);
    chol_solve_neg<L, double>(A, g, x);
#pragma unroll
    for (int i = 0; i < L; ++i) delta[i] = (float)x[i];
    return ok;
}

// Lanes of this wavefront that hold problems of target t in one run of
// consecutive lanes with this one (bit mask).  Called by every lane that
// holds a problem.
PK_DEV uint64_t target_run_mask(int64_t t)
{
    const int lane = threadIdx.x & 63;
    const uint64_t act = __ballot(1);
    const int64_t tp = __shfl(t, (lane + 63) & 63, 64);
    const bool start = lane == 0 || !((act >> (lane - 1)) & 1) || tp != t;
    const uint64_t R = __ballot(start);
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);   // bits 0..lane
    const int s = 63 - __builtin_clzll(R & upto);                      // this run's first lane
    const uint64_t after = R & ~upto;
    const uint64_t from_s = ~0ull << s;
    const uint64_t mask = after ? from_s & ((1ull << __builtin_ctzll(after)) - 1) : from_s;
    return mask & act;
}

template <int C, int L, int KIND>
PK_DEV bool meets_tol(const SolveParams &P, const float *perr, const float *rerr)
{
    bool ok = true;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        ok &= perr[c] <= P.tol_pos;
        if (ee_of(KIND) == PK_EE_POSE) ok &= rerr[c] <= P.tol_rot;
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

// Loads problem p's starting point (from qsrc) into q and its targets into
// the TG slots; false if any of them is not finite.
template <int C, int L, int KIND>
PK_DEV bool load_problem(const SolveParams &P, const LaneLds &S, const float *qsrc, int64_t p, float *q)
{
    using St = Star<C, L, KIND>;
    using SL = Slots<C, L, KIND>;
    const int64_t N = P.N, T = P.T, t = p / P.K;
    bool finite = true;
#pragma unroll
    for (int j = 0; j < St::N; ++j) {
        q[j] = qsrc[j * N + p];
        finite &= isfinite(q[j]);
    }
    const int W = ee_of(KIND) == PK_EE_POSE ? 7 : 3;
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
        if constexpr (ee_of(KIND) == PK_EE_POSE) {
            float R[9];
            quat_to_rot(v[3], v[4], v[5], v[6], R);
#pragma unroll
            for (int u = 0; u < 9; ++u) S[base + 3 + u] = R[u];
        }
    }
    return finite;
}

// Outputs of a problem with a non-finite seed or target.
template <int C, int L, int KIND>
PK_DEV void write_nonfinite(const SolveParams &P, int64_t p, const float *q, bool resumable)
{
    using St = Star<C, L, KIND>;
    const int64_t N = P.N;
#pragma unroll
    for (int j = 0; j < St::N; ++j) P.joints[j * N + p] = q[j];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if (P.pos_err) P.pos_err[c * N + p] = NAN;
        if (P.rot_err) P.rot_err[c * N + p] = NAN;
    }
    if (P.cost) P.cost[p] = NAN;
    if (P.pose_cost) P.pose_cost[p] = NAN;
    if (P.iters) P.iters[p] = 0;
    if (P.accepts) P.accepts[p] = 0;
    if (P.status) P.status[p] = PK_NONFINITE;
    if (P.iters_to_tol) P.iters_to_tol[p] = -1;
    if (resumable) P.st_state[p] = PK_ST_DONE;
    for (int it = 0; it < P.trace_iters; ++it) write_trace<C, L, KIND>(P, it, p, q, false);
}

// Damped step from the Jacobian in LDS: FP32 Cholesky with the pivot test
// against the largest damped diagonal, FP64 re-solve on a small pivot.
// False if that fails too.
template <int C, int L, int KIND>
PK_DEV bool lane_step(const RobotC *__restrict__ rb, const SolveParams &P, const float *__restrict__ qr,
                      const LaneLds &S, const float *q, float lam, int &flags, float *delta)
{
    using St = Star<C, L, KIND>;
    using SL = Slots<C, L, KIND>;
    // Every block first: the pivot threshold needs the largest damped
    // diagonal over all joints, read off the formed blocks (a single chain
    // reads its cached normal equations).
    float Ac[C][St::NA], gc[C][L];
    if constexpr (C == 1) {
#pragma unroll
        for (int i = 0; i < St::NA; ++i) Ac[0][i] = S[SL::AG + i];
#pragma unroll
        for (int i = 0; i < L; ++i) gc[0][i] = S[SL::AG + St::NA + i];
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) form_normal<C, L, KIND, float>(S, c, Ac[c], gc[c]);
    }
    float dmax = 0.f;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const float a = Ac[c][tri(i, i)];
            dmax = fmaxf(dmax, a + lam * fmaxf(a, P.damping_floor));
        }
    const float thresh = P.pivot_rel * dmax;
    bool ok = true;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float x[L];
        ok &= chol_damped<L, float>(Ac[c], lam, P.damping_floor, thresh, Ac[c]);   // in place
        chol_solve_neg<L, float>(Ac[c], gc[c], x);
#pragma unroll
        for (int ii = 0; ii < L; ++ii) delta[c * L + ii] = x[ii];
    }
    if (!ok) {
        flags |= PK_FLAG_FP64;
        // a single chain re-forms its Jacobian for this (the caller does it,
        // where fewer values are live)
        if constexpr (C > 1) ok = step_fp64<C, L, KIND>(P, S, lam, delta);
    }
    return ok;
}

// Final outputs of problem p (and its trace after the last iteration).
template <int C, int L, int KIND>
PK_DEV void write_result(const SolveParams &P, int64_t p, const float *q, float cost, float pcost,
                         const float *perr, const float *rerr, int iters, int accepts, int itt,
                         int flags, bool stalled, bool finished, bool tsolved = false)
{
    using St = Star<C, L, KIND>;
    const int64_t N = P.N;
    if (finished)
        for (int it = iters; it < P.trace_iters; ++it) write_trace<C, L, KIND>(P, it, p, q, false);
    const bool conv = meets_tol<C, L, KIND>(P, perr, rerr);
#pragma unroll
    for (int j = 0; j < St::N; ++j) P.joints[j * N + p] = q[j];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if (P.pos_err) P.pos_err[c * N + p] = perr[c];
        if (P.rot_err) P.rot_err[c * N + p] = rerr[c];
    }
    if (P.cost) P.cost[p] = cost;
    if (P.pose_cost) P.pose_cost[p] = pcost;
    if (P.iters) P.iters[p] = iters;
    if (P.accepts) P.accepts[p] = accepts;
    if (P.status)
        P.status[p] = (conv ? PK_CONVERGED
                            : tsolved ? PK_TARGET_SOLVED : (stalled ? PK_STALLED : PK_MAX_ITERS)) | flags;
    if (P.iters_to_tol) P.iters_to_tol[p] = itt;
}

// A problem's final joints, costs and convergence, for a best-of-K taken in
// the launch that solved it.
template <int N>
struct LaneFinal {
    float q[N];
    float cost, pcost;
    bool conv;
};

// One LM problem (active index i) on this lane.  With P.st_state the run is
// resumable: it continues from the state a previous launch left in HBM and
// stops after P.iter_budget iterations.  Each pass of the loop evaluates one
// point (first the starting point, then each trial), so the cost evaluation
// has a single call site.
template <int C, int L, int KIND, bool RESUMABLE, bool TEXIT = false>
PK_DEV void lane_problem(const RobotC *__restrict__ rb, const float *__restrict__ qr,
                         const SolveParams &P, const LaneLds &S, int64_t i,
                         LaneFinal<Star<C, L, KIND>::N> *fin = nullptr)
{
    using St = Star<C, L, KIND>;
    const int64_t p = P.active ? (int64_t)P.active[i] : i;
    constexpr bool resumable = RESUMABLE;
    const bool resume = RESUMABLE && P.resume;

    float q[St::N], qt[St::N];
    if (!load_problem<C, L, KIND>(P, S, resume ? P.joints : P.seeds, p, q)) {
        write_nonfinite<C, L, KIND>(P, p, q, resumable);
        if (fin) {
#pragma unroll
            for (int j = 0; j < St::N; ++j) fin->q[j] = q[j];
            fin->cost = fin->pcost = NAN;
            fin->conv = false;
        }
        return;
    }
    int iters = 0, accepts = 0, itt = -1, flags = 0;
    bool done = false, stalled = false, tsolved = false;
    float lam = P.lambda0;
    // target_exit: the problem also ends in the pass in which a problem of
    // its target in the same run of lanes meets the tolerance (problems
    // started from their seeds in this launch only)
    const bool texit = TEXIT && !resume;
    const uint64_t trun = texit ? target_run_mask(p / P.K) : 0;
    if (resume) {
        const int st = P.st_state[p];
        iters = P.iters[p];
        accepts = P.accepts[p];
        itt = P.iters_to_tol[p];
        flags = st & 0xffff;
        stalled = (st & PK_ST_STALLED) != 0;
        done = (st & PK_ST_DONE) != 0;
        lam = P.st_lambda[p];
    }
    const int iter_end = resumable ? min(P.max_iters, iters + P.iter_budget) : P.max_iters;
    float cost = 0.f, pcost = 0.f, perr[C], rerr[C];
#pragma unroll
    for (int c = 0; c < C; ++c) perr[c] = rerr[c] = 0.f;
#pragma unroll
    for (int j = 0; j < St::N; ++j) qt[j] = q[j];
    bool first = true, need_j = true;

    for (;;) {
        // keep LDS-resident state out of registers across iterations
        __asm__ volatile("" ::: "memory");
        bool ok = true;
        if (!first) {
            if constexpr (C > 1) {
                if (need_j) {
                    // Jacobian at the current point (after an accept) -> LDS.
#pragma unroll
                    for (int c = 0; c < C; ++c) eval_jacobian_chain<C, L, KIND>(rb, P, qr, S, q, c);
                    need_j = false;
                }
            }
            float delta[St::N];
            ok = lane_step<C, L, KIND>(rb, P, qr, S, q, lam, flags, delta);
            if constexpr (C == 1) {
                if (!ok) ok = step_fp64_1<L, KIND>(rb, P, qr, S, q, lam, delta);
            }
#pragma unroll
            for (int j = 0; j < St::N; ++j) qt[j] = q[j] + delta[j];
        }
        bool met = false;   // the point taken in this pass meets the tolerance
        float ct = INFINITY, pct = 0.f, pe_t[C], re_t[C];
#pragma unroll
        for (int c = 0; c < C; ++c) pe_t[c] = re_t[c] = 0.f;
        if constexpr (C == 1) {
            // a taken point's Jacobian is formed here, from the same FK
            if (ok) (void)eval_point1<L, KIND>(rb, P, qr, S, qt, first, cost, ct, pct, pe_t, re_t);
        } else {
            if (ok) eval_cost<C, L, KIND>(rb, P, qr, S, qt, ct, pct, pe_t, re_t);
        }
        if (first) {
            cost = ct;
            pcost = pct;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                perr[c] = pe_t[c];
                rerr[c] = re_t[c];
            }
            if (!resume) {
                itt = meets_tol<C, L, KIND>(P, perr, rerr) ? 0 : -1;
                done = P.early_exit && itt == 0;
            }
            met = itt == 0;
            first = false;
        } else {
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
                    met = true;
                }
            } else {
                if (lam >= P.lambda_max) {
                    stalled = true;
                    done = true;
                }
                lam = fminf(lam * P.nu_up, P.lambda_max);
            }
            write_trace<C, L, KIND>(P, iters - 1, p, q, acc);
        }
        if (texit) {   // uniform: every lane of the pass takes part
            const uint64_t others = __ballot(met) & trun & ~(1ull << (threadIdx.x & 63));
            if (!done && others) {
                done = true;
                tsolved = true;
            }
        }
        if (done || iters >= iter_end) break;
    }
    const bool finished = done || iters >= P.max_iters;
    write_result<C, L, KIND>(P, p, q, cost, pcost, perr, rerr, iters, accepts, itt, flags, stalled, finished,
                             tsolved);
    if (fin) {
#pragma unroll
        for (int j = 0; j < St::N; ++j) fin->q[j] = q[j];
        fin->cost = cost;
        fin->pcost = pcost;
        fin->conv = meets_tol<C, L, KIND>(P, perr, rerr);
    }
    if (resumable) {
        P.st_lambda[p] = lam;
        P.st_state[p] = flags | (stalled ? PK_ST_STALLED : 0) | (finished ? PK_ST_DONE : 0);
    }
}

}  // namespace lane
}  // namespace pk
