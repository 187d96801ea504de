// Wave-per-problem Levenberg-Marquardt IK kernel for any revolute tree
// (up to 64 joints, 8 EEs): one problem per 64-lane wavefront, lane j owns
// joint j, lane k < m also owns EE k.
//
//  * FK runs level by level over tree depth; a lane reads its parent's frame
//    with a lane shuffle.
//  * EE lanes evaluate the pose log and residual; the right-Jacobian-inverse
//    blocks and the Jacobian columns are formed only for accepted points.
//    Lane j writes its column (6 rows per EE) to LDS.
//  * Tree structure of the normal equations.  (J^T J)_ij is non-zero only
//    when one of i, j is an ancestor of the other (both sit on a path from the
//    root to an EE), so lane j stores row j of the lower triangle indexed by
//    ancestor depth: r[d] = A(j, ancestor of j at depth d), plus its diagonal.
//    Eliminating joints leaves first (descending index, parents have smaller
//    indices) creates no fill: the update of step k touches only the
//    ancestors of k, which already form a dense block.  The factorization is
//    A = L^T D L without square roots; one step costs O(depth) per lane and
//    the back substitution runs level by level over depth.
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

PK_DEV int bcast_i(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

PK_DEV uint64_t bcast_u64(uint64_t v, int lane)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
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

// Orders LDS accesses across the lanes of the wavefront (one lane writes,
// the others read): without it the compiler may treat the lanes as unrelated
// threads and move a lane's read ahead of another lane's write.  The kernel's
// workgroup is a single wavefront, so this is the only ordering its LDS
// exchanges need (LDS accesses of one wavefront complete in order).
// A mimic lane's value from its driver lane's (every lane takes part in the
// exchange; the others keep theirs).
PK_DEV float mimic_rule(float q, int src, float a, float b)
{
    const float qd = __shfl(q, src < 0 ? 0 : src, 64);
    return src >= 0 ? a * qd + b : q;
}

PK_DEV void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

PK_DEV float recip(float x) { return rcp(x); }
PK_DEV double recip(double x) { return 1.0 / x; }

// Byte d of the packed ancestor table of this lane (ancestor at depth d).
template <int DMAX>
PK_DEV int anc_lane(const uint32_t (&ancp)[DMAX / 4], int d)
{
    return (int)((ancp[d >> 2] >> (8 * (d & 3))) & 0xffu);
}

// LDS layout of one wavefront's problem (float offsets).
template <int DMAX, int MMAX>
struct Lds {
    static constexpr int JS = 6 * MMAX;            // floats per Jacobian column row
    static constexpr int ES = 60;                  // floats per EE record
    static constexpr int JC = 0;                   // [64][JS]  Jacobian columns (current point)
    static constexpr int RS = JC + 64 * JS;        // [6 * MMAX] EE residual rows (current point)
    static constexpr int FR = RS + 6 * MMAX;       // [64][12] joint frames O, p (last evaluated point)
    static constexpr int EX = FR + 64 * 12;        // [MMAX][ES] EE records (last evaluated point)
    static constexpr int PV = EX + MMAX * ES;      // pivot rows of an elimination step: DMAX + 2 values each, FP64-sized
    static constexpr int FLOATS = PV + 2 * PK_STEP_PIVOTS * (DMAX + 2);
};
// Slots of an EE record.
enum { E_PE = 0, E_R = 4, E_RE = 12, E_LG = 24, E_M = 36, E_N = 48 };

// Per-lane constants of the joint and EE owned by this lane.
struct LaneConst {
    float G[9], t[3], lo, hi, qr;
    int parent, depth;
    bool pris;            // prismatic joint (else revolute)
    bool var;             // the joint is a variable (not a mimic joint)
    float eG[9], et[3];
    int ee_joint, ee_kind;
    float tp[3], tR[9];   // this lane's EE target
};

// Scalars of one evaluated point (the rest of it is in LDS).
struct PointVal {
    float rl, rr, dl;     // joint lane: limit and rest residuals, limit-row derivative
    float perr, rerr;     // EE lane errors
    float cost, pcost;    // uniform
    bool meets;           // uniform
};

// FK, EE residuals, limit/rest residuals and the cost at q.  Joint frames
// and EE records of the point go to LDS.
template <int DMAX, int MMAX>
PK_DEV void point(const SolveParams &P, const LaneConst &C, int lane, int n, int m, int max_depth,
                  float q, float *lds, PointVal &X)
{
    using L = Lds<DMAX, MMAX>;
    const bool isj = lane < n, ise = lane < m;
    float s = 0.f, c = 1.f;
    if (isj && !C.pris) joint_sincos(q, s, c);
    // FK, one tree level at a time, through LDS.
    for (int d = 0; d <= max_depth; ++d) {
        if (C.depth == d) {
            float Op[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f}, pp[3] = {0.f, 0.f, 0.f};
            if (C.parent >= 0) {
                const float *f = lds + L::FR + C.parent * 12;
#pragma unroll
                for (int u = 0; u < 9; ++u) Op[u] = f[u];
#pragma unroll
                for (int u = 0; u < 3; ++u) pp[u] = f[9 + u];
            }
            float O[9], pos[3];
            joint_step(Op, pp, C.G, C.t, s, c, O, pos);
            if (C.pris) joint_slide(O, q, pos);
            float *f = lds + L::FR + lane * 12;
#pragma unroll
            for (int u = 0; u < 9; ++u) f[u] = O[u];
#pragma unroll
            for (int u = 0; u < 3; ++u) f[9 + u] = pos[u];
        }
        wave_sync();
    }
    // EE lanes: frame of the EE joint, residual, errors.
    float ecost = 0.f;
    X.perr = X.rerr = 0.f;
    if (ise) {
        const float *f = lds + L::FR + C.ee_joint * 12;
        float Oe[9], pj[3], Re[9], pe[3], d[3], r[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int u = 0; u < 9; ++u) Oe[u] = f[u];
#pragma unroll
        for (int u = 0; u < 3; ++u) pj[u] = f[9 + u];
        ee_frame(Oe, pj, C.eG, C.et, Re, pe);
#pragma unroll
        for (int u = 0; u < 3; ++u) d[u] = pe[u] - C.tp[u];
        X.perr = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        float *e = lds + L::EX + lane * L::ES;
        if (C.ee_kind == PK_EE_POSE) {
            const PoseLog lg = pose_log(C.tR, Re, d);
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                r[u] = P.w_pos * lg.rho[u];
                r[3 + u] = P.w_rot * lg.phi[u];
                e[E_LG + u] = lg.rho[u];
                e[E_LG + 3 + u] = lg.phi[u];
            }
            e[E_LG + 6] = lg.theta;
            e[E_LG + 7] = lg.sh;
            e[E_LG + 8] = lg.ch;
            X.rerr = lg.theta;
        } else {
#pragma unroll
            for (int u = 0; u < 3; ++u) r[u] = P.w_pos * d[u];
        }
#pragma unroll
        for (int u = 0; u < 3; ++u) e[E_PE + u] = pe[u];
#pragma unroll
        for (int u = 0; u < 6; ++u) {
            e[E_R + u] = r[u];
            ecost += r[u] * r[u];
        }
#pragma unroll
        for (int u = 0; u < 9; ++u) e[E_RE + u] = Re[u];
    }
    // Joint lanes: limit and rest rows.
    float jcost = 0.f;
    X.rl = X.rr = X.dl = 0.f;
    if (isj && C.var) {
        const float over = q - C.hi, under = C.lo - q;
        X.rl = P.w_limit * (fmaxf(over, 0.f) + fmaxf(under, 0.f));
        X.rr = P.w_rest * (q - C.qr);
        X.dl = over > 0.f ? P.w_limit : (under > 0.f ? -P.w_limit : 0.f);
        jcost = X.rl * X.rl + X.rr * X.rr;
    }
    X.pcost = wave_sum(ecost);
    X.cost = wave_sum(ecost + jcost);
    bool ok = true;
    if (ise) ok = X.perr <= P.tol_pos && (C.ee_kind != PK_EE_POSE || X.rerr <= P.tol_rot);
    X.meets = __all(ok);
}

// Jacobian of the last evaluated point: lane j's column (one 6-row block per
// EE, zero where j is not an ancestor of the EE) and the EE residual rows
// into LDS.
template <int DMAX, int MMAX>
PK_DEV void jacobian(const RobotC *__restrict__ rb, const SolveParams &P, int lane, int n, int m,
                     float *lds)
{
    using L = Lds<DMAX, MMAX>;
    const bool isj = lane < n, ise = lane < m;
    if (ise) {
        float *e = lds + L::EX + lane * L::ES;
        if (rb->e[lane].kind == PK_EE_POSE) {
            PoseLog lg;
            float Re[9], M[9], Nb[9];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                lg.rho[u] = e[E_LG + u];
                lg.phi[u] = e[E_LG + 3 + u];
            }
            lg.theta = e[E_LG + 6];
            lg.sh = e[E_LG + 7];
            lg.ch = e[E_LG + 8];
#pragma unroll
            for (int u = 0; u < 9; ++u) Re[u] = e[E_RE + u];
            jr_inv_blocks(lg, Re, M, Nb);
#pragma unroll
            for (int u = 0; u < 9; ++u) {
                e[E_M + u] = M[u];
                e[E_N + u] = Nb[u];
            }
        }
#pragma unroll
        for (int u = 0; u < 6; ++u) lds[L::RS + 6 * lane + u] = e[E_R + u];
    }
    wave_sync();
    const float *f = lds + L::FR + (isj ? lane : 0) * 12;
    const float om[3] = {f[2], f[5], f[8]}, pj[3] = {f[9], f[10], f[11]};
    const bool pris = isj && rb->j[lane].type == PK_JOINT_PRISMATIC;
    float *jc = lds + L::JC + lane * L::JS;
#pragma unroll
    for (int k = 0; k < MMAX; ++k) {
        if (k < m) {
            const float *e = lds + L::EX + k * L::ES;
            const int kind = rb->e[k].kind;
            const bool anc = isj && ((rb->anc[k] >> lane) & 1ull);
            float col[6], v[3], wv[3];
            joint_twist(pris, om, pj, e + E_PE, v, wv);
            if (kind == PK_EE_POSE) {
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    const float *Mu = e + E_M + 3 * u, *Nu = e + E_N + 3 * u;
                    float mv = Mu[0] * v[0] + Mu[1] * v[1] + Mu[2] * v[2];
                    float nw = Nu[0] * wv[0] + Nu[1] * wv[1] + Nu[2] * wv[2];
                    float mw = Mu[0] * wv[0] + Mu[1] * wv[1] + Mu[2] * wv[2];
                    col[u] = anc ? P.w_pos * (mv + nw) : 0.f;
                    col[3 + u] = anc ? P.w_rot * mw : 0.f;
                }
            } else {
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    col[u] = anc ? P.w_pos * v[u] : 0.f;
                    col[3 + u] = 0.f;
                }
            }
#pragma unroll
            for (int u = 0; u < 6; ++u) jc[6 * k + u] = col[u];
        }
    }
}

// Mimic joints: each adds its column, times its multiplier, into its
// driver's, then drops it (a mimic joint is not a variable).
template <int DMAX, int MMAX>
PK_DEV void merge_mimic(const RobotC *__restrict__ rb, int lane, int n, int m, float *lds)
{
    using L = Lds<DMAX, MMAX>;
    const int nm = rb->n_mimic;
    for (int i = 0; i < nm; ++i) {
        const int ml = rb->mimic_list[i];
        if (lane == rb->j[ml].mimic_src) {
            const float a = rb->j[ml].mimic_a;
            float *jd = lds + L::JC + lane * L::JS;
            const float *jm = lds + L::JC + ml * L::JS;
#pragma unroll
            for (int u = 0; u < L::JS; ++u)
                if (u < 6 * m) jd[u] += a * jm[u];
        }
        wave_sync();
    }
    if (lane < n && rb->j[lane].var < 0) {
        float *jc = lds + L::JC + lane * L::JS;
#pragma unroll
        for (int u = 0; u < L::JS; ++u) jc[u] = 0.f;
    }
    wave_sync();
}

// Row j of J^T J by ancestor depth, r[d] = A(j, ancestor of j at depth d)
// for d < depth j, in precision T from the FP32 columns in LDS (products of
// FP32 entries summed in T), and g = J^T r over the EE rows; returns the
// diagonal A_jj.
template <int DMAX, int MMAX, typename T>
PK_DEV T jtj_rows(const float *lds, const uint32_t (&ancp)[DMAX / 4], int lane, int dep, int m,
                  int max_depth, T (&r)[DMAX], T &g)
{
    using L = Lds<DMAX, MMAX>;
    float cj[6 * MMAX];
    const float *own = lds + L::JC + lane * L::JS;
#pragma unroll
    for (int k = 0; k < MMAX; ++k)
#pragma unroll
        for (int u = 0; u < 6; ++u) cj[6 * k + u] = k < m ? own[6 * k + u] : 0.f;
    g = 0;
#pragma unroll
    for (int k = 0; k < MMAX; ++k)
        if (k < m)
#pragma unroll
            for (int u = 0; u < 6; ++u) g += (T)cj[6 * k + u] * (T)lds[L::RS + 6 * k + u];
    T diag = 0;
    if constexpr (sizeof(T) == 8) {
        // FP64 (cold path): one Jacobian row at a time, all depths at once.
        T acc[DMAX];
#pragma unroll
        for (int d = 0; d < DMAX; ++d) acc[d] = 0;
        for (int e = 0; e < 6 * m; ++e) {
            const T ce = (T)own[e];
#pragma unroll
            for (int d = 0; d < DMAX; ++d)
                if (d <= max_depth) acc[d] += ce * (T)lds[L::JC + anc_lane<DMAX>(ancp, d) * L::JS + e];
        }
#pragma unroll
        for (int d = 0; d < DMAX; ++d) {
            r[d] = d < dep ? acc[d] : (T)0;
            diag = d == dep ? acc[d] : diag;
        }
        return diag;
    }
#pragma unroll
    for (int d = 0; d < DMAX; ++d) {
        T s = 0;
        if (d <= max_depth) {
            const float *ca = lds + L::JC + anc_lane<DMAX>(ancp, d) * L::JS;
#pragma unroll
            for (int k = 0; k < MMAX; ++k)
                if (k < m)
#pragma unroll
                    for (int u = 0; u < 6; ++u) s += (T)cj[6 * k + u] * (T)ca[6 * k + u];
        }
        r[d] = d < dep ? s : (T)0;
        diag = d == dep ? s : diag;
        __asm__ volatile("" ::: "memory");   // one ancestor row in flight at a time
    }
    return diag;
}

// Solve (A + lam diag(max(A_jj, floor))) delta = -g for the tree-structured A
// given as depth-indexed rows r and undamped diagonal dgu (consumed).
// Returns false if a pivot is not above thresh_rel * max damped diagonal
// (thresh_rel > 0) or not positive and finite.  `desc` has bit k set when
// this lane's joint is a proper ancestor of joint k; the lane's joint is
// pivot `pos` of elimination step `step` (-1: no joint).  Lane i's `stab`
// holds pivot i of the schedule (bits 0-7), that pivot's depth (8-15) and
// the first pivot of step i (16-23).  `slots` (LDS, PK_STEP_PIVOTS rows of
// DMAX + 2 values of T) carry a step's pivot rows.
template <int DMAX, typename T>
PK_DEV bool tree_solve(T (&r)[DMAX], T dgu, T g, float lam, float dfloor, float thresh_rel,
                       int lane, int n, int dep, uint64_t desc, int step, int pos, int nstep,
                       uint32_t stab, const uint32_t (&ancp)[DMAX / 4], int max_depth, T *slots,
                       float &delta, bool unit = false)
{
    constexpr int SS = DMAX + 2;
    const bool isj = lane < n;
    T dg = isj ? dgu + (T)lam * (dgu > (T)dfloor ? dgu : (T)dfloor) : (T)0;
    // A mimic joint's row and column are zero: its pivot is set to the
    // largest damped diagonal, so that it passes the test and leaves x = 0.
    const float dmax = wave_max(unit ? 0.f : (float)dg);
    if (unit) dg = (T)(dmax > 0.f ? dmax : 1.f);
    T thresh = 0;
    if (thresh_rel > 0.f) thresh = (T)thresh_rel * (T)dmax;
    T b = isj ? -g : (T)0;
    bool bad = false;
    // Leaves first, one step of mutually unrelated joints at a time: the
    // step's pivot lanes put their rows, pivots and right-hand sides in LDS,
    // then every lane removes from its row the pivots it is an ancestor of.
    // Every pivot is tested; a failed test ends the solve after the loop.
    for (int st = 0; st < nstep; ++st) {
        wave_sync();   // the previous step's reads are done
        if (step == st) {
            // Up to 16 depths the whole row goes out, zero past the joint's
            // own depth, so that readers need no depth-dependent branches.
            T *sl = slots + pos * SS;
#pragma unroll
            for (int d = 0; d < DMAX; ++d) {
                if (DMAX > 16 && (d & 3) == 0 && d >= dep) break;
                sl[d] = d < dep ? r[d] : (T)0;
            }
            sl[DMAX] = dg;
            sl[DMAX + 1] = b;
        }
        wave_sync();   // the step's rows are visible to every lane
        const int i0 = (int)((unsigned)bcast_i((int)stab, st) >> 16);
        const int i1 = st + 1 < nstep ? (int)((unsigned)bcast_i((int)stab, st + 1) >> 16) : n;
        for (int i = i0; i < i1; ++i) {
            const unsigned e = (unsigned)bcast_i((int)stab, i);
            const int k = (int)(e & 0xffu), dk = (int)((e >> 8) & 0xffu);
            const T *sk = slots + (i - i0) * SS;
            const T piv = sk[DMAX], bk = sk[DMAX + 1];
            bad = bad || !(piv > thresh) || !(piv < (T)INFINITY);
            const bool is_anc = (desc >> k) & 1ull;
            const T sk_dep = sk[dep > 0 ? dep : 0];
            const T sel = is_anc ? sk_dep : (T)0;
            const T c = sel * recip(piv);
#pragma unroll
            for (int d = 0; d < DMAX; ++d) {
                if (DMAX > 16 && (d & 3) == 0 && d >= dk) break;
                r[d] -= c * sk[d];
            }
            dg -= c * sel;
            b -= c * bk;
        }
    }
    if (bad) return false;
    // Back substitution, root first: x_j = (b_j - sum_d r_j[d] x_anc(d)) / pivot_j.
    const T ipj = isj ? recip(dg) : (T)0;
    T s = 0, x = 0;
#pragma unroll
    for (int D = 0; D < DMAX; ++D) {
        if (D <= max_depth) {
            if (dep == D) x = (b - s) * ipj;
            const T xa = __shfl(x, anc_lane<DMAX>(ancp, D), 64);
            if (dep > D) s += r[D] * xa;
        }
    }
    delta = isj ? (float)x : 0.f;
    return true;
}

// One LM problem (active index wi) on this wavefront; resumable (state in
// HBM, at most P.iter_budget iterations per launch when P.st_state is set).
template <int DMAX, int MMAX>
PK_DEV void wave_problem(const RobotC *__restrict__ rb, const SolveParams &P, float *lds, int64_t wi)
{
    using L = Lds<DMAX, MMAX>;
    const int lane = threadIdx.x & 63;     // wavefronts of a multi-wave block each run their own problem
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
    C.qr = (P.q_rest && isj && rb->j[jl].var >= 0) ? P.q_rest[rb->j[jl].var] : rb->j[jl].mid;
    C.parent = rb->j[jl].parent;
    C.depth = isj ? rb->j[jl].depth : -1;
    C.pris = isj && rb->j[jl].type == PK_JOINT_PRISMATIC;
    // Lane j holds joint j; its variable (or, for a mimic joint, the rule
    // on its driver's lane).
    const int vi = isj ? rb->j[jl].var : -1, nv = rb->nv;
    C.var = vi >= 0;
    const int msrc = isj ? rb->j[jl].mimic_src : -1;
    const float ma = isj ? rb->j[jl].mimic_a : 0.f, mb = isj ? rb->j[jl].mimic_b : 0.f;
    const bool any_mimic = rb->n_mimic > 0;
#pragma unroll
    for (int u = 0; u < 9; ++u) C.eG[u] = rb->e[el].G[u];
#pragma unroll
    for (int u = 0; u < 3; ++u) C.et[u] = rb->e[el].t[u];
    C.ee_joint = rb->e[el].joint;
    C.ee_kind = rb->e[el].kind;
    uint32_t ancp[DMAX / 4];
    const uint32_t *arow = (const uint32_t *)rb->anc_at[jl];
#pragma unroll
    for (int i = 0; i < DMAX / 4; ++i) ancp[i] = isj ? arow[i] : 0u;
    const uint64_t desc = isj ? rb->jdesc[jl] : 0ull;
    const int step = isj ? rb->step_of[jl] : -1, spos = isj ? rb->step_pos[jl] : 0;
    const int nstep = rb->nstep;
    uint32_t stab = 0;
    if (isj) {
        const int pj = rb->step_joint[lane];
        stab = (uint32_t)pj | ((uint32_t)rb->j[pj].depth << 8);
    }
    if (lane < nstep) stab |= (uint32_t)rb->step_start[lane] << 16;
    const int dep = C.depth;

    bool fin = true;
    float q = 0.f;
    if (C.var) q = (resume ? P.joints : P.seeds)[(int64_t)vi * N + p];
    if (any_mimic) q = mimic_rule(q, msrc, ma, mb);
    if (isj) fin = isfinite(q);
    if (ise) {
        const int off = rb->e[el].tgt_off;
        const int W = C.ee_kind == PK_EE_POSE ? 7 : 3;
        float v[7] = {0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int u = 0; u < 7; ++u) {
            if (u < W) {
                v[u] = P.targets[(int64_t)(off + u) * T + t];
                fin = fin && isfinite(v[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < 3; ++u) C.tp[u] = v[u];
        quat_to_rot(v[3], v[4], v[5], v[6], C.tR);
    }
    const bool finite = __all(fin);
    if (!finite) {
        if (C.var) {
            P.joints[(int64_t)vi * N + p] = q;
            for (int it = 0; it < P.trace_iters; ++it)
                P.trace_q[((int64_t)it * nv + vi) * N + p] = q;
        }
        if (ise) {
            if (P.pos_err) P.pos_err[(int64_t)lane * N + p] = NAN;
            if (P.rot_err) P.rot_err[(int64_t)lane * N + p] = NAN;
        }
        if (lane == 0) {
            if (P.cost) P.cost[p] = NAN;
            if (P.pose_cost) P.pose_cost[p] = NAN;
            if (P.iters) P.iters[p] = 0;
            if (P.accepts) P.accepts[p] = 0;
            if (P.status) P.status[p] = PK_NONFINITE;
            if (P.iters_to_tol) P.iters_to_tol[p] = -1;
            if (resumable) P.st_state[p] = PK_ST_DONE;
            for (int it = 0; it < P.trace_iters; ++it) P.trace_acc[(int64_t)it * N + p] = 0;
        }
        return;
    }

    int iters = 0, accepts = 0, itt = -1, flags = 0;
    bool done = false, stalled = false;
    float lam = P.lambda0;
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

    // Current point: scalars and J^T J rows in registers, Jacobian columns
    // and residual rows in LDS.  Each pass evaluates one point (first the
    // start point, then each trial), so every stage has a single call site.
    PointVal X;
    float cost = INFINITY, pcost = 0.f, perr = 0.f, rerr = 0.f, rl = 0.f, rr = 0.f, dl = 0.f;
    float g = 0.f, dgu = 0.f, rows[DMAX];
#pragma unroll
    for (int d = 0; d < DMAX; ++d) rows[d] = 0.f;
    bool meets = false;
    float qt = q;
    bool first = true, evaluate = true;
    for (;;) {
        bool acc = false;
        if (evaluate) {
            point<DMAX, MMAX>(P, C, lane, n, m, max_depth, qt, lds, X);
            acc = first || X.cost < cost;
        }
        if (!first) ++iters;
        if (acc) {
            q = qt;
            cost = X.cost;
            pcost = X.pcost;
            perr = X.perr;
            rerr = X.rerr;
            rl = X.rl;
            rr = X.rr;
            dl = X.dl;
            meets = X.meets;
            if (first) {
                if (!resume) {
                    itt = meets ? 0 : -1;
                    done = P.early_exit && itt == 0;
                }
            } else {
                lam = fmaxf(lam / P.nu_down, P.lambda_min);
                ++accepts;
                if (meets) {
                    if (itt < 0) itt = iters;
                    if (P.early_exit) done = true;
                }
            }
            if (!done && iters < iter_end) {
                wave_sync();
                jacobian<DMAX, MMAX>(rb, P, lane, n, m, lds);
                wave_sync();
                if (any_mimic) merge_mimic<DMAX, MMAX>(rb, lane, n, m, lds);
                float ge;
                dgu = jtj_rows<DMAX, MMAX, float>(lds, ancp, lane, dep, m, max_depth, rows, ge) +
                      (C.var ? dl * dl + P.w_rest * P.w_rest : 0.f);
                g = isj ? ge + dl * rl + P.w_rest * rr : 0.f;
            }
        } else if (!first) {
            if (lam >= P.lambda_max) {
                stalled = true;
                done = true;
            }
            lam = fminf(lam * P.nu_up, P.lambda_max);
        }
        if (!first && iters - 1 < P.trace_iters) {
            if (C.var) P.trace_q[((int64_t)(iters - 1) * nv + vi) * N + p] = q;
            if (lane == 0) P.trace_acc[(int64_t)(iters - 1) * N + p] = acc ? 1 : 0;
        }
        first = false;
        if (done || iters >= iter_end) break;
        // Damped step from the current point.
        float delta = 0.f;
        bool ok;
        {
            float r[DMAX];
#pragma unroll
            for (int d = 0; d < DMAX; ++d) r[d] = rows[d];
            ok = tree_solve<DMAX, float>(r, dgu, g, lam, P.damping_floor, P.pivot_rel, lane, n, dep,
                                         desc, step, spos, nstep, stab, ancp, max_depth, lds + L::PV,
                                         delta, isj && !C.var);
        }
        if (!ok) {
            // Re-form the damped system and gradient in FP64 from the FP32
            // Jacobian and residuals, and solve again.
            flags |= PK_FLAG_FP64;
            double r[DMAX], gd;
            double dgd = jtj_rows<DMAX, MMAX, double>(lds, ancp, lane, dep, m, max_depth, r, gd) +
                         (C.var ? (double)dl * dl + (double)P.w_rest * P.w_rest : 0.0);
            gd += (double)dl * rl + (double)P.w_rest * rr;
            ok = tree_solve<DMAX, double>(r, dgd, isj ? gd : 0.0, lam, P.damping_floor, 0.f, lane,
                                          n, dep, desc, step, spos, nstep, stab, ancp, max_depth,
                                          (double *)(lds + L::PV), delta, isj && !C.var);
        }
        qt = q + delta;
        if (any_mimic) qt = mimic_rule(qt, msrc, ma, mb);
        evaluate = ok;   // a failed solve counts as a rejected step
    }
    const bool finished = done || iters >= P.max_iters;
    if (finished)
        for (int it = iters; it < P.trace_iters; ++it) {
            if (C.var) P.trace_q[((int64_t)it * nv + vi) * N + p] = q;
            if (lane == 0) P.trace_acc[(int64_t)it * N + p] = 0;
        }
    if (C.var) P.joints[(int64_t)vi * N + p] = q;
    if (ise) {
        if (P.pos_err) P.pos_err[(int64_t)lane * N + p] = perr;
        if (P.rot_err) P.rot_err[(int64_t)lane * N + p] = rerr;
    }
    if (lane == 0) {
        if (P.cost) P.cost[p] = cost;
        if (P.pose_cost) P.pose_cost[p] = pcost;
        if (P.iters) P.iters[p] = iters;
        if (P.accepts) P.accepts[p] = accepts;
        if (P.status)
            P.status[p] = (meets ? PK_CONVERGED : (stalled ? PK_STALLED : PK_MAX_ITERS)) | flags;
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

template <int DMAX, int MMAX>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((DMAX <= 16 && MMAX <= 4) ? 2 : 1))) void lm_wave_kernel(const RobotC *__restrict__ rb, SolveParams P)
{
    using L = Lds<DMAX, MMAX>;
    __shared__ __attribute__((aligned(16))) float lds[L::FLOATS];
    const int64_t nact = P.n_active ? (int64_t)*P.n_active : P.N;
    int64_t wi = P.queue_head ? pop_item_wave(P.queue_head) : (int64_t)blockIdx.x;
    while (wi < nact) {
        wave_problem<DMAX, MMAX>(rb, P, lds, wi);
        if (!P.queue_head) break;
        __syncthreads();
        wi = pop_item_wave(P.queue_head);
    }
}

template <int DMAX, int MMAX>
hipError_t launch_wave(const RobotC *rb, const SolveParams &P, int persist_blocks, hipStream_t s)
{
    int64_t grid = P.N;
    if (P.queue_head && persist_blocks > 0 && persist_blocks < grid) grid = persist_blocks;
    hipLaunchKernelGGL((lm_wave_kernel<DMAX, MMAX>), dim3((unsigned)grid), dim3(64), 0, s, rb, P);
    return hipGetLastError();
}

}  // namespace wave
}  // namespace pk
