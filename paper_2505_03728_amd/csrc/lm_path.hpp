// Wavefront-per-problem Levenberg-Marquardt IK kernel in the path-pair
// layout (PathC): one problem per 64-lane wavefront, lane l holds the pair
// (joint, EE path) -- every joint on the path from the root to EE k has a
// lane in path k, so a joint that several EE paths share has one copy per
// path, and a joint on no EE path has one lane of its own.
//
//  * FK: each lane starts from its joint's transform relative to its parent
//    and, in ceil(log2(levels)) rounds, composes it with the transform held
//    by the ancestor at which its own currently starts (path doubling along
//    the lane's path, through LDS).  Copies of a joint compute the same frame.
//  * Lane (j, k) forms joint j's Jacobian block for EE k and, from the blocks
//    of the ancestors in its path, EE k's part of row j of J^T J
//    ((J^T J)_ja sums over the EEs below both joints).
//  * Elimination follows the tree's leaves-first schedule.  The pivots of a
//    step are mutually unrelated, so at most one of them is owned by a given
//    path and every lane takes at most one update per step: the paths below a
//    shared joint eliminate their own joints side by side, each into its own
//    copies of the shared rows.  Once no path other than the owner's has
//    updates left for a shared joint, the owner copy adds the other copies'
//    rows (one merge phase for a whole run of shared joints); from then on
//    only the owner copy is updated and it becomes the pivot row.
//  * Decisions are uniform across the wavefront, so the LM loop runs without
//    divergence, as in the lane-per-joint kernel.
//
// Method: Sec. III-A (LM on the sum of squared weighted residuals, limits as
// penalties), Sec. III-B (FK), Sec. III-C (joint pose, limit and rest costs).
#pragma once

#include "lm_wave.hpp"

namespace pk {
namespace path {

using wave::bcast_i;
using wave::PointVal;
using wave::recip;
using wave::wave_sync;

// Wave-wide reductions on DPP lane moves (no LDS traffic): an inclusive scan
// within each row of 16 lanes (row shifts by 1, 2, 4, 8), then the row totals
// carried across rows (row broadcasts of lanes 15 and 31); lane 63 ends with
// the total, which readlane makes uniform.  Lanes a move does not reach add
// the identity.
template <typename Op>
PK_DEV float dpp_reduce(float v, int identity, Op op)
{
    v = op(v, __int_as_float(__builtin_amdgcn_update_dpp(identity, __float_as_int(v), 0x111, 0xf, 0xf, false)));
    v = op(v, __int_as_float(__builtin_amdgcn_update_dpp(identity, __float_as_int(v), 0x112, 0xf, 0xf, false)));
    v = op(v, __int_as_float(__builtin_amdgcn_update_dpp(identity, __float_as_int(v), 0x114, 0xf, 0xf, false)));
    v = op(v, __int_as_float(__builtin_amdgcn_update_dpp(identity, __float_as_int(v), 0x118, 0xf, 0xf, false)));
    v = op(v, __int_as_float(__builtin_amdgcn_update_dpp(identity, __float_as_int(v), 0x142, 0xa, 0xf, false)));
    v = op(v, __int_as_float(__builtin_amdgcn_update_dpp(identity, __float_as_int(v), 0x143, 0xc, 0xf, false)));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

PK_DEV float wave_sum(float v)
{
    return dpp_reduce(v, 0, [](float a, float b) { return a + b; });
}

// (of non-negative values)
PK_DEV float wave_max_nonneg(float v)
{
    return dpp_reduce(v, 0, [](float a, float b) { return fmaxf(a, b); });
}

// The call's parameters in the kernel-argument segment (constant memory).
// path_problem reads them through this pointer, so that in its long LM loop
// a field is fetched with a scalar load where it is used instead of every
// field being held in SGPRs (and spilled) across the loop.
using KParams = const __attribute__((address_space(4))) SolveParams;

// The kernel argument at byte `offset` of the argument segment.
PK_DEV KParams *kernel_params_at(size_t offset)
{
    return (KParams *)((const __attribute__((address_space(4))) char *)__builtin_amdgcn_kernarg_segment_ptr() +
                       offset);
}

// A wave-uniform value taken as a new one (in an SGPR) by the compiler: what
// it derives from the value is formed after this point, where it is used,
// rather than hoisted and held from an earlier one.
PK_DEV int fresh_uniform(int v)
{
    v = __builtin_amdgcn_readfirstlane(v);
    __asm__ volatile("" : "+s"(v));
    return v;
}

PK_DEV KParams *fresh_uniform(KParams *p)
{
    const uint64_t a = (uint64_t)p;
    const int lo = fresh_uniform((int)(uint32_t)a), hi = fresh_uniform((int)(uint32_t)(a >> 32));
    return (KParams *)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// LDS layout of one wavefront's problem (float offsets).
template <int DMAX, int MMAX>
struct Lds {
    static constexpr int ES = 60;                   // floats per EE record (slots as wave::E_*)
    static constexpr int SS = DMAX + 4;             // pivot slot stride, in values of the solve's type
    // One region serves three uses in turn within an LM pass: the transform
    // exchange of the FK rounds; then, per lane, the joint axis and origin of
    // the evaluated point (read by the Jacobian); then the pivot rows of the
    // solve (the axes and origins are dead by then).
    static constexpr int XF = 0;                    // [64][12] FK exchange; [64][12] axis, origin
    static constexpr int JA = XF;
    static constexpr int PV = XF;                   // [MMAX][SS] pivot rows by path, FP64-sized
    static constexpr int JC = XF + 64 * 12;         // [64][8]  Jacobian block of the lane's pair
    static constexpr int CS = JC + 64 * 8;          // [64][12] joint constants G (row-major), t
    static constexpr int EC = CS + 64 * 12;         // [MMAX][12] EE constants G, t
    static constexpr int TG = EC + MMAX * 12;       // [MMAX][12] EE targets p, R
    static constexpr int EX = TG + MMAX * 12;       // [MMAX][ES] EE records (last evaluated point)
    static constexpr int RS = EX + MMAX * ES;       // [MMAX][8] EE residual rows (current point)
    static constexpr int FLOATS = RS + MMAX * 8;
    static_assert(2 * MMAX * SS <= 64 * 12, "pivot rows fit the FK exchange region");
};

// A lane's row of the tree-structured normal matrix, by ancestor depth, in
// groups of four (register tuples the LDS stores can take directly).  N
// entries serve trees of up to N + 1 levels (a joint's row has one entry per
// proper ancestor).
template <typename T, int N>
struct Row {
    typedef T V4 __attribute__((ext_vector_type(4)));
    V4 v[N / 4];
    PK_DEV T get(int d) const { return v[d >> 2][d & 3]; }
    PK_DEV void set(int d, T x) { v[d >> 2][d & 3] = x; }
};

// What a lane holds (registers), from PathC and the joint table.
template <int DMAX>
struct LaneInfo {
    int j;          // joint (-1: idle lane)
    int grp;        // EE path (-1: joint on no EE path, or idle)
    int dep;        // depth of j (-1: idle)
    int owner;      // lane of j's owner copy (itself when idle)
    int ee;         // the EE whose joint this lane holds in that EE's path (-1)
    int step;       // elimination step of j
    int mstep;      // owner lanes of shared joints: step of the merge phase
    int gkind;      // kind of the path's EE
    int own;        // owner copy of a joint (0/1)
    int pris;       // prismatic joint (0/1)
    float lo, hi, qr;
    uint32_t ancp[DMAX / 4];   // lane of the path ancestor at depth d (byte d)
    uint64_t upd;   // bit s: this lane's row takes an update at step s
    uint32_t cp0, cp1;         // owner lanes: the other copies' lanes (bytes)
    uint32_t jump;             // byte k: lane of the path ancestor 2^k levels up
};

template <int DMAX>
PK_DEV int copy_lane(const LaneInfo<DMAX> &I, int c)
{
    const uint32_t w = c < 4 ? I.cp0 : I.cp1;
    return (int)((w >> (8 * (c & 3))) & 0xffu);
}

// Owner lanes: v plus the other copies' v (every lane takes part).
template <int DMAX, typename T>
PK_DEV T add_copies(T v, const LaneInfo<DMAX> &I, int lane, int ncopy)
{
    T acc = v;
    for (int c = 0; c < ncopy; ++c) {
        const int cl = copy_lane(I, c);
        const T o = __shfl(v, cl == PK_PATH_NONE ? lane : cl, 64);
        if (I.own && cl != PK_PATH_NONE) acc += o;
    }
    return acc;
}

// FK, EE residuals, limit/rest residuals and the cost at q.  The joint axes
// and origins and the EE records of the point go to LDS.
template <int DMAX, int MMAX>
PK_DEV void point(const SolveParams &P, const LaneInfo<DMAX> &I, int lane, int max_depth, float q,
                  float *lds, PointVal &X)
{
    using L = Lds<DMAX, MMAX>;
    const bool onp = I.grp >= 0;
    // The joint's transform in its parent's frame: R = G Rz(q), p = t, and
    // for a prismatic joint (no rotation) p = t + q G e_z.
    float R[9], p[3];
    {
        const float *cs = lds + L::CS + lane * 12;
        float G[12];
#pragma unroll
        for (int u = 0; u < 12; ++u) G[u] = cs[u];
        float s = 0.f, c = 1.f;
        if (!I.pris) joint_sincos(q, s, c);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            R[3 * r] = G[3 * r] * c + G[3 * r + 1] * s;
            R[3 * r + 1] = G[3 * r + 1] * c - G[3 * r] * s;
            R[3 * r + 2] = G[3 * r + 2];
            p[r] = G[9 + r];
        }
        if (I.pris) {
#pragma unroll
            for (int r = 0; r < 3; ++r) p[r] += q * G[3 * r + 2];
        }
    }
    // Path doubling: after the round with span s the lane's transform starts
    // at its ancestor 2s levels up (or at the root frame).
    float *mine = lds + L::XF + lane * 12;
    for (int k = 0, span = 1; span <= max_depth; ++k, span <<= 1) {
#pragma unroll
        for (int u = 0; u < 9; ++u) mine[u] = R[u];
#pragma unroll
        for (int u = 0; u < 3; ++u) mine[9 + u] = p[u];
        wave_sync();
        if (onp && I.dep >= span) {
            const float *fa = lds + L::XF + (int)((I.jump >> (8 * k)) & 0xffu) * 12;
            float Ra[9], pa[3], Rn[9];
#pragma unroll
            for (int u = 0; u < 9; ++u) Ra[u] = fa[u];
#pragma unroll
            for (int u = 0; u < 3; ++u) pa[u] = fa[9 + u];
            mm3(Ra, R, Rn);
            float pn[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) pn[r] = pa[r] + Ra[3 * r] * p[0] + Ra[3 * r + 1] * p[1] + Ra[3 * r + 2] * p[2];
#pragma unroll
            for (int u = 0; u < 9; ++u) R[u] = Rn[u];
#pragma unroll
            for (int u = 0; u < 3; ++u) p[u] = pn[u];
        }
        wave_sync();
    }
    {
        // (the last round's reads are done: the lane's slot takes its axis and origin)
        float *ja = lds + L::JA + lane * 12;
        ja[0] = R[2];
        ja[1] = R[5];
        ja[2] = R[8];
        ja[3] = p[0];
        ja[4] = p[1];
        ja[5] = p[2];
    }
    // EE lanes: EE frame, residual, errors.
    float ecost = 0.f;
    X.perr = X.rerr = 0.f;
    bool ok = true;
    if (I.ee >= 0) {
        const float *ec = lds + L::EC + I.ee * 12, *tg = lds + L::TG + I.ee * 12;
        float eG[12], Re[9], pe[3], d[3], r[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int u = 0; u < 12; ++u) eG[u] = ec[u];
        ee_frame(R, p, eG, eG + 9, Re, pe);
#pragma unroll
        for (int u = 0; u < 3; ++u) d[u] = pe[u] - tg[u];
        X.perr = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        float *e = lds + L::EX + I.ee * L::ES;
        if (I.gkind == PK_EE_POSE) {
            float Rt[9];
#pragma unroll
            for (int u = 0; u < 9; ++u) Rt[u] = tg[3 + u];
            const PoseLog lg = pose_log(Rt, Re, d);
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                r[u] = P.w_pos * lg.rho[u];
                r[3 + u] = P.w_rot * lg.phi[u];
                e[wave::E_LG + u] = lg.rho[u];
                e[wave::E_LG + 3 + u] = lg.phi[u];
            }
            e[wave::E_LG + 6] = lg.theta;
            e[wave::E_LG + 7] = lg.sh;
            e[wave::E_LG + 8] = lg.ch;
            X.rerr = lg.theta;
        } else {
#pragma unroll
            for (int u = 0; u < 3; ++u) r[u] = P.w_pos * d[u];
        }
#pragma unroll
        for (int u = 0; u < 3; ++u) e[wave::E_PE + u] = pe[u];
#pragma unroll
        for (int u = 0; u < 6; ++u) {
            e[wave::E_R + u] = r[u];
            ecost += r[u] * r[u];
        }
#pragma unroll
        for (int u = 0; u < 9; ++u) e[wave::E_RE + u] = Re[u];
        ok = X.perr <= P.tol_pos && (I.gkind != PK_EE_POSE || X.rerr <= P.tol_rot);
    }
    // Owner lanes: limit and rest rows.
    float jcost = 0.f;
    X.rl = X.rr = X.dl = 0.f;
    if (I.own) {
        const float over = q - I.hi, under = I.lo - q;
        X.rl = P.w_limit * (fmaxf(over, 0.f) + fmaxf(under, 0.f));
        X.rr = P.w_rest * (q - I.qr);
        X.dl = over > 0.f ? P.w_limit : (under > 0.f ? -P.w_limit : 0.f);
        jcost = X.rl * X.rl + X.rr * X.rr;
    }
    X.pcost = wave_sum(ecost);
    X.cost = wave_sum(ecost + jcost);
    X.meets = __all(ok);
}

// Jacobian block of the lane's pair at the last evaluated point (zero for
// lanes on no EE path) into LDS, and the EE residual rows of that point
// (kept for the solves from it while trial points overwrite the records).
template <int DMAX, int MMAX>
PK_DEV void jacobian(const SolveParams &P, const LaneInfo<DMAX> &I, int lane, float *lds)
{
    using L = Lds<DMAX, MMAX>;
    if (I.ee >= 0) {
        const float *e = lds + L::EX + I.ee * L::ES;
        float *rs = lds + L::RS + I.ee * 8;
#pragma unroll
        for (int u = 0; u < 6; ++u) rs[u] = e[wave::E_R + u];
    }
    if (I.ee >= 0 && I.gkind == PK_EE_POSE) {
        float *e = lds + L::EX + I.ee * L::ES;
        PoseLog lg;
        float Re[9], M[9], Nb[9];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            lg.rho[u] = e[wave::E_LG + u];
            lg.phi[u] = e[wave::E_LG + 3 + u];
        }
        lg.theta = e[wave::E_LG + 6];
        lg.sh = e[wave::E_LG + 7];
        lg.ch = e[wave::E_LG + 8];
#pragma unroll
        for (int u = 0; u < 9; ++u) Re[u] = e[wave::E_RE + u];
        jr_inv_blocks(lg, Re, M, Nb);
#pragma unroll
        for (int u = 0; u < 9; ++u) {
            e[wave::E_M + u] = M[u];
            e[wave::E_N + u] = Nb[u];
        }
    }
    wave_sync();
    float col[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (I.grp >= 0) {
        const float *e = lds + L::EX + I.grp * L::ES;
        const float *ja = lds + L::JA + lane * 12;
        const float om[3] = {ja[0], ja[1], ja[2]}, pj[3] = {ja[3], ja[4], ja[5]};
        float v[3], wv[3];
        joint_twist(I.pris, om, pj, e + wave::E_PE, v, wv);
        if (I.gkind == PK_EE_POSE) {
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const float *Mu = e + wave::E_M + 3 * u, *Nu = e + wave::E_N + 3 * u;
                const float mv = Mu[0] * v[0] + Mu[1] * v[1] + Mu[2] * v[2];
                const float nw = Nu[0] * wv[0] + Nu[1] * wv[1] + Nu[2] * wv[2];
                const float mw = Mu[0] * wv[0] + Mu[1] * wv[1] + Mu[2] * wv[2];
                col[u] = P.w_pos * (mv + nw);
                col[3 + u] = P.w_rot * mw;
            }
        } else {
#pragma unroll
            for (int u = 0; u < 3; ++u) col[u] = P.w_pos * v[u];
        }
    }
    float *jc = lds + L::JC + lane * 8;
#pragma unroll
    for (int u = 0; u < 6; ++u) jc[u] = col[u];
}

// The lane's part of row j of J^T J by ancestor depth, r[d] = EE k's term of
// A(j, ancestor at depth d) for d < depth j (later entries: don't-care), in precision T from the FP32
// blocks in LDS, and g = EE k's term of (J^T r)_j; returns EE k's term of A_jj.
template <int DMAX, int MMAX, typename T, int RW>
PK_DEV T jtj_rows(const float *lds, const LaneInfo<DMAX> &I, int lane, int max_depth,
                  Row<T, RW> &r, T &g)
{
    using L = Lds<DMAX, MMAX>;
    // new values (as in path_solve): the per-depth conditions are formed here
    int dep = I.dep;
    __asm__ volatile("" : "+v"(dep));
    max_depth = fresh_uniform(max_depth);
    const float *own = lds + L::JC + lane * 8;
    float cj[6];
#pragma unroll
    for (int u = 0; u < 6; ++u) cj[u] = own[u];
    g = 0;
    if (I.grp >= 0) {
        const float *rs = lds + L::RS + I.grp * 8;
#pragma unroll
        for (int u = 0; u < 6; ++u) g += (T)cj[u] * (T)rs[u];
    }
    T diag = 0;
#pragma unroll
    for (int d = 0; d < DMAX; ++d) {
        T s = 0;
        if (d <= max_depth) {
            const float *ca = lds + L::JC + wave::anc_lane<DMAX>(I.ancp, d) * 8;
#pragma unroll
            for (int u = 0; u < 6; ++u) s += (T)cj[u] * (T)ca[u];
        }
        // entries at and past the lane's depth take values no reader uses
        if (d < RW) r.set(d < RW ? d : 0, s);
        diag = d == dep ? s : diag;
        __asm__ volatile("" ::: "memory");   // one ancestor block in flight at a time
    }
    return diag;
}

// Solve (A + lam diag(max(A_jj, floor))) delta = -g with A given by the
// lanes' partial rows r (consumed), partial diagonals dgu and right-hand
// sides g, and the owners' whole undamped diagonals dfull.  Returns false if
// a pivot is not above thresh_rel * max damped diagonal (thresh_rel > 0) or
// not positive and finite.  sinfo: lane s holds step s's PathC::step_info.
// slots: LDS, one pivot row (SS values of T) per path.
template <int DMAX, typename T, int RW>
PK_DEV bool path_solve(Row<T, RW> &r, T dgu, T dfull, T g, float lam, float dfloor, float thresh_rel,
                       const LaneInfo<DMAX> &I, int lane, int nstep, uint32_t sinfo, int ncopy,
                       uint32_t copy_depths, int max_depth, T *slots, float &delta)
{
    constexpr int SS = DMAX + 4;
    // the lane's depth and ownership and the tree depth as new values:
    // conditions on them are formed here, not shared with (and kept live
    // from) the row forming
    int dep = I.dep, own = I.own;
    __asm__ volatile("" : "+v"(dep), "+v"(own));
    max_depth = fresh_uniform(max_depth);
    const T damp = own ? (T)lam * (dfull > (T)dfloor ? dfull : (T)dfloor) : (T)0;
    T dg = dgu + damp;
    const float dmax = wave_max_nonneg(own ? (float)(dfull + damp) : 0.f);
    T thresh = 0;
    if (thresh_rel > 0.f) thresh = (T)thresh_rel * (T)dmax;
    T b = I.j >= 0 ? -g : (T)0;
    bool bad = false;
    for (int st = 0; st < nstep; ++st) {
        const unsigned si = (unsigned)bcast_i((int)sinfo, st);
        const int mdep = (int)((si >> 8) & 0xffu);
        if (mdep > 0) {
            // Merge phase: the owners of the joints merged at this step add
            // their other copies' rows, diagonals and right-hand sides.
            // Every entry of a copy's row is exchanged, those at and past
            // the owner's depth too (they stay don't-care), so that all of a
            // copy's exchanges are in flight together rather than one per
            // merged depth.
            const bool mg = I.mstep == st;
            for (int c = 0; c < ncopy; ++c) {
                const int cl = copy_lane(I, c);
                const int src = cl == PK_PATH_NONE ? lane : cl;
                const bool use = mg && cl != PK_PATH_NONE;
                Row<T, RW> o;
#pragma unroll
                for (int d = 0; d < RW; ++d) o.set(d, __shfl(r.get(d), src, 64));
                const T od = __shfl(dg, src, 64), ob = __shfl(b, src, 64);
                if (use) {
#pragma unroll
                    for (int i = 0; i < RW / 4; ++i) r.v[i] += o.v[i];
                    dg += od;
                    b += ob;
                }
            }
        }
        wave_sync();   // the previous step's slot reads are done
        if (own && I.step == st) {
            bad = bad || !(dg > thresh) || !(dg < (T)INFINITY);
            if (I.grp >= 0) {
                // Entries at and past the pivot's depth are not part of its
                // row; readers use only those below their own, shallower depth.
                T *sl = slots + I.grp * SS;
#pragma unroll
                for (int i = 0; i < RW / 4; ++i) *(typename Row<T, RW>::V4 *)(sl + 4 * i) = r.v[i];
                sl[DMAX] = dg;
                sl[DMAX + 1] = b;
            }
        }
        wave_sync();   // the step's pivot rows are visible
        if ((I.upd >> st) & 1ull) {
            // The whole slot is read at once (one LDS round trip; loads
            // issued under per-group conditions waited one after another) and
            // applied to the whole row: entries past the lane's own depth take
            // values no reader uses.
            typedef typename Row<T, RW>::V4 V4;
            const T *sk = slots + I.grp * SS;
            V4 sv[RW / 4];
#pragma unroll
            for (int i = 0; i < RW / 4; ++i) sv[i] = *(const V4 *)(sk + 4 * i);
            const T piv = sk[DMAX], bk = sk[DMAX + 1];
            const T sel = sk[dep];
            const T c = sel * recip(piv);
#pragma unroll
            for (int i = 0; i < RW / 4; ++i) r.v[i] -= c * sv[i];
            dg -= c * sel;
            b -= c * bk;
        }
    }
    if (__any(bad)) return false;
    // Back substitution, root first: x_j = (b_j - sum_d r_j[d] x_anc(d)) /
    // pivot_j on the owner.  At depths with shared joints a lane reads its
    // ancestor's x from that joint's owner (whose lane it looks up off the
    // dependent chain); the copies take their owner's x at the end.
    const T ipj = own ? recip(dg) : (T)0;
    T s = 0, x = 0;
#pragma unroll
    for (int D = 0; D < DMAX; ++D) {
        if (D <= max_depth) {
            if (own && dep == D) x = (b - s) * ipj;
            int al = wave::anc_lane<DMAX>(I.ancp, D);
            if ((copy_depths >> D) & 1)   // uniform: some joint at depth D has copies
                al = __shfl(I.owner, al, 64);
            const T xa = __shfl(x, al, 64);
            if (D < RW && dep > D) s += r.get(D < RW ? D : 0) * xa;
        }
    }
    if (copy_depths) x = __shfl(x, I.owner, 64);
    delta = I.j >= 0 ? (float)x : 0.f;
    return true;
}

// One LM problem (active index wi) on this wavefront; resumable (state in
// HBM, at most P.iter_budget iterations per launch when P.st_state is set).
template <int DMAX, int MMAX, int RW = DMAX>
PK_DEV void path_problem(const RobotC *__restrict__ rb, KParams *Pk, float *lds, int64_t wi)
{
    const SolveParams &P = *(const SolveParams *)Pk;
    using L = Lds<DMAX, MMAX>;
    const int lane = threadIdx.x & 63;     // wavefronts of a multi-wave block each run their own problem
    const int64_t p = P.active ? (int64_t)P.active[wi] : wi;
    const int64_t N = P.N, T = P.T, t = p / P.K;
    const PathC &Pc = rb->path;
    const int n = rb->n, m = rb->m, nstep0 = rb->nstep, max_depth0 = rb->max_depth, ncopy0 = Pc.ncopy;
    const uint32_t copy_depths = Pc.copy_depths;
    const bool resumable = P.st_state != nullptr, resume = resumable && P.resume;

    LaneInfo<DMAX> I;
    const bool inl = lane < Pc.lanes;
    const int l = inl ? lane : 0;
    const int jl = inl ? (int)Pc.joint[l] : 0;
    I.j = inl ? jl : -1;
    I.grp = inl ? (int)Pc.group[l] : -1;
    I.dep = inl ? rb->j[jl].depth : -1;
    I.owner = inl ? (int)Pc.owner[l] : lane;
    I.own = inl && I.owner == lane;
    I.ee = inl ? (int)Pc.lane_ee[l] : -1;
    I.step = inl ? (int)rb->step_of[jl] : -1;
    I.mstep = inl ? (int)Pc.merge_step[l] : -1;
    I.gkind = I.grp >= 0 ? rb->e[I.grp].kind : 0;
    I.pris = inl && rb->j[jl].type == PK_JOINT_PRISMATIC;
    I.lo = rb->j[jl].lo;
    I.hi = rb->j[jl].hi;
    I.qr = (P.q_rest && inl) ? P.q_rest[jl] : rb->j[jl].mid;
    {
        const uint32_t *arow = (const uint32_t *)Pc.anc[l];
#pragma unroll
        for (int i = 0; i < DMAX / 4; ++i) I.ancp[i] = inl ? arow[i] : (uint32_t)lane * 0x01010101u;
        const uint32_t *crow = (const uint32_t *)Pc.copies[l];
        I.cp0 = inl ? crow[0] : 0xffffffffu;
        I.cp1 = inl ? crow[1] : 0xffffffffu;
    }
    I.upd = inl ? Pc.upd[l] : 0ull;
    I.jump = inl ? Pc.jump[l] : (uint32_t)lane * 0x01010101u;
    const uint32_t sinfo = lane < nstep0 ? Pc.step_info[lane] : 0u;
    {
        float *cs = lds + L::CS + lane * 12;
#pragma unroll
        for (int u = 0; u < 9; ++u) cs[u] = rb->j[jl].G[u];
#pragma unroll
        for (int u = 0; u < 3; ++u) cs[9 + u] = rb->j[jl].t[u];
    }

    bool fin = true;
    if (lane < m) {
        float *ec = lds + L::EC + lane * 12, *tg = lds + L::TG + lane * 12;
#pragma unroll
        for (int u = 0; u < 9; ++u) ec[u] = rb->e[lane].G[u];
#pragma unroll
        for (int u = 0; u < 3; ++u) ec[9 + u] = rb->e[lane].t[u];
        const int off = rb->e[lane].tgt_off;
        const int W = rb->e[lane].kind == PK_EE_POSE ? 7 : 3;
        float v[7] = {0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int u = 0; u < 7; ++u) {
            if (u < W) {
                v[u] = P.targets[(int64_t)(off + u) * T + t];
                fin = fin && isfinite(v[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < 3; ++u) tg[u] = v[u];
        float Rt[9];
        quat_to_rot(v[3], v[4], v[5], v[6], Rt);
#pragma unroll
        for (int u = 0; u < 9; ++u) tg[3 + u] = Rt[u];
    }
    float q = 0.f;
    if (I.j >= 0) {
        q = (resume ? P.joints : P.seeds)[(int64_t)I.j * N + p];
        fin = fin && isfinite(q);
    }
    const bool finite = __all(fin);
    if (!finite) {
        if (I.own) {
            P.joints[(int64_t)I.j * N + p] = q;
            for (int it = 0; it < P.trace_iters; ++it)
                P.trace_q[((int64_t)it * n + I.j) * N + p] = q;
        }
        if (lane < m) {
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

    // Current point: scalars in registers, Jacobian blocks and EE records in
    // LDS.  Each pass evaluates one point (first the
    // start point, then each trial), so every stage has a single call site.
    PointVal X;
    float cost = INFINITY, pcost = 0.f, perr = 0.f, rerr = 0.f, rl = 0.f, rr = 0.f, dl = 0.f;
    bool meets = false;
    float qt = q;
    bool first = true, evaluate = true;
    for (;;) {
        // The call's parameters are re-read (scalar loads) in each pass
        // rather than held in SGPRs across the loop, which spills them.
        const SolveParams &Q = *(const SolveParams *)fresh_uniform(Pk);
        // likewise the robot's sizes: the per-depth conditions of the unrolled
        // loops are formed at their uses
        const int max_depth = fresh_uniform(max_depth0), nstep = fresh_uniform(nstep0),
                  ncopy = fresh_uniform(ncopy0);
        bool acc = false;
        // The lane tables are taken as new values in each pass, so that what
        // the compiler derives from them (addresses, per-depth lane masks) is
        // formed where it is used instead of held across the whole loop.
#pragma unroll
        for (int i = 0; i < DMAX / 4; ++i) __asm__ volatile("" : "+v"(I.ancp[i]));
        __asm__ volatile("" : "+v"(I.jump), "+v"(I.cp0), "+v"(I.cp1));
        __asm__ volatile("" : "+v"(I.dep), "+v"(I.own), "+v"(I.grp), "+v"(I.ee), "+v"(I.owner));
        __asm__ volatile("" : "+v"(I.j), "+v"(I.step), "+v"(I.mstep));
        if (evaluate) {
            point<DMAX, MMAX>(Q, I, lane, max_depth, qt, lds, X);
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
                    done = Q.early_exit && itt == 0;
                }
            } else {
                lam = fmaxf(lam / Q.nu_down, Q.lambda_min);
                ++accepts;
                if (meets) {
                    if (itt < 0) itt = iters;
                    if (Q.early_exit) done = true;
                }
            }
            if (!done && iters < iter_end) {
                wave_sync();
                jacobian<DMAX, MMAX>(Q, I, lane, lds);
            }
        } else if (!first) {
            if (lam >= Q.lambda_max) {
                stalled = true;
                done = true;
            }
            lam = fminf(lam * Q.nu_up, Q.lambda_max);
        }
        if (!first && iters - 1 < Q.trace_iters) {
            if (I.own) Q.trace_q[((int64_t)(iters - 1) * n + I.j) * N + p] = q;
            if (lane == 0) Q.trace_acc[(int64_t)(iters - 1) * N + p] = acc ? 1 : 0;
        }
        first = false;
        if (done || iters >= iter_end) break;
        // Damped step from the current point: the partial rows of J^T J are
        // formed from the Jacobian blocks in LDS at each solve (a rejected
        // step re-forms the same values) instead of being kept in registers.
        float delta = 0.f;
        bool ok;
        {
            wave_sync();   // the blocks are visible
            Row<float, RW> r;
            float ge;
            const float dgu = jtj_rows<DMAX, MMAX, float, RW>(lds, I, lane, max_depth, r, ge) +
                              (I.own ? dl * dl + Q.w_rest * Q.w_rest : 0.f);
            const float g = ge + (I.own ? dl * rl + Q.w_rest * rr : 0.f);
            const float dfull = add_copies<DMAX, float>(dgu, I, lane, ncopy);
            ok = path_solve<DMAX, float, RW>(r, dgu, dfull, g, lam, Q.damping_floor, Q.pivot_rel, I, lane,
                                         nstep, sinfo, ncopy, copy_depths, max_depth, (float *)(lds + L::PV),
                                         delta);
        }
        if (!ok) {
            // Re-form the damped system and gradient in FP64 from the FP32
            // Jacobian blocks and residuals, and solve again.
            flags |= PK_FLAG_FP64;
            Row<double, RW> r;
            double gd;
            const double dgd = jtj_rows<DMAX, MMAX, double, RW>(lds, I, lane, max_depth, r, gd) +
                               (I.own ? (double)dl * dl + (double)Q.w_rest * Q.w_rest : 0.0);
            if (I.own) gd += (double)dl * rl + (double)Q.w_rest * rr;
            const double dfd = add_copies<DMAX, double>(dgd, I, lane, ncopy);
            ok = path_solve<DMAX, double, RW>(r, dgd, dfd, gd, lam, Q.damping_floor, 0.f, I, lane, nstep,
                                          sinfo, ncopy, copy_depths, max_depth, (double *)(lds + L::PV),
                                          delta);
        }
        qt = q + delta;
        evaluate = ok;   // a failed solve counts as a rejected step
    }
    const bool finished = done || iters >= P.max_iters;
    if (finished)
        for (int it = iters; it < P.trace_iters; ++it) {
            if (I.own) P.trace_q[((int64_t)it * n + I.j) * N + p] = q;
            if (lane == 0) P.trace_acc[(int64_t)it * N + p] = 0;
        }
    if (I.own) P.joints[(int64_t)I.j * N + p] = q;
    if (I.ee >= 0) {
        if (P.pos_err) P.pos_err[(int64_t)I.ee * N + p] = perr;
        if (P.rot_err) P.rot_err[(int64_t)I.ee * N + p] = rerr;
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

struct PathKernelArgs {     // the argument list of lm_path_kernel, for the offset of P
    const RobotC *rb;
    SolveParams P;
};

// Four wavefronts per SIMD where the LDS allows it (<= 4 EEs: 9.4 KiB per
// wavefront), so that a batch of 4 x 256 x 4 problems is resident at once;
// the compiler then keeps the kernel within 128 VGPRs (its spills land in
// the per-problem set-up and in the FP64 re-solve, not in the LM loop).
template <int DMAX, int MMAX, int RW>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MMAX <= 4 ? 4 : 3))) void lm_path_kernel(
    const RobotC *__restrict__ rb, SolveParams P)
{
    KParams *Pk = kernel_params_at(offsetof(PathKernelArgs, P));
    using L = Lds<DMAX, MMAX>;
    __shared__ __attribute__((aligned(16))) float lds[L::FLOATS];
    const int64_t nact = P.n_active ? (int64_t)*P.n_active : P.N;
    int64_t wi = P.queue_head ? wave::pop_item_wave(P.queue_head) : (int64_t)blockIdx.x;
    while (wi < nact) {
        path_problem<DMAX, MMAX, RW>(rb, Pk, lds, wi);
        if (!P.queue_head) break;
        __syncthreads();
        wi = wave::pop_item_wave(P.queue_head);
    }
}

template <int DMAX, int MMAX, int RW>
hipError_t launch_path(const RobotC *rb, const SolveParams &P, int persist_blocks, hipStream_t s)
{
    int64_t grid = P.N;
    if (P.queue_head && persist_blocks > 0 && persist_blocks < grid) grid = persist_blocks;
    hipLaunchKernelGGL((lm_path_kernel<DMAX, MMAX, RW>), dim3((unsigned)grid), dim3(64), 0, s, rb, P);
    return hipGetLastError();
}

}  // namespace path
}  // namespace pk
