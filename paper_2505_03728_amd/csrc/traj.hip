// Trajectory optimisation: LM over a trajectory of T configurations of a
// single-chain robot (Sec. II: a configuration interacts only with its
// temporal neighbours, so the normal equations are banded).  One trajectory
// per workgroup of four wavefronts:
//   * lanes 0 and 1 run FK, the pose log and the pose Jacobian at the first
//     and the last configuration (start and goal pose costs);
//   * every thread takes its share of the T*n variables for the limit,
//     smoothness, velocity-limit and five-point acceleration/jerk terms;
//   * J^T J is banded (half-bandwidth 4n in time-major order): it is formed
//     straight into a band in LDS, damped, factored by a band L D L^T
//     blocked by timestep and solved, all in FP64: the jerk rows outweigh
//     the smoothness rows by ~1e5 in J^T J, and at that conditioning an FP32
//     factorisation steers LM off the FP64 path (FP64 FMAs issue at the
//     unpacked FP32 rate).
#include <string.h>

#include <cmath>

#include "pk_ctx.hpp"
#include "pk_device.hpp"

namespace pk {
namespace {

constexpr int TRAJ_VMAX = 256;   // T * n variables per trajectory
constexpr int TRAJ_THREADS = 256; // four wavefronts per trajectory

struct TrajParams {
    int64_t B;
    int T;
    float dt, w_pos, w_rot, w_limit, w_smooth, w_vel, w_acc, w_jerk;
    const float *vmax;                 // [n] or null (no velocity-limit term)
    const float *start, *goal;         // [7][B]: p, quaternion wxyz
    const float *init;                 // [B][T][n]
    float *out;                        // [B][T][n]
    float *cost, *pos_err, *rot_err;   // [B], [2][B], [2][B]
    int32_t *iters, *accepts, *status;
    float lambda0, nu_up, nu_down, lambda_min, lambda_max, tol_pos, tol_rot, damping_floor,
        pivot_rel;
    int max_iters, early_exit;
};

// Five-point stencils on offsets -2..2: second derivative times dt^2 and
// third derivative times dt^3 (copied to LDS per workgroup).
constexpr float ACC5[5] = {-1.f / 12.f, 16.f / 12.f, -30.f / 12.f, 16.f / 12.f, -1.f / 12.f};
constexpr float JERK5[5] = {-0.5f, 1.f, 0.f, -1.f, 0.5f};

template <int NJ>
struct TrajLds {
    static constexpr int HB = 4 * NJ, W = HB + 1;
    static constexpr int NPAIR = HB * (HB + 1) / 2;
    double band[TRAJ_VMAX * W];
    double b[TRAJ_VMAX];
    double invd[TRAJ_VMAX];                            // 1 / D_j of the L D L^T factorisation
    float Q[TRAJ_VMAX], Qt[TRAJ_VMAX];
    float J0[6 * NJ], J1[6 * NJ], r0[6], r1[6];        // pose rows at the current point
    float Jt0[6 * NJ], Jt1[6 * NJ], rt0[6], rt1[6];    // ... at the trial point
    float err[4], errt[4];                             // pos/rot errors (start, goal)
    // per-joint limits and allowed step, the stencils: read per band entry,
    // so they sit in LDS rather than behind lane-indexed global loads
    float lo[NJ], hi[NJ], vdt[NJ], acc5[5], jerk5[5];
    float red[4];                                      // per-wavefront partials of a reduction
    // the part of the normal matrix that does not depend on the trajectory:
    // smoothness and the two stencils, A(t, t - dtk) per joint at t * 5 + dtk
    double ctab[5 * (TRAJ_VMAX / NJ)];
    float racc[TRAJ_VMAX], rjerk[TRAJ_VMAX];          // stencil rows at the current point
    int fail;                                          // a pivot failed in the factorisation
};

PK_DEV float wsum(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

PK_DEV float wmax(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum and maximum over the workgroup (four wavefronts): butterflies within
// each wavefront, then the four partials through LDS, added in one order so
// that every thread gets the same value.
PK_DEV float block_sum(float v, float *red)
{
    v = wsum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

PK_DEV float block_max(float v, float *red)
{
    v = wmax(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// FK of the chain at q (NJ values), the pose residual rows against target
// tp (p, quaternion) and, with jac, the weighted pose Jacobian [6][NJ].
template <int NJ>
PK_DEV void endpoint(const RobotC *__restrict__ rb, const TrajParams &P, const float *q,
                     const float *tp, float *r6, float *J, float &perr, float &rerr)
{
    float O[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f}, p[3] = {0.f, 0.f, 0.f};
    float om[NJ][3], pj[NJ][3];
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const bool pri = rb->j[i].type == PK_JOINT_PRISMATIC;
        float s = 0.f, c = 1.f, On[9], pn[3];
        if (!pri) joint_sincos(q[i], s, c);
        joint_step(O, p, rb->j[i].G, rb->j[i].t, s, c, On, pn);
        if (pri) joint_slide(On, q[i], pn);
#pragma unroll
        for (int u = 0; u < 9; ++u) O[u] = On[u];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            p[u] = pn[u];
            om[i][u] = O[3 * u + 2];
            pj[i][u] = p[u];
        }
    }
    float Re[9], pe[3], Rt[9], d[3];
    ee_frame(O, p, rb->e[0].G, rb->e[0].t, Re, pe);
#pragma unroll
    for (int u = 0; u < 3; ++u) d[u] = pe[u] - tp[u];
    perr = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    quat_to_rot(tp[3], tp[4], tp[5], tp[6], Rt);
    const PoseLog lg = pose_log(Rt, Re, d);
    rerr = lg.theta;
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        r6[u] = P.w_pos * lg.rho[u];
        r6[3 + u] = P.w_rot * lg.phi[u];
    }
    float M[9], Nb[9];
    jr_inv_blocks(lg, Re, M, Nb);
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        float v[3], w[3];
        joint_twist(rb->j[i].type == PK_JOINT_PRISMATIC, om[i], pj[i], pe, v, w);
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const float mv = M[3 * u] * v[0] + M[3 * u + 1] * v[1] + M[3 * u + 2] * v[2];
            const float nw = Nb[3 * u] * w[0] + Nb[3 * u + 1] * w[1] + Nb[3 * u + 2] * w[2];
            const float mw = M[3 * u] * w[0] + M[3 * u + 1] * w[1] + M[3 * u + 2] * w[2];
            J[u * NJ + i] = P.w_pos * (mv + nw);
            J[(3 + u) * NJ + i] = P.w_rot * mw;
        }
    }
}

// Per-variable pieces at Q: limit residual and derivative, and the
// velocity-limit residual and sign of the step into timestep t.
template <int NJ>
PK_DEV void limit_row(const TrajLds<NJ> &S, const TrajParams &P, float q, int i, float &rl, float &dl)
{
    const float over = q - S.hi[i], under = S.lo[i] - q;
    rl = P.w_limit * (fmaxf(over, 0.f) + fmaxf(under, 0.f));
    dl = over > 0.f ? P.w_limit : (under > 0.f ? -P.w_limit : 0.f);
}

template <int NJ>
PK_DEV void vel_row(const TrajLds<NJ> &S, const TrajParams &P, const float *Q, int v, int i, float &rv,
                    float &sv)
{
    const float d = Q[v] - Q[v - NJ];
    const float ex = fabsf(d) - S.vdt[i];
    rv = ex > 0.f ? P.w_vel * ex : 0.f;
    sv = ex > 0.f ? (d > 0.f ? P.w_vel : -P.w_vel) : 0.f;
}

PK_DEV float acc_row(const TrajParams &P, const float *Q, int v, int n)
{
    float a = 0.f;
#pragma unroll
    for (int k = 0; k < 5; ++k) a += ACC5[k] * Q[v + (k - 2) * n];
    return a * (P.w_acc / (P.dt * P.dt));
}

PK_DEV float jerk_row(const TrajParams &P, const float *Q, int v, int n)
{
    float a = 0.f;
#pragma unroll
    for (int k = 0; k < 5; ++k) a += JERK5[k] * Q[v + (k - 2) * n];
    return a * (P.w_jerk / (P.dt * P.dt * P.dt));
}

// Sum of squares of the non-pose rows at Q (every lane; wave total).
template <int NJ>
PK_DEV float path_cost(TrajLds<NJ> &S, const TrajParams &P, const float *Q, int lane)
{
    const int T = P.T, V = T * NJ;
    float s = 0.f;
    for (int v = lane; v < V; v += TRAJ_THREADS) {
        const int t = v / NJ, i = v - t * NJ;
        float rl, dl;
        limit_row<NJ>(S, P, Q[v], i, rl, dl);
        s += rl * rl;
        if (t >= 1) {
            const float rs = P.w_smooth * (Q[v] - Q[v - NJ]);
            s += rs * rs;
            if (P.vmax) {
                float rv, sv;
                vel_row<NJ>(S, P, Q, v, i, rv, sv);
                s += rv * rv;
            }
        }
        if (t >= 2 && t <= T - 3) {
            const float ra = acc_row(P, Q, v, NJ), rj = jerk_row(P, Q, v, NJ);
            s += ra * ra + rj * rj;
        }
    }
    return block_sum(s, S.red);
}

// Band of A + lambda diag(max(A_vv, floor)) and the right-hand side -J^T r at
// the current point, in precision T: A(v, v - k) at band[v * W + k].
template <int NJ, typename T>
PK_DEV void form_system(const RobotC *__restrict__ rb, const TrajParams &P, TrajLds<NJ> &S,
                        float lam, int lane, T *band, T *rhs)
{
    constexpr int W = TrajLds<NJ>::W;
    const int TT = P.T, V = TT * NJ;
    const T sa = (T)P.w_acc / ((T)P.dt * (T)P.dt), sj = (T)P.w_jerk / ((T)P.dt * (T)P.dt * (T)P.dt);
    for (int v = lane; v < V; v += TRAJ_THREADS) {
        const int t = v / NJ;
        if (t >= 2 && t <= TT - 3) {
            S.racc[v] = acc_row(P, S.Q, v, NJ);
            S.rjerk[v] = jerk_row(P, S.Q, v, NJ);
        }
    }
    // one band row per thread: A(v, v - k) for k = 0 .. W-1.  Nonzero are the
    // same joint's entries (k a multiple of NJ: smoothness, stencils, the
    // velocity rows and, on the diagonal, the limit row) and, at the first
    // and the last timestep, the pose block (k <= i); the rest is zero.
    for (int v = lane; v < V; v += TRAJ_THREADS) {
        const int t = v / NJ, i = v - t * NJ;
        float rl, dl, rv = 0.f, sv = 0.f, rv1 = 0.f, sv1 = 0.f;
        limit_row<NJ>(S, P, S.Q[v], i, rl, dl);
        if (P.vmax) {   // velocity rows tau = t and tau = t + 1, where active
            if (t >= 1) vel_row<NJ>(S, P, S.Q, v, i, rv, sv);
            if (t + 1 <= TT - 1) vel_row<NJ>(S, P, S.Q, v + NJ, i, rv1, sv1);
        }
        const bool endp = t == 0 || t == TT - 1;
        const float *J = t == 0 ? S.J0 : S.J1;
        T *row = band + v * W;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            T a = 0;
            if (v - k >= 0) {
                if (k % NJ == 0) {
                    a = (T)S.ctab[t * 5 + k / NJ];
                    if (k == 0) {
                        a += (T)dl * (T)dl;
                        a += (T)sv * (T)sv + (T)sv1 * (T)sv1;
                    }
                    if (k == NJ) a -= (T)sv * (T)sv;
                }
                if (k < NJ && endp && k <= i) {
#pragma unroll
                    for (int r = 0; r < 6; ++r) a += (T)J[r * NJ + i] * (T)J[r * NJ + i - k];
                }
                if (k == 0) a += (T)lam * (a > (T)P.damping_floor ? a : (T)P.damping_floor);
            }
            row[k] = a;
        }
    }
    __syncthreads();   // stencil rows
    for (int v = lane; v < V; v += TRAJ_THREADS) {
        const int t = v / NJ, i = v - t * NJ;
        T g = 0;
        float rl, dl;
        limit_row<NJ>(S, P, S.Q[v], i, rl, dl);
        g += (T)dl * (T)rl;
        if (t >= 1) g += (T)P.w_smooth * (T)P.w_smooth * ((T)S.Q[v] - (T)S.Q[v - NJ]);
        if (t <= TT - 2) g -= (T)P.w_smooth * (T)P.w_smooth * ((T)S.Q[v + NJ] - (T)S.Q[v]);
        if (P.vmax) {
            float rv, sv;
            if (t >= 1) {
                vel_row<NJ>(S, P, S.Q, v, i, rv, sv);
                g += (T)sv * (T)rv;
            }
            if (t <= TT - 2) {
                vel_row<NJ>(S, P, S.Q, v + NJ, i, rv, sv);
                g -= (T)sv * (T)rv;
            }
        }
        for (int tc = t - 2; tc <= t + 2; ++tc) {
            if (tc < 2 || tc > TT - 3) continue;
            const int o = t - tc + 2, vc = tc * NJ + i;
            g += sa * (T)S.acc5[o] * (T)S.racc[vc] + sj * (T)S.jerk5[o] * (T)S.rjerk[vc];
        }
        if (t == 0 || t == TT - 1) {
            const float *J = t == 0 ? S.J0 : S.J1;
            const float *r = t == 0 ? S.r0 : S.r1;
#pragma unroll
            for (int q = 0; q < 6; ++q) g += (T)J[q * NJ + i] * (T)r[q];
        }
        rhs[v] = -g;
    }
}

// The trailing triangle of a block step at c0: entries (R, R2) =
// (c0 + NJ - 1 + di, c0 + NJ - 1 + dk), 1 <= dk <= di <= HB, in two parts:
// A (dk <= NJ: the next block's columns, which its elimination needs) and B
// (dk > NJ).  A is spread over the workgroup, B over wavefronts 1..3.
template <int NJ>
struct Pairs {
    static constexpr int HB = TrajLds<NJ>::HB;
    static constexpr int NA = NJ * (HB + 1) - NJ * (NJ + 1) / 2;
    static constexpr int NB = (HB - NJ) * (HB - NJ + 1) / 2;
    static constexpr int PA = (NA + TRAJ_THREADS - 1) / TRAJ_THREADS;
    static constexpr int PB = (NB + TRAJ_THREADS - 64 - 1) / (TRAJ_THREADS - 64);
};

// Entries p = t + stride m of the part with dk in [dlo, HB], listed dk-major
// (di = dk .. HB within a dk), packed di | dk << 8; 0 for t < 0 and past total.
template <int NJ, int M>
PK_DEV void part_pairs(int t, int stride, int dlo, int total, int (&mp)[M])
{
    constexpr int HB = TrajLds<NJ>::HB;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int p = t + stride * m;
        int dk = dlo, rem = p;
        while (dk <= HB && rem >= HB - dk + 1) {
            rem -= HB - dk + 1;
            ++dk;
        }
        mp[m] = t >= 0 && p < total ? ((dk + rem) | (dk << 8)) : 0;
    }
}

// Rank-NJ update of the listed entries of the trailing triangle of the block
// step at c0: A(R, R2) -= sum_cc A(R, cc) A(R2, cc) / D_cc over the block's
// columns (unscaled entries).  Addresses are clamped into the band so that
// every load is issued unconditionally; padding entries store nothing.
template <int NJ, typename T, int M>
PK_DEV void trail(T *band, const T *invd, int V, int c0_, const int (&mp)[M])
{
    constexpr int HB = TrajLds<NJ>::HB, W = TrajLds<NJ>::W;
    // the block offset as an opaque uniform value: addresses are recomputed
    // per block step rather than carried as induction variables across the
    // factorisation (which spilled them)
    const int c0 = __builtin_amdgcn_readfirstlane(c0_);
    T dinv[NJ];
#pragma unroll
    for (int cc = 0; cc < NJ; ++cc) dinv[cc] = invd[c0 + cc];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        // likewise for the pair: its offsets are derived here, not hoisted
        int pm = mp[m];
        asm volatile("" : "+v"(pm));
        const int di = pm & 0xff, dk = pm >> 8;
        const int R = c0 + NJ - 1 + di, R2 = c0 + NJ - 1 + dk;
        const bool ok = di && R < V;
        const int Rc = min(R, V - 1), R2c = min(R2, V - 1);
        // every load first (the target included), so that they are in flight
        // together; the band-edge selects come after
        T a1[NJ], a2[NJ];
#pragma unroll
        for (int cc = 0; cc < NJ; ++cc) {
            a1[cc] = band[Rc * W + min(NJ - 1 + di - cc, HB)];
            a2[cc] = band[R2c * W + min(NJ - 1 + dk - cc, HB)];
        }
        const T tv = band[Rc * W + (di - dk)];
        T term[NJ];
#pragma unroll
        for (int cc = 0; cc < NJ; ++cc) {
            const int k1 = NJ - 1 + di - cc, k2 = NJ - 1 + dk - cc;
            term[cc] = (k1 <= HB ? a1[cc] : (T)0) * dinv[cc] * (k2 <= HB ? a2[cc] : (T)0);
        }
        // pairwise sum: a short dependent chain
#pragma unroll
        for (int w = 1; w < NJ; w *= 2)
#pragma unroll
            for (int cc = 0; cc + w < NJ; cc += 2 * w) term[cc] += term[cc + w];
        if (ok) band[R * W + (di - dk)] = tv - term[0];
    }
}

// Value of v in lane l (l uniform) broadcast to the wavefront.
PK_DEV double readlane_d(double v, int l)
{
    const long long u = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// 1 / d for a positive normal d: the hardware reciprocal estimate refined by
// one Newton-Raphson step r <- r + r (1 - d r), which squares its relative
// error (measured on gfx950 over 2^20 values across 60 binades: below
// 2^-24.4 for the estimate, below 2^-48.7 after the step).  It sits on the
// factorisation's dependent chain; the solution is rounded to FP32 anyway.
PK_DEV double recip(double d)
{
    const double r = __builtin_amdgcn_rcp(d);
    return fma(r, fma(-d, r, 1.0), r);
}

// In-place band L D L^T factorisation of band (half-bandwidth HB, unit L)
// and the solve of L D L^T x = rhs (x over rhs).  A pivot D_j not above
// thresh_rel times the largest damped diagonal fails the factorisation
// (returns false).
//
// No square roots; blocked by timestep: after the factorisation band[j * W]
// holds D_j and band[i * W + (i - j)] the unscaled entry D_j L_ij, with
// invd[j] = 1 / D_j.  Each block step of NJ columns eliminates its window
// (the block's rows and the HB rows below it, at most 64) on the first
// wavefront in registers, carrying the right-hand side along as one more
// column (the forward substitution L y = rhs); then all threads apply the
// part of the block's rank-NJ trailing update that falls in the next block's
// columns, and the rest of it runs on wavefronts 1..3 while wavefront 0
// eliminates the next block (look-ahead: the two touch disjoint entries).
// Two workgroup barriers per NJ columns.  The backward solve L^T x = D^-1 y
// runs on the first wavefront with the vector in registers (lane l holds
// entries l, l + 64, ...): per chunk of CH steps the lanes read their
// coefficients at once, then each step broadcasts the finished entry with
// readlane and the lanes holding the previous HB entries take their update,
// with no memory access or branch on that dependent chain.
template <int NJ, typename T>
PK_DEV bool band_solve(T *band, T *rhs, T *invd, int V, float thresh_rel,
                       const int (&mpa)[Pairs<NJ>::PA], const int (&mpb)[Pairs<NJ>::PB], int lane,
                       float *red, int *fail)
{
    constexpr int HB = TrajLds<NJ>::HB, W = TrajLds<NJ>::W;
    constexpr int NS = TRAJ_VMAX / 64, CH = 8, NR = NJ + HB;
    static_assert(NR <= 64, "a block step's window fits one wavefront");
    float mx = 0.f;
    for (int v = lane; v < V; v += TRAJ_THREADS) mx = fmaxf(mx, (float)band[v * W]);
    const T thresh = (T)thresh_rel * (T)block_max(mx, red);
    if (lane == 0) *fail = 0;
    for (int c0 = 0; c0 < V; c0 += NJ) {
        // Block step over columns c0 .. c0 + NJ - 1.  Lane r of the first
        // wavefront holds row R = c0 + r of the window (the block's rows
        // and the HB rows below) restricted to the block's columns, x[cc]
        // = A(R, c0 + cc), 0 outside the band; the NJ elimination steps run
        // in registers, each broadcasting its pivot row's column with
        // readlane.
        if (lane >= 64) {
            // meanwhile: part B of the previous block (entries beyond this
            // block's columns, which the elimination does not touch)
            if (c0 > 0) trail<NJ, T>(band, invd, V, c0 - NJ, mpb);
        } else {
            const int R = c0 + lane;
            const bool live = lane < NR && R < V;
            T x[NJ];
#pragma unroll
            for (int cc = 0; cc < NJ; ++cc) {
                const int k = R - (c0 + cc);
                x[cc] = live && k >= 0 && k <= HB ? band[R * W + k] : (T)0;
            }
            T bv = live ? rhs[R] : (T)0;   // right-hand side as one more column
            bool bad = false;
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
                // a failed pivot discards the whole factorisation, so the
                // test stays off the dependent chain
                const T d = readlane_d(x[jj], jj);
                bad |= !(d > thresh) || !(d < (T)INFINITY);
                const T inv = recip(d);
                if (lane == 0) invd[c0 + jj] = inv;
                const T ell = lane > jj ? x[jj] : (T)0;   // unscaled D_jj L_(R, jj)
#pragma unroll
                for (int cc = jj + 1; cc < NJ; ++cc) x[cc] -= ell * (readlane_d(x[jj], cc) * inv);
                bv -= ell * (readlane_d(bv, jj) * inv);
            }
#pragma unroll
            for (int cc = 0; cc < NJ; ++cc) {
                const int k = R - (c0 + cc);
                if (live && k >= 0 && k <= HB) band[R * W + k] = x[cc];
            }
            if (live) rhs[R] = bv;
            if (bad && lane == 0) *fail = 1;
        }
        __syncthreads();
        trail<NJ, T>(band, invd, V, c0, mpa);   // part A of this block
        __syncthreads();
    }
    if (*fail) return false;
    // rhs now holds y of L y = rhs (forward substitution rode along with the
    // elimination)
    if (lane < 64) {
        T x[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int i = 64 * s + lane;
            x[s] = i < V ? rhs[i] : (T)0;
        }
        // D z = y
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int i = 64 * s + lane;
            if (i < V) x[s] *= invd[i];
        }
        // L^T x = z: the entry finished at step j updates i in [j - HB, j)
        // by -L_ji x_j; the candidate i sits in slot s when lane < j % 64
        // (cs), else in slot s - 1 (cp).
#pragma unroll
        for (int s = NS - 1; s >= 0; --s) {
#pragma unroll 1
            for (int l0 = 64 - CH; l0 >= 0; l0 -= CH) {
                const int jt = 64 * s + l0;
                if (jt >= V) continue;
                T cs[CH], cp[CH];
#pragma unroll
                for (int u = 0; u < CH; ++u) {   // loads first, all in flight together
                    const int l = l0 + CH - 1 - u, j = 64 * s + l;
                    const int i = 64 * s + lane - (lane < l ? 0 : 64);
                    const bool ok = j < V && i >= 0 && j - i <= HB;
                    cs[u] = band[ok ? j * W + (j - i) : 0];
                    cp[u] = invd[ok ? i : 0];
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const int l = l0 + CH - 1 - u, j = 64 * s + l;
                    const bool dn = lane < l;
                    const int i = 64 * s + lane - (dn ? 0 : 64);
                    const bool ok = j < V && i >= 0 && j - i <= HB;
                    const T c = cs[u] * cp[u];
                    cs[u] = ok && dn ? c : (T)0;
                    cp[u] = ok && !dn ? c : (T)0;
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const T y = readlane_d(x[s], l0 + CH - 1 - u);
                    x[s] -= cs[u] * y;
                    if (s > 0) x[s - 1] -= cp[u] * y;
                }
            }
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int i = 64 * s + lane;
            if (i < V) rhs[i] = x[s];
        }
    }
    __syncthreads();
    return true;
}

// Two workgroups per CU where their LDS fits (up to 7 joints), which also
// holds the register budget to 256 per lane.
template <int NJ>
__global__ __launch_bounds__(TRAJ_THREADS, NJ <= 7 ? 2 : 1) void traj_kernel(const RobotC *__restrict__ rb,
                                                                             TrajParams P)
{
    using L = TrajLds<NJ>;
    __shared__ L S;
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    if (b >= P.B) return;   // uniform per workgroup
    const int TT = P.T, V = TT * NJ;
    int mpa[Pairs<NJ>::PA], mpb[Pairs<NJ>::PB];
    part_pairs<NJ>(lane, TRAJ_THREADS, 1, Pairs<NJ>::NA, mpa);
    part_pairs<NJ>(lane - 64, TRAJ_THREADS - 64, NJ + 1, Pairs<NJ>::NB, mpb);
    const float *src = P.init + b * (int64_t)V;
    for (int v = lane; v < V; v += TRAJ_THREADS) S.Q[v] = src[v];
    if (lane < NJ) {
        S.lo[lane] = rb->j[lane].lo;
        S.hi[lane] = rb->j[lane].hi;
        S.vdt[lane] = P.vmax ? P.vmax[lane] * P.dt : 0.f;
    }
    if (lane < 5) {
        S.acc5[lane] = ACC5[lane];
        S.jerk5[lane] = JERK5[lane];
    }
    {
        // smoothness rows q_tau - q_{tau-1} (tau = 1..T-1), then the
        // acceleration and jerk rows centred at tc = 2..T-3
        const double ws2 = (double)P.w_smooth * (double)P.w_smooth;
        const double sa = (double)P.w_acc / ((double)P.dt * (double)P.dt);
        const double sj = (double)P.w_jerk / ((double)P.dt * (double)P.dt * (double)P.dt);
        for (int x = lane; x < 5 * P.T; x += TRAJ_THREADS) {
            const int t = x / 5, dtk = x - 5 * t, t2 = t - dtk;
            double a = 0;
            if (dtk == 0) a += (t >= 1 ? ws2 : 0.0) + (t <= P.T - 2 ? ws2 : 0.0);
            if (dtk == 1) a -= ws2;
            for (int tc = t - 2; tc <= t2 + 2; ++tc) {
                if (tc < 2 || tc > P.T - 3) continue;
                const int o1 = t - tc + 2, o2 = t2 - tc + 2;
                a += sa * sa * (double)ACC5[o1] * (double)ACC5[o2] +
                     sj * sj * (double)JERK5[o1] * (double)JERK5[o2];
            }
            S.ctab[x] = a;
        }
    }
    __syncthreads();

    float tgt[7];
    const float *tplane = lane == 0 ? P.start : P.goal;
#pragma unroll
    for (int u = 0; u < 7; ++u) tgt[u] = tplane[(int64_t)u * P.B + b];

    int iters = 0, accepts = 0;
    bool stalled = false, done = false, first = true, evaluate = true;
    float lam = P.lambda0, cost = 0.f;
    // Each pass evaluates one point (first the initial trajectory, then each
    // trial), takes or rejects it, then forms and solves the next step; a
    // failed solve is a rejected trial.  All decisions are workgroup-uniform.
    for (;;) {
        bool acc = false;
        if (evaluate) {
            const float *Qe = first ? S.Q : S.Qt;
            if (lane < 2) {
                float q[NJ], perr, rerr;
                const int t = lane == 0 ? 0 : TT - 1;
#pragma unroll
                for (int i = 0; i < NJ; ++i) q[i] = Qe[t * NJ + i];
                endpoint<NJ>(rb, P, q, tgt, lane == 0 ? S.rt0 : S.rt1, lane == 0 ? S.Jt0 : S.Jt1,
                             perr, rerr);
                S.errt[lane] = perr;
                S.errt[2 + lane] = rerr;
            }
            const float pc = path_cost<NJ>(S, P, Qe, lane);
            __syncthreads();
            float pose = 0.f;
#pragma unroll
            for (int u = 0; u < 6; ++u) pose += S.rt0[u] * S.rt0[u] + S.rt1[u] * S.rt1[u];
            const float ct = pc + pose;
            acc = first || ct < cost;
            if (acc) {
                if (!first)
                    for (int v = lane; v < V; v += TRAJ_THREADS) S.Q[v] = S.Qt[v];
                for (int e = lane; e < 6 * NJ; e += TRAJ_THREADS) {
                    S.J0[e] = S.Jt0[e];
                    S.J1[e] = S.Jt1[e];
                }
                if (lane < 6) {
                    S.r0[lane] = S.rt0[lane];
                    S.r1[lane] = S.rt1[lane];
                }
                if (lane < 4) S.err[lane] = S.errt[lane];
                cost = ct;
            }
        }
        if (!first) {
            ++iters;
            if (acc) {
                lam = fmaxf(lam / P.nu_down, P.lambda_min);
                ++accepts;
            } else {
                if (lam >= P.lambda_max) {
                    stalled = true;
                    done = true;
                }
                lam = fminf(lam * P.nu_up, P.lambda_max);
            }
        }
        if (acc && P.early_exit && S.errt[0] <= P.tol_pos && S.errt[1] <= P.tol_pos &&
            S.errt[2] <= P.tol_rot && S.errt[3] <= P.tol_rot)
            done = true;
        first = false;
        __syncthreads();
        if (done || iters >= P.max_iters) break;
        // damped step from the current point (a pivot test failure is a
        // rejected trial, as when the IK re-solve fails)
        form_system<NJ, double>(rb, P, S, lam, lane, S.band, S.b);
        __syncthreads();
        const bool ok =
            band_solve<NJ, double>(S.band, S.b, S.invd, V, P.pivot_rel, mpa, mpb, lane, S.red, &S.fail);
        for (int v = lane; v < V; v += TRAJ_THREADS) S.Qt[v] = S.Q[v] + (ok ? (float)S.b[v] : 0.f);
        evaluate = ok;
        __syncthreads();
    }
    float *dst = P.out + b * (int64_t)V;
    for (int v = lane; v < V; v += TRAJ_THREADS) dst[v] = S.Q[v];
    if (lane == 0) {
        const bool meets = S.err[0] <= P.tol_pos && S.err[1] <= P.tol_pos && S.err[2] <= P.tol_rot &&
                           S.err[3] <= P.tol_rot;
        if (P.cost) P.cost[b] = cost;
        if (P.iters) P.iters[b] = iters;
        if (P.accepts) P.accepts[b] = accepts;
        if (P.status) P.status[b] = meets ? PK_CONVERGED : (stalled ? PK_STALLED : PK_MAX_ITERS);
        if (P.pos_err) {
            P.pos_err[b] = S.err[0];
            P.pos_err[P.B + b] = S.err[1];
        }
        if (P.rot_err) {
            P.rot_err[b] = S.err[2];
            P.rot_err[P.B + b] = S.err[3];
        }
    }
}

inline bool traj_variant(int n) { return n == 4 || n == 6 || n == 7 || n == 10; }

hipError_t launch_traj(const RobotC *rb, int n, const TrajParams &P, hipStream_t s)
{
    const dim3 grid((unsigned)P.B), block(TRAJ_THREADS);
    switch (n) {
    case 4: hipLaunchKernelGGL(traj_kernel<4>, grid, block, 0, s, rb, P); break;
    case 6: hipLaunchKernelGGL(traj_kernel<6>, grid, block, 0, s, rb, P); break;
    case 7: hipLaunchKernelGGL(traj_kernel<7>, grid, block, 0, s, rb, P); break;
    case 10: hipLaunchKernelGGL(traj_kernel<10>, grid, block, 0, s, rb, P); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace
}  // namespace pk

using namespace pk;

extern "C" int pk_traj_solve(pk_ctx *ctx, int32_t robot_id, const pk_traj_problem *pr,
                             const pk_traj_costs *c, const pk_lm_options *o,
                             const pk_traj_outputs *out, void *stream)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_traj_solve: ctx is NULL");
    RobotEntry *rb = robot_of(ctx, robot_id);
    if (!rb) return fail(ctx, PK_ENOTFOUND, "pk_traj_solve: unknown robot %d", robot_id);
    if (!pr || !c || !o || !out) return fail(ctx, PK_EINVAL, "pk_traj_solve: NULL argument");
    const RobotC &H = rb->host;
    const int n = H.n;
    if (H.chains != 1 || H.m != 1 || H.e[0].kind != PK_EE_POSE || H.n_mimic != 0 || !traj_variant(n))
        return fail(ctx, PK_EUNSUPPORTED, "pk_traj_solve: needs a single chain of 4, 6, 7 or 10 "
                    "non-mimic joints with one pose EE");
    if (pr->B < 0 || pr->T < 5 || (int64_t)pr->T * n > TRAJ_VMAX)
        return fail(ctx, PK_EINVAL, "pk_traj_solve: B=%lld T=%d (need T >= 5, T * n <= %d)",
                    (long long)pr->B, pr->T, TRAJ_VMAX);
    if (pr->B == 0) return PK_OK;
    if (pr->B >= (int64_t)1 << 31) return fail(ctx, PK_EUNSUPPORTED, "pk_traj_solve: B too large");
    if (!pr->start || !pr->goal || !pr->init || !out->traj)
        return fail(ctx, PK_EINVAL, "pk_traj_solve: NULL start/goal/init/traj");
    if (!(c->dt > 0) || !std::isfinite(c->w_pos) || !std::isfinite(c->w_rot) ||
        !std::isfinite(c->w_limit) || !std::isfinite(c->w_smooth) || !std::isfinite(c->w_vel) ||
        !std::isfinite(c->w_acc) || !std::isfinite(c->w_jerk))
        return fail(ctx, PK_EINVAL, "pk_traj_solve: bad costs");
    if (c->w_vel != 0.f && !c->vmax)
        return fail(ctx, PK_EINVAL, "pk_traj_solve: w_vel != 0 needs vmax (velocity limits)");
    if (o->max_iters < 0 || !(o->lambda0 > 0) || !(o->nu_up > 1) || !(o->nu_down > 1) ||
        !(o->lambda_min > 0) || !(o->lambda_max >= o->lambda_min) || !(o->damping_floor > 0) ||
        !(o->pivot_rel >= 0))
        return fail(ctx, PK_EINVAL, "pk_traj_solve: invalid LM options");
    PK_HIP(ctx, hipSetDevice(ctx->device));
    TrajParams P;
    memset(&P, 0, sizeof P);
    P.B = pr->B;
    P.T = pr->T;
    P.dt = c->dt;
    P.w_pos = c->w_pos; P.w_rot = c->w_rot; P.w_limit = c->w_limit; P.w_smooth = c->w_smooth;
    P.w_vel = c->w_vel; P.w_acc = c->w_acc; P.w_jerk = c->w_jerk; P.vmax = c->vmax;
    P.start = pr->start; P.goal = pr->goal; P.init = pr->init;
    P.out = out->traj; P.cost = out->cost; P.pos_err = out->pos_err; P.rot_err = out->rot_err;
    P.iters = out->iters; P.accepts = out->accepts; P.status = out->status;
    P.lambda0 = o->lambda0; P.nu_up = o->nu_up; P.nu_down = o->nu_down;
    P.lambda_min = o->lambda_min; P.lambda_max = o->lambda_max;
    P.tol_pos = o->tol_pos; P.tol_rot = o->tol_rot;
    P.damping_floor = o->damping_floor; P.pivot_rel = o->pivot_rel;
    P.max_iters = o->max_iters; P.early_exit = o->early_exit ? 1 : 0;
    PK_HIP(ctx, launch_traj(rb->dev, n, P, (hipStream_t)stream));
    return PK_OK;
}
