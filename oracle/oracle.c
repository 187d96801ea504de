/*
 * oracle.c -- plain, slow, FP64 CPU reference for batched Levenberg-Marquardt
 * inverse kinematics (PyRoki, arXiv 2505.03728).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * What it follows:
 *   - Sec. III-A (Solver Backbone): Levenberg-Marquardt on a sum of squared
 *     residuals; joint limits are penalties, not hard constraints.
 *   - Sec. III-B (Variable Abstractions): T_base<-i = FK(q)_i over revolute
 *     joints.
 *   - Sec. III-C (Cost Functions): residuals are weighted, the optimizer
 *     minimises their sum of squares; joint pose cost log(T_target^-1 T_i),
 *     joint limit cost max(0,q-q_upper)+max(0,q_lower-q), joint
 *     regularisation cost q - q_reg.
 *   - Lie-group formulas: SO(3)/SE(3) exp, log, left/right Jacobians and
 *     the SE(3) Q-matrix as given by Barfoot, "State Estimation for
 *     Robotics" (2017), Sec. 7.1, and Sola et al., "A micro Lie theory for
 *     state estimation in robotics" (2018).
 *   - Marquardt (1963) damping lambda*diag(J^T J) with factor-10 updates.
 *
 * Readings where the paper is silent (damping floor, lambda bounds, strict
 * accept test, log near pi, series thresholds, success test, best-of-K rule)
 * are listed in the design notes and restated next to the code below.
 *
 * Everything is double precision; loops are written out plainly, one
 * problem at a time.  Threads only split the batch into contiguous chunks.
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_MAX_N 64
#define ORA_MAX_M 8
#define ORA_MAX_ROWS (6 * ORA_MAX_M + 2 * ORA_MAX_N)

enum { ORA_CONVERGED = 0, ORA_MAX_ITERS = 1, ORA_STALLED = 2, ORA_NONFINITE = 3 };
#define ORA_FLAG_FP64 0x100   /* a pivot fell below pivot_rel * max diagonal */

typedef struct {
    int n;
    const int *parent;          /* [n], -1 = base, parent[j] < j            */
    const double *mount_quat;   /* [n][4] wxyz                               */
    const double *offset;       /* [n][3] in the parent frame                */
    const double *axis;         /* [n][3] unit, after the mount rotation     */
    const double *lower;        /* [n]                                       */
    const double *upper;        /* [n]                                       */
    int m;
    const int *ee_joint;        /* [m]                                       */
    const double *ee_offset;    /* [m][3]                                    */
    const double *ee_quat;      /* [m][4]                                    */
    const int *ee_kind;         /* [m] 0 = full pose, 1 = position only      */
    const int *joint_type;      /* [n] ORA_REVOLUTE / ORA_PRISMATIC / ORA_FIXED,
                                   NULL = all revolute                        */
    const int *mimic_joint;     /* [n] driver of a mimic joint or -1; NULL = none */
    const double *mimic_mult;   /* [n] q_j = mult * q_driver + offset           */
    const double *mimic_offset; /* [n]                                         */
} ora_tree;

/* Joint kinds (Sec. III-B lists fixed, revolute, prismatic and mimic
 * joints): a revolute joint rotates by its value about its axis, a prismatic
 * one translates by it along the axis, a fixed one has no value.  A mimic
 * joint (revolute or prismatic) takes mult * (its driver's value) + offset.
 * The variables are the joints that are neither fixed nor mimic, in index
 * order. */
enum { ORA_REVOLUTE = 0, ORA_PRISMATIC = 1, ORA_FIXED = 2 };

static int jtype(const ora_tree *tr, int j)
{
    return tr->joint_type ? tr->joint_type[j] : ORA_REVOLUTE;
}

static int mimic_of(const ora_tree *tr, int j)
{
    return tr->mimic_joint ? tr->mimic_joint[j] : -1;
}

/* Number of variables. */
int ora_nvar(const ora_tree *tr)
{
    int v = 0;
    for (int j = 0; j < tr->n; ++j) v += jtype(tr, j) != ORA_FIXED && mimic_of(tr, j) < 0;
    return v;
}

/* var_of[j]: variable of joint j (-1 if fixed or mimic); joint_of[v]: joint
 * of variable v. */
static void var_maps(const ora_tree *tr, int *var_of, int *joint_of)
{
    int v = 0;
    for (int j = 0; j < tr->n; ++j) {
        if (jtype(tr, j) == ORA_FIXED || mimic_of(tr, j) >= 0) {
            var_of[j] = -1;
        } else {
            var_of[j] = v;
            if (joint_of) joint_of[v] = j;
            ++v;
        }
    }
}

typedef struct {
    double w_pos, w_rot, w_limit, w_rest;
    const double *q_rest;       /* [n] or NULL = (lower+upper)/2             */
} ora_weights;

typedef struct {
    int max_iters;
    double lambda0, nu_up, nu_down, lambda_min, lambda_max;
    int early_exit;
    double tol_pos, tol_rot;
    double damping_floor;       /* D_jj = max(A_jj, damping_floor)           */
    double pivot_rel;           /* fallback-flag threshold on pivots         */
} ora_options;

/* ---------------------------------------------------------------- 3-vectors */

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static double norm3(const double *a) { return sqrt(dot3(a, a)); }

/* 3x3 matrices are row-major double[9]. */
static void matmul3(const double *A, const double *B, double *C)
{
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            T[3 * i + j] = s;
        }
    memcpy(C, T, sizeof T);
}

static void transpose3(const double *A, double *B)
{
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) T[3 * i + j] = A[3 * j + i];
    memcpy(B, T, sizeof T);
}

static void matvec3(const double *A, const double *x, double *y)
{
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
    memcpy(y, t, sizeof t);
}

static void hat3(const double *w, double *W)
{
    W[0] = 0.0;   W[1] = -w[2]; W[2] = w[1];
    W[3] = w[2];  W[4] = 0.0;   W[5] = -w[0];
    W[6] = -w[1]; W[7] = w[0];  W[8] = 0.0;
}

static void eye3(double *I)
{
    memset(I, 0, 9 * sizeof(double));
    I[0] = I[4] = I[8] = 1.0;
}

/* Unit quaternion (w,x,y,z) -> rotation matrix; the quaternion is
 * normalised first (inputs are FP32-rounded and so not exactly unit). */
void ora_quat_to_R(const double *q_in, double *R)
{
    double n = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
    double w = q_in[0] / n, x = q_in[1] / n, y = q_in[2] / n, z = q_in[3] / n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* ------------------------------------------------------------------ SO(3) */

/* exp: R = I + (sin t / t) W + ((1 - cos t) / t^2) W^2,  W = hat(phi). */
void ora_so3_exp(const double *phi, double *R)
{
    double t = norm3(phi), a, b, W[9], W2[9], I[9];
    if (t < 1e-4) {
        double t2 = t * t;
        a = 1.0 - t2 / 6.0 + t2 * t2 / 120.0;
        b = 0.5 - t2 / 24.0 + t2 * t2 / 720.0;
    } else {
        double sh = sin(0.5 * t);          /* 1 - cos t = 2 sin^2(t/2) */
        a = sin(t) / t;
        b = 2.0 * sh * sh / (t * t);
    }
    hat3(phi, W);
    matmul3(W, W, W2);
    eye3(I);
    for (int i = 0; i < 9; ++i) R[i] = I[i] + a * W[i] + b * W2[i];
}

/* log: theta = atan2(|w|, (tr R - 1)/2) with w = vee(R - R^T)/2 = sin(theta) * axis.
 * Near theta = pi the axis is read from the symmetric part
 * (R + R^T)/2 = cos(theta) I + (1 - cos(theta)) a a^T, column of the largest
 * diagonal, sign taken from w (if w vanishes, the largest-magnitude component
 * is made positive). */
void ora_so3_log(const double *R, double *phi)
{
    double w[3] = {0.5 * (R[7] - R[5]), 0.5 * (R[2] - R[6]), 0.5 * (R[3] - R[1])};
    double s = norm3(w);
    double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    double t = atan2(s, c);
    if (t > M_PI - 1e-3) {
        double B[9];
        double omc = 1.0 - c;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                B[3 * i + j] = (0.5 * (R[3 * i + j] + R[3 * j + i]) - (i == j ? c : 0.0)) / omc;
        int k = 0;
        if (B[4] > B[3 * k + k]) k = 1;
        if (B[8] > B[3 * k + k]) k = 2;
        double a[3] = {B[0 * 3 + k], B[1 * 3 + k], B[2 * 3 + k]};
        double an = norm3(a);
        for (int i = 0; i < 3; ++i) a[i] /= an;
        double sgn = dot3(a, w);
        if (sgn < 0.0) {
            for (int i = 0; i < 3; ++i) a[i] = -a[i];
        } else if (sgn == 0.0) {
            int big = 0;
            for (int i = 1; i < 3; ++i) if (fabs(a[i]) > fabs(a[big])) big = i;
            if (a[big] < 0.0) for (int i = 0; i < 3; ++i) a[i] = -a[i];
        }
        for (int i = 0; i < 3; ++i) phi[i] = t * a[i];
        return;
    }
    double f;
    if (t < 1e-3) {
        double t2 = t * t;                 /* theta / sin(theta) */
        f = 1.0 + t2 / 6.0 + 7.0 * t2 * t2 / 360.0;
    } else {
        f = t / s;
    }
    for (int i = 0; i < 3; ++i) phi[i] = f * w[i];
}

/* Left Jacobian J_l(phi) = I + ((1-cos t)/t^2) W + ((t - sin t)/t^3) W^2. */
void ora_so3_jl(const double *phi, double *J)
{
    double t = norm3(phi), a, b, W[9], W2[9], I[9];
    if (t < 1e-3) {
        double t2 = t * t;
        a = 0.5 - t2 / 24.0 + t2 * t2 / 720.0;
        b = 1.0 / 6.0 - t2 / 120.0 + t2 * t2 / 5040.0;
    } else {
        double sh = sin(0.5 * t);
        a = 2.0 * sh * sh / (t * t);
        b = (t - sin(t)) / (t * t * t);
    }
    hat3(phi, W);
    matmul3(W, W, W2);
    eye3(I);
    for (int i = 0; i < 9; ++i) J[i] = I[i] + a * W[i] + b * W2[i];
}

/* Inverse left Jacobian J_l^-1(phi) = I - W/2 + k W^2,
 * k = 1/t^2 - (1 + cos t)/(2 t sin t), written as 1/t^2 - cot(t/2)/(2t) (the same
 * quantity, well defined up to t = pi, no 1 - cos t cancellation); series
 * below 1e-3. */
void ora_so3_jl_inv(const double *phi, double *J)
{
    double t = norm3(phi), k, W[9], W2[9], I[9];
    if (t < 1e-3) {
        double t2 = t * t;
        k = 1.0 / 12.0 + t2 / 720.0 + t2 * t2 / 30240.0;
    } else {
        k = 1.0 / (t * t) - cos(0.5 * t) / (2.0 * t * sin(0.5 * t));
    }
    hat3(phi, W);
    matmul3(W, W, W2);
    eye3(I);
    for (int i = 0; i < 9; ++i) J[i] = I[i] - 0.5 * W[i] + k * W2[i];
}

/* ------------------------------------------------------------------ SE(3) */
/* Tangent vectors are xi = [rho; phi] (translation first). */

/* Q(rho, phi): upper-right block of the SE(3) left Jacobian (Barfoot 2017). */
void ora_se3_Q(const double *rho, const double *phi, double *Q)
{
    double t = norm3(phi), a1, a2, a3;
    if (t < 1e-2) {
        double t2 = t * t;
        a1 = 1.0 / 6.0 - t2 / 120.0 + t2 * t2 / 5040.0;
        a2 = 1.0 / 24.0 - t2 / 720.0 + t2 * t2 / 40320.0;
        a3 = 1.0 / 120.0 - t2 / 2520.0 + t2 * t2 / 120960.0;
    } else {
        double s = sin(t), c = cos(t), t2 = t * t, sh = sin(0.5 * t);
        a1 = (t - s) / (t2 * t);
        a2 = (t2 - 4.0 * sh * sh) / (2.0 * t2 * t2);   /* 2 cos t - 2 = -4 sin^2(t/2) */
        a3 = (2.0 * t - 3.0 * s + t * c) / (2.0 * t2 * t2 * t);
    }
    double P[9], Rh[9], PR[9], RP[9], PRP[9], PP[9], PPR[9], RPP[9], PRPP[9], PPRP[9];
    hat3(phi, P);
    hat3(rho, Rh);
    matmul3(P, Rh, PR);
    matmul3(Rh, P, RP);
    matmul3(PR, P, PRP);
    matmul3(P, P, PP);
    matmul3(PP, Rh, PPR);
    matmul3(RP, P, RPP);
    matmul3(PRP, P, PRPP);
    matmul3(PP, RP, PPRP);
    for (int i = 0; i < 9; ++i)
        Q[i] = 0.5 * Rh[i]
             + a1 * (PR[i] + RP[i] + PRP[i])
             + a2 * (PPR[i] + RPP[i] - 3.0 * PRP[i])
             + a3 * (PRPP[i] + PPRP[i]);
}

/* exp: R = exp(phi), t = J_l(phi) rho. */
void ora_se3_exp(const double *xi, double *R, double *t)
{
    double J[9];
    ora_so3_exp(xi + 3, R);
    ora_so3_jl(xi + 3, J);
    matvec3(J, xi, t);
}

/* log: phi = log(R), rho = J_l^-1(phi) t. */
void ora_se3_log(const double *R, const double *t, double *xi)
{
    double Ji[9];
    ora_so3_log(R, xi + 3);
    ora_so3_jl_inv(xi + 3, Ji);
    matvec3(Ji, t, xi);
}

/* Inverse of the SE(3) left Jacobian, 6x6 row-major:
 * [[Ji, -Ji Q Ji], [0, Ji]],  Ji = J_l^-1(phi), Q = Q(rho, phi). */
void ora_se3_jl_inv(const double *xi, double *M)
{
    double Ji[9], Q[9], T[9], B[9];
    ora_so3_jl_inv(xi + 3, Ji);
    ora_se3_Q(xi, xi + 3, Q);
    matmul3(Ji, Q, T);
    matmul3(T, Ji, B);
    memset(M, 0, 36 * sizeof(double));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            M[6 * i + j] = Ji[3 * i + j];
            M[6 * i + 3 + j] = -B[3 * i + j];
            M[6 * (i + 3) + 3 + j] = Ji[3 * i + j];
        }
}

/* Right Jacobian inverse: J_r^-1(xi) = J_l^-1(-xi). */
void ora_se3_jr_inv(const double *xi, double *M)
{
    double m[6];
    for (int i = 0; i < 6; ++i) m[i] = -xi[i];
    ora_se3_jl_inv(m, M);
}

/* ------------------------------------------------------ forward kinematics */

/* Rotation by angle q about the unit axis a (Rodrigues). */
static void axis_angle(const double *a, double q, double *R)
{
    double W[9], W2[9], I[9], ah[3];
    double an = norm3(a);
    for (int i = 0; i < 3; ++i) ah[i] = a[i] / an;
    hat3(ah, W);
    matmul3(W, W, W2);
    eye3(I);
    double s = sin(q), c = cos(q);
    for (int i = 0; i < 9; ++i) R[i] = I[i] + s * W[i] + (1.0 - c) * W2[i];
}

/* FK: for j in topological order,
 *   revolute:  p_j = p_parent + R_parent t_j,   R_j = R_parent R_mount,j Rot(a_j, q_j);
 *   prismatic: R_j = R_parent R_mount,j,        p_j = p_parent + R_parent t_j + R_j a_j q_j;
 *   fixed:     R_j = R_parent R_mount,j,        p_j = p_parent + R_parent t_j;
 * q holds one value per variable (non-fixed joint).
 * EE k: R = R_e R_eeoff,  p = p_e + R_e t_eeoff.   Base frame = (I, 0).
 * Outputs (any may be NULL): R[n][9], p[n][3] (every joint), Ree[m][9], pee[m][3]. */
void ora_fk(const ora_tree *tr, const double *q, double *R, double *p, double *Ree,
            double *pee)
{
    double Rl[ORA_MAX_N][9], pl[ORA_MAX_N][3];
    int var_of[ORA_MAX_N];
    var_maps(tr, var_of, NULL);
    for (int j = 0; j < tr->n; ++j) {
        /* joint value: its variable, or the mimic rule on its driver's */
        const int src = mimic_of(tr, j);
        double qj = 0.0;
        if (src >= 0) qj = tr->mimic_mult[j] * q[var_of[src]] + tr->mimic_offset[j];
        else if (var_of[j] >= 0) qj = q[var_of[j]];
        double Rp[9], pp[3] = {0, 0, 0}, Rm[9], Rq[9], tmp[9], v[3];
        int par = tr->parent[j];
        if (par < 0) {
            eye3(Rp);
        } else {
            memcpy(Rp, Rl[par], sizeof Rp);
            memcpy(pp, pl[par], sizeof pp);
        }
        matvec3(Rp, tr->offset + 3 * j, v);
        for (int i = 0; i < 3; ++i) pl[j][i] = pp[i] + v[i];
        ora_quat_to_R(tr->mount_quat + 4 * j, Rm);
        matmul3(Rp, Rm, tmp);
        const int kind = jtype(tr, j);
        if (kind == ORA_REVOLUTE) {
            axis_angle(tr->axis + 3 * j, qj, Rq);
            matmul3(tmp, Rq, Rl[j]);
        } else {
            memcpy(Rl[j], tmp, sizeof tmp);
            if (kind == ORA_PRISMATIC) {
                double a[3], wa[3], an = norm3(tr->axis + 3 * j);
                for (int i = 0; i < 3; ++i) a[i] = tr->axis[3 * j + i] / an;
                matvec3(Rl[j], a, wa);
                for (int i = 0; i < 3; ++i) pl[j][i] += wa[i] * qj;
            }
        }
        if (R) memcpy(R + 9 * j, Rl[j], sizeof(double) * 9);
        if (p) memcpy(p + 3 * j, pl[j], sizeof(double) * 3);
    }
    for (int k = 0; k < tr->m; ++k) {
        int e = tr->ee_joint[k];
        double Ro[9], v[3], Rk[9];
        ora_quat_to_R(tr->ee_quat + 4 * k, Ro);
        matmul3(Rl[e], Ro, Rk);
        matvec3(Rl[e], tr->ee_offset + 3 * k, v);
        if (Ree) memcpy(Ree + 9 * k, Rk, sizeof Rk);
        if (pee) for (int i = 0; i < 3; ++i) pee[3 * k + i] = pl[e][i] + v[i];
    }
}

/* EE poses in the target layout [m][7] = (p, quat wxyz).  The quaternion of a
 * rotation matrix is taken with Shepperd's method, then w >= 0. */
void ora_fk_pose7(const ora_tree *tr, const double *q, double *out)
{
    double Ree[ORA_MAX_M * 9], pee[ORA_MAX_M * 3];
    ora_fk(tr, q, NULL, NULL, Ree, pee);
    for (int k = 0; k < tr->m; ++k) {
        const double *R = Ree + 9 * k;
        double *o = out + 7 * k, qw, qx, qy, qz;
        double tr_ = R[0] + R[4] + R[8];
        if (tr_ >= R[0] && tr_ >= R[4] && tr_ >= R[8]) {
            double s = 2.0 * sqrt(1.0 + tr_);
            qw = 0.25 * s; qx = (R[7] - R[5]) / s; qy = (R[2] - R[6]) / s; qz = (R[3] - R[1]) / s;
        } else if (R[0] >= R[4] && R[0] >= R[8]) {
            double s = 2.0 * sqrt(1.0 + R[0] - R[4] - R[8]);
            qw = (R[7] - R[5]) / s; qx = 0.25 * s; qy = (R[1] + R[3]) / s; qz = (R[2] + R[6]) / s;
        } else if (R[4] >= R[8]) {
            double s = 2.0 * sqrt(1.0 + R[4] - R[0] - R[8]);
            qw = (R[2] - R[6]) / s; qx = (R[1] + R[3]) / s; qy = 0.25 * s; qz = (R[5] + R[7]) / s;
        } else {
            double s = 2.0 * sqrt(1.0 + R[8] - R[0] - R[4]);
            qw = (R[3] - R[1]) / s; qx = (R[2] + R[6]) / s; qy = (R[5] + R[7]) / s; qz = 0.25 * s;
        }
        if (qw < 0.0) { qw = -qw; qx = -qx; qy = -qy; qz = -qz; }
        o[0] = pee[3 * k]; o[1] = pee[3 * k + 1]; o[2] = pee[3 * k + 2];
        o[3] = qw; o[4] = qx; o[5] = qy; o[6] = qz;
    }
}

/* ------------------------------------------------------- residuals, cost */

int ora_rows(const ora_tree *tr)
{
    int r = 0;
    for (int k = 0; k < tr->m; ++k) r += tr->ee_kind[k] == 0 ? 6 : 3;
    return r + 2 * ora_nvar(tr);
}

/* Rest value of variable v (joint j). */
static double rest_of(const ora_tree *tr, const ora_weights *w, int v, int j)
{
    return w->q_rest ? w->q_rest[v] : 0.5 * (tr->lower[j] + tr->upper[j]);
}

/* Residual vector, row order: per EE (pose: [w_pos rho; w_rot phi] with
 * [rho; phi] = log(T_target^-1 T_ee); position: w_pos (p_ee - p_target)),
 * then n limit rows, then n rest rows.
 * targets: [m][7] (p, quat wxyz); position EEs use the first three values.
 * Optional per-EE errors: pos_err = |p_ee - p_t|, rot_err = |log(R_t^T R_ee)|. */
void ora_residual(const ora_tree *tr, const double *targets, const ora_weights *w,
                  const double *q, double *r, double *pos_err, double *rot_err)
{
    double Ree[ORA_MAX_M * 9], pee[ORA_MAX_M * 3];
    ora_fk(tr, q, NULL, NULL, Ree, pee);
    int row = 0;
    for (int k = 0; k < tr->m; ++k) {
        const double *tg = targets + 7 * k;
        double d[3] = {pee[3 * k] - tg[0], pee[3 * k + 1] - tg[1], pee[3 * k + 2] - tg[2]};
        if (pos_err) pos_err[k] = norm3(d);
        if (tr->ee_kind[k] == 0) {
            double Rt[9], RtT[9], RE[9], tE[3], xi[6];
            ora_quat_to_R(tg + 3, Rt);
            transpose3(Rt, RtT);
            matmul3(RtT, Ree + 9 * k, RE);
            matvec3(RtT, d, tE);
            ora_se3_log(RE, tE, xi);
            for (int i = 0; i < 3; ++i) r[row + i] = w->w_pos * xi[i];
            for (int i = 0; i < 3; ++i) r[row + 3 + i] = w->w_rot * xi[3 + i];
            if (rot_err) rot_err[k] = norm3(xi + 3);
            row += 6;
        } else {
            for (int i = 0; i < 3; ++i) r[row + i] = w->w_pos * d[i];
            if (rot_err) rot_err[k] = 0.0;
            row += 3;
        }
    }
    int joint_of[ORA_MAX_N], var_of[ORA_MAX_N];
    var_maps(tr, var_of, joint_of);
    const int nv = ora_nvar(tr);
    for (int v = 0; v < nv; ++v) {
        const int j = joint_of[v];
        double over = q[v] - tr->upper[j], under = tr->lower[j] - q[v];
        r[row + v] = w->w_limit * ((over > 0.0 ? over : 0.0) + (under > 0.0 ? under : 0.0));
    }
    row += nv;
    for (int v = 0; v < nv; ++v) r[row + v] = w->w_rest * (q[v] - rest_of(tr, w, v, joint_of[v]));
}

double ora_cost(const ora_tree *tr, const double *targets, const ora_weights *w,
                const double *q)
{
    double r[ORA_MAX_ROWS];
    ora_residual(tr, targets, w, q, r, NULL, NULL);
    int rows = ora_rows(tr);
    double c = 0.0;
    for (int i = 0; i < rows; ++i) c += r[i] * r[i];
    return c;
}

static int is_ancestor(const ora_tree *tr, int j, int e)
{
    for (int a = e; a >= 0; a = tr->parent[a])
        if (a == j) return 1;
    return 0;
}

/* Analytic Jacobian dr/dq, row-major [rows][nvar].
 * Pose EE k, ancestor revolute joint j: world axis w_j = R_j a_j, point
 * velocity v_j = w_j x (p_ee - p_j); ancestor prismatic joint j: v_j = R_j a_j,
 * w_j = 0.  Body twist s_j = [R_ee^T v_j; R_ee^T w_j];
 * d xi / d q_j = J_r^-1(xi) s_j, rows weighted by w_pos / w_rot.
 * Position EE: w_pos v_j.  Limit rows: +-w_limit outside the limits, else 0.
 * Rest rows: w_rest on the diagonal. */
void ora_jacobian(const ora_tree *tr, const double *targets, const ora_weights *w,
                  const double *q, double *J)
{
    int n = ora_nvar(tr), rows = ora_rows(tr);
    int joint_of[ORA_MAX_N], var_of[ORA_MAX_N];
    var_maps(tr, var_of, joint_of);
    double R[ORA_MAX_N * 9], p[ORA_MAX_N * 3], Ree[ORA_MAX_M * 9], pee[ORA_MAX_M * 3];
    memset(J, 0, sizeof(double) * rows * n);
    ora_fk(tr, q, R, p, Ree, pee);
    int row = 0;
    for (int k = 0; k < tr->m; ++k) {
        const double *tg = targets + 7 * k;
        double Jr[36] = {0}, ReT[9] = {0};
        int pose = tr->ee_kind[k] == 0;
        if (pose) {
            double Rt[9], RtT[9], RE[9], tE[3], xi[6];
            double d[3] = {pee[3 * k] - tg[0], pee[3 * k + 1] - tg[1], pee[3 * k + 2] - tg[2]};
            ora_quat_to_R(tg + 3, Rt);
            transpose3(Rt, RtT);
            matmul3(RtT, Ree + 9 * k, RE);
            matvec3(RtT, d, tE);
            ora_se3_log(RE, tE, xi);
            ora_se3_jr_inv(xi, Jr);
            transpose3(Ree + 9 * k, ReT);
        }
        for (int j = 0; j < tr->n; ++j) {
            if (jtype(tr, j) == ORA_FIXED || !is_ancestor(tr, j, tr->ee_joint[k])) continue;
            /* column of joint j, added into its variable's (a mimic joint's
             * into its driver's, times the multiplier) */
            const int src = mimic_of(tr, j);
            const int jv = src >= 0 ? var_of[src] : var_of[j];
            const double mul = src >= 0 ? tr->mimic_mult[j] : 1.0;
            double om[3], lev[3], v[3];
            const double *Rj = R + 9 * j;
            double a[3];
            /* R_j a_j: the axis is fixed by the joint's own rotation. */
            double an = norm3(tr->axis + 3 * j);
            for (int i = 0; i < 3; ++i) a[i] = tr->axis[3 * j + i] / an;
            matvec3(Rj, a, om);
            if (jtype(tr, j) == ORA_PRISMATIC) {
                for (int i = 0; i < 3; ++i) {
                    v[i] = om[i];
                    om[i] = 0.0;
                }
            } else {
                for (int i = 0; i < 3; ++i) lev[i] = pee[3 * k + i] - p[3 * j + i];
                cross3(om, lev, v);
            }
            if (pose) {
                double s[6], col[6];
                matvec3(ReT, v, s);
                matvec3(ReT, om, s + 3);
                for (int i = 0; i < 6; ++i) {
                    double acc = 0.0;
                    for (int l = 0; l < 6; ++l) acc += Jr[6 * i + l] * s[l];
                    col[i] = acc;
                }
                for (int i = 0; i < 3; ++i) J[(row + i) * n + jv] += mul * w->w_pos * col[i];
                for (int i = 0; i < 3; ++i) J[(row + 3 + i) * n + jv] += mul * w->w_rot * col[3 + i];
            } else {
                for (int i = 0; i < 3; ++i) J[(row + i) * n + jv] += mul * w->w_pos * v[i];
            }
        }
        row += pose ? 6 : 3;
    }
    for (int v = 0; v < n; ++v) {
        const int j = joint_of[v];
        double d = 0.0;
        if (q[v] > tr->upper[j]) d = w->w_limit;
        else if (q[v] < tr->lower[j]) d = -w->w_limit;
        J[(row + v) * n + v] = d;
    }
    row += n;
    for (int v = 0; v < n; ++v) J[(row + v) * n + v] = w->w_rest;
}

/* ----------------------------------------------------------- linear algebra */

/* In-place lower Cholesky A = L L^T of the n x n row-major matrix (only the
 * lower triangle is read).  Returns 1 on success, 0 if a pivot d_k <= 0 or is
 * not finite.  *min_ratio receives min_k d_k / max_i A_ii. */
int ora_cholesky(int n, double *A, double *min_ratio)
{
    double maxd = 0.0, mr = INFINITY;
    for (int i = 0; i < n; ++i) if (A[i * n + i] > maxd) maxd = A[i * n + i];
    for (int k = 0; k < n; ++k) {
        double d = A[k * n + k];
        for (int l = 0; l < k; ++l) d -= A[k * n + l] * A[k * n + l];
        double ratio = d / maxd;
        if (ratio < mr) mr = ratio;
        if (!(d > 0.0) || !isfinite(d)) {
            if (min_ratio) *min_ratio = mr;
            return 0;
        }
        double lkk = sqrt(d);
        A[k * n + k] = lkk;
        for (int i = k + 1; i < n; ++i) {
            double s = A[i * n + k];
            for (int l = 0; l < k; ++l) s -= A[i * n + l] * A[k * n + l];
            A[i * n + k] = s / lkk;
        }
    }
    if (min_ratio) *min_ratio = mr;
    return 1;
}

/* Solve L L^T x = b given the factor from ora_cholesky. */
void ora_chol_solve(int n, const double *L, const double *b, double *x)
{
    double y[ORA_MAX_N];
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int l = 0; l < i; ++l) s -= L[i * n + l] * y[l];
        y[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int l = i + 1; l < n; ++l) s -= L[l * n + i] * x[l];
        x[i] = s / L[i * n + i];
    }
}

/* One damped Gauss-Newton step at q:
 *   A = J^T J,  g = J^T r,  D_jj = max(A_jj, floor),  (A + lambda D) delta = -g.
 * Returns 1 if the factorisation succeeded.  *fallback is set when the
 * smallest pivot ratio is at or below pivot_rel. */
int ora_lm_step(const ora_tree *tr, const double *targets, const ora_weights *w,
                const ora_options *o, const double *q, double lambda, double *delta,
                int *fallback)
{
    int n = ora_nvar(tr), rows = ora_rows(tr);
    double r[ORA_MAX_ROWS];
    double *J = malloc(sizeof(double) * rows * n);
    double *A = malloc(sizeof(double) * n * n);
    double g[ORA_MAX_N];
    ora_residual(tr, targets, w, q, r, NULL, NULL);
    ora_jacobian(tr, targets, w, q, J);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int l = 0; l < rows; ++l) s += J[l * n + i] * J[l * n + j];
            A[i * n + j] = s;
        }
        double s = 0.0;
        for (int l = 0; l < rows; ++l) s += J[l * n + i] * r[l];
        g[i] = s;
    }
    for (int i = 0; i < n; ++i) {
        double D = A[i * n + i] > o->damping_floor ? A[i * n + i] : o->damping_floor;
        A[i * n + i] += lambda * D;
    }
    double mr;
    int ok = ora_cholesky(n, A, &mr);
    if (fallback) *fallback = !(mr > o->pivot_rel);
    if (ok) {
        double mg[ORA_MAX_N];
        for (int i = 0; i < n; ++i) mg[i] = -g[i];
        ora_chol_solve(n, A, mg, delta);
    }
    free(J);
    free(A);
    return ok;
}

/* ------------------------------------------------------------------- LM */

typedef struct {
    double cost, pose_cost;
    int iters, accepts, status, iters_to_tol, flags;
} ora_result;

/* All EEs meet the tolerance (inclusive); position EEs test position only. */
static int meets_tol(const ora_tree *tr, const double *targets, const ora_weights *w,
                     const ora_options *o, const double *q, double *pos_err,
                     double *rot_err)
{
    double r[ORA_MAX_ROWS];
    ora_residual(tr, targets, w, q, r, pos_err, rot_err);
    for (int k = 0; k < tr->m; ++k) {
        if (!(pos_err[k] <= o->tol_pos)) return 0;
        if (tr->ee_kind[k] == 0 && !(rot_err[k] <= o->tol_rot)) return 0;
    }
    return 1;
}

static double pose_cost_of(const ora_tree *tr, const double *targets,
                           const ora_weights *w, const double *q)
{
    double r[ORA_MAX_ROWS];
    ora_residual(tr, targets, w, q, r, NULL, NULL);
    int prow = ora_rows(tr) - 2 * ora_nvar(tr);
    double c = 0.0;
    for (int i = 0; i < prow; ++i) c += r[i] * r[i];
    return c;
}

/* Levenberg-Marquardt on one problem.
 *   accept iff c(q + delta) < c(q) (strict; NaN rejects), then
 *   lambda <- max(lambda / nu_down, lambda_min);
 *   otherwise lambda <- min(lambda * nu_up, lambda_max), and a reject while
 *   lambda already sits at lambda_max stops the problem as STALLED.
 * Every trial (accepted or not) is one iteration.  The tolerance is checked
 * at the seed and after every accepted step (iters_to_tol records the first
 * iteration count at which it holds; -1 if never).
 * trace_* (optional, length n_trace): state after iterations 1..n_trace. */
void ora_lm_solve(const ora_tree *tr, const double *targets, const ora_weights *w,
                  const ora_options *o, const double *q0, double *q_out,
                  double *pos_err, double *rot_err, ora_result *res, int n_trace,
                  double *trace_q, int *trace_acc, double *trace_cost, int *trace_tie)
{
    int n = ora_nvar(tr);
    double q[ORA_MAX_N], qt[ORA_MAX_N], delta[ORA_MAX_N];
    memset(res, 0, sizeof *res);
    res->iters_to_tol = -1;
    int finite = 1;
    for (int j = 0; j < n; ++j) finite &= isfinite(q0[j]);
    for (int k = 0; k < tr->m; ++k)
        for (int i = 0; i < (tr->ee_kind[k] == 0 ? 7 : 3); ++i) finite &= isfinite(targets[7 * k + i]);
    memcpy(q, q0, sizeof(double) * n);
    if (!finite) {
        memcpy(q_out, q0, sizeof(double) * n);
        for (int k = 0; k < tr->m; ++k) pos_err[k] = rot_err[k] = NAN;
        res->cost = res->pose_cost = NAN;
        res->status = ORA_NONFINITE;
        return;
    }
    double c = ora_cost(tr, targets, w, q);
    double lambda = o->lambda0;
    int stalled = 0;
    if (meets_tol(tr, targets, w, o, q, pos_err, rot_err)) res->iters_to_tol = 0;
    int done = o->early_exit && res->iters_to_tol == 0;
    while (!done && res->iters < o->max_iters) {
        int fb = 0;
        int ok = ora_lm_step(tr, targets, w, o, q, lambda, delta, &fb);
        if (fb) res->flags |= ORA_FLAG_FP64;
        double ct = INFINITY;
        if (ok) {
            for (int j = 0; j < n; ++j) qt[j] = q[j] + delta[j];
            ct = ora_cost(tr, targets, w, qt);
        }
        int t = res->iters;
        res->iters++;
        int acc = ct < c;
        if (trace_tie && t < n_trace) trace_tie[t] = isfinite(ct) && fabs(ct - c) <= 1e-5 * c;
        if (acc) {
            memcpy(q, qt, sizeof(double) * n);
            c = ct;
            lambda = lambda / o->nu_down;
            if (lambda < o->lambda_min) lambda = o->lambda_min;
            res->accepts++;
            if (meets_tol(tr, targets, w, o, q, pos_err, rot_err)) {
                if (res->iters_to_tol < 0) res->iters_to_tol = res->iters;
                if (o->early_exit) done = 1;
            }
        } else {
            if (lambda >= o->lambda_max) {
                stalled = 1;
                done = 1;
            }
            lambda = lambda * o->nu_up;
            if (lambda > o->lambda_max) lambda = o->lambda_max;
        }
        if (t < n_trace) {
            if (trace_q) memcpy(trace_q + (size_t)t * n, q, sizeof(double) * n);
            if (trace_acc) trace_acc[t] = acc;
            if (trace_cost) trace_cost[t] = c;
        }
    }
    memcpy(q_out, q, sizeof(double) * n);
    int ok = meets_tol(tr, targets, w, o, q, pos_err, rot_err);
    res->cost = c;
    res->pose_cost = pose_cost_of(tr, targets, w, q);
    res->status = ok ? ORA_CONVERGED : (stalled ? ORA_STALLED : ORA_MAX_ITERS);
}

/* --------------------------------------------------------- batched driver */

typedef struct {
    const ora_tree *tr;
    const double *targets;      /* [T][m][7] */
    const double *seeds;        /* [N][n]    */
    const ora_weights *w;
    const ora_options *o;
    int K;
    long begin, end;
    double *q_out, *pos_err, *rot_err, *cost, *pose_cost;
    int *iters, *accepts, *status, *iters_to_tol, *flags;
} ora_chunk;

static void *run_chunk(void *arg)
{
    ora_chunk *c = arg;
    int n = ora_nvar(c->tr), m = c->tr->m;
    for (long p = c->begin; p < c->end; ++p) {
        ora_result r;
        ora_lm_solve(c->tr, c->targets + (size_t)(p / c->K) * m * 7, c->w, c->o,
                     c->seeds + (size_t)p * n, c->q_out + (size_t)p * n,
                     c->pos_err + (size_t)p * m, c->rot_err + (size_t)p * m, &r, 0,
                     NULL, NULL, NULL, NULL);
        c->cost[p] = r.cost;
        c->pose_cost[p] = r.pose_cost;
        c->iters[p] = r.iters;
        c->accepts[p] = r.accepts;
        c->status[p] = r.status | r.flags;
        c->iters_to_tol[p] = r.iters_to_tol;
    }
    return NULL;
}

/* N = T*K problems, problem p uses target p / K.  Work is split into
 * contiguous chunks over `threads` POSIX threads. */
void ora_lm_solve_batch(const ora_tree *tr, const double *targets, const double *seeds,
                        long N, int K, const ora_weights *w, const ora_options *o,
                        double *q_out, double *pos_err, double *rot_err, double *cost,
                        double *pose_cost, int *iters, int *accepts, int *status,
                        int *iters_to_tol, int threads)
{
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t th[256];
    ora_chunk ch[256];
    long per = (N + threads - 1) / threads;
    int used = 0;
    for (int t = 0; t < threads; ++t) {
        long b = t * per, e = b + per < N ? b + per : N;
        if (b >= e) break;
        ch[t] = (ora_chunk){tr, targets, seeds, w, o, K, b, e, q_out, pos_err, rot_err,
                            cost, pose_cost, iters, accepts, status, iters_to_tol, NULL};
        pthread_create(&th[t], NULL, run_chunk, &ch[t]);
        used++;
    }
    for (int t = 0; t < used; ++t) pthread_join(th[t], NULL);
}

/* Best of K seeds per target:
 *   if any seed meets the tolerance, the one with the lowest total cost among
 *   those; otherwise the lowest pose-only residual sum of squares; ties go to
 *   the lowest seed index.  success[t] = some seed meets the tolerance. */
void ora_best_of_k(long T, int K, const int *status, const double *cost,
                   const double *pose_cost, int *best, int *success)
{
    for (long t = 0; t < T; ++t) {
        int b = -1, any = 0;
        for (int k = 0; k < K; ++k) {
            long p = t * K + k;
            if ((status[p] & 0xff) == ORA_CONVERGED) {
                if (!any || cost[p] < cost[t * K + b]) b = k;
                any = 1;
            }
        }
        if (!any) {
            for (int k = 0; k < K; ++k) {
                long p = t * K + k;
                if (b < 0 || pose_cost[p] < pose_cost[t * K + b]) b = k;
            }
        }
        best[t] = b;
        success[t] = any;
    }
}

/* IK-Beam survivor order (Sec. V-C keeps the seeds of lowest error): seed a
 * comes before seed b if it meets the tolerance and b does not; otherwise by
 * the error measure of their class (total cost for seeds within tolerance,
 * pose-only residual sum of squares for the others), a NaN after every
 * number; then the lower seed index.  The first seed in this order is the
 * best-of-K choice whenever no value is NaN. */
static int beam_before(int conv_a, double va, int ka, int conv_b, double vb, int kb)
{
    if (conv_a != conv_b) return conv_a;
    int na = isnan(va), nb = isnan(vb);
    if (na != nb) return nb;
    if (!na && va != vb) return va < vb;
    return ka < kb;
}

/* Per target, the `keep` first of its K seeds in the survivor order, first
 * one first: kept[t * keep + r] = seed index (0..K-1).  A plain selection:
 * pass r takes the earliest seed not taken by passes 0..r-1. */
void ora_beam_select(long T, int K, int keep, const int *status, const double *cost,
                     const double *pose_cost, int *kept)
{
    for (long t = 0; t < T; ++t) {
        for (int r = 0; r < keep; ++r) {
            int b = -1;
            int conv_b = 0;
            double vb = 0;
            for (int k = 0; k < K; ++k) {
                int taken = 0;
                for (int u = 0; u < r; ++u)
                    if (kept[t * keep + u] == k) taken = 1;
                if (taken) continue;
                long p = t * K + k;
                int conv = (status[p] & 0xff) == ORA_CONVERGED;
                double v = conv ? cost[p] : pose_cost[p];
                if (b < 0 || beam_before(conv, v, k, conv_b, vb, b)) {
                    b = k;
                    conv_b = conv;
                    vb = v;
                }
            }
            kept[t * keep + r] = b;
        }
    }
}
