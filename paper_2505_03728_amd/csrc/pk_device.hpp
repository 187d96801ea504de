// Device-side FP32 arithmetic shared by the LM kernels: the joint step of
// forward kinematics, the SE(3) pose residual log(T_target^-1 T_ee) and the
// right-Jacobian-inverse blocks used by the analytic Jacobian.
//
// Lie-group formulas: Barfoot, "State Estimation for Robotics" (2017),
// Sec. 7.1 (SO(3)/SE(3) left Jacobians and the Q block), with
// J_r^-1(xi) = J_l^-1(-xi).  Tangent order is xi = [rho; phi].
#pragma once

#include <hip/hip_runtime.h>

#include "pk_internal.hpp"

#define PK_DEV __device__ __forceinline__

namespace pk {

// 3x3 matrices are row-major float[9].

// Hardware sin/cos (v_sin_f32 / v_cos_f32 on q / 2pi): joint angles stay
// within a few turns, where the absolute error is ~1e-7.
PK_DEV void joint_sincos(float q, float &s, float &c)
{
    s = __sinf(q);
    c = __cosf(q);
}

// 1/x: v_rcp_f32 (about 1 ulp).
PK_DEV float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// 1/sqrt(d): v_rsq_f32 (about 1 ulp) in FP32, exact in FP64.
PK_DEV float rsqrt_t(float d) { return __builtin_amdgcn_rsqf(d); }
PK_DEV double rsqrt_t(double d) { return 1.0 / sqrt(d); }

// p = pp + Op t;  O = Op G Rz(q) with (s, c) = (sin q, cos q).
PK_DEV void joint_step(const float *Op, const float *pp, const float *G, const float *t,
                       float s, float c, float *O, float *p)
{
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        p[r] = pp[r] + Op[3 * r] * t[0] + Op[3 * r + 1] * t[1] + Op[3 * r + 2] * t[2];
        float m0 = Op[3 * r] * G[0] + Op[3 * r + 1] * G[3] + Op[3 * r + 2] * G[6];
        float m1 = Op[3 * r] * G[1] + Op[3 * r + 1] * G[4] + Op[3 * r + 2] * G[7];
        float m2 = Op[3 * r] * G[2] + Op[3 * r + 1] * G[5] + Op[3 * r + 2] * G[8];
        O[3 * r] = m0 * c + m1 * s;
        O[3 * r + 1] = m1 * c - m0 * s;
        O[3 * r + 2] = m2;
    }
}

// Prismatic joint: joint_step with s = 0, c = 1 leaves the frame unrotated;
// then the origin slides by q along the joint axis, the frame's third column.
PK_DEV void joint_slide(const float *O, float q, float *p)
{
    p[0] += q * O[2];
    p[1] += q * O[5];
    p[2] += q * O[8];
}

// EE frame: R = O G, p = pe + O t.
PK_DEV void ee_frame(const float *O, const float *p, const float *G, const float *t,
                     float *R, float *pe)
{
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        pe[r] = p[r] + O[3 * r] * t[0] + O[3 * r + 1] * t[1] + O[3 * r + 2] * t[2];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            R[3 * r + c] = O[3 * r] * G[c] + O[3 * r + 1] * G[3 + c] + O[3 * r + 2] * G[6 + c];
    }
}

PK_DEV void mm3(const float *A, const float *B, float *C)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// C = A B^T
PK_DEV void mmT3(const float *A, const float *B, float *C)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A[3 * i] * B[3 * j] + A[3 * i + 1] * B[3 * j + 1] + A[3 * i + 2] * B[3 * j + 2];
}

// C = A^T B
PK_DEV void mTm3(const float *A, const float *B, float *C)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A[i] * B[j] + A[3 + i] * B[3 + j] + A[6 + i] * B[6 + j];
}

PK_DEV void hat(const float *w, float *W)
{
    W[0] = 0.f;   W[1] = -w[2]; W[2] = w[1];
    W[3] = w[2];  W[4] = 0.f;   W[5] = -w[0];
    W[6] = -w[1]; W[7] = w[0];  W[8] = 0.f;
}

PK_DEV void cross(const float *a, const float *b, float *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Velocity of a joint with world axis om at origin pj, seen at the point pe:
// revolute (v, w) = (om x (pe - pj), om); prismatic (v, w) = (om, 0).
PK_DEV void joint_twist(bool prismatic, const float *om, const float *pj, const float *pe, float *v,
                        float *w)
{
    if (prismatic) {
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            v[u] = om[u];
            w[u] = 0.f;
        }
    } else {
        const float lev[3] = {pe[0] - pj[0], pe[1] - pj[1], pe[2] - pj[2]};
        cross(om, lev, v);
#pragma unroll
        for (int u = 0; u < 3; ++u) w[u] = om[u];
    }
}

// Unit quaternion (w >= 0) of a rotation matrix, Shepperd's method: the
// largest of |w|, |x|, |y|, |z| comes from a square root, the other three from
// sums and differences of off-diagonal entries over it.  The case is chosen
// per lane with selects around one square root (no divergent branches).
PK_DEV void rot_to_quat(const float *R, float &w, float &x, float &y, float &z)
{
    const float tr = R[0] + R[4] + R[8];
    const bool c0 = tr >= R[0] && tr >= R[4] && tr >= R[8];
    const bool c1 = !c0 && R[0] >= R[4] && R[0] >= R[8];
    const bool c2 = !c0 && !c1 && R[4] >= R[8];
    const float t = c0 ? 1.f + tr
                  : c1 ? 1.f + R[0] - R[4] - R[8]
                  : c2 ? 1.f + R[4] - R[0] - R[8]
                       : 1.f + R[8] - R[0] - R[4];
    const float s = 2.f * sqrtf(t), is = rcp(s), big = 0.25f * s;
    const float d1 = (R[7] - R[5]) * is, d2 = (R[2] - R[6]) * is, d3 = (R[3] - R[1]) * is;
    const float s1 = (R[1] + R[3]) * is, s2 = (R[2] + R[6]) * is, s3 = (R[5] + R[7]) * is;
    // (w, x, y, z) per case: 0 (big, d1, d2, d3), 1 (d1, big, s1, s2),
    // 2 (d2, s1, big, s3), 3 (d3, s2, s3, big)
    w = c0 ? big : c1 ? d1 : c2 ? d2 : d3;
    x = c0 ? d1 : c1 ? big : c2 ? s1 : s2;
    y = c0 ? d2 : c1 ? s1 : c2 ? big : s3;
    z = c0 ? d3 : c1 ? s2 : c2 ? s3 : big;
    if (w < 0.f) { w = -w; x = -x; y = -y; z = -z; }
    float in = rsqrtf(w * w + x * x + y * y + z * z);
    w *= in; x *= in; y *= in; z *= in;
}

// Rotation matrix of a (not necessarily unit) quaternion wxyz.
PK_DEV void quat_to_rot(float w, float x, float y, float z, float *R)
{
    float in = rsqrtf(w * w + x * x + y * y + z * z);
    w *= in; x *= in; y *= in; z *= in;
    R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
}

// SE(3) logarithm of E = (R_E, t_E) = T_target^-1 T_ee.
struct PoseLog {
    float rho[3], phi[3];
    float theta;
    float sh, ch;      // sin(theta/2), cos(theta/2)
};

// Rt: target rotation; Re: EE rotation; d = p_ee - p_target (world frame).
PK_DEV PoseLog pose_log(const float *Rt, const float *Re, const float *d)
{
    PoseLog L;
    float RE[9], tE[3];
    mTm3(Rt, Re, RE);
#pragma unroll
    for (int i = 0; i < 3; ++i) tE[i] = Rt[i] * d[0] + Rt[3 + i] * d[1] + Rt[6 + i] * d[2];
    float w, x, y, z;
    rot_to_quat(RE, w, x, y, z);
    float s = sqrtf(x * x + y * y + z * z);
    float theta = 2.f * atan2f(s, w);
    // phi = theta * v / |v|;  theta / s -> 2 / w (1 - s^2 / (3 w^2)) as s -> 0.
    const float iw = rcp(w);
    float f = s < 1e-4f ? 2.f * iw * (1.f - (1.f / 3.f) * s * s * iw * iw) : theta * rcp(s);
    L.phi[0] = f * x; L.phi[1] = f * y; L.phi[2] = f * z;
    L.theta = theta;
    L.sh = s;
    L.ch = w;
    // rho = J_l^-1(phi) t_E = t_E - phi x t_E / 2 + k phi x (phi x t_E),
    // k = (1 - (theta/2) cot(theta/2)) / theta^2, cot(theta/2) = w / s.
    float t2 = theta * theta, k;
    if (theta < 0.1f)
        k = 1.f / 12.f + t2 * (1.f / 720.f + t2 * (1.f / 30240.f));
    else
        k = (1.f - 0.5f * theta * w * rcp(s)) * rcp(t2);
    float a[3], b[3];
    cross(L.phi, tE, a);
    cross(L.phi, a, b);
#pragma unroll
    for (int i = 0; i < 3; ++i) L.rho[i] = tE[i] - 0.5f * a[i] + k * b[i];
    return L;
}

// Blocks of the right-Jacobian inverse folded with the EE rotation:
//   J_r^-1(xi) = [[P, B], [0, P]],  P = J_l^-1(-phi),  B = -P Q(-rho,-phi) P,
// M = P Re^T, N = B Re^T, so that for a joint with world axis w and point
// velocity v (world), d xi / d q = [M v + N w ; M w].
PK_DEV void jr_inv_blocks(const PoseLog &L, const float *Re, float *M, float *N)
{
    const float th = L.theta, t2 = th * th;
    float k, a1, a2, a3;
    if (th < 0.1f)
        k = 1.f / 12.f + t2 * (1.f / 720.f + t2 * (1.f / 30240.f));
    else
        k = (1.f - 0.5f * th * L.ch * rcp(L.sh)) * rcp(t2);
    if (th < 0.5f) {
        a1 = 1.f / 6.f + t2 * (-1.f / 120.f + t2 * (1.f / 5040.f - t2 * (1.f / 362880.f)));
        a2 = 1.f / 24.f + t2 * (-1.f / 720.f + t2 * (1.f / 40320.f - t2 * (1.f / 3628800.f)));
        a3 = 1.f / 120.f + t2 * (-1.f / 2520.f + t2 * (1.f / 120960.f - t2 * (1.f / 9979200.f)));
    } else {
        const float st = 2.f * L.sh * L.ch, ct = L.ch * L.ch - L.sh * L.sh;
        const float it = rcp(th), it2 = it * it, it3 = it2 * it;
        a1 = (th - st) * it3;
        a2 = (t2 - 4.f * L.sh * L.sh) * (0.5f * it2 * it2);   // 2 cos - 2 = -4 sin^2(th/2)
        a3 = (2.f * th - 3.f * st + th * ct) * (0.5f * it3 * it2);
    }
    // With f = phi, r = rho, d = f.r, c = f x r, t2 = |f|^2 and the identity
    // hat(a) hat(b) = b a^T - (a.b) I, the products of hats in P and Q reduce
    // to outer products:
    //   Ph Ph = f f^T - t2 I,
    //   Ph Rh + Rh Ph - Ph Rh Ph = r f^T + f r^T - 2 d I + d Ph,
    //   3 Ph Rh Ph - Ph Ph Rh - Rh Ph Ph = f c^T - c f^T - d Ph,
    //   Ph Rh Ph Ph + Ph Ph Rh Ph = -2 d (f f^T - t2 I),
    // so P = I + Ph/2 + k (f f^T - t2 I) and
    //   Q(-rho,-phi) = hat((a1 - a2) d f - r/2) + a1 (r f^T + f r^T)
    //                + a2 (f c^T - c f^T) - 2 a3 d f f^T + 2 d (a3 t2 - a1) I.
    const float *f = L.phi, *r = L.rho;
    const float d = f[0] * r[0] + f[1] * r[1] + f[2] * r[2];
    const float ff2 = f[0] * f[0] + f[1] * f[1] + f[2] * f[2];   // t2 of the identities
    float c[3];
    cross(f, r, c);
    float P[9], Q[9];
    const float pd = 1.f - k * ff2;                       // diagonal of P
    const float qd = 2.f * d * (a3 * ff2 - a1);           // diagonal of Q
    const float qf = -2.f * a3 * d;                       // f f^T coefficient of Q
    float sk[3];                                          // skew part of Q
#pragma unroll
    for (int i = 0; i < 3; ++i) sk[i] = (a1 - a2) * d * f[i] - 0.5f * r[i];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const float ff = f[i] * f[j];
            P[3 * i + j] = k * ff + (i == j ? pd : 0.f);
            Q[3 * i + j] = a1 * (r[i] * f[j] + f[i] * r[j]) + a2 * (f[i] * c[j] - c[i] * f[j]) + qf * ff +
                           (i == j ? qd : 0.f);
        }
    // + hat(f)/2 on P, + hat(sk) on Q
    P[1] -= 0.5f * f[2]; P[2] += 0.5f * f[1]; P[5] -= 0.5f * f[0];
    P[3] += 0.5f * f[2]; P[6] -= 0.5f * f[1]; P[7] += 0.5f * f[0];
    Q[1] -= sk[2]; Q[2] += sk[1]; Q[5] -= sk[0];
    Q[3] += sk[2]; Q[6] -= sk[1]; Q[7] += sk[0];
    // M = P Re^T;  N = B Re^T = -P Q P Re^T = -P (Q M)
    mmT3(P, Re, M);
    float QM[9], PQM[9];
    mm3(Q, M, QM);
    mm3(P, QM, PQM);
#pragma unroll
    for (int i = 0; i < 9; ++i) N[i] = -PQM[i];
}

// Best of K problems base .. base+K-1: the lowest total cost among those
// that converged, else the lowest pose-only cost; ties to the lower index.
PK_DEV int best_of_k_pick(const int32_t *status, const float *cost, const float *pcost, int64_t base,
                          int K, bool &any)
{
    int b = -1;
    any = false;
    for (int k = 0; k < K; ++k) {
        const int64_t p = base + k;
        if ((status[p] & 0xff) == PK_CONVERGED) {
            if (!any || cost[p] < cost[base + b]) b = k;
            any = true;
        }
    }
    if (!any)
        for (int k = 0; k < K; ++k) {
            const int64_t p = base + k;
            if (b < 0 || pcost[p] < pcost[base + b]) b = k;
        }
    return b;
}

}  // namespace pk
