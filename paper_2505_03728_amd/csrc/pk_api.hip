// C ABI of the batched-LM IK library: contexts, robot upload, validation,
// workspace and kernel dispatch.  See include/pkmi.h for the contract.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "tree_layout.hpp"
#include "pk_ctx.hpp"

using namespace pk;

static std::string g_err_noctx;

int pk::fail(pk_ctx *ctx, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_err_noctx = buf;
    return code;
}

// ------------------------------------------------------------ host geometry (FP64)

namespace {

struct M3 {
    double a[9];
};

M3 eye()
{
    M3 m{};
    m.a[0] = m.a[4] = m.a[8] = 1.0;
    return m;
}

M3 mul(const M3 &A, const M3 &B)
{
    M3 C{};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) C.a[3 * i + j] += A.a[3 * i + k] * B.a[3 * k + j];
    return C;
}

M3 tr(const M3 &A)
{
    M3 T{};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) T.a[3 * i + j] = A.a[3 * j + i];
    return T;
}

M3 quat(const double *q)
{
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    M3 R{};
    R.a[0] = 1 - 2 * (y * y + z * z); R.a[1] = 2 * (x * y - w * z); R.a[2] = 2 * (x * z + w * y);
    R.a[3] = 2 * (x * y + w * z); R.a[4] = 1 - 2 * (x * x + z * z); R.a[5] = 2 * (y * z - w * x);
    R.a[6] = 2 * (x * z - w * y); R.a[7] = 2 * (y * z + w * x); R.a[8] = 1 - 2 * (x * x + y * y);
    return R;
}

// A rotation taking e_z to the unit vector a (Rodrigues about e_z x a).
M3 z_to(const double *a)
{
    if (a[2] > 1.0 - 1e-15) return eye();
    if (a[2] < -1.0 + 1e-15) {
        M3 R{};
        R.a[0] = 1; R.a[4] = -1; R.a[8] = -1;
        return R;
    }
    double k[3] = {-a[1], a[0], 0.0};          // e_z x a
    double s = sqrt(k[0] * k[0] + k[1] * k[1]);
    double c = a[2];
    k[0] /= s; k[1] /= s;
    double K[9] = {0, -k[2], k[1], k[2], 0, -k[0], -k[1], k[0], 0};
    M3 K2{}, R = eye();
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int l = 0; l < 3; ++l) K2.a[3 * i + j] += K[3 * i + l] * K[3 * l + j];
    for (int i = 0; i < 9; ++i) R.a[i] += s * K[i] + (1 - c) * K2.a[i];
    return R;
}

void mv(const M3 &A, const double *x, double *y)
{
    for (int i = 0; i < 3; ++i) y[i] = A.a[3 * i] * x[0] + A.a[3 * i + 1] * x[1] + A.a[3 * i + 2] * x[2];
}

float snap(double v) { return fabs(v) < 1e-12 ? 0.f : (float)v; }

bool finite_all(const double *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return false;
    return true;
}

}  // namespace

RobotEntry *pk::robot_of(pk_ctx *ctx, int32_t id)
{
    if (id < 0 || id >= (int)ctx->robots.size()) return nullptr;
    return &ctx->robots[id];
}

static void weights_into(const pk_cost_weights *w, SolveParams &P)
{
    P.w_pos = w->w_pos;
    P.w_rot = w->w_rot;
    P.w_limit = w->w_limit;
    P.w_rest = w->w_rest;
    P.q_rest = w->q_rest;
}

static bool finite_w(const pk_cost_weights *w)
{
    return isfinite(w->w_pos) && isfinite(w->w_rot) && isfinite(w->w_limit) && isfinite(w->w_rest);
}


int pk::prepare_solve(pk_ctx *ctx, const RobotEntry &rb, const pk_cost_weights *w,
                      const pk_lm_options *o, SolveParams &P, int &variant)
{
    if (o->max_iters < 0) return fail(ctx, PK_EINVAL, "LM options: max_iters < 0");
    if (!(o->lambda0 > 0) || !(o->nu_up > 1) || !(o->nu_down > 1) || !(o->lambda_min > 0) ||
        !(o->lambda_max >= o->lambda_min) || !(o->damping_floor > 0) || !(o->pivot_rel >= 0) ||
        !(o->tol_pos >= 0) || !(o->tol_rot >= 0))
        return fail(ctx, PK_EINVAL, "LM options: invalid value");
    if (!finite_w(w)) return fail(ctx, PK_EINVAL, "cost weights: non-finite value");
    const RobotC &H = rb.host;
    variant = o->variant;
    // the per-lane kernel: no mimic joints; prismatic joints on single chains
    const bool lane_ok = H.chains > 0 && H.n_mimic == 0 && (H.prismatic == 0 || H.chains == 1) &&
                         lane_variant_available(H.chains, H.chain_len, H.e[0].kind);
    const bool wave_ok = wave_variant_available(H.n);
    if (variant == PK_VARIANT_AUTO) variant = lane_ok ? PK_VARIANT_LANE : PK_VARIANT_WAVE;
    if (variant == PK_VARIANT_LANE && !lane_ok)
        return fail(ctx, PK_EUNSUPPORTED, "no per-lane kernel for this robot shape");
    if ((variant == PK_VARIANT_WAVE || variant == PK_VARIANT_WAVE_JOINT) && !wave_ok)
        return fail(ctx, PK_EUNSUPPORTED, "no wave kernel for n=%d", H.n);
    if (variant != PK_VARIANT_LANE && variant != PK_VARIANT_WAVE && variant != PK_VARIANT_WAVE_JOINT)
        return fail(ctx, PK_EINVAL, "unknown variant %d", variant);
    memset(&P, 0, sizeof P);
    weights_into(w, P);
    P.lambda0 = o->lambda0; P.nu_up = o->nu_up; P.nu_down = o->nu_down;
    P.lambda_min = o->lambda_min; P.lambda_max = o->lambda_max;
    P.tol_pos = o->tol_pos; P.tol_rot = o->tol_rot;
    P.damping_floor = o->damping_floor; P.pivot_rel = o->pivot_rel;
    P.max_iters = o->max_iters; P.early_exit = o->early_exit ? 1 : 0;
    P.target_exit = o->early_exit && o->target_exit ? 1 : 0;
    return PK_OK;
}

hipError_t pk::launch_lm(const RobotEntry &rb, const SolveParams &P, int variant, hipStream_t s,
                         int persist_blocks, const BestOut *best)
{
    if (variant == PK_VARIANT_LANE) return launch_lm_lane(rb.dev, rb.host, P, s, persist_blocks, best);
    if (best) return hipErrorInvalidValue;
    if (variant == PK_VARIANT_WAVE && path_variant_available(rb.host))
        return launch_lm_path(rb.dev, rb.host, P, s, persist_blocks);
    return launch_lm_wave(rb.dev, rb.host, P, s, persist_blocks);
}

// Scratch of the allocation-free solve: pose-only cost, total cost and status
// of up to PK_NOALLOC_MAX_PROBLEMS problems when best-of-K needs them and the
// caller did not ask for them.  One copy per GPU, held until the process
// ends; its device address is looked up once per device (scratch_ptr).
static __device__ __align__(256) float scratch[3 * (size_t)PK_NOALLOC_MAX_PROBLEMS];

namespace {
std::mutex g_scratch_mu;
float *g_scratch_dev[PK_MAX_DEVICES] = {};
}  // namespace

// Device address of `scratch` on `device` (current), looked up on the first
// call for that device.  The host-side name of the array is not a device
// address and is never passed to a kernel or a copy.
static int scratch_ptr(pk_ctx *ctx, int device, float **ptr)
{
    if (device < 0 || device >= PK_MAX_DEVICES)
        return fail(ctx, PK_EUNSUPPORTED, "device %d beyond the %d devices the scratch table holds",
                    device, PK_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ctx, PK_EHIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", device,
                        hipGetErrorString(e));
        g_scratch_dev[device] = (float *)p;
    }
    *ptr = g_scratch_dev[device];
    return PK_OK;
}

// ------------------------------------------------------------------- API

extern "C" {

int pk_create(pk_ctx **out, int device_ordinal)
{
    if (!out) return fail(nullptr, PK_EINVAL, "pk_create: out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return fail(nullptr, PK_EHIP, "pk_create: no HIP device");
    if (device_ordinal < 0 || device_ordinal >= count)
        return fail(nullptr, PK_EINVAL, "pk_create: device %d out of range [0,%d)", device_ordinal, count);
    if (hipSetDevice(device_ordinal) != hipSuccess)
        return fail(nullptr, PK_EHIP, "pk_create: hipSetDevice(%d) failed", device_ordinal);
    pk_ctx *c = new pk_ctx;
    c->device = device_ordinal;
    float *scr = nullptr;
    int rc = scratch_ptr(c, device_ordinal, &scr);      // once per device, device current
    if (rc) {
        g_err_noctx = c->err;
        delete c;
        return rc;
    }
    sched_load_env(c);
    *out = c;
    return PK_OK;
}

int pk_destroy(pk_ctx *ctx)
{
    if (!ctx) return PK_OK;
    (void)hipSetDevice(ctx->device);
    for (auto &r : ctx->robots)
        if (r.dev) (void)hipFree(r.dev);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->ws2) (void)hipFree(ctx->ws2);
    if (ctx->ws3) (void)hipFree(ctx->ws3);
    for (auto *sd : ctx->seeders) seeder_free(sd);
    sched_free(ctx);
    delete ctx;
    return PK_OK;
}

const char *pk_last_error(pk_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_err_noctx.c_str();
}


int pk_robot_upload(pk_ctx *ctx, const pk_tree *t, int32_t *robot_id)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_robot_upload: ctx is NULL");
    if (!t || !robot_id) return fail(ctx, PK_EINVAL, "pk_robot_upload: NULL argument");
    const int nt = t->n_joints, m = t->n_ee;
    if (nt < 1 || m < 1) return fail(ctx, PK_EINVAL, "pk_robot_upload: need >= 1 joint and EE");
    if (nt > PK_MAX_TREE_JOINTS || m > PK_MAX_EES)
        return fail(ctx, PK_EUNSUPPORTED, "pk_robot_upload: %d joints / %d EEs above %d / %d", nt, m,
                    PK_MAX_TREE_JOINTS, PK_MAX_EES);
    if (!t->parent || !t->mount_quat || !t->offset || !t->axis || !t->lower || !t->upper ||
        !t->ee_joint || !t->ee_offset || !t->ee_quat || !t->ee_kind)
        return fail(ctx, PK_EINVAL, "pk_robot_upload: NULL array in tree");
    if (!finite_all(t->mount_quat, 4 * nt) || !finite_all(t->offset, 3 * nt) ||
        !finite_all(t->axis, 3 * nt) || !finite_all(t->lower, nt) || !finite_all(t->upper, nt) ||
        !finite_all(t->ee_offset, 3 * m) || !finite_all(t->ee_quat, 4 * m))
        return fail(ctx, PK_EINVAL, "pk_robot_upload: non-finite tree value");

    // Fold fixed joints: a fixed joint's transform (mount, offset) is composed
    // into the mounts and offsets of its children and into its EEs, which are
    // then expressed in the frame of its nearest non-fixed ancestor.  Every
    // joint left is a variable.  rel_R / rel_p: a fixed joint's frame in its
    // anchor's frame.
    struct Folded {
        int parent;
        M3 mount;
        double offset[3], axis[3], lo, hi;
        int kind;
    };
    std::vector<Folded> F;
    std::vector<int> kind(nt), var(nt, -1), anchor(nt, -1);
    std::vector<M3> rel_R(nt);
    std::vector<double> rel_p(3 * nt, 0.0);
    for (int j = 0; j < nt; ++j) {
        const int par = t->parent[j];
        if (par < -1 || par >= j)
            return fail(ctx, PK_EINVAL, "pk_robot_upload: parent[%d] = %d not in [-1, %d)", j, par, j);
        kind[j] = t->joint_type ? t->joint_type[j] : PK_JOINT_REVOLUTE;
        if (kind[j] != PK_JOINT_REVOLUTE && kind[j] != PK_JOINT_PRISMATIC && kind[j] != PK_JOINT_FIXED)
            return fail(ctx, PK_EINVAL, "pk_robot_upload: joint_type[%d] = %d", j, kind[j]);
        const double *mq = t->mount_quat + 4 * j;
        double qn = sqrt(mq[0] * mq[0] + mq[1] * mq[1] + mq[2] * mq[2] + mq[3] * mq[3]);
        if (qn < 1e-6) return fail(ctx, PK_EINVAL, "pk_robot_upload: mount quaternion %d is zero", j);
        // parent frame in the anchor frame
        int anc = -1;
        M3 Rb = eye();
        double pb[3] = {0.0, 0.0, 0.0};
        if (par >= 0 && kind[par] != PK_JOINT_FIXED) {
            anc = var[par];
        } else if (par >= 0) {
            anc = anchor[par];
            Rb = rel_R[par];
            for (int i = 0; i < 3; ++i) pb[i] = rel_p[3 * par + i];
        }
        Folded f;
        f.parent = anc;
        f.mount = mul(Rb, quat(mq));
        mv(Rb, t->offset + 3 * j, f.offset);
        for (int i = 0; i < 3; ++i) f.offset[i] += pb[i];
        if (kind[j] == PK_JOINT_FIXED) {
            anchor[j] = anc;
            rel_R[j] = f.mount;
            for (int i = 0; i < 3; ++i) rel_p[3 * j + i] = f.offset[i];
            continue;
        }
        const double *a = t->axis + 3 * j;
        double an = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        if (fabs(an - 1.0) > 1e-3) return fail(ctx, PK_EINVAL, "pk_robot_upload: axis %d not unit (|a|=%g)", j, an);
        if (!(t->lower[j] <= t->upper[j]))
            return fail(ctx, PK_EINVAL, "pk_robot_upload: lower[%d] > upper[%d]", j, j);
        for (int i = 0; i < 3; ++i) f.axis[i] = a[i] / an;
        f.lo = t->lower[j];
        f.hi = t->upper[j];
        f.kind = kind[j];
        var[j] = (int)F.size();
        anchor[j] = var[j];
        F.push_back(f);
    }
    const int n = (int)F.size();
    if (n < 1) return fail(ctx, PK_EINVAL, "pk_robot_upload: every joint is fixed");
    if (n > PK_MAX_JOINTS)
        return fail(ctx, PK_EUNSUPPORTED, "pk_robot_upload: %d non-fixed joints above %d", n, PK_MAX_JOINTS);
    // Mimic joints (folded indices): driver, multiplier, offset.
    std::vector<int> msrc(n, -1), vidx(n, -1);
    std::vector<double> ma(n, 0.0), mb(n, 0.0);
    if (t->mimic_joint) {
        if (!t->mimic_multiplier || !t->mimic_offset)
            return fail(ctx, PK_EINVAL, "pk_robot_upload: mimic_joint without multiplier/offset");
        for (int j = 0; j < nt; ++j) {
            const int d = t->mimic_joint[j];
            if (d < 0) continue;
            if (kind[j] == PK_JOINT_FIXED) continue;   // a fixed joint ignores it
            if (d >= nt || var[d] < 0 || (t->mimic_joint[d] >= 0))
                return fail(ctx, PK_EINVAL, "pk_robot_upload: mimic_joint[%d] = %d is not a non-fixed, "
                            "non-mimic joint", j, d);
            if (!isfinite(t->mimic_multiplier[j]) || !isfinite(t->mimic_offset[j]))
                return fail(ctx, PK_EINVAL, "pk_robot_upload: non-finite mimic rule %d", j);
            msrc[var[j]] = var[d];
            ma[var[j]] = t->mimic_multiplier[j];
            mb[var[j]] = t->mimic_offset[j];
        }
    }

    RobotC R;
    memset(&R, 0, sizeof R);
    R.n = n;
    R.m = m;
    for (int j = 0; j < n; ++j) {
        if (msrc[j] >= 0) {
            R.mimic_list[R.n_mimic++] = (uint8_t)j;
        } else {
            vidx[j] = R.nv++;
        }
    }
    std::vector<M3> U(n);
    for (int j = 0; j < n; ++j) {
        const Folded &f = F[j];
        const int par = f.parent;
        U[j] = z_to(f.axis);
        M3 Upt = par < 0 ? eye() : tr(U[par]);
        M3 G = mul(mul(Upt, f.mount), U[j]);
        double tt[3];
        mv(Upt, f.offset, tt);
        JointC &J = R.j[j];
        M3 Ut = tr(U[j]);
        for (int i = 0; i < 9; ++i) {
            J.G[i] = snap(G.a[i]);
            J.Ut[i] = snap(Ut.a[i]);
        }
        for (int i = 0; i < 3; ++i) J.t[i] = snap(tt[i]);
        J.lo = (float)f.lo;
        J.hi = (float)f.hi;
        J.mid = (float)(0.5 * (f.lo + f.hi));
        J.type = f.kind;
        J.var = vidx[j];
        J.mimic_src = msrc[j];
        J.mimic_a = (float)ma[j];
        J.mimic_b = (float)mb[j];
        R.prismatic += f.kind == PK_JOINT_PRISMATIC;
        R.mid[j] = J.mid;
        J.parent = par;
        J.depth = par < 0 ? 0 : R.j[par].depth + 1;
        if (J.depth > R.max_depth) R.max_depth = J.depth;
        R.janc[j] = par < 0 ? 0 : (R.janc[par] | (1ull << par));
        for (int d = 0; d < J.depth; ++d) R.anc_at[j][d] = R.anc_at[par][d];
        R.anc_at[j][J.depth] = (uint8_t)j;
    }
    for (int j = 0; j < n; ++j) {
        R.jdesc[j] = 0;
        for (int k = 0; k < n; ++k)
            if ((R.janc[k] >> j) & 1ull) R.jdesc[j] |= 1ull << k;
    }
    build_step_schedule(R);
    int tgt = 0, rows = 0;
    std::vector<int> ee_var(m);
    for (int k = 0; k < m; ++k) {
        const int ej = t->ee_joint[k], kind = t->ee_kind[k];
        if (ej < 0 || ej >= nt) return fail(ctx, PK_EINVAL, "pk_robot_upload: ee_joint[%d] = %d out of range", k, ej);
        if (kind != PK_EE_POSE && kind != PK_EE_POSITION)
            return fail(ctx, PK_EINVAL, "pk_robot_upload: ee_kind[%d] = %d", k, kind);
        // the EE in the frame of its joint's anchor (the joint itself unless fixed)
        const int e = anchor[ej];
        if (e < 0) return fail(ctx, PK_EUNSUPPORTED, "pk_robot_upload: EE %d has no non-fixed ancestor", k);
        M3 Rrel = quat(t->ee_quat + 4 * k);
        double prel[3];
        for (int i = 0; i < 3; ++i) prel[i] = t->ee_offset[3 * k + i];
        if (var[ej] < 0) {
            double pr[3];
            mv(rel_R[ej], prel, pr);
            for (int i = 0; i < 3; ++i) prel[i] = rel_p[3 * ej + i] + pr[i];
            Rrel = mul(rel_R[ej], Rrel);
        }
        ee_var[k] = e;
        EEC &E = R.e[k];
        M3 Uet = tr(U[e]);
        M3 G = mul(Uet, Rrel);
        double tt[3];
        mv(Uet, prel, tt);
        for (int i = 0; i < 9; ++i) E.G[i] = snap(G.a[i]);
        for (int i = 0; i < 3; ++i) E.t[i] = snap(tt[i]);
        E.joint = e;
        E.kind = kind;
        E.tgt_off = tgt;
        E.row_off = rows;
        tgt += kind == PK_EE_POSE ? 7 : 3;
        rows += kind == PK_EE_POSE ? 6 : 3;
        uint64_t mask = 0;
        for (int a = e; a >= 0; a = F[a].parent) mask |= 1ull << a;
        R.anc[k] = mask;
        for (int j = 0; j < n; ++j)
            if (msrc[j] >= 0 && ((mask >> j) & 1ull) && !((mask >> msrc[j]) & 1ull))
                return fail(ctx, PK_EUNSUPPORTED, "pk_robot_upload: EE %d is below mimic joint %d but "
                            "not below its driver", k, j);
    }
    R.tgt_floats = tgt;
    R.pose_rows = rows;

    // Star-of-chains shape: C chains of L joints from the base, contiguous
    // indices, EE c at the tip of chain c, one EE kind.
    {
        int roots = 0;
        for (int j = 0; j < n; ++j) roots += F[j].parent < 0;
        bool star = roots >= 1 && n % roots == 0 && m == roots;
        const int L = star ? n / roots : 0;
        for (int j = 0; star && j < n; ++j)
            star = (j % L == 0) ? F[j].parent == -1 : F[j].parent == j - 1;
        for (int k = 0; star && k < m; ++k)
            star = ee_var[k] == k * L + L - 1 && t->ee_kind[k] == t->ee_kind[0];
        R.chains = star ? roots : 0;
        R.chain_len = star ? L : 0;
    }
    build_path_layout(R);

    RobotEntry ent;
    ent.host = R;
    PK_HIP(ctx, hipSetDevice(ctx->device));
    if (hipMalloc(&ent.dev, sizeof(RobotC)) != hipSuccess)
        return fail(ctx, PK_ENOMEM, "pk_robot_upload: hipMalloc failed");
    PK_HIP(ctx, hipMemcpy(ent.dev, &R, sizeof(RobotC), hipMemcpyHostToDevice));
    ctx->robots.push_back(ent);
    *robot_id = (int32_t)ctx->robots.size() - 1;
    return PK_OK;
}

int pk_robot_info(pk_ctx *ctx, int32_t id, int32_t *n, int32_t *m, int32_t *tf, int32_t *rows,
                  int32_t *chains, int32_t *chain_len)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_robot_info: ctx is NULL");
    if (id < 0 || id >= (int)ctx->robots.size()) return fail(ctx, PK_ENOTFOUND, "unknown robot %d", id);
    const RobotC &R = ctx->robots[id].host;
    if (n) *n = R.nv;
    if (m) *m = R.m;
    if (tf) *tf = R.tgt_floats;
    if (rows) *rows = R.pose_rows + 2 * R.nv;
    if (chains) *chains = R.chains;
    if (chain_len) *chain_len = R.chain_len;
    return PK_OK;
}


int pk_fk(pk_ctx *ctx, int32_t id, int64_t N, const float *q, float *ee_pose, float *frames,
          void *stream)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_fk: ctx is NULL");
    RobotEntry *r = robot_of(ctx, id);
    if (!r) return fail(ctx, PK_ENOTFOUND, "pk_fk: unknown robot %d", id);
    if (N < 0) return fail(ctx, PK_EINVAL, "pk_fk: N < 0");
    if (N == 0) return PK_OK;
    if (!q || !ee_pose) return fail(ctx, PK_EINVAL, "pk_fk: NULL q or ee_pose");
    if (N > (int64_t)INT32_MAX * 32) return fail(ctx, PK_EUNSUPPORTED, "pk_fk: N too large");
    PK_HIP(ctx, hipSetDevice(ctx->device));
    PK_HIP(ctx, launch_fk(r->dev, N, q, ee_pose, frames, (hipStream_t)stream));
    return PK_OK;
}

int pk_residual_jacobian(pk_ctx *ctx, int32_t id, int64_t N, int32_t K, const float *targets,
                         const float *q, const pk_cost_weights *w, float *r, float *J, void *stream)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_residual_jacobian: ctx is NULL");
    RobotEntry *rb = robot_of(ctx, id);
    if (!rb) return fail(ctx, PK_ENOTFOUND, "pk_residual_jacobian: unknown robot %d", id);
    if (N < 0 || K < 1 || N % K) return fail(ctx, PK_EINVAL, "pk_residual_jacobian: bad N=%lld K=%d", (long long)N, K);
    if (N == 0) return PK_OK;
    if (!targets || !q || !w || !r) return fail(ctx, PK_EINVAL, "pk_residual_jacobian: NULL argument");
    if (!finite_w(w)) return fail(ctx, PK_EINVAL, "pk_residual_jacobian: non-finite weight");
    SolveParams P;
    memset(&P, 0, sizeof P);
    weights_into(w, P);
    PK_HIP(ctx, hipSetDevice(ctx->device));
    PK_HIP(ctx, launch_residual_jacobian(rb->dev, N, K, targets, q, P, r, J, (hipStream_t)stream));
    return PK_OK;
}

static int ensure_ws(pk_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->ws_bytes) return PK_OK;
    if (ctx->ws) (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    if (hipMalloc(&ctx->ws, bytes) != hipSuccess) return fail(ctx, PK_ENOMEM, "workspace hipMalloc(%zu) failed", bytes);
    ctx->ws_bytes = bytes;
    return PK_OK;
}

// Shared body of pk_ik_solve and pk_ik_solve_noalloc.  noalloc: the
// best-of-K scratch comes from `scratch` (problem count bounded) instead of
// the context's grow-only workspace.
static int ik_solve_impl(pk_ctx *ctx, int32_t id, const pk_ik_problem *pr, const pk_cost_weights *w,
                         const pk_lm_options *o, const pk_ik_outputs *out, void *stream, bool noalloc)
{
    const char *fn = noalloc ? "pk_ik_solve_noalloc" : "pk_ik_solve";
    if (!ctx) return fail(nullptr, PK_EINVAL, "%s: ctx is NULL", fn);
    RobotEntry *rb = robot_of(ctx, id);
    if (!rb) return fail(ctx, PK_ENOTFOUND, "%s: unknown robot %d", fn, id);
    if (!pr || !w || !o || !out) return fail(ctx, PK_EINVAL, "%s: NULL argument", fn);
    if (pr->n_targets < 0 || pr->K < 1) return fail(ctx, PK_EINVAL, "%s: bad T=%lld K=%d", fn, (long long)pr->n_targets, pr->K);
    const int64_t N = pr->n_targets * pr->K;
    if (N == 0) return PK_OK;
    if (N >= (int64_t)1 << 31) return fail(ctx, PK_EUNSUPPORTED, "%s: %lld problems, limit 2^31 - 1", fn, (long long)N);
    if (!pr->targets || !pr->seeds || !out->joints) return fail(ctx, PK_EINVAL, "%s: NULL targets/seeds/joints", fn);
    if (out->trace_iters < 0 || out->trace_iters > 64 ||
        (out->trace_iters > 0 && (!out->trace_q || !out->trace_accept)))
        return fail(ctx, PK_EINVAL, "%s: bad trace request", fn);

    SolveParams P;
    int variant = 0;
    int rc0 = prepare_solve(ctx, *rb, w, o, P, variant);
    if (rc0) return rc0;
    const RobotC &H = rb->host;

    PK_HIP(ctx, hipSetDevice(ctx->device));
    const bool want_best = out->best_index || out->best_joints || out->target_success;
    // The per-lane kernel takes best-of-K itself when a target's K problems
    // share a wavefront (K divides 64): one launch instead of two, and the
    // costs and statuses need not go through memory.
    const bool fuse = want_best && variant == PK_VARIANT_LANE && 64 % pr->K == 0;
    // Workspace: pose-only cost, total cost and status when a separate
    // best-of-K pass needs them and the caller did not ask for them.
    float *ws_f = nullptr;
    if (want_best && !fuse && !(out->pose_cost && out->cost && out->status)) {
        if (noalloc) {
            int rc = scratch_ptr(ctx, ctx->device, &ws_f);
            if (rc) return rc;
        } else {
            int rc = ensure_ws(ctx, (size_t)N * 4 * 3);
            if (rc) return rc;
            ws_f = (float *)ctx->ws;
        }
    }

    P.K = pr->K; P.N = N; P.T = pr->n_targets;
    P.targets = pr->targets; P.seeds = pr->seeds;
    P.joints = out->joints; P.pos_err = out->pos_err; P.rot_err = out->rot_err;
    P.pose_cost = out->pose_cost ? out->pose_cost : (ws_f ? ws_f : nullptr);
    P.cost = out->cost ? out->cost : (ws_f ? ws_f + N : nullptr);
    P.status = out->status ? out->status : (ws_f ? (int32_t *)(ws_f + 2 * N) : nullptr);
    P.iters = out->iters; P.accepts = out->accepts; P.iters_to_tol = out->iters_to_tol;
    P.trace_iters = out->trace_iters; P.trace_q = out->trace_q; P.trace_acc = out->trace_accept;

    hipStream_t s = (hipStream_t)stream;
    if (fuse) {
        const BestOut B{out->best_index, out->best_joints, out->target_success};
        PK_HIP(ctx, launch_lm(*rb, P, variant, s, 0, &B));
        return PK_OK;
    }
    PK_HIP(ctx, launch_lm(*rb, P, variant, s));
    if (want_best)
        PK_HIP(ctx, launch_best_of_k(P, H.nv, out->best_index, out->best_joints, out->target_success, s));
    return PK_OK;
}

int pk_ik_solve(pk_ctx *ctx, int32_t id, const pk_ik_problem *pr, const pk_cost_weights *w,
                const pk_lm_options *o, const pk_ik_outputs *out, void *stream)
{
    return ik_solve_impl(ctx, id, pr, w, o, out, stream, false);
}

int pk_ik_solve_noalloc(pk_ctx *ctx, int32_t id, const pk_ik_problem *pr, const pk_cost_weights *w,
                        const pk_lm_options *o, const pk_ik_outputs *out, void *stream)
{
    if (pr && pr->n_targets > 0 && pr->K > 0 &&
        pr->n_targets * (int64_t)pr->K > (int64_t)PK_NOALLOC_MAX_PROBLEMS)
        return fail(ctx, PK_EUNSUPPORTED, "pk_ik_solve_noalloc: %lld problems, limit %d",
                    (long long)(pr->n_targets * (int64_t)pr->K), PK_NOALLOC_MAX_PROBLEMS);
    return ik_solve_impl(ctx, id, pr, w, o, out, stream, true);
}

}  // extern "C"
