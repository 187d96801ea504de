// Learned seeder: an MLP from an EE target to K joint-space seeds, trained on
// (FK(q), q) pairs with a min-over-seeds loss and Adam, run as BF16
// matrix-core (MFMA) GEMMs with FP32 accumulation.
//
//   x = [p / reach, quat (w >= 0)]  (7 inputs, zero-padded to 32)
//   h_l = SiLU(W_l h_{l-1} + b_l)   (hidden width H, `depth` layers)
//   y = W_out h + b_out             (7K <= 64 outputs, padded to 64)
//   L = mean_b min_k |y_{b,k} - q_b|^2
//
// The GEMMs (BF16 MFMA, FP32 accumulation, fused epilogues) are in sd_gemm.hpp.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "pk_ctx.hpp"
#include "pk_device.hpp"

#include "sd_gemm.hpp"
#include "sd_mlp.hpp"

namespace pk {
namespace sd {

// out[i] = sum over z of part[z * count + i] (fixed order).
__global__ void split_reduce_kernel(int64_t count, int splits, const float *__restrict__ part, float *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[z * count + i];
    out[i] = s;
}

// ------------------------------------------------------------ small kernels

// Network input from poses: [p / reach, quat with w >= 0] -> bf16 row, zero pad.
__global__ void encode_kernel(int64_t rows, int64_t valid, const float *__restrict__ planes,
                              int64_t plane_stride, float inv_reach, int in_pad, __bf16 *X0,
                              float *x32)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    float v[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (i < valid) {
        for (int u = 0; u < 7; ++u) v[u] = planes[u * plane_stride + i];
        float w = v[3], x = v[4], y = v[5], z = v[6];
        const float in = rsqrtf(w * w + x * x + y * y + z * z);
        const float sg = w < 0.f ? -in : in;
        v[3] = w * sg; v[4] = x * sg; v[5] = y * sg; v[6] = z * sg;
        v[0] *= inv_reach; v[1] *= inv_reach; v[2] *= inv_reach;
    }
    if (x32)
        for (int u = 0; u < 7; ++u) x32[i * 7 + u] = v[u];
    if (X0)
        for (int u = 0; u < in_pad; ++u) X0[i * in_pad + u] = (__bf16)(u < 7 ? v[u] : 0.f);
}

// One training batch: X0 rows from the pre-encoded inputs, Q from the joint
// values, sample order from the caller's permutation.
// Training rows of local step (*dstep - step0) of a train call with nsteps
// steps: epoch e uses perm row e (or index order), batch b its rows b*B...
__global__ void gather_kernel(int B, int64_t S, int n, int in_pad, int steps_per_epoch, int nsteps,
                              int step0, const int *__restrict__ dstep, const int *__restrict__ perm,
                              const float *__restrict__ xall, const float *__restrict__ qtrain,
                              __bf16 *X0, float *Q)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    const int local = *dstep - step0;
    if (local < 0 || local >= nsteps) return;
    const int64_t e = local / steps_per_epoch, b = local % steps_per_epoch;
    const int64_t pos = b * B + i;
    const int64_t idx = perm ? perm[e * S + pos] : pos;
    if (idx < 0 || idx >= S) return;
    for (int u = 0; u < in_pad; ++u) X0[(int64_t)i * in_pad + u] = (__bf16)(u < 7 ? xall[idx * 7 + u] : 0.f);
    for (int j = 0; j < n; ++j) Q[(int64_t)i * n + j] = qtrain[(int64_t)j * S + idx];
}

// Min-over-seeds loss: per sample the closest seed (ties -> lowest k) gets
// the gradient 2 (y - q) / B.  One wavefront per row, lane = output column
// (K n <= 64), four rows per wavefront, sixteen per block; per-block partial
// sums of the loss in a fixed order.  Rows in [B, rows) get zero gradients.
__global__ __launch_bounds__(256) void loss_kernel(int rows, int B, int n, int K, int out_pad,
                                                   const float *__restrict__ Y,
                                                   const float *__restrict__ Q, float *dY,
                                                   __bf16 *dYb, float *partial)
{
    __shared__ float red[4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kn = K * n;
    const float sc = 2.f / (float)B;
    float wl = 0.f;
    for (int rr = 0; rr < 4; ++rr) {
        const int64_t i = (int64_t)blockIdx.x * 16 + w * 4 + rr;
        if (i >= rows) break;                          // uniform per wavefront
        const bool valid = i < B;
        float diff = 0.f;
        if (valid && lane < kn) diff = Y[i * out_pad + lane] - Q[i * n + lane % n];
        const float s2 = diff * diff;
        // squared distance of seed k = lane (sum over j in order)
        float dk = 0.f;
        for (int j = 0; j < n; ++j) dk += __shfl(s2, (lane < K ? lane : 0) * n + j, 64);
        float bd = lane < K ? dk : INFINITY;
        int bi = lane;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const float od = __shfl_xor(bd, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (od < bd || (od == bd && oi < bi)) {
                bd = od;
                bi = oi;
            }
        }
        const float g = (valid && lane < kn && lane / n == bi) ? sc * diff : 0.f;
        for (int c = lane; c < out_pad; c += 64) {
            const float gc = c == lane ? g : 0.f;
            dY[i * out_pad + c] = gc;
            dYb[i * out_pad + c] = (__bf16)gc;
        }
        if (valid) wl += bd;
    }
    if (lane == 0) red[w] = wl;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// loss_log[*dstep - step0] (when within [0, nlog)) and/or *loss_out: the sum
// of the partials / B, as a fixed-order 256-thread reduction.
__global__ __launch_bounds__(256) void loss_finish_kernel(int nparts, int B, const float *__restrict__ partial,
                                                          const int *__restrict__ dstep, int step0, int nlog,
                                                          float *loss_log, float *loss_out)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < nparts; i += 256) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const float v = red[0] / (float)B;
    const int li = *dstep - step0;
    if (loss_log && li >= 0 && li < nlog) loss_log[li] = v;
    if (loss_out) *loss_out = v;
}

// Column sums of dZ [R][C] (bias gradient), two deterministic passes.  Pass
// 1: per 128-row chunk, 64 columns x 4 row phases per block.
constexpr int COLSUM_ROWS = 128;
__global__ __launch_bounds__(256) void colsum_pass1(int R, int C, const float *__restrict__ X, float *part)
{
    __shared__ float red[4][64];
    const int cl = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + cl, r0 = blockIdx.y * COLSUM_ROWS;
    const int r1 = min(r0 + COLSUM_ROWS, R);
    float s = 0.f;
    if (c < C)
        for (int r = r0 + ph; r < r1; r += 4) s += X[(int64_t)r * C + c];
    red[ph][cl] = s;
    __syncthreads();
    if (ph == 0 && c < C) part[(int64_t)blockIdx.y * C + c] = ((red[0][cl] + red[1][cl]) + red[2][cl]) + red[3][cl];
}
// Pass 2: out[c] = sum of the chunk partials, 64 columns x 4 chunk phases
// per block, fixed order.
__global__ __launch_bounds__(256) void colsum_pass2(int nchunk, int C, const float *__restrict__ part, float *out)
{
    __shared__ float red[4][64];
    const int cl = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + cl;
    float s = 0.f;
    if (c < C)
        for (int i = ph; i < nchunk; i += 4) s += part[(int64_t)i * C + c];
    red[ph][cl] = s;
    __syncthreads();
    if (ph == 0 && c < C) out[c] = ((red[0][cl] + red[1][cl]) + red[2][cl]) + red[3][cl];
}

// Adam (Kingma & Ba 2015) with bias correction; t = step + 1 from the device
// counter.  Writes the BF16 copy used by the GEMMs.
__global__ void adam_kernel(int64_t count, float lr, float b1, float b2, float eps,
                            const int *__restrict__ dstep, float *P, const float *__restrict__ G,
                            float *Mo, float *V, __bf16 *Pb)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float t = (float)(*dstep + 1);
    const float c1 = 1.f - powf(b1, t), c2 = 1.f - powf(b2, t);
    const float g = G[i];
    const float m = b1 * Mo[i] + (1.f - b1) * g;
    const float v = b2 * V[i] + (1.f - b2) * g * g;
    Mo[i] = m;
    V[i] = v;
    const float p = P[i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
    P[i] = p;
    Pb[i] = (__bf16)p;
}

__global__ void tick_kernel(int *dstep)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dstep += 1;
}

__global__ void to_bf16_kernel(int64_t count, const float *__restrict__ P, __bf16 *Pb)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) Pb[i] = (__bf16)P[i];
}

__global__ void fill_kernel(int64_t count, float v, float *p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// Seeds [n][T*K] from the network output, clamped to the joint limits.  One
// thread per (target, seed): its n outputs are contiguous in Y, and
// neighbouring threads write neighbouring seeds of each joint plane.
__global__ void seeds_kernel(int64_t T, int K, int n, int out_pad, const float *__restrict__ Y,
                             const RobotC *__restrict__ rb, float *seeds)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // = t * K + k
    const int64_t NK = T * K;
    if (i >= NK) return;
    const int64_t t = i / K;
    const int k = (int)(i - t * K);
    const float *y = Y + t * out_pad + k * n;
    for (int j = 0; j < n; ++j) seeds[(int64_t)j * NK + i] = fminf(fmaxf(y[j], rb->j[j].lo), rb->j[j].hi);
}

// Encoded inputs x [B][7] (and optionally joints q [B][n]) into the padded
// BF16 input rows (rows >= B are zero).
__global__ void load_rows_kernel(int64_t rows, int64_t B, int in_pad, int n, const float *__restrict__ x,
                                 const float *__restrict__ q, __bf16 *X0, float *Q)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    for (int u = 0; u < in_pad; ++u) X0[i * in_pad + u] = (__bf16)(i < B && u < 7 ? x[i * 7 + u] : 0.f);
    if (q && Q)
        for (int j = 0; j < n; ++j) Q[i * n + j] = i < B ? q[i * n + j] : 0.f;
}

__global__ void store_out_kernel(int64_t B, int out_real, int out_pad, const float *__restrict__ Y,
                                 float *y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    for (int c = 0; c < out_real; ++c) y[i * out_real + c] = Y[i * out_pad + c];
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace sd

// ------------------------------------------------------------------ state

struct SeederState {
    int robot_id, n, K, H, depth, in_pad, out_real, out_pad;
    float reach;
    std::vector<int> lin, lout;         // per layer padded in / out widths
    std::vector<int64_t> woff, boff;    // offsets in the parameter buffer
    int64_t nparam;
    float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;
    __bf16 *Pb = nullptr;
    int *dstep = nullptr;
    int host_step = 0;
    // activations for up to `cap` rows
    int64_t cap = 0;
    __bf16 *X0 = nullptr, *Hb = nullptr, *dZb = nullptr, *dYb = nullptr;
    float *Z = nullptr, *Y = nullptr, *dZ = nullptr, *dY = nullptr, *Q = nullptr, *part = nullptr;
    float *splitbuf = nullptr;          // split-K partial weight gradients
    size_t splitbuf_floats = 0;
    // BF16 weights in MFMA fragment order for the fused inference pass,
    // rebuilt from Pb after the parameters change.
    __bf16 *Wf = nullptr;
    std::vector<int64_t> wfoff;
    bool wf_dirty = true;
    std::vector<void *> extra;
};

void seeder_free(SeederState *s)
{
    if (!s) return;
    void *ptrs[] = {s->P, s->G, s->M, s->V, s->Pb, s->dstep, s->X0, s->Hb, s->dZb, s->dYb, s->Z,
                    s->Y, s->dZ, s->dY, s->Q, s->part, s->splitbuf, s->Wf};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (void *p : s->extra)
        if (p) (void)hipFree(p);
    delete s;
}

namespace {

int alloc_acts(pk_ctx *ctx, SeederState *s, int64_t rows)
{
    if (rows <= s->cap) return PK_OK;
    void *ptrs[] = {s->X0, s->Hb, s->dZb, s->dYb, s->Z, s->Y, s->dZ, s->dY, s->Q, s->part};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    const int L = s->depth;
    const int64_t hsz = rows * s->H;
    bool ok = true;
    ok &= hipMalloc(&s->X0, rows * s->in_pad * sizeof(__bf16)) == hipSuccess;
    ok &= hipMalloc(&s->Hb, (size_t)L * hsz * sizeof(__bf16)) == hipSuccess;
    ok &= hipMalloc(&s->dZb, hsz * sizeof(__bf16)) == hipSuccess;
    ok &= hipMalloc(&s->dYb, rows * s->out_pad * sizeof(__bf16)) == hipSuccess;
    ok &= hipMalloc(&s->Z, (size_t)L * hsz * sizeof(float)) == hipSuccess;
    ok &= hipMalloc(&s->Y, rows * s->out_pad * sizeof(float)) == hipSuccess;
    ok &= hipMalloc(&s->dZ, hsz * sizeof(float)) == hipSuccess;
    ok &= hipMalloc(&s->dY, rows * s->out_pad * sizeof(float)) == hipSuccess;
    ok &= hipMalloc(&s->Q, rows * s->n * sizeof(float)) == hipSuccess;
    // column-sum partials (one row per 128-row chunk) or loss partials (one per 16 rows)
    ok &= hipMalloc(&s->part, ((rows / sd::COLSUM_ROWS + 1) * (size_t)std::max(s->H, s->out_pad) +
                               rows / 16 + 1) * sizeof(float) + 4096) == hipSuccess;
    // Split-K partials: sized for the largest split any row count can pick.
    size_t need = 0;
    for (int l = 0; l <= L; ++l) {
        const int M = s->lout[l], N = s->lin[l];
        need = std::max(need, (size_t)sd::split_max(M, N) * M * N);
    }
    if (s->splitbuf) (void)hipFree(s->splitbuf);
    s->splitbuf = nullptr;
    s->splitbuf_floats = 0;
    if (hipMalloc(&s->splitbuf, need * sizeof(float)) == hipSuccess)
        s->splitbuf_floats = need;
    else
        ok = false;
    if (!ok) {
        s->cap = 0;
        return fail(ctx, PK_ENOMEM, "seeder: activation allocation for %lld rows failed", (long long)rows);
    }
    s->cap = rows;
    return PK_OK;
}

SeederState *seeder_of(pk_ctx *ctx, int32_t id)
{
    if (id < 0 || id >= (int)ctx->seeders.size()) return nullptr;
    return ctx->seeders[id];
}

// Forward pass over `rows` rows of X0 (a multiple of 128).  train=true keeps
// the FP32 pre-activations for backward.
hipError_t forward(SeederState *s, int64_t rows, bool train, hipStream_t st)
{
    using namespace sd;
    const __bf16 *in = s->X0;
    int ld_in = s->in_pad;
    hipError_t e;
    for (int l = 0; l < s->depth; ++l) {
        __bf16 *Hl = s->Hb + (size_t)l * rows * s->H;
        float *Zl = train ? s->Z + (size_t)l * rows * s->H : nullptr;
        e = gemm<A_MK, B_NK>((int)rows, s->H, s->lin[l], in, ld_in, s->Pb + s->woff[l], s->lin[l],
                             EpiHidden{s->P + s->boff[l], Zl, Hl, s->H}, st);
        if (e != hipSuccess) return e;
        in = Hl;
        ld_in = s->H;
    }
    const int L = s->depth;
    return gemm<A_MK, B_NK>((int)rows, s->out_pad, s->H, in, s->H, s->Pb + s->woff[L], s->H,
                            EpiOut{s->P + s->boff[L], s->Y, s->out_pad}, st);
}

// Inference forward pass over `rows` rows of X0 into Y: the fused kernel for
// the shapes it covers (hidden width 128, 256 or 512, padded output width
// 64), else the layer-by-layer GEMMs.  Both give the same values.
hipError_t forward_infer(SeederState *s, int64_t rows, hipStream_t st)
{
    using namespace sd;
    const int JT = s->H / 64;
    const bool fused = s->in_pad == 32 && s->out_pad == 64 && (JT == 2 || JT == 4 || JT == 8) &&
                       s->depth + 1 <= MLP_MAX_LAYERS;
    if (!fused) return forward(s, rows, false, st);
    if (s->wf_dirty) {
        for (int l = 0; l <= s->depth; ++l) {
            const int N = s->lout[l], K = s->lin[l];
            const int64_t pieces = (int64_t)(N / 16) * (K / 32) * 64;
            hipLaunchKernelGGL(frag_layout_kernel, dim3(blocks(pieces, 256)), dim3(256), 0, st, N, K, K,
                               (const __bf16 *)(s->Pb + s->woff[l]), l < s->depth ? 1 : 0, s->Wf + s->wfoff[l]);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        s->wf_dirty = false;
    }
    MlpArgs a{};
    a.depth = s->depth;
    a.out_pad = s->out_pad;
    for (int l = 0; l <= s->depth; ++l) {
        a.wf[l] = s->Wf + s->wfoff[l];
        a.bias[l] = s->P + s->boff[l];
    }
    const dim3 grid((unsigned)(rows / 64)), block(256);
    if (JT == 2)
        hipLaunchKernelGGL((mlp_infer_kernel<2, 1>), grid, block, 0, st, a, s->X0, s->Y);
    else if (JT == 4)
        hipLaunchKernelGGL((mlp_infer_kernel<4, 1>), grid, block, 0, st, a, s->X0, s->Y);
    else
        hipLaunchKernelGGL((mlp_infer_kernel<8, 1>), grid, block, 0, st, a, s->X0, s->Y);
    return hipGetLastError();
}

// Weight gradient dW [M][N] = A^T B reduced over `rows` (split-K + fixed-order sum).
hipError_t weight_grad(SeederState *s, int M, int N, int64_t rows, const __bf16 *A, int lda,
                       const __bf16 *B, int ldb, float *out, hipStream_t st)
{
    using namespace sd;
    int sp = split_for(M, N, (int)rows);
    while (sp > 1 && (size_t)sp * M * N > s->splitbuf_floats) sp /= 2;
    if (sp == 1)
        return gemm<A_KM, B_KN>(M, N, (int)rows, A, lda, B, ldb, EpiStore{out, N, 0}, st);
    const size_t cnt = (size_t)M * N;
    hipError_t e = gemm<A_KM, B_KN>(M, N, (int)rows, A, lda, B, ldb, EpiStore{s->splitbuf, N, cnt}, st, sp);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(split_reduce_kernel, dim3(blocks((int64_t)cnt, 256)), dim3(256), 0, st, (int64_t)cnt, sp,
                       s->splitbuf, out);
    return hipGetLastError();
}

// Loss gradient in dY/dYb -> parameter gradients in G.
hipError_t backward(SeederState *s, int64_t rows, hipStream_t st)
{
    using namespace sd;
    hipError_t e;
    const int L = s->depth;
    const int nchunk = (int)((rows + sd::COLSUM_ROWS - 1) / sd::COLSUM_ROWS);
    // output layer
    const __bf16 *Hlast = s->Hb + (size_t)(L - 1) * rows * s->H;
    e = weight_grad(s, s->out_pad, s->H, rows, s->dYb, s->out_pad, Hlast, s->H, s->G + s->woff[L], st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colsum_pass1, dim3(blocks(s->out_pad, 64), nchunk), dim3(256), 0, st, (int)rows,
                       s->out_pad, s->dY, s->part);
    hipLaunchKernelGGL(colsum_pass2, dim3(blocks(s->out_pad, 64)), dim3(256), 0, st, nchunk, s->out_pad,
                       s->part, s->G + s->boff[L]);
    // dZ of the last hidden layer = (dY W_out) * SiLU'(Z)
    const __bf16 *gin = s->dYb;
    int gld = s->out_pad, gk = s->out_pad;
    for (int l = L - 1; l >= 0; --l) {
        const float *Zl = s->Z + (size_t)l * rows * s->H;
        e = gemm<A_MK, B_KN>((int)rows, s->H, gk, gin, gld, s->Pb + s->woff[l + 1], s->H,
                             EpiBackHidden{Zl, s->dZ, s->dZb, s->H}, st);
        if (e != hipSuccess) return e;
        const __bf16 *inl = l == 0 ? s->X0 : s->Hb + (size_t)(l - 1) * rows * s->H;
        const int ldin = l == 0 ? s->in_pad : s->H;
        e = weight_grad(s, s->H, s->lin[l], rows, s->dZb, s->H, inl, ldin, s->G + s->woff[l], st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(colsum_pass1, dim3(blocks(s->H, 64), nchunk), dim3(256), 0, st, (int)rows,
                           s->H, s->dZ, s->part);
        hipLaunchKernelGGL(colsum_pass2, dim3(blocks(s->H, 64)), dim3(256), 0, st, nchunk, s->H,
                           s->part, s->G + s->boff[l]);
        gin = s->dZb;
        gld = s->H;
        gk = s->H;
    }
    return hipGetLastError();
}

float tree_reach(const RobotC &R)
{
    // Sum of link and EE offset lengths (an upper bound on the EE distance).
    double r = 0.0;
    for (int j = 0; j < R.n; ++j)
        r += sqrt((double)R.j[j].t[0] * R.j[j].t[0] + (double)R.j[j].t[1] * R.j[j].t[1] +
                  (double)R.j[j].t[2] * R.j[j].t[2]);
    double re = 0.0;
    for (int k = 0; k < R.m; ++k)
        re = fmax(re, sqrt((double)R.e[k].t[0] * R.e[k].t[0] + (double)R.e[k].t[1] * R.e[k].t[1] +
                           (double)R.e[k].t[2] * R.e[k].t[2]));
    return (float)(r + re);
}

}  // namespace
}  // namespace pk

using namespace pk;

extern "C" {

int pk_seeder_create(pk_ctx *ctx, int32_t robot_id, int32_t K, int32_t hidden, int32_t depth,
                     const float *init, int64_t init_count, int32_t *seeder_id)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_seeder_create: ctx is NULL");
    RobotEntry *rb = robot_of(ctx, robot_id);
    if (!rb) return fail(ctx, PK_ENOTFOUND, "pk_seeder_create: unknown robot %d", robot_id);
    if (!seeder_id) return fail(ctx, PK_EINVAL, "pk_seeder_create: seeder_id is NULL");
    const RobotC &R = rb->host;
    if (R.m != 1 || R.e[0].kind != PK_EE_POSE)
        return fail(ctx, PK_EUNSUPPORTED, "pk_seeder_create: needs a robot with one pose EE");
    if (K < 1 || depth < 1 || depth > 8 || hidden < 128 || hidden % 128)
        return fail(ctx, PK_EINVAL, "pk_seeder_create: bad K=%d hidden=%d depth=%d", K, hidden, depth);
    if (R.n_mimic)
        return fail(ctx, PK_EUNSUPPORTED, "pk_seeder_create: robots with mimic joints are not supported");
    if (R.n * K > 64)
        return fail(ctx, PK_EUNSUPPORTED, "pk_seeder_create: K * n = %d above 64 outputs", R.n * K);
    SeederState *s = new SeederState;
    s->robot_id = robot_id;
    s->n = R.n;
    s->K = K;
    s->H = hidden;
    s->depth = depth;
    s->in_pad = 32;
    s->out_real = R.n * K;
    s->out_pad = 64;   // n*K <= 64 outputs, padded to the GEMM tile's 64 rows
    s->reach = tree_reach(R);
    int64_t off = 0;
    for (int l = 0; l <= depth; ++l) {
        const int in = l == 0 ? s->in_pad : hidden, out = l == depth ? s->out_pad : hidden;
        s->lin.push_back(in);
        s->lout.push_back(out);
        s->woff.push_back(off);
        off += (int64_t)in * out;
        s->boff.push_back(off);
        off += out;
    }
    s->nparam = off;
    // Unpadded parameter count in the caller's layout: W0 [H][n_in=7] b0, ..., W_L [7K][H] b_L.
    int64_t want = 0;
    for (int l = 0; l <= depth; ++l) {
        const int in = l == 0 ? 7 : hidden, out = l == depth ? s->out_real : hidden;
        want += (int64_t)in * out + out;
    }
    if (init && init_count != want) {
        seeder_free(s);
        return fail(ctx, PK_EINVAL, "pk_seeder_create: init has %lld values, expected %lld",
                    (long long)init_count, (long long)want);
    }
    PK_HIP(ctx, hipSetDevice(ctx->device));
    bool ok = hipMalloc(&s->P, off * 4) == hipSuccess && hipMalloc(&s->G, off * 4) == hipSuccess &&
              hipMalloc(&s->M, off * 4) == hipSuccess && hipMalloc(&s->V, off * 4) == hipSuccess &&
              hipMalloc(&s->Pb, off * 2) == hipSuccess && hipMalloc(&s->dstep, 4) == hipSuccess;
    int64_t wfn = 0;
    for (int l = 0; l <= depth; ++l) {
        s->wfoff.push_back(wfn);
        wfn += (int64_t)s->lin[l] * s->lout[l];
    }
    ok = ok && hipMalloc(&s->Wf, wfn * 2) == hipSuccess;
    if (!ok) {
        seeder_free(s);
        return fail(ctx, PK_ENOMEM, "pk_seeder_create: allocation failed");
    }
    std::vector<float> host(off, 0.f);
    if (init) {
        const float *src = init;
        for (int l = 0; l <= depth; ++l) {
            const int in = l == 0 ? 7 : hidden, out = l == depth ? s->out_real : hidden;
            for (int o = 0; o < out; ++o)
                for (int i = 0; i < in; ++i) host[s->woff[l] + (int64_t)o * s->lin[l] + i] = *src++;
            for (int o = 0; o < out; ++o) host[s->boff[l] + o] = *src++;
        }
    }
    std::vector<float> zeros(off, 0.f);
    int zero = 0;
    PK_HIP(ctx, hipMemcpy(s->P, host.data(), off * 4, hipMemcpyHostToDevice));
    PK_HIP(ctx, hipMemcpy(s->M, zeros.data(), off * 4, hipMemcpyHostToDevice));
    PK_HIP(ctx, hipMemcpy(s->V, zeros.data(), off * 4, hipMemcpyHostToDevice));
    PK_HIP(ctx, hipMemcpy(s->G, zeros.data(), off * 4, hipMemcpyHostToDevice));
    PK_HIP(ctx, hipMemcpy(s->dstep, &zero, 4, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(sd::to_bf16_kernel, dim3(sd::blocks(off, 256)), dim3(256), 0, 0, off, s->P, s->Pb);
    PK_HIP(ctx, hipDeviceSynchronize());
    ctx->seeders.push_back(s);
    *seeder_id = (int32_t)ctx->seeders.size() - 1;
    return PK_OK;
}

int pk_seeder_param_count(pk_ctx *ctx, int32_t id, int64_t *count)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_seeder_param_count: ctx is NULL");
    SeederState *s = seeder_of(ctx, id);
    if (!s || !count) return fail(ctx, PK_ENOTFOUND, "pk_seeder_param_count: unknown seeder %d", id);
    int64_t want = 0;
    for (int l = 0; l <= s->depth; ++l) {
        const int in = l == 0 ? 7 : s->H, out = l == s->depth ? s->out_real : s->H;
        want += (int64_t)in * out + out;
    }
    *count = want;
    return PK_OK;
}

// which: 0 = parameters, 1 = last gradients, 2 = Adam first moments, 3 = second moments.
int pk_seeder_get(pk_ctx *ctx, int32_t id, int32_t which, float *host_out, int64_t count)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_seeder_get: ctx is NULL");
    SeederState *s = seeder_of(ctx, id);
    if (!s) return fail(ctx, PK_ENOTFOUND, "pk_seeder_get: unknown seeder %d", id);
    int64_t want;
    pk_seeder_param_count(ctx, id, &want);
    if (!host_out || count != want || which < 0 || which > 3)
        return fail(ctx, PK_EINVAL, "pk_seeder_get: bad buffer (%lld values, expected %lld)",
                    (long long)count, (long long)want);
    const float *src = which == 0 ? s->P : which == 1 ? s->G : which == 2 ? s->M : s->V;
    std::vector<float> host(s->nparam);
    PK_HIP(ctx, hipSetDevice(ctx->device));
    PK_HIP(ctx, hipDeviceSynchronize());
    PK_HIP(ctx, hipMemcpy(host.data(), src, s->nparam * 4, hipMemcpyDeviceToHost));
    float *dst = host_out;
    for (int l = 0; l <= s->depth; ++l) {
        const int in = l == 0 ? 7 : s->H, out = l == s->depth ? s->out_real : s->H;
        for (int o = 0; o < out; ++o)
            for (int i = 0; i < in; ++i) *dst++ = host[s->woff[l] + (int64_t)o * s->lin[l] + i];
        for (int o = 0; o < out; ++o) *dst++ = host[s->boff[l] + o];
    }
    return PK_OK;
}

}  // extern "C"

namespace pk {
namespace {

// Loss + gradients for `rows` rows already in X0 / Q; loss_out (device) gets
// the mean loss.  `B` is the number of real rows (the loss averages over B).
// Loss (into loss_log[step - step0] for steps within [step0, step0 + nlog),
// and/or *loss_out) and parameter gradients of rows rows (B of them valid).
hipError_t loss_and_grads(SeederState *s, int64_t rows, int64_t B, float *loss_log, int step0, int nlog,
                          float *loss_out, hipStream_t st)
{
    using namespace sd;
    hipError_t e = forward(s, rows, true, st);
    if (e != hipSuccess) return e;
    const unsigned nb = blocks(rows, 16);
    hipLaunchKernelGGL(loss_kernel, dim3(nb), dim3(256), 0, st, (int)rows, (int)B, s->n, s->K, s->out_pad,
                       s->Y, s->Q, s->dY, s->dYb, s->part);
    hipLaunchKernelGGL(loss_finish_kernel, dim3(1), dim3(256), 0, st, (int)nb, (int)B, s->part, s->dstep,
                       step0, nlog, loss_log, loss_out);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return backward(s, rows, st);
}

}  // namespace

int seeder_infer_into(pk_ctx *ctx, int32_t id, const float *targets, int64_t T, float *seeds,
                      hipStream_t st, int32_t *K_out, int32_t *robot_out)
{
    SeederState *s = seeder_of(ctx, id);
    if (!s) return fail(ctx, PK_ENOTFOUND, "seeder: unknown seeder %d", id);
    if (K_out) *K_out = s->K;
    if (robot_out) *robot_out = s->robot_id;
    if (T < 0 || (T > 0 && (!targets || !seeds))) return fail(ctx, PK_EINVAL, "seeder inference: bad arguments");
    if (T == 0) return PK_OK;
    const int64_t rows = (T + 127) / 128 * 128;
    PK_HIP(ctx, hipSetDevice(ctx->device));
    int rc = alloc_acts(ctx, s, rows);
    if (rc) return rc;
    RobotEntry *rb = robot_of(ctx, s->robot_id);
    hipLaunchKernelGGL(sd::encode_kernel, dim3(sd::blocks(rows, 256)), dim3(256), 0, st, rows, T, targets, T,
                       1.f / s->reach, s->in_pad, s->X0, (float *)nullptr);
    PK_HIP(ctx, hipGetLastError());
    PK_HIP(ctx, forward_infer(s, rows, st));
    hipLaunchKernelGGL(sd::seeds_kernel, dim3(sd::blocks(T * s->K, 256)), dim3(256), 0, st, T, s->K, s->n, s->out_pad,
                       s->Y, rb->dev, seeds);
    PK_HIP(ctx, hipGetLastError());
    return PK_OK;
}

}  // namespace pk

extern "C" {

// x [B][7] (device) -> y [B][7K] (device), fused or layer by layer.
static int seeder_forward(pk_ctx *ctx, int32_t id, const float *x, int64_t B, float *y, hipStream_t st,
                   bool layers, const char *who)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "%s: ctx is NULL", who);
    SeederState *s = seeder_of(ctx, id);
    if (!s) return fail(ctx, PK_ENOTFOUND, "%s: unknown seeder %d", who, id);
    if (B < 0 || (B > 0 && (!x || !y))) return fail(ctx, PK_EINVAL, "%s: bad arguments", who);
    if (B == 0) return PK_OK;
    const int64_t rows = (B + 127) / 128 * 128;
    PK_HIP(ctx, hipSetDevice(ctx->device));
    int rc = alloc_acts(ctx, s, rows);
    if (rc) return rc;
    hipLaunchKernelGGL(sd::load_rows_kernel, dim3(sd::blocks(rows, 256)), dim3(256), 0, st, rows, B,
                       s->in_pad, s->n, x, nullptr, s->X0, nullptr);
    PK_HIP(ctx, hipGetLastError());
    PK_HIP(ctx, layers ? forward(s, rows, false, st) : forward_infer(s, rows, st));
    hipLaunchKernelGGL(sd::store_out_kernel, dim3(sd::blocks(B, 256)), dim3(256), 0, st, B, s->out_real,
                       s->out_pad, s->Y, y);
    PK_HIP(ctx, hipGetLastError());
    return PK_OK;
}

// Raw network output for encoded inputs x [B][7] (device) -> y [B][7K] (device).
int pk_seeder_forward(pk_ctx *ctx, int32_t id, const float *x, int64_t B, float *y, void *stream)
{
    return seeder_forward(ctx, id, x, B, y, (hipStream_t)stream, false, "pk_seeder_forward");
}

// The same through the layer-by-layer GEMMs.
int pk_seeder_forward_layers(pk_ctx *ctx, int32_t id, const float *x, int64_t B, float *y, void *stream)
{
    return seeder_forward(ctx, id, x, B, y, (hipStream_t)stream, true, "pk_seeder_forward_layers");
}

// Loss and parameter gradients for one batch x [B][7], q [B][n] (device);
// B a multiple of 128.  The gradients stay in the seeder (pk_seeder_get(..., 1, ...)).
int pk_seeder_grad(pk_ctx *ctx, int32_t id, const float *x, const float *q, int64_t B, float *loss,
                   void *stream)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_seeder_grad: ctx is NULL");
    SeederState *s = seeder_of(ctx, id);
    if (!s) return fail(ctx, PK_ENOTFOUND, "pk_seeder_grad: unknown seeder %d", id);
    if (B <= 0 || B % 128 || !x || !q) return fail(ctx, PK_EINVAL, "pk_seeder_grad: B must be a positive multiple of 128");
    hipStream_t st = (hipStream_t)stream;
    PK_HIP(ctx, hipSetDevice(ctx->device));
    int rc = alloc_acts(ctx, s, B);
    if (rc) return rc;
    hipLaunchKernelGGL(sd::load_rows_kernel, dim3(sd::blocks(B, 256)), dim3(256), 0, st, B, B, s->in_pad,
                       s->n, x, q, s->X0, s->Q);
    PK_HIP(ctx, hipGetLastError());
    PK_HIP(ctx, loss_and_grads(s, B, B, nullptr, 0, 0, loss, st));
    return PK_OK;
}

// Train on q_train [n][S] (device): targets are FK(q) computed here; per
// epoch the samples are visited in the order perm[e][0..S) (device, int32,
// epochs x S) or in index order when perm is NULL; S / batch steps per epoch.
// loss_log (device, optional) receives one mean loss per step.
int pk_seeder_train(pk_ctx *ctx, int32_t id, const float *q_train, int64_t S, int32_t batch,
                    int32_t epochs, float lr, const int32_t *perm, float *loss_log, void *stream)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_seeder_train: ctx is NULL");
    SeederState *s = seeder_of(ctx, id);
    if (!s) return fail(ctx, PK_ENOTFOUND, "pk_seeder_train: unknown seeder %d", id);
    if (!q_train || S < batch || batch <= 0 || batch % 128 || epochs < 0 || !(lr > 0.f))
        return fail(ctx, PK_EINVAL, "pk_seeder_train: bad arguments (S=%lld batch=%d epochs=%d)",
                    (long long)S, batch, epochs);
    if (S > INT32_MAX) return fail(ctx, PK_EUNSUPPORTED, "pk_seeder_train: S above 2^31");
    hipStream_t st = (hipStream_t)stream;
    RobotEntry *rb = robot_of(ctx, s->robot_id);
    PK_HIP(ctx, hipSetDevice(ctx->device));
    int rc = alloc_acts(ctx, s, batch);
    if (rc) return rc;
    // Inputs of every training sample: FK pose, encoded once.
    float *pose = nullptr, *xall = nullptr;
    if (hipMalloc(&pose, (size_t)S * 7 * 4) != hipSuccess || hipMalloc(&xall, (size_t)S * 7 * 4) != hipSuccess) {
        if (pose) (void)hipFree(pose);
        return fail(ctx, PK_ENOMEM, "pk_seeder_train: input buffers");
    }
    hipError_t e = launch_fk(rb->dev, S, q_train, pose, nullptr, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(sd::encode_kernel, dim3(sd::blocks(S, 256)), dim3(256), 0, st, S, S, pose, S,
                           1.f / s->reach, s->in_pad, (__bf16 *)nullptr, xall);
        e = hipGetLastError();
    }
    const int spe = (int)(S / batch);
    const int steps = spe * epochs;
    for (int t = 0; t < steps && e == hipSuccess; ++t) {
        hipLaunchKernelGGL(sd::gather_kernel, dim3(sd::blocks(batch, 256)), dim3(256), 0, st, batch, S, s->n,
                           s->in_pad, spe, steps, s->host_step, s->dstep, perm, xall, q_train, s->X0, s->Q);
        e = loss_and_grads(s, batch, batch, loss_log, s->host_step, steps, nullptr, st);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(sd::adam_kernel, dim3(sd::blocks(s->nparam, 256)), dim3(256), 0, st, s->nparam, lr,
                           0.9f, 0.999f, 1e-8f, s->dstep, s->P, s->G, s->M, s->V, s->Pb);
        hipLaunchKernelGGL(sd::tick_kernel, dim3(1), dim3(1), 0, st, s->dstep);
        e = hipGetLastError();
    }
    hipError_t e2 = hipStreamSynchronize(st);
    s->wf_dirty = true;
    (void)hipFree(pose);
    (void)hipFree(xall);
    if (e != hipSuccess) return fail(ctx, PK_EHIP, "pk_seeder_train: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(ctx, PK_EHIP, "pk_seeder_train: %s", hipGetErrorString(e2));
    // the next call's local steps count from the device counter
    PK_HIP(ctx, hipMemcpy(&s->host_step, s->dstep, sizeof(int), hipMemcpyDeviceToHost));
    return PK_OK;
}

// K seeds per target: targets planes [7][T] (device, pose EE layout) ->
// seeds [n][T*K] (device), clamped to the joint limits.
int pk_seeder_infer(pk_ctx *ctx, int32_t id, const float *targets, int64_t T, float *seeds, void *stream)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_seeder_infer: ctx is NULL");
    return seeder_infer_into(ctx, id, targets, T, seeds, (hipStream_t)stream, nullptr, nullptr);
}

// Versioned binary checkpoint: magic, dims, step, then parameters and the two
// Adam moments (FP32, padded layout).  Synchronous.
int pk_seeder_save(pk_ctx *ctx, int32_t id, const char *path)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_seeder_save: ctx is NULL");
    SeederState *s = seeder_of(ctx, id);
    if (!s || !path) return fail(ctx, PK_EINVAL, "pk_seeder_save: bad arguments");
    PK_HIP(ctx, hipSetDevice(ctx->device));
    PK_HIP(ctx, hipDeviceSynchronize());
    std::vector<float> buf(3 * s->nparam);
    PK_HIP(ctx, hipMemcpy(buf.data(), s->P, s->nparam * 4, hipMemcpyDeviceToHost));
    PK_HIP(ctx, hipMemcpy(buf.data() + s->nparam, s->M, s->nparam * 4, hipMemcpyDeviceToHost));
    PK_HIP(ctx, hipMemcpy(buf.data() + 2 * s->nparam, s->V, s->nparam * 4, hipMemcpyDeviceToHost));
    int step = 0;
    PK_HIP(ctx, hipMemcpy(&step, s->dstep, 4, hipMemcpyDeviceToHost));
    FILE *f = fopen(path, "wb");
    if (!f) return fail(ctx, PK_EINVAL, "pk_seeder_save: cannot open %s", path);
    const int32_t hdr[8] = {0x44534b50 /* "PKSD" */, 1, s->n, s->K, s->H, s->depth, step, 0};
    const int64_t np = s->nparam;
    bool ok = fwrite(hdr, sizeof hdr, 1, f) == 1 && fwrite(&np, 8, 1, f) == 1 &&
              fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    ok &= fclose(f) == 0;
    return ok ? PK_OK : fail(ctx, PK_EINVAL, "pk_seeder_save: write to %s failed", path);
}

int pk_seeder_load(pk_ctx *ctx, int32_t id, const char *path)
{
    if (!ctx) return fail(nullptr, PK_EINVAL, "pk_seeder_load: ctx is NULL");
    SeederState *s = seeder_of(ctx, id);
    if (!s || !path) return fail(ctx, PK_EINVAL, "pk_seeder_load: bad arguments");
    FILE *f = fopen(path, "rb");
    if (!f) return fail(ctx, PK_EINVAL, "pk_seeder_load: cannot open %s", path);
    int32_t hdr[8];
    int64_t np = 0;
    bool ok = fread(hdr, sizeof hdr, 1, f) == 1 && fread(&np, 8, 1, f) == 1;
    if (!ok || hdr[0] != 0x44534b50 || hdr[1] != 1 || hdr[2] != s->n || hdr[3] != s->K || hdr[4] != s->H ||
        hdr[5] != s->depth || np != s->nparam) {
        fclose(f);
        return fail(ctx, PK_EINVAL, "pk_seeder_load: %s does not match this seeder", path);
    }
    std::vector<float> buf(3 * np);
    ok = fread(buf.data(), 4, buf.size(), f) == buf.size();
    fclose(f);
    if (!ok) return fail(ctx, PK_EINVAL, "pk_seeder_load: %s is truncated", path);
    PK_HIP(ctx, hipSetDevice(ctx->device));
    PK_HIP(ctx, hipMemcpy(s->P, buf.data(), np * 4, hipMemcpyHostToDevice));
    PK_HIP(ctx, hipMemcpy(s->M, buf.data() + np, np * 4, hipMemcpyHostToDevice));
    PK_HIP(ctx, hipMemcpy(s->V, buf.data() + 2 * np, np * 4, hipMemcpyHostToDevice));
    PK_HIP(ctx, hipMemcpy(s->dstep, &hdr[6], 4, hipMemcpyHostToDevice));
    s->host_step = hdr[6];
    s->wf_dirty = true;
    hipLaunchKernelGGL(sd::to_bf16_kernel, dim3(sd::blocks(np, 256)), dim3(256), 0, 0, np, s->P, s->Pb);
    PK_HIP(ctx, hipGetLastError());
    PK_HIP(ctx, hipDeviceSynchronize());
    return PK_OK;
}

}  // extern "C"
