// Fused inference pass of the learned seeder: every layer of the MLP for a
// block of 64 rows in one kernel, the hidden activations kept in LDS.
//
// Each layer is the same BF16 MFMA product with FP32 accumulation, bias and
// SiLU as the layer-by-layer GEMMs, with the reduction over K taken in the
// same order, so both passes give the same values.  Per layer, a 256-thread
// block (4 waves) computes a 64 x N tile: a wave owns the 64 rows and N/4
// columns.  Two blocks share a CU, so one block's epilogue (bias, SiLU)
// overlaps the other's MFMAs.  A fragments come from the LDS activation tile (layer 0: from the
// input rows in global memory); B fragments come from a copy of the weights
// kept in MFMA fragment order, one contiguous 1 KB load per 16 x 32 block.
// Only the network input and output touch HBM.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sd_gemm.hpp"

namespace pk {
namespace sd {

constexpr int MLP_MAX_LAYERS = 9;   // depth <= 8 hidden layers + output

struct MlpArgs {
    int depth, out_pad;
    const __bf16 *wf[MLP_MAX_LAYERS];   // fragment-order weights per layer
    const float *bias[MLP_MAX_LAYERS];
};

// Output column of row c of B block nb.  Hidden layers pair the blocks
// (`pair`): blocks 2p, 2p+1 cover columns 32p .. 32p+31 so that lane group g
// of the MFMA result holds the 8 contiguous columns 32p + 8g .. 32p + 8g + 7.
PK_DEV int frag_col(int nb, int c, bool pair)
{
    return pair ? 32 * (nb >> 1) + 8 * (c >> 2) + 4 * (nb & 1) + (c & 3) : 16 * nb + c;
}

// W [N][ldw] (bf16, K used) -> Wf: block (nb, kb) at ((nb * K/32) + kb) * 512,
// lane l = (c = l % 16, g = l / 16) holding W[frag_col(nb, c)][32 kb + 8 g ..].
__global__ void frag_layout_kernel(int N, int K, int ldw, const __bf16 *__restrict__ W, int pair,
                                   __bf16 *__restrict__ Wf)
{
    const int KB = K / 32;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // one 16-byte piece
    if (p >= (int64_t)(N / 16) * KB * 64) return;
    const int l = (int)(p % 64);
    const int64_t blk = p / 64;
    const int kb = (int)(blk % KB), nb = (int)(blk / KB);
    const int col = frag_col(nb, l & 15, pair != 0);
    *(uint4 *)&Wf[p * 8] = *(const uint4 *)&W[(size_t)col * ldw + 32 * kb + 8 * (l >> 4)];
}

// acc[i][j] += A(rows of i) x B(block wn * NT + j) over KB steps of 32.
// A fragments: ld_a(i, kb).  B block j of the next step is fetched as soon as
// the MFMAs of this step that read it have issued, so each load has most of
// a step to arrive without a second set of registers.
template <int NT, class LoadA>
PK_DEV void mlp_kloop(f32x4 (&acc)[4][NT], const __bf16 *__restrict__ wf, int KB, int wn, int lane,
                      LoadA ld_a)
{
    const __bf16 *wb = wf + (size_t)wn * NT * KB * 512 + lane * 8;
    bf16x8 b[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) b[j] = *(const bf16x8 *)&wb[(size_t)j * KB * 512];
#pragma unroll 1
    for (int kb = 0; kb < KB; ++kb) {
        // The last step refetches its own blocks: the loads stay
        // unconditional, so every wait counts exactly the 8 in flight.
        const int kn = kb + 1 < KB ? kb + 1 : kb;
        bf16x8 a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = ld_a(i, kb);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j], a[i], acc[i][j], 0, 0, 0);
            b[j] = *(const bf16x8 *)&wb[((size_t)j * KB + kn) * 512];
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// JT = hidden width / 64 (B blocks per wave in a hidden layer), NO = output
// width / 64.  Grid: rows / 64 blocks of 256 threads; X0 [rows][32], Y
// [rows][out_pad].
template <int JT, int NO>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(JT >= 8 ? 2 : 4))) void mlp_infer_kernel(MlpArgs args, const __bf16 *__restrict__ X0,
                                                        float *__restrict__ Y)
{
    constexpr int H = 64 * JT;
    // Activation tile [64][H]; the 16-byte chunk ch of row R sits at chunk
    // ch ^ (R % 16), so a fragment read (16 rows, one chunk) hits 16 banks.
    __shared__ __attribute__((aligned(16))) __bf16 act[64 * H];
    const int tid = threadIdx.x, wn = tid >> 6, lane = tid & 63;
    const int r16 = lane & 15, g = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.x * 64;
    auto row = [&](int i) { return 16 * i + r16; };
    auto act_at = [&](int R, int ch) { return &act[R * H + 8 * (ch ^ (R & 15))]; };

    f32x4 acc[4][JT];
    // Hidden-layer epilogue: z = acc + b, h = bf16(SiLU(z)) into the tile.
    auto to_act = [&](const float *b) {
#pragma unroll
        for (int p = 0; p < JT / 2; ++p) {
            const f32x4 cv[2] = {*(const f32x4 *)&b[frag_col(wn * JT + 2 * p, 4 * g, true)],
                                 *(const f32x4 *)&b[frag_col(wn * JT + 2 * p + 1, 4 * g, true)]};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const f32x4 z0 = acc[i][2 * p] + cv[0], z1 = acc[i][2 * p + 1] + cv[1];
                const bf16x8 h = {(__bf16)silu(z0[0]), (__bf16)silu(z0[1]), (__bf16)silu(z0[2]),
                                  (__bf16)silu(z0[3]), (__bf16)silu(z1[0]), (__bf16)silu(z1[1]),
                                  (__bf16)silu(z1[2]), (__bf16)silu(z1[3])};
                *(bf16x8 *)act_at(row(i), 4 * (wn * JT / 2 + p) + g) = h;
            }
        }
    };
    auto zero = [&]() {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < JT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    };

    // layer 0: K = 32 from the input rows
    zero();
    mlp_kloop<JT>(acc, args.wf[0], 1, wn, lane, [&](int i, int) {
        return *(const bf16x8 *)&X0[(m0 + row(i)) * 32 + 8 * g];
    });
    to_act(args.bias[0]);
    __syncthreads();
    auto from_act = [&](int i, int kb) { return *(const bf16x8 *)act_at(row(i), 4 * kb + g); };
    for (int l = 1; l < args.depth; ++l) {
        zero();
        mlp_kloop<JT>(acc, args.wf[l], H / 32, wn, lane, from_act);
        __syncthreads();   // every wave has read the layer input
        to_act(args.bias[l]);
        __syncthreads();
    }
    // output layer: y = acc + b (FP32)
    f32x4 ao[4][NO], co[NO];
    const float *bo = args.bias[args.depth];
#pragma unroll
    for (int j = 0; j < NO; ++j) co[j] = *(const f32x4 *)&bo[frag_col(wn * NO + j, 4 * g, false)];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NO; ++j) ao[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    mlp_kloop<NO>(ao, args.wf[args.depth], H / 32, wn, lane, from_act);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NO; ++j)
            *(f32x4 *)&Y[(m0 + row(i)) * args.out_pad + frag_col(wn * NO + j, 4 * g, false)] = ao[i][j] + co[j];
}

}  // namespace sd
}  // namespace pk
