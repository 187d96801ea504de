// BF16 matrix-core GEMMs of the learned seeder with fused epilogues.
//
// C[M,N] = A[M,K] B[K,N] with v_mfma_f32_16x16x32_bf16 and FP32
// accumulation; a 256-thread block (2x2 waves) computes a (32 WM) x (32 WN)
// tile.  Epilogues fuse bias, SiLU / SiLU', the BF16 down-conversion and the
// FP32 copies backward needs.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include <algorithm>
#include <type_traits>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace pk {
namespace sd {

#ifndef PK_DEV
#define PK_DEV __device__ __forceinline__
#endif

enum { A_MK = 0, A_KM = 1 };   // A(m,k) = A[m*lda + k]  or  A[k*lda + m]
enum { B_NK = 0, B_KN = 1 };   // B(k,n) = B[n*ldb + k]  or  B[k*ldb + n]

// z * sigmoid(z) with the hardware reciprocal (1 ulp) in place of a division.
PK_DEV float silu(float z) { return z * __builtin_amdgcn_rcpf(1.f + __expf(-z)); }
PK_DEV float silu_grad(float z)
{
    const float s = 1.f / (1.f + __expf(-z));
    return s * (1.f + z * (1.f - s));
}

// Epilogues receive four consecutive output columns n..n+3 of row m.  Their
// inputs are fetched apart from the stores so that a tile's loads are all in
// flight together: col(n) (per column, fetched before the K loop) and
// elem(m, n) (per element, fetched for the whole tile before any store).
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

struct EpiStore {           // C[z] = acc (FP32); z = split-K slice, slices `zstride` apart
    float *C;
    int ld;
    size_t zstride;
    PK_DEV f32x4 col(int) const { return f32x4{0.f, 0.f, 0.f, 0.f}; }
    PK_DEV f32x4 elem(int, int) const { return f32x4{0.f, 0.f, 0.f, 0.f}; }
    PK_DEV void operator()(int m, int n, int z, f32x4 v, f32x4, f32x4) const
    {
        *(f32x4 *)&C[z * zstride + (size_t)m * ld + n] = v;
    }
};
struct EpiHidden {          // z = acc + b; Z = z; H = bf16(SiLU(z))
    const float *bias;
    float *Z;
    __bf16 *H;
    int ld;
    PK_DEV f32x4 col(int n) const { return *(const f32x4 *)&bias[n]; }
    PK_DEV f32x4 elem(int, int) const { return f32x4{0.f, 0.f, 0.f, 0.f}; }
    PK_DEV void operator()(int m, int n, int, f32x4 v, f32x4 b, f32x4) const
    {
        const f32x4 z = v + b;
        const size_t i = (size_t)m * ld + n;
        if (Z) *(f32x4 *)&Z[i] = z;
        const bf16x4 h = {(__bf16)silu(z[0]), (__bf16)silu(z[1]), (__bf16)silu(z[2]), (__bf16)silu(z[3])};
        *(bf16x4 *)&H[i] = h;
    }
};
struct EpiOut {             // y = acc + b
    const float *bias;
    float *Y;
    int ld;
    PK_DEV f32x4 col(int n) const { return *(const f32x4 *)&bias[n]; }
    PK_DEV f32x4 elem(int, int) const { return f32x4{0.f, 0.f, 0.f, 0.f}; }
    PK_DEV void operator()(int m, int n, int, f32x4 v, f32x4 b, f32x4) const
    {
        *(f32x4 *)&Y[(size_t)m * ld + n] = v + b;
    }
};
struct EpiBackHidden {      // dZ = acc * SiLU'(Z): FP32 and BF16 copies
    const float *Z;
    float *dZ;
    __bf16 *dZb;
    int ld;
    PK_DEV f32x4 col(int) const { return f32x4{0.f, 0.f, 0.f, 0.f}; }
    PK_DEV f32x4 elem(int m, int n) const { return *(const f32x4 *)&Z[(size_t)m * ld + n]; }
    PK_DEV void operator()(int m, int n, int, f32x4 v, f32x4, f32x4 z) const
    {
        const size_t i = (size_t)m * ld + n;
        const f32x4 g = {v[0] * silu_grad(z[0]), v[1] * silu_grad(z[1]), v[2] * silu_grad(z[2]),
                         v[3] * silu_grad(z[3])};
        *(f32x4 *)&dZ[i] = g;
        const bf16x4 gb = {(__bf16)g[0], (__bf16)g[1], (__bf16)g[2], (__bf16)g[3]};
        *(bf16x4 *)&dZb[i] = gb;
    }
};

// Runs the epilogue over a wave's (16 WM) x (16 WN) accumulator tile.
template <int WM, int WN, class Epi>
PK_DEV void epilogue(const Epi &epi, const f32x4 (&acc)[WM][WN], const f32x4 (&cv)[WN], int mb, int nb,
                     int lane, int z)
{
    f32x4 ev[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) ev[i][j] = epi.elem(mb + 16 * i + (lane & 15), nb + 16 * j + 4 * (lane >> 4));
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
            epi(mb + 16 * i + (lane & 15), nb + 16 * j + 4 * (lane >> 4), z, acc[i][j], cv[j], ev[i][j]);
}

// Element e of R row vectors, packed along k: R consecutive bf16 in one store.
// (The vectors are reinterpreted whole as 16-bit integers and then indexed.)
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
template <int R>
PK_DEV void store_kpack(__bf16 *dst, const bf16x8 (&v)[R], int e)
{
    u16x8 w[R];
#pragma unroll
    for (int i = 0; i < R; ++i) w[i] = __builtin_bit_cast(u16x8, v[i]);
    if constexpr (R == 4) {
        *(uint2 *)dst = make_uint2((unsigned)w[0][e] | ((unsigned)w[1][e] << 16),
                                   (unsigned)w[2][e] | ((unsigned)w[3][e] << 16));
    } else if constexpr (R == 2) {
        *(unsigned *)dst = (unsigned)w[0][e] | ((unsigned)w[1][e] << 16);
    } else {
        unsigned short *d = (unsigned short *)dst;
#pragma unroll
        for (int i = 0; i < R; ++i) d[i] = w[i][e];
    }
}

// blockIdx.z selects one of gridDim.z equal slices of K (split-K); the
// epilogue receives the slice index so partial products can be kept apart.
// The next K stage is fetched from global memory into registers while the
// current stage, staged in LDS with the reduction dimension contiguous, feeds
// the MFMAs.
template <int AL, int BL, int WM, int WN, int BK, class Epi>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, const __bf16 *__restrict__ A,
                                                   int lda, const __bf16 *__restrict__ B, int ldb,
                                                   Epi epi)
{
    constexpr int BM = 32 * WM, BN = 32 * WN, LDK = BK + 8;
    constexpr int NVA = BM * BK / 8, NVB = BN * BK / 8;             // 8-element vectors per stage
    constexpr int RA = (NVA + 255) / 256, RB = (NVB + 255) / 256;   // per thread
    __shared__ __attribute__((aligned(16))) __bf16 sA[BM * LDK];
    __shared__ __attribute__((aligned(16))) __bf16 sB[BN * LDK];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    // Workgroups are handed to the 8 XCDs in turn (linear id mod 8).  Give
    // each XCD a contiguous run of tiles instead, so the N tiles that share
    // an A row block run together behind one L2.
    const int nx = (int)gridDim.x, ntile = nx * (int)gridDim.y;
    int b = (int)blockIdx.x + nx * (int)blockIdx.y;
    if (ntile % 8 == 0) b = (b % 8) * (ntile / 8) + b / 8;
    const int m0 = (b / nx) * BM, n0 = (b % nx) * BN;
    f32x4 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    f32x4 cv[WN];
#pragma unroll
    for (int j = 0; j < WN; ++j) cv[j] = epi.col(n0 + wn * 16 * WN + 16 * j + 4 * (lane >> 4));

    bf16x8 ra[RA], rb[RB];
    // MK/NK layouts: vector v of a stage is (row v / (BK/8), k 8 * (v % (BK/8))).
    // KM/KN layouts: thread t owns R consecutive k rows (R = RA or RB) of the
    // 8-wide row group t % (rows/8), so its LDS writes pack R values per row.
    constexpr int GA = BM / 8, GB = BN / 8;
    const int amg = tid % GA, akq = tid / GA, bng = tid % GB, bkq = tid / GB;
    auto gload = [&](int k0) {
#pragma unroll
        for (int i = 0; i < RA; ++i) {
            if (AL == A_MK) {
                const int v = tid + 256 * i;
                if (v < NVA)
                    ra[i] = *(const bf16x8 *)&A[(size_t)(m0 + v / (BK / 8)) * lda + k0 + 8 * (v % (BK / 8))];
            } else {
                const int kk = akq * RA + i;
                if (kk < BK) ra[i] = *(const bf16x8 *)&A[(size_t)(k0 + kk) * lda + m0 + 8 * amg];
            }
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            if (BL == B_NK) {
                const int v = tid + 256 * i;
                if (v < NVB)
                    rb[i] = *(const bf16x8 *)&B[(size_t)(n0 + v / (BK / 8)) * ldb + k0 + 8 * (v % (BK / 8))];
            } else {
                const int kk = bkq * RB + i;
                if (kk < BK) rb[i] = *(const bf16x8 *)&B[(size_t)(k0 + kk) * ldb + n0 + 8 * bng];
            }
        }
    };
    auto lstore = [&]() {
        if (AL == A_MK) {
#pragma unroll
            for (int i = 0; i < RA; ++i) {
                const int v = tid + 256 * i;
                if (v < NVA) *(bf16x8 *)&sA[(v / (BK / 8)) * LDK + 8 * (v % (BK / 8))] = ra[i];
            }
        } else if (akq * RA < BK) {
#pragma unroll
            for (int e = 0; e < 8; ++e) store_kpack<RA>(&sA[(8 * amg + e) * LDK + akq * RA], ra, e);
        }
        if (BL == B_NK) {
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const int v = tid + 256 * i;
                if (v < NVB) *(bf16x8 *)&sB[(v / (BK / 8)) * LDK + 8 * (v % (BK / 8))] = rb[i];
            }
        } else if (bkq * RB < BK) {
#pragma unroll
            for (int e = 0; e < 8; ++e) store_kpack<RB>(&sB[(8 * bng + e) * LDK + bkq * RB], rb, e);
        }
    };

    const int kslice = K / (int)gridDim.z;
    const int kbeg = (int)blockIdx.z * kslice, kend = kbeg + kslice;
    gload(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        __syncthreads();
        lstore();
        __syncthreads();
        if (k0 + BK < kend) gload(k0 + BK);
        const int r16 = lane & 15;
#pragma unroll
        for (int ks = 0; ks < BK; ks += 32) {
            const int kq = ks + 8 * (lane >> 4);
            bf16x8 af[WM], bfr[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i) af[i] = *(const bf16x8 *)&sA[(wm * 16 * WM + 16 * i + r16) * LDK + kq];
#pragma unroll
            for (int j = 0; j < WN; ++j) bfr[j] = *(const bf16x8 *)&sB[(wn * 16 * WN + 16 * j + r16) * LDK + kq];
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[i][j], 0, 0, 0);
        }
    }
    // The B fragment is the MFMA's first operand, so the 16x16 result is the
    // transposed tile: lane l holds row l%16 and columns 4*(l/16)..+3.
    epilogue<WM, WN>(epi, acc, cv, m0 + wm * 16 * WM, n0 + wn * 16 * WN, lane, (int)blockIdx.z);
}

template <int AL, int BL, int WM, int WN, class Epi>
hipError_t gemm_tile(int M, int N, int K, const __bf16 *A, int lda, const __bf16 *B, int ldb, Epi epi,
                     hipStream_t s, int splits)
{
    dim3 grid(N / (32 * WN), M / (32 * WM), splits);
    if ((K / splits) % 64 == 0)
        hipLaunchKernelGGL((gemm_kernel<AL, BL, WM, WN, 64, Epi>), grid, dim3(256), 0, s, M, N, K, A, lda,
                           B, ldb, epi);
    else
        hipLaunchKernelGGL((gemm_kernel<AL, BL, WM, WN, 32, Epi>), grid, dim3(256), 0, s, M, N, K, A, lda,
                           B, ldb, epi);
    return hipGetLastError();
}

// Picks the tile for the shape (M % 64 == 0, N % 32 == 0, K % (32 * splits) == 0).
template <int AL, int BL, class Epi>
hipError_t gemm(int M, int N, int K, const __bf16 *A, int lda, const __bf16 *B, int ldb, Epi epi,
                hipStream_t s, int splits = 1)
{
    if (M % 64 || N % 32 || splits < 1 || K % (32 * splits)) return hipErrorInvalidValue;
    const bool m128 = M % 128 == 0;
    if (N % 128 == 0)
        return m128 ? gemm_tile<AL, BL, 4, 4>(M, N, K, A, lda, B, ldb, epi, s, splits)
                    : gemm_tile<AL, BL, 2, 4>(M, N, K, A, lda, B, ldb, epi, s, splits);
    if (N % 64 == 0)
        return m128 ? gemm_tile<AL, BL, 4, 2>(M, N, K, A, lda, B, ldb, epi, s, splits)
                    : gemm_tile<AL, BL, 2, 2>(M, N, K, A, lda, B, ldb, epi, s, splits);
    return m128 ? gemm_tile<AL, BL, 4, 1>(M, N, K, A, lda, B, ldb, epi, s, splits)
                : gemm_tile<AL, BL, 2, 1>(M, N, K, A, lda, B, ldb, epi, s, splits);
}

// Number of K slices so that an (M x N) output with a K-long reduction
// fills the device: about 256 workgroups, each slice at least 256 long.
inline int split_for(int M, int N, int K)
{
    const int tm = M % 128 == 0 ? 128 : 64, tn = N % 128 == 0 ? 128 : N % 64 == 0 ? 64 : 32;
    const int tiles = std::max(1, (M / tm) * (N / tn));
    int sp = 1;
    while (tiles * sp < 256 && K % (64 * sp) == 0 && K / (2 * sp) >= 256) sp *= 2;
    return sp;
}

// Largest split_for(M, N, K) over all K: the smallest power of two that
// brings the tile count to 256.
inline int split_max(int M, int N)
{
    const int tm = M % 128 == 0 ? 128 : 64, tn = N % 128 == 0 ? 128 : N % 64 == 0 ? 64 : 32;
    const int tiles = std::max(1, (M / tm) * (N / tn));
    int sp = 1;
    while (tiles * sp < 256) sp *= 2;
    return sp;
}

}  // namespace sd
}  // namespace pk
