// Kernels and launcher of the per-lane LM path (device code in lm_lane.hpp),
// instantiated per robot shape by the lm_lane*.hip units: one 64-problem
// block per launch item, or persistent blocks popping items from a device
// queue.
#pragma once

#include "lm_lane.hpp"

namespace pk {
namespace lane {

// Next work item of this block: the block index for a plain grid, else an
// atomic pop from the device queue (block = one wavefront).
PK_DEV int64_t pop_item(int32_t *head)
{
    int v = 0;
    if (threadIdx.x == 0) v = atomicAdd(head, 1);
    return (int64_t)__shfl(v, 0, 64);
}

// Best-of-K over the K problems of each target in this wavefront (K divides
// 64, problems in index order): the rule of best_of_k_pick (the lowest total
// cost among those that met the tolerance, else the lowest pose-only cost,
// ties to the lower index), taken in the same order on the values the
// problems ended with.  Every lane of the wavefront takes part.
template <int N>
PK_DEV void best_in_wave(const SolveParams &P, const LaneFinal<N> &f, int64_t i, const BestOut &B)
{
    const int K = P.K, lane = threadIdx.x & 63, gb = lane & ~(K - 1);
    int b = -1;
    bool any = false;
    float bv = 0.f;
    for (int k = 0; k < K; ++k) {
        const bool cv = __shfl((int)f.conv, gb + k, 64) != 0;
        const float c = __shfl(f.cost, gb + k, 64);
        if (cv && (!any || c < bv)) {
            b = k;
            bv = c;
        }
        any = any || cv;
    }
    if (!any)
        for (int k = 0; k < K; ++k) {
            const float c = __shfl(f.pcost, gb + k, 64);
            if (b < 0 || c < bv) {
                b = k;
                bv = c;
            }
        }
    if (i >= P.N) return;
    const int64_t t = i / K, T = P.T;
    if (B.joints && lane == gb + b)
#pragma unroll
        for (int j = 0; j < N; ++j) B.joints[(int64_t)j * T + t] = f.q[j];
    if (lane == gb) {
        if (B.index) B.index[t] = b;
        if (B.success) B.success[t] = any ? 1 : 0;
    }
}

// One 64-problem item per block; no state kept between launches.  With B's
// pointers set, the block's targets' best-of-K as well.
// TEXIT: the instantiation for target_exit (separate kernels, so that the
// others' loops carry no trace of it).
template <int C, int L, int KIND, bool TEXIT>
__global__ __launch_bounds__(BLOCK) void lm_lane_kernel(const RobotC *__restrict__ rb,
                                                        const float *__restrict__ qr, SolveParams P,
                                                        BestOut B)
{
    using SL = Slots<C, L, KIND>;
    __shared__ float smem[SL::TOTAL * BLOCK];
    const LaneLds S{smem + threadIdx.x};
    const int64_t nact = P.n_active ? (int64_t)*P.n_active : P.N;
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    LaneFinal<Star<C, L, KIND>::N> fin;
    fin.cost = fin.pcost = NAN;
    fin.conv = false;
    if (i < nact) lane_problem<C, L, KIND, false, TEXIT>(rb, qr, P, S, i, &fin);
    if (B.index || B.joints || B.success) best_in_wave(P, fin, i, B);
}

// Persistent variant: blocks pop 64-problem items from P.queue_head until
// the active list is exhausted; problem state is resumable.
template <int C, int L, int KIND, bool TEXIT>
PK_DEV void persist_loop(const RobotC *__restrict__ rb, const float *__restrict__ qr,
                         const SolveParams &P, float *smem)
{
    const LaneLds S{smem + threadIdx.x};
    const int64_t nact = P.n_active ? (int64_t)*P.n_active : P.N;
    const int64_t nitems = (nact + BLOCK - 1) / BLOCK;
    int64_t item = pop_item(P.queue_head);
    while (item < nitems) {
        const int64_t i = item * BLOCK + threadIdx.x;
        if (i < nact) lane_problem<C, L, KIND, true, TEXIT>(rb, qr, P, S, i);
        item = pop_item(P.queue_head);
    }
}

template <int C, int L, int KIND, bool TEXIT>
__global__ __launch_bounds__(BLOCK) void lm_lane_persist_kernel(const RobotC *__restrict__ rb,
                                                                const float *__restrict__ qr,
                                                                SolveParams P)
{
    __shared__ float smem[Slots<C, L, KIND>::TOTAL * BLOCK];
    persist_loop<C, L, KIND, TEXIT>(rb, qr, P, smem);
}

template <int C, int L, int KIND>
hipError_t launch_star(const RobotC *rb, const SolveParams &P, int persist_blocks, hipStream_t s,
                       const BestOut *best = nullptr)
{
    const int block = BLOCK;
    int64_t grid = (P.N + block - 1) / block;
    const bool persist = P.queue_head != nullptr;
    if (persist && persist_blocks > 0 && persist_blocks < grid) grid = persist_blocks;
    // rest pose: caller's array, else the robot's mid-range table
    const float *qr = P.q_rest ? P.q_rest : rb->mid;
    const dim3 g((unsigned)grid), b(block);
    if (best && (persist || P.active || P.n_active || 64 % P.K != 0)) return hipErrorInvalidValue;
    const BestOut B = best ? *best : BestOut{nullptr, nullptr, nullptr};
    if (persist && P.target_exit)
        hipLaunchKernelGGL((lm_lane_persist_kernel<C, L, KIND, true>), g, b, 0, s, rb, qr, P);
    else if (persist)
        hipLaunchKernelGGL((lm_lane_persist_kernel<C, L, KIND, false>), g, b, 0, s, rb, qr, P);
    else if (P.target_exit)
        hipLaunchKernelGGL((lm_lane_kernel<C, L, KIND, true>), g, b, 0, s, rb, qr, P, B);
    else
        hipLaunchKernelGGL((lm_lane_kernel<C, L, KIND, false>), g, b, 0, s, rb, qr, P, B);
    return hipGetLastError();
}

}  // namespace lane

// Launchers of the single-chain instantiations (defined in lm_lane_chain*.hip):
// chain length L with a pose (kind PK_EE_POSE) or position EE.
hipError_t launch_lane_chain_a(int L, int kind, const RobotC *rb, const SolveParams &P, int pb, hipStream_t s,
                               const BestOut *best);
hipError_t launch_lane_chain_b(int L, int kind, const RobotC *rb, const SolveParams &P, int pb, hipStream_t s,
                               const BestOut *best);
hipError_t launch_lane_chain_c(int L, int kind, const RobotC *rb, const SolveParams &P, int pb, hipStream_t s,
                               const BestOut *best);

}  // namespace pk
