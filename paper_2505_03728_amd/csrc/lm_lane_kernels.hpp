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

// One 64-problem item per block; no state kept between launches.
// TEXIT: the instantiation for target_exit (separate kernels, so that the
// others' loops carry no trace of it).
template <int C, int L, int KIND, bool TEXIT>
__global__ __launch_bounds__(BLOCK) void lm_lane_kernel(const RobotC *__restrict__ rb,
                                                        const float *__restrict__ qr, SolveParams P)
{
    using SL = Slots<C, L, KIND>;
    __shared__ float smem[SL::TOTAL * BLOCK];
    const LaneLds S{smem + threadIdx.x};
    const int64_t nact = P.n_active ? (int64_t)*P.n_active : P.N;
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < nact) lane_problem<C, L, KIND, false, TEXIT>(rb, qr, P, S, i);
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
hipError_t launch_star(const RobotC *rb, const SolveParams &P, int persist_blocks, hipStream_t s)
{
    const int block = BLOCK;
    int64_t grid = (P.N + block - 1) / block;
    const bool persist = P.queue_head != nullptr;
    if (persist && persist_blocks > 0 && persist_blocks < grid) grid = persist_blocks;
    // rest pose: caller's array, else the robot's mid-range table
    const float *qr = P.q_rest ? P.q_rest : rb->mid;
    const dim3 g((unsigned)grid), b(block);
    if (persist && P.target_exit)
        hipLaunchKernelGGL((lm_lane_persist_kernel<C, L, KIND, true>), g, b, 0, s, rb, qr, P);
    else if (persist)
        hipLaunchKernelGGL((lm_lane_persist_kernel<C, L, KIND, false>), g, b, 0, s, rb, qr, P);
    else if (P.target_exit)
        hipLaunchKernelGGL((lm_lane_kernel<C, L, KIND, true>), g, b, 0, s, rb, qr, P);
    else
        hipLaunchKernelGGL((lm_lane_kernel<C, L, KIND, false>), g, b, 0, s, rb, qr, P);
    return hipGetLastError();
}

}  // namespace lane

// Launchers of the single-chain instantiations (defined in lm_lane_chain*.hip):
// chain length L with a pose (kind PK_EE_POSE) or position EE.
hipError_t launch_lane_chain_a(int L, int kind, const RobotC *rb, const SolveParams &P, int pb, hipStream_t s);
hipError_t launch_lane_chain_b(int L, int kind, const RobotC *rb, const SolveParams &P, int pb, hipStream_t s);
hipError_t launch_lane_chain_c(int L, int kind, const RobotC *rb, const SolveParams &P, int pb, hipStream_t s);

}  // namespace pk
