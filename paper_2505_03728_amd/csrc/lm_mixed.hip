// Single persistent LM launch over a mixed batch: the wavefronts of one grid
// pop work items from one device queue; an item is (group, range of that
// group's active problems): 64 problems for a per-lane path, one for a
// per-wavefront path.  The wavefront branches (uniformly) to the device path
// of the item's group, which runs the problems for at most k more LM
// iterations with their state in HBM (resumable), so a problem's result does
// not depend on k, on the grid or on which wavefront takes it.
//
// Method: Sec. III-A (LM over the sum of squared weighted residuals) for each
// problem, as in the per-lane and per-wavefront kernels it instantiates.
#include "lm_lane.hpp"
#include "lm_path.hpp"
#include "lm_wave.hpp"
#include "sched_table.hpp"

namespace pk {
namespace {

constexpr int align4(int f) { return (f + 3) & ~3; }

// Work items per group for this round, the queue head reset, and the next
// round's list size cleared (the compaction after this round fills it).
__global__ void mixed_plan_kernel(MixedArgs a, int32_t *item_end, int32_t *head)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int cur = a.round & 1;
    int acc = 0;
    for (int g = 0; g < a.n_groups; ++g) {
        const MixedGroup &G = a.g[g];
        const int64_t cnt = a.round > 0 ? (int64_t)G.count[cur] : G.P.N;
        acc += (int)((cnt + G.per_item - 1) / G.per_item);
        item_end[g] = acc;
        G.count[cur ^ 1] = 0;
    }
    *head = 0;
}

// Unfinished problems of this round's list -> next round's list (one grid
// row per group).
__global__ void mixed_compact_kernel(MixedArgs a)
{
    const int g = blockIdx.y;
    if (g >= a.n_groups) return;
    const MixedGroup &G = a.g[g];
    const int cur = a.round & 1;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nc = a.round > 0 ? (int64_t)G.count[cur] : G.P.N;
    if (i >= nc) return;
    const int32_t p = a.round > 0 ? G.list[cur][i] : (int32_t)i;
    if (!(G.P.st_state[p] & PK_ST_DONE)) G.list[cur ^ 1][atomicAdd(&G.count[cur ^ 1], 1)] = p;
}

// Per-lane path: problems first*64 + lane of the group's active list.
template <int C, int L, int KIND>
PK_DEV void run_lane(const MixedGroup &G, float *ws, int64_t first, int lane)
{
    const SolveParams &P = G.P;
    const int64_t nact = P.n_active ? (int64_t)*P.n_active : P.N;
    const int64_t i = first * 64 + lane;
    if (i < nact) lane::lane_problem<C, L, KIND, true>(G.rb, G.qr, P, lane::LaneLds{ws + lane}, i);
}

// MixedArgs is the first kernel argument (offset 0 of the argument segment).
template <int WG>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(2))) void lm_mixed_kernel(
    const MixedArgs a, const int32_t *__restrict__ item_end, int32_t *head, int lds_floats)
{
    extern __shared__ __attribute__((aligned(16))) float smem[];
    const int lane = threadIdx.x & 63;
    float *ws = smem + (threadIdx.x >> 6) * lds_floats;
    const int ng = a.n_groups;
    const int total = item_end[ng - 1];
    for (;;) {
        int v = 0;
        if (lane == 0) v = atomicAdd(head, 1);
        const int item = __builtin_amdgcn_readfirstlane(__shfl(v, 0, 64));
        if (item >= total) break;
        int g = 0;
        while (g < ng - 1 && item >= item_end[g]) ++g;
        g = __builtin_amdgcn_readfirstlane(g);   // uniform: item is
        const MixedGroup &G = a.g[g];
        const int64_t first = item - (g > 0 ? item_end[g - 1] : 0);
        switch (G.path) {
        case MIX_LANE_ARM:
            run_lane<1, 7, PK_EE_POSE>(G, ws, first, lane);
            break;
        case MIX_LANE_HAND:
            run_lane<4, 4, PK_EE_POSITION>(G, ws, first, lane);
            break;
        case MIX_PATH_16_4:
            path::path_problem<16, 4>(
                G.rb, path::kernel_params_at(offsetof(MixedArgs, g) + g * sizeof(MixedGroup) + offsetof(MixedGroup, P)),
                ws, first);
            break;
        default:
            wave::wave_problem<16, 4>(G.rb, G.P, ws, first);
            break;
        }
        // the next item reuses this wavefront's LDS slice
        wave::wave_sync();
    }
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

int mixed_lds_floats(int path)
{
    switch (path) {
    case MIX_LANE_ARM: return align4(lane::Slots<1, 7, PK_EE_POSE>::TOTAL * lane::BLOCK);
    case MIX_LANE_HAND: return align4(lane::Slots<4, 4, PK_EE_POSITION>::TOTAL * lane::BLOCK);
    case MIX_WAVE_16_4: return align4(wave::Lds<16, 4>::FLOATS);
    case MIX_PATH_16_4: return align4(path::Lds<16, 4>::FLOATS);
    default: return 0;
    }
}

hipError_t launch_mixed_round(const MixedArgs &a, int32_t *item_end, int32_t *head, int max_n,
                              bool last, int waves, int wg, int lds_floats, hipStream_t s)
{
    hipLaunchKernelGGL(mixed_plan_kernel, dim3(1), dim3(64), 0, s, a, item_end, head);
    const int wpb = wg / 64;
    const unsigned blocks = nblk(waves, wpb);
    const size_t lds = (size_t)wpb * lds_floats * sizeof(float);
    switch (wg) {
    case 64:
        hipLaunchKernelGGL(lm_mixed_kernel<64>, dim3(blocks), dim3(64), lds, s, a, item_end, head, lds_floats);
        break;
    case 128:
        hipLaunchKernelGGL(lm_mixed_kernel<128>, dim3(blocks), dim3(128), lds, s, a, item_end, head, lds_floats);
        break;
    case 256:
        hipLaunchKernelGGL(lm_mixed_kernel<256>, dim3(blocks), dim3(256), lds, s, a, item_end, head, lds_floats);
        break;
    default:
        return hipErrorInvalidValue;
    }
    if (!last)
        hipLaunchKernelGGL(mixed_compact_kernel, dim3(nblk(max_n, 256), a.n_groups), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace pk
