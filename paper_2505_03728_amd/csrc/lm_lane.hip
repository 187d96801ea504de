// Per-lane LM path: the 7-joint arm and the 4 x 4 hand star instantiated
// here, other single chains (2 to 10 joints, pose or position EE, revolute
// or prismatic joints) in lm_lane_chain*.hip; dispatch by robot shape.
#include "lm_lane_kernels.hpp"

namespace pk {

bool lane_variant_available(int chains, int chain_len, int kind)
{
    return (chains == 1 && chain_len >= 2 && chain_len <= PK_LANE_MAX_CHAIN) ||
           (chains == 4 && chain_len == 4 && kind == PK_EE_POSITION);
}

hipError_t launch_lm_lane(const RobotC *dev_robot, const RobotC &h, const SolveParams &P,
                          hipStream_t s, int persist_blocks, const BestOut *best)
{
    const int kind = h.e[0].kind | (h.prismatic ? lane::LANE_PRISMATIC : 0), L = h.chain_len;
    if (h.chains == 1 && L == 7 && kind == PK_EE_POSE)
        return lane::launch_star<1, 7, PK_EE_POSE>(dev_robot, P, persist_blocks, s, best);
    if (h.chains == 4 && L == 4 && kind == PK_EE_POSITION)
        return lane::launch_star<4, 4, PK_EE_POSITION>(dev_robot, P, persist_blocks, s, best);
    if (h.chains == 1) {
        if (L <= 4) return launch_lane_chain_a(L, kind, dev_robot, P, persist_blocks, s, best);
        if (L <= 7) return launch_lane_chain_b(L, kind, dev_robot, P, persist_blocks, s, best);
        return launch_lane_chain_c(L, kind, dev_robot, P, persist_blocks, s, best);
    }
    return hipErrorInvalidValue;
}

}  // namespace pk
