// Per-lane LM instantiations for single chains of 2 to 4 joints (pose or
// position EE; revolute-only and with-prismatic code), split from lm_lane.hip
// so that the units compile in parallel.
#include "lm_lane_kernels.hpp"

namespace pk {

// kind: the EE kind, plus lane::LANE_PRISMATIC if the chain has prismatic joints.
hipError_t launch_lane_chain_a(int L, int kind, const RobotC *rb, const SolveParams &P, int pb, hipStream_t s,
                               const BestOut *best)
{
    if (L == 2) {
        switch (kind) {
        case PK_EE_POSE: return lane::launch_star<1, 2, PK_EE_POSE>(rb, P, pb, s, best);
        case PK_EE_POSITION: return lane::launch_star<1, 2, PK_EE_POSITION>(rb, P, pb, s, best);
        case PK_EE_POSE | lane::LANE_PRISMATIC:
            return lane::launch_star<1, 2, PK_EE_POSE | lane::LANE_PRISMATIC>(rb, P, pb, s, best);
        case PK_EE_POSITION | lane::LANE_PRISMATIC:
            return lane::launch_star<1, 2, PK_EE_POSITION | lane::LANE_PRISMATIC>(rb, P, pb, s, best);
        default: return hipErrorInvalidValue;
        }
    }
    if (L == 3) {
        switch (kind) {
        case PK_EE_POSE: return lane::launch_star<1, 3, PK_EE_POSE>(rb, P, pb, s, best);
        case PK_EE_POSITION: return lane::launch_star<1, 3, PK_EE_POSITION>(rb, P, pb, s, best);
        case PK_EE_POSE | lane::LANE_PRISMATIC:
            return lane::launch_star<1, 3, PK_EE_POSE | lane::LANE_PRISMATIC>(rb, P, pb, s, best);
        case PK_EE_POSITION | lane::LANE_PRISMATIC:
            return lane::launch_star<1, 3, PK_EE_POSITION | lane::LANE_PRISMATIC>(rb, P, pb, s, best);
        default: return hipErrorInvalidValue;
        }
    }
    if (L == 4) {
        switch (kind) {
        case PK_EE_POSE: return lane::launch_star<1, 4, PK_EE_POSE>(rb, P, pb, s, best);
        case PK_EE_POSITION: return lane::launch_star<1, 4, PK_EE_POSITION>(rb, P, pb, s, best);
        case PK_EE_POSE | lane::LANE_PRISMATIC:
            return lane::launch_star<1, 4, PK_EE_POSE | lane::LANE_PRISMATIC>(rb, P, pb, s, best);
        case PK_EE_POSITION | lane::LANE_PRISMATIC:
            return lane::launch_star<1, 4, PK_EE_POSITION | lane::LANE_PRISMATIC>(rb, P, pb, s, best);
        default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace pk
