// Per-lane LM instantiations for single chains of 5 to 7 joints (pose or
// position EE; revolute-only and with-prismatic code), split from lm_lane.hip
// so that the units compile in parallel.
#include "lm_lane_kernels.hpp"

namespace pk {

// kind: the EE kind, plus lane::LANE_PRISMATIC if the chain has prismatic joints.
hipError_t launch_lane_chain_b(int L, int kind, const RobotC *rb, const SolveParams &P, int pb, hipStream_t s,
                               const BestOut *best)
{
    if (L == 7) {
        switch (kind) {
        case PK_EE_POSITION: return lane::launch_star<1, 7, PK_EE_POSITION>(rb, P, pb, s, best);
        case PK_EE_POSE | lane::LANE_PRISMATIC:
            return lane::launch_star<1, 7, PK_EE_POSE | lane::LANE_PRISMATIC>(rb, P, pb, s, best);
        case PK_EE_POSITION | lane::LANE_PRISMATIC:
            return lane::launch_star<1, 7, PK_EE_POSITION | lane::LANE_PRISMATIC>(rb, P, pb, s, best);
        default: return hipErrorInvalidValue;
        }
    }
    if (L == 5) {
        switch (kind) {
        case PK_EE_POSE: return lane::launch_star<1, 5, PK_EE_POSE>(rb, P, pb, s, best);
        case PK_EE_POSITION: return lane::launch_star<1, 5, PK_EE_POSITION>(rb, P, pb, s, best);
        case PK_EE_POSE | lane::LANE_PRISMATIC:
            return lane::launch_star<1, 5, PK_EE_POSE | lane::LANE_PRISMATIC>(rb, P, pb, s, best);
        case PK_EE_POSITION | lane::LANE_PRISMATIC:
            return lane::launch_star<1, 5, PK_EE_POSITION | lane::LANE_PRISMATIC>(rb, P, pb, s, best);
        default: return hipErrorInvalidValue;
        }
    }
    if (L == 6) {
        switch (kind) {
        case PK_EE_POSE: return lane::launch_star<1, 6, PK_EE_POSE>(rb, P, pb, s, best);
        case PK_EE_POSITION: return lane::launch_star<1, 6, PK_EE_POSITION>(rb, P, pb, s, best);
        case PK_EE_POSE | lane::LANE_PRISMATIC:
            return lane::launch_star<1, 6, PK_EE_POSE | lane::LANE_PRISMATIC>(rb, P, pb, s, best);
        case PK_EE_POSITION | lane::LANE_PRISMATIC:
            return lane::launch_star<1, 6, PK_EE_POSITION | lane::LANE_PRISMATIC>(rb, P, pb, s, best);
        default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace pk
