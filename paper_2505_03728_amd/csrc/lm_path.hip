// Instantiations and dispatch of the path-pair wavefront LM kernel (one
// problem per 64-lane wavefront, one lane per (joint, EE path) pair) for
// trees of depth <= 8 or <= 16 with up to 4 or 8 EEs.
#include "lm_path.hpp"

namespace pk {

bool path_variant_available(const RobotC &h) { return h.path.ok != 0; }

hipError_t launch_lm_path(const RobotC *dev_robot, const RobotC &h, const SolveParams &P,
                          hipStream_t s, int persist_blocks)
{
    if (!h.path.ok) return hipErrorInvalidValue;
    const int levels = h.max_depth + 1;
    if (levels <= 8) {
        if (h.m <= 4) return path::launch_path<8, 4>(dev_robot, P, persist_blocks, s);
        return path::launch_path<8, 8>(dev_robot, P, persist_blocks, s);
    }
    if (h.m <= 4) return path::launch_path<16, 4>(dev_robot, P, persist_blocks, s);
    return path::launch_path<16, 8>(dev_robot, P, persist_blocks, s);
}

}  // namespace pk
