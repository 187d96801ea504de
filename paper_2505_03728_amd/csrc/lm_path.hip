// Dispatch of the path-pair wavefront LM kernel (one problem per 64-lane
// wavefront, one lane per (joint, EE path) pair) and its instantiations for
// trees of up to 8 levels.  Rows of 8, 12 or 16 entries serve trees of up to
// 8, 13 or 16 levels (a joint's row has one entry per proper ancestor).
#include "lm_path.hpp"

namespace pk {

hipError_t launch_lm_path_d16(const RobotC *rb, const SolveParams &P, int levels, int m, int pb, hipStream_t s);

bool path_variant_available(const RobotC &h) { return h.path.ok != 0; }

hipError_t launch_lm_path(const RobotC *dev_robot, const RobotC &h, const SolveParams &P,
                          hipStream_t s, int persist_blocks)
{
    if (!h.path.ok) return hipErrorInvalidValue;
    const int levels = h.max_depth + 1;
    if (levels <= 8) {
        if (h.m <= 4) return path::launch_path<8, 4, 8>(dev_robot, P, persist_blocks, s);
        return path::launch_path<8, 8, 8>(dev_robot, P, persist_blocks, s);
    }
    return launch_lm_path_d16(dev_robot, P, levels, h.m, persist_blocks, s);
}

}  // namespace pk
