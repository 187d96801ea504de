// Dispatch of the wave-per-problem LM kernel (one problem per 64-lane
// wavefront, any revolute tree up to 64 joints and 8 EEs) to the
// instantiation sized for the robot's depth and EE count.
#include "pk_internal.hpp"

namespace pk {

hipError_t launch_lm_wave_d8(const RobotC *rb, const SolveParams &P, int m, int pb, hipStream_t s);
hipError_t launch_lm_wave_d16(const RobotC *rb, const SolveParams &P, int m, int pb, hipStream_t s);
hipError_t launch_lm_wave_d32(const RobotC *rb, const SolveParams &P, int m, int pb, hipStream_t s);
hipError_t launch_lm_wave_d64(const RobotC *rb, const SolveParams &P, int m, int pb, hipStream_t s);

bool wave_variant_available(int n) { return n >= 1 && n <= 64; }

hipError_t launch_lm_wave(const RobotC *dev_robot, const RobotC &h, const SolveParams &P,
                          hipStream_t s, int persist_blocks)
{
    const int levels = h.max_depth + 1;
    if (levels <= 8) return launch_lm_wave_d8(dev_robot, P, h.m, persist_blocks, s);
    if (levels <= 16) return launch_lm_wave_d16(dev_robot, P, h.m, persist_blocks, s);
    if (levels <= 32) return launch_lm_wave_d32(dev_robot, P, h.m, persist_blocks, s);
    return launch_lm_wave_d64(dev_robot, P, h.m, persist_blocks, s);
}

}  // namespace pk
