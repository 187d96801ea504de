// Dispatch of the wave-per-problem LM kernel (one problem per 64-lane
// wavefront, any revolute tree up to 64 joints and 8 EEs) to the
// instantiation sized for the robot.
#include "pk_internal.hpp"

namespace pk {

hipError_t launch_lm_wave_16(const RobotC *rb, const SolveParams &P, int pb, hipStream_t s);
hipError_t launch_lm_wave_40(const RobotC *rb, const SolveParams &P, int pb, hipStream_t s);
hipError_t launch_lm_wave_64(const RobotC *rb, const SolveParams &P, int pb, hipStream_t s);

bool wave_variant_available(int n) { return n >= 1 && n <= 64; }

hipError_t launch_lm_wave(const RobotC *dev_robot, const RobotC &h, const SolveParams &P,
                          hipStream_t s, int persist_blocks)
{
    if (h.m <= 4) {
        if (h.n <= 16) return launch_lm_wave_16(dev_robot, P, persist_blocks, s);
        if (h.n <= 40) return launch_lm_wave_40(dev_robot, P, persist_blocks, s);
    }
    return launch_lm_wave_64(dev_robot, P, persist_blocks, s);
}

}  // namespace pk
