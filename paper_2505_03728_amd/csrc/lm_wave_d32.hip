// Instantiations of the wave-per-problem LM kernel for trees of depth <= 32
// (up to 4 or 8 EEs).
#include "lm_wave.hpp"

namespace pk {

hipError_t launch_lm_wave_d32(const RobotC *rb, const SolveParams &P, int m, int pb, hipStream_t s)
{
    if (m <= 4) return wave::launch_wave<32, 4>(rb, P, pb, s);
    return wave::launch_wave<32, 8>(rb, P, pb, s);
}

}  // namespace pk
