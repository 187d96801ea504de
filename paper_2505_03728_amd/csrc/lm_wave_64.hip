// Instantiation of the wave-per-problem LM kernel for n <= 64, m <= 8.
#include "lm_wave.hpp"

namespace pk {

hipError_t launch_lm_wave_64(const RobotC *rb, const SolveParams &P, int pb, hipStream_t s)
{
    return wave::launch_wave<64, 8>(rb, P, pb, s);
}

}  // namespace pk
