// Instantiation of the wave-per-problem LM kernel for n <= 40, m <= 4.
#include "lm_wave.hpp"

namespace pk {

hipError_t launch_lm_wave_40(const RobotC *rb, const SolveParams &P, int pb, hipStream_t s)
{
    return wave::launch_wave<40, 4>(rb, P, pb, s);
}

}  // namespace pk
