// Instantiations of the path-pair wavefront LM kernel for trees of 9 to 16
// levels (rows of 12 entries up to 13 levels, else 16) with up to 4 or 8 EEs.
#include "lm_path.hpp"

namespace pk {

hipError_t launch_lm_path_d16(const RobotC *rb, const SolveParams &P, int levels, int m, int pb, hipStream_t s)
{
    if (levels <= 13) {
        if (m <= 4) return path::launch_path<16, 4, 12>(rb, P, pb, s);
        return path::launch_path<16, 8, 12>(rb, P, pb, s);
    }
    if (m <= 4) return path::launch_path<16, 4, 16>(rb, P, pb, s);
    return path::launch_path<16, 8, 16>(rb, P, pb, s);
}

}  // namespace pk
