// ntd_setup_g2.hip -- factorization kernels for 10, 12 elements per lane (the
// instantiations are split over several files so that they compile in parallel).
#include "ntd_sweep.h"

namespace ntd {

hipError_t launch_setup_g2(const SetupArgs &a, int epl, hipStream_t s) {
    switch (epl) {
    case 10: return setup_impl<10>(a, s);
    case 12: return setup_impl<12>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ntd
