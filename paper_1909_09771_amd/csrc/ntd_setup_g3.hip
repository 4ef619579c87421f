// ntd_setup_g3.hip -- factorization kernels for 14, 16 elements per lane (the
// instantiations are split over several files so that they compile in parallel).
#include "ntd_sweep.h"

namespace ntd {

hipError_t launch_setup_g3(const SetupArgs &a, int epl, hipStream_t s) {
    switch (epl) {
    case 14: return setup_impl<14>(a, s);
    case 16: return setup_impl<16>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ntd
