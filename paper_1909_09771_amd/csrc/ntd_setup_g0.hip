// ntd_setup_g0.hip -- factorization kernels for 1, 2, 3, 4 elements per lane (the
// instantiations are split over several files so that they compile in parallel).
#include "ntd_sweep.h"

namespace ntd {

hipError_t launch_setup_g0(const SetupArgs &a, int epl, hipStream_t s) {
    switch (epl) {
    case 1: return setup_impl<1>(a, s);
    case 2: return setup_impl<2>(a, s);
    case 3: return setup_impl<3>(a, s);
    case 4: return setup_impl<4>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_setup_batch_g0(const SetupArgs *tab, int count, int max_nx, int epl,
                                 hipStream_t s) {
    switch (epl) {
    case 1: return setup_batch_impl<1>(tab, count, max_nx, s);
    case 2: return setup_batch_impl<2>(tab, count, max_nx, s);
    case 3: return setup_batch_impl<3>(tab, count, max_nx, s);
    case 4: return setup_batch_impl<4>(tab, count, max_nx, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ntd
