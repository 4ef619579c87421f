// ntd_setup_g1.hip -- factorization kernels for 5, 6, 7, 8 elements per lane (the
// instantiations are split over several files so that they compile in parallel).
#include "ntd_sweep.h"

namespace ntd {

hipError_t launch_setup_g1(const SetupArgs &a, int epl, hipStream_t s) {
    switch (epl) {
    case 5: return setup_impl<5>(a, s);
    case 6: return setup_impl<6>(a, s);
    case 7: return setup_impl<7>(a, s);
    case 8: return setup_impl<8>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_setup_batch_g1(const SetupArgs *tab, int count, int max_nx, int epl,
                                 hipStream_t s) {
    switch (epl) {
    case 5: return setup_batch_impl<5>(tab, count, max_nx, s);
    case 6: return setup_batch_impl<6>(tab, count, max_nx, s);
    case 7: return setup_batch_impl<7>(tab, count, max_nx, s);
    case 8: return setup_batch_impl<8>(tab, count, max_nx, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ntd
