// ntd_apply_multi_f64.hip -- instantiation of the batched sweeps with several
// right-hand sides per wavefront pair, in double.
#include "ntd_apply_multi.h"

namespace ntd {

hipError_t launch_apply_batch_multi_f64(const ApplyArgs<double> *tab, const int *active, int count,
                                        int nrhs, int epl, int nr, hipStream_t s, hipEvent_t *ev) {
    if (nr < 2 || nrhs % nr != 0 || !batch_multi_ok((int)sizeof(double), epl, nr))
        return hipErrorInvalidValue;
    if (nr == 2) {
        switch (epl) {
        case 1: return apply_batch_multi_impl<double, 1, 2>(tab, active, count, nrhs, s, ev);
        case 2: return apply_batch_multi_impl<double, 2, 2>(tab, active, count, nrhs, s, ev);
        default: break;
        }
    } else if (nr == 4) {
        switch (epl) {
        case 1: return apply_batch_multi_impl<double, 1, 4>(tab, active, count, nrhs, s, ev);
        default: break;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace ntd
