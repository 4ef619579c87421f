// ntd_apply_multi_f32.hip -- instantiation of the batched sweeps with several
// right-hand sides per wavefront pair, in float.
#include "ntd_apply_multi.h"

namespace ntd {

bool batch_multi_ok(int elem_bytes, int epl, int nr) {
    if (nr == 1) return true;
    if (elem_bytes == 4) return (nr == 2 && epl >= 1 && epl <= 4) || (nr == 4 && epl >= 1 && epl <= 2);
    if (elem_bytes == 8) return (nr == 2 && epl >= 1 && epl <= 2) || (nr == 4 && epl == 1);
    return false;
}

hipError_t launch_apply_batch_multi_f32(const ApplyArgs<float> *tab, const int *active, int count,
                                        int nrhs, int epl, int nr, hipStream_t s, hipEvent_t *ev) {
    if (nr < 2 || nrhs % nr != 0 || !batch_multi_ok((int)sizeof(float), epl, nr))
        return hipErrorInvalidValue;
    if (nr == 2) {
        switch (epl) {
        case 1: return apply_batch_multi_impl<float, 1, 2>(tab, active, count, nrhs, s, ev);
        case 2: return apply_batch_multi_impl<float, 2, 2>(tab, active, count, nrhs, s, ev);
        case 3: return apply_batch_multi_impl<float, 3, 2>(tab, active, count, nrhs, s, ev);
        case 4: return apply_batch_multi_impl<float, 4, 2>(tab, active, count, nrhs, s, ev);
        default: break;
        }
    } else if (nr == 4) {
        switch (epl) {
        case 1: return apply_batch_multi_impl<float, 1, 4>(tab, active, count, nrhs, s, ev);
        case 2: return apply_batch_multi_impl<float, 2, 4>(tab, active, count, nrhs, s, ev);
        default: break;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace ntd
