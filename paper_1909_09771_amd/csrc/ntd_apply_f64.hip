// ntd_apply_f64.hip -- instantiation of the preconditioner apply in double.
#include "ntd_sweep.h"

namespace ntd {

hipError_t launch_apply_f64(const ApplyArgs<double> &a, int epl, hipStream_t s, hipEvent_t *ev) {
    switch (epl) {
#define NTD_CASE(E) case E: return apply_impl<double, E>(a, s, ev);
        NTD_EPL_LIST(NTD_CASE)
#undef NTD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pack_f64(const PackArgs<double> &p, int epl, hipStream_t s) {
    switch (epl) {
#define NTD_CASE(E) case E: return pack_impl<double, E>(p, s);
        NTD_EPL_LIST(NTD_CASE)
#undef NTD_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ntd
