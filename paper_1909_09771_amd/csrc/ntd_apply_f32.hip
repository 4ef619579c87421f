// ntd_apply_f32.hip -- instantiation of the preconditioner apply in float.
#include "ntd_sweep.h"

namespace ntd {

hipError_t launch_apply_f32(const ApplyArgs<float> &a, int epl, hipStream_t s, hipEvent_t *ev) {
    switch (epl) {
#define NTD_CASE(E) case E: return apply_impl<float, E>(a, s, ev);
        NTD_EPL_LIST(NTD_CASE)
#undef NTD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pack_f32(const PackArgs<float> &p, int epl, hipStream_t s) {
    switch (epl) {
#define NTD_CASE(E) case E: return pack_impl<float, E>(p, s);
        NTD_EPL_LIST(NTD_CASE)
#undef NTD_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ntd
