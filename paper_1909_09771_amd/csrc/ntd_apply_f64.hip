// ntd_apply_f64.hip -- instantiation of the preconditioner apply, the factor
// packing and the natural/packed moves in double.
#include "ntd_apply.h"

namespace ntd {

hipError_t launch_apply_f64(const ApplyArgs<double> &a, int epl, hipStream_t s, hipEvent_t *ev) {
    switch (epl) {
#define NTD_CASE(E) case E: return apply_impl<double, E>(a, s, ev);
        NTD_EPL_LIST(NTD_CASE)
#undef NTD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pack_f64(const PackArgs &p, int epl, hipStream_t s) {
    switch (epl) {
#define NTD_CASE(E) case E: return pack_impl<double, E>(p, s);
        NTD_EPL_LIST(NTD_CASE)
#undef NTD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pack_rhs_f64(const XferArgs<double> &x, int epl, hipStream_t s) {
    switch (epl) {
#define NTD_CASE(E) case E: return pack_rhs_impl<double, E>(x, s);
        NTD_EPL_LIST(NTD_CASE)
#undef NTD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_unpack_f64(const XferArgs<double> &x, int epl, hipStream_t s, int *np) {
    switch (epl) {
#define NTD_CASE(E) case E: return unpack_impl<double, E>(x, s, np);
        NTD_EPL_LIST(NTD_CASE)
#undef NTD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_apply_batch_f64(const ApplyArgs<double> *tab, const int *active, int count,
                                  int nrhs, int epl, size_t plane_lds, hipStream_t s,
                                  hipEvent_t *ev) {
    switch (epl) {
#define NTD_CASE(E) \
    case E: return apply_batch_impl<double, E>(tab, active, count, nrhs, plane_lds, s, ev);
        NTD_BATCH_EPL_LIST(NTD_CASE)
#undef NTD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t allow_apply_batch_lds_f64(int epl, size_t bytes) {
    switch (epl) {
#define NTD_CASE(E) case E: return apply_batch_lds_impl<double, E>(bytes);
        NTD_BATCH_EPL_LIST(NTD_CASE)
#undef NTD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pack_rhs_batch_f64(const XferArgs<double> *tab, const int *active, int count,
                                     int gx, int epl, hipStream_t s) {
    switch (epl) {
#define NTD_CASE(E) case E: return pack_rhs_batch_impl<double, E>(tab, active, count, gx, s);
        NTD_BATCH_EPL_LIST(NTD_CASE)
#undef NTD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_unpack_batch_f64(const XferArgs<double> *tab, const int *active, int count,
                                   int gx, int epl, hipStream_t s) {
    switch (epl) {
#define NTD_CASE(E) case E: return unpack_batch_impl<double, E>(tab, active, count, gx, s);
        NTD_BATCH_EPL_LIST(NTD_CASE)
#undef NTD_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ntd
