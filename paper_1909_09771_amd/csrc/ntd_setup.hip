// ntd_setup.hip -- instantiation of the factorization kernels and the choice
// of the per-lane chain length.
#include "ntd_sweep.h"

namespace ntd {

int epl_for(int nx) {
    if (nx < 1) return 0;
    const int ca = (nx + 1) / 2;
    const int need = (ca + 31) / 32;
#define NTD_PICK(E) if (need <= E) return E;
    NTD_EPL_LIST(NTD_PICK)
#undef NTD_PICK
    return 0;
}

hipError_t launch_setup(const SetupArgs &a, int epl, hipStream_t s) {
    switch (epl) {
#define NTD_CASE(E) case E: return setup_impl<E>(a, s);
        NTD_EPL_LIST(NTD_CASE)
#undef NTD_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_setup_batch(const SetupArgs *tab, int count, int max_nx, int epl,
                              hipStream_t s) {
    switch (epl) {
#define NTD_CASE(E) case E: return setup_batch_impl<E>(tab, count, max_nx, s);
        NTD_BATCH_EPL_LIST(NTD_CASE)
#undef NTD_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ntd
