// ntd_setup.hip -- the choice of the per-lane chain length and the dispatch
// of the factorization to the file that instantiates it for that length.
#include "ntd_sweep.h"

namespace ntd {

hipError_t launch_setup_g0(const SetupArgs &a, int epl, hipStream_t s);
hipError_t launch_setup_g1(const SetupArgs &a, int epl, hipStream_t s);
hipError_t launch_setup_g2(const SetupArgs &a, int epl, hipStream_t s);
hipError_t launch_setup_g3(const SetupArgs &a, int epl, hipStream_t s);
hipError_t launch_setup_batch_g0(const SetupArgs *tab, int count, int max_nx, int epl,
                                 hipStream_t s);
hipError_t launch_setup_batch_g1(const SetupArgs *tab, int count, int max_nx, int epl,
                                 hipStream_t s);

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
    if (epl >= 1 && epl <= 4) return launch_setup_g0(a, epl, s);
    if (epl >= 5 && epl <= 8) return launch_setup_g1(a, epl, s);
    if (epl >= 10 && epl <= 12) return launch_setup_g2(a, epl, s);
    if (epl >= 14 && epl <= 16) return launch_setup_g3(a, epl, s);
    return hipErrorInvalidValue;
}

hipError_t launch_setup_batch(const SetupArgs *tab, int count, int max_nx, int epl,
                              hipStream_t s) {
    if (epl >= 1 && epl <= 4) return launch_setup_batch_g0(tab, count, max_nx, epl, s);
    if (epl >= 5 && epl <= 8) return launch_setup_batch_g1(tab, count, max_nx, epl, s);
    return hipErrorInvalidValue;
}

}  // namespace ntd
