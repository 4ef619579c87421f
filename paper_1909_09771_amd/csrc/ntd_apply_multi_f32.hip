// ntd_apply_multi_f32.hip -- instantiation of the batched sweeps with several
// right-hand sides per wavefront pair, in float.
#include <utility>

#include "ntd_apply_multi.h"

namespace ntd {

bool batch_multi_ok(int elem_bytes, int epl, int nr) {
    if (nr == 1) return true;
    if (elem_bytes == 4) return (nr == 2 && epl >= 1 && epl <= 4) || (nr == 4 && epl >= 1 && epl <= 2);
    if (elem_bytes == 8) return (nr == 2 && epl >= 1 && epl <= 2) || (nr == 4 && epl == 1);
    return false;
}

namespace {

// The built (EPL, NR) instances, as ntd::batch_multi_ok lists them.
template <template <typename, int, int> class F, typename... A>
hipError_t dispatch_f32(int epl, int nr, A &&...args) {
    if (nr == 2) {
        switch (epl) {
        case 1: return F<float, 1, 2>::run(std::forward<A>(args)...);
        case 2: return F<float, 2, 2>::run(std::forward<A>(args)...);
        case 3: return F<float, 3, 2>::run(std::forward<A>(args)...);
        case 4: return F<float, 4, 2>::run(std::forward<A>(args)...);
        default: break;
        }
    } else if (nr == 4) {
        switch (epl) {
        case 1: return F<float, 1, 4>::run(std::forward<A>(args)...);
        case 2: return F<float, 2, 4>::run(std::forward<A>(args)...);
        default: break;
        }
    }
    return hipErrorInvalidValue;
}

template <typename T, int EPL, int NR>
struct Sweeps {
    static hipError_t run(const ApplyArgs<T> *tab, const int *active, int count, int nrhs,
                          size_t plane_lds, hipStream_t s, hipEvent_t *ev) {
        return apply_batch_multi_impl<T, EPL, NR>(tab, active, count, nrhs, plane_lds, s, ev);
    }
};
template <typename T, int EPL, int NR>
struct AllowLds {
    static hipError_t run(size_t bytes) { return apply_batch_multi_lds_impl<T, EPL, NR>(bytes); }
};

}  // namespace

hipError_t launch_apply_batch_multi_f32(const ApplyArgs<float> *tab, const int *active, int count,
                                        int nrhs, int epl, int nr, size_t plane_lds, hipStream_t s,
                                        hipEvent_t *ev) {
    if (nr < 2 || nrhs % nr != 0 || !batch_multi_ok((int)sizeof(float), epl, nr))
        return hipErrorInvalidValue;
    return dispatch_f32<Sweeps>(epl, nr, tab, active, count, nrhs, plane_lds, s, ev);
}

hipError_t allow_apply_batch_multi_lds_f32(int epl, int nr, size_t bytes) {
    if (nr < 2 || !batch_multi_ok((int)sizeof(float), epl, nr)) return hipErrorInvalidValue;
    return dispatch_f32<AllowLds>(epl, nr, bytes);
}

}  // namespace ntd
