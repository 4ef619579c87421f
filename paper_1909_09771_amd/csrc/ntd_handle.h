// ntd_handle.h -- host-side state of one system (the handle of the C ABI) and
// the internal set-up and launch helpers that the batched solve shares with
// the single-system entry points.  Private to the library.
#pragma once

#include <stddef.h>

#include "ntd.h"
#include "ntd_internal.h"

struct ntd_handle {
    int nx, ny, nz, prec, schur, smoother, epl;
    ntd::IluGrid ilu;                         // ILU(0) level schedule (smoother only)
    double *dt, *dtinv, *zi, *tv;             // ILU(0) diagonal, its inverse, two work vectors
    float *fcoef;                             // MIXED: ax, ay, az, 1/dt in FP32 for the ILU(0) sweeps
    long long N, nxy, npack;                  // npack = ny*nz*64*epl packed slots
    size_t used;
    double *d, *ax, *ay, *az;                 // bands of A
    double *e1, *mv, *f2, *dT, *dP, *xP;      // factors (FP64, natural layout) and setup state
    double *r, *z, *p, *q;                    // PCG vectors
    void *rec;                                // line records of the apply (float in MIXED)
    void *pZ, *rp;                            // packed result and right-hand side
    void *scratch;                            // setup planes / packed apply planes
    double *partials;
    ntd::Scalars *sc;
    int *flag;
};

namespace ntd_host {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// Walks a workspace: identical for sizing (base == nullptr) and carving.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base((char *)b) {}
    template <typename T>
    T *take(size_t count) {
        size_t o = off;
        off = align_up(off + count * sizeof(T));
        return base ? (T *)(base + o) : nullptr;
    }
};

// Bytes of a handle's workspace.  epl: elements per lane of the apply (at
// least epl_for(nx)).  A lean handle (member of a batch) holds no PCG vectors
// and no packed right-hand side or result: the batch keeps those per
// right-hand side.
size_t handle_bytes(int nx, int ny, int nz, int prec, int smoother, int epl, bool lean);
bool grid_ok(int nx, int ny, int nz, int epl);

// The phases of a setup, for callers that run them over many systems at once:
// validation and layout (no GPU work; *out is a new handle), the check of kappa
// and t (result in the handle's device flag), the asynchronous read of that
// flag, the assembly of A, the factorization arguments, and the packing of the
// factors (after the factorization).
int handle_create(int nx, int ny, int nz, const int *bc, int prec, int schur, int smoother,
                  int epl, bool lean, void *workspace, size_t workspace_bytes, ntd_handle **out);
int handle_check(ntd_handle *h, const double *kappa, const double *t, hipStream_t s);
int handle_flag_async(const ntd_handle *h, int *flag, hipStream_t s);
int handle_assemble(ntd_handle *h, const double *kappa, const int *bc, hipStream_t s);
ntd::SetupArgs handle_setup_args(const ntd_handle *h, const double *t);
int handle_finish(ntd_handle *h, hipStream_t s);

// Validation, assembly, factorization and packing of one system into a
// workspace of handle_bytes(); on success *out is a new handle.
int setup_handle(int nx, int ny, int nz, const double *kappa, const int *bc, const double *t,
                 int prec, int schur, int smoother, int epl, bool lean, void *workspace,
                 size_t workspace_bytes, hipStream_t s, ntd_handle **out);

template <typename T>
ntd::ApplyArgs<T> apply_args(const ntd_handle *h) {
    ntd::ApplyArgs<T> a;
    a.nx = h->nx; a.ny = h->ny; a.nz = h->nz;
    a.rec = h->rec; a.rp = (const T *)h->rp; a.Z = (T *)h->pZ; a.scratch = (T *)h->scratch;
    return a;
}

template <typename T>
ntd::XferArgs<T> xfer_args(const ntd_handle *h) {
    ntd::XferArgs<T> x;
    x.nx = h->nx; x.ny = h->ny; x.nz = h->nz;
    x.r = nullptr; x.zi = nullptr;
    x.d = h->d; x.ax = h->ax; x.ay = h->ay; x.az = h->az;
    x.rp = (T *)h->rp; x.Z = (const T *)h->pZ; x.zout = nullptr; x.partials = nullptr;
    return x;
}

}  // namespace ntd_host
