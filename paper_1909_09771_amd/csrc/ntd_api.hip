// ntd_api.hip -- host side of the C ABI declared in include/ntd.h: argument
// validation, the layout of the caller's workspace, kernel launches and the
// PCG driver loop.  Nothing here allocates device memory: every device array
// lives in the workspace the caller passes to ntd_setup.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "ntd.h"
#include "ntd_handle.h"

using ntd::Scalars;

namespace ntd_host {

bool grid_ok(int nx, int ny, int nz, int epl) {
    if (nx < 1 || ny < 1 || nz < 1) return false;
    if (nx > NTD_MAX_NX || epl < ntd::epl_for(nx) || ntd::epl_for(nx) == 0) return false;
    // FP64 arrays are addressed with 32-bit byte offsets, the records and packed
    // vectors of one plane too
    const long long N = (long long)nx * ny * nz;
    const long long npack = (long long)ny * nz * 64 * epl;
    const long long plane_rec = (long long)ny * ntd::rec_bytes(sizeof(double), epl);
    return N * 8 < 0x7fffffffLL && npack * 8 < 0x7fffffffLL && plane_rec < 0x7fffffffLL;
}

}  // namespace ntd_host

namespace {

using ntd_host::Carver;
using ntd_host::apply_args;
using ntd_host::xfer_args;
using ntd_host::kAlign;

size_t layout(ntd_handle *h, void *ws, int nx, int ny, int nz, int prec, int smoother, int epl,
              bool lean) {
    const long long N = (long long)nx * ny * nz, nxy = (long long)nx * ny;
    const long long lane_slots = 64LL * epl;
    const long long npack = (long long)ny * nz * lane_slots;
    const size_t tsz = prec == NTD_PREC_MIXED ? sizeof(float) : sizeof(double);
    Carver c(ws);
    double **f64[] = {&h->d, &h->ax, &h->ay, &h->az, &h->e1, &h->mv, &h->f2, &h->dT, &h->dP, &h->xP};
    for (double **a : f64) *a = c.take<double>(N);
    h->r = h->z = h->p = h->q = nullptr;
    h->pZ = h->rp = nullptr;
    if (!lean) {
        double **vec[] = {&h->r, &h->z, &h->p, &h->q};
        for (double **a : vec) *a = c.take<double>(N);
    }
    h->rec = (void *)c.take<char>((size_t)ny * nz * ntd::rec_bytes((unsigned)tsz, epl));
    if (!lean) {
        h->pZ = (void *)c.take<char>(npack * tsz);
        h->rp = (void *)c.take<char>(npack * tsz);
    }
    h->dt = h->dtinv = h->zi = h->tv = nullptr;
    h->fcoef = nullptr;
    if (smoother != NTD_SMOOTHER_NONE) {
        double **ilu[] = {&h->dt, &h->dtinv, &h->zi, &h->tv};
        for (double **a : ilu) *a = c.take<double>(N);
        if (prec == NTD_PREC_MIXED) h->fcoef = c.take<float>(4 * N);
    }
    const size_t setup_scr = 6 * (size_t)nxy * sizeof(double);
    const size_t apply_scr = 2 * (size_t)ny * lane_slots * tsz;
    h->scratch = (void *)c.take<char>(setup_scr > apply_scr ? setup_scr : apply_scr);
    h->partials = c.take<double>(ntd::kMaxBlocks);
    h->sc = c.take<Scalars>(1);
    h->flag = c.take<int>(4);
    return c.off;
}

#define CK(expr)                                 \
    do {                                         \
        if ((expr) != hipSuccess) return NTD_EHIP; \
    } while (0)

inline hipStream_t S(void *s) { return (hipStream_t)s; }

ntd::Grid grid_of(const ntd_handle *h) {
    ntd::Grid g;
    g.nx = h->nx; g.ny = h->ny; g.nz = h->nz; g.nxy = h->nxy; g.N = h->N;
    return g;
}

ntd::PackArgs pack_args(const ntd_handle *h) {
    ntd::PackArgs p;
    p.nx = h->nx; p.ny = h->ny; p.nz = h->nz;
    p.e1 = h->e1; p.mv = h->mv; p.f2 = h->f2; p.g3 = h->az;
    p.rec = h->rec;
    return p;
}

// Launchers of one precision, picked by overload.
hipError_t pack_rhs(const ntd::XferArgs<float> &x, int epl, hipStream_t s) {
    return ntd::launch_pack_rhs_f32(x, epl, s);
}
hipError_t pack_rhs(const ntd::XferArgs<double> &x, int epl, hipStream_t s) {
    return ntd::launch_pack_rhs_f64(x, epl, s);
}
hipError_t sweeps(const ntd::ApplyArgs<float> &a, int epl, hipStream_t s, hipEvent_t *ev) {
    return ntd::launch_apply_f32(a, epl, s, ev);
}
hipError_t sweeps(const ntd::ApplyArgs<double> &a, int epl, hipStream_t s, hipEvent_t *ev) {
    return ntd::launch_apply_f64(a, epl, s, ev);
}
hipError_t unpack(const ntd::XferArgs<float> &x, int epl, hipStream_t s, int *np) {
    return ntd::launch_unpack_f32(x, epl, s, np);
}
hipError_t unpack(const ntd::XferArgs<double> &x, int epl, hipStream_t s, int *np) {
    return ntd::launch_unpack_f64(x, epl, s, np);
}

// z = B^{-1} rhs with rhs = r, or r - A zi when zi is given (then z = zi +
// B^{-1}(r - A zi)): pack the right-hand side, run the three sweep launches,
// unpack.  With partials, the unpack also writes per-block partials of r.z and
// *np their count.  ev (if not null, 6 events): ev[0] before the pack, ev[1..4]
// bracket the sweeps, ev[5] after the unpack.
template <typename T>
int ntd_solve(ntd_handle *h, const double *r, const double *zi, double *z, double *partials,
              int *np, hipStream_t s, hipEvent_t *ev) {
    ntd::XferArgs<T> x = xfer_args<T>(h);
    x.r = r;
    x.zi = zi;
    if (ev) CK(hipEventRecord(ev[0], s));
    CK(pack_rhs(x, h->epl, s));
    CK(sweeps(apply_args<T>(h), h->epl, s, ev ? ev + 1 : nullptr));
    x.zout = z;
    x.partials = partials;
    CK(unpack(x, h->epl, s, np));
    if (ev) CK(hipEventRecord(ev[5], s));
    return NTD_OK;
}

int ntd_solve_any(ntd_handle *h, const double *r, const double *zi, double *z, double *partials,
                  int *np, hipStream_t s, hipEvent_t *ev) {
    if (h->prec == NTD_PREC_FP64) return ntd_solve<double>(h, r, zi, z, partials, np, s, ev);
    return ntd_solve<float>(h, r, zi, z, partials, np, s, ev);
}

// z = B_ILU^{-1} r (block-diagonal ILU(0)).
int ilu_internal(ntd_handle *h, const double *r, double *z, hipStream_t s) {
    CK(ntd::launch_ilu_apply(h->ilu, h->ax, h->ay, h->az, h->dtinv, h->fcoef, r, z, s));
    return NTD_OK;
}

// The handle's preconditioner: B^{-1} r; with the ILU(0) smoother the
// combination of eq. com evaluated as z = B_ILU^{-1} r + B^{-1}(r - A B_ILU^{-1} r);
// with the symmetric smoother that z followed by z += B_ILU^{-1}(r - A z).
// ev: as for ntd_solve, with ev[0] recorded before the ILU(0) sweeps and ev[5]
// after the last stage.
int precond_internal(ntd_handle *h, const double *r, double *z, double *partials, int *np,
                     hipStream_t s, hipEvent_t *ev = nullptr) {
    if (h->smoother == NTD_SMOOTHER_NONE)
        return ntd_solve_any(h, r, nullptr, z, partials, np, s, ev);
    if (ev) CK(hipEventRecord(ev[0], s));
    int st = ilu_internal(h, r, h->zi, s);
    if (st != NTD_OK) return st;
    hipEvent_t ev2[6];
    if (ev) {
        for (int i = 1; i < 6; ++i) ev2[i] = ev[i];
        ev2[0] = ev[6];  // a spare event: the pack start inside the smoother region
    }
    const bool sym = h->smoother == NTD_SMOOTHER_ILU0_SYM;
    st = ntd_solve_any(h, r, h->zi, z, sym ? nullptr : partials, sym ? nullptr : np, s,
                       ev ? ev2 : nullptr);
    if (st != NTD_OK || !sym) return st;
    // third stage: tv = r - A z, zi = B_ILU^{-1} tv, z += zi with the r.z partials
    CK(ntd::launch_spmv(grid_of(h), h->d, h->ax, h->ay, h->az, z, h->tv, nullptr, nullptr, s));
    CK(ntd::launch_residual(h->tv, r, h->tv, h->N, s));
    if ((st = ilu_internal(h, h->tv, h->zi, s)) != NTD_OK) return st;
    CK(ntd::launch_add_dot(z, h->zi, r, h->N, partials, np, s));
    if (ev) CK(hipEventRecord(ev[5], s));
    return NTD_OK;
}

// Pack the FP64 natural-layout factors into the line records of the apply.
int pack_factors(ntd_handle *h, hipStream_t s) {
    if (h->prec == NTD_PREC_FP64) {
        CK(ntd::launch_pack_f64(pack_args(h), h->epl, s));
    } else {
        CK(ntd::launch_pack_f32(pack_args(h), h->epl, s));
    }
    return NTD_OK;
}

int read_scalars(const ntd_handle *h, Scalars *out, hipStream_t s) {
    CK(hipMemcpyAsync(out, h->sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    return NTD_OK;
}

// ||v||^2 into sc->result and onto the host.
int norm2(ntd_handle *h, const double *v, double *out, hipStream_t s) {
    int np = 0;
    CK(ntd::launch_dot(v, v, h->N, h->partials, &np, s));
    CK(ntd::launch_finalize(h->partials, np, h->sc, ntd::kOpResult, s));
    Scalars hs;
    int st = read_scalars(h, &hs, s);
    if (st != NTD_OK) return st;
    *out = hs.result;
    return NTD_OK;
}

// True relative residual ||b - A x|| / bn, using q as scratch.
int true_relres(ntd_handle *h, const double *b, const double *x, double bn, double *out,
                hipStream_t s) {
    ntd::Grid g = grid_of(h);
    CK(ntd::launch_spmv(g, h->d, h->ax, h->ay, h->az, x, h->q, nullptr, nullptr, s));
    CK(ntd::launch_residual(h->q, b, h->q, h->N, s));
    double rr = 0.0;
    int st = norm2(h, h->q, &rr, s);
    if (st != NTD_OK) return st;
    *out = sqrt(rr) / bn;
    return NTD_OK;
}

}  // namespace

namespace ntd_host {

size_t handle_bytes(int nx, int ny, int nz, int prec, int smoother, int epl, bool lean) {
    if (!grid_ok(nx, ny, nz, epl) || (prec != NTD_PREC_FP64 && prec != NTD_PREC_MIXED)) return 0;
    if (smoother != NTD_SMOOTHER_NONE && smoother != NTD_SMOOTHER_ILU0 &&
        smoother != NTD_SMOOTHER_ILU0_SYM)
        return 0;
    ntd_handle tmp;
    return layout(&tmp, nullptr, nx, ny, nz, prec, smoother, epl, lean);
}

int handle_create(int nx, int ny, int nz, const int *bc, int prec, int schur, int smoother,
                  int epl, bool lean, void *workspace, size_t workspace_bytes, ntd_handle **out) {
    *out = nullptr;
    if (!bc || !workspace) return NTD_EINVAL;
    if (!grid_ok(nx, ny, nz, epl)) return NTD_EINVAL;
    if (prec != NTD_PREC_FP64 && prec != NTD_PREC_MIXED) return NTD_EINVAL;
    if (schur != NTD_SCHUR_NEWTON && schur != NTD_SCHUR_DIAG) return NTD_EINVAL;
    if (smoother != NTD_SMOOTHER_NONE && smoother != NTD_SMOOTHER_ILU0 &&
        smoother != NTD_SMOOTHER_ILU0_SYM)
        return NTD_EINVAL;
    int ndir = 0;
    for (int f = 0; f < 6; ++f) {
        if (bc[f] != NTD_BC_DIRICHLET && bc[f] != NTD_BC_NEUMANN) return NTD_EINVAL;
        ndir += bc[f] == NTD_BC_DIRICHLET;
    }
    if (ndir == 0) return NTD_EINVAL;  // pure Neumann: A is singular
    if (((uintptr_t)workspace) % kAlign) return NTD_EINVAL;
    if (workspace_bytes < handle_bytes(nx, ny, nz, prec, smoother, epl, lean)) return NTD_EINVAL;
    ntd_handle *h = (ntd_handle *)calloc(1, sizeof(ntd_handle));
    if (!h) return NTD_ENOMEM;
    h->nx = nx; h->ny = ny; h->nz = nz; h->prec = prec; h->schur = schur;
    h->smoother = smoother;
    h->epl = epl;
    h->N = (long long)nx * ny * nz;
    h->nxy = (long long)nx * ny;
    h->npack = (long long)ny * nz * 64 * h->epl;
    h->used = layout(h, workspace, nx, ny, nz, prec, smoother, epl, lean);
    h->ilu = ntd::ilu_grid(nx, ny, nz, 2);
    *out = h;
    return NTD_OK;
}

int handle_check(ntd_handle *h, const double *kappa, const double *t, hipStream_t s) {
    CK(hipMemsetAsync(h->flag, 0, 4 * sizeof(int), s));
    CK(hipMemsetAsync(h->sc, 0, sizeof(Scalars), s));
    CK(ntd::launch_check_positive(kappa, t, h->N, h->flag, s));
    return NTD_OK;
}

int handle_flag_async(const ntd_handle *h, int *flag, hipStream_t s) {
    CK(hipMemcpyAsync(flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, s));
    return NTD_OK;
}

int handle_assemble(ntd_handle *h, const double *kappa, const int *bc, hipStream_t s) {
    CK(ntd::launch_assemble(grid_of(h), kappa, bc, h->d, h->ax, h->ay, h->az, s));
    return NTD_OK;
}

ntd::SetupArgs handle_setup_args(const ntd_handle *h, const double *t) {
    ntd::SetupArgs a;
    a.nx = h->nx; a.ny = h->ny; a.nz = h->nz; a.schur = h->schur;
    a.d = h->d; a.ax = h->ax; a.ay = h->ay; a.az = h->az; a.t = t;
    a.dP = h->dP; a.xP = h->xP; a.f2 = h->f2; a.dT = h->dT; a.e1 = h->e1; a.mv = h->mv;
    a.scratch = (double *)h->scratch; a.flag = h->flag;
    return a;
}

int handle_finish(ntd_handle *h, hipStream_t s) {
    int st = pack_factors(h, s);
    if (st != NTD_OK) return st;
    // unused slots of the packed right-hand side are never written by the
    // packing of a right-hand side and must read as 0
    if (h->rp)
        CK(ntd::launch_fill((double *)h->rp, 0.0,
                             h->npack * (h->prec == NTD_PREC_FP64 ? 8 : 4) / 8, s));
    return NTD_OK;
}

int setup_handle(int nx, int ny, int nz, const double *kappa, const int *bc, const double *t,
                 int prec, int schur, int smoother, int epl, bool lean, void *workspace,
                 size_t workspace_bytes, hipStream_t s, ntd_handle **out) {
    if (out) *out = nullptr;
    if (!out || !kappa) return NTD_EINVAL;
    ntd_handle *h = nullptr;
    int st = handle_create(nx, ny, nz, bc, prec, schur, smoother, epl, lean, workspace,
                           workspace_bytes, &h);
    if (st != NTD_OK) return st;
    int hflag = 0;
#define FAIL(code) do { st = (code); goto fail; } while (0)
#define HK(expr) do { if ((expr) != hipSuccess) FAIL(NTD_EHIP); } while (0)
    if ((st = handle_check(h, kappa, t, s)) != NTD_OK) goto fail;
    if ((st = handle_flag_async(h, &hflag, s)) != NTD_OK) goto fail;
    HK(hipStreamSynchronize(s));
    if (hflag & ntd::kFlagBadInput) FAIL(NTD_EINVAL);
    if ((st = handle_assemble(h, kappa, bc, s)) != NTD_OK) goto fail;
    HK(ntd::launch_setup(handle_setup_args(h, t), h->epl, s));
    if (smoother != NTD_SMOOTHER_NONE)
        HK(ntd::launch_ilu_factor(h->ilu, h->d, h->ax, h->ay, h->az, h->dt, h->dtinv, h->flag, s));
    if (h->fcoef)
        HK(ntd::launch_ilu_coef_f32(h->ilu, h->ax, h->ay, h->az, h->dtinv, h->fcoef, s));
    if ((st = handle_flag_async(h, &hflag, s)) != NTD_OK) goto fail;
    HK(hipStreamSynchronize(s));
    if (hflag & ntd::kFlagNotSPD) FAIL(NTD_ENOTSPD);
    if ((st = handle_finish(h, s)) != NTD_OK) goto fail;
    HK(hipStreamSynchronize(s));
    *out = h;
    return NTD_OK;
fail:
    free(h);
    return st;
#undef FAIL
#undef HK
}

}  // namespace ntd_host

extern "C" {

size_t ntd_workspace_bytes(int nx, int ny, int nz, int prec, int smoother) {
    if (nx < 1) return 0;
    return ntd_host::handle_bytes(nx, ny, nz, prec, smoother, ntd::epl_for(nx), false);
}

int ntd_setup(int nx, int ny, int nz, const double *kappa, const int *bc, const double *t,
              int prec, int schur, int smoother, void *workspace, size_t workspace_bytes,
              void *stream, ntd_handle **out) {
    if (out) *out = nullptr;
    if (nx < 1) return NTD_EINVAL;
    return ntd_host::setup_handle(nx, ny, nz, kappa, bc, t, prec, schur, smoother,
                                  ntd::epl_for(nx), false, workspace, workspace_bytes,
                                  S(stream), out);
}

int ntd_apply_precond(ntd_handle *h, const double *r, double *z, void *stream) {
    if (!h || !r || !z || r == z) return NTD_EINVAL;
    return precond_internal(h, r, z, nullptr, nullptr, S(stream));
}

int ntd_apply_ntd(ntd_handle *h, const double *r, double *z, void *stream) {
    if (!h || !r || !z || r == z) return NTD_EINVAL;
    return ntd_solve_any(h, r, nullptr, z, nullptr, nullptr, S(stream), nullptr);
}

int ntd_apply_ilu0(ntd_handle *h, const double *r, double *z, void *stream) {
    if (!h || !r || !z || r == z || h->smoother == NTD_SMOOTHER_NONE) return NTD_EINVAL;
    return ilu_internal(h, r, z, S(stream));
}

int ntd_apply_profile(ntd_handle *h, const double *r, double *z, float *ms, void *stream) {
    if (!h || !r || !z || r == z || !ms) return NTD_EINVAL;
    hipStream_t s = S(stream);
    // ev[0]: start; ev[1..4] bracket the sweeps; ev[5]: end; ev[6]: spare
    hipEvent_t ev[7];
    int made = 0, st = NTD_OK, np = 0;
    for (; made < 7; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess) { st = NTD_EHIP; break; }
    // The preconditioner as the PCG loop launches it, r.z partials included.
    if (st == NTD_OK) st = precond_internal(h, r, z, h->partials, &np, s, ev);
    if (st == NTD_OK && hipEventSynchronize(ev[5]) != hipSuccess) st = NTD_EHIP;
    for (int i = 0; st == NTD_OK && i < 3; ++i)
        if (hipEventElapsedTime(&ms[i], ev[i + 1], ev[i + 2]) != hipSuccess) st = NTD_EHIP;
    float pre = 0.0f, post = 0.0f;
    if (st == NTD_OK && (hipEventElapsedTime(&pre, ev[0], ev[1]) != hipSuccess ||
                         hipEventElapsedTime(&post, ev[4], ev[5]) != hipSuccess))
        st = NTD_EHIP;
    ms[3] = pre + post;
    for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    return st;
}

int ntd_spmv(ntd_handle *h, const double *x, double *y, void *stream) {
    if (!h || !x || !y || x == y) return NTD_EINVAL;
    ntd::Grid g = grid_of(h);
    CK(ntd::launch_spmv(g, h->d, h->ax, h->ay, h->az, x, y, nullptr, nullptr, S(stream)));
    return NTD_OK;
}

int ntd_dot(ntd_handle *h, const double *x, const double *y, double *result, void *stream) {
    if (!h || !x || !y || !result) return NTD_EINVAL;
    hipStream_t s = S(stream);
    int np = 0;
    CK(ntd::launch_dot(x, y, h->N, h->partials, &np, s));
    CK(ntd::launch_finalize(h->partials, np, h->sc, ntd::kOpResult, s));
    Scalars hs;
    int st = read_scalars(h, &hs, s);
    if (st != NTD_OK) return st;
    *result = hs.result;
    return NTD_OK;
}

int ntd_pcg_solve(ntd_handle *h, const double *b, double *x, double tol, int maxit, int *iters,
                  double *relres, void *stream) {
    return ntd_pcg_solve_history(h, b, x, tol, maxit, iters, relres, nullptr, stream);
}

int ntd_pcg_solve_history(ntd_handle *h, const double *b, double *x, double tol, int maxit,
                          int *iters, double *relres, double *hist, void *stream) {
    return ntd_pcg_solve_progress(h, b, x, tol, maxit, iters, relres, hist, 0, nullptr, nullptr,
                                  stream);
}

int ntd_pcg_solve_progress(ntd_handle *h, const double *b, double *x, double tol, int maxit,
                           int *iters, double *relres, double *hist, int every,
                           ntd_progress_fn progress, void *ctx, void *stream) {
    if (!h || !b || !x || b == x || !iters || !relres) return NTD_EINVAL;
    if (!(tol > 0.0) || maxit < 1 || every < 0 || (progress && every < 1)) return NTD_EINVAL;
    hipStream_t s = S(stream);
    const long long N = h->N;
    ntd::Grid g = grid_of(h);
    *iters = 0;
    *relres = 0.0;
    int st, np = 0;
    double bb = 0.0;
    CK(hipMemsetAsync(h->sc, 0, sizeof(Scalars), s));
    if ((st = norm2(h, b, &bb, s)) != NTD_OK) return st;
    const double bn = sqrt(bb);
    CK(ntd::launch_fill(x, 0.0, N, s));
    CK(ntd::launch_copy(h->r, b, N, s));
    if (bn == 0.0) {
        CK(hipStreamSynchronize(s));
        return NTD_OK;
    }
    if ((st = precond_internal(h, h->r, h->z, h->partials, &np, s)) != NTD_OK) return st;
    CK(ntd::launch_finalize(h->partials, np, h->sc, ntd::kOpRhoInit, s));
    CK(ntd::launch_copy(h->p, h->z, N, s));
    int it = 0, status = NTD_OK;
    Scalars hs;
    for (;;) {
        if (it >= maxit) { status = NTD_ENOCONV; break; }
        CK(ntd::launch_spmv(g, h->d, h->ax, h->ay, h->az, h->p, h->q, h->partials, &np, s));
        CK(ntd::launch_finalize(h->partials, np, h->sc, ntd::kOpAlpha, s));
        CK(ntd::launch_axpy2_norm(x, h->r, h->p, h->q, h->sc, N, h->partials, &np, s));
        CK(ntd::launch_finalize(h->partials, np, h->sc, ntd::kOpRR, s));
        if ((st = read_scalars(h, &hs, s)) != NTD_OK) return st;
        if (hs.flag & (ntd::kFlagPqBreakdown | ntd::kFlagRhoBreakdown)) {
            status = NTD_EBREAKDOWN;
            break;
        }
        ++it;
        if (hist) hist[it - 1] = sqrt(hs.rr) / bn;
        if (progress && it % every == 0) progress(it, sqrt(hs.rr) / bn, ctx);
        if (sqrt(hs.rr) / bn <= tol) {
            double tr = 0.0;
            if ((st = true_relres(h, b, x, bn, &tr, s)) != NTD_OK) return st;
            if (tr <= tol) break;
        }
        if ((st = precond_internal(h, h->r, h->z, h->partials, &np, s)) != NTD_OK) return st;
        CK(ntd::launch_finalize(h->partials, np, h->sc, ntd::kOpBeta, s));
        CK(ntd::launch_xpay(h->p, h->z, h->sc, N, s));
    }
    *iters = it;
    if ((st = true_relres(h, b, x, bn, relres, s)) != NTD_OK) return st;
    return status;
}

int ntd_export(const ntd_handle *h, int which, double *dst, void *stream) {
    if (!h || !dst) return NTD_EINVAL;
    const double *src[] = {h->d, h->ax, h->ay, h->az, h->e1, h->mv, h->f2, h->dT, h->dP, h->xP, h->dt};
    if (which < 0 || which >= (int)(sizeof(src) / sizeof(src[0])) || !src[which]) return NTD_EINVAL;
    CK(hipMemcpyAsync(dst, src[which], sizeof(double) * h->N, hipMemcpyDeviceToDevice,
                      S(stream)));
    return NTD_OK;
}

int ntd_load_factors(ntd_handle *h, const double *e1, const double *pivots, const double *f2,
                     void *stream) {
    if (!h || !e1 || !pivots || !f2) return NTD_EINVAL;
    hipStream_t s = S(stream);
    CK(ntd::launch_copy(h->e1, e1, h->N, s));
    CK(ntd::launch_recip(h->mv, pivots, h->N, s));
    CK(ntd::launch_copy(h->f2, f2, h->N, s));
    return pack_factors(h, s);
}

size_t ntd_footprint_bytes(const ntd_handle *h) { return h ? h->used : 0; }

int ntd_destroy(ntd_handle *h) {
    free(h);
    return NTD_OK;
}

const char *ntd_strerror(int status) {
    switch (status) {
    case NTD_OK: return "ok";
    case NTD_EINVAL: return "invalid argument";
    case NTD_ENOMEM: return "host allocation failed";
    case NTD_ENOTSPD: return "factorization pivot not positive";
    case NTD_EBREAKDOWN: return "PCG breakdown (p'Ap or r'z not positive)";
    case NTD_ENOCONV: return "PCG did not converge within maxit";
    case NTD_EHIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

}  // extern "C"
