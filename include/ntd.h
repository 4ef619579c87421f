/*
 * ntd.h -- C ABI of the MI355X (gfx950) library for the nested, twisted
 * frequency-filtering preconditioned conjugate gradient method of
 * Aggarwal, Kakkar and Kumar, arXiv:1909.09771 ("NTD").
 *
 * Problem (Sec. 1, eq. diffeqn): -div(kappa grad u) = f on a structured
 * nx x ny x nz grid, u = 0 on Dirichlet faces, du/dn = 0 on Neumann faces,
 * discretised by the 7-point finite-difference stencil.  The matrix A is the
 * nested block tridiagonal matrix of Sec. 2 (planes -> lines -> points).
 *
 * Layout of every grid vector: FP64, x fastest, C-contiguous [nz][ny][nx],
 * unknown p = i + nx*(j + ny*k).  Unless a comment says "host", every pointer
 * is a DEVICE pointer on the current HIP device and stays owned by the caller.
 * `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *
 * Error behaviour: every entry point returns an int status (NTD_OK = 0 or one
 * of the codes below); nothing throws across the ABI and nothing aborts.  On
 * an error the output buffers are unspecified unless stated otherwise.
 *
 * Threading: a handle must not be used from two host threads or two streams
 * at the same time; distinct handles are independent.
 */
#ifndef NTD_H
#define NTD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ntd_handle ntd_handle;

/* Status codes. */
#define NTD_OK 0
#define NTD_EINVAL 1       /* bad argument: size, pointer, workspace, kappa or t not finite > 0, ... */
#define NTD_ENOMEM 2       /* host-side allocation failed */
#define NTD_ENOTSPD 3      /* a pivot of the factorization is not positive and finite */
#define NTD_EBREAKDOWN 4   /* PCG: p'Ap or r'z not positive, or not finite */
#define NTD_ENOCONV 5      /* PCG: maxit reached before the tolerance */
#define NTD_EHIP 6         /* a HIP runtime call failed */

/* Boundary type of a face; faces are ordered x-, x+, y-, y+, z-, z+. */
#define NTD_BC_DIRICHLET 0
#define NTD_BC_NEUMANN 1

/* Arithmetic of the preconditioner.  FP64: factors and sweeps in double.
 * MIXED: factors rounded to float after an FP64 setup and sweeps in float,
 * except the twist (meeting) row of every line, whose pivot and update stay in
 * double; with an ILU(0) smoother its sweeps read the couplings and 1/dt
 * rounded to float and compute in double.  CG vectors, SpMV, dot products and
 * residual updates are always FP64. */
#define NTD_PREC_FP64 0
#define NTD_PREC_MIXED 1

/* Approximate Schur block of a neighbour block (Sec. 2.1).
 * NEWTON: 2b - b P b with b = diag((Pt^{-1} w)./w), w = coupling .* t (the
 *   paper's formula), plus a diagonal compensation at the plane level so that
 *   B t = A t holds exactly although the inner plane solve is approximate.
 * DIAG: the diagonal b itself (classical tangential filtering); filter-exact
 *   without compensation.  Both give an SPD B whenever every pivot is > 0. */
#define NTD_SCHUR_NEWTON 0
#define NTD_SCHUR_DIAG 1

/* Smoother combined with B (Sec. 3, eq. com): none, or ILU(0) of the
 * block-diagonal approximation blkD(A(1:M,1:M), A(M+1:N,M+1:N)), M = floor(N/2),
 * giving the combination Bc^{-1} = B^{-1} + B_ILU^{-1} - B^{-1} A B_ILU^{-1}
 * (the preconditioner of the paper's experiments, Table 1). */
#define NTD_SMOOTHER_NONE 0
#define NTD_SMOOTHER_ILU0 1
/* Symmetric combination (an addition to the paper): z1 = B_ILU^{-1} r,
 * z2 = z1 + B^{-1}(r - A z1), z = z2 + B_ILU^{-1}(r - A z2).  B and B_ILU are
 * symmetric, so this preconditioner is symmetric, which CG assumes; the
 * combination of eq. com is not, and CG with it diverges on high-contrast
 * inclusions.  Costs one more ILU(0) solve and one more SpMV per application. */
#define NTD_SMOOTHER_ILU0_SYM 2

/* Largest supported line length nx (one wavefront solves one line).  The
 * grid must also satisfy 8*nx*ny*nz < 2^31 (32-bit byte offsets). */
#define NTD_MAX_NX 1024

/* Bytes of device workspace that ntd_setup needs for this grid, precision and
 * smoother.  Returns 0 for invalid arguments. */
size_t ntd_workspace_bytes(int nx, int ny, int nz, int prec, int smoother);

/* Assemble A from kappa and the face types, then factor B (Sec. 2.1: the
 * level-3 plane recurrence, the level-2 line recurrence of every plane, the
 * level-1 twisted pivots of every line) and, with the ILU(0) smoother, the
 * block-diagonal ILU(0) (Sec. 3).
 *   kappa     [N] device, finite and > 0
 *   bc        [6] HOST, NTD_BC_* per face; at least one Dirichlet face
 *   t         [N] device filter vector, finite and > 0, or NULL for t = 1
 *             (the rowsum filter, eq. rowsum); B depends only on its direction
 *   prec      NTD_PREC_*; schur NTD_SCHUR_*; smoother NTD_SMOOTHER_*
 *   workspace device buffer of >= ntd_workspace_bytes() bytes, 256-byte
 *             aligned, owned by the caller and used by the handle until
 *             ntd_destroy; its contents need no initialisation
 * Synchronises `stream`.  On success *out receives a new handle; on failure
 * *out = NULL (NTD_ENOTSPD if a pivot is not positive). */
int ntd_setup(int nx, int ny, int nz, const double *kappa, const int *bc, const double *t,
              int prec, int schur, int smoother, void *workspace, size_t workspace_bytes,
              void *stream, ntd_handle **out);

/* z = (the handle's preconditioner)^{-1} r: B^{-1} r, or with the ILU(0)
 * smoother the combination of eq. com, or the symmetric combination
 * (NTD_SMOOTHER_ILU0_SYM).  r and z are [N] device FP64 and must
 * not overlap.  Stream-ordered, asynchronous. */
int ntd_apply_precond(ntd_handle *h, const double *r, double *z, void *stream);

/* z = B^{-1} r alone (Sec. 2.2, Algorithms 1-7: level-3 twisted block sweeps
 * over planes, each plane block solved by level-2 sweeps over lines, each line
 * by the exact twisted tridiagonal solve).  Same conventions. */
int ntd_apply_ntd(ntd_handle *h, const double *r, double *z, void *stream);

/* z = B_ILU^{-1} r alone (forward and backward sweeps of the block-diagonal
 * ILU(0)); NTD_EINVAL if the handle has no smoother.  Same conventions. */
int ntd_apply_ilu0(ntd_handle *h, const double *r, double *z, void *stream);

/* Same as ntd_apply_precond (launched exactly as inside ntd_pcg_solve, with
 * the fused r.z partials), but synchronous; ms[0..3] (HOST) receive durations
 * in milliseconds measured with HIP events on `stream`: ms[0..2] the three
 * sweep launches (lower level-3 sweep of the two half chains, twist plane,
 * upper level-3 sweep), ms[3] the rest of the application: the ILU(0) sweeps
 * when the handle has the smoother, the packing of the right-hand side into
 * the sweep layout (with r - A zi fused in when there is a smoother) and the
 * unpacking of the result to FP64 (with the r.z partials), and with the
 * symmetric smoother its third stage (SpMV, ILU(0) sweeps, update).  For
 * benchmarking. */
int ntd_apply_profile(ntd_handle *h, const double *r, double *z, float *ms, void *stream);

/* y = A x with the assembled 7-point bands.  [N] device FP64, no overlap.
 * Stream-ordered, asynchronous. */
int ntd_spmv(ntd_handle *h, const double *x, double *y, void *stream);

/* *result (HOST) = x . y over the N entries, FP64, fixed summation order
 * (bitwise reproducible run to run).  Synchronises `stream`. */
int ntd_dot(ntd_handle *h, const double *x, const double *y, double *result, void *stream);

/* ntd_dot without a handle and without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  *result (DEVICE, one double) =
 * x . y over n entries (x, y [n] device FP64), in the same summation order as
 * ntd_dot, so the two agree bitwise on the same vectors.  Stream-ordered and
 * asynchronous (nothing synchronises), so it can be captured.
 * Scratch: a fixed static device array per GPU (2048 block partial sums and
 * one 64-byte scalar record, 16.4 KiB), held until the process ends; its use
 * does not grow with n.  n must lie in [0, NTD_DOT_NOALLOC_MAX_N], else
 * NTD_EINVAL.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (two streams, or two host threads) race and must be
 * ordered by the caller.  The current device must be the device of x, y,
 * result and stream.  Allocates nothing; returns NTD_EHIP if a launch fails. */
#define NTD_DOT_NOALLOC_MAX_N (1LL << 50)
int ntd_dot_noalloc(const double *x, const double *y, long long n, double *result, void *stream);

/* Preconditioned CG for A x = b (Sec. 1; stopping rule of Sec. 3): x0 = 0,
 * iterate until ||r||/||b|| <= tol on the recursively updated residual and the
 * true residual ||b - A x||/||b|| confirms it.  b, x [N] device FP64.
 * *iters (HOST) = products with A taken in the loop; *relres (HOST) = final
 * true relative residual.  Returns NTD_ENOCONV after maxit iterations and
 * NTD_EBREAKDOWN when p'Ap or r'z is not positive and finite (r'z can turn
 * non-positive with the non-symmetric combination of eq. com); x then holds
 * the last iterate.  Synchronises. */
int ntd_pcg_solve(ntd_handle *h, const double *b, double *x, double tol, int maxit, int *iters,
                  double *relres, void *stream);

/* ntd_pcg_solve that also records the recursively updated relative residual
 * ||r||/||b|| after every iteration: hist (HOST, maxit doubles, may be NULL)
 * receives entries 0..*iters-1. */
int ntd_pcg_solve_history(ntd_handle *h, const double *b, double *x, double tol, int maxit,
                          int *iters, double *relres, double *hist, void *stream);

/* Progress callback of ntd_pcg_solve_progress: iteration count and recursive
 * relative residual ||r||/||b|| after that iteration, and the caller's ctx. */
typedef void (*ntd_progress_fn)(int iteration, double relres, void *ctx);

/* ntd_pcg_solve_history that also calls progress(it, ||r||/||b||, ctx) on the
 * calling host thread after every `every`-th iteration (every >= 1 when
 * progress is not NULL; progress NULL: no calls).  The loop already reads its
 * scalars back every iteration, so the calls change neither the iterates nor
 * the number of synchronisations; they let a long solve report as it goes.
 * The callback must not call into this handle. */
int ntd_pcg_solve_progress(ntd_handle *h, const double *b, double *x, double tol, int maxit,
                           int *iters, double *relres, double *hist, int every,
                           ntd_progress_fn progress, void *ctx, void *stream);

/* Filter-vector target from the handle's own preconditioner (Sec. 1: the
 * error components that the filtered iteration (I - B^{-1}A)^n damps slowest
 * are the eigenvectors of B^{-1}A of smallest eigenvalue).  Inverse iteration
 * on M = B^{-1}A (B as set up, without smoother): `outer` times,
 * y = M^{-1} v by conjugate gradients in the A-inner product (M is self-adjoint
 * and positive definite there; one B^{-1} application and one product with A
 * per step) to ||v - M y||_A <= inner_tol ||v||_A, then v = y / (the entry of
 * y of largest magnitude); each solve starts at y = 0.  On return
 * v = max(v, floor).
 * v: [N] device FP64, the start vector in, the target out.  The start must
 * carry components along the eigenvector sought: t = 1 (the handle's own filter
 * vector when set up with t = NULL) is itself an eigenvector of B^{-1}A with
 * eigenvalue 1 (B t = A t), and the iteration would stay there.  work: [7 N] device FP64 scratch owned by the caller.  *inner_iters
 * (HOST): CG steps over all outer iterations; *lambda (HOST): v'Av / y'Av of
 * the last step, the estimate of the smallest eigenvalue of B^{-1}A.
 * Returns NTD_ENOCONV if an inner solve misses inner_tol in inner_maxit
 * steps, NTD_EBREAKDOWN on a non-positive curvature.  Synchronises. */
int ntd_filter_target(ntd_handle *h, double *v, int outer, double inner_tol, int inner_maxit,
                      double floor, double *work, int *inner_iters, double *lambda, void *stream);

/* v[0..n) <- max(v / m, floor), m = the entry of v of largest magnitude (the
 * first one on ties), so that the largest entry becomes +1; floor <= -1 leaves
 * the scaled vector unclipped.  partials: [2048] device FP64 scratch owned by
 * the caller; *scale (HOST) = 1/m.  NTD_EINVAL if v is zero or not finite.
 * Synchronises. */
int ntd_vec_normalize(double *v, long long n, double floor, double *partials, double *scale,
                      void *stream);

/* Copy an internal array of the handle into dst ([N] device FP64), for tests
 * and diagnostics.  which: 0..3 = bands d, ax, ay, az of A; 4 = e1 (x-band of
 * the line blocks T); 5 = 1/pivot of T; 6 = f2 (y-band of the plane blocks P);
 * 7 = diagonal of T; 8 = diagonal of P; 9 = x-band of P; 10 = diagonal of the
 * ILU(0) factor (smoother only). Stream-ordered. */
int ntd_export(const ntd_handle *h, int which, double *dst, void *stream);

/* Replace the factors of the handle by given FP64 ones (e1, pivots M -- not
 * their inverse --, f2; [N] device each), e.g. those of a reference setup, so
 * that the apply can be checked on its own.  MIXED handles re-round them to
 * float.  Stream-ordered. */
int ntd_load_factors(ntd_handle *h, const double *e1, const double *pivots, const double *f2,
                     void *stream);

/* Device bytes the handle keeps in use inside its workspace. */
size_t ntd_footprint_bytes(const ntd_handle *h);

/* Release the host-side state of the handle (not the caller's workspace). */
int ntd_destroy(ntd_handle *h);

/* ---------------------------------------------------------------------------
 * Batches: many independent systems, each with several right-hand sides,
 * preconditioned with B (Sec. 2; no smoother) and solved together.  Every
 * launch of a batched step covers all right-hand sides of the batch, so the
 * sweeps of B run as 4 * count * nrhs independent chains at once instead of 4.
 * A batch entry computes the same operators as the single-system entry points
 * for its system, up to rounding (its lines may carry pass-through slots, see
 * ntd_batch_setup).
 * ------------------------------------------------------------------------- */
typedef struct ntd_batch ntd_batch;

/* Most systems in one batch, most right-hand sides per system, and the
 * longest line (the batched sweeps cover up to 8 elements per lane). */
#define NTD_BATCH_MAX_SYSTEMS 4096
#define NTD_BATCH_MAX_RHS 16
#define NTD_BATCH_MAX_NX 512

/* Flags of ntd_batch_pcg_solve. */
#define NTD_BATCH_GRAPH 1  /* run the iterations as replays of one captured HIP graph */

/* Bytes of device workspace for a batch of `count` systems with grid sizes
 * dims[3*s + 0..2] = (nx, ny, nz) (HOST) and nrhs right-hand sides each.
 * Returns 0 for invalid arguments. */
size_t ntd_batch_workspace_bytes(int count, const int *dims, int nrhs, int prec);

/* Set up every system of a batch as ntd_setup would (smoother none):
 *   dims   [3*count] HOST grid sizes; nx <= NTD_BATCH_MAX_NX
 *   kappa  [count] HOST array of device pointers, kappa[s] of N_s values
 *   bc     [6*count] HOST face types, 6 per system
 *   nrhs   1..NTD_BATCH_MAX_RHS; prec NTD_PREC_*; schur NTD_SCHUR_*
 *   workspace device buffer of >= ntd_batch_workspace_bytes(), 256-byte
 *          aligned, owned by the caller until ntd_batch_destroy
 * Every system of the batch is packed with the elements per lane of its
 * longest line (shorter lines carry pass-through slots), so that one launch
 * runs all of them.  Synchronises `stream`.  On failure *out = NULL and the
 * status of the first failing system is returned. */
int ntd_batch_setup(int count, const int *dims, const double *const *kappa, const int *bc,
                    int nrhs, int prec, int schur, void *workspace, size_t workspace_bytes,
                    void *stream, ntd_batch **out);

/* z[e] = B_s^{-1} r[e] for every entry e = s*nrhs + q (system s, right-hand
 * side q).  r, z: [count*nrhs] HOST arrays of device pointers to [N_s] FP64
 * vectors; r[e] and z[e] must not overlap.  Stream-ordered, asynchronous. */
int ntd_batch_apply(ntd_batch *b, const double *const *r, double *const *z, void *stream);

/* As ntd_batch_apply, but synchronous, with ms[0..3] (HOST) the durations in
 * milliseconds of the lower sweep, the twist planes, the upper sweep and the
 * rest (packing and unpacking), measured with HIP events on `stream`. */
int ntd_batch_apply_profile(ntd_batch *b, const double *const *r, double *const *z, float *ms,
                            void *stream);

/* PCG for every entry (rules of ntd_pcg_solve, applied per entry): rhs[e] and
 * x[e] as r and z above; iters, relres, status: [count*nrhs] HOST outputs per
 * entry (iterations, final true relative residual, NTD_OK / NTD_ENOCONV /
 * NTD_EBREAKDOWN).  Every entry keeps its scalars on the device and stops on
 * its own; the host checks the batch between runs of iterations.  flags:
 * NTD_BATCH_GRAPH or 0.  Returns NTD_OK when the batch ran (per-entry outcomes
 * are in status) or an error.  Synchronises `stream`. */
int ntd_batch_pcg_solve(ntd_batch *b, const double *const *rhs, double *const *x, double tol,
                        int maxit, int flags, int *iters, double *relres, int *status,
                        void *stream);

/* Statistics of the batch's last ntd_batch_pcg_solve (HOST outputs): passes =
 * runs of iterations between host checks of the entries' active flags;
 * gap_ms = time the stream spent between the end of a run and the start of
 * the next (the host's read of the flags and its decision), summed over the
 * solve; solve_ms = the iterations' time from the first run to the end, both
 * measured with HIP events on the solve's stream. */
int ntd_batch_solve_stats(const ntd_batch *b, int *passes, double *gap_ms, double *solve_ms);

/* Device bytes the batch keeps in use inside its workspace. */
size_t ntd_batch_footprint_bytes(const ntd_batch *b);

/* Autotune the launch shape of the batch's bandwidth kernels (SpMV, vector
 * updates, packing of the right-hand sides and unpacking of the results): time
 * one round of them, on zero-filled vectors, for 1, 1/2, 1/4 and 1/8 of the
 * workgroups per entry that the setup sized (one per 1024 points of the
 * largest system, at most 512), and keep the fastest; *gx (HOST) receives
 * it.  Until it is called the sized maximum is used, so results are bitwise
 * repeatable run to run; a tuned batch is repeatable with the same choice (the
 * reductions are fixed-order for a given count).  Discards a captured
 * iteration graph.  Synchronises `stream`; must not overlap a solve. */
int ntd_batch_tune(ntd_batch *b, int *gx, void *stream);

/* Right-hand sides per wavefront pair in the batch's line sweeps.  nr = 1
 * (the default): one wavefront pair per right-hand side, each reading its
 * system's line records.  nr = 2 or 4: one pair runs nr right-hand sides of one
 * system through the same chain and reads each line record once for all of
 * them (nr must divide nrhs; nr = 2 for lines of up to 256 points in MIXED and
 * 128 in FP64, nr = 4 for up to 128 in MIXED and 64 in FP64).  Results are the
 * same operations as with nr = 1 (bitwise).  Returns NTD_EINVAL for an
 * unsupported nr.  Discards a captured iteration graph if nr changes. */
int ntd_batch_set_sweep_group(ntd_batch *b, int nr);

/* Plane buffers of the batch's line sweeps in LDS (on = 1, the default) or in
 * device memory (on = 0).  Each level-3 step hands a plane to the next: the
 * finished neighbour plane, the level-2 lower results and the plane's final
 * values.  With on = 1 each workgroup keeps that plane in its own LDS, so it
 * passes through no memory.  Only the final results and the right-hand sides
 * still move through HBM.  This is used when the device can hold every
 * workgroup of a sweep at once with its nr buffers (ntd_batch_set_sweep_group)
 * of (2 + ny_max) * 64 * epl values each.  For example, 64 systems at 128^3
 * with 4 right-hand sides in MIXED need 65 KB per workgroup at nr = 1 (two
 * workgroups per CU) and 130 KB at nr = 2 (one per CU).
 * Results are bitwise the same either way.  *used (HOST, may be NULL) is set to
 * 1 when the sweeps will use the LDS buffers.  Returns NTD_EINVAL for on
 * other than 0 or 1.  Discards a captured iteration graph if on changes. */
int ntd_batch_set_plane_lds(ntd_batch *b, int on, int *used);

/* Autotune the line-sweep shape: time one batched sweep (on zero right-hand
 * sides) for every supported right-hand sides per wavefront pair (1, 2, 4) and
 * keep the fastest; *nr (HOST) receives it.  Overwrites the batch's CG vectors
 * and packed right-hand sides.  Synchronises `stream`; must not overlap a solve. */
int ntd_batch_tune_sweeps(ntd_batch *b, int *nr, void *stream);

/* Release the host-side state of the batch (not the caller's workspace). */
int ntd_batch_destroy(ntd_batch *b);

/* ------------------------------------------------------------------------
 * Learned filter vector (Sec. 1: B(t) t = A t, and a t close to A's lowest
 * eigenvectors treats that end of the spectrum best; t = 1 is the rowsum
 * choice).  A 3D convolutional network predicts t from kappa:
 *   H0 = bf16((log10 kappa - mean(log10 kappa)) / 3)          1 channel
 *   H_l = relu(conv_l(H_{l-1})), l = 1..3                      16 channels
 *   y = conv_4(H3);  t = softplus(y) + 1e-3                    1 channel
 * conv_l is a 3x3x3 cross-correlation with zero padding plus a bias, taken on
 * bfloat16 operands with float32 accumulation (matrix cores).
 *
 * Parameters: NTD_CNN_NPARAMS floats (device), per layer W[cout][tap][cin]
 * then b[cout], tap = 9 (dz+1) + 3 (dy+1) + (dx+1) for the neighbour
 * (z+dz, y+dy, x+dx); layers (cin, cout) = (1,16), (16,16), (16,16), (16,1).
 * Fields are [nz][ny][nx] as everywhere else; 1 <= nx*ny*nz <= 2^28.
 * The workspace (device, caller-owned, 256-byte aligned) holds activations,
 * gradient maps and packed weights: about 168 bytes per voxel + 7 MB.
 * ------------------------------------------------------------------------ */
#define NTD_CNN_NPARAMS 14737

/* Bytes of workspace for one grid (0 if the grid is out of range). */
size_t ntd_cnn_workspace_bytes(int nx, int ny, int nz);

/* t = the network's filter vector for kappa (FP64 [N]); if y is not NULL it
 * also receives the output before the softplus (float [N]).  Checks kappa
 * (finite and > 0, else NTD_EINVAL) with one read-back, so it synchronises the
 * stream once; the rest is stream-ordered. */
int ntd_cnn_predict(int nx, int ny, int nz, const double *kappa, const float *params, double *t,
                    float *y, void *workspace, size_t ws_bytes, void *stream);

/* *loss (host) = mean over the grid of (t - target)^2 and grad (device, float
 * [NTD_CNN_NPARAMS], same layout as params) = its gradient, with every
 * back-propagated map rounded to bfloat16 as the forward activations are.
 * Synchronises the stream (it returns the loss). */
int ntd_cnn_loss_grad(int nx, int ny, int nz, const double *kappa, const double *target,
                      const float *params, float *grad, double *loss, void *workspace,
                      size_t ws_bytes, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; `step`
 * counts from 1) on params with the moment vectors m and v (device, float
 * [NTD_CNN_NPARAMS] each, zero before step 1).  Stream-ordered. */
int ntd_cnn_adam(float *params, float *m, float *v, const float *grad, int step, float lr,
                 void *stream);

/* Static text for a status code. */
const char *ntd_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* NTD_H */
