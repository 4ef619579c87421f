// ntd_internal.h -- shared declarations of the HIP library behind include/ntd.h.
// Grid vectors are x-fastest [nz][ny][nx]; p = i + nx*(j + ny*k).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ntd {

// Scalars of one PCG solve, kept on the device so that a step never waits for
// the host except for the single convergence read per iteration.
struct Scalars {
    double rho;    // r.z of the current iterate
    double pq;     // p.Ap
    double alpha;  // rho / pq
    double beta;   // rho_new / rho
    double rr;     // r.r
    double result; // generic reduction result (ntd_dot, norms)
    int flag;      // bit 0: breakdown (pq <= 0 or not finite)
    int pad;
};

// Reduction partial slots: vector kernels write one partial per block (at most
// kMaxBlocks); the preconditioner apply writes kApplySlots per-wave partials.
constexpr int kMaxBlocks = 2048;
constexpr int kApplySlots = 8;
constexpr int kBlock = 256;

enum FinalizeOp : int {
    kOpResult = 0,  // result = sum
    kOpAlpha = 1,   // pq = sum; alpha = rho / pq; flag on breakdown
    kOpRR = 2,      // rr = sum
    kOpRhoInit = 3, // rho = sum
    kOpBeta = 4,    // beta = sum / rho; rho = sum
};

// Device error flags (int, OR-ed by kernels).
constexpr int kFlagBadInput = 1;   // kappa or t not finite and > 0
constexpr int kFlagNotSPD = 2;     // a pivot not positive and finite

struct Grid {
    int nx, ny, nz;
    long long nxy, N;
};

// Packed ("lane order") layout of the apply: every grid line (nx elements) is
// stored as 64*EPL slots, slot lane*EPL + s holding the element that lane's
// position s solves (lanes 0-31: elements 0..j, lanes 32-63: elements nx-1 down
// to j+1, j = floor((nx-1)/2), both right-aligned in their half); unused slots
// hold identity values.  Line L = k*ny + m starts at slot L*64*EPL.

// Arguments of the nested sweeps (apply) in the sweep precision T.
template <typename T>
struct ApplyArgs {
    int nx, ny, nz;
    const T *pmv, *pa, *pu;       // packed 1/M, a = -cp/M, u = -cn/M
    const T *pf2, *pg3;           // packed y-band of P and z-band of A
    const double *tw;             // per line: 1/M_j, e1[j-1], e1[j], 0 (FP64 twist row)
    const double *r;              // right-hand side (FP64, natural layout)
    T *Z;                         // packed intermediate / final result
    double *zout;                 // final result (FP64, natural layout)
    T *scratch;                   // two packed plane buffers (one per half chain)
    double *partials;             // kApplySlots partial sums of rdot.z (may be null)
    const double *zbase;          // if not null, the output is zbase + B^{-1} r
    const double *rdot;           // vector dotted with the output (null: r)
};

// Geometry of the ILU(0) level schedule: rows split at M (nblocks = 2) or not.
struct IluGrid {
    int nx, ny, nz, nblocks;
    long long nxy, N, M;
    int kz;       // plane of row M (start plane of the second block's level frame)
    int levels;   // number of hyperplane levels
};

// Arguments of the packing of FP64 natural-layout factors into the apply layout.
template <typename T>
struct PackArgs {
    int nx;
    long long nlines;             // ny*nz
    const double *e1, *mv, *f2, *g3;
    T *pmv, *pa, *pu, *pf2, *pg3;
    double *tw;
};

// Arguments of the factorization.
struct SetupArgs {
    int nx, ny, nz, schur;
    const double *d, *ax, *ay, *az, *t;  // bands of A; t may be null (t = 1)
    double *dP, *xP, *f2;                // bands of the plane blocks P
    double *dT, *e1, *mv;                // diagonal, x-band and 1/pivot of the line blocks T
    double *scratch;                     // 3 x 2 plane-sized buffers (w, z per block)
    int *flag;
};

// Host-side launchers (defined in the .hip files).
int epl_for(int nx);  // elements per lane of a half-wave chain, 0 if unsupported
hipError_t launch_apply_f64(const ApplyArgs<double> &a, int epl, hipStream_t s, hipEvent_t *ev);
hipError_t launch_apply_f32(const ApplyArgs<float> &a, int epl, hipStream_t s, hipEvent_t *ev);
hipError_t launch_setup(const SetupArgs &a, int epl, hipStream_t s);
hipError_t launch_pack_f64(const PackArgs<double> &p, int epl, hipStream_t s);
hipError_t launch_pack_f32(const PackArgs<float> &p, int epl, hipStream_t s);

IluGrid ilu_grid(int nx, int ny, int nz, int nblocks);
hipError_t launch_ilu_factor(const IluGrid &g, const double *d, const double *ax, const double *ay,
                             const double *az, double *dt, double *dtinv, int *flag,
                             hipStream_t s);
hipError_t launch_ilu_apply(const IluGrid &g, const double *ax, const double *ay, const double *az,
                            const double *dtinv, const double *r, double *z, hipStream_t s);
hipError_t launch_spmv_residual(const Grid &g, const double *d, const double *ax, const double *ay,
                                const double *az, const double *x, const double *b, double *out,
                                hipStream_t s);

hipError_t launch_check_positive(const double *kappa, const double *t, long long N, int *flag,
                                 hipStream_t s);
hipError_t launch_assemble(const Grid &g, const double *kappa, const int *bc, double *d,
                           double *ax, double *ay, double *az, hipStream_t s);
hipError_t launch_spmv(const Grid &g, const double *d, const double *ax, const double *ay,
                       const double *az, const double *x, double *y, double *partials,
                       int *nparts, hipStream_t s);
hipError_t launch_dot(const double *x, const double *y, long long N, double *partials,
                      int *nparts, hipStream_t s);
hipError_t launch_finalize(const double *partials, int nparts, Scalars *sc, int op, hipStream_t s);
hipError_t launch_axpy2_norm(double *x, double *r, const double *p, const double *q,
                             const Scalars *sc, long long N, double *partials, int *nparts,
                             hipStream_t s);
hipError_t launch_xpay(double *p, const double *z, const Scalars *sc, long long N, hipStream_t s);
hipError_t launch_residual(double *out, const double *b, const double *Ax, long long N,
                           hipStream_t s);
hipError_t launch_fill(double *x, double v, long long N, hipStream_t s);
hipError_t launch_copy(double *dst, const double *src, long long N, hipStream_t s);
hipError_t launch_cast_f32(float *dst, const double *src, long long N, hipStream_t s);
hipError_t launch_recip(double *dst, const double *src, long long N, hipStream_t s);

}  // namespace ntd
