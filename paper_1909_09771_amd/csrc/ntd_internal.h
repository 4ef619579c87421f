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
    int flag;      // kFlagPqBreakdown | kFlagRhoBreakdown
    int pad;
};

// Reduction partial slots: vector kernels write one partial per block (at most
// kMaxBlocks).
constexpr int kMaxBlocks = 2048;
constexpr int kBlock = 256;

enum FinalizeOp : int {
    kOpResult = 0,  // result = sum
    kOpAlpha = 1,   // pq = sum; alpha = rho / pq; flag on breakdown
    kOpRR = 2,      // rr = sum
    kOpRhoInit = 3, // rho = sum; flag if not positive
    kOpBeta = 4,    // beta = sum / rho; rho = sum; flag if sum not positive
};

// Breakdown bits of Scalars::flag.
constexpr int kFlagPqBreakdown = 1;   // p.Ap not positive and finite
constexpr int kFlagRhoBreakdown = 2;  // r.z not positive and finite

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
// to j+1, j = floor((nx-1)/2), both right-aligned in their half).  Vectors in
// this layout (the packed right-hand side and results) take 64*EPL*sizeof(T)
// bytes per line, line L = k*ny + m at L*64*EPL slots.
//
// The factors of line L form one record of rec_bytes() bytes: four packed
// arrays (1/M; p, the coupling of the slot's element to its chain predecessor,
// 0 at a chain's start and in unused slots; f, the y-coupling to line m+1; g,
// the z-coupling to plane k+1; f and g are 0 past the last line and plane),
// then the FP64 twist row (1/M_j, e1[j-1], e1[j], and the chain-B seed: the
// coefficient u of element j+1 toward the twist element).  A coupling is stored
// once: a sweep that needs line m's coupling to line m-1 (plane k's to plane
// k-1) reads f of line m-1 (g of plane k-1).  The sweeps form the recurrence
// coefficients a = -p/M and u = -p'/M (p' the next chain position's coupling)
// and the kRecMul scan multipliers of a lane themselves.
constexpr int kRecArrays = 4;
constexpr int kRecMul = 11;  // forward stage multipliers 0-4, backward 0-4, chain-B seed
enum RecArray : int { kRecMv = 0, kRecP = 1, kRecF = 2, kRecG = 3 };

__host__ __device__ constexpr unsigned rec_arr_bytes(unsigned tsz, int epl) {
    return 64u * (unsigned)epl * tsz;
}
__host__ __device__ constexpr unsigned rec_tw_off(unsigned tsz, int epl) {
    return kRecArrays * rec_arr_bytes(tsz, epl);
}
__host__ __device__ constexpr unsigned rec_bytes(unsigned tsz, int epl) {
    return (rec_tw_off(tsz, epl) + 32u + 255u) & ~255u;
}

// Arguments of the nested sweeps (apply) in the sweep precision T.
template <typename T>
struct ApplyArgs {
    int nx, ny, nz;
    const void *rec;              // line records (rec_bytes each)
    const T *rp;                  // packed right-hand side
    T *Z;                         // packed intermediate, then final result
    T *scratch;                   // two packed plane buffers (one per half chain) for the
                                  // upper sweep's level-2 lower results, unless in LDS
};

// Arguments of the moves between the natural FP64 layout and the packed one.
template <typename T>
struct XferArgs {
    int nx, ny, nz;
    const double *r;              // pack: right-hand side; unpack: dot operand (may be null)
    const double *zi;             // pack: rhs = r - A zi if set; unpack: added to the output
    const double *d, *ax, *ay, *az;  // bands of A (pack with zi)
    T *rp;                        // pack output
    const T *Z;                   // unpack input
    double *zout;                 // unpack output
    double *partials;             // unpack: per-block partials of r.zout (may be null)
};

// Geometry of the ILU(0) level schedule: rows split at M (nblocks = 2) or not.
struct IluGrid {
    int nx, ny, nz, nblocks;
    long long nxy, N, M;
    int kz;       // plane of row M (start plane of the second block's level frame)
    int levels;   // number of point hyperplane levels (factorization)
    // tiled sweeps: block b covers planes kb0[b]..kb1[b] (empty if kb1 < kb0),
    // cut into tiles of kIluTile x kIluTile x-lines, TY along y, TZ[b] along z
    int kb0[2], kb1[2];
    int TY, TZ[2];
    int tlevels;  // tile anti-diagonals
};
constexpr int kIluTile = 8;

// Arguments of the packing of FP64 natural-layout factors into the line records.
struct PackArgs {
    int nx, ny, nz;
    const double *e1, *mv, *f2, *g3;
    void *rec;
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

// One right-hand side of a batched PCG: the bands of its system and its
// vectors (device memory; one table entry per system and right-hand side).
struct BatchVec {
    int nx, ny, nz, pad;
    const double *d, *ax, *ay, *az;  // bands of the system
    const double *b;                 // right-hand side (caller's)
    double *x;                       // solution (caller's)
    double *r, *z, *p, *q;           // PCG vectors
    double *partials;                // per-block partials (gx per entry)
    Scalars *sc;
};

// Per right-hand side control state of a batched PCG.
struct BatchCtl {
    double bn;      // ||b||
    double relres;  // recursive relative residual, then the true one at exit
    double tol;
    int maxit;
    int iters;
    int status;     // NTD_OK, NTD_EBREAKDOWN or NTD_ENOCONV
    int pad;
};

enum BatchOp : int {
    kBOpInit = 16,  // bn = sqrt(sum); reset the scalars; active = bn > 0
    kBOpTrue = 17,  // true relative residual; reactivate if above tol with iterations left
};

// Host-side launchers (defined in the .hip files).
int epl_for(int nx);  // elements per lane of a half-wave chain, 0 if unsupported
hipError_t launch_apply_f64(const ApplyArgs<double> &a, int epl, hipStream_t s, hipEvent_t *ev);
hipError_t launch_apply_f32(const ApplyArgs<float> &a, int epl, hipStream_t s, hipEvent_t *ev);
hipError_t launch_pack_rhs_f64(const XferArgs<double> &x, int epl, hipStream_t s);
hipError_t launch_pack_rhs_f32(const XferArgs<float> &x, int epl, hipStream_t s);
// np receives the number of partials written (0 when x.partials is null)
hipError_t launch_unpack_f64(const XferArgs<double> &x, int epl, hipStream_t s, int *np);
hipError_t launch_unpack_f32(const XferArgs<float> &x, int epl, hipStream_t s, int *np);
hipError_t launch_setup(const SetupArgs &a, int epl, hipStream_t s);
// the factorizations of `count` systems (a table of arguments in device
// memory, all with the same elements per lane) in one pair of launches
hipError_t launch_setup_batch(const SetupArgs *tab, int count, int max_nx, int epl,
                              hipStream_t s);
hipError_t launch_pack_f64(const PackArgs &p, int epl, hipStream_t s);
hipError_t launch_pack_f32(const PackArgs &p, int epl, hipStream_t s);

// Batched launches over the table entries e = s*nrhs + q of count systems
// with nrhs right-hand sides each (the moves: `count` = all entries, one grid
// row per entry); an entry whose active flag is 0 does nothing (active may be
// null: all entries run).
// plane_lds > 0: the lower and upper sweeps keep each plane in LDS, that many
// bytes per workgroup (plane_lds_bytes of the batch's largest ny), after
// allow_apply_batch_lds_* has allowed it; 0: planes go through memory.
hipError_t launch_apply_batch_f32(const ApplyArgs<float> *tab, const int *active, int count,
                                  int nrhs, int epl, size_t plane_lds, hipStream_t s,
                                  hipEvent_t *ev);
hipError_t launch_apply_batch_f64(const ApplyArgs<double> *tab, const int *active, int count,
                                  int nrhs, int epl, size_t plane_lds, hipStream_t s,
                                  hipEvent_t *ev);
hipError_t allow_apply_batch_lds_f32(int epl, size_t bytes);
hipError_t allow_apply_batch_lds_f64(int epl, size_t bytes);
// Dynamic LDS of the LDS-plane sweeps: the twist exchange (two lines) and one
// plane of ny lines, 64*epl slots each.
constexpr size_t plane_lds_bytes(int ny, int epl, size_t tsz) {
    return (size_t)(2 + ny) * 64u * (size_t)epl * tsz;
}
// The same sweeps with nr right-hand sides of one system per wavefront pair
// (nr = 2 or 4 dividing nrhs; batch_multi_ok tells which (precision, EPL, nr)
// are built).
bool batch_multi_ok(int elem_bytes, int epl, int nr);
// plane_lds as for launch_apply_batch_*: NR plane buffers, NR times
// plane_lds_bytes of the largest ny, after allow_apply_batch_multi_lds_*.
hipError_t launch_apply_batch_multi_f32(const ApplyArgs<float> *tab, const int *active, int count,
                                        int nrhs, int epl, int nr, size_t plane_lds, hipStream_t s,
                                        hipEvent_t *ev);
hipError_t launch_apply_batch_multi_f64(const ApplyArgs<double> *tab, const int *active,
                                        int count, int nrhs, int epl, int nr, size_t plane_lds,
                                        hipStream_t s, hipEvent_t *ev);
hipError_t allow_apply_batch_multi_lds_f32(int epl, int nr, size_t bytes);
hipError_t allow_apply_batch_multi_lds_f64(int epl, int nr, size_t bytes);
hipError_t launch_pack_rhs_batch_f32(const XferArgs<float> *tab, const int *active, int count,
                                     int gx, int epl, hipStream_t s);
hipError_t launch_pack_rhs_batch_f64(const XferArgs<double> *tab, const int *active, int count,
                                     int gx, int epl, hipStream_t s);
hipError_t launch_unpack_batch_f32(const XferArgs<float> *tab, const int *active, int count,
                                   int gx, int epl, hipStream_t s);
hipError_t launch_unpack_batch_f64(const XferArgs<double> *tab, const int *active, int count,
                                   int gx, int epl, hipStream_t s);
// x = 0, r = b, partials of b.b
hipError_t launch_batch_init(const BatchVec *tab, int count, int gx, hipStream_t s);
// which = 0: q = A p with partials of p.q; which = 1: q = b - A x with partials of q.q
hipError_t launch_batch_spmv(const BatchVec *tab, const int *active, int count, int gx, int which,
                             hipStream_t s);
hipError_t launch_batch_axpy2(const BatchVec *tab, const int *active, int count, int gx,
                              hipStream_t s);
// p = z + beta p (or p = z when copy is set)
hipError_t launch_batch_xpay(const BatchVec *tab, const int *active, int count, int gx, bool copy,
                             hipStream_t s);
// one block per entry: sums the entry's gx partials and applies op (a
// FinalizeOp or a BatchOp); kBOpInit (which stores tol and maxit in the
// entry's control state) and kBOpTrue run for every entry
hipError_t launch_batch_finalize(const BatchVec *tab, BatchCtl *ctl, int *active, int count,
                                 int gx, int op, double tol, int maxit, hipStream_t s);

IluGrid ilu_grid(int nx, int ny, int nz, int nblocks);
hipError_t launch_ilu_factor(const IluGrid &g, const double *d, const double *ax, const double *ay,
                             const double *az, double *dt, double *dtinv, int *flag,
                             hipStream_t s);
// z = B_ILU^{-1} r; fcoef (MIXED, else NULL): ax, ay, az and 1/dt in FP32,
// 4 N floats, which the sweeps then read instead of the FP64 arrays (the
// arithmetic stays FP64).
hipError_t launch_ilu_apply(const IluGrid &g, const double *ax, const double *ay, const double *az,
                            const double *dtinv, const float *fcoef, const double *r, double *z,
                            hipStream_t s);
hipError_t launch_ilu_coef_f32(const IluGrid &g, const double *ax, const double *ay,
                               const double *az, const double *dtinv, float *fcoef,
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
hipError_t launch_add_dot(double *z, const double *w, const double *r, long long N,
                          double *partials, int *nparts, hipStream_t s);
hipError_t launch_residual(double *out, const double *b, const double *Ax, long long N,
                           hipStream_t s);
hipError_t launch_fill(double *x, double v, long long N, hipStream_t s);
hipError_t launch_copy(double *dst, const double *src, long long N, hipStream_t s);
hipError_t launch_cast_f32(float *dst, const double *src, long long N, hipStream_t s);
hipError_t launch_recip(double *dst, const double *src, long long N, hipStream_t s);

}  // namespace ntd
