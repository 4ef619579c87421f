// ntd_ilu.hip -- the ILU(0) smoother of the combination preconditioner
// (arXiv:1909.09771, Sec. 3: "Smoothing high frequency components of error",
// eq. com, and "Parallel Solve with Preconditioner").
//
// ILU(0) is taken of the block-diagonal approximation blkD(A(1:M,1:M),
// A(M+1:N,M+1:N)), M = floor(N/2): couplings between a row below M and a row
// at or above M are dropped.  For the 7-point pattern ILU(0) produces no fill
// inside the pattern, so the factorization only changes the diagonal:
//   dt_p = d_p - sum over kept lower neighbours q of a_pq^2 / dt_q,
// and B_ILU = (Dt + L) Dt^{-1} (Dt + U).
//
// Scheduling: row p depends only on its lower neighbours p-1, p-nx, p-nx*ny, so
// all rows on one hyperplane i + j + (k - k0) = level (k0 = 0 in the first
// block, k0 = the plane of row M in the second) are independent.  One launch
// per level processes both blocks at once; a thread owns one (j, k) pair and
// the row of each block that falls on the level.
#include "ntd_internal.h"

namespace ntd {

namespace {

__device__ __forceinline__ bool kept(long long q, long long p, const IluGrid &g) {
    return g.nblocks == 1 || !(q < g.M && p >= g.M);
}

// Calls f(p, i, j, k) for every row of the level owned by this thread.
template <class F>
__device__ __forceinline__ void for_level_rows(const IluGrid &g, int level, F f) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= (long long)g.ny * g.nz) return;
    const int j = (int)(t % g.ny), k = (int)(t / g.ny);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        if (b == 1 && (g.nblocks == 1 || k < g.kz)) break;
        const int k0 = b == 0 ? 0 : g.kz;
        const int i = level - j - (k - k0);
        if (i < 0 || i >= g.nx) continue;
        const long long p = i + (long long)g.nx * j + g.nxy * k;
        const int blk = (g.nblocks == 2 && p >= g.M) ? 1 : 0;
        if (blk != b) continue;
        f(p, i, j, k);
    }
}

__global__ void __launch_bounds__(256) k_ilu_factor_level(IluGrid g, const double *__restrict__ d,
                                                          const double *__restrict__ ax,
                                                          const double *__restrict__ ay,
                                                          const double *__restrict__ az,
                                                          double *__restrict__ dt, int level,
                                                          int *flag) {
    for_level_rows(g, level, [&](long long p, int i, int j, int k) {
        double v = d[p];
        if (i > 0 && kept(p - 1, p, g)) v -= ax[p - 1] * ax[p - 1] / dt[p - 1];
        if (j > 0 && kept(p - g.nx, p, g)) v -= ay[p - g.nx] * ay[p - g.nx] / dt[p - g.nx];
        if (k > 0 && kept(p - g.nxy, p, g)) v -= az[p - g.nxy] * az[p - g.nxy] / dt[p - g.nxy];
        if (!(v > 0.0) || !isfinite(v)) atomicOr(flag, kFlagNotSPD);
        dt[p] = v;
    });
}

// Forward sweep (Dt + L) y = r.
__global__ void __launch_bounds__(256) k_ilu_fwd_level(IluGrid g, const double *__restrict__ ax,
                                                       const double *__restrict__ ay,
                                                       const double *__restrict__ az,
                                                       const double *__restrict__ dtinv,
                                                       const double *__restrict__ r,
                                                       double *__restrict__ y, int level) {
    for_level_rows(g, level, [&](long long p, int i, int j, int k) {
        double v = r[p];
        if (i > 0 && kept(p - 1, p, g)) v -= ax[p - 1] * y[p - 1];
        if (j > 0 && kept(p - g.nx, p, g)) v -= ay[p - g.nx] * y[p - g.nx];
        if (k > 0 && kept(p - g.nxy, p, g)) v -= az[p - g.nxy] * y[p - g.nxy];
        y[p] = v * dtinv[p];
    });
}

// Backward sweep (I + Dt^{-1} U) z = y, in place (z holds y on entry).
__global__ void __launch_bounds__(256) k_ilu_bwd_level(IluGrid g, const double *__restrict__ ax,
                                                       const double *__restrict__ ay,
                                                       const double *__restrict__ az,
                                                       const double *__restrict__ dtinv,
                                                       double *__restrict__ z, int level) {
    for_level_rows(g, level, [&](long long p, int i, int j, int k) {
        double v = 0.0;
        if (i < g.nx - 1 && kept(p, p + 1, g)) v += ax[p] * z[p + 1];
        if (j < g.ny - 1 && kept(p, p + g.nx, g)) v += ay[p] * z[p + g.nx];
        if (k < g.nz - 1 && kept(p, p + g.nxy, g)) v += az[p] * z[p + g.nxy];
        z[p] -= v * dtinv[p];
    });
}

inline int level_blocks(const IluGrid &g) {
    const long long t = (long long)g.ny * g.nz;
    return (int)((t + 255) / 256);
}

}  // namespace

IluGrid ilu_grid(int nx, int ny, int nz, int nblocks) {
    IluGrid g;
    g.nx = nx; g.ny = ny; g.nz = nz; g.nblocks = nblocks;
    g.nxy = (long long)nx * ny;
    g.N = g.nxy * nz;
    g.M = nblocks == 2 ? g.N / 2 : g.N;
    g.kz = (int)(g.M / g.nxy);
    if (g.kz > nz - 1) g.kz = nz - 1;
    // highest level of either block, plus one
    const int span = nblocks == 2 ? (g.kz > nz - 1 - g.kz ? g.kz : nz - 1 - g.kz) : nz - 1;
    g.levels = nx + ny - 2 + span + 1;
    return g;
}

hipError_t launch_ilu_factor(const IluGrid &g, const double *d, const double *ax, const double *ay,
                             const double *az, double *dt, double *dtinv, int *flag,
                             hipStream_t s) {
    const int nb = level_blocks(g);
    for (int l = 0; l < g.levels; ++l)
        hipLaunchKernelGGL(k_ilu_factor_level, dim3(nb), dim3(256), 0, s, g, d, ax, ay, az, dt, l,
                           flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_recip(dtinv, dt, g.N, s);
}

hipError_t launch_ilu_apply(const IluGrid &g, const double *ax, const double *ay, const double *az,
                            const double *dtinv, const double *r, double *z, hipStream_t s) {
    const int nb = level_blocks(g);
    for (int l = 0; l < g.levels; ++l)
        hipLaunchKernelGGL(k_ilu_fwd_level, dim3(nb), dim3(256), 0, s, g, ax, ay, az, dtinv, r, z, l);
    for (int l = g.levels - 1; l >= 0; --l)
        hipLaunchKernelGGL(k_ilu_bwd_level, dim3(nb), dim3(256), 0, s, g, ax, ay, az, dtinv, z, l);
    return hipGetLastError();
}

}  // namespace ntd
