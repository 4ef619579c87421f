// ntd_batch.hip -- the bandwidth-bound kernels of a batched PCG: many
// independent systems, several right-hand sides each, advanced together.  Every
// launch covers all right-hand sides of the batch (blockIdx.y selects one entry
// of a table of BatchVec in device memory, gx blocks per entry), and every
// right-hand side keeps its scalars and convergence state on the device, so an
// iteration never waits for the host and a run of iterations can be captured
// in a graph and replayed.  A right-hand side that has converged (or broken
// down, or used its iterations) is switched off through its active flag, which
// every kernel reads first.
//
// The arithmetic of each entry is that of the single-system kernels (same
// operation order); reductions are fixed-order for a given gx, so a batch is
// bitwise repeatable, and an entry matches the single-system PCG of its system
// up to the rounding of its dot products.
#include <math.h>

#include "ntd.h"
#include "ntd_internal.h"

namespace ntd {

namespace {

__device__ __forceinline__ double block_sum_b(double v) {
    __shared__ double red[kBlock];
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    return red[0];
}

// The table entry of this block, in scalar registers.
__device__ __forceinline__ BatchVec entry(const BatchVec *tab) {
    BatchVec out;
    const unsigned *src = (const unsigned *)(tab + blockIdx.y);
    unsigned *dst = (unsigned *)&out;
#pragma unroll
    for (unsigned i = 0; i < sizeof(BatchVec) / 4; ++i)
        dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return out;
}

__device__ __forceinline__ bool on(const int *active) {
    return !active || __builtin_amdgcn_readfirstlane(active[blockIdx.y]) != 0;
}

__device__ __forceinline__ long long npoints(const BatchVec &v) {
    return (long long)v.nx * v.ny * v.nz;
}

__global__ void __launch_bounds__(kBlock) k_batch_init(const BatchVec *tab) {
    const BatchVec v = entry(tab);
    const long long N = npoints(v);
    double acc = 0.0;
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < N;
         i += (long long)gridDim.x * kBlock) {
        const double bv = v.b[i];
        v.x[i] = 0.0;
        v.r[i] = bv;
        acc += bv * bv;
    }
    const double t = block_sum_b(acc);
    if (threadIdx.x == 0) v.partials[blockIdx.x] = t;
}

// which = 0: q = A p, partial of p.q; which = 1: q = b - A x, partial of q.q.
__global__ void __launch_bounds__(kBlock) k_batch_spmv(const BatchVec *tab, const int *active,
                                                       int which) {
    if (!on(active)) return;
    const BatchVec v = entry(tab);
    const long long nxy = (long long)v.nx * v.ny, N = nxy * v.nz;
    const double *x = which == 0 ? v.p : v.x;
    double acc = 0.0;
    for (long long p = blockIdx.x * (long long)kBlock + threadIdx.x; p < N;
         p += (long long)gridDim.x * kBlock) {
        const int i = (int)(p % v.nx);
        const int j = (int)((p / v.nx) % v.ny);
        const int k = (int)(p / nxy);
        const double xp = x[p];
        double s = v.d[p] * xp;
        if (i > 0) s += v.ax[p - 1] * x[p - 1];
        if (i < v.nx - 1) s += v.ax[p] * x[p + 1];
        if (j > 0) s += v.ay[p - v.nx] * x[p - v.nx];
        if (j < v.ny - 1) s += v.ay[p] * x[p + v.nx];
        if (k > 0) s += v.az[p - nxy] * x[p - nxy];
        if (k < v.nz - 1) s += v.az[p] * x[p + nxy];
        if (which == 0) {
            v.q[p] = s;
            acc += xp * s;
        } else {
            const double res = v.b[p] - s;
            v.q[p] = res;
            acc += res * res;
        }
    }
    const double t = block_sum_b(acc);
    if (threadIdx.x == 0) v.partials[blockIdx.x] = t;
}

// x += alpha p; r -= alpha q; partial of r.r.
__global__ void __launch_bounds__(kBlock) k_batch_axpy2(const BatchVec *tab, const int *active) {
    if (!on(active)) return;
    const BatchVec v = entry(tab);
    const long long N = npoints(v);
    const double alpha = v.sc->alpha;
    double acc = 0.0;
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < N;
         i += (long long)gridDim.x * kBlock) {
        v.x[i] += alpha * v.p[i];
        const double rv = v.r[i] - alpha * v.q[i];
        v.r[i] = rv;
        acc += rv * rv;
    }
    const double t = block_sum_b(acc);
    if (threadIdx.x == 0) v.partials[blockIdx.x] = t;
}

// p = z + beta p, or p = z.
__global__ void __launch_bounds__(kBlock) k_batch_xpay(const BatchVec *tab, const int *active,
                                                       int copy) {
    if (!on(active)) return;
    const BatchVec v = entry(tab);
    const long long N = npoints(v);
    const double beta = copy ? 0.0 : v.sc->beta;
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < N;
         i += (long long)gridDim.x * kBlock)
        v.p[i] = copy ? v.z[i] : v.z[i] + beta * v.p[i];
}

// One block per entry (blockIdx.y): the sum of its gx partials in a fixed
// order, then the scalar step of op.
__global__ void __launch_bounds__(kBlock) k_batch_finalize(const BatchVec *tab, BatchCtl *ctl,
                                                           int *active, int gx, int op,
                                                           double tol, int maxit) {
    const bool every = op == kBOpInit || op == kBOpTrue;
    if (!every && !on(active)) return;
    const BatchVec v = entry(tab);
    double acc = 0.0;
    for (int q = threadIdx.x; q < gx; q += kBlock) acc += v.partials[q];
    const double s = block_sum_b(acc);
    if (threadIdx.x != 0) return;
    Scalars *sc = v.sc;
    BatchCtl &c = ctl[blockIdx.y];
    int *act = active + blockIdx.y;
    switch (op) {
    case kBOpInit: {
        const double bn = sqrt(s);
        sc->rho = sc->pq = sc->alpha = sc->beta = sc->rr = sc->result = 0.0;
        sc->flag = 0;
        c.bn = bn;
        c.relres = 0.0;
        c.tol = tol;
        c.maxit = maxit;
        c.iters = 0;
        c.status = NTD_OK;
        *act = bn > 0.0 ? 1 : 0;
        break;
    }
    case kOpRhoInit:
        sc->rho = s;
        if (!(s > 0.0) || !isfinite(s)) {  // r.z of a preconditioner that is not SPD
            sc->flag |= kFlagRhoBreakdown;
            c.status = NTD_EBREAKDOWN;
            *act = 0;
        }
        break;
    case kOpAlpha:
        sc->pq = s;
        if (!(s > 0.0) || !isfinite(s)) {
            sc->flag |= kFlagPqBreakdown;
            sc->alpha = 0.0;
            c.status = NTD_EBREAKDOWN;
            *act = 0;
        } else {
            sc->alpha = sc->rho / s;
        }
        break;
    case kOpRR:
        sc->rr = s;
        c.iters += 1;
        c.relres = sqrt(s) / c.bn;
        if (c.relres <= c.tol) {
            *act = 0;
        } else if (c.iters >= c.maxit) {
            c.status = NTD_ENOCONV;
            *act = 0;
        }
        break;
    case kOpBeta:
        if (!(s > 0.0) || !isfinite(s)) {
            sc->flag |= kFlagRhoBreakdown;
            sc->beta = 0.0;
            c.status = NTD_EBREAKDOWN;
            *act = 0;
        } else {
            sc->beta = s / sc->rho;
            sc->rho = s;
        }
        break;
    case kBOpTrue:
        if (c.bn == 0.0) break;
        c.relres = sqrt(s) / c.bn;
        if (c.status == NTD_OK && c.relres > c.tol) {
            if (c.iters < c.maxit) *act = 1;
            else c.status = NTD_ENOCONV;
        }
        break;
    default: break;
    }
}

}  // namespace

hipError_t launch_batch_init(const BatchVec *tab, int count, int gx, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_init, dim3(gx, count), dim3(kBlock), 0, s, tab);
    return hipGetLastError();
}

hipError_t launch_batch_spmv(const BatchVec *tab, const int *active, int count, int gx, int which,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_batch_spmv, dim3(gx, count), dim3(kBlock), 0, s, tab, active, which);
    return hipGetLastError();
}

hipError_t launch_batch_axpy2(const BatchVec *tab, const int *active, int count, int gx,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_batch_axpy2, dim3(gx, count), dim3(kBlock), 0, s, tab, active);
    return hipGetLastError();
}

hipError_t launch_batch_xpay(const BatchVec *tab, const int *active, int count, int gx, bool copy,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_batch_xpay, dim3(gx, count), dim3(kBlock), 0, s, tab, active,
                       copy ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_batch_finalize(const BatchVec *tab, BatchCtl *ctl, int *active, int count,
                                 int gx, int op, double tol, int maxit, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_finalize, dim3(1, count), dim3(kBlock), 0, s, tab, ctl, active, gx,
                       op, tol, maxit);
    return hipGetLastError();
}

}  // namespace ntd
