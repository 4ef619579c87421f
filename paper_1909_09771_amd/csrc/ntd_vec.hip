// ntd_vec.hip -- bandwidth-bound kernels of the PCG step: assembly of the
// 7-point matrix, SpMV with a fused dot partial, the CG vector updates and the
// fixed-order FP64 reductions.
//
// Reductions are deterministic: every launch uses a grid that depends only on
// N, each thread sums a fixed set of entries in a fixed order, blocks reduce
// in LDS with a fixed tree, and one finalize block sums the block partials in
// a fixed order.
#include "ntd_internal.h"

namespace ntd {

namespace {

__device__ __forceinline__ double face_coef(double kp, double kq) {
    return 2.0 * kp * kq / (kp + kq);
}

// Blocks for an N-element grid-stride kernel (deterministic in N only).
inline int blocks_for(long long N) {
    long long b = (N + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > kMaxBlocks) b = kMaxBlocks;
    return (int)b;
}

// Fixed-order block reduction of one double per thread; thread 0 gets the sum.
__device__ __forceinline__ double block_sum(double v) {
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

__global__ void __launch_bounds__(kBlock) k_check_positive(const double *__restrict__ kappa,
                                                           const double *__restrict__ t,
                                                           long long N, int *flag) {
    int bad = 0;
    for (long long p = blockIdx.x * (long long)kBlock + threadIdx.x; p < N;
         p += (long long)gridDim.x * kBlock) {
        double k = kappa[p];
        if (!(k > 0.0) || !isfinite(k)) bad = 1;
        if (t) {
            double v = t[p];
            if (!(v > 0.0) || !isfinite(v)) bad = 1;
        }
    }
    if (bad) atomicOr(flag, kFlagBadInput);
}

// One thread per grid point; faces in the order x-, x+, y-, y+, z-, z+.  A
// Dirichlet face adds kappa_p to the diagonal, a Neumann face nothing, an
// interior face the harmonic mean of the two node values.
__global__ void __launch_bounds__(kBlock) k_assemble(Grid g, const double *__restrict__ kappa,
                                                     int b0, int b1, int b2, int b3, int b4,
                                                     int b5, double *__restrict__ d,
                                                     double *__restrict__ ax,
                                                     double *__restrict__ ay,
                                                     double *__restrict__ az) {
    for (long long p = blockIdx.x * (long long)kBlock + threadIdx.x; p < g.N;
         p += (long long)gridDim.x * kBlock) {
        int i = (int)(p % g.nx);
        int j = (int)((p / g.nx) % g.ny);
        int k = (int)(p / g.nxy);
        double kp = kappa[p];
        double diag = 0.0, c;
        if (i > 0) diag += face_coef(kp, kappa[p - 1]);
        else if (b0 == 0) diag += kp;
        if (i < g.nx - 1) { c = face_coef(kp, kappa[p + 1]); diag += c; ax[p] = -c; }
        else { ax[p] = 0.0; if (b1 == 0) diag += kp; }
        if (j > 0) diag += face_coef(kp, kappa[p - g.nx]);
        else if (b2 == 0) diag += kp;
        if (j < g.ny - 1) { c = face_coef(kp, kappa[p + g.nx]); diag += c; ay[p] = -c; }
        else { ay[p] = 0.0; if (b3 == 0) diag += kp; }
        if (k > 0) diag += face_coef(kp, kappa[p - g.nxy]);
        else if (b4 == 0) diag += kp;
        if (k < g.nz - 1) { c = face_coef(kp, kappa[p + g.nxy]); diag += c; az[p] = -c; }
        else { az[p] = 0.0; if (b5 == 0) diag += kp; }
        d[p] = diag;
    }
}

// y = A x (7-point, symmetric bands), plus the block partial of x.y.
__global__ void __launch_bounds__(kBlock) k_spmv(Grid g, const double *__restrict__ d,
                                                 const double *__restrict__ ax,
                                                 const double *__restrict__ ay,
                                                 const double *__restrict__ az,
                                                 const double *__restrict__ x,
                                                 double *__restrict__ y,
                                                 double *__restrict__ partials) {
    double acc = 0.0;
    for (long long p = blockIdx.x * (long long)kBlock + threadIdx.x; p < g.N;
         p += (long long)gridDim.x * kBlock) {
        int i = (int)(p % g.nx);
        int j = (int)((p / g.nx) % g.ny);
        int k = (int)(p / g.nxy);
        // every neighbour term is one fused multiply-add onto the running sum
        // (written out, so that no contraction choice can reorder it)
        double xp = x[p];
        double s = d[p] * xp;
        if (i > 0) s = fma(ax[p - 1], x[p - 1], s);
        if (i < g.nx - 1) s = fma(ax[p], x[p + 1], s);
        if (j > 0) s = fma(ay[p - g.nx], x[p - g.nx], s);
        if (j < g.ny - 1) s = fma(ay[p], x[p + g.nx], s);
        if (k > 0) s = fma(az[p - g.nxy], x[p - g.nxy], s);
        if (k < g.nz - 1) s = fma(az[p], x[p + g.nxy], s);
        y[p] = s;
        acc += xp * s;
    }
    if (partials) {
        double t = block_sum(acc);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

// y = A x for two consecutive points of a line per thread, with 16-byte loads
// of every pair (nx even, all arrays 16-byte aligned, N < 2^31), one pair per
// thread.  The stencil is bound by the load instructions it issues, not by its
// bytes, and a pair needs 14 where two single points need 28.  Each point's sum
// is formed in k_spmv's order, so y is bitwise k_spmv's.  It serves the
// products without a dot partial; the PCG's q = A p keeps k_spmv, whose fixed
// grid also fixes the summation order of p.q.
typedef double dbl2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ dbl2 ld2(const double *p) { return *(const dbl2 *)p; }

__global__ void __launch_bounds__(kBlock) k_spmv2(Grid g, const double *__restrict__ d,
                                                  const double *__restrict__ ax,
                                                  const double *__restrict__ ay,
                                                  const double *__restrict__ az,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ y) {
    const unsigned nx = (unsigned)g.nx, ny = (unsigned)g.ny, nz = (unsigned)g.nz;
    const unsigned nxy = (unsigned)g.nxy, P = (unsigned)(g.N / 2);
    for (unsigned q = blockIdx.x * (unsigned)kBlock + threadIdx.x; q < P;
         q += gridDim.x * (unsigned)kBlock) {
        const unsigned p = 2 * q;
        const unsigned line = p / nx;
        const unsigned i = p - line * nx, j = line % ny, k = line / ny;
        const dbl2 xv = ld2(x + p), dv = ld2(d + p), axv = ld2(ax + p);
        const dbl2 ayv = ld2(ay + p), azv = ld2(az + p);
        double s0 = dv.x * xv.x, s1 = dv.y * xv.y;
        if (i > 0) s0 = fma(ax[p - 1], x[p - 1], s0);
        s0 = fma(axv.x, xv.y, s0);  // i + 1 < nx: the pair never ends a line
        s1 = fma(axv.x, xv.x, s1);
        if (i + 1 < nx - 1) s1 = fma(axv.y, x[p + 2], s1);
        if (j > 0) {
            const dbl2 a = ld2(ay + p - nx), v = ld2(x + p - nx);
            s0 = fma(a.x, v.x, s0);
            s1 = fma(a.y, v.y, s1);
        }
        if (j < ny - 1) {
            const dbl2 v = ld2(x + p + nx);
            s0 = fma(ayv.x, v.x, s0);
            s1 = fma(ayv.y, v.y, s1);
        }
        if (k > 0) {
            const dbl2 a = ld2(az + p - nxy), v = ld2(x + p - nxy);
            s0 = fma(a.x, v.x, s0);
            s1 = fma(a.y, v.y, s1);
        }
        if (k < nz - 1) {
            const dbl2 v = ld2(x + p + nxy);
            s0 = fma(azv.x, v.x, s0);
            s1 = fma(azv.y, v.y, s1);
        }
        dbl2 o;
        o.x = s0;
        o.y = s1;
        *(dbl2 *)(y + p) = o;
    }
}

__global__ void __launch_bounds__(kBlock) k_dot(const double *__restrict__ x,
                                                const double *__restrict__ y, long long N,
                                                double *__restrict__ partials) {
    double acc = 0.0;
    for (long long p = blockIdx.x * (long long)kBlock + threadIdx.x; p < N;
         p += (long long)gridDim.x * kBlock)
        acc += x[p] * y[p];
    double t = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kBlock) k_finalize(const double *__restrict__ partials,
                                                     int nparts, Scalars *sc, int op) {
    double acc = 0.0;
    for (int q = threadIdx.x; q < nparts; q += kBlock) acc += partials[q];
    double s = block_sum(acc);
    if (threadIdx.x == 0) {
        // CG needs p'Ap > 0 and r'z > 0; a failure sets a breakdown bit (1:
        // p'Ap, 2: r'z) and zeroes the step, so x and r keep the last iterate.
        switch (op) {
        case kOpAlpha:
            sc->pq = s;
            if (sc->flag & kFlagRhoBreakdown) sc->alpha = 0.0;
            else if (!(s > 0.0) || !isfinite(s)) { sc->flag |= kFlagPqBreakdown; sc->alpha = 0.0; }
            else sc->alpha = sc->rho / s;
            break;
        case kOpRR: sc->rr = s; break;
        case kOpRhoInit:
            sc->rho = s;
            if (!(s > 0.0) || !isfinite(s)) sc->flag |= kFlagRhoBreakdown;
            break;
        case kOpBeta:
            if (!(s > 0.0) || !isfinite(s)) { sc->flag |= kFlagRhoBreakdown; sc->beta = 0.0; }
            else { sc->beta = s / sc->rho; sc->rho = s; }
            break;
        default: sc->result = s; break;
        }
    }
}

// x += alpha p; r -= alpha q; partial of r.r.
__global__ void __launch_bounds__(kBlock) k_axpy2_norm(double *__restrict__ x,
                                                       double *__restrict__ r,
                                                       const double *__restrict__ p,
                                                       const double *__restrict__ q,
                                                       const Scalars *__restrict__ sc,
                                                       long long N,
                                                       double *__restrict__ partials) {
    const double alpha = sc->alpha;
    double acc = 0.0;
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < N;
         i += (long long)gridDim.x * kBlock) {
        x[i] += alpha * p[i];
        double rv = r[i] - alpha * q[i];
        r[i] = rv;
        acc += rv * rv;
    }
    double t = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// p = z + beta p.
__global__ void __launch_bounds__(kBlock) k_xpay(double *__restrict__ p,
                                                 const double *__restrict__ z,
                                                 const Scalars *__restrict__ sc, long long N) {
    const double beta = sc->beta;
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < N;
         i += (long long)gridDim.x * kBlock)
        p[i] = z[i] + beta * p[i];
}

__global__ void __launch_bounds__(kBlock) k_residual(double *__restrict__ out,
                                                     const double *__restrict__ b,
                                                     const double *__restrict__ Ax, long long N) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < N;
         i += (long long)gridDim.x * kBlock)
        out[i] = b[i] - Ax[i];
}

// z += w; partials of r.z (the last stage of the symmetric combination).
__global__ void __launch_bounds__(kBlock) k_add_dot(double *__restrict__ z,
                                                    const double *__restrict__ w,
                                                    const double *__restrict__ r, long long N,
                                                    double *__restrict__ partials) {
    double acc = 0.0;
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < N;
         i += (long long)gridDim.x * kBlock) {
        const double zv = z[i] + w[i];
        z[i] = zv;
        acc += r[i] * zv;
    }
    const double t = block_sum(acc);
    if (partials && threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kBlock) k_fill(double *__restrict__ x, double v, long long N) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < N;
         i += (long long)gridDim.x * kBlock)
        x[i] = v;
}

__global__ void __launch_bounds__(kBlock) k_copy(double *__restrict__ dst,
                                                 const double *__restrict__ src, long long N) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < N;
         i += (long long)gridDim.x * kBlock)
        dst[i] = src[i];
}

__global__ void __launch_bounds__(kBlock) k_cast_f32(float *__restrict__ dst,
                                                     const double *__restrict__ src, long long N) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < N;
         i += (long long)gridDim.x * kBlock)
        dst[i] = (float)src[i];
}

__global__ void __launch_bounds__(kBlock) k_recip(double *__restrict__ dst,
                                                  const double *__restrict__ src, long long N) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < N;
         i += (long long)gridDim.x * kBlock)
        dst[i] = 1.0 / src[i];
}

}  // namespace

hipError_t launch_check_positive(const double *kappa, const double *t, long long N, int *flag,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_check_positive, dim3(blocks_for(N)), dim3(kBlock), 0, s, kappa, t, N,
                       flag);
    return hipGetLastError();
}

hipError_t launch_assemble(const Grid &g, const double *kappa, const int *bc, double *d,
                           double *ax, double *ay, double *az, hipStream_t s) {
    hipLaunchKernelGGL(k_assemble, dim3(blocks_for(g.N)), dim3(kBlock), 0, s, g, kappa, bc[0],
                       bc[1], bc[2], bc[3], bc[4], bc[5], d, ax, ay, az);
    return hipGetLastError();
}

hipError_t launch_spmv(const Grid &g, const double *d, const double *ax, const double *ay,
                       const double *az, const double *x, double *y, double *partials,
                       int *nparts, hipStream_t s) {
    const uintptr_t al = (uintptr_t)d | (uintptr_t)ax | (uintptr_t)ay | (uintptr_t)az |
                         (uintptr_t)x | (uintptr_t)y;
    if (!partials && g.nx % 2 == 0 && g.N < (1LL << 31) && (al & 15) == 0) {
        long long nb = (g.N / 2 + kBlock - 1) / kBlock;  // one pair per thread
        if (nb < 1) nb = 1;
        if (nparts) *nparts = 0;
        hipLaunchKernelGGL(k_spmv2, dim3((unsigned)nb), dim3(kBlock), 0, s, g, d, ax, ay, az, x, y);
        return hipGetLastError();
    }
    int nb = blocks_for(g.N);
    if (nparts) *nparts = nb;
    hipLaunchKernelGGL(k_spmv, dim3(nb), dim3(kBlock), 0, s, g, d, ax, ay, az, x, y, partials);
    return hipGetLastError();
}

hipError_t launch_dot(const double *x, const double *y, long long N, double *partials,
                      int *nparts, hipStream_t s) {
    int nb = blocks_for(N);
    *nparts = nb;
    hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kBlock), 0, s, x, y, N, partials);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, int nparts, Scalars *sc, int op,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, partials, nparts, sc, op);
    return hipGetLastError();
}

hipError_t launch_axpy2_norm(double *x, double *r, const double *p, const double *q,
                             const Scalars *sc, long long N, double *partials, int *nparts,
                             hipStream_t s) {
    int nb = blocks_for(N);
    *nparts = nb;
    hipLaunchKernelGGL(k_axpy2_norm, dim3(nb), dim3(kBlock), 0, s, x, r, p, q, sc, N, partials);
    return hipGetLastError();
}

hipError_t launch_xpay(double *p, const double *z, const Scalars *sc, long long N,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_xpay, dim3(blocks_for(N)), dim3(kBlock), 0, s, p, z, sc, N);
    return hipGetLastError();
}

hipError_t launch_residual(double *out, const double *b, const double *Ax, long long N,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_residual, dim3(blocks_for(N)), dim3(kBlock), 0, s, out, b, Ax, N);
    return hipGetLastError();
}

hipError_t launch_add_dot(double *z, const double *w, const double *r, long long N,
                          double *partials, int *nparts, hipStream_t s) {
    const int nb = blocks_for(N);
    if (nparts) *nparts = nb;
    hipLaunchKernelGGL(k_add_dot, dim3(nb), dim3(kBlock), 0, s, z, w, r, N, partials);
    return hipGetLastError();
}

hipError_t launch_fill(double *x, double v, long long N, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(N)), dim3(kBlock), 0, s, x, v, N);
    return hipGetLastError();
}

hipError_t launch_copy(double *dst, const double *src, long long N, hipStream_t s) {
    hipLaunchKernelGGL(k_copy, dim3(blocks_for(N)), dim3(kBlock), 0, s, dst, src, N);
    return hipGetLastError();
}

hipError_t launch_cast_f32(float *dst, const double *src, long long N, hipStream_t s) {
    hipLaunchKernelGGL(k_cast_f32, dim3(blocks_for(N)), dim3(kBlock), 0, s, dst, src, N);
    return hipGetLastError();
}

hipError_t launch_recip(double *dst, const double *src, long long N, hipStream_t s) {
    hipLaunchKernelGGL(k_recip, dim3(blocks_for(N)), dim3(kBlock), 0, s, dst, src, N);
    return hipGetLastError();
}

}  // namespace ntd
