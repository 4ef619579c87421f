// ntd_target.hip -- filter-vector targets from the preconditioner itself.
//
// Sec. 1 of the paper: the error of the filtered iteration evolves as
// (I - B^{-1}A)^n e^0, so the error components that survive longest are the
// eigenvectors of B^{-1}A with the smallest eigenvalues, and a filter vector t
// should approximate them.  ntd_filter_target computes that eigenvector for
// the handle's own B by inverse iteration on B^{-1}A:
//     v <- M^{-1} v, M = B^{-1}A, normalised to a largest entry of +1,
// and returns max(v, floor) as a filter vector.  M is self-adjoint and
// positive definite in the A-inner product <u, w>_A = u'Aw (B and A are SPD),
// so each inner solve M y = v is a conjugate-gradient iteration in that inner
// product: it needs one application of B^{-1} and one product with A per step,
// never B itself.
#include <math.h>

#include <vector>

#include "ntd.h"
#include "ntd_handle.h"

namespace {

constexpr int kTB = 256;
constexpr int kTMaxBlocks = ntd::kMaxBlocks;  // the partials of a handle hold this many

inline int tblocks(long long n) {
    long long b = (n + kTB - 1) / kTB;
    if (b < 1) b = 1;
    if (b > kTMaxBlocks) b = kTMaxBlocks;
    return (int)b;
}

// y += a p; r -= a q; s -= a w
__global__ void __launch_bounds__(kTB) k_tgt_step(double *__restrict__ y, double *__restrict__ r,
                                                  double *__restrict__ s,
                                                  const double *__restrict__ p,
                                                  const double *__restrict__ q,
                                                  const double *__restrict__ w, double a,
                                                  long long n) {
    for (long long i = blockIdx.x * (long long)kTB + threadIdx.x; i < n;
         i += (long long)gridDim.x * kTB) {
        y[i] += a * p[i];
        r[i] -= a * q[i];
        s[i] -= a * w[i];
    }
}

// p = r + b p; u = s + b u
__global__ void __launch_bounds__(kTB) k_tgt_dir(double *__restrict__ p, double *__restrict__ u,
                                                 const double *__restrict__ r,
                                                 const double *__restrict__ s, double b,
                                                 long long n) {
    for (long long i = blockIdx.x * (long long)kTB + threadIdx.x; i < n;
         i += (long long)gridDim.x * kTB) {
        p[i] = r[i] + b * p[i];
        u[i] = s[i] + b * u[i];
    }
}

// Per block: the entry of largest magnitude (the first in index order on
// ties), as a signed value; a NaN entry wins, so that the caller sees it.
__global__ void __launch_bounds__(kTB) k_tgt_maxabs(const double *__restrict__ v, long long n,
                                                    double *__restrict__ part) {
    __shared__ double best[kTB];
    __shared__ long long where[kTB];
    double b = 0.0;
    long long bi = -1;
    for (long long i = blockIdx.x * (long long)kTB + threadIdx.x; i < n;
         i += (long long)gridDim.x * kTB) {
        const double x = v[i];
        if (bi < 0 || (b == b && !(fabs(x) <= fabs(b)))) { b = x; bi = i; }
    }
    best[threadIdx.x] = b;
    where[threadIdx.x] = bi < 0 ? n : bi;
    __syncthreads();
    for (int h = kTB / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            const double o = best[threadIdx.x + h], mine = best[threadIdx.x];
            const long long oi = where[threadIdx.x + h];
            const bool nan_o = o != o, nan_m = mine != mine;
            if ((nan_o && !nan_m) || (!nan_m && fabs(o) > fabs(mine)) ||
                (nan_o == nan_m && fabs(o) == fabs(mine) && oi < where[threadIdx.x]) ||
                (nan_o && nan_m && oi < where[threadIdx.x])) {
                best[threadIdx.x] = o;
                where[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = best[0];
}

// v = max(v * c, floor)  (floor <= -1 leaves the scaled values as they are)
__global__ void __launch_bounds__(kTB) k_tgt_scale(double *__restrict__ v, double c, double floor_,
                                                   long long n) {
    for (long long i = blockIdx.x * (long long)kTB + threadIdx.x; i < n;
         i += (long long)gridDim.x * kTB) {
        const double x = v[i] * c;
        v[i] = x < floor_ ? floor_ : x;
    }
}

#define TCK(expr)                                  \
    do {                                           \
        if ((expr) != hipSuccess) return NTD_EHIP; \
    } while (0)
#define TST(expr)                      \
    do {                               \
        const int st_ = (expr);        \
        if (st_ != NTD_OK) return st_; \
    } while (0)

// The signed entry of largest magnitude of v[0..n), from per-block partials in
// `part` (at least 2048 doubles of device memory); synchronises s.
int signed_maxabs(const double *v, long long n, double *part, double *out, hipStream_t s) {
    const int nb = tblocks(n);
    hipLaunchKernelGGL(k_tgt_maxabs, dim3(nb), dim3(kTB), 0, s, v, n, part);
    TCK(hipGetLastError());
    std::vector<double> h(nb);
    TCK(hipMemcpyAsync(h.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    TCK(hipStreamSynchronize(s));
    double b = 0.0;
    for (int i = 0; i < nb; ++i) {
        if (h[i] != h[i]) { b = h[i]; break; }  // NaN: reported as not finite
        if (fabs(h[i]) > fabs(b)) b = h[i];
    }
    *out = b;
    return NTD_OK;
}

}  // namespace

extern "C" int ntd_vec_normalize(double *v, long long n, double floor_, double *partials,
                                 double *scale, void *stream) {
    if (!v || !partials || !scale || n < 1) return NTD_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    double m = 0.0;
    TST(signed_maxabs(v, n, partials, &m, s));
    if (!(m != 0.0) || !isfinite(m)) return NTD_EINVAL;
    hipLaunchKernelGGL(k_tgt_scale, dim3(tblocks(n)), dim3(kTB), 0, s, v, 1.0 / m, floor_, n);
    TCK(hipGetLastError());
    *scale = 1.0 / m;
    return NTD_OK;
}

extern "C" int ntd_filter_target(ntd_handle *h, double *v, int outer, double inner_tol,
                                 int inner_maxit, double floor_, double *work, int *inner_iters,
                                 double *lambda, void *stream) {
    if (!h || !v || !work || !inner_iters || !lambda) return NTD_EINVAL;
    if (outer < 1 || inner_maxit < 1 || !(inner_tol > 0.0) || !(floor_ > 0.0)) return NTD_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const long long n = h->N;
    double *y = work, *r = work + n, *p = work + 2 * n, *q = work + 3 * n, *w = work + 4 * n,
           *u = work + 5 * n, *sv = work + 6 * n;
    const int nb = tblocks(n);
    auto dot = [&](const double *a, const double *b, double *res) {
        return ntd_dot(h, a, b, res, stream);
    };
    *inner_iters = 0;
    *lambda = 0.0;
    double m = 0.0;
    TST(signed_maxabs(v, n, h->partials, &m, s));     // start from v / (its largest entry)
    if (!(m != 0.0) || !isfinite(m)) return NTD_EINVAL;
    hipLaunchKernelGGL(k_tgt_scale, dim3(nb), dim3(kTB), 0, s, v, 1.0 / m, -2.0, n);
    TCK(hipGetLastError());
    for (int k = 0; k < outer; ++k) {
        // y = M^{-1} v by CG in the A-inner product from y = 0: r = v - M y,
        // s = A r, p (direction), u = A p, q = M p = B^{-1} u, w = A q.  (Once v
        // is close to the eigenvector the first step already finds y = v /
        // lambda, so a start at y = v / lambda would save nothing; it would add
        // the rounding error of computing v - M y, amplified by 1 / lambda.)
        TCK(hipMemsetAsync(y, 0, n * sizeof(double), s));
        TCK(hipMemcpyAsync(r, v, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        TST(ntd_spmv(h, r, sv, stream));
        TCK(hipMemcpyAsync(p, r, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        TCK(hipMemcpyAsync(u, sv, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        double rho = 0.0;
        TST(dot(r, sv, &rho));
        const double vAv = rho;
        if (!(vAv > 0.0) || !isfinite(vAv)) return NTD_EBREAKDOWN;
        int it = 0;
        while (it < inner_maxit && rho > 0.0 && sqrt(rho / vAv) > inner_tol) {
            TST(ntd_apply_ntd(h, u, q, stream));
            TST(ntd_spmv(h, q, w, stream));
            double uq = 0.0;
            TST(dot(u, q, &uq));
            if (!(uq > 0.0) || !isfinite(uq)) return NTD_EBREAKDOWN;
            const double a = rho / uq;
            hipLaunchKernelGGL(k_tgt_step, dim3(nb), dim3(kTB), 0, s, y, r, sv, p, q, w, a, n);
            TCK(hipGetLastError());
            double rho1 = 0.0;
            TST(dot(r, sv, &rho1));
            if (!(rho1 >= 0.0) || !isfinite(rho1)) return NTD_EBREAKDOWN;
            hipLaunchKernelGGL(k_tgt_dir, dim3(nb), dim3(kTB), 0, s, p, u, r, sv, rho1 / rho, n);
            TCK(hipGetLastError());
            rho = rho1;
            ++it;
        }
        *inner_iters += it;
        if (sqrt(rho / vAv) > inner_tol) return NTD_ENOCONV;
        // Rayleigh-type estimate of the smallest eigenvalue: v'Av / y'Av
        TST(ntd_spmv(h, v, w, stream));
        double yAv = 0.0;
        TST(dot(y, w, &yAv));
        if (!(yAv > 0.0) || !isfinite(yAv)) return NTD_EBREAKDOWN;
        *lambda = vAv / yAv;
        TST(signed_maxabs(y, n, h->partials, &m, s));
        if (!(m != 0.0) || !isfinite(m)) return NTD_EBREAKDOWN;
        const bool last = k + 1 == outer;
        hipLaunchKernelGGL(k_tgt_scale, dim3(nb), dim3(kTB), 0, s, y, 1.0 / m,
                           last ? floor_ : -2.0, n);
        TCK(hipGetLastError());
        TCK(hipMemcpyAsync(v, y, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    TCK(hipStreamSynchronize(s));
    return NTD_OK;
}
