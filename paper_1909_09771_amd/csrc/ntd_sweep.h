// ntd_sweep.h -- device templates of the nested twisted sweeps of the preconditioner
// (arXiv:1909.09771, Sec. 2.2, Algorithms 1-7) and its factorization (Sec. 2.1).
//
// Execution model on gfx950.  The sweeps are one long chain of dependent line
// solves: plane k of a level-3 sweep needs the finished plane k-1, line m of a
// level-2 sweep the finished line m-1.  The twists at levels 3 and 2 split each
// chain into two independent halves, so four chains run at once:
//   * a level-3 half (planes below / above the twist plane) is one workgroup;
//   * a level-2 half (lines below / above the twist line) is one wavefront of
//     that workgroup; the two wavefronts meet at the twist line through LDS;
//   * one line (level 1) is solved by one wavefront: lanes 0-31 hold the chain
//     from element 0 up to the twist element j = floor((nx-1)/2), lanes 32-63
//     the chain from element nx-1 down to j+1, EPL consecutive chain positions
//     per lane.  Each of the two recurrences of the twisted tridiagonal solve
//     is an affine map x_c = a_c x_{c-1} + b_c along a chain, evaluated as a
//     lane-local composition plus a 32-lane inclusive scan of affine maps.
// The level-3 twist plane and the switch from the lower to the upper level-3
// sweep are kernel boundaries (lower halves, twist plane, upper halves), so no
// workgroup ever waits for another.
#pragma once

#include "ntd_internal.h"

namespace ntd {

namespace {

constexpr int kApplyThreads = 128;  // two wavefronts: the two level-2 half chains
constexpr int kSetupThreads = 256;  // two chain wavefronts + two helpers for plane-wide work

// ---------------------------------------------------------------------------
// Level 1: one line per wavefront.
// ---------------------------------------------------------------------------

struct LineGeom {
    int n;     // line length (nx)
    int ca;    // chain A length: elements 0..j (j = ca - 1 is the twist element)
    int cb;    // chain B length: elements n-1 down to j+1
    int half;  // 0: this lane holds chain A, 1: chain B
    int hl;    // lane index inside the half, 0..31
    int cnt;   // length of this lane's chain
    __device__ explicit LineGeom(int n_) : n(n_) {
        ca = (n_ + 1) / 2;
        cb = n_ - ca;
        int lane = threadIdx.x & 63;
        half = lane >> 5;
        hl = lane & 31;
        cnt = half ? cb : ca;
    }
    __device__ __forceinline__ int pos(int s, int epl) const { return hl * epl + s; }
    __device__ __forceinline__ bool ok(int c) const { return c < cnt; }
    __device__ __forceinline__ int elem(int c) const { return half ? n - 1 - c : c; }
};

template <typename T, int EPL>
__device__ __forceinline__ T pick(const T (&v)[EPL], int s) {
    T r = v[0];
#pragma unroll
    for (int q = 1; q < EPL; ++q)
        if (q == s) r = v[q];
    return r;
}

template <typename T, int EPL>
__device__ __forceinline__ void put(T (&v)[EPL], int s, T x) {
#pragma unroll
    for (int q = 0; q < EPL; ++q)
        if (q == s) v[q] = x;
}

// Load v[s] = src[element of slot s] (0 outside the chain).
template <typename T, int EPL>
__device__ __forceinline__ void load_line(const LineGeom &G, const T *__restrict__ src,
                                          T (&v)[EPL]) {
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        int c = G.pos(s, EPL);
        v[s] = G.ok(c) ? src[G.elem(c)] : T(0);
    }
}

template <typename T, int EPL>
__device__ __forceinline__ void store_line(const LineGeom &G, T *__restrict__ dst,
                                           const T (&v)[EPL]) {
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        int c = G.pos(s, EPL);
        if (G.ok(c)) dst[G.elem(c)] = v[s];
    }
}

// Coefficients of the line solve T^{-1} y with T = (M + L1)(I + M^{-1} U1):
// mv = 1/M at the slot's element, cp = coupling to the chain predecessor
// (chain A: e1[e-1]; chain B: e1[e]), cn = coupling toward the twist
// (chain A: e1[e]; chain B: e1[e-1]); mvj = FP64 1/M of the twist element.
template <typename T, int EPL>
struct LineCoef {
    T mv[EPL], cp[EPL], cn[EPL];
    double mvj;
};

template <typename T, int EPL>
__device__ __forceinline__ void load_coef(const LineGeom &G, const T *__restrict__ e1,
                                          const T *__restrict__ mv,
                                          const double *__restrict__ mv64,
                                          LineCoef<T, EPL> &C) {
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        int c = G.pos(s, EPL);
        bool ok = G.ok(c);
        int e = G.elem(c);
        C.mv[s] = ok ? mv[e] : T(0);
        if (G.half == 0) {
            C.cp[s] = (ok && e > 0) ? e1[e - 1] : T(0);
            C.cn[s] = ok ? e1[e] : T(0);
        } else {
            C.cp[s] = ok ? e1[e] : T(0);
            C.cn[s] = ok ? e1[e - 1] : T(0);
        }
    }
    C.mvj = mv64[G.ca - 1];
}

// Inclusive scan of affine maps over the 32 lanes of each half, forward
// (lane hl composes lanes 0..hl): x -> A x + B.
template <typename T>
__device__ __forceinline__ void scan_fwd32(T &A, T &B, int hl) {
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
        T Ap = __shfl_up(A, off, 32);
        T Bp = __shfl_up(B, off, 32);
        if (hl >= off) {
            B = A * Bp + B;
            A = A * Ap;
        }
    }
}

// Same, backward (lane hl composes lanes hl..31).
template <typename T>
__device__ __forceinline__ void scan_bwd32(T &U, T &G, int hl) {
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
        T Un = __shfl_down(U, off, 32);
        T Gn = __shfl_down(G, off, 32);
        if (hl + off < 32) {
            G = U * Gn + G;
            U = U * Un;
        }
    }
}

// x = T^{-1} y for one line held by the calling wavefront (all 64 lanes).
// Lower sweep: g_c = a_c g_{c-1} + b_c along each chain toward the twist with
// a_c = -cp/M, b_c = y/M; the twist row takes both neighbours, in FP64.
// Upper sweep: x_c = u_c x_{c+1} + g_c from the twist outward, u_c = -cn/M,
// the top of chain B being seeded with the twist value.
template <typename T, int EPL>
__device__ __forceinline__ void line_solve(const LineGeom &G, const LineCoef<T, EPL> &C,
                                           const T (&y)[EPL], T (&x)[EPL]) {
    T a[EPL], g[EPL], gm1[EPL];
    T A = T(1), B = T(0);
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        bool ok = G.ok(G.pos(s, EPL));
        a[s] = ok ? -C.mv[s] * C.cp[s] : T(1);
        g[s] = ok ? C.mv[s] * y[s] : T(0);
        B = a[s] * B + g[s];
        A = a[s] * A;
    }
    scan_fwd32(A, B, G.hl);
    T carry = __shfl_up(B, 1, 32);
    if (G.hl == 0) carry = T(0);
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        gm1[s] = carry;
        g[s] = a[s] * carry + g[s];
        carry = g[s];
    }
    // Twist element j: chain A position ca-1, neighbour j+1 = last of chain B.
    const int cta = G.ca - 1, lt = cta / EPL, st = cta % EPL;
    T gB = T(0);
    if (G.cb > 0) {
        const int ctb = G.cb - 1;
        T v = pick(g, ctb % EPL);
        gB = __shfl(v, 32 + ctb / EPL, 64);
    }
    double gj = 0.0;
    if (G.half == 0 && G.hl == lt) {
        double yj = (double)pick(y, st), gjm1 = (double)pick(gm1, st);
        double cpj = (double)pick(C.cp, st), cnj = (double)pick(C.cn, st);
        gj = C.mvj * (yj - cpj * gjm1 - cnj * (double)gB);
        put(g, st, (T)gj);
    }
    gj = __shfl(gj, lt, 64);
    const T xj = (T)gj;
    T u[EPL];
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        bool ok = G.ok(G.pos(s, EPL));
        u[s] = ok ? -C.mv[s] * C.cn[s] : T(0);
        if (!ok) g[s] = T(0);
    }
    if (G.half == 0) {
        if (G.hl == lt) put(u, st, T(0));
    } else if (G.cb > 0) {
        const int ctb = G.cb - 1;
        if (G.hl == ctb / EPL) {
            const int sb = ctb % EPL;
            put(g, sb, pick(g, sb) + pick(u, sb) * xj);
            put(u, sb, T(0));
        }
    }
    T U = T(1), Gs = T(0);
#pragma unroll
    for (int s = EPL - 1; s >= 0; --s) {
        Gs = u[s] * Gs + g[s];
        U = u[s] * U;
    }
    scan_bwd32(U, Gs, G.hl);
    T xn = __shfl_down(Gs, 1, 32);
    if (G.hl == 31) xn = T(0);
#pragma unroll
    for (int s = EPL - 1; s >= 0; --s) {
        x[s] = u[s] * xn + g[s];
        xn = x[s];
    }
}

// ---------------------------------------------------------------------------
// Level 2: one plane per workgroup, two wavefronts (the two half chains).
// ---------------------------------------------------------------------------

// Solve Pt x = y for the plane whose factors start at e1p/mvp/mv64p/f2p:
//   lower: w_m = T_m^{-1}(y_m - f*w_{m-1}) for m < j2 (wave 0), mirrored for
//          m > j2 (wave 1), the twist line j2 taking both neighbours;
//   upper: x_{j2} = w_{j2}; x_m = w_m - T_m^{-1}(f*x_{m+-1}) outward.
// rhs(m, G, y) fills the right-hand side of line m; W (plane-sized) keeps the
// lower results; out(m, G, x) receives the final value of line m exactly once.
// All threads of the block must call it (it holds two block barriers).
template <typename T, int EPL, class Rhs, class Out>
__device__ void plane_solve(int nx, int ny, const T *__restrict__ e1p, const T *__restrict__ mvp,
                            const double *__restrict__ mv64p, const T *__restrict__ f2p,
                            T *__restrict__ W, Rhs rhs, Out out, T *lds /* [2][64*EPL] */) {
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const LineGeom G(nx);
    const int j2 = (ny - 1) / 2;
    T y[EPL], w[EPL], prev[EPL], f[EPL];
    LineCoef<T, EPL> C;
#pragma unroll
    for (int s = 0; s < EPL; ++s) prev[s] = T(0);

    if (wv == 0) {
        for (int m = 0; m < j2; ++m) {
            const long long lo = (long long)m * nx;
            rhs(m, G, y);
            if (m > 0) {
                load_line(G, f2p + lo - nx, f);
#pragma unroll
                for (int s = 0; s < EPL; ++s) y[s] -= f[s] * prev[s];
            }
            load_coef(G, e1p + lo, mvp + lo, mv64p + lo, C);
            line_solve(G, C, y, w);
            store_line(G, W + lo, w);
#pragma unroll
            for (int s = 0; s < EPL; ++s) prev[s] = w[s];
        }
    } else if (wv == 1) {
        for (int m = ny - 1; m > j2; --m) {
            const long long lo = (long long)m * nx;
            rhs(m, G, y);
            if (m < ny - 1) {
                load_line(G, f2p + lo, f);
#pragma unroll
                for (int s = 0; s < EPL; ++s) y[s] -= f[s] * prev[s];
            }
            load_coef(G, e1p + lo, mvp + lo, mv64p + lo, C);
            line_solve(G, C, y, w);
            store_line(G, W + lo, w);
#pragma unroll
            for (int s = 0; s < EPL; ++s) prev[s] = w[s];
        }
#pragma unroll
        for (int s = 0; s < EPL; ++s) lds[64 * EPL + lane * EPL + s] = prev[s];
    }
    __syncthreads();
    if (wv == 0) {  // twist line: both neighbours
        const long long lo = (long long)j2 * nx;
        rhs(j2, G, y);
        if (j2 > 0) {
            load_line(G, f2p + lo - nx, f);
#pragma unroll
            for (int s = 0; s < EPL; ++s) y[s] -= f[s] * prev[s];
        }
        if (j2 < ny - 1) {
            load_line(G, f2p + lo, f);
#pragma unroll
            for (int s = 0; s < EPL; ++s) y[s] -= f[s] * lds[64 * EPL + lane * EPL + s];
        }
        load_coef(G, e1p + lo, mvp + lo, mv64p + lo, C);
        line_solve(G, C, y, w);
        out(j2, G, w);
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
            prev[s] = w[s];
            lds[lane * EPL + s] = w[s];
        }
    }
    __syncthreads();
    if (wv == 1) {
#pragma unroll
        for (int s = 0; s < EPL; ++s) prev[s] = lds[lane * EPL + s];
        for (int m = j2 + 1; m < ny; ++m) {
            const long long lo = (long long)m * nx;
            load_line(G, f2p + lo - nx, f);
#pragma unroll
            for (int s = 0; s < EPL; ++s) y[s] = f[s] * prev[s];
            load_coef(G, e1p + lo, mvp + lo, mv64p + lo, C);
            line_solve(G, C, y, w);
            load_line(G, W + lo, f);
#pragma unroll
            for (int s = 0; s < EPL; ++s) w[s] = f[s] - w[s];
            out(m, G, w);
#pragma unroll
            for (int s = 0; s < EPL; ++s) prev[s] = w[s];
        }
    } else if (wv == 0) {
        for (int m = j2 - 1; m >= 0; --m) {
            const long long lo = (long long)m * nx;
            load_line(G, f2p + lo, f);
#pragma unroll
            for (int s = 0; s < EPL; ++s) y[s] = f[s] * prev[s];
            load_coef(G, e1p + lo, mvp + lo, mv64p + lo, C);
            line_solve(G, C, y, w);
            load_line(G, W + lo, f);
#pragma unroll
            for (int s = 0; s < EPL; ++s) w[s] = f[s] - w[s];
            out(m, G, w);
#pragma unroll
            for (int s = 0; s < EPL; ++s) prev[s] = w[s];
        }
    }
}

// Wave-level sum (fixed butterfly order) of a double.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Level 3: the apply z = B^{-1} r as three launches.
// ---------------------------------------------------------------------------

// Lower level-3 sweep of one half: block 0 takes planes 0..j3-1 upward, block 1
// planes nz-1..j3+1 downward; z_k = Pt_k^{-1}(r_k - g3 * z_{k-+1}) into Z.
template <typename T, int EPL>
__global__ void __launch_bounds__(kApplyThreads) k_apply_lower(ApplyArgs<T> a) {
    __shared__ T lds[2 * 64 * EPL];
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long long nxy = (long long)nx * ny;
    const int j3 = (nz - 1) / 2;
    const int h = blockIdx.x;
    const int k0 = h == 0 ? 0 : nz - 1;
    const int kend = h == 0 ? j3 : j3;  // exclusive bound, walked toward the twist
    const int dk = h == 0 ? 1 : -1;
    for (int k = k0; h == 0 ? k < kend : k > kend; k += dk) {
        const long long pk = k * nxy;
        const int kn = k - dk;  // neighbour already solved (toward the chain start)
        const bool has = (kn >= 0 && kn < nz);
        const long long pn = kn * nxy, pc = (has ? (k < kn ? k : kn) : 0) * nxy;
        auto rhs = [&](int m, const LineGeom &G, T (&y)[EPL]) {
            const long long lo = (long long)m * nx;
#pragma unroll
            for (int s = 0; s < EPL; ++s) {
                int c = G.pos(s, EPL);
                if (G.ok(c)) {
                    long long e = lo + G.elem(c);
                    T v = (T)a.r[pk + e];
                    if (has) v -= a.g3[pc + e] * a.Z[pn + e];
                    y[s] = v;
                } else {
                    y[s] = T(0);
                }
            }
        };
        auto out = [&](int m, const LineGeom &G, const T (&x)[EPL]) {
            store_line(G, a.Z + pk + (long long)m * nx, x);
        };
        plane_solve<T, EPL>(nx, ny, a.e1 + pk, a.mv + pk, a.mv64 + pk, a.f2 + pk, a.Z + pk, rhs,
                            out, lds);
    }
}

// The twist plane j3 takes both neighbours; its result is final.
template <typename T, int EPL>
__global__ void __launch_bounds__(kApplyThreads) k_apply_twist(ApplyArgs<T> a) {
    __shared__ T lds[2 * 64 * EPL];
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long long nxy = (long long)nx * ny;
    const int k = (nz - 1) / 2;
    const long long pk = k * nxy;
    const bool lo_nb = k > 0, hi_nb = k < nz - 1;
    double acc = 0.0;
    auto rhs = [&](int m, const LineGeom &G, T (&y)[EPL]) {
        const long long lo = (long long)m * nx;
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
            int c = G.pos(s, EPL);
            if (G.ok(c)) {
                long long e = lo + G.elem(c);
                T v = (T)a.r[pk + e];
                if (lo_nb) v -= a.g3[pk - nxy + e] * a.Z[pk - nxy + e];
                if (hi_nb) v -= a.g3[pk + e] * a.Z[pk + nxy + e];
                y[s] = v;
            } else {
                y[s] = T(0);
            }
        }
    };
    auto out = [&](int m, const LineGeom &G, const T (&x)[EPL]) {
        const long long lo = pk + (long long)m * nx;
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
            int c = G.pos(s, EPL);
            if (G.ok(c)) {
                long long e = lo + G.elem(c);
                a.Z[e] = x[s];
                double xd = (double)x[s];
                if ((void *)a.zout != (void *)a.Z) a.zout[e] = xd;
                acc += a.r[e] * xd;
            }
        }
    };
    plane_solve<T, EPL>(nx, ny, a.e1 + pk, a.mv + pk, a.mv64 + pk, a.f2 + pk, a.Z + pk, rhs, out,
                        lds);
    if (a.partials) {
        double sum = wave_sum(acc);
        if ((threadIdx.x & 63) == 0) a.partials[threadIdx.x >> 6] = sum;
    }
}

// Upper level-3 sweep: block 0 takes planes j3-1..0, block 1 planes j3+1..nz-1;
// x_k = z_k - Pt_k^{-1}(g3 * x_{k+-1}), written over Z (and zout).
template <typename T, int EPL>
__global__ void __launch_bounds__(kApplyThreads) k_apply_upper(ApplyArgs<T> a) {
    __shared__ T lds[2 * 64 * EPL];
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long long nxy = (long long)nx * ny;
    const int j3 = (nz - 1) / 2;
    const int h = blockIdx.x;
    const int dk = h == 0 ? -1 : 1;
    T *W = a.scratch + h * nxy;
    double acc = 0.0;
    for (int k = j3 + dk; k >= 0 && k < nz; k += dk) {
        const long long pk = k * nxy;
        const int kn = k - dk;  // final neighbour, toward the twist plane
        const long long pn = kn * nxy, pc = (k < kn ? k : kn) * nxy;
        auto rhs = [&](int m, const LineGeom &G, T (&y)[EPL]) {
            const long long lo = (long long)m * nx;
#pragma unroll
            for (int s = 0; s < EPL; ++s) {
                int c = G.pos(s, EPL);
                if (G.ok(c)) {
                    long long e = lo + G.elem(c);
                    y[s] = a.g3[pc + e] * a.Z[pn + e];
                } else {
                    y[s] = T(0);
                }
            }
        };
        auto out = [&](int m, const LineGeom &G, const T (&cv)[EPL]) {
            const long long lo = pk + (long long)m * nx;
#pragma unroll
            for (int s = 0; s < EPL; ++s) {
                int c = G.pos(s, EPL);
                if (G.ok(c)) {
                    long long e = lo + G.elem(c);
                    T xv = a.Z[e] - cv[s];
                    a.Z[e] = xv;
                    double xd = (double)xv;
                    if ((void *)a.zout != (void *)a.Z) a.zout[e] = xd;
                    acc += a.r[e] * xd;
                }
            }
        };
        plane_solve<T, EPL>(nx, ny, a.e1 + pk, a.mv + pk, a.mv64 + pk, a.f2 + pk, W, rhs, out,
                            lds);
    }
    if (a.partials) {
        double sum = wave_sum(acc);
        if ((threadIdx.x & 63) == 0) a.partials[2 + 2 * h + (threadIdx.x >> 6)] = sum;
    }
}

// ---------------------------------------------------------------------------
// Factorization (Sec. 2.1).
// ---------------------------------------------------------------------------

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double tval(const double *t, long long p) { return t ? t[p] : 1.0; }

// Line m of plane k (one wavefront): T_m starts as the line block of P_k and
// loses, for each neighbour line nb, phi Y phi with g = (T_nb^{-1} v)./v,
// v = phi .* t_m, phi = the y-coupling of the two lines and Y = 2g - g T_nb g
// (Newton) or Y = g (diagonal); then the twisted pivots of T_m.
template <int EPL>
__device__ void line_setup(const SetupArgs &a, long long pk, int m, int nnb, int nb0, int nb1,
                           double *sh /* per-wave LDS: 5 * nx doubles */) {
    const int nx = a.nx;
    const LineGeom G(nx);
    const int lane = threadIdx.x & 63;
    double *sd = sh, *se = sh + nx, *sM = sh + 2 * nx, *sg = sh + 3 * nx, *sp = sh + 4 * nx;
    const long long lm = pk + (long long)m * nx;
    double dT[EPL], ev[EPL];
    load_line(G, a.dP + lm, dT);
    load_line(G, a.xP + lm, ev);
    for (int q = 0; q < nnb; ++q) {
        const int nb = q == 0 ? nb0 : nb1;
        const long long ln = pk + (long long)nb * nx;
        const long long lc = pk + (long long)(m < nb ? m : nb) * nx;
        double phi[EPL], v[EPL], zl[EPL], gam[EPL], dTn[EPL], en[EPL];
        load_line(G, a.f2 + lc, phi);
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
            int c = G.pos(s, EPL);
            v[s] = G.ok(c) ? phi[s] * tval(a.t, lm + G.elem(c)) : 0.0;
        }
        LineCoef<double, EPL> C;
        load_coef(G, a.e1 + ln, a.mv + ln, a.mv + ln, C);
        line_solve(G, C, v, zl);
        load_line(G, a.dT + ln, dTn);
        load_line(G, a.e1 + ln, en);
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
            bool ok = G.ok(G.pos(s, EPL));
            gam[s] = ok ? zl[s] / v[s] : 0.0;
        }
        if (a.schur == 1) {  // diagonal
#pragma unroll
            for (int s = 0; s < EPL; ++s) dT[s] -= phi[s] * phi[s] * gam[s];
        } else {
#pragma unroll
            for (int s = 0; s < EPL; ++s) {
                double yii = 2.0 * gam[s] - gam[s] * dTn[s] * gam[s];
                dT[s] -= phi[s] * yii * phi[s];
            }
            store_line(G, sg, gam);
            store_line(G, sp, phi);
            wave_sync();
#pragma unroll
            for (int s = 0; s < EPL; ++s) {
                int c = G.pos(s, EPL);
                int e = G.elem(c);
                if (G.ok(c) && e + 1 < nx) {
                    double yi1 = -gam[s] * en[s] * sg[e + 1];
                    ev[s] -= phi[s] * yi1 * sp[e + 1];
                }
            }
            wave_sync();
        }
    }
    // Twisted pivots: lane 0 walks chain A up to j-1, lane 32 chain B down to
    // j+1, then lane 0 takes the twist row with both neighbours.
    store_line(G, sd, dT);
    store_line(G, se, ev);
    wave_sync();
    const int j = G.ca - 1;
    if (G.hl == 0) {
        const int len = G.half ? G.cb : j;
        for (int q = 0; q < len; ++q) {
            const int i = G.half ? nx - 1 - q : q;
            double Mi;
            if (q == 0) {
                Mi = sd[i];
            } else {
                const int ip = G.half ? i + 1 : i - 1;
                const double ec = G.half ? se[i] : se[i - 1];
                Mi = sd[i] - ec * ec / sM[ip];
            }
            sM[i] = Mi;
        }
    }
    wave_sync();
    if (lane == 0) {
        double Mj = sd[j];
        if (j > 0) Mj -= se[j - 1] * se[j - 1] / sM[j - 1];
        if (j < nx - 1) Mj -= se[j] * se[j] / sM[j + 1];
        sM[j] = Mj;
    }
    wave_sync();
    double mv[EPL];
    bool bad = false;
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        int c = G.pos(s, EPL);
        if (G.ok(c)) {
            double M = sM[G.elem(c)];
            if (!(M > 0.0) || !isfinite(M)) bad = true;
            mv[s] = 1.0 / M;
        } else {
            mv[s] = 0.0;
        }
    }
    wave_sync();
    store_line(G, a.mv + lm, mv);
    store_line(G, a.dT + lm, dT);
    store_line(G, a.e1 + lm, ev);
    if (bad) atomicOr(a.flag, kFlagNotSPD);
}

// Level-2 factorization of plane k (the line recurrence of its P_k block).
template <int EPL>
__device__ void plane_lines_setup(const SetupArgs &a, int k, double *sh) {
    const int ny = a.ny;
    const long long pk = (long long)k * a.nx * ny;
    const int wv = threadIdx.x >> 6;
    const int j2 = (ny - 1) / 2;
    double *mine = sh + (wv & 1) * 5 * a.nx;
    if (wv == 0) {
        for (int m = 0; m < j2; ++m) line_setup<EPL>(a, pk, m, m > 0 ? 1 : 0, m - 1, 0, mine);
    } else if (wv == 1) {
        for (int m = ny - 1; m > j2; --m)
            line_setup<EPL>(a, pk, m, m < ny - 1 ? 1 : 0, m + 1, 0, mine);
    }
    __syncthreads();
    if (wv == 0) {
        int nnb = 0, n0 = 0, n1 = 0;
        if (j2 > 0) { n0 = j2 - 1; ++nnb; }
        if (j2 < ny - 1) { if (nnb == 0) n0 = j2 + 1; else n1 = j2 + 1; ++nnb; }
        line_setup<EPL>(a, pk, j2, nnb, n0, n1, mine);
    }
    __syncthreads();
}

// Plane k: P_k starts as D^_k and loses, for each neighbour plane nb,
// psi X psi with b = (Pt_nb^{-1} w)./w, w = psi .* t_k, psi = the z-coupling,
// X = 2b - b P_nb b (Newton, plus the diagonal compensation
// psi b (w - P_nb z)./t_k) or X = b (diagonal); then the level-2 recurrence.
template <int EPL>
__device__ void plane_setup(const SetupArgs &a, int k, int nnb, int nb0, int nb1, double *wbuf,
                            double *zbuf, double *lds_lines, double *lds_x) {
    const int nx = a.nx, ny = a.ny;
    const long long nxy = (long long)nx * ny;
    const long long pk = k * nxy;
    for (long long u = threadIdx.x; u < nxy; u += blockDim.x) {
        a.dP[pk + u] = a.d[pk + u];
        a.xP[pk + u] = a.ax[pk + u];
        a.f2[pk + u] = a.ay[pk + u];
    }
    __syncthreads();
    for (int q = 0; q < nnb; ++q) {
        const int nb = q == 0 ? nb0 : nb1;
        const long long pn = nb * nxy;
        const double *psi = a.az + (k < nb ? k : nb) * nxy;
        for (long long u = threadIdx.x; u < nxy; u += blockDim.x)
            wbuf[u] = psi[u] * tval(a.t, pk + u);
        __syncthreads();
        auto rhs = [&](int m, const LineGeom &G, double (&y)[EPL]) {
            load_line(G, wbuf + (long long)m * nx, y);
        };
        auto out = [&](int m, const LineGeom &G, const double (&x)[EPL]) {
            store_line(G, zbuf + (long long)m * nx, x);
        };
        plane_solve<double, EPL>(nx, ny, a.e1 + pn, a.mv + pn, a.mv + pn, a.f2 + pn, zbuf, rhs,
                                 out, lds_x);
        __syncthreads();
        const double *dPn = a.dP + pn, *xPn = a.xP + pn, *yPn = a.f2 + pn;
        for (long long u = threadIdx.x; u < nxy; u += blockDim.x) {
            const int i = (int)(u % nx), jl = (int)(u / nx);
            const double b = zbuf[u] / wbuf[u];
            if (a.schur == 1) {
                a.dP[pk + u] -= psi[u] * psi[u] * b;
                continue;
            }
            double Pz = dPn[u] * zbuf[u];
            if (i > 0) Pz += xPn[u - 1] * zbuf[u - 1];
            if (i < nx - 1) Pz += xPn[u] * zbuf[u + 1];
            if (jl > 0) Pz += yPn[u - nx] * zbuf[u - nx];
            if (jl < ny - 1) Pz += yPn[u] * zbuf[u + nx];
            const double xuu = 2.0 * b - b * dPn[u] * b;
            double dnew = a.dP[pk + u] - psi[u] * xuu * psi[u];
            if (i < nx - 1) {
                const double b1 = zbuf[u + 1] / wbuf[u + 1];
                const double x01 = -b * xPn[u] * b1;
                a.xP[pk + u] -= psi[u] * x01 * psi[u + 1];
            }
            if (jl < ny - 1) {
                const double bn = zbuf[u + nx] / wbuf[u + nx];
                const double x0n = -b * yPn[u] * bn;
                a.f2[pk + u] -= psi[u] * x0n * psi[u + nx];
            }
            dnew += psi[u] * b * (wbuf[u] - Pz) / tval(a.t, pk + u);
            a.dP[pk + u] = dnew;
        }
        __syncthreads();
    }
    plane_lines_setup<EPL>(a, k, lds_lines);
}

// Setup of the two level-3 half chains (block 0: planes 0..j3-1 upward, each
// with neighbour k-1; block 1: planes nz-1..j3+1 downward, neighbour k+1).
template <int EPL>
__global__ void __launch_bounds__(kSetupThreads) k_setup_halves(SetupArgs a) {
    extern __shared__ double smem[];
    double *lds_lines = smem;                  // 2 waves x 5 lines
    double *lds_x = smem + 10 * a.nx;          // 2 x 64*EPL exchange lines
    const long long nxy = (long long)a.nx * a.ny;
    const int j3 = (a.nz - 1) / 2;
    const int h = blockIdx.x;
    double *wbuf = a.scratch + (2 * h) * nxy, *zbuf = a.scratch + (2 * h + 1) * nxy;
    if (h == 0) {
        for (int k = 0; k < j3; ++k)
            plane_setup<EPL>(a, k, k > 0 ? 1 : 0, k - 1, 0, wbuf, zbuf, lds_lines, lds_x);
    } else {
        for (int k = a.nz - 1; k > j3; --k)
            plane_setup<EPL>(a, k, k < a.nz - 1 ? 1 : 0, k + 1, 0, wbuf, zbuf, lds_lines, lds_x);
    }
}

template <int EPL>
__global__ void __launch_bounds__(kSetupThreads) k_setup_twist(SetupArgs a) {
    extern __shared__ double smem[];
    double *lds_lines = smem;
    double *lds_x = smem + 10 * a.nx;
    const long long nxy = (long long)a.nx * a.ny;
    const int j3 = (a.nz - 1) / 2;
    int nnb = 0, n0 = 0, n1 = 0;
    if (j3 > 0) { n0 = j3 - 1; ++nnb; }
    if (j3 < a.nz - 1) { if (nnb == 0) n0 = j3 + 1; else n1 = j3 + 1; ++nnb; }
    plane_setup<EPL>(a, j3, nnb, n0, n1, a.scratch + 4 * nxy, a.scratch + 5 * nxy, lds_lines,
                     lds_x);
}

template <typename T, int EPL>
hipError_t apply_impl(const ApplyArgs<T> &a, hipStream_t s) {
    hipLaunchKernelGGL((k_apply_lower<T, EPL>), dim3(2), dim3(kApplyThreads), 0, s, a);
    hipLaunchKernelGGL((k_apply_twist<T, EPL>), dim3(1), dim3(kApplyThreads), 0, s, a);
    hipLaunchKernelGGL((k_apply_upper<T, EPL>), dim3(2), dim3(kApplyThreads), 0, s, a);
    return hipGetLastError();
}

template <int EPL>
hipError_t setup_impl(const SetupArgs &a, hipStream_t s) {
    size_t sh = sizeof(double) * (10 * (size_t)a.nx + 2 * 64 * EPL);
    if (sh > 65536) {
        hipFuncSetAttribute((const void *)k_setup_halves<EPL>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        hipFuncSetAttribute((const void *)k_setup_twist<EPL>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    }
    hipLaunchKernelGGL((k_setup_halves<EPL>), dim3(2), dim3(kSetupThreads), sh, s, a);
    hipLaunchKernelGGL((k_setup_twist<EPL>), dim3(1), dim3(kSetupThreads), sh, s, a);
    return hipGetLastError();
}

}  // namespace

// Supported elements per lane: a half chain holds up to 32*EPL positions.
#define NTD_EPL_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(10) X(12) X(14) X(16)

}  // namespace ntd
