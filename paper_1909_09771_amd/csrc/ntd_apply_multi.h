// ntd_apply_multi.h -- the batched sweeps with several right-hand sides of one
// system per wavefront.
//
// In a batch every right-hand side of a system reads the same line records.
// With one right-hand side per wavefront pair each of them loads every record
// itself.  Here one wavefront pair runs NR right-hand sides of one system (and
// level-3 half) through the same chain: each line step loads the line's record
// once and runs NR independent twisted solves with it, interleaved, so the
// record is loaded once per NR right-hand sides and the NR dependency chains
// fill each other's latency.  The pairs of one system mostly share their record
// reads in L2 already, so this pays only where the steps are short next to the
// loads; the batch's tuner chooses.  The steps, the twists and the memory
// layouts are those of ntd_apply.h.
#pragma once

#include "ntd_apply.h"

namespace ntd {

namespace {

// Inputs of one line step for NR right-hand sides: the shared coefficients
// and couplings, and three per-right-hand-side lines (their use depends on the
// sweep: see the policies below).
template <typename T, int EPL, int NR>
struct LineInM {
    T c0[EPL], c1[EPL], c2[EPL];  // 1/M, a, u
    T f[EPL];                     // y-coupling to the chain predecessor
    T g[EPL], g2[EPL];            // z-couplings (level 3)
    double mvj, cpj, cnj, seed;
    T q0[NR][EPL], q1[NR][EPL], q2[NR][EPL];
};

template <typename T, int EPL, int NR>
struct RecFmtM {
    using Ty = T;
    static constexpr int kEPL = EPL;
    static constexpr int kNR = NR;
    using R = RecFmt<T, EPL>;
    rsrc_t rec;
    rsrc_t W[NR];  // lower-sweep results of the plane, one buffer per right-hand side
    unsigned vA;
    __device__ RecFmtM() {
        const unsigned lane = threadIdx.x & 63;
        vA = lane * EPL * (unsigned)sizeof(T);
    }
    __device__ void load_coef(int m, LineInM<T, EPL, NR> &in) const {
        const unsigned so = (unsigned)m * R::kRec;
        vload(rec, vA + kRecMv * R::kArr, so, in.c0);
        vload(rec, vA + kRecP * R::kArr, so, in.c1);
        double tw[4];
        vload(rec, R::kTw, so, tw);
        in.mvj = tw[0];
        in.cpj = tw[1];
        in.cnj = tw[2];
        in.seed = tw[3];
    }
    // f of line m (up) or m-1 (down), 0 below line 0, as RecFmt::load_fc
    __device__ void load_fc(int m, bool up, T (&f)[EPL]) const {
        const int lc = up ? m : m - 1;
        vload(rec, lc < 0 ? kOOB : vA + kRecF * R::kArr, lc < 0 ? 0u : (unsigned)lc * R::kRec, f);
    }
    __device__ void load_w(int m, T (&w)[NR][EPL]) const {
#pragma unroll
        for (int q = 0; q < NR; ++q) vload(W[q], vA, (unsigned)m * R::kLine, w[q]);
    }
    __device__ void store_w(int m, int q, const T (&w)[EPL]) const {
        vstore(W[q], vA, (unsigned)m * R::kLine, w);
    }
    // the recurrence coefficients and scan multipliers of the step's line,
    // shared by its NR solves
    struct Prep {
        T a[EPL], u[EPL], m[kRecMul];
    };
    __device__ void prep(const LineInM<T, EPL, NR> &in, Prep &p) const {
        line_coefs(in.c0, in.c1, p.a, p.u);
        scan_mults(p.a, p.u, (T)in.seed, p.m);
    }
    __device__ void solve(const LineInM<T, EPL, NR> &in, const Prep &p, const T (&y)[EPL],
                          T (&x)[EPL]) const {
        solve_rec(p.a, in.c0, p.u, p.m, in.mvj, in.cpj, in.cnj, y, x);
    }
};

// RecFmtM with the level-2 lower results in LDS plane buffers, one per
// right-hand side (plane q at pl + q*ps), as RecFmtL.
template <typename T, int EPL, int NR>
struct RecFmtML : RecFmtM<T, EPL, NR> {
    T *pl;  // this lane's slots of line 0 of plane buffer 0
    int ps; // values per plane buffer (ny lines)
    __device__ void load_w(int m, T (&w)[NR][EPL]) const {
#pragma unroll
        for (int q = 0; q < NR; ++q) lds_ld<T, EPL>(pl + q * ps + m * 64 * EPL, w[q]);
    }
    __device__ void store_w(int m, int q, const T (&w)[EPL]) const {
        lds_st<T, EPL>(pl + q * ps + m * 64 * EPL, w);
    }
};

// Lower level-3 step of plane k for NR right-hand sides: rhs_q = r_q - g z_q(kn).
// LP: z_q(kn) comes from the LDS plane buffers (pl, ps as RecFmtML), and
// z_q(k) goes there too.
template <typename T, int EPL, int NR, bool HAS, bool LP = false>
struct PolLowerM {
    rsrc_t rp[NR], Zn[NR], Zk[NR], Gr;  // Gr: the records holding g
    unsigned vA, vG;
    T *pl;
    int ps;
    __device__ void load_rhs(int m, const RecFmtM<T, EPL, NR> &, LineInM<T, EPL, NR> &in) const {
        constexpr unsigned kLine = RecFmt<T, EPL>::kLine;
#pragma unroll
        for (int q = 0; q < NR; ++q) vload(rp[q], vA, (unsigned)m * kLine, in.q2[q]);
        if constexpr (HAS) {
            vload(Gr, vG, (unsigned)m * RecFmt<T, EPL>::kRec, in.g);
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                if constexpr (LP) lds_ld<T, EPL>(pl + q * ps + m * 64 * EPL, in.q1[q]);
                else vload(Zn[q], vA, (unsigned)m * kLine, in.q1[q]);
            }
        }
    }
    __device__ T rhs(const LineInM<T, EPL, NR> &in, int q, int s) const {
        if constexpr (HAS) return fmad(-in.g[s], in.q1[q][s], in.q2[q][s]);
        else return in.q2[q][s];
    }
    __device__ void load_out(int, const RecFmtM<T, EPL, NR> &, LineInM<T, EPL, NR> &) const {}
    __device__ void out(int m, int q, const T (&x)[EPL], const LineInM<T, EPL, NR> &) {
        vstore(Zk[q], vA, (unsigned)m * RecFmt<T, EPL>::kLine, x);
        if constexpr (LP) lds_st<T, EPL>(pl + q * ps + m * 64 * EPL, x);
    }
};

// The twist plane for NR right-hand sides.
template <typename T, int EPL, int NR>
struct PolTwistM {
    rsrc_t rp[NR], Zlo[NR], Zhi[NR], Zk[NR], Glo, Ghi;  // g of planes k-1 and k
    unsigned vA, vG;
    bool lo_nb, hi_nb;
    __device__ void load_rhs(int m, const RecFmtM<T, EPL, NR> &, LineInM<T, EPL, NR> &in) const {
        constexpr unsigned kLine = RecFmt<T, EPL>::kLine;
        const unsigned so = (unsigned)m * RecFmt<T, EPL>::kRec;
#pragma unroll
        for (int q = 0; q < NR; ++q) vload(rp[q], vA, (unsigned)m * kLine, in.q2[q]);
        if (lo_nb) {
            vload(Glo, vG, so, in.g);
#pragma unroll
            for (int q = 0; q < NR; ++q) vload(Zlo[q], vA, (unsigned)m * kLine, in.q1[q]);
        } else {
            zero_line(in.g);
#pragma unroll
            for (int q = 0; q < NR; ++q) zero_line(in.q1[q]);
        }
        if (hi_nb) {
            vload(Ghi, vG, so, in.g2);
#pragma unroll
            for (int q = 0; q < NR; ++q) vload(Zhi[q], vA, (unsigned)m * kLine, in.q0[q]);
        } else {
            zero_line(in.g2);
#pragma unroll
            for (int q = 0; q < NR; ++q) zero_line(in.q0[q]);
        }
    }
    __device__ T rhs(const LineInM<T, EPL, NR> &in, int q, int s) const {
        return fmad(-in.g2[s], in.q0[q][s], fmad(-in.g[s], in.q1[q][s], in.q2[q][s]));
    }
    __device__ void load_out(int, const RecFmtM<T, EPL, NR> &, LineInM<T, EPL, NR> &) const {}
    __device__ void out(int m, int q, const T (&x)[EPL], const LineInM<T, EPL, NR> &) {
        vstore(Zk[q], vA, (unsigned)m * RecFmt<T, EPL>::kLine, x);
    }
};

// Upper level-3 step of plane k for NR right-hand sides: c_q = Pt_k^{-1}(g x_q(kn)),
// x_q(k) = z_q(k) - c_q over Z_q.  q0 carries the level-2 lower result (load_w).
// LPN: x_q(kn) comes from the LDS plane buffers; LPO: x_q(k) goes there too.
template <typename T, int EPL, int NR, bool LPN = false, bool LPO = false>
struct PolUpperM {
    rsrc_t Zn[NR], Zk[NR], Gr;  // Gr: the records holding g (the lower of planes k, kn)
    unsigned vA, vG;
    T *pl;
    int ps;
    __device__ void load_rhs(int m, const RecFmtM<T, EPL, NR> &, LineInM<T, EPL, NR> &in) const {
        vload(Gr, vG, (unsigned)m * RecFmt<T, EPL>::kRec, in.g);
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            if constexpr (LPN) lds_ld<T, EPL>(pl + q * ps + m * 64 * EPL, in.q1[q]);
            else vload(Zn[q], vA, (unsigned)m * RecFmt<T, EPL>::kLine, in.q1[q]);
        }
    }
    __device__ T rhs(const LineInM<T, EPL, NR> &in, int q, int s) const {
        return in.g[s] * in.q1[q][s];
    }
    __device__ void load_out(int m, const RecFmtM<T, EPL, NR> &, LineInM<T, EPL, NR> &in) const {
#pragma unroll
        for (int q = 0; q < NR; ++q)
            vload(Zk[q], vA, (unsigned)m * RecFmt<T, EPL>::kLine, in.q2[q]);
    }
    __device__ void out(int m, int q, const T (&c)[EPL], const LineInM<T, EPL, NR> &in) {
        T xv[EPL];
#pragma unroll
        for (int s = 0; s < EPL; ++s) xv[s] = in.q2[q][s] - c[s];
        vstore(Zk[q], vA, (unsigned)m * RecFmt<T, EPL>::kLine, xv);
        if constexpr (LPO) lds_st<T, EPL>(pl + q * ps + m * 64 * EPL, xv);
    }
};

// plane_solve (ntd_sweep.h) for NR right-hand sides: the same two half chains
// and twist line, each step solving the NR lines of the step's line index with
// one set of coefficients; q0 carries the level-2 lower results into the upper
// steps.  lds holds 2 * 64 * EPL * NR values.
template <int DEPTH, class Fmt, class Pol>
__device__ void plane_solve_m(int ny, const Fmt &fmt, Pol &pol, typename Fmt::Ty *lds) {
    using T = typename Fmt::Ty;
    constexpr int EPL = Fmt::kEPL;
    constexpr int NR = Fmt::kNR;
    using In = LineInM<T, EPL, NR>;
    static_assert(DEPTH == 1 || DEPTH == 2, "prefetch depth");
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int j2 = (ny - 1) / 2;
    T y[NR][EPL], w[NR][EPL], prev[NR][EPL], fhi[EPL];
    In A, B;
    [[maybe_unused]] In C;
#pragma unroll
    for (int q = 0; q < NR; ++q) zero_line(prev[q]);
    auto L2 = [&](int q, int half, int s) -> T & {  // LDS slot of a half's line
        return lds[((q * 2 + half) * 64 + lane) * EPL + s];
    };

    auto load_lower = [&](int m, bool up, In &in) {
        pol.load_rhs(m, fmt, in);
        fmt.load_fc(m, up, in.f);
        fmt.load_coef(m, in);
    };
    auto load_upper = [&](int m, bool up, In &in) {
        fmt.load_w(m, in.q0);
        fmt.load_fc(m, up, in.f);
        fmt.load_coef(m, in);
        pol.load_out(m, fmt, in);
    };
    auto lower_step = [&](int m, const In &in) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
            for (int s = 0; s < EPL; ++s) y[q][s] = pol.rhs(in, q, s) - in.f[s] * prev[q][s];
        {
            typename Fmt::Prep pp;
            fmt.prep(in, pp);
#pragma unroll
            for (int q = 0; q < NR; ++q) fmt.solve(in, pp, y[q], w[q]);
        }
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            fmt.store_w(m, q, w[q]);
#pragma unroll
            for (int s = 0; s < EPL; ++s) prev[q][s] = w[q][s];
        }
    };
    auto upper_step = [&](int m, const In &in) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
            for (int s = 0; s < EPL; ++s) y[q][s] = in.f[s] * prev[q][s];
        {
            typename Fmt::Prep pp;
            fmt.prep(in, pp);
#pragma unroll
            for (int q = 0; q < NR; ++q) fmt.solve(in, pp, y[q], w[q]);
        }
#pragma unroll
        for (int q = 0; q < NR; ++q) {
#pragma unroll
            for (int s = 0; s < EPL; ++s) w[q][s] = in.q0[q][s] - w[q][s];
            pol.out(m, q, w[q], in);
#pragma unroll
            for (int s = 0; s < EPL; ++s) prev[q][s] = w[q][s];
        }
    };
    auto chain = [&](int count, bool tail, bool pre, auto &&load, auto &&step) {
        const int nl = count + (tail ? 1 : 0);
        if (nl <= 0) return;
        const int last = nl - 1;
        auto cl = [last](int i) { return i < last ? i : last; };
        if (!pre) load(0, A);
        if constexpr (DEPTH == 2) {
            __builtin_amdgcn_sched_barrier(0);
            load(cl(1), B);
            __builtin_amdgcn_sched_barrier(0);
            int i = 0;
            for (; i + 2 < count; i += 3) {
                load(cl(i + 2), C);
                step(i, A);
                load(cl(i + 3), A);
                step(i + 1, B);
                load(cl(i + 4), B);
                step(i + 2, C);
            }
            const int rest = count - i;
            if (rest >= 1) {
                if (i + 2 < nl) load(i + 2, C);
                step(i, A);
            }
            if (rest == 2) step(i + 1, B);
            if (tail) {
                if (rest == 1) A = B;
                else if (rest == 2) A = C;
            }
        } else {
            __builtin_amdgcn_sched_barrier(0);
            int i = 0;
            for (; i + 1 < count; i += 2) {
                load(cl(i + 1), B);
                step(i, A);
                load(cl(i + 2), A);
                step(i + 1, B);
            }
            if (i < count) {
                if (i + 1 < nl) load(i + 1, B);
                step(i, A);
                if (tail) A = B;
            }
        }
    };

    if (wv == 0) {
        chain(j2, true, false, [&](int i, In &in) { load_lower(i, false, in); },
              [&](int i, const In &in) { lower_step(i, in); });
        pol.load_out(j2, fmt, A);
        fmt.load_fc(j2, true, fhi);
    } else if (wv == 1) {
        chain(ny - 1 - j2, false, false, [&](int i, In &in) { load_lower(ny - 1 - i, true, in); },
              [&](int i, const In &in) { lower_step(ny - 1 - i, in); });
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
            for (int s = 0; s < EPL; ++s) L2(q, 1, s) = prev[q][s];
        if (j2 + 1 < ny) load_upper(j2 + 1, false, A);
    }
    __syncthreads();
    if (wv == 0) {  // the twist line takes both neighbours
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
            for (int s = 0; s < EPL; ++s)
                y[q][s] = pol.rhs(A, q, s) - A.f[s] * prev[q][s] - fhi[s] * L2(q, 1, s);
        {
            typename Fmt::Prep pp;
            fmt.prep(A, pp);
#pragma unroll
            for (int q = 0; q < NR; ++q) fmt.solve(A, pp, y[q], w[q]);
        }
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            pol.out(j2, q, w[q], A);
#pragma unroll
            for (int s = 0; s < EPL; ++s) {
                prev[q][s] = w[q][s];
                L2(q, 0, s) = w[q][s];
            }
        }
        if (j2 > 0) load_upper(j2 - 1, true, A);
    }
    __syncthreads();
    if (wv == 1) {
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
            for (int s = 0; s < EPL; ++s) prev[q][s] = L2(q, 0, s);
        chain(ny - 1 - j2, false, true, [&](int i, In &in) { load_upper(j2 + 1 + i, false, in); },
              [&](int i, const In &in) { upper_step(j2 + 1 + i, in); });
    } else if (wv == 0) {
        chain(j2, false, true, [&](int i, In &in) { load_upper(j2 - 1 - i, true, in); },
              [&](int i, const In &in) { upper_step(j2 - 1 - i, in); });
    }
}

// Prefetch depth: two lines ahead while three input buffers stay small.
template <typename T, int EPL, int NR>
constexpr int kApplyDepthM = (sizeof(T) * EPL * NR <= 32) ? 2 : 1;

template <typename T, int EPL, int NR, class Fmt = RecFmtM<T, EPL, NR>>
__device__ __forceinline__ Fmt rec_fmt_m(const ApplyArgs<T> (&a)[NR], int k) {
    Fmt F;
    F.rec = rec_plane<T, EPL>(a[0].rec, k, a[0].ny);
    return F;
}

// The plane format for NR right-hand sides; with LP the level-2 lower results
// go to the LDS plane buffers (pl, ps).
template <typename T, int EPL, int NR, bool LP>
using PlaneFmtM =
    typename std::conditional<LP, RecFmtML<T, EPL, NR>, RecFmtM<T, EPL, NR>>::type;

template <typename T, int EPL, int NR, bool LP>
__device__ __forceinline__ PlaneFmtM<T, EPL, NR, LP> plane_fmt_m(const ApplyArgs<T> (&a)[NR],
                                                                 int k, T *pl, int ps) {
    PlaneFmtM<T, EPL, NR, LP> F = rec_fmt_m<T, EPL, NR, PlaneFmtM<T, EPL, NR, LP>>(a, k);
    if constexpr (LP) {
        F.pl = pl;
        F.ps = ps;
    }
    return F;
}

template <typename T, int EPL, int NR, bool HAS, bool LP>
__device__ __forceinline__ void lower_plane_m(const ApplyArgs<T> (&a)[NR], int k, int kn, T *lds,
                                              T *pl) {
    constexpr unsigned kArr = RecFmt<T, EPL>::kArr;
    const int ny = a[0].ny;
    PolLowerM<T, EPL, NR, HAS, LP> pol;
    auto F = plane_fmt_m<T, EPL, NR, LP>(a, k, pl, ny * 64 * EPL);
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        pol.rp[q] = plane_rsrc<T, EPL>(a[q].rp, k, ny);
        pol.Zk[q] = plane_rsrc<T, EPL>(a[q].Z, k, ny);
        pol.Zn[q] = plane_rsrc<T, EPL>(a[q].Z, HAS ? kn : k, ny);
        F.W[q] = pol.Zk[q];
    }
    pol.pl = pl;
    pol.ps = ny * 64 * EPL;
    pol.Gr = rec_plane<T, EPL>(a[0].rec, kn < k ? kn : k, ny);
    pol.vA = F.vA;
    pol.vG = F.vA + kRecG * kArr;
    plane_solve_m<kApplyDepthM<T, EPL, NR>>(ny, F, pol, lds);
}

// With LP, pl is this lane's slots of the first of NR LDS plane buffers of ny
// lines each.
template <typename T, int EPL, int NR, bool LP = false>
__device__ __forceinline__ void apply_lower_m(const ApplyArgs<T> (&a)[NR], int h, T *lds,
                                              T *pl = nullptr) {
    const int nz = a[0].nz, j3 = (nz - 1) / 2;
    const int dk = h == 0 ? 1 : -1;
    const int k0 = h == 0 ? 0 : nz - 1;
    if (h == 0 ? k0 >= j3 : k0 <= j3) return;
    lower_plane_m<T, EPL, NR, false, LP>(a, k0, k0, lds, pl);
    for (int k = k0 + dk; h == 0 ? k < j3 : k > j3; k += dk)
        lower_plane_m<T, EPL, NR, true, LP>(a, k, k - dk, lds, pl);
}

template <typename T, int EPL, int NR>
__device__ __forceinline__ void apply_twist_m(const ApplyArgs<T> (&a)[NR], T *lds) {
    constexpr unsigned kArr = RecFmt<T, EPL>::kArr;
    const int ny = a[0].ny, nz = a[0].nz, k = (nz - 1) / 2;
    PolTwistM<T, EPL, NR> pol;
    RecFmtM<T, EPL, NR> F = rec_fmt_m<T, EPL, NR>(a, k);
    pol.lo_nb = k > 0;
    pol.hi_nb = k < nz - 1;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        pol.rp[q] = plane_rsrc<T, EPL>(a[q].rp, k, ny);
        pol.Zk[q] = plane_rsrc<T, EPL>(a[q].Z, k, ny);
        pol.Zlo[q] = plane_rsrc<T, EPL>(a[q].Z, pol.lo_nb ? k - 1 : k, ny);
        pol.Zhi[q] = plane_rsrc<T, EPL>(a[q].Z, pol.hi_nb ? k + 1 : k, ny);
        F.W[q] = pol.Zk[q];
    }
    pol.Glo = rec_plane<T, EPL>(a[0].rec, pol.lo_nb ? k - 1 : k, ny);
    pol.Ghi = F.rec;
    pol.vA = F.vA;
    pol.vG = F.vA + kRecG * kArr;
    plane_solve_m<kApplyDepthM<T, EPL, NR>>(ny, F, pol, lds);
}

template <typename T, int EPL, int NR, bool LPN, bool LP>
__device__ __forceinline__ void upper_plane_m(const ApplyArgs<T> (&a)[NR], int h, int k, int kn,
                                              T *lds, T *pl) {
    constexpr unsigned kArr = RecFmt<T, EPL>::kArr;
    const int ny = a[0].ny;
    PolUpperM<T, EPL, NR, LPN, LP> pol;
    auto F = plane_fmt_m<T, EPL, NR, LP>(a, k, pl, ny * 64 * EPL);
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        pol.Zk[q] = plane_rsrc<T, EPL>(a[q].Z, k, ny);
        pol.Zn[q] = plane_rsrc<T, EPL>(a[q].Z, kn, ny);
        F.W[q] = make_rsrc(a[q].scratch + (size_t)h * ny * 64 * EPL);
    }
    pol.pl = pl;
    pol.ps = ny * 64 * EPL;
    pol.Gr = rec_plane<T, EPL>(a[0].rec, kn < k ? kn : k, ny);
    pol.vA = F.vA;
    pol.vG = F.vA + kRecG * kArr;
    plane_solve_m<kApplyDepthM<T, EPL, NR>>(ny, F, pol, lds);
}

// With LP the first plane reads the twist plane from Z and the others their
// neighbour from the LDS plane buffers.
template <typename T, int EPL, int NR, bool LP = false>
__device__ __forceinline__ void apply_upper_m(const ApplyArgs<T> (&a)[NR], int h, T *lds,
                                              T *pl = nullptr) {
    const int nz = a[0].nz, j3 = (nz - 1) / 2;
    const int dk = h == 0 ? -1 : 1;
    for (int k = j3 + dk; k >= 0 && k < nz; k += dk) {
        const int kn = k - dk;
        if (LP && kn != j3) upper_plane_m<T, EPL, NR, LP, LP>(a, h, k, kn, lds, pl);
        else upper_plane_m<T, EPL, NR, false, LP>(a, h, k, kn, lds, pl);
    }
}

// Workgroup w runs right-hand sides q0..q0+NR-1 of system s, level-3 half h
// (halves = 2), or the twist plane (halves = 1): group g = w / halves with
// g = s * (nrhs / NR) + (q0 / NR).  The group's entries are s*nrhs + q0 + r.
// The block returns when none of its entries is active; inactive entries of a
// partly active group are swept too (their buffers are their own and their
// results unused).
template <typename T, int NR>
__device__ __forceinline__ bool multi_slot(const ApplyArgs<T> *tab, const int *active, int count,
                                           int nrhs, int halves, ApplyArgs<T> (&a)[NR], int &h) {
    const int groups_per_sys = nrhs / NR;
    const int g = blockIdx.x / halves;
    h = blockIdx.x % halves;
    if (g >= count * groups_per_sys) return false;
    const int e0 = (g / groups_per_sys) * nrhs + (g % groups_per_sys) * NR;
    bool any = false;
#pragma unroll
    for (int q = 0; q < NR; ++q) any = any || entry_active(active, e0 + q);
    if (!any) return false;
#pragma unroll
    for (int q = 0; q < NR; ++q) a[q] = load_uniform(tab + e0 + q);
    return true;
}

template <typename T, int EPL, int NR>
__global__ void __launch_bounds__(kApplyThreads) k_apply_lower_bm(const ApplyArgs<T> *tab,
                                                                  const int *active, int count,
                                                                  int nrhs) {
    __shared__ T lds[2 * 64 * EPL * NR];
    ApplyArgs<T> a[NR];
    int h;
    if (!multi_slot<T, NR>(tab, active, count, nrhs, 2, a, h)) return;
    apply_lower_m<T, EPL, NR>(a, h, lds);
}
template <typename T, int EPL, int NR>
__global__ void __launch_bounds__(kApplyThreads) k_apply_twist_bm(const ApplyArgs<T> *tab,
                                                                  const int *active, int count,
                                                                  int nrhs) {
    __shared__ T lds[2 * 64 * EPL * NR];
    ApplyArgs<T> a[NR];
    int h;
    if (!multi_slot<T, NR>(tab, active, count, nrhs, 1, a, h)) return;
    apply_twist_m<T, EPL, NR>(a, lds);
}
template <typename T, int EPL, int NR>
__global__ void __launch_bounds__(kApplyThreads) k_apply_upper_bm(const ApplyArgs<T> *tab,
                                                                  const int *active, int count,
                                                                  int nrhs) {
    __shared__ T lds[2 * 64 * EPL * NR];
    ApplyArgs<T> a[NR];
    int h;
    if (!multi_slot<T, NR>(tab, active, count, nrhs, 2, a, h)) return;
    apply_upper_m<T, EPL, NR>(a, h, lds);
}

// The same with NR plane buffers in dynamic LDS: the twist exchange
// (2*64*EPL*NR values), then NR planes of the group's ny lines.
template <typename T, int EPL, int NR>
__global__ void __launch_bounds__(kApplyThreads) k_apply_lower_bml(const ApplyArgs<T> *tab,
                                                                   const int *active, int count,
                                                                   int nrhs) {
    T *lds = (T *)ntd_plane_lds;
    T *pl = lds + 2 * 64 * EPL * NR + (threadIdx.x & 63) * EPL;
    ApplyArgs<T> a[NR];
    int h;
    if (!multi_slot<T, NR>(tab, active, count, nrhs, 2, a, h)) return;
    apply_lower_m<T, EPL, NR, true>(a, h, lds, pl);
}
template <typename T, int EPL, int NR>
__global__ void __launch_bounds__(kApplyThreads) k_apply_upper_bml(const ApplyArgs<T> *tab,
                                                                   const int *active, int count,
                                                                   int nrhs) {
    T *lds = (T *)ntd_plane_lds;
    T *pl = lds + 2 * 64 * EPL * NR + (threadIdx.x & 63) * EPL;
    ApplyArgs<T> a[NR];
    int h;
    if (!multi_slot<T, NR>(tab, active, count, nrhs, 2, a, h)) return;
    apply_upper_m<T, EPL, NR, true>(a, h, lds, pl);
}

// The sweeps of a batch with NR right-hand sides per wavefront pair (nrhs a
// multiple of NR), as three launches; ev (optional, 4 events) brackets them.
// plane_lds > 0: the lower and upper sweeps keep their NR planes in that many
// bytes of LDS (NR * plane_lds_bytes of the largest ny, after
// apply_batch_multi_lds_impl has allowed it).
template <typename T, int EPL, int NR>
hipError_t apply_batch_multi_impl(const ApplyArgs<T> *tab, const int *active, int count, int nrhs,
                                  size_t plane_lds, hipStream_t s, hipEvent_t *ev) {
    const dim3 g2(2 * (unsigned)(count * (nrhs / NR))), g1((unsigned)(count * (nrhs / NR)));
    const dim3 blk(kApplyThreads);
    if (ev) (void)hipEventRecord(ev[0], s);
    if (plane_lds)
        hipLaunchKernelGGL((k_apply_lower_bml<T, EPL, NR>), g2, blk, plane_lds, s, tab, active,
                           count, nrhs);
    else
        hipLaunchKernelGGL((k_apply_lower_bm<T, EPL, NR>), g2, blk, 0, s, tab, active, count, nrhs);
    if (ev) (void)hipEventRecord(ev[1], s);
    hipLaunchKernelGGL((k_apply_twist_bm<T, EPL, NR>), g1, blk, 0, s, tab, active, count, nrhs);
    if (ev) (void)hipEventRecord(ev[2], s);
    if (plane_lds)
        hipLaunchKernelGGL((k_apply_upper_bml<T, EPL, NR>), g2, blk, plane_lds, s, tab, active,
                           count, nrhs);
    else
        hipLaunchKernelGGL((k_apply_upper_bm<T, EPL, NR>), g2, blk, 0, s, tab, active, count, nrhs);
    if (ev) (void)hipEventRecord(ev[3], s);
    return hipGetLastError();
}

template <typename T, int EPL, int NR>
hipError_t apply_batch_multi_lds_impl(size_t bytes) {
    hipError_t e = hipFuncSetAttribute((const void *)&k_apply_lower_bml<T, EPL, NR>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)&k_apply_upper_bml<T, EPL, NR>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    return e;
}

}  // namespace

}  // namespace ntd
