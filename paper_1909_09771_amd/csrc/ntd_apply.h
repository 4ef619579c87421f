// ntd_apply.h -- the preconditioner apply z = B^{-1} r (arXiv:1909.09771, Sec. 2.2,
// Algorithms 1-7) on packed line records, the packing of the factors into
// those records, and the moves of right-hand side and result between the
// natural FP64 layout and the packed one.
//
// A line step is a chain of dependent operations run by one wavefront, and a
// wavefront issues at most one instruction every four cycles, so the step time
// is its instruction count.  Everything here serves to keep that count low:
//   * one record per line holds every factor the step reads (one buffer
//     descriptor, one scalar offset per line, no per-array address updates);
//   * the lane-level products of the recurrence coefficients do not depend on
//     the right-hand side, so the multipliers of every scan stage are
//     precomputed at packing: a stage is one zero-filling DPP move and one FMA;
//   * the twist row (FP64) exchanges its neighbours with one permlane32 swap
//     each way, and the twist and chain-B seed are inserted without branches;
//   * the sweeps read a packed right-hand side in the sweep precision and write
//     packed results only; the FP64 natural-layout gather, the ILU(0) base and
//     the r.z partials live in bandwidth-bound kernels before and after them.
#pragma once

#include <type_traits>

#include "ntd_sweep.h"

namespace ntd {

namespace {

constexpr int kApplyThreads = 128;  // two wavefronts: the two level-2 half chains
constexpr int kRowNewBcast0 = 0x150;  // broadcast lane 0 of each row within the row

// ---------------------------------------------------------------------------
// Cross-lane moves of the apply.
// ---------------------------------------------------------------------------

// DPP move in which a lane whose source lane does not exist reads 0.
template <int CTRL>
__device__ __forceinline__ float zmov(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double zmov(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xF, 0xF, true);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// permlane32 swap of v with itself: .lo gives every lane of the low half the
// value of the lane 32 above it, .hi gives every lane of the high half the value
// of the lane 32 below it.
struct Swap32f { float lo, hi; };
__device__ __forceinline__ Swap32f swap32(float v) {
    const unsigned u = __builtin_bit_cast(unsigned, v);
    const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    return {__builtin_bit_cast(float, (unsigned)r[1]), __builtin_bit_cast(float, (unsigned)r[0])};
}
struct Swap32d { double lo, hi; };
__device__ __forceinline__ Swap32d swap32(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned l = (unsigned)u, h = (unsigned)(u >> 32);
    const auto rl = __builtin_amdgcn_permlane32_swap(l, l, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(h, h, false, false);
    const unsigned long long lo = ((unsigned long long)(unsigned)rh[1] << 32) | (unsigned)rl[1];
    const unsigned long long hi = ((unsigned long long)(unsigned)rh[0] << 32) | (unsigned)rl[0];
    return {__builtin_bit_cast(double, lo), __builtin_bit_cast(double, hi)};
}

// Rows 0 and 2 receive rows 1 and 3 (lane i gets lane i+16); rows 1 and 3
// keep their own values.
__device__ __forceinline__ float rows_down16(float v) {
    const unsigned u = __builtin_bit_cast(unsigned, v);
    const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    return __builtin_bit_cast(float, (unsigned)r[1]);
}
__device__ __forceinline__ double rows_down16(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned l = (unsigned)u, h = (unsigned)(u >> 32);
    const auto rl = __builtin_amdgcn_permlane16_swap(l, l, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(h, h, false, false);
    return __builtin_bit_cast(double,
                              ((unsigned long long)(unsigned)rh[1] << 32) | (unsigned)rl[1]);
}

__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------------------
// Level 1: the twisted solve of one line on the packed layout.
// ---------------------------------------------------------------------------

// Per-lane multipliers (kRecMul values) of the two 32-lane scans.  With A_l the
// product of the lane's lower-sweep coefficients a and U_l that of its upper
// coefficients u, entry q < 4 of the forward set is the product of A over the
// 2^q lanes ending at this one (clipped at the start of its 16-lane row), entry
// 4 the product over the row up to this lane (0 in rows 0 and 2, which the
// cross-row step does not feed); the backward set 5..9 is the same over the
// lanes starting at this one toward the end of the row (entry 9 is 0 in rows 1
// and 3).  Entry 10 is the chain-B seed: in lane 63 the coefficient u of
// element j+1 (its coupling to the twist value), 0 elsewhere; in the packed u
// array that coefficient is replaced by 0.  They depend on the factors only,
// and are formed in the sweep from the loaded a and u (scan_mults): reading
// them from the record would add 44 B per lane to every line step's loads.
// The recurrence coefficients of the packed slots, from 1/M and the coupling p
// to the chain predecessor: a = -p/M (lower) and u = -p'/M (upper, p' that of
// the next chain position: the lane's next slot, or the next lane's first).
// The last slot of chain A (the twist element) takes p' from chain B's first
// slot and the last of chain B from beyond lane 63: both 0, the first as the
// twist row takes both couplings itself, the second as the chain-B seed does.
// Unused slots (1/M = 0) get a = u = 0: they hold zeros, and a zero a at a
// chain's start already cuts every scan window that reaches back into them.
template <typename T, int EPL>
__device__ __forceinline__ void line_coefs(const T (&mv)[EPL], const T (&p)[EPL], T (&a)[EPL],
                                           T (&u)[EPL]) {
    const T pn = zmov<kWaveShl1>(p[0]);  // the next lane's first coupling
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        a[s] = -mv[s] * p[s];
        u[s] = -mv[s] * (s + 1 < EPL ? p[s + 1] : pn);
    }
}

template <typename T, int EPL>
__device__ __forceinline__ void scan_mults(const T (&a)[EPL], const T (&u)[EPL], T seed,
                                           T (&m)[kRecMul]) {
    T A = T(1), U = T(1);
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        A *= a[s];
        U *= u[s];
    }
    m[0] = A;
    m[1] = m[0] * dpp<kRowShr1>(T(1), m[0]);
    m[2] = m[1] * dpp<kRowShr2>(T(1), m[1]);
    m[3] = m[2] * dpp<kRowShr4>(T(1), m[2]);
    m[4] = m[3] * dpp<kRowShr8>(T(1), m[3]);
    m[5] = U;
    m[6] = m[5] * dpp<kRowShl1>(T(1), m[5]);
    m[7] = m[6] * dpp<kRowShl2>(T(1), m[6]);
    m[8] = m[7] * dpp<kRowShl4>(T(1), m[7]);
    m[9] = m[8] * dpp<kRowShl8>(T(1), m[8]);
    const int lane = threadIdx.x & 63;
    const bool odd_row = ((lane >> 4) & 1) != 0;
    m[4] = odd_row ? m[4] : T(0);  // the forward cross-row step feeds rows 1 and 3
    m[9] = odd_row ? T(0) : m[9];  // the backward one rows 0 and 2
    m[10] = lane == 63 ? seed : T(0);
}
template <typename T>
__device__ __forceinline__ T scan_fwd(T B, const T (&m)[kRecMul]) {
    B = fmad(zmov<kRowShr1>(B), m[0], B);
    B = fmad(zmov<kRowShr2>(B), m[1], B);
    B = fmad(zmov<kRowShr4>(B), m[2], B);
    B = fmad(zmov<kRowShr8>(B), m[3], B);
    return fmad(zmov<kRowBcast15>(B), m[4], B);
}

template <typename T>
__device__ __forceinline__ T scan_bwd(T G, const T (&m)[kRecMul]) {
    G = fmad(zmov<kRowShl1>(G), m[5], G);
    G = fmad(zmov<kRowShl2>(G), m[6], G);
    G = fmad(zmov<kRowShl4>(G), m[7], G);
    G = fmad(zmov<kRowShl8>(G), m[8], G);
    return fmad(zmov<kRowNewBcast0>(rows_down16(G)), m[9], G);
}

// x = T^{-1} y for the line held by the wavefront (layout of LineGeom), given
// per slot a, 1/M and u as packed, the lane's multipliers, and the FP64 twist
// row (1/M_j and the couplings of element j to j-1 and j+1).
// Lower sweep: g_c = a_c g_{c-1} + y_c/M_c along each chain toward the twist,
// the twist row taking both neighbours in FP64; upper sweep: x_c = u_c x_{c+1}
// + g_c from the twist outward.
template <typename T, int EPL>
__device__ __forceinline__ void solve_rec(const T (&a)[EPL], const T (&mv)[EPL], const T (&u)[EPL],
                                          const T (&m)[kRecMul], double mvj, double cpj, double cnj,
                                          const T (&y)[EPL], T (&x)[EPL]) {
    constexpr int L = EPL - 1;
    const int lane = threadIdx.x & 63;
    T g[EPL];
#pragma unroll
    for (int s = 0; s < EPL; ++s) g[s] = mv[s] * y[s];
    T B = g[0];
#pragma unroll
    for (int s = 1; s < EPL; ++s) B = fmad(a[s], B, g[s]);
    B = scan_fwd(B, m);
    // lane 0 reads 0; lane 32 reads the end of chain A, which the zero a of
    // chain B's first element (or the unused slots before it) discards
    T carry = zmov<kWaveShr1>(B);
    T gm1 = carry;
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        if (s == L) gm1 = carry;
        g[s] = fmad(a[s], carry, g[s]);
        carry = g[s];
    }
    // twist element j: lane 31, slot L; element j+1 ends chain B in lane 63
    const T gB = swap32(g[L]).lo;
    const double gj = mvj * ((double)y[L] - cpj * (double)gm1 - cnj * (double)gB);
    const T xj = (T)gj;
    g[L] = lane == 31 ? xj : g[L];
    g[L] = fmad(m[10], swap32(xj).hi, g[L]);
    T G = g[L];
#pragma unroll
    for (int s = L - 1; s >= 0; --s) G = fmad(u[s], G, g[s]);
    G = scan_bwd(G, m);
    // lane 63 reads 0; lane 31 reads chain B, discarded by u = 0 at the twist
    T xn = zmov<kWaveShl1>(G);
#pragma unroll
    for (int s = L; s >= 0; --s) {
        x[s] = fmad(u[s], xn, g[s]);
        xn = x[s];
    }
}

// ---------------------------------------------------------------------------
// The packed format seen by plane_solve.
// ---------------------------------------------------------------------------

template <typename T, int EPL>
struct RecFmt {
    using Ty = T;
    static constexpr int kEPL = EPL;
    static constexpr unsigned kArr = rec_arr_bytes(sizeof(T), EPL);
    static constexpr unsigned kTw = rec_tw_off(sizeof(T), EPL);
    static constexpr unsigned kRec = rec_bytes(sizeof(T), EPL);
    static constexpr unsigned kLine = 64u * EPL * sizeof(T);
    rsrc_t rec;       // the records of the plane
    rsrc_t W;         // lower-sweep results of the plane
    unsigned vA;      // this lane's byte offset inside a packed array
    __device__ RecFmt() {
        const unsigned lane = threadIdx.x & 63;
        vA = lane * EPL * (unsigned)sizeof(T);
    }
    __device__ void load_coef(int m, LineIn<T, EPL> &in) const {
        const unsigned so = (unsigned)m * kRec;
        vload(rec, vA + kRecMv * kArr, so, in.c0);
        vload(rec, vA + kRecP * kArr, so, in.c1);
        double tw[4];
        vload(rec, kTw, so, tw);
        in.mvj = tw[0];
        in.cpj = tw[1];
        in.cnj = tw[2];
        in.seed = tw[3];
    }
    // y-coupling of line m to line m+1 (up) or m-1 (down): f of line m or m-1,
    // 0 below line 0 (an out-of-range offset: the load is still issued)
    __device__ void load_fc(int m, bool up, T (&f)[EPL]) const {
        const int lc = up ? m : m - 1;
        vload(rec, lc < 0 ? kOOB : vA + kRecF * kArr, lc < 0 ? 0u : (unsigned)lc * kRec, f);
    }
    __device__ void load_w(int m, T (&w)[EPL]) const { vload(W, vA, (unsigned)m * kLine, w); }
    __device__ void store_w(int m, const T (&w)[EPL]) const {
        vstore(W, vA, (unsigned)m * kLine, w);
    }
    __device__ void solve(const LineIn<T, EPL> &in, const T (&y)[EPL], T (&x)[EPL]) const {
        T a[EPL], u[EPL], m[kRecMul];
        line_coefs(in.c0, in.c1, a, u);
        scan_mults(a, u, (T)in.seed, m);
        solve_rec(a, in.c0, u, m, in.mvj, in.cpj, in.cnj, y, x);
    }
};

// One lane's EPL slots of a line in LDS.
template <typename T, int EPL>
__device__ __forceinline__ void lds_ld(const T *p, T (&v)[EPL]) {
#pragma unroll
    for (int s = 0; s < EPL; ++s) v[s] = p[s];
}
template <typename T, int EPL>
__device__ __forceinline__ void lds_st(T *p, const T (&v)[EPL]) {
#pragma unroll
    for (int s = 0; s < EPL; ++s) p[s] = v[s];
}

// The packed format with a plane buffer in LDS (batched sweeps whose planes fit
// the workgroup's LDS): line m of the plane at pl + m*64*EPL.  Along a level-3
// sweep the buffer holds, line by line, the finished neighbour plane's values,
// then the level-2 lower results written over them as each line's right-hand
// side is formed, then the plane's final values, which the next plane reads as
// its neighbour.  Each line is read and written by one wavefront only (the
// level-2 half that owns it), in program order, so no barrier guards it.
template <typename T, int EPL>
struct RecFmtL : RecFmt<T, EPL> {
    T *pl;  // this lane's slots of line 0
    __device__ void load_w(int m, T (&w)[EPL]) const { lds_ld<T, EPL>(pl + m * 64 * EPL, w); }
    __device__ void store_w(int m, const T (&w)[EPL]) const {
        lds_st<T, EPL>(pl + m * 64 * EPL, w);
    }
};

// Prefetch depth of the sweeps: two lines ahead while three input buffers fit
// the register file comfortably, else one.
template <typename T, int EPL>
constexpr int kApplyDepth = (sizeof(T) * EPL <= 16) ? 2 : 1;

// ---------------------------------------------------------------------------
// Level 3: three launches over the packed vectors.
// ---------------------------------------------------------------------------

template <typename T, int EPL>
__device__ __forceinline__ rsrc_t plane_rsrc(const T *base, int k, int ny) {
    return make_rsrc(base + (size_t)k * ny * 64 * EPL);
}

// The records of plane k.
template <typename T, int EPL>
__device__ __forceinline__ rsrc_t rec_plane(const void *rec, int k, int ny) {
    return make_rsrc((const char *)rec + (size_t)k * ny * RecFmt<T, EPL>::kRec);
}

template <typename T, int EPL, class Fmt = RecFmt<T, EPL>>
__device__ __forceinline__ Fmt rec_fmt(const ApplyArgs<T> &a, int k, rsrc_t W) {
    Fmt F;
    F.rec = rec_plane<T, EPL>(a.rec, k, a.ny);
    F.W = W;
    return F;
}

// Lower level-3 step of plane k: rhs = r_k - g * z_kn, with g the z-coupling of
// planes k and kn (absent for the first plane), held by the lower of the two.
// LP: z_kn comes from the LDS plane buffer, and z_k goes there too.
template <typename T, int EPL, bool HAS, bool LP = false>
struct PolLower {
    rsrc_t rp, Zn, Zk, Gr;  // Gr: the records holding g
    unsigned vA, vG;        // lane offsets: in a packed line; of g in a record
    T *pl;                  // LP: this lane's slots of the plane buffer
    __device__ void load_rhs(int m, const RecFmt<T, EPL> &, LineIn<T, EPL> &in) const {
        constexpr unsigned kLine = RecFmt<T, EPL>::kLine;
        vload(rp, vA, (unsigned)m * kLine, in.a2);
        if constexpr (HAS) {
            vload(Gr, vG, (unsigned)m * RecFmt<T, EPL>::kRec, in.a0);
            if constexpr (LP) lds_ld<T, EPL>(pl + m * 64 * EPL, in.a1);
            else vload(Zn, vA, (unsigned)m * kLine, in.a1);
        }
    }
    __device__ T rhs(const LineIn<T, EPL> &in, int s) const {
        if constexpr (HAS) return fmad(-in.a0[s], in.a1[s], in.a2[s]);
        else return in.a2[s];
    }
    __device__ void load_out(int, const RecFmt<T, EPL> &, LineIn<T, EPL> &) const {}
    __device__ void out(int m, const RecFmt<T, EPL> &, const T (&x)[EPL], const LineIn<T, EPL> &) {
        vstore(Zk, vA, (unsigned)m * RecFmt<T, EPL>::kLine, x);
        if constexpr (LP) lds_st<T, EPL>(pl + m * 64 * EPL, x);
    }
};

// The twist plane: rhs = r - g_dn * z_{k-1} - g_up * z_{k+1}; the result is final.
// g_dn is g of plane k-1 (records Glo), g_up g of plane k (records Ghi).
template <typename T, int EPL>
struct PolTwist {
    rsrc_t rp, Zlo, Zhi, Zk, Glo, Ghi;
    unsigned vA, vG;
    bool lo_nb, hi_nb;
    __device__ void load_rhs(int m, const RecFmt<T, EPL> &, LineIn<T, EPL> &in) const {
        constexpr unsigned kLine = RecFmt<T, EPL>::kLine;
        const unsigned so = (unsigned)m * RecFmt<T, EPL>::kRec;
        vload(rp, vA, (unsigned)m * kLine, in.a2);
        if (lo_nb) {
            vload(Glo, vG, so, in.a0);
            vload(Zlo, vA, (unsigned)m * kLine, in.a1);
        } else {
            zero_line(in.a0);
            zero_line(in.a1);
        }
        if (hi_nb) {
            vload(Ghi, vG, so, in.a3);
            vload(Zhi, vA, (unsigned)m * kLine, in.w);
        } else {
            zero_line(in.a3);
            zero_line(in.w);
        }
    }
    __device__ T rhs(const LineIn<T, EPL> &in, int s) const {
        return fmad(-in.a3[s], in.w[s], fmad(-in.a0[s], in.a1[s], in.a2[s]));
    }
    __device__ void load_out(int, const RecFmt<T, EPL> &, LineIn<T, EPL> &) const {}
    __device__ void out(int m, const RecFmt<T, EPL> &, const T (&x)[EPL], const LineIn<T, EPL> &) {
        vstore(Zk, vA, (unsigned)m * RecFmt<T, EPL>::kLine, x);
    }
};

// Upper level-3 step of plane k: c = Pt_k^{-1}(g * x_kn) with kn the final
// neighbour toward the twist plane; x_k = z_k - c over Z.
// LPN: x_kn comes from the LDS plane buffer; LPO: x_k goes there too.
template <typename T, int EPL, bool LPN = false, bool LPO = false>
struct PolUpper {
    rsrc_t Zn, Zk, Gr;  // Gr: the records holding g (the lower of planes k, kn)
    unsigned vA, vG;
    T *pl;              // LPN or LPO: this lane's slots of the plane buffer
    __device__ void load_rhs(int m, const RecFmt<T, EPL> &, LineIn<T, EPL> &in) const {
        vload(Gr, vG, (unsigned)m * RecFmt<T, EPL>::kRec, in.a0);
        if constexpr (LPN) lds_ld<T, EPL>(pl + m * 64 * EPL, in.a1);
        else vload(Zn, vA, (unsigned)m * RecFmt<T, EPL>::kLine, in.a1);
    }
    __device__ T rhs(const LineIn<T, EPL> &in, int s) const { return in.a0[s] * in.a1[s]; }
    __device__ void load_out(int m, const RecFmt<T, EPL> &, LineIn<T, EPL> &in) const {
        vload(Zk, vA, (unsigned)m * RecFmt<T, EPL>::kLine, in.a2);
    }
    __device__ void out(int m, const RecFmt<T, EPL> &, const T (&c)[EPL], const LineIn<T, EPL> &in) {
        T xv[EPL];
#pragma unroll
        for (int s = 0; s < EPL; ++s) xv[s] = in.a2[s] - c[s];
        vstore(Zk, vA, (unsigned)m * RecFmt<T, EPL>::kLine, xv);
        if constexpr (LPO) lds_st<T, EPL>(pl + m * 64 * EPL, xv);
    }
};

// The plane format: records in memory, the level-2 lower results in memory
// (W) or, with LP, in the LDS plane buffer pl (this lane's slots).
template <typename T, int EPL, bool LP>
using PlaneFmt = typename std::conditional<LP, RecFmtL<T, EPL>, RecFmt<T, EPL>>::type;

template <typename T, int EPL, bool LP>
__device__ __forceinline__ PlaneFmt<T, EPL, LP> plane_fmt(const ApplyArgs<T> &a, int k, rsrc_t W,
                                                          T *pl) {
    PlaneFmt<T, EPL, LP> F = rec_fmt<T, EPL, PlaneFmt<T, EPL, LP>>(a, k, W);
    if constexpr (LP) F.pl = pl;
    return F;
}

template <typename T, int EPL, bool HAS, bool LP>
__device__ __forceinline__ void lower_plane(const ApplyArgs<T> &a, int k, int kn, T *lds, T *pl) {
    constexpr unsigned kArr = RecFmt<T, EPL>::kArr;
    PolLower<T, EPL, HAS, LP> pol;
    pol.rp = plane_rsrc<T, EPL>(a.rp, k, a.ny);
    pol.Zk = plane_rsrc<T, EPL>(a.Z, k, a.ny);
    pol.Zn = plane_rsrc<T, EPL>(a.Z, HAS ? kn : k, a.ny);
    pol.pl = pl;
    const auto F = plane_fmt<T, EPL, LP>(a, k, pol.Zk, pl);
    pol.Gr = rec_plane<T, EPL>(a.rec, kn < k ? kn : k, a.ny);
    pol.vA = F.vA;
    pol.vG = F.vA + kRecG * kArr;
    plane_solve<kApplyDepth<T, EPL>>(a.ny, F, pol, lds);
}

// Lower level-3 sweep of one half: half 0 takes planes 0..j3-1 upward, half 1
// planes nz-1..j3+1 downward; z_k = Pt_k^{-1}(r_k - g * z_{k-+1}) into Z.
// With LP, pl is this lane's slots of the LDS plane buffer (RecFmtL).
template <typename T, int EPL, bool LP = false>
__device__ __forceinline__ void apply_lower(const ApplyArgs<T> &a, int h, T *lds, T *pl = nullptr) {
    const int nz = a.nz, j3 = (nz - 1) / 2;
    const int dk = h == 0 ? 1 : -1;
    const int k0 = h == 0 ? 0 : nz - 1;
    if (h == 0 ? k0 >= j3 : k0 <= j3) return;
    lower_plane<T, EPL, false, LP>(a, k0, k0, lds, pl);
    for (int k = k0 + dk; h == 0 ? k < j3 : k > j3; k += dk)
        lower_plane<T, EPL, true, LP>(a, k, k - dk, lds, pl);
}

// The twist plane j3 takes both neighbours; its result is final.
template <typename T, int EPL>
__device__ __forceinline__ void apply_twist(const ApplyArgs<T> &a, T *lds) {
    constexpr unsigned kArr = RecFmt<T, EPL>::kArr;
    const int nz = a.nz, k = (nz - 1) / 2;
    PolTwist<T, EPL> pol;
    pol.rp = plane_rsrc<T, EPL>(a.rp, k, a.ny);
    pol.Zk = plane_rsrc<T, EPL>(a.Z, k, a.ny);
    pol.lo_nb = k > 0;
    pol.hi_nb = k < nz - 1;
    pol.Zlo = plane_rsrc<T, EPL>(a.Z, pol.lo_nb ? k - 1 : k, a.ny);
    pol.Zhi = plane_rsrc<T, EPL>(a.Z, pol.hi_nb ? k + 1 : k, a.ny);
    const RecFmt<T, EPL> F = rec_fmt<T, EPL>(a, k, pol.Zk);
    pol.Glo = rec_plane<T, EPL>(a.rec, pol.lo_nb ? k - 1 : k, a.ny);
    pol.Ghi = F.rec;
    pol.vA = F.vA;
    pol.vG = F.vA + kRecG * kArr;
    plane_solve<kApplyDepth<T, EPL>>(a.ny, F, pol, lds);
}

template <typename T, int EPL, bool LPN, bool LP>
__device__ __forceinline__ void upper_plane(const ApplyArgs<T> &a, int k, int kn, rsrc_t W, T *lds,
                                            T *pl) {
    constexpr unsigned kArr = RecFmt<T, EPL>::kArr;
    PolUpper<T, EPL, LPN, LP> pol;
    pol.Zk = plane_rsrc<T, EPL>(a.Z, k, a.ny);
    pol.Zn = plane_rsrc<T, EPL>(a.Z, kn, a.ny);
    pol.pl = pl;
    const auto F = plane_fmt<T, EPL, LP>(a, k, W, pl);
    pol.Gr = rec_plane<T, EPL>(a.rec, kn < k ? kn : k, a.ny);
    pol.vA = F.vA;
    pol.vG = F.vA + kRecG * kArr;
    plane_solve<kApplyDepth<T, EPL>>(a.ny, F, pol, lds);
}

// Upper level-3 sweep: half 0 takes planes j3-1..0, half 1 planes j3+1..nz-1;
// x_k = z_k - Pt_k^{-1}(g * x_{k+-1}), written over Z.  With LP the first plane
// reads the twist plane from Z and the others their neighbour from the LDS
// plane buffer (pl, this lane's slots).
template <typename T, int EPL, bool LP = false>
__device__ __forceinline__ void apply_upper(const ApplyArgs<T> &a, int h, T *lds, T *pl = nullptr) {
    const int ny = a.ny, nz = a.nz, j3 = (nz - 1) / 2;
    const int dk = h == 0 ? -1 : 1;
    const rsrc_t W = make_rsrc(a.scratch + (size_t)h * ny * 64 * EPL);
    for (int k = j3 + dk; k >= 0 && k < nz; k += dk) {
        const int kn = k - dk;  // final neighbour, toward the twist plane
        if (LP && kn != j3) upper_plane<T, EPL, LP, LP>(a, k, kn, W, lds, pl);
        else upper_plane<T, EPL, false, LP>(a, k, kn, W, lds, pl);
    }
}

// One system: blockIdx.x is the level-3 half (lower and upper sweeps).
template <typename T, int EPL>
__global__ void __launch_bounds__(kApplyThreads) k_apply_lower(ApplyArgs<T> a) {
    __shared__ T lds[2 * 64 * EPL];
    apply_lower<T, EPL>(a, blockIdx.x, lds);
}
template <typename T, int EPL>
__global__ void __launch_bounds__(kApplyThreads) k_apply_twist(ApplyArgs<T> a) {
    __shared__ T lds[2 * 64 * EPL];
    apply_twist<T, EPL>(a, lds);
}
template <typename T, int EPL>
__global__ void __launch_bounds__(kApplyThreads) k_apply_upper(ApplyArgs<T> a) {
    __shared__ T lds[2 * 64 * EPL];
    apply_upper<T, EPL>(a, blockIdx.x, lds);
}

// A batch: a table of arguments in device memory, entry e = s*nrhs + q for
// right-hand side q of system s; entries whose active flag is 0 (when active
// is given) do nothing.  The entry is read once per block into scalar
// registers, so the sweeps see wave-uniform arguments as above.
__device__ __forceinline__ bool entry_active(const int *active, int e) {
    return !active || __builtin_amdgcn_readfirstlane(active[e]) != 0;
}

// Workgroups are dispatched round-robin over the XCDs (workgroup id mod 8), and
// each XCD has its own L2.  The sweeps of the right-hand sides of one system
// (and level-3 half) read the same line records at nearly the same time, so
// they are given workgroup ids that are equal mod 8: group g = s*halves + h
// goes to XCD g mod 8, its nrhs members to consecutive ids of that XCD.  The
// grid holds 8*nrhs*ceil(count*halves/8) workgroups; the padding ones exit.
constexpr int kXcds = 8;

struct BatchSlot {
    int e, h;
    bool ok;
};

__device__ __forceinline__ BatchSlot batch_slot(int count, int nrhs, int halves) {
    const int w = blockIdx.x;
    const int j = w / kXcds;
    const int q = j % nrhs;
    const int g = kXcds * (j / nrhs) + w % kXcds;
    BatchSlot b;
    b.ok = g < count * halves;
    b.e = (g / halves) * nrhs + q;
    b.h = g % halves;
    return b;
}

inline unsigned batch_grid(int count, int nrhs, int halves) {
    return (unsigned)(kXcds * nrhs * ((count * halves + kXcds - 1) / kXcds));
}

template <typename T, int EPL>
__global__ void __launch_bounds__(kApplyThreads) k_apply_lower_b(const ApplyArgs<T> *tab,
                                                                 const int *active, int count,
                                                                 int nrhs) {
    __shared__ T lds[2 * 64 * EPL];
    const BatchSlot b = batch_slot(count, nrhs, 2);
    if (!b.ok || !entry_active(active, b.e)) return;
    apply_lower<T, EPL>(load_uniform(tab + b.e), b.h, lds);
}
template <typename T, int EPL>
__global__ void __launch_bounds__(kApplyThreads) k_apply_twist_b(const ApplyArgs<T> *tab,
                                                                 const int *active, int count,
                                                                 int nrhs) {
    __shared__ T lds[2 * 64 * EPL];
    const BatchSlot b = batch_slot(count, nrhs, 1);
    if (!b.ok || !entry_active(active, b.e)) return;
    apply_twist<T, EPL>(load_uniform(tab + b.e), lds);
}
template <typename T, int EPL>
__global__ void __launch_bounds__(kApplyThreads) k_apply_upper_b(const ApplyArgs<T> *tab,
                                                                 const int *active, int count,
                                                                 int nrhs) {
    __shared__ T lds[2 * 64 * EPL];
    const BatchSlot b = batch_slot(count, nrhs, 2);
    if (!b.ok || !entry_active(active, b.e)) return;
    apply_upper<T, EPL>(load_uniform(tab + b.e), b.h, lds);
}

// The same with the plane buffer in LDS: plane_lds_bytes() of dynamic LDS, the
// twist exchange (2*64*EPL values) and then the plane (ny lines of 64*EPL).
extern __shared__ __attribute__((aligned(16))) unsigned char ntd_plane_lds[];

template <typename T, int EPL>
__global__ void __launch_bounds__(kApplyThreads) k_apply_lower_bl(const ApplyArgs<T> *tab,
                                                                  const int *active, int count,
                                                                  int nrhs) {
    T *lds = (T *)ntd_plane_lds;
    T *pl = lds + 2 * 64 * EPL + (threadIdx.x & 63) * EPL;
    const BatchSlot b = batch_slot(count, nrhs, 2);
    if (!b.ok || !entry_active(active, b.e)) return;
    apply_lower<T, EPL, true>(load_uniform(tab + b.e), b.h, lds, pl);
}
template <typename T, int EPL>
__global__ void __launch_bounds__(kApplyThreads) k_apply_upper_bl(const ApplyArgs<T> *tab,
                                                                  const int *active, int count,
                                                                  int nrhs) {
    T *lds = (T *)ntd_plane_lds;
    T *pl = lds + 2 * 64 * EPL + (threadIdx.x & 63) * EPL;
    const BatchSlot b = batch_slot(count, nrhs, 2);
    if (!b.ok || !entry_active(active, b.e)) return;
    apply_upper<T, EPL, true>(load_uniform(tab + b.e), b.h, lds, pl);
}

// ---------------------------------------------------------------------------
// Packing of the factors into the line records (one wavefront per line).
// ---------------------------------------------------------------------------

template <typename T, int EPL>
__global__ void __launch_bounds__(256) k_pack(PackArgs p) {
    using R = RecFmt<T, EPL>;
    const long long line = blockIdx.x * 4LL + (threadIdx.x >> 6);
    if (line >= (long long)p.ny * p.nz) return;  // whole wavefronts; no barrier below
    const int n = p.nx, ny = p.ny;
    const int k = (int)(line / ny), m = (int)(line - (long long)k * ny);
    const LineGeom G(n, EPL);
    const int lane = threadIdx.x & 63;
    const int j = G.ca - 1;
    const long long base = line * n;
    double v[kRecArrays][EPL];
    double seed = 0.0;
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        const int c = G.pos(s, EPL);
        if (!G.ok(c)) {  // unused slot
            v[kRecMv][s] = v[kRecP][s] = 0.0;
            v[kRecF][s] = v[kRecG][s] = 0.0;
            continue;
        }
        const int e = G.elem(c);
        const double M = p.mv[base + e];
        double cp, cn;
        if (G.half == 0) {
            cp = c > 0 ? p.e1[base + e - 1] : 0.0;
            cn = e == j ? 0.0 : p.e1[base + e];
        } else {
            cp = c > 0 ? p.e1[base + e] : 0.0;
            cn = p.e1[base + e - 1];
        }
        v[kRecMv][s] = M;
        v[kRecP][s] = cp;
        if (G.half == 1 && c == G.cb - 1) seed = -M * cn;  // element j+1: it seeds chain B
        v[kRecF][s] = m < ny - 1 ? p.f2[base + e] : 0.0;
        v[kRecG][s] = k < p.nz - 1 ? p.g3[base + e] : 0.0;
    }
    char *rec = (char *)p.rec + (size_t)line * R::kRec;
#pragma unroll
    for (int q = 0; q < kRecArrays; ++q) {
        T *arr = (T *)(rec + q * R::kArr);
#pragma unroll
        for (int s = 0; s < EPL; ++s) arr[lane * EPL + s] = (T)v[q][s];
    }
    // the chain-B seed (held by the lane of element j+1) goes with the twist row
    {
        const unsigned long long sb = __builtin_bit_cast(unsigned long long, seed);
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)sb, 63);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(sb >> 32), 63);
        seed = __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
    }
    if (lane == 0) {
        double *tw = (double *)(rec + R::kTw);
        tw[0] = p.mv[base + j];
        tw[1] = j > 0 ? p.e1[base + j - 1] : 0.0;
        tw[2] = j < n - 1 ? p.e1[base + j] : 0.0;
        tw[3] = seed;
    }
}

// ---------------------------------------------------------------------------
// Natural FP64 <-> packed moves (one thread per grid point).
// ---------------------------------------------------------------------------

// Packed slot of element i of a line (layout of LineGeom).
template <int EPL>
__device__ __forceinline__ int slot_of(int i, int n) {
    const int ca = (n + 1) / 2, cb = n - ca;
    if (i < ca) return i + 32 * EPL - ca;
    return 32 * EPL + (n - 1 - i) + 32 * EPL - cb;
}

// rp = r (or r - A zi), packed in the sweep precision, over the points
// blk*kBlock + t + i*nblk*kBlock.  Grids hold fewer than 2^28 points, so 32-bit
// indices suffice.
template <typename T, int EPL>
__device__ __forceinline__ void pack_rhs_body(const XferArgs<T> &x, unsigned blk, unsigned nblk) {
    const unsigned nx = (unsigned)x.nx, ny = (unsigned)x.ny, nz = (unsigned)x.nz;
    const unsigned nxy = nx * ny, N = nxy * nz;
    for (unsigned p = blk * kBlock + threadIdx.x; p < N; p += nblk * kBlock) {
        const unsigned line = p / nx;
        const unsigned i = p - line * nx;
        double v = x.r[p];
        if (x.zi) {
            const unsigned jj = line % ny, kk = line / ny;
            // each neighbour term one fused multiply-add onto the running sum
            const double *z = x.zi;
            double s = x.d[p] * z[p];
            if (i > 0) s = fma(x.ax[p - 1], z[p - 1], s);
            if (i + 1 < nx) s = fma(x.ax[p], z[p + 1], s);
            if (jj > 0) s = fma(x.ay[p - nx], z[p - nx], s);
            if (jj + 1 < ny) s = fma(x.ay[p], z[p + nx], s);
            if (kk > 0) s = fma(x.az[p - nxy], z[p - nxy], s);
            if (kk + 1 < nz) s = fma(x.az[p], z[p + nxy], s);
            v -= s;
        }
        x.rp[line * (64u * EPL) + slot_of<EPL>((int)i, (int)nx)] = (T)v;
    }
}

template <typename T, int EPL>
__global__ void __launch_bounds__(kBlock) k_pack_rhs(XferArgs<T> x) {
    pack_rhs_body<T, EPL>(x, blockIdx.x, gridDim.x);
}

// k_pack_rhs for two consecutive points of a line per thread, one pair per
// thread, with 16-byte loads of every pair (nx even, the FP64 arrays 16-byte
// aligned): the stencil r - A zi is bound by the load instructions it issues,
// and a pair needs 16 where two single points need 32.  Each point's value is
// formed in pack_rhs_body's order (bitwise the same packed right-hand side);
// the two slots are stored one by one, since the chain split can fall inside a
// pair (ceil(nx/2) odd).
template <typename T, int EPL>
__global__ void __launch_bounds__(kBlock) k_pack_rhs2(XferArgs<T> x) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const unsigned nx = (unsigned)x.nx, ny = (unsigned)x.ny, nz = (unsigned)x.nz;
    const unsigned nxy = nx * ny, P = nxy * nz / 2;
    const unsigned q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= P) return;
    const unsigned p = 2 * q;
    const unsigned line = p / nx;
    const unsigned i = p - line * nx;
    const d2 rv = *(const d2 *)(x.r + p);
    double v0 = rv.x, v1 = rv.y;
    if (x.zi) {
        const unsigned jj = line % ny, kk = line / ny;
        const double *z = x.zi;
        const d2 zv = *(const d2 *)(z + p), dv = *(const d2 *)(x.d + p);
        const d2 axv = *(const d2 *)(x.ax + p), ayv = *(const d2 *)(x.ay + p);
        const d2 azv = *(const d2 *)(x.az + p);
        double s0 = dv.x * zv.x, s1 = dv.y * zv.y;
        if (i > 0) s0 = fma(x.ax[p - 1], z[p - 1], s0);
        s0 = fma(axv.x, zv.y, s0);  // i + 1 < nx: the pair never ends a line
        s1 = fma(axv.x, zv.x, s1);
        if (i + 2 < nx) s1 = fma(axv.y, z[p + 2], s1);
        if (jj > 0) {
            const d2 a = *(const d2 *)(x.ay + p - nx), w = *(const d2 *)(z + p - nx);
            s0 = fma(a.x, w.x, s0);
            s1 = fma(a.y, w.y, s1);
        }
        if (jj + 1 < ny) {
            const d2 w = *(const d2 *)(z + p + nx);
            s0 = fma(ayv.x, w.x, s0);
            s1 = fma(ayv.y, w.y, s1);
        }
        if (kk > 0) {
            const d2 a = *(const d2 *)(x.az + p - nxy), w = *(const d2 *)(z + p - nxy);
            s0 = fma(a.x, w.x, s0);
            s1 = fma(a.y, w.y, s1);
        }
        if (kk + 1 < nz) {
            const d2 w = *(const d2 *)(z + p + nxy);
            s0 = fma(azv.x, w.x, s0);
            s1 = fma(azv.y, w.y, s1);
        }
        v0 -= s0;
        v1 -= s1;
    }
    T *row = x.rp + line * (64u * EPL);
    row[slot_of<EPL>((int)i, (int)nx)] = (T)v0;
    row[slot_of<EPL>((int)i + 1, (int)nx)] = (T)v1;
}

// Fixed-order block reduction of one double per thread; thread 0 gets the sum.
__device__ __forceinline__ double block_sum_apply(double v) {
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

// zout = Z (+ zi), natural FP64; the block's partial of r.zout into
// partials[blk].
template <typename T, int EPL>
__device__ __forceinline__ void unpack_body(const XferArgs<T> &x, unsigned blk, unsigned nblk) {
    const unsigned nx = (unsigned)x.nx;
    const unsigned N = nx * (unsigned)x.ny * (unsigned)x.nz;
    double acc = 0.0;
    for (unsigned p = blk * kBlock + threadIdx.x; p < N; p += nblk * kBlock) {
        const unsigned line = p / nx;
        const unsigned i = p - line * nx;
        double z = (double)x.Z[line * (64u * EPL) + slot_of<EPL>((int)i, (int)nx)];
        if (x.zi) z += x.zi[p];
        x.zout[p] = z;
        if (x.partials) acc += x.r[p] * z;
    }
    if (x.partials) {
        const double t = block_sum_apply(acc);
        if (threadIdx.x == 0) x.partials[blk] = t;
    }
}

template <typename T, int EPL>
__global__ void __launch_bounds__(kBlock) k_unpack(XferArgs<T> x) {
    unpack_body<T, EPL>(x, blockIdx.x, gridDim.x);
}

// Batched moves: blockIdx.y selects the table entry, gridDim.x blocks per entry.
template <typename T, int EPL>
__global__ void __launch_bounds__(kBlock) k_pack_rhs_b(const XferArgs<T> *tab, const int *active) {
    if (!entry_active(active, blockIdx.y)) return;
    pack_rhs_body<T, EPL>(load_uniform(tab + blockIdx.y), blockIdx.x, gridDim.x);
}
template <typename T, int EPL>
__global__ void __launch_bounds__(kBlock) k_unpack_b(const XferArgs<T> *tab, const int *active) {
    if (!entry_active(active, blockIdx.y)) return;
    unpack_body<T, EPL>(load_uniform(tab + blockIdx.y), blockIdx.x, gridDim.x);
}

inline int xfer_blocks(long long N) {
    long long b = (N + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > kMaxBlocks) b = kMaxBlocks;
    return (int)b;
}

// The apply as three stream-ordered launches; ev (optional, 4 events) brackets
// them for per-launch timing.
template <typename T, int EPL>
hipError_t apply_impl(const ApplyArgs<T> &a, hipStream_t s, hipEvent_t *ev) {
    if (ev) (void)hipEventRecord(ev[0], s);
    hipLaunchKernelGGL((k_apply_lower<T, EPL>), dim3(2), dim3(kApplyThreads), 0, s, a);
    if (ev) (void)hipEventRecord(ev[1], s);
    hipLaunchKernelGGL((k_apply_twist<T, EPL>), dim3(1), dim3(kApplyThreads), 0, s, a);
    if (ev) (void)hipEventRecord(ev[2], s);
    hipLaunchKernelGGL((k_apply_upper<T, EPL>), dim3(2), dim3(kApplyThreads), 0, s, a);
    if (ev) (void)hipEventRecord(ev[3], s);
    return hipGetLastError();
}

// The sweeps of a batch of count systems x nrhs right-hand sides, as three
// launches; plane_lds > 0: the lower and upper sweeps keep their planes in that
// many bytes of LDS (plane_lds_bytes of the largest ny, after
// apply_batch_lds_impl has allowed it).
template <typename T, int EPL>
hipError_t apply_batch_impl(const ApplyArgs<T> *tab, const int *active, int count, int nrhs,
                            size_t plane_lds, hipStream_t s, hipEvent_t *ev) {
    const dim3 g2(batch_grid(count, nrhs, 2)), g1(batch_grid(count, nrhs, 1));
    const dim3 blk(kApplyThreads);
    if (ev) (void)hipEventRecord(ev[0], s);
    if (plane_lds)
        hipLaunchKernelGGL((k_apply_lower_bl<T, EPL>), g2, blk, plane_lds, s, tab, active, count,
                           nrhs);
    else
        hipLaunchKernelGGL((k_apply_lower_b<T, EPL>), g2, blk, 0, s, tab, active, count, nrhs);
    if (ev) (void)hipEventRecord(ev[1], s);
    hipLaunchKernelGGL((k_apply_twist_b<T, EPL>), g1, blk, 0, s, tab, active, count, nrhs);
    if (ev) (void)hipEventRecord(ev[2], s);
    if (plane_lds)
        hipLaunchKernelGGL((k_apply_upper_bl<T, EPL>), g2, blk, plane_lds, s, tab, active, count,
                           nrhs);
    else
        hipLaunchKernelGGL((k_apply_upper_b<T, EPL>), g2, blk, 0, s, tab, active, count, nrhs);
    if (ev) (void)hipEventRecord(ev[3], s);
    return hipGetLastError();
}

// Allow the LDS-plane sweeps up to `bytes` of dynamic LDS (a limit of the
// kernels, shared by every batch: the callers pass the device's maximum).
template <typename T, int EPL>
hipError_t apply_batch_lds_impl(size_t bytes) {
    hipError_t e = hipFuncSetAttribute((const void *)&k_apply_lower_bl<T, EPL>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)&k_apply_upper_bl<T, EPL>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    return e;
}

template <typename T, int EPL>
hipError_t pack_rhs_batch_impl(const XferArgs<T> *tab, const int *active, int count, int gx,
                               hipStream_t s) {
    hipLaunchKernelGGL((k_pack_rhs_b<T, EPL>), dim3(gx, count), dim3(kBlock), 0, s, tab, active);
    return hipGetLastError();
}

template <typename T, int EPL>
hipError_t unpack_batch_impl(const XferArgs<T> *tab, const int *active, int count, int gx,
                             hipStream_t s) {
    hipLaunchKernelGGL((k_unpack_b<T, EPL>), dim3(gx, count), dim3(kBlock), 0, s, tab, active);
    return hipGetLastError();
}

template <typename T, int EPL>
hipError_t pack_impl(const PackArgs &p, hipStream_t s) {
    const long long nlines = (long long)p.ny * p.nz;
    hipLaunchKernelGGL((k_pack<T, EPL>), dim3((unsigned)((nlines + 3) / 4)), dim3(256), 0, s, p);
    return hipGetLastError();
}

template <typename T, int EPL>
hipError_t pack_rhs_impl(const XferArgs<T> &x, hipStream_t s) {
    const long long N = (long long)x.nx * x.ny * x.nz;
    uintptr_t al = (uintptr_t)x.r;
    if (x.zi)
        al |= (uintptr_t)x.zi | (uintptr_t)x.d | (uintptr_t)x.ax | (uintptr_t)x.ay |
              (uintptr_t)x.az;
    if (x.nx % 2 == 0 && N < (1LL << 31) && (al & 15) == 0) {
        const long long nb = (N / 2 + kBlock - 1) / kBlock;  // one pair per thread
        hipLaunchKernelGGL((k_pack_rhs2<T, EPL>), dim3((unsigned)(nb > 0 ? nb : 1)), dim3(kBlock),
                           0, s, x);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_pack_rhs<T, EPL>), dim3(xfer_blocks(N)), dim3(kBlock), 0, s, x);
    return hipGetLastError();
}

template <typename T, int EPL>
hipError_t unpack_impl(const XferArgs<T> &x, hipStream_t s, int *np) {
    const long long N = (long long)x.nx * x.ny * x.nz;
    const int nb = xfer_blocks(N);
    if (np) *np = x.partials ? nb : 0;
    hipLaunchKernelGGL((k_unpack<T, EPL>), dim3(nb), dim3(kBlock), 0, s, x);
    return hipGetLastError();
}

}  // namespace

}  // namespace ntd
