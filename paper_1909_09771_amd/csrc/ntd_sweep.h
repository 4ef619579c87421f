// ntd_sweep.h -- device templates shared by the nested twisted sweeps of the
// preconditioner (arXiv:1909.09771, Sec. 2.2, Algorithms 1-7) and its
// factorization (Sec. 2.1): line geometry, buffer I/O, cross-lane primitives,
// the level-2 plane solve, and the factorization kernels.  The apply's own
// layout and kernels are in ntd_apply.h.
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
//     lane-local composition plus a 32-lane scan of affine maps built from DPP
//     row shifts, a row broadcast and readlane.
// The level-3 twist plane and the switch from the lower to the upper level-3
// sweep are kernel boundaries (lower halves, twist plane, upper halves), so no
// workgroup ever waits for another.
//
// Memory access: a chain step is latency-bound, so every input of line m+1 is
// issued while line m is solved, through raw buffer loads with a uniform
// per-line byte offset and per-lane 32-bit element offsets.  Slots outside a
// chain use an offset past the end of every buffer: their loads return 0 and
// their stores are dropped, so no load or store needs a branch.
#pragma once

#include "ntd_internal.h"

namespace ntd {

namespace {

// Threads of a factorization workgroup: two chain wavefronts plus helpers for
// the plane-wide work.  Up to 4 values per lane, 512 (two waves per SIMD); with
// more, 256, so that a wave may use 512 registers (VGPRs and AGPRs) and spill
// into AGPRs rather than scratch.
template <int EPL>
constexpr int kSetupThreads = EPL <= 4 ? 512 : 256;

// ---------------------------------------------------------------------------
// Buffer I/O.
// ---------------------------------------------------------------------------

using rsrc_t = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned int))));

constexpr unsigned kOOB = 0x80000000u;  // beyond every buffer: load -> 0, store dropped

// Raw buffer over [p, p + 2 GiB); gfx9 resource word 3.
__device__ __forceinline__ rsrc_t make_rsrc(const void *p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, 0x7fffffff,
                                             0x00020000);
}

__device__ __forceinline__ float bload(float *, rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
}
__device__ __forceinline__ double bload(double *, rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(double,
                              __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0));
}
__device__ __forceinline__ void bstore(float v, rsrc_t r, unsigned vo, unsigned so) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ void bstore(double v, rsrc_t r, unsigned vo, unsigned so) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)vo, (int)so, 0);
}

// An argument struct read from device memory into scalar registers (one
// entry of a batched launch's table; the whole wavefront reads the same one).
template <typename S>
__device__ __forceinline__ S load_uniform(const S *p) {
    static_assert(sizeof(S) % 4 == 0, "word-sized descriptor");
    S out;
    const unsigned *src = (const unsigned *)p;
    unsigned *dst = (unsigned *)&out;
#pragma unroll
    for (unsigned i = 0; i < sizeof(S) / 4; ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return out;
}

// ---------------------------------------------------------------------------
// Level 1: one line per wavefront.
// ---------------------------------------------------------------------------

// Lane layout of one line: lanes 0-31 hold chain A (elements 0..j, j = ca-1 the
// twist element), lanes 32-63 chain B (elements n-1 down to j+1), EPL
// consecutive chain positions per lane.  Both chains are right-aligned in their
// half so that the twist element always sits in lane 31, slot EPL-1, and the
// end of chain B (element j+1) in lane 63, slot EPL-1; the unused positions are
// at the start of each half.
struct LineGeom {
    int n;     // line length (nx)
    int ca;    // chain A length: elements 0..j (j = ca - 1 is the twist element)
    int cb;    // chain B length: elements n-1 down to j+1
    int half;  // 0: this lane holds chain A, 1: chain B
    int hl;    // lane index inside the half, 0..31
    int cnt;   // length of this lane's chain
    int skip;  // unused positions at the start of this half
    __device__ LineGeom(int n_, int epl) : n(n_) {
        ca = (n_ + 1) / 2;
        cb = n_ - ca;
        int lane = threadIdx.x & 63;
        half = lane >> 5;
        hl = lane & 31;
        cnt = half ? cb : ca;
        skip = 32 * epl - cnt;
    }
    // chain position of slot s (negative: unused slot)
    __device__ __forceinline__ int pos(int s, int epl) const { return hl * epl + s - skip; }
    __device__ __forceinline__ bool ok(int c) const { return c >= 0; }
    __device__ __forceinline__ int elem(int c) const { return half ? n - 1 - c : c; }
};

// Per-lane byte offsets, inside a line, of the element of each slot (o4 for
// 4-byte, o8 for 8-byte arrays) and of its left neighbour e-1 (p4, p8); kOOB
// where the slot is outside the chain or the neighbour does not exist.
template <int EPL>
struct Slots {
    unsigned o4[EPL], o8[EPL], p4[EPL], p8[EPL];
    __device__ explicit Slots(const LineGeom &G) {
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
            const int c = G.pos(s, EPL);
            const bool ok = G.ok(c);
            const int e = G.elem(c);
            o4[s] = ok ? 4u * e : kOOB;
            o8[s] = ok ? 8u * e : kOOB;
            p4[s] = (ok && e > 0) ? 4u * (e - 1) : kOOB;
            p8[s] = (ok && e > 0) ? 8u * (e - 1) : kOOB;
        }
    }
    __device__ __forceinline__ bool valid(int s) const { return o4[s] != kOOB; }
    __device__ __forceinline__ unsigned off(float *, int s) const { return o4[s]; }
    __device__ __forceinline__ unsigned off(double *, int s) const { return o8[s]; }
    __device__ __forceinline__ unsigned offm1(float *, int s) const { return p4[s]; }
    __device__ __forceinline__ unsigned offm1(double *, int s) const { return p8[s]; }
};

template <typename T, int EPL>
__device__ __forceinline__ void bload_line(const Slots<EPL> &S, rsrc_t r, unsigned so,
                                           T (&v)[EPL]) {
#pragma unroll
    for (int s = 0; s < EPL; ++s) v[s] = bload((T *)nullptr, r, S.off((T *)nullptr, s), so);
}

template <typename T, int EPL>
__device__ __forceinline__ void bstore_line(const Slots<EPL> &S, rsrc_t r, unsigned so,
                                            const T (&v)[EPL]) {
#pragma unroll
    for (int s = 0; s < EPL; ++s) bstore(v[s], r, S.off((T *)nullptr, s), so);
}

template <typename T, int EPL>
__device__ __forceinline__ void zero_line(T (&v)[EPL]) {
#pragma unroll
    for (int s = 0; s < EPL; ++s) v[s] = T(0);
}

// Pointer-based line access (setup only).
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

// ---------------------------------------------------------------------------
// Cross-lane primitives: DPP moves inside the 16-lane rows, row broadcast and
// readlane across rows.  `old` is what a lane keeps when its source lane does
// not exist (the identity of the operation being scanned).
// ---------------------------------------------------------------------------

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp(float old, float src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                 __builtin_bit_cast(int, src), CTRL,
                                                                 ROW_MASK, 0xF, false));
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp(double old, double src) {
    const unsigned long long o = __builtin_bit_cast(unsigned long long, old);
    const unsigned long long s = __builtin_bit_cast(unsigned long long, src);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)s,
                                                              CTRL, ROW_MASK, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32),
                                                              (int)(unsigned)(s >> 32), CTRL,
                                                              ROW_MASK, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ float rdlane(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

__device__ __forceinline__ double rdlane(double v, int lane) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// DPP controls (GFX9 encoding).
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowShl1 = 0x101, kRowShl2 = 0x102, kRowShl4 = 0x104, kRowShl8 = 0x108;
constexpr int kWaveShl1 = 0x130, kWaveShr1 = 0x138, kRowBcast15 = 0x142;

// Inclusive scan of affine maps x -> A x + B over the 32 lanes of each half,
// forward (lane hl composes lanes 0..hl).  Four in-row steps, then row 1
// (row 3) takes the composite of row 0 (row 2) through lane 15 (47).
template <typename T>
__device__ __forceinline__ void scan_fwd32(T &A, T &B) {
#define NTD_FWD_STEP(CTRL, RM)                                            \
    {                                                                     \
        const T Ap = dpp<CTRL, RM>(T(1), A), Bp = dpp<CTRL, RM>(T(0), B); \
        B = A * Bp + B;                                                   \
        A = A * Ap;                                                       \
    }
    NTD_FWD_STEP(kRowShr1, 0xF)
    NTD_FWD_STEP(kRowShr2, 0xF)
    NTD_FWD_STEP(kRowShr4, 0xF)
    NTD_FWD_STEP(kRowShr8, 0xF)
    {
        const T Bp = dpp<kRowBcast15, 0xA>(T(0), B);
        B = A * Bp + B;
    }
#undef NTD_FWD_STEP
}

// Same, backward (lane hl composes lanes hl..31): four in-row steps, then rows
// 0 and 2 take the composite of rows 1 and 3 read from lanes 16 and 48.
template <typename T>
__device__ __forceinline__ void scan_bwd32(T &U, T &G, int lane) {
#define NTD_BWD_STEP(CTRL)                                        \
    {                                                             \
        const T Un = dpp<CTRL>(T(1), U), Gn = dpp<CTRL>(T(0), G); \
        G = U * Gn + G;                                           \
        U = U * Un;                                               \
    }
    NTD_BWD_STEP(kRowShl1)
    NTD_BWD_STEP(kRowShl2)
    NTD_BWD_STEP(kRowShl4)
    NTD_BWD_STEP(kRowShl8)
#undef NTD_BWD_STEP
    const T g16 = rdlane(G, 16), g48 = rdlane(G, 48);
    const T gn = lane < 32 ? g16 : g48;
    if (((lane >> 4) & 1) == 0) G = U * gn + G;
}

// Vector access to one lane's EPL consecutive values of a packed line, in the
// widest chunks (16, 8 or 4 bytes) that divide EPL*sizeof(T); lane bases are
// multiples of EPL*sizeof(T) and line bases of 64*EPL*sizeof(T), so every chunk
// is aligned to its size.
// (Elements of the returned vectors are first copied into plain unsigned
// scalars: a bit cast applied directly to a vector element is mis-compiled by
// this toolchain, which then loads only the first dword.)
template <typename T, int EPL>
__device__ __forceinline__ void vload(rsrc_t r, unsigned vo, unsigned so, T (&v)[EPL]) {
    typedef unsigned int u32x4 __attribute__((__vector_size__(4 * sizeof(unsigned int))));
    constexpr int PB = EPL * (int)sizeof(T);
    constexpr int CH = (PB % 16 == 0) ? 16 : (PB % 8 == 0) ? 8 : 4;
    static_assert(CH >= (int)sizeof(T), "chunk");
#pragma unroll
    for (int c = 0; c < PB / CH; ++c) {
        const int vo_c = (int)(vo + c * CH);
        if constexpr (CH == 16) {
            const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, vo_c, (int)so, 0);
            const unsigned w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3];
            if constexpr (sizeof(T) == 4) {
                v[c * 4 + 0] = __builtin_bit_cast(T, w0);
                v[c * 4 + 1] = __builtin_bit_cast(T, w1);
                v[c * 4 + 2] = __builtin_bit_cast(T, w2);
                v[c * 4 + 3] = __builtin_bit_cast(T, w3);
            } else {
                v[c * 2 + 0] = __builtin_bit_cast(T, ((unsigned long long)w1 << 32) | w0);
                v[c * 2 + 1] = __builtin_bit_cast(T, ((unsigned long long)w3 << 32) | w2);
            }
        } else if constexpr (CH == 8) {
            const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, vo_c, (int)so, 0);
            const unsigned w0 = w[0], w1 = w[1];
            if constexpr (sizeof(T) == 4) {
                v[c * 2 + 0] = __builtin_bit_cast(T, w0);
                v[c * 2 + 1] = __builtin_bit_cast(T, w1);
            } else {
                v[c] = __builtin_bit_cast(T, ((unsigned long long)w1 << 32) | w0);
            }
        } else {
            const unsigned w0 = __builtin_amdgcn_raw_buffer_load_b32(r, vo_c, (int)so, 0);
            v[c] = __builtin_bit_cast(T, w0);
        }
    }
}

template <typename T, int EPL>
__device__ __forceinline__ void vstore(rsrc_t r, unsigned vo, unsigned so, const T (&v)[EPL]) {
    typedef unsigned int u32x4 __attribute__((__vector_size__(4 * sizeof(unsigned int))));
    constexpr int PB = EPL * (int)sizeof(T);
    constexpr int CH = (PB % 16 == 0) ? 16 : (PB % 8 == 0) ? 8 : 4;
#pragma unroll
    for (int c = 0; c < PB / CH; ++c) {
        const int vo_c = (int)(vo + c * CH);
        if constexpr (CH == 16) {
            u32x4 w;
            if constexpr (sizeof(T) == 4) {
                w[0] = __builtin_bit_cast(unsigned, v[c * 4 + 0]);
                w[1] = __builtin_bit_cast(unsigned, v[c * 4 + 1]);
                w[2] = __builtin_bit_cast(unsigned, v[c * 4 + 2]);
                w[3] = __builtin_bit_cast(unsigned, v[c * 4 + 3]);
            } else {
                const unsigned long long x0 = __builtin_bit_cast(unsigned long long, v[c * 2 + 0]);
                const unsigned long long x1 = __builtin_bit_cast(unsigned long long, v[c * 2 + 1]);
                w[0] = (unsigned)x0; w[1] = (unsigned)(x0 >> 32);
                w[2] = (unsigned)x1; w[3] = (unsigned)(x1 >> 32);
            }
            __builtin_amdgcn_raw_buffer_store_b128(w, r, vo_c, (int)so, 0);
        } else if constexpr (CH == 8) {
            u32x2 w;
            if constexpr (sizeof(T) == 4) {
                w[0] = __builtin_bit_cast(unsigned, v[c * 2 + 0]);
                w[1] = __builtin_bit_cast(unsigned, v[c * 2 + 1]);
            } else {
                const unsigned long long x0 = __builtin_bit_cast(unsigned long long, v[c]);
                w[0] = (unsigned)x0; w[1] = (unsigned)(x0 >> 32);
            }
            __builtin_amdgcn_raw_buffer_store_b64(w, r, vo_c, (int)so, 0);
        } else {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v[c]), r, vo_c,
                                                  (int)so, 0);
        }
    }
}

// The twisted solve of one line held by the calling wavefront, given per slot
// the lower-sweep coefficient a (-cp/M; 1 on unused slots), 1/M (0 on unused
// slots) and the upper-sweep coefficient u (-cn/M; 0 on unused slots and on
// the twist slot), and, for the twist row, 1/M, cp and cn in FP64.
// Lower sweep: g_c = a_c g_{c-1} + y_c/M_c along each chain toward the twist;
// the twist row takes both neighbours, in FP64.  Upper sweep: x_c = u_c x_{c+1}
// + g_c from the twist outward, the top of chain B (lane 63, last slot) being
// seeded with the twist value.
template <typename T, int EPL>
__device__ __forceinline__ void solve_core(const T (&a)[EPL], const T (&mv)[EPL],
                                           const T (&uin)[EPL], double mvj, double cpj,
                                           double cnj, const T (&y)[EPL], T (&x)[EPL]) {
    const int lane = threadIdx.x & 63;
    const int hl = lane & 31;
    T g[EPL], gm1[EPL], u[EPL];
    T A = T(1), B = T(0);
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        g[s] = mv[s] * y[s];
        B = a[s] * B + g[s];
        A = a[s] * A;
    }
    scan_fwd32(A, B);
    T carry = dpp<kWaveShr1>(T(0), B);
    if (hl == 0) carry = T(0);
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        gm1[s] = carry;
        g[s] = a[s] * carry + g[s];
        carry = g[s];
    }
    // Twist element j: lane 31, slot EPL-1; its neighbour j+1 ends chain B in
    // lane 63, slot EPL-1 (0 there when chain B is empty).
    constexpr int L = EPL - 1;
    const T gB = rdlane(g[L], 63);
    double gj = mvj * ((double)y[L] - cpj * (double)gm1[L] - cnj * (double)gB);
    gj = rdlane(gj, 31);
    const T xj = (T)gj;
#pragma unroll
    for (int s = 0; s < EPL; ++s) u[s] = uin[s];
    if (lane == 31) {
        g[L] = xj;
        u[L] = T(0);
    }
    if (lane == 63) {  // seed chain B with x_j
        g[L] = g[L] + u[L] * xj;
        u[L] = T(0);
    }
    T U = T(1), Gs = T(0);
#pragma unroll
    for (int s = EPL - 1; s >= 0; --s) {
        Gs = u[s] * Gs + g[s];
        U = u[s] * U;
    }
    scan_bwd32(U, Gs, lane);
    T xn = dpp<kWaveShl1>(T(0), Gs);
    if (hl == 31) xn = T(0);
#pragma unroll
    for (int s = EPL - 1; s >= 0; --s) {
        x[s] = u[s] * xn + g[s];
        xn = x[s];
    }
}

// Everything one line step reads from memory, loaded ahead of use: the line's
// solve coefficients (format dependent), the y-coupling f to the neighbour
// line, the lower-sweep result w (upper sweeps), and raw inputs a*, d0 of the
// caller's right-hand side and output (combined only when used, so that the
// loads stay in flight).
template <typename T, int EPL>
struct LineIn {
    T c0[EPL], c1[EPL], c2[EPL];  // natural: 1/M, e1[e], e1[e-1]; packed: 1/M, a, u
    T f[EPL], w[EPL];
    T a0[EPL], a1[EPL], a2[EPL], a3[EPL];
    double d0[EPL], d1[EPL], d2[EPL];
    double mvj, cpj, cnj, seed;  // packed: the twist row and the chain-B seed
};

// Natural layout (the factorization's own arrays, FP64): lines of nx elements,
// couplings taken from the x-band e1 around each slot's element.
template <typename T, int EPL>
struct NatFmt {
    using Ty = T;
    static constexpr int kEPL = EPL;
    LineGeom G;
    Slots<EPL> S;
    rsrc_t e1, mv, f2, W;
    const double *mv64;  // FP64 1/M of the plane
    unsigned soT, soW, lineB;
    int ny;
    __device__ NatFmt(int nx) : G(nx, EPL), S(G), ny(1) {}
    __device__ void load_coef(int m, LineIn<T, EPL> &in) const {
        const unsigned so = soT + (unsigned)m * lineB;
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
            in.c0[s] = bload((T *)nullptr, mv, S.off((T *)nullptr, s), so);
            in.c1[s] = bload((T *)nullptr, e1, S.off((T *)nullptr, s), so);
            in.c2[s] = bload((T *)nullptr, e1, S.offm1((T *)nullptr, s), so);
        }
        in.mvj = mv64[(long long)m * G.n + G.ca - 1];
    }
    // y-coupling of line m to line m+1 (up) or m-1 (down); 0 past the plane edge
    __device__ void load_fc(int m, bool up, T (&f)[EPL]) const {
        const int lc = up ? m : m - 1;
        if (lc < 0 || lc >= ny - 1) zero_line(f);
        else bload_line(S, f2, soT + (unsigned)lc * lineB, f);
    }
    __device__ void load_w(int m, T (&w)[EPL]) const {
        bload_line(S, W, soW + (unsigned)m * lineB, w);
    }
    __device__ void store_w(int m, const T (&w)[EPL]) const {
        bstore_line(S, W, soW + (unsigned)m * lineB, w);
    }
    __device__ void solve(const LineIn<T, EPL> &in, const T (&y)[EPL], T (&x)[EPL]) const {
        T a[EPL], u[EPL];
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
            const T cp = G.half ? in.c1[s] : in.c2[s];
            const T cn = G.half ? in.c2[s] : in.c1[s];
            a[s] = S.valid(s) ? -in.c0[s] * cp : T(1);
            u[s] = -in.c0[s] * cn;
        }
        constexpr int L = EPL - 1;
        const double cpj = (double)(G.half ? in.c1[L] : in.c2[L]);
        const double cnj = (double)(G.half ? in.c2[L] : in.c1[L]);
        solve_core(a, in.c0, u, in.mvj, cpj, cnj, y, x);
    }
};

// ---------------------------------------------------------------------------
// Level 2: one plane per workgroup, two wavefronts (the two half chains).
// ---------------------------------------------------------------------------

// Solve Pt x = y for one plane:
//   lower: w_m = T_m^{-1}(y_m - f*w_{m-1}) for m < j2 (wave 0), mirrored for
//          m > j2 (wave 1), the twist line j2 taking both neighbours;
//   upper: x_{j2} = w_{j2}; x_m = w_m - T_m^{-1}(f*x_{m+-1}) outward.
// `fmt` addresses the plane's factors and the lower-result buffer W; the
// policy `pol` supplies the right-hand side and takes the results:
//   pol.load_rhs(m, fmt, in)  issue the loads of line m's right-hand side
//   pol.rhs(in, s)            the right-hand side value of slot s
//   pol.load_out(m, fmt, in)  issue the loads the output of line m needs
//   pol.out(m, fmt, x, in)    receive the final x of line m (exactly once)
// The inputs of the next DEPTH lines are in flight while a line is solved.
// All threads of the block must call it (it holds two block barriers).
template <int DEPTH, class Fmt, class Pol>
__device__ void plane_solve(int ny, const Fmt &fmt, Pol &pol, typename Fmt::Ty *lds) {
    using T = typename Fmt::Ty;
    constexpr int EPL = Fmt::kEPL;
    static_assert(DEPTH == 1 || DEPTH == 2, "prefetch depth");
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int j2 = (ny - 1) / 2;
    T y[EPL], w[EPL], prev[EPL], fhi[EPL];
    LineIn<T, EPL> A, B;
    [[maybe_unused]] LineIn<T, EPL> C;
    zero_line(prev);

    // inputs of the lower step of line m, coupled to its chain predecessor
    // m+1 (up) or m-1 (down)
    auto load_lower = [&](int m, bool up, LineIn<T, EPL> &in) {
        pol.load_rhs(m, fmt, in);
        fmt.load_fc(m, up, in.f);
        fmt.load_coef(m, in);
    };
    // inputs of the upper step of line m, coupled to its final neighbour toward
    // the twist, m+1 (up) or m-1 (down)
    auto load_upper = [&](int m, bool up, LineIn<T, EPL> &in) {
        fmt.load_w(m, in.w);
        fmt.load_fc(m, up, in.f);
        fmt.load_coef(m, in);
        pol.load_out(m, fmt, in);
    };
    // Each step starts with a scheduling barrier: work of the next step moved
    // into this one would wait for loads issued only one step earlier.
    auto lower_step = [&](int m, const LineIn<T, EPL> &in) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < EPL; ++s) y[s] = pol.rhs(in, s) - in.f[s] * prev[s];
        fmt.solve(in, y, w);
        fmt.store_w(m, w);
#pragma unroll
        for (int s = 0; s < EPL; ++s) prev[s] = w[s];
    };
    auto upper_step = [&](int m, const LineIn<T, EPL> &in) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < EPL; ++s) y[s] = in.f[s] * prev[s];
        fmt.solve(in, y, w);
#pragma unroll
        for (int s = 0; s < EPL; ++s) w[s] = in.w[s] - w[s];
        pol.out(m, fmt, w, in);
#pragma unroll
        for (int s = 0; s < EPL; ++s) prev[s] = w[s];
    };
    // Steps i = 0..count-1 of a chain.  DEPTH 2: three rotating input buffers,
    // the inputs of steps i+1 and i+2 are in flight while step i runs; DEPTH 1:
    // two buffers, one step ahead.  With `tail`, the inputs of step `count` are
    // issued too and left in A; with `pre`, those of step 0 are already in A.
    // Inside the loop every load is issued, past the end of the chain on its
    // last line again: a conditional load would make the wait counts at the
    // loop's merge points assume it was skipped and wait for the newest loads.
    auto chain = [&](int count, bool tail, bool pre, auto &&load, auto &&step) {
        const int nl = count + (tail ? 1 : 0);
        if (nl <= 0) return;
        const int last = nl - 1;
        auto cl = [last](int q) { return q < last ? q : last; };
        // The batches of the first steps are issued in step order: interleaved
        // by the scheduler, the wait counts at the loop header (merged with the
        // back edge) would assume the older batch was issued last.
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
            const int rest = count - i;  // 0, 1 or 2 steps left, in A then B
            if (rest >= 1) {
                if (i + 2 < nl) load(i + 2, C);
                step(i, A);
            }
            if (rest == 2) step(i + 1, B);
            if (tail) {  // the inputs of step `count` are in A, B or C
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
        // lines 0..j2-1 upward, then the inputs of the twist line j2 in A
        chain(j2, true, false,
              [&](int i, LineIn<T, EPL> &in) { load_lower(i, false, in); },
              [&](int i, const LineIn<T, EPL> &in) { lower_step(i, in); });
        pol.load_out(j2, fmt, A);
        fmt.load_fc(j2, true, fhi);
    } else if (wv == 1) {
        // lines ny-1..j2+1 downward (line m couples to m+1 through f2 line m)
        chain(ny - 1 - j2, false, false,
              [&](int i, LineIn<T, EPL> &in) { load_lower(ny - 1 - i, true, in); },
              [&](int i, const LineIn<T, EPL> &in) { lower_step(ny - 1 - i, in); });
#pragma unroll
        for (int s = 0; s < EPL; ++s) lds[64 * EPL + lane * EPL + s] = prev[s];
        if (j2 + 1 < ny) load_upper(j2 + 1, false, A);
    }
    __syncthreads();
    if (wv == 0) {  // twist line: both neighbours
#pragma unroll
        for (int s = 0; s < EPL; ++s)
            y[s] = pol.rhs(A, s) - A.f[s] * prev[s] - fhi[s] * lds[64 * EPL + lane * EPL + s];
        fmt.solve(A, y, w);
        pol.out(j2, fmt, w, A);
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
            prev[s] = w[s];
            lds[lane * EPL + s] = w[s];
        }
        if (j2 > 0) load_upper(j2 - 1, true, A);
    }
    __syncthreads();
    if (wv == 1) {
#pragma unroll
        for (int s = 0; s < EPL; ++s) prev[s] = lds[lane * EPL + s];
        // lines j2+1..ny-1 upward (line m couples to m-1 through f2 line m-1)
        chain(ny - 1 - j2, false, true,
              [&](int i, LineIn<T, EPL> &in) { load_upper(j2 + 1 + i, false, in); },
              [&](int i, const LineIn<T, EPL> &in) { upper_step(j2 + 1 + i, in); });
    } else if (wv == 0) {
        // lines j2-1..0 downward (line m couples to m+1 through f2 line m)
        chain(j2, false, true,
              [&](int i, LineIn<T, EPL> &in) { load_upper(j2 - 1 - i, true, in); },
              [&](int i, const LineIn<T, EPL> &in) { upper_step(j2 - 1 - i, in); });
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

// Plain plane solve x = Pt^{-1} y with y and x plane-sized buffers (natural layout).
template <int EPL>
struct PolPlain {
    rsrc_t y, x;
    unsigned line8;
    __device__ void load_rhs(int m, const NatFmt<double, EPL> &F,
                             LineIn<double, EPL> &in) const {
        bload_line(F.S, y, m * line8, in.a0);
    }
    __device__ double rhs(const LineIn<double, EPL> &in, int s) const { return in.a0[s]; }
    __device__ void load_out(int, const NatFmt<double, EPL> &, LineIn<double, EPL> &) const {}
    __device__ void out(int m, const NatFmt<double, EPL> &F, const double (&v)[EPL],
                        const LineIn<double, EPL> &) {
        bstore_line(F.S, x, m * line8, v);
    }
};

// Line m of plane k (one wavefront): T_m starts as the line block of P_k and
// loses, for each neighbour line nb, phi Y phi with g = (T_nb^{-1} v)./v,
// v = phi .* t_m, phi = the y-coupling of the two lines and Y = 2g - g T_nb g
// (Newton) or Y = g (diagonal); then the twisted pivots of T_m.
// The LDS of a wave (5 * nx doubles: dT, e, M then 1/M, and two work lines)
// keeps the factors of the last line it set up; a neighbour's factors are read
// from there (nbsh0, nbsh1: the LDS of the wave that set up nb0, nb1), not
// from the global arrays it has just written.
template <int EPL>
__device__ void line_setup(const SetupArgs &a, long long pk, int m, int nnb, int nb0, int nb1,
                           double *sh /* this wave's LDS */, const double *nbsh0,
                           const double *nbsh1) {
    const int nx = a.nx;
    const LineGeom G(nx, EPL);
    const int lane = threadIdx.x & 63;
    double *sd = sh, *se = sh + nx, *sM = sh + 2 * nx, *sg = sh + 3 * nx, *sp = sh + 4 * nx;
    const long long lm = pk + (long long)m * nx;
    double dT[EPL], ev[EPL];
    load_line(G, a.dP + lm, dT);
    load_line(G, a.xP + lm, ev);
    for (int q = 0; q < nnb; ++q) {
        const int nb = q == 0 ? nb0 : nb1;
        const double *nbs = q == 0 ? nbsh0 : nbsh1;
        const double *nd = nbs, *ne = nbs + nx, *nmv = nbs + 2 * nx;
        const long long lc = pk + (long long)(m < nb ? m : nb) * nx;
        double phi[EPL], v[EPL], zl[EPL], gam[EPL], dTn[EPL], en[EPL];
        load_line(G, a.f2 + lc, phi);
        LineIn<double, EPL> C;
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
            const int c = G.pos(s, EPL);
            const bool ok = G.ok(c);
            const int e = G.elem(c);
            v[s] = ok ? phi[s] * tval(a.t, lm + e) : 0.0;
            C.c0[s] = ok ? nmv[e] : 0.0;                 // 1/M of the neighbour
            C.c1[s] = ok ? ne[e] : 0.0;                  // its coupling e -- e+1
            C.c2[s] = (ok && e > 0) ? ne[e - 1] : 0.0;   // and e-1 -- e
            dTn[s] = ok ? nd[e] : 0.0;
            en[s] = C.c1[s];
        }
        C.mvj = nmv[G.ca - 1];
        const NatFmt<double, EPL> F(nx);
        F.solve(C, v, zl);
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
    // Twisted pivots M_c = d_c - e_c^2 / M_{c-1} along chain A (elements 0..j-1)
    // and chain B (n-1 down to j+1), e_c the coupling of c to its predecessor;
    // then the twist row j with both neighbours.  With the continuants p_c =
    // d_c p_{c-1} - e_c^2 p_{c-2} (p_{-1} = 1, p_0 = d_0), M_c = p_c / p_{c-1}.
    // Scaled as q_c = p_c / (d_0 ... d_c) they obey
    //     q_c = q_{c-1} - alpha_c q_{c-2},  alpha_c = e_c^2 / (d_c d_{c-1}),
    // so the walk along a chain is one FMA per element (the alphas and the
    // ratios M_c = d_c q_c / q_{c-1} are formed by all lanes in parallel), and a
    // rounding error propagates exactly as in the recurrence for M_c itself.
    // An exact power-of-2 rescale every 16 elements keeps q from underflowing.
    store_line(G, sd, dT);
    store_line(G, se, ev);
    wave_sync();
    const int j = G.ca - 1;
    const int len = G.half ? G.cb : j;  // this lane's chain, without the twist element
    double *sA = sg, *sP = sp, *sQ = sM;  // alpha_c; q_c and q_{c-1} in one scale
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        const int c = G.pos(s, EPL);
        if (G.ok(c) && c >= 1 && c < len) {
            const int e = G.elem(c);
            const int ep = G.half ? e + 1 : e - 1;
            const double ec = G.half ? ev[s] : se[e - 1];
            sA[e] = ec * ec / (dT[s] * sd[ep]);
        }
    }
    wave_sync();
    if (G.hl == 0 && len > 0) {  // lanes 0 and 32: the two chains side by side
        const int di = G.half ? -1 : 1;
        int e = G.half ? nx - 1 : 0;
        double q2 = 1.0, q1 = 1.0;  // q_{c-2}, q_{c-1}
        sP[e] = 1.0;
        sQ[e] = 1.0;
        // 16 elements at a time: their alphas are read first and their q stored
        // after the walk, so that no LDS access waits inside the FMA chain
        // (the lines share one LDS block, and the compiler cannot move a read
        // of one above a write of another).
        int c = 1;
        for (; c + 16 <= len; c += 16) {
            double al[16], qv[16], qp[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) al[u] = sA[e + (u + 1) * di];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                qv[u] = __builtin_fma(-al[u], q2, q1);
                qp[u] = q1;
                q2 = q1;
                q1 = qv[u];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                sP[e + (u + 1) * di] = qv[u];
                sQ[e + (u + 1) * di] = qp[u];
            }
            e += 16 * di;
            const int x = -__builtin_amdgcn_frexp_exp(q1);
            q1 = __builtin_amdgcn_ldexp(q1, x);
            q2 = __builtin_amdgcn_ldexp(q2, x);
        }
        for (; c < len; ++c) {
            e += di;
            const double q = __builtin_fma(-sA[e], q2, q1);
            sP[e] = q;
            sQ[e] = q1;
            q2 = q1;
            q1 = q;
        }
    }
    wave_sync();
    // 1/M_c = q_{c-1} / (d_c q_c) for the chain elements, into sM (over q_{c-1})
    double mv[EPL];
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        const int c = G.pos(s, EPL);
        mv[s] = 0.0;
        if (G.ok(c) && c < len) {
            const int e = G.elem(c);
            mv[s] = sQ[e] / (dT[s] * sP[e]);
            sM[e] = mv[s];
        }
    }
    wave_sync();
    if (lane == 0) {
        double Mj = sd[j];
        if (j > 0) Mj -= se[j - 1] * se[j - 1] * sM[j - 1];
        if (j < nx - 1) Mj -= se[j] * se[j] * sM[j + 1];
        sM[j] = 1.0 / Mj;
    }
    wave_sync();
    bool bad = false;
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        const int c = G.pos(s, EPL);
        if (G.ok(c)) {
            if (c == len) mv[s] = sM[G.elem(c)];  // the twist element (chain A)
            if (!(mv[s] > 0.0) || !isfinite(mv[s])) bad = true;
        }
    }
    wave_sync();
    store_line(G, a.mv + lm, mv);
    store_line(G, a.dT + lm, dT);
    store_line(G, a.e1 + lm, ev);  // LDS holds this line's dT, e and 1/M
    wave_sync();
    if (bad) atomicOr(a.flag, kFlagNotSPD);
}

// Level-2 factorization of plane k (the line recurrence of its P_k block).
template <int EPL>
__device__ void plane_lines_setup(const SetupArgs &a, int k, double *sh) {
    const int ny = a.ny;
    const long long pk = (long long)k * a.nx * ny;
    const int wv = threadIdx.x >> 6;
    const int j2 = (ny - 1) / 2;
    double *lds0 = sh, *lds1 = sh + 5 * a.nx;  // the LDS of waves 0 and 1
    double *mine = (wv & 1) ? lds1 : lds0;
    if (wv == 0) {
        for (int m = 0; m < j2; ++m)
            line_setup<EPL>(a, pk, m, m > 0 ? 1 : 0, m - 1, 0, mine, mine, mine);
    } else if (wv == 1) {
        for (int m = ny - 1; m > j2; --m)
            line_setup<EPL>(a, pk, m, m < ny - 1 ? 1 : 0, m + 1, 0, mine, mine, mine);
    }
    __syncthreads();
    if (wv == 0) {  // the twist line: line j2-1 in wave 0's LDS, j2+1 in wave 1's
        int nnb = 0, n0 = 0, n1 = 0;
        const double *s0 = lds0, *s1 = lds1;
        if (j2 > 0) { n0 = j2 - 1; ++nnb; }
        if (j2 < ny - 1) {
            if (nnb == 0) { n0 = j2 + 1; s0 = lds1; }
            else n1 = j2 + 1;
            ++nnb;
        }
        line_setup<EPL>(a, pk, j2, nnb, n0, n1, mine, s0, s1);
    }
    __syncthreads();
}

// One neighbour's correction of plane k's blocks (the plane recurrence of
// Sec. 2.1), element by element over the plane: with b = z./w, z = Pt_nb^{-1} w,
// the diagonal loses psi^2 b (diagonal Schur blocks) or psi (2b - b P_nb b) psi
// plus the compensation psi b (w - P_nb z)./t (Newton), and the x- and
// y-couplings lose psi_u (-b_u P_uv b_v) psi_v.  FROM_BANDS: the plane's first
// correction, which starts from the assembled bands (no separate copy pass);
// else the blocks are corrected in place.  The pointers are restrict-qualified:
// the plane's own blocks, the neighbour's and the work lines do not overlap.
template <bool FROM_BANDS>
__device__ __forceinline__ void plane_update(const SetupArgs &a, long long pk, long long pn,
                                             const double *__restrict__ psi,
                                             const double *__restrict__ w,
                                             const double *__restrict__ z) {
    const int nx = a.nx, ny = a.ny;
    const long long nxy = (long long)nx * ny;
    double *__restrict__ dP = a.dP + pk, *__restrict__ xP = a.xP + pk;
    double *__restrict__ yP = a.f2 + pk;
    const double *__restrict__ d0 = a.d + pk, *__restrict__ x0 = a.ax + pk;
    const double *__restrict__ y0 = a.ay + pk;
    const double *__restrict__ dPn = a.dP + pn, *__restrict__ xPn = a.xP + pn;
    const double *__restrict__ yPn = a.f2 + pn;
    const double *__restrict__ t = a.t;
    for (long long u = threadIdx.x; u < nxy; u += blockDim.x) {
        const int i = (int)(u % nx), jl = (int)(u / nx);
        double dv, xv, yv;
        if constexpr (FROM_BANDS) {
            dv = d0[u];
            xv = x0[u];
            yv = y0[u];
        } else {
            dv = dP[u];
            xv = xP[u];
            yv = yP[u];
        }
        const double b = z[u] / w[u];
        if (a.schur == 1) {
            dv -= psi[u] * psi[u] * b;
        } else {
            double Pz = dPn[u] * z[u];
            if (i > 0) Pz += xPn[u - 1] * z[u - 1];
            if (i < nx - 1) Pz += xPn[u] * z[u + 1];
            if (jl > 0) Pz += yPn[u - nx] * z[u - nx];
            if (jl < ny - 1) Pz += yPn[u] * z[u + nx];
            const double xuu = 2.0 * b - b * dPn[u] * b;
            dv -= psi[u] * xuu * psi[u];
            if (i < nx - 1) {
                const double b1 = z[u + 1] / w[u + 1];
                xv -= psi[u] * (-b * xPn[u] * b1) * psi[u + 1];
            }
            if (jl < ny - 1) {
                const double bn = z[u + nx] / w[u + nx];
                yv -= psi[u] * (-b * yPn[u] * bn) * psi[u + nx];
            }
            dv += psi[u] * b * (w[u] - Pz) / (t ? t[pk + u] : 1.0);
        }
        dP[u] = dv;
        xP[u] = xv;
        yP[u] = yv;
    }
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
    if (nnb == 0) {  // no neighbour plane: the blocks are the assembled bands
        double *__restrict__ dP = a.dP + pk, *__restrict__ xP = a.xP + pk;
        double *__restrict__ yP = a.f2 + pk;
        const double *__restrict__ d0 = a.d + pk, *__restrict__ x0 = a.ax + pk;
        const double *__restrict__ y0 = a.ay + pk;
#pragma unroll 4
        for (long long u = threadIdx.x; u < nxy; u += blockDim.x) {
            dP[u] = d0[u];
            xP[u] = x0[u];
            yP[u] = y0[u];
        }
        __syncthreads();
    }
    for (int q = 0; q < nnb; ++q) {
        const int nb = q == 0 ? nb0 : nb1;
        const long long pn = nb * nxy;
        const double *__restrict__ psi = a.az + (k < nb ? k : nb) * nxy;
        {
            double *__restrict__ w = wbuf;
            const double *__restrict__ t = a.t;
#pragma unroll 4
            for (long long u = threadIdx.x; u < nxy; u += blockDim.x)
                w[u] = psi[u] * (t ? t[pk + u] : 1.0);
        }
        __syncthreads();
        PolPlain<EPL> pol;
        pol.y = make_rsrc(wbuf);
        pol.x = make_rsrc(zbuf);
        pol.line8 = (unsigned)nx * 8u;
        NatFmt<double, EPL> F(nx);
        F.e1 = make_rsrc(a.e1 + pn);
        F.mv = make_rsrc(a.mv + pn);
        F.f2 = make_rsrc(a.f2 + pn);
        F.W = pol.x;
        F.mv64 = a.mv + pn;
        F.soT = 0;
        F.soW = 0;
        F.lineB = (unsigned)nx * 8u;
        F.ny = ny;
        plane_solve<1>(ny, F, pol, lds_x);
        __syncthreads();
        if (q == 0) plane_update<true>(a, pk, pn, psi, wbuf, zbuf);
        else plane_update<false>(a, pk, pn, psi, wbuf, zbuf);
        __syncthreads();
    }
    plane_lines_setup<EPL>(a, k, lds_lines);
}

// Setup of the two level-3 half chains (h = 0: planes 0..j3-1 upward, each
// with neighbour k-1; h = 1: planes nz-1..j3+1 downward, neighbour k+1).
template <int EPL>
__device__ __forceinline__ void setup_halves(const SetupArgs &a, int h, double *smem) {
    double *lds_lines = smem;          // 2 waves x 5 lines
    double *lds_x = smem + 10 * a.nx;  // 2 x 64*EPL exchange lines
    const long long nxy = (long long)a.nx * a.ny;
    const int j3 = (a.nz - 1) / 2;
    double *wbuf = a.scratch + (2 * h) * nxy, *zbuf = a.scratch + (2 * h + 1) * nxy;
    if (h == 0) {
        for (int k = 0; k < j3; ++k)
            plane_setup<EPL>(a, k, k > 0 ? 1 : 0, k - 1, 0, wbuf, zbuf, lds_lines, lds_x);
    } else {
        for (int k = a.nz - 1; k > j3; --k)
            plane_setup<EPL>(a, k, k < a.nz - 1 ? 1 : 0, k + 1, 0, wbuf, zbuf, lds_lines, lds_x);
    }
}

// The twist plane j3 (after both halves): both neighbours.
template <int EPL>
__device__ __forceinline__ void setup_twist(const SetupArgs &a, double *smem) {
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

template <int EPL>
__global__ void __launch_bounds__(kSetupThreads<EPL>) k_setup_halves(SetupArgs a) {
    extern __shared__ double smem[];
    setup_halves<EPL>(a, blockIdx.x, smem);
}

template <int EPL>
__global__ void __launch_bounds__(kSetupThreads<EPL>) k_setup_twist(SetupArgs a) {
    extern __shared__ double smem[];
    setup_twist<EPL>(a, smem);
}

// A batch of independent systems (blockIdx.y selects the system's arguments):
// their level-3 chains run at the same time.
template <int EPL>
__global__ void __launch_bounds__(kSetupThreads<EPL>) k_setup_halves_b(const SetupArgs *tab) {
    extern __shared__ double smem[];
    setup_halves<EPL>(load_uniform(tab + blockIdx.y), blockIdx.x, smem);
}

template <int EPL>
__global__ void __launch_bounds__(kSetupThreads<EPL>) k_setup_twist_b(const SetupArgs *tab) {
    extern __shared__ double smem[];
    setup_twist<EPL>(load_uniform(tab + blockIdx.y), smem);
}

template <int EPL>
size_t setup_smem(int nx) {
    return sizeof(double) * (10 * (size_t)nx + 2 * 64 * EPL);
}

template <int EPL>
hipError_t setup_impl(const SetupArgs &a, hipStream_t s) {
    const size_t sh = setup_smem<EPL>(a.nx);
    if (sh > 65536) {
        (void)hipFuncSetAttribute((const void *)k_setup_halves<EPL>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        (void)hipFuncSetAttribute((const void *)k_setup_twist<EPL>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    }
    hipLaunchKernelGGL((k_setup_halves<EPL>), dim3(2), dim3(kSetupThreads<EPL>), sh, s, a);
    hipLaunchKernelGGL((k_setup_twist<EPL>), dim3(1), dim3(kSetupThreads<EPL>), sh, s, a);
    return hipGetLastError();
}

template <int EPL>
hipError_t setup_batch_impl(const SetupArgs *tab, int count, int max_nx, hipStream_t s) {
    const size_t sh = setup_smem<EPL>(max_nx);
    if (sh > 65536) {
        (void)hipFuncSetAttribute((const void *)k_setup_halves_b<EPL>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        (void)hipFuncSetAttribute((const void *)k_setup_twist_b<EPL>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    }
    hipLaunchKernelGGL((k_setup_halves_b<EPL>), dim3(2, count), dim3(kSetupThreads<EPL>), sh, s, tab);
    hipLaunchKernelGGL((k_setup_twist_b<EPL>), dim3(1, count), dim3(kSetupThreads<EPL>), sh, s, tab);
    return hipGetLastError();
}

}  // namespace

// Supported elements per lane: a half chain holds up to 32*EPL positions.
#define NTD_EPL_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(10) X(12) X(14) X(16)
// Elements per lane of the batched apply (lines of up to 512 points).
#define NTD_BATCH_EPL_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)

}  // namespace ntd
