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
// Scheduling.  Row p depends only on its lower neighbours p-1, p-nx, p-nx*ny.
// The factorization (once per setup) takes all rows of a hyperplane
// i + j + (k - k0) = level (k0 = 0 in the first block, the plane of row M in
// the second) in one launch, both blocks at once.  The sweeps of every
// application are tiled instead: an x-line (j, k) depends on lines (j-1, k)
// and (j, k-1) only through elementwise terms, and along x it is a first-order
// linear recurrence, solved by one wavefront as a 64-lane affine scan.  A
// workgroup of kIluTile wavefronts owns a tile of kIluTile x kIluTile lines
// and walks its line anti-diagonals with one barrier each, passing each line
// to its successors through LDS; tiles on one anti-diagonal of the tile grid
// (both blocks) form one launch, so a sweep takes about (ny + nz/2)/kIluTile
// launches instead of nx + ny + nz/2.
#include "ntd_sweep.h"

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

constexpr int kIluThreads = 64 * kIluTile;  // one wavefront per tile row
constexpr int kRowBcast31 = 0x143;

// x_c = a_c x_{c-1} + b_c over the 64*E positions c = lane*E + s of the
// wavefront (x_{-1} = 0), in place of b: lane composites, a 64-lane scan of
// affine maps (rows, then rows 1 and 3 from lanes 15 and 47, then rows 2 and 3
// from lane 31), then the lane-local recurrence from the exclusive carry.
template <int E>
__device__ __forceinline__ void line_recurrence(const double (&a)[E], double (&b)[E]) {
    double A = 1.0, B = 0.0;
#pragma unroll
    for (int s = 0; s < E; ++s) {
        B = a[s] * B + b[s];
        A = a[s] * A;
    }
#define NTD_ILU_STEP(CTRL, RM)                                                   \
    {                                                                            \
        const double Ap = dpp<CTRL, RM>(1.0, A), Bp = dpp<CTRL, RM>(0.0, B);     \
        B = A * Bp + B;                                                          \
        A = A * Ap;                                                              \
    }
    NTD_ILU_STEP(kRowShr1, 0xF)
    NTD_ILU_STEP(kRowShr2, 0xF)
    NTD_ILU_STEP(kRowShr4, 0xF)
    NTD_ILU_STEP(kRowShr8, 0xF)
    NTD_ILU_STEP(kRowBcast15, 0xA)
#undef NTD_ILU_STEP
    B = A * dpp<kRowBcast31, 0xC>(0.0, B) + B;
    double carry = dpp<kWaveShr1>(0.0, B);
#pragma unroll
    for (int s = 0; s < E; ++s) {
        b[s] = a[s] * carry + b[s];
        carry = b[s];
    }
}

// Tile (block b, ty, tz) of tile anti-diagonal L served by this workgroup.
__device__ __forceinline__ bool tile_of(const IluGrid &g, int L, int &b, int &ty, int &tz) {
    int idx = blockIdx.x;
    for (b = 0; b < 2; ++b) {
        const int lo = L - (g.TY - 1) > 0 ? L - (g.TY - 1) : 0;
        const int hi = L < g.TZ[b] - 1 ? L : g.TZ[b] - 1;
        const int cnt = hi >= lo ? hi - lo + 1 : 0;
        if (idx < cnt) {
            tz = lo + idx;
            ty = L - tz;
            return true;
        }
        idx -= cnt;
    }
    return false;
}

__device__ __forceinline__ bool in_block(long long p, int b, const IluGrid &g) {
    return g.nblocks == 1 || ((p >= g.M) == (b == 1));
}

// Grid line (j, k) at tile row w, line anti-diagonal ll of tile (ty, tz) of
// the block that spans planes kb0..kb1, or false if it does not exist.
__device__ __forceinline__ bool tile_line(const IluGrid &g, int kb0, int kb1, int ty, int tz,
                                          int w, int ll, int &j, int &k) {
    const int kl = ll - w;
    j = ty * kIluTile + w;
    k = kb0 + tz * kIluTile + kl;
    return kl >= 0 && kl < kIluTile && j < g.ny && k <= kb1;
}

// The plane range of block b, read once per workgroup: selected from both
// entries rather than indexed, so that it stays in scalar registers (an
// indexed read of the argument would be a scalar memory load, and its wait
// would also drain the LDS accesses in flight, on every line diagonal).
__device__ __forceinline__ void block_planes(const IluGrid &g, int b, int &kb0, int &kb1) {
    kb0 = b == 0 ? g.kb0[0] : g.kb0[1];
    kb1 = b == 0 ? g.kb1[0] : g.kb1[1];
}

// Does row M (the block split) fall strictly inside the x-line starting at base?
__device__ __forceinline__ bool cut_by_split(const IluGrid &g, long long base) {
    return g.nblocks == 2 && base < g.M && g.M < base + g.nx;
}

// Element offsets of the positions c = lane*E + s of a line: element i = c
// (forward) or i = 64E - 1 - c (backward), 8*i bytes, or kOOB past the line.
// With VEC (nx a multiple of E) a lane's elements are one aligned chunk, at
// byte offset co (kOOB when outside the line).
template <int E, bool REV>
struct IluLanes {
    unsigned eo[E], eo4[E];  // for 8- and 4-byte arrays
    unsigned co, co4;
    __device__ IluLanes(int nx) {
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int c = lane * E + s;
            const int i = REV ? 64 * E - 1 - c : c;
            eo[s] = i < nx ? 8u * (unsigned)i : kOOB;
            eo4[s] = i < nx ? 4u * (unsigned)i : kOOB;
        }
        const int i0 = REV ? 64 * E - E - lane * E : lane * E;
        co = i0 + E - 1 < nx ? 8u * (unsigned)i0 : kOOB;
        co4 = i0 + E - 1 < nx ? 4u * (unsigned)i0 : kOOB;
    }
    __device__ int elem(int s) const {
        const int c = (threadIdx.x & 63) * E + s;
        return REV ? 64 * E - 1 - c : c;
    }
};

template <int E, bool REV, bool VEC>
__device__ __forceinline__ void ld(rsrc_t r, unsigned so, const IluLanes<E, REV> &L,
                                   double (&v)[E]) {
    if constexpr (VEC) {
        double t[E];
        vload(r, L.co, so, t);
#pragma unroll
        for (int s = 0; s < E; ++s) v[s] = REV ? t[E - 1 - s] : t[s];
    } else {
#pragma unroll
        for (int s = 0; s < E; ++s) v[s] = bload((double *)nullptr, r, L.eo[s], so);
    }
}

// A coefficient line of type CT (double, or float in MIXED): so is the byte
// offset of the line in an 8-byte array (halved for a 4-byte one).
template <int E, bool REV, bool VEC, typename CT>
__device__ __forceinline__ void ldc(rsrc_t r, unsigned so, const IluLanes<E, REV> &L,
                                    CT (&v)[E]) {
    if constexpr (sizeof(CT) == 8) {
        ld<E, REV, VEC>(r, so, L, v);
    } else if constexpr (VEC) {
        CT t[E];
        vload(r, L.co4, so >> 1, t);
#pragma unroll
        for (int s = 0; s < E; ++s) v[s] = REV ? t[E - 1 - s] : t[s];
    } else {
#pragma unroll
        for (int s = 0; s < E; ++s) v[s] = bload((CT *)nullptr, r, L.eo4[s], so >> 1);
    }
}

// ld, or (use false) the same load with every lane out of bounds: zeros, and
// no data moved through the cache path.
template <int E, bool REV, bool VEC>
__device__ __forceinline__ void ld_if(rsrc_t r, unsigned so, const IluLanes<E, REV> &L,
                                      double (&v)[E], bool use) {
    if constexpr (VEC) {
        double t[E];
        vload(r, use ? L.co : kOOB, so, t);
#pragma unroll
        for (int s = 0; s < E; ++s) v[s] = REV ? t[E - 1 - s] : t[s];
    } else {
#pragma unroll
        for (int s = 0; s < E; ++s) v[s] = bload((double *)nullptr, r, use ? L.eo[s] : kOOB, so);
    }
}

template <int E, bool REV, bool VEC>
__device__ __forceinline__ void st(rsrc_t r, unsigned so, const IluLanes<E, REV> &L,
                                   const double (&v)[E]) {
    if constexpr (VEC) {
        double t[E];
#pragma unroll
        for (int s = 0; s < E; ++s) t[REV ? E - 1 - s : s] = v[s];
        vstore(r, L.co, so, t);
    } else {
#pragma unroll
        for (int s = 0; s < E; ++s) bstore(v[s], r, L.eo[s], so);
    }
}

// Inputs of one line of a tiled sweep that do not depend on the sweep's own
// results inside the tile (loaded one anti-diagonal ahead): the right-hand
// side (forward) or forward result (backward), 1/dt, the couplings, and the
// neighbour lines that lie in earlier tiles (zero when absent).
// The coefficients (1/dt and the couplings) are stored as CT and used in FP64.
template <int E, typename CT>
struct IluLine {
    double rv[E], vy[E], vz[E];
    CT di[E], cx[E], cy[E], cz[E];
};

template <typename CT>
struct IluPtrs {
    const CT *ax, *ay, *az, *di;
    const double *r;
    double *y;
};

struct IluBufs {
    rsrc_t ax, ay, az, di, r, y;
    template <typename CT>
    __device__ explicit IluBufs(const IluPtrs<CT> &p)
        : ax(make_rsrc(p.ax)), ay(make_rsrc(p.ay)), az(make_rsrc(p.az)), di(make_rsrc(p.di)),
          r(make_rsrc(p.r)), y(make_rsrc(p.y)) {}
};

// Rows of the x-lines starting at base and base2 lie in the same block.
__device__ __forceinline__ bool same_block(const IluGrid &g, long long base, long long base2) {
    return g.nblocks == 1 || ((base >= g.M) == (base2 >= g.M));
}

// Forward sweep (Dt + L) y = r on the tiles of anti-diagonal L:
// y_p = (r_p - sum over kept lower neighbours q of a_qp y_q) / dt_p.
template <int E, bool VEC, typename CT>
__global__ void __launch_bounds__(kIluThreads) k_ilu_fwd_tile(IluGrid g, int L, IluPtrs<CT> P) {
    extern __shared__ double lds[];  // two anti-diagonals of kIluTile lines, [s][lane]
    int b, ty, tz;
    if (!tile_of(g, L, b, ty, tz)) return;
    int kb0, kb1;
    block_planes(g, b, kb0, kb1);
    const IluBufs B(P);
    // the wavefront index is uniform per wavefront; say so, or every buffer
    // access with an offset derived from it becomes a per-lane loop
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int nx = g.nx;
    const unsigned nx8 = 8u * nx, nxy8 = 8u * (unsigned)g.nxy;
    const IluLanes<E, false> Ln(nx);
    // Every load is issued, at line 0 for a line outside the grid and at the
    // line itself for an absent neighbour: a skipped load would leave the
    // waits before the next solve unable to count, and they would drain the
    // loads in flight.  Values of absent neighbours, and neighbours that solve
    // takes from LDS instead, are never used.
    auto load = [&](int ll, IluLine<E, CT> &d) {
        int j, k;
        const bool ok = tile_line(g, kb0, kb1, ty, tz, w, ll, j, k);
        const unsigned so = ok ? 8u * (unsigned)(((long long)k * g.ny + j) * nx) : 0u;
        const unsigned sy = ok && j > 0 ? so - nx8 : so;
        const unsigned sz = ok && k > 0 ? so - nxy8 : so;
        ld<E, false, VEC>(B.r, so, Ln, d.rv);
        ldc<E, false, VEC>(B.di, so, Ln, d.di);
        // ax of element i-1 (0 at i = 0 and past the line)
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const bool in = Ln.eo[s] != kOOB && Ln.elem(s) > 0;
            if constexpr (sizeof(CT) == 8)
                d.cx[s] = bload((CT *)nullptr, B.ax, in ? Ln.eo[s] - 8u : kOOB, so);
            else
                d.cx[s] = bload((CT *)nullptr, B.ax, in ? Ln.eo4[s] - 4u : kOOB, so >> 1);
        }
        ldc<E, false, VEC>(B.ay, sy, Ln, d.cy);
        ld_if<E, false, VEC>(B.y, sy, Ln, d.vy, w == 0);  // used at w = 0: tile ty-1
        ldc<E, false, VEC>(B.az, sz, Ln, d.cz);
        ld_if<E, false, VEC>(B.y, sz, Ln, d.vz, ll - w == 0);  // at ll - w = 0: tile tz-1
    };
    auto solve = [&](int ll, const IluLine<E, CT> &d) {
        int j, k;
        if (!tile_line(g, kb0, kb1, ty, tz, w, ll, j, k)) return;
        const int kl = ll - w;
        const long long base = ((long long)k * g.ny + j) * nx;
        const unsigned so = 8u * (unsigned)base;
        double *cur = lds + (ll & 1) * kIluTile * 64 * E;
        const double *prv = lds + ((ll + 1) & 1) * kIluTile * 64 * E;
        double a[E], v[E], ny_[E], nz_[E];
#pragma unroll
        for (int s = 0; s < E; ++s) {
            ny_[s] = w > 0 ? prv[((w - 1) * E + s) * 64 + lane] : d.vy[s];
            nz_[s] = kl > 0 ? prv[(w * E + s) * 64 + lane] : d.vz[s];
        }
        const bool generic = cut_by_split(g, base) || cut_by_split(g, base - nx) ||
                             cut_by_split(g, base - g.nxy);
        if (!generic) {
            // the line and its neighbour lines lie wholly on one side of row M
            const bool mine = g.nblocks == 1 || ((base >= g.M) == (b == 1));
            if (!mine) return;  // only in the plane shared by the two blocks
            const bool yk = j > 0 && same_block(g, base, base - nx);
            const bool zk = k > 0 && same_block(g, base, base - g.nxy);
#pragma unroll
            for (int s = 0; s < E; ++s) {
                double c = d.rv[s];
                if (yk) c -= d.cy[s] * ny_[s];
                if (zk) c -= d.cz[s] * nz_[s];
                v[s] = Ln.eo[s] != kOOB ? d.di[s] * c : 0.0;
                a[s] = -(double)d.di[s] * (double)d.cx[s];
            }
        } else {
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int i = Ln.elem(s);
                const long long p = base + i;
                a[s] = 0.0;
                v[s] = 0.0;
                if (i < nx && in_block(p, b, g)) {
                    double c = d.rv[s];
                    if (j > 0 && kept(p - nx, p, g)) c -= d.cy[s] * ny_[s];
                    if (k > 0 && kept(p - g.nxy, p, g)) c -= d.cz[s] * nz_[s];
                    v[s] = d.di[s] * c;
                    if (i > 0 && kept(p - 1, p, g)) a[s] = -(double)d.di[s] * (double)d.cx[s];
                }
            }
        }
        line_recurrence<E>(a, v);
#pragma unroll
        for (int s = 0; s < E; ++s) cur[(w * E + s) * 64 + lane] = v[s];
        if (!generic) {
            st<E, false, VEC>(B.y, so, Ln, v);
        } else {
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int i = Ln.elem(s);
                if (i < nx && in_block(base + i, b, g)) bstore(v[s], B.y, Ln.eo[s], so);
            }
        }
    };
    constexpr int NL = 2 * kIluTile - 1;
    IluLine<E, CT> A, Bq;
#pragma unroll
    for (int s = 0; s < E; ++s) A.cy[s] = A.cz[s] = A.vy[s] = A.vz[s] = Bq.cy[s] = Bq.cz[s] =
        Bq.vy[s] = Bq.vz[s] = 0.0;
    // pairs of line diagonals with the next one's inputs in flight, then the
    // last diagonal: no conditional half-steps, so the two input buffers keep
    // their registers and no wait drains the prefetched loads
    static_assert(NL % 2 == 1, "odd number of line diagonals");
    load(0, A);
    for (int ll = 0; ll + 2 < NL; ll += 2) {
        load(ll + 1, Bq);
        solve(ll, A);
        __syncthreads();
        load(ll + 2, A);
        solve(ll + 1, Bq);
        __syncthreads();
    }
    solve(NL - 1, A);
}

// Backward sweep (I + Dt^{-1} U) z = y in place on the tiles of anti-diagonal L
// (visited in decreasing order): z_p = y_p - (sum over kept upper neighbours q
// of a_pq z_q) / dt_p.  Lanes take the positions of the line in reverse
// (c = 0 is element nx-1 padded to 64*E), so the recurrence runs forward in c.
template <int E, bool VEC, typename CT>
__global__ void __launch_bounds__(kIluThreads) k_ilu_bwd_tile(IluGrid g, int L, IluPtrs<CT> P) {
    extern __shared__ double lds[];
    int b, ty, tz;
    if (!tile_of(g, L, b, ty, tz)) return;
    int kb0, kb1;
    block_planes(g, b, kb0, kb1);
    const IluBufs B(P);
    // the wavefront index is uniform per wavefront; say so, or every buffer
    // access with an offset derived from it becomes a per-lane loop
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int nx = g.nx;
    const unsigned nx8 = 8u * nx, nxy8 = 8u * (unsigned)g.nxy;
    const IluLanes<E, true> Ln(nx);
    // every load issued, as in the forward sweep
    auto load = [&](int ll, IluLine<E, CT> &d) {
        int j, k;
        const bool ok = tile_line(g, kb0, kb1, ty, tz, w, ll, j, k);
        const unsigned so = ok ? 8u * (unsigned)(((long long)k * g.ny + j) * nx) : 0u;
        const unsigned sy = ok && j < g.ny - 1 ? so + nx8 : so;
        const unsigned sz = ok && k < g.nz - 1 ? so + nxy8 : so;
        ld<E, true, VEC>(B.y, so, Ln, d.rv);  // the forward result of this line
        ldc<E, true, VEC>(B.di, so, Ln, d.di);
        ldc<E, true, VEC>(B.ax, so, Ln, d.cx);
        ldc<E, true, VEC>(B.ay, so, Ln, d.cy);
        ld_if<E, true, VEC>(B.y, sy, Ln, d.vy, w == kIluTile - 1);  // tile ty+1
        ldc<E, true, VEC>(B.az, so, Ln, d.cz);
        ld_if<E, true, VEC>(B.y, sz, Ln, d.vz, ll - w == kIluTile - 1);  // tile tz+1
    };
    auto solve = [&](int ll, const IluLine<E, CT> &d) {
        int j, k;
        if (!tile_line(g, kb0, kb1, ty, tz, w, ll, j, k)) return;
        const int kl = ll - w;
        const long long base = ((long long)k * g.ny + j) * nx;
        const unsigned so = 8u * (unsigned)base;
        double *cur = lds + (ll & 1) * kIluTile * 64 * E;
        const double *prv = lds + ((ll + 1) & 1) * kIluTile * 64 * E;
        double a[E], v[E], ny_[E], nz_[E];
#pragma unroll
        for (int s = 0; s < E; ++s) {
            ny_[s] = w < kIluTile - 1 ? prv[((w + 1) * E + s) * 64 + lane] : d.vy[s];
            nz_[s] = kl < kIluTile - 1 ? prv[(w * E + s) * 64 + lane] : d.vz[s];
        }
        const bool generic = cut_by_split(g, base) || cut_by_split(g, base + nx) ||
                             cut_by_split(g, base + g.nxy);
        if (!generic) {
            const bool mine = g.nblocks == 1 || ((base >= g.M) == (b == 1));
            if (!mine) return;
            const bool yk = j < g.ny - 1 && same_block(g, base, base + nx);
            const bool zk = k < g.nz - 1 && same_block(g, base, base + g.nxy);
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int i = Ln.elem(s);
                double c = 0.0;
                if (yk) c += d.cy[s] * ny_[s];
                if (zk) c += d.cz[s] * nz_[s];
                v[s] = Ln.eo[s] != kOOB ? d.rv[s] - d.di[s] * c : 0.0;
                a[s] = i < nx - 1 ? -(double)d.di[s] * (double)d.cx[s] : 0.0;
            }
        } else {
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int i = Ln.elem(s);
                const long long p = base + i;
                a[s] = 0.0;
                v[s] = 0.0;
                if (i < nx && in_block(p, b, g)) {
                    double c = 0.0;
                    if (j < g.ny - 1 && kept(p, p + nx, g)) c += d.cy[s] * ny_[s];
                    if (k < g.nz - 1 && kept(p, p + g.nxy, g)) c += d.cz[s] * nz_[s];
                    v[s] = d.rv[s] - d.di[s] * c;
                    if (i < nx - 1 && kept(p, p + 1, g)) a[s] = -(double)d.di[s] * (double)d.cx[s];
                }
            }
        }
        line_recurrence<E>(a, v);
#pragma unroll
        for (int s = 0; s < E; ++s) cur[(w * E + s) * 64 + lane] = v[s];
        if (!generic) {
            st<E, true, VEC>(B.y, so, Ln, v);
        } else {
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int i = Ln.elem(s);
                if (i < nx && in_block(base + i, b, g)) bstore(v[s], B.y, Ln.eo[s], so);
            }
        }
    };
    constexpr int NL = 2 * kIluTile - 1;
    IluLine<E, CT> A, Bq;
#pragma unroll
    for (int s = 0; s < E; ++s) A.cy[s] = A.cz[s] = A.vy[s] = A.vz[s] = Bq.cy[s] = Bq.cz[s] =
        Bq.vy[s] = Bq.vz[s] = 0.0;
    static_assert(NL % 2 == 1, "odd number of line diagonals");
    load(NL - 1, A);
    for (int ll = NL - 1; ll - 2 >= 0; ll -= 2) {
        load(ll - 1, Bq);
        solve(ll, A);
        __syncthreads();
        load(ll - 2, A);
        solve(ll - 1, Bq);
        __syncthreads();
    }
    solve(0, A);
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
    g.kb0[0] = 0;
    g.kb1[0] = nblocks == 2 ? (g.M > 0 ? (int)((g.M - 1) / g.nxy) : -1) : nz - 1;
    g.kb0[1] = nblocks == 2 ? (int)(g.M / g.nxy) : 0;
    g.kb1[1] = nblocks == 2 ? nz - 1 : -1;
    g.TY = (ny + kIluTile - 1) / kIluTile;
    int tzmax = 0;
    for (int b = 0; b < 2; ++b) {
        const int np = g.kb1[b] >= g.kb0[b] ? g.kb1[b] - g.kb0[b] + 1 : 0;
        g.TZ[b] = (np + kIluTile - 1) / kIluTile;
        if (g.TZ[b] > tzmax) tzmax = g.TZ[b];
    }
    g.tlevels = tzmax > 0 ? g.TY + tzmax - 1 : 0;
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

namespace {

int tiles_on(const IluGrid &g, int L) {
    int n = 0;
    for (int b = 0; b < 2; ++b) {
        const int lo = L - (g.TY - 1) > 0 ? L - (g.TY - 1) : 0;
        const int hi = L < g.TZ[b] - 1 ? L : g.TZ[b] - 1;
        if (hi >= lo) n += hi - lo + 1;
    }
    return n;
}

template <int E, bool VEC, typename CT>
hipError_t ilu_apply_e(const IluGrid &g, const IluPtrs<CT> &fb, hipStream_t s) {
    const size_t sh = 2 * (size_t)kIluTile * 64 * E * sizeof(double);
    if (sh > 65536) {
        (void)hipFuncSetAttribute((const void *)k_ilu_fwd_tile<E, VEC, CT>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        (void)hipFuncSetAttribute((const void *)k_ilu_bwd_tile<E, VEC, CT>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    }
    for (int L = 0; L < g.tlevels; ++L)
        hipLaunchKernelGGL((k_ilu_fwd_tile<E, VEC, CT>), dim3(tiles_on(g, L)), dim3(kIluThreads),
                           sh, s, g, L, fb);
    for (int L = g.tlevels - 1; L >= 0; --L)
        hipLaunchKernelGGL((k_ilu_bwd_tile<E, VEC, CT>), dim3(tiles_on(g, L)), dim3(kIluThreads),
                           sh, s, g, L, fb);
    return hipGetLastError();
}

template <int E, typename CT>
hipError_t ilu_apply_v(const IluGrid &g, const IluPtrs<CT> &fb, hipStream_t s) {
    if (g.nx % E == 0) return ilu_apply_e<E, true>(g, fb, s);
    return ilu_apply_e<E, false>(g, fb, s);
}

template <typename CT>
hipError_t ilu_apply_t(const IluGrid &g, const IluPtrs<CT> &fb, hipStream_t s) {
    const int e = (g.nx + 63) / 64;
    if (e <= 1) return ilu_apply_v<1>(g, fb, s);
    if (e <= 2) return ilu_apply_v<2>(g, fb, s);
    if (e <= 4) return ilu_apply_v<4>(g, fb, s);
    // 6 per lane (nx up to 384, e.g. 350) keeps the two input buffers in registers,
    // where 8 per lane spills
    if (e <= 6) return ilu_apply_v<6>(g, fb, s);
    if (e <= 8) return ilu_apply_v<8>(g, fb, s);
    return ilu_apply_v<16>(g, fb, s);
}

// The coefficients of the sweeps in FP32: ax, ay, az, 1/dt one after another.
__global__ void __launch_bounds__(256) k_ilu_coef_f32(const double *__restrict__ ax,
                                                      const double *__restrict__ ay,
                                                      const double *__restrict__ az,
                                                      const double *__restrict__ dtinv,
                                                      float *__restrict__ out, long long n) {
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        out[i] = (float)ax[i];
        out[n + i] = (float)ay[i];
        out[2 * n + i] = (float)az[i];
        out[3 * n + i] = (float)dtinv[i];
    }
}

}  // namespace

hipError_t launch_ilu_apply(const IluGrid &g, const double *ax, const double *ay, const double *az,
                            const double *dtinv, const float *fcoef, const double *r, double *z,
                            hipStream_t s) {
    if (fcoef) {
        const long long n = g.N;
        const IluPtrs<float> fb{fcoef, fcoef + n, fcoef + 2 * n, fcoef + 3 * n, r, z};
        return ilu_apply_t(g, fb, s);
    }
    const IluPtrs<double> fb{ax, ay, az, dtinv, r, z};
    return ilu_apply_t(g, fb, s);
}

hipError_t launch_ilu_coef_f32(const IluGrid &g, const double *ax, const double *ay,
                               const double *az, const double *dtinv, float *fcoef,
                               hipStream_t s) {
    long long nb = (g.N + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_ilu_coef_f32, dim3((unsigned)nb), dim3(256), 0, s, ax, ay, az, dtinv,
                       fcoef, g.N);
    return hipGetLastError();
}

}  // namespace ntd
