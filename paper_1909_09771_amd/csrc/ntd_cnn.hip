// ntd_cnn.hip -- the learned filter vector: a four-layer 3D convolutional
// network kappa -> t > 0 (layers 1-16-16-16-1, 3x3x3 taps, zero padding, ReLU
// between layers, softplus + 1e-3 at the output), its loss gradient and an
// Adam step.  The premise (Sec. 1 of arXiv:1909.09771): B(t) reproduces A on
// the filter vector t, so a t close to A's lowest eigenvectors is the natural
// thing to predict; t = 1 is the rowsum choice.
//
// Layouts (N = nx*ny*nz voxels, x fastest):
//   feature H0          bf16 [N]
//   hidden H1..H3       bf16 [N][16] (channels last)
//   output y            fp32 [N];  t = softplus(y) + 1e-3 as fp64 [N]
//   parameters          fp32, per layer W[cout][tap][cin] then b[cout],
//                       tap = 9 (dz+1) + 3 (dy+1) + (dx+1)
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16: M = 16 voxels
// along x, N = 16 output channels, K = 27 taps x cin (padded to a multiple of
// 32).  One wavefront walks one grid row (y, z) in tiles of 16 voxels and keeps
// the packed weights of its layer in registers.  The gradient with respect to
// a layer's input is the same kernel run with the adjoint weights (taps
// mirrored, cin and cout swapped), masked by the ReLU derivative.  The weight
// gradient is a correlation over the whole grid: plain FP32 FMAs per block,
// then a fixed-order sum over the blocks.
#include "ntd.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16_t;  // bfloat16 bits in storage

constexpr int kTaps = 27;
constexpr int kHid = 16;
constexpr float kEpsT = 1.0e-3f;
constexpr double kFeatureScale = 3.0;
constexpr int kWgMaxBlocks = 256;   // weight-gradient partial blocks
constexpr int kRedBlocks = 1024;    // reduction partial blocks
constexpr size_t kAlign = 256;
constexpr long long kMaxVoxels = 1LL << 28;

struct Layer {
    int cin, cout, woff, boff;
};

__host__ __device__ constexpr Layer layer_desc(int l) {
    return l == 0 ? Layer{1, 16, 0, 432}
         : l == 1 ? Layer{16, 16, 448, 448 + 6912}
         : l == 2 ? Layer{16, 16, 448 + 6928, 448 + 6928 + 6912}
                  : Layer{16, 1, 448 + 2 * 6928, 448 + 2 * 6928 + 432};
}
static_assert(448 + 2 * 6928 + 433 == NTD_CNN_NPARAMS, "parameter layout");

// Packed weights of one convolution: the MFMA B operand, [kb][lane][8] bf16,
// lane = 16 g + n holding B[k = 32 kb + 8 g + j][n], j = 0..7.
__host__ __device__ constexpr int pack_kb(int cin) { return (kTaps * cin + 31) / 32; }
// Jobs 0-3: forward weights of layers 0-3; jobs 4-6: adjoint weights of layers 1-3.
__host__ __device__ constexpr int pack_off(int job) {
    return job == 0 ? 0 : job == 1 ? 512 : job == 2 ? 7680 : job == 3 ? 14848
         : job == 4 ? 22016 : job == 5 ? 29184 : job == 6 ? 36352 : 36864;
}
constexpr int kPackElems = pack_off(7);
constexpr int kPackMaxJob = 14 * 512;  // elements of the largest job (27 x 16 inputs)
static_assert(pack_off(2) - pack_off(1) == kPackMaxJob && pack_off(7) - pack_off(6) == 512,
              "pack sizes");

__device__ inline bf16_t f2bf(float f) {  // round to nearest, ties to even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__device__ inline float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline float softplusf(float y) { return fmaxf(y, 0.0f) + log1pf(expf(-fabsf(y))); }

__global__ __launch_bounds__(256) void k_cnn_pack(const float *__restrict__ params,
                                                  bf16_t *__restrict__ packs) {
    const int job = blockIdx.y;
    const int layer = job < 4 ? job : job - 3;
    const bool adj = job >= 4;
    const Layer L = layer_desc(layer);
    const int cin = adj ? L.cout : L.cin, cout = adj ? L.cin : L.cout;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= pack_off(job + 1) - pack_off(job)) return;
    const int j = e & 7, lane = (e >> 3) & 63, kb = e >> 9;
    const int n = lane & 15, k = kb * 32 + 8 * (lane >> 4) + j;
    const int tap = k / cin, c = k % cin;
    float w = 0.0f;
    if (tap < kTaps && n < cout) {
        // forward: W[co = n][tap][ci = c]; adjoint: W[co = c][26 - tap][ci = n]
        const int co = adj ? c : n, ci = adj ? n : c, tp = adj ? kTaps - 1 - tap : tap;
        w = params[L.woff + (co * kTaps + tp) * L.cin + ci];
    }
    packs[pack_off(job) + e] = f2bf(w);
}

enum Epi : int { kEpiRelu = 0, kEpiFinal = 1, kEpiMask = 2 };

struct ConvArgs {
    const bf16_t *in;    // [N][CIN]
    const bf16_t *wp;    // packed weights
    const float *bias;   // kEpiRelu: [16]; kEpiFinal: [1]
    const bf16_t *mask;  // kEpiMask: [N][16], the layer input whose ReLU gates the gradient
    bf16_t *out;         // kEpiRelu, kEpiMask: [N][16]
    float *y;            // kEpiFinal: [N]
    double *t;           // kEpiFinal: [N] or null
    int nx, ny, nz;
};

// A-operand fragments of the 16-voxel tile whose lane row is voxel (x, y, z):
// k = 32 kb + 8 g + j.  Every load is issued (at voxel 0 where the neighbour
// is outside the grid or the tile) and masked afterwards, so that the wait
// counts stay exact when the next tile's loads are in flight.
template <int CIN>
__device__ __forceinline__ void conv_frag(const ConvArgs &a, int x, int y, int z, int g,
                                          bf16x8 (&av)[pack_kb(CIN)]) {
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    if constexpr (CIN == kHid) {
#pragma unroll
        for (int kb = 0; kb < pack_kb(CIN); ++kb) {
            // tap 2 kb + g/2, channels 8 (g%2) .. +7
            const int tap = 2 * kb + (g >> 1);
            const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
            const int xx = x + dx, yy = y + dy, zz = z + dz;
            const bool ok = tap < kTaps && x < nx && xx >= 0 && xx < nx && yy >= 0 && yy < ny &&
                            zz >= 0 && zz < nz;
            const size_t vox = ok ? ((size_t)zz * ny + yy) * nx + xx : 0;
            const bf16x8 v = *reinterpret_cast<const bf16x8 *>(a.in + vox * kHid +
                                                                (size_t)((g & 1) << 3));
            const bf16x8 zero = {};
            av[kb] = ok ? v : zero;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {  // one input channel: k = tap = 8 g + j
            const int tap = 8 * g + j;
            const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
            const int xx = x + dx, yy = y + dy, zz = z + dz;
            const bool ok = tap < kTaps && x < nx && xx >= 0 && xx < nx && yy >= 0 && yy < ny &&
                            zz >= 0 && zz < nz;
            const size_t vox = ok ? ((size_t)zz * ny + yy) * nx + xx : 0;
            const bf16_t h = a.in[vox];
            av[0][j] = __builtin_bit_cast(__bf16, ok ? h : (bf16_t)0);
        }
    }
}

// Values the epilogue of the tile at x0 reads besides the accumulators: the
// ReLU mask of its outputs (kEpiMask), loaded before the next tile's fragments
// are issued so that waiting for them leaves those in flight.
struct ConvPre {
    bf16_t mask[4];
};

template <int EPI>
__device__ __forceinline__ ConvPre conv_pre(const ConvArgs &a, int x0, int y, int z, int lane) {
    ConvPre p{};
    if constexpr (EPI == kEpiMask) {
        const int g = lane >> 4, n = lane & 15;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int xo = x0 + 4 * g + i;
            const size_t v = ((size_t)z * a.ny + y) * a.nx + (xo < a.nx ? xo : a.nx - 1);
            p.mask[i] = a.mask[v * kHid + n];
        }
    }
    return p;
}

// D[4 g + i][n] of the tile at x0 sits in lane 16 g + n, element i; bias is
// this lane's output-channel bias (kEpiRelu: channel n, kEpiFinal: channel 0).
template <int EPI>
__device__ __forceinline__ void conv_out(const ConvArgs &a, int x0, int y, int z, int lane,
                                         float bias, const ConvPre &pre, const f32x4 &acc) {
    const int g = lane >> 4, n = lane & 15;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int xo = x0 + 4 * g + i;
        if (xo >= a.nx) continue;
        const size_t v = ((size_t)z * a.ny + y) * a.nx + xo;
        if constexpr (EPI == kEpiRelu) {
            a.out[v * kHid + n] = f2bf(fmaxf(acc[i] + bias, 0.0f));
        } else if constexpr (EPI == kEpiMask) {
            a.out[v * kHid + n] = pre.mask[i] != 0 ? f2bf(acc[i]) : (bf16_t)0;
        } else {
            if (n == 0) {
                const float yv = acc[i] + bias;
                a.y[v] = yv;
                if (a.t) a.t[v] = (double)(softplusf(yv) + kEpsT);
            }
        }
    }
}

template <int NKB>
__device__ __forceinline__ f32x4 conv_mma(const bf16x8 (&av)[NKB], const bf16x8 (&wb)[NKB]) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[kb], wb[kb], acc, 0, 0, 0);
    return acc;
}

// One wavefront per grid row (y, z), tiles of 16 voxels along x; the
// fragments of the next tile load while the current tile's MFMAs run.
template <int CIN, int EPI>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a) {
    constexpr int NKB = pack_kb(CIN);
    const int lane = threadIdx.x & 63;
    const long long row = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= (long long)a.ny * a.nz) return;  // whole wavefront
    const int y = (int)(row % a.ny), z = (int)(row / a.ny);
    const int nx = a.nx;
    const bf16x8 *wp = reinterpret_cast<const bf16x8 *>(a.wp);
    bf16x8 wb[NKB];
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) wb[kb] = wp[kb * 64 + lane];
    const int m = lane & 15, g = lane >> 4;
    float bias = 0.0f;
    if constexpr (EPI == kEpiRelu) bias = a.bias[m];
    if constexpr (EPI == kEpiFinal) bias = a.bias[0];
    bf16x8 fa[NKB], fb[NKB];
    conv_frag<CIN>(a, m, y, z, g, fa);
    for (int x0 = 0;;) {
        // past the last tile the "next" loads repeat the current tile
        ConvPre pre = conv_pre<EPI>(a, x0, y, z, lane);
        const int xa = x0 + 16 < nx ? x0 + 16 : x0;
        conv_frag<CIN>(a, xa + m, y, z, g, fb);
        conv_out<EPI>(a, x0, y, z, lane, bias, pre, conv_mma<NKB>(fa, wb));
        if (x0 + 16 >= nx) break;
        x0 += 16;
        pre = conv_pre<EPI>(a, x0, y, z, lane);
        const int xb = x0 + 16 < nx ? x0 + 16 : x0;
        conv_frag<CIN>(a, xb + m, y, z, g, fa);
        conv_out<EPI>(a, x0, y, z, lane, bias, pre, conv_mma<NKB>(fb, wb));
        if (x0 + 16 >= nx) break;
        x0 += 16;
    }
}

struct WgArgs {
    const bf16_t *h;  // layer input [N][CIN]
    const bf16_t *g;  // gradient at the layer output [N][COUT]
    float *partial;   // [blocks][COUT*27*CIN + COUT]
    int nx, ny, nz, rows_per_block;
};

// Thread tid < 27*CIN owns (tap, ci) = (tid / CIN, tid % CIN) and accumulates
// dW[co][tap][ci] for every co over the block's rows; thread 27*CIN sums the
// bias gradient.  No barrier: the spare threads of the last wavefront leave.
template <int CIN, int COUT>
__global__ __launch_bounds__(448) void k_wgrad(WgArgs a) {
    constexpr int NW = kTaps * CIN;
    constexpr int STRIDE = COUT * NW + COUT;
    const int tid = threadIdx.x;
    if (tid > NW) return;
    const int tap = tid / CIN, ci = tid % CIN;
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    float acc[COUT];
#pragma unroll
    for (int c = 0; c < COUT; ++c) acc[c] = 0.0f;
    const long long rows = (long long)ny * nz;
    const long long r0 = (long long)blockIdx.x * a.rows_per_block;
    const long long r1 = r0 + a.rows_per_block < rows ? r0 + a.rows_per_block : rows;
    for (long long r = r0; r < r1; ++r) {
        const int y = (int)(r % ny), z = (int)(r / ny);
        const int yy = y + dy, zz = z + dz;
        const bool rowok = tid < NW && yy >= 0 && yy < ny && zz >= 0 && zz < nz;
        const size_t hrow = ((size_t)zz * ny + yy) * nx;
        const size_t grow = ((size_t)z * ny + y) * nx;
        for (int x = 0; x < nx; ++x) {
            float hv;
            if (tid == NW) {
                hv = 1.0f;
            } else {
                const int xx = x + dx;
                hv = (rowok && xx >= 0 && xx < nx) ? bf2f(a.h[(hrow + xx) * CIN + ci]) : 0.0f;
            }
            if constexpr (COUT == kHid) {
                const uint4 *gp = reinterpret_cast<const uint4 *>(a.g + (grow + x) * kHid);
                const uint4 q0 = gp[0], q1 = gp[1];
                const uint32_t w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    acc[2 * c] += __uint_as_float(w[c] << 16) * hv;
                    acc[2 * c + 1] += __uint_as_float(w[c] & 0xFFFF0000u) * hv;
                }
            } else {
                acc[0] += bf2f(a.g[grow + x]) * hv;
            }
        }
    }
    float *out = a.partial + (size_t)blockIdx.x * STRIDE;
    if (tid < NW) {
#pragma unroll
        for (int c = 0; c < COUT; ++c) out[c * NW + tid] = acc[c];
    } else {
#pragma unroll
        for (int c = 0; c < COUT; ++c) out[COUT * NW + c] = acc[c];
    }
}

// grad[p] = sum over the blocks of partial[b][p]: 64 outputs per workgroup,
// its four wavefronts summing every fourth block, combined in a fixed order.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *__restrict__ partial, int blocks,
                                                      int stride, float *__restrict__ grad) {
    __shared__ double sh[4][64];
    const int seg = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int p = blockIdx.x * 64 + l;
    double s = 0.0;
    if (p < stride) {
#pragma unroll 8
        for (int b = seg; b < blocks; b += 4) s += partial[(size_t)b * stride + p];
    }
    sh[seg][l] = s;
    __syncthreads();
    if (seg == 0 && p < stride) grad[p] = (float)(((sh[0][l] + sh[1][l]) + sh[2][l]) + sh[3][l]);
}

// Fixed-order block sum of 256 values in LDS; the result is valid in thread 0.
__device__ inline double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    return sh[0];
}

// Partial sums of log10(kappa) per block; flags kappa that is not finite > 0.
__global__ __launch_bounds__(256) void k_cnn_logsum(const double *__restrict__ kappa, long long n,
                                                    double *__restrict__ partial,
                                                    int *__restrict__ bad) {
    __shared__ double sh[256];
    double s = 0.0;
    int flag = 0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (long long)gridDim.x * 256) {
        const double k = kappa[i];
        if (!(k > 0.0) || !isfinite(k)) flag = 1;
        else s += log10(k);
    }
    if (flag) atomicOr(bad, 1);
    const double tot = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Every block re-sums the partials in the same order (so all see one mean) and
// writes the feature bf16((log10 kappa - mean) / 3).
__global__ __launch_bounds__(256) void k_cnn_feature(const double *__restrict__ kappa, long long n,
                                                     const double *__restrict__ partial, int parts,
                                                     bf16_t *__restrict__ x0) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < parts; i += 256) s += partial[i];
    const double mean = block_sum(s, sh) / (double)n;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (long long)gridDim.x * 256)
        x0[i] = f2bf((float)((log10(kappa[i]) - mean) / kFeatureScale));
}

// Loss partials sum (t - t*)^2 and the output gradient bf16(2 (t - t*) sigmoid(y) / n).
__global__ __launch_bounds__(256) void k_cnn_loss(const float *__restrict__ y,
                                                  const double *__restrict__ target, long long n,
                                                  bf16_t *__restrict__ g,
                                                  double *__restrict__ partial) {
    __shared__ double sh[256];
    double s = 0.0;
    const double inv_n = 1.0 / (double)n;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (long long)gridDim.x * 256) {
        const float yv = y[i];
        const double d = (double)(softplusf(yv) + kEpsT) - target[i];
        s += d * d;
        const float sig = 1.0f / (1.0f + expf(-yv));
        g[i] = f2bf((float)(2.0 * d * inv_n) * sig);
    }
    const double tot = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_cnn_total(const double *__restrict__ partial, int parts,
                                                   double scale, double *__restrict__ out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < parts; i += 256) s += partial[i];
    const double tot = block_sum(s, sh);
    if (threadIdx.x == 0) out[0] = tot * scale;
}

__global__ __launch_bounds__(256) void k_cnn_adam(float *__restrict__ p, float *__restrict__ m,
                                                  float *__restrict__ v,
                                                  const float *__restrict__ g, int n, float lr,
                                                  float b1, float b2, float c1, float c2,
                                                  float eps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// ---------------------------------------------------------------- host side

#define CKH(expr)                                 \
    do {                                          \
        if ((expr) != hipSuccess) return NTD_EHIP; \
    } while (0)

struct Ws {
    bf16_t *x0, *h[3], *g4, *da, *db, *packs;
    float *y, *wpart;
    double *red, *scal;
    int *flag;
    size_t bytes;
};

size_t up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// Sizing when base is null (no pointer is formed then).
Ws carve(char *base, long long N) {
    Ws w{};
    size_t o = 0;
    auto take = [&](size_t b) {
        char *p = base ? base + o : nullptr;
        o += up(b);
        return p;
    };
    w.x0 = (bf16_t *)take((size_t)N * 2);
    for (int l = 0; l < 3; ++l) w.h[l] = (bf16_t *)take((size_t)N * kHid * 2);
    w.y = (float *)take((size_t)N * 4);
    w.g4 = (bf16_t *)take((size_t)N * 2);
    w.da = (bf16_t *)take((size_t)N * kHid * 2);
    w.db = (bf16_t *)take((size_t)N * kHid * 2);
    w.packs = (bf16_t *)take((size_t)kPackElems * 2);
    w.wpart = (float *)take((size_t)kWgMaxBlocks * (kHid * kTaps * kHid + kHid) * 4);
    w.red = (double *)take((size_t)kRedBlocks * 8);
    w.scal = (double *)take(64);
    w.flag = (int *)take(64);
    w.bytes = o;
    return w;
}

bool grid_ok(int nx, int ny, int nz) {
    return nx >= 1 && ny >= 1 && nz >= 1 && (long long)nx * ny * nz <= kMaxVoxels;
}

int red_blocks(long long N) {
    const long long b = (N + 255) / 256;
    return (int)(b < kRedBlocks ? b : kRedBlocks);
}

template <int CIN, int EPI>
hipError_t conv(const ConvArgs &a, hipStream_t s) {
    const long long rows = (long long)a.ny * a.nz;
    hipLaunchKernelGGL((k_conv<CIN, EPI>), dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Packs the weights, checks kappa and writes the feature; runs the forward
// pass into w (y always, t when t != null).
int forward(int nx, int ny, int nz, const double *kappa, const float *params, double *t,
            const Ws &w, hipStream_t s) {
    const long long N = (long long)nx * ny * nz;
    const int rb = red_blocks(N);
    hipLaunchKernelGGL(k_cnn_pack, dim3((kPackMaxJob + 255) / 256, 7), dim3(256), 0, s, params,
                       w.packs);
    CKH(hipGetLastError());
    CKH(hipMemsetAsync(w.flag, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_cnn_logsum, dim3(rb), dim3(256), 0, s, kappa, N, w.red, w.flag);
    CKH(hipGetLastError());
    int bad = 0;
    CKH(hipMemcpyAsync(&bad, w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    CKH(hipStreamSynchronize(s));
    if (bad) return NTD_EINVAL;
    hipLaunchKernelGGL(k_cnn_feature, dim3(rb), dim3(256), 0, s, kappa, N, w.red, rb, w.x0);
    CKH(hipGetLastError());
    ConvArgs a{};
    a.nx = nx, a.ny = ny, a.nz = nz;
    const bf16_t *in = w.x0;
    for (int l = 0; l < 3; ++l) {
        a.in = in;
        a.wp = w.packs + pack_off(l);
        a.bias = params + layer_desc(l).boff;
        a.out = w.h[l];
        CKH((l == 0 ? conv<1, kEpiRelu>(a, s) : conv<kHid, kEpiRelu>(a, s)));
        in = w.h[l];
    }
    a.in = in;
    a.wp = w.packs + pack_off(3);
    a.bias = params + layer_desc(3).boff;
    a.out = nullptr;
    a.y = w.y;
    a.t = t;
    CKH((conv<kHid, kEpiFinal>(a, s)));
    return NTD_OK;
}

template <int CIN, int COUT>
hipError_t wgrad(int nx, int ny, int nz, const bf16_t *h, const bf16_t *g, float *part,
                 float *grad, hipStream_t s) {
    const long long rows = (long long)ny * nz;
    const int rpb = (int)((rows + kWgMaxBlocks - 1) / kWgMaxBlocks);
    const int blocks = (int)((rows + rpb - 1) / rpb);
    constexpr int threads = ((kTaps * CIN + 1 + 63) / 64) * 64;
    constexpr int stride = COUT * kTaps * CIN + COUT;
    WgArgs a{h, g, part, nx, ny, nz, rpb};
    hipLaunchKernelGGL((k_wgrad<CIN, COUT>), dim3(blocks), dim3(threads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((stride + 63) / 64), dim3(256), 0, s, part, blocks,
                       stride, grad);
    return hipGetLastError();
}

}  // namespace

extern "C" {

size_t ntd_cnn_workspace_bytes(int nx, int ny, int nz) {
    if (!grid_ok(nx, ny, nz)) return 0;
    return carve(nullptr, (long long)nx * ny * nz).bytes;
}

int ntd_cnn_predict(int nx, int ny, int nz, const double *kappa, const float *params, double *t,
                    float *y, void *workspace, size_t ws_bytes, void *stream) {
    if (!grid_ok(nx, ny, nz) || !kappa || !params || !t || !workspace) return NTD_EINVAL;
    const long long N = (long long)nx * ny * nz;
    const Ws w = carve((char *)workspace, N);
    if (ws_bytes < w.bytes || ((uintptr_t)workspace % kAlign) != 0) return NTD_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int st = forward(nx, ny, nz, kappa, params, t, w, s);
    if (st != NTD_OK) return st;
    if (y) CKH(hipMemcpyAsync(y, w.y, (size_t)N * 4, hipMemcpyDeviceToDevice, s));
    return NTD_OK;
}

int ntd_cnn_loss_grad(int nx, int ny, int nz, const double *kappa, const double *target,
                      const float *params, float *grad, double *loss, void *workspace,
                      size_t ws_bytes, void *stream) {
    if (!grid_ok(nx, ny, nz) || !kappa || !target || !params || !grad || !loss || !workspace)
        return NTD_EINVAL;
    const long long N = (long long)nx * ny * nz;
    const Ws w = carve((char *)workspace, N);
    if (ws_bytes < w.bytes || ((uintptr_t)workspace % kAlign) != 0) return NTD_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int st = forward(nx, ny, nz, kappa, params, nullptr, w, s);
    if (st != NTD_OK) return st;
    const int rb = red_blocks(N);
    hipLaunchKernelGGL(k_cnn_loss, dim3(rb), dim3(256), 0, s, w.y, target, N, w.g4, w.red);
    CKH(hipGetLastError());
    hipLaunchKernelGGL(k_cnn_total, dim3(1), dim3(256), 0, s, w.red, rb, 1.0 / (double)N, w.scal);
    CKH(hipGetLastError());
    // layer 3 (16 -> 1): its input H3, its output gradient g4
    CKH((wgrad<kHid, 1>(nx, ny, nz, w.h[2], w.g4, w.wpart, grad + layer_desc(3).woff, s)));
    ConvArgs a{};
    a.nx = nx, a.ny = ny, a.nz = nz;
    a.in = w.g4;
    a.wp = w.packs + pack_off(6);
    a.mask = w.h[2];
    a.out = w.da;
    CKH((conv<1, kEpiMask>(a, s)));  // dZ of layer 2
    // layer 2: input H2, output gradient da
    CKH((wgrad<kHid, kHid>(nx, ny, nz, w.h[1], w.da, w.wpart, grad + layer_desc(2).woff, s)));
    a.in = w.da;
    a.wp = w.packs + pack_off(5);
    a.mask = w.h[1];
    a.out = w.db;
    CKH((conv<kHid, kEpiMask>(a, s)));  // dZ of layer 1
    CKH((wgrad<kHid, kHid>(nx, ny, nz, w.h[0], w.db, w.wpart, grad + layer_desc(1).woff, s)));
    a.in = w.db;
    a.wp = w.packs + pack_off(4);
    a.mask = w.h[0];
    a.out = w.da;
    CKH((conv<kHid, kEpiMask>(a, s)));  // dZ of layer 0
    CKH((wgrad<1, kHid>(nx, ny, nz, w.x0, w.da, w.wpart, grad + layer_desc(0).woff, s)));
    CKH(hipMemcpyAsync(loss, w.scal, sizeof(double), hipMemcpyDeviceToHost, s));
    CKH(hipStreamSynchronize(s));
    return NTD_OK;
}

int ntd_cnn_adam(float *params, float *m, float *v, const float *grad, int step, float lr,
                 void *stream) {
    if (!params || !m || !v || !grad || step < 1 || !(lr > 0.0f) || !isfinite(lr))
        return NTD_EINVAL;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - pow(b1, step)));
    const float c2 = (float)(1.0 / (1.0 - pow(b2, step)));
    hipLaunchKernelGGL(k_cnn_adam, dim3((NTD_CNN_NPARAMS + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, params, m, v, grad, NTD_CNN_NPARAMS, lr, (float)b1,
                       (float)b2, c1, c2, 1.0e-8f);
    CKH(hipGetLastError());
    return NTD_OK;
}

}  // extern "C"
