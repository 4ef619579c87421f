// ntd_batch_api.hip -- host side of the batched solve declared in include/ntd.h:
// the layout of a batch in the caller's workspace, its argument tables in
// device memory, the batched apply and the batched PCG driver.
//
// A batch holds one lean handle per system (bands, factors and line records,
// all packed with the batch's elements per lane) and, per entry (system s,
// right-hand side q), the PCG vectors, the packed right-hand side and result,
// the plane scratch of the upper sweep, the reduction partials and the scalars.
// Three tables in device memory describe the entries to the batched kernels:
// the sweep arguments, the pack/unpack arguments of the PCG, and the CG
// vectors.  The caller's vectors enter through a fourth table (batched apply)
// or through the CG table (PCG), uploaded at each call.
//
// The PCG loop runs kIterChunk iterations between host checks.  Each entry
// stops on its own (its active flag); the host only reads the flags after a
// chunk, and when every entry has stopped it confirms the true residuals and
// resumes the entries that do not meet the tolerance.  With NTD_BATCH_GRAPH the
// chunk is captured once per batch as a HIP graph on a private stream (the
// kernels read every call-dependent value from device memory, so the same graph
// serves every call) and replayed; without it the same launches are issued one
// by one.  The graph holds kernel launches only.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "ntd.h"
#include "ntd_handle.h"

namespace {

constexpr int kIterChunk = 8;
constexpr int kMaxGx = 512;

using ntd_host::Carver;

}  // namespace

struct ntd_batch {
    int count = 0, nrhs = 0, prec = 0, epl = 0, gx = 0, gx_max = 0, D = 0;
    int nr = 1;  // right-hand sides per wavefront pair in the line sweeps
    // LDS plane buffers of the line sweeps: wanted (the default), and for
    // nr = 1, 2, 4 the dynamic LDS per workgroup when the device holds every
    // workgroup of a sweep at once with its nr buffers (else 0: planes go
    // through memory)
    int lds_want = 1;
    size_t plane_lds[3] = {0, 0, 0};
    size_t used = 0;
    std::vector<ntd_handle *> sys;
    // device tables
    void *tabA = nullptr;       // ApplyArgs<T>[D]
    void *tabXp = nullptr;      // XferArgs<T>[D]: r -> rp, Z -> z with r.z partials
    void *tabXu = nullptr;      // XferArgs<T>[D]: the caller's r and z (batched apply)
    ntd::BatchVec *tabV = nullptr;
    ntd::BatchCtl *ctl = nullptr;
    int *active = nullptr;
    // host mirrors of the tables written per call
    std::vector<ntd::BatchVec> hV;
    std::vector<char> hXu;
    std::vector<int> hact;
    std::vector<ntd::BatchCtl> hctl;
    std::vector<const double *> last_r;
    std::vector<double *> last_z;
    // captured chunk of PCG iterations
    hipStream_t gs = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // statistics of the last solve: host checks of the active flags, and the
    // time the GPU spent between the end of a run of iterations and the start
    // of the next (the host's read and decision in between)
    hipEvent_t ev_gap[4] = {nullptr, nullptr, nullptr, nullptr};  // gap start, end; solve start, end
    int passes = 0;
    double gap_ms = 0.0, solve_ms = 0.0;
};

namespace {

#define CK(expr)                                   \
    do {                                           \
        if ((expr) != hipSuccess) return NTD_EHIP; \
    } while (0)

inline hipStream_t S(void *s) { return (hipStream_t)s; }

int batch_epl(int count, const int *dims) {
    int epl = 0;
    for (int s = 0; s < count; ++s) {
        const int e = ntd::epl_for(dims[3 * s]);
        if (e > epl) epl = e;
    }
    return epl;
}

long long points(const int *dims, int s) {
    return (long long)dims[3 * s] * dims[3 * s + 1] * dims[3 * s + 2];
}

int gx_for(int count, const int *dims) {
    long long nmax = 1;
    for (int s = 0; s < count; ++s)
        if (points(dims, s) > nmax) nmax = points(dims, s);
    long long g = (nmax + 4LL * ntd::kBlock - 1) / (4LL * ntd::kBlock);
    if (g < 1) g = 1;
    if (g > kMaxGx) g = kMaxGx;
    return (int)g;
}

bool args_ok(int count, const int *dims, int nrhs, int prec) {
    if (count < 1 || count > NTD_BATCH_MAX_SYSTEMS || !dims) return false;
    if (nrhs < 1 || nrhs > NTD_BATCH_MAX_RHS) return false;
    if (prec != NTD_PREC_FP64 && prec != NTD_PREC_MIXED) return false;
    for (int s = 0; s < count; ++s) {
        const int nx = dims[3 * s], ny = dims[3 * s + 1], nz = dims[3 * s + 2];
        if (nx < 1 || ny < 1 || nz < 1 || nx > NTD_BATCH_MAX_NX) return false;
    }
    const int epl = batch_epl(count, dims);
    for (int s = 0; s < count; ++s)
        if (!ntd_host::grid_ok(dims[3 * s], dims[3 * s + 1], dims[3 * s + 2], epl)) return false;
    return true;
}

// Per-entry device arrays of the batch, in carving order.
struct EntryArrays {
    double *r, *z, *p, *q;
    void *rp, *pZ, *scratch;
    double *partials;
    ntd::Scalars *sc;
};

// Walks the batch workspace: the lean handles' regions, the entry arrays, the
// tables.  Sizing when base is null.
struct BatchWalk {
    size_t off_sys[NTD_BATCH_MAX_SYSTEMS];
    size_t sys_bytes[NTD_BATCH_MAX_SYSTEMS];
    std::vector<EntryArrays> ent;
    void *tabA, *tabXp, *tabXu;
    ntd::BatchVec *tabV;
    ntd::BatchCtl *ctl;
    int *active;
    ntd::SetupArgs *tabS;  // factorization arguments of the systems
};

size_t batch_walk(BatchWalk &w, void *ws, int count, const int *dims, int nrhs, int prec) {
    const int epl = batch_epl(count, dims);
    const int gx = gx_for(count, dims);
    const size_t tsz = prec == NTD_PREC_MIXED ? sizeof(float) : sizeof(double);
    const int D = count * nrhs;
    Carver c(ws);
    for (int s = 0; s < count; ++s) {
        const size_t hb = ntd_host::handle_bytes(dims[3 * s], dims[3 * s + 1], dims[3 * s + 2],
                                                 prec, NTD_SMOOTHER_NONE, epl, true);
        w.off_sys[s] = c.off;
        w.sys_bytes[s] = hb;
        c.take<char>(hb);
    }
    w.ent.resize(D);
    for (int s = 0; s < count; ++s) {
        const long long N = points(dims, s);
        const long long ny = dims[3 * s + 1], nz = dims[3 * s + 2];
        const long long npack = ny * nz * 64 * epl;
        for (int q = 0; q < nrhs; ++q) {
            EntryArrays &e = w.ent[s * nrhs + q];
            e.r = c.take<double>(N);
            e.z = c.take<double>(N);
            e.p = c.take<double>(N);
            e.q = c.take<double>(N);
            e.rp = (void *)c.take<char>(npack * tsz);
            e.pZ = (void *)c.take<char>(npack * tsz);
            e.scratch = (void *)c.take<char>(2 * ny * 64 * epl * tsz);
            e.partials = c.take<double>(gx);
            e.sc = c.take<ntd::Scalars>(1);
        }
    }
    const size_t xsz = prec == NTD_PREC_MIXED ? sizeof(ntd::XferArgs<float>)
                                              : sizeof(ntd::XferArgs<double>);
    const size_t asz = prec == NTD_PREC_MIXED ? sizeof(ntd::ApplyArgs<float>)
                                              : sizeof(ntd::ApplyArgs<double>);
    w.tabA = (void *)c.take<char>(D * asz);
    w.tabXp = (void *)c.take<char>(D * xsz);
    w.tabXu = (void *)c.take<char>(D * xsz);
    w.tabV = c.take<ntd::BatchVec>(D);
    w.ctl = c.take<ntd::BatchCtl>(D);
    w.active = c.take<int>(D);
    w.tabS = c.take<ntd::SetupArgs>(count);
    return c.off;
}

template <typename T>
hipError_t upload_static_tables(ntd_batch *b, const BatchWalk &w, hipStream_t s) {
    const int D = b->D;
    std::vector<ntd::ApplyArgs<T>> A(D);
    std::vector<ntd::XferArgs<T>> X(D);
    for (int e = 0; e < D; ++e) {
        const ntd_handle *h = b->sys[e / b->nrhs];
        const EntryArrays &E = w.ent[e];
        A[e] = ntd_host::apply_args<T>(h);
        A[e].rp = (const T *)E.rp;
        A[e].Z = (T *)E.pZ;
        A[e].scratch = (T *)E.scratch;
        X[e] = ntd_host::xfer_args<T>(h);
        X[e].rp = (T *)E.rp;
        X[e].Z = (const T *)E.pZ;
        X[e].r = E.r;
        X[e].zout = E.z;
        X[e].partials = E.partials;
        ntd::BatchVec &V = b->hV[e];
        V.nx = h->nx; V.ny = h->ny; V.nz = h->nz; V.pad = 0;
        V.d = h->d; V.ax = h->ax; V.ay = h->ay; V.az = h->az;
        V.b = nullptr; V.x = nullptr;
        V.r = E.r; V.z = E.z; V.p = E.p; V.q = E.q;
        V.partials = E.partials;
        V.sc = E.sc;
    }
    hipError_t err;
    if ((err = hipMemcpyAsync(b->tabA, A.data(), D * sizeof(A[0]), hipMemcpyHostToDevice, s)))
        return err;
    if ((err = hipMemcpyAsync(b->tabXp, X.data(), D * sizeof(X[0]), hipMemcpyHostToDevice, s)))
        return err;
    // the caller's table starts as a copy; its r, zout are set per call
    b->hXu.assign((const char *)X.data(), (const char *)X.data() + D * sizeof(X[0]));
    return hipStreamSynchronize(s);
}

// The caller's r[e], z[e] into the batched-apply table (uploaded only when
// they differ from the previous call's).
template <typename T>
hipError_t upload_user_xfer(ntd_batch *b, const double *const *r, double *const *z, hipStream_t s) {
    bool same = (int)b->last_r.size() == b->D;
    for (int e = 0; same && e < b->D; ++e) same = b->last_r[e] == r[e] && b->last_z[e] == z[e];
    if (same) return hipSuccess;
    // the previous upload from this mirror has completed before it changes
    hipError_t err = hipStreamSynchronize(s);
    if (err != hipSuccess) return err;
    ntd::XferArgs<T> *X = (ntd::XferArgs<T> *)b->hXu.data();
    for (int e = 0; e < b->D; ++e) {
        X[e].r = r[e];
        X[e].zout = z[e];
        X[e].partials = nullptr;
    }
    b->last_r.assign(r, r + b->D);
    b->last_z.assign(z, z + b->D);
    return hipMemcpyAsync(b->tabXu, b->hXu.data(), b->hXu.size(), hipMemcpyHostToDevice, s);
}

hipError_t pack_b(const ntd_batch *b, const void *tab, const int *act, hipStream_t s) {
    if (b->prec == NTD_PREC_FP64)
        return ntd::launch_pack_rhs_batch_f64((const ntd::XferArgs<double> *)tab, act, b->D, b->gx,
                                              b->epl, s);
    return ntd::launch_pack_rhs_batch_f32((const ntd::XferArgs<float> *)tab, act, b->D, b->gx,
                                          b->epl, s);
}
int nr_index(int nr) { return nr == 1 ? 0 : nr == 2 ? 1 : 2; }

size_t sweep_lds(const ntd_batch *b) { return b->lds_want ? b->plane_lds[nr_index(b->nr)] : 0; }

hipError_t sweeps_b(const ntd_batch *b, const int *act, hipStream_t s, hipEvent_t *ev) {
    if (b->prec == NTD_PREC_FP64) {
        const auto *tab = (const ntd::ApplyArgs<double> *)b->tabA;
        if (b->nr > 1)
            return ntd::launch_apply_batch_multi_f64(tab, act, b->count, b->nrhs, b->epl, b->nr,
                                                     sweep_lds(b), s, ev);
        return ntd::launch_apply_batch_f64(tab, act, b->count, b->nrhs, b->epl, sweep_lds(b), s,
                                           ev);
    }
    const auto *tab = (const ntd::ApplyArgs<float> *)b->tabA;
    if (b->nr > 1)
        return ntd::launch_apply_batch_multi_f32(tab, act, b->count, b->nrhs, b->epl, b->nr,
                                                 sweep_lds(b), s, ev);
    return ntd::launch_apply_batch_f32(tab, act, b->count, b->nrhs, b->epl, sweep_lds(b), s, ev);
}

// Dynamic LDS per workgroup for the LDS-plane sweeps of the batch with nr
// right-hand sides per wavefront pair, or 0 when the device cannot hold every
// workgroup of a sweep at once with its nr plane buffers: the sweeps are a
// latency-bound chain per workgroup, and workgroups waiting for a free CU would
// double the launch.
size_t plane_lds_fit(int count, const int *dims, int nrhs, int prec, int epl, int nr) {
    int ny_max = 1;
    for (int s = 0; s < count; ++s)
        if (dims[3 * s + 1] > ny_max) ny_max = dims[3 * s + 1];
    const size_t tsz = prec == NTD_PREC_MIXED ? sizeof(float) : sizeof(double);
    const size_t bytes = (size_t)nr * ntd::plane_lds_bytes(ny_max, epl, tsz);
    int dev = 0, per_block = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess ||
        hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (bytes > (size_t)per_block || per_cu <= 0 || cus <= 0) return 0;
    const long long per = (long long)((size_t)per_cu / bytes);  // workgroups per CU
    const long long wgs = 2LL * count * (nrhs / nr);            // two level-3 halves each
    if (per * cus < wgs) return 0;
    // The limit belongs to the kernel, not to this batch: allow the device's
    // maximum, so that a later batch with smaller planes cannot lower it below
    // what an earlier one launches with.
    hipError_t e;
    if (nr == 1)
        e = prec == NTD_PREC_MIXED ? ntd::allow_apply_batch_lds_f32(epl, (size_t)per_block)
                                   : ntd::allow_apply_batch_lds_f64(epl, (size_t)per_block);
    else
        e = prec == NTD_PREC_MIXED
                ? ntd::allow_apply_batch_multi_lds_f32(epl, nr, (size_t)per_block)
                : ntd::allow_apply_batch_multi_lds_f64(epl, nr, (size_t)per_block);
    return e == hipSuccess ? bytes : 0;
}

// Can the batch's sweeps run nr right-hand sides per wavefront pair?
bool nr_ok(const ntd_batch *b, int nr) {
    if (nr == 1) return true;
    if (nr != 2 && nr != 4) return false;
    if (b->nrhs % nr != 0) return false;
    return ntd::batch_multi_ok(b->prec == NTD_PREC_FP64 ? 8 : 4, b->epl, nr);
}

void drop_graph(ntd_batch *b) {
    if (b->gexec) {  // captured with the old launch shape
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
}
hipError_t unpack_b(const ntd_batch *b, const void *tab, const int *act, hipStream_t s) {
    if (b->prec == NTD_PREC_FP64)
        return ntd::launch_unpack_batch_f64((const ntd::XferArgs<double> *)tab, act, b->D, b->gx,
                                            b->epl, s);
    return ntd::launch_unpack_batch_f32((const ntd::XferArgs<float> *)tab, act, b->D, b->gx,
                                        b->epl, s);
}

int fin(ntd_batch *b, int op, double tol, int maxit, hipStream_t s) {
    CK(ntd::launch_batch_finalize(b->tabV, b->ctl, b->active, b->D, b->gx, op, tol, maxit, s));
    return NTD_OK;
}

// z = B^{-1} r for the active entries, with the r.z partials.
int precond_b(ntd_batch *b, hipStream_t s) {
    CK(pack_b(b, b->tabXp, b->active, s));
    CK(sweeps_b(b, b->active, s, nullptr));
    CK(unpack_b(b, b->tabXp, b->active, s));
    return NTD_OK;
}

// One PCG iteration of every active entry.
int iterate(ntd_batch *b, hipStream_t s) {
    int st;
    CK(ntd::launch_batch_spmv(b->tabV, b->active, b->D, b->gx, 0, s));
    if ((st = fin(b, ntd::kOpAlpha, 0.0, 0, s)) != NTD_OK) return st;
    CK(ntd::launch_batch_axpy2(b->tabV, b->active, b->D, b->gx, s));
    if ((st = fin(b, ntd::kOpRR, 0.0, 0, s)) != NTD_OK) return st;
    if ((st = precond_b(b, s)) != NTD_OK) return st;
    if ((st = fin(b, ntd::kOpBeta, 0.0, 0, s)) != NTD_OK) return st;
    CK(ntd::launch_batch_xpay(b->tabV, b->active, b->D, b->gx, false, s));
    return NTD_OK;
}

int ensure_graph(ntd_batch *b) {
    if (b->gexec) return NTD_OK;
    if (!b->gs) CK(hipStreamCreateWithFlags(&b->gs, hipStreamNonBlocking));
    if (!b->ev_in) CK(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    if (!b->ev_out) CK(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    CK(hipStreamBeginCapture(b->gs, hipStreamCaptureModeThreadLocal));
    int st = NTD_OK;
    for (int k = 0; k < kIterChunk && st == NTD_OK; ++k) st = iterate(b, b->gs);
    hipGraph_t g = nullptr;
    const hipError_t end = hipStreamEndCapture(b->gs, &g);
    if (st != NTD_OK || end != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return st != NTD_OK ? st : NTD_EHIP;
    }
    const hipError_t inst = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (inst != hipSuccess) {
        b->gexec = nullptr;
        return NTD_EHIP;
    }
    return NTD_OK;
}

// kIterChunk iterations on stream s (graph replay on the private stream,
// ordered after and before the work of s).
int run_chunk(ntd_batch *b, bool graph, hipStream_t s) {
    if (!graph) {
        for (int k = 0; k < kIterChunk; ++k) {
            const int st = iterate(b, s);
            if (st != NTD_OK) return st;
        }
        return NTD_OK;
    }
    const int st = ensure_graph(b);
    if (st != NTD_OK) return st;
    CK(hipEventRecord(b->ev_in, s));
    CK(hipStreamWaitEvent(b->gs, b->ev_in, 0));
    CK(hipGraphLaunch(b->gexec, b->gs));
    CK(hipEventRecord(b->ev_out, b->gs));
    CK(hipStreamWaitEvent(s, b->ev_out, 0));
    return NTD_OK;
}

int any_active(ntd_batch *b, hipStream_t s, bool *any) {
    CK(hipMemcpyAsync(b->hact.data(), b->active, b->D * sizeof(int), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    *any = false;
    for (int e = 0; e < b->D; ++e) *any = *any || b->hact[e] != 0;
    return NTD_OK;
}

void release(ntd_batch *b) {
    if (!b) return;
    for (hipEvent_t e : b->ev_gap)
        if (e) (void)hipEventDestroy(e);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->gs) (void)hipStreamDestroy(b->gs);
    for (ntd_handle *h : b->sys) ntd_destroy(h);
    delete b;
}

}  // namespace

extern "C" {

size_t ntd_batch_workspace_bytes(int count, const int *dims, int nrhs, int prec) {
    if (!args_ok(count, dims, nrhs, prec)) return 0;
    BatchWalk *w = new (std::nothrow) BatchWalk;
    if (!w) return 0;
    const size_t bytes = batch_walk(*w, nullptr, count, dims, nrhs, prec);
    delete w;
    return bytes;
}

int ntd_batch_setup(int count, const int *dims, const double *const *kappa, const int *bc,
                    int nrhs, int prec, int schur, void *workspace, size_t workspace_bytes,
                    void *stream, ntd_batch **out) {
    if (out) *out = nullptr;
    if (!out || !kappa || !bc || !workspace) return NTD_EINVAL;
    if (!args_ok(count, dims, nrhs, prec)) return NTD_EINVAL;
    if (schur != NTD_SCHUR_NEWTON && schur != NTD_SCHUR_DIAG) return NTD_EINVAL;
    if (((uintptr_t)workspace) % ntd_host::kAlign) return NTD_EINVAL;
    for (int s = 0; s < count; ++s)
        if (!kappa[s]) return NTD_EINVAL;
    BatchWalk *w = new (std::nothrow) BatchWalk;
    if (!w) return NTD_ENOMEM;
    const size_t need = batch_walk(*w, workspace, count, dims, nrhs, prec);
    if (workspace_bytes < need) {
        delete w;
        return NTD_EINVAL;
    }
    ntd_batch *b = new (std::nothrow) ntd_batch;
    if (!b) {
        delete w;
        return NTD_ENOMEM;
    }
    hipStream_t s = S(stream);
    b->count = count;
    b->nrhs = nrhs;
    b->prec = prec;
    b->epl = batch_epl(count, dims);
    b->gx = gx_for(count, dims);
    b->gx_max = b->gx;  // the entries' partials hold this many blocks
    b->D = count * nrhs;
    b->used = need;
    b->tabA = w->tabA;
    b->tabXp = w->tabXp;
    b->tabXu = w->tabXu;
    b->tabV = w->tabV;
    b->ctl = w->ctl;
    b->active = w->active;
    b->hV.resize(b->D);
    b->hact.resize(b->D);
    b->hctl.resize(b->D);
    // The setups of the systems, phase by phase over the whole batch: every
    // factorization runs in one pair of launches.
    int st = NTD_OK;
    for (int sy = 0; sy < count && st == NTD_OK; ++sy) {
        ntd_handle *h = nullptr;
        st = ntd_host::handle_create(dims[3 * sy], dims[3 * sy + 1], dims[3 * sy + 2],
                                     bc + 6 * sy, prec, schur, NTD_SMOOTHER_NONE, b->epl, true,
                                     (char *)workspace + w->off_sys[sy], w->sys_bytes[sy], &h);
        if (st == NTD_OK) b->sys.push_back(h);
    }
    std::vector<int> flags(count, 0);
    auto read_flags = [&](int mask, int code) {
        for (int sy = 0; sy < count && st == NTD_OK; ++sy)
            st = ntd_host::handle_flag_async(b->sys[sy], &flags[sy], s);
        if (st == NTD_OK && hipStreamSynchronize(s) != hipSuccess) st = NTD_EHIP;
        for (int sy = 0; sy < count && st == NTD_OK; ++sy)
            if (flags[sy] & mask) st = code;
    };
    for (int sy = 0; sy < count && st == NTD_OK; ++sy)
        st = ntd_host::handle_check(b->sys[sy], kappa[sy], nullptr, s);
    if (st == NTD_OK) read_flags(ntd::kFlagBadInput, NTD_EINVAL);
    for (int sy = 0; sy < count && st == NTD_OK; ++sy)
        st = ntd_host::handle_assemble(b->sys[sy], kappa[sy], bc + 6 * sy, s);
    if (st == NTD_OK) {
        std::vector<ntd::SetupArgs> args(count);
        int max_nx = 1;
        for (int sy = 0; sy < count; ++sy) {
            args[sy] = ntd_host::handle_setup_args(b->sys[sy], nullptr);
            if (dims[3 * sy] > max_nx) max_nx = dims[3 * sy];
        }
        if (hipMemcpyAsync(w->tabS, args.data(), count * sizeof(ntd::SetupArgs),
                           hipMemcpyHostToDevice, s) != hipSuccess ||
            ntd::launch_setup_batch(w->tabS, count, max_nx, b->epl, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = NTD_EHIP;
    }
    if (st == NTD_OK) read_flags(ntd::kFlagNotSPD, NTD_ENOTSPD);
    for (int sy = 0; sy < count && st == NTD_OK; ++sy)
        st = ntd_host::handle_finish(b->sys[sy], s);
    if (st == NTD_OK) {
        // unused slots of the packed right-hand sides must read as 0
        const size_t tsz = prec == NTD_PREC_MIXED ? sizeof(float) : sizeof(double);
        for (int e = 0; e < b->D && st == NTD_OK; ++e) {
            const ntd_handle *h = b->sys[e / nrhs];
            if (ntd::launch_fill((double *)w->ent[e].rp, 0.0, h->npack * tsz / 8, s) != hipSuccess)
                st = NTD_EHIP;
        }
    }
    if (st == NTD_OK) {
        const hipError_t err = prec == NTD_PREC_MIXED ? upload_static_tables<float>(b, *w, s)
                                                      : upload_static_tables<double>(b, *w, s);
        if (err != hipSuccess) st = NTD_EHIP;
    }
    for (int nr : {1, 2, 4})
        if (st == NTD_OK && nr_ok(b, nr))
            b->plane_lds[nr_index(nr)] = plane_lds_fit(count, dims, nrhs, prec, b->epl, nr);
    delete w;
    if (st != NTD_OK) {
        release(b);
        return st;
    }
    *out = b;
    return NTD_OK;
}

int ntd_batch_apply(ntd_batch *b, const double *const *r, double *const *z, void *stream) {
    if (!b || !r || !z) return NTD_EINVAL;
    for (int e = 0; e < b->D; ++e)
        if (!r[e] || !z[e] || r[e] == z[e]) return NTD_EINVAL;
    hipStream_t s = S(stream);
    CK(b->prec == NTD_PREC_MIXED ? upload_user_xfer<float>(b, r, z, s)
                                 : upload_user_xfer<double>(b, r, z, s));
    CK(pack_b(b, b->tabXu, nullptr, s));
    CK(sweeps_b(b, nullptr, s, nullptr));
    CK(unpack_b(b, b->tabXu, nullptr, s));
    return NTD_OK;
}

int ntd_batch_apply_profile(ntd_batch *b, const double *const *r, double *const *z, float *ms,
                            void *stream) {
    if (!b || !r || !z || !ms) return NTD_EINVAL;
    for (int e = 0; e < b->D; ++e)
        if (!r[e] || !z[e] || r[e] == z[e]) return NTD_EINVAL;
    hipStream_t s = S(stream);
    CK(b->prec == NTD_PREC_MIXED ? upload_user_xfer<float>(b, r, z, s)
                                 : upload_user_xfer<double>(b, r, z, s));
    hipEvent_t ev[6];
    int made = 0, st = NTD_OK;
    for (; made < 6; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess) { st = NTD_EHIP; break; }
    if (st == NTD_OK) {
        if (hipEventRecord(ev[0], s) != hipSuccess || pack_b(b, b->tabXu, nullptr, s) != hipSuccess ||
            sweeps_b(b, nullptr, s, ev + 1) != hipSuccess ||
            unpack_b(b, b->tabXu, nullptr, s) != hipSuccess || hipEventRecord(ev[5], s) != hipSuccess ||
            hipEventSynchronize(ev[5]) != hipSuccess)
            st = NTD_EHIP;
    }
    float pre = 0.0f, post = 0.0f;
    for (int i = 0; st == NTD_OK && i < 3; ++i)
        if (hipEventElapsedTime(&ms[i], ev[i + 1], ev[i + 2]) != hipSuccess) st = NTD_EHIP;
    if (st == NTD_OK && (hipEventElapsedTime(&pre, ev[0], ev[1]) != hipSuccess ||
                         hipEventElapsedTime(&post, ev[4], ev[5]) != hipSuccess))
        st = NTD_EHIP;
    if (st == NTD_OK) ms[3] = pre + post;
    for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    return st;
}

int ntd_batch_pcg_solve(ntd_batch *b, const double *const *rhs, double *const *x, double tol,
                        int maxit, int flags, int *iters, double *relres, int *status,
                        void *stream) {
    if (!b || !rhs || !x || !iters || !relres || !status) return NTD_EINVAL;
    if (!(tol > 0.0) || maxit < 1 || (flags & ~NTD_BATCH_GRAPH)) return NTD_EINVAL;
    for (int e = 0; e < b->D; ++e)
        if (!rhs[e] || !x[e] || rhs[e] == x[e]) return NTD_EINVAL;
    hipStream_t s = S(stream);
    const bool graph = (flags & NTD_BATCH_GRAPH) != 0;
    for (int e = 0; e < b->D; ++e) {
        b->hV[e].b = rhs[e];
        b->hV[e].x = x[e];
    }
    CK(hipMemcpyAsync(b->tabV, b->hV.data(), b->D * sizeof(ntd::BatchVec), hipMemcpyHostToDevice,
                      s));
    int st;
    CK(ntd::launch_batch_init(b->tabV, b->D, b->gx, s));
    if ((st = fin(b, ntd::kBOpInit, tol, maxit, s)) != NTD_OK) return st;
    if ((st = precond_b(b, s)) != NTD_OK) return st;
    if ((st = fin(b, ntd::kOpRhoInit, 0.0, 0, s)) != NTD_OK) return st;
    CK(ntd::launch_batch_xpay(b->tabV, b->active, b->D, b->gx, true, s));
    // every pass advances some entry by at least one iteration, and no entry
    // passes maxit, so the loop ends; the bound guards against a logic error
    const long long max_pass = (long long)b->D * maxit + 2;
    bool any = true;
    for (hipEvent_t &e : b->ev_gap)
        if (!e) CK(hipEventCreate(&e));
    b->passes = 0;
    b->gap_ms = 0.0;
    CK(hipEventRecord(b->ev_gap[2], s));  // start of the solve's iterations
    for (long long pass = 0; pass < max_pass; ++pass) {
        // the end of the previous run of iterations, then the host's check
        CK(hipEventRecord(b->ev_gap[0], s));
        if ((st = any_active(b, s, &any)) != NTD_OK) return st;
        ++b->passes;
        if (!any) {
            CK(ntd::launch_batch_spmv(b->tabV, nullptr, b->D, b->gx, 1, s));
            if ((st = fin(b, ntd::kBOpTrue, 0.0, 0, s)) != NTD_OK) return st;
            if ((st = any_active(b, s, &any)) != NTD_OK) return st;
            if (!any) break;
            // the recursive test stopped these entries right after their
            // residual update; finish that iteration (z = B^{-1} r, beta,
            // p = z + beta p) so that CG continues as the single-system solve does
            if ((st = precond_b(b, s)) != NTD_OK) return st;
            if ((st = fin(b, ntd::kOpBeta, 0.0, 0, s)) != NTD_OK) return st;
            CK(ntd::launch_batch_xpay(b->tabV, b->active, b->D, b->gx, false, s));
        }
        // the next run starts here: the gap since ev_gap[0] is the check's cost
        CK(hipEventRecord(b->ev_gap[1], s));
        if ((st = run_chunk(b, graph, s)) != NTD_OK) return st;
        float g = 0.0f;
        CK(hipEventSynchronize(b->ev_gap[1]));
        CK(hipEventElapsedTime(&g, b->ev_gap[0], b->ev_gap[1]));
        b->gap_ms += g;
    }
    if (any) return NTD_EHIP;
    {
        float ms = 0.0f;
        CK(hipEventRecord(b->ev_gap[3], s));
        CK(hipEventSynchronize(b->ev_gap[3]));
        CK(hipEventElapsedTime(&ms, b->ev_gap[2], b->ev_gap[3]));
        b->solve_ms = ms;
    }
    CK(hipMemcpyAsync(b->hctl.data(), b->ctl, b->D * sizeof(ntd::BatchCtl),
                      hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    for (int e = 0; e < b->D; ++e) {
        iters[e] = b->hctl[e].iters;
        relres[e] = b->hctl[e].relres;
        status[e] = b->hctl[e].status;
    }
    return NTD_OK;
}

int ntd_batch_tune(ntd_batch *b, int *gx_out, void *stream) {
    if (!b || !gx_out) return NTD_EINVAL;
    hipStream_t s = S(stream);
    // clean inputs for the timed kernels (every CG vector is rewritten by a solve)
    for (int e = 0; e < b->D; ++e) {
        const long long N = (long long)b->hV[e].nx * b->hV[e].ny * b->hV[e].nz;
        for (double *v : {b->hV[e].r, b->hV[e].z, b->hV[e].p, b->hV[e].q})
            CK(ntd::launch_fill(v, 0.0, N, s));
    }
    hipEvent_t ev[2];
    int made = 0, st = NTD_OK;
    for (; made < 2; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess) { st = NTD_EHIP; break; }
    // one round: the bandwidth kernels of an iteration that touch only the
    // entries' own arrays (q = A p, p = z, pack of r, unpack into z)
    auto round = [&](void) -> hipError_t {
        hipError_t e;
        if ((e = ntd::launch_batch_spmv(b->tabV, nullptr, b->D, b->gx, 0, s))) return e;
        if ((e = ntd::launch_batch_xpay(b->tabV, nullptr, b->D, b->gx, true, s))) return e;
        if ((e = pack_b(b, b->tabXp, nullptr, s))) return e;
        return unpack_b(b, b->tabXp, nullptr, s);
    };
    int best = b->gx_max;
    float best_ms = 0.0f;
    for (int k = 0, last = 0; k < 4 && st == NTD_OK; ++k) {
        const int g = (b->gx_max + (1 << k) - 1) >> k;
        if (g < 1 || g == last) break;
        last = g;
        b->gx = g;
        float ms = 0.0f;
        if (round() != hipSuccess || hipEventRecord(ev[0], s) != hipSuccess) { st = NTD_EHIP; break; }
        for (int r = 0; r < 3 && st == NTD_OK; ++r)
            if (round() != hipSuccess) st = NTD_EHIP;
        if (st != NTD_OK || hipEventRecord(ev[1], s) != hipSuccess ||
            hipEventSynchronize(ev[1]) != hipSuccess ||
            hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) {
            st = NTD_EHIP;
            break;
        }
        if (k == 0 || ms < best_ms) {
            best = g;
            best_ms = ms;
        }
    }
    for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    b->gx = best;
    drop_graph(b);
    if (st != NTD_OK) return st;
    *gx_out = best;
    return NTD_OK;
}

int ntd_batch_set_sweep_group(ntd_batch *b, int nr) {
    if (!b || !nr_ok(b, nr)) return NTD_EINVAL;
    if (b->nr != nr) drop_graph(b);
    b->nr = nr;
    return NTD_OK;
}

int ntd_batch_set_plane_lds(ntd_batch *b, int on, int *used) {
    if (!b || (on != 0 && on != 1)) return NTD_EINVAL;
    if (b->lds_want != on) drop_graph(b);
    b->lds_want = on;
    if (used) *used = sweep_lds(b) > 0 ? 1 : 0;
    return NTD_OK;
}

int ntd_batch_tune_sweeps(ntd_batch *b, int *nr_out, void *stream) {
    if (!b || !nr_out) return NTD_EINVAL;
    hipStream_t s = S(stream);
    // the sweeps read only the packed right-hand sides and write only the
    // packed results and scratch planes: start from zero right-hand sides
    for (int e = 0; e < b->D; ++e) {
        const long long N = (long long)b->hV[e].nx * b->hV[e].ny * b->hV[e].nz;
        CK(ntd::launch_fill(b->hV[e].r, 0.0, N, s));
    }
    if (pack_b(b, b->tabXp, nullptr, s) != hipSuccess) return NTD_EHIP;
    hipEvent_t ev[2];
    int made = 0, st = NTD_OK;
    for (; made < 2; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess) { st = NTD_EHIP; break; }
    const int keep = b->nr;
    int best = keep;
    float best_ms = 0.0f;
    bool first = true;
    for (int nr : {1, 2, 4}) {
        if (st != NTD_OK) break;
        if (!nr_ok(b, nr)) continue;
        b->nr = nr;
        float ms = 0.0f;
        if (sweeps_b(b, nullptr, s, nullptr) != hipSuccess ||     // warm-up
            hipEventRecord(ev[0], s) != hipSuccess || sweeps_b(b, nullptr, s, nullptr) != hipSuccess ||
            hipEventRecord(ev[1], s) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
            hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) {
            st = NTD_EHIP;
            break;
        }
        if (first || ms < best_ms) {
            best = nr;
            best_ms = ms;
            first = false;
        }
    }
    for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    b->nr = st == NTD_OK ? best : keep;
    if (b->nr != keep) drop_graph(b);
    if (st != NTD_OK) return st;
    *nr_out = best;
    return NTD_OK;
}

size_t ntd_batch_footprint_bytes(const ntd_batch *b) { return b ? b->used : 0; }

int ntd_batch_solve_stats(const ntd_batch *b, int *passes, double *gap_ms, double *solve_ms) {
    if (!b || !passes || !gap_ms || !solve_ms) return NTD_EINVAL;
    *passes = b->passes;
    *gap_ms = b->gap_ms;
    *solve_ms = b->solve_ms;
    return NTD_OK;
}

int ntd_batch_destroy(ntd_batch *b) {
    release(b);
    return NTD_OK;
}

}  // extern "C"
