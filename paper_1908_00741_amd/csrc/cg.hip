// IC(0)-preconditioned CG on gfx950 (Section 2; stopping test of Section 5.1):
// the SpMV on the sliced-ELL Abar, the inner products and vector updates, the
// permutations between numberings, and the solver loop.
//
// Reductions never communicate between workgroups inside a kernel: each
// workgroup writes one partial sum (wavefront butterfly, then across the
// waves of the workgroup), and a one-workgroup kernel adds the partials in a
// fixed order and updates the CG scalars held on the device.  Results are
// therefore deterministic, and no device-wide fence is needed.
//
// The loop keeps all scalars (rho, alpha, beta, ||r||^2) and the stop flag on
// the device, so the host only reads the state every check_every
// iterations; with use_graph the check_every iterations are captured once as
// a hipGraph and replayed.  Every kernel of an iteration returns at once when
// the flag is set, so iterations past the stopping point change nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <vector>

#include "hbmc_internal.h"

using namespace hbmc;

#define HIP_TRY(call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(HBMC_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

namespace {

constexpr int kLanes = kTileLanes;
constexpr int kBlock = 256;      // threads of the vector kernels: one element each
constexpr int kFin = 1024;       // threads of the one-workgroup finalizing kernels

// Stop flag values
enum { kRunning = 0, kConverged = 1, kBreakdown = 2, kMaxIt = 3 };

struct CgState {
    double rho, alpha, beta, sigma, rr, bb, res, tol;
    int32_t it, maxit, done, pad;
};

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup (at most 1024 threads); the result is valid in
// thread 0.
__device__ inline double block_sum(double v) {
    __shared__ double sh[16];
    v = wave_sum(v);
    const int wid = threadIdx.x >> 6, ln = threadIdx.x & 63;
    if (ln == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (wid == 0) t = wave_sum(ln < int(blockDim.x >> 6) ? sh[ln] : 0.0);
    __syncthreads();
    return t;
}

// Fixed-order total of g partial sums, computed by one workgroup of kFin
// threads; valid in thread 0.
__device__ inline double total(const double *part, int g) {
    double s = 0.0;
    for (int i = threadIdx.x; i < g; i += kFin) s += part[i];
    return block_sum(s);
}

// Abar: diagonal plus off-diagonal couplings in 64-row groups of strided
// and indexed slots (a wavefront is one group).
struct Mat {
    const double *diag;
    const int32_t *soff;
    const int32_t *sbase;
    const uint64_t *smask;
    const double *sval;
    const int32_t *ioff;
    const int32_t *icol;
    const double *ival;
    int64_t n;
};

__device__ inline uint64_t readlane64(uint64_t v, int lane) {
    const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(v), lane);
    const uint32_t hi = __builtin_amdgcn_readlane(uint32_t(v >> 32), lane);
    return (uint64_t(hi) << 32) | lo;
}

// One row of y = A x.  A wavefront is one 64-row group, so the group index
// is uniform; the group's strided-slot bases and masks (at most 64) come in
// with one vector load, one slot per lane, and are broadcast with readlane.
template <class X>
__device__ inline double spmv_row_with(const Mat &m, X x, int64_t row) {
    const int64_t g = __builtin_amdgcn_readfirstlane(int(row >> 6));
    const int lane = int(row & 63);
    double acc = m.diag[row] * x(row);
    const int32_t s0 = m.soff[g], ns = m.soff[g + 1] - s0;
    const int64_t ms = s0 + (lane < ns ? lane : 0);
    const int32_t mbase = m.sbase[ms];
    const uint64_t mmask = m.smask[ms];
#pragma unroll 4
    for (int k = 0; k < ns; ++k) {
        const int32_t base = __builtin_amdgcn_readlane(mbase, k);
        const bool on = (readlane64(mmask, k) >> lane) & 1;
        const double v = m.sval[(s0 + k) * int64_t(kLanes) + lane];
        const double xv = x(base + lane);
        acc = on ? acc + v * xv : acc;
    }
#pragma unroll 4
    for (int64_t s = m.ioff[g]; s < m.ioff[g + 1]; ++s) {
        const int64_t e = s * kLanes + lane;
        const int32_t c = m.icol[e];
        const double v = m.ival[e];
        const double xv = x(c >= 0 ? c : 0);
        acc = c >= 0 ? acc + v * xv : acc;
    }
    return acc;
}

__device__ inline double spmv_row(const Mat &m, const double *__restrict__ x, int64_t row) {
    return spmv_row_with(m, [=](int64_t i) { return x[i]; }, row);
}

// one element per thread (the grid covers n)
#define GRID_STRIDE(i, n) \
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < (n); i = (n))

__global__ void __launch_bounds__(kBlock) k_spmv(Mat m, const double *__restrict__ x,
                                                 double *__restrict__ y) {
    GRID_STRIDE(row, m.n) y[row] = spmv_row(m, x, row);
}

// r = b - q; partials of ||b||^2 and ||r||^2
__global__ void __launch_bounds__(kBlock) k_init_r(int64_t n, const double *__restrict__ b,
                                                   const double *__restrict__ q,
                                                   double *__restrict__ r, double *part) {
    double sb = 0.0, sr = 0.0;
    GRID_STRIDE(i, n) {
        const double ri = b[i] - q[i];
        r[i] = ri;
        sb += b[i] * b[i];
        sr += ri * ri;
    }
    sb = block_sum(sb);
    sr = block_sum(sr);
    if (threadIdx.x == 0) { part[blockIdx.x] = sb; part[gridDim.x + blockIdx.x] = sr; }
}

__global__ void __launch_bounds__(kFin) k_fin_init(const double *part, int g, CgState *st,
                                                     double tol, int32_t maxit, double *hist) {
    const double bb = total(part, g);
    const double rr = total(part + g, g);
    if (threadIdx.x) return;
    st->bb = bb;
    st->rr = rr;
    st->tol = tol;
    st->maxit = maxit;
    st->it = 0;
    st->res = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    if (hist) hist[0] = st->res;
    st->done = (bb == 0.0 || st->res < tol) ? kConverged : (maxit <= 0 ? kMaxIt : kRunning);
    if (!isfinite(st->res)) st->done = kBreakdown;
}

// p = z; partial of (r, z)   (beta = 0 for the first iteration)
__global__ void __launch_bounds__(kBlock) k_init_p(int64_t n, const double *__restrict__ r,
                                                   const double *__restrict__ z,
                                                   double *__restrict__ p, double *part) {
    double s = 0.0;
    GRID_STRIDE(i, n) {
        p[i] = z[i];
        s += r[i] * z[i];
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kFin) k_fin_rho(const double *part, int g, CgState *st) {
    const double t = total(part, g);
    if (threadIdx.x == 0) { st->rho = t; st->beta = 0.0; }
}

// p = z + beta p_old (formed on the fly, also at the columns the row
// couples to), written to p_new; q = A p; partial of (p, q)
__global__ void __launch_bounds__(kBlock) k_spmv_dot_p(Mat m, const double *__restrict__ z,
                                                       const double *__restrict__ p_old,
                                                       double *__restrict__ p_new,
                                                       double *__restrict__ q, double *part,
                                                       const CgState *st) {
    if (st->done) return;
    const double beta = st->beta;
    double s = 0.0;
    GRID_STRIDE(row, m.n) {
        auto pv = [=](int64_t i) { return z[i] + beta * p_old[i]; };
        const double pi = pv(row);
        const double qi = spmv_row_with(m, pv, row);
        p_new[row] = pi;
        q[row] = qi;
        s += pi * qi;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// sigma = (p, Ap); alpha = rho / sigma
__global__ void __launch_bounds__(kFin) k_fin_alpha(const double *part, int g, CgState *st) {
    if (st->done) return;
    const double sigma = total(part, g);
    if (threadIdx.x) return;
    st->sigma = sigma;
    if (!(sigma > 0.0) || !isfinite(sigma)) { st->done = kBreakdown; st->it += 1; return; }
    st->alpha = st->rho / sigma;
}

// After the preconditioning step: ||r||^2 and (r, z) from the per-tile
// partials; one more iteration done; stopping test ||r|| / ||b|| < tol;
// then beta = rho' / rho, rho = rho' for the next direction.
__global__ void __launch_bounds__(kFin) k_fin_rr_beta(const double *part_rr, const double *part_rz,
                                                      int ntiles, CgState *st, double *hist,
                                                      int32_t hist_len) {
    if (st->done) return;
    const double rr = total(part_rr, ntiles);
    const double rz = total(part_rz, ntiles);
    if (threadIdx.x) return;
    st->rr = rr;
    st->it += 1;
    st->res = sqrt(rr / st->bb);
    if (hist && st->it < hist_len) hist[st->it] = st->res;
    if (!isfinite(st->res)) st->done = kBreakdown;
    else if (st->res < st->tol) st->done = kConverged;
    else if (st->it >= st->maxit) st->done = kMaxIt;
    else {
        st->beta = rz / st->rho;
        st->rho = rz;
    }
}

// partial of ||b - q||^2 (true residual)
__global__ void __launch_bounds__(kBlock) k_resid(int64_t n, const double *__restrict__ b,
                                                  const double *__restrict__ q, double *part) {
    double s = 0.0;
    GRID_STRIDE(i, n) { const double d = b[i] - q[i]; s += d * d; }
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kFin) k_fin_resid(const double *part, int g, double *out) {
    const double t = total(part, g);
    if (threadIdx.x == 0) *out = t;
}

__global__ void __launch_bounds__(kBlock) k_to_hbmc(int64_t n_pad, const int32_t *__restrict__ iperm,
                                                    const double *__restrict__ v,
                                                    double *__restrict__ vb) {
    GRID_STRIDE(r, n_pad) { const int32_t i = iperm[r]; vb[r] = i >= 0 ? v[i] : 0.0; }
}

__global__ void __launch_bounds__(kBlock) k_from_hbmc(int64_t n, const int32_t *__restrict__ perm,
                                                      const double *__restrict__ vb,
                                                      double *__restrict__ v) {
    GRID_STRIDE(i, n) v[i] = vb[perm[i]];
}

__global__ void __launch_bounds__(kBlock) k_zero(int64_t n, double *__restrict__ v) {
    GRID_STRIDE(i, n) v[i] = 0.0;
}

inline int grid_for(int64_t n) { return int(std::max<int64_t>(1, (n + kBlock - 1) / kBlock)); }

template <class P>
P *at(void *base, size_t off) {
    return reinterpret_cast<P *>(static_cast<uint8_t *>(base) + off);
}

Mat mat_of(const hbmc_matrix_s *m) {
    const PackedOffsets &o = m->offs;
    return Mat{at<double>(m->dev, m->off_diag), at<int32_t>(m->dev, o.soff),
               at<int32_t>(m->dev, o.sbase), at<uint64_t>(m->dev, o.smask),
               at<double>(m->dev, o.sval), at<int32_t>(m->dev, o.ioff),
               at<int32_t>(m->dev, o.icol), at<double>(m->dev, o.ival), m->n_pad};
}

std::atomic<uint64_t> g_uid{1};

// Workspace: b, x, r, z, p, q in HBMC order, partial sums, the CG state,
// the true-residual slot and the residual history.
// Workspace: b, x, r, z, p (two, used in turn), q in HBMC order, partial
// sums (per workgroup and per tile), the CG state, the true-residual slot
// and the residual history.
struct Work {
    double *bb, *xb, *r, *z, *p[2], *q, *part, *part_rr, *part_rz, *resid, *hist;
    CgState *st;
    int32_t hist_len;
};

constexpr int32_t kHistLen = 65536;

size_t work_layout(int64_t n_pad, int64_t ntiles, Work *w, void *base) {
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t vec = up(size_t(n_pad) * sizeof(double));
    const size_t part = up(size_t(2) * grid_for(n_pad) * sizeof(double));
    const size_t tp = up(size_t(ntiles) * sizeof(double));
    const size_t hist = size_t(kHistLen) * sizeof(double);
    const size_t total = 7 * vec + part + 2 * tp + 256 + 256 + hist;
    if (w && base) {
        auto *b = static_cast<uint8_t *>(base);
        double **v[7] = {&w->bb, &w->xb, &w->r, &w->z, &w->p[0], &w->p[1], &w->q};
        for (int i = 0; i < 7; ++i) *v[i] = reinterpret_cast<double *>(b + i * vec);
        size_t at = 7 * vec;
        w->part = reinterpret_cast<double *>(b + at); at += part;
        w->part_rr = reinterpret_cast<double *>(b + at); at += tp;
        w->part_rz = reinterpret_cast<double *>(b + at); at += tp;
        w->st = reinterpret_cast<CgState *>(b + at); at += 256;
        w->resid = reinterpret_cast<double *>(b + at); at += 256;
        w->hist = reinterpret_cast<double *>(b + at);
        w->hist_len = kHistLen;
    }
    return total;
}

// One CG iteration (everything after the first preconditioning step); the
// direction is read from p[parity] and written to p[1 - parity].
//   q = A p, p = z + beta p_old  |  alpha = rho / (p, q)  |
//   x += alpha p, r -= alpha q, z = M^-1 r, partials of ||r||^2 and (r, z)  |
//   stopping test, beta
int enqueue_iteration(const hbmc_factor_s *f, const Mat &m, const Work &w, hipStream_t s,
                      bool history, int parity) {
    const int64_t n = f->n_pad;
    const int g = grid_for(n);
    const int ntiles = int(f->tile_base[f->nc]);
    double *p_old = w.p[parity], *p_new = w.p[1 - parity];
    hipLaunchKernelGGL(k_spmv_dot_p, dim3(g), dim3(kBlock), 0, s, m, w.z, p_old, p_new, w.q, w.part, w.st);
    hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(kFin), 0, s, w.part, g, w.st);
    HIP_TRY(hipGetLastError());
    const ApplyCg cg{w.xb, p_new, w.q, w.r, &w.st->alpha, w.part_rr, w.part_rz};
    int st = apply_launch(f, w.r, w.z, s, &w.st->done, &cg);
    if (st) return st;
    hipLaunchKernelGGL(k_fin_rr_beta, dim3(1), dim3(kFin), 0, s, w.part_rr, w.part_rz, ntiles, w.st,
                       history ? w.hist : nullptr, w.hist_len);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

// A private stream to capture graphs on (the caller's stream may be the
// legacy null stream, which cannot be captured).  Default priority.
hipStream_t capture_stream() {
    static thread_local hipStream_t cs = nullptr;
    static thread_local int dev = -1;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (!cs || dev != cur) {
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return nullptr;
        dev = cur;
    }
    return cs;
}

int get_graph(hbmc_factor_s *f, const hbmc_matrix_s *A, const Mat &m, const Work &w, void *work,
              int iters, bool history, hipGraphExec_t *out) {
    for (const auto &gph : f->graphs)
        if (gph.matrix_uid == A->uid && gph.work == work && gph.iters == iters * (history ? -1 : 1)) {
            *out = static_cast<hipGraphExec_t>(gph.exec);
            return HBMC_OK;
        }
    hipStream_t cs = capture_stream();
    if (!cs) return fail(HBMC_EHIP, "cannot create a capture stream");
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int st = HBMC_OK;
    for (int k = 0; k < iters && st == HBMC_OK; ++k) st = enqueue_iteration(f, m, w, cs, history, k & 1);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &graph);
    if (st) { if (graph) hipGraphDestroy(graph); return st; }
    if (e != hipSuccess) return fail(HBMC_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(HBMC_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    f->graphs.push_back({A->uid, work, iters * (history ? -1 : 1), exec});
    *out = exec;
    return HBMC_OK;
}

}  // namespace

uint64_t hbmc::next_uid() { return g_uid.fetch_add(1); }

void hbmc::release_graphs(hbmc_factor_s *f) {
    for (auto &gph : f->graphs) hipGraphExecDestroy(static_cast<hipGraphExec_t>(gph.exec));
    f->graphs.clear();
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int hbmc_matrix_upload(hbmc_matrix_t *m, void *dev, size_t bytes, void *stream) {
    clear_error();
    if (!m || !dev) return fail(HBMC_EINVAL, "null argument");
    if (bytes < m->image.bytes.size())
        return fail(HBMC_EINVAL, "device buffer too small (%zu < %zu)", bytes, m->image.bytes.size());
    if (reinterpret_cast<uintptr_t>(dev) % 256) return fail(HBMC_EINVAL, "device buffer not 256-byte aligned");
    auto s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(dev, m->image.bytes.data(), m->image.bytes.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    m->dev = dev;
    m->dev_bytes = bytes;
    m->uid = next_uid();
    return HBMC_OK;
}

extern "C" int hbmc_spmv(const hbmc_matrix_t *m, const double *x, double *y, int32_t nrhs, void *stream) {
    if (!m || !x || !y) return fail(HBMC_EINVAL, "null argument");
    if (!m->dev) return fail(HBMC_ENOTREADY, "matrix not uploaded");
    if (nrhs != 1) return fail(HBMC_EINVAL, "nrhs = %d not supported", nrhs);
    if (x == y) return fail(HBMC_EINVAL, "y must not alias x");
    hipLaunchKernelGGL(k_spmv, dim3(grid_for(m->n_pad)), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), mat_of(m), x, y);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int hbmc_to_hbmc(const hbmc_factor_t *f, const double *v, double *vb, int32_t nrhs, void *stream) {
    if (!f || !v || !vb) return fail(HBMC_EINVAL, "null argument");
    if (!f->dev) return fail(HBMC_ENOTREADY, "factor not uploaded");
    if (nrhs != 1) return fail(HBMC_EINVAL, "nrhs = %d not supported", nrhs);
    hipLaunchKernelGGL(k_to_hbmc, dim3(grid_for(f->n_pad)), dim3(kBlock), 0, static_cast<hipStream_t>(stream),
                       f->n_pad, at<int32_t>(f->dev, f->off_iperm), v, vb);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int hbmc_from_hbmc(const hbmc_factor_t *f, const double *vb, double *v, int32_t nrhs, void *stream) {
    if (!f || !v || !vb) return fail(HBMC_EINVAL, "null argument");
    if (!f->dev) return fail(HBMC_ENOTREADY, "factor not uploaded");
    if (nrhs != 1) return fail(HBMC_EINVAL, "nrhs = %d not supported", nrhs);
    hipLaunchKernelGGL(k_from_hbmc, dim3(grid_for(f->n)), dim3(kBlock), 0, static_cast<hipStream_t>(stream),
                       int64_t(f->n), at<int32_t>(f->dev, f->off_perm), vb, v);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int iccg_workspace_bytes(const hbmc_factor_t *f, int32_t nrhs, size_t *bytes) {
    if (!f || !bytes) return fail(HBMC_EINVAL, "null argument");
    if (nrhs != 1) return fail(HBMC_EINVAL, "nrhs = %d not supported", nrhs);
    *bytes = work_layout(f->n_pad, f->tile_base[f->nc], nullptr, nullptr);
    return HBMC_OK;
}

extern "C" int iccg_solve(const hbmc_factor_t *fc, const hbmc_matrix_t *A, const double *b, double *x,
                          int32_t nrhs, double tol, int32_t maxit, const hbmc_solve_opts_t *opts,
                          hbmc_solve_stats_t *stats, void *work, size_t work_bytes, void *stream) {
    clear_error();
    auto *f = const_cast<hbmc_factor_s *>(fc);   // the graph cache is mutable state
    if (!f || !A || !b || !x || !work) return fail(HBMC_EINVAL, "null argument");
    if (!f->dev) return fail(HBMC_ENOTREADY, "factor not uploaded");
    if (!A->dev) return fail(HBMC_ENOTREADY, "matrix not uploaded");
    if (A->n_pad != f->n_pad || A->n != f->n) return fail(HBMC_EINVAL, "matrix and factor sizes differ");
    if (nrhs != 1) return fail(HBMC_EINVAL, "nrhs = %d not supported", nrhs);
    if (maxit < 0 || !(tol >= 0.0)) return fail(HBMC_EINVAL, "bad tol or maxit");
    const int64_t ntiles = f->tile_base[f->nc];
    if (work_bytes < work_layout(f->n_pad, ntiles, nullptr, nullptr))
        return fail(HBMC_EINVAL, "workspace too small");
    Work w{};
    work_layout(f->n_pad, ntiles, &w, work);
    const bool x0_zero = opts && opts->x0_zero;
    const bool use_graph = opts && opts->use_graph;
    const bool history = opts && opts->record_history;
    int check = opts && opts->check_every > 0 ? opts->check_every : (use_graph ? 16 : 1);
    if (use_graph) check = (check + 1) & ~1;   // graphs hold whole pairs of iterations
    auto s = static_cast<hipStream_t>(stream);
    const int64_t n = f->n_pad;
    const int g = grid_for(n);
    const Mat m = mat_of(A);
    const int32_t *iperm = at<int32_t>(f->dev, f->off_iperm);
    const int32_t *perm = at<int32_t>(f->dev, f->off_perm);

    hipLaunchKernelGGL(k_to_hbmc, dim3(g), dim3(kBlock), 0, s, n, iperm, b, w.bb);
    if (x0_zero) hipLaunchKernelGGL(k_zero, dim3(g), dim3(kBlock), 0, s, n, w.xb);
    else hipLaunchKernelGGL(k_to_hbmc, dim3(g), dim3(kBlock), 0, s, n, iperm, x, w.xb);
    hipLaunchKernelGGL(k_spmv, dim3(g), dim3(kBlock), 0, s, m, w.xb, w.q);
    hipLaunchKernelGGL(k_init_r, dim3(g), dim3(kBlock), 0, s, n, w.bb, w.q, w.r, w.part);
    hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(kFin), 0, s, w.part, g, w.st, tol, maxit,
                       history ? w.hist : nullptr);
    HIP_TRY(hipGetLastError());
    CgState h{};
    HIP_TRY(hipMemcpyAsync(&h, w.st, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));

    if (h.bb == 0.0) {
        hipLaunchKernelGGL(k_zero, dim3(g), dim3(kBlock), 0, s, n, w.xb);
    } else if (h.done == kRunning) {
        int st = apply_launch(f, w.r, w.z, s, nullptr, nullptr);
        if (st) return st;
        hipLaunchKernelGGL(k_init_p, dim3(g), dim3(kBlock), 0, s, n, w.r, w.z, w.p[0], w.part);
        hipLaunchKernelGGL(k_fin_rho, dim3(1), dim3(kFin), 0, s, w.part, g, w.st);
        HIP_TRY(hipGetLastError());
        hipGraphExec_t exec = nullptr;
        if (use_graph && (st = get_graph(f, A, m, w, work, check, history, &exec))) return st;
        int parity = 0;
        while (h.done == kRunning) {
            if (use_graph) HIP_TRY(hipGraphLaunch(exec, s));
            else
                for (int k = 0; k < check; ++k, parity ^= 1)
                    if ((st = enqueue_iteration(f, m, w, s, history, parity))) return st;
            HIP_TRY(hipMemcpyAsync(&h, w.st, sizeof h, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
    }
    // solution back to the caller's numbering, and the true residual
    hipLaunchKernelGGL(k_from_hbmc, dim3(grid_for(f->n)), dim3(kBlock), 0, s, int64_t(f->n), perm, w.xb, x);
    hipLaunchKernelGGL(k_spmv, dim3(g), dim3(kBlock), 0, s, m, w.xb, w.q);
    hipLaunchKernelGGL(k_resid, dim3(g), dim3(kBlock), 0, s, n, w.bb, w.q, w.part);
    hipLaunchKernelGGL(k_fin_resid, dim3(1), dim3(kFin), 0, s, w.part, g, w.resid);
    HIP_TRY(hipGetLastError());
    double rr_true = 0.0;
    HIP_TRY(hipMemcpyAsync(&rr_true, w.resid, sizeof rr_true, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int status = h.done == kConverged ? HBMC_OK
                       : h.done == kBreakdown ? HBMC_EBREAKDOWN : HBMC_ENOCONV;
    if (stats) {
        stats->iters = h.it;
        stats->status = status;
        stats->rel_res = h.res;
        stats->true_rel_res = h.bb > 0.0 ? std::sqrt(rr_true / h.bb) : 0.0;
    }
    if (status == HBMC_EBREAKDOWN) return fail(HBMC_EBREAKDOWN, "CG breakdown: (p, Ap) <= 0 or not finite");
    if (status == HBMC_ENOCONV) fail(HBMC_ENOCONV, "maxit = %d reached", maxit);
    return status;
}

// Residual history of the last iccg_solve that ran with record_history:
// hist[0..count) = ||r_k|| / ||b|| for k = 0..count-1, read from the
// workspace (synchronous copy to host memory).
extern "C" int iccg_history(const void *work, size_t work_bytes, const hbmc_factor_t *f, double *hist,
                            int32_t count, void *stream) {
    if (!work || !f || !hist || count < 0) return fail(HBMC_EINVAL, "null argument");
    const int64_t ntiles = f->tile_base[f->nc];
    if (work_bytes < work_layout(f->n_pad, ntiles, nullptr, nullptr))
        return fail(HBMC_EINVAL, "workspace too small");
    Work w{};
    work_layout(f->n_pad, ntiles, &w, const_cast<void *>(work));
    if (count > w.hist_len) return fail(HBMC_EINVAL, "history holds at most %d entries", w.hist_len);
    auto s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(hist, w.hist, size_t(count) * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return HBMC_OK;
}
