// IC(0)-preconditioned CG on gfx950 (Section 2; stopping test of Section 5.1):
// the SpMV on the sliced-ELL Abar, the inner products and vector updates, the
// permutations between numberings, and the solver loop.
//
// One call may solve several independent systems at once (an ordering made
// by hbmc_order_batch): each keeps its own CG scalars and stopping test,
// while every kernel covers all of them.  Vector kernels work in parts of
// kPartRows rows (one workgroup each) and the substitution in tiles; each
// part and each tile belongs to one system.
//
// Reductions never communicate between workgroups inside a kernel (a
// device-scope release fence per workgroup costs far more than the data):
// each workgroup writes the partial sum of its part or tile, and a
// finalizing kernel with one workgroup per system adds that system's
// partials in a fixed order and updates its scalars on the device.  Results
// are deterministic.
//
// All scalars and stop flags stay on the device; the host reads the number of
// stopped systems every check_every iterations.  With use_graph those
// iterations are captured once as a hipGraph (in pairs: the search direction
// lives in two buffers used in turn) and replayed.  Every kernel of an
// iteration skips stopped systems, so iterations past a system's stopping
// point change nothing for it.
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
constexpr int kBlock = kPartRows;   // threads of the vector kernels: one row each
constexpr int kFin = 1024;       // threads of the finalizing kernels (one workgroup per system)

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup (at most 1024 threads); valid in thread 0.
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

// Tables of the systems of one factor.
struct Sys {
    const int32_t *part_sys;    // [parts] system of each part
    const int32_t *tiles;       // [nsys][nc][2] tile range of each (system, color)
    const int32_t *parts;       // [nsys][nc][2] part range of each (system, color)
    int32_t nc, nsys;
};

// Fixed-order total of one system's partials (one per part, or one per
// tile), by one workgroup of kFin threads; valid in thread 0.  Each thread
// issues kLoads independent loads before it adds them (in index order), so
// that the latency of the partials' loads is paid once per kLoads, not once
// per partial.
constexpr int kLoads = 16;
__device__ inline double sys_total(const double *part, const int32_t *ranges, int nc, int s) {
    double acc = 0.0;
    for (int c = 0; c < nc; ++c) {
        const int a = ranges[(s * nc + c) * 2], b = ranges[(s * nc + c) * 2 + 1];
        for (int i0 = a + int(threadIdx.x); i0 < b; i0 += kFin * kLoads) {
            double v[kLoads];
#pragma unroll
            for (int k = 0; k < kLoads; ++k) v[k] = i0 + k * kFin < b ? part[i0 + k * kFin] : 0.0;
#pragma unroll
            for (int k = 0; k < kLoads; ++k) acc += v[k];
        }
    }
    return block_sum(acc);
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

// Rows of the vector kernels: one thread per row, one part of kPartRows
// rows per workgroup.  In the last part (n need not be a multiple of it) a
// wavefront whose 64 rows all lie past n does no work; in the wavefront that
// holds row n - 1 all 64 lanes stay active (the SpMV broadcasts slot
// metadata from any lane), the lanes past n computing on row n - 1 and
// storing nothing.  Every thread still reaches the workgroup's reduction.
struct RowOf {
    int64_t row;     // this thread's row
    int64_t rc;      // the row it reads (row, or n - 1 past the end)
    int64_t g;       // its 64-row group (wave-uniform)
    bool wave_on;    // the wavefront has rows below n
    bool valid;      // row < n
};
__device__ inline RowOf row_of(int64_t n) {
    RowOf r;
    r.row = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    r.g = __builtin_amdgcn_readfirstlane(int(r.row >> 6));
    r.wave_on = r.g * kLanes < n;
    r.valid = r.row < n;
    r.rc = r.valid ? r.row : n - 1;
    return r;
}

// One row of y = A x with x(i) given by an accessor; all 64 lanes of the
// group must be active.  The group's strided-slot bases and masks (at most
// 64) come in with one vector load, one slot per lane, and are broadcast
// with readlane.
template <class X>
__device__ inline double spmv_row_with(const Mat &m, X x, const RowOf &r) {
    const int64_t g = r.g;
    const int lane = int(threadIdx.x & 63);
    double acc = m.diag[r.rc] * x(r.rc);
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

__global__ void __launch_bounds__(kBlock) k_spmv(Mat m, const double *__restrict__ x,
                                                 double *__restrict__ y) {
    const RowOf r = row_of(m.n);
    if (!r.wave_on) return;
    const double v = spmv_row_with(m, [=](int64_t i) { return x[i]; }, r);
    if (r.valid) y[r.row] = v;
}

// the part's partial sum of a vector kernel (all threads of the workgroup)
__device__ inline void store_part(double *part, double value) {
    const double s = block_sum(value);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// r = b - q; part partials of ||b||^2 and ||r||^2
__global__ void __launch_bounds__(kBlock) k_init_r(int64_t n, const double *__restrict__ b,
                                                   const double *__restrict__ q,
                                                   double *__restrict__ rv, double *part, int64_t np) {
    const RowOf r = row_of(n);
    double sb = 0.0, sr = 0.0;
    if (r.valid) {
        const double ri = b[r.row] - q[r.row];
        rv[r.row] = ri;
        sb = b[r.row] * b[r.row];
        sr = ri * ri;
    }
    store_part(part, sb);
    store_part(part + np, sr);
}

// one stopped system more; the last one raises the all-stopped flag
__device__ inline void count_done(int32_t *ndone, int32_t *alldone, int nsys) {
    if (atomicAdd(ndone, 1) + 1 == nsys) *alldone = 1;
}

// per system: ||b||^2, ||r0||^2, the state, and whether it is already done
__global__ void __launch_bounds__(kFin) k_fin_init(const double *part, int64_t np, Sys sys, CgState *st,
                                                   double tol, int32_t maxit, double *hist,
                                                   int32_t *ndone, int32_t *alldone) {
    const int s = blockIdx.x;
    const double bb = sys_total(part, sys.parts, sys.nc, s);
    const double rr = sys_total(part + np, sys.parts, sys.nc, s);
    if (threadIdx.x) return;
    CgState &c = st[s];
    c.bb = bb;
    c.rr = rr;
    c.tol = tol;
    c.maxit = maxit;
    c.it = 0;
    c.alpha = 0.0;
    c.beta = 0.0;
    c.res = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    if (hist && s == 0) hist[0] = c.res;
    c.done = (bb == 0.0 || c.res < tol) ? kConverged : (maxit <= 0 ? kMaxIt : kRunning);
    if (!isfinite(c.res)) c.done = kBreakdown;
    if (c.done) count_done(ndone, alldone, sys.nsys);
}

// p = z; part partials of (r, z)
__global__ void __launch_bounds__(kBlock) k_init_p(int64_t n, const double *__restrict__ rv,
                                                   const double *__restrict__ z,
                                                   double *__restrict__ p, double *part) {
    const RowOf r = row_of(n);
    double s = 0.0;
    if (r.valid) {
        p[r.row] = z[r.row];
        s = rv[r.row] * z[r.row];
    }
    store_part(part, s);
}

__global__ void __launch_bounds__(kFin) k_fin_rho(const double *part, Sys sys, CgState *st) {
    const int s = blockIdx.x;
    const double t = sys_total(part, sys.parts, sys.nc, s);
    if (threadIdx.x == 0) { st[s].rho = t; st[s].beta = 0.0; }
}

// p = z + beta p_old (formed on the fly, also at the columns the row
// couples to), written to p_new; q = A p; part partials of (p, q)
__global__ void __launch_bounds__(kBlock) k_spmv_dot_p(Mat m, Sys sys, const double *__restrict__ z,
                                                       const double *__restrict__ p_old,
                                                       double *__restrict__ p_new,
                                                       double *__restrict__ q, double *part,
                                                       const CgState *st, const int32_t *alldone) {
    if (*alldone) return;
    const CgState &c = st[sys.part_sys[blockIdx.x]];
    if (c.done) return;                       // workgroup-uniform: a part lies in one system
    const RowOf r = row_of(m.n);
    double pq = 0.0;
    if (r.wave_on) {
        const double beta = c.beta;
        auto pv = [=](int64_t i) { return z[i] + beta * p_old[i]; };
        const double pi = pv(r.rc);
        const double qi = spmv_row_with(m, pv, r);
        if (r.valid) {
            p_new[r.row] = pi;
            q[r.row] = qi;
            pq = pi * qi;
        }
    }
    store_part(part, pq);
}

// sigma = (p, Ap); alpha = rho / sigma
__global__ void __launch_bounds__(kFin) k_fin_alpha(const double *part, Sys sys, CgState *st,
                                                    int32_t *ndone, int32_t *alldone) {
    const int s = blockIdx.x;
    CgState &c = st[s];
    if (c.done) return;
    const double sigma = sys_total(part, sys.parts, sys.nc, s);
    if (threadIdx.x) return;
    c.sigma = sigma;
    if (!(sigma > 0.0) || !isfinite(sigma)) {
        c.done = kBreakdown;
        c.it += 1;
        count_done(ndone, alldone, sys.nsys);
        return;
    }
    c.alpha = c.rho / sigma;
}

// After the preconditioning step: ||r||^2 and (r, z) from the per-tile
// partials; one more iteration done; stopping test ||r|| / ||b|| < tol;
// then beta = rho' / rho, rho = rho' for the next direction.
__global__ void __launch_bounds__(kFin) k_fin_rr_beta(const double *part_rr, const double *part_rz,
                                                      Sys sys, CgState *st, double *hist,
                                                      int32_t hist_len, int32_t *ndone,
                                                      int32_t *alldone) {
    const int s = blockIdx.x;
    CgState &c = st[s];
    if (c.done) return;
    const double rr = sys_total(part_rr, sys.tiles, sys.nc, s);
    const double rz = sys_total(part_rz, sys.tiles, sys.nc, s);
    if (threadIdx.x) return;
    c.rr = rr;
    c.it += 1;
    c.res = sqrt(rr / c.bb);
    if (hist && s == 0 && c.it < hist_len) hist[c.it] = c.res;
    if (!isfinite(c.res)) c.done = kBreakdown;
    else if (c.res < c.tol) c.done = kConverged;
    else if (c.it >= c.maxit) c.done = kMaxIt;
    else {
        c.beta = rz / c.rho;
        c.rho = rz;
    }
    if (c.done) count_done(ndone, alldone, sys.nsys);
}

// part partials of ||b - q||^2 (true residual)
__global__ void __launch_bounds__(kBlock) k_resid(int64_t n, const double *__restrict__ b,
                                                  const double *__restrict__ q, double *part) {
    const RowOf r = row_of(n);
    double s = 0.0;
    if (r.valid) { const double d = b[r.row] - q[r.row]; s = d * d; }
    store_part(part, s);
}

__global__ void __launch_bounds__(kFin) k_fin_resid(const double *part, Sys sys, double *out) {
    const int s = blockIdx.x;
    const double t = sys_total(part, sys.parts, sys.nc, s);
    if (threadIdx.x == 0) out[s] = t;
}

__global__ void __launch_bounds__(kBlock) k_to_hbmc(int64_t n_pad, const int32_t *__restrict__ iperm,
                                                    const double *__restrict__ v,
                                                    double *__restrict__ vb) {
    const int64_t r = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (r < n_pad) { const int32_t i = iperm[r]; vb[r] = i >= 0 ? v[i] : 0.0; }
}

__global__ void __launch_bounds__(kBlock) k_from_hbmc(int64_t n, const int32_t *__restrict__ perm,
                                                      const double *__restrict__ vb,
                                                      double *__restrict__ v) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) v[i] = vb[perm[i]];
}

// x = 0 on the rows of the systems whose right-hand side is zero
__global__ void __launch_bounds__(kBlock) k_zero_b0(int64_t n, const int32_t *__restrict__ part_sys,
                                                    const CgState *st, double *__restrict__ x) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n && st[part_sys[blockIdx.x]].bb == 0.0) x[i] = 0.0;
}

__global__ void __launch_bounds__(kBlock) k_zero(int64_t n, double *__restrict__ v) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) v[i] = 0.0;
}

__global__ void k_zero_int(int32_t *a, int n) {
    if (int(threadIdx.x) < n) a[threadIdx.x] = 0;
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

Sys sys_of(const hbmc_factor_s *f) {
    return Sys{at<int32_t>(f->dev, f->off_part_sys), at<int32_t>(f->dev, f->off_sys_tiles),
               at<int32_t>(f->dev, f->off_sys_parts), f->nc, f->nsys};
}

std::atomic<uint64_t> g_uid{1};

// Workspace: b, x, r, z, p (two, used in turn), q in HBMC order; partial
// sums per part (two slots) and per tile (two); the CG state of each
// system; the stopped-system counter and the all-stopped flag; the true
// residuals; the residual history of system 0.
struct Work {
    double *bb, *xb, *r, *z, *p[2], *q, *part_g, *part_rr, *part_rz, *resid, *hist;
    CgState *st;
    int32_t *ndone, *alldone;
    int64_t np;
    int32_t hist_len;
};

constexpr int32_t kHistLen = 65536;

size_t work_layout(const hbmc_factor_s *f, Work *w, void *base) {
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const int64_t np = (f->n_pad + kPartRows - 1) / kPartRows;
    const int64_t ntiles = f->tile_base[f->nc];
    const size_t vec = up(size_t(f->n_pad) * sizeof(double));
    const size_t pg = up(size_t(2) * np * sizeof(double));
    const size_t tp = up(size_t(ntiles) * sizeof(double));
    const size_t sts = up(size_t(f->nsys) * sizeof(CgState));
    const size_t res = up(size_t(f->nsys) * sizeof(double));
    const size_t hist = size_t(kHistLen) * sizeof(double);
    const size_t total = 7 * vec + pg + 2 * tp + sts + 256 + res + hist;
    if (w && base) {
        auto *b = static_cast<uint8_t *>(base);
        double **v[7] = {&w->bb, &w->xb, &w->r, &w->z, &w->p[0], &w->p[1], &w->q};
        for (int i = 0; i < 7; ++i) *v[i] = reinterpret_cast<double *>(b + i * vec);
        size_t a = 7 * vec;
        w->part_g = reinterpret_cast<double *>(b + a); a += pg;
        w->part_rr = reinterpret_cast<double *>(b + a); a += tp;
        w->part_rz = reinterpret_cast<double *>(b + a); a += tp;
        w->st = reinterpret_cast<CgState *>(b + a); a += sts;
        w->ndone = reinterpret_cast<int32_t *>(b + a);
        w->alldone = w->ndone + 1; a += 256;
        w->resid = reinterpret_cast<double *>(b + a); a += res;
        w->hist = reinterpret_cast<double *>(b + a);
        w->hist_len = kHistLen;
        w->np = np;
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
    const int g = grid_for(f->n_pad);
    const Sys sys = sys_of(f);
    double *p_old = w.p[parity], *p_new = w.p[1 - parity];
    hipLaunchKernelGGL(k_spmv_dot_p, dim3(g), dim3(kBlock), 0, s, m, sys, w.z, p_old, p_new, w.q,
                       w.part_g, w.st, w.alldone);
    hipLaunchKernelGGL(k_fin_alpha, dim3(f->nsys), dim3(kFin), 0, s, w.part_g, sys, w.st, w.ndone,
                       w.alldone);
    HIP_TRY(hipGetLastError());
    const ApplyCg cg{w.xb, p_new, w.q, w.r, w.st, at<int32_t>(f->dev, f->off_tile_sys),
                     w.part_rr, w.part_rz};
    int st = apply_launch(f, w.r, w.z, s, w.alldone, &cg);
    if (st) return st;
    hipLaunchKernelGGL(k_fin_rr_beta, dim3(f->nsys), dim3(kFin), 0, s, w.part_rr, w.part_rz, sys, w.st,
                       history ? w.hist : nullptr, w.hist_len, w.ndone, w.alldone);
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
    const int32_t key = iters * (history ? -1 : 1);
    for (const auto &gph : f->graphs)
        if (gph.matrix_uid == A->uid && gph.work == work && gph.iters == key) {
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
    f->graphs.push_back({A->uid, work, key, exec});
    *out = exec;
    return HBMC_OK;
}

int check_ready(const hbmc_factor_s *f, int32_t nrhs) {
    if (!f) return fail(HBMC_EINVAL, "null handle");
    if (!f->dev) return fail(HBMC_ENOTREADY, "factor not uploaded");
    if (nrhs != 1) return fail(HBMC_EINVAL, "nrhs = %d not supported", nrhs);
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
    int st = check_ready(f, nrhs);
    if (st) return st;
    if (!v || !vb) return fail(HBMC_EINVAL, "null argument");
    hipLaunchKernelGGL(k_to_hbmc, dim3(grid_for(f->n_pad)), dim3(kBlock), 0, static_cast<hipStream_t>(stream),
                       f->n_pad, at<int32_t>(f->dev, f->off_iperm), v, vb);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int hbmc_from_hbmc(const hbmc_factor_t *f, const double *vb, double *v, int32_t nrhs, void *stream) {
    int st = check_ready(f, nrhs);
    if (st) return st;
    if (!v || !vb) return fail(HBMC_EINVAL, "null argument");
    hipLaunchKernelGGL(k_from_hbmc, dim3(grid_for(f->n)), dim3(kBlock), 0, static_cast<hipStream_t>(stream),
                       int64_t(f->n), at<int32_t>(f->dev, f->off_perm), vb, v);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int iccg_workspace_bytes(const hbmc_factor_t *f, int32_t nrhs, size_t *bytes) {
    if (!f || !bytes) return fail(HBMC_EINVAL, "null argument");
    if (nrhs != 1) return fail(HBMC_EINVAL, "nrhs = %d not supported", nrhs);
    *bytes = work_layout(f, nullptr, nullptr);
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
    if (work_bytes < work_layout(f, nullptr, nullptr)) return fail(HBMC_EINVAL, "workspace too small");
    Work w{};
    work_layout(f, &w, work);
    const bool x0_zero = opts && opts->x0_zero;
    const bool use_graph = opts && opts->use_graph;
    const bool history = opts && opts->record_history;
    int check = opts && opts->check_every > 0 ? opts->check_every : (use_graph ? 16 : 1);
    if (use_graph) check = (check + 1) & ~1;   // graphs hold whole pairs of iterations
    auto s = static_cast<hipStream_t>(stream);
    const int64_t n = f->n_pad;
    const int g = grid_for(n);
    const Mat m = mat_of(A);
    const Sys sys = sys_of(f);
    const int32_t *iperm = at<int32_t>(f->dev, f->off_iperm);
    const int32_t *perm = at<int32_t>(f->dev, f->off_perm);

    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, w.ndone, 2);
    hipLaunchKernelGGL(k_to_hbmc, dim3(g), dim3(kBlock), 0, s, n, iperm, b, w.bb);
    if (x0_zero) hipLaunchKernelGGL(k_zero, dim3(g), dim3(kBlock), 0, s, n, w.xb);
    else hipLaunchKernelGGL(k_to_hbmc, dim3(g), dim3(kBlock), 0, s, n, iperm, x, w.xb);
    hipLaunchKernelGGL(k_spmv, dim3(g), dim3(kBlock), 0, s, m, w.xb, w.q);
    hipLaunchKernelGGL(k_init_r, dim3(g), dim3(kBlock), 0, s, n, w.bb, w.q, w.r, w.part_g, w.np);
    hipLaunchKernelGGL(k_fin_init, dim3(f->nsys), dim3(kFin), 0, s, w.part_g, w.np, sys, w.st, tol, maxit,
                       history ? w.hist : nullptr, w.ndone, w.alldone);
    HIP_TRY(hipGetLastError());
    int32_t hd[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(hd, w.ndone, sizeof hd, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));

    if (hd[0] < f->nsys) {
        int st = apply_launch(f, w.r, w.z, s, nullptr, nullptr);
        if (st) return st;
        hipLaunchKernelGGL(k_init_p, dim3(g), dim3(kBlock), 0, s, n, w.r, w.z, w.p[0], w.part_g);
        hipLaunchKernelGGL(k_fin_rho, dim3(f->nsys), dim3(kFin), 0, s, w.part_g, sys, w.st);
        HIP_TRY(hipGetLastError());
        hipGraphExec_t exec = nullptr;
        if (use_graph && (st = get_graph(f, A, m, w, work, check, history, &exec))) return st;
        int parity = 0;
        while (hd[0] < f->nsys) {
            if (use_graph) HIP_TRY(hipGraphLaunch(exec, s));
            else
                for (int k = 0; k < check; ++k, parity ^= 1)
                    if ((st = enqueue_iteration(f, m, w, s, history, parity))) return st;
            HIP_TRY(hipMemcpyAsync(hd, w.ndone, sizeof hd, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
    }
    // systems with b = 0 get x = 0; the solution back to the caller's
    // numbering; the true residuals
    hipLaunchKernelGGL(k_zero_b0, dim3(g), dim3(kBlock), 0, s, n, sys.part_sys, w.st, w.xb);
    hipLaunchKernelGGL(k_from_hbmc, dim3(grid_for(f->n)), dim3(kBlock), 0, s, int64_t(f->n), perm, w.xb, x);
    hipLaunchKernelGGL(k_spmv, dim3(g), dim3(kBlock), 0, s, m, w.xb, w.q);
    hipLaunchKernelGGL(k_resid, dim3(g), dim3(kBlock), 0, s, n, w.bb, w.q, w.part_g);
    hipLaunchKernelGGL(k_fin_resid, dim3(f->nsys), dim3(kFin), 0, s, w.part_g, sys, w.resid);
    HIP_TRY(hipGetLastError());
    std::vector<CgState> hs(f->nsys);
    std::vector<double> rt(f->nsys);
    HIP_TRY(hipMemcpyAsync(hs.data(), w.st, hs.size() * sizeof(CgState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(rt.data(), w.resid, rt.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int status = HBMC_OK;
    for (int32_t k = 0; k < f->nsys; ++k) {
        const int sk = hs[k].done == kConverged ? HBMC_OK
                       : hs[k].done == kBreakdown ? HBMC_EBREAKDOWN : HBMC_ENOCONV;
        if (sk == HBMC_EBREAKDOWN) status = HBMC_EBREAKDOWN;
        else if (sk == HBMC_ENOCONV && status == HBMC_OK) status = HBMC_ENOCONV;
        if (stats) {
            stats[k].iters = hs[k].it;
            stats[k].status = sk;
            stats[k].rel_res = hs[k].res;
            stats[k].true_rel_res = hs[k].bb > 0.0 ? std::sqrt(rt[k] / hs[k].bb) : 0.0;
        }
    }
    if (status == HBMC_EBREAKDOWN) return fail(HBMC_EBREAKDOWN, "CG breakdown: (p, Ap) <= 0 or not finite");
    if (status == HBMC_ENOCONV) fail(HBMC_ENOCONV, "maxit = %d reached", maxit);
    return status;
}

// Residual history of system 0 from the last iccg_solve that ran with
// record_history on this workspace: hist[k] = ||r_k|| / ||b||
// (synchronous copy to host memory).
extern "C" int iccg_history(const void *work, size_t work_bytes, const hbmc_factor_t *f, double *hist,
                            int32_t count, void *stream) {
    if (!work || !f || !hist || count < 0) return fail(HBMC_EINVAL, "null argument");
    if (work_bytes < work_layout(f, nullptr, nullptr)) return fail(HBMC_EINVAL, "workspace too small");
    Work w{};
    work_layout(f, &w, const_cast<void *>(work));
    if (count > w.hist_len) return fail(HBMC_EINVAL, "history holds at most %d entries", w.hist_len);
    auto s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(hist, w.hist, size_t(count) * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return HBMC_OK;
}
