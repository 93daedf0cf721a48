// Device side of the HBMC-ordered IC(0)-CG library for gfx950.
//
// Substitution (Section 4.2.2): colors run one after another (one kernel
// launch per color phase, the launch boundary being the synchronization of
// Section 4.4.3).  A workgroup owns one tile: 64 chain lanes, i.e. 64/w
// level-1 blocks of w BMC blocks each, and all bs steps of them
// (eqs. "y2-2", "y2-3").
//   1. Row pass: every row of the tile gets its own thread, which folds in
//      the couplings to other colors (eq. "for3") from a sliced-ELL layout
//      whose slices are the 64 rows of one wavefront -- coalesced, and fully
//      parallel.  The partial results land in LDS.
//   2. Chain pass: one wavefront, one lane per BMC block, walks the bs steps
//      of its block; a step only needs earlier (forward) or later (backward)
//      steps of the same lane, which sit in LDS.
// The last color runs its forward and backward chains in one launch, since
// it has no later color to wait for.
#include <hip/hip_runtime.h>

#include <algorithm>
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
constexpr int kBlock = 256;              // threads of the vector kernels
constexpr size_t kMaxLds = 64 * 1024;    // LDS budget of one phase workgroup

struct Tri {
    const int32_t *ext_off;
    const void *ext_val;
    const int32_t *ext_col;
    const int32_t *int_off;
    const void *int_val;
    const int32_t *int_lp;
};

struct Phase {
    int64_t row0, row1;   // rows of the color
    int64_t slice0;       // first global 64-row slice of the color
    int64_t tile0;        // first global tile of the color
    int64_t nlane;        // chain lanes of the color (level-1 blocks * w)
    int32_t w;
    int32_t lds_int;      // internal couplings staged in LDS
    int32_t fslots, bslots;
    Tri f, b;
    const void *dinv;
};

enum { kForward = 0, kBackward = 1, kLast = 2 };

// One color phase.  MODE kForward: y of color c; kBackward: z of color c;
// kLast: y then z of the last color.  z holds y of the colors whose forward
// step is done and z of the colors whose backward step is done.
template <int BS, typename T, int MODE>
__global__ void __launch_bounds__(512) k_phase(Phase ph, const double *__restrict__ r,
                                               double *__restrict__ z) {
    extern __shared__ __align__(16) unsigned char smem[];
    T *q = reinterpret_cast<T *>(smem);   // [BS][64]: partial sums, then y / z
    T *dv = q + BS * kLanes;              // [BS][64]: diaginv (forward)
    T *fval = dv + BS * kLanes;
    T *bval = fval + ph.fslots * kLanes;
    int32_t *flp = reinterpret_cast<int32_t *>(bval + ph.bslots * kLanes);
    int32_t *blp = flp + ph.fslots * kLanes;

    const int tile = blockIdx.x;
    const int64_t trow0 = ph.row0 + int64_t(tile) * BS * kLanes;
    const int w = ph.w;
    const int bw = BS * w;
    const int64_t gt = (ph.tile0 + tile) * BS;   // first (tile, step) slot list

    // 1. row pass: couplings to other colors
    for (int t = threadIdx.x; t < BS * kLanes; t += blockDim.x) {
        const int64_t row = trow0 + t;
        if (row >= ph.row1) break;
        const int kl = t / bw, rem = t - kl * bw, l = rem / w, m = rem - l * w;
        const int slot = l * kLanes + kl * w + m;
        const int64_t slice = ph.slice0 + int64_t(tile) * BS + (t >> 6);
        const int lane = t & (kLanes - 1);
        if (MODE != kBackward) {
            const T *ev = static_cast<const T *>(ph.f.ext_val);
            T acc = T(r[row]);
            for (int64_t s = ph.f.ext_off[slice]; s < ph.f.ext_off[slice + 1]; ++s) {
                const int64_t e = s * kLanes + lane;
                const int32_t c = ph.f.ext_col[e];
                if (c >= 0) acc -= ev[e] * T(z[c]);
            }
            q[slot] = acc;
            dv[slot] = static_cast<const T *>(ph.dinv)[row];
        } else {
            const T *ev = static_cast<const T *>(ph.b.ext_val);
            T acc = T(z[row]);
            for (int64_t s = ph.b.ext_off[slice]; s < ph.b.ext_off[slice + 1]; ++s) {
                const int64_t e = s * kLanes + lane;
                const int32_t c = ph.b.ext_col[e];
                if (c >= 0) acc -= ev[e] * T(z[c]);
            }
            q[slot] = acc;
        }
    }
    // stage the couplings inside the level-1 blocks
    const int64_t fib = MODE != kBackward ? ph.f.int_off[gt] : 0;
    const int64_t bib = MODE != kForward ? ph.b.int_off[gt] : 0;
    if (ph.lds_int) {
        if (MODE != kBackward) {
            const int64_t cnt = (ph.f.int_off[gt + BS] - fib) * kLanes;
            const T *sv = static_cast<const T *>(ph.f.int_val) + fib * kLanes;
            const int32_t *sl = ph.f.int_lp + fib * kLanes;
            for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) { fval[e] = sv[e]; flp[e] = sl[e]; }
        }
        if (MODE != kForward) {
            const int64_t cnt = (ph.b.int_off[gt + BS] - bib) * kLanes;
            const T *sv = static_cast<const T *>(ph.b.int_val) + bib * kLanes;
            const int32_t *sl = ph.b.int_lp + bib * kLanes;
            for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) { bval[e] = sv[e]; blp[e] = sl[e]; }
        }
    }
    __syncthreads();

    // 2. chain pass: one lane per BMC block
    if (threadIdx.x >= kLanes) return;
    const int j = threadIdx.x;
    if (int64_t(tile) * kLanes + j >= ph.nlane) return;
    const int64_t rb = trow0 + int64_t(j / w) * bw + (j % w);   // row of step 0

    if (MODE != kBackward) {
        const T *gv = static_cast<const T *>(ph.f.int_val);
#pragma unroll
        for (int l = 0; l < BS; ++l) {
            T acc = q[l * kLanes + j];
            const int64_t s0 = ph.f.int_off[gt + l], s1 = ph.f.int_off[gt + l + 1];
            for (int64_t s = s0; s < s1; ++s) {
                int32_t lp;
                T v;
                if (ph.lds_int) { const int64_t e = (s - fib) * kLanes + j; lp = flp[e]; v = fval[e]; }
                else { const int64_t e = s * kLanes + j; lp = ph.f.int_lp[e]; v = gv[e]; }
                acc -= v * q[lp * kLanes + j];
            }
            const T y = acc * dv[l * kLanes + j];
            q[l * kLanes + j] = y;
            if (MODE == kForward) z[rb + int64_t(l) * w] = double(y);
        }
    }
    if (MODE != kForward) {
        const T *gv = static_cast<const T *>(ph.b.int_val);
#pragma unroll
        for (int l = BS - 1; l >= 0; --l) {
            T acc = q[l * kLanes + j];
            const int64_t s0 = ph.b.int_off[gt + l], s1 = ph.b.int_off[gt + l + 1];
            for (int64_t s = s0; s < s1; ++s) {
                int32_t lp;
                T v;
                if (ph.lds_int) { const int64_t e = (s - bib) * kLanes + j; lp = blp[e]; v = bval[e]; }
                else { const int64_t e = s * kLanes + j; lp = ph.b.int_lp[e]; v = gv[e]; }
                acc -= v * q[lp * kLanes + j];
            }
            q[l * kLanes + j] = acc;
            z[rb + int64_t(l) * w] = double(acc);
        }
    }
}

// ---------------------------------------------------------------------------
// reductions: wavefront butterfly, then across the waves of the block, then
// across blocks by the last block to finish (fixed order: deterministic)
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int N>
__device__ inline void block_sum(double (&v)[N], double *sh) {   // sh: [N][16]
    const int wid = threadIdx.x >> 6, ln = threadIdx.x & 63, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
    if (ln == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) sh[k * 16 + wid] = v[k];
    __syncthreads();
    if (wid == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = wave_sum(ln < nw ? sh[k * 16 + ln] : 0.0);
    }
    __syncthreads();
}

// Sums v over the grid.  Returns true in thread 0 of the last block, where
// out[] then holds the totals.  partials: [N][gridDim.x].
template <int N>
__device__ bool grid_sum(double (&v)[N], double *partials, unsigned *counter, double (&out)[N]) {
    __shared__ double sh[N * 16];
    __shared__ int last;
    block_sum<N>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) partials[k * gridDim.x + blockIdx.x] = v[k];
        __threadfence();
        last = atomicAdd(counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    double s[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        s[k] = 0.0;
        for (unsigned i = threadIdx.x; i < gridDim.x; i += blockDim.x)
            s[k] += __builtin_nontemporal_load(&partials[k * gridDim.x + i]);
    }
    block_sum<N>(s, sh);
    if (threadIdx.x != 0) return false;
#pragma unroll
    for (int k = 0; k < N; ++k) out[k] = s[k];
    *counter = 0;
    return true;
}

struct Mat {
    const double *diag;
    const int32_t *soff;
    const double *val;
    const int32_t *col;
    int64_t n;
};

__device__ inline double spmv_row(const Mat &m, const double *__restrict__ x, int64_t row) {
    const int64_t slice = row >> 6;
    const int lane = int(row & 63);
    double acc = m.diag[row] * x[row];
    for (int64_t s = m.soff[slice]; s < m.soff[slice + 1]; ++s) {
        const int64_t e = s * kLanes + lane;
        const int32_t c = m.col[e];
        if (c >= 0) acc += m.val[e] * x[c];
    }
    return acc;
}

__global__ void __launch_bounds__(kBlock) k_spmv(Mat m, const double *__restrict__ x,
                                                 double *__restrict__ y) {
    const int64_t row = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (row < m.n) y[row] = spmv_row(m, x, row);
}

// CG state kept on the device between kernels
struct CgState {
    double rho, sigma, alpha, beta, rr, bb, rz, res;
    int32_t flag;   // 1 = breakdown
    int32_t pad;
    unsigned counter;
};

// r = b - q, with ||b||^2 and ||r||^2
__global__ void __launch_bounds__(kBlock) k_cg_init_r(int64_t n, const double *__restrict__ b,
                                                      const double *__restrict__ q,
                                                      double *__restrict__ r, double *partials,
                                                      CgState *st) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (i < n) {
        const double ri = b[i] - q[i];
        r[i] = ri;
        v[0] = b[i] * b[i];
        v[1] = ri * ri;
    }
    double out[2];
    if (grid_sum<2>(v, partials, &st->counter, out)) {
        st->bb = out[0];
        st->rr = out[1];
        st->res = out[0] > 0.0 ? sqrt(out[1] / out[0]) : 0.0;
        st->flag = 0;
    }
}

// p = z, rho = (r, z)
__global__ void __launch_bounds__(kBlock) k_cg_init_p(int64_t n, const double *__restrict__ r,
                                                      const double *__restrict__ z,
                                                      double *__restrict__ p, double *partials,
                                                      CgState *st) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (i < n) {
        p[i] = z[i];
        v[0] = r[i] * z[i];
    }
    double out[1];
    if (grid_sum<1>(v, partials, &st->counter, out)) st->rho = out[0];
}

// q = A p, sigma = (p, q), alpha = rho / sigma
__global__ void __launch_bounds__(kBlock) k_cg_spmv(Mat m, const double *__restrict__ p,
                                                    double *__restrict__ q, double *partials,
                                                    CgState *st) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (i < m.n) {
        const double qi = spmv_row(m, p, i);
        q[i] = qi;
        v[0] = p[i] * qi;
    }
    double out[1];
    if (grid_sum<1>(v, partials, &st->counter, out)) {
        st->sigma = out[0];
        if (!(out[0] > 0.0) || !isfinite(out[0])) st->flag = 1;
        st->alpha = st->rho / out[0];
    }
}

// x += alpha p, r -= alpha q, ||r||^2
__global__ void __launch_bounds__(kBlock) k_cg_xr(int64_t n, const double *__restrict__ p,
                                                  const double *__restrict__ q,
                                                  double *__restrict__ x, double *__restrict__ r,
                                                  double *partials, CgState *st) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    const double alpha = st->alpha;
    double v[1] = {0.0};
    if (i < n) {
        x[i] = x[i] + alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        v[0] = ri * ri;
    }
    double out[1];
    if (grid_sum<1>(v, partials, &st->counter, out)) {
        st->rr = out[0];
        st->res = sqrt(out[0] / st->bb);
        if (!isfinite(out[0])) st->flag = 1;
    }
}

// rho' = (r, z), beta = rho' / rho, rho = rho'
__global__ void __launch_bounds__(kBlock) k_cg_rz(int64_t n, const double *__restrict__ r,
                                                  const double *__restrict__ z, double *partials,
                                                  CgState *st) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    double v[1] = {i < n ? r[i] * z[i] : 0.0};
    double out[1];
    if (grid_sum<1>(v, partials, &st->counter, out)) {
        st->rz = out[0];
        st->beta = out[0] / st->rho;
        st->rho = out[0];
    }
}

// p = z + beta p
__global__ void __launch_bounds__(kBlock) k_cg_p(int64_t n, const double *__restrict__ z,
                                                 double *__restrict__ p, const CgState *st) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    const double beta = st->beta;
    if (i < n) p[i] = z[i] + beta * p[i];
}

// ||b - q||^2 (true residual)
__global__ void __launch_bounds__(kBlock) k_resid(int64_t n, const double *__restrict__ b,
                                                  const double *__restrict__ q, double *partials,
                                                  CgState *st) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (i < n) { const double d = b[i] - q[i]; v[0] = d * d; }
    double out[1];
    if (grid_sum<1>(v, partials, &st->counter, out)) st->rz = out[0];
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

__global__ void __launch_bounds__(kBlock) k_zero(int64_t n, double *__restrict__ v) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) v[i] = 0.0;
}

inline unsigned nblocks(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
template <class P>
const P *at(const void *base, size_t off) {
    return reinterpret_cast<const P *>(static_cast<const uint8_t *>(base) + off);
}

Tri tri_of(const hbmc_factor_s *f, const TriOffsets &o) {
    return Tri{at<int32_t>(f->dev, o.ext_off), at<void>(f->dev, o.ext_val),
               at<int32_t>(f->dev, o.ext_col), at<int32_t>(f->dev, o.int_off),
               at<void>(f->dev, o.int_val), at<int32_t>(f->dev, o.int_lp)};
}

Mat mat_of(const hbmc_matrix_s *m) {
    return Mat{at<double>(m->dev, m->off_diag), at<int32_t>(m->dev, m->off_soff),
               at<double>(m->dev, m->off_val), at<int32_t>(m->dev, m->off_col), m->n_pad};
}

template <int BS, typename T>
int launch_phases(const hbmc_factor_s *f, const double *r, double *z, hipStream_t s) {
    const size_t tsz = sizeof(T);
    Phase ph{};
    ph.w = f->w;
    ph.f = tri_of(f, f->fwd);
    ph.b = tri_of(f, f->bwd);
    ph.dinv = at<void>(f->dev, f->off_dinv);
    const size_t base = 2 * size_t(BS) * kLanes * tsz;
    const size_t staged =
        size_t(f->max_int_slots_f + f->max_int_slots_b) * kLanes * (tsz + sizeof(int32_t));
    ph.lds_int = base + staged <= kMaxLds;
    ph.fslots = ph.lds_int ? f->max_int_slots_f : 0;
    ph.bslots = ph.lds_int ? f->max_int_slots_b : 0;
    const size_t lds = ph.lds_int ? base + staged : base;
    const unsigned threads = unsigned(std::min(BS * kLanes, 512));
    auto run = [&](int c, auto kernel) -> int {
        ph.row0 = f->color_start[c];
        ph.row1 = f->color_start[c + 1];
        ph.slice0 = f->slice_base[c];
        ph.tile0 = f->tile_base[c];
        ph.nlane = (ph.row1 - ph.row0) / BS;
        const unsigned grid = unsigned(f->tile_base[c + 1] - f->tile_base[c]);
        if (grid == 0) return HBMC_OK;
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), lds, s, ph, r, z);
        HIP_TRY(hipGetLastError());
        return HBMC_OK;
    };
    const int nc = f->nc;
    int st;
    for (int c = 0; c + 1 < nc; ++c)
        if ((st = run(c, k_phase<BS, T, kForward>))) return st;
    if ((st = run(nc - 1, k_phase<BS, T, kLast>))) return st;
    for (int c = nc - 2; c >= 0; --c)
        if ((st = run(c, k_phase<BS, T, kBackward>))) return st;
    return HBMC_OK;
}

template <typename T>
int dispatch_bs(const hbmc_factor_s *f, const double *r, double *z, hipStream_t s) {
    switch (f->bs) {
        case 1: return launch_phases<1, T>(f, r, z, s);
        case 2: return launch_phases<2, T>(f, r, z, s);
        case 4: return launch_phases<4, T>(f, r, z, s);
        case 8: return launch_phases<8, T>(f, r, z, s);
        case 16: return launch_phases<16, T>(f, r, z, s);
        case 32: return launch_phases<32, T>(f, r, z, s);
        default: return fail(HBMC_EINVAL, "bs = %d has no device kernel (1, 2, 4, 8, 16, 32)", f->bs);
    }
}

int apply_impl(const hbmc_factor_s *f, const double *r, double *z, hipStream_t s) {
    return f->precision == HBMC_F64 ? dispatch_bs<double>(f, r, z, s)
                                    : dispatch_bs<float>(f, r, z, s);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI (device side)
// ---------------------------------------------------------------------------
extern "C" int hbmc_factor_upload(hbmc_factor_t *f, void *dev, size_t bytes, void *stream) {
    clear_error();
    if (!f || !dev) return fail(HBMC_EINVAL, "null argument");
    if (bytes < f->image.bytes.size())
        return fail(HBMC_EINVAL, "device buffer too small (%zu < %zu)", bytes, f->image.bytes.size());
    if (reinterpret_cast<uintptr_t>(dev) % 256) return fail(HBMC_EINVAL, "device buffer not 256-byte aligned");
    if (f->bs != 1 && f->bs != 2 && f->bs != 4 && f->bs != 8 && f->bs != 16 && f->bs != 32)
        return fail(HBMC_EINVAL, "bs = %d has no device kernel (1, 2, 4, 8, 16, 32)", f->bs);
    auto s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(dev, f->image.bytes.data(), f->image.bytes.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    f->dev = dev;
    f->dev_bytes = bytes;
    return HBMC_OK;
}

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
    return HBMC_OK;
}

extern "C" int ic0_apply(const hbmc_factor_t *f, const double *r, double *z, int32_t nrhs, void *stream) {
    if (!f || !r || !z) return fail(HBMC_EINVAL, "null argument");
    if (!f->dev) return fail(HBMC_ENOTREADY, "factor not uploaded");
    if (nrhs != 1) return fail(HBMC_EINVAL, "nrhs = %d not supported", nrhs);
    if (r == z) return fail(HBMC_EINVAL, "z must not alias r");
    return apply_impl(f, r, z, static_cast<hipStream_t>(stream));
}

extern "C" int hbmc_spmv(const hbmc_matrix_t *m, const double *x, double *y, int32_t nrhs, void *stream) {
    if (!m || !x || !y) return fail(HBMC_EINVAL, "null argument");
    if (!m->dev) return fail(HBMC_ENOTREADY, "matrix not uploaded");
    if (nrhs != 1) return fail(HBMC_EINVAL, "nrhs = %d not supported", nrhs);
    if (x == y) return fail(HBMC_EINVAL, "y must not alias x");
    hipLaunchKernelGGL(k_spmv, dim3(nblocks(m->n_pad)), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), mat_of(m), x, y);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int hbmc_to_hbmc(const hbmc_factor_t *f, const double *v, double *vb, int32_t nrhs, void *stream) {
    if (!f || !v || !vb) return fail(HBMC_EINVAL, "null argument");
    if (!f->dev) return fail(HBMC_ENOTREADY, "factor not uploaded");
    if (nrhs != 1) return fail(HBMC_EINVAL, "nrhs = %d not supported", nrhs);
    hipLaunchKernelGGL(k_to_hbmc, dim3(nblocks(f->n_pad)), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), f->n_pad, at<int32_t>(f->dev, f->off_iperm), v, vb);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int hbmc_from_hbmc(const hbmc_factor_t *f, const double *vb, double *v, int32_t nrhs, void *stream) {
    if (!f || !v || !vb) return fail(HBMC_EINVAL, "null argument");
    if (!f->dev) return fail(HBMC_ENOTREADY, "factor not uploaded");
    if (nrhs != 1) return fail(HBMC_EINVAL, "nrhs = %d not supported", nrhs);
    hipLaunchKernelGGL(k_from_hbmc, dim3(nblocks(f->n)), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), int64_t(f->n), at<int32_t>(f->dev, f->off_perm), vb, v);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

namespace {
struct Work {
    double *bb, *xb, *r, *z, *p, *q, *partials;
    CgState *st;
};

size_t work_layout(int64_t n_pad, Work *w, void *base) {
    const size_t vec = (size_t(n_pad) * sizeof(double) + 255) & ~size_t(255);
    const size_t part = (size_t(2) * nblocks(n_pad) * sizeof(double) + 255) & ~size_t(255);
    const size_t total = 6 * vec + part + 256;
    if (w && base) {
        auto *b = static_cast<uint8_t *>(base);
        double **v[6] = {&w->bb, &w->xb, &w->r, &w->z, &w->p, &w->q};
        for (int i = 0; i < 6; ++i) *v[i] = reinterpret_cast<double *>(b + i * vec);
        w->partials = reinterpret_cast<double *>(b + 6 * vec);
        w->st = reinterpret_cast<CgState *>(b + 6 * vec + part);
    }
    return total;
}
}  // namespace

extern "C" int iccg_workspace_bytes(const hbmc_factor_t *f, int32_t nrhs, size_t *bytes) {
    if (!f || !bytes) return fail(HBMC_EINVAL, "null argument");
    if (nrhs != 1) return fail(HBMC_EINVAL, "nrhs = %d not supported", nrhs);
    *bytes = work_layout(f->n_pad, nullptr, nullptr);
    return HBMC_OK;
}

extern "C" int iccg_solve(const hbmc_factor_t *f, const hbmc_matrix_t *A, const double *b, double *x,
                          int32_t nrhs, double tol, int32_t maxit, const hbmc_solve_opts_t *opts,
                          hbmc_solve_stats_t *stats, void *work, size_t work_bytes, void *stream) {
    clear_error();
    if (!f || !A || !b || !x || !work) return fail(HBMC_EINVAL, "null argument");
    if (!f->dev) return fail(HBMC_ENOTREADY, "factor not uploaded");
    if (!A->dev) return fail(HBMC_ENOTREADY, "matrix not uploaded");
    if (A->n_pad != f->n_pad || A->n != f->n) return fail(HBMC_EINVAL, "matrix and factor sizes differ");
    if (nrhs != 1) return fail(HBMC_EINVAL, "nrhs = %d not supported", nrhs);
    if (maxit < 0 || !(tol >= 0.0)) return fail(HBMC_EINVAL, "bad tol or maxit");
    Work w{};
    if (work_bytes < work_layout(f->n_pad, nullptr, nullptr)) return fail(HBMC_EINVAL, "workspace too small");
    work_layout(f->n_pad, &w, work);
    const int check = opts && opts->check_every > 0 ? opts->check_every : 1;
    const bool x0_zero = opts && opts->x0_zero;
    auto s = static_cast<hipStream_t>(stream);
    const int64_t n = f->n_pad;
    const unsigned g = nblocks(n);
    const Mat m = mat_of(A);
    const int32_t *iperm = at<int32_t>(f->dev, f->off_iperm);
    const int32_t *perm = at<int32_t>(f->dev, f->off_perm);

    HIP_TRY(hipMemsetAsync(w.st, 0, sizeof(CgState), s));
    hipLaunchKernelGGL(k_to_hbmc, dim3(g), dim3(kBlock), 0, s, n, iperm, b, w.bb);
    if (x0_zero) hipLaunchKernelGGL(k_zero, dim3(g), dim3(kBlock), 0, s, n, w.xb);
    else hipLaunchKernelGGL(k_to_hbmc, dim3(g), dim3(kBlock), 0, s, n, iperm, x, w.xb);
    hipLaunchKernelGGL(k_spmv, dim3(g), dim3(kBlock), 0, s, m, w.xb, w.q);
    hipLaunchKernelGGL(k_cg_init_r, dim3(g), dim3(kBlock), 0, s, n, w.bb, w.q, w.r, w.partials, w.st);
    HIP_TRY(hipGetLastError());
    CgState h{};
    HIP_TRY(hipMemcpyAsync(&h, w.st, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));

    int status = HBMC_OK, iters = 0;
    double res = h.res;
    if (h.bb == 0.0) {
        hipLaunchKernelGGL(k_zero, dim3(g), dim3(kBlock), 0, s, n, w.xb);
        res = 0.0;
    } else if (!(res < tol)) {
        int st = apply_impl(f, w.r, w.z, s);
        if (st) return st;
        hipLaunchKernelGGL(k_cg_init_p, dim3(g), dim3(kBlock), 0, s, n, w.r, w.z, w.p, w.partials, w.st);
        status = HBMC_ENOCONV;
        for (int it = 1; it <= maxit; ++it) {
            hipLaunchKernelGGL(k_cg_spmv, dim3(g), dim3(kBlock), 0, s, m, w.p, w.q, w.partials, w.st);
            hipLaunchKernelGGL(k_cg_xr, dim3(g), dim3(kBlock), 0, s, n, w.p, w.q, w.xb, w.r, w.partials, w.st);
            HIP_TRY(hipGetLastError());
            iters = it;
            if (it % check == 0 || it == maxit) {
                HIP_TRY(hipMemcpyAsync(&h, w.st, sizeof h, hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                res = h.res;
                if (h.flag) { status = HBMC_EBREAKDOWN; break; }
                if (res < tol) { status = HBMC_OK; break; }
            }
            if ((st = apply_impl(f, w.r, w.z, s))) return st;
            hipLaunchKernelGGL(k_cg_rz, dim3(g), dim3(kBlock), 0, s, n, w.r, w.z, w.partials, w.st);
            hipLaunchKernelGGL(k_cg_p, dim3(g), dim3(kBlock), 0, s, n, w.z, w.p, w.st);
        }
    }
    // solution back to the caller's numbering, and the true residual
    hipLaunchKernelGGL(k_from_hbmc, dim3(nblocks(f->n)), dim3(kBlock), 0, s, int64_t(f->n), perm, w.xb, x);
    hipLaunchKernelGGL(k_spmv, dim3(g), dim3(kBlock), 0, s, m, w.xb, w.q);
    hipLaunchKernelGGL(k_resid, dim3(g), dim3(kBlock), 0, s, n, w.bb, w.q, w.partials, w.st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(&h, w.st, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (stats) {
        stats->iters = iters;
        stats->status = status;
        stats->rel_res = res;
        stats->true_rel_res = h.bb > 0.0 ? std::sqrt(h.rz / h.bb) : 0.0;
    }
    if (status == HBMC_EBREAKDOWN) return fail(HBMC_EBREAKDOWN, "CG breakdown: (p, Ap) <= 0 or not finite");
    return status;
}
