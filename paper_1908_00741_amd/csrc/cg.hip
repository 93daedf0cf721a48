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
#include <mutex>
#include <vector>

#include "flow.h"
#include "fold.h"
#include "xcd.h"
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
constexpr int64_t kFinFillRows = 32768;   // largest system whose α finalizer marks the step's vectors empty

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

// Fixed-order total of one system's partials (one per part, or tmul per
// tile), by one workgroup of kFin threads; valid in thread 0.  Each thread
// issues kLoads independent loads before it adds them (in index order), so
// that the latency of the partials' loads is paid once per kLoads, not once
// per partial.
constexpr int kLoads = 16;
__device__ inline double sys_total(const double *part, const int32_t *ranges, int nc, int s, int tmul,
                                   int64_t all = -1) {
    double acc = 0.0;
    if (all >= 0) {   // one system: its partials are all of them, no range table to wait for
        for (int64_t i0 = threadIdx.x; i0 < all; i0 += int64_t(kFin) * kLoads) {
            double v[kLoads];
#pragma unroll
            for (int k = 0; k < kLoads; ++k) v[k] = i0 + k * kFin < all ? part[i0 + k * kFin] : 0.0;
#pragma unroll
            for (int k = 0; k < kLoads; ++k) acc += v[k];
        }
        return block_sum(acc);
    }
    for (int c = 0; c < nc;) {
        // ranges of consecutive colors that meet are summed as one (a single
        // system's partials are one range over all colors)
        const int a = ranges[(s * nc + c) * 2] * tmul;
        int b = ranges[(s * nc + c) * 2 + 1] * tmul;
        for (++c; c < nc && ranges[(s * nc + c) * 2] * tmul == b; ++c) b = ranges[(s * nc + c) * 2 + 1] * tmul;
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

// sys_total of two partial arrays over the same ranges in one pass (loads of
// both in flight together); each total is added in the same order as by
// sys_total, so the results are the same bits.  Valid in thread 0.
__device__ inline void sys_total2(const double *pa, const double *pb, const int32_t *ranges, int nc, int s,
                                  int tmul, double &ta, double &tb, int64_t all = -1) {
    double acc_a = 0.0, acc_b = 0.0;
    if (all >= 0) {   // one system (as sys_total)
        for (int64_t i0 = threadIdx.x; i0 < all; i0 += int64_t(kFin) * kLoads) {
            double va[kLoads], vb[kLoads];
#pragma unroll
            for (int k = 0; k < kLoads; ++k) {
                const bool in = i0 + k * kFin < all;
                va[k] = in ? pa[i0 + k * kFin] : 0.0;
                vb[k] = in ? pb[i0 + k * kFin] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < kLoads; ++k) acc_a += va[k];
#pragma unroll
            for (int k = 0; k < kLoads; ++k) acc_b += vb[k];
        }
        ta = block_sum(acc_a);
        tb = block_sum(acc_b);
        return;
    }
    for (int c = 0; c < nc;) {
        const int a = ranges[(s * nc + c) * 2] * tmul;
        int b = ranges[(s * nc + c) * 2 + 1] * tmul;
        for (++c; c < nc && ranges[(s * nc + c) * 2] * tmul == b; ++c) b = ranges[(s * nc + c) * 2 + 1] * tmul;
        for (int i0 = a + int(threadIdx.x); i0 < b; i0 += kFin * kLoads) {
            double va[kLoads], vb[kLoads];
#pragma unroll
            for (int k = 0; k < kLoads; ++k) {
                const bool in = i0 + k * kFin < b;
                va[k] = in ? pa[i0 + k * kFin] : 0.0;
                vb[k] = in ? pb[i0 + k * kFin] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < kLoads; ++k) acc_a += va[k];
#pragma unroll
            for (int k = 0; k < kLoads; ++k) acc_b += vb[k];
        }
    }
    ta = block_sum(acc_a);
    tb = block_sum(acc_b);
}

// Abar: diagonal plus off-diagonal couplings in 64-row groups of strided
// and indexed slots (a wavefront covers rows of one group).
struct Mat {
    const double *diag;
    const int32_t *soff;
    const int32_t *sbase;
    const uint64_t *smask;
    const double *sval;
    const int32_t *ioff;
    const uint64_t *imask;   // lanes of each indexed slot
    const int64_t *ivoff;    // first packed entry of each indexed slot
    const int32_t *icol;
    const double *ival;
    int64_t n;
    bool fuse_p;             // host side: one right-hand side forms p inside the product
};

__device__ inline uint64_t readlane64(uint64_t v, int lane) {
    const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(v), lane);
    const uint32_t hi = __builtin_amdgcn_readlane(uint32_t(v >> 32), lane);
    return (uint64_t(hi) << 32) | lo;
}

// Sum over the lanes j' of the wavefront with j' = j mod NR (the lanes of
// one right-hand side).
template <int NR>
__device__ inline double rhs_sum(double v) {
#pragma unroll
    for (int o = 32; o >= NR; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Elements of the vector kernels.  Vectors are [n][K] (the K right-hand
// sides of a row adjacent).  A wavefront covers 64/NR consecutive rows (of
// one 64-row group) for NR right-hand sides (group blockIdx.y), lane j taking
// row j / NR and right-hand side j % NR: with NR = K its loads and stores are
// whole contiguous rows.  A part of kPartRows rows is split over SB(NR)
// workgroups (blockIdx.x = part * SB + sub-block), each covering its share in
// ROUNDS(NR) rounds.  In the last part (n need not be a multiple of it) a
// wavefront whose rows all lie past n does no work; in the wavefront that
// holds row n - 1 all lanes stay active (the SpMV broadcasts slot metadata
// from any lane), the lanes past n computing on row n - 1 and storing
// nothing.  Every thread still reaches the workgroup's reduction.
__host__ __device__ constexpr int sub_blocks(int NR) { return NR <= 4 ? 1 : NR / 4; }

// The workgroup's place in the row order.  Workgroups are dealt to the
// chip's 8 XCDs (each with its own L2) in turn; renumbering them so that XCD
// x gets a contiguous range of the row order keeps rows whose neighbours
// overlap (the gathers of the SpMV) in the same L2.
__device__ inline int64_t logical_block() { return xcd_block(blockIdx.x, gridDim.x); }
__host__ __device__ constexpr int rounds(int NR) { return NR / sub_blocks(NR); }

struct Elem {
    int64_t row;     // this lane's row
    int64_t rc;      // the row it reads (row, or n - 1 past the end)
    int64_t g;       // 64-row group (wave-uniform)
    int64_t e;       // element index rc * K + q
    int jc;          // row within the group
    int q;           // right-hand side (clamped to K - 1)
    bool wave_on;    // the wavefront has rows below n
    bool valid;      // row < n and right-hand side < K
};
template <int NR>
__device__ inline Elem elem(int64_t n, int K, int m) {
    if (NR == 1) K = 1;   // one right-hand side: compile-time stride
    constexpr int SB = sub_blocks(NR);
    Elem r;
    const int wave = threadIdx.x >> 6, j = threadIdx.x & 63;
    const int64_t lb = logical_block();
    const int64_t part = lb / SB, sb = lb % SB;
    const int64_t base = part * kPartRows + sb * (kPartRows / SB) + m * (kPartRows / NR) + wave * (kLanes / NR);
    const int q0 = int(blockIdx.y) * NR + j % NR;
    r.row = base + j / NR;
    r.g = __builtin_amdgcn_readfirstlane(int(base >> 6));
    r.jc = int(r.row & 63);
    r.q = q0 < K ? q0 : K - 1;
    r.wave_on = base < n;
    r.valid = r.row < n && q0 < K;
    r.rc = r.row < n ? r.row : n - 1;
    r.e = r.rc * K + r.q;
    return r;
}

// the part of the workgroup (for the system tables)
template <int NR>
__device__ inline int64_t part_of_block() { return logical_block() / sub_blocks(NR); }

// The CG state of the workgroup's part for right-hand side q: with one
// system no table lookup (the state is st[q]).
template <int NR>
__device__ inline const CgState &state_of(const Sys &sys, const CgState *st, int K, int q) {
    return st[(sys.nsys == 1 ? 0 : int64_t(sys.part_sys[part_of_block<NR>()]) * K) + q];
}

// One row of y = A x for one right-hand side, x(i) given by an accessor of
// element indices; all 64 lanes of the wavefront must be active.  The
// group's strided-slot bases and masks (at most 64) come in with one vector
// load, one slot per lane, and are broadcast with readlane.  CHUNKED: the
// packed slots are read in chunks (below), for matrices that hold most of
// their couplings there (fuse_p false).
template <bool CHUNKED, class X>
__device__ inline double spmv_row_with(const Mat &m, X x, const Elem &r, int K) {
    const int64_t g = r.g;
    const int lane = int(threadIdx.x & 63);
    const int jc = r.jc;
    double acc = m.diag[r.rc] * x(r.e);
    const int32_t s0 = m.soff[g], ns = m.soff[g + 1] - s0;
    const int64_t ms = s0 + (lane < ns ? lane : 0);
    const int32_t mbase = m.sbase[ms];
    const uint64_t mmask = m.smask[ms];
    // strided slots kS at a time, all loads of a chunk issued before its
    // products are added in slot order (past the last slot a chunk repeats
    // that slot's loads and adds nothing).  128^3 product: 48.0 us one slot
    // at a time, 46.5 us two, 51.5 us four (the repeated loads and the
    // registers cost more than the overlap gains)
    constexpr int kS = 2;
    for (int k0 = 0; k0 < ns; k0 += kS) {
        double v[kS], xv[kS];
        bool on[kS];
#pragma unroll
        for (int kk = 0; kk < kS; ++kk) {
            const int k = min(k0 + kk, ns - 1);
            const int32_t base = __builtin_amdgcn_readlane(mbase, k);
            on[kk] = k0 + kk < ns && ((readlane64(mmask, k) >> jc) & 1);
            v[kk] = m.sval[(s0 + k) * int64_t(kLanes) + jc];
            xv[kk] = x((base + jc) * int64_t(K) + r.q);
        }
#pragma unroll
        for (int kk = 0; kk < kS; ++kk) acc = on[kk] ? acc + v[kk] * xv[kk] : acc;
    }
    if constexpr (!CHUNKED) {
#pragma unroll 4
        for (int64_t s = m.ioff[g]; s < m.ioff[g + 1]; ++s) {
            // packed slot: lane jc's entry is its rank among the slot's lanes
            const uint64_t mask = m.imask[s];
            const bool on = (mask >> jc) & 1;
            const int64_t e = m.ivoff[s] + (on ? __builtin_popcountll(mask & ((uint64_t(1) << jc) - 1)) : 0);
            const int32_t c = on ? m.icol[e] : -1;
            const double v = m.ival[e];
            const double xv = x((c >= 0 ? c : 0) * int64_t(K) + r.q);
            acc = c >= 0 ? acc + v * xv : acc;
        }
        return acc;
    }
    // packed slots kC at a time: the slots' masks and offsets, then their
    // columns and values, then the gathers, each step issued for the whole
    // chunk (lane jc's entry is its rank among the slot's lanes), so that a
    // row of an unstructured matrix waits for three round trips per chunk,
    // not per slot (1M-point 13-NN product 146 against 140 us).  Past the
    // last slot a chunk repeats that slot's loads (in range) and adds
    // nothing.  The product of the grids (strided slots, p formed on the
    // fly) reads its packed slots one at a time: the chunks' registers cost
    // it occupancy (128^3 product 69 against 48 us with chunks of eight
    // for both kinds of slot).
    constexpr int kC = 8;
    const int64_t i0 = m.ioff[g], i1 = m.ioff[g + 1];
    for (int64_t s0i = i0; s0i < i1; s0i += kC) {
        int32_t c[kC];
        double v[kC], xv[kC];
#pragma unroll
        for (int kk = 0; kk < kC; ++kk) {
            const int64_t s = min(s0i + kk, i1 - 1);
            const uint64_t mask = m.imask[s];
            const bool on = s0i + kk < i1 && ((mask >> jc) & 1);
            const int64_t e = m.ivoff[s] + (on ? __builtin_popcountll(mask & ((uint64_t(1) << jc) - 1)) : 0);
            c[kk] = on ? m.icol[e] : -1;
            v[kk] = m.ival[e];
        }
#pragma unroll
        for (int kk = 0; kk < kC; ++kk) xv[kk] = x((c[kk] >= 0 ? c[kk] : 0) * int64_t(K) + r.q);
#pragma unroll
        for (int kk = 0; kk < kC; ++kk) acc = c[kk] >= 0 ? acc + v[kk] * xv[kk] : acc;
    }
    return acc;
}

// CH: the matrix holds most couplings in packed slots (spmv_row_with)
template <int NR, bool CH>
__global__ void __launch_bounds__(kBlock) k_spmv(Mat m, int K, const double *__restrict__ x,
                                                 double *__restrict__ y) {
    if (NR == 1) K = 1;
#pragma unroll 1
    for (int mm = 0; mm < rounds(NR); ++mm) {
        const Elem r = elem<NR>(m.n, K, mm);
        if (!r.wave_on) continue;
        const double v = spmv_row_with<CH>(m, [=](int64_t i) { return x[i]; }, r, K);
        if (r.valid) y[r.row * K + r.q] = v;
    }
}

// The part's partial sum of each right-hand side of the workgroup's group:
// part[q * np + part].  All threads of the workgroup call it.
template <int NR>
__device__ inline void store_part(double *part, int64_t np, int K, double v) {
    __shared__ double sh[kBlock / kLanes][NR];
    v = rhs_sum<NR>(v);
    const int wave = threadIdx.x >> 6, j = threadIdx.x & 63;
    if (j < NR) sh[wave][j] = v;
    __syncthreads();
    if (int(threadIdx.x) < NR) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < kBlock / kLanes; ++k) t += sh[k][threadIdx.x];
        const int q = int(blockIdx.y) * NR + threadIdx.x;
        if (q < K) part[q * np + logical_block()] = t;
    }
    __syncthreads();
}

// r = b - q; part partials of ||b||^2 and ||r||^2
template <int NR>
__global__ void __launch_bounds__(kBlock) k_init_r(int64_t n, int K, const double *__restrict__ b,
                                                   const double *__restrict__ q,
                                                   double *__restrict__ rv, double *part, int64_t np) {
    if (NR == 1) K = 1;
    double sb = 0.0, sr = 0.0;
#pragma unroll 1
    for (int mm = 0; mm < rounds(NR); ++mm) {
        const Elem r = elem<NR>(n, K, mm);
        if (r.valid) {
            const int64_t e = r.row * K + r.q;
            const double ri = b[e] - q[e];
            rv[e] = ri;
            sb += b[e] * b[e];
            sr += ri * ri;
        }
    }
    store_part<NR>(part, np, K, sb);
    store_part<NR>(part + int64_t(K) * np, np, K, sr);
}

// part partials of (b, x0) and (x0, A x0) (q = A x0), for the scaling of a
// given start vector
template <int NR>
__global__ void __launch_bounds__(kBlock) k_init_dots(int64_t n, int K, const double *__restrict__ b,
                                                      const double *__restrict__ x, const double *__restrict__ q,
                                                      double *part, int64_t np) {
    if (NR == 1) K = 1;
    double bx = 0.0, xq = 0.0;
#pragma unroll 1
    for (int mm = 0; mm < rounds(NR); ++mm) {
        const Elem r = elem<NR>(n, K, mm);
        if (r.valid) {
            const int64_t e = r.row * K + r.q;
            bx += b[e] * x[e];
            xq += x[e] * q[e];
        }
    }
    store_part<NR>(part, np, K, bx);
    store_part<NR>(part + int64_t(K) * np, np, K, xq);
}

// c = (b, x0) / (x0, A x0) per (system, right-hand side), 0 when either is
// not > 0 (start from 0)
__global__ void __launch_bounds__(kFin) k_fin_scale(const double *part, int64_t np, int pmul, int K, Sys sys,
                                                    CgState *st) {
    const int b = blockIdx.x, s = b / K, q = b % K;
    const double bx = sys_total(part + q * np, sys.parts, sys.nc, s, pmul);
    const double xq = sys_total(part + (K + q) * np, sys.parts, sys.nc, s, pmul);
    if (threadIdx.x == 0) st[b].c0 = (bx > 0.0 && xq > 0.0 && isfinite(bx / xq)) ? bx / xq : 0.0;
}

// x0 *= c, q *= c (q = A x0 stays the product of the scaled start)
__global__ void __launch_bounds__(kBlock) k_scale_x(int64_t n_pad, int K, const int32_t *__restrict__ part_sys,
                                                    const CgState *st, double *__restrict__ x,
                                                    double *__restrict__ q) {
    const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (e >= n_pad * K) return;
    const int64_t row = e / K;
    const double c = st[int64_t(part_sys[row / kPartRows]) * K + (e - row * K)].c0;
    x[e] *= c;
    q[e] *= c;
}

// per (system s, right-hand side q) = blockIdx.x = s * K + q: ||b||^2,
// ||r0||^2, the state, and whether it is already done
__global__ void __launch_bounds__(kFin) k_fin_init(const double *part, int64_t np, int pmul, int K, Sys sys,
                                                   CgState *st, double tol, int32_t maxit, double *hist,
                                                   int32_t *ndone, int32_t *alldone) {
    const int b = blockIdx.x, s = b / K, q = b % K;
    const double bb = sys_total(part + q * np, sys.parts, sys.nc, s, pmul);
    const double rr = sys_total(part + (K + q) * np, sys.parts, sys.nc, s, pmul);
    if (threadIdx.x) return;
    CgState &c = st[b];
    c.bb = bb;
    c.rr = rr;
    c.tol = tol;
    c.maxit = maxit;
    c.it = 0;
    c.alpha = 0.0;
    c.beta = 0.0;
    c.res = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    if (hist && b == 0) hist[0] = c.res;
    c.done = (bb == 0.0 || c.res < tol) ? kConverged : (maxit <= 0 ? kMaxIt : kRunning);
    if (!isfinite(c.res)) c.done = kBreakdown;
    if (c.done) count_done(ndone, alldone, sys.nsys * K);
}

// p = z; part partials of (r, z)
template <int NR>
__global__ void __launch_bounds__(kBlock) k_init_p(int64_t n, int K, const double *__restrict__ rv,
                                                   const double *__restrict__ z,
                                                   double *__restrict__ p, double *part, int64_t np) {
    if (NR == 1) K = 1;
    double s = 0.0;
#pragma unroll 1
    for (int mm = 0; mm < rounds(NR); ++mm) {
        const Elem r = elem<NR>(n, K, mm);
        if (r.valid) {
            const int64_t e = r.row * K + r.q;
            p[e] = z[e];
            s += rv[e] * z[e];
        }
    }
    store_part<NR>(part, np, K, s);
}

__global__ void __launch_bounds__(kFin) k_fin_rho(const double *part, int64_t np, int pmul, int K, Sys sys,
                                                  CgState *st) {
    const int b = blockIdx.x, s = b / K, q = b % K;
    const double t = sys_total(part + q * np, sys.parts, sys.nc, s, pmul);
    if (threadIdx.x == 0) { st[b].rho = t; st[b].beta = 0.0; st[b].alpha = 0.0; }
}

// p = z + beta p_old (formed on the fly, also at the columns the row
// couples to), written to p_new; q = A p; part partials of (p, q); and the
// previous iteration's x += alpha p_old at the row (lagged: this kernel
// reads p_old there anyway; k_finish_x adds the last one)
template <int NR>
__global__ void __launch_bounds__(kBlock) k_spmv_dot_p(Mat m, int K, Sys sys, const double *__restrict__ z,
                                                       const double *__restrict__ p_old,
                                                       double *__restrict__ p_new, double *__restrict__ x,
                                                       double *__restrict__ q, double *part, int64_t np,
                                                       const CgState *st, const int32_t *alldone) {
    if (*alldone) return;
    if (NR == 1) K = 1;
    const int q0 = int(blockIdx.y) * NR + int(threadIdx.x & 63) % NR;
    const CgState &c = state_of<NR>(sys, st, K, q0 < K ? q0 : K - 1);
    // a part lies in one system; with one system and one right-hand side its
    // stop is the all-stopped flag above, and the loads need not wait for it
    const bool live = q0 < K && ((NR == 1 && sys.nsys == 1) || !c.done);
    if (NR == 1 && !live) return;                  // workgroup-uniform with one right-hand side
    const double beta = c.beta, alpha = c.alpha;
    auto pv = [=](int64_t i) { return z[i] + beta * p_old[i]; };
    double pq = 0.0;
#pragma unroll 1
    for (int mm = 0; mm < rounds(NR); ++mm) {
        const Elem r = elem<NR>(m.n, K, mm);
        if (!r.wave_on || !__any(live)) continue;
        const double po = p_old[r.e], xo = x[r.e];
        const double pi = z[r.e] + beta * po;
        const double qi = spmv_row_with<false>(m, pv, r, K);
        if (r.valid && live) {
            const int64_t e = r.row * K + r.q;
            x[e] = xo + alpha * po;
            p_new[e] = pi;
            q[e] = qi;
            pq += pi * qi;
        }
    }
    store_part<NR>(part, np, K, pq);
}

// Several right-hand sides: p = z + beta p_old first (elementwise), so that
// the product below gathers p alone at the columns a row couples to (with
// [n][K] vectors the gathered rows are K times longer and miss the caches;
// forming p on the fly would gather z and p_old both).
// With empty (one system, one right-hand side, the substitution in one
// launch), z and p_old, dead once read, are marked kFlowEmpty for the next
// preconditioning step, which computes into them (p_old holding its
// forward values).
template <int NR>
__global__ void __launch_bounds__(kBlock) k_update_p(int64_t n, int K, Sys sys, double *__restrict__ z,
                                                     double *__restrict__ p_old, double *__restrict__ p_new,
                                                     double *__restrict__ x, const CgState *st,
                                                     const int32_t *alldone, bool empty) {
    if (*alldone) return;
    const int q0 = int(blockIdx.y) * NR + int(threadIdx.x & 63) % NR;
    const CgState &c = state_of<NR>(sys, st, K, q0 < K ? q0 : K - 1);
    if (q0 >= K || (!(K == 1 && sys.nsys == 1) && c.done)) return;   // (one system and K = 1: the flag above)
    const double beta = c.beta, alpha = c.alpha;
#pragma unroll 1
    for (int mm = 0; mm < rounds(NR); ++mm) {
        const Elem r = elem<NR>(n, K, mm);
        if (r.valid) {
            const int64_t e = r.row * K + r.q;
            const double po = p_old[e];
            x[e] = x[e] + alpha * po;   // the previous iteration's step (lagged)
            p_new[e] = z[e] + beta * po;
            if (empty) {
                reinterpret_cast<uint64_t *>(z)[e] = kFlowEmpty;
                reinterpret_cast<uint64_t *>(p_old)[e] = kFlowEmpty;
            }
        }
    }
}

// After the loop: the step x += alpha p of each stopped system's last
// iteration, which no direction update applied (none after a breakdown in
// alpha, which leaves alpha = 0).  The direction of iteration k is p[k % 2].
template <int NR>
__global__ void __launch_bounds__(kBlock) k_finish_x(int64_t n, int K, Sys sys, const double *__restrict__ p0,
                                                     const double *__restrict__ p1, double *__restrict__ x,
                                                     const CgState *st) {
    const int q0 = int(blockIdx.y) * NR + int(threadIdx.x & 63) % NR;
    const CgState &c = state_of<NR>(sys, st, K, q0 < K ? q0 : K - 1);
    if (q0 >= K || c.it < 1 || c.alpha == 0.0) return;
    const double alpha = c.alpha;
    const double *p = (c.it & 1) ? p1 : p0;
#pragma unroll 1
    for (int mm = 0; mm < rounds(NR); ++mm) {
        const Elem r = elem<NR>(n, K, mm);
        if (r.valid) {
            const int64_t e = r.row * K + r.q;
            x[e] = x[e] + alpha * p[e];
        }
    }
}

// q = A p for p formed by k_update_p; part partials of (p, q)
template <int NR, bool CH>
__global__ void __launch_bounds__(kBlock) k_spmv_dot(Mat m, int K, Sys sys, const double *__restrict__ p,
                                                     double *__restrict__ q, double *part, int64_t np,
                                                     const CgState *st, const int32_t *alldone) {
    if (*alldone) return;
    const int q0 = int(blockIdx.y) * NR + int(threadIdx.x & 63) % NR;
    const CgState &c = state_of<NR>(sys, st, K, q0 < K ? q0 : K - 1);
    const bool live = q0 < K && ((K == 1 && sys.nsys == 1) || !c.done);
    auto pv = [=](int64_t i) { return p[i]; };
    double pq = 0.0;
#pragma unroll 1
    for (int mm = 0; mm < rounds(NR); ++mm) {
        const Elem r = elem<NR>(m.n, K, mm);
        if (!r.wave_on || !__any(live)) continue;
        const double qi = spmv_row_with<CH>(m, pv, r, K);
        if (r.valid && live) {
            const int64_t e = r.row * K + r.q;
            q[e] = qi;
            pq += p[e] * qi;
        }
    }
    store_part<NR>(part, np, K, pq);
}

// sigma = (p, Ap); alpha = rho / sigma
// With fy (one system, one right-hand side, a small system whose
// preconditioning step runs in one launch after the product that forms p):
// also marks fy and fz ([fn]) empty for that step, in place of a kernel of
// its own, unless the system has stopped (the old direction in fy may then
// hold the last step's direction).
__global__ void __launch_bounds__(kFin) k_fin_alpha(const double *part, int64_t np, int pmul, int K, Sys sys,
                                                    CgState *st, int32_t *ndone, int32_t *alldone,
                                                    double *fy, double *fz, int64_t fn) {
    const int b = blockIdx.x, s = b / K, q = b % K;
    CgState &c = st[b];
    // the stop flag is read beside the partials, not before them
    const int32_t done = c.done;
    const double sigma = sys_total(part + q * np, sys.parts, sys.nc, s, pmul, sys.nsys == 1 ? np : -1);
    if (fy && !done)
        for (int64_t i = threadIdx.x; i < fn; i += blockDim.x) {
            reinterpret_cast<uint64_t *>(fy)[i] = kFlowEmpty;
            reinterpret_cast<uint64_t *>(fz)[i] = kFlowEmpty;
        }
    if (threadIdx.x || done) return;
    c.sigma = sigma;
    if (!(sigma > 0.0) || !isfinite(sigma)) {
        c.done = kBreakdown;
        c.alpha = 0.0;   // no x update pending
        c.it += 1;
        count_done(ndone, alldone, sys.nsys * K);
        return;
    }
    c.alpha = c.rho / sigma;
}

// After the preconditioning step: ||r||^2 and (r, z) from the partials per
// (tile, sub-tile) (tmul sub-tiles per tile); one more iteration done;
// stopping test ||r|| / ||b|| < tol; then beta = rho' / rho, rho = rho' for
// the next direction.
__global__ void __launch_bounds__(kFin) k_fin_rr_beta(const double *part_rr, const double *part_rz,
                                                      int64_t ptiles, int tmul, int K, Sys sys,
                                                      CgState *st, double *hist, int32_t hist_len,
                                                      int32_t *ndone, int32_t *alldone) {
    const int b = blockIdx.x, s = b / K, q = b % K;
    CgState &c = st[b];
    const int32_t done = c.done;   // read beside the partials, not before them
    double rr, rz;
    sys_total2(part_rr + q * ptiles, part_rz + q * ptiles, sys.tiles, sys.nc, s, tmul, rr, rz,
               sys.nsys == 1 ? ptiles : -1);
    if (threadIdx.x || done) return;
    c.rr = rr;
    c.it += 1;
    c.res = sqrt(rr / c.bb);
    if (hist && b == 0 && c.it < hist_len) hist[c.it] = c.res;
    if (!isfinite(c.res)) c.done = kBreakdown;
    else if (c.res < c.tol) c.done = kConverged;
    else if (c.it >= c.maxit) c.done = kMaxIt;
    else {
        c.beta = rz / c.rho;
        c.rho = rz;
    }
    if (c.done) count_done(ndone, alldone, sys.nsys * K);
}

// part partials of ||b - q||^2 (true residual)
template <int NR>
__global__ void __launch_bounds__(kBlock) k_resid(int64_t n, int K, const double *__restrict__ b,
                                                  const double *__restrict__ q, double *part, int64_t np) {
    if (NR == 1) K = 1;
    double s = 0.0;
#pragma unroll 1
    for (int mm = 0; mm < rounds(NR); ++mm) {
        const Elem r = elem<NR>(n, K, mm);
        if (r.valid) { const int64_t e = r.row * K + r.q; const double d = b[e] - q[e]; s += d * d; }
    }
    store_part<NR>(part, np, K, s);
}

__global__ void __launch_bounds__(kFin) k_fin_resid(const double *part, int64_t np, int pmul, int K, Sys sys,
                                                    double *out) {
    const int b = blockIdx.x, s = b / K, q = b % K;
    const double t = sys_total(part + q * np, sys.parts, sys.nc, s, pmul);
    if (threadIdx.x == 0) out[b] = t;
}

// r = b - A x (the residual of a smoothing step)
template <int NR, bool CH>
__global__ void __launch_bounds__(kBlock) k_smooth_r(Mat m, int K, const double *__restrict__ b,
                                                     const double *__restrict__ x, double *__restrict__ r) {
    if (NR == 1) K = 1;
#pragma unroll 1
    for (int mm = 0; mm < rounds(NR); ++mm) {
        const Elem e = elem<NR>(m.n, K, mm);
        if (!e.wave_on) continue;
        const double ax = spmv_row_with<CH>(m, [=](int64_t i) { return x[i]; }, e, K);
        if (e.valid) r[e.row * K + e.q] = b[e.row * K + e.q] - ax;
    }
}

// element-wise kernels over [rows][K]
__global__ void __launch_bounds__(kBlock) k_axpy(int64_t n, double c, const double *__restrict__ z,
                                                 double *__restrict__ x) {
    const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (e < n) x[e] += c * z[e];
}

__global__ void __launch_bounds__(kBlock) k_to_hbmc(int64_t n_pad, int K, const int32_t *__restrict__ iperm,
                                                    const double *__restrict__ v,
                                                    double *__restrict__ vb) {
    const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (e >= n_pad * K) return;
    const int64_t row = e / K;
    const int32_t i = iperm[row];
    vb[e] = i >= 0 ? v[int64_t(i) * K + (e - row * K)] : 0.0;
}

__global__ void __launch_bounds__(kBlock) k_from_hbmc(int64_t n, int K, const int32_t *__restrict__ perm,
                                                      const double *__restrict__ vb,
                                                      double *__restrict__ v) {
    const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (e >= n * K) return;
    const int64_t i = e / K;
    v[e] = vb[int64_t(perm[i]) * K + (e - i * K)];
}

// x = 0 for the (system, right-hand side) pairs whose right-hand side is zero
__global__ void __launch_bounds__(kBlock) k_zero_b0(int64_t n_pad, int K, const int32_t *__restrict__ part_sys,
                                                    const CgState *st, double *__restrict__ x) {
    const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (e >= n_pad * K) return;
    const int64_t row = e / K;
    if (st[int64_t(part_sys[row / kPartRows]) * K + (e - row * K)].bb == 0.0) x[e] = 0.0;
}

__global__ void __launch_bounds__(kBlock) k_zero(int64_t n, double *__restrict__ v) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) v[i] = 0.0;
}

// the solve's counters and flags zero; the words that carry alpha unpublished
__global__ void k_init_flags(int32_t *ints, uint64_t *words) {
    if (threadIdx.x < 4) ints[threadIdx.x] = 0;
    for (int i = int(threadIdx.x); i < kFoldWords; i += int(blockDim.x)) words[i] = kNotYet;
}

template <class P>
P *at(void *base, size_t off) {
    return reinterpret_cast<P *>(static_cast<uint8_t *>(base) + off);
}

Mat mat_of(const hbmc_matrix_s *m) {
    const PackedOffsets &o = m->offs;
    return Mat{at<double>(m->dev, m->off_diag), at<int32_t>(m->dev, o.soff),
               at<int32_t>(m->dev, o.sbase), at<uint64_t>(m->dev, o.smask),
               at<double>(m->dev, o.sval), at<int32_t>(m->dev, o.ioff),
               at<uint64_t>(m->dev, o.imask), at<int64_t>(m->dev, o.ivoff),
               at<int32_t>(m->dev, o.icol), at<double>(m->dev, o.ival),
               m->n_pad, m->fuse_p};
}

Sys sys_of(const hbmc_factor_s *f) {
    return Sys{at<int32_t>(f->dev, f->off_part_sys), at<int32_t>(f->dev, f->off_sys_tiles),
               at<int32_t>(f->dev, f->off_sys_parts), f->nc, f->nsys};
}

std::atomic<uint64_t> g_uid{1};

// Right-hand sides per wavefront of the vector kernels for K right-hand
// sides: K rounded up to a power of two, at most 64 (1 for one).
inline int vec_nr(int K) {
    if (K == 1) return 1;
    int nr = 4;
    while (nr < K && nr < 64) nr *= 2;
    return nr;
}

// Workspace, for K right-hand sides: b, x, r, z, p (two, used in turn), q
// in HBMC order ([n_pad][K]); partial sums per part (two slots) and per
// (tile, sub-tile) (two); the CG state of each (system, right-hand side);
// the stopped counter and the all-stopped flag; the true residuals; the
// residual history of system 0, right-hand side 0.
struct Work {
    double *bb, *xb, *r, *z, *p[2], *q, *part_g, *part_rr, *part_rz, *resid, *hist;
    CgState *st;
    int32_t *ndone, *alldone;
    int32_t *err;      // a wait inside a kernel ran past its time limit (1: alpha, 2: substitution)
    uint64_t *awords;  // [kFoldWords] alpha published inside a kernel (both parities, replicated)
    int64_t np;        // part partial slots per right-hand side (parts * pmul)
    int32_t pmul;      // sub-blocks per part of the vector kernels
    int64_t ptiles;    // tile partial slots per right-hand side
    int32_t K, nr;     // right-hand sides; right-hand sides per wavefront
    int32_t hist_len;
};

constexpr int32_t kHistLen = 65536;
constexpr int kMaxTile = 16;   // largest right-hand-side tile

// Byte layout of the workspace for K right-hand sides (tile partials sized
// for the largest tile, so that the tile may change after allocation).
size_t work_layout(const hbmc_factor_s *f, int K, Work *w, void *base) {
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const int64_t np = (f->n_pad + kPartRows - 1) / kPartRows;
    const int64_t tmul = K == 1 ? 1 : kMaxTile;
    const int64_t ptiles = f->tile_base[f->nc] * tmul;
    const size_t vec = up(size_t(f->n_pad) * K * sizeof(double));
    const size_t pg = up(size_t(2) * K * np * sub_blocks(64) * sizeof(double));
    const size_t tp = up(size_t(ptiles) * K * sizeof(double));
    const size_t sts = up(size_t(f->nsys) * K * sizeof(CgState));
    const size_t res = up(size_t(f->nsys) * K * sizeof(double));
    const size_t hist = size_t(kHistLen) * sizeof(double);
    const size_t total = hist + 7 * vec + pg + 2 * tp + sts + 256 + kFoldWords * sizeof(uint64_t) + res;
    if (w && base) {
        auto *b = static_cast<uint8_t *>(base);
        w->hist = reinterpret_cast<double *>(b);   // first: its place does not depend on K
        b += hist;
        double **v[7] = {&w->bb, &w->xb, &w->r, &w->z, &w->p[0], &w->p[1], &w->q};
        for (int i = 0; i < 7; ++i) *v[i] = reinterpret_cast<double *>(b + i * vec);
        size_t a = 7 * vec;
        w->part_g = reinterpret_cast<double *>(b + a); a += pg;
        w->part_rr = reinterpret_cast<double *>(b + a); a += tp;
        w->part_rz = reinterpret_cast<double *>(b + a); a += tp;
        w->st = reinterpret_cast<CgState *>(b + a); a += sts;
        w->ndone = reinterpret_cast<int32_t *>(b + a);
        w->alldone = w->ndone + 1;
        w->err = w->ndone + 2;
        a += 256;
        w->awords = reinterpret_cast<uint64_t *>(b + a);
        a += kFoldWords * sizeof(uint64_t);
        w->resid = reinterpret_cast<double *>(b + a);
        w->hist_len = kHistLen;
        w->pmul = sub_blocks(vec_nr(K));
        w->np = np * w->pmul;
        w->K = K;
        w->nr = rhs_tile(f, K);
        w->ptiles = f->tile_base[f->nc] * w->nr;
    }
    return total;
}

// Launches a vector kernel template on the workgroups (parts of n_pad rows
// times sub-blocks, groups of NR right-hand sides).
#define VEC_LAUNCH(kernel, n_pad, K, s, ...)                                                      \
    do {                                                                                          \
        const int nr_ = vec_nr(K);                                                                \
        const unsigned px_ = unsigned(((n_pad) + kPartRows - 1) / kPartRows * sub_blocks(nr_));   \
        const dim3 g_(px_, unsigned(((K) + nr_ - 1) / nr_));                                      \
        switch (nr_) {                                                                            \
            case 1: hipLaunchKernelGGL(kernel<1>, g_, dim3(kBlock), 0, s, __VA_ARGS__); break;    \
            case 4: hipLaunchKernelGGL(kernel<4>, g_, dim3(kBlock), 0, s, __VA_ARGS__); break;    \
            case 8: hipLaunchKernelGGL(kernel<8>, g_, dim3(kBlock), 0, s, __VA_ARGS__); break;    \
            case 16: hipLaunchKernelGGL(kernel<16>, g_, dim3(kBlock), 0, s, __VA_ARGS__); break;  \
            case 32: hipLaunchKernelGGL(kernel<32>, g_, dim3(kBlock), 0, s, __VA_ARGS__); break;  \
            default: hipLaunchKernelGGL(kernel<64>, g_, dim3(kBlock), 0, s, __VA_ARGS__); break;  \
        }                                                                                         \
    } while (0)

// VEC_LAUNCH for the product kernels, with the packed-slot form chosen by
// the matrix (chunks for matrices held mostly in packed slots, the others
// one slot at a time: the chunks' registers would cost them occupancy).
#define VEC_LAUNCH_MAT(kernel, mat, n_pad, K, s, ...)                                              \
    do {                                                                                          \
        const int nr_ = vec_nr(K);                                                                \
        const bool ch_ = !(mat).fuse_p;                                                           \
        const unsigned px_ = unsigned(((n_pad) + kPartRows - 1) / kPartRows * sub_blocks(nr_));   \
        const dim3 g_(px_, unsigned(((K) + nr_ - 1) / nr_));                                      \
        switch (nr_) {                                                                            \
            case 1: if (ch_) hipLaunchKernelGGL((kernel<1, true>), g_, dim3(kBlock), 0, s, __VA_ARGS__);     \
                    else hipLaunchKernelGGL((kernel<1, false>), g_, dim3(kBlock), 0, s, __VA_ARGS__); break;  \
            case 4: if (ch_) hipLaunchKernelGGL((kernel<4, true>), g_, dim3(kBlock), 0, s, __VA_ARGS__);     \
                    else hipLaunchKernelGGL((kernel<4, false>), g_, dim3(kBlock), 0, s, __VA_ARGS__); break;  \
            case 8: if (ch_) hipLaunchKernelGGL((kernel<8, true>), g_, dim3(kBlock), 0, s, __VA_ARGS__);     \
                    else hipLaunchKernelGGL((kernel<8, false>), g_, dim3(kBlock), 0, s, __VA_ARGS__); break;  \
            case 16: if (ch_) hipLaunchKernelGGL((kernel<16, true>), g_, dim3(kBlock), 0, s, __VA_ARGS__);   \
                     else hipLaunchKernelGGL((kernel<16, false>), g_, dim3(kBlock), 0, s, __VA_ARGS__); break;\
            case 32: if (ch_) hipLaunchKernelGGL((kernel<32, true>), g_, dim3(kBlock), 0, s, __VA_ARGS__);   \
                     else hipLaunchKernelGGL((kernel<32, false>), g_, dim3(kBlock), 0, s, __VA_ARGS__); break;\
            default: if (ch_) hipLaunchKernelGGL((kernel<64, true>), g_, dim3(kBlock), 0, s, __VA_ARGS__);   \
                     else hipLaunchKernelGGL((kernel<64, false>), g_, dim3(kBlock), 0, s, __VA_ARGS__); break;\
        }                                                                                         \
    } while (0)

inline int grid_elems(int64_t n) { return int(std::max<int64_t>(1, (n + kBlock - 1) / kBlock)); }

// One CG iteration (everything after the first preconditioning step); the
// direction is read from p[parity] and written to p[1 - parity].
//   q = A p, p = z + beta p_old, the previous iteration's x += alpha p_old (two kernels for several
//   right-hand sides or a mostly indexed matrix)  |  alpha = rho / (p, q)  |
//   r -= alpha q, z = M^-1 r, partials of ||r||^2 and (r, z)  |  stopping test, beta
int enqueue_iteration(const hbmc_factor_s *f, const Mat &m, const Work &w, hipStream_t s,
                      bool history, int parity) {
    const Sys sys = sys_of(f);
    const int K = w.K;
    const unsigned nst = unsigned(f->nsys) * K;
    double *p_old = w.p[parity], *p_new = w.p[1 - parity];
    // The row kernel's phases in one launch (flow.h): p_old, dead once the
    // direction update has read it (the lagged x update included), holds
    // the forward values.  The update marks it and z empty where it streams
    // them anyway; after the product that forms p itself a kernel does.
    const bool flow = flow_ok(f, K);
    const bool fused = K == 1 && m.fuse_p;
    // small systems: the α finalizer marks them, one launch fewer per
    // iteration (64x64 grid, 64 iterations: 2.95 -> 2.88 ms eager, 1.62 ->
    // 1.55 ms replayed as a graph; a launch per phase: 3.07 / 1.63 ms)
    const bool fin_fill = flow && fused && f->n_pad <= kFinFillRows;
    const Flow fl{p_old, w.err, fused && !fin_fill, false};
    if (fused) {
        VEC_LAUNCH(k_spmv_dot_p, f->n_pad, K, s, m, K, sys, w.z, p_old, p_new, w.xb, w.q, w.part_g, w.np, w.st,
                   w.alldone);
    } else {
        VEC_LAUNCH(k_update_p, f->n_pad, K, s, f->n_pad, K, sys, w.z, p_old, p_new, w.xb, w.st, w.alldone, flow);
        VEC_LAUNCH_MAT(k_spmv_dot, m, f->n_pad, K, s, m, K, sys, p_new, w.q, w.part_g, w.np, w.st, w.alldone);
    }
    ApplyCg cg{w.q, w.r, w.st, at<int32_t>(f->dev, f->off_tile_sys), w.part_rr, w.part_rz,
               nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr, nullptr};
    if (K == 1 && f->nsys == 1 && !use_rows(f, f->bs, 1, 1)) {
        // one system, one right-hand side, one wavefront per tile: alpha is
        // computed by the first phase of the preconditioning step (fold.h)
        // instead of a kernel of its own (128^3, bs 8: 6.7 us less per
        // iteration).  Not with one workgroup per tile, where it measured
        // slower (1M-point 13-NN graph: 134.1 against 137.3 ms per solve).
        cg.stw = w.st;
        cg.fpart = w.part_g;
        cg.fnp = w.np;
        cg.fwords = w.awords;
        cg.fparity = parity;
        cg.ferr = w.err;
        cg.ndone = w.ndone;
        cg.alldone = w.alldone;
    } else {
        hipLaunchKernelGGL(k_fin_alpha, dim3(nst), dim3(kFin), 0, s, w.part_g, w.np, w.pmul, K, sys, w.st, w.ndone,
                           w.alldone, fin_fill ? p_old : nullptr, fin_fill ? w.z : nullptr, f->n_pad);
        HIP_TRY(hipGetLastError());
    }
    int st = apply_launch(f, w.r, w.z, s, w.alldone, &cg, K, false, flow ? &fl : nullptr);
    if (st) return st;
    hipLaunchKernelGGL(k_fin_rr_beta, dim3(nst), dim3(kFin), 0, s, w.part_rr, w.part_rz, w.ptiles, w.nr, K,
                       sys, w.st, history ? w.hist : nullptr, w.hist_len, w.ndone, w.alldone);
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
        if (gph.matrix_uid == A->uid && gph.work == work && gph.iters == key && gph.K == w.K &&
            gph.nr == w.nr) {
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
    if (st) { if (graph) (void)hipGraphDestroy(graph); return st; }
    if (e != hipSuccess) return fail(HBMC_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(HBMC_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    f->graphs.push_back({A->uid, work, key, w.K, w.nr, exec});
    *out = exec;
    return HBMC_OK;
}

int check_ready(const hbmc_factor_s *f, int32_t nrhs) {
    if (!f) return fail(HBMC_EINVAL, "null handle");
    if (!f->dev) return fail(HBMC_ENOTREADY, "factor not uploaded");
    if (nrhs < 1) return fail(HBMC_EINVAL, "nrhs = %d", nrhs);
    return HBMC_OK;
}

}  // namespace

uint64_t hbmc::next_uid() { return g_uid.fetch_add(1); }

void hbmc::release_graphs(hbmc_factor_s *f) {
    for (auto &gph : f->graphs) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(gph.exec));
    f->graphs.clear();
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int hbmc_matrix_upload(hbmc_matrix_t *m, void *dev, size_t bytes, void *stream) {
    clear_error();
    if (!m || !dev) return fail(HBMC_EINVAL, "null argument");
    if (m->device_built) return fail(HBMC_EINVAL, "a matrix built on the device is already uploaded");
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
    if (nrhs < 1) return fail(HBMC_EINVAL, "nrhs = %d", nrhs);
    if (x == y) return fail(HBMC_EINVAL, "y must not alias x");
    const int K = nrhs;
    const Mat mm = mat_of(m);
    VEC_LAUNCH_MAT(k_spmv, mm, m->n_pad, K, static_cast<hipStream_t>(stream), mm, K, x, y);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int hbmc_to_hbmc(const hbmc_factor_t *f, const double *v, double *vb, int32_t nrhs, void *stream) {
    int st = check_ready(f, nrhs);
    if (st) return st;
    if (!v || !vb) return fail(HBMC_EINVAL, "null argument");
    hipLaunchKernelGGL(k_to_hbmc, dim3(grid_elems(f->n_pad * nrhs)), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), f->n_pad, nrhs, at<int32_t>(f->dev, f->off_iperm), v, vb);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int hbmc_from_hbmc(const hbmc_factor_t *f, const double *vb, double *v, int32_t nrhs, void *stream) {
    int st = check_ready(f, nrhs);
    if (st) return st;
    if (!v || !vb) return fail(HBMC_EINVAL, "null argument");
    hipLaunchKernelGGL(k_from_hbmc, dim3(grid_elems(int64_t(f->n) * nrhs)), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), int64_t(f->n), nrhs, at<int32_t>(f->dev, f->off_perm),
                       vb, v);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int iccg_workspace_bytes(const hbmc_factor_t *f, int32_t nrhs, size_t *bytes) {
    if (!f || !bytes) return fail(HBMC_EINVAL, "null argument");
    if (nrhs < 1) return fail(HBMC_EINVAL, "nrhs = %d", nrhs);
    *bytes = work_layout(f, nrhs, nullptr, nullptr);
    return HBMC_OK;
}

namespace {

// Checks shared by the solve entry points.
int solve_args(const hbmc_factor_s *f, const hbmc_matrix_t *A, const double *b, double *x, int32_t nrhs,
               double tol, int32_t maxit) {
    if (!f || !A || !b || !x) return fail(HBMC_EINVAL, "null argument");
    if (!f->dev) return fail(HBMC_ENOTREADY, "factor not uploaded");
    if (!A->dev) return fail(HBMC_ENOTREADY, "matrix not uploaded");
    if (A->n_pad != f->n_pad || A->n != f->n) return fail(HBMC_EINVAL, "matrix and factor sizes differ");
    if (nrhs < 1) return fail(HBMC_EINVAL, "nrhs = %d", nrhs);
    if (maxit < 0 || !(tol >= 0.0)) return fail(HBMC_EINVAL, "bad tol or maxit");
    return HBMC_OK;
}

// The solve on a checked workspace of at least work_layout(f, nrhs) bytes.
// Allocates nothing on the device or the host unless use_graph is set (the
// graph is instantiated on first use).
int solve_in(hbmc_factor_s *f, const hbmc_matrix_t *A, const double *b, double *x, int32_t nrhs, double tol,
             int32_t maxit, const hbmc_solve_opts_t *opts, hbmc_solve_stats_t *stats, void *work,
             void *stream) {
    const int K = nrhs;
    Work w{};
    work_layout(f, K, &w, work);
    const bool x0_zero = opts && opts->x0_zero;
    const bool x0_scale = !x0_zero && opts && opts->x0_scale;
    const bool use_graph = opts && opts->use_graph;
    const bool history = opts && opts->record_history;
    int check = opts && opts->check_every > 0 ? opts->check_every : (use_graph ? 16 : 1);
    if (use_graph) check = (check + 1) & ~1;   // graphs hold whole pairs of iterations
    auto s = static_cast<hipStream_t>(stream);
    const int64_t n = f->n_pad;
    const int ge = grid_elems(n * K);
    const Mat m = mat_of(A);
    const Sys sys = sys_of(f);
    const int32_t nst = f->nsys * K;
    const int32_t *iperm = at<int32_t>(f->dev, f->off_iperm);
    const int32_t *perm = at<int32_t>(f->dev, f->off_perm);

    hipLaunchKernelGGL(k_init_flags, dim3(1), dim3(256), 0, s, w.ndone, w.awords);
    hipLaunchKernelGGL(k_to_hbmc, dim3(ge), dim3(kBlock), 0, s, n, K, iperm, b, w.bb);
    if (x0_zero) hipLaunchKernelGGL(k_zero, dim3(ge), dim3(kBlock), 0, s, n * K, w.xb);
    else hipLaunchKernelGGL(k_to_hbmc, dim3(ge), dim3(kBlock), 0, s, n, K, iperm, x, w.xb);
    VEC_LAUNCH_MAT(k_spmv, m, n, K, s, m, K, w.xb, w.q);
    if (x0_scale) {
        VEC_LAUNCH(k_init_dots, n, K, s, n, K, w.bb, w.xb, w.q, w.part_g, w.np);
        hipLaunchKernelGGL(k_fin_scale, dim3(nst), dim3(kFin), 0, s, w.part_g, w.np, w.pmul, K, sys, w.st);
        hipLaunchKernelGGL(k_scale_x, dim3(ge), dim3(kBlock), 0, s, n, K, sys.part_sys, w.st, w.xb, w.q);
    }
    VEC_LAUNCH(k_init_r, n, K, s, n, K, w.bb, w.q, w.r, w.part_g, w.np);
    hipLaunchKernelGGL(k_fin_init, dim3(nst), dim3(kFin), 0, s, w.part_g, w.np, w.pmul, K, sys, w.st, tol, maxit,
                       history ? w.hist : nullptr, w.ndone, w.alldone);
    HIP_TRY(hipGetLastError());
    int32_t hd[3] = {0, 0, 0};   // stopped count, all-stopped flag, wait time-out
    HIP_TRY(hipMemcpyAsync(hd, w.ndone, sizeof hd, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));

    if (hd[0] < nst) {
        // the first direction is written after this step, the second in
        // the first iteration: p[1] is free to hold the forward values
        const Flow fl{w.p[1], w.err, true, false};
        int st = apply_launch(f, w.r, w.z, s, nullptr, nullptr, K, false, &fl);
        if (st) return st;
        VEC_LAUNCH(k_init_p, n, K, s, n, K, w.r, w.z, w.p[0], w.part_g, w.np);
        hipLaunchKernelGGL(k_fin_rho, dim3(nst), dim3(kFin), 0, s, w.part_g, w.np, w.pmul, K, sys, w.st);
        HIP_TRY(hipGetLastError());
        hipGraphExec_t exec = nullptr;
        if (use_graph && (st = get_graph(f, A, m, w, work, check, history, &exec))) return st;
        int parity = 0;
        while (hd[0] < nst) {
            if (use_graph) HIP_TRY(hipGraphLaunch(exec, s));
            else
                for (int k = 0; k < check; ++k, parity ^= 1)
                    if ((st = enqueue_iteration(f, m, w, s, history, parity))) return st;
            HIP_TRY(hipMemcpyAsync(hd, w.ndone, sizeof hd, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (hd[2])
                return fail(HBMC_EHIP, "a wait inside a kernel timed out (%s)",
                            hd[2] & 2 ? "a value of the substitution" : "alpha");
        }
    }
    // the last step of each system; pairs with b = 0 get x = 0; the
    // solution back to the caller's numbering; the true residuals
    VEC_LAUNCH(k_finish_x, n, K, s, n, K, sys, w.p[0], w.p[1], w.xb, w.st);
    hipLaunchKernelGGL(k_zero_b0, dim3(ge), dim3(kBlock), 0, s, n, K, sys.part_sys, w.st, w.xb);
    hipLaunchKernelGGL(k_from_hbmc, dim3(grid_elems(int64_t(f->n) * K)), dim3(kBlock), 0, s, int64_t(f->n), K,
                       perm, w.xb, x);
    VEC_LAUNCH_MAT(k_spmv, m, n, K, s, m, K, w.xb, w.q);
    VEC_LAUNCH(k_resid, n, K, s, n, K, w.bb, w.q, w.part_g, w.np);
    hipLaunchKernelGGL(k_fin_resid, dim3(nst), dim3(kFin), 0, s, w.part_g, w.np, w.pmul, K, sys, w.resid);
    HIP_TRY(hipGetLastError());
    // states and true residuals back in fixed-size chunks
    constexpr int kChunk = 64;
    CgState hs[kChunk];
    double rt[kChunk];
    int status = HBMC_OK;
    for (int32_t k0 = 0; k0 < nst; k0 += kChunk) {
        const int32_t nk = std::min<int32_t>(kChunk, nst - k0);
        HIP_TRY(hipMemcpyAsync(hs, w.st + k0, nk * sizeof(CgState), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(rt, w.resid + k0, nk * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int32_t i = 0; i < nk; ++i) {
            const int sk = hs[i].done == kConverged ? HBMC_OK
                           : hs[i].done == kBreakdown ? HBMC_EBREAKDOWN : HBMC_ENOCONV;
            if (sk == HBMC_EBREAKDOWN) status = HBMC_EBREAKDOWN;
            else if (sk == HBMC_ENOCONV && status == HBMC_OK) status = HBMC_ENOCONV;
            if (stats) {
                hbmc_solve_stats_t &o = stats[k0 + i];
                o.iters = hs[i].it;
                o.status = sk;
                o.rel_res = hs[i].res;
                o.true_rel_res = hs[i].bb > 0.0 ? std::sqrt(rt[i] / hs[i].bb) : 0.0;
                o.x0_scale = x0_zero ? 0.0 : (x0_scale ? hs[i].c0 : 1.0);
            }
        }
    }
    if (status == HBMC_EBREAKDOWN) return fail(HBMC_EBREAKDOWN, "CG breakdown: (p, Ap) <= 0 or not finite");
    if (status == HBMC_ENOCONV) fail(HBMC_ENOCONV, "maxit = %d reached", maxit);
    return status;
}

}  // namespace

extern "C" int iccg_solve(const hbmc_factor_t *fc, const hbmc_matrix_t *A, const double *b, double *x,
                          int32_t nrhs, double tol, int32_t maxit, const hbmc_solve_opts_t *opts,
                          hbmc_solve_stats_t *stats, void *work, size_t work_bytes, void *stream) {
    clear_error();
    auto *f = const_cast<hbmc_factor_s *>(fc);   // the graph cache is mutable state
    int st = solve_args(f, A, b, x, nrhs, tol, maxit);
    if (st) return st;
    if (!work) return fail(HBMC_EINVAL, "null argument");
    if (work_bytes < work_layout(f, nrhs, nullptr, nullptr)) return fail(HBMC_EINVAL, "workspace too small");
    return solve_in(f, A, b, x, nrhs, tol, maxit, opts, stats, work, stream);
}

// ---------------------------------------------------------------------------
// iccg_solve without allocation: the workspace is a static device array
// ---------------------------------------------------------------------------
namespace {

// The workspace of iccg_solve_noalloc.  Host code never uses this name as an
// address: hipGetSymbolAddress gives each device's copy, kept in g_scratch.
__device__ __align__(256) unsigned char scratch[HBMC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// The current device's copy of scratch (looked up once per device).
int scratch_of_device(void **out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(HBMC_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HBMC_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return HBMC_OK;
}

}  // namespace

extern "C" int iccg_solve_noalloc(const hbmc_factor_t *fc, const hbmc_matrix_t *A, const double *b, double *x,
                                  int32_t nrhs, double tol, int32_t maxit, const hbmc_solve_opts_t *opts,
                                  hbmc_solve_stats_t *stats, void *stream) {
    clear_error();
    auto *f = const_cast<hbmc_factor_s *>(fc);
    int st = solve_args(f, A, b, x, nrhs, tol, maxit);
    if (st) return st;
    if (opts && opts->use_graph) return fail(HBMC_EINVAL, "use_graph: instantiating a graph allocates");
    if (opts && opts->record_history)
        return fail(HBMC_EINVAL, "record_history: the history would stay in the library's scratch");
    const size_t need = work_layout(f, nrhs, nullptr, nullptr);
    if (need > size_t(HBMC_NOALLOC_SCRATCH_BYTES))
        return fail(HBMC_EINVAL, "the solve needs %zu bytes of workspace; the static scratch holds %zu "
                    "(use iccg_solve with a caller workspace)", need, size_t(HBMC_NOALLOC_SCRATCH_BYTES));
    void *work = nullptr;
    if ((st = scratch_of_device(&work))) return st;
    return solve_in(f, A, b, x, nrhs, tol, maxit, opts, stats, work, stream);
}

// Residual history of system 0, right-hand side 0, from the last iccg_solve
// that ran with record_history on this workspace: hist[k] = ||r_k|| / ||b||
// (synchronous copy to host memory).  The history is at the start of the
// workspace, whatever the number of right-hand sides.
extern "C" int iccg_history(const void *work, size_t work_bytes, const hbmc_factor_t *f, double *hist,
                            int32_t count, void *stream) {
    if (!work || !f || !hist || count < 0) return fail(HBMC_EINVAL, "null argument");
    if (count > kHistLen) return fail(HBMC_EINVAL, "history holds at most %d entries", kHistLen);
    if (work_bytes < size_t(kHistLen) * sizeof(double)) return fail(HBMC_EINVAL, "workspace too small");
    auto s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(hist, work, size_t(count) * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return HBMC_OK;
}

// ---------------------------------------------------------------------------
// Smoothing (Section 2: the GS and SOR iterations are substitutions with the
// triangles of A).  One step is  x <- x + c M^-1 (b - A x):  with the SSOR
// splitting (ssor_factor) and both substitutions it is one forward and one
// backward SOR sweep (c = 2 - omega; symmetric Gauss-Seidel at omega = 1),
// with the forward substitution alone one forward SOR sweep (c = 1); with an
// IC(0) factor it is the IC smoother (c = 1).
// ---------------------------------------------------------------------------
namespace {
size_t smooth_vec_bytes(const hbmc_factor_s *f, int K) {
    return (size_t(f->n_pad) * K * sizeof(double) + 255) & ~size_t(255);
}
}  // namespace

extern "C" int hbmc_smooth_workspace_bytes(const hbmc_factor_t *f, int32_t nrhs, size_t *bytes) {
    if (!f || !bytes) return fail(HBMC_EINVAL, "null argument");
    if (nrhs < 1) return fail(HBMC_EINVAL, "nrhs = %d", nrhs);
    *bytes = 2 * smooth_vec_bytes(f, nrhs);
    return HBMC_OK;
}

extern "C" int hbmc_smooth(const hbmc_factor_t *f, const hbmc_matrix_t *A, const double *b, double *x,
                           int32_t nrhs, int32_t sweeps, int32_t mode, void *work, size_t work_bytes,
                           void *stream) {
    clear_error();
    int st = check_ready(f, nrhs);
    if (st) return st;
    if (!A || !b || !x || !work) return fail(HBMC_EINVAL, "null argument");
    if (!A->dev) return fail(HBMC_ENOTREADY, "matrix not uploaded");
    if (A->n_pad != f->n_pad || A->n != f->n) return fail(HBMC_EINVAL, "matrix and factor sizes differ");
    if (sweeps < 0) return fail(HBMC_EINVAL, "sweeps = %d", sweeps);
    if (mode != HBMC_SMOOTH_SYMMETRIC && mode != HBMC_SMOOTH_FORWARD)
        return fail(HBMC_EINVAL, "unknown smoothing mode %d", mode);
    if (static_cast<const void *>(b) == static_cast<const void *>(x)) return fail(HBMC_EINVAL, "x must not alias b");
    const int K = nrhs;
    const size_t vb = smooth_vec_bytes(f, K);
    if (work_bytes < 2 * vb) return fail(HBMC_EINVAL, "workspace too small (%zu < %zu)", work_bytes, 2 * vb);
    if (reinterpret_cast<uintptr_t>(work) % 256) return fail(HBMC_EINVAL, "workspace not 256-byte aligned");
    auto s = static_cast<hipStream_t>(stream);
    double *r = at<double>(work, 0), *z = at<double>(work, vb);
    const Mat m = mat_of(A);
    const bool fwd = mode == HBMC_SMOOTH_FORWARD;
    const double c = fwd ? 1.0 : f->smooth_scale;
    const int64_t ne = f->n_pad * K;
    for (int32_t k = 0; k < sweeps; ++k) {
        VEC_LAUNCH_MAT(k_smooth_r, m, f->n_pad, K, s, m, K, b, x, r);
        HIP_TRY(hipGetLastError());
        if ((st = apply_launch(f, r, z, s, nullptr, nullptr, K, fwd))) return st;
        hipLaunchKernelGGL(k_axpy, dim3(grid_elems(ne)), dim3(kBlock), 0, s, ne, c, z, x);
        HIP_TRY(hipGetLastError());
    }
    return HBMC_OK;
}
