// Preconditioning step z = M^-1 r of the HBMC-ordered IC(0) method, gfx950.
//
// Forward substitution y = L^-1 r, then backward substitution z = U^-1 y
// (Section 2), color by color (Section 4.2.2): one kernel launch per color
// phase, the launch boundary being the synchronization between colors
// (Section 4.4.3).  The last color runs its forward and backward sweeps in
// one launch, since no later color feeds its backward sweep.
//
// Inside a phase every wavefront owns one tile of 64 chain lanes, one lane
// per BMC block (64/w level-1 blocks of w lanes each), and walks the bs
// steps of eqs. "y2-2", "y2-3": at step l the 64 lanes solve 64 independent
// rows, as the w SIMD lanes do in the paper.  The couplings to other colors
// (eq. "for3") do not depend on the chain, so each lane first issues the
// loads of all of them for all bs steps -- values, indices and the gathered
// y or z -- and only then runs the chain in registers.  Wavefronts never
// wait for each other inside a phase: there is no LDS traffic and no
// barrier on the main path.
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
constexpr size_t kMaxLds = 64 * 1024;      // LDS budget of one workgroup (general path)

// Device pointers of a Packed layout (strided and indexed slots per group),
// each array with a trailing all-padding slot.
struct Ext {
    const int32_t *soff;
    const int32_t *sbase;
    const uint64_t *smask;
    const void *sval;
    const int32_t *ioff;
    const int32_t *icol;
    const void *ival;
    int64_t spad, ipad;   // index of the padding slots
};

// One direction: couplings to other colors (ext) and inside the level-1
// block (int).
struct Tri {
    Ext ext;
    const int32_t *int_off;
    const void *int_val;
    const int32_t *int_lp;
    int64_t int_pad;
};

// CG work folded into the sweep (iccg_solve only; all null for ic0_apply):
// the forward sweep of a color first applies x += alpha p, r -= alpha q to
// the rows it reads and adds up ||r||^2; the sweeps that finish z add up
// (r, z).  One partial sum per tile, in tile order.
struct CgFuse {
    double *x;
    const double *p;
    const double *q;
    double *r;
    const CgState *st;         // per system: alpha, done
    const int32_t *tile_sys;   // system of each tile
    double *part_rr;
    double *part_rz;
};

struct Phase {
    int64_t row0, row1;   // rows of the color
    int64_t tile0;        // first global tile of the color
    int64_t ntile;        // tiles of the color
    int64_t nlane;        // chain lanes of the color (level-1 blocks * w)
    int32_t w;
    int32_t lw;           // log2(w)
    int32_t lds_slots;    // general path: LDS slots per wavefront
    Tri f, b;
    const void *dinv;
    const int32_t *done;  // if set and *done != 0 the phase does nothing
    CgFuse cg;
};

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

enum { kForward = 0, kBackward = 1, kLast = 2 };

// y[idx] among the compile-time candidates lo <= idx < hi, else 0.
template <int BS, typename T>
__device__ inline T pick(const T (&y)[BS], int idx, int lo, int hi) {
    T r = T(0);
#pragma unroll
    for (int i = 0; i < BS; ++i)
        if (i >= lo && i < hi) r = idx == i ? y[i] : r;
    return r;
}

__device__ inline uint64_t readlane64(uint64_t v, int lane) {
    const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(v), lane);
    const uint32_t hi = __builtin_amdgcn_readlane(uint32_t(v >> 32), lane);
    return (uint64_t(hi) << 32) | lo;
}

// acc[l] -= sum of the couplings to other colors of step l, for all steps.
// Chunks of CH slots: within a chunk every step's slot loads are issued
// before any of them is used; a slot past a step's count reads the padding
// slot, whose empty lane mask (strided) or column -1 (indexed) drops the
// product.  Strided slots read z[base + j]; the bases and lane masks of the
// tile's strided slots (at most 64) are fetched by one vector load, one slot
// per lane, and broadcast with readlane, so no load waits on another.
// Indexed slots first load the lane's column.
template <int BS, int CH, typename T>
__device__ inline void ext_sweep(T (&acc)[BS], const Ext E, int64_t gt, int j,
                                 const double *__restrict__ z) {
    int32_t so[BS + 1], io[BS + 1];
#pragma unroll
    for (int l = 0; l <= BS; ++l) {
        so[l] = E.soff[gt + l];
        io[l] = E.ioff[gt + l];
    }
    {
        const T *val = static_cast<const T *>(E.sval);
        const int nst = so[BS] - so[0];
        const int64_t mslot = so[0] + (j < nst ? j : 0);
        const int32_t mbase = E.sbase[mslot];
        const uint64_t mmask = E.smask[mslot];
        int smax = 0;
#pragma unroll
        for (int l = 0; l < BS; ++l) smax = max(smax, so[l + 1] - so[l]);
        for (int c0 = 0; c0 < smax; c0 += CH) {
            T v[BS][CH], g[BS][CH];
            bool on[BS][CH];
#pragma unroll
            for (int l = 0; l < BS; ++l)
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const bool has = c0 + k < so[l + 1] - so[l];
                    const int q = has ? so[l] + c0 + k - so[0] : 0;
                    const int32_t base = has ? __builtin_amdgcn_readlane(mbase, q) : 0;
                    const uint64_t mask = has ? readlane64(mmask, q) : 0;
                    const int64_t slot = has ? so[l] + c0 + k : E.spad;
                    on[l][k] = (mask >> j) & 1;
                    v[l][k] = val[slot * kLanes + j];
                    g[l][k] = T(z[base + j]);
                }
#pragma unroll
            for (int l = 0; l < BS; ++l)
#pragma unroll
                for (int k = 0; k < CH; ++k) acc[l] = on[l][k] ? acc[l] - v[l][k] * g[l][k] : acc[l];
        }
    }
    const T *val = static_cast<const T *>(E.ival);
    int smax = 0;
#pragma unroll
    for (int l = 0; l < BS; ++l) smax = max(smax, io[l + 1] - io[l]);
    for (int c0 = 0; c0 < smax; c0 += CH) {
        int32_t col[BS][CH];
        T v[BS][CH];
#pragma unroll
        for (int l = 0; l < BS; ++l)
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int64_t e = (c0 + k < io[l + 1] - io[l] ? int64_t(io[l]) + c0 + k : E.ipad) * kLanes + j;
                col[l][k] = E.icol[e];
                v[l][k] = val[e];
            }
        T g[BS][CH];
#pragma unroll
        for (int l = 0; l < BS; ++l)
#pragma unroll
            for (int k = 0; k < CH; ++k) g[l][k] = T(z[col[l][k] >= 0 ? col[l][k] : 0]);
#pragma unroll
        for (int l = 0; l < BS; ++l)
#pragma unroll
            for (int k = 0; k < CH; ++k) acc[l] = col[l][k] >= 0 ? acc[l] - v[l][k] * g[l][k] : acc[l];
    }
}

// Couplings inside the level-1 block for all steps, at most MI per step,
// into registers (padding: index -1, value 0).
template <int BS, int MI, typename T>
__device__ inline void int_load(T (&v)[BS][MI], int32_t (&lp)[BS][MI], const Tri E, int64_t gt, int j) {
    const T *val = static_cast<const T *>(E.int_val);
    int32_t off[BS + 1];
#pragma unroll
    for (int l = 0; l <= BS; ++l) off[l] = E.int_off[gt + l];   // one batch of scalar loads
#pragma unroll
    for (int l = 0; l < BS; ++l) {
#pragma unroll
        for (int k = 0; k < MI; ++k) {
            const int64_t e = (k < off[l + 1] - off[l] ? int64_t(off[l]) + k : E.int_pad) * kLanes + j;
            v[l][k] = val[e];
            lp[l][k] = E.int_lp[e];
        }
    }
}

// One color phase for the tile of wavefront blockIdx.x * WAVES + wave.
// MODE kForward: y of color c; kBackward: z of color c; kLast: y then z of
// the last color.  z holds y of the colors whose forward sweep is done and
// z of the colors whose backward sweep is done.
// MI > 0: at most MI couplings per step inside a level-1 block, held in
// registers.  MI == 0: any number, staged per wavefront in LDS when they fit
// (each lane reads back only what it wrote, so no barrier is needed), else
// read from global memory step by step.
// The bs-step chains of one lane (eqs. "y2-2", "y2-3"): forward (y) and/or
// backward (z) sweeps inside the level-1 block, with acc holding each step's
// right-hand side after the couplings to other colors.  Stores y (forward
// phases) or z, and with CG the tile's (r, z) partial.  MI == 0: couplings
// inside the block are staged into this wavefront's LDS region sv/sl (each
// lane reads back only its own entries) when lds, else read in place.
// Copies this lane's couplings inside the level-1 blocks of steps [l0, l1)
// of the tile into an LDS region laid out like the slot lists (slot s of the
// tile at s * 64 + lane).  Loads are issued in groups before the stores.
template <typename T>
__device__ inline void stage_steps(const Tri &E, int64_t gt, int l0, int l1, int j, T *sv, int32_t *sl) {
    const int64_t ib = E.int_off[gt];
    const int64_t s0 = E.int_off[gt + l0] - ib, s1 = E.int_off[gt + l1] - ib;
    const T *val = static_cast<const T *>(E.int_val) + ib * kLanes;
    const int32_t *lp = E.int_lp + ib * kLanes;
#pragma unroll 4
    for (int64_t s = s0; s < s1; ++s) {
        sv[s * kLanes + j] = val[s * kLanes + j];
        sl[s * kLanes + j] = lp[s * kLanes + j];
    }
}

template <int BS, typename T, int MODE, int MI, bool CG>
__device__ inline void chains(const Phase &ph, T (&acc)[BS], const T (&dv)[BS], const double (&rn)[BS],
                              const T (&fv)[BS][MI > 0 ? MI : 1], const int32_t (&fl)[BS][MI > 0 ? MI : 1],
                              const T (&bv)[BS][MI > 0 ? MI : 1], const int32_t (&bl)[BS][MI > 0 ? MI : 1],
                              T *sv, int32_t *sl, bool lds, int64_t gt, int j, int64_t rb, bool valid,
                              double *__restrict__ z, int64_t gtile, T *svb = nullptr,
                              int32_t *slb = nullptr) {
    constexpr int RM = MI > 0 ? MI : 1;
    const int w = ph.w;
    // svb: couplings already staged by the caller (forward at sv/sl,
    // backward at svb/slb); else staged here, one direction at a time
    const bool staged = svb != nullptr;
    auto stage = [&](const Tri &E) -> int64_t {
        const int64_t ib = E.int_off[gt];
        if (lds && !staged) stage_steps<T>(E, gt, 0, BS, j, sv, sl);
        return ib;
    };
    auto ival = [&](const Tri &E, int64_t s) -> T {
        if (!lds) return static_cast<const T *>(E.int_val)[(s + E.int_off[gt]) * kLanes + j];
        return (staged && &E == &ph.b ? svb : sv)[s * kLanes + j];
    };
    auto ilp = [&](const Tri &E, int64_t s) -> int32_t {
        if (!lds) return E.int_lp[(s + E.int_off[gt]) * kLanes + j];
        return (staged && &E == &ph.b ? slb : sl)[s * kLanes + j];
    };

    T y[BS];
    if (MODE != kBackward) {
        int64_t ib = 0;
        if constexpr (MI == 0) ib = stage(ph.f);
#pragma unroll
        for (int l = 0; l < BS; ++l) {
            T a = acc[l];
            if constexpr (MI > 0) {
#pragma unroll
                for (int k = 0; k < RM; ++k) a -= fv[l][k] * pick<BS, T>(y, fl[l][k], 0, l);
            } else {
                const int64_t s0 = ph.f.int_off[gt + l] - ib, s1 = ph.f.int_off[gt + l + 1] - ib;
                for (int64_t s = s0; s < s1; ++s) a -= ival(ph.f, s) * pick<BS, T>(y, ilp(ph.f, s), 0, l);
            }
            y[l] = a * dv[l];
            if (MODE == kForward && valid) z[rb + int64_t(l) * w] = double(y[l]);
        }
    } else {
#pragma unroll
        for (int l = 0; l < BS; ++l) y[l] = acc[l];
    }
    if (MODE != kForward) {
        int64_t ib = 0;
        if constexpr (MI == 0) ib = stage(ph.b);
        // y becomes z, from the last step down
#pragma unroll
        for (int l = BS - 1; l >= 0; --l) {
            T a = y[l];
            if constexpr (MI > 0) {
#pragma unroll
                for (int k = 0; k < RM; ++k) a -= bv[l][k] * pick<BS, T>(y, bl[l][k], l + 1, BS);
            } else {
                const int64_t s0 = ph.b.int_off[gt + l] - ib, s1 = ph.b.int_off[gt + l + 1] - ib;
                for (int64_t s = s0; s < s1; ++s) a -= ival(ph.b, s) * pick<BS, T>(y, ilp(ph.b, s), l + 1, BS);
            }
            y[l] = a;
            if (valid) z[rb + int64_t(l) * w] = double(a);
        }
        if (CG) {
            double rz = 0.0;
#pragma unroll
            for (int l = 0; l < BS; ++l) rz += valid ? rn[l] * double(y[l]) : 0.0;
            rz = wave_sum(rz);
            if (j == 0) ph.cg.part_rz[gtile] = rz;
        }
    }
}

// Loads the right-hand side of one row (r, or y for a backward phase); with
// CG in a forward phase first applies x += alpha p, r -= alpha q to it.
template <typename T, int MODE, bool CG>
__device__ inline T row_rhs(const Phase &ph, const double *__restrict__ r, const double *__restrict__ z,
                            int64_t row, bool valid, double alpha, double &rn, double &rr) {
    if (CG && MODE != kBackward) {
        const double pv = ph.cg.p[row];
        const double xn = ph.cg.x[row] + alpha * pv;
        rn = ph.cg.r[row] - alpha * ph.cg.q[row];
        if (valid) { ph.cg.x[row] = xn; ph.cg.r[row] = rn; rr += rn * rn; }
        return T(rn);
    }
    if (CG) rn = ph.cg.r[row];   // backward: r of these rows is final
    return T(MODE == kBackward ? z[row] : r[row]);
}

// One color phase, one wavefront per tile (tile = blockIdx.x * WAVES + wave):
// the wavefront loads the couplings of all bs steps itself, then runs the
// chains.  Best when a color has many tiles.
// MODE kForward: y of color c; kBackward: z of color c; kLast: y then z of
// the last color.  z holds y of the colors whose forward sweep is done and
// z of the colors whose backward sweep is done.
// MI > 0: at most MI couplings per step inside a level-1 block, held in
// registers.  MI == 0: any number, staged per wavefront in LDS when they fit.
template <int BS, typename T, int MODE, int MI, int CH, int WAVES, bool CG>
__global__ void __launch_bounds__(WAVES * kLanes) k_sweep(Phase ph, const double *__restrict__ r,
                                                          double *__restrict__ z) {
    if (ph.done && *ph.done) return;
    // the wavefront index is uniform: say so, so that everything indexed by
    // the tile (slot offsets, strided bases and masks) uses scalar loads
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kLanes);
    const int j = threadIdx.x % kLanes;
    const int64_t tile = int64_t(blockIdx.x) * WAVES + wave;
    if (tile >= ph.ntile) return;
    const CgState *cs = CG ? &ph.cg.st[ph.cg.tile_sys[ph.tile0 + tile]] : nullptr;
    if (CG && cs->done) return;                  // this tile's system has stopped
    const int64_t lam = tile * kLanes + j;       // chain lane in the color
    const bool valid = lam < ph.nlane;
    const int w = ph.w;
    // lanes past the color's last level-1 block (a partial last tile) work
    // on the last lane's rows and store nothing
    const int64_t lc = valid ? lam : ph.nlane - 1;
    const int64_t rb = ph.row0 + ((lc >> ph.lw) << ph.lw) * BS + (lc & (w - 1));
    const int64_t gt = (ph.tile0 + tile) * BS;   // (tile, step 0) slot list

    constexpr int RM = MI > 0 ? MI : 1;
    T fv[BS][RM], bv[BS][RM];
    int32_t fl[BS][RM], bl[BS][RM];
    if constexpr (MI > 0) {
        if (MODE != kBackward) int_load<BS, RM, T>(fv, fl, ph.f, gt, j);
        if (MODE != kForward) int_load<BS, RM, T>(bv, bl, ph.b, gt, j);
    }
    T acc[BS], dv[BS];
    double rn[BS];   // CG: the updated residual of the lane's rows
    double rr = 0.0;
    const double alpha = CG && MODE != kBackward ? cs->alpha : 0.0;
#pragma unroll
    for (int l = 0; l < BS; ++l) {
        const int64_t row = rb + int64_t(l) * w;
        if (MODE != kBackward) dv[l] = static_cast<const T *>(ph.dinv)[row];
        acc[l] = row_rhs<T, MODE, CG>(ph, r, z, row, valid, alpha, rn[l], rr);
    }
    if (CG && MODE != kBackward) {
        rr = wave_sum(rr);
        if (j == 0) ph.cg.part_rr[ph.tile0 + tile] = rr;
    }
    ext_sweep<BS, CH, T>(acc, MODE == kBackward ? ph.b.ext : ph.f.ext, gt, j, z);

    extern __shared__ __align__(16) unsigned char smem[];
    T *sv = reinterpret_cast<T *>(smem) + int64_t(wave) * ph.lds_slots * kLanes;
    int32_t *sl = reinterpret_cast<int32_t *>(reinterpret_cast<T *>(smem) +
                                              int64_t(WAVES) * ph.lds_slots * kLanes) +
                  int64_t(wave) * ph.lds_slots * kLanes;
    chains<BS, T, MODE, MI, CG>(ph, acc, dv, rn, fv, fl, bv, bl, sv, sl, ph.lds_slots > 0, gt, j, rb,
                                valid, z, ph.tile0 + tile);
}

// One color phase, one workgroup per tile with one wavefront per step: each
// wavefront folds in the couplings to other colors of its step for the 64
// lanes, the partial right-hand sides meet in LDS, and wavefront 0 runs the
// chains.  Eight times the wavefronts of k_sweep, each with one step's loads:
// best when a color has few tiles or its steps have many couplings.
template <int BS, typename T, int MODE, int MI, int CH, bool CG>
__global__ void __launch_bounds__(BS <= 16 ? BS * kLanes : 1024) k_rows(Phase ph, const double *__restrict__ r,
                                                      double *__restrict__ z) {
    if (ph.done && *ph.done) return;
    const int l = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kLanes);   // this wave's step
    const int j = threadIdx.x % kLanes;
    const int64_t tile = blockIdx.x;
    const CgState *cs = CG ? &ph.cg.st[ph.cg.tile_sys[ph.tile0 + tile]] : nullptr;
    if (CG && cs->done) return;                  // the whole workgroup: one tile
    const int64_t lam = tile * kLanes + j;
    const bool valid = lam < ph.nlane;
    const int w = ph.w;
    const int64_t lc = valid ? lam : ph.nlane - 1;
    const int64_t rb = ph.row0 + ((lc >> ph.lw) << ph.lw) * BS + (lc & (w - 1));
    const int64_t gt = (ph.tile0 + tile) * BS;

    extern __shared__ __align__(16) unsigned char smem[];
    double *srn = reinterpret_cast<double *>(smem);          // [BS][64] (CG)
    double *srr = srn + BS * kLanes;                         // [BS]     (CG)
    T *sq = reinterpret_cast<T *>(srr + BS);                 // [BS][64]
    T *sd = sq + BS * kLanes;                                // [BS][64]
    T *svf = sd + BS * kLanes;                               // [lds_slots][64] (MI == 0)
    T *svb = svf + ph.lds_slots * kLanes;                    // [lds_slots][64]
    int32_t *slf = reinterpret_cast<int32_t *>(svb + ph.lds_slots * kLanes);
    int32_t *slb = slf + ph.lds_slots * kLanes;

    constexpr int RM = MI > 0 ? MI : 1;
    T fv[BS][RM], bv[BS][RM];
    int32_t fl[BS][RM], bl[BS][RM];
    if constexpr (MI > 0) {
        if (l == 0) {
            if (MODE != kBackward) int_load<BS, RM, T>(fv, fl, ph.f, gt, j);
            if (MODE != kForward) int_load<BS, RM, T>(bv, bl, ph.b, gt, j);
        }
    }
    const int64_t row = rb + int64_t(l) * w;
    double rn1 = 0.0, rr = 0.0;
    const double alpha = CG && MODE != kBackward ? cs->alpha : 0.0;
    T acc1[1] = {row_rhs<T, MODE, CG>(ph, r, z, row, valid, alpha, rn1, rr)};
    if (MODE != kBackward) sd[l * kLanes + j] = static_cast<const T *>(ph.dinv)[row];
    if (MI == 0 && ph.lds_slots > 0) {   // this step's couplings inside the block
        if (MODE != kBackward) stage_steps<T>(ph.f, gt, l, l + 1, j, svf, slf);
        if (MODE != kForward) stage_steps<T>(ph.b, gt, l, l + 1, j, svb, slb);
    }
    ext_sweep<1, CH, T>(acc1, MODE == kBackward ? ph.b.ext : ph.f.ext, gt + l, j, z);
    sq[l * kLanes + j] = acc1[0];
    if (CG) {
        srn[l * kLanes + j] = rn1;
        if (MODE != kBackward) {
            rr = wave_sum(rr);
            if (j == 0) srr[l] = rr;
        }
    }
    __syncthreads();
    if (l != 0) return;

    T acc[BS], dv[BS];
    double rn[BS];
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        acc[k] = sq[k * kLanes + j];
        dv[k] = MODE != kBackward ? sd[k * kLanes + j] : T(1);
        rn[k] = CG ? srn[k * kLanes + j] : 0.0;
    }
    if (CG && MODE != kBackward && j == 0) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < BS; ++k) t += srr[k];
        ph.cg.part_rr[ph.tile0 + tile] = t;
    }
    chains<BS, T, MODE, MI, CG>(ph, acc, dv, rn, fv, fl, bv, bl, svf, slf, ph.lds_slots > 0, gt, j, rb,
                                valid, z, ph.tile0 + tile, svb, slb);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <class P>
const P *at(const void *base, size_t off) {
    return reinterpret_cast<const P *>(static_cast<const uint8_t *>(base) + off);
}

Tri tri_of(const hbmc_factor_s *f, const TriOffsets &o, const Packed &e, const Sell &i) {
    const PackedOffsets &x = o.ext;
    return Tri{Ext{at<int32_t>(f->dev, x.soff), at<int32_t>(f->dev, x.sbase),
                   at<uint64_t>(f->dev, x.smask), at<void>(f->dev, x.sval),
                   at<int32_t>(f->dev, x.ioff), at<int32_t>(f->dev, x.icol),
                   at<void>(f->dev, x.ival), e.strided(), e.indexed()},
               at<int32_t>(f->dev, o.int_off), at<void>(f->dev, o.int_val),
               at<int32_t>(f->dev, o.int_lp), i.slots()};
}

// Which kernel runs the phases: one wavefront per tile (k_sweep) or one
// workgroup of bs wavefronts per tile (k_rows).  Automatic choice: k_rows
// when the colors have few tiles on average (fewer than 1024: a phase would
// not fill the chip with one wavefront per tile).
bool use_rows(const hbmc_factor_s *f, int bs) {
    if (bs > 16) return false;                      // bs wavefronts per workgroup
    if (f->kernel == HBMC_KERNEL_SWEEP) return false;
    if (f->kernel == HBMC_KERNEL_ROWS) return true;
    return f->tile_base[f->nc] < 1024 * int64_t(f->nc);
}

template <int BS, typename T, int MI, bool CG>
int launch_phases(const hbmc_factor_s *f, const double *r, double *z, hipStream_t s,
                  const int32_t *done, const CgFuse &cg) {
    constexpr int CH = BS <= 4 ? 4 : (BS <= 8 ? 2 : 1);   // measured best on 128^3, bs 8
    constexpr int WAVES = MI > 0 ? 4 : 1;                 // k_sweep: tiles per workgroup
    constexpr int CHR = 16;                               // k_rows: slots per chunk
    const bool rows = use_rows(f, BS);
    Phase ph{};
    ph.w = f->w;
    ph.lw = __builtin_ctz(unsigned(f->w));
    ph.f = tri_of(f, f->fwd, f->fext, f->fint);
    ph.b = tri_of(f, f->bwd, f->bext, f->bint);
    ph.dinv = at<void>(f->dev, f->off_dinv);
    ph.done = done;
    ph.cg = cg;
    const size_t tw = sizeof(T) + sizeof(int32_t);
    size_t lds = 0;
    ph.lds_slots = 0;
    if (MI == 0) {
        ph.lds_slots = std::max(std::max(f->max_int_slots_f, f->max_int_slots_b), 1);
        const size_t per = size_t(ph.lds_slots) * kLanes * tw;
        if ((rows ? 2 * per + size_t(BS) * kLanes * (8 + 2 * sizeof(T)) + 8 * BS : WAVES * per) > kMaxLds)
            ph.lds_slots = 0;
    }
    if (rows)
        lds = size_t(BS) * kLanes * (8 + 2 * sizeof(T)) + 8 * BS + 2 * size_t(ph.lds_slots) * kLanes * tw;
    else
        lds = size_t(WAVES) * ph.lds_slots * kLanes * tw;
    auto run = [&](int c, auto sweep, auto rowk) -> int {
        ph.row0 = f->color_start[c];
        ph.row1 = f->color_start[c + 1];
        ph.tile0 = f->tile_base[c];
        ph.ntile = f->tile_base[c + 1] - f->tile_base[c];
        ph.nlane = (ph.row1 - ph.row0) / BS;
        if (ph.ntile == 0) return HBMC_OK;
        if (rows) {
            hipLaunchKernelGGL(rowk, dim3(unsigned(ph.ntile)), dim3(BS * kLanes), lds, s, ph, r, z);
        } else {
            const unsigned grid = unsigned((ph.ntile + WAVES - 1) / WAVES);
            hipLaunchKernelGGL(sweep, dim3(grid), dim3(WAVES * kLanes), lds, s, ph, r, z);
        }
        HIP_TRY(hipGetLastError());
        return HBMC_OK;
    };
    const int nc = f->nc;
    int st;
    for (int c = 0; c + 1 < nc; ++c)
        if ((st = run(c, k_sweep<BS, T, kForward, MI, CH, WAVES, CG>,
                      k_rows<BS, T, kForward, MI, CHR, CG>))) return st;
    if ((st = run(nc - 1, k_sweep<BS, T, kLast, MI, CH, WAVES, CG>,
                  k_rows<BS, T, kLast, MI, CHR, CG>))) return st;
    for (int c = nc - 2; c >= 0; --c)
        if ((st = run(c, k_sweep<BS, T, kBackward, MI, CH, WAVES, CG>,
                      k_rows<BS, T, kBackward, MI, CHR, CG>))) return st;
    return HBMC_OK;
}

// couplings per step inside a level-1 block: <= 1, <= 2, or more (LDS path)
template <int BS, typename T, bool CG>
int dispatch_mi(const hbmc_factor_s *f, const double *r, double *z, hipStream_t s,
                const int32_t *done, const CgFuse &cg) {
    const int mi = std::max(f->max_int_step_f, f->max_int_step_b);
    if (mi <= 1) return launch_phases<BS, T, 1, CG>(f, r, z, s, done, cg);
    if (BS <= 16 && mi <= 2) return launch_phases<BS, T, 2, CG>(f, r, z, s, done, cg);
    return launch_phases<BS, T, 0, CG>(f, r, z, s, done, cg);
}

template <typename T, bool CG>
int dispatch_bs(const hbmc_factor_s *f, const double *r, double *z, hipStream_t s,
                const int32_t *done, const CgFuse &cg) {
    switch (f->bs) {
        case 1: return dispatch_mi<1, T, CG>(f, r, z, s, done, cg);
        case 2: return dispatch_mi<2, T, CG>(f, r, z, s, done, cg);
        case 4: return dispatch_mi<4, T, CG>(f, r, z, s, done, cg);
        case 8: return dispatch_mi<8, T, CG>(f, r, z, s, done, cg);
        case 16: return dispatch_mi<16, T, CG>(f, r, z, s, done, cg);
        case 32: return dispatch_mi<32, T, CG>(f, r, z, s, done, cg);
        default: return fail(HBMC_EINVAL, "bs = %d has no device kernel (1, 2, 4, 8, 16, 32)", f->bs);
    }
}

}  // namespace

int hbmc::apply_launch(const hbmc_factor_s *f, const double *r, double *z, void *stream,
                       const int32_t *done, const ApplyCg *cgp) {
    auto s = static_cast<hipStream_t>(stream);
    if (!cgp) {
        const CgFuse none{};
        return f->precision == HBMC_F64 ? dispatch_bs<double, false>(f, r, z, s, done, none)
                                        : dispatch_bs<float, false>(f, r, z, s, done, none);
    }
    const CgFuse cg{cgp->x, cgp->p, cgp->q, cgp->r, cgp->st, cgp->tile_sys, cgp->part_rr, cgp->part_rz};
    return f->precision == HBMC_F64 ? dispatch_bs<double, true>(f, cgp->r, z, s, done, cg)
                                    : dispatch_bs<float, true>(f, cgp->r, z, s, done, cg);
}

// ---------------------------------------------------------------------------
// C ABI
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
    release_graphs(f);
    f->dev = dev;
    f->dev_bytes = bytes;
    f->uid = next_uid();
    return HBMC_OK;
}

extern "C" int hbmc_factor_set_kernel(hbmc_factor_t *f, int32_t kernel) {
    if (!f) return fail(HBMC_EINVAL, "null handle");
    if (kernel != HBMC_KERNEL_AUTO && kernel != HBMC_KERNEL_SWEEP && kernel != HBMC_KERNEL_ROWS)
        return fail(HBMC_EINVAL, "unknown kernel %d", kernel);
    f->kernel = kernel;
    release_graphs(f);
    return HBMC_OK;
}

extern "C" int ic0_apply(const hbmc_factor_t *f, const double *r, double *z, int32_t nrhs, void *stream) {
    if (!f || !r || !z) return fail(HBMC_EINVAL, "null argument");
    if (!f->dev) return fail(HBMC_ENOTREADY, "factor not uploaded");
    if (nrhs != 1) return fail(HBMC_EINVAL, "nrhs = %d not supported", nrhs);
    if (r == z) return fail(HBMC_EINVAL, "z must not alias r");
    return apply_launch(f, r, z, stream, nullptr, nullptr);
}
