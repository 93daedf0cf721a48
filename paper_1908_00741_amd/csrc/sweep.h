// Preconditioning step z = M^-1 r of the HBMC-ordered IC(0) method, gfx950:
// the device kernels and their launcher, included by one translation unit
// per block size (sweep_bs*.hip) so that the instantiations compile in
// parallel.
//
// Forward substitution y = L^-1 r, then backward substitution z = U^-1 y
// (Section 2), color by color (Section 4.3): one kernel launch per color
// phase, the launch boundary being the synchronization between colors
// (Section 4.4.3).  The last color runs its forward and backward sweeps in
// one launch, since no later color feeds its backward sweep.
//
// Inside a phase a tile is 64 chain lanes, one per BMC block (64/w level-1
// blocks of w lanes each); a chain walks the bs steps of eqs. "y2-2",
// "y2-3", so at step l the 64 lanes solve 64 independent rows, as the w SIMD
// lanes do in the paper.  The couplings to other colors (eq. "for3") do not
// depend on the chain, so each lane first issues the loads of all of them
// for all bs steps -- values, indices and the gathered y or z -- and only
// then runs the chain in registers.  Wavefronts never wait for each other
// inside a phase: there is no barrier on the main path.
//
// Several right-hand sides (vectors stored [n_pad][K], the K values of a row
// adjacent): a wavefront covers 64/NR chains of a tile for NR right-hand
// sides, lane j taking chain j / NR and right-hand side j % NR of its group.
// The NR lanes of a chain load the same factor entries (one access serves
// them) and their y/z gathers are adjacent in memory; the wavefronts of the
// K/NR right-hand-side groups of a tile are neighbours in the grid, so they
// share the factor through the caches and HBM delivers it about once per
// apply.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "flow.h"
#include "fold.h"
#include "xcd.h"
#include "hbmc_internal.h"

namespace hbmc {

// Launches the phases of one apply for factors of block size BS (defined in
// sweep_bs<BS>.hip).  K right-hand sides, nr of them per wavefront.  With
// fwd_only, only the forward substitution runs (z = (D + L)^-1 r, every
// color in the forward form).  With fl, the row kernel's phases run in one
// launch (flow.h; the caller has checked flow_ok).
int launch_bs1(const ::hbmc_factor_s *f, const double *r, double *z, hipStream_t s, const int32_t *done,
               const ApplyCg *cg, int K, int nr, bool fwd_only, const Flow *fl);
int launch_bs2(const ::hbmc_factor_s *f, const double *r, double *z, hipStream_t s, const int32_t *done,
               const ApplyCg *cg, int K, int nr, bool fwd_only, const Flow *fl);
int launch_bs4(const ::hbmc_factor_s *f, const double *r, double *z, hipStream_t s, const int32_t *done,
               const ApplyCg *cg, int K, int nr, bool fwd_only, const Flow *fl);
int launch_bs8(const ::hbmc_factor_s *f, const double *r, double *z, hipStream_t s, const int32_t *done,
               const ApplyCg *cg, int K, int nr, bool fwd_only, const Flow *fl);
int launch_bs16(const ::hbmc_factor_s *f, const double *r, double *z, hipStream_t s, const int32_t *done,
               const ApplyCg *cg, int K, int nr, bool fwd_only, const Flow *fl);
int launch_bs32(const ::hbmc_factor_s *f, const double *r, double *z, hipStream_t s, const int32_t *done,
               const ApplyCg *cg, int K, int nr, bool fwd_only, const Flow *fl);

}  // namespace hbmc

#ifdef HBMC_SWEEP_KERNELS
namespace {

using namespace hbmc;

#define SWEEP_TRY(call)                                                               \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(HBMC_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

constexpr int kLanes = kTileLanes;
constexpr size_t kMaxLds = 64 * 1024;      // LDS budget of one workgroup (general path)
constexpr size_t kLdsPerCu = 160 * 1024;   // LDS of one CU

// Device pointers of a factor's Packed layout: strided slots per group,
// then the left-over couplings either in indexed slots or in flat form
// (lane by lane per group); every array with a trailing padding slot or
// entry.
struct Ext {
    const int32_t *soff;
    const int32_t *sbase;
    const uint64_t *smask;
    const void *sval;
    const int32_t *ioff;      // indexed slots
    const uint64_t *imask;    // lanes of each indexed slot
    const int64_t *ivoff;     // first packed entry of each indexed slot
    const int32_t *icol;
    const void *ival;
    const int64_t *goff;      // flat form: [groups + 1] first entry of each group
    const uint16_t *lstart;   // flat form: [groups][64] first entry of each chain lane, relative to goff
    const int32_t *fcol;
    const void *fval;
    int64_t spad, ipad, fpad;   // the padding slots and the flat padding entry
    bool flat;
};

// Entry of chain lane jc in a packed indexed slot (mask, first entry): its
// rank among the slot's lanes; a lane without an entry reads the slot's
// first entry (every slot has one) and must not use it.
__device__ inline int64_t packed_entry(uint64_t mask, int64_t first, int jc, bool &on) {
    on = (mask >> jc) & 1;
    return first + (on ? __builtin_popcountll(mask & ((uint64_t(1) << jc) - 1)) : 0);
}

// Lanes 0..63 of one wavefront: the largest of v.
__device__ inline int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

// The flat entries of chain lane jc in group g: [first, first + count).
__device__ inline void lane_range(const Ext &E, int64_t g, int jc, int64_t &first, int &count) {
    const int64_t g0 = E.goff[g];
    const int ne = int(E.goff[g + 1] - g0);
    const int a = E.lstart[g * kLanes + jc];
    const int b = jc + 1 < kLanes ? int(E.lstart[g * kLanes + jc + 1]) : ne;
    first = g0 + a;
    count = b - a;
}

// One direction: couplings to other colors (ext) and inside the level-1
// block (int).
struct Tri {
    Ext ext;
    const int32_t *int_off;
    const void *int_val;
    const int8_t *int_lp;    // source step of each in-block coupling (-1: none)
    int64_t int_pad;
};

struct Phase {
    int64_t row0, row1;   // rows of the color
    int64_t tile0;        // first global tile of the color
    int64_t ntile;        // tiles of the color
    int64_t nlane;        // chain lanes of the color (level-1 blocks * w)
    int64_t ptiles;       // CG partial slots per right-hand side (all tiles * NR)
    int32_t w;
    int32_t lw;           // log2(w)
    int32_t lds_slots;    // general path: LDS slots per wavefront
    int32_t K;            // right-hand sides (row stride of the vectors)
    int32_t G;            // right-hand-side groups: ceil(K / NR)
    Tri f, b;
    const void *dinv;
    const int32_t *done;  // if set and *done != 0 the phase does nothing
    ApplyCg cg;
    bool fold;            // CG, first phase, k_sweep: alpha computed here (fold.h)
    bool xcd;             // k_rows: tiles in XCD-contiguous order
    bool one_sys;         // CG: one system (its states are st[0 .. K), no tile lookup)
};

// Sum over the lanes j' of the wavefront with j' = j mod NR (the lanes of
// one right-hand side).
template <int NR>
__device__ inline double rhs_sum(double v) {
#pragma unroll
    for (int o = 32; o >= NR; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

enum { kForward = 0, kBackward = 1, kLast = 2 };

// Row-splitting window of k_rows: chunks of 64 entries per wavefront, so
// that the bs wavefronts of a workgroup stage at most 32 KB.
template <int BS, typename T>
__host__ __device__ constexpr int split_window() {
    return 32768 / (BS * kLanes * 2 * int(sizeof(T))) < 16 ? 32768 / (BS * kLanes * 2 * int(sizeof(T))) : 16;
}

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

// Where a lane's values live: chain lane jc of the tile (factor entries are
// [slot][64] by chain lane), right-hand side q (vector entry row * K + q).
struct Lane {
    int jc;
    int q;
    int K;
    __device__ int64_t at(int64_t row) const { return row * K + q; }
};

// acc[l] -= sum of the couplings to other colors of step l, for all steps,
// each lane over its own couplings in column order: the strided slots, then
// its flat entries.  Chunks of CH slots (entries): within a chunk every
// step's loads are issued before any of them is used; a slot past a step's
// count reads the padding slot, whose empty lane mask drops the product, and
// an entry past a lane's count reads the padding entry and is dropped.
// Strided slots read z[base + jc]; the bases and lane masks of the tile's
// strided slots (at most 64) are fetched by one vector load, one slot per
// lane, and broadcast with readlane, so no load waits on another.
// WAIT (all phases in one launch, flow.h): a gathered value a lane uses is
// waited for once the chunk's loads are back; lanes that drop the product
// never wait (their address may belong to a later phase).
template <int BS, int CH, typename T, bool WAIT = false>
__device__ inline void ext_strided(T (&acc)[BS], const Ext E, int64_t gt, int j, const Lane &L,
                                   const double *__restrict__ z, const FlowWait &fw = FlowWait{}) {
    const int jc = L.jc;
    int32_t so[BS + 1];
#pragma unroll
    for (int l = 0; l <= BS; ++l) so[l] = E.soff[gt + l];
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
        double gd[BS][CH];
        int32_t ix[BS][CH];
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
                on[l][k] = (mask >> jc) & 1;
                v[l][k] = val[slot * kLanes + jc];
                ix[l][k] = base + jc;
                gd[l][k] = z[L.at(ix[l][k])];
            }
#pragma unroll
        for (int l = 0; l < BS; ++l)
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                if (WAIT && on[l][k]) gd[l][k] = flow_take(gd[l][k], z + L.at(ix[l][k]), fw);
                g[l][k] = T(gd[l][k]);
            }
#pragma unroll
        for (int l = 0; l < BS; ++l)
#pragma unroll
            for (int k = 0; k < CH; ++k) acc[l] = on[l][k] ? acc[l] - v[l][k] * g[l][k] : acc[l];
    }
}

// Indexed slots: each loads the slot's lane mask and first entry, then the
// lane's column.
template <int BS, int CH, typename T, bool WAIT = false>
__device__ inline void ext_packed(T (&acc)[BS], const Ext E, int64_t gt, const Lane &L,
                                  const double *__restrict__ z, const FlowWait &fw = FlowWait{}) {
    const int jc = L.jc;
    int32_t io[BS + 1];
#pragma unroll
    for (int l = 0; l <= BS; ++l) io[l] = E.ioff[gt + l];
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
                const int64_t slot = c0 + k < io[l + 1] - io[l] ? int64_t(io[l]) + c0 + k : E.ipad;
                bool on;
                const int64_t e = packed_entry(E.imask[slot], E.ivoff[slot], jc, on);
                const int32_t c = E.icol[e];
                col[l][k] = on ? c : -1;
                v[l][k] = val[e];
            }
        T g[BS][CH];
        double gd[BS][CH];
#pragma unroll
        for (int l = 0; l < BS; ++l)
#pragma unroll
            for (int k = 0; k < CH; ++k) gd[l][k] = z[L.at(col[l][k] >= 0 ? col[l][k] : 0)];
#pragma unroll
        for (int l = 0; l < BS; ++l)
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                if (WAIT && col[l][k] >= 0) gd[l][k] = flow_take(gd[l][k], z + L.at(col[l][k]), fw);
                g[l][k] = T(gd[l][k]);
            }
#pragma unroll
        for (int l = 0; l < BS; ++l)
#pragma unroll
            for (int k = 0; k < CH; ++k) acc[l] = col[l][k] >= 0 ? acc[l] - v[l][k] * g[l][k] : acc[l];
    }
}

// Flat form, each lane over its own entries.
template <int BS, int CH, typename T>
__device__ inline void ext_lanes(T (&acc)[BS], const Ext E, int64_t gt, const Lane &L,
                                 const double *__restrict__ z) {
    int64_t e0[BS];
    int cnt[BS];
    int cmax = 0;
#pragma unroll
    for (int l = 0; l < BS; ++l) {
        lane_range(E, gt + l, L.jc, e0[l], cnt[l]);
        cmax = max(cmax, cnt[l]);
    }
    cmax = wave_max(cmax);
    const T *val = static_cast<const T *>(E.fval);
    for (int c0 = 0; c0 < cmax; c0 += CH) {
        int32_t col[BS][CH];
        T v[BS][CH];
#pragma unroll
        for (int l = 0; l < BS; ++l)
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const bool has = c0 + k < cnt[l];
                const int64_t e = has ? e0[l] + c0 + k : E.fpad;
                const int32_t c = E.fcol[e];
                col[l][k] = has ? c : -1;
                v[l][k] = val[e];
            }
        T g[BS][CH];
#pragma unroll
        for (int l = 0; l < BS; ++l)
#pragma unroll
            for (int k = 0; k < CH; ++k) g[l][k] = T(z[L.at(col[l][k] >= 0 ? col[l][k] : 0)]);
#pragma unroll
        for (int l = 0; l < BS; ++l)
#pragma unroll
            for (int k = 0; k < CH; ++k) acc[l] = col[l][k] >= 0 ? acc[l] - v[l][k] * g[l][k] : acc[l];
    }
}

template <int BS, int CH, typename T>
__device__ inline void ext_sweep(T (&acc)[BS], const Ext E, int64_t gt, int j, const Lane &L,
                                 const double *__restrict__ z) {
    ext_strided<BS, CH, T>(acc, E, gt, j, L, z);
    if (E.flat) ext_lanes<BS, CH, T>(acc, E, gt, L, z);
    else ext_packed<BS, CH, T>(acc, E, gt, L, z);
}

// Row splitting (one right-hand side): the flat entries of group g,
// however unevenly they fall on the rows, are shared evenly by the 64 lanes
// (entry w0 + 64 k + j to lane j), which load them with coalesced loads,
// gather z and stage (value, z) pairs in this wavefront's LDS window
// (win: 2 * NW * 64 values); each chain lane then adds up its own entries
// from the window in column order, the order and arithmetic of ext_lanes.
// Groups longer than the window take several rounds.
template <int NW, typename T, bool WAIT = false>
__device__ inline T ext_split(T acc, const Ext &E, int64_t g, int j, const double *__restrict__ z, T *win,
                             const FlowWait &fw = FlowWait{}) {
    const int64_t g0 = E.goff[g];
    const int ne = int(E.goff[g + 1] - g0);
    if (ne == 0) return acc;
    const int a = E.lstart[g * kLanes + j];
    const int b = j + 1 < kLanes ? int(E.lstart[g * kLanes + j + 1]) : ne;
    const T *val = static_cast<const T *>(E.fval);
    T *wv = win, *wz = win + NW * kLanes;
    for (int w0 = 0; w0 < ne; w0 += NW * kLanes) {
        const int nk = min(NW, (ne - w0 + kLanes - 1) / kLanes);
        T v[NW];
        double gz[NW];
        int32_t col[NW];
#pragma unroll
        for (int k = 0; k < NW; ++k)
            if (k < nk) {
                const int64_t e = g0 + min(w0 + k * kLanes + j, ne - 1);
                col[k] = E.fcol[e];
                v[k] = val[e];
            }
#pragma unroll
        for (int k = 0; k < NW; ++k)
            if (k < nk) gz[k] = z[col[k]];
#pragma unroll
        for (int k = 0; k < NW; ++k)
            if (k < nk) {
                if (WAIT) gz[k] = flow_take(gz[k], z + col[k], fw);
                wv[k * kLanes + j] = v[k];
                wz[k * kLanes + j] = T(gz[k]);
            }
        // the window is written by other lanes of this wavefront
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int lo = max(a, w0), hi = min(b, w0 + NW * kLanes);
        for (int e = lo; e < hi; ++e) acc = acc - wv[e - w0] * wz[e - w0];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    return acc;
}

// Couplings inside the level-1 block for all steps, at most MI per step,
// into registers (padding: index -1, value 0).
template <int BS, int MI, typename T>
__device__ inline void int_load(T (&v)[BS][MI], int32_t (&lp)[BS][MI], const Tri E, int64_t gt, int jc) {
    const T *val = static_cast<const T *>(E.int_val);
    int32_t off[BS + 1];
#pragma unroll
    for (int l = 0; l <= BS; ++l) off[l] = E.int_off[gt + l];   // one batch of scalar loads
#pragma unroll
    for (int l = 0; l < BS; ++l) {
#pragma unroll
        for (int k = 0; k < MI; ++k) {
            const int64_t e = (k < off[l + 1] - off[l] ? int64_t(off[l]) + k : E.int_pad) * kLanes + jc;
            v[l][k] = val[e];
            lp[l][k] = E.int_lp[e];
        }
    }
}

// Copies chain lane jc's couplings inside the level-1 blocks of steps
// [l0, l1) of the tile into an LDS region laid out like the slot lists
// (slot s of the tile at s * 64 + jc).  The NR lanes of a chain write the
// same values to the same places; each lane reads back only its chain's.
template <typename T>
__device__ inline void stage_steps(const Tri &E, int64_t gt, int l0, int l1, int jc, T *sv, int32_t *sl) {
    const int64_t ib = E.int_off[gt];
    const int64_t s0 = E.int_off[gt + l0] - ib, s1 = E.int_off[gt + l1] - ib;
    const T *val = static_cast<const T *>(E.int_val) + ib * kLanes;
    const int8_t *lp = E.int_lp + ib * kLanes;
#pragma unroll 4
    for (int64_t s = s0; s < s1; ++s) {
        sv[s * kLanes + jc] = val[s * kLanes + jc];
        sl[s * kLanes + jc] = lp[s * kLanes + jc];
    }
}

// The bs-step chains of one lane (eqs. "y2-2", "y2-3"): forward (y) and/or
// backward (z) sweeps inside the level-1 block, with acc holding each step's
// right-hand side after the couplings to other colors.  Stores y (forward
// phases) or z, and with CG the (r, z) partial of the lane's right-hand side
// at pslot.  MI == 0: couplings inside the block are staged into this
// wavefront's LDS region sv/sl when lds, else read in place.  Forward
// values go to yout when set (all phases in one launch), else to z; WT
// stores them with agent-scope atomic stores (flow.h).
template <int BS, typename T, int MODE, int MI, bool CG, int NR, bool WT = false>
__device__ inline void chains(const Phase &ph, T (&acc)[BS], const T (&dv)[BS], const double (&rn)[BS],
                              const T (&fv)[BS][MI > 0 ? MI : 1], const int32_t (&fl)[BS][MI > 0 ? MI : 1],
                              const T (&bv)[BS][MI > 0 ? MI : 1], const int32_t (&bl)[BS][MI > 0 ? MI : 1],
                              T *sv, int32_t *sl, bool lds, int64_t gt, int j, const Lane &L, int64_t rb,
                              bool valid, bool qv, double *__restrict__ z, int64_t pslot,
                              T *svb = nullptr, int32_t *slb = nullptr, double *yout = nullptr) {
    constexpr int RM = MI > 0 ? MI : 1;
    const int w = ph.w;
    const int jc = L.jc;
    // svb: couplings already staged by the caller (forward at sv/sl,
    // backward at svb/slb); else staged here, one direction at a time
    const bool staged = svb != nullptr;
    auto stage = [&](const Tri &E) -> int64_t {
        const int64_t ib = E.int_off[gt];
        if (lds && !staged) stage_steps<T>(E, gt, 0, BS, jc, sv, sl);
        return ib;
    };
    auto ival = [&](const Tri &E, int64_t s) -> T {
        if (!lds) return static_cast<const T *>(E.int_val)[(s + E.int_off[gt]) * kLanes + jc];
        return (staged && &E == &ph.b ? svb : sv)[s * kLanes + jc];
    };
    auto ilp = [&](const Tri &E, int64_t s) -> int32_t {
        if (!lds) return E.int_lp[(s + E.int_off[gt]) * kLanes + jc];
        return (staged && &E == &ph.b ? slb : sl)[s * kLanes + jc];
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
            if (MODE == kForward && valid) {
                double *d = (yout ? yout : z) + L.at(rb + int64_t(l) * w);
                if (WT) flow_put(d, double(y[l]));
                else *d = double(y[l]);
            }
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
            if (valid) {
                double *d = z + L.at(rb + int64_t(l) * w);
                if (WT) flow_put(d, double(a));
                else *d = double(a);
            }
        }
        if (CG) {
            double rz = 0.0;
#pragma unroll
            for (int l = 0; l < BS; ++l) rz += valid ? rn[l] * double(y[l]) : 0.0;
            rz = rhs_sum<NR>(rz);
            if (j < NR && qv) ph.cg.part_rz[int64_t(L.q) * ph.ptiles + pslot] = rz;
        }
    }
}

// Loads the right-hand side of one row (r, or y for a backward phase); with
// CG in a forward phase first applies r -= alpha q to it.
template <typename T, int MODE, bool CG>
__device__ inline T row_rhs(const Phase &ph, const double *__restrict__ r, const double *__restrict__ z,
                            int64_t e, bool valid, double alpha, double &rn, double &rr) {
    if (CG && MODE != kBackward) {
        rn = ph.cg.r[e] - alpha * ph.cg.q[e];
        if (valid) { ph.cg.r[e] = rn; rr += rn * rn; }
        return T(rn);
    }
    if (CG) rn = ph.cg.r[e];   // backward: r of these rows is final
    return T(MODE == kBackward ? z[e] : r[e]);
}

// One color phase, one wavefront per (tile, sub-tile, right-hand-side
// group): the wavefront loads the couplings of all bs steps itself, then
// runs the chains.  Best when a color has many tiles.
// MODE kForward: y of color c; kBackward: z of color c; kLast: y then z of
// the last color.  z holds y of the colors whose forward sweep is done and
// z of the colors whose backward sweep is done.
// MI > 0: at most MI couplings per step inside a level-1 block, held in
// registers.  MI == 0: any number, staged per wavefront in LDS when they fit.
template <int BS, typename T, int MODE, int MI, int CH, int WAVES, bool CG, int NR>
__global__ void __launch_bounds__(WAVES * kLanes) k_sweep(Phase ph, const double *__restrict__ r,
                                                          double *__restrict__ z) {
    if (ph.done && *ph.done) return;
    if (CG && ph.fold && blockIdx.x == 0) fold_alpha(ph.cg);   // every thread, before any return
    // the wavefront index is uniform: say so, so that everything indexed by
    // the tile (slot offsets, strided bases and masks) uses scalar loads
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kLanes);
    const int j = threadIdx.x % kLanes;
    // NR == 1 runs one right-hand side only (K == 1 at compile time)
    constexpr bool ONE = NR == 1;
    const int K = ONE ? 1 : ph.K;
    const int64_t W = int64_t(blockIdx.x) * WAVES + wave;
    const int64_t ts = ONE ? W : W / ph.G;       // tile * NR + sub-tile
    const int grp = int(W - ts * (ONE ? 1 : ph.G));   // right-hand-side group
    const int64_t tile = ts / NR;
    const int sub = int(ts % NR);
    if (tile >= ph.ntile) return;
    const int q0 = grp * NR + j % NR;
    const bool qv = q0 < K;
    const Lane L{sub * (kLanes / NR) + j / NR, qv ? q0 : K - 1, K};
    // The state of the lane's (system, right-hand side).  With one system
    // and one right-hand side its stop is the all-stopped flag checked above,
    // so nothing waits for the state here (alpha is read where it is used).
    const CgState *cs = CG ? &ph.cg.st[(ph.one_sys ? 0 : int64_t(ph.cg.tile_sys[ph.tile0 + tile]) * K) + L.q]
                           : nullptr;
    const bool live = qv && !(CG && !(ONE && ph.one_sys) && cs->done);
    if (CG && !__any(live)) return;              // every right-hand side of this wave has stopped
    const int64_t lam = tile * kLanes + L.jc;    // chain lane in the color
    const bool valid = lam < ph.nlane && live;
    const int w = ph.w;
    // lanes past the color's last level-1 block (a partial last tile) work
    // on the last lane's rows and store nothing
    const int64_t lc = lam < ph.nlane ? lam : ph.nlane - 1;
    const int64_t rb = ph.row0 + ((lc >> ph.lw) << ph.lw) * BS + (lc & (w - 1));
    const int64_t gt = (ph.tile0 + tile) * BS;   // (tile, step 0) slot list
    const int64_t pslot = (ph.tile0 + tile) * NR + sub;

    constexpr int RM = MI > 0 ? MI : 1;
    T fv[BS][RM], bv[BS][RM];
    int32_t fl[BS][RM], bl[BS][RM];
    if constexpr (MI > 0) {
        if (MODE != kBackward) int_load<BS, RM, T>(fv, fl, ph.f, gt, L.jc);
        if (MODE != kForward) int_load<BS, RM, T>(bv, bl, ph.b, gt, L.jc);
    }
    T acc[BS], dv[BS];
    double rn[BS];   // CG: the updated residual of the lane's rows
    double rr = 0.0;
    if constexpr (CG && MODE != kBackward) {
        // r -= alpha q on the lane's rows: their loads first, then (first
        // phase of a folded iteration) the wait for alpha
        double rv[BS], qv[BS];
#pragma unroll
        for (int l = 0; l < BS; ++l) {
            const int64_t row = rb + int64_t(l) * w, e = L.at(row);
            dv[l] = static_cast<const T *>(ph.dinv)[row];
            rv[l] = ph.cg.r[e];
            qv[l] = ph.cg.q[e];
        }
        double alpha;
        if (ph.fold) {
            const uint64_t v = fold_wait(ph.cg.fwords, ph.cg.fparity, ph.cg.ferr);
            if (v == kStopped) return;
            alpha = __longlong_as_double(int64_t(v));
        } else {
            alpha = cs->alpha;
        }
#pragma unroll
        for (int l = 0; l < BS; ++l) {
            const int64_t e = L.at(rb + int64_t(l) * w);
            rn[l] = rv[l] - alpha * qv[l];
            if (valid) { ph.cg.r[e] = rn[l]; rr += rn[l] * rn[l]; }
            acc[l] = T(rn[l]);
        }
    } else {
#pragma unroll
        for (int l = 0; l < BS; ++l) {
            const int64_t row = rb + int64_t(l) * w;
            if (MODE != kBackward) dv[l] = static_cast<const T *>(ph.dinv)[row];
            acc[l] = row_rhs<T, MODE, CG>(ph, r, z, L.at(row), valid, 0.0, rn[l], rr);
        }
    }
    if (CG && MODE != kBackward) {
        rr = rhs_sum<NR>(rr);
        if (j < NR && qv) ph.cg.part_rr[int64_t(L.q) * ph.ptiles + pslot] = rr;
    }
    ext_sweep<BS, CH, T>(acc, MODE == kBackward ? ph.b.ext : ph.f.ext, gt, j, L, z);

    extern __shared__ __align__(16) unsigned char smem[];
    T *sv = reinterpret_cast<T *>(smem) + int64_t(wave) * ph.lds_slots * kLanes;
    int32_t *sl = reinterpret_cast<int32_t *>(reinterpret_cast<T *>(smem) +
                                              int64_t(WAVES) * ph.lds_slots * kLanes) +
                  int64_t(wave) * ph.lds_slots * kLanes;
    chains<BS, T, MODE, MI, CG, NR>(ph, acc, dv, rn, fv, fl, bv, bl, sv, sl, ph.lds_slots > 0, gt, j, L,
                                    rb, valid, qv, z, pslot);
}

// Where a tile of the row kernel reads and writes.  One launch per color:
// everything in z (y of the colors whose forward sweep is done, z of those
// whose backward sweep is done).  All phases in one launch (flow.h): the
// forward values in y, the result in z, each waited for where it is read.
struct RowsIo {
    const double *gsrc;   // values gathered from other colors
    const double *own;    // backward: y of the tile's own rows
    double *yout;         // forward: y of the tile's own rows
    FlowWait fw;          // error word and time limit of the waits
};

// One tile of one color phase, one workgroup per tile with one wavefront
// per step: each wavefront folds in the couplings to other colors of its
// step for the 64 lanes, the partial right-hand sides meet in LDS, and
// wavefront 0 runs the chains.  Eight times the wavefronts of k_sweep, each
// with one step's loads: best when a color has few tiles or its steps have
// many couplings.  One right-hand side only.
// With FLOW and CG, r's update (r -= alpha q) is computed by the forward
// tile for its sums and again, with the same single rounding, by the
// backward tile of the same rows, which stores it: the forward tile never
// writes r, so that no tile reads a value of r another workgroup stored.
// The backward tile stores it only after the barrier that follows its wait
// for the rows' own forward values, i.e. after the forward tile has read
// the old r (it reads r before it stores those values).
template <int BS, typename T, int MODE, int MI, int CH, bool CG, bool FLOW>
__device__ inline void rows_tile(const Phase &ph, int64_t tile, int64_t row0, int64_t tile0, int64_t nlane,
                                 const double *__restrict__ r, double *__restrict__ z, const RowsIo &io) {
    const int l = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kLanes);   // this wave's step
    const int j = threadIdx.x % kLanes;
    // the tile's system state; with one system its stop is the all-stopped
    // flag checked on entry, and nothing waits for the state here
    const CgState *cs = CG ? &ph.cg.st[ph.one_sys ? 0 : ph.cg.tile_sys[tile0 + tile]] : nullptr;
    if (CG && !ph.one_sys && cs->done) return;   // the whole workgroup: one tile
    const Lane L{j, 0, 1};
    const int64_t lam = tile * kLanes + j;
    const bool valid = lam < nlane;
    const int w = ph.w;
    const int64_t lc = valid ? lam : nlane - 1;
    const int64_t rb = row0 + ((lc >> ph.lw) << ph.lw) * BS + (lc & (w - 1));
    const int64_t gt = (tile0 + tile) * BS;

    extern __shared__ __align__(16) unsigned char smem[];
    double *srn = reinterpret_cast<double *>(smem);          // [BS][64] (CG)
    double *srr = srn + BS * kLanes;                         // [BS]     (CG)
    T *sq = reinterpret_cast<T *>(srr + BS);                 // [BS][64]
    T *sd = sq + BS * kLanes;                                // [BS][64]
    T *svf = sd + BS * kLanes;                               // [lds_slots][64] (MI == 0)
    T *svb = svf + ph.lds_slots * kLanes;                    // [lds_slots][64]
    int32_t *slf = reinterpret_cast<int32_t *>(svb + ph.lds_slots * kLanes);
    int32_t *slb = slf + ph.lds_slots * kLanes;
    constexpr int NW = split_window<BS, T>();
    T *win = reinterpret_cast<T *>(slb + ph.lds_slots * kLanes) + l * (2 * NW * kLanes);   // this wave's window

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
    T acc1[1];
    if constexpr (FLOW) {
        if (CG) {
            const double alpha = cs->alpha;
            rn1 = __builtin_fma(-alpha, ph.cg.q[row], ph.cg.r[row]);
            if (MODE != kBackward && valid) rr += rn1 * rn1;
        }
        if (MODE == kBackward) acc1[0] = T(flow_take(io.own[row], io.own + row, io.fw));
        else acc1[0] = T(CG ? rn1 : r[row]);
    } else {
        const double alpha = CG && MODE != kBackward ? cs->alpha : 0.0;
        acc1[0] = row_rhs<T, MODE, CG>(ph, r, z, row, valid, alpha, rn1, rr);
    }
    if (MODE != kBackward) sd[l * kLanes + j] = static_cast<const T *>(ph.dinv)[row];
    if (MI == 0 && ph.lds_slots > 0) {   // this step's couplings inside the block
        if (MODE != kBackward) stage_steps<T>(ph.f, gt, l, l + 1, j, svf, slf);
        if (MODE != kForward) stage_steps<T>(ph.b, gt, l, l + 1, j, svb, slb);
    }
    const Ext &ext = MODE == kBackward ? ph.b.ext : ph.f.ext;
    const double *src = FLOW ? io.gsrc : z;
    ext_strided<1, CH, T, FLOW>(acc1, ext, gt + l, j, L, src, io.fw);
    if (ext.flat) acc1[0] = ext_split<NW, T, FLOW>(acc1[0], ext, gt + l, j, src, win, io.fw);
    else ext_packed<1, CH, T, FLOW>(acc1, ext, gt + l, L, src, io.fw);
    sq[l * kLanes + j] = acc1[0];
    if (CG) {
        srn[l * kLanes + j] = rn1;
        if (MODE != kBackward) {
            rr = rhs_sum<1>(rr);
            if (j == 0) srr[l] = rr;
        }
    }
    __syncthreads();
    if (FLOW && CG && MODE != kForward && valid) ph.cg.r[row] = rn1;   // see above
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
        ph.cg.part_rr[tile0 + tile] = t;
    }
    chains<BS, T, MODE, MI, CG, 1, FLOW>(ph, acc, dv, rn, fv, fl, bv, bl, svf, slf, ph.lds_slots > 0, gt, j, L,
                                         rb, valid, true, z, tile0 + tile, svb, slb, FLOW ? io.yout : nullptr);
}

// One color phase of the row kernel, a workgroup per tile.
template <int BS, typename T, int MODE, int MI, int CH, bool CG>
__global__ void __launch_bounds__(BS <= 16 ? BS * kLanes : 1024) k_rows(Phase ph, const double *__restrict__ r,
                                                      double *__restrict__ z) {
    if (ph.done && *ph.done) return;
    // XCD-contiguous tiles for an ordering with locality (after the
    // renumbering): the tiles one XCD takes gather from neighbouring places
    // (1M-point 13-NN graph after reverse Cuthill-McKee: 217.7 -> 198.5 us
    // per apply, solve 104.9 -> 101.8 ms).  In the shuffled numbering the
    // hardware order is faster (solve 131.9 against 134.7 ms), and the
    // wavefront-per-tile kernel keeps it too (128^3 apply 51.5 against 53.2 us)
    const int64_t tile = ph.xcd ? xcd_block(blockIdx.x, gridDim.x) : int64_t(blockIdx.x);
    rows_tile<BS, T, MODE, MI, CH, CG, false>(ph, tile, ph.row0, ph.tile0, ph.nlane, r, z, RowsIo{});
}

// The phases of one apply in one launch (flow.h).  Workgroups
// [pblock[p], pblock[p + 1]) run phase p: forward color p for p < nc - 1,
// the last color for p = nc - 1, then backward color 2 nc - 2 - p.  Tiles
// in the hardware order: the XCD-contiguous order that helps k_rows after
// the renumbering measured slightly slower here (1M-point 13-NN graph,
// renumbered, FP64: apply 153.6 against 152.6 us, solve 80.3 against
// 79.2 ms).
struct FlowTab {
    int64_t color_start[kFlowMaxColors + 1];
    int64_t tile_base[kFlowMaxColors + 1];
    int32_t pblock[2 * kFlowMaxColors];
    int32_t nc;
    double *y;        // forward values, kFlowEmpty on entry
    FlowWait fw;
};

template <int BS, typename T, int MI, int CH, bool CG>
__global__ void __launch_bounds__(BS <= 16 ? BS * kLanes : 1024) k_flow(Phase ph, FlowTab ft,
                                                      const double *__restrict__ r, double *__restrict__ z) {
    if (ph.done && *ph.done) return;
    const int32_t b = int32_t(blockIdx.x);
    const int np = 2 * ft.nc - 1;
    int lo = 0, hi = np - 1;   // the last phase starting at or before b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ft.pblock[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const int p = lo;
    const int c = p < ft.nc ? p : 2 * ft.nc - 2 - p;
    const int64_t tile = b - ft.pblock[p];
    const int64_t tile0 = ft.tile_base[c];
    if (tile >= ft.tile_base[c + 1] - tile0) return;
    const int64_t row0 = ft.color_start[c];
    const int64_t nlane = (ft.color_start[c + 1] - row0) / BS;
    if (p < ft.nc - 1)
        rows_tile<BS, T, kForward, MI, CH, CG, true>(ph, tile, row0, tile0, nlane, r, z,
                                                    RowsIo{ft.y, nullptr, ft.y, ft.fw});
    else if (p == ft.nc - 1)
        rows_tile<BS, T, kLast, MI, CH, CG, true>(ph, tile, row0, tile0, nlane, r, z,
                                                 RowsIo{ft.y, nullptr, nullptr, ft.fw});
    else
        rows_tile<BS, T, kBackward, MI, CH, CG, true>(ph, tile, row0, tile0, nlane, r, z,
                                                     RowsIo{z, ft.y, nullptr, ft.fw});
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <class P>
const P *dev_at(const void *base, size_t off) {
    return reinterpret_cast<const P *>(static_cast<const uint8_t *>(base) + off);
}

Tri tri_of(const ::hbmc_factor_s *f, const TriOffsets &o, const LayoutCounts &e) {
    const PackedOffsets &x = o.ext;
    return Tri{Ext{dev_at<int32_t>(f->dev, x.soff), dev_at<int32_t>(f->dev, x.sbase),
                   dev_at<uint64_t>(f->dev, x.smask), dev_at<void>(f->dev, x.sval),
                   dev_at<int32_t>(f->dev, x.ioff), dev_at<uint64_t>(f->dev, x.imask),
                   dev_at<int64_t>(f->dev, x.ivoff), dev_at<int32_t>(f->dev, x.icol),
                   dev_at<void>(f->dev, x.ival),
                   dev_at<int64_t>(f->dev, x.goff), dev_at<uint16_t>(f->dev, x.lstart),
                   dev_at<int32_t>(f->dev, x.fcol), dev_at<void>(f->dev, x.fval),
                   e.strided, e.indexed, e.fpad, e.flat},
               dev_at<int32_t>(f->dev, o.int_off), dev_at<void>(f->dev, o.int_val),
               dev_at<int8_t>(f->dev, o.int_lp), o.int_slots};
}

template <int BS, typename T, int MI, bool CG, int NR>
int launch_phases(const ::hbmc_factor_s *f, const double *r, double *z, hipStream_t s,
                  const int32_t *done, const ApplyCg &cg, int K, bool fwd_only, const Flow *fl) {
    constexpr int CH = BS <= 4 ? 4 : (BS <= 8 ? 2 : 1);   // measured best on 128^3, bs 8
    constexpr int WAVES = MI > 0 ? 4 : 1;                 // k_sweep: wavefronts per workgroup
    constexpr int CHR = 16;                               // k_rows: slots per chunk
    if (NR == 1 && K != 1) return fail(HBMC_EINVAL, "right-hand-side tile 1 runs one right-hand side");
    const bool rows = hbmc::use_rows(f, BS, K, NR);
    Phase ph{};
    ph.w = f->w;
    ph.lw = __builtin_ctz(unsigned(f->w));
    ph.K = K;
    ph.G = (K + NR - 1) / NR;
    ph.ptiles = f->tile_base[f->nc] * NR;
    ph.f = tri_of(f, f->fwd, f->fcnt);
    ph.b = tri_of(f, f->bwd, f->bcnt);
    ph.dinv = dev_at<void>(f->dev, f->off_dinv);
    ph.done = done;
    ph.cg = cg;
    ph.xcd = f->local;   // tiles in XCD-contiguous order after the renumbering
    ph.one_sys = f->nsys == 1;
    bool first_phase = CG && cg.stw != nullptr;   // the next launch computes alpha
    const size_t tw = sizeof(T) + sizeof(int32_t);
    size_t lds = 0;
    ph.lds_slots = 0;
    const size_t split = size_t(BS) * 2 * split_window<BS, T>() * kLanes * sizeof(T);   // k_rows windows
    if (MI == 0) {
        ph.lds_slots = std::max(std::max(f->max_int_slots_f, f->max_int_slots_b), 1);
        const size_t per = size_t(ph.lds_slots) * kLanes * tw;
        if ((rows ? 2 * per + size_t(BS) * kLanes * (8 + 2 * sizeof(T)) + 8 * BS + split : WAVES * per) > kMaxLds)
            ph.lds_slots = 0;
    }
    if (rows)
        lds = size_t(BS) * kLanes * (8 + 2 * sizeof(T)) + 8 * BS + 2 * size_t(ph.lds_slots) * kLanes * tw + split;
    else
        lds = size_t(WAVES) * ph.lds_slots * kLanes * tw;
    const int nc = f->nc;
    if (fl) {
        if constexpr (NR == 1 && BS <= kFlowMaxBs) {
            if (!rows || K != 1 || fwd_only || nc > kFlowMaxColors || f->nsys != 1)
                return fail(HBMC_EINVAL, "internal: the one-launch form does not apply");
            FlowTab ft{};
            ft.nc = nc;
            ft.y = fl->y;
            ft.fw = FlowWait{fl->err, f->wait_ticks};
            for (int c = 0; c <= nc; ++c) {
                ft.color_start[c] = f->color_start[c];
                ft.tile_base[c] = f->tile_base[c];
            }
            int64_t blocks = 0;
            for (int p = 0; p < 2 * nc - 1; ++p) {
                const int c = p < nc ? p : 2 * nc - 2 - p;
                ft.pblock[p] = int32_t(blocks);
                blocks += f->tile_base[c + 1] - f->tile_base[c];
                if (blocks > int64_t(INT32_MAX)) return fail(HBMC_EINVAL, "too many workgroups for one launch");
            }
            if (blocks == 0) return HBMC_OK;
            // At most four workgroups per CU (five for an ordering with
            // locality, i.e. after the renumbering), set through the LDS each takes: more resident tiles
            // only wait longer and crowd the caches.  1M-point 13-NN graph,
            // bs 2, w 32, FP32 apply (FP64 takes four by its own LDS):
            // shuffled 239 us with eight per CU, 196 with four, 204 with
            // five, 220 with three; renumbered 158 / 148 / 142 / 166 us.
            const int per_cu = f->local ? 5 : 4;
            const size_t lds_flow = std::max(lds, kLdsPerCu / size_t(per_cu + 1) + 1);
            hipLaunchKernelGGL((k_flow<BS, T, MI, CHR, CG>), dim3(unsigned(blocks)), dim3(BS * kLanes), lds_flow, s,
                               ph, ft, r, z);
            SWEEP_TRY(hipGetLastError());
            return HBMC_OK;
        } else {
            return fail(HBMC_EINVAL, "internal: the one-launch form runs one right-hand side, bs <= %d", kFlowMaxBs);
        }
    }
    auto run = [&](int c, auto sweep, auto rowk) -> int {
        ph.row0 = f->color_start[c];
        ph.row1 = f->color_start[c + 1];
        ph.tile0 = f->tile_base[c];
        ph.ntile = f->tile_base[c + 1] - f->tile_base[c];
        ph.nlane = (ph.row1 - ph.row0) / BS;
        if (ph.ntile == 0) return HBMC_OK;
        ph.fold = first_phase;
        first_phase = false;
        if (rows) {
            hipLaunchKernelGGL(rowk, dim3(unsigned(ph.ntile)), dim3(BS * kLanes), lds, s, ph, r, z);
        } else {
            const int64_t waves = ph.ntile * NR * ph.G;
            if ((waves + WAVES - 1) / WAVES > int64_t(INT32_MAX))
                return fail(HBMC_EINVAL, "too many wavefronts for one launch");
            const unsigned grid = unsigned((waves + WAVES - 1) / WAVES);
            hipLaunchKernelGGL(sweep, dim3(grid), dim3(WAVES * kLanes), lds, s, ph, r, z);
        }
        SWEEP_TRY(hipGetLastError());
        return HBMC_OK;
    };
    int st;
    if (fwd_only) {
        if (CG) return fail(HBMC_EINVAL, "internal: forward-only substitution inside CG");
        for (int c = 0; c < nc; ++c)
            if ((st = run(c, k_sweep<BS, T, kForward, MI, CH, WAVES, CG, NR>,
                          k_rows<BS, T, kForward, MI, CHR, CG>))) return st;
        return HBMC_OK;
    }
    for (int c = 0; c + 1 < nc; ++c)
        if ((st = run(c, k_sweep<BS, T, kForward, MI, CH, WAVES, CG, NR>,
                      k_rows<BS, T, kForward, MI, CHR, CG>))) return st;
    if ((st = run(nc - 1, k_sweep<BS, T, kLast, MI, CH, WAVES, CG, NR>,
                  k_rows<BS, T, kLast, MI, CHR, CG>))) return st;
    for (int c = nc - 2; c >= 0; --c)
        if ((st = run(c, k_sweep<BS, T, kBackward, MI, CH, WAVES, CG, NR>,
                      k_rows<BS, T, kBackward, MI, CHR, CG>))) return st;
    return HBMC_OK;
}

// right-hand sides per wavefront: 1 (one right-hand side), 4, 8 or 16
template <int BS, typename T, int MI, bool CG>
int dispatch_nr(const ::hbmc_factor_s *f, const double *r, double *z, hipStream_t s, const int32_t *done,
                const ApplyCg &cg, int K, int nr, bool fo, const Flow *fl) {
    switch (nr) {
        case 1: return launch_phases<BS, T, MI, CG, 1>(f, r, z, s, done, cg, K, fo, fl);
        case 4: return launch_phases<BS, T, MI, CG, 4>(f, r, z, s, done, cg, K, fo, fl);
        case 8: return launch_phases<BS, T, MI, CG, 8>(f, r, z, s, done, cg, K, fo, fl);
        case 16: return launch_phases<BS, T, MI, CG, 16>(f, r, z, s, done, cg, K, fo, fl);
        default: return fail(HBMC_EINVAL, "right-hand-side tile %d (1, 4, 8, 16)", nr);
    }
}

// couplings per step inside a level-1 block: <= 1, <= 2, or more (LDS path)
template <int BS, typename T, bool CG>
int dispatch_mi(const ::hbmc_factor_s *f, const double *r, double *z, hipStream_t s, const int32_t *done,
                const ApplyCg &cg, int K, int nr, bool fo, const Flow *fl) {
    const int mi = std::max(f->max_int_step_f, f->max_int_step_b);
    if (mi <= 1) return dispatch_nr<BS, T, 1, CG>(f, r, z, s, done, cg, K, nr, fo, fl);
    if (BS <= 16 && mi <= 2) return dispatch_nr<BS, T, 2, CG>(f, r, z, s, done, cg, K, nr, fo, fl);
    return dispatch_nr<BS, T, 0, CG>(f, r, z, s, done, cg, K, nr, fo, fl);
}

template <int BS>
int launch_bs(const ::hbmc_factor_s *f, const double *r, double *z, hipStream_t s, const int32_t *done,
              const ApplyCg *cgp, int K, int nr, bool fo, const Flow *fl) {
    if (!cgp) {
        const ApplyCg none{};
        return f->precision == HBMC_F64 ? dispatch_mi<BS, double, false>(f, r, z, s, done, none, K, nr, fo, fl)
                                        : dispatch_mi<BS, float, false>(f, r, z, s, done, none, K, nr, fo, fl);
    }
    return f->precision == HBMC_F64 ? dispatch_mi<BS, double, true>(f, cgp->r, z, s, done, *cgp, K, nr, fo, fl)
                                    : dispatch_mi<BS, float, true>(f, cgp->r, z, s, done, *cgp, K, nr, fo, fl);
}

}  // namespace
#endif  // HBMC_SWEEP_KERNELS
