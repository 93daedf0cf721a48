// Internal declarations shared by the host setup (order.cpp, factor.cpp) and
// the device code (hbmc.hip).  Not part of the public interface.
#pragma once

#include <cstddef>
#include <cstdint>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hbmc.h"

namespace hbmc {

// Records a message for hbmc_last_error() and returns code.
int fail(int code, const char *fmt, ...);
void clear_error();

// A color is processed in tiles of kTileLanes chain lanes (one lane per BMC
// block) x bs steps; each tile is one wavefront of gfx950.  The SpMV uses
// sliced ELL with slices of kTileLanes consecutive rows.
constexpr int kTileLanes = 64;
// Rows per partial sum of the CG vector kernels (one workgroup of those
// kernels); a batch keeps every part inside one system.
constexpr int kPartRows = 256;
// A base shared by at least this many lanes of a group makes a strided slot.
constexpr int kMinStridedLanes = 48;

// Checks a CSR pattern: sizes, sorted in-range columns, diagonal present,
// symmetric pattern.  Values (if given) must be symmetric with a positive
// diagonal.
int check_csr(int32_t n, const int64_t *rowptr, const int32_t *col, const double *val);

// A sliced-ELL array on the host: slot offsets per slice, then slot-major
// values and columns, kTileLanes entries per slot.  Used for the couplings
// inside level-1 blocks, whose "column" is the source step (0..bs-1, -1 for
// none): one byte each.
struct Sell {
    std::vector<int32_t> off;   // [slices + 1]
    std::vector<double> val;    // [slots * kTileLanes]
    std::vector<int8_t> col;    // [slots * kTileLanes]
    int64_t slots() const { return off.empty() ? 0 : off.back(); }
    // room for the slices of parts (before appending them)
    void reserve_for(const std::vector<const Sell *> &parts) {
        size_t o = off.size(), v = val.size();
        for (const Sell *p : parts) { o += p->off.size(); v += p->val.size(); }
        off.reserve(o); val.reserve(v); col.reserve(v);
    }
    // o's slices after this one's (both started with off = {0}, no padding slot yet)
    void append(const Sell &o) {
        const int32_t base = off.back();
        for (size_t i = 1; i < o.off.size(); ++i) off.push_back(base + o.off[i]);
        val.insert(val.end(), o.val.begin(), o.val.end());
        col.insert(col.end(), o.col.begin(), o.col.end());
    }
};

// CG state of one system, kept on the device between kernels.
struct CgState {
    double rho, alpha, beta, sigma, rr, bb, res, tol;
    double c0;   // scale applied to a given start vector (x0_scale)
    int32_t it, maxit, done, pad;
};
// Stop flag values
enum { kRunning = 0, kConverged = 1, kBreakdown = 2, kMaxIt = 3 };

// CG work folded into the preconditioning step (iccg_solve only): the
// forward sweep of a color first applies r -= alpha q to the rows it reads
// and adds up ||r||^2; the sweeps that finish z add up (r, z).  (x += alpha
// p waits for the next iteration's direction update, which streams p
// anyway.)  Partial sums per (right-hand side, tile, sub-tile):
// [K][tiles * NR].
struct ApplyCg {
    const double *q;
    double *r;
    const CgState *st;          // [systems][K]: alpha, and done (stopped ones are skipped)
    const int32_t *tile_sys;    // [tiles] system of each tile
    double *part_rr;            // [K][tiles * NR]
    double *part_rz;            // [K][tiles * NR]
    // one system, one right-hand side: alpha computed in the first phase
    // (workgroup 0 adds the product's partials fpart[0 .. fnp)), published
    // in fwords (replicated, by iteration parity fparity)
    CgState *stw;
    const double *fpart;
    int64_t fnp;
    uint64_t *fwords;
    int32_t fparity;
    int32_t *ferr, *ndone, *alldone;
};
// All phases of the row kernel in one launch (flow.h): y ([n_pad]) holds
// the forward values, err is set by a wait past its time limit.  With
// fill the launcher first marks y and z empty (and with reset_err clears
// *err); else the caller has (the CG direction update does).
constexpr int kFlowMaxColors = 64;
// Largest block size that takes the one-launch form: with bs 8 a tile's
// chain is long and its workgroup of bs wavefronts large, and a launch per
// phase is faster (1M-point 13-NN graph, row kernel, w 64: solve 254.9
// against 284.7 ms; bs 1 w 64, bs 2 w 32, bs 4 w 16 gain: 139.1 -> 133.8,
// 128.7 -> 110.4, 148.8 -> 134.4 ms).
constexpr int kFlowMaxBs = 4;
struct Flow {
    double *y;
    int32_t *err;
    bool fill;
    bool reset_err;
};
// Whether the one-launch form applies to z = M^-1 r for K right-hand sides.
bool flow_ok(const ::hbmc_factor_s *f, int K, bool fwd_only = false);

// Enqueues z = M^-1 r for K right-hand sides ([n_pad][K]) on stream (a
// hipStream_t).  When done is not null the kernels return at once while
// *done != 0 (used inside captured CG loops).  With cg, r is taken from
// cg->r after the update.  With fwd_only (and no cg), only the forward
// substitution runs: z = (D + L)^-1 r.  With flow (and flow_ok) all phases
// run in one launch.
int apply_launch(const ::hbmc_factor_s *f, const double *r, double *z, void *stream,
                 const int32_t *done, const ApplyCg *cg, int K, bool fwd_only = false,
                 const Flow *flow = nullptr);
// Right-hand sides per wavefront (NR) used for K right-hand sides.
int rhs_tile(const ::hbmc_factor_s *f, int K);
// Whether the phases run as one workgroup per tile (k_rows) rather than one
// wavefront per tile (k_sweep), for bs, K right-hand sides and tile NR.
bool use_rows(const ::hbmc_factor_s *f, int bs, int K, int nr);
// hbmc_factor_export of a factor built on the device (copies from the
// build workspace; synchronous).
int device_export(const ::hbmc_factor_s *f, double *d, int64_t *lrp, int32_t *lcol, double *lval);
// Destroys the hipGraph executables cached by iccg_solve for this factor.
void release_graphs(::hbmc_factor_s *f);
// Unique id for each upload of a device image (keys the graph cache).
uint64_t next_uid();

// Allocator whose resize() leaves new elements of trivial types
// uninitialized: large setup arrays are first written by the threads that
// fill them, not zeroed by one thread beforehand.
template <class T>
struct NoInit : std::allocator<T> {
    template <class U> struct rebind { using other = NoInit<U>; };
    NoInit() = default;
    template <class U> NoInit(const NoInit<U> &) noexcept {}
    template <class U> void construct(U *p) noexcept { ::new (static_cast<void *>(p)) U; }
    template <class U, class... A> void construct(U *p, A &&...a) { ::new (static_cast<void *>(p)) U(std::forward<A>(a)...); }
};
template <class T> using RawVec = std::vector<T, NoInit<T>>;

// One coupling: column (or source step) and value.
struct Coupling {
    int32_t first;
    double second;
};
// Couplings of one row, sorted by column; empty for a lane without a row.
struct CouplingSpan {
    const Coupling *p = nullptr;
    size_t n = 0;
    size_t size() const { return n; }
    const Coupling &operator[](size_t i) const { return p[i]; }
};
// Couplings of all rows in one array: row r is data[ptr[r] .. ptr[r + 1]).
struct CouplingRows {
    std::vector<int64_t> ptr;
    RawVec<Coupling> data;
    CouplingSpan row(int64_t r) const { return {data.data() + ptr[r], size_t(ptr[r + 1] - ptr[r])}; }
};
// Couplings of groups of kTileLanes rows, one row per lane, in two kinds of
// slots.  A strided slot has one base per slot: lane j couples to column
// base + j when bit j of the slot's lane mask is set.  On HBMC-ordered
// structured grids most couplings line up this way, because the 64 lanes
// are 64 consecutive BMC blocks whose neighbours are consecutive too; such
// a slot needs no index array and its loads do not wait for indices.  What
// does not line up goes to indexed slots: slot t of a group holds the t-th
// left-over coupling of every lane that has one, packed in lane order (the
// lane mask says which lanes; lane j's entry is number popcount(mask below
// j) from the slot's first entry), so that lanes without one cost nothing.
// Each array ends with one all-padding slot that loads may target instead
// of branching.
//
// Flat form of the left-over couplings (substitution factors build it
// beside the slots when `both` is set before adding groups, and upload one
// of the two forms, `flat` saying which): a group's left-over couplings
// stored lane by lane (lane j's in column order, the order the slots visit
// them), with the group's first entry (goff) and each lane's first entry
// relative to it (lstart, 64 per group; lane 63's entries end where the
// next group's begin).  A lane can then read its own entries in place, or
// the lanes of a wavefront can share the group's entries evenly whatever
// the length of each row (row splitting).  Slots suit grids (few left-over
// couplings, each slot's entries adjacent across lanes); the flat form
// suits unstructured graphs (mostly left-over couplings of uneven count).
struct Packed {
    std::vector<int32_t> soff{0};   // [groups + 1] strided slots per group
    std::vector<int32_t> sbase;     // [strided + 1]
    std::vector<uint64_t> smask;    // [strided + 1]
    std::vector<double> sval;       // [(strided + 1) * kTileLanes]
    std::vector<int32_t> ioff{0};   // [groups + 1] indexed slots per group
    std::vector<uint64_t> imask;    // [indexed + 1] lanes with an entry in the slot
    std::vector<int64_t> ivoff;     // [indexed + 1] the slot's first entry in icol / ival
    std::vector<int32_t> icol;      // [entries in indexed slots + 1] columns
    std::vector<double> ival;       // [entries in indexed slots + 1] values
    int32_t max_strided = 0, max_indexed = 0;   // per group (flat: most left-over couplings of a lane)
    int64_t entries = 0;                        // couplings stored
    int64_t left = 0;                           // left-over couplings (in indexed slots)
    bool both = false;                          // build the flat form too
    bool flat = false;                          // the device image holds the flat form, not the slots
    std::vector<int64_t> goff{0};               // flat: [groups + 1] first entry of each group
    std::vector<uint16_t> lstart;               // flat: [groups * kTileLanes] lane starts in the group
    std::vector<int32_t> fcol;                  // flat: [left + 1] columns (+ padding entry)
    std::vector<double> fval;                   // flat: [left + 1] values
    int32_t max_group = 0;                      // flat: most entries of a group
    bool overflow = false;                      // flat: a group held more entries than lstart can address
    // lanes[j]: couplings of lane j's row (sorted by column), or null.
    // Columns base + j of strided slots stay below limit; at most budget
    // strided slots are made (the rest of the couplings go to indexed slots).
    // Returns the number of strided slots made.
    int add_group(const std::vector<CouplingSpan> &lanes, int64_t limit, int budget);
    void append(const Packed &o);   // o's groups after this one's (neither finished)
    void reserve_for(const std::vector<const Packed *> &parts);   // room for appending parts
    void finish();   // appends the padding slots
    int64_t strided() const { return soff.back(); }
    int64_t indexed() const { return ioff.back(); }
};

// Byte layout of a device image: every array starts on a 256-byte boundary.
struct ImageBuilder {
    std::vector<uint8_t> bytes;
    size_t add(const void *src, size_t n);
    template <class T> size_t add(const std::vector<T> &v) { return add(v.data(), v.size() * sizeof(T)); }
};

}  // namespace hbmc

struct hbmc_dbuild_s;

struct hbmc_order_s {
    int32_t n = 0, bs = 0, w = 0, nc = 0, nsys = 1;
    bool local = false;                // ordered after the locality renumbering (hbmc_order_rcm)
    int64_t n_pad = 0, nblocks = 0;
    std::vector<int64_t> sys_ptr;      // [nsys + 1] original rows of each system
    std::vector<int64_t> seg;          // [nc * (nsys + 1)] HBMC rows of (color, system)
    std::vector<int32_t> perm;         // [n]    original -> HBMC
    std::vector<int32_t> iperm;        // [n_pad] HBMC -> original, -1 for dummies
    std::vector<int64_t> color_start;  // [nc + 1]
};

// Offsets (bytes, inside a device image) of a Packed layout.
struct PackedOffsets {
    size_t soff, sbase, smask, sval, ioff, imask, ivoff, icol, ival;
    size_t goff, lstart, fcol, fval;   // flat form only
};

// What the launchers need to know of one direction's coupling layout
// (host builds take it from their Packed arrays, device builds from the
// counts computed on the device).
struct LayoutCounts {
    int64_t strided = 0;   // strided slots: the padding slot's index
    int64_t indexed = 0;   // indexed slots: the padding slot's index
    int64_t fpad = 0;      // flat form: the padding entry's index
    int64_t left = 0;      // left-over couplings
    bool flat = false;     // the image holds the flat form
};

// Offsets of one triangular direction.
struct TriOffsets {
    PackedOffsets ext;                  // per (tile, step): couplings to other colors
    size_t int_off, int_val, int_lp;    // per (tile, step): couplings inside the level-1 block
    int64_t int_slots;                  // in-block slots (the padding slot's index)
};

struct hbmc_factor_s {
    int32_t n = 0, bs = 0, w = 0, nc = 0, precision = HBMC_F64;
    int32_t kernel = HBMC_KERNEL_AUTO;
    int32_t sync = HBMC_SYNC_AUTO;
    uint64_t wait_ticks = 5000000;     // time limit of a wait in the one-launch form (100 MHz ticks: 50 ms)
    bool local = false;                // ordered after a locality renumbering (hbmc_order_rcm): the row
                                       // kernel takes tiles in XCD-contiguous order, its one-launch form
                                       // admits five workgroups per CU
    int32_t rhs_tile = 0;              // right-hand sides per wavefront, 0 = automatic
    int32_t nsys = 1;
    int64_t n_pad = 0;
    double smooth_scale = 1.0;         // c of the smoothing step x += c M^-1 r: 1 (IC(0)), 2 - omega (SSOR)
    bool ssor = false;                 // the SSOR splitting rather than IC(0)
    std::vector<int64_t> color_start;
    std::vector<int64_t> sys_ptr;      // [nsys + 1] original rows of each system
    // systems: tile and 64-row group -> system; per system and color the
    // ranges of its tiles and groups ([nsys][nc][2])
    std::vector<int32_t> tile_sys, part_sys, sys_tiles, sys_parts;
    size_t off_tile_sys = 0, off_part_sys = 0, off_sys_tiles = 0, off_sys_parts = 0;
    std::vector<int64_t> tile_base;    // [nc + 1] first global tile of each color
    std::vector<int32_t> perm, iperm;
    // FP64 factor: strictly lower L in CSR over HBMC indices, and d
    std::vector<int64_t> lrp;
    std::vector<int32_t> lcol;
    std::vector<double> lval, d;
    // substitution layout
    hbmc::Packed fext, bext;   // forward: L to earlier colors; backward: U to later colors
    hbmc::Sell fint, bint;   // inside level-1 blocks; col = source step (0..bs-1)
    LayoutCounts fcnt, bcnt;   // of fext, bext
    int64_t nnz_lower = 0;     // entries of L
    // built on the device (hbmc_device_build): no host image; the image's
    // size, and where d and L stay in the build workspace (for export)
    bool device_built = false;
    size_t dev_image_bytes = 0;
    const void *dev_d = nullptr, *dev_lrp = nullptr, *dev_lcol = nullptr, *dev_lval = nullptr;
    int32_t max_int_slots_f = 0, max_int_slots_b = 0;   // per tile, summed over steps
    int32_t max_int_step_f = 0, max_int_step_b = 0;     // per (tile, step)
    // device image
    hbmc::ImageBuilder image;
    size_t off_dinv = 0, off_perm = 0, off_iperm = 0;
    TriOffsets fwd{}, bwd{};
    void *dev = nullptr;
    size_t dev_bytes = 0;
    uint64_t uid = 0;
    // captured CG iteration graphs: (matrix upload, workspace, iterations
    // and history flag, right-hand sides, right-hand-side tile) -> exec
    struct Graph {
        uint64_t matrix_uid;
        const void *work;
        int32_t iters;
        int32_t K, nr;
        void *exec;
    };
    std::vector<Graph> graphs;
};

// Pattern data for recomputing a factor and a matrix from new values of
// the same matrix on the device (ic0_refactor, hbmc_matrix_revalue).
struct hbmc_revalue_s {
    int32_t n = 0, bs = 0, w = 0, nc = 0;
    int64_t n_pad = 0, nnz = 0;           // nnz: entries of the caller's CSR
    std::vector<int64_t> color_start, tile_base;
    std::vector<int64_t> arp, amap;       // Abar rows; source entry of each Abar entry (-1: dummy diagonal 1)
    std::vector<int32_t> aci;
    std::vector<int64_t> lrp;             // strictly lower pattern of Abar
    std::vector<int32_t> lcol;
    hbmc::ImageBuilder image;             // the arrays above; device scratch follows the image
    size_t off_cs = 0, off_tb = 0, off_arp = 0, off_aci = 0, off_amap = 0, off_lrp = 0, off_lcol = 0;
    size_t off_lval = 0, off_d = 0, off_flag = 0, scratch_end = 0;
    void *dev = nullptr;
};

struct hbmc_matrix_s {
    int32_t n = 0;
    int64_t n_pad = 0;
    std::vector<double> diag;   // [n_pad]
    hbmc::Packed off;           // off-diagonal entries, 64-row slices from row 0
    // CG forms the search direction inside the product (gathering z and the
    // old direction at every coupling) when most couplings sit in strided
    // slots; otherwise it updates the direction first and gathers it alone
    bool fuse_p = true;
    hbmc::ImageBuilder image;
    size_t off_diag = 0;
    PackedOffsets offs{};
    void *dev = nullptr;
    size_t dev_bytes = 0;
    uint64_t uid = 0;
    bool device_built = false;   // built on the device: no host image
    size_t dev_image_bytes = 0;
    size_t image_bytes() const { return device_built ? dev_image_bytes : image.bytes.size(); }
};
