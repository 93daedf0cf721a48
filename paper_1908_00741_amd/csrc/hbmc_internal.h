// Internal declarations shared by the host setup (order.cpp, factor.cpp) and
// the device code (hbmc.hip).  Not part of the public interface.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hbmc.h"

namespace hbmc {

// Records a message for hbmc_last_error() and returns code.
int fail(int code, const char *fmt, ...);
void clear_error();

// Rows of one phase are processed in tiles of kTileLanes lanes x bs steps;
// the sliced-ELL slices are kTileLanes rows high.  kTileLanes is the
// wavefront width of gfx950.
constexpr int kTileLanes = 64;

// Checks a CSR pattern: sizes, sorted in-range columns, diagonal present,
// symmetric pattern.  Values (if given) must be symmetric with a positive
// diagonal.
int check_csr(int32_t n, const int64_t *rowptr, const int32_t *col, const double *val);

// A sliced-ELL array on the host: slot offsets per slice, then slot-major
// values and columns, kTileLanes entries per slot.
struct Sell {
    std::vector<int32_t> off;   // [slices + 1]
    std::vector<double> val;    // [slots * kTileLanes]
    std::vector<int32_t> col;   // [slots * kTileLanes]
    int64_t slots() const { return off.empty() ? 0 : off.back(); }
};

// Byte layout of a device image: every array starts on a 256-byte boundary.
struct ImageBuilder {
    std::vector<uint8_t> bytes;
    size_t add(const void *src, size_t n);
    template <class T> size_t add(const std::vector<T> &v) { return add(v.data(), v.size() * sizeof(T)); }
};

}  // namespace hbmc

struct hbmc_order_s {
    int32_t n = 0, bs = 0, w = 0, nc = 0;
    int64_t n_pad = 0, nblocks = 0;
    std::vector<int32_t> perm;         // [n]    original -> HBMC
    std::vector<int32_t> iperm;        // [n_pad] HBMC -> original, -1 for dummies
    std::vector<int64_t> color_start;  // [nc + 1]
};

// Offsets (bytes, inside the device image) of one triangular direction.
struct TriOffsets {
    size_t ext_off, ext_val, ext_col;   // per 64-row slice: couplings to other colors
    size_t int_off, int_val, int_lp;    // per (tile, step): couplings inside the level-1 block
};

struct hbmc_factor_s {
    int32_t n = 0, bs = 0, w = 0, nc = 0, precision = HBMC_F64;
    int64_t n_pad = 0;
    std::vector<int64_t> color_start;
    std::vector<int64_t> slice_base;   // [nc + 1] first global slice of each color
    std::vector<int64_t> tile_base;    // [nc + 1] first global tile of each color
    std::vector<int32_t> perm, iperm;
    // FP64 factor: strictly lower L in CSR over HBMC indices, and d
    std::vector<int64_t> lrp;
    std::vector<int32_t> lcol;
    std::vector<double> lval, d;
    // substitution layout
    hbmc::Sell fext, bext;   // forward: L to earlier colors; backward: U to later colors
    hbmc::Sell fint, bint;   // inside level-1 blocks; col = source step (0..bs-1)
    int32_t max_int_slots_f = 0, max_int_slots_b = 0;   // per tile, summed over steps
    // device image
    hbmc::ImageBuilder image;
    size_t off_dinv = 0, off_perm = 0, off_iperm = 0;
    TriOffsets fwd{}, bwd{};
    void *dev = nullptr;
    size_t dev_bytes = 0;
};

struct hbmc_matrix_s {
    int32_t n = 0;
    int64_t n_pad = 0;
    std::vector<double> diag;   // [n_pad]
    hbmc::Sell off;             // off-diagonal entries, 64-row slices from row 0
    hbmc::ImageBuilder image;
    size_t off_diag = 0, off_soff = 0, off_val = 0, off_col = 0;
    void *dev = nullptr;
    size_t dev_bytes = 0;
};
