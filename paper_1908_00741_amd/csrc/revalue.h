// Device kernels shared by the device refactorization (refactor.hip) and
// the device build of factors and matrices (devbuild.hip): IC(0) on the
// device (Section 2, eq. "ILU", the same arithmetic in the same order as the
// host factorization, one launch per color, one thread per BMC block, its
// rows in order: a row needs only rows of earlier colors and earlier rows
// of its own block, Section 4.3) and the values of the factor's and the
// matrix's device layouts.  Included by one translation unit each; the
// kernels live in an anonymous namespace.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "hbmc_internal.h"

#define HIP_TRY(call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return hbmc::fail(HBMC_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

using namespace hbmc;

namespace {

constexpr int kLanes = kTileLanes;

template <class P>
P *at(void *base, size_t off) {
    return reinterpret_cast<P *>(static_cast<uint8_t *>(base) + off);
}

// The pattern data and scratch on the device.
struct Rv {
    const int64_t *cs, *tb;          // color starts, first tile of each color
    const int64_t *arp, *amap;       // Abar rows, source entry of each value (-1: dummy diagonal)
    const int32_t *aci;
    const int64_t *lrp;              // strictly lower pattern
    const int32_t *lcol;
    double *lval, *d;                // the factor being computed
    int32_t *flag;                   // set when a pivot is not > 0
    int32_t nc, bs, w;
    int64_t n_pad;
};

Rv rv_of(const hbmc_revalue_s *r) {
    void *b = r->dev;
    return Rv{at<int64_t>(b, r->off_cs), at<int64_t>(b, r->off_tb), at<int64_t>(b, r->off_arp),
              at<int64_t>(b, r->off_amap), at<int32_t>(b, r->off_aci), at<int64_t>(b, r->off_lrp),
              at<int32_t>(b, r->off_lcol), at<double>(b, r->off_lval), at<double>(b, r->off_d),
              at<int32_t>(b, r->off_flag), r->nc, r->bs, r->w, r->n_pad};
}

// Position of column c in the sorted columns [lo, hi) of a row, or -1.
__device__ inline int64_t find_col(const int32_t *cols, int64_t lo, int64_t hi, int32_t c) {
    const int64_t end = hi;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cols[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return lo < end && cols[lo] == c ? lo : -1;
}

// Abar(r, c) from the caller's values; 0 outside the pattern.
__device__ inline double abar_at(const Rv &R, const double *val, int64_t r, int32_t c) {
    const int64_t q = find_col(R.aci, R.arp[r], R.arp[r + 1], c);
    if (q < 0) return 0.0;
    const int64_t m = R.amap[q];
    return m >= 0 ? val[m] : 1.0;
}

// L(r, c), c < r, of the factor being computed; 0 outside the pattern.
__device__ inline double l_at(const Rv &R, int64_t r, int32_t c) {
    const int64_t q = find_col(R.lcol, R.lrp[r], R.lrp[r + 1], c);
    return q < 0 ? 0.0 : R.lval[q];
}

// The color of global tile t.
__device__ inline int color_of_tile(const Rv &R, int64_t t) {
    int c = 0;
    while (c + 1 < R.nc && R.tb[c + 1] <= t) ++c;
    return c;
}

// Row of chain lane lam at step l of color c.
__device__ inline int64_t row_of(const Rv &R, int c, int64_t lam, int l) {
    const int64_t l1 = int64_t(R.bs) * R.w;
    return R.cs[c] + (lam / R.w) * l1 + int64_t(l) * R.w + lam % R.w;
}

// Lower values and diagonals of Abar, from the caller's values: the
// diagonal times (1 + shift) for IC(0), divided by omega for the SSOR
// splitting (ssor != 0).
__global__ void k_rv_gather(Rv R, const double *__restrict__ val, double shift, int ssor, double omega) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= R.n_pad) return;
    int64_t q = R.lrp[r];
    for (int64_t p = R.arp[r]; p < R.arp[r + 1]; ++p) {
        const int32_t c = R.aci[p];
        const double v = R.amap[p] >= 0 ? val[R.amap[p]] : 1.0;
        if (c < r) R.lval[q++] = v;
        else if (c == r) R.d[r] = ssor ? v / omega : v * (1.0 + shift);
    }
}

// IC(0) of the rows of color c, one thread per BMC block, its rows in order:
// for each lower entry (i, k) in ascending k, L_ik = a_ik - sum over the
// common lower pattern of rows i and k of L_im L_km / d_m; then d_i = a_ii -
// sum of L_im^2 / d_m.
__global__ void k_rv_ic0(Rv R, int c) {
    const int64_t lam = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (lam >= (R.cs[c + 1] - R.cs[c]) / R.bs) return;
    bool bad = false;
    for (int l = 0; l < R.bs; ++l) {
        const int64_t i = row_of(R, c, lam, l);
        const int64_t b = R.lrp[i], e = R.lrp[i + 1];
        for (int64_t p = b; p < e; ++p) {
            const int32_t k = R.lcol[p];
            double s = R.lval[p];
            int64_t x = b, y = R.lrp[k];
            const int64_t ye = R.lrp[k + 1];
            while (x < p && y < ye) {
                const int32_t cx = R.lcol[x], cy = R.lcol[y];
                if (cx < cy) ++x;
                else if (cx > cy) ++y;
                else { s = s - R.lval[x] * R.lval[y] / R.d[cx]; ++x; ++y; }
            }
            R.lval[p] = s;
        }
        double s = R.d[i];
        for (int64_t p = b; p < e; ++p) s = s - R.lval[p] * R.lval[p] / R.d[R.lcol[p]];
        R.d[i] = s;
        bad = bad || !(s > 0.0) || !isfinite(s);
    }
    if (bad) R.flag[0] = 1;
}

// Where one direction's values live in the factor image.
template <typename T>
struct Dir {
    const int32_t *soff, *sbase;
    const uint64_t *smask;
    T *sval;
    const int32_t *ioff;      // indexed slots
    const uint64_t *imask;
    const int64_t *ivoff;
    const int32_t *icol;
    T *ival;
    const int64_t *goff;      // flat form: first entry of each group
    const uint16_t *lstart;   // first entry of each lane, relative to goff
    const int32_t *fcol;
    T *fval;
    bool flat;
    const int32_t *int_off;
    const int8_t *int_lp;
    T *int_val;
};

// Rewrites the values of one direction, one workgroup of 64 lanes per
// (tile, step) group: forward L(row, col); backward, with the row as the
// upper side, (1 / d_row) L(col, row).
template <typename T, bool BACKWARD>
__global__ void __launch_bounds__(kLanes) k_rv_pack(Rv R, Dir<T> D) {
    const int64_t g = blockIdx.x;
    const int j = threadIdx.x;
    const int64_t t = g / R.bs;
    const int l = int(g % R.bs);
    const int c = color_of_tile(R, t);
    const int64_t lam = (t - R.tb[c]) * kLanes + j;
    if (lam >= (R.cs[c + 1] - R.cs[c]) / R.bs) return;   // no row: no entries in any slot
    const int64_t row = row_of(R, c, lam, l);
    auto value = [&](int32_t col) -> T {
        if (BACKWARD) {
            const double dinv = 1.0 / R.d[row];
            return T(dinv * l_at(R, col, int32_t(row)));
        }
        return T(l_at(R, row, col));
    };
    for (int32_t s = D.soff[g]; s < D.soff[g + 1]; ++s)
        if ((D.smask[s] >> j) & 1) D.sval[int64_t(s) * kLanes + j] = value(D.sbase[s] + j);
    if (D.flat) {
        const int64_t g0 = D.goff[g];
        const int64_t a = g0 + D.lstart[g * kLanes + j];
        const int64_t b = j + 1 < kLanes ? g0 + D.lstart[g * kLanes + j + 1] : D.goff[g + 1];
        for (int64_t e = a; e < b; ++e) D.fval[e] = value(D.fcol[e]);
    } else {
        for (int32_t s = D.ioff[g]; s < D.ioff[g + 1]; ++s) {
            const uint64_t mask = D.imask[s];
            if (!((mask >> j) & 1)) continue;
            const int64_t e = D.ivoff[s] + __builtin_popcountll(mask & ((uint64_t(1) << j) - 1));
            D.ival[e] = value(D.icol[e]);
        }
    }
    for (int32_t s = D.int_off[g]; s < D.int_off[g + 1]; ++s) {
        const int lp = D.int_lp[int64_t(s) * kLanes + j];
        if (lp >= 0) D.int_val[int64_t(s) * kLanes + j] = value(int32_t(row_of(R, c, lam, lp)));
    }
}

template <typename T>
__global__ void k_rv_dinv(Rv R, T *__restrict__ dinv) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < R.n_pad) dinv[i] = T(1.0 / R.d[i]);
}

// Abar's values in the SpMV layout, one workgroup per 64-row group.
struct MatVals {
    double *diag;
    const int32_t *soff, *sbase;
    const uint64_t *smask;
    double *sval;
    const int32_t *ioff;
    const uint64_t *imask;
    const int64_t *ivoff;
    const int32_t *icol;
    double *ival;
};

__global__ void __launch_bounds__(kLanes) k_rv_matrix(Rv R, MatVals M, const double *__restrict__ val) {
    const int64_t g = blockIdx.x;
    const int j = threadIdx.x;
    const int64_t row = g * kLanes + j;
    if (row >= R.n_pad) return;
    M.diag[row] = abar_at(R, val, row, int32_t(row));
    for (int32_t s = M.soff[g]; s < M.soff[g + 1]; ++s)
        if ((M.smask[s] >> j) & 1) M.sval[int64_t(s) * kLanes + j] = abar_at(R, val, row, M.sbase[s] + j);
    for (int32_t s = M.ioff[g]; s < M.ioff[g + 1]; ++s) {
        const uint64_t mask = M.imask[s];
        if (!((mask >> j) & 1)) continue;
        const int64_t e = M.ivoff[s] + __builtin_popcountll(mask & ((uint64_t(1) << j) - 1));
        M.ival[e] = abar_at(R, val, row, M.icol[e]);
    }
}

template <typename T>
Dir<T> dir_of(hbmc_factor_s *f, const TriOffsets &o, bool flat) {
    void *b = f->dev;
    const PackedOffsets &x = o.ext;
    return Dir<T>{at<int32_t>(b, x.soff), at<int32_t>(b, x.sbase), at<uint64_t>(b, x.smask), at<T>(b, x.sval),
                  at<int32_t>(b, x.ioff), at<uint64_t>(b, x.imask), at<int64_t>(b, x.ivoff),
                  at<int32_t>(b, x.icol), at<T>(b, x.ival),
                  at<int64_t>(b, x.goff), at<uint16_t>(b, x.lstart), at<int32_t>(b, x.fcol), at<T>(b, x.fval), flat,
                  at<int32_t>(b, o.int_off), at<int8_t>(b, o.int_lp), at<T>(b, o.int_val)};
}

template <typename T>
int pack_factor(hbmc_factor_s *f, const Rv &R, hipStream_t s) {
    const int64_t groups = f->tile_base[f->nc] * f->bs;
    if (groups > 0) {
        hipLaunchKernelGGL((k_rv_pack<T, false>), dim3(unsigned(groups)), dim3(kLanes), 0, s, R,
                           dir_of<T>(f, f->fwd, f->fcnt.flat));
        hipLaunchKernelGGL((k_rv_pack<T, true>), dim3(unsigned(groups)), dim3(kLanes), 0, s, R,
                           dir_of<T>(f, f->bwd, f->bcnt.flat));
    }
    hipLaunchKernelGGL(k_rv_dinv<T>, dim3(unsigned((f->n_pad + 255) / 256)), dim3(256), 0, s, R,
                       at<T>(f->dev, f->off_dinv));
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

bool same_order(const hbmc_revalue_s *rv, int64_t n_pad, int32_t n, int32_t bs, int32_t w, int32_t nc,
                const std::vector<int64_t> &cs) {
    return rv->n_pad == n_pad && rv->n == n && rv->bs == bs && rv->w == w && rv->nc == nc && rv->color_start == cs;
}

}  // namespace
