// Preconditioning step z = M^-1 r: dispatch by block size to the
// substitution kernels (sweep.h, instantiated per block size in
// sweep_bs*.hip), the choice of the right-hand-side tile, and the C ABI of
// the factor's device side.
#include <hip/hip_runtime.h>

#include "sweep.h"

using namespace hbmc;

#define HIP_TRY(call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(HBMC_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

namespace {
bool tile_ok(int nr) { return nr == 4 || nr == 8 || nr == 16; }
}  // namespace

// Right-hand sides per wavefront: 1 for one right-hand side; else the
// factor's setting, or 4 below eight right-hand sides and 8 from eight on
// (lanes past K idle, so the tile should not exceed K by much).
int hbmc::rhs_tile(const hbmc_factor_s *f, int K) {
    if (K == 1) return 1;
    if (f->rhs_tile > 0) return f->rhs_tile;
    return K < 8 ? 4 : 8;
}

// Which kernel runs the phases: one wavefront per tile (k_sweep) or one
// workgroup of bs wavefronts per tile (k_rows, one right-hand side only).
// Automatic choice: k_rows when the colors have few tiles on average (fewer
// than 1024: a phase would not fill the chip with one wavefront per tile)
// and the factor holds its left-over couplings in flat form (unstructured
// graphs: each step has many couplings, whose loads k_rows spreads over bs
// wavefronts, and with row splitting evenly over the lanes).  On
// grids a step has a few strided slots, and k_rows' single chain wavefront
// after the barrier costs more than it saves (96^3, bs 8: 75.7 against
// 38.0 us per apply; 1M-point 13-NN graph, bs 2: 300 against 370 us).
bool hbmc::use_rows(const hbmc_factor_s *f, int bs, int K, int nr) {
    if (bs > 16 || K != 1 || nr != 1) return false;
    if (f->kernel == HBMC_KERNEL_SWEEP) return false;
    if (f->kernel == HBMC_KERNEL_ROWS) return true;
    return f->tile_base[f->nc] < 1024 * int64_t(f->nc) && f->fcnt.flat;
}

int hbmc::apply_launch(const hbmc_factor_s *f, const double *r, double *z, void *stream,
                       const int32_t *done, const ApplyCg *cg, int K, bool fo) {
    auto s = static_cast<hipStream_t>(stream);
    const int nr = rhs_tile(f, K);
    switch (f->bs) {
        case 1: return launch_bs1(f, r, z, s, done, cg, K, nr, fo);
        case 2: return launch_bs2(f, r, z, s, done, cg, K, nr, fo);
        case 4: return launch_bs4(f, r, z, s, done, cg, K, nr, fo);
        case 8: return launch_bs8(f, r, z, s, done, cg, K, nr, fo);
        case 16: return launch_bs16(f, r, z, s, done, cg, K, nr, fo);
        case 32: return launch_bs32(f, r, z, s, done, cg, K, nr, fo);
        default: return fail(HBMC_EINVAL, "bs = %d has no device kernel (1, 2, 4, 8, 16, 32)", f->bs);
    }
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int hbmc_factor_upload(hbmc_factor_t *f, void *dev, size_t bytes, void *stream) {
    clear_error();
    if (!f || !dev) return fail(HBMC_EINVAL, "null argument");
    if (f->device_built) return fail(HBMC_EINVAL, "a factor built on the device is already uploaded");
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

extern "C" int hbmc_factor_set_rhs_tile(hbmc_factor_t *f, int32_t nr) {
    if (!f) return fail(HBMC_EINVAL, "null handle");
    if (nr != 0 && !tile_ok(nr)) return fail(HBMC_EINVAL, "right-hand-side tile %d (0, 4, 8, 16)", nr);
    f->rhs_tile = nr;
    release_graphs(f);
    return HBMC_OK;
}

extern "C" int ic0_apply(const hbmc_factor_t *f, const double *r, double *z, int32_t nrhs, void *stream) {
    if (!f || !r || !z) return fail(HBMC_EINVAL, "null argument");
    if (!f->dev) return fail(HBMC_ENOTREADY, "factor not uploaded");
    if (nrhs < 1) return fail(HBMC_EINVAL, "nrhs = %d", nrhs);
    if (r == z) return fail(HBMC_EINVAL, "z must not alias r");
    return apply_launch(f, r, z, stream, nullptr, nullptr, nrhs);
}
