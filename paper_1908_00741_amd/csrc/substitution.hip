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

// The one-launch form of the row kernel (flow.h): one system, one
// right-hand side, both substitutions, colors within the kernel's table,
// block sizes up to kFlowMaxBs.
bool hbmc::flow_ok(const hbmc_factor_s *f, int K, bool fo) {
    return f->sync == HBMC_SYNC_AUTO && !fo && K == 1 && f->nsys == 1 && f->nc >= 1 &&
           f->nc <= kFlowMaxColors && f->bs <= kFlowMaxBs && use_rows(f, f->bs, 1, 1);
}

namespace {
// Marks y and z empty for the one-launch form (rows [0, n)) unless *done;
// with err, clears it.
__global__ void __launch_bounds__(256) k_flow_fill(int64_t n, double *y, double *z, int32_t *err,
                                                   const int32_t *done) {
    if (done && *done) return;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (err && i == 0) *err = 0;
    if (i < n) {
        reinterpret_cast<uint64_t *>(y)[i] = kFlowEmpty;
        reinterpret_cast<uint64_t *>(z)[i] = kFlowEmpty;
    }
}
}  // namespace

int hbmc::apply_launch(const hbmc_factor_s *f, const double *r, double *z, void *stream,
                       const int32_t *done, const ApplyCg *cg, int K, bool fo, const Flow *flow) {
    auto s = static_cast<hipStream_t>(stream);
    const int nr = rhs_tile(f, K);
    const Flow *fl = flow && flow_ok(f, K, fo) ? flow : nullptr;
    if (fl && fl->fill) {
        const int64_t n = f->n_pad;
        hipLaunchKernelGGL(k_flow_fill, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, fl->y, z,
                           fl->reset_err ? fl->err : nullptr, done);
        HIP_TRY(hipGetLastError());
    }
    switch (f->bs) {
        case 1: return launch_bs1(f, r, z, s, done, cg, K, nr, fo, fl);
        case 2: return launch_bs2(f, r, z, s, done, cg, K, nr, fo, fl);
        case 4: return launch_bs4(f, r, z, s, done, cg, K, nr, fo, fl);
        case 8: return launch_bs8(f, r, z, s, done, cg, K, nr, fo, fl);
        case 16: return launch_bs16(f, r, z, s, done, cg, K, nr, fo, fl);
        case 32: return launch_bs32(f, r, z, s, done, cg, K, nr, fo, fl);
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

extern "C" int hbmc_factor_set_sync(hbmc_factor_t *f, int32_t sync) {
    if (!f) return fail(HBMC_EINVAL, "null handle");
    if (sync != HBMC_SYNC_AUTO && sync != HBMC_SYNC_LAUNCH) return fail(HBMC_EINVAL, "unknown sync %d", sync);
    f->sync = sync;
    release_graphs(f);
    return HBMC_OK;
}

extern "C" int hbmc_factor_set_wait_limit(hbmc_factor_t *f, int64_t us) {
    if (!f) return fail(HBMC_EINVAL, "null handle");
    if (us < 0 || us > 60000000) return fail(HBMC_EINVAL, "wait limit %lld us (0 .. 60000000)", (long long)us);
    f->wait_ticks = us == 0 ? 5000000 : uint64_t(us) * 100;
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

// Workspace of ic0_apply_ws: the error word, then y ([n_pad] doubles).
constexpr size_t kWsHead = 256;

extern "C" int ic0_apply_ws_bytes(const hbmc_factor_t *f, size_t *bytes) {
    if (!f || !bytes) return fail(HBMC_EINVAL, "null argument");
    *bytes = kWsHead + size_t(f->n_pad) * sizeof(double);
    return HBMC_OK;
}

extern "C" int ic0_apply_ws(const hbmc_factor_t *f, const double *r, double *z, int32_t nrhs, void *ws,
                            size_t ws_bytes, void *stream) {
    if (!f || !r || !z) return fail(HBMC_EINVAL, "null argument");
    if (!f->dev) return fail(HBMC_ENOTREADY, "factor not uploaded");
    if (nrhs < 1) return fail(HBMC_EINVAL, "nrhs = %d", nrhs);
    if (r == z) return fail(HBMC_EINVAL, "z must not alias r");
    if (!ws || !flow_ok(f, nrhs)) return apply_launch(f, r, z, stream, nullptr, nullptr, nrhs);
    const size_t need = kWsHead + size_t(f->n_pad) * sizeof(double);
    if (ws_bytes < need) return fail(HBMC_EINVAL, "workspace too small (%zu < %zu)", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(HBMC_EINVAL, "workspace not 256-byte aligned");
    auto *b = static_cast<uint8_t *>(ws);
    const Flow fl{reinterpret_cast<double *>(b + kWsHead), reinterpret_cast<int32_t *>(b), true, true};
    return apply_launch(f, r, z, stream, nullptr, nullptr, nrhs, false, &fl);
}
