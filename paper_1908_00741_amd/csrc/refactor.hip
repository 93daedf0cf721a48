// New values, same pattern: IC(0) recomputed on the device (Section 2, eq.
// "ILU", the same arithmetic in the same order as the host factorization)
// and the device layouts of the factor and of Abar rewritten in place.
//
// The factorization runs one launch per color; inside a color one thread
// per BMC block walks the block's bs rows in order.  A row needs only rows
// of earlier colors (earlier launches) and earlier rows of its own block
// (Section 4.3: couplings inside a level-1 block join rows of the same lane
// only), so the threads of a launch never wait on each other.
#include <cstring>

#include "revalue.h"

extern "C" int hbmc_revalue_upload(hbmc_revalue_t *rv, void *dev, size_t bytes, void *stream) {
    clear_error();
    if (!rv || !dev) return fail(HBMC_EINVAL, "null argument");
    if (bytes < rv->scratch_end) return fail(HBMC_EINVAL, "device buffer too small (%zu < %zu)", bytes, rv->scratch_end);
    if (reinterpret_cast<uintptr_t>(dev) % 256) return fail(HBMC_EINVAL, "device buffer not 256-byte aligned");
    auto s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(dev, rv->image.bytes.data(), rv->image.bytes.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    rv->dev = dev;
    return HBMC_OK;
}

namespace {

// The factor of either splitting from new values, then its device values.
int refactor(hbmc_factor_s *f, const hbmc_revalue_s *rv, const double *val, bool ssor, double param,
             void *stream) {
    clear_error();
    if (!f || !rv || !val) return fail(HBMC_EINVAL, "null argument");
    if (!f->dev) return fail(HBMC_ENOTREADY, "factor not uploaded");
    if (!rv->dev) return fail(HBMC_ENOTREADY, "revalue data not uploaded");
    if (f->ssor != ssor)
        return fail(HBMC_EINVAL, ssor ? "ssor_refactor needs an SSOR factor" : "ic0_refactor needs an IC(0) factor");
    if (!ssor && !(param >= 0.0)) return fail(HBMC_EINVAL, "shift must be >= 0");
    if (ssor && !(param > 0.0 && param < 2.0)) return fail(HBMC_EINVAL, "omega must lie in (0, 2) (got %g)", param);
    if (!same_order(rv, f->n_pad, f->n, f->bs, f->w, f->nc, f->color_start) ||
        int64_t(rv->lcol.size()) != f->nnz_lower)
        return fail(HBMC_EINVAL, "revalue data of another order or pattern");
    auto s = static_cast<hipStream_t>(stream);
    const Rv R = rv_of(rv);
    hipLaunchKernelGGL(k_rv_gather, dim3(unsigned((rv->n_pad + 255) / 256)), dim3(256), 0, s, R, val,
                       ssor ? 0.0 : param, ssor ? 1 : 0, ssor ? param : 1.0);
    HIP_TRY(hipGetLastError());
    if (!ssor) {
        HIP_TRY(hipMemsetAsync(R.flag, 0, sizeof(int32_t), s));
        for (int c = 0; c < rv->nc; ++c) {
            const int64_t lanes = (rv->color_start[c + 1] - rv->color_start[c]) / rv->bs;
            if (lanes > 0)
                hipLaunchKernelGGL(k_rv_ic0, dim3(unsigned((lanes + 127) / 128)), dim3(128), 0, s, R, c);
        }
        HIP_TRY(hipGetLastError());
        int32_t bad = 0;
        HIP_TRY(hipMemcpyAsync(&bad, R.flag, sizeof bad, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (bad) return fail(HBMC_EBREAKDOWN, "IC(0) pivot not > 0 on the device");
    }
    const int st = f->precision == HBMC_F64 ? pack_factor<double>(f, R, s) : pack_factor<float>(f, R, s);
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(s));
    return HBMC_OK;
}

}  // namespace

extern "C" int ic0_refactor(hbmc_factor_t *f, const hbmc_revalue_t *rv, const double *val, double shift,
                            void *stream) {
    return refactor(f, rv, val, false, shift, stream);
}

extern "C" int ssor_refactor(hbmc_factor_t *f, const hbmc_revalue_t *rv, const double *val, double omega,
                             void *stream) {
    return refactor(f, rv, val, true, omega, stream);
}

extern "C" int hbmc_matrix_revalue(hbmc_matrix_t *m, const hbmc_revalue_t *rv, const double *val, void *stream) {
    clear_error();
    if (!m || !rv || !val) return fail(HBMC_EINVAL, "null argument");
    if (!m->dev) return fail(HBMC_ENOTREADY, "matrix not uploaded");
    if (!rv->dev) return fail(HBMC_ENOTREADY, "revalue data not uploaded");
    if (rv->n_pad != m->n_pad || rv->n != m->n) return fail(HBMC_EINVAL, "revalue data of another order");
    const PackedOffsets &o = m->offs;
    void *b = m->dev;
    const MatVals M{at<double>(b, m->off_diag), at<int32_t>(b, o.soff), at<int32_t>(b, o.sbase),
                    at<uint64_t>(b, o.smask), at<double>(b, o.sval), at<int32_t>(b, o.ioff),
                    at<uint64_t>(b, o.imask), at<int64_t>(b, o.ivoff), at<int32_t>(b, o.icol),
                    at<double>(b, o.ival)};
    const int64_t groups = (m->n_pad + kLanes - 1) / kLanes;
    hipLaunchKernelGGL(k_rv_matrix, dim3(unsigned(groups)), dim3(kLanes), 0, static_cast<hipStream_t>(stream),
                       rv_of(rv), M, val);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}
