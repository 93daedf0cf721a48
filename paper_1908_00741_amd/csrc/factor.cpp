// Host side of the factorization and of the device layouts:
//  - Abar = P A P^T with identity rows for dummy unknowns (Section 3, eq. "AB");
//  - IC(0) with zero fill (Section 2, eq. "ILU"), computed row by row;
//  - the sliced-ELL layouts used by the substitutions (Section 4.4.2) and by
//    the SpMV.
// Compiled without floating-point contraction (-ffp-contract=off).
#include <algorithm>
#include <cmath>
#include <new>

#include "hbmc_internal.h"

using namespace hbmc;

namespace {

struct Csr {
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> v;
};

// Abar in HBMC numbering, rows sorted by column, dummy rows = identity.
Csr permute(const hbmc_order_s &o, const int64_t *rp, const int32_t *ci, const double *v) {
    Csr a;
    a.rp.assign(o.n_pad + 1, 0);
    for (int64_t r = 0; r < o.n_pad; ++r) {
        const int32_t i = o.iperm[r];
        a.rp[r + 1] = a.rp[r] + (i < 0 ? 1 : rp[i + 1] - rp[i]);
    }
    a.ci.resize(a.rp.back());
    a.v.resize(a.rp.back());
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t r = 0; r < o.n_pad; ++r) {
        const int32_t i = o.iperm[r];
        int64_t at = a.rp[r];
        if (i < 0) {
            a.ci[at] = int32_t(r);
            a.v[at] = 1.0;
            continue;
        }
        row.clear();
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) row.emplace_back(o.perm[ci[p]], v ? v[p] : 0.0);
        std::sort(row.begin(), row.end(),
                  [](const auto &x, const auto &y) { return x.first < y.first; });
        for (const auto &e : row) { a.ci[at] = e.first; a.v[at] = e.second; ++at; }
    }
    return a;
}

// IC(0), row by row: for each row i and each lower entry (i, k) in
// ascending k,  L_ik = a_ik - sum_{m<k} L_im L_km / d_m  over the common
// lower pattern of rows i and k; then d_i = a_ii - sum_{m<i} L_im^2 / d_m.
// This is the same arithmetic, term for term and in the same order, as the
// right-looking elimination with overwriting, organised by rows so that
// each row is finished before the next starts.
int ic0_rows(const Csr &a, int64_t n, double shift, std::vector<int64_t> &lrp,
             std::vector<int32_t> &lcol, std::vector<double> &lval, std::vector<double> &d) {
    lrp.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        int64_t cnt = 0;
        for (int64_t p = a.rp[i]; p < a.rp[i + 1] && a.ci[p] < i; ++p) ++cnt;
        lrp[i + 1] = lrp[i] + cnt;
    }
    lcol.resize(lrp[n]);
    lval.resize(lrp[n]);
    d.assign(n, 0.0);
    for (int64_t i = 0; i < n; ++i) {
        double aii = 0.0;
        int64_t q = lrp[i];
        for (int64_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
            if (a.ci[p] < i) { lcol[q] = a.ci[p]; lval[q] = a.v[p]; ++q; }
            else if (a.ci[p] == i) aii = a.v[p];
        }
        for (int64_t p = lrp[i]; p < lrp[i + 1]; ++p) {
            const int32_t k = lcol[p];
            double s = lval[p];
            // merge row i (entries before p) with the lower row k
            int64_t x = lrp[i], y = lrp[k];
            while (x < p && y < lrp[k + 1]) {
                if (lcol[x] < lcol[y]) ++x;
                else if (lcol[x] > lcol[y]) ++y;
                else { s = s - lval[x] * lval[y] / d[lcol[x]]; ++x; ++y; }
            }
            lval[p] = s;
        }
        double s = aii * (1.0 + shift);
        for (int64_t p = lrp[i]; p < lrp[i + 1]; ++p) s = s - lval[p] * lval[p] / d[lcol[p]];
        if (!(s > 0.0) || !std::isfinite(s))
            return fail(HBMC_EBREAKDOWN, "IC(0) pivot %lld is not > 0 (%g)", (long long)i, s);
        d[i] = s;
    }
    return HBMC_OK;
}

// A list of (column, value) couplings per row, packed as sliced ELL with
// slices of kTileLanes rows; missing slots get column -1 and value 0.
void pack_ext(const std::vector<std::vector<std::pair<int32_t, double>>> &rows, int64_t row0,
              int64_t row1, Sell &s) {
    const int64_t nslices = (row1 - row0 + kTileLanes - 1) / kTileLanes;
    for (int64_t g = 0; g < nslices; ++g) {
        size_t len = 0;
        for (int64_t r = row0 + g * kTileLanes; r < std::min(row1, row0 + (g + 1) * kTileLanes); ++r)
            len = std::max(len, rows[r].size());
        const int64_t base = s.off.back();
        s.off.push_back(int32_t(base + len));
        s.val.resize((base + len) * kTileLanes, 0.0);
        s.col.resize((base + len) * kTileLanes, -1);
        for (int64_t r = row0 + g * kTileLanes; r < std::min(row1, row0 + (g + 1) * kTileLanes); ++r) {
            const int lane = int((r - row0) % kTileLanes);
            for (size_t t = 0; t < rows[r].size(); ++t) {
                s.col[(base + t) * kTileLanes + lane] = rows[r][t].first;
                s.val[(base + t) * kTileLanes + lane] = rows[r][t].second;
            }
        }
    }
}

template <class T>
std::vector<T> cast(const std::vector<double> &v) {
    return std::vector<T>(v.begin(), v.end());
}

}  // namespace

extern "C" int ic0_factor(const hbmc_order_t *o, const int64_t *rowptr, const int32_t *col,
                          const double *val, int32_t precision, double shift, hbmc_factor_t **out) {
    clear_error();
    if (!out) return fail(HBMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!o || !val) return fail(HBMC_EINVAL, "null argument");
    if (precision != HBMC_F64 && precision != HBMC_F32)
        return fail(HBMC_EINVAL, "precision must be HBMC_F64 or HBMC_F32");
    if (!(shift >= 0.0)) return fail(HBMC_EINVAL, "shift must be >= 0");
    int st = check_csr(o->n, rowptr, col, val);
    if (st) return st;
    try {
        auto *f = new hbmc_factor_s;
        f->n = o->n; f->bs = o->bs; f->w = o->w; f->nc = o->nc; f->precision = precision;
        f->n_pad = o->n_pad;
        f->color_start = o->color_start;
        f->perm = o->perm;
        f->iperm = o->iperm;
        const Csr a = permute(*o, rowptr, col, val);
        st = ic0_rows(a, f->n_pad, shift, f->lrp, f->lcol, f->lval, f->d);
        if (st) { delete f; return st; }

        const int64_t n = f->n_pad;
        const int bs = f->bs, w = f->w;
        const int64_t l1 = int64_t(bs) * w;
        std::vector<double> dinv(n);
        for (int64_t i = 0; i < n; ++i) dinv[i] = 1.0 / f->d[i];
        // color of each HBMC row
        std::vector<int32_t> color(n);
        for (int c = 0; c < f->nc; ++c)
            for (int64_t r = f->color_start[c]; r < f->color_start[c + 1]; ++r) color[r] = c;
        // the step of row r inside its level-1 block, and its chain lane
        auto step_of = [&](int64_t r) { return int(((r - f->color_start[color[r]]) % l1) / w); };

        // couplings of each row: forward (lower) and backward (upper, scaled
        // by diaginv of the row: U = I + D^-1 L^T), split into couplings to
        // other colors (ext) and inside the level-1 block (int)
        std::vector<std::vector<std::pair<int32_t, double>>> fe(n), fi(n), be(n), bi(n);
        for (int64_t r = 0; r < n; ++r) {
            const int64_t lb = (r - f->color_start[color[r]]) / l1;
            for (int64_t p = f->lrp[r]; p < f->lrp[r + 1]; ++p) {
                const int32_t k = f->lcol[p];
                const double lv = f->lval[p];
                // (r, k) lower: forward coupling of r; (k, r) upper: backward of k
                if (color[k] != color[r]) {
                    fe[r].emplace_back(k, lv);
                    be[k].emplace_back(int32_t(r), dinv[k] * lv);
                } else {
                    const int64_t lbk = (k - f->color_start[color[k]]) / l1;
                    if (lbk != lb || (r - k) % w != 0) {
                        delete f;
                        return fail(HBMC_EINVAL, "internal: coupling (%lld,%d) crosses level-1 blocks",
                                    (long long)r, k);
                    }
                    fi[r].emplace_back(step_of(k), lv);
                    bi[k].emplace_back(step_of(r), dinv[k] * lv);
                }
            }
        }
        // be and bi were filled in ascending r, so they are already sorted

        // forward/backward ext: per color, 64-row slices from the color start
        f->slice_base.assign(f->nc + 1, 0);
        f->tile_base.assign(f->nc + 1, 0);
        f->fext.off.assign(1, 0);
        f->bext.off.assign(1, 0);
        for (int c = 0; c < f->nc; ++c) {
            const int64_t r0 = f->color_start[c], r1 = f->color_start[c + 1];
            f->slice_base[c + 1] = f->slice_base[c] + (r1 - r0 + kTileLanes - 1) / kTileLanes;
            const int64_t lanes = (r1 - r0) / bs;   // = level-1 blocks * w
            f->tile_base[c + 1] = f->tile_base[c] + (lanes + kTileLanes - 1) / kTileLanes;
            pack_ext(fe, r0, r1, f->fext);
            pack_ext(be, r0, r1, f->bext);
        }
        // int: per tile (kTileLanes chain lanes) and step l, slot-major over lanes
        auto pack_int = [&](const std::vector<std::vector<std::pair<int32_t, double>>> &rows,
                            Sell &s, int32_t &max_slots) {
            s.off.assign(1, 0);
            max_slots = 0;
            for (int c = 0; c < f->nc; ++c) {
                const int64_t r0 = f->color_start[c];
                const int64_t lanes = (f->color_start[c + 1] - r0) / bs;
                for (int64_t t0 = 0; t0 < lanes; t0 += kTileLanes) {
                    int32_t tile_slots = 0;
                    for (int l = 0; l < bs; ++l) {
                        auto row_of = [&](int64_t lam) {
                            return r0 + (lam / w) * l1 + int64_t(l) * w + lam % w;
                        };
                        size_t len = 0;
                        for (int64_t lam = t0; lam < std::min(lanes, t0 + kTileLanes); ++lam)
                            len = std::max(len, rows[row_of(lam)].size());
                        const int64_t base = s.off.back();
                        s.off.push_back(int32_t(base + len));
                        s.val.resize((base + len) * kTileLanes, 0.0);
                        s.col.resize((base + len) * kTileLanes, l);   // padding reads its own step
                        for (int64_t lam = t0; lam < std::min(lanes, t0 + kTileLanes); ++lam) {
                            const auto &e = rows[row_of(lam)];
                            for (size_t t = 0; t < e.size(); ++t) {
                                s.col[(base + t) * kTileLanes + (lam - t0)] = e[t].first;
                                s.val[(base + t) * kTileLanes + (lam - t0)] = e[t].second;
                            }
                        }
                        tile_slots += int32_t(len);
                    }
                    max_slots = std::max(max_slots, tile_slots);
                }
            }
        };
        pack_int(fi, f->fint, f->max_int_slots_f);
        pack_int(bi, f->bint, f->max_int_slots_b);

        // device image
        auto &im = f->image;
        auto add_tri = [&](const Sell &e, const Sell &i, TriOffsets &t) {
            t.ext_off = im.add(e.off);
            t.ext_col = im.add(e.col);
            t.int_off = im.add(i.off);
            t.int_lp = im.add(i.col);
            if (precision == HBMC_F64) {
                t.ext_val = im.add(e.val);
                t.int_val = im.add(i.val);
            } else {
                t.ext_val = im.add(cast<float>(e.val));
                t.int_val = im.add(cast<float>(i.val));
            }
        };
        f->off_dinv = precision == HBMC_F64 ? im.add(dinv) : im.add(cast<float>(dinv));
        f->off_perm = im.add(f->perm);
        f->off_iperm = im.add(f->iperm);
        add_tri(f->fext, f->fint, f->fwd);
        add_tri(f->bext, f->bint, f->bwd);
        im.bytes.resize((im.bytes.size() + 255) & ~size_t(255));
        *out = f;
        return HBMC_OK;
    } catch (const std::bad_alloc &) {
        return fail(HBMC_ENOMEM, "out of host memory in ic0_factor");
    }
}

extern "C" int hbmc_factor_export(const hbmc_factor_t *f, double *d, int64_t *lower_rowptr,
                                  int32_t *lower_col, double *lower_val, int64_t *lower_nnz) {
    if (!f) return fail(HBMC_EINVAL, "null handle");
    if (lower_nnz) *lower_nnz = int64_t(f->lcol.size());
    if (d) std::copy(f->d.begin(), f->d.end(), d);
    if (lower_rowptr) std::copy(f->lrp.begin(), f->lrp.end(), lower_rowptr);
    if (lower_col) std::copy(f->lcol.begin(), f->lcol.end(), lower_col);
    if (lower_val) std::copy(f->lval.begin(), f->lval.end(), lower_val);
    return HBMC_OK;
}

extern "C" int hbmc_factor_device_bytes(const hbmc_factor_t *f, size_t *bytes) {
    if (!f || !bytes) return fail(HBMC_EINVAL, "null argument");
    *bytes = f->image.bytes.size();
    return HBMC_OK;
}

extern "C" void hbmc_factor_destroy(hbmc_factor_t *f) { delete f; }

extern "C" int hbmc_matrix_create(const hbmc_order_t *o, const int64_t *rowptr, const int32_t *col,
                                  const double *val, hbmc_matrix_t **out) {
    clear_error();
    if (!out) return fail(HBMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!o || !val) return fail(HBMC_EINVAL, "null argument");
    int st = check_csr(o->n, rowptr, col, val);
    if (st) return st;
    try {
        auto *m = new hbmc_matrix_s;
        m->n = o->n;
        m->n_pad = o->n_pad;
        const Csr a = permute(*o, rowptr, col, val);
        m->diag.assign(m->n_pad, 0.0);
        std::vector<std::vector<std::pair<int32_t, double>>> rows(m->n_pad);
        for (int64_t r = 0; r < m->n_pad; ++r)
            for (int64_t p = a.rp[r]; p < a.rp[r + 1]; ++p) {
                if (a.ci[p] == r) m->diag[r] = a.v[p];
                else rows[r].emplace_back(a.ci[p], a.v[p]);
            }
        m->off.off.assign(1, 0);
        pack_ext(rows, 0, m->n_pad, m->off);
        m->off_diag = m->image.add(m->diag);
        m->off_soff = m->image.add(m->off.off);
        m->off_val = m->image.add(m->off.val);
        m->off_col = m->image.add(m->off.col);
        m->image.bytes.resize((m->image.bytes.size() + 255) & ~size_t(255));
        *out = m;
        return HBMC_OK;
    } catch (const std::bad_alloc &) {
        return fail(HBMC_ENOMEM, "out of host memory in hbmc_matrix_create");
    }
}

extern "C" int hbmc_matrix_device_bytes(const hbmc_matrix_t *m, size_t *bytes) {
    if (!m || !bytes) return fail(HBMC_EINVAL, "null argument");
    *bytes = m->image.bytes.size();
    return HBMC_OK;
}

extern "C" void hbmc_matrix_destroy(hbmc_matrix_t *m) { delete m; }
