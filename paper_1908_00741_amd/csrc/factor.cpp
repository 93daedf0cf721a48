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

template <class T>
std::vector<T> cast(const std::vector<double> &v) {
    return std::vector<T>(v.begin(), v.end());
}

template <class T>
size_t add_packed(ImageBuilder &im, const Packed &p, bool f32, PackedOffsets &o) {
    o.soff = im.add(p.soff);
    o.sbase = im.add(p.sbase);
    o.smask = im.add(p.smask);
    o.sval = f32 ? im.add(cast<float>(p.sval)) : im.add(p.sval);
    o.ioff = im.add(p.ioff);
    o.icol = im.add(p.icol);
    o.ival = f32 ? im.add(cast<float>(p.ival)) : im.add(p.ival);
    return o.soff;
}

}  // namespace

int Packed::add_group(const std::vector<const Couplings *> &lanes, int64_t limit, int budget) {
    const int nl = int(lanes.size());
    // every coupling (lane j, column c) proposes the strided base c - j
    struct Entry { int64_t key; int lane; int idx; };
    std::vector<Entry> all;
    for (int j = 0; j < nl; ++j)
        if (lanes[j])
            for (int t = 0; t < int(lanes[j]->size()); ++t)
                all.push_back({int64_t((*lanes[j])[t].first) - j, j, t});
    entries += int64_t(all.size());
    std::sort(all.begin(), all.end(), [](const Entry &a, const Entry &b) {
        return a.key != b.key ? a.key < b.key : a.lane < b.lane;
    });
    // bases shared by enough lanes become strided slots, most shared first
    struct Cand { int64_t key; size_t first, count; };
    std::vector<Cand> cands;
    for (size_t i = 0; i < all.size();) {
        size_t k = i;
        while (k < all.size() && all[k].key == all[i].key) ++k;
        const int64_t key = all[i].key;
        if (int(k - i) >= kMinStridedLanes && key >= 0 && key + kTileLanes <= limit)
            cands.push_back({key, i, k - i});
        i = k;
    }
    std::stable_sort(cands.begin(), cands.end(),
                     [](const Cand &a, const Cand &b) { return a.count > b.count; });
    if (int(cands.size()) > std::max(budget, 0)) cands.resize(std::max(budget, 0));
    std::vector<std::vector<uint8_t>> used(nl);
    for (int j = 0; j < nl; ++j)
        if (lanes[j]) used[j].assign(lanes[j]->size(), 0);
    for (const Cand &c : cands) {
        const int64_t slot = int64_t(sbase.size());
        sbase.push_back(int32_t(c.key));
        uint64_t mask = 0;
        sval.resize((slot + 1) * kTileLanes, 0.0);
        for (size_t i = c.first; i < c.first + c.count; ++i) {
            const Entry &e = all[i];
            mask |= uint64_t(1) << e.lane;
            sval[slot * kTileLanes + e.lane] = (*lanes[e.lane])[e.idx].second;
            used[e.lane][e.idx] = 1;
        }
        smask.push_back(mask);
    }
    soff.push_back(int32_t(sbase.size()));
    max_strided = std::max(max_strided, int32_t(cands.size()));
    // the rest, per lane in column order, as indexed slots
    size_t len = 0;
    for (int j = 0; j < nl; ++j)
        if (lanes[j]) {
            size_t left = 0;
            for (uint8_t u : used[j]) left += !u;
            len = std::max(len, left);
        }
    const int64_t base = ioff.back();
    ioff.push_back(int32_t(base + len));
    icol.resize((base + len) * kTileLanes, -1);
    ival.resize((base + len) * kTileLanes, 0.0);
    for (int j = 0; j < nl; ++j) {
        if (!lanes[j]) continue;
        int64_t t = 0;
        for (size_t i = 0; i < lanes[j]->size(); ++i)
            if (!used[j][i]) {
                icol[(base + t) * kTileLanes + j] = (*lanes[j])[i].first;
                ival[(base + t) * kTileLanes + j] = (*lanes[j])[i].second;
                ++t;
            }
    }
    max_indexed = std::max(max_indexed, int32_t(len));
    return int(cands.size());
}

void Packed::finish() {
    sbase.push_back(0);
    smask.push_back(0);
    sval.resize(sval.size() + kTileLanes, 0.0);
    icol.resize(icol.size() + kTileLanes, -1);
    ival.resize(ival.size() + kTileLanes, 0.0);
}

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
        f->nsys = o->nsys;
        f->sys_ptr = o->sys_ptr;
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
        std::vector<Couplings> fe(n), fi(n), be(n), bi(n);
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

        // Layout of the substitutions: per color, the chain lanes (one per BMC
        // block, lam = level-1 block * w + m) are cut into tiles of 64 lanes;
        // for each (tile, step l) a sliced-ELL slot list holds, slot-major,
        // one entry per lane: the couplings of row  S_c + (lam / w) bs w +
        // l w + lam % w.  Missing entries have column -1 and value 0.  Each
        // array ends with one extra all-padding slot that loads may target
        // instead of branching.
        f->tile_base.assign(f->nc + 1, 0);
        for (int c = 0; c < f->nc; ++c) {
            const int64_t lanes = (f->color_start[c + 1] - f->color_start[c]) / bs;
            f->tile_base[c + 1] = f->tile_base[c] + (lanes + kTileLanes - 1) / kTileLanes;
        }
        // couplings to other colors: one Packed group per (tile, step)
        std::vector<const Couplings *> lanes_f, lanes_b;
        for (int c = 0; c < f->nc; ++c) {
            const int64_t r0 = f->color_start[c];
            const int64_t lanes = (f->color_start[c + 1] - r0) / bs;
            for (int64_t t0 = 0; t0 < lanes; t0 += kTileLanes) {
                // the kernel fetches a tile's strided-slot metadata one slot per lane
                int budget_f = kTileLanes, budget_b = kTileLanes;
                for (int l = 0; l < bs; ++l) {
                    lanes_f.assign(kTileLanes, nullptr);
                    lanes_b.assign(kTileLanes, nullptr);
                    for (int64_t lam = t0; lam < std::min(lanes, t0 + kTileLanes); ++lam) {
                        const int64_t row = r0 + (lam / w) * l1 + int64_t(l) * w + lam % w;
                        lanes_f[lam - t0] = &fe[row];
                        lanes_b[lam - t0] = &be[row];
                    }
                    budget_f -= f->fext.add_group(lanes_f, n, budget_f);
                    budget_b -= f->bext.add_group(lanes_b, n, budget_b);
                }
            }
        }
        f->fext.finish();
        f->bext.finish();
        // couplings inside the level-1 blocks: per (tile, step) a list of
        // slots, one entry per lane (column = source step, -1 = none)
        auto pack_lanes = [&](const std::vector<Couplings> &rows, Sell &s, int32_t &max_slots,
                              int32_t &max_step) {
            s.off.assign(1, 0);
            max_slots = 0;
            max_step = 0;
            for (int c = 0; c < f->nc; ++c) {
                const int64_t r0 = f->color_start[c];
                const int64_t lanes = (f->color_start[c + 1] - r0) / bs;
                for (int64_t t0 = 0; t0 < lanes; t0 += kTileLanes) {
                    const int64_t t1 = std::min(lanes, t0 + kTileLanes);
                    int32_t tile_slots = 0;
                    for (int l = 0; l < bs; ++l) {
                        auto row_of = [&](int64_t lam) {
                            return r0 + (lam / w) * l1 + int64_t(l) * w + lam % w;
                        };
                        size_t len = 0;
                        for (int64_t lam = t0; lam < t1; ++lam) len = std::max(len, rows[row_of(lam)].size());
                        const int64_t base = s.off.back();
                        s.off.push_back(int32_t(base + len));
                        s.val.resize((base + len) * kTileLanes, 0.0);
                        s.col.resize((base + len) * kTileLanes, -1);
                        for (int64_t lam = t0; lam < t1; ++lam) {
                            const auto &e = rows[row_of(lam)];
                            for (size_t t = 0; t < e.size(); ++t) {
                                s.col[(base + t) * kTileLanes + (lam - t0)] = e[t].first;
                                s.val[(base + t) * kTileLanes + (lam - t0)] = e[t].second;
                            }
                        }
                        tile_slots += int32_t(len);
                        max_step = std::max(max_step, int32_t(len));
                    }
                    max_slots = std::max(max_slots, tile_slots);
                }
            }
            s.val.resize(s.val.size() + kTileLanes, 0.0);   // the padding slot
            s.col.resize(s.col.size() + kTileLanes, -1);
        };
        pack_lanes(fi, f->fint, f->max_int_slots_f, f->max_int_step_f);
        pack_lanes(bi, f->bint, f->max_int_slots_b, f->max_int_step_b);

        // systems: each tile and each kPartRows-row part lies in one system
        // (a single system trivially; batches pad every system's share of a
        // color to whole tiles of kTileLanes lanes and whole parts)
        {
            const int nsys = f->nsys, nc = f->nc;
            const int64_t ntiles = f->tile_base[nc];
            const int64_t nparts = (n + kPartRows - 1) / kPartRows;
            const int64_t trows = int64_t(kTileLanes) * bs;
            auto sys_of_row = [&](int64_t row) -> int32_t {
                if (nsys == 1) return 0;
                int c = int(std::upper_bound(f->color_start.begin(), f->color_start.end(), row) -
                            f->color_start.begin()) - 1;
                const int64_t *sg = &o->seg[int64_t(c) * (nsys + 1)];
                return int32_t(std::upper_bound(sg, sg + nsys + 1, row) - sg) - 1;
            };
            f->tile_sys.assign(ntiles, 0);
            for (int c = 0; c < nc; ++c)
                for (int64_t t = f->tile_base[c]; t < f->tile_base[c + 1]; ++t)
                    f->tile_sys[t] = sys_of_row(f->color_start[c] + (t - f->tile_base[c]) * trows);
            f->part_sys.assign(nparts, 0);
            for (int64_t g = 0; g < nparts; ++g) f->part_sys[g] = sys_of_row(g * kPartRows);
            // tile and part ranges of each (system, color); a tile or part
            // that a color ends inside (one system) is counted with the color
            // it starts in
            f->sys_tiles.assign(int64_t(nsys) * nc * 2, 0);
            f->sys_parts.assign(int64_t(nsys) * nc * 2, 0);
            auto ceil_div = [](int64_t a, int64_t b) { return (a + b - 1) / b; };
            for (int sy = 0; sy < nsys; ++sy)
                for (int c = 0; c < nc; ++c) {
                    const int64_t a = o->seg[int64_t(c) * (nsys + 1) + sy];
                    const int64_t b = o->seg[int64_t(c) * (nsys + 1) + sy + 1];
                    const int64_t k = (int64_t(sy) * nc + c) * 2;
                    f->sys_tiles[k] = int32_t(f->tile_base[c] + ceil_div(a - f->color_start[c], trows));
                    f->sys_tiles[k + 1] = int32_t(f->tile_base[c] + ceil_div(b - f->color_start[c], trows));
                    f->sys_parts[k] = int32_t(ceil_div(a, kPartRows));
                    f->sys_parts[k + 1] = int32_t(ceil_div(b, kPartRows));
                }
        }

        // device image
        auto &im = f->image;
        auto add_tri = [&](const Packed &e, const Sell &i, TriOffsets &t) {
            add_packed<double>(im, e, precision == HBMC_F32, t.ext);
            t.int_off = im.add(i.off);
            t.int_lp = im.add(i.col);
            t.int_val = precision == HBMC_F64 ? im.add(i.val) : im.add(cast<float>(i.val));
        };
        f->off_dinv = precision == HBMC_F64 ? im.add(dinv) : im.add(cast<float>(dinv));
        f->off_perm = im.add(f->perm);
        f->off_iperm = im.add(f->iperm);
        f->off_tile_sys = im.add(f->tile_sys);
        f->off_part_sys = im.add(f->part_sys);
        f->off_sys_tiles = im.add(f->sys_tiles);
        f->off_sys_parts = im.add(f->sys_parts);
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

extern "C" void hbmc_factor_destroy(hbmc_factor_t *f) {
    if (!f) return;
    release_graphs(f);
    delete f;
}

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
        std::vector<Couplings> rows(m->n_pad);
        for (int64_t r = 0; r < m->n_pad; ++r)
            for (int64_t p = a.rp[r]; p < a.rp[r + 1]; ++p) {
                if (a.ci[p] == r) m->diag[r] = a.v[p];
                else rows[r].emplace_back(a.ci[p], a.v[p]);
            }
        // one Packed group per 64-row slice
        std::vector<const Couplings *> lanes;
        for (int64_t r0 = 0; r0 < m->n_pad; r0 += kTileLanes) {
            lanes.assign(kTileLanes, nullptr);
            for (int64_t r = r0; r < std::min(m->n_pad, r0 + kTileLanes); ++r) lanes[r - r0] = &rows[r];
            m->off.add_group(lanes, m->n_pad, kTileLanes);
        }
        m->off.finish();
        m->off_diag = m->image.add(m->diag);
        add_packed<double>(m->image, m->off, false, m->offs);
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
