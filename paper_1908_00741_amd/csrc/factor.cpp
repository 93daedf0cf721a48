// Host side of the factorization and of the device layouts:
//  - Abar = P A P^T with identity rows for dummy unknowns (Section 3, eq. "AB");
//  - IC(0) with zero fill (Section 2, eq. "ILU"), computed row by row;
//  - the sliced-ELL layouts used by the substitutions (Section 4.4.2) and by
//    the SpMV.
// Compiled without floating-point contraction (-ffp-contract=off).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "hbmc_internal.h"
#include "parallel.h"

using namespace hbmc;

namespace {

constexpr int64_t kGrain = 16384;   // rows per chunk of the parallel setup, at least

struct Csr {
    RawVec<int64_t> rp;
    RawVec<int32_t> ci;
    RawVec<double> v;
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
    parallel_chunks(o.n_pad, chunks_for(o.n_pad, kGrain), [&](int64_t lo, int64_t hi, int) {
        std::vector<std::pair<int32_t, double>> row;
        for (int64_t r = lo; r < hi; ++r) {
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
    });
    return a;
}

// Where the rows of Abar sit in the HBMC layout: color starts and the
// level-1 block size bs * w (a color's rows are whole level-1 blocks).
struct Levels {
    const std::vector<int64_t> &color_start;
    int64_t l1;
    int w;
};

// The strictly lower pattern of Abar (row pointers); checks that no
// coupling joins two level-1 blocks of one color or two lanes of one
// level-1 block (Section 4.3, eq. "BAMC1": the level-1 blocks of a color are
// independent), which the parallel factorization relies on.
int lower_pattern(const Csr &a, int64_t n, const Levels &lv, std::vector<int64_t> &lrp) {
    lrp.assign(n + 1, 0);
    for (size_t c = 0; c + 1 < lv.color_start.size(); ++c) {
        const int64_t r0 = lv.color_start[c], r1 = lv.color_start[c + 1];
        const int chunks = chunks_for(r1 - r0, kGrain);
        std::vector<int64_t> bad(chunks, -1);
        parallel_chunks(r1 - r0, chunks, [&](int64_t lo, int64_t hi, int ch) {
            for (int64_t t = lo; t < hi; ++t) {
                const int64_t i = r0 + t;
                int64_t cnt = 0;
                for (int64_t p = a.rp[i]; p < a.rp[i + 1] && a.ci[p] < i; ++p) {
                    const int64_t k = a.ci[p];
                    if (k >= r0 && ((k - r0) / lv.l1 != t / lv.l1 || (i - k) % lv.w != 0) && bad[ch] < 0)
                        bad[ch] = i;
                    ++cnt;
                }
                lrp[i + 1] = cnt;
            }
        });
        for (int64_t x : bad)
            if (x >= 0)
                return fail(HBMC_EINVAL, "internal: a coupling of row %lld crosses level-1 blocks", (long long)x);
    }
    for (int64_t i = 0; i < n; ++i) lrp[i + 1] += lrp[i];
    return HBMC_OK;
}

// IC(0), row by row: for each row i and each lower entry (i, k) in
// ascending k,  L_ik = a_ik - sum_{m<k} L_im L_km / d_m  over the common
// lower pattern of rows i and k; then d_i = a_ii - sum_{m<i} L_im^2 / d_m.
// This is the same arithmetic, term for term and in the same order, as the
// right-looking elimination with overwriting, organised by rows so that
// each row is finished before the next starts.  A row needs only rows of
// earlier colors and earlier rows of its own level-1 block, so the colors
// run in turn and the level-1 blocks of a color in parallel (each block's
// rows in order): the same arithmetic as one row after another.
int ic0_rows(const Csr &a, int64_t n, double shift, const Levels &lv, std::vector<int64_t> &lrp,
             std::vector<int32_t> &lcol, std::vector<double> &lval, std::vector<double> &d) {
    int st = lower_pattern(a, n, lv, lrp);
    if (st) return st;
    lcol.resize(lrp[n]);
    lval.resize(lrp[n]);
    d.assign(n, 0.0);
    auto row = [&](int64_t i) -> bool {
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
        d[i] = s;
        return s > 0.0 && std::isfinite(s);
    };
    for (size_t c = 0; c + 1 < lv.color_start.size(); ++c) {
        const int64_t r0 = lv.color_start[c], r1 = lv.color_start[c + 1];
        const int64_t blocks = (r1 - r0) / lv.l1;
        const int chunks = chunks_for(blocks, std::max<int64_t>(1, kGrain / lv.l1));
        std::vector<int64_t> first_bad(chunks, -1);
        parallel_chunks(blocks, chunks, [&](int64_t lo, int64_t hi, int ch) {
            for (int64_t b = lo; b < hi; ++b)
                for (int64_t i = r0 + b * lv.l1; i < r0 + (b + 1) * lv.l1; ++i)
                    if (!row(i) && (first_bad[ch] < 0 || i < first_bad[ch])) first_bad[ch] = i;
        });
        int64_t bad = -1;
        for (int64_t x : first_bad)
            if (x >= 0 && (bad < 0 || x < bad)) bad = x;
        if (bad >= 0)
            return fail(HBMC_EBREAKDOWN, "IC(0) pivot %lld is not > 0 (%g)", (long long)bad, d[bad]);
    }
    return HBMC_OK;
}

// The SSOR splitting (Section 2: the GS and SOR steps are substitutions
// with the triangles of A itself): L = strict lower triangle of Abar, copied
// without any update, and d_i = a_ii / omega.  With these, the
// preconditioner (D + L) D^-1 (D + L^T) is (2 - omega) times the inverse of
// the SSOR matrix, and omega = 1 gives symmetric Gauss-Seidel.
int ssor_rows(const Csr &a, int64_t n, double omega, const Levels &lv, std::vector<int64_t> &lrp,
              std::vector<int32_t> &lcol, std::vector<double> &lval, std::vector<double> &d) {
    int st = lower_pattern(a, n, lv, lrp);
    if (st) return st;
    lcol.resize(lrp[n]);
    lval.resize(lrp[n]);
    d.assign(n, 0.0);
    parallel_for(n, kGrain, [&](int64_t i) {
        int64_t q = lrp[i];
        for (int64_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
            if (a.ci[p] < i) { lcol[q] = a.ci[p]; lval[q] = a.v[p]; ++q; }
            else if (a.ci[p] == i) d[i] = a.v[p] / omega;
        }
    });
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
    // the left-over couplings: indexed slots, or their flat form
    o = PackedOffsets{o.soff, o.sbase, o.smask, o.sval, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (p.flat) {
        o.goff = im.add(p.goff);
        o.lstart = im.add(p.lstart);
        o.fcol = im.add(p.fcol);
        o.fval = f32 ? im.add(cast<float>(p.fval)) : im.add(p.fval);
    } else {
        o.ioff = im.add(p.ioff);
        o.imask = im.add(p.imask);
        o.ivoff = im.add(p.ivoff);
        o.icol = im.add(p.icol);
        o.ival = f32 ? im.add(cast<float>(p.ival)) : im.add(p.ival);
    }
    return o.soff;
}

}  // namespace

int Packed::add_group(const std::vector<CouplingSpan> &lanes, int64_t limit, int budget) {
    const int nl = int(lanes.size());
    // every coupling (lane j, column c) proposes the strided base c - j
    struct Entry { int64_t key; int lane; int idx; };
    thread_local std::vector<Entry> all;
    thread_local std::vector<int32_t> first;   // first entry of each lane in `used`
    thread_local std::vector<uint8_t> used;
    all.clear();
    first.assign(nl + 1, 0);
    for (int j = 0; j < nl; ++j) {
        for (int t = 0; t < int(lanes[j].size()); ++t) all.push_back({int64_t(lanes[j][t].first) - j, j, t});
        first[j + 1] = first[j] + int32_t(lanes[j].size());
    }
    entries += int64_t(all.size());
    std::sort(all.begin(), all.end(), [](const Entry &a, const Entry &b) {
        return a.key != b.key ? a.key < b.key : a.lane < b.lane;
    });
    // bases shared by enough lanes become strided slots, most shared first
    struct Cand { int64_t key; size_t first, count; };
    thread_local std::vector<Cand> cands;
    cands.clear();
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
    used.assign(first[nl], 0);
    for (const Cand &c : cands) {
        const int64_t slot = int64_t(sbase.size());
        sbase.push_back(int32_t(c.key));
        uint64_t mask = 0;
        sval.resize((slot + 1) * kTileLanes, 0.0);
        for (size_t i = c.first; i < c.first + c.count; ++i) {
            const Entry &e = all[i];
            mask |= uint64_t(1) << e.lane;
            sval[slot * kTileLanes + e.lane] = lanes[e.lane][e.idx].second;
            used[first[e.lane] + e.idx] = 1;
        }
        smask.push_back(mask);
    }
    soff.push_back(int32_t(sbase.size()));
    max_strided = std::max(max_strided, int32_t(cands.size()));
    // the rest, per lane in column order, as indexed slots: slot t holds the
    // t-th left-over coupling of each lane that has one, in lane order
    thread_local std::vector<int32_t> left_of;   // left-over entries of each lane, lane by lane
    thread_local std::vector<int32_t> lfirst;
    left_of.clear();
    lfirst.assign(nl + 1, 0);
    int32_t len = 0;
    for (int j = 0; j < nl; ++j) {
        for (int32_t i = first[j]; i < first[j + 1]; ++i)
            if (!used[i]) left_of.push_back(i - first[j]);
        lfirst[j + 1] = int32_t(left_of.size());
        len = std::max(len, lfirst[j + 1] - lfirst[j]);
    }
    left += int64_t(left_of.size());
    if (both) {
        // the flat form: lane by lane, each lane's in column order
        const int64_t g0 = int64_t(fcol.size());
        for (int j = 0; j < kTileLanes; ++j) {
            const int64_t rel = int64_t(fcol.size()) - g0;
            if (rel > 0xFFFF) overflow = true;
            lstart.push_back(uint16_t(rel));
            if (j >= nl) continue;
            for (int32_t k = lfirst[j]; k < lfirst[j + 1]; ++k) {
                const Coupling &c = lanes[j][left_of[k]];
                fcol.push_back(c.first);
                fval.push_back(c.second);
            }
        }
        goff.push_back(int64_t(fcol.size()));
        max_group = std::max(max_group, int32_t(int64_t(fcol.size()) - g0));
    }
    const int64_t base = ioff.back();
    ioff.push_back(int32_t(base + len));
    for (int32_t t = 0; t < len; ++t) {
        uint64_t mask = 0;
        ivoff.push_back(int64_t(icol.size()));
        for (int j = 0; j < nl; ++j) {
            if (lfirst[j] + t >= lfirst[j + 1]) continue;
            const Coupling &c = lanes[j][left_of[lfirst[j] + t]];
            mask |= uint64_t(1) << j;
            icol.push_back(c.first);
            ival.push_back(c.second);
        }
        imask.push_back(mask);
    }
    max_indexed = std::max(max_indexed, len);
    return int(cands.size());
}

void Packed::reserve_for(const std::vector<const Packed *> &parts) {
    size_t so = soff.size(), sb = sbase.size(), sv = sval.size(), io = ioff.size(), is = imask.size(),
           iv = icol.size();
    for (const Packed *p : parts) {
        so += p->soff.size(); sb += p->sbase.size(); sv += p->sval.size();
        io += p->ioff.size(); is += p->imask.size(); iv += p->icol.size();
    }
    soff.reserve(so); sbase.reserve(sb + 1); smask.reserve(sb + 1); sval.reserve(sv + kTileLanes);
    ioff.reserve(io); imask.reserve(is + 1); ivoff.reserve(is + 1); icol.reserve(iv + 1); ival.reserve(iv + 1);
    if (both) {
        size_t go = goff.size(), ls = lstart.size(), fc = fcol.size();
        for (const Packed *p : parts) { go += p->goff.size(); ls += p->lstart.size(); fc += p->fcol.size(); }
        goff.reserve(go);
        lstart.reserve(ls);
        fcol.reserve(fc + 1);
        fval.reserve(fc + 1);
    }
}

void Packed::append(const Packed &o) {
    const int32_t sb = soff.back(), ib = ioff.back();
    const int64_t eb = int64_t(icol.size());
    for (size_t i = 1; i < o.soff.size(); ++i) soff.push_back(sb + o.soff[i]);
    for (size_t i = 1; i < o.ioff.size(); ++i) ioff.push_back(ib + o.ioff[i]);
    for (int64_t v : o.ivoff) ivoff.push_back(eb + v);
    imask.insert(imask.end(), o.imask.begin(), o.imask.end());
    sbase.insert(sbase.end(), o.sbase.begin(), o.sbase.end());
    smask.insert(smask.end(), o.smask.begin(), o.smask.end());
    sval.insert(sval.end(), o.sval.begin(), o.sval.end());
    icol.insert(icol.end(), o.icol.begin(), o.icol.end());
    ival.insert(ival.end(), o.ival.begin(), o.ival.end());
    max_strided = std::max(max_strided, o.max_strided);
    max_indexed = std::max(max_indexed, o.max_indexed);
    entries += o.entries;
    left += o.left;
    if (both) {
        const int64_t fb = int64_t(fcol.size());
        for (size_t i = 1; i < o.goff.size(); ++i) goff.push_back(fb + o.goff[i]);
        lstart.insert(lstart.end(), o.lstart.begin(), o.lstart.end());
        fcol.insert(fcol.end(), o.fcol.begin(), o.fcol.end());
        fval.insert(fval.end(), o.fval.begin(), o.fval.end());
        max_group = std::max(max_group, o.max_group);
        overflow = overflow || o.overflow;
    }
}

void Packed::finish() {
    sbase.push_back(0);
    smask.push_back(0);
    sval.resize(sval.size() + kTileLanes, 0.0);
    imask.push_back(0);                       // the padding slot: no lanes, one dummy entry
    ivoff.push_back(int64_t(icol.size()));
    icol.push_back(-1);
    ival.push_back(0.0);
    if (both) {                               // the padding entry of the flat form
        fcol.push_back(-1);
        fval.push_back(0.0);
    }
}

namespace {

enum class Split { kIc0, kSsor };

// Factor of either splitting, its substitution layout and its device image.
int make_factor(const hbmc_order_t *o, const int64_t *rowptr, const int32_t *col, const double *val,
                int32_t precision, Split kind, double param, hbmc_factor_t **out) {
    clear_error();
    if (!out) return fail(HBMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!o || !val) return fail(HBMC_EINVAL, "null argument");
    if (precision != HBMC_F64 && precision != HBMC_F32)
        return fail(HBMC_EINVAL, "precision must be HBMC_F64 or HBMC_F32");
    if (kind == Split::kIc0 && !(param >= 0.0)) return fail(HBMC_EINVAL, "shift must be >= 0");
    if (kind == Split::kSsor && !(param > 0.0 && param < 2.0))
        return fail(HBMC_EINVAL, "omega must lie in (0, 2) (got %g)", param);
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
        f->local = o->local;
        const Csr a = permute(*o, rowptr, col, val);
        const int64_t n = f->n_pad;
        const int bs = f->bs, w = f->w;
        const int64_t l1 = int64_t(bs) * w;
        const Levels lv{f->color_start, l1, w};
        st = kind == Split::kIc0 ? ic0_rows(a, n, param, lv, f->lrp, f->lcol, f->lval, f->d)
                                 : ssor_rows(a, n, param, lv, f->lrp, f->lcol, f->lval, f->d);
        if (st) { delete f; return st; }
        f->smooth_scale = kind == Split::kSsor ? 2.0 - param : 1.0;
        f->ssor = kind == Split::kSsor;

        std::vector<double> dinv(n);
        // color of each HBMC row
        std::vector<int32_t> color(n);
        for (int c = 0; c < f->nc; ++c)
            std::fill(color.begin() + f->color_start[c], color.begin() + f->color_start[c + 1], c);
        parallel_for(n, kGrain, [&](int64_t i) { dinv[i] = 1.0 / f->d[i]; });
        // the step of row r inside its level-1 block
        auto step_of = [&](int64_t r) { return int(((r - f->color_start[color[r]]) % l1) / w); };

        // couplings of each row: forward (lower) and backward (upper, scaled
        // by diaginv of the row: U = I + D^-1 L^T), split into couplings to
        // other colors (ext) and inside the level-1 block (int, column = the
        // source step).  The upper couplings of row k are the columns r > k
        // of Abar's row k (the pattern is symmetric), each with L_rk found in
        // row r; they come out in ascending r.
        CouplingRows fe, fi, be, bi;
        for (CouplingRows *cr : {&fe, &fi, &be, &bi}) cr->ptr.assign(n + 1, 0);
        auto lower_at = [&](int64_t r, int32_t k) {
            const int32_t *b = f->lcol.data() + f->lrp[r], *e = f->lcol.data() + f->lrp[r + 1];
            return f->lval[f->lrp[r] + (std::lower_bound(b, e, k) - b)];
        };
        parallel_for(n, kGrain, [&](int64_t r) {
            int64_t ne = 0, ni = 0;
            for (int64_t p = f->lrp[r]; p < f->lrp[r + 1]; ++p) (color[f->lcol[p]] != color[r] ? ne : ni) += 1;
            fe.ptr[r + 1] = ne;
            fi.ptr[r + 1] = ni;
            ne = ni = 0;
            for (int64_t p = a.rp[r]; p < a.rp[r + 1]; ++p)
                if (a.ci[p] > r) (color[a.ci[p]] != color[r] ? ne : ni) += 1;
            be.ptr[r + 1] = ne;
            bi.ptr[r + 1] = ni;
        });
        for (CouplingRows *cr : {&fe, &fi, &be, &bi}) {
            for (int64_t r = 0; r < n; ++r) cr->ptr[r + 1] += cr->ptr[r];
            cr->data.resize(cr->ptr[n]);
        }
        parallel_for(n, kGrain, [&](int64_t r) {
            int64_t xe = fe.ptr[r], xi = fi.ptr[r];
            for (int64_t p = f->lrp[r]; p < f->lrp[r + 1]; ++p) {
                const int32_t k = f->lcol[p];
                if (color[k] != color[r]) fe.data[xe++] = {k, f->lval[p]};
                else fi.data[xi++] = {step_of(k), f->lval[p]};
            }
            xe = be.ptr[r];
            xi = bi.ptr[r];
            for (int64_t p = a.rp[r]; p < a.rp[r + 1]; ++p) {
                const int32_t q = a.ci[p];
                if (q <= r) continue;
                const double u = dinv[r] * lower_at(q, int32_t(r));
                if (color[q] != color[r]) be.data[xe++] = {q, u};
                else bi.data[xi++] = {step_of(q), u};
            }
        });

        // Layout of the substitutions: per color, the chain lanes (one per BMC
        // block, lam = level-1 block * w + m) are cut into tiles of 64 lanes;
        // for each (tile, step l) a sliced-ELL slot list holds, slot-major,
        // one entry per lane: the couplings of row  S_c + (lam / w) bs w +
        // l w + lam % w.  Missing entries have column -1 and value 0.  Each
        // array ends with one extra all-padding slot that loads may target
        // instead of branching.  Tiles are packed in parallel chunks, which
        // are then joined in tile order.
        f->tile_base.assign(f->nc + 1, 0);
        for (int c = 0; c < f->nc; ++c) {
            const int64_t lanes = (f->color_start[c + 1] - f->color_start[c]) / bs;
            f->tile_base[c + 1] = f->tile_base[c] + (lanes + kTileLanes - 1) / kTileLanes;
        }
        const int64_t ntiles = f->tile_base[f->nc];
        struct Chunk {
            Packed fext, bext;                 // couplings to other colors, one group per (tile, step)
            Sell fint, bint;                   // couplings inside level-1 blocks, one slice per (tile, step)
            int32_t slots_f = 0, slots_b = 0;  // most in-block slots of a tile
            int32_t step_f = 0, step_b = 0;    // most in-block slots of a (tile, step)
        };
        const int nchunks = chunks_for(ntiles, std::max<int64_t>(1, kGrain / (int64_t(kTileLanes) * bs)));
        std::vector<Chunk> chunks(nchunks);
        parallel_chunks(ntiles, nchunks, [&](int64_t t_lo, int64_t t_hi, int ch) {
            Chunk &k = chunks[ch];
            k.fext.both = k.bext.both = true;
            k.fint.off.assign(1, 0);
            k.bint.off.assign(1, 0);
            std::vector<CouplingSpan> lanes_f(kTileLanes), lanes_b(kTileLanes), lanes_fi(kTileLanes),
                lanes_bi(kTileLanes);
            // in-block couplings of one (tile, step): slots of (source step, value)
            auto pack_int = [](const std::vector<CouplingSpan> &ls, Sell &s, int32_t &tile_slots,
                               int32_t &max_step) {
                size_t len = 0;
                for (const auto &e : ls) len = std::max(len, e.size());
                const int64_t base = s.off.back();
                s.off.push_back(int32_t(base + len));
                s.val.resize((base + len) * kTileLanes, 0.0);
                s.col.resize((base + len) * kTileLanes, -1);
                for (int j = 0; j < kTileLanes; ++j)
                    for (size_t t = 0; t < ls[j].size(); ++t) {
                        s.col[(base + t) * kTileLanes + j] = int8_t(ls[j][t].first);
                        s.val[(base + t) * kTileLanes + j] = ls[j][t].second;
                    }
                tile_slots += int32_t(len);
                max_step = std::max(max_step, int32_t(len));
            };
            for (int64_t t = t_lo; t < t_hi; ++t) {
                const int c = int(std::upper_bound(f->tile_base.begin(), f->tile_base.end(), t) -
                                  f->tile_base.begin()) - 1;
                const int64_t r0 = f->color_start[c];
                const int64_t lanes = (f->color_start[c + 1] - r0) / bs;
                const int64_t t0 = (t - f->tile_base[c]) * kTileLanes;
                // the kernel fetches a tile's strided-slot metadata one slot per lane
                int budget_f = kTileLanes, budget_b = kTileLanes;
                int32_t tile_f = 0, tile_b = 0;
                for (int l = 0; l < bs; ++l) {
                    for (int j = 0; j < kTileLanes; ++j) {
                        const int64_t lam = t0 + j;
                        if (lam < lanes) {
                            const int64_t row = r0 + (lam / w) * l1 + int64_t(l) * w + lam % w;
                            lanes_f[j] = fe.row(row);
                            lanes_b[j] = be.row(row);
                            lanes_fi[j] = fi.row(row);
                            lanes_bi[j] = bi.row(row);
                        } else {
                            lanes_f[j] = lanes_b[j] = lanes_fi[j] = lanes_bi[j] = CouplingSpan{};
                        }
                    }
                    budget_f -= k.fext.add_group(lanes_f, n, budget_f);
                    budget_b -= k.bext.add_group(lanes_b, n, budget_b);
                    pack_int(lanes_fi, k.fint, tile_f, k.step_f);
                    pack_int(lanes_bi, k.bint, tile_b, k.step_b);
                }
                k.slots_f = std::max(k.slots_f, tile_f);
                k.slots_b = std::max(k.slots_b, tile_b);
            }
        });
        f->fint.off.assign(1, 0);
        f->bint.off.assign(1, 0);
        f->fext.both = f->bext.both = true;
        f->max_int_slots_f = f->max_int_slots_b = f->max_int_step_f = f->max_int_step_b = 0;
        {
            std::vector<const Packed *> pf, pb;
            std::vector<const Sell *> sf, sb;
            for (const Chunk &k : chunks) {
                pf.push_back(&k.fext); pb.push_back(&k.bext);
                sf.push_back(&k.fint); sb.push_back(&k.bint);
            }
            f->fext.reserve_for(pf);
            f->bext.reserve_for(pb);
            f->fint.reserve_for(sf);
            f->bint.reserve_for(sb);
        }
        for (const Chunk &k : chunks) {
            f->fext.append(k.fext);
            f->bext.append(k.bext);
            f->fint.append(k.fint);
            f->bint.append(k.bint);
            f->max_int_slots_f = std::max(f->max_int_slots_f, k.slots_f);
            f->max_int_slots_b = std::max(f->max_int_slots_b, k.slots_b);
            f->max_int_step_f = std::max(f->max_int_step_f, k.step_f);
            f->max_int_step_b = std::max(f->max_int_step_b, k.step_b);
        }
        chunks.clear();
        f->fext.finish();
        f->bext.finish();
        // the device gets the flat form where the left-over couplings
        // outweigh the strided slots (unstructured graphs), else the slots
        {
            const bool flat = (f->fext.left + f->bext.left) / kTileLanes > f->fext.strided() + f->bext.strided();
            if (flat && (f->fext.overflow || f->bext.overflow)) {
                delete f;
                return fail(HBMC_EINVAL, "a (tile, step) group has more than 65535 couplings to other colors");
            }
            f->fext.flat = f->bext.flat = flat;
            for (auto [e, c] : {std::pair{&f->fext, &f->fcnt}, std::pair{&f->bext, &f->bcnt}})
                *c = LayoutCounts{e->strided(), e->indexed(), int64_t(e->fcol.size()) - 1, e->left, flat};
        }
        f->nnz_lower = int64_t(f->lcol.size());
        for (Sell *sl : {&f->fint, &f->bint}) {   // the padding slot
            sl->val.resize(sl->val.size() + kTileLanes, 0.0);
            sl->col.resize(sl->col.size() + kTileLanes, -1);
        }

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
        {
            auto vb = [](const auto &v) { return v.size() * sizeof(v[0]) + 256; };
            size_t est = 256 + vb(dinv) + vb(f->perm) + vb(f->iperm) + vb(f->tile_sys) + vb(f->part_sys) +
                         vb(f->sys_tiles) + vb(f->sys_parts);
            for (const Packed *e : {&f->fext, &f->bext})
                est += vb(e->soff) + vb(e->sbase) + vb(e->smask) + vb(e->sval) + vb(e->ioff) + vb(e->imask) +
                       vb(e->ivoff) + vb(e->icol) + vb(e->ival);
            for (const Sell *i : {&f->fint, &f->bint}) est += vb(i->off) + vb(i->col) + vb(i->val);
            im.bytes.reserve(est);
        }
        auto add_tri = [&](const Packed &e, const Sell &i, TriOffsets &t) {
            add_packed<double>(im, e, precision == HBMC_F32, t.ext);
            t.int_off = im.add(i.off);
            t.int_lp = im.add(i.col);
            t.int_val = precision == HBMC_F64 ? im.add(i.val) : im.add(cast<float>(i.val));
            t.int_slots = i.slots();
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
        return fail(HBMC_ENOMEM, "out of host memory in %s", kind == Split::kIc0 ? "ic0_factor" : "ssor_factor");
    }
}

}  // namespace

extern "C" int ic0_factor(const hbmc_order_t *o, const int64_t *rowptr, const int32_t *col,
                          const double *val, int32_t precision, double shift, hbmc_factor_t **out) {
    return make_factor(o, rowptr, col, val, precision, Split::kIc0, shift, out);
}

extern "C" int ssor_factor(const hbmc_order_t *o, const int64_t *rowptr, const int32_t *col,
                           const double *val, int32_t precision, double omega, hbmc_factor_t **out) {
    return make_factor(o, rowptr, col, val, precision, Split::kSsor, omega, out);
}

extern "C" int hbmc_factor_export(const hbmc_factor_t *f, double *d, int64_t *lower_rowptr,
                                  int32_t *lower_col, double *lower_val, int64_t *lower_nnz) {
    if (!f) return fail(HBMC_EINVAL, "null handle");
    if (lower_nnz) *lower_nnz = f->nnz_lower;
    if (f->device_built) return device_export(f, d, lower_rowptr, lower_col, lower_val);
    if (d) std::copy(f->d.begin(), f->d.end(), d);
    if (lower_rowptr) std::copy(f->lrp.begin(), f->lrp.end(), lower_rowptr);
    if (lower_col) std::copy(f->lcol.begin(), f->lcol.end(), lower_col);
    if (lower_val) std::copy(f->lval.begin(), f->lval.end(), lower_val);
    return HBMC_OK;
}

extern "C" int hbmc_factor_image(const hbmc_factor_t *f, void *host, size_t bytes) {
    if (!f || !host) return fail(HBMC_EINVAL, "null argument");
    if (f->device_built) return fail(HBMC_EINVAL, "a factor built on the device has no host image");
    if (bytes < f->image.bytes.size())
        return fail(HBMC_EINVAL, "buffer too small (%zu < %zu)", bytes, f->image.bytes.size());
    std::memcpy(host, f->image.bytes.data(), f->image.bytes.size());
    return HBMC_OK;
}

extern "C" int hbmc_matrix_image(const hbmc_matrix_t *m, void *host, size_t bytes) {
    if (!m || !host) return fail(HBMC_EINVAL, "null argument");
    if (m->device_built) return fail(HBMC_EINVAL, "a matrix built on the device has no host image");
    if (bytes < m->image.bytes.size())
        return fail(HBMC_EINVAL, "buffer too small (%zu < %zu)", bytes, m->image.bytes.size());
    std::memcpy(host, m->image.bytes.data(), m->image.bytes.size());
    return HBMC_OK;
}

extern "C" int hbmc_factor_device_bytes(const hbmc_factor_t *f, size_t *bytes) {
    if (!f || !bytes) return fail(HBMC_EINVAL, "null argument");
    *bytes = f->device_built ? f->dev_image_bytes : f->image.bytes.size();
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
        const int64_t n = m->n_pad;
        m->diag.assign(n, 0.0);
        CouplingRows rows;
        rows.ptr.assign(n + 1, 0);
        parallel_for(n, kGrain, [&](int64_t r) { rows.ptr[r + 1] = a.rp[r + 1] - a.rp[r] - 1; });
        for (int64_t r = 0; r < n; ++r) rows.ptr[r + 1] += rows.ptr[r];
        rows.data.resize(rows.ptr[n]);
        parallel_for(n, kGrain, [&](int64_t r) {
            int64_t x = rows.ptr[r];
            for (int64_t p = a.rp[r]; p < a.rp[r + 1]; ++p) {
                if (a.ci[p] == r) m->diag[r] = a.v[p];
                else rows.data[x++] = {a.ci[p], a.v[p]};
            }
        });
        // one Packed group per 64-row slice, slices packed in parallel chunks
        // and joined in slice order
        const int64_t slices = (n + kTileLanes - 1) / kTileLanes;
        const int nchunks = chunks_for(slices, kGrain / kTileLanes);
        std::vector<Packed> part(nchunks);
        parallel_chunks(slices, nchunks, [&](int64_t lo, int64_t hi, int ch) {
            std::vector<CouplingSpan> lanes(kTileLanes);
            for (int64_t sl = lo; sl < hi; ++sl) {
                for (int j = 0; j < kTileLanes; ++j) {
                    const int64_t r = sl * kTileLanes + j;
                    lanes[j] = r < n ? rows.row(r) : CouplingSpan{};
                }
                part[ch].add_group(lanes, n, kTileLanes);
            }
        });
        {
            std::vector<const Packed *> pp;
            for (const Packed &pk : part) pp.push_back(&pk);
            m->off.reserve_for(pp);
        }
        for (const Packed &pk : part) m->off.append(pk);
        part.clear();
        {
            int64_t strided = 0;
            for (uint64_t mask : m->off.smask) strided += __builtin_popcountll(mask);
            m->fuse_p = 2 * strided >= m->off.entries;
        }
        m->off.finish();
        {
            const Packed &e = m->off;
            auto vb = [](const auto &v) { return v.size() * sizeof(v[0]) + 256; };
            m->image.bytes.reserve(256 + vb(m->diag) + vb(e.soff) + vb(e.sbase) + vb(e.smask) + vb(e.sval) +
                                   vb(e.ioff) + vb(e.imask) + vb(e.ivoff) + vb(e.icol) + vb(e.ival));
        }
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
    *bytes = m->image_bytes();
    return HBMC_OK;
}

extern "C" void hbmc_matrix_destroy(hbmc_matrix_t *m) { delete m; }

// ---------------------------------------------------------------------------
// Pattern data for device refactorization
// ---------------------------------------------------------------------------
extern "C" int hbmc_revalue_create(const hbmc_order_t *o, const int64_t *rowptr, const int32_t *col,
                                   hbmc_revalue_t **out) {
    clear_error();
    if (!out) return fail(HBMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!o) return fail(HBMC_EINVAL, "null argument");
    int st = check_csr(o->n, rowptr, col, nullptr);
    if (st) return st;
    try {
        auto *rv = new hbmc_revalue_s;
        rv->n = o->n; rv->bs = o->bs; rv->w = o->w; rv->nc = o->nc;
        rv->n_pad = o->n_pad;
        rv->nnz = rowptr[o->n];
        rv->color_start = o->color_start;
        rv->tile_base.assign(o->nc + 1, 0);
        for (int c = 0; c < o->nc; ++c) {
            const int64_t lanes = (o->color_start[c + 1] - o->color_start[c]) / o->bs;
            rv->tile_base[c + 1] = rv->tile_base[c] + (lanes + kTileLanes - 1) / kTileLanes;
        }
        // Abar's pattern with the source entry of every value: the caller's
        // entry positions, permuted like the values
        std::vector<double> pos(size_t(rv->nnz));
        for (int64_t p = 0; p < rv->nnz; ++p) pos[p] = double(p);   // exact below 2^53
        const Csr a = permute(*o, rowptr, col, pos.data());
        pos.clear();
        pos.shrink_to_fit();
        const int64_t n = rv->n_pad;
        rv->arp.assign(a.rp.begin(), a.rp.end());
        rv->aci.assign(a.ci.begin(), a.ci.end());
        rv->amap.resize(a.v.size());
        parallel_for(n, kGrain, [&](int64_t r) {
            for (int64_t p = a.rp[r]; p < a.rp[r + 1]; ++p)
                rv->amap[p] = o->iperm[r] < 0 ? -1 : int64_t(a.v[p]);
        });
        const Levels lv{rv->color_start, int64_t(o->bs) * o->w, o->w};
        if ((st = lower_pattern(a, n, lv, rv->lrp))) { delete rv; return st; }
        rv->lcol.resize(rv->lrp[n]);
        parallel_for(n, kGrain, [&](int64_t r) {
            int64_t q = rv->lrp[r];
            for (int64_t p = a.rp[r]; p < a.rp[r + 1] && a.ci[p] < r; ++p) rv->lcol[q++] = a.ci[p];
        });
        auto &im = rv->image;
        rv->off_cs = im.add(rv->color_start);
        rv->off_tb = im.add(rv->tile_base);
        rv->off_arp = im.add(rv->arp);
        rv->off_aci = im.add(rv->aci);
        rv->off_amap = im.add(rv->amap);
        rv->off_lrp = im.add(rv->lrp);
        rv->off_lcol = im.add(rv->lcol);
        auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
        rv->off_lval = up(im.bytes.size());
        rv->off_d = up(rv->off_lval + rv->lcol.size() * sizeof(double));
        rv->off_flag = up(rv->off_d + size_t(n) * sizeof(double));
        rv->scratch_end = up(rv->off_flag + 256);
        *out = rv;
        return HBMC_OK;
    } catch (const std::bad_alloc &) {
        return fail(HBMC_ENOMEM, "out of host memory in hbmc_revalue_create");
    }
}

extern "C" int hbmc_revalue_device_bytes(const hbmc_revalue_t *rv, size_t *bytes) {
    if (!rv || !bytes) return fail(HBMC_EINVAL, "null argument");
    *bytes = rv->scratch_end;
    return HBMC_OK;
}

extern "C" void hbmc_revalue_destroy(hbmc_revalue_t *rv) { delete rv; }
