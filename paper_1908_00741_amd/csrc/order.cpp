// Host side of the ordering: block multi-color ordering (BMC) and the HBMC
// secondary reordering (Sections 4.1-4.3; blocking and coloring heuristics
// of Section 5.1).
#include <algorithm>
#include <numeric>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <thread>
#include <atomic>

#include "hbmc_internal.h"
#include "parallel.h"

namespace hbmc {

static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

namespace {
std::atomic<int> g_threads{0};
}  // namespace

int setup_threads() {
    const int t = g_threads.load();
    if (t > 0) return t;
    return int(std::max(1u, std::thread::hardware_concurrency()));
}

size_t ImageBuilder::add(const void *src, size_t n) {
    size_t at = (bytes.size() + 255) & ~size_t(255);
    bytes.resize(at + n);
    constexpr int64_t kPiece = int64_t(1) << 22;   // bytes per thread of a large copy, at least
    parallel_chunks(int64_t(n), chunks_for(int64_t(n), kPiece), [&](int64_t lo, int64_t hi, int) {
        if (hi > lo) std::memcpy(bytes.data() + at + lo, static_cast<const uint8_t *>(src) + lo, size_t(hi - lo));
    });
    return at;
}

int check_csr(int32_t n, const int64_t *rp, const int32_t *ci, const double *v) {
    if (n < 1) return fail(HBMC_EINVAL, "n must be >= 1 (got %d)", n);
    if (!rp || !ci) return fail(HBMC_EINVAL, "null CSR pointer");
    if (rp[0] != 0) return fail(HBMC_EINVAL, "rowptr[0] must be 0");
    for (int32_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return fail(HBMC_EINVAL, "rowptr decreases at row %d", i);
    // Rows are checked in parallel chunks; the error reported is the one of
    // the first offending row (as a row-by-row check would find it).
    struct Bad { int32_t row = -1, code = 0, other = 0; const char *what = nullptr; };
    constexpr int64_t kRows = 16384;
    auto first_bad = [&](auto &&check_row) -> Bad {
        const int chunks = chunks_for(n, kRows);
        std::vector<Bad> bad(chunks);
        parallel_chunks(n, chunks, [&](int64_t lo, int64_t hi, int c) {
            for (int64_t i = lo; i < hi && bad[c].row < 0; ++i) check_row(int32_t(i), bad[c]);
        });
        for (const Bad &x : bad)
            if (x.row >= 0) return x;
        return Bad{};
    };
    Bad e = first_bad([&](int32_t i, Bad &b) {
        bool diag = false;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] < 0 || ci[p] >= n) { b = {i, HBMC_EINVAL, 0, "column out of range in row %d"}; return; }
            if (p > rp[i] && ci[p] <= ci[p - 1]) {
                b = {i, HBMC_EINVAL, 0, "columns of row %d not strictly ascending"};
                return;
            }
            if (ci[p] == i) {
                diag = true;
                if (v && !(v[p] > 0.0)) { b = {i, HBMC_EDIAG, 0, "diagonal of row %d is not > 0"}; return; }
            }
        }
        if (!diag) b = {i, HBMC_EDIAG, 0, "row %d has no diagonal entry"};
    });
    if (e.row >= 0) return fail(e.code, e.what, e.row);
    // symmetry: every off-diagonal entry (i, j) has a mirror (j, i) with the
    // same value (rows are sorted: binary search in row j)
    e = first_bad([&](int32_t i, Bad &b) {
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            const int32_t j = ci[p];
            if (j == i) continue;
            const int32_t *lo = ci + rp[j], *hi = ci + rp[j + 1];
            const int32_t *q = std::lower_bound(lo, hi, i);
            if (q == hi || *q != i) { b = {i, HBMC_ENOTSYM, j, "pattern not symmetric: (%d,%d) has no mirror"}; return; }
            if (v && v[q - ci] != v[p]) { b = {i, HBMC_ENOTSYM, j, "values not symmetric at (%d,%d)"}; return; }
        }
    });
    if (e.row >= 0) return fail(e.code, e.what, e.row, e.other);
    return HBMC_OK;
}

}  // namespace hbmc

using namespace hbmc;

namespace {

// Blocking: blocks of bs unknowns grown from the minimal-numbered
// unassigned unknown through its smallest unassigned neighbours.  The
// frontier is kept as an unsorted candidate list; each pick scans it for the
// smallest unassigned entry and drops entries that became assigned.
void build_blocks(int32_t n, const int64_t *rp, const int32_t *ci, int32_t bs,
                  std::vector<int32_t> &members) {
    members.clear();
    members.reserve(n);
    std::vector<uint8_t> taken(n, 0);
    std::vector<int32_t> cand;
    int32_t scan = 0;   // every unknown below scan is assigned
    while (true) {
        while (scan < n && taken[scan]) ++scan;
        if (scan >= n) break;
        cand.clear();
        int32_t u = scan;
        for (int32_t size = 1;; ++size) {
            taken[u] = 1;
            members.push_back(u);
            if (size == bs) break;
            for (int64_t p = rp[u]; p < rp[u + 1]; ++p)
                if (!taken[ci[p]]) cand.push_back(ci[p]);
            int32_t best = -1;
            size_t keep = 0;
            for (size_t t = 0; t < cand.size(); ++t) {
                int32_t v = cand[t];
                if (taken[v]) continue;
                cand[keep++] = v;
                if (best < 0 || v < best) best = v;
            }
            cand.resize(keep);
            if (best < 0) {
                while (scan < n && taken[scan]) ++scan;
                if (scan >= n) break;
                best = scan;
            }
            u = best;
        }
    }
}

// Greedy coloring of the block graph: blocks in id order, smallest color
// not present among already-colored adjacent blocks.  The colors of the
// neighbours are collected in a bitmap that grows with the color count.
int32_t color_blocks(int32_t n, const int64_t *rp, const int32_t *ci, int32_t bs,
                     const std::vector<int32_t> &members, std::vector<int32_t> &color) {
    const int64_t nb = (int64_t(n) + bs - 1) / bs;
    std::vector<int32_t> block(n);
    for (int64_t t = 0; t < n; ++t) block[members[t]] = int32_t(t / bs);
    color.assign(nb, -1);
    std::vector<uint64_t> used;
    int32_t ncolors = 0;
    for (int64_t b = 0; b < nb; ++b) {
        std::fill(used.begin(), used.end(), 0);
        const int64_t t1 = std::min<int64_t>((b + 1) * bs, n);
        for (int64_t t = b * bs; t < t1; ++t) {
            const int32_t u = members[t];
            for (int64_t p = rp[u]; p < rp[u + 1]; ++p) {
                const int32_t c = color[block[ci[p]]];
                if (c < 0) continue;   // not colored yet (or this block)
                if (size_t(c / 64) >= used.size()) used.resize(c / 64 + 1, 0);
                used[c / 64] |= uint64_t(1) << (c % 64);
            }
        }
        int32_t c = 0;
        for (size_t wd = 0;; ++wd) {
            const uint64_t bits = wd < used.size() ? used[wd] : 0;
            if (bits != ~uint64_t(0)) {
                c = int32_t(wd * 64) + __builtin_ctzll(~bits);
                break;
            }
        }
        color[b] = c;
        ncolors = std::max(ncolors, c + 1);
    }
    return ncolors;
}

}  // namespace

// Orders nsys independent systems stored as one block-diagonal CSR (rows
// [sys_ptr[s], sys_ptr[s+1]) of system s couple only among themselves).  Each
// system is blocked, colored and reordered exactly as it would be alone; the
// union is laid out color-major: color c holds, system after system, that
// system's color-c unknowns.  With one system each color is padded to a
// multiple of w blocks (Section 4.3); with several, each system's part of a
// color is padded to a multiple of kTileLanes blocks, so that no tile of
// kTileLanes lanes (one lane per BMC block) spans two systems.
// unit: padding of each (color, system) segment, in BMC blocks
static int order_systems(int32_t nsys, const int64_t *sys_ptr, int32_t n, const int64_t *rowptr,
                         const int32_t *col, int32_t bs, int32_t w, bool batch, hbmc_order_t **out) {
    clear_error();
    if (!out) return fail(HBMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (bs < 1 || bs > 32) return fail(HBMC_EINVAL, "bs must be in [1, 32] (got %d)", bs);
    if (w < 1 || w > kTileLanes || kTileLanes % w != 0)
        return fail(HBMC_EINVAL, "w must divide %d (got %d)", kTileLanes, w);
    if (nsys < 1 || !sys_ptr) return fail(HBMC_EINVAL, "need at least one system");
    if (sys_ptr[0] != 0 || sys_ptr[nsys] != n) return fail(HBMC_EINVAL, "system offsets must run from 0 to n");
    for (int32_t s = 0; s < nsys; ++s)
        if (sys_ptr[s + 1] <= sys_ptr[s]) return fail(HBMC_EINVAL, "system %d is empty", s);
    int st = check_csr(n, rowptr, col, nullptr);
    if (st) return st;
    try {
        auto *h = new hbmc_order_s;
        h->n = n; h->bs = bs; h->w = w; h->nsys = nsys;
        h->sys_ptr.assign(sys_ptr, sys_ptr + nsys + 1);
        // padding unit in blocks: w for one system (Section 3); in a batch,
        // whole tiles of kTileLanes blocks that also fill whole parts of
        // kPartRows rows, so that no tile and no part spans two systems
        const int64_t unit = batch ? std::lcm<int64_t>(kTileLanes, kPartRows / std::gcd(kPartRows, bs)) : w;
        // per system: blocks (global unknown ids) and their colors
        std::vector<std::vector<int32_t>> members(nsys), color(nsys);
        std::vector<int64_t> lrp;
        std::vector<int32_t> lci;
        h->nc = 0;
        h->nblocks = 0;
        for (int32_t s = 0; s < nsys; ++s) {
            const int64_t a = sys_ptr[s], b = sys_ptr[s + 1];
            const int32_t ns = int32_t(b - a);
            lrp.assign(ns + 1, 0);
            lci.clear();
            for (int64_t i = a; i < b; ++i) {
                for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
                    if (col[p] < a || col[p] >= b) {
                        delete h;
                        return fail(HBMC_EINVAL, "row %lld of system %d couples outside it", (long long)i, s);
                    }
                    lci.push_back(int32_t(col[p] - a));
                }
                lrp[i - a + 1] = int64_t(lci.size());
            }
            build_blocks(ns, lrp.data(), lci.data(), bs, members[s]);
            const int32_t nc = color_blocks(ns, lrp.data(), lci.data(), bs, members[s], color[s]);
            for (auto &u : members[s]) u += int32_t(a);
            h->nc = std::max(h->nc, nc);
            h->nblocks += int64_t(color[s].size());
        }
        // segment of (color c, system s): rows seg[c * (nsys + 1) + s] ..
        h->seg.assign(int64_t(h->nc) * (nsys + 1), 0);
        h->color_start.assign(h->nc + 1, 0);
        std::vector<std::vector<std::vector<int32_t>>> of_color(h->nc, std::vector<std::vector<int32_t>>(nsys));
        for (int32_t s = 0; s < nsys; ++s)
            for (int64_t b = 0; b < int64_t(color[s].size()); ++b) of_color[color[s][b]][s].push_back(int32_t(b));
        int64_t at = 0;
        for (int32_t c = 0; c < h->nc; ++c) {
            h->color_start[c] = at;
            for (int32_t s = 0; s < nsys; ++s) {
                h->seg[int64_t(c) * (nsys + 1) + s] = at;
                const int64_t padded = (int64_t(of_color[c][s].size()) + unit - 1) / unit * unit;
                at += padded * bs;
            }
            h->seg[int64_t(c) * (nsys + 1) + nsys] = at;
        }
        h->color_start[h->nc] = at;
        h->n_pad = at;
        if (h->n_pad > INT32_MAX) { delete h; return fail(HBMC_EINVAL, "n_pad exceeds int32"); }
        h->perm.assign(n, -1);
        h->iperm.assign(h->n_pad, -1);
        // the q-th block of (color c, system s) is BMC block m = q mod w of
        // level-1 block k' = q / w of that segment; its j-th member goes to
        // segment start + k' bs w + j w + m
        for (int32_t c = 0; c < h->nc; ++c)
            for (int32_t s = 0; s < nsys; ++s) {
                const auto &list = of_color[c][s];
                const int64_t s0 = h->seg[int64_t(c) * (nsys + 1) + s];
                const int64_t ns = sys_ptr[s + 1] - sys_ptr[s];
                for (size_t q = 0; q < list.size(); ++q) {
                    const int64_t kp = int64_t(q) / w, m = int64_t(q) % w;
                    const int64_t first = int64_t(list[q]) * bs;
                    for (int32_t j = 0; j < bs && first + j < ns; ++j) {
                        const int64_t dst = s0 + kp * bs * w + int64_t(j) * w + m;
                        const int32_t u = members[s][first + j];
                        h->perm[u] = int32_t(dst);
                        h->iperm[dst] = u;
                    }
                }
            }
        *out = h;
        return HBMC_OK;
    } catch (const std::bad_alloc &) {
        return fail(HBMC_ENOMEM, "out of host memory in hbmc_order");
    }
}

extern "C" int hbmc_order(int32_t n, const int64_t *rowptr, const int32_t *col, int32_t bs,
                          int32_t w, hbmc_order_t **out) {
    const int64_t sys_ptr[2] = {0, n};
    if (n < 1) return fail(HBMC_EINVAL, "n must be >= 1 (got %d)", n);
    return order_systems(1, sys_ptr, n, rowptr, col, bs, w, false, out);
}

// Reverse Cuthill-McKee numbering of a symmetric pattern: order[k] is the
// unknown numbered k.  The degree of an unknown counts its off-diagonal
// entries.  Each connected component starts at its unvisited unknown of
// least degree (the smallest index among equals; components in the order of
// those starts); every unknown taken from the queue appends its unvisited
// neighbours by (degree, index); the whole Cuthill-McKee sequence is then
// reversed.
static void rcm_order(int32_t n, const int64_t *rp, const int32_t *ci, std::vector<int32_t> &order) {
    std::vector<int32_t> deg(n), by_deg(n);
    parallel_for(n, 1 << 16, [&](int64_t i) {
        int32_t d = 0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) d += ci[p] != i;
        deg[i] = d;
    });
    std::iota(by_deg.begin(), by_deg.end(), 0);
    std::stable_sort(by_deg.begin(), by_deg.end(), [&](int32_t a, int32_t b) { return deg[a] < deg[b]; });
    std::vector<char> seen(n, 0);
    order.assign(size_t(n), 0);
    int64_t len = 0, head = 0, next_start = 0;
    // (degree, index) order of the neighbours an unknown appends: rows are
    // short, so an insertion sort in place in the sequence
    auto before = [&](int32_t a, int32_t b) { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; };
    while (len < n) {
        while (seen[by_deg[next_start]]) ++next_start;
        const int32_t s = by_deg[next_start];
        seen[s] = 1;
        order[len++] = s;
        for (; head < len; ++head) {
            const int32_t u = order[head];
            const int64_t first = len;
            for (int64_t p = rp[u]; p < rp[u + 1]; ++p) {
                const int32_t v = ci[p];
                if (seen[v]) continue;
                seen[v] = 1;
                int64_t k = len++;
                while (k > first && before(v, order[k - 1])) { order[k] = order[k - 1]; --k; }
                order[k] = v;
            }
        }
    }
    std::reverse(order.begin(), order.end());
}

extern "C" int hbmc_rcm(int32_t n, const int64_t *rowptr, const int32_t *col, int32_t *order) {
    clear_error();
    if (!order) return fail(HBMC_EINVAL, "order is NULL");
    int st = check_csr(n, rowptr, col, nullptr);
    if (st) return st;
    try {
        std::vector<int32_t> o;
        rcm_order(n, rowptr, col, o);
        std::memcpy(order, o.data(), size_t(n) * sizeof(int32_t));
        return HBMC_OK;
    } catch (const std::bad_alloc &) {
        return fail(HBMC_ENOMEM, "out of host memory in hbmc_rcm");
    }
}

extern "C" int hbmc_order_rcm(int32_t n, const int64_t *rowptr, const int32_t *col, int32_t bs, int32_t w,
                              hbmc_order_t **out) {
    clear_error();
    if (!out) return fail(HBMC_EINVAL, "out is NULL");
    *out = nullptr;
    int st = check_csr(n, rowptr, col, nullptr);
    if (st) return st;
    try {
        // the pattern renumbered: row k of it is row order[k] of the input
        std::vector<int32_t> ord, inv(n);
        rcm_order(n, rowptr, col, ord);
        parallel_for(n, 1 << 16, [&](int64_t k) { inv[ord[k]] = int32_t(k); });
        std::vector<int64_t> rp(int64_t(n) + 1, 0);
        std::vector<int32_t> ci(size_t(rowptr[n]));
        for (int32_t k = 0; k < n; ++k) rp[k + 1] = rp[k] + (rowptr[ord[k] + 1] - rowptr[ord[k]]);
        parallel_for(n, 1 << 14, [&](int64_t k) {
            const int32_t u = ord[k];
            int64_t at = rp[k];
            for (int64_t p = rowptr[u]; p < rowptr[u + 1]; ++p) ci[size_t(at++)] = inv[col[p]];
            std::sort(ci.begin() + rp[k], ci.begin() + at);
        });
        const int64_t sys_ptr[2] = {0, n};
        hbmc_order_t *h = nullptr;
        if ((st = order_systems(1, sys_ptr, n, rp.data(), ci.data(), bs, w, false, &h))) return st;
        // back to the input's numbering
        std::vector<int32_t> perm(n);
        parallel_for(n, 1 << 16, [&](int64_t u) { perm[u] = h->perm[inv[u]]; });
        h->perm.swap(perm);
        parallel_for(int64_t(h->iperm.size()), 1 << 16, [&](int64_t x) {
            if (h->iperm[x] >= 0) h->iperm[x] = ord[h->iperm[x]];
        });
        h->local = true;
        *out = h;
        return HBMC_OK;
    } catch (const std::bad_alloc &) {
        return fail(HBMC_ENOMEM, "out of host memory in hbmc_order_rcm");
    }
}

extern "C" int hbmc_order_batch(int32_t nsys, const int64_t *sys_ptr, int32_t n, const int64_t *rowptr,
                                const int32_t *col, int32_t bs, int32_t w, hbmc_order_t **out) {
    return order_systems(nsys, sys_ptr, n, rowptr, col, bs, w, true, out);
}

extern "C" int hbmc_order_info(const hbmc_order_t *h, hbmc_order_info_t *info) {
    if (!h || !info) return fail(HBMC_EINVAL, "null argument");
    info->n = h->n;
    info->n_pad = h->n_pad;
    info->n_blocks = h->nblocks;
    info->n_colors = h->nc;
    info->bs = h->bs;
    info->w = h->w;
    info->n_systems = h->nsys;
    return HBMC_OK;
}

extern "C" int hbmc_order_perm(const hbmc_order_t *h, int32_t *perm, int64_t *color_start) {
    if (!h) return fail(HBMC_EINVAL, "null handle");
    if (perm) std::memcpy(perm, h->perm.data(), h->perm.size() * sizeof(int32_t));
    if (color_start)
        std::memcpy(color_start, h->color_start.data(), h->color_start.size() * sizeof(int64_t));
    return HBMC_OK;
}

extern "C" void hbmc_order_destroy(hbmc_order_t *h) { delete h; }

extern "C" const char *hbmc_last_error(void) { return hbmc::g_last_error.c_str(); }

extern "C" int hbmc_set_num_threads(int32_t threads) {
    if (threads < 0) return fail(HBMC_EINVAL, "threads = %d", threads);
    hbmc::g_threads.store(threads);
    return HBMC_OK;
}
