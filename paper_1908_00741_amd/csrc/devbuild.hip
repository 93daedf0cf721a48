// The factor and the matrix built on the device, from a CSR matrix in
// device memory and an ordering made on the host (blocking and coloring
// stay there: they are greedy sequential procedures, Section 5.1, and the
// ordering is the contract the oracle checks bit for bit):
//  - Abar = P A P^T with identity rows for the dummy unknowns (Section 3,
//    eq. "AB"), rows sorted by new column;
//  - its strictly lower pattern, and IC(0) (Section 2, eq. "ILU") with the
//    kernels of revalue.h: the host's arithmetic in the host's order;
//  - the sliced-ELL layouts of the substitutions (Section 4.4.2; per
//    (tile, step) group, the couplings to other colors in strided slots and
//    indexed slots or the flat form, the couplings inside the level-1 block
//    in slots of their own) and of the SpMV (per 64-row slice).
// The images are the host build's byte for byte: the same strided slots
// (bases col - lane shared by at least 48 lanes, most shared first, ties to
// the smaller base, at most 64 per tile and direction or per slice), the
// same left-over couplings in the same places, the same in-block slots.
//
// Two passes over the layouts, one workgroup of 64 lanes per tile (the
// steps of a tile in order: the strided-slot budget runs over them) or per
// 64-row slice: the first counts each group's slots and entries, prefix
// sums place the groups, the second writes the structure; the value
// kernels of revalue.h then write the values.
#include <cstring>
#include <vector>

#include "revalue.h"

namespace {

constexpr int kMaxLane = 64;    // couplings of one row in one group (width of the used-entry mask)
constexpr int kMaxCand = 128;   // bases shared by >= 48 lanes in one group
constexpr int kScanBlock = 1024;
constexpr int kScanPer = 8;     // elements per thread of the scan

enum : int32_t {
    kBadCsr = 1,       // columns unsorted or out of range
    kNotSym = 2,       // pattern or values not symmetric
    kBadDiag = 4,      // diagonal missing or not > 0
    kCrossL1 = 8,      // internal: a coupling joins two level-1 blocks of one color
    kLongRow = 16,     // a row has more than kMaxLane couplings in one group
    kManyCand = 32,    // more than kMaxCand strided bases in one group
    kWideGroup = 64,   // a flat group holds more than 65535 entries
};

// ---- prefix sums -----------------------------------------------------------

// a[0..len) <- exclusive prefix sums, in three launches: per block of
// kScanBlock * kScanPer elements the local sums (block total to tmp), the
// block totals in one workgroup, the block offsets added back.
__global__ void __launch_bounds__(kScanBlock) k_scan_local(int64_t *a, int64_t len, int64_t *tmp) {
    __shared__ int64_t sh[kScanBlock];
    const int64_t base = (int64_t(blockIdx.x) * kScanBlock + threadIdx.x) * kScanPer;
    int64_t v[kScanPer], s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = base + k < len ? a[base + k] : 0;
        s += v[k];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < kScanBlock; o <<= 1) {
        const int64_t t = threadIdx.x >= unsigned(o) ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t run = sh[threadIdx.x] - s;   // exclusive within the block
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < len) a[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == kScanBlock - 1) tmp[blockIdx.x] = sh[kScanBlock - 1];
}

__global__ void __launch_bounds__(kScanBlock) k_scan_tops(int64_t *tmp, int64_t nb) {
    __shared__ int64_t sh[kScanBlock];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanBlock) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t v = i < nb ? tmp[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kScanBlock; o <<= 1) {
            const int64_t t = threadIdx.x >= unsigned(o) ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) tmp[i] = carry + sh[threadIdx.x] - v;
        carry += sh[kScanBlock - 1];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_add(int64_t *a, int64_t len, const int64_t *tmp) {
    const int64_t base = (int64_t(blockIdx.x) * kScanBlock + threadIdx.x) * kScanPer;
    const int64_t add = tmp[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < len) a[base + k] += add;
}

int scan(int64_t *a, int64_t len, int64_t *tmp, hipStream_t s) {
    const int64_t per = int64_t(kScanBlock) * kScanPer;
    const int64_t nb = (len + per - 1) / per;
    if (nb == 0) return HBMC_OK;
    hipLaunchKernelGGL(k_scan_local, dim3(unsigned(nb)), dim3(kScanBlock), 0, s, a, len, tmp);
    hipLaunchKernelGGL(k_scan_tops, dim3(1), dim3(kScanBlock), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_add, dim3(unsigned(nb)), dim3(kScanBlock), 0, s, a, len, tmp);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

// ---- Abar and its lower pattern -------------------------------------------

struct In {
    const int64_t *rp;   // the caller's CSR (original numbering)
    const int32_t *ci;
    const double *v;
    int32_t n;
};

__device__ inline int64_t find_in(const int32_t *c, int64_t lo, int64_t hi, int32_t x) {
    const int64_t end = hi;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (c[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo < end && c[lo] == x ? lo : -1;
}

// Checks of the caller's CSR, one thread per row: columns strictly
// ascending and in range, a positive diagonal, and for every entry (i, j)
// the entry (j, i) with the same value.
__global__ void k_b_check(In A, int32_t *flag) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    int32_t bad = 0;
    const int64_t lo = A.rp[i], hi = A.rp[i + 1];
    if (hi < lo) { atomicOr(flag, kBadCsr); return; }
    bool diag = false;
    for (int64_t p = lo; p < hi; ++p) {
        const int32_t c = A.ci[p];
        if (c < 0 || c >= A.n || (p > lo && A.ci[p - 1] >= c)) { bad |= kBadCsr; break; }
        if (c == i) {
            diag = true;
            if (!(A.v[p] > 0.0)) bad |= kBadDiag;
            continue;
        }
        const int64_t q = find_in(A.ci, A.rp[c], A.rp[c + 1], int32_t(i));
        if (q < 0 || A.v[q] != A.v[p]) bad |= kNotSym;
    }
    if (!diag) bad |= kBadDiag;
    if (bad) atomicOr(flag, bad);
}

struct Ord {
    const int32_t *perm, *iperm;
    const int64_t *cs, *tb;
    int32_t nc, bs, w;
    int64_t n_pad;
};

__device__ inline int color_of_row(const Ord &O, int64_t r) {
    int c = 0;
    while (c + 1 < O.nc && O.cs[c + 1] <= r) ++c;
    return c;
}

__global__ void k_b_rowlen(In A, Ord O, int64_t *arp) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r > O.n_pad) return;
    if (r == O.n_pad) { arp[r] = 0; return; }
    const int32_t i = O.iperm[r];
    arp[r] = i < 0 ? 1 : A.rp[i + 1] - A.rp[i];
}

// Row r of Abar: the columns of row iperm[r] renumbered and sorted
// (insertion), with the caller's entry index of each (amap); a dummy row
// holds its diagonal only (amap -1: the value 1).
__global__ void k_b_abar(In A, Ord O, const int64_t *arp, int32_t *aci, int64_t *amap) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= O.n_pad) return;
    const int64_t b = arp[r];
    const int32_t i = O.iperm[r];
    if (i < 0) {
        aci[b] = int32_t(r);
        amap[b] = -1;
        return;
    }
    int64_t len = 0;
    for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p, ++len) {
        const int32_t c = O.perm[A.ci[p]];
        int64_t k = len;
        while (k > 0 && aci[b + k - 1] > c) {
            aci[b + k] = aci[b + k - 1];
            amap[b + k] = amap[b + k - 1];
            --k;
        }
        aci[b + k] = c;
        amap[b + k] = p;
    }
}

// Lower entries per row; a lower coupling inside a color must stay inside
// one level-1 block and one lane (Section 4.3, eq. "BAMC1").
__global__ void k_b_lowlen(Ord O, const int64_t *arp, const int32_t *aci, int64_t *lrp, int32_t *flag) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r > O.n_pad) return;
    if (r == O.n_pad) { lrp[r] = 0; return; }
    const int c = color_of_row(O, r);
    const int64_t r0 = O.cs[c], l1 = int64_t(O.bs) * O.w;
    int64_t cnt = 0;
    for (int64_t p = arp[r]; p < arp[r + 1] && aci[p] < r; ++p, ++cnt) {
        const int64_t k = aci[p];
        if (k >= r0 && ((k - r0) / l1 != (r - r0) / l1 || (r - k) % O.w != 0)) atomicOr(flag, kCrossL1);
    }
    lrp[r] = cnt;
}

__global__ void k_b_lower(Ord O, const int64_t *arp, const int32_t *aci, const int64_t *lrp, int32_t *lcol) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= O.n_pad) return;
    int64_t q = lrp[r];
    for (int64_t p = arp[r]; p < arp[r + 1] && aci[p] < r; ++p) lcol[q++] = aci[p];
}

// ---- layouts -----------------------------------------------------------------

// A lane's couplings in one group: the sorted columns col[lo, hi) of its
// row, without index skip (the diagonal, for the matrix; -1: none).
struct Span {
    int64_t lo = 0, hi = 0, skip = -1;
    __device__ int size() const { return int(hi - lo) - (skip >= lo && skip < hi ? 1 : 0); }
    __device__ int64_t at(int t) const {
        const int64_t p = lo + t;
        return skip >= lo && p >= skip ? p + 1 : p;
    }
    // position t of column x in the span, or -1
    __device__ int find(const int32_t *col, int32_t x) const {
        const int64_t p = find_in(col, lo, hi, x);
        if (p < 0 || p == skip) return -1;
        return int(p - lo) - (skip >= lo && p > skip ? 1 : 0);
    }
};

// The strided slots a group gets, in slot order (LDS of a 64-lane workgroup).
struct Sel {
    int64_t key[kMaxCand];
    uint64_t mask[kMaxCand];
    int32_t cnt[kMaxCand];
    int64_t okey[kMaxCand];
    uint64_t omask[kMaxCand];
    int32_t n;
};

__device__ inline int wsum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline int wmax(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}
// exclusive prefix sum over the 64 lanes
__device__ inline int wexcl(int v, int j) {
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(x, o, 64);
        if (j >= o) x += t;
    }
    return x - v;
}

// The host's choice of strided slots for one group (all 64 lanes call it):
// bases shared by at least kMinStridedLanes lanes with base >= 0 and
// base + 64 <= limit, most shared first, ties to the smaller base, at most
// budget.  A base shared by 48 of 64 lanes appears in one of lanes 0..16,
// so their couplings propose every candidate; a base counts once, at the
// first lane that has it.  Returns the number chosen (S.okey / S.omask in
// slot order) and, per lane, the mask of its couplings they take.
__device__ int choose_strided(Sel &S, const int32_t *col, const Span &sp, int j, int64_t limit, int budget,
                              uint64_t &used, int32_t *flag) {
    if (j == 0) S.n = 0;
    __syncthreads();
    for (int src = 0; src < 64 - kMinStridedLanes + 1; ++src) {
        Span ss;
        ss.lo = __shfl(sp.lo, src, 64);
        ss.hi = __shfl(sp.hi, src, 64);
        ss.skip = __shfl(sp.skip, src, 64);
        const int ms = ss.size();
        for (int t = 0; t < ms; ++t) {
            const int64_t key = int64_t(col[ss.at(t)]) - src;
            const int64_t want = key + j;
            const bool has = want >= 0 && want <= INT32_MAX && sp.find(col, int32_t(want)) >= 0;
            const uint64_t b = __ballot(has);
            const int nb = __popcll(b);
            if (nb >= kMinStridedLanes && key >= 0 && key + kTileLanes <= limit && __ffsll((long long)b) - 1 == src && j == 0) {
                if (S.n < kMaxCand) {
                    S.key[S.n] = key;
                    S.mask[S.n] = b;
                    S.cnt[S.n] = nb;
                } else {
                    atomicOr(flag, kManyCand);
                }
                ++S.n;
            }
        }
    }
    __syncthreads();
    const int n = min(S.n, kMaxCand);
    for (int i = j; i < n; i += 64) {
        int rank = 0;
        for (int k = 0; k < n; ++k) rank += S.cnt[k] > S.cnt[i] || (S.cnt[k] == S.cnt[i] && S.key[k] < S.key[i]);
        S.okey[rank] = S.key[i];
        S.omask[rank] = S.mask[i];
    }
    __syncthreads();
    const int nsel = min(n, max(budget, 0));
    used = 0;
    for (int k = 0; k < nsel; ++k)
        if ((S.omask[k] >> j) & 1) used |= uint64_t(1) << sp.find(col, int32_t(S.okey[k] + j));
    return nsel;
}

// t-th coupling of the span not taken by a strided slot
__device__ inline int64_t left_at(const Span &sp, uint64_t used, int t) {
    for (int k = 0;; ++k)
        if (!((used >> k) & 1) && t-- == 0) return sp.at(k);
}

// Group counts (per direction for the factor): [kind][group], kinds:
// strided slots, indexed slots, left-over entries, in-block slots (factor)
// or strided lanes (matrix).
struct Counts {
    int64_t *c[4];
};

// Where the second pass writes one direction (or the matrix).
struct Out {
    int32_t *sbase;
    uint64_t *smask;
    uint64_t *imask;     // indexed slots
    int64_t *ivoff;
    int32_t *icol;
    uint16_t *lstart;    // flat form
    int32_t *fcol;
    int8_t *int_lp;      // in-block slots
    bool flat;
};

// The left-over couplings of one group: indexed slots or the flat form.
__device__ void write_left(const Out &o, const int32_t *col, const Span &sp, uint64_t used, int left, int j,
                           int64_t g, int64_t i0, int64_t e0, int32_t *flag) {
    if (o.flat) {
        const int st = wexcl(left, j);
        if (j == 63 && st + left > 0xFFFF) atomicOr(flag, kWideGroup);
        o.lstart[g * kLanes + j] = uint16_t(st);
        for (int t = 0; t < left; ++t) o.fcol[e0 + st + t] = col[left_at(sp, used, t)];
        return;
    }
    const int len = wmax(left);
    int64_t cum = 0;
    for (int t = 0; t < len; ++t) {
        const uint64_t m = __ballot(left > t);
        if (j == 0) {
            o.imask[i0 + t] = m;
            o.ivoff[i0 + t] = e0 + cum;
        }
        if (left > t) o.icol[e0 + cum + __popcll(m & ((uint64_t(1) << j) - 1))] = col[left_at(sp, used, t)];
        cum += __popcll(m);
    }
}

struct Fac {
    const int64_t *arp;
    const int32_t *aci;
    Counts cnt[2];           // forward, backward
    Counts scan[2];          // their exclusive prefix sums (second pass)
    Out out[2];
    int64_t *maxes;          // [0..1] in-block slots of a group, [2..3] of a tile (forward, backward)
    int32_t *flag;
};

// One workgroup of 64 lanes per tile; FILL = false counts, true writes.
template <bool FILL>
__global__ void __launch_bounds__(kLanes) k_b_factor(Ord O, Fac F) {
    __shared__ Sel S;
    const int64_t t = blockIdx.x;
    const int j = threadIdx.x;
    int c = 0;
    while (c + 1 < O.nc && O.tb[c + 1] <= t) ++c;
    const int64_t lanes = (O.cs[c + 1] - O.cs[c]) / O.bs;
    const int64_t lam = (t - O.tb[c]) * kLanes + j;
    const bool valid = lam < lanes;
    const int64_t l1 = int64_t(O.bs) * O.w;
    int budget[2] = {kTileLanes, kTileLanes};
    int64_t tile_int[2] = {0, 0};
    for (int l = 0; l < O.bs; ++l) {
        const int64_t g = t * O.bs + l;
        Span ext[2], in[2];
        if (valid) {
            const int64_t row = O.cs[c] + (lam / O.w) * l1 + int64_t(l) * O.w + lam % O.w;
            const int64_t lo = F.arp[row], hi = F.arp[row + 1];
            int64_t p1 = lo, pd = lo, p2 = lo;   // first column >= cs[c], the diagonal, first >= cs[c + 1]
            while (p1 < hi && F.aci[p1] < O.cs[c]) ++p1;
            pd = p1;
            while (pd < hi && F.aci[pd] < row) ++pd;
            p2 = pd;
            while (p2 < hi && F.aci[p2] < O.cs[c + 1]) ++p2;
            ext[0] = Span{lo, p1, -1};
            in[0] = Span{p1, pd, -1};
            in[1] = Span{pd + 1, p2, -1};
            ext[1] = Span{p2, hi, -1};
        }
        for (int d = 0; d < 2; ++d) {
            if (ext[d].size() > kMaxLane || in[d].size() > kMaxLane) atomicOr(F.flag, kLongRow);
            uint64_t used = 0;
            const int ns = choose_strided(S, F.aci, ext[d], j, O.n_pad, budget[d], used, F.flag);
            budget[d] -= ns;
            const int left = ext[d].size() - __popcll(used);
            const int nint = wmax(in[d].size());
            if (!FILL) {
                const int ni = wmax(left), ne = wsum(left);
                if (j == 0) {
                    F.cnt[d].c[0][g] = ns;
                    F.cnt[d].c[1][g] = ni;
                    F.cnt[d].c[2][g] = ne;
                    F.cnt[d].c[3][g] = nint;
                    atomicMax(reinterpret_cast<unsigned long long *>(&F.maxes[d]), (unsigned long long)nint);
                }
                tile_int[d] += nint;
                continue;
            }
            const Out &o = F.out[d];
            const int64_t s0 = F.scan[d].c[0][g];
            if (j == 0)
                for (int k = 0; k < ns; ++k) {
                    o.sbase[s0 + k] = int32_t(S.okey[k]);
                    o.smask[s0 + k] = S.omask[k];
                }
            write_left(o, F.aci, ext[d], used, left, j, g, F.scan[d].c[1][g], F.scan[d].c[2][g], F.flag);
            const int64_t n0 = F.scan[d].c[3][g];
            for (int k = 0; k < nint; ++k) {
                int8_t lp = -1;
                if (k < in[d].size()) lp = int8_t(((F.aci[in[d].at(k)] - O.cs[c]) % l1) / O.w);
                o.int_lp[(n0 + k) * kLanes + j] = lp;
            }
            __syncthreads();   // S is reused by the next choose_strided
        }
    }
    if (!FILL && j == 0)
        for (int d = 0; d < 2; ++d)
            atomicMax(reinterpret_cast<unsigned long long *>(&F.maxes[2 + d]), (unsigned long long)tile_int[d]);
}

struct Mat {
    const int64_t *arp;
    const int32_t *aci;
    Counts cnt, scan;
    Out out;
    int32_t *flag;
};

// One workgroup of 64 lanes per 64-row slice of Abar (its off-diagonal
// couplings, both triangles).
template <bool FILL>
__global__ void __launch_bounds__(kLanes) k_b_matrix(Ord O, Mat M) {
    __shared__ Sel S;
    const int64_t g = blockIdx.x;
    const int j = threadIdx.x;
    const int64_t r = g * kLanes + j;
    Span sp;
    if (r < O.n_pad) {
        sp.lo = M.arp[r];
        sp.hi = M.arp[r + 1];
        sp.skip = find_in(M.aci, sp.lo, sp.hi, int32_t(r));
    }
    if (sp.size() > kMaxLane) atomicOr(M.flag, kLongRow);
    uint64_t used = 0;
    const int ns = choose_strided(S, M.aci, sp, j, O.n_pad, kTileLanes, used, M.flag);
    const int left = sp.size() - __popcll(used);
    if (!FILL) {
        const int ni = wmax(left), ne = wsum(left), sl = wsum(__popcll(used));
        if (j == 0) {
            M.cnt.c[0][g] = ns;
            M.cnt.c[1][g] = ni;
            M.cnt.c[2][g] = ne;
            M.cnt.c[3][g] = sl;
        }
        return;
    }
    const int64_t s0 = M.scan.c[0][g];
    if (j == 0)
        for (int k = 0; k < ns; ++k) {
            M.out.sbase[s0 + k] = int32_t(S.okey[k]);
            M.out.smask[s0 + k] = S.omask[k];
        }
    write_left(M.out, M.aci, sp, used, left, j, g, M.scan.c[1][g], M.scan.c[2][g], M.flag);
}

// The slot-offset arrays from the prefix sums (groups + 1 entries).
__global__ void k_b_offsets(int64_t groups, const int64_t *ss, const int64_t *si, const int64_t *se,
                            const int64_t *sn, int32_t *soff, int32_t *ioff, int64_t *goff, int32_t *int_off) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g > groups) return;
    soff[g] = int32_t(ss[g]);
    if (ioff) ioff[g] = int32_t(si[g]);
    if (goff) goff[g] = se[g];
    if (int_off) int_off[g] = int32_t(sn[g]);
}

// The padding slots and entries at the ends of the arrays (zeros except
// these; int_lp of the in-block padding slot: -1 in every lane).
__global__ void k_b_pad(Out o, int64_t islots, int64_t entries, int64_t nslots) {
    const int j = threadIdx.x;
    if (o.int_lp) o.int_lp[nslots * kLanes + j] = -1;
    if (j) return;
    if (o.flat) {
        o.fcol[entries] = -1;
    } else {
        o.ivoff[islots] = entries;
        o.icol[entries] = -1;
    }
}

// ---- the build's workspace ---------------------------------------------------

size_t up(size_t x) { return (x + 255) & ~size_t(255); }

struct Work {
    size_t perm, iperm, cs, tb, arp, aci, amap, lrp, lcol, lval, d, flag, maxes, fcnt, mcnt, tmp, end;
    int64_t G, Sl;   // factor groups, matrix slices
};

Work work_of(const hbmc_order_s *o, int64_t nnz) {
    Work w{};
    const int64_t n = o->n, np = o->n_pad, nnzA = nnz + (np - n);
    int64_t tiles = 0;
    for (int c = 0; c < o->nc; ++c)
        tiles += ((o->color_start[c + 1] - o->color_start[c]) / o->bs + kTileLanes - 1) / kTileLanes;
    w.G = tiles * o->bs;
    w.Sl = (np + kTileLanes - 1) / kTileLanes;
    size_t at = 0;
    auto add = [&](size_t bytes) { const size_t a = up(at); at = a + bytes; return a; };
    w.perm = add(size_t(n) * 4);
    w.iperm = add(size_t(np) * 4);
    w.cs = add(size_t(o->nc + 1) * 8);
    w.tb = add(size_t(o->nc + 1) * 8);
    w.arp = add(size_t(np + 1) * 8);
    w.aci = add(size_t(nnzA) * 4);
    w.amap = add(size_t(nnzA) * 8);
    w.lrp = add(size_t(np + 1) * 8);
    w.lcol = add(size_t(nnz) * 4);
    w.lval = add(size_t(nnz) * 8);
    w.d = add(size_t(np) * 8);
    w.flag = add(256);
    w.maxes = add(8 * 8);
    w.fcnt = add(size_t(8) * (w.G + 1) * 8);
    w.mcnt = add(size_t(4) * (w.Sl + 1) * 8);
    const int64_t longest = std::max<int64_t>({np + 1, w.G + 1, w.Sl + 1});
    w.tmp = add(size_t(longest / (int64_t(kScanBlock) * kScanPer) + 2) * 8);
    w.end = up(at);
    return w;
}

template <class P>
P *wp(void *base, size_t off) {
    return reinterpret_cast<P *>(static_cast<uint8_t *>(base) + off);
}

// Byte planner with the host image's rules (each array on a 256-byte
// boundary, in the host's order).
struct Plan {
    size_t at = 0;
    size_t add(size_t bytes) {
        const size_t a = up(at);
        at = a + bytes;
        return a;
    }
};

// Totals after the counting pass.
struct Tot {
    int64_t s, i, e, n;   // strided slots, indexed slots, left-over entries, in-block slots (or strided lanes)
};

unsigned blocks(int64_t n, int per) { return unsigned(std::max<int64_t>(1, (n + per - 1) / per)); }

int read_flag(void *work, const Work &W, hipStream_t s, int32_t &flag) {
    HIP_TRY(hipMemcpyAsync(&flag, wp<int32_t>(work, W.flag), sizeof flag, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return HBMC_OK;
}

int flag_error(int32_t flag) {
    if (flag & kBadCsr) return fail(HBMC_EINVAL, "CSR columns unsorted, duplicated or out of range");
    if (flag & kBadDiag) return fail(HBMC_EDIAG, "a diagonal entry is missing or not > 0");
    if (flag & kNotSym) return fail(HBMC_ENOTSYM, "pattern or values not symmetric");
    if (flag & kCrossL1) return fail(HBMC_EINVAL, "internal: a coupling crosses level-1 blocks");
    if (flag & kLongRow)
        return fail(HBMC_EINVAL, "a row has more than %d couplings in one layout group (use the host build)", kMaxLane);
    if (flag & kManyCand) return fail(HBMC_EINVAL, "more than %d strided bases in one layout group", kMaxCand);
    if (flag & kWideGroup) return fail(HBMC_EINVAL, "a (tile, step) group has more than 65535 couplings to other colors");
    return HBMC_OK;
}

}  // namespace

// Build state kept between hbmc_device_build and hbmc_device_build_fill.
struct hbmc_dbuild_s {
    Work W{};
    const hbmc_order_s *o = nullptr;
    In A{};
    int32_t precision = HBMC_F64;
    Tot ft[2]{}, mt{};
    bool flat = false;
    int64_t maxes[4]{};
};

namespace {

Counts counts_at(void *work, size_t off, int64_t len, int k0) {
    Counts c;
    for (int k = 0; k < 4; ++k) c.c[k] = wp<int64_t>(work, off) + (k0 + k) * len;
    return c;
}

Ord ord_of(const hbmc_order_s *o, void *work, const Work &W) {
    return Ord{wp<int32_t>(work, W.perm), wp<int32_t>(work, W.iperm), wp<int64_t>(work, W.cs),
               wp<int64_t>(work, W.tb), o->nc, o->bs, o->w, o->n_pad};
}

Rv rv_in(const hbmc_order_s *o, void *work, const Work &W) {
    return Rv{wp<int64_t>(work, W.cs), wp<int64_t>(work, W.tb), wp<int64_t>(work, W.arp), wp<int64_t>(work, W.amap),
              wp<int32_t>(work, W.aci), wp<int64_t>(work, W.lrp), wp<int32_t>(work, W.lcol),
              wp<double>(work, W.lval), wp<double>(work, W.d), wp<int32_t>(work, W.flag), o->nc, o->bs, o->w,
              o->n_pad};
}

}  // namespace

extern "C" int hbmc_device_build_bytes(const hbmc_order_t *o, int64_t nnz, size_t *bytes) {
    clear_error();
    if (!o || !bytes) return fail(HBMC_EINVAL, "null argument");
    if (nnz < o->n) return fail(HBMC_EINVAL, "nnz = %lld is below n", (long long)nnz);
    if (o->nsys != 1) return fail(HBMC_EINVAL, "the device build takes a single system (not a batch ordering)");
    *bytes = work_of(o, nnz).end;
    return HBMC_OK;
}

extern "C" int hbmc_device_build(const hbmc_order_t *o, const int64_t *rowptr, const int32_t *col,
                                 const double *val, int64_t nnz, int32_t precision, double shift, void *work,
                                 size_t work_bytes, void *stream, hbmc_dbuild_t **out) {
    clear_error();
    if (!out) return fail(HBMC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!o || !rowptr || !col || !val || !work) return fail(HBMC_EINVAL, "null argument");
    if (o->nsys != 1) return fail(HBMC_EINVAL, "the device build takes a single system (not a batch ordering)");
    if (precision != HBMC_F64 && precision != HBMC_F32) return fail(HBMC_EINVAL, "precision must be HBMC_F64 or HBMC_F32");
    if (!(shift >= 0.0)) return fail(HBMC_EINVAL, "shift must be >= 0");
    if (nnz < o->n) return fail(HBMC_EINVAL, "nnz = %lld is below n", (long long)nnz);
    if (o->bs > 127) return fail(HBMC_EINVAL, "bs = %d: in-block steps are stored as bytes", o->bs);
    const Work W = work_of(o, nnz);
    if (work_bytes < W.end) return fail(HBMC_EINVAL, "workspace too small (%zu < %zu)", work_bytes, W.end);
    if (reinterpret_cast<uintptr_t>(work) % 256) return fail(HBMC_EINVAL, "workspace not 256-byte aligned");
    auto s = static_cast<hipStream_t>(stream);
    {
        int64_t ends[2] = {-1, -1};
        HIP_TRY(hipMemcpyAsync(&ends[0], rowptr, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&ends[1], rowptr + o->n, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (ends[0] != 0 || ends[1] != nnz)
            return fail(HBMC_EINVAL, "rowptr[0] = %lld, rowptr[n] = %lld (nnz = %lld)", (long long)ends[0],
                        (long long)ends[1], (long long)nnz);
    }
    const In A{rowptr, col, val, o->n};
    const int64_t np = o->n_pad;
    std::vector<int64_t> tb(o->nc + 1, 0);
    for (int c = 0; c < o->nc; ++c)
        tb[c + 1] = tb[c] + ((o->color_start[c + 1] - o->color_start[c]) / o->bs + kTileLanes - 1) / kTileLanes;
    HIP_TRY(hipMemcpyAsync(wp<void>(work, W.perm), o->perm.data(), size_t(o->n) * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(wp<void>(work, W.iperm), o->iperm.data(), size_t(np) * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(wp<void>(work, W.cs), o->color_start.data(), size_t(o->nc + 1) * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(wp<void>(work, W.tb), tb.data(), size_t(o->nc + 1) * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(wp<void>(work, W.flag), 0, 256 + 64, s));   // flag and maxes
    const Ord O = ord_of(o, work, W);
    int32_t *flag = wp<int32_t>(work, W.flag);
    int64_t *tmp = wp<int64_t>(work, W.tmp);
    int64_t *arp = wp<int64_t>(work, W.arp), *lrp = wp<int64_t>(work, W.lrp);
    hipLaunchKernelGGL(k_b_check, dim3(blocks(o->n, 256)), dim3(256), 0, s, A, flag);
    int32_t fl = 0;
    int st;
    if ((st = read_flag(work, W, s, fl))) return st;
    if (fl) return flag_error(fl);
    hipLaunchKernelGGL(k_b_rowlen, dim3(blocks(np + 1, 256)), dim3(256), 0, s, A, O, arp);
    if ((st = scan(arp, np + 1, tmp, s))) return st;
    hipLaunchKernelGGL(k_b_abar, dim3(blocks(np, 256)), dim3(256), 0, s, A, O, arp, wp<int32_t>(work, W.aci),
                       wp<int64_t>(work, W.amap));
    hipLaunchKernelGGL(k_b_lowlen, dim3(blocks(np + 1, 256)), dim3(256), 0, s, O, arp, wp<int32_t>(work, W.aci),
                       lrp, flag);
    if ((st = scan(lrp, np + 1, tmp, s))) return st;
    hipLaunchKernelGGL(k_b_lower, dim3(blocks(np, 256)), dim3(256), 0, s, O, arp, wp<int32_t>(work, W.aci), lrp,
                       wp<int32_t>(work, W.lcol));
    HIP_TRY(hipGetLastError());
    if ((st = read_flag(work, W, s, fl))) return st;
    if (fl) return flag_error(fl);
    // IC(0), colors in turn
    const Rv R = rv_in(o, work, W);
    hipLaunchKernelGGL(k_rv_gather, dim3(blocks(np, 256)), dim3(256), 0, s, R, val, shift, 0, 1.0);
    for (int c = 0; c < o->nc; ++c) {
        const int64_t lanes = (o->color_start[c + 1] - o->color_start[c]) / o->bs;
        if (lanes > 0) hipLaunchKernelGGL(k_rv_ic0, dim3(blocks(lanes, 128)), dim3(128), 0, s, R, c);
    }
    HIP_TRY(hipGetLastError());
    if ((st = read_flag(work, W, s, fl))) return st;
    if (fl) return fail(HBMC_EBREAKDOWN, "IC(0) pivot not > 0 on the device");
    // layout counts and their prefix sums
    Fac F{};
    F.arp = arp;
    F.aci = wp<int32_t>(work, W.aci);
    for (int d = 0; d < 2; ++d) F.cnt[d] = counts_at(work, W.fcnt, W.G + 1, 4 * d);
    F.maxes = wp<int64_t>(work, W.maxes);
    F.flag = flag;
    Mat M{};
    M.arp = arp;
    M.aci = F.aci;
    M.cnt = counts_at(work, W.mcnt, W.Sl + 1, 0);
    M.flag = flag;
    for (int d = 0; d < 2; ++d)
        for (int k = 0; k < 4; ++k) HIP_TRY(hipMemsetAsync(F.cnt[d].c[k] + W.G, 0, 8, s));
    for (int k = 0; k < 4; ++k) HIP_TRY(hipMemsetAsync(M.cnt.c[k] + W.Sl, 0, 8, s));
    if (W.G > 0) hipLaunchKernelGGL(k_b_factor<false>, dim3(unsigned(W.G / o->bs)), dim3(kLanes), 0, s, O, F);
    hipLaunchKernelGGL(k_b_matrix<false>, dim3(unsigned(W.Sl)), dim3(kLanes), 0, s, O, M);
    HIP_TRY(hipGetLastError());
    for (int d = 0; d < 2; ++d)
        for (int k = 0; k < 4; ++k)
            if ((st = scan(F.cnt[d].c[k], W.G + 1, tmp, s))) return st;
    for (int k = 0; k < 4; ++k)
        if ((st = scan(M.cnt.c[k], W.Sl + 1, tmp, s))) return st;
    if ((st = read_flag(work, W, s, fl))) return st;
    if (fl) return flag_error(fl);
    try {
        auto *b = new hbmc_dbuild_s;
        b->W = W;
        b->o = o;
        b->A = A;
        b->precision = precision;
        int64_t t[4];
        for (int d = 0; d < 2; ++d) {
            for (int k = 0; k < 4; ++k) HIP_TRY(hipMemcpyAsync(&t[k], F.cnt[d].c[k] + W.G, 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            b->ft[d] = Tot{t[0], t[1], t[2], t[3]};
        }
        for (int k = 0; k < 4; ++k) HIP_TRY(hipMemcpyAsync(&t[k], M.cnt.c[k] + W.Sl, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(b->maxes, F.maxes, sizeof b->maxes, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        b->mt = Tot{t[0], t[1], t[2], t[3]};
        // the flat form where the left-over couplings outweigh the strided
        // slots (the host build's rule)
        b->flat = (b->ft[0].e + b->ft[1].e) / kTileLanes > b->ft[0].s + b->ft[1].s;
        *out = b;
    } catch (const std::bad_alloc &) {
        return fail(HBMC_ENOMEM, "out of host memory in hbmc_device_build");
    }
    return HBMC_OK;
}

extern "C" void hbmc_device_build_destroy(hbmc_dbuild_t *b) { delete b; }

namespace {

// The factor's and the matrix's host handles and image layouts.
void plan_factor(const hbmc_dbuild_s &b, hbmc_factor_s *f) {
    const hbmc_order_s *o = b.o;
    const Work &W = b.W;
    const size_t sT = b.precision == HBMC_F64 ? 8 : 4;
    f->n = o->n; f->bs = o->bs; f->w = o->w; f->nc = o->nc; f->precision = b.precision;
    f->n_pad = o->n_pad;
    f->nsys = 1;
    f->local = o->local;
    f->color_start = o->color_start;
    f->sys_ptr = {0, o->n};
    f->tile_base.assign(o->nc + 1, 0);
    for (int c = 0; c < o->nc; ++c)
        f->tile_base[c + 1] = f->tile_base[c] + ((o->color_start[c + 1] - o->color_start[c]) / o->bs + kTileLanes - 1) /
                                                    kTileLanes;
    const int64_t tiles = f->tile_base[o->nc];
    const int64_t parts = (o->n_pad + kPartRows - 1) / kPartRows;
    Plan p;
    f->off_dinv = p.add(size_t(o->n_pad) * sT);
    f->off_perm = p.add(size_t(o->n) * 4);
    f->off_iperm = p.add(size_t(o->n_pad) * 4);
    f->off_tile_sys = p.add(size_t(tiles) * 4);
    f->off_part_sys = p.add(size_t(parts) * 4);
    f->off_sys_tiles = p.add(size_t(o->nc) * 2 * 4);
    f->off_sys_parts = p.add(size_t(o->nc) * 2 * 4);
    for (int d = 0; d < 2; ++d) {
        const Tot &t = b.ft[d];
        TriOffsets &to = d == 0 ? f->fwd : f->bwd;
        PackedOffsets &x = to.ext;
        x = PackedOffsets{};
        x.soff = p.add(size_t(W.G + 1) * 4);
        x.sbase = p.add(size_t(t.s + 1) * 4);
        x.smask = p.add(size_t(t.s + 1) * 8);
        x.sval = p.add(size_t(t.s + 1) * kTileLanes * sT);
        if (b.flat) {
            x.goff = p.add(size_t(W.G + 1) * 8);
            x.lstart = p.add(size_t(W.G) * kTileLanes * 2);
            x.fcol = p.add(size_t(t.e + 1) * 4);
            x.fval = p.add(size_t(t.e + 1) * sT);
        } else {
            x.ioff = p.add(size_t(W.G + 1) * 4);
            x.imask = p.add(size_t(t.i + 1) * 8);
            x.ivoff = p.add(size_t(t.i + 1) * 8);
            x.icol = p.add(size_t(t.e + 1) * 4);
            x.ival = p.add(size_t(t.e + 1) * sT);
        }
        to.int_off = p.add(size_t(W.G + 1) * 4);
        to.int_lp = p.add(size_t(t.n + 1) * kTileLanes);
        to.int_val = p.add(size_t(t.n + 1) * kTileLanes * sT);
        to.int_slots = t.n;
        LayoutCounts &lc = d == 0 ? f->fcnt : f->bcnt;
        lc = LayoutCounts{t.s, t.i, t.e, t.e, b.flat};
    }
    f->dev_image_bytes = up(p.at);
    f->max_int_step_f = int32_t(b.maxes[0]);
    f->max_int_step_b = int32_t(b.maxes[1]);
    f->max_int_slots_f = int32_t(b.maxes[2]);
    f->max_int_slots_b = int32_t(b.maxes[3]);
    f->device_built = true;
}

void plan_matrix(const hbmc_dbuild_s &b, hbmc_matrix_s *m) {
    const hbmc_order_s *o = b.o;
    const Tot &t = b.mt;
    m->n = o->n;
    m->n_pad = o->n_pad;
    Plan p;
    m->off_diag = p.add(size_t(o->n_pad) * 8);
    PackedOffsets &x = m->offs;
    x = PackedOffsets{};
    x.soff = p.add(size_t(b.W.Sl + 1) * 4);
    x.sbase = p.add(size_t(t.s + 1) * 4);
    x.smask = p.add(size_t(t.s + 1) * 8);
    x.sval = p.add(size_t(t.s + 1) * kTileLanes * 8);
    x.ioff = p.add(size_t(b.W.Sl + 1) * 4);
    x.imask = p.add(size_t(t.i + 1) * 8);
    x.ivoff = p.add(size_t(t.i + 1) * 8);
    x.icol = p.add(size_t(t.e + 1) * 4);
    x.ival = p.add(size_t(t.e + 1) * 8);
    m->dev_image_bytes = up(p.at);
    m->fuse_p = 2 * t.n >= t.n + t.e;   // strided lanes against all couplings
    m->device_built = true;
}

Out out_of(void *img, const PackedOffsets &x, const TriOffsets *to, bool flat) {
    Out o{};
    o.sbase = wp<int32_t>(img, x.sbase);
    o.smask = wp<uint64_t>(img, x.smask);
    o.flat = flat;
    if (flat) {
        o.lstart = wp<uint16_t>(img, x.lstart);
        o.fcol = wp<int32_t>(img, x.fcol);
    } else {
        o.imask = wp<uint64_t>(img, x.imask);
        o.ivoff = wp<int64_t>(img, x.ivoff);
        o.icol = wp<int32_t>(img, x.icol);
    }
    o.int_lp = to ? wp<int8_t>(img, to->int_lp) : nullptr;
    return o;
}

}  // namespace

extern "C" int hbmc_device_build_create(const hbmc_dbuild_t *b, hbmc_factor_t **f, hbmc_matrix_t **m) {
    clear_error();
    if (!b || !f || !m) return fail(HBMC_EINVAL, "null argument");
    *f = nullptr;
    *m = nullptr;
    try {
        auto *fa = new hbmc_factor_s;
        auto *ma = new hbmc_matrix_s;
        plan_factor(*b, fa);
        plan_matrix(*b, ma);
        *f = fa;
        *m = ma;
    } catch (const std::bad_alloc &) {
        return fail(HBMC_ENOMEM, "out of host memory in hbmc_device_build_create");
    }
    return HBMC_OK;
}

extern "C" int hbmc_device_build_fill(const hbmc_dbuild_t *b, hbmc_factor_t *f, hbmc_matrix_t *m, void *fdev,
                                      size_t fbytes, void *mdev, size_t mbytes, void *work, void *stream) {
    clear_error();
    if (!b || !f || !m || !fdev || !mdev || !work) return fail(HBMC_EINVAL, "null argument");
    if (!f->device_built || !m->device_built) return fail(HBMC_EINVAL, "handles not made by hbmc_device_build_create");
    if (f->dev || m->dev) return fail(HBMC_EINVAL, "handles already filled");
    if (fbytes < f->dev_image_bytes || mbytes < m->dev_image_bytes) return fail(HBMC_EINVAL, "device buffer too small");
    if (reinterpret_cast<uintptr_t>(fdev) % 256 || reinterpret_cast<uintptr_t>(mdev) % 256)
        return fail(HBMC_EINVAL, "device buffer not 256-byte aligned");
    auto s = static_cast<hipStream_t>(stream);
    const Work &W = b->W;
    const hbmc_order_s *o = b->o;
    const Ord O = ord_of(o, work, W);
    int32_t *flag = wp<int32_t>(work, W.flag);
    HIP_TRY(hipMemsetAsync(fdev, 0, f->dev_image_bytes, s));
    HIP_TRY(hipMemsetAsync(mdev, 0, m->dev_image_bytes, s));
    HIP_TRY(hipMemsetAsync(flag, 0, 4, s));
    // the factor's tables
    HIP_TRY(hipMemcpyAsync(wp<void>(fdev, f->off_perm), wp<void>(work, W.perm), size_t(o->n) * 4,
                           hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(wp<void>(fdev, f->off_iperm), wp<void>(work, W.iperm), size_t(o->n_pad) * 4,
                           hipMemcpyDeviceToDevice, s));
    std::vector<int32_t> sys_t(size_t(o->nc) * 2), sys_p(size_t(o->nc) * 2);
    for (int c = 0; c < o->nc; ++c) {
        sys_t[2 * c] = int32_t(f->tile_base[c]);
        sys_t[2 * c + 1] = int32_t(f->tile_base[c + 1]);
        sys_p[2 * c] = int32_t((o->color_start[c] + kPartRows - 1) / kPartRows);
        sys_p[2 * c + 1] = int32_t((o->color_start[c + 1] + kPartRows - 1) / kPartRows);
    }
    HIP_TRY(hipMemcpyAsync(wp<void>(fdev, f->off_sys_tiles), sys_t.data(), sys_t.size() * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(wp<void>(fdev, f->off_sys_parts), sys_p.data(), sys_p.size() * 4, hipMemcpyHostToDevice, s));
    // the factor's structure
    Fac F{};
    F.arp = wp<int64_t>(work, W.arp);
    F.aci = wp<int32_t>(work, W.aci);
    F.flag = flag;
    F.maxes = wp<int64_t>(work, W.maxes);
    for (int d = 0; d < 2; ++d) {
        F.scan[d] = counts_at(work, W.fcnt, W.G + 1, 4 * d);
        const TriOffsets &to = d == 0 ? f->fwd : f->bwd;
        F.out[d] = out_of(fdev, to.ext, &to, b->flat);
        const Counts &sc = F.scan[d];
        const PackedOffsets &x = to.ext;
        hipLaunchKernelGGL(k_b_offsets, dim3(blocks(W.G + 1, 256)), dim3(256), 0, s, W.G, sc.c[0], sc.c[1], sc.c[2],
                           sc.c[3], wp<int32_t>(fdev, x.soff), b->flat ? nullptr : wp<int32_t>(fdev, x.ioff),
                           b->flat ? wp<int64_t>(fdev, x.goff) : nullptr, wp<int32_t>(fdev, to.int_off));
        hipLaunchKernelGGL(k_b_pad, dim3(1), dim3(kLanes), 0, s, F.out[d], b->ft[d].i, b->ft[d].e, b->ft[d].n);
    }
    if (W.G > 0) hipLaunchKernelGGL(k_b_factor<true>, dim3(unsigned(W.G / o->bs)), dim3(kLanes), 0, s, O, F);
    // the matrix's structure
    Mat M{};
    M.arp = F.arp;
    M.aci = F.aci;
    M.scan = counts_at(work, W.mcnt, W.Sl + 1, 0);
    M.out = out_of(mdev, m->offs, nullptr, false);
    M.flag = flag;
    hipLaunchKernelGGL(k_b_offsets, dim3(blocks(W.Sl + 1, 256)), dim3(256), 0, s, W.Sl, M.scan.c[0], M.scan.c[1],
                       M.scan.c[2], M.scan.c[3], wp<int32_t>(mdev, m->offs.soff), wp<int32_t>(mdev, m->offs.ioff),
                       nullptr, nullptr);
    hipLaunchKernelGGL(k_b_pad, dim3(1), dim3(kLanes), 0, s, M.out, b->mt.i, b->mt.e, int64_t(0));
    hipLaunchKernelGGL(k_b_matrix<true>, dim3(unsigned(W.Sl)), dim3(kLanes), 0, s, O, M);
    HIP_TRY(hipGetLastError());
    int32_t fl = 0;
    int st;
    if ((st = read_flag(work, W, s, fl))) return st;
    if (fl) return flag_error(fl);
    // values: the factor (L, U = D^-1 L^T, diaginv), the matrix
    f->dev = fdev;
    f->dev_bytes = fbytes;
    const Rv R = rv_in(o, work, W);
    st = f->precision == HBMC_F64 ? pack_factor<double>(f, R, s) : pack_factor<float>(f, R, s);
    if (st) { f->dev = nullptr; return st; }
    const PackedOffsets &x = m->offs;
    const MatVals MV{wp<double>(mdev, m->off_diag), wp<int32_t>(mdev, x.soff), wp<int32_t>(mdev, x.sbase),
                     wp<uint64_t>(mdev, x.smask), wp<double>(mdev, x.sval), wp<int32_t>(mdev, x.ioff),
                     wp<uint64_t>(mdev, x.imask), wp<int64_t>(mdev, x.ivoff), wp<int32_t>(mdev, x.icol),
                     wp<double>(mdev, x.ival)};
    hipLaunchKernelGGL(k_rv_matrix, dim3(unsigned(W.Sl)), dim3(kLanes), 0, s, R, MV, b->A.v);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    m->dev = mdev;
    m->dev_bytes = mbytes;
    m->uid = next_uid();
    f->uid = next_uid();
    // d and L stay in the workspace (hbmc_factor_export reads them there)
    f->nnz_lower = 0;
    HIP_TRY(hipMemcpy(&f->nnz_lower, wp<int64_t>(work, W.lrp) + o->n_pad, 8, hipMemcpyDeviceToHost));
    f->dev_d = wp<double>(work, W.d);
    f->dev_lrp = wp<int64_t>(work, W.lrp);
    f->dev_lcol = wp<int32_t>(work, W.lcol);
    f->dev_lval = wp<double>(work, W.lval);
    return HBMC_OK;
}

int hbmc::device_export(const hbmc_factor_s *f, double *d, int64_t *lrp, int32_t *lcol, double *lval) {
    if (!f->dev_d) return fail(HBMC_ENOTREADY, "device build not filled");
    const int64_t np = f->n_pad, nl = f->nnz_lower;
    if (d) HIP_TRY(hipMemcpy(d, f->dev_d, size_t(np) * 8, hipMemcpyDeviceToHost));
    if (lrp) HIP_TRY(hipMemcpy(lrp, f->dev_lrp, size_t(np + 1) * 8, hipMemcpyDeviceToHost));
    if (lcol) HIP_TRY(hipMemcpy(lcol, f->dev_lcol, size_t(nl) * 4, hipMemcpyDeviceToHost));
    if (lval) HIP_TRY(hipMemcpy(lval, f->dev_lval, size_t(nl) * 8, hipMemcpyDeviceToHost));
    return HBMC_OK;
}
