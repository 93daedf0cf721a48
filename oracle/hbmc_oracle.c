/*
 * hbmc_oracle.c -- plain, sequential, FP64 CPU reference for the
 * HBMC-ordered IC(0)-preconditioned CG method of Iwashita, Li and Fukaya,
 * "Hierarchical block multi-color ordering" (arXiv 1908.00741).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP library is
 * checked against.  It shares no code, header or table with the library, and
 * only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It is written for clarity, not speed: every step follows the
 * paper's definitions in the paper's order, one unknown at a time.
 *
 * Readings taken where the paper is silent (each is listed with its reason in
 * the design notes of the repository):
 *   - blocking: a block grows from the smallest unassigned unknown by
 *     repeatedly taking the smallest unassigned unknown adjacent to any
 *     member, else the smallest unassigned unknown overall (Section 5.1 names
 *     the minimal-number seed; the growth rule is not printed);
 *   - greedy block coloring in block-id order, smallest free color;
 *   - members of a block keep their insertion order;
 *   - padding (Section 4.3): the short last block is completed with dummy
 *     unknowns, and each color gets all-dummy blocks appended until its block
 *     count is a multiple of w; dummy rows are identity rows;
 *   - IC(0) in the form M = (D + L) D^-1 (D + L^T), computed by the
 *     right-looking update with overwriting of Appendix A, with diaginv = 1/d
 *     multiplied in as in the forward-substitution listing (Fig. 6);
 *   - PCG stops when ||r||_2 / ||b||_2 < tol for the recurrence residual
 *     (Section 5.1), checked after every update of r.
 *   - the optional locality pre-pass (not in the paper: its blocking takes
 *     seeds in the input numbering): reverse Cuthill-McKee, each component
 *     started at its unvisited unknown of least off-diagonal degree (the
 *     smallest index among equals), neighbours queued by (degree, index).
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -o liboracle.so hbmc_oracle.c
 * (no FMA contraction, so every product and sum rounds separately).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOTSYM (-2)
#define ORC_EDIAG (-3)
#define ORC_EBREAKDOWN (-4)
#define ORC_ENOMEM (-6)
#define ORC_ENOCONV 1

/* Position of entry (i, j) in a CSR matrix with sorted rows, or -1. */
static int64_t csr_find(const int64_t *rp, const int32_t *ci, int32_t i, int32_t j)
{
    int64_t lo = rp[i], hi = rp[i + 1] - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (ci[mid] == j) return mid;
        if (ci[mid] < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------------
 * Input checks.  The method assumes a symmetric positive (semi)definite
 * matrix (Section 2); here: square CSR, 0-based, strictly ascending columns,
 * a positive diagonal, and an exactly symmetric pattern and value set.
 * ---------------------------------------------------------------------- */
int orc_check(int32_t n, const int64_t *rp, const int32_t *ci, const double *v)
{
    if (n < 1 || !rp || !ci) return ORC_EINVAL;
    if (rp[0] != 0) return ORC_EINVAL;
    for (int32_t i = 0; i < n; i++) {
        if (rp[i + 1] < rp[i]) return ORC_EINVAL;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            if (ci[p] < 0 || ci[p] >= n) return ORC_EINVAL;
            if (p > rp[i] && ci[p] <= ci[p - 1]) return ORC_EINVAL;
        }
    }
    for (int32_t i = 0; i < n; i++) {
        int64_t dpos = csr_find(rp, ci, i, i);
        if (dpos < 0) return ORC_EDIAG;
        if (v && !(v[dpos] > 0.0)) return ORC_EDIAG;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            int64_t q = csr_find(rp, ci, ci[p], i);
            if (q < 0) return ORC_ENOTSYM;
            if (v && v[q] != v[p]) return ORC_ENOTSYM;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * A binary min-heap of unknown indices, used as the blocking frontier.
 * ---------------------------------------------------------------------- */
typedef struct { int32_t *a; int64_t len, cap; } heap_t;

static int heap_push(heap_t *h, int32_t x)
{
    if (h->len == h->cap) {
        int64_t cap = h->cap ? 2 * h->cap : 64;
        int32_t *a = (int32_t *)realloc(h->a, (size_t)cap * sizeof(int32_t));
        if (!a) return ORC_ENOMEM;
        h->a = a; h->cap = cap;
    }
    int64_t k = h->len++;
    h->a[k] = x;
    while (k > 0) {
        int64_t parent = (k - 1) / 2;
        if (h->a[parent] <= h->a[k]) break;
        int32_t t = h->a[parent]; h->a[parent] = h->a[k]; h->a[k] = t;
        k = parent;
    }
    return ORC_OK;
}

static int32_t heap_pop(heap_t *h)
{
    int32_t top = h->a[0];
    h->a[0] = h->a[--h->len];
    int64_t k = 0;
    for (;;) {
        int64_t l = 2 * k + 1, r = l + 1, m = k;
        if (l < h->len && h->a[l] < h->a[m]) m = l;
        if (r < h->len && h->a[r] < h->a[m]) m = r;
        if (m == k) break;
        int32_t t = h->a[m]; h->a[m] = h->a[k]; h->a[k] = t;
        k = m;
    }
    return top;
}

/* ------------------------------------------------------------------------
 * BMC blocking (Section 4.1; heuristic of Section 5.1).  The unknowns are
 * divided into blocks of b_s unknowns.  A new block starts at the smallest
 * unassigned unknown; it then grows by the smallest unassigned unknown
 * adjacent to any of its members, or, if there is none, by the smallest
 * unassigned unknown overall, so that every block but the last has exactly
 * b_s members.
 *
 * Output: members[n], the unknowns listed block by block (block b occupies
 * members[b*bs .. min((b+1)*bs, n)) in insertion order); *nblocks.
 * ---------------------------------------------------------------------- */
int orc_blocking(int32_t n, const int64_t *rp, const int32_t *ci, int32_t bs,
                 int32_t *members, int32_t *nblocks)
{
    if (n < 1 || bs < 1) return ORC_EINVAL;
    char *assigned = (char *)calloc((size_t)n, 1);
    heap_t frontier = {0, 0, 0};
    if (!assigned) return ORC_ENOMEM;
    int32_t next = 0, nb = 0;
    int64_t pos = 0;
    int status = ORC_OK;
    for (;;) {
        while (next < n && assigned[next]) next++;
        if (next == n) break;
        frontier.len = 0;
        int32_t u = next;               /* seed: minimal-numbered unassigned */
        int32_t size = 0;
        for (;;) {
            assigned[u] = 1;
            members[pos++] = u;
            size++;
            if (size == bs) break;
            for (int64_t p = rp[u]; p < rp[u + 1]; p++)
                if (!assigned[ci[p]] && (status = heap_push(&frontier, ci[p])) != ORC_OK)
                    goto done;
            u = -1;
            while (frontier.len > 0) {
                int32_t cand = heap_pop(&frontier);
                if (!assigned[cand]) { u = cand; break; }
            }
            if (u < 0) {                 /* no unassigned neighbour left */
                while (next < n && assigned[next]) next++;
                if (next == n) break;
                u = next;
            }
        }
        nb++;
    }
    *nblocks = nb;
done:
    free(frontier.a);
    free(assigned);
    return status;
}

/* ------------------------------------------------------------------------
 * Reverse Cuthill-McKee numbering (the locality pre-pass; not a step of the
 * paper's method).  deg(i) = number of j != i with a_ij != 0.  Repeat until
 * every unknown is numbered: start a breadth-first sweep at the unnumbered
 * unknown of least degree (smallest index among equals); when an unknown
 * leaves the queue, its unnumbered neighbours are numbered next, by
 * increasing (degree, index).  The resulting sequence is reversed.
 * Output: order[k] = the unknown numbered k.
 * ---------------------------------------------------------------------- */
int orc_rcm(int32_t n, const int64_t *rp, const int32_t *ci, int32_t *order)
{
    if (n < 1) return ORC_EINVAL;
    int32_t *deg = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    char *numbered = (char *)calloc((size_t)n, 1);
    int32_t *cm = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!deg || !numbered || !cm) { free(deg); free(numbered); free(cm); return ORC_ENOMEM; }
    for (int32_t i = 0; i < n; i++) {
        deg[i] = 0;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++)
            if (ci[p] != i) deg[i]++;
    }
    int32_t count = 0, head = 0;
    while (count < n) {
        int32_t s = -1;
        for (int32_t i = 0; i < n; i++)
            if (!numbered[i] && (s < 0 || deg[i] < deg[s])) s = i;
        numbered[s] = 1;
        cm[count++] = s;
        while (head < count) {
            int32_t u = cm[head++];
            int32_t first = count;
            for (int64_t p = rp[u]; p < rp[u + 1]; p++) {
                int32_t v = ci[p];
                if (numbered[v]) continue;
                /* insert v into cm[first .. count) kept sorted by (deg, index) */
                int32_t k = count++;
                while (k > first && (deg[cm[k - 1]] > deg[v] ||
                                     (deg[cm[k - 1]] == deg[v] && cm[k - 1] > v))) {
                    cm[k] = cm[k - 1];
                    k--;
                }
                cm[k] = v;
                numbered[v] = 1;
            }
        }
    }
    for (int32_t k = 0; k < n; k++) order[k] = cm[n - 1 - k];
    free(deg);
    free(numbered);
    free(cm);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Greedy multi-coloring of the blocks (Section 5.1).  Blocks p != q are
 * adjacent when some a_ij != 0 with i in p and j in q.  Blocks are visited
 * in id order and each takes the smallest color that no already-colored
 * adjacent block has.  Colors are numbered 0..nc-1.
 * Outputs: block_of[n] (block id of each unknown), color[nblocks], *ncolors.
 * ---------------------------------------------------------------------- */
int orc_coloring(int32_t n, const int64_t *rp, const int32_t *ci, int32_t bs,
                 const int32_t *members, int32_t nblocks,
                 int32_t *block_of, int32_t *color, int32_t *ncolors)
{
    for (int64_t p = 0; p < n; p++) block_of[members[p]] = (int32_t)(p / bs);
    int32_t *seen = (int32_t *)malloc(((size_t)nblocks + 1) * sizeof(int32_t));
    if (!seen) return ORC_ENOMEM;
    for (int32_t c = 0; c <= nblocks; c++) seen[c] = -1;
    int32_t nc = 0;
    for (int32_t b = 0; b < nblocks; b++) {
        int64_t first = (int64_t)b * bs, last = first + bs;
        if (last > n) last = n;
        for (int64_t t = first; t < last; t++) {
            int32_t u = members[t];
            for (int64_t p = rp[u]; p < rp[u + 1]; p++) {
                int32_t other = block_of[ci[p]];
                if (other < b) seen[color[other]] = b;   /* colored neighbour */
            }
        }
        int32_t c = 0;
        while (seen[c] == b) c++;
        color[b] = c;
        if (c + 1 > nc) nc = c + 1;
    }
    free(seen);
    *ncolors = nc;
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Padding, BMC numbering and the HBMC secondary reordering.
 *
 * BMC numbering (Section 4.1): colors in order; inside a color its blocks in
 * ascending id; inside a block its members in insertion order.  Each color's
 * block count is padded to a multiple of w with all-dummy blocks at its end,
 * and the short last block is completed with dummies (Section 4.3), so the
 * color segment has a multiple of b_s*w unknowns.
 *
 * Secondary reordering (Section 4.2, eq. "simd-block"): the level-1 block k'
 * of color c is made of the w consecutive BMC blocks k'w .. k'w+w-1 of that
 * color.  Inside it, the first unknown of each of the w blocks is taken, then
 * the second, and so on, b_s times.  For the unknown at offset u from the
 * color start S_c in BMC numbering, with level-1 block k' = u / (b_s w), BMC
 * block m = (u mod b_s w) / b_s inside it, and position j = u mod b_s inside
 * that block, the new index is  S_c + k' b_s w + j w + m.
 *
 * Outputs: perm[n] (original index -> HBMC index), color_start[nc+1] (first
 * HBMC index of each color; color_start[nc] = n_pad), *n_pad.
 * ---------------------------------------------------------------------- */
int orc_hbmc_perm(int32_t n, int32_t bs, int32_t w, const int32_t *members,
                  int32_t nblocks, const int32_t *color, int32_t ncolors,
                  int32_t *perm, int64_t *color_start, int64_t *n_pad)
{
    if (w < 1) return ORC_EINVAL;
    int64_t *count = (int64_t *)calloc((size_t)ncolors, sizeof(int64_t));
    int64_t *rank = (int64_t *)calloc((size_t)ncolors, sizeof(int64_t));
    if (!count || !rank) { free(count); free(rank); return ORC_ENOMEM; }
    for (int32_t b = 0; b < nblocks; b++) count[color[b]]++;
    color_start[0] = 0;
    for (int32_t c = 0; c < ncolors; c++) {
        int64_t padded_blocks = (count[c] + w - 1) / w * w;
        color_start[c + 1] = color_start[c] + padded_blocks * bs;
    }
    *n_pad = color_start[ncolors];
    for (int32_t b = 0; b < nblocks; b++) {
        int32_t c = color[b];
        int64_t q = rank[c]++;                       /* rank of b in color c */
        for (int32_t j = 0; j < bs; j++) {
            int64_t t = (int64_t)b * bs + j;
            if (t >= n) break;                       /* dummy tail */
            int64_t u = q * bs + j;                  /* BMC offset in color */
            int64_t kprime = u / ((int64_t)bs * w);
            int64_t m = (u % ((int64_t)bs * w)) / bs;
            int64_t jj = u % bs;
            perm[members[t]] = (int32_t)(color_start[c] + kprime * bs * w + jj * w + m);
        }
    }
    free(count);
    free(rank);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Reordered system (Section 3, eq. "AB"): Abar = P A P^T on n_pad unknowns;
 * dummy unknowns get an identity row.  Output arrays have room for
 * nnz + (n_pad - n) entries; rows come out sorted by column.
 * ---------------------------------------------------------------------- */
int orc_permute(int32_t n, const int64_t *rp, const int32_t *ci, const double *v,
                const int32_t *perm, int64_t n_pad,
                int64_t *rp2, int32_t *ci2, double *v2)
{
    int32_t *iperm = (int32_t *)malloc((size_t)n_pad * sizeof(int32_t));
    if (!iperm) return ORC_ENOMEM;
    for (int64_t r = 0; r < n_pad; r++) iperm[r] = -1;
    for (int32_t i = 0; i < n; i++) iperm[perm[i]] = i;
    rp2[0] = 0;
    for (int64_t r = 0; r < n_pad; r++) {
        int32_t i = iperm[r];
        int64_t out = rp2[r];
        if (i < 0) {
            ci2[out] = (int32_t)r; v2[out] = 1.0;
            rp2[r + 1] = out + 1;
            continue;
        }
        int64_t len = rp[i + 1] - rp[i];
        for (int64_t p = 0; p < len; p++) {          /* insertion sort by new column */
            int32_t c = perm[ci[rp[i] + p]];
            double x = v[rp[i] + p];
            int64_t k = out + p;
            while (k > out && ci2[k - 1] > c) { ci2[k] = ci2[k - 1]; v2[k] = v2[k - 1]; k--; }
            ci2[k] = c; v2[k] = x;
        }
        rp2[r + 1] = out + len;
    }
    free(iperm);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * IC(0) (Section 2, eq. "ILU"; Appendix A).  The factors have the nonzero
 * pattern of the triangles of A.  Right-looking elimination with
 * overwriting, updates restricted to the pattern: for k = 0..n-1 and every
 * pair k < j <= i with (i,k), (j,k) and (i,j) in the pattern,
 *     a_ij <- a_ij - a_ik a_jk / a_kk .
 * Afterwards d = diag(a) and the strictly lower part of a is L, so that
 * M = (D + L) D^-1 (D + L^T).  shift multiplies the diagonal by (1 + shift)
 * first (shifted IC, Section 5.1).
 *
 * Outputs: d[n], fac[nnz] (a copy of the pattern; only the strictly lower
 * entries carry L).  Returns ORC_EBREAKDOWN on a pivot that is not > 0.
 * ---------------------------------------------------------------------- */
int orc_ic0(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
            double shift, double *d, double *fac)
{
    memcpy(fac, v, (size_t)rp[n] * sizeof(double));
    for (int64_t i = 0; i < n; i++) {
        int64_t pd = csr_find(rp, ci, (int32_t)i, (int32_t)i);
        if (pd < 0) return ORC_EDIAG;
        fac[pd] = fac[pd] * (1.0 + shift);
    }
    for (int64_t k = 0; k < n; k++) {
        double akk = fac[csr_find(rp, ci, (int32_t)k, (int32_t)k)];
        if (!(akk > 0.0)) return ORC_EBREAKDOWN;
        /* rows i > k with a_ik != 0 are the columns i > k of row k */
        for (int64_t p = rp[k]; p < rp[k + 1]; p++) {
            int32_t i = ci[p];
            if (i <= k) continue;
            double aik = fac[csr_find(rp, ci, i, (int32_t)k)];
            for (int64_t q = rp[k]; q < rp[k + 1]; q++) {
                int32_t j = ci[q];
                if (j <= k || j > i) continue;
                int64_t pij = csr_find(rp, ci, i, j);
                if (pij < 0) continue;                 /* outside the pattern: dropped */
                double ajk = fac[csr_find(rp, ci, j, (int32_t)k)];
                fac[pij] = fac[pij] - aik * ajk / akk;
            }
        }
    }
    for (int64_t i = 0; i < n; i++) d[i] = fac[csr_find(rp, ci, (int32_t)i, (int32_t)i)];
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Preconditioning step z = M^-1 r (Section 2, eqs. "for", "back").
 * Forward, i ascending:  y_i = (r_i - sum_{j<i} L_ij y_j) * diaginv_i.
 * Backward, i descending: z_i = y_i - diaginv_i * sum_{j>i} L_ji z_j.
 * Sums run over ascending j.  y may alias nothing; z may not alias r.
 * ---------------------------------------------------------------------- */
void orc_apply(int64_t n, const int64_t *rp, const int32_t *ci, const double *fac,
               const double *d, const double *r, double *y, double *z)
{
    for (int64_t i = 0; i < n; i++) {
        double s = r[i];
        for (int64_t p = rp[i]; p < rp[i + 1] && ci[p] < i; p++)
            s = s - fac[p] * y[ci[p]];
        y[i] = s * (1.0 / d[i]);
    }
    for (int64_t i = n - 1; i >= 0; i--) {
        double s = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            int32_t j = ci[p];
            if (j <= i) continue;
            s = s + fac[csr_find(rp, ci, j, (int32_t)i)] * z[j];
        }
        z[i] = y[i] - (1.0 / d[i]) * s;
    }
}

/* Same preconditioning step with the factor rounded to FP32 and every
 * operation of the substitutions carried out in FP32 (the FP32-storage,
 * FP32-arithmetic preconditioner); r is rounded to FP32 on entry and z is
 * widened back to FP64 on exit. */
void orc_apply_f32(int64_t n, const int64_t *rp, const int32_t *ci, const double *fac,
                   const double *d, const double *r, float *y, double *z)
{
    float *zf = (float *)malloc((size_t)n * sizeof(float));
    for (int64_t i = 0; i < n; i++) {
        float s = (float)r[i];
        for (int64_t p = rp[i]; p < rp[i + 1] && ci[p] < i; p++)
            s = s - (float)fac[p] * y[ci[p]];
        y[i] = s * (float)(1.0 / d[i]);
    }
    for (int64_t i = n - 1; i >= 0; i--) {
        float s = 0.0f;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            int32_t j = ci[p];
            if (j <= i) continue;
            s = s + (float)fac[csr_find(rp, ci, j, (int32_t)i)] * zf[j];
        }
        zf[i] = y[i] - (float)(1.0 / d[i]) * s;
    }
    for (int64_t i = 0; i < n; i++) z[i] = (double)zf[i];
    free(zf);
}

/* ------------------------------------------------------------------------
 * SOR sweep (Section 2: the GS and SOR iterations, textbook form), in place,
 * one unknown at a time in the given numbering:
 *     x_i <- (1 - omega) x_i + omega (b_i - sum_{j != i} a_ij x_j) / a_ii ,
 * with i ascending (backward == 0) or descending (backward != 0); every x_j
 * read is the current value (already updated for the unknowns visited
 * earlier in the sweep).  Sums run over the row's entries in ascending
 * column order.  omega = 1 is Gauss-Seidel; a forward sweep followed by a
 * backward sweep is one SSOR (symmetric GS) step.
 * ---------------------------------------------------------------------- */
void orc_sor_sweep(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                   const double *b, double *x, double omega, int32_t backward)
{
    for (int64_t t = 0; t < n; t++) {
        int64_t i = backward ? n - 1 - t : t;
        double s = b[i], aii = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            if (ci[p] == i) aii = v[p];
            else s = s - v[p] * x[ci[p]];
        }
        x[i] = (1.0 - omega) * x[i] + omega * (s / aii);
    }
}

/* The SSOR splitting as a "factor" for orc_apply / orc_pcg: d_i = a_ii /
 * omega and the strictly lower entries of A unchanged, so that
 * (D + L) D^-1 (D + L^T) = (2 - omega) M_SSOR with
 * M_SSOR = (D_A + omega L)(omega (2 - omega))^-1 D_A^-1 (D_A + omega L^T). */
int orc_ssor_split(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                   double omega, double *d, double *fac)
{
    if (!(omega > 0.0 && omega < 2.0)) return ORC_EINVAL;
    memcpy(fac, v, (size_t)rp[n] * sizeof(double));
    for (int64_t i = 0; i < n; i++) {
        int64_t pd = csr_find(rp, ci, (int32_t)i, (int32_t)i);
        if (pd < 0) return ORC_EDIAG;
        d[i] = v[pd] / omega;
    }
    return ORC_OK;
}

/* y = A x, rows in order, entries in ascending column order. */
void orc_spmv(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
              const double *x, double *y)
{
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) s = s + v[p] * x[ci[p]];
        y[i] = s;
    }
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s = s + a[i] * b[i];
    return s;
}

/* ------------------------------------------------------------------------
 * IC(0)-preconditioned CG (Section 2; convergence test of Section 5.1).
 * Textbook preconditioned CG:
 *   r = b - A x;  z = M^-1 r;  p = z;  rho = (r, z)
 *   repeat:  q = A p;  alpha = rho / (p, q);  x += alpha p;  r -= alpha q;
 *            stop if ||r|| / ||b|| < tol;
 *            z = M^-1 r;  rho' = (r, z);  p = z + (rho'/rho) p;  rho = rho'.
 * *iters counts the products A p made in the loop.  hist (maxit + 1 entries,
 * may be NULL) receives ||r|| / ||b|| before the loop and after every update.
 * With precision32 != 0 the preconditioner is orc_apply_f32.
 * Returns ORC_OK, ORC_ENOCONV (maxit reached) or ORC_EBREAKDOWN.
 * ---------------------------------------------------------------------- */
int orc_pcg(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
            const double *fac, const double *d, int32_t precision32,
            const double *b, double *x, double tol, int32_t maxit,
            int32_t *iters, double *hist)
{
    double *r = (double *)malloc((size_t)n * sizeof(double));
    double *z = (double *)malloc((size_t)n * sizeof(double));
    double *p = (double *)malloc((size_t)n * sizeof(double));
    double *q = (double *)malloc((size_t)n * sizeof(double));
    double *y = (double *)malloc((size_t)n * sizeof(double));
    float *yf = (float *)malloc((size_t)n * sizeof(float));
    int status = ORC_ENOCONV;
    *iters = 0;
    if (!r || !z || !p || !q || !y || !yf) { status = ORC_ENOMEM; goto out; }

    double bnorm = sqrt(dot(n, b, b));
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; i++) x[i] = 0.0;
        if (hist) hist[0] = 0.0;
        status = ORC_OK;
        goto out;
    }
    orc_spmv(n, rp, ci, v, x, q);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
    double res = sqrt(dot(n, r, r)) / bnorm;
    if (hist) hist[0] = res;
    if (res < tol) { status = ORC_OK; goto out; }

    if (precision32) orc_apply_f32(n, rp, ci, fac, d, r, yf, z);
    else orc_apply(n, rp, ci, fac, d, r, y, z);
    for (int64_t i = 0; i < n; i++) p[i] = z[i];
    double rho = dot(n, r, z);
    for (int32_t it = 1; it <= maxit; it++) {
        orc_spmv(n, rp, ci, v, p, q);
        double sigma = dot(n, p, q);
        if (!(sigma > 0.0) || !isfinite(sigma)) { *iters = it; status = ORC_EBREAKDOWN; goto out; }
        double alpha = rho / sigma;
        for (int64_t i = 0; i < n; i++) x[i] = x[i] + alpha * p[i];
        for (int64_t i = 0; i < n; i++) r[i] = r[i] - alpha * q[i];
        res = sqrt(dot(n, r, r)) / bnorm;
        if (hist) hist[it] = res;
        *iters = it;
        if (!isfinite(res)) { status = ORC_EBREAKDOWN; goto out; }
        if (res < tol) { status = ORC_OK; goto out; }
        if (precision32) orc_apply_f32(n, rp, ci, fac, d, r, yf, z);
        else orc_apply(n, rp, ci, fac, d, r, y, z);
        double rho_new = dot(n, r, z);
        double beta = rho_new / rho;
        for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        rho = rho_new;
    }
out:
    free(r); free(z); free(p); free(q); free(y); free(yf);
    return status;
}
