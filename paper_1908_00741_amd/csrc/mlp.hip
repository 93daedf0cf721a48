// Kernels of the warm-start network x0 = s * MLP(theta) (12 -> 256 -> 256 ->
// n, ReLU, mean squared error, Adam): dense products on the matrix cores in
// BF16 with FP32 accumulation (or FP32 throughout, for checking), with the
// bias, activation and loss folded into the products' epilogues.
//
// The products: a workgroup of four wavefronts computes a 64 x 64 tile of
// C = A B, each wavefront a 32 x 32 quarter with 32x32 MFMA instructions
// (K = 16 per instruction in BF16, 2 in FP32).  Tiles of A and B pass
// through LDS in a k-contiguous layout, whatever their layout in memory, so
// one kernel serves the three products of a linear layer: X W (forward),
// X^T dY (weight gradient) and dY W^T (input gradient, split over K into
// partial products that a second kernel adds in a fixed order).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "hbmc_internal.h"
#include "../../include/hbmc_mlp.h"

using namespace hbmc;

#define HIP_TRY(call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(HBMC_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// BF16 storage as 16-bit patterns; conversion from FP32 rounds to nearest
// even (NaN stays NaN).
__device__ inline float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }
__device__ inline uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40);   // quiet NaN
    return uint16_t((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

template <typename T> __device__ inline float ld(const T *p, int64_t i);
template <> __device__ inline float ld<uint16_t>(const uint16_t *p, int64_t i) { return bf2f(p[i]); }
template <> __device__ inline float ld<float>(const float *p, int64_t i) { return p[i]; }
template <typename T> __device__ inline T cvt(float v);
template <> __device__ inline uint16_t cvt<uint16_t>(float v) { return f2bf(v); }
template <> __device__ inline float cvt<float>(float v) { return v; }

constexpr int BM = 64, BN = 64, KT = 64, LDK = KT + 8;   // LDS rows padded by 16 bytes
constexpr int kThreads = 256;

enum { EPI_STORE = 0, EPI_BIAS_ACT = 1, EPI_MSE = 2, EPI_ADAM = 3 };

struct Epi {
    // EPI_STORE: C[z * zstride + i * ldc + j] = acc (FP32)
    float *C;
    int64_t ldc, zstride;
    // EPI_BIAS_ACT: Y[i * ldc + j] = act(acc + bias[j]) in the compute type,
    // and Yf in FP32 when not null
    const float *bias;
    int relu;
    void *Y;
    float *Yf;
    // EPI_MSE: y = acc + bias[j], d = y - T[i * ldc + j]; dY = scale * d in
    // the compute type; loss_part[tile] = sum d^2; dbias_part[row tile][j] =
    // sum over the tile's rows of scale * d
    const void *T;
    float scale;
    float *loss_part, *dbias_part;
    // EPI_ADAM: acc is the gradient of parameter e = i * ldc + j of
    // (aw, am, av, awc); one Adam update of it (adam_one), nothing stored
    float *aw, *am, *av;
    void *awc;
    float lr, b1, b2, eps, c1, c2;
};

// One Adam update of parameter e with gradient g: moments m, v, master
// weight w, and (when wc is not null) its compute-type copy.  c1 and c2 are
// the bias corrections 1 / (1 - beta1^t) and 1 / (1 - beta2^t).  The one
// definition serves the stand-alone update and the product epilogue, so the
// two give the same bits.
__device__ inline void adam_math(float g, float m, float v, float w, float lr, float b1, float b2, float eps,
                                 float c1, float c2, float &mo, float &vo, float &wo) {
    // no fused multiply-adds: whether b1 m + (1 - b1) g fuses one product or
    // the other would otherwise depend on the surrounding code
#pragma clang fp contract(off)
    mo = b1 * m + (1.0f - b1) * g;
    vo = b2 * v + (1.0f - b2) * g * g;
    wo = w - lr * (mo * c1) / (sqrtf(vo * c2) + eps);
}

template <typename T>
__device__ inline void adam_one(int64_t e, float g, float *__restrict__ w, float *__restrict__ m,
                                float *__restrict__ v, T *__restrict__ wc, float lr, float b1, float b2, float eps,
                                float c1, float c2) {
    float mo, vo, wo;
    adam_math(g, m[e], v[e], w[e], lr, b1, b2, eps, c1, c2, mo, vo, wo);
    m[e] = mo;
    v[e] = vo;
    w[e] = wo;
    if (wc) wc[e] = cvt<T>(wo);
}

// Column of k in LDS row `row`.  BF16 rows hold eight 16-byte chunks of 8 k;
// chunk c sits at c ^ ((row / 16) % 4).  Staging an m- or n-contiguous
// operand writes, in one instruction, one k of rows 8 apart (rows 8 j + i,
// j = 0..7), which the 144-byte row pitch alone puts on two bank groups;
// the XOR spreads them over the 64 banks.  Sixteen consecutive rows share
// one permutation, so the MFMA's 16-byte reads of 16 consecutive rows stay
// as they were.  FP32 rows are not permuted.
template <typename T> __device__ inline int swz(int row, int k);
template <> __device__ inline int swz<uint16_t>(int row, int k) { return (((k >> 3) ^ ((row >> 4) & 3)) << 3) | (k & 7); }
template <> __device__ inline int swz<float>(int, int k) { return k; }

// The MFMA step for one K slice of KT held in LDS: acc += A[32 rows of the
// wavefront][KT] * B[KT][32 columns of the wavefront].  A fragment is 8
// consecutive k of one row (BF16) or 1 (FP32); the instruction pairs the
// same k positions of A and B, so the order of k inside a slice is free.
template <typename T>
__device__ inline void mma_slice(f32x16 &acc, const T (*sA)[LDK], const T (*sB)[LDK], int ra, int cb, int l);
template <>
__device__ inline void mma_slice<uint16_t>(f32x16 &acc, const uint16_t (*sA)[LDK], const uint16_t (*sB)[LDK],
                                           int ra, int cb, int l) {
#pragma unroll
    for (int kk = 0; kk < KT; kk += 16) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&sA[ra][swz<uint16_t>(ra, kk + 8 * (l >> 5))]);
        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&sB[cb][swz<uint16_t>(cb, kk + 8 * (l >> 5))]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
}
template <>
__device__ inline void mma_slice<float>(f32x16 &acc, const float (*sA)[LDK], const float (*sB)[LDK], int ra,
                                        int cb, int l) {
#pragma unroll
    for (int kk = 0; kk < KT; kk += 2) {
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(sA[ra][kk + (l >> 5)], sB[cb][kk + (l >> 5)], acc, 0, 0, 0);
    }
}

// One K slice of a BF16 tile pair staged with 16-byte loads, two per thread
// and operand (BM x KT and BN x KT values are 2 x 256 x 8; half h = 0, 1
// covers 32 of the 64 rows in memory): the caller guarantees whole tiles
// (M, N multiples of 64, the slice inside K) and 16-byte aligned rows.
// vec_load_* fetch a slice into registers (issued a slice ahead, so that
// the loads overlap the MFMA work); vec_store puts it into LDS:
// k-contiguous rows as they are, m- or n-contiguous rows transposed on the
// way.
template <int LAYOUT>
__device__ inline uint4 vec_load_a(const uint16_t *__restrict__ A, int64_t lda, int m0, int k0, int tid, int h) {
    const int row = (tid >> 3) + 32 * h, col = (tid & 7) * 8;
    if (LAYOUT == MLP_TN)   // A stored [K][M]: a row holds 64 m
        return *reinterpret_cast<const uint4 *>(A + int64_t(k0 + row) * lda + m0 + col);
    // A stored [M][K]: a row holds the slice's 64 k
    return *reinterpret_cast<const uint4 *>(A + int64_t(m0 + row) * lda + k0 + col);
}

template <int LAYOUT>
__device__ inline uint4 vec_load_b(const uint16_t *__restrict__ B, int64_t ldb, int n0, int k0, int tid, int h) {
    const int row = (tid >> 3) + 32 * h, col = (tid & 7) * 8;
    if (LAYOUT == MLP_NT)   // B stored [N][K]
        return *reinterpret_cast<const uint4 *>(B + int64_t(n0 + row) * ldb + k0 + col);
    // B stored [K][N]: a row holds 64 n
    return *reinterpret_cast<const uint4 *>(B + int64_t(k0 + row) * ldb + n0 + col);
}

// Value i (0..7) of the eight BF16 values held in v, taken with shifts so
// that v stays in registers.
__device__ inline uint16_t half_of(uint4 v, int i) {
    const uint32_t w = i < 2 ? v.x : i < 4 ? v.y : i < 6 ? v.z : v.w;
    return uint16_t(w >> (16 * (i & 1)));
}

template <bool TRANSPOSED>
__device__ inline void vec_store(uint4 v, uint16_t (*s)[LDK], int tid, int h) {
    const int row = (tid >> 3) + 32 * h, col = (tid & 7) * 8;   // as loaded
    if (TRANSPOSED) {   // row is a k; col the first of eight m (or n)
#pragma unroll
        for (int i = 0; i < 8; ++i) s[col + i][swz<uint16_t>(col + i, row)] = half_of(v, i);
    } else {            // row is an m (or n); col the first of eight k
        *reinterpret_cast<uint4 *>(&s[row][swz<uint16_t>(row, col)]) = v;
    }
}

// Output tile (mt, nt) and K range z of a workgroup in a one-dimensional
// grid of Mt * Nt * nsplit.  Workgroups go to the eight XCDs in turn (g % 8),
// each with its own L2; the remap hands XCD x a contiguous range of tile
// numbers t, which run m fastest, then n, then z, so the row tiles that
// share a column block of B (and, under a K split, all tiles of one z) run
// side by side on one XCD and read that block from HBM once.
__device__ inline void tile_of(int Mt, int Nt, int &mt, int &nt, int &z) {
    const int64_t G = gridDim.x, g = blockIdx.x;
    const int64_t per = G / 8, rem = G % 8, x = g % 8;
    const int64_t t = x * per + (x < rem ? x : rem) + g / 8;
    mt = int(t % Mt);
    nt = int((t / Mt) % Nt);
    z = int(t / (int64_t(Mt) * Nt));
}

// C = A B for logical A [M][K] and B [K][N].  LAYOUT: MLP_NN (A stored
// [M][K], B stored [K][N]), MLP_TN (A stored [K][M]), MLP_NT (B stored
// [N][K]).  z: K split (k in [z * kchunk, (z + 1) * kchunk)).
// VEC: BF16 whole tiles with aligned rows, staged with 16-byte loads.
template <typename T, int LAYOUT, int EPI, bool VEC>
__global__ void __launch_bounds__(kThreads) k_gemm(int M, int N, int K, const T *__restrict__ A, int64_t lda,
                                                   const T *__restrict__ B, int64_t ldb, int kchunk, Epi ep) {
    // the staging tiles of A and B; after the K loop the whole-tile loss
    // epilogue reuses the space for the FP32 output tile
    constexpr int kStage = (BM + BN) * LDK * int(sizeof(T)), kOut = BM * (BN + 4) * 4;
    __shared__ __align__(16) unsigned char smem[kStage > kOut ? kStage : kOut];
    T (*sA)[LDK] = reinterpret_cast<T (*)[LDK]>(smem);
    T (*sB)[LDK] = reinterpret_cast<T (*)[LDK]>(smem + BM * LDK * sizeof(T));
    const int tid = threadIdx.x, l = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int Mt = (M + BM - 1) / BM, Nt = (N + BN - 1) / BN;
    int mt, nt, z;
    tile_of(Mt, Nt, mt, nt, z);
    const int m0 = mt * BM, n0 = nt * BN;
    const int kbeg = z * kchunk, kend = min(K, kbeg + kchunk);
    f32x16 acc = {};
    if constexpr (VEC) {
        const auto *A16 = reinterpret_cast<const uint16_t *>(A);
        const auto *B16 = reinterpret_cast<const uint16_t *>(B);
        auto *sA16 = reinterpret_cast<uint16_t (*)[LDK]>(sA);
        auto *sB16 = reinterpret_cast<uint16_t (*)[LDK]>(sB);
        uint4 ra0 = {}, ra1 = {}, rb0 = {}, rb1 = {};
        if (kbeg < kend) {
            ra0 = vec_load_a<LAYOUT>(A16, lda, m0, kbeg, tid, 0);
            ra1 = vec_load_a<LAYOUT>(A16, lda, m0, kbeg, tid, 1);
            rb0 = vec_load_b<LAYOUT>(B16, ldb, n0, kbeg, tid, 0);
            rb1 = vec_load_b<LAYOUT>(B16, ldb, n0, kbeg, tid, 1);
        }
        for (int k0 = kbeg; k0 < kend; k0 += KT) {
            vec_store<LAYOUT == MLP_TN>(ra0, sA16, tid, 0);
            vec_store<LAYOUT == MLP_TN>(ra1, sA16, tid, 1);
            vec_store<LAYOUT != MLP_NT>(rb0, sB16, tid, 0);
            vec_store<LAYOUT != MLP_NT>(rb1, sB16, tid, 1);
            __syncthreads();
            if (k0 + KT < kend) {
                ra0 = vec_load_a<LAYOUT>(A16, lda, m0, k0 + KT, tid, 0);
                ra1 = vec_load_a<LAYOUT>(A16, lda, m0, k0 + KT, tid, 1);
                rb0 = vec_load_b<LAYOUT>(B16, ldb, n0, k0 + KT, tid, 0);
                rb1 = vec_load_b<LAYOUT>(B16, ldb, n0, k0 + KT, tid, 1);
            }
            mma_slice<T>(acc, sA, sB, wm * 32 + (l & 31), wn * 32 + (l & 31), l);
            __syncthreads();
        }
    }
    for (int k0 = kbeg; !VEC && k0 < kend; k0 += KT) {
#pragma unroll
        for (int e = 0; e < BM * KT / kThreads; ++e) {
            const int idx = tid + kThreads * e;
            int m, k;
            if (LAYOUT == MLP_TN) { k = idx / BM; m = idx % BM; }   // A stored [K][M]: m contiguous
            else { m = idx / KT; k = idx % KT; }                   // A stored [M][K]: k contiguous
            const int gm = m0 + m, gk = k0 + k;
            float v = 0.0f;
            if (gm < M && gk < kend)
                v = LAYOUT == MLP_TN ? ld(A, int64_t(gk) * lda + gm) : ld(A, int64_t(gm) * lda + gk);
            sA[m][swz<T>(m, k)] = cvt<T>(v);
        }
#pragma unroll
        for (int e = 0; e < BN * KT / kThreads; ++e) {
            const int idx = tid + kThreads * e;
            int n, k;
            if (LAYOUT == MLP_NT) { n = idx / KT; k = idx % KT; }   // B stored [N][K]: k contiguous
            else { k = idx / BN; n = idx % BN; }                   // B stored [K][N]: n contiguous
            const int gn = n0 + n, gk = k0 + k;
            float v = 0.0f;
            if (gn < N && gk < kend)
                v = LAYOUT == MLP_NT ? ld(B, int64_t(gn) * ldb + gk) : ld(B, int64_t(gk) * ldb + gn);
            sB[n][swz<T>(n, k)] = cvt<T>(v);
        }
        __syncthreads();
        mma_slice<T>(acc, sA, sB, wm * 32 + (l & 31), wn * 32 + (l & 31), l);
        __syncthreads();
    }
    // element r of the accumulator: row 8 (r / 4) + 4 (l / 32) + r % 4 and
    // column l % 32 of the wavefront's 32 x 32 quarter
    const int j = n0 + wn * 32 + (l & 31);
    if (EPI == EPI_STORE) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = m0 + wm * 32 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
            if (i < M && j < N) ep.C[z * ep.zstride + int64_t(i) * ep.ldc + j] = acc[r];
        }
    } else if (EPI == EPI_ADAM) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = m0 + wm * 32 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
            if (i < M && j < N)
                adam_one<T>(int64_t(i) * ep.ldc + j, acc[r], ep.aw, ep.am, ep.av, static_cast<T *>(ep.awc), ep.lr,
                            ep.b1, ep.b2, ep.eps, ep.c1, ep.c2);
        }
    } else if (EPI == EPI_BIAS_ACT) {
        const float bj = ep.bias && j < N ? ep.bias[j] : 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = m0 + wm * 32 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
            if (i < M && j < N) {
                float y = acc[r] + bj;
                if (ep.relu) y = fmaxf(y, 0.0f);
                static_cast<T *>(ep.Y)[int64_t(i) * ep.ldc + j] = cvt<T>(y);
                if (ep.Yf) ep.Yf[int64_t(i) * ep.ldc + j] = y;
            }
        }
    } else if (VEC) {   // EPI_MSE, whole BF16 tiles
        // The FP32 tile goes through LDS so that a thread owns runs of four
        // columns (8-byte loads of T, 8-byte stores of dY): rows rg and
        // rg + 32, columns c4..c4+3 and 32+c4..32+c4+3.
        __shared__ float sCol[kThreads / 64][BN];
        __shared__ float sLoss[kThreads / 64];
        float (*sC)[BN + 4] = reinterpret_cast<float (*)[BN + 4]>(smem);
#pragma unroll
        for (int r = 0; r < 16; ++r) sC[wm * 32 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3)][wn * 32 + (l & 31)] = acc[r];
        __syncthreads();
        const int c4 = (tid & 7) * 4, rg = tid >> 3;
        const auto *T16 = static_cast<const uint16_t *>(ep.T);
        auto *Y16 = static_cast<uint16_t *>(ep.Y);
        float bj[8], col[8], loss = 0.0f;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            bj[k] = ep.bias ? ep.bias[n0 + 32 * (k >> 2) + c4 + (k & 3)] : 0.0f;
            col[k] = 0.0f;
        }
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int ii = rg + 32 * p;
            const int64_t row = int64_t(m0 + ii) * ep.ldc + n0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int jj = 32 * h + c4;
                const float4 a = *reinterpret_cast<const float4 *>(&sC[ii][jj]);
                const uint2 t = *reinterpret_cast<const uint2 *>(T16 + row + jj);
                const float av[4] = {a.x, a.y, a.z, a.w};
                const uint32_t tw[2] = {t.x, t.y};
                uint32_t out[2] = {0u, 0u};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float d = av[q] + bj[4 * h + q] - bf2f(uint16_t(tw[q >> 1] >> (16 * (q & 1))));
                    const float g = ep.scale * d;
                    out[q >> 1] |= uint32_t(f2bf(g)) << (16 * (q & 1));
                    col[4 * h + q] += g;
                    loss += d * d;
                }
                *reinterpret_cast<uint2 *>(Y16 + row + jj) = make_uint2(out[0], out[1]);
            }
        }
        // column partials over the wavefront's eight row groups (lane bits
        // 3..5), then over the four wavefronts in order
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            col[k] += __shfl_xor(col[k], 8, 64);
            col[k] += __shfl_xor(col[k], 16, 64);
            col[k] += __shfl_xor(col[k], 32, 64);
        }
        if (l < 8) {
#pragma unroll
            for (int k = 0; k < 8; ++k) sCol[wave][32 * (k >> 2) + c4 + (k & 3)] = col[k];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
        if (l == 0) sLoss[wave] = loss;
        __syncthreads();
        if (tid < BN) ep.dbias_part[int64_t(mt) * N + n0 + tid] = (sCol[0][tid] + sCol[1][tid]) + (sCol[2][tid] + sCol[3][tid]);
        if (tid == 0) ep.loss_part[int64_t(mt) * Nt + nt] = (sLoss[0] + sLoss[1]) + (sLoss[2] + sLoss[3]);
    } else {   // EPI_MSE
        __shared__ float sCol[2][BN];
        __shared__ float sLoss[kThreads / 64];
        const float bj = ep.bias && j < N ? ep.bias[j] : 0.0f;
        float col = 0.0f, loss = 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = m0 + wm * 32 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
            if (i < M && j < N) {
                const int64_t e = int64_t(i) * ep.ldc + j;
                const float d = acc[r] + bj - ld(static_cast<const T *>(ep.T), e);
                const float g = ep.scale * d;
                static_cast<T *>(ep.Y)[e] = cvt<T>(g);
                col += g;
                loss += d * d;
            }
        }
        col += __shfl_xor(col, 32, 64);              // the two lanes of one column
        if (l < 32) sCol[wm][wn * 32 + l] = col;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
        if (l == 0) sLoss[wave] = loss;
        __syncthreads();
        if (tid < BN && n0 + tid < N) ep.dbias_part[int64_t(mt) * N + n0 + tid] = sCol[0][tid] + sCol[1][tid];
        if (tid == 0)
            ep.loss_part[int64_t(mt) * Nt + nt] = (sLoss[0] + sLoss[1]) + (sLoss[2] + sLoss[3]);
    }
}

// out[j] = sum over i < R of src[i * ld + j], i in order; the loads of
// sixteen rows are issued before they are added (few columns, many rows:
// one load latency per sixteen rows rather than per row)
__global__ void k_sum_rows(int64_t R, int64_t N, const float *__restrict__ src, int64_t ld,
                           float *__restrict__ out) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= N) return;
    constexpr int kRows = 16;
    float s = 0.0f;
    int64_t i = 0;
    for (; i + kRows <= R; i += kRows) {
        float v[kRows];
#pragma unroll
        for (int k = 0; k < kRows; ++k) v[k] = src[(i + k) * ld + j];
#pragma unroll
        for (int k = 0; k < kRows; ++k) s += v[k];
    }
    for (; i < R; ++i) s += src[i * ld + j];
    out[j] = s;
}

// *out = sum of src[0 .. n) by one workgroup, in a fixed order
__global__ void __launch_bounds__(1024) k_total(int64_t n, const float *__restrict__ src, float *__restrict__ out) {
    __shared__ double sh[16];
    double acc = 0.0;
    int64_t i = threadIdx.x;
    // sixteen loads in flight per thread, added in the order of i
    for (; i + 15 * 1024 < n; i += 16 * 1024) {
        float v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = src[i + k * 1024];
#pragma unroll
        for (int k = 0; k < 16; ++k) acc += v[k];
    }
    for (; i < n; i += 1024) acc += src[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < 16; ++k) t += sh[k];
        *out = float(t);
    }
}

// dz = dh * (h > 0): dz in the compute type and, when dzf is set, FP32
template <typename T>
__global__ void k_relu_bwd(int64_t n, const float *__restrict__ dh, const T *__restrict__ h, T *__restrict__ dz,
                           float *__restrict__ dzf) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = ld(h, i) > 0.0f ? dh[i] : 0.0f;
    dz[i] = cvt<T>(v);
    if (dzf) dzf[i] = v;
}

// Adam with bias corrections c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t);
// the compute-type copy of the updated weights is written too
template <typename T>
__global__ void k_adam(int64_t n, float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, T *__restrict__ wc, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) adam_one<T>(i, g[i], w, m, v, wc, lr, b1, b2, eps, c1, c2);
}

template <typename T>
__global__ void k_cast_f32(int64_t n, const float *__restrict__ src, T *__restrict__ dst) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = cvt<T>(src[i]);
}

template <typename T>
__global__ void k_cast_f64(int64_t n, const double *__restrict__ src, double scale, T *__restrict__ dst) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = cvt<T>(float(src[i] * scale));
}

__global__ void k_to_f64(int64_t n, const float *__restrict__ src, double scale, double *__restrict__ dst) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = double(src[i]) * scale;
}

// b at the N^3 cell centres (index x + N y + N^2 z) for theta = (positions
// s_q along the four body diagonals, widths, amplitudes)
__global__ void k_gaussian_rhs(int N, double s0, double s1, double s2, double s3, double w0, double w1,
                               double w2, double w3, double a0, double a1, double a2, double a3,
                               double *__restrict__ b) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = int64_t(N) * N * N;
    if (idx >= n) return;
    const double h = 1.0 / N;
    const double x = (double(idx % N) + 0.5) * h;
    const double y = (double((idx / N) % N) + 0.5) * h;
    const double z = (double(idx / (int64_t(N) * N)) + 0.5) * h;
    // diagonal q starts at o_q and runs along d_q
    const double ox[4] = {0, 1, 0, 0}, oy[4] = {0, 0, 1, 0}, oz[4] = {0, 0, 0, 1};
    const double dx[4] = {1, -1, 1, 1}, dy[4] = {1, 1, -1, 1}, dz[4] = {1, 1, 1, -1};
    const double s[4] = {s0, s1, s2, s3}, w[4] = {w0, w1, w2, w3}, a[4] = {a0, a1, a2, a3};
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double cx = ox[q] + s[q] * dx[q], cy = oy[q] + s[q] * dy[q], cz = oz[q] + s[q] * dz[q];
        const double r2 = (x - cx) * (x - cx) + (y - cy) * (y - cy) + (z - cz) * (z - cz);
        v += a[q] * exp(-r2 / (2.0 * w[q] * w[q]));
    }
    b[idx] = v;
}

// Y = act(X W + b) for a few rows (M <= MM): a matrix-vector product bound
// by reading W once.  A workgroup covers 512 columns, each lane 8 adjacent
// ones (one 16-byte load of W per k in BF16); its four wavefronts take a
// quarter of k each and meet in LDS.
template <typename T> struct Vec8;
template <> struct Vec8<uint16_t> {
    uint16_t v[8];
    __device__ void load(const uint16_t *p) {
        const uint4 u = *reinterpret_cast<const uint4 *>(p);
        v[0] = u.x & 0xffff; v[1] = u.x >> 16; v[2] = u.y & 0xffff; v[3] = u.y >> 16;
        v[4] = u.z & 0xffff; v[5] = u.z >> 16; v[6] = u.w & 0xffff; v[7] = u.w >> 16;
    }
    __device__ float at(int c) const { return bf2f(v[c]); }
};
template <> struct Vec8<float> {
    float v[8];
    __device__ void load(const float *p) {
        const float4 a = *reinterpret_cast<const float4 *>(p), b = *reinterpret_cast<const float4 *>(p + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    }
    __device__ float at(int c) const { return v[c]; }
};

constexpr int GV_COLS = 512;   // columns per workgroup
template <typename T, int MM>
__global__ void __launch_bounds__(kThreads) k_gemv(int M, int N, int K, const T *__restrict__ X,
                                                   const T *__restrict__ W, const float *__restrict__ bias,
                                                   int relu, T *__restrict__ Y, float *__restrict__ Yf) {
    __shared__ float sred[kThreads / 64][MM][GV_COLS];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j0 = blockIdx.x * GV_COLS + lane * 8;
    const int kq = (K + 3) / 4, kb = wave * kq, ke = min(K, kb + kq);
    const bool vec = (N % 8 == 0) && (j0 + 8 <= N);
    float acc[MM][8];
#pragma unroll
    for (int m = 0; m < MM; ++m)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[m][c] = 0.0f;
#pragma unroll 4
    for (int k = kb; k < ke; ++k) {
        Vec8<T> w;
        if (vec) w.load(W + int64_t(k) * N + j0);
        else
#pragma unroll
            for (int c = 0; c < 8; ++c) w.v[c] = j0 + c < N ? W[int64_t(k) * N + j0 + c] : T(0);
#pragma unroll
        for (int m = 0; m < MM; ++m) {
            const float xm = m < M ? ld(X, int64_t(m) * K + k) : 0.0f;
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[m][c] += xm * w.at(c);
        }
    }
#pragma unroll
    for (int m = 0; m < MM; ++m)
#pragma unroll
        for (int c = 0; c < 8; ++c) sred[wave][m][lane * 8 + c] = acc[m][c];
    __syncthreads();
    // thread t finishes columns t and t + 256 of the workgroup for every row
    for (int cc = threadIdx.x; cc < GV_COLS; cc += kThreads) {
        const int j = blockIdx.x * GV_COLS + cc;
        if (j >= N) continue;
        const float bj = bias ? bias[j] : 0.0f;
        for (int m = 0; m < M; ++m) {
            float y = (sred[0][m][cc] + sred[1][m][cc]) + (sred[2][m][cc] + sred[3][m][cc]) + bj;
            if (relu) y = fmaxf(y, 0.0f);
            Y[int64_t(m) * N + j] = cvt<T>(y);
            if (Yf) Yf[int64_t(m) * N + j] = y;
        }
    }
}

// T[m][i] = scale * sum over q < 4 of amp[m][q] * G[idx[m][q]][i]
template <typename T>
__global__ void k_combine(int M, int64_t n, const T *__restrict__ G, const int32_t *__restrict__ idx,
                          const float *__restrict__ amp, float scale, T *__restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    if (i >= n || m >= M) return;
    float v = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) v += amp[m * 4 + q] * ld(G, int64_t(idx[m * 4 + q]) * n + i);
    out[int64_t(m) * n + i] = cvt<T>(scale * v);
}

inline unsigned blocks_for(int64_t n, int t = 256) { return unsigned((n + t - 1) / t); }

template <typename T, int EPI, bool VEC>
int launch_layout(int layout, dim3 grid, hipStream_t s, int M, int N, int K, const T *a, int64_t lda,
                  const T *b, int64_t ldb, int kchunk, const Epi &ep) {
    switch (layout) {
        case MLP_NN: hipLaunchKernelGGL((k_gemm<T, MLP_NN, EPI, VEC>), grid, dim3(kThreads), 0, s, M, N, K, a, lda, b, ldb, kchunk, ep); break;
        case MLP_TN: hipLaunchKernelGGL((k_gemm<T, MLP_TN, EPI, VEC>), grid, dim3(kThreads), 0, s, M, N, K, a, lda, b, ldb, kchunk, ep); break;
        case MLP_NT: hipLaunchKernelGGL((k_gemm<T, MLP_NT, EPI, VEC>), grid, dim3(kThreads), 0, s, M, N, K, a, lda, b, ldb, kchunk, ep); break;
        default: return fail(HBMC_EINVAL, "unknown layout %d", layout);
    }
    return HBMC_OK;
}

template <typename T, int EPI>
int launch_gemm(int layout, int M, int N, int K, const void *A, int64_t lda, const void *B, int64_t ldb,
                int nsplit, const Epi &ep, hipStream_t s) {
    const int kchunk = ((K + nsplit - 1) / nsplit + KT - 1) / KT * KT;
    const dim3 grid(unsigned(int64_t((N + BN - 1) / BN) * ((M + BM - 1) / BM) * nsplit));
    const T *a = static_cast<const T *>(A);
    const T *b = static_cast<const T *>(B);
    // the 16-byte staging: BF16, whole tiles, every K slice whole, rows and
    // bases 16-byte aligned
    bool vec = false;
    if constexpr (sizeof(T) == 2)
        vec = M % BM == 0 && N % BN == 0 && K % KT == 0 && lda % 8 == 0 &&
                     ldb % 8 == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(B) % 16 == 0;
    if (EPI == EPI_MSE)   // the whole-tile loss epilogue: 8-byte runs of T and dY
        vec = vec && ep.ldc % 4 == 0 && reinterpret_cast<uintptr_t>(ep.T) % 8 == 0 &&
              reinterpret_cast<uintptr_t>(ep.Y) % 8 == 0;
    int st;
    if constexpr (sizeof(T) == 2)
        st = vec ? launch_layout<T, EPI, true>(layout, grid, s, M, N, K, a, lda, b, ldb, kchunk, ep)
                 : launch_layout<T, EPI, false>(layout, grid, s, M, N, K, a, lda, b, ldb, kchunk, ep);
    else
        st = launch_layout<T, EPI, false>(layout, grid, s, M, N, K, a, lda, b, ldb, kchunk, ep);
    if (st) return st;
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

template <int EPI>
int gemm_dtype(int dtype, int layout, int M, int N, int K, const void *A, int64_t lda, const void *B,
               int64_t ldb, int nsplit, const Epi &ep, hipStream_t s) {
    if (dtype == MLP_BF16) return launch_gemm<uint16_t, EPI>(layout, M, N, K, A, lda, B, ldb, nsplit, ep, s);
    if (dtype == MLP_F32) return launch_gemm<float, EPI>(layout, M, N, K, A, lda, B, ldb, nsplit, ep, s);
    return fail(HBMC_EINVAL, "unknown dtype %d", dtype);
}

// Adam's bias corrections for step t (1-based): 1 / (1 - beta^t), in FP64
// and rounded once.
void bias_corrections(float beta1, float beta2, int step, float &c1, float &c2) {
    c1 = float(1.0 / (1.0 - std::pow(double(beta1), step)));
    c2 = float(1.0 / (1.0 - std::pow(double(beta2), step)));
}

int check_dims(int M, int N, int K, int nsplit) {
    if (M < 1 || N < 1 || K < 1) return fail(HBMC_EINVAL, "bad sizes M=%d N=%d K=%d", M, N, K);
    if (nsplit < 1 || nsplit > 65535) return fail(HBMC_EINVAL, "bad split %d", nsplit);
    // one-dimensional grid: fewer than 2^32 threads
    if (int64_t((N + BN - 1) / BN) * ((M + BM - 1) / BM) * nsplit * kThreads > int64_t(UINT32_MAX))
        return fail(HBMC_EINVAL, "grid too large");
    return HBMC_OK;
}

}  // namespace

extern "C" int mlp_gemm(int32_t dtype, int32_t layout, int32_t M, int32_t N, int32_t K, const void *A,
                        int64_t lda, const void *B, int64_t ldb, float *C, int64_t ldc, int32_t nsplit,
                        void *stream) {
    if (!A || !B || !C) return fail(HBMC_EINVAL, "null argument");
    int st = check_dims(M, N, K, nsplit);
    if (st) return st;
    if (layout < MLP_NN || layout > MLP_NT) return fail(HBMC_EINVAL, "unknown layout %d", layout);
    const int64_t wa = layout == MLP_TN ? M : K, wb = layout == MLP_NT ? K : N;
    if (lda < wa || ldb < wb || ldc < N)
        return fail(HBMC_EINVAL, "leading dimension below the row width (lda %lld of %lld, ldb %lld of %lld, ldc %lld of %d)",
                    (long long)lda, (long long)wa, (long long)ldb, (long long)wb, (long long)ldc, N);
    Epi ep{};
    ep.C = C;
    ep.ldc = ldc;
    ep.zstride = int64_t(M) * ldc;
    return gemm_dtype<EPI_STORE>(dtype, layout, M, N, K, A, lda, B, ldb, nsplit, ep, static_cast<hipStream_t>(stream));
}

extern "C" int mlp_linear_fwd(int32_t dtype, int32_t M, int32_t N, int32_t K, const void *X, const void *W,
                              const float *bias, int32_t relu, void *Y, float *Yf, void *stream) {
    if (!X || !W || !Y) return fail(HBMC_EINVAL, "null argument");
    int st = check_dims(M, N, K, 1);
    if (st) return st;
    auto s = static_cast<hipStream_t>(stream);
    if (M <= 4) {   // a few rows: bound by reading W once
        const dim3 grid(unsigned((N + GV_COLS - 1) / GV_COLS));
        if (dtype == MLP_BF16)
            hipLaunchKernelGGL((k_gemv<uint16_t, 4>), grid, dim3(kThreads), 0, s, M, N, K,
                               static_cast<const uint16_t *>(X), static_cast<const uint16_t *>(W), bias, relu,
                               static_cast<uint16_t *>(Y), Yf);
        else if (dtype == MLP_F32)
            hipLaunchKernelGGL((k_gemv<float, 4>), grid, dim3(kThreads), 0, s, M, N, K, static_cast<const float *>(X),
                               static_cast<const float *>(W), bias, relu, static_cast<float *>(Y), Yf);
        else return fail(HBMC_EINVAL, "unknown dtype %d", dtype);
        HIP_TRY(hipGetLastError());
        return HBMC_OK;
    }
    Epi ep{};
    ep.bias = bias;
    ep.relu = relu;
    ep.Y = Y;
    ep.Yf = Yf;
    ep.ldc = N;
    return gemm_dtype<EPI_BIAS_ACT>(dtype, MLP_NN, M, N, K, X, K, W, N, 1, ep, s);
}

extern "C" int mlp_linear_fwd_mse(int32_t dtype, int32_t M, int32_t N, int32_t K, const void *X, const void *W,
                                  const float *bias, const void *T, float scale, void *dY, float *loss_part,
                                  float *dbias_part, void *stream) {
    if (!X || !W || !T || !dY || !loss_part || !dbias_part) return fail(HBMC_EINVAL, "null argument");
    int st = check_dims(M, N, K, 1);
    if (st) return st;
    Epi ep{};
    ep.bias = bias;
    ep.T = T;
    ep.scale = scale;
    ep.Y = dY;
    ep.ldc = N;
    ep.loss_part = loss_part;
    ep.dbias_part = dbias_part;
    return gemm_dtype<EPI_MSE>(dtype, MLP_NN, M, N, K, X, K, W, N, 1, ep, static_cast<hipStream_t>(stream));
}

extern "C" int mlp_mse_parts(int32_t M, int32_t N, int64_t *loss_parts, int64_t *dbias_rows) {
    if (!loss_parts || !dbias_rows || M < 1 || N < 1) return fail(HBMC_EINVAL, "bad argument");
    *loss_parts = int64_t((M + BM - 1) / BM) * ((N + BN - 1) / BN);
    *dbias_rows = (M + BM - 1) / BM;
    return HBMC_OK;
}

extern "C" int mlp_sum_rows(int64_t R, int64_t N, const float *src, int64_t ld, float *out, void *stream) {
    if (!src || !out || R < 1 || N < 1 || ld < N) return fail(HBMC_EINVAL, "bad argument");
    hipLaunchKernelGGL(k_sum_rows, dim3(blocks_for(N)), dim3(256), 0, static_cast<hipStream_t>(stream), R, N, src,
                       ld, out);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int mlp_relu_bwd(int32_t dtype, int64_t n, const float *dh, const void *h, void *dz, float *dzf,
                            void *stream) {
    if (!dh || !h || !dz || n < 1) return fail(HBMC_EINVAL, "bad argument");
    auto s = static_cast<hipStream_t>(stream);
    if (dtype == MLP_BF16)
        hipLaunchKernelGGL(k_relu_bwd<uint16_t>, dim3(blocks_for(n)), dim3(256), 0, s, n, dh,
                           static_cast<const uint16_t *>(h), static_cast<uint16_t *>(dz), dzf);
    else if (dtype == MLP_F32)
        hipLaunchKernelGGL(k_relu_bwd<float>, dim3(blocks_for(n)), dim3(256), 0, s, n, dh,
                           static_cast<const float *>(h), static_cast<float *>(dz), dzf);
    else return fail(HBMC_EINVAL, "unknown dtype %d", dtype);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int mlp_adam(int32_t dtype, int64_t n, float *w, float *m, float *v, const float *g, void *wc,
                        float lr, float beta1, float beta2, float eps, int32_t step, void *stream) {
    if (!w || !m || !v || !g || n < 1 || step < 1) return fail(HBMC_EINVAL, "bad argument");
    float c1, c2;
    bias_corrections(beta1, beta2, step, c1, c2);
    auto s = static_cast<hipStream_t>(stream);
    if (dtype == MLP_BF16)
        hipLaunchKernelGGL(k_adam<uint16_t>, dim3(blocks_for(n)), dim3(256), 0, s, n, w, m, v, g,
                           static_cast<uint16_t *>(wc), lr, beta1, beta2, eps, c1, c2);
    else if (dtype == MLP_F32)
        hipLaunchKernelGGL(k_adam<float>, dim3(blocks_for(n)), dim3(256), 0, s, n, w, m, v, g,
                           static_cast<float *>(wc), lr, beta1, beta2, eps, c1, c2);
    else return fail(HBMC_EINVAL, "unknown dtype %d", dtype);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int mlp_cast(int32_t dtype, int64_t n, const float *src, void *dst, void *stream) {
    if (!src || !dst || n < 1) return fail(HBMC_EINVAL, "bad argument");
    auto s = static_cast<hipStream_t>(stream);
    if (dtype == MLP_BF16)
        hipLaunchKernelGGL(k_cast_f32<uint16_t>, dim3(blocks_for(n)), dim3(256), 0, s, n, src,
                           static_cast<uint16_t *>(dst));
    else if (dtype == MLP_F32)
        hipLaunchKernelGGL(k_cast_f32<float>, dim3(blocks_for(n)), dim3(256), 0, s, n, src, static_cast<float *>(dst));
    else return fail(HBMC_EINVAL, "unknown dtype %d", dtype);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int mlp_cast_f64(int32_t dtype, int64_t n, const double *src, double scale, void *dst, void *stream) {
    if (!src || !dst || n < 1) return fail(HBMC_EINVAL, "bad argument");
    auto s = static_cast<hipStream_t>(stream);
    if (dtype == MLP_BF16)
        hipLaunchKernelGGL(k_cast_f64<uint16_t>, dim3(blocks_for(n)), dim3(256), 0, s, n, src, scale,
                           static_cast<uint16_t *>(dst));
    else if (dtype == MLP_F32)
        hipLaunchKernelGGL(k_cast_f64<float>, dim3(blocks_for(n)), dim3(256), 0, s, n, src, scale,
                           static_cast<float *>(dst));
    else return fail(HBMC_EINVAL, "unknown dtype %d", dtype);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int mlp_to_f64(int64_t n, const float *src, double scale, double *dst, void *stream) {
    if (!src || !dst || n < 1) return fail(HBMC_EINVAL, "bad argument");
    hipLaunchKernelGGL(k_to_f64, dim3(blocks_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), n, src, scale,
                       dst);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int mlp_gaussian_rhs(int32_t N, const double *theta, double *b, void *stream) {
    if (!theta || !b || N < 1) return fail(HBMC_EINVAL, "bad argument");
    const double *t = theta;
    hipLaunchKernelGGL(k_gaussian_rhs, dim3(blocks_for(int64_t(N) * N * N)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), N, t[0], t[1], t[2], t[3], t[4], t[5], t[6], t[7], t[8],
                       t[9], t[10], t[11], b);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

extern "C" int mlp_combine(int32_t dtype, int32_t M, int64_t n, const void *G, int64_t rows, const int32_t *idx,
                           const float *amp, float scale, void *T, void *stream) {
    if (!G || !idx || !amp || !T || M < 1 || M > 65535 || n < 1 || rows < 1) return fail(HBMC_EINVAL, "bad argument");
    auto s = static_cast<hipStream_t>(stream);
    const dim3 grid(blocks_for(n), unsigned(M));
    if (dtype == MLP_BF16)
        hipLaunchKernelGGL(k_combine<uint16_t>, grid, dim3(256), 0, s, M, n, static_cast<const uint16_t *>(G), idx, amp,
                           scale, static_cast<uint16_t *>(T));
    else if (dtype == MLP_F32)
        hipLaunchKernelGGL(k_combine<float>, grid, dim3(256), 0, s, M, n, static_cast<const float *>(G), idx, amp, scale,
                           static_cast<float *>(T));
    else return fail(HBMC_EINVAL, "unknown dtype %d", dtype);
    HIP_TRY(hipGetLastError());
    return HBMC_OK;
}

// ---------------------------------------------------------------------------
// The whole network: forward, backward (with the loss) and the Adam step,
// composed from the kernels above.
// ---------------------------------------------------------------------------
namespace {

struct NetWork {   // workspace carve-up for a batch of M rows
    void *h1, *h2, *dY, *dz;
    float *loss, *dbias, *part, *dh, *dzf;
    int64_t nloss, nrows;
    int split;    // K split of dY W3^T
    int xsplit;   // K split of x^T dz1 (K = batch)
};

size_t elem_size(int dtype) { return dtype == MLP_BF16 ? 2 : 4; }

size_t net_layout(int dtype, int M, int n_in, int hid, int n_out, NetWork *w, void *base) {
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const int64_t nloss = int64_t((M + BM - 1) / BM) * ((n_out + BN - 1) / BN);
    const int64_t nrows = (M + BM - 1) / BM;
    // K split of dY W3^T (K = n_out) into about 1024 workgroups over the
    // output tiles, K ranges of at least 4096: more splits only add
    // partial products to write and add up
    const int tiles = ((M + BM - 1) / BM) * ((hid + BN - 1) / BN);
    const int split = std::max(1, std::min((1024 + tiles - 1) / tiles, n_out / 4096));
    // x^T dz1 has few output tiles (n_in rows): one K slice per split, at
    // most four; its partials share the buffer of dY W3^T's
    const int xsplit = std::max(1, std::min(4, M / KT));
    const size_t part = std::max(size_t(split) * M * hid, xsplit > 1 ? size_t(xsplit) * n_in * hid : size_t(0));
    const size_t es = elem_size(dtype);
    const size_t sz[9] = {up(size_t(M) * hid * es), up(size_t(M) * hid * es), up(size_t(M) * n_out * es),
                          up(size_t(M) * hid * es), up(size_t(nloss) * 4), up(size_t(nrows) * n_out * 4),
                          up(part * 4), up(size_t(M) * hid * 4), up(size_t(M) * hid * 4)};
    size_t total = 0;
    for (size_t v : sz) total += v;
    if (w && base) {
        auto *b = static_cast<uint8_t *>(base);
        void **ptrs[9] = {&w->h1, &w->h2, &w->dY, &w->dz, reinterpret_cast<void **>(&w->loss),
                          reinterpret_cast<void **>(&w->dbias), reinterpret_cast<void **>(&w->part),
                          reinterpret_cast<void **>(&w->dh), reinterpret_cast<void **>(&w->dzf)};
        size_t a = 0;
        for (int i = 0; i < 9; ++i) { *ptrs[i] = b + a; a += sz[i]; }
        w->nloss = nloss;
        w->nrows = nrows;
        w->split = split;
        w->xsplit = xsplit;
    }
    return total;
}

int check_net(int dtype, int M, int n_in, int hid, int n_out, const void *const *W, const float *const *b) {
    if (dtype != MLP_BF16 && dtype != MLP_F32) return fail(HBMC_EINVAL, "unknown dtype %d", dtype);
    if (M < 1 || n_in < 1 || hid < 1 || n_out < 1 || M > 65535 * BM) return fail(HBMC_EINVAL, "bad sizes");
    if (!W || !b || !W[0] || !W[1] || !W[2]) return fail(HBMC_EINVAL, "null weights");
    return HBMC_OK;
}

#define MLP_TRY(call)           \
    do {                        \
        int st_ = (call);       \
        if (st_) return st_;    \
    } while (0)

}  // namespace

extern "C" int mlp_workspace_bytes(int32_t dtype, int32_t M, int32_t n_in, int32_t hidden, int32_t n_out,
                                   size_t *bytes) {
    if (!bytes || M < 1 || n_in < 1 || hidden < 1 || n_out < 1) return fail(HBMC_EINVAL, "bad argument");
    *bytes = net_layout(dtype, M, n_in, hidden, n_out, nullptr, nullptr);
    return HBMC_OK;
}

extern "C" int mlp_forward(int32_t dtype, int32_t M, int32_t n_in, int32_t hidden, int32_t n_out, const void *X,
                           const void *const *W, const float *const *b, void *Y, float *Yf, void *work,
                           size_t work_bytes, void *stream) {
    MLP_TRY(check_net(dtype, M, n_in, hidden, n_out, W, b));
    if (!X || (!Y && !Yf) || !work) return fail(HBMC_EINVAL, "null argument");
    if (work_bytes < net_layout(dtype, M, n_in, hidden, n_out, nullptr, nullptr))
        return fail(HBMC_EINVAL, "workspace too small");
    NetWork w{};
    net_layout(dtype, M, n_in, hidden, n_out, &w, work);
    // the output in the compute type goes to Y, or to the dY slot when only FP32 is wanted
    MLP_TRY(mlp_linear_fwd(dtype, M, hidden, n_in, X, W[0], b[0], 1, w.h1, nullptr, stream));
    MLP_TRY(mlp_linear_fwd(dtype, M, hidden, hidden, w.h1, W[1], b[1], 1, w.h2, nullptr, stream));
    MLP_TRY(mlp_linear_fwd(dtype, M, n_out, hidden, w.h2, W[2], b[2], 0, Y ? Y : w.dY, Yf, stream));
    return HBMC_OK;
}

namespace {

// Optimizer state of the six parameters for a training step whose output
// layer takes its Adam update in the weight-gradient product.
struct FusedAdam {
    float *const *w, *const *m, *const *v;
    void *const *wc;
    float lr, b1, b2, eps, c1, c2;
};

// Loss and gradients of the network (mlp_backward).  With fa, the gradient
// of W3 is not stored: the product h2^T dY applies Adam to W3 (master, moments
// and compute copy W[2]) in its epilogue, after dY W3^T has read W3.
int backward_impl(int dtype, int M, int n_in, int h, int n, const void *X, const void *T, const void *const *W,
                  const float *const *b, float *const *grad, float *loss, const NetWork &w, hipStream_t s,
                  const FusedAdam *fa) {
    void *stream = s;
    MLP_TRY(mlp_linear_fwd(dtype, M, h, n_in, X, W[0], b[0], 1, w.h1, nullptr, stream));
    MLP_TRY(mlp_linear_fwd(dtype, M, h, h, w.h1, W[1], b[1], 1, w.h2, nullptr, stream));
    MLP_TRY(mlp_linear_fwd_mse(dtype, M, n, h, w.h2, W[2], b[2], T, 2.0f / (float(M) * float(n)), w.dY, w.loss,
                               w.dbias, stream));
    if (loss) {
        hipLaunchKernelGGL(k_total, dim3(1), dim3(1024), 0, s, w.nloss, w.loss, loss);
        HIP_TRY(hipGetLastError());
    }
    MLP_TRY(mlp_sum_rows(w.nrows, n, w.dbias, n, grad[5], stream));                          // db3
    MLP_TRY(mlp_gemm(dtype, MLP_NT, M, h, n, w.dY, n, W[2], n, w.part, h, w.split, stream));   // dY W3^T
    MLP_TRY(mlp_sum_rows(w.split, int64_t(M) * h, w.part, int64_t(M) * h, w.dh, stream));
    if (fa) {                                                                                 // h2^T dY -> Adam
        Epi ep{};
        ep.ldc = n;
        ep.aw = fa->w[4];
        ep.am = fa->m[4];
        ep.av = fa->v[4];
        ep.awc = fa->wc[4];
        ep.lr = fa->lr;
        ep.b1 = fa->b1;
        ep.b2 = fa->b2;
        ep.eps = fa->eps;
        ep.c1 = fa->c1;
        ep.c2 = fa->c2;
        MLP_TRY(check_dims(h, n, M, 1));
        MLP_TRY(gemm_dtype<EPI_ADAM>(dtype, MLP_TN, h, n, M, w.h2, h, w.dY, n, 1, ep, s));
    } else {
        MLP_TRY(mlp_gemm(dtype, MLP_TN, h, n, M, w.h2, h, w.dY, n, grad[4], n, 1, stream));   // h2^T dY
    }
    MLP_TRY(mlp_relu_bwd(dtype, int64_t(M) * h, w.dh, w.h2, w.dz, w.dzf, stream));
    MLP_TRY(mlp_sum_rows(M, h, w.dzf, h, grad[3], stream));                                    // db2
    MLP_TRY(mlp_gemm(dtype, MLP_TN, h, h, M, w.h1, h, w.dz, h, grad[2], h, 1, stream));        // h1^T dz2
    MLP_TRY(mlp_gemm(dtype, MLP_NT, M, h, h, w.dz, h, W[1], h, w.dh, h, 1, stream));           // dz2 W2^T
    MLP_TRY(mlp_relu_bwd(dtype, int64_t(M) * h, w.dh, w.h1, w.dz, w.dzf, stream));
    MLP_TRY(mlp_sum_rows(M, h, w.dzf, h, grad[1], stream));                                    // db1
    if (w.xsplit > 1) {                                                                         // x^T dz1
        MLP_TRY(mlp_gemm(dtype, MLP_TN, n_in, h, M, X, n_in, w.dz, h, w.part, h, w.xsplit, stream));
        MLP_TRY(mlp_sum_rows(w.xsplit, int64_t(n_in) * h, w.part, int64_t(n_in) * h, grad[0], stream));
    } else {
        MLP_TRY(mlp_gemm(dtype, MLP_TN, n_in, h, M, X, n_in, w.dz, h, grad[0], h, 1, stream));
    }
    return HBMC_OK;
}

}  // namespace

extern "C" int mlp_backward(int32_t dtype, int32_t M, int32_t n_in, int32_t hidden, int32_t n_out, const void *X,
                            const void *T, const void *const *W, const float *const *b, float *const *grad,
                            float *loss, void *work, size_t work_bytes, void *stream) {
    MLP_TRY(check_net(dtype, M, n_in, hidden, n_out, W, b));
    if (!X || !T || !grad || !work) return fail(HBMC_EINVAL, "null argument");
    for (int i = 0; i < 6; ++i)
        if (!grad[i]) return fail(HBMC_EINVAL, "null gradient %d", i);
    if (work_bytes < net_layout(dtype, M, n_in, hidden, n_out, nullptr, nullptr))
        return fail(HBMC_EINVAL, "workspace too small");
    NetWork w{};
    net_layout(dtype, M, n_in, hidden, n_out, &w, work);
    return backward_impl(dtype, M, n_in, hidden, n_out, X, T, W, b, grad, loss, w, static_cast<hipStream_t>(stream),
                         nullptr);
}

extern "C" int mlp_train_step(int32_t dtype, int32_t M, int32_t n_in, int32_t hidden, int32_t n_out, const void *X,
                              const void *T, float *const *w, float *const *m, float *const *v, float *const *grad,
                              void *const *wc, float lr, float beta1, float beta2, float eps, int32_t step,
                              float *loss, void *work, size_t work_bytes, void *stream) {
    if (!w || !m || !v || !grad || !wc) return fail(HBMC_EINVAL, "null argument");
    for (int i = 0; i < 6; ++i)
        if (!w[i] || !m[i] || !v[i] || !grad[i]) return fail(HBMC_EINVAL, "null parameter array %d", i);
    if (step < 1) return fail(HBMC_EINVAL, "step %d < 1", step);
    const void *W[3] = {wc[0], wc[2], wc[4]};
    const float *b[3] = {w[1], w[3], w[5]};
    MLP_TRY(check_net(dtype, M, n_in, hidden, n_out, W, b));
    if (!X || !T || !work) return fail(HBMC_EINVAL, "null argument");
    if (work_bytes < net_layout(dtype, M, n_in, hidden, n_out, nullptr, nullptr))
        return fail(HBMC_EINVAL, "workspace too small");
    NetWork nw{};
    net_layout(dtype, M, n_in, hidden, n_out, &nw, work);
    FusedAdam fa{w, m, v, wc, lr, beta1, beta2, eps, 0.0f, 0.0f};
    bias_corrections(beta1, beta2, step, fa.c1, fa.c2);
    MLP_TRY(backward_impl(dtype, M, n_in, hidden, n_out, X, T, W, b, grad, loss, nw,
                          static_cast<hipStream_t>(stream), &fa));
    const int64_t sizes[6] = {int64_t(n_in) * hidden, hidden, int64_t(hidden) * hidden, hidden,
                              int64_t(hidden) * n_out, n_out};
    for (int i = 0; i < 6; ++i)
        if (i != 4)
            MLP_TRY(mlp_adam(dtype, sizes[i], w[i], m[i], v[i], grad[i], wc[i], lr, beta1, beta2, eps, step,
                             stream));
    return HBMC_OK;
}

extern "C" int mlp_adam_step(int32_t dtype, int32_t count, const int64_t *sizes, float *const *w, float *const *m,
                             float *const *v, const float *const *g, void *const *wc, float lr, float beta1,
                             float beta2, float eps, int32_t step, void *stream) {
    if (count < 1 || !sizes || !w || !m || !v || !g) return fail(HBMC_EINVAL, "null argument");
    for (int i = 0; i < count; ++i)
        MLP_TRY(mlp_adam(dtype, sizes[i], w[i], m[i], v[i], g[i], wc ? wc[i] : nullptr, lr, beta1, beta2, eps,
                         step, stream));
    return HBMC_OK;
}
