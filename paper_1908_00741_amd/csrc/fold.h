// alpha = rho / (p, A p) computed inside the first phase of the
// preconditioning step (one system, one right-hand side), in place of a
// kernel of its own: workgroup 0 of that phase adds up the product's
// partials and publishes alpha; every workgroup first loads the rows it
// updates (r -= alpha q), then waits for the publication.
// Workgroup 0 is dispatched first and waits on nobody before publishing, so
// the wait always ends; it is also bounded in time.
//
// Publication is an agent-scope atomic store of a 64-bit word: alpha's
// bits, or kStopped when the system stopped (its state, written with
// ordinary stores, is read by later kernels only); kNotYet marks a word not
// yet published.  The word is replicated kReplicas times on separate
// 128-byte lines (the 64 lanes of one wavefront store them at once) and
// each waiting wavefront polls one replica with one lane.  Each iteration
// uses one of two sets of words by its parity and resets the other, which
// the previous iteration (completed: same stream) used.
#pragma once
#include <hip/hip_runtime.h>

#include "hbmc_internal.h"

namespace hbmc {

constexpr uint64_t kFoldWaitTicks = 5000000;   // 50 ms of the 100 MHz real-time counter

template <class T>
__device__ inline void put(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ inline T get(const T *p) {
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Words that are no value of a scalar (NaN bit patterns no arithmetic
// produces)
constexpr uint64_t kNotYet = 0x7FF8DEAD0000BEEFull;
constexpr uint64_t kStopped = 0x7FF8DEAD0000D0E0ull;

constexpr int kReplicas = 64;
constexpr int kReplicaStride = 16;                       // words: 128 bytes apart
constexpr int kParityWords = kReplicas * kReplicaStride;   // one parity's replicas
constexpr int kFoldWords = 2 * kParityWords;               // one scalar's words, both parities

// Called by the 64 lanes of one wavefront: publishes value in parity's
// replicas and resets the other parity's.
__device__ inline void fold_publish(uint64_t *words, int parity, uint64_t value) {
    const int j = threadIdx.x & 63;
    put(words + (1 - parity) * kParityWords + j * kReplicaStride, kNotYet);
    put(words + parity * kParityWords + j * kReplicaStride, value);
}

// One lane of the calling wavefront polls its replica until the word is
// published; past the time limit sets *err and returns kStopped (the host
// then reports the error).  Returns the word to every lane.
__device__ inline uint64_t fold_wait(const uint64_t *words, int parity, int32_t *err) {
    const int wave = int(threadIdx.x >> 6);
    const int rep = int((int64_t(blockIdx.x) * ((blockDim.x + 63) >> 6) + wave) % kReplicas);
    const uint64_t *w = words + parity * kParityWords + rep * kReplicaStride;
    uint64_t v = kNotYet;
    if ((threadIdx.x & 63) == 0) {
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        while ((v = get(w)) == kNotYet) {
            if (__builtin_amdgcn_s_memrealtime() - t0 > kFoldWaitTicks) {
                atomicOr(err, 1);
                v = kStopped;
                break;
            }
            __builtin_amdgcn_s_sleep(4);
        }
    }
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
    return (uint64_t(hi) << 32) | lo;
}

// Sum of a[0 .. n) by every thread of the workgroup (at most 1024), in a
// fixed order: thread t adds elements t, t + blockDim, ... (sixteen loads
// in flight), then the wavefronts' sums, then the workgroup's in wavefront
// order.  Valid in thread 0; calls __syncthreads.
__device__ inline double wg_total(const double *a, int64_t n) {
    __shared__ double sh[16];
    constexpr int kIn = 16;
    const int64_t nt = blockDim.x;
    double sum = 0.0;
    for (int64_t i0 = threadIdx.x; i0 < n; i0 += nt * kIn) {
        double v[kIn];
#pragma unroll
        for (int k = 0; k < kIn; ++k) v[k] = i0 + k * nt < n ? a[i0 + k * nt] : 0.0;
#pragma unroll
        for (int k = 0; k < kIn; ++k) sum += v[k];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    const int wid = threadIdx.x >> 6, waves = int((nt + 63) >> 6);
    if ((threadIdx.x & 63) == 0) sh[wid] = sum;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < waves; ++k) t += sh[k];
    __syncthreads();
    return t;
}

// one stopped (system, right-hand side) more; the last raises the
// all-stopped flag
__device__ inline void count_done(int32_t *ndone, int32_t *alldone, int total) {
    if (atomicAdd(ndone, 1) + 1 == total) *alldone = 1;
}

// alpha = rho / (p, A p) from the product's partials, by workgroup 0 of the
// first phase (all its threads call it; wavefront 0 publishes); breakdown
// ((p, A p) not > 0 or not finite) stops the system
__device__ inline void fold_alpha(const ApplyCg &cg) {
    const double sigma = wg_total(cg.fpart, cg.fnp);
    uint64_t v = kStopped;
    if (threadIdx.x == 0) {
        CgState &c = cg.stw[0];
        c.sigma = sigma;
        const double alpha = c.rho / sigma;
        if (!(sigma > 0.0) || !isfinite(sigma) || !isfinite(alpha)) {
            c.it += 1;
            c.alpha = 0.0;   // no x update pending
            c.done = kBreakdown;
            count_done(cg.ndone, cg.alldone, 1);
        } else {
            c.alpha = alpha;
            v = __double_as_longlong(alpha);
        }
    }
    if (threadIdx.x < 64) {
        const uint32_t lo = __shfl(uint32_t(v), 0, 64), hi = __shfl(uint32_t(v >> 32), 0, 64);
        fold_publish(cg.fwords, cg.fparity, (uint64_t(hi) << 32) | lo);
    }
}

}  // namespace hbmc
