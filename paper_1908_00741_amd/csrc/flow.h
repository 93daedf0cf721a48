// All color phases of the workgroup-per-tile substitution in one launch
// (one system, one right-hand side).  The synchronization between colors
// (Section 4.4.3) becomes a wait on each value a tile reads: the forward
// values y and the result z start as kFlowEmpty, each tile stores its rows'
// values once, with agent-scope atomic stores, and a tile that finds
// kFlowEmpty where it gathers polls that word with agent-scope loads until
// the tile that owns the row has stored it.  The grid holds the phases in
// their sequential order (forward colors, the last color, backward colors),
// so a tile waits only on tiles of earlier workgroups: workgroups are
// dispatched in order, hence the earliest unfinished one always has its
// values and finishes.  Every wait is also bounded in time; past the limit
// it sets the error word, yields a NaN, and every later wait gives up at
// once, so a broken ordering shows as NaN results, never as a hang.
//
// The forward values live in a buffer of their own (y), not in z as in the
// one-launch-per-color form: a backward tile must tell z of a later color,
// which it waits for, from y of that color, which it must not take.
#pragma once
#include <hip/hip_runtime.h>

#include "fold.h"

namespace hbmc {

// A signalling NaN: arithmetic only yields quiet NaNs (an operand's
// signalling NaN comes out quieted), so no computed value has these bits.
constexpr uint64_t kFlowEmpty = 0x7FF00000DEADBEEFull;

// The error word and the time limit of every wait (ticks of the 100 MHz
// real-time counter).
struct FlowWait {
    int32_t *err;
    uint64_t ticks;
};

// The value at p once it is stored; past the time limit, or once another
// wait has timed out, a quiet NaN.
__device__ inline double flow_wait(const double *p, const FlowWait &fw) {
    const uint64_t *w = reinterpret_cast<const uint64_t *>(p);
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    int32_t *err = fw.err;
    uint64_t v;
    while ((v = get(w)) == kFlowEmpty) {
        if (get(err) != 0) return __builtin_nan("");
        if (__builtin_amdgcn_s_memrealtime() - t0 > fw.ticks) {
            atomicOr(err, 2);
            return __builtin_nan("");
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return __longlong_as_double(int64_t(v));
}

// v, loaded from p by an ordinary load (which may see a stale empty line in
// a cache), or the stored value once it is there.
__device__ inline double flow_take(double v, const double *p, const FlowWait &fw) {
    return __double_as_longlong(v) == int64_t(kFlowEmpty) ? flow_wait(p, fw) : v;
}

__device__ inline void flow_put(double *p, double v) {
    put(reinterpret_cast<uint64_t *>(p), uint64_t(__double_as_longlong(v)));
}

}  // namespace hbmc
