// Host stand-in for the few HIP device features the persistent tile
// pipeline (paper_2607_01735_amd/csrc/blocked_pipeline.h) uses, so that the
// pipeline's indexing and dependency logic can be compiled for the CPU and
// checked with AddressSanitizer against the oracle.  One wave = 64 lanes run
// as cooperative fibers on one host thread; a cross-lane operation (DPP
// shift, vote, broadcast) is a wave barrier, at which each lane hands over
// to the next in round-robin order, so every lane has reached it before any
// lane goes on.  The pipeline reaches every barrier uniformly (no lane skips
// one).  Test infrastructure only.
#pragma once
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <setjmp.h>
#include <ucontext.h>

#include <algorithm>

typedef int hipError_t;
typedef void* hipStream_t;
typedef void* hipEvent_t;
#define __device__
#define __global__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __HIP_MEMORY_SCOPE_AGENT 0

using std::max;
using std::min;

namespace emu {
struct Dim {
    unsigned x, y, z;
};
constexpr int kLanes = 64;
extern int current;               // lane whose fiber runs
extern jmp_buf lane_jmp[kLanes];  // where each parked lane resumes
extern bool lane_done[kLanes];
extern uint64_t lane_slot[kLanes];

inline Dim thread_idx() { return Dim{unsigned(current), 0, 0}; }

// Hand over to the next lane that has not finished (round robin).  The
// switch is _setjmp/_longjmp between the lanes' own stacks (no signal-mask
// system call per switch, unlike swapcontext).
inline void switch_to_next() {
    const int me = current;
    for (int k = 1; k <= kLanes; ++k) {
        const int nx = (me + k) % kLanes;
        if (!lane_done[nx]) {
            if (nx == me) return;
            if (_setjmp(lane_jmp[me]) == 0) {
                current = nx;
                _longjmp(lane_jmp[nx], 1);
            }
            current = me;
            return;
        }
    }
}

inline void wave_barrier() { switch_to_next(); }

// Value of `v` in lane `src`, as every lane sees it.
inline uint64_t from_lane(uint64_t v, int src) {
    lane_slot[current] = v;
    wave_barrier();
    const uint64_t r = lane_slot[src];
    wave_barrier();
    return r;
}

// Whole-wave DPP shifts: 0x130 = wave_shl:1 (lane i takes lane i+1),
// 0x138 = wave_shr:1 (lane i takes lane i-1).  A lane without a source
// keeps `old` (bound_ctrl off) or receives 0 (bound_ctrl on).
inline int dpp(int old, int src, int ctrl, bool bound_ctrl) {
    const int me = current;
    int from;
    if (ctrl == 0x130)
        from = me + 1;
    else if (ctrl == 0x138)
        from = me - 1;
    else {
        fprintf(stderr, "unsupported DPP control %#x\n", ctrl);
        abort();
    }
    const bool valid = from >= 0 && from < kLanes;
    const uint64_t r = from_lane(uint32_t(src), valid ? from : me);
    if (valid) return int(uint32_t(r));
    return bound_ctrl ? 0 : old;
}

inline bool vote(bool p, bool want_all) {
    lane_slot[current] = p;
    wave_barrier();
    bool r = want_all;
    for (int i = 0; i < kLanes; ++i) r = want_all ? (r && lane_slot[i]) : (r || lane_slot[i]);
    wave_barrier();
    return r;
}
}  // namespace emu

#define threadIdx (emu::thread_idx())
#define __builtin_amdgcn_update_dpp(o, s, c, rm, bm, bc) emu::dpp(o, s, c, bc)
#define __builtin_amdgcn_mov_dpp(s, c, rm, bm, bc) emu::dpp(0, s, c, bc)
#define __builtin_amdgcn_readfirstlane(v) int(uint32_t(emu::from_lane(uint32_t(v), 0)))
#define __builtin_amdgcn_sched_barrier(m) ((void)0)
#define __builtin_amdgcn_s_sleep(n) ((void)0)
#define __builtin_amdgcn_fence(order, scope) __atomic_thread_fence(__ATOMIC_SEQ_CST)
#define __all(p) emu::vote(p, true)
#define __any(p) emu::vote(p, false)
#define __hip_atomic_load(p, order, scope) __atomic_load_n(p, __ATOMIC_SEQ_CST)
#define __hip_atomic_store(p, v, order, scope) __atomic_store_n(p, v, __ATOMIC_SEQ_CST)
#define __hip_atomic_fetch_add(p, v, order, scope) __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST)

template <class To, class From>
inline To emu_bits(From f) {
    To t;
    memcpy(&t, &f, sizeof t);
    return t;
}
inline double __hiloint2double(int hi, int lo) {
    return emu_bits<double>((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
}
inline int __double2hiint(double d) { return int(emu_bits<uint64_t>(d) >> 32); }
inline int __double2loint(double d) { return int(uint32_t(emu_bits<uint64_t>(d))); }
inline float __int_as_float(int i) { return emu_bits<float>(i); }
inline int __float_as_int(float f) { return emu_bits<int>(f); }
inline float __uint_as_float(uint32_t i) { return emu_bits<float>(i); }
inline uint32_t __float_as_uint(float f) { return emu_bits<uint32_t>(f); }
inline double __longlong_as_double(long long i) { return emu_bits<double>(i); }
inline long long __double_as_longlong(double d) { return emu_bits<long long>(d); }
