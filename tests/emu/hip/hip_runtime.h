// Host stand-in for the few HIP device features the persistent tile
// pipeline (paper_2607_01735_amd/csrc/blocked_pipeline.h) uses, so that its
// indexing, data flow and dependency protocol can be compiled for the CPU
// and checked with a sanitizer against the oracle.
//
// One workgroup = up to 128 lanes (one or two waves) run as cooperative
// fibers on one host thread; several workgroups are several host threads
// that share the grid arrays, tickets and progress flags through real
// atomics.  Inside a workgroup a cross-lane operation (DPP shift, vote,
// broadcast) and a fence are wave barriers: each lane hands over to the next
// in round-robin order, so every lane of the wave has reached the same
// operation before any lane goes on (the lanes of one wave run the same
// sequence of such operations, as on the GPU).  __syncthreads is a barrier
// over the whole workgroup.  LDS (__shared__) is per workgroup: static
// thread_local.  Test infrastructure only.
#pragma once
#include <sched.h>
#include <setjmp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <ucontext.h>

#include <algorithm>
#include <atomic>
#include <chrono>

#if defined(__SANITIZE_THREAD__)
#define EMU_TSAN 1
#elif defined(__has_feature)
#if __has_feature(thread_sanitizer)
#define EMU_TSAN 1
#endif
#endif
#ifdef EMU_TSAN
extern "C" {
void* __tsan_get_current_fiber(void);
void* __tsan_create_fiber(unsigned flags);
void __tsan_switch_to_fiber(void* fiber, unsigned flags);
}
#endif

typedef int hipError_t;
typedef void* hipStream_t;
typedef void* hipEvent_t;
#define __device__
#define __global__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static thread_local
#define __HIP_MEMORY_SCOPE_AGENT 0

using std::max;
using std::min;

namespace emu {
struct Dim {
    unsigned x, y, z;
};
constexpr int kLanes = 64;         // wave size
constexpr int kMaxThreads = 128;   // lanes per workgroup
extern thread_local int nthreads;  // lanes of this workgroup
extern thread_local int current;   // lane whose fiber runs
extern thread_local jmp_buf lane_jmp[kMaxThreads];  // where each parked lane resumes
extern thread_local bool lane_done[kMaxThreads];
extern thread_local uint64_t lane_slot[kMaxThreads];
extern thread_local int bar_arrived, bar_generation;
extern int yield_every;  // > 0: the host thread yields the CPU every so many switches
extern thread_local unsigned switches;
#ifdef EMU_TSAN
extern thread_local void* lane_fiber[kMaxThreads];
extern thread_local void* host_fiber;
#endif

extern thread_local int workgroup;  // this host thread's workgroup index

inline Dim thread_idx() { return Dim{unsigned(current), 0, 0}; }
inline Dim block_idx() { return Dim{unsigned(workgroup), 0, 0}; }

inline void jump_to_lane(int nx) {
#ifdef EMU_TSAN
    __tsan_switch_to_fiber(lane_fiber[nx], 0);
#endif
    current = nx;
    _longjmp(lane_jmp[nx], 1);
}

// Hand over to the next lane that has not finished (round robin).  The
// switch is _setjmp/_longjmp between the lanes' own stacks (no signal-mask
// system call per switch, unlike swapcontext).
inline void switch_to_next() {
    const int me = current;
    if (yield_every > 0 && ++switches % unsigned(yield_every) == 0) sched_yield();
    for (int k = 1; k <= nthreads; ++k) {
        const int nx = (me + k) % nthreads;
        if (!lane_done[nx]) {
            if (nx == me) return;
            if (_setjmp(lane_jmp[me]) == 0) jump_to_lane(nx);
            current = me;
            return;
        }
    }
}

inline void wave_barrier() { switch_to_next(); }

// The device's constant-rate counter, as a host steady clock (10 ns ticks).
inline unsigned long long realtime_ticks() {
    return (unsigned long long)(std::chrono::steady_clock::now().time_since_epoch().count() / 10);
}

inline int wave_base() { return current & ~(kLanes - 1); }

// Value of `v` in lane `src` (of this workgroup), as every lane sees it.
inline uint64_t from_lane(uint64_t v, int src) {
    lane_slot[current] = v;
    wave_barrier();
    const uint64_t r = lane_slot[src];
    wave_barrier();
    return r;
}

// Whole-wave DPP shifts: 0x130 = wave_shl:1 (lane i takes lane i+1),
// 0x138 = wave_shr:1 (lane i takes lane i-1), within the lane's wave.  A
// lane without a source keeps `old` (bound_ctrl off) or receives 0
// (bound_ctrl on).
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
    const bool valid = from >= wave_base() && from < wave_base() + kLanes;
    const uint64_t r = from_lane(uint32_t(src), valid ? from : me);
    if (valid) return int(uint32_t(r));
    return bound_ctrl ? 0 : old;
}

inline bool vote(bool p, bool want_all) {
    lane_slot[current] = p;
    wave_barrier();
    bool r = want_all;
    for (int i = wave_base(); i < wave_base() + kLanes; ++i)
        r = want_all ? (r && lane_slot[i]) : (r || lane_slot[i]);
    wave_barrier();
    return r;
}

// Workgroup barrier: every lane of the workgroup arrives before any leaves.
inline void block_barrier() {
    const int gen = bar_generation;
    if (++bar_arrived == nthreads) {
        bar_arrived = 0;
        ++bar_generation;
        return;
    }
    while (bar_generation == gen) switch_to_next();
}

// A fence is executed by a whole wave at once on the GPU: all of its lanes'
// earlier memory operations precede it.
inline void fence(int order) {
    wave_barrier();
    std::atomic_thread_fence(order == __ATOMIC_RELEASE ? std::memory_order_release
                             : order == __ATOMIC_ACQUIRE ? std::memory_order_acquire
                                                         : std::memory_order_seq_cst);
}
}  // namespace emu

#define threadIdx (emu::thread_idx())
#define blockIdx (emu::block_idx())
#define __syncthreads() emu::block_barrier()
#define __builtin_amdgcn_update_dpp(o, s, c, rm, bm, bc) emu::dpp(o, s, c, bc)
#define __builtin_amdgcn_mov_dpp(s, c, rm, bm, bc) emu::dpp(0, s, c, bc)
#define __builtin_amdgcn_readfirstlane(v) int(uint32_t(emu::from_lane(uint32_t(v), emu::wave_base())))
#define __builtin_amdgcn_sched_barrier(m) ((void)0)
#define __builtin_amdgcn_s_sleep(n) ((void)0)
#define __builtin_amdgcn_s_memrealtime() emu::realtime_ticks()
#define __builtin_amdgcn_fence(order, scope) emu::fence(order)
#define __all(p) emu::vote(p, true)
#define __any(p) emu::vote(p, false)
#ifdef EMU_TSAN
// ThreadSanitizer does not model stand-alone fences, so under it the flag
// protocol (relaxed store after a release fence, relaxed poll followed by
// an acquire fence) is checked in its equivalent acquire/release form.
#define __hip_atomic_load(p, order, scope) __atomic_load_n(p, __ATOMIC_ACQUIRE)
#define __hip_atomic_store(p, v, order, scope) __atomic_store_n(p, v, __ATOMIC_RELEASE)
#else
#define __hip_atomic_load(p, order, scope) __atomic_load_n(p, order)
#define __hip_atomic_store(p, v, order, scope) __atomic_store_n(p, v, order)
#endif
#define __hip_atomic_fetch_add(p, v, order, scope) __atomic_fetch_add(p, v, order)

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
