// Two-wave tiles for the persistent blocked sweep: the tile pipeline of
// blocked_pipeline.h with its L levels split over the two waves of a
// workgroup.  The front wave loads the tile's input rows (several steps
// ahead) and runs levels 0 .. LA-1; the back wave runs levels LA .. L-1 one
// step behind it and stores the results.  Per step the front wave hands
// the back wave the row its last level produced (and, on edge tiles, the
// row before it, which carries the Dirichlet ring through the level that
// follows) through LDS; both waves read the right-hand sides h^2 f from the
// one LDS ring the front wave fills.  One workgroup barrier per step keeps
// the two apart by exactly one step.
//
// Why: with all L levels in one wave a tile needs about 300 registers and a
// 32 KB ring, so each SIMD holds one wave and nothing hides the waits for
// HBM or LDS.  Split, each wave needs about half the registers, two waves
// share one ring, and the front wave has registers left to load its inputs
// five steps ahead instead of three, so more bytes are in flight per tile.
//
// Every point still receives Eq. (1)'s operations in the canonical order
// from the same neighbour values, so the result is the plain sweep's bit
// for bit (the schedule inside a tile changes, the data flow does not).
#pragma once

#include "blocked_pipeline.h"

namespace rbgs {
namespace blocked {

constexpr int kSplitThreads = 2 * kLanes;

template <int L>
constexpr int split_front_levels() { return L / 2; }

// Steps ahead that the front wave loads its inputs (the ring of input slots
// has 6 entries, one of them the step being processed).
constexpr int kSplitPrefetch = 5;

template <typename T, int V, int L>
struct SplitShared {
    FRing<T, V, L> fr;
    Vec<T, V> c1[2][kLanes];  // output row of level LA-1 at step x (slot x & 1)
    Vec<T, V> c0[2][kLanes];  // edge tiles: output row of level LA-2 at step x
};

template <typename T, int V, int NL>
struct Levels {
    Vec<T, V> win[NL][3];
};

// One Eq. (1) update of level l's row from its window and right-hand side
// (the same operations, in the same order, as pipe_step).
template <typename T, int V, int l, int S, bool EDGE>
__device__ __forceinline__ Vec<T, V> level_update(const Vec<T, V>& up, const Vec<T, V>& mid,
                                                  const Vec<T, V>& dn, const Vec<T, V>& fl,
                                                  const Vec<T, V>& prev, int x, int n,
                                                  int64_t q0) {
    constexpr int p = pmod(S - 1 - l + (l & 1), 2);
    T extra;
    if constexpr (p == 1)
        extra = lane_shift<kWaveShl1>(mid.v[0]);
    else
        extra = lane_shift<kWaveShr1>(mid.v[V - 1]);
    const int y = x - 1 - l;
    const bool row_in = y >= 1 && y <= n;
    const int64_t q_lo = 1 - p, q_hi = (int64_t(n) - p) >> 1;
    Vec<T, V> out;
#pragma unroll
    for (int e = 0; e < V; ++e) {
        T right = p ? (e + 1 < V ? mid.v[e + 1] : extra) : mid.v[e];
        T left = p ? mid.v[e] : (e > 0 ? mid.v[e - 1] : extra);
        T s = dn.v[e] + up.v[e];
        s = s + right;
        s = s + left;
        s = s - fl.v[e];
        T nv = T(0.25) * s;
        if constexpr (EDGE) {
            const int64_t q = q0 + e;
            out.v[e] = blend(row_in && q >= q_lo && q <= q_hi, nv, prev.v[e]);
        } else {
            out.v[e] = nv;
        }
    }
    return out;
}

template <int R>
__device__ __forceinline__ int ring_slot(int x, int back) {
    if constexpr ((R & (R - 1)) == 0) {
        return (x - back) & (R - 1);
    } else {
        const int base = x % R;
        return base - back < 0 ? base - back + R : base - back;
    }
}

// Front wave, step x (S = x mod 6): loads step x + kSplitPrefetch, puts this
// step's right-hand sides into the ring, runs levels 0 .. LA-1 and hands
// level LA-1's output (and on edge tiles level LA-2's) to the back wave.
template <typename T, int V, int L, int S, bool EDGE>
__device__ __forceinline__ void front_step(Levels<T, V, split_front_levels<L>()>& st,
                                           StepIn<T, V> (&in)[6], Vec<T, V> (&red_in)[2],
                                           SplitShared<T, V, L>& sh, const GridDesc<T>& a,
                                           const T* __restrict__ xr, const T* __restrict__ xb,
                                           int x, int xs, int xe, int64_t q0, int64_t qv) {
    constexpr int LA = split_front_levels<L>();
    constexpr int R = fring_rows<L>();
    const int lane = threadIdx.x & (kLanes - 1);
    const StepIn<T, V> cur = in[S];
    in[(S + kSplitPrefetch) % 6] = load_in<T, V, EDGE>(a, xr, xb, x + kSplitPrefetch, xs, xe, qv);
    Vec<T, V> hf[LA];
#pragma unroll
    for (int e = 0; e < V; ++e) {
        hf[0].v[e] = a.h2 * cur.f0.v[e];
        hf[1].v[e] = a.h2 * cur.f1.v[e];
    }
    sh.fr.row[0][ring_slot<R>(x, 1)][lane] = hf[0];
    sh.fr.row[1][ring_slot<R>(x, 2)][lane] = hf[1];
    static_for<2, LA>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        hf[l] = sh.fr.row[l & 1][ring_slot<R>(x, 1 + l)][lane];
    });
    __builtin_amdgcn_sched_barrier(0);
    Vec<T, V> carry = cur.b;
    Vec<T, V> before = carry;  // input of the last level (output of level LA-2)
    static_for<0, LA>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        st.win[l][pmod(S - l, 3)] = carry;
        if constexpr (l == LA - 1) before = carry;
        auto upd = [&](const Vec<T, V>& prev) {
            return level_update<T, V, l, S, EDGE>(st.win[l][pmod(S - l - 2, 3)],
                                                  st.win[l][pmod(S - l - 1, 3)],
                                                  st.win[l][pmod(S - l, 3)], hf[l], prev, x, a.n,
                                                  q0);
        };
        if constexpr (l == 0)
            carry = upd(red_in[pmod(S - 1, 2)]);
        else
            carry = upd(st.win[l - 1][pmod(S - l - 1, 3)]);
    });
    if constexpr (EDGE) red_in[S & 1] = cur.r;
    sh.c1[x & 1][lane] = carry;
    if constexpr (EDGE) sh.c0[x & 1][lane] = before;
}

// Back wave, step x (S = x mod 6): takes the front wave's rows of step x,
// runs levels LA .. L-1 and stores row x - L (black, and red when asked).
// pw mirrors the window of level LA-1 (edge tiles: the pass-through values).
template <typename T, int V, int L, int S, bool EDGE>
__device__ __forceinline__ void back_step(Levels<T, V, L - split_front_levels<L>()>& st,
                                          Vec<T, V> (&pw)[3], SplitShared<T, V, L>& sh,
                                          const GridDesc<T>& a, T* __restrict__ yr,
                                          T* __restrict__ yb, int x, int r0, int r1, int64_t q0,
                                          int64_t qc0, int64_t qc1, bool in_core,
                                          bool store_red) {
    constexpr int LA = split_front_levels<L>();
    constexpr int NB = L - LA;
    constexpr int R = fring_rows<L>();
    const int lane = threadIdx.x & (kLanes - 1);
    const int n = a.n;
    const int64_t P = a.pitch;
    Vec<T, V> carry = sh.c1[x & 1][lane];
    if constexpr (EDGE) pw[pmod(S - (LA - 1), 3)] = sh.c0[x & 1][lane];
    Vec<T, V> hf[NB];
    static_for<0, NB>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int l = LA + k;
        hf[k] = sh.fr.row[l & 1][ring_slot<R>(x, 1 + l)][lane];
    });
    __builtin_amdgcn_sched_barrier(0);
    static_for<0, NB>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int l = LA + k;
        st.win[k][pmod(S - l, 3)] = carry;
        auto upd = [&](const Vec<T, V>& prev) {
            return level_update<T, V, l, S, EDGE>(st.win[k][pmod(S - l - 2, 3)],
                                                  st.win[k][pmod(S - l - 1, 3)],
                                                  st.win[k][pmod(S - l, 3)], hf[k], prev, x, n, q0);
        };
        if constexpr (k == 0)
            carry = upd(pw[pmod(S - l - 1, 3)]);
        else
            carry = upd(st.win[k - 1][pmod(S - l - 1, 3)]);
    });
    const int y = x - L;
    if (y >= r0 && y <= r1) {
        if constexpr (EDGE) {
            store_core<T, V>(yb + int64_t(y) * P, carry, q0, qc0, qc1, pmod(S - L + 1, 2), n);
            if (store_red)
                store_core<T, V>(yr + int64_t(y) * P, st.win[NB - 1][pmod(S - L, 3)], q0, qc0,
                                 qc1, pmod(S - L, 2), n);
        } else if (in_core) {
            *reinterpret_cast<Vec<T, V>*>(yb + int64_t(y) * P + q0) = carry;
            if (store_red)
                *reinterpret_cast<Vec<T, V>*>(yr + int64_t(y) * P + q0) =
                    st.win[NB - 1][pmod(S - L, 3)];
        }
    }
}

template <typename T, int V, int L, bool EDGE>
__device__ __forceinline__ void run_tile_split(SplitShared<T, V, L>& sh, const GridDesc<T>& a,
                                               int pass, int r0, int r1, int64_t qc0,
                                               int64_t qc1, bool store_red) {
    constexpr int LA = split_front_levels<L>();
    // a scalar, so that each wave takes its branch as a whole (the barriers
    // inside must be met by both waves, never by a wave with no lanes on)
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int lane = threadIdx.x & (kLanes - 1);
    const int64_t q0 = qc0 - a.halo_q + int64_t(lane) * V;
    const int64_t qv = q0 < 0 ? 0 : (q0 > a.pitch - V ? a.pitch - V : q0);
    const bool in_core = q0 >= qc0 && q0 + V <= qc1;
    const int xs = max(0, r0 - L);
    const int xe = min(a.n + 1, r1 + L);
    const int x_last = r1 + L;
    const int x0 = xs - xs % 6;
    // both waves run the same number of steps (one barrier each); the back
    // wave is one step behind, so the loop runs one step past x_last
    if (wave == 0) {
        const T* xr = a.red[pass & 1];
        const T* xb = a.black[pass & 1];
        Levels<T, V, LA> st;
#pragma unroll
        for (int l = 0; l < LA; ++l)
#pragma unroll
            for (int r = 0; r < 3; ++r) st.win[l][r] = vzero<T, V>();
        Vec<T, V> red_in[2] = {vzero<T, V>(), vzero<T, V>()};
        StepIn<T, V> in[6];
#pragma unroll
        for (int d = 0; d < kSplitPrefetch; ++d)
            in[d] = load_in<T, V, EDGE>(a, xr, xb, x0 + d, xs, xe, qv);
        for (int x = x0; x <= x_last + 1; x += 6) {
            front_step<T, V, L, 0, EDGE>(st, in, red_in, sh, a, xr, xb, x + 0, xs, xe, q0, qv);
            __syncthreads();
            front_step<T, V, L, 1, EDGE>(st, in, red_in, sh, a, xr, xb, x + 1, xs, xe, q0, qv);
            __syncthreads();
            front_step<T, V, L, 2, EDGE>(st, in, red_in, sh, a, xr, xb, x + 2, xs, xe, q0, qv);
            __syncthreads();
            front_step<T, V, L, 3, EDGE>(st, in, red_in, sh, a, xr, xb, x + 3, xs, xe, q0, qv);
            __syncthreads();
            front_step<T, V, L, 4, EDGE>(st, in, red_in, sh, a, xr, xb, x + 4, xs, xe, q0, qv);
            __syncthreads();
            front_step<T, V, L, 5, EDGE>(st, in, red_in, sh, a, xr, xb, x + 5, xs, xe, q0, qv);
            __syncthreads();
        }
    } else {
        T* yr = a.red[(pass + 1) & 1];
        T* yb = a.black[(pass + 1) & 1];
        Levels<T, V, L - LA> st;
#pragma unroll
        for (int l = 0; l < L - LA; ++l)
#pragma unroll
            for (int r = 0; r < 3; ++r) st.win[l][r] = vzero<T, V>();
        Vec<T, V> pw[3] = {vzero<T, V>(), vzero<T, V>(), vzero<T, V>()};
        // the first step (x0 - 1) precedes the tile's loaded rows: its values
        // only reach rows outside every stored row's dependency cone
        for (int x = x0; x <= x_last + 1; x += 6) {
            back_step<T, V, L, 5, EDGE>(st, pw, sh, a, yr, yb, x - 1, r0, r1, q0, qc0, qc1, in_core,
                                        store_red);
            __syncthreads();
            back_step<T, V, L, 0, EDGE>(st, pw, sh, a, yr, yb, x + 0, r0, r1, q0, qc0, qc1, in_core,
                                        store_red);
            __syncthreads();
            back_step<T, V, L, 1, EDGE>(st, pw, sh, a, yr, yb, x + 1, r0, r1, q0, qc0, qc1, in_core,
                                        store_red);
            __syncthreads();
            back_step<T, V, L, 2, EDGE>(st, pw, sh, a, yr, yb, x + 2, r0, r1, q0, qc0, qc1, in_core,
                                        store_red);
            __syncthreads();
            back_step<T, V, L, 3, EDGE>(st, pw, sh, a, yr, yb, x + 3, r0, r1, q0, qc0, qc1, in_core,
                                        store_red);
            __syncthreads();
            back_step<T, V, L, 4, EDGE>(st, pw, sh, a, yr, yb, x + 4, r0, r1, q0, qc0, qc1, in_core,
                                        store_red);
            __syncthreads();
        }
    }
}

template <typename T, int V, int L>
__device__ __forceinline__ void process_tile_split(SplitShared<T, V, L>& sh, const GridDesc<T>& a,
                                                   int pass, int tile, bool store_red) {
    const int strip = tile / a.bands;
    const int band = tile - strip * a.bands;
    const int r0 = 1 + strip * a.rows;
    const int r1 = min(a.n, r0 + a.rows - 1);
    const int64_t qc0 = int64_t(band) * a.q_core;
    const int64_t qmax = int64_t(a.n >> 1);
    const int64_t qc1 = qc0 + a.q_core < qmax + 1 ? qc0 + a.q_core : qmax + 1;
    const int64_t qa = qc0 - a.halo_q;
    const bool interior = r0 - L >= 1 && r1 + L <= a.n && qa >= 1 &&
                          qa + int64_t(kLanes) * V - 1 <= (int64_t(a.n) - 1) >> 1 &&
                          qc1 - qc0 == a.q_core;
    if (interior)
        run_tile_split<T, V, L, false>(sh, a, pass, r0, r1, qc0, qc1, store_red);
    else
        run_tile_split<T, V, L, true>(sh, a, pass, r0, r1, qc0, qc1, store_red);
}

// The persistent loop for two-wave tiles: wave 0 takes the ticket and waits
// for the tile's dependencies, the workgroup runs the tile, both waves make
// their stores visible at agent scope, then thread 0 publishes the progress
// flag (the same protocol as run_item, at workgroup granularity).
template <typename T, int V, int L>
__device__ __forceinline__ void persistent_split(const GridDesc<T>& g, const Queue& qu) {
    __shared__ SplitShared<T, V, L> sh;
    __shared__ int s_ticket, s_ok;
    const int total = qu.passes * g.ntiles;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    for (;;) {
        if (threadIdx.x == 0)
            s_ticket = __hip_atomic_fetch_add(qu.ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int tk = __builtin_amdgcn_readfirstlane(s_ticket);
        if (tk >= total) break;
        const int pass = tk / g.ntiles;
        const int tile = tk - pass * g.ntiles;
        if (wave == 0) {
            const bool ok = wait_deps(g, qu, pass, tile);
            if (ok && qu.delay > 0) {
                uint32_t loops = mix32(uint32_t(pass) * 0x9e3779b9u + uint32_t(g.flag_base + tile)) %
                                 uint32_t(qu.delay + 1);
                for (uint32_t i = 0; i < loops; ++i) __builtin_amdgcn_s_sleep(127);
            }
            if (threadIdx.x == 0) s_ok = ok ? 1 : 0;
        }
        __syncthreads();
        if (!__builtin_amdgcn_readfirstlane(s_ok)) break;
        process_tile_split<T, V, L>(sh, g, pass + qu.buf_offset, tile, pass == qu.passes - 1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0 && g.flag_base + tile + 1 != qu.stall_tile)
            __hip_atomic_store(qu.progress + g.flag_base + tile, pass + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace blocked
}  // namespace rbgs
