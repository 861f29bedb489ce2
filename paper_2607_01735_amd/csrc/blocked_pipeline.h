// Device-side tile pipeline shared by the single-grid and batched
// persistent sweep kernels (see sweep_blocked.hip for the method).
#pragma once

#include <climits>
#include <type_traits>

#include "rbgs_internal.h"

namespace rbgs {
namespace blocked {


constexpr int kLanes = 64;
constexpr int kDefaultSpinLimit = 1 << 22;

template <typename T, int V>
struct alignas(sizeof(T) * V) Vec {
    T v[V];
};

template <int N>
using IC = std::integral_constant<int, N>;

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(IC<B>{});
        static_for<B + 1, E>(f);
    }
}

constexpr int pmod(int a, int m) { return ((a % m) + m) % m; }

// One grid as the persistent kernels see it (split layout, two buffers).
template <typename T>
struct GridDesc {
    T* red[2];  // ping-pong buffers of the split iterate: pass p reads [p & 1]
    T* black[2];
    const T* f_red;
    const T* f_black;
    int n;
    int64_t pitch;
    T h2;
    int rows;         // interior rows per strip
    int halo_q;       // halo q-columns on each side (multiple of V)
    int q_core;       // q-columns written per band
    int strips, bands, ntiles;
    int flag_base;    // index of this grid's first tile in the progress array
    T omega;          // relaxation of a batched SOR launch (the single-grid
                      // kernels take it as an argument)
};

// Work queue shared by all waves of one persistent launch.
struct Queue {
    int passes;
    int* progress;    // passes completed, per tile (all grids)
    int* ticket;
    int* error;
    int spin_limit;
    int delay;
    int stall_tile;   // debug: global tile index + 1 that never publishes (0 = off)
    int buf_offset;   // pass p reads buffer (p + buf_offset) & 1
    const int* stop;  // converged flag of a graph-captured solve (nullptr: none)
};

// Verification modes of the single-grid kernel.  They run in a separate
// instantiation (DBG = true), so the production kernel carries none of
// their code or arguments.
struct DebugModes {
    int order = 0;          // tiles of a pass in ticket order: 0 as numbered,
                            // 1 reversed, 2 a pseudo-random permutation per pass
    uint32_t seed = 0;      // of the order-2 permutations
    int stamp_check = 0;    // 1: check the neighbours' pass counts around each item
    unsigned long long* trace = nullptr;  // per-item records (kTraceWords each), or none
    long long trace_items = 0;            // records the array holds
    long long trace_base = 0;             // record index of this launch's first ticket
};

// Error-word values: a bounded wait expired / the stamp check failed.
constexpr int kErrTimeout = 1;
constexpr int kErrOrder = 2;

// A trace record: start and end of the item (the device's constant-rate
// real-time counter, read after the dependency wait and after the item's
// writes were released), (pass << 32) | tile, and (workgroup << 32) |
// ticket-within-launch.
constexpr int kTraceWords = 4;

__device__ __forceinline__ uint32_t mix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    return h;
}

__device__ __forceinline__ int gcd_int(int a, int b) {
    while (b != 0) {
        const int t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Tile of the t-th ticket of a pass.  Tickets stay in pass-major order, so
// every order is a topological order of the dependency graph (a pass-p item
// waits only on pass p-1 items, all ticketed before any of pass p) and no
// order can deadlock.  Order 2 maps t to (a t + b) mod ntiles with a coprime
// to ntiles, a and b drawn from the seed and the pass.
__device__ __forceinline__ int tile_of_ticket(const DebugModes& dm, int ntiles, int pass, int t) {
    if (dm.order == 1) return ntiles - 1 - t;
    if (dm.order == 2 && ntiles > 1) {
        const uint32_t h = mix32(dm.seed * 0x9e3779b9u + uint32_t(pass) * 0x85ebca6bu + 1u);
        int a = int(h % uint32_t(ntiles));
        if (a == 0) a = 1;
        while (gcd_int(a, ntiles) != 1) a = a + 1 < ntiles ? a + 1 : 1;
        const int b = int(mix32(h ^ 0x68e31da4u) % uint32_t(ntiles));
        return int((int64_t(a) * t + b) % ntiles);
    }
    return t;
}

// True when a graph-captured solve has converged before this launch (the
// flag is written by an earlier kernel of the stream, so every wave reads
// the same value and leaves together).
__device__ __forceinline__ bool stopped(const Queue& qu) {
    return qu.stop != nullptr && __hip_atomic_load(qu.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

template <typename T, int V>
__device__ __forceinline__ Vec<T, V> vload(const T* p) {
    return *reinterpret_cast<const Vec<T, V>*>(p);
}

template <typename T, int V>
__device__ __forceinline__ Vec<T, V> vzero() {
    Vec<T, V> z;
#pragma unroll
    for (int e = 0; e < V; ++e) z.v[e] = T(0);
    return z;
}

// Inputs that a step consumes first-hand from HBM: the black and red rows x
// of the pass input, and the right-hand sides of levels 0 and 1 (f_red row
// x-1 and f_black row x-2, their first use).  The right-hand sides of levels
// >= 2 are rows that levels 0 and 1 brought in earlier (kept in LDS).
template <typename T, int V>
struct StepIn {
    Vec<T, V> b, r, f0, f1;
};

// Steps ahead that a tile loads its inputs.  The deep pipelines run one
// wave per SIMD, so the loads in flight alone must cover HBM latency: three
// steps ahead was 5% faster than two for FP64 at 8191^2 and 2% at 4095^2
// (four was no better than two); FP32 and the deepest pipelines (L > 14),
// short of registers, keep two.
template <typename T, int L>
constexpr int prefetch_steps() {
#ifdef RBGS_EMU_PREFETCH_STEPS  // the CPU emulation replays other depths (1..5)
    return RBGS_EMU_PREFETCH_STEPS;
#else
    return sizeof(T) == 8 && L <= 14 ? 3 : 2;
#endif
}

// Whole-wave lane shifts through DPP (register to register, no LDS trip):
// from_next_lane gives lane i the value of lane i+1 (wave_shl:1), and
// from_prev_lane the value of lane i-1 (wave_shr:1).  The lane with no
// source receives 0 (bound_ctrl); it lies in the tile's halo, whose values
// are never stored.  Not asking for the old value to be kept saves a copy of
// the source register per shift.
template <int CTRL>
__device__ __forceinline__ int dpp_shift(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}

constexpr int kWaveShl1 = 0x130;
constexpr int kWaveShr1 = 0x138;

template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(dpp_shift<CTRL>(hi), dpp_shift<CTRL>(lo));
}

template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
    return __int_as_float(dpp_shift<CTRL>(__float_as_int(v)));
}

// c ? a : b as a bitwise blend, so the compiler cannot turn it into a
// branch around the computation of a (it did, with exec-mask juggling and
// scalar-register spills, when this was a plain conditional).
__device__ __forceinline__ double blend(bool c, double a, double b) {
    const uint64_t m = uint64_t(0) - uint64_t(c);
    return __longlong_as_double(
        (long long)((uint64_t(__double_as_longlong(a)) & m) | (uint64_t(__double_as_longlong(b)) & ~m)));
}

__device__ __forceinline__ float blend(bool c, float a, float b) {
    const uint32_t m = uint32_t(0) - uint32_t(c);
    return __uint_as_float((__float_as_uint(a) & m) | (__float_as_uint(b) & ~m));
}

template <typename T, int V, int L>
struct Pipe {
    Vec<T, V> win[L][3];   // level l: other-colour rows (ring buffer of 3), version l-1
    Vec<T, V> red_in[2];   // red input rows x-1, x (ring values pass through level 0)
    StepIn<T, V> in[6];    // inputs of steps x .. x+D (slot x mod 6), D = prefetch_steps
};

// Right-hand-side rows of a wave (as the products h^2 f), kept in LDS for
// the deeper levels.  Level l of step x needs f of colour l & 1 at row
// x-1-l, a row that levels 0 (red) or 1 (black) loaded l or l-1 steps
// earlier; each wave keeps the rows it loaded in a ring of L + 2 rows per
// colour, one 16-byte slot per lane,
// instead of fetching them again from memory for every level (those
// re-reads missed L2 and doubled the HBM read traffic at 6 fused sweeps).
// The ring holds at least L + 2 rows per colour (rows x-1 .. x-L are live
// at step x): the next power of two up to L = 14, so that the slot is a
// mask; L + 2 beyond, so that the ring stays within 40 KB and four waves
// fit a CU.
template <int L>
constexpr int fring_rows() { return L <= 2 ? 4 : L <= 6 ? 8 : L <= 14 ? 16 : L + 2; }

template <typename T, int V, int R>
struct FRingRows {
    Vec<T, V> row[2][R][kLanes];
};

template <typename T, int V, int L>
using FRing = FRingRows<T, V, fring_rows<L>()>;

// The wave's ring in LDS, one allocation per (type, vector, ring height):
// pipelines of different depth with the same ring height (the passes of one
// launch whose depths differ by one sweep) share it.
template <typename T, int V, int R>
__device__ __forceinline__ FRingRows<T, V, R>& wave_fring() {
    __shared__ FRingRows<T, V, R> fr;
    return fr;
}

// Loads never branch: row and column indices are clamped into the grid,
// and rows of the iterate into the tile's loaded region [lo, hi] = [xs, xe]
// (its rows plus L halo rows each side, inside the dependency region that
// the tile waited for), so that no load touches rows another tile may be
// writing.  A clamped load only ever feeds rows or columns outside the
// region the tile writes (the warm-up rows above xs, the drain rows below
// xe, lanes beyond the grid edge), whose values are recomputed garbage
// anyway.
__device__ __forceinline__ int clamp_row(int x, int lo, int hi) {
    return x < lo ? lo : (x > hi ? hi : x);
}

template <typename T, int V, bool EDGE, bool SOR = false>
__device__ __forceinline__ StepIn<T, V> load_in(const GridDesc<T>& a, const T* __restrict__ xr,
                                                const T* __restrict__ xb, int x, int lo, int hi,
                                                int64_t qv) {
    StepIn<T, V> in;
    const int64_t P = a.pitch;
    const int64_t row = int64_t(clamp_row(x, lo, hi)) * P + qv;
    in.b = vload<T, V>(xb + row);
    // red input values matter only where they pass through unchanged
    // (the ring); interior tiles never see the ring.  SOR relaxes every
    // red point from its old value, so it reads them everywhere.
    if constexpr (EDGE || SOR)
        in.r = vload<T, V>(xr + row);
    else
        in.r = vzero<T, V>();
    in.f0 = vload<T, V>(a.f_red + int64_t(clamp_row(x - 1, 1, a.n)) * P + qv);
    in.f1 = vload<T, V>(a.f_black + int64_t(clamp_row(x - 2, 1, a.n)) * P + qv);
    return in;
}

// Store the core part of one row: q in [qc0, qc1) and interior for parity p.
template <typename T, int V>
__device__ __forceinline__ void store_core(T* row, const Vec<T, V>& v, int64_t q0, int64_t qc0,
                                           int64_t qc1, int p, int n) {
    const int64_t lo = qc0 > 1 - p ? qc0 : 1 - p;
    const int64_t hi_in = (int64_t(n) - p) >> 1;
    const int64_t hi = qc1 - 1 < hi_in ? qc1 - 1 : hi_in;
    if (q0 >= lo && q0 + V - 1 <= hi) {
        *reinterpret_cast<Vec<T, V>*>(row + q0) = v;
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e)
            if (q0 + e >= lo && q0 + e <= hi) row[q0 + e] = v.v[e];
    }
}

// One pipeline step at input row x; S = x mod 6 fixes, at compile time, the
// ring-buffer slots (period 3) and the row parities (period 2).  SOR: each
// level relaxes the Gauss-Seidel value g of a point from its previous
// version u, u + omega (g - u), each operation rounded once (as the plain
// kernel does).
template <typename T, int V, int L, int S, bool EDGE, bool SOR = false>
__device__ __forceinline__ void pipe_step(Pipe<T, V, L>& st, FRing<T, V, L>& fr, const GridDesc<T>& a,
                                          const T* __restrict__ xr, const T* __restrict__ xb,
                                          T* __restrict__ yr, T* __restrict__ yb, int x, int xs,
                                          int xe, int r0, int r1, int64_t q0, int64_t qv,
                                          int64_t qc0, int64_t qc1, bool in_core, bool store_red,
                                          T omega = T(1)) {
    const int n = a.n;
    const int64_t P = a.pitch;
    constexpr int D = prefetch_steps<T, L>();
    const StepIn<T, V> cur = st.in[S];
    // prefetch: step x+D's rows into a slot no pending step holds
    st.in[(S + D) % 6] = load_in<T, V, EDGE, SOR>(a, xr, xb, x + D, xs, xe, qv);
    // this step's right-hand-side rows join the ring (red row x-1, black
    // row x-2) as the products h^2 f that Eq. (1) subtracts: each is formed
    // once here, not once per fused level (the same product, so the same
    // bits).  The deeper levels read older rows from the ring.  Row r sits in
    // slot r mod R; base = x mod R (x >= 0), and every slot below is base
    // minus a compile-time offset, wrapped once.
    constexpr int R = fring_rows<L>();
    const int lane = threadIdx.x;
    const int base = (R & (R - 1)) == 0 ? (x & (R - 1)) : x % R;
    auto slot = [&](int back) {
        if constexpr ((R & (R - 1)) == 0)
            return (base - back) & (R - 1);
        else
            return base - back < 0 ? base - back + R : base - back;
    };
    Vec<T, V> hf[L];  // h^2 f for each level's row y = x - 1 - l
#pragma unroll
    for (int e = 0; e < V; ++e) {
        hf[0].v[e] = a.h2 * cur.f0.v[e];
        hf[1].v[e] = a.h2 * cur.f1.v[e];
    }
    fr.row[0][slot(1)][lane] = hf[0];
    fr.row[1][slot(2)][lane] = hf[1];
    // all ring reads of the step are issued up front, so that their LDS
    // latency overlaps the first levels instead of stalling each level
    static_for<2, L>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        hf[l] = fr.row[l & 1][slot(1 + l)][lane];
    });
    // keep the scheduler from sinking those reads back next to their uses
    __builtin_amdgcn_sched_barrier(0);
    const Vec<T, V> bin = cur.b;
    const Vec<T, V> rin = cur.r;
    Vec<T, V> carry = bin;  // row entering level l's window
    static_for<0, L>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        constexpr int s_new = pmod(S - l, 3);      // row x - l
        constexpr int s_mid = pmod(S - l - 1, 3);  // row y = x - 1 - l
        constexpr int s_up = pmod(S - l - 2, 3);   // row y - 1
        // parity of (y + colour): P = 1 -> right neighbour q+1, left q
        constexpr int p = pmod(S - 1 - l + (l & 1), 2);
        st.win[l][s_new] = carry;
        const Vec<T, V>& up = st.win[l][s_up];
        const Vec<T, V>& mid = st.win[l][s_mid];
        const Vec<T, V>& dn = st.win[l][s_new];
        T extra;
        if constexpr (p == 1)
            extra = lane_shift<kWaveShl1>(mid.v[0]);
        else
            extra = lane_shift<kWaveShr1>(mid.v[V - 1]);
        const int y = x - 1 - l;
        const bool row_in = y >= 1 && y <= n;
        const int64_t q_lo = 1 - p, q_hi = (int64_t(n) - p) >> 1;
        Vec<T, V> out;
        // prev: this colour's previous version of row y, kept where nothing
        // is updated (the Dirichlet ring and rows outside the interior)
        const Vec<T, V>& fl = hf[l];
        auto update = [&](const Vec<T, V>& prev) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                T right = p ? (e + 1 < V ? mid.v[e + 1] : extra) : mid.v[e];
                T left = p ? mid.v[e] : (e > 0 ? mid.v[e - 1] : extra);
                T s = dn.v[e] + up.v[e];
                s = s + right;
                s = s + left;
                s = s - fl.v[e];
                T nv = T(0.25) * s;
                if constexpr (SOR) {
                    const T d = nv - prev.v[e];
                    const T w = omega * d;
                    nv = prev.v[e] + w;
                }
                if constexpr (EDGE) {
                    const int64_t q = q0 + e;
                    out.v[e] = blend(row_in && q >= q_lo && q <= q_hi, nv, prev.v[e]);
                } else {
                    out.v[e] = nv;  // every loaded point of an interior tile is interior
                }
            }
        };
        if constexpr (l == 0)
            update(st.red_in[pmod(S - 1, 2)]);
        else
            update(st.win[l - 1][pmod(S - l - 1, 3)]);
        carry = out;
    });
    if constexpr (EDGE || SOR) st.red_in[S & 1] = rin;
    const int y = x - L;
    if (y >= r0 && y <= r1) {
        // black (level L-1) and red (level L-2, still in level L-1's window)
        if constexpr (EDGE) {
            store_core<T, V>(yb + int64_t(y) * P, carry, q0, qc0, qc1, pmod(S - L + 1, 2), n);
            if (store_red)
                store_core<T, V>(yr + int64_t(y) * P, st.win[L - 1][pmod(S - L, 3)], q0, qc0,
                                 qc1, pmod(S - L, 2), n);
        } else if (in_core) {
            *reinterpret_cast<Vec<T, V>*>(yb + int64_t(y) * P + q0) = carry;
            if (store_red)
                *reinterpret_cast<Vec<T, V>*>(yr + int64_t(y) * P + q0) =
                    st.win[L - 1][pmod(S - L, 3)];
        }
    }
}

template <typename T, int V, int L, bool EDGE, bool SOR = false>
__device__ __forceinline__ void run_tile(FRing<T, V, L>& fr, const GridDesc<T>& a, int pass, int r0,
                                         int r1, int64_t qc0, int64_t qc1, bool store_red,
                                         T omega = T(1)) {
    const int lane = threadIdx.x;
    const int64_t q0 = qc0 - a.halo_q + int64_t(lane) * V;
    // column actually loaded: q0 clamped into the row (lanes past the grid
    // edge load a valid vector whose values only feed the halo)
    const int64_t qv = q0 < 0 ? 0 : (q0 > a.pitch - V ? a.pitch - V : q0);
    const bool in_core = q0 >= qc0 && q0 + V <= qc1;
    const T* xr = a.red[pass & 1];
    const T* xb = a.black[pass & 1];
    T* yr = a.red[(pass + 1) & 1];
    T* yb = a.black[(pass + 1) & 1];
    const int xs = max(0, r0 - L);
    const int xe = min(a.n + 1, r1 + L);
    const int x_last = r1 + L;
    Pipe<T, V, L> st;
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
        for (int r = 0; r < 3; ++r) st.win[l][r] = vzero<T, V>();
    st.red_in[0] = st.red_in[1] = vzero<T, V>();
    const int x0 = xs - xs % 6;
#pragma unroll
    for (int d = 0; d < prefetch_steps<T, L>(); ++d)
        st.in[d] = load_in<T, V, EDGE, SOR>(a, xr, xb, x0 + d, xs, xe, qv);
    for (int x = x0; x <= x_last; x += 6) {
        pipe_step<T, V, L, 0, EDGE, SOR>(st, fr, a, xr, xb, yr, yb, x + 0, xs, xe, r0, r1, q0, qv,
                                         qc0, qc1, in_core, store_red, omega);
        pipe_step<T, V, L, 1, EDGE, SOR>(st, fr, a, xr, xb, yr, yb, x + 1, xs, xe, r0, r1, q0, qv,
                                         qc0, qc1, in_core, store_red, omega);
        pipe_step<T, V, L, 2, EDGE, SOR>(st, fr, a, xr, xb, yr, yb, x + 2, xs, xe, r0, r1, q0, qv,
                                         qc0, qc1, in_core, store_red, omega);
        pipe_step<T, V, L, 3, EDGE, SOR>(st, fr, a, xr, xb, yr, yb, x + 3, xs, xe, r0, r1, q0, qv,
                                         qc0, qc1, in_core, store_red, omega);
        pipe_step<T, V, L, 4, EDGE, SOR>(st, fr, a, xr, xb, yr, yb, x + 4, xs, xe, r0, r1, q0, qv,
                                         qc0, qc1, in_core, store_red, omega);
        pipe_step<T, V, L, 5, EDGE, SOR>(st, fr, a, xr, xb, yr, yb, x + 5, xs, xe, r0, r1, q0, qv,
                                         qc0, qc1, in_core, store_red, omega);
    }
}

// A tile is interior when every point it loads (core plus halo, both
// colours) is an interior grid point: then no ring value needs to pass
// through, no red input row is needed and every core vector is stored whole.
// store_red: a pass reads only the black colour of its input (level 0
// recomputes every interior red point from black), so the red colour is
// written only by the launch's last pass, whose output leaves the kernel;
// the Dirichlet ring, the only red input that is read, is never written.
template <typename T, int V, int L, bool SOR = false>
__device__ __forceinline__ void process_tile(const GridDesc<T>& a, int pass, int tile,
                                             bool store_red, T omega = T(1)) {
    const int strip = tile / a.bands;
    const int band = tile - strip * a.bands;
    const int r0 = 1 + strip * a.rows;
    const int r1 = min(a.n, r0 + a.rows - 1);
    const int64_t qc0 = int64_t(band) * a.q_core;
    const int64_t qmax = int64_t(a.n >> 1);
    const int64_t qc1 = qc0 + a.q_core < qmax + 1 ? qc0 + a.q_core : qmax + 1;
    const int64_t qa = qc0 - a.halo_q;  // first loaded q
    const bool interior = r0 - L >= 1 && r1 + L <= a.n && qa >= 1 &&
                          qa + int64_t(kLanes) * V - 1 <= (int64_t(a.n) - 1) >> 1 &&
                          qc1 - qc0 == a.q_core;
    FRing<T, V, L>& fr = wave_fring<T, V, fring_rows<L>()>();
    if (interior)
        run_tile<T, V, L, false, SOR>(fr, a, pass, r0, r1, qc0, qc1, store_red, omega);
    else
        run_tile<T, V, L, true, SOR>(fr, a, pass, r0, r1, qc0, qc1, store_red, omega);
}

// Waits until the 3 x 3 neighbourhood of `tile` has finished pass-1.
// Returns false when the wait timed out or another wave reported an error.
template <typename T>
__device__ bool wait_deps(const GridDesc<T>& a, const Queue& qu, int pass, int tile) {
#ifdef RBGS_EMU_NO_WAIT  // the CPU emulation's planted mistake for the stamp check's own test
    return true;
#endif
    if (pass == 0) return true;
    const int lane = threadIdx.x;
    const int strip = tile / a.bands;
    const int band = tile - strip * a.bands;
    const int ns = strip + lane / 3 - 1;
    const int nb = band + lane % 3 - 1;
    const bool mine = lane < 9 && ns >= 0 && ns < a.strips && nb >= 0 && nb < a.bands;
    const int* flag = qu.progress + a.flag_base + (mine ? ns * a.bands + nb : 0);
    for (int polls = 0;; ++polls) {
        int v = mine ? __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : INT_MAX;
        if (__all(v >= pass)) break;
        if (polls >= qu.spin_limit) {
            if (lane == 0) __hip_atomic_store(qu.error, kErrTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        if ((polls & 255) == 255) {
            int e = __hip_atomic_load(qu.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__any(e != 0)) return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// Stamp check: every tile of the 3 x 3 neighbourhood has completed at least
// `pass` passes (the dependency wait saw that) and at most pass + 1: a
// neighbour at pass + 2 would have finished a pass that needs this item's
// output, i.e. written the buffer this item reads.  Called after the wait and
// again after the item's last write; false (and the error word set to
// kErrOrder) on a violation.
template <typename T>
__device__ bool stamps_ok(const GridDesc<T>& a, const Queue& qu, int pass, int tile) {
    const int lane = threadIdx.x;
    const int strip = tile / a.bands;
    const int band = tile - strip * a.bands;
    const int ns = strip + lane / 3 - 1;
    const int nb = band + lane % 3 - 1;
    const bool mine = lane < 9 && ns >= 0 && ns < a.strips && nb >= 0 && nb < a.bands &&
                      !(ns == strip && nb == band);
    const int* flag = qu.progress + a.flag_base + (mine ? ns * a.bands + nb : 0);
    const int v = mine ? __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : pass;
    const bool bad = v < pass || v > pass + 1;
    if (__any(bad)) {
        if (lane == 0) __hip_atomic_store(qu.error, kErrOrder, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
    }
    return true;
}

__device__ __forceinline__ unsigned long long realtime() {
    return (unsigned long long)__builtin_amdgcn_s_memrealtime();
}

// Runs one work item after its dependencies are met and publishes it.
// Returns false when the wave must leave (timeout or error elsewhere).
// DBG: the verification modes of `dm` apply (ticket: the item's ticket
// within the launch, for the trace).  SOR: the over-relaxed sweep with
// `omega`; it relaxes red from its old value, so every pass writes red.
template <typename T, int V, int L, bool DBG = false, bool SOR = false>
__device__ __forceinline__ bool run_item(const GridDesc<T>& g, const Queue& qu, int pass,
                                         int tile, const DebugModes& dm = DebugModes(),
                                         int ticket = 0, T omega = T(1)) {
    if (!wait_deps(g, qu, pass, tile)) return false;
    unsigned long long t0 = 0ull;
    if constexpr (DBG) {
        if (dm.trace) t0 = realtime();
        if (dm.stamp_check && !stamps_ok(g, qu, pass, tile)) return false;
    }
    if (qu.delay > 0) {
        // debug: a pseudo-random stall per work item (schedule stress)
        uint32_t loops = mix32(uint32_t(pass) * 0x9e3779b9u + uint32_t(g.flag_base + tile)) %
                         uint32_t(qu.delay + 1);
        for (uint32_t i = 0; i < loops; ++i) __builtin_amdgcn_s_sleep(127);
    }
    process_tile<T, V, L, SOR>(g, pass + qu.buf_offset, tile, SOR || pass == qu.passes - 1, omega);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if constexpr (DBG) {
        if (dm.stamp_check && !stamps_ok(g, qu, pass, tile)) return false;
        if (dm.trace && threadIdx.x == 0) {
            const long long k = dm.trace_base + ticket;
            if (k >= 0 && k < dm.trace_items) {
                unsigned long long* rec = dm.trace + k * kTraceWords;
                rec[0] = t0;
                rec[1] = realtime();
                rec[2] = ((unsigned long long)uint32_t(pass) << 32) | uint32_t(tile);
                rec[3] = ((unsigned long long)blockIdx.x << 32) | uint32_t(ticket);
            }
        }
    }
    if (threadIdx.x == 0 && g.flag_base + tile + 1 != qu.stall_tile)
        __hip_atomic_store(qu.progress + g.flag_base + tile, pass + 1, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// The ticket is read back with readfirstlane (lane 0 is the first active
// lane here), which makes it, and every tile coordinate and row index
// derived from it, a wave-uniform scalar: the row loops then run on scalar
// branches and the row addressing on the scalar unit.
__device__ __forceinline__ int next_ticket(const Queue& qu) {
    int tk = 0;
    if (threadIdx.x == 0) tk = __hip_atomic_fetch_add(qu.ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_amdgcn_readfirstlane(tk);
}

}  // namespace blocked
}  // namespace rbgs
