// Persistent, temporally blocked red-black sweep.
//
// The paper removes the global barrier between colours by running each
// colour of each stripe as a task that starts once its neighbouring stripes
// of the other colour are up to date (Algorithm 2, Section 2.3).  Here the
// same dependency rule orders tiles of a persistent kernel, and each tile
// does several half-sweeps per trip through HBM:
//
// * Work item = (pass p, tile t).  A pass fuses k full sweeps (L = 2k
//   half-sweeps).  Tiles are (row strip) x (q-column band) of the split
//   colour layout; one wave of 64 lanes owns one tile, each lane V
//   consecutive q-columns (a 16-byte vector) of the band.
// * Inside a tile the L half-sweeps are pipelined down the strip in
//   registers: at input row x, level l (colour l & 1, red first) updates row
//   x-1-l from the three other-colour rows that level l-1 produced last.
//   Rows are visited once per pass, so HBM sees one read of u and f and one
//   write of u per k sweeps.  Horizontal neighbours outside a lane's vector
//   come from the adjacent lane (cross-lane shuffle).
// * Overlapped tiling: a tile loads a halo of L rows above and below and
//   halo_q columns left and right; values there are recomputed redundantly,
//   lose validity by one point per level at the halo edge, and are never
//   written.  Passes alternate between two buffers (read X_p, write
//   Y_p = X_{p+1}), so a tile's writes cannot disturb neighbours that still
//   read the previous pass.
// * Dependencies: (p, t) may start when every tile in t's 3 x 3
//   neighbourhood has finished pass p-1 (progress flag >= p).  That covers
//   read-after-write on X_p and write-after-read on Y_p = X_{p-1}, the two
//   conflicts the task runtime serialises in Algorithm 2.  Flags are
//   published with an agent-scope release and read with acquire, so the
//   data crosses XCD L2 caches correctly.
// * Work items are handed out by one atomic ticket counter in (pass, tile)
//   order, a topological order of the dependency graph: a wave waits only
//   on items with smaller tickets, which running waves already hold, so no
//   co-residency of the grid is assumed and the kernel cannot deadlock.
// * Every wait is bounded (watchdog); on expiry the kernel records an error
//   word and every wave leaves, and the host returns RBGS_ETIMEOUT.
//
// Each point receives exactly the operations of Eq. (1) in the canonical
// order, from exactly the neighbour values a sequential red-black sweep
// would use, so the result equals the plain kernel bit for bit.
#include <climits>
#include <type_traits>

#include "rbgs_blocked.h"
#include "rbgs_internal.h"

namespace rbgs {
namespace {

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

template <typename T>
struct BlockedArgs {
    T* red[2];  // ping-pong buffers of the split iterate
    T* black[2];
    const T* f_red;
    const T* f_black;
    int n;
    int64_t pitch;
    T h2;
    int rows;     // interior rows per strip
    int halo_q;   // halo q-columns on each side (multiple of V)
    int q_core;   // q-columns written per band
    int strips, bands, ntiles, passes;
    int* progress;  // passes completed, per tile
    int* ticket;
    int* error;
    int spin_limit;
    int delay;
    int stall_tile;  // debug: tile + 1 whose progress is never published (0 = off)
};

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
// x-1 and f_black row x-2, their first use).  They are loaded two steps
// ahead; the right-hand sides of levels >= 2 (rows already brought in by
// levels 0 and 1) are loaded one step ahead.
template <typename T, int V>
struct StepIn {
    Vec<T, V> b, r, f0, f1;
};

// Whole-wave lane shifts through DPP (register to register, no LDS trip):
// from_next_lane gives lane i the value of lane i+1 (wave_shl:1), and
// from_prev_lane the value of lane i-1 (wave_shr:1).  The lane with no
// source keeps its own value; it lies in the tile's halo.
template <int CTRL>
__device__ __forceinline__ int dpp_shift(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
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

template <typename T, int V, int L>
struct Pipe {
    Vec<T, V> win[L][3];   // level l: other-colour rows (ring buffer of 3), version l-1
    Vec<T, V> red_in[2];   // red input rows x-1, x (ring values pass through level 0)
    StepIn<T, V> in[3];    // inputs of steps x, x+1, x+2 (slot x mod 3)
    Vec<T, V> fl[2][L];    // right-hand sides of levels >= 2 for steps x, x+1 (slot x mod 2)
};

// Loads never branch: row and column indices are clamped into the grid.
// A clamped load only ever feeds rows or columns outside the region the
// tile writes (the warm-up rows above xs, the drain rows below xe, lanes
// beyond the grid edge), whose values are recomputed garbage anyway.
__device__ __forceinline__ int clamp_row(int x, int lo, int hi) {
    return x < lo ? lo : (x > hi ? hi : x);
}

template <typename T, int V, bool EDGE>
__device__ __forceinline__ StepIn<T, V> load_in(const BlockedArgs<T>& a, const T* __restrict__ xr,
                                                const T* __restrict__ xb, int x, int64_t qv) {
    StepIn<T, V> in;
    const int64_t P = a.pitch;
    const int64_t row = int64_t(clamp_row(x, 0, a.n + 1)) * P + qv;
    in.b = vload<T, V>(xb + row);
    // red input values matter only where they pass through unchanged
    // (the ring); interior tiles never see the ring
    if constexpr (EDGE)
        in.r = vload<T, V>(xr + row);
    else
        in.r = vzero<T, V>();
    in.f0 = vload<T, V>(a.f_red + int64_t(clamp_row(x - 1, 1, a.n)) * P + qv);
    in.f1 = vload<T, V>(a.f_black + int64_t(clamp_row(x - 2, 1, a.n)) * P + qv);
    return in;
}

template <typename T, int V, int L>
__device__ __forceinline__ void load_fl(const BlockedArgs<T>& a, Vec<T, V> (&dst)[L], int x,
                                        int64_t qv) {
    static_for<2, L>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        const int y = clamp_row(x - 1 - l, 1, a.n);
        dst[l] = vload<T, V>(((l & 1) ? a.f_black : a.f_red) + int64_t(y) * a.pitch + qv);
    });
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
// ring-buffer slots (period 3) and the row parities (period 2).
template <typename T, int V, int L, int S, bool EDGE>
__device__ __forceinline__ void pipe_step(Pipe<T, V, L>& st, const BlockedArgs<T>& a,
                                          const T* __restrict__ xr, const T* __restrict__ xb,
                                          T* __restrict__ yr, T* __restrict__ yb, int x, int xs,
                                          int xe, int r0, int r1, int64_t q0, int64_t qv,
                                          int64_t qc0, int64_t qc1, bool in_core) {
    const int n = a.n;
    const int64_t P = a.pitch;
    const StepIn<T, V> cur = st.in[S % 3];
    // prefetch: step x+2's rows into the slot step x-1 used, step x+1's
    // right-hand sides into the other half of the double buffer
    st.in[(S + 2) % 3] = load_in<T, V, EDGE>(a, xr, xb, x + 2, qv);
    load_fl<T, V, L>(a, st.fl[(S + 1) % 2], x + 1, qv);
    const Vec<T, V> bin = cur.b;
    const Vec<T, V> rin = cur.r;
    auto rhs = [&](auto lc) -> const Vec<T, V>& {
        constexpr int l = decltype(lc)::value;
        if constexpr (l == 0)
            return cur.f0;
        else if constexpr (l == 1)
            return cur.f1;
        else
            return st.fl[S % 2][l];
    };
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
        auto update = [&](const Vec<T, V>& prev) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                T right = p ? (e + 1 < V ? mid.v[e + 1] : extra) : mid.v[e];
                T left = p ? mid.v[e] : (e > 0 ? mid.v[e - 1] : extra);
                T s = dn.v[e] + up.v[e];
                s = s + right;
                s = s + left;
                T t = a.h2 * rhs(lc).v[e];
                s = s - t;
                T nv = T(0.25) * s;
                if constexpr (EDGE) {
                    const int64_t q = q0 + e;
                    out.v[e] = (row_in && q >= q_lo && q <= q_hi) ? nv : prev.v[e];
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
    if constexpr (EDGE) st.red_in[S & 1] = rin;
    const int y = x - L;
    if (y >= r0 && y <= r1) {
        // black (level L-1) and red (level L-2, still in level L-1's window)
        if constexpr (EDGE) {
            store_core<T, V>(yb + int64_t(y) * P, carry, q0, qc0, qc1, pmod(S - L + 1, 2), n);
            store_core<T, V>(yr + int64_t(y) * P, st.win[L - 1][pmod(S - L, 3)], q0, qc0, qc1,
                             pmod(S - L, 2), n);
        } else if (in_core) {
            *reinterpret_cast<Vec<T, V>*>(yb + int64_t(y) * P + q0) = carry;
            *reinterpret_cast<Vec<T, V>*>(yr + int64_t(y) * P + q0) = st.win[L - 1][pmod(S - L, 3)];
        }
    }
}

template <typename T, int V, int L, bool EDGE>
__device__ __forceinline__ void run_tile(const BlockedArgs<T>& a, int pass, int r0, int r1,
                                         int64_t qc0, int64_t qc1) {
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
    st.in[0] = load_in<T, V, EDGE>(a, xr, xb, x0, qv);
    st.in[1] = load_in<T, V, EDGE>(a, xr, xb, x0 + 1, qv);
    load_fl<T, V, L>(a, st.fl[0], x0, qv);
    for (int x = x0; x <= x_last; x += 6) {
        pipe_step<T, V, L, 0, EDGE>(st, a, xr, xb, yr, yb, x + 0, xs, xe, r0, r1, q0, qv, qc0, qc1, in_core);
        pipe_step<T, V, L, 1, EDGE>(st, a, xr, xb, yr, yb, x + 1, xs, xe, r0, r1, q0, qv, qc0, qc1, in_core);
        pipe_step<T, V, L, 2, EDGE>(st, a, xr, xb, yr, yb, x + 2, xs, xe, r0, r1, q0, qv, qc0, qc1, in_core);
        pipe_step<T, V, L, 3, EDGE>(st, a, xr, xb, yr, yb, x + 3, xs, xe, r0, r1, q0, qv, qc0, qc1, in_core);
        pipe_step<T, V, L, 4, EDGE>(st, a, xr, xb, yr, yb, x + 4, xs, xe, r0, r1, q0, qv, qc0, qc1, in_core);
        pipe_step<T, V, L, 5, EDGE>(st, a, xr, xb, yr, yb, x + 5, xs, xe, r0, r1, q0, qv, qc0, qc1, in_core);
    }
}

// A tile is interior when every point it loads (core plus halo, both
// colours) is an interior grid point: then no ring value needs to pass
// through, no red input row is needed and every core vector is stored whole.
template <typename T, int V, int L>
__device__ __forceinline__ void process_tile(const BlockedArgs<T>& a, int pass, int tile) {
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
    if (interior)
        run_tile<T, V, L, false>(a, pass, r0, r1, qc0, qc1);
    else
        run_tile<T, V, L, true>(a, pass, r0, r1, qc0, qc1);
}

// Waits until the 3 x 3 neighbourhood of `tile` has finished pass-1.
// Returns false when the wait timed out or another wave reported an error.
template <typename T>
__device__ bool wait_deps(const BlockedArgs<T>& a, int pass, int tile) {
    if (pass == 0) return true;
    const int lane = threadIdx.x;
    const int strip = tile / a.bands;
    const int band = tile - strip * a.bands;
    const int ns = strip + lane / 3 - 1;
    const int nb = band + lane % 3 - 1;
    const bool mine = lane < 9 && ns >= 0 && ns < a.strips && nb >= 0 && nb < a.bands;
    const int* flag = a.progress + (mine ? ns * a.bands + nb : 0);
    for (int polls = 0;; ++polls) {
        int v = mine ? __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : INT_MAX;
        if (__all(v >= pass)) break;
        if (polls >= a.spin_limit) {
            if (lane == 0) __hip_atomic_store(a.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        if ((polls & 255) == 255) {
            int e = __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__any(e != 0)) return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

__device__ __forceinline__ uint32_t mix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    return h;
}

template <typename T, int V, int L>
__global__ __launch_bounds__(kLanes) void k_blocked(BlockedArgs<T> a) {
    const int lane = threadIdx.x;
    const int total = a.passes * a.ntiles;
    for (;;) {
        int tk = 0;
        if (lane == 0) tk = __hip_atomic_fetch_add(a.ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        tk = __shfl(tk, 0);
        if (tk >= total) break;
        const int pass = tk / a.ntiles;
        const int tile = tk - pass * a.ntiles;
        if (!wait_deps(a, pass, tile)) break;
        if (a.delay > 0) {
            // debug: a pseudo-random stall per work item (schedule stress)
            uint32_t loops = mix32(uint32_t(pass) * 0x9e3779b9u + uint32_t(tile)) % uint32_t(a.delay + 1);
            for (uint32_t i = 0; i < loops; ++i) __builtin_amdgcn_s_sleep(127);
        }
        process_tile<T, V, L>(a, pass, tile);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0 && tile + 1 != a.stall_tile)
            __hip_atomic_store(a.progress + tile, pass + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct Geometry {
    int V, L, halo_q, q_core, rows, strips, bands, ntiles;
};

Geometry geometry(int n, int elem_bytes, int fuse, int rows) {
    Geometry g;
    g.V = 16 / elem_bytes;
    g.L = 2 * fuse;
    const int need = g.L / 2 + 1;                      // validity loss per side, in q
    g.halo_q = (need + g.V - 1) / g.V * g.V;
    g.q_core = kLanes * g.V - 2 * g.halo_q;
    g.rows = rows;
    g.strips = (n + rows - 1) / rows;
    g.bands = int(((int64_t(n) >> 1) + 1 + g.q_core - 1) / g.q_core);
    g.ntiles = g.strips * g.bands;
    return g;
}

constexpr int kMinRows = 8;
constexpr int kMaxFuse = 4;

int max_tiles(int n) {
    // the smallest tile has kMinRows rows and the narrowest core (FP32? no:
    // FP64, V = 2, fuse = kMaxFuse): bound both dimensions generously
    int64_t strips = (int64_t(n) + kMinRows - 1) / kMinRows;
    int64_t bands = ((int64_t(n) >> 1) + 1 + 63) / 64 + 1;
    return int(strips * bands);
}

int default_rows(int n, int L) {
    int r = 256;
    while (r > 2 * L && r > kMinRows && r * 4 > n) r >>= 1;
    return r < L ? L : r;
}

template <typename T, int V, int L>
hipError_t launch_k(const BlockedArgs<T>& a, hipStream_t s) {
    static int per_cu = 0;
    static int cus = 0;
    if (per_cu == 0) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_blocked<T, V, L>, kLanes, 0);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
    }
    int64_t total = int64_t(a.passes) * a.ntiles;
    int64_t grid = int64_t(cus) * per_cu;
    if (grid > total) grid = total;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((k_blocked<T, V, L>), dim3(unsigned(grid)), dim3(kLanes), 0, s, a);
    return hipGetLastError();
}

template <typename T, int V>
hipError_t launch_by_fuse(int fuse, const BlockedArgs<T>& a, hipStream_t s) {
    switch (fuse) {
        case 1: return launch_k<T, V, 2>(a, s);
        case 2: return launch_k<T, V, 4>(a, s);
        case 3: return launch_k<T, V, 6>(a, s);
        default: return launch_k<T, V, 8>(a, s);
    }
}

}  // namespace

size_t blocked_state_bytes(int n, int) { return 256 + align256(size_t(max_tiles(n)) * 4); }

int validate_blocked_opts(int fuse, int tile_rows, int tile_cols, std::string* why) {
    if (fuse > kMaxFuse) {
        *why = "fuse must be in [1, 4] (0 = default)";
        return RBGS_EINVAL;
    }
    if (tile_rows != 0 && tile_rows < kMinRows) {
        *why = "tile_rows must be >= 8 (0 = default)";
        return RBGS_EINVAL;
    }
    if (tile_cols != 0) {
        *why = "tile_cols must be 0: a tile is one wave wide (64 lanes x 16 bytes)";
        return RBGS_EINVAL;
    }
    return RBGS_OK;
}

int auto_kernel(int n, size_t) { return n >= 1024 ? RBGS_KERNEL_BLOCKED : RBGS_KERNEL_PLAIN; }

BlockedParams blocked_params(int n, size_t, const rbgs_sweep_opts* o) {
    BlockedParams bp;
    bp.fuse = (o && o->fuse > 0) ? o->fuse : kMaxFuse;
    bp.tile_rows = (o && o->tile_rows > 0) ? o->tile_rows : default_rows(n, 2 * bp.fuse);
    if (bp.tile_rows < 2 * bp.fuse) bp.tile_rows = 2 * bp.fuse;  // halo rows must fit one strip
    bp.delay = o ? o->debug_delay : 0;
    bp.spin_limit = (o && o->debug_spin_limit > 0) ? o->debug_spin_limit : kDefaultSpinLimit;
    bp.stall_tile = o ? o->debug_stall_tile : 0;
    return bp;
}

template <typename T>
hipError_t run_blocked(T* const buf_red[2], T* const buf_black[2], const T* f_red,
                       const T* f_black, int n, int64_t pitch, T h2, int nsweeps,
                       const BlockedParams& bp, void* state, size_t state_bytes, hipStream_t s,
                       int* launches) {
    constexpr int V = 16 / int(sizeof(T));
    const int k = bp.fuse;
    const int passes = nsweeps / k;
    const int rem = nsweeps - passes * k;
    const size_t colour_bytes = size_t(n + 2) * size_t(pitch) * sizeof(T);
    *launches = 0;
    hipError_t e;
    if (passes > 0) {
        Geometry g = geometry(n, int(sizeof(T)), k, bp.tile_rows);
        if (g.ntiles > max_tiles(n)) return hipErrorInvalidValue;
        // the second buffer needs the Dirichlet ring: start from a full copy
        e = hipMemcpyAsync(buf_red[1], buf_red[0], colour_bytes, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(buf_black[1], buf_black[0], colour_bytes, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        // tickets are ints: split very long runs into launches of at most
        // 2^30 work items, each starting from freshly zeroed flags
        const int max_passes = int((int64_t(1) << 30) / g.ntiles) > 0
                                   ? int((int64_t(1) << 30) / g.ntiles) : 1;
        int done = 0;
        while (done < passes) {
            const int chunk = passes - done < max_passes ? passes - done : max_passes;
            e = launch_zero(state, 256 + size_t(g.ntiles) * 4, s);
            if (e != hipSuccess) return e;
            const int in = done & 1;  // buffer holding the input of this chunk
            BlockedArgs<T> a;
            a.red[0] = buf_red[in];
            a.red[1] = buf_red[in ^ 1];
            a.black[0] = buf_black[in];
            a.black[1] = buf_black[in ^ 1];
            a.f_red = f_red;
            a.f_black = f_black;
            a.n = n;
            a.pitch = pitch;
            a.h2 = h2;
            a.rows = g.rows;
            a.halo_q = g.halo_q;
            a.q_core = g.q_core;
            a.strips = g.strips;
            a.bands = g.bands;
            a.ntiles = g.ntiles;
            a.passes = chunk;
            char* base = static_cast<char*>(state);
            a.ticket = reinterpret_cast<int*>(base);
            a.error = reinterpret_cast<int*>(base + 64);
            a.progress = reinterpret_cast<int*>(base + 256);
            a.spin_limit = bp.spin_limit;
            a.delay = bp.delay;
            a.stall_tile = bp.stall_tile;
            e = launch_by_fuse<T, V>(k, a, s);
            if (e != hipSuccess) return e;
            *launches += 1;
            done += chunk;
        }
        if (passes & 1) {
            e = hipMemcpyAsync(buf_red[0], buf_red[1], colour_bytes, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return e;
            e = hipMemcpyAsync(buf_black[0], buf_black[1], colour_bytes, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return e;
        }
    } else {
        // no persistent launch: make sure a stale error word cannot be reported
        e = launch_zero(state, 256, s);
        if (e != hipSuccess) return e;
    }
    for (int it = 0; it < rem; ++it) {
        e = launch_half_sweep<T>(buf_red[0], buf_black[0], f_red, n, pitch, h2, 0, 0, s);
        if (e != hipSuccess) return e;
        e = launch_half_sweep<T>(buf_black[0], buf_red[0], f_black, n, pitch, h2, 1, 0, s);
        if (e != hipSuccess) return e;
        *launches += 2;
    }
    return hipSuccess;
}

template hipError_t run_blocked<double>(double* const[2], double* const[2], const double*,
                                        const double*, int, int64_t, double, int,
                                        const BlockedParams&, void*, size_t, hipStream_t, int*);
template hipError_t run_blocked<float>(float* const[2], float* const[2], const float*,
                                       const float*, int, int64_t, float, int,
                                       const BlockedParams&, void*, size_t, hipStream_t, int*);

int blocked_check_error(void* state, hipStream_t s, std::string* why) {
    int err = 0;
    hipError_t e = hipMemcpyAsync(&err, static_cast<char*>(state) + 64, sizeof err,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        *why = std::string("reading the persistent kernel's error word: ") + hipGetErrorString(e);
        return RBGS_EHIP;
    }
    if (err != 0) {
        *why = "a tile dependency wait in the persistent kernel timed out";
        return RBGS_ETIMEOUT;
    }
    return RBGS_OK;
}

}  // namespace rbgs
