// Persistent, temporally blocked red-black sweep.
//
// The paper removes the global barrier between colours by running each
// colour of each stripe as a task that starts once its neighbouring stripes
// of the other colour are up to date (Algorithm 2, Section 2.3).  Here the
// same dependency rule orders tiles of a persistent kernel, and each tile
// does several half-sweeps per trip through HBM:
//
// * Work item = (pass p, tile t).  A pass fuses k full sweeps (L = 2k
//   half-sweeps, k = 1..10).  Tiles are (row strip) x (q-column band) of the split
//   colour layout; one wave of 64 lanes owns one tile, each lane V
//   consecutive q-columns (a 16-byte vector) of the band.
// * Inside a tile the L half-sweeps are pipelined down the strip in
//   registers: at input row x, level l (colour l & 1, red first) updates row
//   x-1-l from the three other-colour rows that level l-1 produced last.
//   Rows are visited once per pass, so HBM sees one read of u (its black
//   colour: level 0 recomputes red from it) and of f, and one write of
//   black, per k sweeps; red is written by the last pass of a launch only.  Horizontal neighbours outside a lane's vector
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
#include <type_traits>

#include "blocked_pipeline.h"
#include "rbgs_blocked.h"
#include "rbgs_internal.h"

namespace rbgs {
namespace {

using namespace blocked;

template <typename T, int V, int L>
__global__ __launch_bounds__(kLanes) void k_blocked(GridDesc<T> g, Queue qu) {
    if (stopped(qu)) return;
    const int total = qu.passes * g.ntiles;
    for (;;) {
        const int tk = next_ticket(qu);
        if (tk >= total) break;
        const int pass = tk / g.ntiles;
        if (!run_item<T, V, L>(g, qu, pass, tk - pass * g.ntiles)) break;
    }
}

// A launch whose passes differ in depth by one sweep: passes [0, n_hi) run
// L1 / 2 fused sweeps, the rest L2 / 2 = L1 / 2 - 1, over the same tiles
// (the host merges only when both depths give the same tile geometry), so
// the shallower passes follow the deeper ones without a launch boundary:
// the first of them start while the last deeper ones drain, instead of the
// second launch ramping up from an idle GPU.  The dependency rule is the
// same for every pass (3 x 3 neighbourhood, pass p - 1), and both pipelines
// share the wave's LDS ring.
template <typename T, int V, int L1, int L2>
__global__ __launch_bounds__(kLanes) void k_blocked2(GridDesc<T> g, Queue qu, int n_hi) {
    static_assert(fring_rows<L1>() == fring_rows<L2>(), "the two depths share one LDS ring");
    if (stopped(qu)) return;
    const int total = qu.passes * g.ntiles;
    for (;;) {
        const int tk = next_ticket(qu);
        if (tk >= total) break;
        const int pass = tk / g.ntiles;
        const int tile = tk - pass * g.ntiles;
        const bool ok = pass < n_hi ? run_item<T, V, L1>(g, qu, pass, tile)
                                    : run_item<T, V, L2>(g, qu, pass, tile);
        if (!ok) break;
    }
}

// Red-black SOR (an extension: the paper's method is omega = 1) through the
// same tiles: every level relaxes from the point's previous version, so red
// is read and written by every pass (32 B per point and pass in FP64).
template <typename T, int V, int L>
__global__ __launch_bounds__(kLanes) void k_blocked_sor(GridDesc<T> g, Queue qu, T omega) {
    if (stopped(qu)) return;
    const int total = qu.passes * g.ntiles;
    for (;;) {
        const int tk = next_ticket(qu);
        if (tk >= total) break;
        const int pass = tk / g.ntiles;
        if (!run_item<T, V, L, false, true>(g, qu, pass, tk - pass * g.ntiles, DebugModes(), 0, omega))
            break;
    }
}

// The same kernel with the verification modes (tile order, stamp check,
// trace); launched only when a caller asks for one of them.
template <typename T, int V, int L>
__global__ __launch_bounds__(kLanes) void k_blocked_dbg(GridDesc<T> g, Queue qu, DebugModes dm) {
    if (stopped(qu)) return;
    const int total = qu.passes * g.ntiles;
    for (;;) {
        const int tk = next_ticket(qu);
        if (tk >= total) break;
        const int pass = tk / g.ntiles;
        const int tile = tile_of_ticket(dm, g.ntiles, pass, tk - pass * g.ntiles);
        if (!run_item<T, V, L, true>(g, qu, pass, tile, dm, tk)) break;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
// omega != 1 launches the SOR kernel (FP64 only: the callers refuse FP32
// SOR), dm the verification kernel; else the production kernel.
template <typename T, int V, int L>
hipError_t launch_k(const GridDesc<T>& g, const Queue& qu, const DebugModes* dm, T omega,
                    hipStream_t s) {
    constexpr bool kSor = std::is_same<T, double>::value;
    const bool sor = omega != T(1);
    if (sor && (!kSor || dm)) return hipErrorInvalidValue;
    int per_cu = 0, cus = 0;
    const void* k = dm ? reinterpret_cast<const void*>(&k_blocked_dbg<T, V, L>)
                       : reinterpret_cast<const void*>(&k_blocked<T, V, L>);
    if constexpr (kSor)
        if (sor) k = reinterpret_cast<const void*>(&k_blocked_sor<T, V, L>);
    hipError_t e = persistent_occupancy(k, &per_cu, &cus);
    if (e != hipSuccess) return e;
    int64_t total = int64_t(qu.passes) * g.ntiles;
    int64_t grid = int64_t(cus) * per_cu;
    if (grid > total) grid = total;
    if (grid < 1) grid = 1;
    if (dm) {
        hipLaunchKernelGGL((k_blocked_dbg<T, V, L>), dim3(unsigned(grid)), dim3(kLanes), 0, s, g, qu, *dm);
    } else if (sor) {
        if constexpr (kSor)
            hipLaunchKernelGGL((k_blocked_sor<T, V, L>), dim3(unsigned(grid)), dim3(kLanes), 0, s, g,
                               qu, omega);
    } else {
        hipLaunchKernelGGL((k_blocked<T, V, L>), dim3(unsigned(grid)), dim3(kLanes), 0, s, g, qu);
    }
    return hipGetLastError();
}

template <typename T, int V, int L1, int L2>
hipError_t launch_k2(const GridDesc<T>& g, const Queue& qu, int n_hi, hipStream_t s) {
    int per_cu = 0, cus = 0;
    hipError_t e = persistent_occupancy(reinterpret_cast<const void*>(&k_blocked2<T, V, L1, L2>),
                                        &per_cu, &cus);
    if (e != hipSuccess) return e;
    int64_t total = int64_t(qu.passes) * g.ntiles;
    int64_t grid = int64_t(cus) * per_cu;
    if (grid > total) grid = total;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((k_blocked2<T, V, L1, L2>), dim3(unsigned(grid)), dim3(kLanes), 0, s, g, qu,
                       n_hi);
    return hipGetLastError();
}

// Depth pairs (fuse, fuse - 1) whose pipelines share a ring height; the
// others run as two launches.
bool mergeable_fuse(int fuse) { return fuse == 3 || fuse == 5 || fuse == 6 || fuse == 7; }

template <typename T, int V>
hipError_t launch_by_fuse2(int fuse, const GridDesc<T>& g, const Queue& qu, int n_hi, hipStream_t s) {
    switch (fuse) {
        case 3: return launch_k2<T, V, 6, 4>(g, qu, n_hi, s);
        case 5: return launch_k2<T, V, 10, 8>(g, qu, n_hi, s);
        case 6: return launch_k2<T, V, 12, 10>(g, qu, n_hi, s);
        case 7: return launch_k2<T, V, 14, 12>(g, qu, n_hi, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int V>
hipError_t launch_by_fuse(int fuse, const GridDesc<T>& g, const Queue& qu, const DebugModes* dm,
                          T omega, hipStream_t s) {
    switch (fuse) {
        case 1: return launch_k<T, V, 2>(g, qu, dm, omega, s);
        case 2: return launch_k<T, V, 4>(g, qu, dm, omega, s);
        case 3: return launch_k<T, V, 6>(g, qu, dm, omega, s);
        case 4: return launch_k<T, V, 8>(g, qu, dm, omega, s);
        case 5: return launch_k<T, V, 10>(g, qu, dm, omega, s);
        case 6: return launch_k<T, V, 12>(g, qu, dm, omega, s);
        case 7: return launch_k<T, V, 14>(g, qu, dm, omega, s);
        case 8: return launch_k<T, V, 16>(g, qu, dm, omega, s);
        case 9: return launch_k<T, V, 18>(g, qu, dm, omega, s);
        default: return launch_k<T, V, 20>(g, qu, dm, omega, s);
    }
}

}  // namespace

hipError_t persistent_occupancy(const void* kernel, int* per_cu, int* cus) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kernel, kLanes, 0);
    if (e != hipSuccess) return e;
    if (*per_cu < 1) *per_cu = 1;
    return hipSuccess;
}

namespace {
template <typename T>
const void* blocked_kernel_of(int fuse) {
    constexpr int V = 16 / int(sizeof(T));
    switch (fuse) {
        case 1: return reinterpret_cast<const void*>(&k_blocked<T, V, 2>);
        case 2: return reinterpret_cast<const void*>(&k_blocked<T, V, 4>);
        case 3: return reinterpret_cast<const void*>(&k_blocked<T, V, 6>);
        case 4: return reinterpret_cast<const void*>(&k_blocked<T, V, 8>);
        case 5: return reinterpret_cast<const void*>(&k_blocked<T, V, 10>);
        case 6: return reinterpret_cast<const void*>(&k_blocked<T, V, 12>);
        case 7: return reinterpret_cast<const void*>(&k_blocked<T, V, 14>);
        case 8: return reinterpret_cast<const void*>(&k_blocked<T, V, 16>);
        case 9: return reinterpret_cast<const void*>(&k_blocked<T, V, 18>);
        default: return reinterpret_cast<const void*>(&k_blocked<T, V, 20>);
    }
}
}  // namespace

int blocked_wave_slots(size_t elem_bytes, int fuse) {
    const void* k = elem_bytes == 8 ? blocked_kernel_of<double>(fuse) : blocked_kernel_of<float>(fuse);
    int per_cu = 0, cus = 0;
    if (persistent_occupancy(k, &per_cu, &cus) != hipSuccess || cus < 1) {
        (void)hipGetLastError();
        return 1024;
    }
    return per_cu * cus;
}

size_t blocked_state_bytes(int n, int) { return 256 + align256(size_t(max_tiles(n)) * 4); }

int validate_blocked_opts(int fuse, int tile_rows, int tile_cols, std::string* why) {
    if (fuse > kMaxFuse) {
        *why = "fuse must be in [1, 10] (0 = default)";
        return RBGS_EINVAL;
    }
    if (tile_rows != 0 && (tile_rows < kMinRows || tile_rows > kMaxRows)) {
        *why = "tile_rows must be in [8, 65536] (0 = default)";
        return RBGS_EINVAL;
    }
    if (tile_cols != 0) {
        *why = "tile_cols must be 0: a tile is one wave wide (64 lanes x 16 bytes)";
        return RBGS_EINVAL;
    }
    return RBGS_OK;
}

int validate_blocked_debug(const rbgs_sweep_opts* o, std::string* why) {
    if (!o) return RBGS_OK;
    if (o->debug_tile_order < 0 || o->debug_tile_order > 2) {
        *why = "debug_tile_order must be 0 (as numbered), 1 (reversed) or 2 (seeded permutation)";
        return RBGS_EINVAL;
    }
    if (o->debug_stamp_check != 0 && o->debug_stamp_check != 1) {
        *why = "debug_stamp_check must be 0 or 1";
        return RBGS_EINVAL;
    }
    if (o->debug_trace_items < 0 || (o->debug_trace_items > 0) != (o->debug_trace != nullptr)) {
        *why = "debug_trace and debug_trace_items > 0 go together (both unset: no trace)";
        return RBGS_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(o->debug_trace) % 8 != 0) {
        *why = "debug_trace must be 8-byte aligned";
        return RBGS_EINVAL;
    }
    return RBGS_OK;
}

// Kernel choice measured on MI355X (time per sweep over thousands of
// sweeps): the resident band kernel up to n = 384 (FP64) or 768 (FP32),
// where it holds the grid in registers; above that the persistent blocked
// kernel, except FP32 below 1536, where it has too few tiles and the plain
// kernel is as fast.  A handful of sweeps does not pay for a persistent
// launch.
int auto_kernel(int n, size_t elem_bytes, int nsweeps) {
    if (nsweeps < 8) return RBGS_KERNEL_PLAIN;
    if (elem_bytes == 8) return n <= 384 ? RBGS_KERNEL_RESIDENT : RBGS_KERNEL_BLOCKED;
    if (n <= 768) return RBGS_KERNEL_RESIDENT;
    return n < 1536 ? RBGS_KERNEL_PLAIN : RBGS_KERNEL_BLOCKED;
}

BlockedParams blocked_params(int n, size_t elem_bytes, const rbgs_sweep_opts* o) {
    BlockedParams bp;
    bp.fuse = (o && o->fuse > 0) ? o->fuse : default_fuse(int(elem_bytes), n);
    bp.tile_rows = (o && o->tile_rows > 0)
                       ? o->tile_rows
                       : single_grid_rows(n, 2 * bp.fuse, int(elem_bytes),
                                          blocked_wave_slots(elem_bytes, bp.fuse));
    if (bp.tile_rows < 2 * bp.fuse) bp.tile_rows = 2 * bp.fuse;  // halo rows must fit one strip
    bp.delay = o ? o->debug_delay : 0;
    bp.spin_limit = (o && o->debug_spin_limit > 0) ? o->debug_spin_limit : kDefaultSpinLimit;
    bp.stall_tile = o ? o->debug_stall_tile : 0;
    if (o) {
        bp.order = o->debug_tile_order;
        bp.seed = o->debug_seed;
        bp.stamp_check = o->debug_stamp_check;
        bp.trace = reinterpret_cast<unsigned long long*>(o->debug_trace);
        bp.trace_items = o->debug_trace_items;
    }
    return bp;
}

template <typename T>
hipError_t run_blocked(T* const buf_red[2], T* const buf_black[2], const T* f_red,
                       const T* f_black, int n, int64_t pitch, T h2, int nsweeps,
                       const BlockedParams& bp, void* state, size_t state_bytes, hipStream_t s,
                       int* launches, hipEvent_t ev_begin, hipEvent_t ev_end,
                       int* persistent_launches, int* passes_done, int* timed_fuse, T omega,
                       bool result_in_last) {
    constexpr int V = 16 / int(sizeof(T));
    *persistent_launches = 0;
    *passes_done = 0;
    *timed_fuse = 0;
    *launches = 0;
    const int k = bp.fuse;
    const size_t colour_bytes = size_t(n + 2) * size_t(pitch) * sizeof(T);
    char* base = static_cast<char*>(state);
    // the error word starts at zero once per call (once per solve for the
    // rounds of a captured graph); tickets and flags before every launch (an
    // error seen by an earlier launch must survive)
    hipError_t e = bp.keep_error ? hipSuccess : launch_zero(base, 256, s);
    if (e != hipSuccess) return e;
    if (nsweeps < 2) {  // a single sweep does not pay for a persistent launch
        for (int it = 0; it < nsweeps; ++it) {
            e = launch_half_sweep<T>(buf_red[0], buf_black[0], f_red, n, pitch, h2, 0, 0, s,
                                     bp.stop, omega);
            if (e != hipSuccess) return e;
            e = launch_half_sweep<T>(buf_black[0], buf_red[0], f_black, n, pitch, h2, 1, 0, s,
                                     bp.stop, omega);
            if (e != hipSuccess) return e;
            *launches += 2;
        }
        return hipSuccess;
    }
    // ceil(nsweeps / k) passes whose depths differ by at most one: n_hi of
    // depth d_hi, then n_lo of depth d_hi - 1 (200 sweeps at k = 7: 26 x 7 +
    // 3 x 6), rather than full passes and one much shallower remainder pass,
    // whose fixed cost per pass buys few sweeps
    const int total_passes = (nsweeps + k - 1) / k;
    const int d_hi = (nsweeps + total_passes - 1) / total_passes;
    const int n_hi = nsweeps - total_passes * (d_hi - 1);
    const int n_lo = total_passes - n_hi;
    // The second buffer needs the Dirichlet ring, and only that: a pass
    // writes every interior black point of its output before the next pass
    // reads it, and reads no interior red point (red is written by the last
    // pass of a launch only).
    e = launch_copy_ring(buf_red[1], buf_black[1], buf_red[0], buf_black[0], n, pitch,
                         int(sizeof(T)), s);
    if (e != hipSuccess) return e;
    int cur = 0;  // buffer holding the current iterate
    bool started = false;
    // `count` passes of `fuse` sweeps starting from buffer cur; `timed`
    // launches are bracketed by the events and counted.  split >= 0: one
    // merged launch of `count` passes, the first `split` of depth `fuse`,
    // the rest one sweep shallower (the caller checked it applies).
    auto run_passes = [&](int fuse, int count, bool timed, int split = -1) -> hipError_t {
        const int rows = bp.tile_rows < 2 * fuse ? 2 * fuse : bp.tile_rows;
        const Geometry geo = geometry(n, int(sizeof(T)), fuse, rows);
        if (geo.ntiles < 1 || geo.ntiles > max_tiles(n)) return hipErrorInvalidValue;
        // tickets are ints: split very long runs into launches of at most
        // 2^30 work items, each starting from freshly zeroed flags
        const int max_passes = int((int64_t(1) << 30) / geo.ntiles) > 0
                                   ? int((int64_t(1) << 30) / geo.ntiles) : 1;
        if (split >= 0 && count > max_passes) return hipErrorInvalidValue;
        int done = 0;
        while (done < count) {
            const int chunk = count - done < max_passes ? count - done : max_passes;
            hipError_t r = launch_zero(base, 64, s);  // ticket
            if (r != hipSuccess) return r;
            r = launch_zero(base + 256, size_t(geo.ntiles) * 4, s);  // progress flags
            if (r != hipSuccess) return r;
            GridDesc<T> g;
            g.red[0] = buf_red[cur];
            g.red[1] = buf_red[cur ^ 1];
            g.black[0] = buf_black[cur];
            g.black[1] = buf_black[cur ^ 1];
            g.f_red = f_red;
            g.f_black = f_black;
            g.n = n;
            g.pitch = pitch;
            g.h2 = h2;
            g.rows = geo.rows;
            g.halo_q = geo.halo_q;
            g.q_core = geo.q_core;
            g.strips = geo.strips;
            g.bands = geo.bands;
            g.ntiles = geo.ntiles;
            g.flag_base = 0;
            g.omega = T(1);
            Queue qu;
            qu.passes = chunk;
            qu.ticket = reinterpret_cast<int*>(base);
            qu.error = reinterpret_cast<int*>(base + 64);
            qu.progress = reinterpret_cast<int*>(base + 256);
            qu.spin_limit = bp.spin_limit;
            qu.delay = bp.delay;
            qu.stall_tile = bp.stall_tile;
            qu.buf_offset = 0;
            qu.stop = bp.stop;
            DebugModes dm;
            dm.order = bp.order;
            dm.seed = bp.seed;
            dm.stamp_check = bp.stamp_check;
            // the trace holds the deeper passes' items, launch after launch
            dm.trace = timed ? bp.trace : nullptr;
            dm.trace_items = bp.trace_items;
            dm.trace_base = int64_t(done) * geo.ntiles;
            const bool debug = dm.order != 0 || dm.stamp_check != 0 || dm.trace != nullptr;
            if (timed && ev_begin && !started) {
                r = hipEventRecord(ev_begin, s);
                if (r != hipSuccess) return r;
                started = true;
            }
            r = split >= 0 ? launch_by_fuse2<T, V>(fuse, g, qu, split, s)
                           : launch_by_fuse<T, V>(fuse, g, qu, debug ? &dm : nullptr, omega, s);
            if (r != hipSuccess) return r;
            *launches += 1;
            if (timed) {
                *persistent_launches += 1;
                *passes_done += chunk;
            }
            done += chunk;
            cur ^= chunk & 1;
        }
        return hipSuccess;
    };
    // Passes of both depths in one launch when their tiles are the same
    // (the production kernel only: not with SOR or a verification mode);
    // else the n_hi passes of depth d_hi, timed by the events so that their
    // duration is that of one kernel, then the n_lo shallower ones.
    bool merge = false;
    if (n_lo > 0 && omega == T(1) && bp.order == 0 && bp.stamp_check == 0 && !bp.trace &&
        mergeable_fuse(d_hi)) {
        const int rows = bp.tile_rows < 2 * d_hi ? 2 * d_hi : bp.tile_rows;
        const Geometry a = geometry(n, int(sizeof(T)), d_hi, rows);
        const Geometry b = geometry(n, int(sizeof(T)), d_hi - 1, rows);
        merge = a.halo_q == b.halo_q && a.q_core == b.q_core && a.rows == b.rows &&
                a.strips == b.strips && a.bands == b.bands && a.ntiles >= 1 &&
                int64_t(total_passes) * a.ntiles < (int64_t(1) << 30);
    }
    if (merge) {
        if ((e = run_passes(d_hi, total_passes, true, n_hi)) != hipSuccess) return e;
        if (ev_end && started) {
            e = hipEventRecord(ev_end, s);
            if (e != hipSuccess) return e;
        }
        *timed_fuse = d_hi;
    } else {
        if ((e = run_passes(d_hi, n_hi, true)) != hipSuccess) return e;
        if (ev_end && started) {
            e = hipEventRecord(ev_end, s);
            if (e != hipSuccess) return e;
        }
        *timed_fuse = d_hi;
        if (n_lo > 0 && (e = run_passes(d_hi - 1, n_lo, false)) != hipSuccess) return e;
    }
    if (result_in_last && cur == 0) {  // an even count after all: move it to where the caller wants it
        e = launch_copy_unless(buf_red[1], buf_red[0], colour_bytes, bp.stop, s);
        if (e != hipSuccess) return e;
        e = launch_copy_unless(buf_black[1], buf_black[0], colour_bytes, bp.stop, s);
        if (e != hipSuccess) return e;
    }
    if (cur != 0 && !result_in_last) {  // a kernel, so that a converged graph-captured solve skips it too
        e = launch_copy_unless(buf_red[0], buf_red[1], colour_bytes, bp.stop, s);
        if (e != hipSuccess) return e;
        e = launch_copy_unless(buf_black[0], buf_black[1], colour_bytes, bp.stop, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t run_blocked<double>(double* const[2], double* const[2], const double*,
                                        const double*, int, int64_t, double, int,
                                        const BlockedParams&, void*, size_t, hipStream_t, int*,
                                        hipEvent_t, hipEvent_t, int*, int*, int*, double, bool);
template hipError_t run_blocked<float>(float* const[2], float* const[2], const float*,
                                       const float*, int, int64_t, float, int,
                                       const BlockedParams&, void*, size_t, hipStream_t, int*,
                                       hipEvent_t, hipEvent_t, int*, int*, int*, float, bool);

int blocked_pass_parity(int n, size_t elem_bytes, int nsweeps, const rbgs_sweep_opts* o) {
    if (nsweeps < 2) return 0;  // the plain kernel runs a single sweep in place
    const int k = blocked_params(n, elem_bytes, o).fuse;
    return ((nsweeps + k - 1) / k) & 1;
}

int blocked_check_error(void* state, hipStream_t s, std::string* why) {
    int err = 0;
    hipError_t e = hipMemcpyAsync(&err, static_cast<char*>(state) + 64, sizeof err,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        *why = std::string("reading the persistent kernel's error word: ") + hipGetErrorString(e);
        return RBGS_EHIP;
    }
    if (err == kErrOrder) {
        *why = "the stamp check saw a neighbour more than one pass ahead of a tile's work item";
        return RBGS_EORDER;
    }
    if (err != 0) {
        *why = "a dependency wait in a persistent kernel timed out";
        return RBGS_ETIMEOUT;
    }
    return RBGS_OK;
}

}  // namespace rbgs
