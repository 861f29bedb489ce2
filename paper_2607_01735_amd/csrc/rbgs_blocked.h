// Persistent, temporally blocked sweep (internal interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "rbgs.h"

namespace rbgs {

constexpr int kBlockedLanes = 64;  // one wave per tile
constexpr int kMinRows = 8;
constexpr int kMaxRows = 65536;  // no grid is taller (n <= 65533)
constexpr int kMaxFuse = 10;

// Full sweeps per pass when the caller leaves fuse = 0, from time per sweep
// measured on MI355X: a pass costs about the same per row step whatever
// its depth (the row's HBM traffic sets the pace), so deep fusion pays on
// large grids (8191^2 FP64: fuse 7 53 us per sweep, fuse 4 96 us, fuse 8
// 55 us, where the deeper pipeline runs out of registers); small grids
// prefer shallow fusion, their short tiles being mostly halo.
inline int default_fuse(int elem_bytes, int n) {
    (void)elem_bytes;
    if (n < 768) return 4;
    if (n < 1536) return 5;
    return 7;
}

// Tile geometry of one grid: a tile is kBlockedLanes lanes x V q-columns
// wide (V = 16 bytes / element size) with halo_q columns of halo on each
// side, and `rows` interior rows tall.
struct Geometry {
    int V, L, halo_q, q_core, rows, strips, bands, ntiles;
};

inline Geometry geometry(int n, int elem_bytes, int fuse, int rows) {
    Geometry g;
    g.V = 16 / elem_bytes;
    g.L = 2 * fuse;
    const int need = g.L / 2 + 1;  // validity lost per side over L half-sweeps, in q
    g.halo_q = (need + g.V - 1) / g.V * g.V;
    g.q_core = kBlockedLanes * g.V - 2 * g.halo_q;
    g.rows = rows;
    g.strips = (n + rows - 1) / rows;
    g.bands = int(((int64_t(n) >> 1) + 1 + g.q_core - 1) / g.q_core);
    g.ntiles = g.strips * g.bands;
    return g;
}

// Upper bound on the tile count of any allowed geometry (rows >= kMinRows,
// q_core >= 64) for grid size n.
inline int max_tiles(int n) {
    int64_t strips = (int64_t(n) + kMinRows - 1) / kMinRows;
    int64_t bands = ((int64_t(n) >> 1) + 1 + 63) / 64 + 1;
    return int(strips * bands);
}

inline int default_rows(int n, int L) {
    int r = 256;
    while (r > 2 * L && r > kMinRows && r * 4 > n) r >>= 1;
    return r < L ? L : r;
}

// Tile height for one grid on its own.  Taller tiles spend less of their
// work on the L halo rows (a fraction rows / (rows + 2L) is useful) but give
// fewer tiles, and fewer tiles than the launch has wave slots leave waves
// idle.  The height (a power of two from kMinRows to 1024, at least L)
// maximises the product of the two, with 0.8 x wave_slots as the tile count
// that keeps the chip busy (waves finish their tiles at different times),
// up to 512 rows in FP64 and 256 in FP32.  On MI355X this picks the measured
// best power-of-two height at 1023..8191 in FP64 and FP32.  The caps come
// from 16383^2 (fuse 7), where every height fills the chip and the score
// alone would take 1024 rows: FP64 1253 GLUP/s at 1024 rows, 1353 at 512,
// 1371 at 768; FP32 1814 at 1024, 1819 at 512, 2234 at 256, 1962 at 128.
// FP64 then takes one more strip of equal height when the chosen height
// gives fewer tiles than 1.2 x wave_slots: waves drain a pass's tiles
// unevenly, and a few more tiles than slots pay.  Measured at 8191^2 (fuse
// 7, 1024 slots, 37 bands), a whole 200-sweep step: 256 rows (32 strips,
// 1184 tiles) 10.05-10.17 ms, 249 rows (33 strips) 9.87, 241 rows 9.87,
// 228 rows 10.12, 272 rows 10.36.
inline int single_grid_rows(int n, int L, int elem_bytes, int wave_slots) {
    const double busy = 0.8 * (wave_slots > 0 ? wave_slots : 1024);
    const int cap = elem_bytes == 8 ? 512 : 256;
    int best = 0;
    double best_score = -1.0;
    for (int r = kMinRows; r <= cap; r <<= 1) {
        const int rows = r < L ? L : r;
        const Geometry g = geometry(n, elem_bytes, L / 2, rows);
        const double fill = g.ntiles >= busy ? 1.0 : g.ntiles / busy;
        const double score = double(rows) / double(rows + 2 * L) * fill;
        if (score >= best_score) {
            best_score = score;
            best = rows;
        }
    }
    const double plenty = 1.2 * (wave_slots > 0 ? wave_slots : 1024);
    if (elem_bytes == 8) {
        const Geometry g = geometry(n, elem_bytes, L / 2, best);
        const int more = (n + g.strips) / (g.strips + 1);  // ceil(n / (strips + 1))
        if (g.ntiles < plenty && more >= L && more >= kMinRows) best = more;
    } else if (best == cap) {
        // FP32 takes 1.25 x its cap when that still leaves plenty of tiles:
        // 16383^2 (fuse 7, 100 sweeps) 10.68 ms at 320 rows (1820 tiles)
        // against 11.05 at 256; 384 rows 11.1, 512 rows 13.6
        const int taller = cap + cap / 4;
        if (geometry(n, elem_bytes, L / 2, taller).ntiles >= plenty) best = taller;
    }
    return best;
}

// Resident one-wave workgroups per CU for a persistent kernel, and CU count.
hipError_t persistent_occupancy(const void* kernel, int* per_cu, int* cus);
// Waves the single-grid persistent kernel of this depth runs at once on the
// current device (CUs x resident waves per CU); 1024 if the query fails.
int blocked_wave_slots(size_t elem_bytes, int fuse);

struct BlockedParams {
    int fuse = 0;       // full sweeps per pass
    int tile_rows = 0;  // interior rows per tile
    int tile_cols = 0;  // interior columns per tile
    int delay = 0;      // debug: per-tile delay injection
    int spin_limit = 0; // debug: bound on each flag wait
    int stall_tile = 0; // debug: tile + 1 that never publishes its progress
    const int* stop = nullptr;  // converged flag of a graph-captured solve
    bool keep_error = false;    // the caller cleared the error word (graph rounds)
    int order = 0;              // debug: tile order within a pass (0, 1, 2)
    uint32_t seed = 0;          // debug: seed of order 2
    int stamp_check = 0;        // debug: neighbour pass-count check per item
    unsigned long long* trace = nullptr;  // debug: per-item trace records
    int64_t trace_items = 0;
};

// Bytes of device state (flags, ticket counter, error word) for grid size n.
size_t blocked_state_bytes(int n, int elem_bytes);
// Checks fuse / tile options; writes a message to *why on failure.
int validate_blocked_opts(int fuse, int tile_rows, int tile_cols, std::string* why);
// Checks the debug tile order, stamp check and trace options.
int validate_blocked_debug(const rbgs_sweep_opts* o, std::string* why);
// Kernel the library picks for RBGS_KERNEL_AUTO.
int auto_kernel(int n, size_t elem_bytes, int nsweeps);
BlockedParams blocked_params(int n, size_t elem_bytes, const rbgs_sweep_opts* o);
// nsweeps sweeps of the split iterate in buffer 0 (buf_red[0], buf_black[0])
// with the persistent kernel; buffer 1 is scratch of the same size.  The
// result is left in buffer 0.  The sweeps run as ceil(nsweeps / fuse)
// passes whose depths differ by at most one (one launch of the deeper
// passes, then one of the shallower ones); a single sweep runs with the
// plain kernel.  When ev_begin/ev_end are given they are recorded around the
// launch(es) of the deeper passes; *persistent_launches, *passes_done and
// *timed_fuse receive what those launches did.  omega != 1: red-black SOR
// (FP64 only; not with the verification modes).  result_in_last: after an
// odd number of passes leave the result in buffer 1 (the caller packed the
// input into buffer 0 knowing the parity, so buffer 1 is where it wants
// it) instead of copying it back into buffer 0.
template <typename T>
hipError_t run_blocked(T* const buf_red[2], T* const buf_black[2], const T* f_red,
                       const T* f_black, int n, int64_t pitch, T h2, int nsweeps,
                       const BlockedParams& bp, void* state, size_t state_bytes, hipStream_t s,
                       int* launches, hipEvent_t ev_begin, hipEvent_t ev_end,
                       int* persistent_launches, int* passes_done, int* timed_fuse,
                       T omega = T(1), bool result_in_last = false);
// 1 when nsweeps sweeps with these options run an odd number of persistent
// passes (the result then lands in the second buffer), else 0.
int blocked_pass_parity(int n, size_t elem_bytes, int nsweeps, const rbgs_sweep_opts* o);
// Reads the persistent kernel's error word (synchronising the stream when
// the kernel ran); returns RBGS_OK or RBGS_ETIMEOUT.
int blocked_check_error(void* state, hipStream_t s, std::string* why);

}  // namespace rbgs
