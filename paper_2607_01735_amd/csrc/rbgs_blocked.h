// Persistent, temporally blocked sweep (internal interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "rbgs.h"

namespace rbgs {

constexpr int kBlockedLanes = 64;  // one wave per tile
constexpr int kMinRows = 8;
constexpr int kMaxFuse = 10;

// Full sweeps per pass when the caller leaves fuse = 0, from time per sweep
// measured on MI355X: deep fusion pays on large grids (8191^2: FP64 fuse 7
// with 256-row tiles 1157 GLUP/s, fuse 6 1036, fuse 9 1111; FP32 fuse 7 with
// 128-row tiles 1520), shallow fusion on small ones, whose short tiles
// would be mostly halo.
inline int default_fuse(int elem_bytes, int n) {
    (void)elem_bytes;
    if (n < 768) return 4;
    if (n < 1536) return 5;
    if (n < 4096) return 6;
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

// Tile height for one grid on its own: small grids need many tiles to keep
// waves busy (about 64 row tiles up to n = 2047, measured best on MI355X
// at 255..2047), large ones need tall tiles for fewer halo rows (256 at
// 8191 in FP64).  FP32 tiles are twice as wide, so half as tall.  The tile
// also has to hold the L halo rows.
inline int single_grid_rows(int n, int L, int elem_bytes) {
    const int64_t m = int64_t(n) + 1;
    int64_t want = m <= 2048 ? m / 64 : m / 32;
    if (elem_bytes == 4) want /= 2;
    int r = kMinRows;
    while (r * 2 <= want && r < 256) r <<= 1;
    return r < L ? L : r;
}

// Resident one-wave workgroups per CU for a persistent kernel, and CU count.
hipError_t persistent_occupancy(const void* kernel, int* per_cu, int* cus);

struct BlockedParams {
    int fuse = 0;       // full sweeps per pass
    int tile_rows = 0;  // interior rows per tile
    int tile_cols = 0;  // interior columns per tile
    int delay = 0;      // debug: per-tile delay injection
    int spin_limit = 0; // debug: bound on each flag wait
    int stall_tile = 0; // debug: tile + 1 that never publishes its progress
};

// Bytes of device state (flags, ticket counter, error word) for grid size n.
size_t blocked_state_bytes(int n, int elem_bytes);
// Checks fuse / tile options; writes a message to *why on failure.
int validate_blocked_opts(int fuse, int tile_rows, int tile_cols, std::string* why);
// Kernel the library picks for RBGS_KERNEL_AUTO.
int auto_kernel(int n, size_t elem_bytes, int nsweeps);
BlockedParams blocked_params(int n, size_t elem_bytes, const rbgs_sweep_opts* o);
// nsweeps sweeps of the split iterate in buffer 0 (buf_red[0], buf_black[0])
// with the persistent kernel; buffer 1 is scratch of the same size.  The
// result is left in buffer 0.  Sweeps that do not fill a whole pass of
// `fuse` sweeps run as one shallower pass (a single one with the plain
// kernel).  When ev_begin/ev_end are given
// they are recorded right before the first and after the last full-depth
// persistent launch (around the shallower pass when there is no full one);
// *persistent_launches and *passes_done receive what those launches did.
template <typename T>
hipError_t run_blocked(T* const buf_red[2], T* const buf_black[2], const T* f_red,
                       const T* f_black, int n, int64_t pitch, T h2, int nsweeps,
                       const BlockedParams& bp, void* state, size_t state_bytes, hipStream_t s,
                       int* launches, hipEvent_t ev_begin, hipEvent_t ev_end,
                       int* persistent_launches, int* passes_done);
// Reads the persistent kernel's error word (synchronising the stream when
// the kernel ran); returns RBGS_OK or RBGS_ETIMEOUT.
int blocked_check_error(void* state, hipStream_t s, std::string* why);

}  // namespace rbgs
