// Persistent, temporally blocked sweep (internal interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "rbgs.h"

namespace rbgs {

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
int auto_kernel(int n, size_t elem_bytes);
BlockedParams blocked_params(int n, size_t elem_bytes, const rbgs_sweep_opts* o);
// nsweeps sweeps of the split iterate in buffer 0 (buf_red[0], buf_black[0])
// with the persistent kernel; buffer 1 is scratch of the same size.  The
// result is left in buffer 0.  Sweeps that do not fill a whole pass of
// `fuse` sweeps run with the plain kernel.
template <typename T>
hipError_t run_blocked(T* const buf_red[2], T* const buf_black[2], const T* f_red,
                       const T* f_black, int n, int64_t pitch, T h2, int nsweeps,
                       const BlockedParams& bp, void* state, size_t state_bytes, hipStream_t s,
                       int* launches);
// Reads the persistent kernel's error word (synchronising the stream when
// the kernel ran); returns RBGS_OK or RBGS_ETIMEOUT.
int blocked_check_error(void* state, hipStream_t s, std::string* why);

}  // namespace rbgs
