// Resident band sweep (sweep_resident.hip): parameters shared with the host.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rbgs {
namespace resident {

constexpr int kH = 8;                 // halo rows on each side = half-sweeps per epoch
constexpr int kK = kH / 2;            // full sweeps per epoch
constexpr int kR = 2 * (kH + 1);      // most rows a band owns
constexpr int kW = kR + 2 * kH + 2;   // window rows held per lane
constexpr int kMaxWaves = 16;         // one lane per interior column, 1024 lanes at most

template <typename T>
struct Args {
    T* u_red;
    T* u_black;
    const T* f_red;
    const T* f_black;
    int64_t pitch;   // split pitch (elements)
    int n;
    T h2;
    int bands;
    int sweeps;      // full sweeps in this launch
    T* xbuf;         // exchange rows: [2][bands][2][kH + 1][xld]
    int64_t xld;
    int* flags;      // per band, zero before the launch
    int* error;      // zero before the launch; 1 after a timed-out wait
    int spin_limit;
    int delay;       // debug: pseudo-random stalls between epochs
    int stall_band;  // debug: band b+1 = stall_band never publishes
    const int* stop; // converged flag of a graph-captured solve (nullptr: none)
    T omega;         // relaxation factor when sor != 0
    int sor;         // 1: red-black SOR, u <- u + omega (g - u) (its own kernel
                     // instance); 0: Gauss-Seidel, u <- g
};

// Bands for an n x n grid: ceil(n / kR), so every band owns between kH + 1
// and kR rows (one band when n < kR).
inline int bands_for(int n) { return n < kR ? 1 : (n + kR - 1) / kR; }

inline int64_t exchange_ld(int n) { return (int64_t(n) + 2 + 63) / 64 * 64; }

inline size_t exchange_elems(int n) {
    return size_t(2) * size_t(bands_for(n)) * 2 * (kH + 1) * size_t(exchange_ld(n));
}

// Kernel state in the caller's workspace: a 256-byte header whose int at
// kErrorOffset is the error word (the same place as the blocked kernel's,
// so one check serves both), the per-band flags, then the exchange rows.
constexpr size_t kHeader = 256;
constexpr size_t kErrorOffset = 64;

// Bytes of state for an n x n grid with elements of elem_bytes; 0 when the
// kernel does not take n in any precision.
size_t state_bytes(int n, size_t elem_bytes);

// nsweeps sweeps of the split arrays in one cooperative launch (clears the
// state's header and flags first, with a kernel).  Fails with
// hipErrorInvalidValue when n is above max_n<T>(), and with the cooperative
// launch's error when the bands do not fit on the device at once.
// omega != 1: red-black SOR (the Gauss-Seidel value g relaxes the old value,
// difference, product and sum each rounded once).
template <typename T>
hipError_t run(T* u_red, T* u_black, const T* f_red, const T* f_black, int n, int64_t pitch, T h2,
               int nsweeps, int spin_limit, int delay, int stall_band, void* state, hipStream_t s,
               const int* stop = nullptr, bool keep_error = false, T omega = T(1));

template <typename T>
hipError_t launch_resident(const Args<T>& a, hipStream_t s);

// How many workgroups of the resident kernel fit on the device at once.
template <typename T>
int max_resident_bands(int n);

// Largest n the kernel takes for this type (u and f of the window are held
// in registers: 512 lanes per workgroup in FP64, 1024 in FP32).
template <typename T>
int max_n();

}  // namespace resident
}  // namespace rbgs
