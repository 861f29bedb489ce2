// Resident band sweep: many red-black sweeps of one small grid (n <= 512 in
// FP64, n <= 1024 in FP32) in one cooperative launch, with the grid held in
// registers.
//
// This is the paper's stripe decomposition (Section 2.3, Algorithm 2) made
// resident: the interior rows are split into horizontal bands, one
// workgroup per band, all co-resident.  A workgroup keeps its band plus a
// halo of H = 2K rows above and below in registers (one column per lane)
// and runs K full sweeps (an epoch) without talking to anyone: after 2K
// half-sweeps the halo has absorbed every stale value, so the owned rows are
// exactly those of K plain sweeps.  Between epochs each band publishes its
// top and bottom H+1 owned rows and waits only for its two neighbours'
// rows (per-band progress flags, as the paper's tasks wait only for the
// stripes they read), instead of a grid-wide barrier after every colour.
//
// Register layout.  Lane j (column j = 1..n) holds window rows
// P[w] = u(base + w + s, j), w = 0..W-1, base = r0 - H - 1, s = (j + base) & 1.
// The lane-parity shift s makes the colour of P[w] equal to w & 1 in every
// lane, so a half-sweep of colour c updates P[w] for w = c (mod 2) with the
// same register indices everywhere.  Vertical neighbours are P[w -+ 1];
// the horizontal neighbours sit in lanes j -+ 1 at their index w + 2s - 1,
// so every lane exports X[w] = s ? P[w-1] : P[w+1] and takes its left and
// right values from the neighbouring lanes through DPP.  Lanes at a wave
// boundary exchange X through LDS; the Dirichlet columns 0 and n+1 are in
// LDS as well.  P[0] and P[W-1] are never updated; the window is sized so
// that their staleness cannot reach the owned rows within one epoch.
//
// Term order as Eq. (1) everywhere in the library:
//   s = u(i+1,j) + u(i-1,j); s += u(i,j+1); s += u(i,j-1); s -= h2*f; u = s/4 (as 0.25*s)
// so the result is bitwise that of the plain sweep.
#include <hip/hip_runtime.h>

#include <climits>

#include "rbgs_internal.h"
#include "rbgs_resident.h"

namespace rbgs {
namespace resident {
namespace {

template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}
constexpr int kFromNext = 0x130;  // wave_shl:1 - lane i receives lane i+1
constexpr int kFromPrev = 0x138;  // wave_shr:1 - lane i receives lane i-1

template <int CTRL>
__device__ __forceinline__ double shift(double v) {
    return __hiloint2double(dpp<CTRL>(__double2hiint(v)), dpp<CTRL>(__double2loint(v)));
}
template <int CTRL>
__device__ __forceinline__ float shift(float v) {
    return __int_as_float(dpp<CTRL>(__float_as_int(v)));
}

// c ? a : b without a branch
__device__ __forceinline__ double pick(bool c, double a, double b) {
    const uint64_t m = uint64_t(0) - uint64_t(c);
    return __longlong_as_double((long long)((uint64_t(__double_as_longlong(a)) & m) |
                                            (uint64_t(__double_as_longlong(b)) & ~m)));
}
__device__ __forceinline__ float pick(bool c, float a, float b) {
    const uint32_t m = uint32_t(0) - uint32_t(c);
    return __uint_as_float((__float_as_uint(a) & m) | (__float_as_uint(b) & ~m));
}

// Wave-boundary exchange: edge[colour][wave + 1][0: lane 0, 1: lane 63][w / 2].
// Slot 0 side 1 holds the Dirichlet column 0 as seen by column 1, and slot
// waves + 1 side 0 the column n+1 as seen by column n, so every lane whose
// neighbour is not in its wave reads slot wave (left) or wave + 2 (right).
template <typename T>
struct Lds {
    T edge[2][kMaxWaves + 2][2][kW / 2];
    int go;  // broadcast of the wait result
};

template <typename T>
struct Band {
    int n, b, bands, r0, r1, base;
    int j, s, lane, wave, waves;
    bool col_in;  // 1 <= j <= n
};

template <typename T>
__device__ __forceinline__ T* colour_ptr(const Args<T>& a, int colour) {
    return colour ? a.u_black : a.u_red;
}

// Value of u(i, j) from the split arrays (i, j inside the stored grid).
template <typename T>
__device__ __forceinline__ T load_u(const Args<T>& a, int i, int j) {
    const T* c = ((i + j) & 1) ? a.u_black : a.u_red;
    return c[int64_t(i) * a.pitch + (j >> 1)];
}

// One half-sweep of colour C over the window (rows 1 .. W-2).  EDGE: the
// window contains a ring row or rows outside the grid, so updates are
// restricted to 1 <= i <= n.
template <typename T, int C, bool EDGE, bool SOR>
__device__ __forceinline__ void half_sweep(const Args<T>& a, const Band<T>& bd, T (&P)[kW],
                                           const T (&F)[kW], Lds<T>& lds) {
    // The exports read only rows of the other colour, which this half-sweep
    // does not change, so they are formed twice (before the barrier for the
    // wave-boundary lanes, after it for the DPP shifts) instead of being
    // kept live across it.
    if (bd.lane == 0 || bd.lane == 63) {
        const int side = bd.lane == 0 ? 0 : 1;
#pragma unroll
        for (int w = 1; w < kW - 1; ++w)
            if ((w & 1) == C)
                lds.edge[C][bd.wave + 1][side][w >> 1] = pick(bd.s != 0, P[w - 1], P[w + 1]);
    }
    __syncthreads();
    const bool need_left = bd.lane == 0, need_right = bd.lane == 63 || bd.j == bd.n;
    const T* lsrc = &lds.edge[C][bd.wave][1][0];
    const T* rsrc = &lds.edge[C][bd.wave + 2][0][0];
#pragma unroll
    for (int w = 1; w < kW - 1; ++w) {
        if ((w & 1) != C) continue;
        const T x = pick(bd.s != 0, P[w - 1], P[w + 1]);
        const T right = pick(need_right, rsrc[w >> 1], shift<kFromNext>(x));
        const T left = pick(need_left, lsrc[w >> 1], shift<kFromPrev>(x));
        T sum = P[w + 1] + P[w - 1];
        sum = sum + right;
        sum = sum + left;
        const T t = a.h2 * F[w];
        sum = sum - t;
        const T g = T(0.25) * sum;
        T nv = g;
        if constexpr (SOR) {  // red-black SOR relaxes the old value towards g
            const T d = g - P[w];
            const T wd = a.omega * d;
            nv = P[w] + wd;
        }
        if constexpr (EDGE) {
            const int i = bd.base + w + bd.s;
            P[w] = pick(i >= 1 && i <= bd.n, nv, P[w]);
        } else {
            P[w] = nv;
        }
    }
}

template <typename T, bool EDGE, bool SOR>
__device__ __forceinline__ void epoch(const Args<T>& a, const Band<T>& bd, T (&P)[kW],
                                      const T (&F)[kW], Lds<T>& lds, int sweeps) {
    for (int k = 0; k < sweeps; ++k) {
        half_sweep<T, 0, EDGE, SOR>(a, bd, P, F, lds);
        half_sweep<T, 1, EDGE, SOR>(a, bd, P, F, lds);
    }
}

// Exchange slots: [parity][band][side 0 top / 1 bottom][H+1 rows][xld].
template <typename T>
__device__ __forceinline__ T* xrow(const Args<T>& a, int parity, int band, int side, int r) {
    return a.xbuf + ((int64_t(parity) * a.bands + band) * 2 + side) * (kH + 1) * a.xld +
           int64_t(r) * a.xld;
}

// Publishes the top rows r0 .. r0+H and bottom rows r1-H-1 .. r1-1.
template <typename T>
__device__ __forceinline__ void export_rows(const Args<T>& a, const Band<T>& bd, const T (&P)[kW],
                                            int parity) {
    if (!bd.col_in) return;
    // global row g sits at window index g - base - s; for the uniform index
    // t = g - base the lane's value is P[t] (s = 0) or P[t-1] (s = 1)
#pragma unroll
    for (int t = kH + 1; t <= 2 * kH + 1; ++t)
        xrow(a, parity, bd.b, 0, t - (kH + 1))[bd.j] = pick(bd.s != 0, P[t - 1], P[t]);
    const int tb = bd.r1 - kH - 1 - bd.base;  // first bottom export row, runtime
#pragma unroll
    for (int t = 1; t < kW; ++t) {
        if (t >= tb && t <= tb + kH)
            xrow(a, parity, bd.b, 1, t - tb)[bd.j] = pick(bd.s != 0, P[t - 1], P[t]);
    }
}

// Reloads the halo rows r0-H-1 .. r0-1 (from the band above) and
// r1 .. r1+H (from the band below) that lie inside the interior.
template <typename T>
__device__ __forceinline__ void import_rows(const Args<T>& a, const Band<T>& bd, T (&P)[kW],
                                            int parity) {
    if (!bd.col_in) return;
#pragma unroll
    for (int w = 0; w < kW; ++w) {
        const int i = bd.base + w + bd.s;
        if (i < 1 || i > bd.n) continue;
        if (i < bd.r0 && bd.b > 0) {
            P[w] = xrow(a, parity, bd.b - 1, 1, i - (bd.r0 - kH - 1))[bd.j];
        } else if (i >= bd.r1 && i <= bd.r1 + kH && bd.b + 1 < bd.bands) {
            P[w] = xrow(a, parity, bd.b + 1, 0, i - bd.r1)[bd.j];
        }
    }
}

__device__ __forceinline__ uint32_t mix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    return h;
}

// Publishes `value` as this band's progress: every thread's prior stores
// are released at agent scope before thread 0 writes the flag.
template <typename T>
__device__ __forceinline__ void publish(const Args<T>& a, const Band<T>& bd, int value) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0 && bd.b + 1 != a.stall_band)
        __hip_atomic_store(a.flags + bd.b, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until both neighbouring bands have published at least `value`.
// Returns false (for the whole workgroup) on timeout or a reported error.
template <typename T>
__device__ bool wait_neighbours(const Args<T>& a, const Band<T>& bd, Lds<T>& lds, int value) {
    if (threadIdx.x == 0) {
        int ok = 1;
        for (int polls = 0;; ++polls) {
            const int up = bd.b > 0 ? __hip_atomic_load(a.flags + bd.b - 1, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT)
                                    : INT_MAX;
            const int dn = bd.b + 1 < bd.bands ? __hip_atomic_load(a.flags + bd.b + 1,
                                                                   __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT)
                                               : INT_MAX;
            if (up >= value && dn >= value) break;
            if (polls >= a.spin_limit) {
                __hip_atomic_store(a.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            if ((polls & 255) == 255 &&
                __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        lds.go = ok;
    }
    __syncthreads();
    const bool ok = lds.go != 0;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok;
}

template <typename T, bool EDGE, bool SOR>
__device__ __forceinline__ void run_band(const Args<T>& a, const Band<T>& bd, T (&P)[kW],
                                         const T (&F)[kW], Lds<T>& lds) {
    int left = a.sweeps;
    int e = 0;
    while (true) {
        const int k = left < kK ? left : kK;
        epoch<T, EDGE, SOR>(a, bd, P, F, lds, k);
        left -= k;
        if (left == 0) break;
        if (a.delay > 0) {
            const uint32_t loops = mix32(uint32_t(e) * 0x9e3779b9u + uint32_t(bd.b)) %
                                   uint32_t(a.delay + 1);
            for (uint32_t i = 0; i < loops; ++i) __builtin_amdgcn_s_sleep(127);
        }
        export_rows(a, bd, P, e & 1);
        publish(a, bd, e + 2);
        if (!wait_neighbours(a, bd, lds, e + 2)) return;
        import_rows(a, bd, P, e & 1);
        ++e;
    }
    // the neighbours' first loads read rows this band now overwrites
    if (!wait_neighbours(a, bd, lds, 1)) return;
#pragma unroll
    for (int w = 0; w < kW; ++w) {
        const int i = bd.base + w + bd.s;
        if (bd.col_in && i >= bd.r0 && i < bd.r1) {
            T* c = (w & 1) ? a.u_black : a.u_red;
            c[int64_t(i) * a.pitch + (bd.j >> 1)] = P[w];
        }
    }
}

// One workgroup per band, one lane per interior column; MAXT threads at
// most (the register budget: u and f of the window live in registers).
template <typename T, int MAXT, bool SOR>
__global__ __launch_bounds__(MAXT) void k_resident(Args<T> a) {
    // a converged graph-captured solve: every workgroup leaves before any
    // exchange (the flag was written by an earlier kernel of the stream)
    if (a.stop != nullptr && *a.stop != 0) return;
    __shared__ Lds<T> lds;
    Band<T> bd;
    bd.n = a.n;
    bd.b = blockIdx.x;
    bd.bands = a.bands;
    bd.r0 = 1 + int((int64_t(bd.b) * a.n) / a.bands);
    bd.r1 = 1 + int((int64_t(bd.b + 1) * a.n) / a.bands);
    bd.base = bd.r0 - kH - 1;
    bd.lane = threadIdx.x & 63;
    bd.wave = threadIdx.x >> 6;
    bd.waves = blockDim.x >> 6;
    bd.j = threadIdx.x + 1;
    bd.s = (bd.j + bd.base) & 1;
    bd.col_in = bd.j <= a.n;
    // Dirichlet columns, stored where columns 1 and n look for their outer
    // neighbour (see Lds)
    {
        const int waves = (a.n + 63) / 64;
        const int s1 = (1 + bd.base) & 1, sn = (a.n + bd.base) & 1;
        for (int t = threadIdx.x; t < 2 * kW; t += blockDim.x) {
            const int side = t / kW, w = t % kW;
            if (w < 1 || w > kW - 2) continue;
            const int i = bd.base + w + (side ? sn : s1);
            T v = T(0);
            if (i >= 0 && i <= a.n + 1) v = load_u(a, i, side ? a.n + 1 : 0);
            if (side)
                lds.edge[w & 1][waves + 1][0][w >> 1] = v;
            else
                lds.edge[w & 1][0][1][w >> 1] = v;
        }
    }
    T P[kW], F[kW];
#pragma unroll
    for (int w = 0; w < kW; ++w) {
        const int i = bd.base + w + bd.s;
        P[w] = T(0);
        F[w] = T(0);
        if (bd.col_in && i >= 0 && i <= a.n + 1) {
            P[w] = load_u(a, i, bd.j);
            const T* fc = (w & 1) ? a.f_black : a.f_red;
            if (i >= 1 && i <= a.n) F[w] = fc[int64_t(i) * a.pitch + (bd.j >> 1)];
        }
    }
    publish(a, bd, 1);  // also makes the ring columns visible to the whole workgroup
    const bool edge = bd.base < 1 || bd.base + kW > a.n;
    if (edge)
        run_band<T, true, SOR>(a, bd, P, F, lds);
    else
        run_band<T, false, SOR>(a, bd, P, F, lds);
}

}  // namespace

template <typename T>
constexpr int max_threads() { return sizeof(T) == 8 ? 512 : 1024; }

template <typename T>
hipError_t launch_resident(const Args<T>& a, hipStream_t s) {
    const int threads = (a.n + 63) / 64 * 64;
    if (threads > max_threads<T>()) return hipErrorInvalidValue;
    void* args[] = {const_cast<Args<T>*>(&a)};
    const void* kernel = a.sor ? reinterpret_cast<const void*>(&k_resident<T, max_threads<T>(), true>)
                               : reinterpret_cast<const void*>(&k_resident<T, max_threads<T>(), false>);
    return hipLaunchCooperativeKernel(kernel, dim3(a.bands), dim3(threads), args, 0, s);
}

template <typename T>
int max_n() { return max_threads<T>(); }

template <typename T>
int max_resident_bands(int n) {
    const int threads = (n + 63) / 64 * 64;
    if (threads > max_threads<T>()) return 0;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(&k_resident<T, max_threads<T>(), false>), threads, 0) !=
        hipSuccess)
        return 0;
    return per_cu * cus;
}

size_t state_bytes(int n, size_t elem_bytes) {
    if (n > max_threads<float>()) return 0;
    return kHeader + align256(size_t(bands_for(n)) * 4) + align256(exchange_elems(n) * elem_bytes);
}

template <typename T>
hipError_t run(T* u_red, T* u_black, const T* f_red, const T* f_black, int n, int64_t pitch, T h2,
               int nsweeps, int spin_limit, int delay, int stall_band, void* state, hipStream_t s,
               const int* stop, bool keep_error, T omega) {
    if (nsweeps <= 0) return hipSuccess;
    char* base = static_cast<char*>(state);
    const int bands = bands_for(n);
    const size_t flag_bytes = align256(size_t(bands) * 4);
    // error word (at kErrorOffset) and flags start at zero in every launch;
    // the rounds of a captured solve keep the error word, which the caller
    // cleared once
    hipError_t e = keep_error ? launch_zero(base + kHeader, flag_bytes, s)
                              : launch_zero(base, kHeader + flag_bytes, s);
    if (e != hipSuccess) return e;
    Args<T> a;
    a.u_red = u_red;
    a.u_black = u_black;
    a.f_red = f_red;
    a.f_black = f_black;
    a.pitch = pitch;
    a.n = n;
    a.h2 = h2;
    a.bands = bands;
    a.sweeps = nsweeps;
    a.xbuf = reinterpret_cast<T*>(base + kHeader + flag_bytes);
    a.xld = exchange_ld(n);
    a.flags = reinterpret_cast<int*>(base + kHeader);
    a.error = reinterpret_cast<int*>(base + kErrorOffset);
    a.spin_limit = spin_limit;
    a.delay = delay;
    a.stall_band = stall_band;
    a.stop = stop;
    a.omega = omega;
    a.sor = omega != T(1) ? 1 : 0;
    return launch_resident<T>(a, s);
}

template hipError_t launch_resident<double>(const Args<double>&, hipStream_t);
template hipError_t launch_resident<float>(const Args<float>&, hipStream_t);
template hipError_t run<double>(double*, double*, const double*, const double*, int, int64_t,
                                double, int, int, int, int, void*, hipStream_t, const int*, bool,
                                double);
template hipError_t run<float>(float*, float*, const float*, const float*, int, int64_t, float,
                               int, int, int, int, void*, hipStream_t, const int*, bool, float);
template int max_resident_bands<double>(int);
template int max_resident_bands<float>(int);
template int max_n<double>();
template int max_n<float>();

}  // namespace resident
}  // namespace rbgs
