// Red-black Gauss-Seidel in three dimensions, 7-point Laplacian (an
// extension: the conclusion, Section 5, names higher dimensions as future
// work).  Red points have i + j + k even.
//
// Layout: the 2D split layout with a row per (i, j) pair: point (i, j, k) of
// colour C = (i + j + k) & 1 sits at C[(i (n+2) + j) pitch + (k >> 1)].  In
// row (i, j) the points of colour C have k = 2q + p, p = (i + j + C) & 1, and
// the neighbours of C[i][j][q] (all of the other colour O) are
//     (i +- 1, j, k) -> O[i +- 1][j][q]      (i, j +- 1, k) -> O[i][j +- 1][q]
//     (i, j, k + 1)  -> O[i][j][q + p]       (i, j, k - 1)  -> O[i][j][q - 1 + p]
// so a half-sweep streams the other colour, its own f and its own colour
// once: 24 B per grid point and sweep, as in 2D.
//
// The half-sweep marches each thread down kPlanes planes (2.5D streaming):
// O[i-1][j][q], O[i][j][q] and O[i+1][j][q] stay in registers, so each step
// loads one new element of that column; the j +- 1 rows and the other k
// neighbour are mostly loads of the same workgroup (cache hits).
//
// Update (each operation rounded once, no contraction):
//   s = ((((u[i+1] + u[i-1]) + u[j+1]) + u[j-1]) + u[k+1]) + u[k-1]
//   u = (s - (h h) f) / 6.
#include <algorithm>
#include <cmath>

#include "rb3_flags.h"
#include "rbgs_internal.h"

namespace rbgs {
namespace {

constexpr int kThreads = 256;
constexpr int kPlanes = 16;
constexpr int kResidualBlocks = 2048;

__global__ __launch_bounds__(kThreads) void k_rb3_pack(const double* __restrict__ nat, int64_t ld,
                                                       double* __restrict__ red,
                                                       double* __restrict__ black, int n,
                                                       int64_t pitch) {
    const int64_t q = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t j = blockIdx.y, i = blockIdx.z;
    if (q >= pitch) return;
    const int64_t row = i * (n + 2) + j;
    // (i, j, 2q) has colour (i + j) & 1, (i, j, 2q + 1) the other
    double* even_dst = ((i + j) & 1) ? black : red;
    double* odd_dst = ((i + j) & 1) ? red : black;
    const double* src = nat + row * ld;
    const int64_t k0 = 2 * q, k1 = 2 * q + 1;
    even_dst[row * pitch + q] = k0 <= n + 1 ? src[k0] : 0.0;
    odd_dst[row * pitch + q] = k1 <= n + 1 ? src[k1] : 0.0;
}

__global__ __launch_bounds__(kThreads) void k_rb3_unpack(double* __restrict__ nat, int64_t ld,
                                                         const double* __restrict__ red,
                                                         const double* __restrict__ black, int n,
                                                         int64_t pitch) {
    const int64_t q = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t j = int64_t(blockIdx.y) + 1, i = int64_t(blockIdx.z) + 1;
    if (q >= pitch) return;
    const int64_t row = i * (n + 2) + j;
    const double* even_src = ((i + j) & 1) ? black : red;
    const double* odd_src = ((i + j) & 1) ? red : black;
    double* dst = nat + row * ld;
    const int64_t k0 = 2 * q, k1 = 2 * q + 1;
    if (k0 >= 1 && k0 <= n) dst[k0] = even_src[row * pitch + q];
    if (k1 >= 1 && k1 <= n) dst[k1] = odd_src[row * pitch + q];
}

// Workgroups of kQ x kJ threads (kQ threads of two q-columns each along kJ
// consecutive rows j), so that most j +- 1 loads hit rows the same
// workgroup loads; the 1-D grid is remapped so that each XCD receives a
// contiguous range of workgroups (rows next to each other share that XCD's
// L2).  A thread loads the other colour and f as 16-byte pairs (q, q + 1):
// twice the bytes in flight per load of a one-column thread; the one k
// neighbour outside the pair (q + 2 or q - 1) is the neighbouring lane's
// value, passed by a cross-lane shuffle (a wave is 64 consecutive pairs of
// one row), and loaded only at the wave's ends or next to a lane without
// points.
constexpr int kQ = 64, kJ = 8;
// Grid size from which each thread takes two q-columns: measured on MI355X,
// 767^3 runs 2.22 ms per sweep with two against 2.33 with one, while 63^3
// and 127^3 solves take 1.38x longer with two (too few threads).
constexpr int kPairMinN = 384;

typedef double dvec2 __attribute__((ext_vector_type(2)));

struct D2 {
    double x, y;
};

__device__ __forceinline__ D2 load2(const double* p) {
    const dvec2 v = *reinterpret_cast<const dvec2*>(p);
    return D2{v.x, v.y};
}

__device__ __forceinline__ D2 load2_nt(const double* p) {
    const dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(p));
    return D2{v.x, v.y};
}

// Gauss-Seidel value of one point from its six neighbours, in the order the
// update fixes (each operation rounded once).
__device__ __forceinline__ double rb3_update(double up, double dn, double jp, double jm, double kp,
                                             double km, double h2, double fv) {
    double s = up + dn;
    s = s + jp;
    s = s + jm;
    s = s + kp;
    s = s + km;
    const double t = h2 * fv;
    s = s - t;
    return s / 6.0;
}

// One q-column per thread: the form for grids below kPairMinN, where half
// as many threads (two columns each) leave the chip short of waves.
__global__ __launch_bounds__(kQ * kJ) void k_rb3_half1(double* __restrict__ self,
                                                      const double* __restrict__ other,
                                                      const double* __restrict__ f, int n,
                                                      int64_t pitch, double h2, int colour,
                                                      int qblocks, int jblocks, const int* stop) {
    if (stop && *stop) return;
    const int nb = int(gridDim.x);
    const int b = xcd_logical_block(int(blockIdx.x), nb);
    const int bq = b % qblocks, bj = (b / qblocks) % jblocks, bz = b / (qblocks * jblocks);
    const int64_t q = int64_t(bq) * kQ + (threadIdx.x % kQ);
    const int64_t j = int64_t(bj) * kJ + (threadIdx.x / kQ) + 1;
    const int64_t i0 = int64_t(bz) * kPlanes + 1;
    if (j > n || q >= pitch || 2 * q > n) return;  // no interior point of either parity beyond
    const int64_t i1 = i0 + kPlanes - 1 < n ? i0 + kPlanes - 1 : n;
    const int64_t np2 = int64_t(n) + 2;
    auto row = [&](int64_t i, int64_t jj) { return (i * np2 + jj) * pitch; };
    double o_dn = other[row(i0 - 1, j) + q];
    double o_c = other[row(i0, j) + q];
    for (int64_t i = i0; i <= i1; ++i) {
        const double o_up = other[row(i + 1, j) + q];
        const int64_t p = (i + j + colour) & 1;
        const int64_t k = 2 * q + p;
        if (k >= 1 && k <= n) {
            const int64_t r = row(i, j);
            const double jp = other[row(i, j + 1) + q];
            const double jm = other[row(i, j - 1) + q];
            const double kp = p ? other[r + q + 1] : o_c;
            const double km = p ? o_c : other[r + q - 1];
            double s = o_up + o_dn;
            s = s + jp;
            s = s + jm;
            s = s + kp;
            s = s + km;
            // f is read once per sweep and the new value is not read again
            // before the other colour's half-sweep has streamed the whole
            // grid: both go through the caches as streaming (non-temporal)
            const double t = h2 * __builtin_nontemporal_load(f + r + q);
            s = s - t;
            __builtin_nontemporal_store(s / 6.0, self + r + q);
        }
        o_dn = o_c;
        o_c = o_up;
    }
}

__global__ __launch_bounds__(kQ * kJ) void k_rb3_half(double* __restrict__ self,
                                                      const double* __restrict__ other,
                                                      const double* __restrict__ f, int n,
                                                      int64_t pitch, double h2, int colour,
                                                      int qblocks, int jblocks, const int* stop) {
    if (stop && *stop) return;
    const int nb = int(gridDim.x);
    const int b = xcd_logical_block(int(blockIdx.x), nb);
    const int bq = b % qblocks, bj = (b / qblocks) % jblocks, bz = b / (qblocks * jblocks);
    const int lane = int(threadIdx.x % kQ);
    const int64_t q = 2 * (int64_t(bq) * kQ + lane);  // pair (q, q + 1)
    const int64_t j = int64_t(bj) * kJ + (threadIdx.x / kQ) + 1;
    const int64_t i0 = int64_t(bz) * kPlanes + 1;
    // no interior point of either parity beyond; such lanes stay for the
    // shuffles but load and store nothing
    const bool act = j <= n && q < pitch && 2 * q <= n;
    // the lane to the right holds the pair (q + 2, q + 3) when it is active
    const bool right_act = lane + 1 < kQ && j <= n && q + 2 < pitch && 2 * (q + 2) <= n;
    const int64_t i1 = i0 + kPlanes - 1 < n ? i0 + kPlanes - 1 : n;
    const int64_t np2 = int64_t(n) + 2;
    auto row = [&](int64_t i, int64_t jj) { return (i * np2 + jj) * pitch; };
    const D2 zero{0.0, 0.0};
    D2 o_dn = act ? load2(other + row(i0 - 1, j) + q) : zero;
    D2 o_c = act ? load2(other + row(i0, j) + q) : zero;
    for (int64_t i = i0; i <= i1; ++i) {
        const D2 o_up = act ? load2(other + row(i + 1, j) + q) : zero;
        // the k neighbours just outside the pair, other[q + 2] and
        // other[q - 1], from the lanes next to this one
        const double from_right = __shfl_down(o_c.x, 1, kQ);
        const double from_left = __shfl_up(o_c.y, 1, kQ);
        const int64_t p = (i + j + colour) & 1;
        const int64_t k0 = 2 * q + p, k1 = k0 + 2;  // the points of q and q + 1
        const bool v0 = act && k0 >= 1 && k0 <= n, v1 = act && k1 <= n;
        if (v0 || v1) {
            const int64_t r = row(i, j);
            const D2 jp = load2(other + r + pitch + q);  // row j + 1 of plane i
            const D2 jm = load2(other + r - pitch + q);
            // p = 1: q's k neighbours are o_c.y (k + 1) and o_c.x (k - 1), and
            // q + 1's are other[q + 2] and o_c.y; p = 0: q's are o_c.x and
            // other[q - 1], q + 1's are o_c.y and o_c.x
            double outer = 0.0;
            if (p) {
                if (v1) outer = right_act ? from_right : other[r + q + 2];
            } else {
                if (v0) outer = lane > 0 ? from_left : other[r + q - 1];
            }
            // f is read once per sweep and the new values are not read again
            // before the other colour's half-sweep has streamed the whole
            // grid: both go through the caches as streaming (non-temporal)
            const D2 fv = load2_nt(f + r + q);
            const double kp0 = p ? o_c.y : o_c.x, km0 = p ? o_c.x : outer;
            const double kp1 = p ? outer : o_c.y, km1 = p ? o_c.y : o_c.x;
            const double u0 = rb3_update(o_up.x, o_dn.x, jp.x, jm.x, kp0, km0, h2, fv.x);
            const double u1 = rb3_update(o_up.y, o_dn.y, jp.y, jm.y, kp1, km1, h2, fv.y);
            if (v0 && v1) {
                const dvec2 w = {u0, u1};
                __builtin_nontemporal_store(w, reinterpret_cast<dvec2*>(self + r + q));
            } else if (v0) {
                __builtin_nontemporal_store(u0, self + r + q);
            } else {
                __builtin_nontemporal_store(u1, self + r + q + 1);
            }
        }
        o_dn = o_c;
        o_c = o_up;
    }
}

__device__ __forceinline__ double rb3_at(const double* red, const double* black, int64_t i,
                                         int64_t j, int64_t k, int64_t np2, int64_t pitch) {
    const double* a = ((i + j + k) & 1) ? black : red;
    return a[(i * np2 + j) * pitch + (k >> 1)];
}

// Residual norms: block b takes (i, j) rows b, b + gridDim.x, ... of the
// interior; each thread the points k = 2q and 2q + 1 of its column.
__global__ __launch_bounds__(kThreads) void k_rb3_residual(
    const double* __restrict__ ur, const double* __restrict__ ub, const double* __restrict__ fr,
    const double* __restrict__ fb, int n, int64_t pitch, double inv_h2, double* partials) {
    __shared__ double sr[kThreads], sb[kThreads];
    double acc_r = 0.0, acc_b = 0.0;
    const int64_t np2 = int64_t(n) + 2, n1 = int64_t(n) + 1;
    const int64_t rows = int64_t(n) * n;
    for (int64_t rr = blockIdx.x; rr < rows; rr += gridDim.x) {
        const int64_t i = rr / n + 1, j = rr % n + 1;
        for (int64_t q = threadIdx.x; q < pitch; q += kThreads) {
            for (int e = 0; e < 2; ++e) {
                const int64_t k = 2 * q + e;
                if (k < 1 || k > n) continue;
                auto at = [&](int64_t a, int64_t b, int64_t c) {
                    return rb3_at(ur, ub, a, b, c, np2, pitch);
                };
                auto ring = [&](int64_t a, int64_t b, int64_t c) {
                    return (a == 0 || b == 0 || c == 0 || a == n1 || b == n1 || c == n1)
                               ? at(a, b, c)
                               : 0.0;
                };
                double s = at(i + 1, j, k) + at(i - 1, j, k);
                s = s + at(i, j + 1, k);
                s = s + at(i, j - 1, k);
                s = s + at(i, j, k + 1);
                s = s + at(i, j, k - 1);
                const double fc = rb3_at(fr, fb, i, j, k, np2, pitch);
                const double lap = (s - 6.0 * at(i, j, k)) * inv_h2;
                const double r = fc - lap;
                double sbv = ring(i + 1, j, k) + ring(i - 1, j, k);
                sbv = sbv + ring(i, j + 1, k);
                sbv = sbv + ring(i, j - 1, k);
                sbv = sbv + ring(i, j, k + 1);
                sbv = sbv + ring(i, j, k - 1);
                const double b = fc - sbv * inv_h2;
                acc_r += r * r;
                acc_b += b * b;
            }
        }
    }
    sr[threadIdx.x] = acc_r;
    sb[threadIdx.x] = acc_b;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
            sr[threadIdx.x] += sr[threadIdx.x + w];
            sb[threadIdx.x] += sb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = sr[0];
        partials[2 * blockIdx.x + 1] = sb[0];
    }
}

__global__ __launch_bounds__(kThreads) void k_rb3_reduce(const double* __restrict__ partials,
                                                         int count, double* __restrict__ out) {
    __shared__ double sr[kThreads], sb[kThreads];
    double r = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < count; k += kThreads) {
        r += partials[2 * k];
        b += partials[2 * k + 1];
    }
    sr[threadIdx.x] = r;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
            sr[threadIdx.x] += sr[threadIdx.x + w];
            sb[threadIdx.x] += sb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sr[0];
        out[1] = sb[0];
    }
}

// The flag-driven form (rb3_flags.h): one launch for every half-sweep.
template <int C>
__global__ __launch_bounds__(rb3f::kLanes) void k_rb3_flags(rb3f::Args a) { rb3f::run<C>(a); }

// Resident one-wave workgroups of the kernel with chunk C (0 if the query
// fails).
template <int C>
int capacity_of() {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(&k_rb3_flags<C>), rb3f::kLanes, 0) !=
            hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const int64_t c = int64_t(cus) * per_cu;
    return int(c < kRb3MaxBlocks ? c : kRb3MaxBlocks);
}

double wanted_items(int n) { return std::sqrt(double(n) * double(n) * double(n) / 10.0); }

// The lean chunk from this size up.  Per sweep, flag-driven, FP64, deep
// (one wave per SIMD) against lean (four): 127^3 0.053 / 0.068 ms, 255^3
// 0.192 / 0.222, 383^3 0.564 / 0.618, 511^3 1.107 / 1.217, 767^3 3.933 /
// 3.396; the deep kernel then holds 1024 waves for 864 blocks of 64 x 64 x
// 64, the lean one 3456 blocks of 64 x 32 x 32.
constexpr int kRb3LeanMinN = 640;

bool use_deep_chunk(int n) { return n < kRb3LeanMinN; }

}  // namespace

int rb3_flags_capacity(int n) {
    return use_deep_chunk(n) ? capacity_of<rb3f::kDeepChunk>() : capacity_of<rb3f::kLeanChunk>();
}

// Bound on the blocks per half-sweep.  Every item costs one ticket, and
// tickets of the whole device go through one counter (about 40 ns each on
// MI355X), while an item's time grows with its size; the two balance near
// sqrt(n^3 / 10) items per half-sweep, capped at the waves the chip holds.
int rb3_flags_target(int n, int capacity) {
    return int(std::max(64.0, std::min(double(capacity), wanted_items(n))));
}

int rb3_flags_blocks(int n, int capacity) {
    if (capacity < 64) return 0;
    return rb3f::geometry(n, rb3_flags_target(n, capacity)).nblocks;
}

hipError_t launch_rb3_flags(double* red, double* black, const double* f_red,
                            const double* f_black, int n, int64_t pitch, double h2, int levels,
                            int capacity, int* ticket, int* progress, int* error, int spin_limit,
                            int delay, int stall_block, const int* stop, hipStream_t s) {
    if (capacity < 64) return hipErrorInvalidValue;
    const rb3f::Geometry geo = rb3f::geometry(n, rb3_flags_target(n, capacity));
    if (int64_t(levels) * geo.nblocks >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    rb3f::Args a;
    a.red = red;
    a.black = black;
    a.f_red = f_red;
    a.f_black = f_black;
    a.n = n;
    a.pitch = pitch;
    a.h2 = h2;
    a.qw = geo.qw;
    a.rj = geo.rj;
    a.rz = geo.rz;
    a.qblocks = geo.qblocks;
    a.jblocks = geo.jblocks;
    a.zblocks = geo.zblocks;
    a.nblocks = geo.nblocks;
    a.levels = levels;
    a.ticket = ticket;
    a.progress = progress;
    a.error = error;
    a.spin_limit = spin_limit;
    a.delay = delay;
    a.stall_block = stall_block;
    a.stop = stop;
    // one wave per block: each takes the next level's item as it finishes
    // one, and more waves would only wait
    const int64_t items = int64_t(levels) * geo.nblocks;
    int64_t waves = std::min<int64_t>(capacity, geo.nblocks);
    if (waves > items) waves = items;
    if (waves < 1) waves = 1;
    if (use_deep_chunk(n))
        hipLaunchKernelGGL(k_rb3_flags<rb3f::kDeepChunk>, dim3(unsigned(waves)),
                           dim3(rb3f::kLanes), 0, s, a);
    else
        hipLaunchKernelGGL(k_rb3_flags<rb3f::kLeanChunk>, dim3(unsigned(waves)),
                           dim3(rb3f::kLanes), 0, s, a);
    return hipGetLastError();
}

int rb3_residual_blocks(int n) {
    const int64_t rows = int64_t(n) * n;
    return rows < kResidualBlocks ? int(rows) : kResidualBlocks;
}

hipError_t launch_rb3_pack(const double* nat, int64_t ld, double* red, double* black, int n,
                           int64_t pitch, hipStream_t s) {
    const dim3 grid(unsigned((pitch + kThreads - 1) / kThreads), unsigned(n + 2), unsigned(n + 2));
    hipLaunchKernelGGL(k_rb3_pack, grid, dim3(kThreads), 0, s, nat, ld, red, black, n, pitch);
    return hipGetLastError();
}

hipError_t launch_rb3_unpack(double* nat, int64_t ld, const double* red, const double* black,
                             int n, int64_t pitch, hipStream_t s) {
    const dim3 grid(unsigned((pitch + kThreads - 1) / kThreads), unsigned(n), unsigned(n));
    hipLaunchKernelGGL(k_rb3_unpack, grid, dim3(kThreads), 0, s, nat, ld, red, black, n, pitch);
    return hipGetLastError();
}

hipError_t launch_rb3_half(double* self, const double* other, const double* f, int n,
                           int64_t pitch, double h2, int colour, const int* stop, hipStream_t s) {
    const int64_t qs = int64_t(n) / 2 + 1;  // q = 0 .. n / 2
    const int per = n >= kPairMinN ? 2 : 1;  // q-columns per thread
    const int qblocks = int((qs + per * kQ - 1) / (per * kQ)), jblocks = (n + kJ - 1) / kJ;
    const int64_t blocks = int64_t(qblocks) * jblocks * ((n + kPlanes - 1) / kPlanes);
    if (per == 2)
        hipLaunchKernelGGL(k_rb3_half, dim3(unsigned(blocks)), dim3(kQ * kJ), 0, s, self, other, f,
                           n, pitch, h2, colour, qblocks, jblocks, stop);
    else
        hipLaunchKernelGGL(k_rb3_half1, dim3(unsigned(blocks)), dim3(kQ * kJ), 0, s, self, other,
                           f, n, pitch, h2, colour, qblocks, jblocks, stop);
    return hipGetLastError();
}

hipError_t launch_rb3_residual(const double* ur, const double* ub, const double* fr,
                               const double* fb, int n, int64_t pitch, double inv_h2,
                               double* partials, double* out, hipStream_t s) {
    const int blocks = rb3_residual_blocks(n);
    hipLaunchKernelGGL(k_rb3_residual, dim3(blocks), dim3(kThreads), 0, s, ur, ub, fr, fb, n,
                       pitch, inv_h2, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rb3_reduce, dim3(1), dim3(kThreads), 0, s, partials, blocks, out);
    return hipGetLastError();
}

}  // namespace rbgs
