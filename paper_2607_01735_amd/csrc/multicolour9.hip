// Four-colour Gauss-Seidel for the 9-point Laplacian (an extension: the
// conclusion, Section 5, names multi-colour variants for wider stencils as
// future work).  The 9-point stencil couples diagonal neighbours, so the
// red-black split no longer separates the points of one colour; colour
// (i & 1) + 2 (j & 1) does, and one sweep is four quarter-sweeps (colours
// 0, 1, 2, 3), each a kernel launch: twice the barriers of red-black.
//
// Layout: one array per colour, the generalisation of the red/black split
// (Section 2.1 stores the colours apart): point (i, j) of colour c sits at
// C_c[i >> 1][j >> 1], rows 0 .. (n+1) >> 1 of `pitch` elements.  A
// quarter-sweep then streams the other three colours, its own right-hand
// side and its own colour once each: 5 words per updated point, 40 B per
// grid point per sweep (the natural layout would move every cache line of
// the grid on each of the four passes).
//
// Update (each operation rounded once, no contraction):
//   e = ((u[i+1][j] + u[i-1][j]) + u[i][j+1]) + u[i][j-1]
//   c = ((u[i+1][j+1] + u[i+1][j-1]) + u[i-1][j+1]) + u[i-1][j-1]
//   u[i][j] = ((4 e + c) - c6 f[i][j]) / 20,   c6 = 6 (h h).
#include <algorithm>
#include <cmath>

#include "mc9_flags.h"
#include "rbgs_internal.h"

namespace rbgs {
namespace {

constexpr int kThreads = 256;
// Colour rows one thread marches (the rows of the i-flipped colours are
// reused from registers): measured on MI355X, two rows per thread is the
// fastest at 8191^2 (0.489 ms per sweep against 0.540 with one row and 0.502
// with four), one row at 255^2 (more threads for a small grid).
inline int rows_per_thread(int n) { return n <= 1024 ? 1 : 2; }
constexpr int kResidualBlocks = 1024;

struct Colours {
    double* c[4];
};
struct ConstColours {
    const double* c[4];
};

// natural (n+2) x ld -> four colour arrays; the 2 x 2 block (2I .. 2I+1,
// 2J .. 2J+1) holds one point of each colour.  Points beyond the grid get 0.
__global__ __launch_bounds__(kThreads) void k_mc9_pack(const double* __restrict__ nat, int64_t ld,
                                                       Colours dst, int n, int64_t pitch,
                                                       int rows) {
    const int64_t J = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t I = blockIdx.y;
    if (J >= pitch || I >= rows) return;
    for (int pi = 0; pi < 2; ++pi) {
        const int64_t i = 2 * I + pi;
        for (int pj = 0; pj < 2; ++pj) {
            const int64_t j = 2 * J + pj;
            const bool in = i <= n + 1 && j <= n + 1;
            dst.c[pi + 2 * pj][I * pitch + J] = in ? nat[i * ld + j] : 0.0;
        }
    }
}

// four colour arrays -> natural interior (the ring is not written).
__global__ __launch_bounds__(kThreads) void k_mc9_unpack(double* __restrict__ nat, int64_t ld,
                                                         ConstColours src, int n, int64_t pitch,
                                                         int rows) {
    const int64_t J = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t I = blockIdx.y;
    if (J >= pitch || I >= rows) return;
    for (int pi = 0; pi < 2; ++pi) {
        const int64_t i = 2 * I + pi;
        for (int pj = 0; pj < 2; ++pj) {
            const int64_t j = 2 * J + pj;
            if (i >= 1 && i <= n && j >= 1 && j <= n)
                nat[i * ld + j] = src.c[pi + 2 * pj][I * pitch + J];
        }
    }
}

// One quarter-sweep of colour (pi, pj): thread J of a strip of rpt colour
// rows updates points (2I + pi, 2J + pj).  The rows of
// the i-flipped colours it needs are I - 1 + pi and I + pi; each step loads
// the new row I + pi of both and reuses I - 1 + pi from the last step.
__global__ __launch_bounds__(kThreads) void k_mc9_quarter(
    double* __restrict__ self, const double* __restrict__ ns, const double* __restrict__ ew,
    const double* __restrict__ cc, const double* __restrict__ f, int n, int64_t pitch, int pi,
    int pj, double c6, int rpt, const int* stop) {
    if (stop && *stop) return;
    const int64_t J = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t j = 2 * J + pj;
    if (j < 1 || j > n) return;
    const int64_t I0 = int64_t(blockIdx.y) * rpt;
    const int64_t Jw = J - 1 + pj, Je = J + pj;  // columns of j - 1 and j + 1
    // row I0 - 1 + pi of the i-flipped colours (clamped; only read when i >= 1)
    int64_t Iu = I0 - 1 + pi;
    double up_ns = 0.0, up_w = 0.0, up_e = 0.0;
    if (Iu >= 0) {
        up_ns = ns[Iu * pitch + J];
        up_w = cc[Iu * pitch + Jw];
        up_e = cc[Iu * pitch + Je];
    }
    for (int k = 0; k < rpt; ++k) {
        const int64_t I = I0 + k;
        const int64_t i = 2 * I + pi;
        if (i > n) break;
        const int64_t Id = I + pi;  // row of i + 1 in the i-flipped colours
        const double dn_ns = ns[Id * pitch + J];
        const double dn_w = cc[Id * pitch + Jw];
        const double dn_e = cc[Id * pitch + Je];
        if (i >= 1) {
            double e = dn_ns + up_ns;
            e = e + ew[I * pitch + Je];
            e = e + ew[I * pitch + Jw];
            double c = dn_e + dn_w;
            c = c + up_e;
            c = c + up_w;
            double s = 4.0 * e + c;
            // f is read once per sweep and the new value is not read again
            // before the next quarter-sweep has streamed its colours: both
            // go through the caches as streaming (non-temporal)
            const double t = c6 * __builtin_nontemporal_load(f + I * pitch + J);
            s = s - t;
            __builtin_nontemporal_store(s / 20.0, self + I * pitch + J);
        }
        up_ns = dn_ns;
        up_w = dn_w;
        up_e = dn_e;
    }
}

__device__ __forceinline__ double colour_at(const ConstColours& u, int64_t i, int64_t j,
                                            int64_t pitch) {
    return u.c[(i & 1) + 2 * (j & 1)][(i >> 1) * pitch + (j >> 1)];
}

// Residual norms: block b takes colour rows b, b + gridDim.x, ...; each
// thread the four points of its 2 x 2 block in the order (pi, pj) = (0,0),
// (1,0), (0,1), (1,1); fixed-order tree in LDS; one partial pair per block.
__global__ __launch_bounds__(kThreads) void k_mc9_residual(ConstColours u, ConstColours f, int n,
                                                           int64_t pitch, int rows,
                                                           double inv6h2, double* partials) {
    __shared__ double sr[kThreads], sb[kThreads];
    double acc_r = 0.0, acc_b = 0.0;
    const int64_t n1 = int64_t(n) + 1;
    for (int64_t I = blockIdx.x; I < rows; I += gridDim.x) {
        for (int64_t J = threadIdx.x; J < pitch; J += kThreads) {
            for (int pj = 0; pj < 2; ++pj) {
                for (int pi = 0; pi < 2; ++pi) {
                    const int64_t i = 2 * I + pi, j = 2 * J + pj;
                    if (i < 1 || i > n || j < 1 || j > n) continue;
                    const double uN = colour_at(u, i + 1, j, pitch), uS = colour_at(u, i - 1, j, pitch);
                    const double uE = colour_at(u, i, j + 1, pitch), uW = colour_at(u, i, j - 1, pitch);
                    const double uNE = colour_at(u, i + 1, j + 1, pitch);
                    const double uNW = colour_at(u, i + 1, j - 1, pitch);
                    const double uSE = colour_at(u, i - 1, j + 1, pitch);
                    const double uSW = colour_at(u, i - 1, j - 1, pitch);
                    double e = uN + uS;
                    e = e + uE;
                    e = e + uW;
                    double c = uNE + uNW;
                    c = c + uSE;
                    c = c + uSW;
                    const double fc = colour_at(f, i, j, pitch);
                    const double lap = ((4.0 * e + c) - 20.0 * colour_at(u, i, j, pitch)) * inv6h2;
                    const double r = fc - lap;
                    // b: only the ring's values (the interior of u set to zero)
                    auto ring = [&](int64_t a, int64_t b2, double v) {
                        return (a == 0 || a == n1 || b2 == 0 || b2 == n1) ? v : 0.0;
                    };
                    double eb = ring(i + 1, j, uN) + ring(i - 1, j, uS);
                    eb = eb + ring(i, j + 1, uE);
                    eb = eb + ring(i, j - 1, uW);
                    double cb = ring(i + 1, j + 1, uNE) + ring(i + 1, j - 1, uNW);
                    cb = cb + ring(i - 1, j + 1, uSE);
                    cb = cb + ring(i - 1, j - 1, uSW);
                    const double b = fc - (4.0 * eb + cb) * inv6h2;
                    acc_r += r * r;
                    acc_b += b * b;
                }
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

__global__ __launch_bounds__(kThreads) void k_mc9_reduce(const double* __restrict__ partials,
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

// The flag-driven form (mc9_flags.h): one launch for every quarter-sweep.
__global__ __launch_bounds__(mc9f::kLanes) void k_mc9_flags(mc9f::Args a) { mc9f::run(a); }

// Bound on the blocks per quarter-sweep: every item costs a ticket on one
// device-wide counter while an item's time grows with its size; as in the
// 3D form about sqrt(points / 10), capped at the waves the chip holds.
int mc9_flags_target(int n, int capacity) {
    const double items = std::sqrt(double(n) * double(n) / 10.0);
    return int(std::max(64.0, std::min(double(capacity), items)));
}

}  // namespace

int mc9_flags_capacity() {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(&k_mc9_flags), mc9f::kLanes, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const int64_t c = int64_t(cus) * per_cu;
    return int(c < kMc9MaxBlocks ? c : kMc9MaxBlocks);
}

int mc9_flags_blocks(int n, int capacity) {
    if (capacity < 64) return 0;
    return mc9f::geometry(n, mc9_flags_target(n, capacity)).nblocks;
}

hipError_t launch_mc9_flags(double* const u[4], double* const f[4], int n, double c6, int levels,
                            int capacity, int* ticket, int* progress, int* error, int spin_limit,
                            int delay, int stall_block, hipStream_t s) {
    if (capacity < 64) return hipErrorInvalidValue;
    const mc9f::Geometry geo = mc9f::geometry(n, mc9_flags_target(n, capacity));
    if (int64_t(levels) * geo.nblocks >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    mc9f::Args a;
    for (int c = 0; c < 4; ++c) {
        a.u[c] = u[c];
        a.f[c] = f[c];
    }
    a.n = n;
    a.pitch = mc9_pitch(n);
    a.rows = geo.rows;
    a.cols = geo.cols;
    a.c6 = c6;
    a.qw = geo.qw;
    a.ri = geo.ri;
    a.qblocks = geo.qblocks;
    a.iblocks = geo.iblocks;
    a.nblocks = geo.nblocks;
    a.levels = levels;
    a.ticket = ticket;
    a.progress = progress;
    a.error = error;
    a.spin_limit = spin_limit;
    a.delay = delay;
    a.stall_block = stall_block;
    // one wave per block: each takes the next level's item as it finishes one
    int64_t waves = std::min<int64_t>(capacity, geo.nblocks);
    const int64_t items = int64_t(levels) * geo.nblocks;
    if (waves > items) waves = items;
    if (waves < 1) waves = 1;
    hipLaunchKernelGGL(k_mc9_flags, dim3(unsigned(waves)), dim3(mc9f::kLanes), 0, s, a);
    return hipGetLastError();
}

int mc9_rows(int n) { return ((n + 1) >> 1) + 1; }

int64_t mc9_pitch(int n) {
    const int64_t cols = ((int64_t(n) + 1) >> 1) + 1;
    return (cols + 31) / 32 * 32;
}

int mc9_residual_blocks(int n) { return mc9_rows(n) < kResidualBlocks ? mc9_rows(n) : kResidualBlocks; }

hipError_t launch_mc9_pack(const double* nat, int64_t ld, double* const colours[4], int n,
                           hipStream_t s) {
    const int64_t pitch = mc9_pitch(n);
    const int rows = mc9_rows(n);
    Colours d{{colours[0], colours[1], colours[2], colours[3]}};
    hipLaunchKernelGGL(k_mc9_pack, dim3(unsigned((pitch + kThreads - 1) / kThreads), unsigned(rows)),
                       dim3(kThreads), 0, s, nat, ld, d, n, pitch, rows);
    return hipGetLastError();
}

hipError_t launch_mc9_unpack(double* nat, int64_t ld, double* const colours[4], int n,
                             hipStream_t s) {
    const int64_t pitch = mc9_pitch(n);
    const int rows = mc9_rows(n);
    ConstColours c{{colours[0], colours[1], colours[2], colours[3]}};
    hipLaunchKernelGGL(k_mc9_unpack, dim3(unsigned((pitch + kThreads - 1) / kThreads), unsigned(rows)),
                       dim3(kThreads), 0, s, nat, ld, c, n, pitch, rows);
    return hipGetLastError();
}

hipError_t launch_mc9_quarter(double* const u[4], double* const f[4], int n, double c6,
                              int colour, const int* stop, hipStream_t s) {
    const int64_t pitch = mc9_pitch(n);
    const int rows = mc9_rows(n);
    const int pi = colour & 1, pj = (colour >> 1) & 1;
    const int rpt = rows_per_thread(n);
    const dim3 grid(unsigned((pitch + kThreads - 1) / kThreads), unsigned((rows + rpt - 1) / rpt));
    hipLaunchKernelGGL(k_mc9_quarter, grid, dim3(kThreads), 0, s, u[colour], u[colour ^ 1],
                       u[colour ^ 2], u[colour ^ 3], f[colour], n, pitch, pi, pj, c6, rpt, stop);
    return hipGetLastError();
}

hipError_t launch_mc9_residual(double* const u[4], double* const f[4], int n, double inv6h2,
                               double* partials, double* out, hipStream_t s) {
    const int64_t pitch = mc9_pitch(n);
    const int rows = mc9_rows(n);
    const int blocks = mc9_residual_blocks(n);
    ConstColours cu{{u[0], u[1], u[2], u[3]}}, cf{{f[0], f[1], f[2], f[3]}};
    hipLaunchKernelGGL(k_mc9_residual, dim3(blocks), dim3(kThreads), 0, s, cu, cf, n, pitch, rows,
                       inv6h2, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mc9_reduce, dim3(1), dim3(kThreads), 0, s, partials, blocks, out);
    return hipGetLastError();
}

}  // namespace rbgs
