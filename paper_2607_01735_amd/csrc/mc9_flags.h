// Flag-driven four-colour Gauss-Seidel for the 9-point Laplacian: every
// quarter-sweep of a call in one launch, with per-block progress counters in
// place of the three barriers between a sweep's colours and the one between
// sweeps.  This is the dependency rule of Algorithm 2 (Section 2.3) carried
// to the multi-colour stencils the conclusion (Section 5) names.
//
// The four colour arrays of multicolour9.hip (point (i, j) of colour
// (i & 1) + 2 (j & 1) at C[i >> 1][j >> 1]) share one (I, J) index grid,
// cut into blocks of qw columns J x ri rows I.  Quarter-sweep `level`
// (colour level & 3) of block B reads the other three colours in B and in
// the first row or column of its eight neighbours (the stencil has
// corners), and writes its own colour in B.  So it may run once B and its
// eight neighbours have completed `level` quarter-sweeps: every value it
// reads is then the latest, and no neighbour still needs the values it
// overwrites (those are read at the levels before; a neighbour at level + 1
// waits for B).  Every block publishes its counter at every level, also
// where it holds no interior point of that colour, so every counter a wait
// looks at has a producer.
//
// Work items (level, block) are handed out by an atomic ticket in
// level-major order, one one-wave workgroup per item at a time; an item
// waits only on smaller tickets, so the schedule cannot deadlock whatever
// number of workgroups is resident.  Waits are bounded (spin_limit polls,
// then the error word, which makes every workgroup leave).
//
// Within a block lane l takes column J0 + l % qw of rows I0 + l / qw,
// I0 + l / qw + 64 / qw, ..., kChunk rows at a time; each point is updated
// with the plain quarter-sweep's operations in its order (so the result is
// bitwise the same):
//   e = ((u[i+1][j] + u[i-1][j]) + u[i][j+1]) + u[i][j-1]
//   c = ((u[i+1][j+1] + u[i+1][j-1]) + u[i-1][j+1]) + u[i-1][j-1]
//   u[i][j] = ((4 e + c) - c6 f[i][j]) / 20,   c6 = 6 (h h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>

namespace rbgs {
namespace mc9f {

constexpr int kLanes = 64;
constexpr int kErrTimeout = 1;
constexpr int kChunk = 4;  // rows of a lane whose loads are in flight together

struct Args {
    double* u[4];       // colour arrays of u
    const double* f[4]; // colour arrays of f
    int n;
    int64_t pitch;      // elements per colour row
    int rows, cols;     // colour rows I = 0 .. rows - 1, columns J = 0 .. cols - 1
    double c6;          // 6 h^2
    int qw;             // columns per row of lanes (64, 32, 16 or 8)
    int ri;             // rows per block (a multiple of 64 / qw)
    int qblocks, iblocks, nblocks;
    int levels;         // quarter-sweeps of the launch, colour 0 first
    int* ticket;        // next work item (level-major: level * nblocks + block)
    int* progress;      // per block: quarter-sweeps completed
    int* error;         // raised by an expired wait
    int spin_limit;     // polls per wait before giving up
    int delay;          // debug: pseudo-random stall per block and level (0 = off)
    int stall_block;    // debug: block + 1 that never publishes (0 = off)
};

struct Geometry {
    int rows, cols, qw, ri, qblocks, iblocks, nblocks;
};

// Block shape for grid size n with at most max_blocks blocks (>= 64): as
// many blocks as fit, growing the rows per block.
inline Geometry geometry(int n, int max_blocks) {
    Geometry g;
    g.rows = ((n + 1) >> 1) + 1;
    g.cols = ((n + 1) >> 1) + 1;
    g.qw = g.cols > 32 ? 64 : g.cols > 16 ? 32 : g.cols > 8 ? 16 : 8;
    g.qblocks = (g.cols + g.qw - 1) / g.qw;
    g.ri = kLanes / g.qw;
    for (;;) {
        g.iblocks = (g.rows + g.ri - 1) / g.ri;
        const int64_t count = int64_t(g.qblocks) * g.iblocks;
        if (count <= max_blocks || g.ri >= g.rows) {
            g.nblocks = int(count);
            return g;
        }
        g.ri *= 2;
    }
}

__device__ __forceinline__ uint32_t stall_hash(uint32_t h) {
    h ^= h >> 15;
    h *= 0x2c1b3c6du;
    h ^= h >> 12;
    h *= 0x297a2d39u;
    h ^= h >> 15;
    return h;
}

// Waits until block b and its eight neighbours have completed `level`
// quarter-sweeps; false when the wait expired or another wave raised the error.
__device__ __forceinline__ bool wait_neighbours(const Args& a, int b, int level) {
    if (level == 0) return true;
    const int lane = int(threadIdx.x);
    const int bq = b % a.qblocks, bi = b / a.qblocks;
    // lanes 0 .. 8: the 3 x 3 neighbourhood, row by row
    const int ni = bi + lane / 3 - 1, nq = bq + lane % 3 - 1;
    const bool mine = lane < 9 && ni >= 0 && ni < a.iblocks && nq >= 0 && nq < a.qblocks;
    const int* flag = a.progress + (mine ? ni * a.qblocks + nq : 0);
    for (int polls = 0;; ++polls) {
        const int v =
            mine ? __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : INT_MAX;
        if (__all(v >= level)) break;
        if (polls >= a.spin_limit) {
            if (lane == 0)
                __hip_atomic_store(a.error, kErrTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        if ((polls & 255) == 255) {
            const int e = __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__any(e != 0)) return false;
        }
        // back off as the wait grows (polling at full rate from thousands of
        // waves takes cache bandwidth from the waves being waited for)
        if (polls < 16)
            __builtin_amdgcn_s_sleep(1);
        else if (polls < 256)
            __builtin_amdgcn_s_sleep(8);
        else
            __builtin_amdgcn_s_sleep(32);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// Quarter-sweep of colour `colour` over block b.  A lane's rows go kChunk
// at a time: the chunk's loads are issued before any of its stores (the
// stores go to the colour being updated, which none of the loads read).
__device__ __forceinline__ void sweep_block(const Args& a, int b, int colour) {
    const int pi = colour & 1, pj = colour >> 1;
    double* __restrict__ self = a.u[colour];
    const double* __restrict__ ns = a.u[colour ^ 1];  // i +- 1, same j
    const double* __restrict__ ew = a.u[colour ^ 2];  // j +- 1, same i
    const double* __restrict__ cc = a.u[colour ^ 3];  // the corners
    const double* __restrict__ f = a.f[colour];
    const int bq = b % a.qblocks, bi = b / a.qblocks;
    const int lane = int(threadIdx.x);
    const int64_t J = int64_t(bq) * a.qw + lane % a.qw;
    const int64_t j = 2 * J + pj;
    if (J >= a.cols || j < 1 || j > a.n) return;
    const int64_t P = a.pitch;
    const int64_t Jw = J - 1 + pj, Je = J + pj;  // columns of j - 1 and j + 1
    const int64_t I0 = int64_t(bi) * a.ri;
    const int64_t I1 = I0 + a.ri - 1 < a.rows - 1 ? I0 + a.ri - 1 : a.rows - 1;
    const int64_t step = kLanes / a.qw;
    for (int64_t Ic = I0 + lane / a.qw; Ic <= I1; Ic += kChunk * step) {
        double nd[kChunk], nu[kChunk], we[kChunk], ww[kChunk];
        double cde[kChunk], cdw[kChunk], cue[kChunk], cuw[kChunk], fv[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            const int64_t I = Ic + k * step;
            const int64_t i = 2 * I + pi;
            nd[k] = nu[k] = we[k] = ww[k] = cde[k] = cdw[k] = cue[k] = cuw[k] = fv[k] = 0.0;
            if (I > I1 || i < 1 || i > a.n) continue;
            const int64_t Iu = I - 1 + pi, Id = I + pi;  // rows of i - 1 and i + 1
            nd[k] = ns[Id * P + J];
            nu[k] = ns[Iu * P + J];
            we[k] = ew[I * P + Je];
            ww[k] = ew[I * P + Jw];
            cde[k] = cc[Id * P + Je];
            cdw[k] = cc[Id * P + Jw];
            cue[k] = cc[Iu * P + Je];
            cuw[k] = cc[Iu * P + Jw];
            fv[k] = f[I * P + J];
        }
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            const int64_t I = Ic + k * step;
            const int64_t i = 2 * I + pi;
            if (I > I1 || i < 1 || i > a.n) continue;
            double e = nd[k] + nu[k];
            e = e + we[k];
            e = e + ww[k];
            double c = cde[k] + cdw[k];
            c = c + cue[k];
            c = c + cuw[k];
            double s = 4.0 * e + c;
            const double t = a.c6 * fv[k];
            s = s - t;
            self[I * P + J] = s / 20.0;
        }
    }
}

// The persistent kernel's body, run by every workgroup of the launch.
__device__ __forceinline__ void run(const Args& a) {
    const int total = a.levels * a.nblocks;
    for (;;) {
        int t = 0;
        if (threadIdx.x == 0)
            t = __hip_atomic_fetch_add(a.ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= total) return;
        const int level = t / a.nblocks;
        const int b = t - level * a.nblocks;
        if (!wait_neighbours(a, b, level)) return;
        if (a.delay > 0) {
            const uint32_t loops =
                stall_hash(uint32_t(level) * 0x9e3779b9u + uint32_t(b)) % uint32_t(a.delay + 1);
            for (uint32_t w = 0; w < loops; ++w) __builtin_amdgcn_s_sleep(127);
        }
        sweep_block(a, b, level & 3);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (threadIdx.x == 0 && b + 1 != a.stall_block)
            __hip_atomic_store(a.progress + b, level + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace mc9f
}  // namespace rbgs
