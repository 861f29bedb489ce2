// Flag-driven red-black Gauss-Seidel in three dimensions: every half-sweep
// of a call in one launch, with per-block progress counters in place of the
// barrier between half-sweeps.  This is the dependency rule of Algorithm 2
// (Section 2.3), a stripe waiting only on the stripes next to it, carried
// to blocks of a 3D grid (the conclusion, Section 5, names higher
// dimensions as future work).
//
// The interior is cut into blocks of qw q-columns x rj rows (index j) x rz
// planes (index i) of the split layout of sweep3d.hip.  Half-sweep `level`
// (red for even levels) of block B reads the other colour inside B and on
// the faces of its six face neighbours, and writes its own colour inside B.
// So it may run once B and its six face neighbours have completed `level`
// half-sweeps: then every value it reads is the previous half-sweep's, and
// no neighbour still needs the values it overwrites (a neighbour at level
// - 1 reads them; a neighbour at level + 1 waits for B).  A block's
// counter holds the half-sweeps it has completed.
//
// Work items (level, block) are handed out by an atomic ticket in
// level-major order, one wave per workgroup taking one item at a time.  An
// item waits only on items of the previous level, whose tickets are
// smaller, so the unfinished item with the smallest ticket always has its
// dependencies met and the wave holding it runs it: the schedule cannot
// deadlock however many of the launch's workgroups are resident at once.
// Waits are bounded all the same: a wait that outlasts spin_limit polls
// raises the error word and the wave leaves, and the others leave when they
// see the error word.
//
// Within a block a lane takes the q-column q0 + lane % qw of rows j0 +
// lane / qw, j0 + lane / qw + 64 / qw, ..., marching each row's column down
// the block's planes C planes at a time: the loads of a chunk are issued
// before any of its stores, then the points are updated with the same
// operations in the same order as the plain half-sweep (so the result is
// bitwise the same).  Two chunk sizes are built: kDeepChunk keeps more
// loads of one wave in flight (one wave per SIMD), kLeanChunk needs fewer
// registers, so four waves fit on a SIMD and the largest grids get more
// and smaller blocks in flight; the launch picks one by grid size.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>

namespace rbgs {
namespace rb3f {

constexpr int kLanes = 64;
constexpr int kErrTimeout = 1;
constexpr int kDeepChunk = 8;  // planes whose loads are in flight together: 1 wave per SIMD
constexpr int kLeanChunk = 2;  // 4 waves per SIMD

struct Args {
    double* red;
    double* black;
    const double* f_red;
    const double* f_black;
    int n;
    int64_t pitch;
    double h2;
    int qw;            // q-columns a wave covers at once (64, 32, 16 or 8)
    int rj, rz;        // rows and planes per block (rj a multiple of 64 / qw)
    int qblocks, jblocks, zblocks, nblocks;
    int levels;        // half-sweeps of the launch, red first
    int* ticket;       // next work item (level-major: level * nblocks + block)
    int* progress;     // per block: half-sweeps completed
    int* error;        // raised by an expired wait
    int spin_limit;    // polls per wait before giving up
    int delay;         // debug: pseudo-random stall per block and level (0 = off)
    int stall_block;   // debug: block + 1 that never publishes (0 = off)
    const int* stop;   // converged flag of a graph-captured solve (nullptr: none)
};

struct Geometry {
    int qw, rj, rz, qblocks, jblocks, zblocks, nblocks;
};

// Block shape for grid size n with at most max_blocks blocks (>= 64): the
// smallest blocks that fit, so that the waves of the launch share each
// half-sweep.  Planes grow to 16 first (each plane step of a column loads
// one new value of the other colour), then rows and planes in turn.
inline Geometry geometry(int n, int max_blocks) {
    Geometry g;
    const int qs = n / 2 + 1;  // q = 0 .. n / 2
    g.qw = qs > 32 ? 64 : qs > 16 ? 32 : qs > 8 ? 16 : 8;
    g.qblocks = (qs + g.qw - 1) / g.qw;
    g.rj = kLanes / g.qw;
    g.rz = 1;
    for (;;) {
        g.jblocks = (n + g.rj - 1) / g.rj;
        g.zblocks = (n + g.rz - 1) / g.rz;
        const int64_t count = int64_t(g.qblocks) * g.jblocks * g.zblocks;
        if (count <= max_blocks || (g.rj >= n && g.rz >= n)) {
            g.nblocks = int(count);
            return g;
        }
        if (g.rz < 16 || (g.rj >= g.rz && g.rz < n) || g.rj >= n)
            g.rz *= 2;
        else
            g.rj *= 2;
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

// Waits until block b and its face neighbours have completed `level`
// half-sweeps; false when the wait expired or another wave raised the error.
__device__ __forceinline__ bool wait_neighbours(const Args& a, int b, int level) {
    if (level == 0) return true;
    const int lane = int(threadIdx.x);
    const int bq = b % a.qblocks, bj = (b / a.qblocks) % a.jblocks,
              bz = b / (a.qblocks * a.jblocks);
    // lanes 0 .. 6: the block itself, then q -/+ 1, j -/+ 1, i -/+ 1
    const int d = lane - 1;
    const int nq = bq + (d == 0 ? -1 : d == 1 ? 1 : 0);
    const int nj = bj + (d == 2 ? -1 : d == 3 ? 1 : 0);
    const int nz = bz + (d == 4 ? -1 : d == 5 ? 1 : 0);
    const bool mine = lane < 7 && nq >= 0 && nq < a.qblocks && nj >= 0 && nj < a.jblocks &&
                      nz >= 0 && nz < a.zblocks;
    const int* flag = a.progress + (mine ? (nz * a.jblocks + nj) * a.qblocks + nq : 0);
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
        // back off as the wait grows: thousands of waves polling at full
        // rate would take cache bandwidth from the waves they wait for
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

// Half-sweep of colour `colour` over block b, C planes at a time.
template <int C>
__device__ __forceinline__ void sweep_block(const Args& a, int b, int colour) {
    double* __restrict__ self = colour ? a.black : a.red;
    const double* __restrict__ other = colour ? a.red : a.black;
    const double* __restrict__ f = colour ? a.f_black : a.f_red;
    const int bq = b % a.qblocks, bj = (b / a.qblocks) % a.jblocks,
              bz = b / (a.qblocks * a.jblocks);
    const int lane = int(threadIdx.x);
    const int64_t q = int64_t(bq) * a.qw + lane % a.qw;
    if (q >= a.pitch || 2 * q > a.n) return;  // no interior point of either parity beyond
    const int step = kLanes / a.qw;
    const int64_t n = a.n, np2 = n + 2, P = a.pitch;
    const int64_t i0 = int64_t(bz) * a.rz + 1;
    const int64_t i1 = i0 + a.rz - 1 < n ? i0 + a.rz - 1 : n;
    const int64_t j0 = int64_t(bj) * a.rj + 1;
    const int64_t j1 = j0 + a.rj - 1 < n ? j0 + a.rj - 1 : n;
    for (int64_t j = j0 + lane / a.qw; j <= j1; j += step) {
        // o_dn, o_c: the other colour's column at the planes below and at the
        // current one
        double o_dn = other[((i0 - 1) * np2 + j) * P + q];
        double o_c = other[(i0 * np2 + j) * P + q];
        for (int64_t ic = i0; ic <= i1; ic += C) {
            double up[C], jp[C], jm[C], kx[C], fv[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int64_t i = ic + c;
                up[c] = jp[c] = jm[c] = kx[c] = fv[c] = 0.0;
                if (i > i1) continue;
                up[c] = other[((i + 1) * np2 + j) * P + q];
                const int64_t p = (i + j + colour) & 1;
                const int64_t k = 2 * q + p;
                if (k >= 1 && k <= n) {
                    const int64_t r = (i * np2 + j) * P;
                    jp[c] = other[r + P + q];  // row j + 1 of plane i
                    jm[c] = other[r - P + q];
                    kx[c] = other[r + q + (p ? 1 : -1)];  // the k neighbour not at q
                    fv[c] = f[r + q];
                }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int64_t i = ic + c;
                if (i > i1) break;
                const int64_t p = (i + j + colour) & 1;
                const int64_t k = 2 * q + p;
                if (k >= 1 && k <= n) {
                    const double kp = p ? kx[c] : o_c;
                    const double km = p ? o_c : kx[c];
                    double s = up[c] + o_dn;
                    s = s + jp[c];
                    s = s + jm[c];
                    s = s + kp;
                    s = s + km;
                    const double t = a.h2 * fv[c];
                    s = s - t;
                    self[(i * np2 + j) * P + q] = s / 6.0;
                }
                o_dn = o_c;
                o_c = up[c];
            }
        }
    }
}

// The persistent kernel's body, run by every workgroup of the launch.
template <int C>
__device__ __forceinline__ void run(const Args& a) {
    if (a.stop && *a.stop) return;
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
        sweep_block<C>(a, b, level & 1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (threadIdx.x == 0 && b + 1 != a.stall_block)
            __hip_atomic_store(a.progress + b, level + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace rb3f
}  // namespace rbgs
