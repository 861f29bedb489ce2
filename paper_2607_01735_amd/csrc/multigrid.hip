// Grid transfers of the multigrid cycle on split (red/black) arrays.
//
// The cycle uses red-black Gauss-Seidel as its smoother: an extension beyond
// the paper, whose conclusion (Section 5) names multilevel odd-even
// techniques as future work.  The hierarchy is vertex-centred: a fine grid of
// n_f = 2 n_c + 1 interior points per side holds coarse point (I, J) at fine
// point (2I, 2J), the ring being index 0 and n+1 on every level.
//
// k_mg_restrict: the fine residual r = f - A_h u (the residual of Eq. (1)'s
//   system, same operations in the same order as the residual kernel), its
//   full weighting onto the coarse right-hand side, and a zero coarse
//   iterate, in one pass.  The fine residual is never stored.
// k_mg_prolong_add: u += bilinear interpolation of the coarse iterate.
//
// Rounding order (every + and * rounded once, no contraction):
//   full weighting: row_a = (r[a][2J-1] + 2 r[a][2J]) + r[a][2J+1] for the
//   fine rows a = 2I-1, 2I, 2I+1, then ((row_0 + 2 row_1) + row_2) * 0.0625;
//   prolongation at fine (i, j) with I = i >> 1, J = j >> 1: e[I][J] (both
//   even), (e[I][J] + e[I+1][J]) * 0.5 (i odd), (e[I][J] + e[I][J+1]) * 0.5
//   (j odd), ((e[I][J] + e[I][J+1]) + (e[I+1][J] + e[I+1][J+1])) * 0.25
//   (both odd); then u + v.
#include "rbgs_internal.h"

namespace rbgs {
namespace {

constexpr int kMgThreads = 256;
constexpr int kRestrictRows = 4;  // coarse rows one thread marches down

// Element k of a split row, 0 outside [0, pitch): only ever used for points
// whose values are discarded.
__device__ __forceinline__ double at_or_zero(const double* row, int64_t k, int64_t pitch) {
    return (k >= 0 && k < pitch) ? row[k] : 0.0;
}

// The seven u values of fine row i at columns 4q-2 .. 4q+4.  Even columns
// of row i have colour i & 1, odd columns the other; column j sits at j >> 1.
__device__ __forceinline__ void load_u7(const double* __restrict__ u_red,
                                        const double* __restrict__ u_black, int64_t i, int64_t q,
                                        int64_t pitch, double out[7]) {
    const double* ev = ((i & 1) ? u_black : u_red) + i * pitch;
    const double* od = ((i & 1) ? u_red : u_black) + i * pitch;
    out[0] = at_or_zero(ev, 2 * q - 1, pitch);  // 4q - 2
    out[1] = at_or_zero(od, 2 * q - 1, pitch);  // 4q - 1
    out[2] = at_or_zero(ev, 2 * q, pitch);      // 4q
    out[3] = at_or_zero(od, 2 * q, pitch);      // 4q + 1
    out[4] = at_or_zero(ev, 2 * q + 1, pitch);  // 4q + 2
    out[5] = at_or_zero(od, 2 * q + 1, pitch);  // 4q + 3
    out[6] = at_or_zero(ev, 2 * q + 2, pitch);  // 4q + 4
}

// Residual of fine row i at columns 4q-1 .. 4q+3 from u rows i-1, i, i+1.
__device__ __forceinline__ void residual5(const double up[7], const double mid[7],
                                          const double dn[7], const double* __restrict__ f_red,
                                          const double* __restrict__ f_black, int64_t i,
                                          int64_t q, int64_t pitch, double inv_h2,
                                          double r[5]) {
    const double* ev = ((i & 1) ? f_black : f_red) + i * pitch;
    const double* od = ((i & 1) ? f_red : f_black) + i * pitch;
    double f[5];
    f[0] = at_or_zero(od, 2 * q - 1, pitch);  // 4q - 1
    f[1] = at_or_zero(ev, 2 * q, pitch);      // 4q
    f[2] = at_or_zero(od, 2 * q, pitch);      // 4q + 1
    f[3] = at_or_zero(ev, 2 * q + 1, pitch);  // 4q + 2
    f[4] = at_or_zero(od, 2 * q + 1, pitch);  // 4q + 3
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        double s = dn[k + 1] + up[k + 1];
        s = s + mid[k + 2];
        s = s + mid[k];
        const double lap = (s - 4.0 * mid[k + 1]) * inv_h2;
        r[k] = f[k] - lap;
    }
}

__device__ __forceinline__ double weight_row(double a, double b, double c) {
    return (a + 2.0 * b) + c;
}

// One thread per coarse q (coarse columns J = 2q and 2q + 1) and a strip of
// kRestrictRows coarse rows; it keeps three fine u rows and the previous
// fine residual row in registers while marching down.
__global__ __launch_bounds__(kMgThreads) void k_mg_restrict(
    const double* __restrict__ u_red, const double* __restrict__ u_black,
    const double* __restrict__ f_red, const double* __restrict__ f_black, int64_t pitch,
    double inv_h2, double* __restrict__ fc_red, double* __restrict__ fc_black,
    double* __restrict__ uc_red, double* __restrict__ uc_black, int nc, int64_t cpitch,
    const int* stop) {
    if (stop && *stop) return;
    const int64_t q = int64_t(blockIdx.x) * kMgThreads + threadIdx.x;
    if (q >= cpitch) return;
    const int64_t I0 = int64_t(blockIdx.y) * kRestrictRows + 1;
    const int64_t I1 = I0 + kRestrictRows - 1 < nc ? I0 + kRestrictRows - 1 : nc;
    for (int64_t I = I0; I <= I1; ++I) {  // a zero coarse iterate (ring columns stay zero)
        uc_red[I * cpitch + q] = 0.0;
        uc_black[I * cpitch + q] = 0.0;
    }
    const bool j0_ok = q >= 1 && 2 * q <= nc;
    const bool j1_ok = 2 * q + 1 <= nc;
    if (!j0_ok && !j1_ok) return;
    double a[7], b[7], c[7];
    double r_top[5], r_mid[5], r_bot[5];
    load_u7(u_red, u_black, 2 * I0 - 2, q, pitch, a);
    load_u7(u_red, u_black, 2 * I0 - 1, q, pitch, b);
    load_u7(u_red, u_black, 2 * I0, q, pitch, c);
    residual5(a, b, c, f_red, f_black, 2 * I0 - 1, q, pitch, inv_h2, r_top);
    // window now: a = row 2I-2, b = 2I-1, c = 2I
    for (int64_t I = I0; I <= I1; ++I) {
        const int64_t i = 2 * I;
#pragma unroll
        for (int m = 0; m < 7; ++m) a[m] = b[m];
#pragma unroll
        for (int m = 0; m < 7; ++m) b[m] = c[m];
        load_u7(u_red, u_black, i + 1, q, pitch, c);  // a, b, c = rows 2I-1, 2I, 2I+1
        residual5(a, b, c, f_red, f_black, i, q, pitch, inv_h2, r_mid);
#pragma unroll
        for (int m = 0; m < 7; ++m) a[m] = b[m];
#pragma unroll
        for (int m = 0; m < 7; ++m) b[m] = c[m];
        load_u7(u_red, u_black, i + 2, q, pitch, c);  // rows 2I, 2I+1, 2I+2
        residual5(a, b, c, f_red, f_black, i + 1, q, pitch, inv_h2, r_bot);
        // coarse (I, 2q) has colour I & 1; (I, 2q + 1) the other
        double* even_dst = (I & 1) ? fc_black : fc_red;
        double* odd_dst = (I & 1) ? fc_red : fc_black;
        if (j0_ok) {
            const double t = weight_row(r_top[0], r_top[1], r_top[2]);
            const double m = weight_row(r_mid[0], r_mid[1], r_mid[2]);
            const double bt = weight_row(r_bot[0], r_bot[1], r_bot[2]);
            even_dst[I * cpitch + q] = ((t + 2.0 * m) + bt) * 0.0625;
        }
        if (j1_ok) {
            const double t = weight_row(r_top[2], r_top[3], r_top[4]);
            const double m = weight_row(r_mid[2], r_mid[3], r_mid[4]);
            const double bt = weight_row(r_bot[2], r_bot[3], r_bot[4]);
            odd_dst[I * cpitch + q] = ((t + 2.0 * m) + bt) * 0.0625;
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) r_top[k] = r_bot[k];
    }
}

// Coarse value e[I][J] of a split coarse grid.
__device__ __forceinline__ double coarse_at(const double* __restrict__ e_red,
                                            const double* __restrict__ e_black, int64_t I,
                                            int64_t J, int64_t cpitch) {
    const double* a = ((I + J) & 1) ? e_black : e_red;
    return a[I * cpitch + (J >> 1)];
}

// One thread per fine (i, q): the two fine points (i, 2q) and (i, 2q + 1),
// one of each colour, both at split column q.
__global__ __launch_bounds__(kMgThreads) void k_mg_prolong_add(
    double* __restrict__ u_red, double* __restrict__ u_black, int64_t pitch, int nf,
    const double* __restrict__ e_red, const double* __restrict__ e_black, int64_t cpitch,
    const int* stop) {
    if (stop && *stop) return;
    const int64_t q = int64_t(blockIdx.x) * kMgThreads + threadIdx.x;
    const int64_t i = int64_t(blockIdx.y) + 1;
    if (2 * q > nf) return;
    const int64_t I = i >> 1;
    double* ev = ((i & 1) ? u_black : u_red) + i * pitch + q;  // (i, 2q)
    double* od = ((i & 1) ? u_red : u_black) + i * pitch + q;  // (i, 2q + 1)
    const double e00 = coarse_at(e_red, e_black, I, q, cpitch);
    const double e01 = coarse_at(e_red, e_black, I, q + 1, cpitch);
    double v_even, v_odd;
    if ((i & 1) == 0) {
        v_even = e00;
        v_odd = (e00 + e01) * 0.5;
    } else {
        const double e10 = coarse_at(e_red, e_black, I + 1, q, cpitch);
        const double e11 = coarse_at(e_red, e_black, I + 1, q + 1, cpitch);
        v_even = (e00 + e10) * 0.5;
        v_odd = ((e00 + e01) + (e10 + e11)) * 0.25;
    }
    if (q >= 1) *ev = *ev + v_even;
    if (2 * q + 1 <= nf) *od = *od + v_odd;
}

// ----- prolongation fused into the first post-smoothing red half-sweep ------
// The red half-sweep after the coarse correction overwrites every red value
// without reading it, and the black half-sweep after it overwrites every
// black value without reading it; so "u += P e, red half-sweep" needs the
// corrected values of the black neighbours only, formed on the fly (black +
// interpolant, ring values unchanged) and never stored.  The red values and,
// after the black half-sweep, the black values are bitwise those of the
// unfused sequence.  13 B per fine point (black and red f read, red written,
// the coarse grid through the cache) instead of 18 + 12.

// One thread per red point (i, j), i + j even.  The interpolants of its four
// black neighbours need five coarse values when i and j are even (the cross
// around (I, J) = (i/2, j/2)) and four when both are odd (the block (I, J) ..
// (I+1, J+1), I = i >> 1, J = j >> 1); each is loaded once and every
// interpolant is formed exactly as k_mg_prolong_add forms it for that
// point's parity.  Neighbours on the ring take no correction.
__global__ __launch_bounds__(kMgThreads) void k_mg_prolong_red(
    double* __restrict__ u_red, const double* __restrict__ u_black,
    const double* __restrict__ f_red, int64_t pitch, int nf, double h2,
    const double* __restrict__ e_red, const double* __restrict__ e_black, int64_t cpitch,
    const int* stop) {
    if (stop && *stop) return;
    const int64_t q = int64_t(blockIdx.x) * kMgThreads + threadIdx.x;
    const int64_t i = int64_t(blockIdx.y) + 1;
    const int64_t p = i & 1;
    if (q < 1 - p || q > ((int64_t(nf) - p) >> 1)) return;
    const int64_t j = 2 * q + p;
    const int64_t I = i >> 1, J = j >> 1;
    // black neighbours: (i+1, j), (i-1, j), (i, j+1), (i, j-1); black (i', j')
    // sits at u_black[i' pitch + (j' >> 1)]
    const double b_dn = u_black[(i + 1) * pitch + (j >> 1)];
    const double b_up = u_black[(i - 1) * pitch + (j >> 1)];
    const double b_rt = u_black[i * pitch + ((j + 1) >> 1)];
    const double b_lt = u_black[i * pitch + ((j - 1) >> 1)];
    double v_dn, v_up, v_rt, v_lt;
    if (p == 0) {  // i, j even
        const double c = coarse_at(e_red, e_black, I, J, cpitch);
        const double cn = coarse_at(e_red, e_black, I + 1, J, cpitch);
        const double cs = coarse_at(e_red, e_black, I - 1, J, cpitch);
        const double ce = coarse_at(e_red, e_black, I, J + 1, cpitch);
        const double cw = coarse_at(e_red, e_black, I, J - 1, cpitch);
        v_dn = (c + cn) * 0.5;   // (i+1, j): i+1 odd, j even, I' = I
        v_up = (cs + c) * 0.5;   // (i-1, j): I' = I - 1
        v_rt = (c + ce) * 0.5;   // (i, j+1): i even, j+1 odd, J' = J
        v_lt = (cw + c) * 0.5;   // (i, j-1): J' = J - 1
    } else {  // i, j odd
        const double e00 = coarse_at(e_red, e_black, I, J, cpitch);
        const double e01 = coarse_at(e_red, e_black, I, J + 1, cpitch);
        const double e10 = coarse_at(e_red, e_black, I + 1, J, cpitch);
        const double e11 = coarse_at(e_red, e_black, I + 1, J + 1, cpitch);
        v_dn = (e10 + e11) * 0.5;  // (i+1, j): i+1 even, j odd, I' = I + 1, J' = J
        v_up = (e00 + e01) * 0.5;  // (i-1, j): I' = I
        v_rt = (e01 + e11) * 0.5;  // (i, j+1): i odd, j+1 even, J' = J + 1
        v_lt = (e00 + e10) * 0.5;  // (i, j-1): J' = J
    }
    const double dn = i + 1 <= nf ? b_dn + v_dn : b_dn;
    const double up = i - 1 >= 1 ? b_up + v_up : b_up;
    const double right = j + 1 <= nf ? b_rt + v_rt : b_rt;
    const double left = j - 1 >= 1 ? b_lt + v_lt : b_lt;
    double s = dn + up;
    s = s + right;
    s = s + left;
    const double t = h2 * __builtin_nontemporal_load(f_red + i * pitch + q);  // read once
    s = s - t;
    u_red[i * pitch + q] = 0.25 * s;
}

// ----- the coarse end of the cycle in one workgroup ------------------------
// Levels of at most kMgCoarseN points per side cost little work but two
// launches per sweep; below that size the rest of the V-cycle (its smoothing,
// transfers and coarsest sweeps, in the order of the level-by-level cycle)
// runs in one workgroup of kCoarseThreads threads with a barrier between
// phases; the arrays stay in the level workspaces (L2-resident at these
// sizes).  Every point's arithmetic is the kernels' above, so the iterate is
// the same bit for bit.

constexpr int kCoarseThreads = 1024;

__device__ __forceinline__ double split_at(const double* red, const double* black, int64_t i,
                                           int64_t j, int64_t pitch) {
    return (((i + j) & 1) ? black : red)[i * pitch + (j >> 1)];
}

__device__ void cw_half_sweep(const MgCoarseLevel& L, int colour) {
    double* self = colour ? L.u_black : L.u_red;
    const double* other = colour ? L.u_red : L.u_black;
    const double* f = colour ? L.f_black : L.f_red;
    const int64_t pitch = L.pitch;
    const int W = (L.n >> 1) + 1;
    for (int idx = threadIdx.x; idx < L.n * W; idx += kCoarseThreads) {
        const int64_t i = idx / W + 1, q = idx % W;
        const int64_t p = (i + colour) & 1;
        if (q < 1 - p || q > ((int64_t(L.n) - p) >> 1)) continue;
        const double* orow = other + i * pitch;
        double s = other[(i + 1) * pitch + q] + other[(i - 1) * pitch + q];
        s = s + orow[q + p];
        s = s + orow[q - 1 + p];
        const double t = L.h2 * f[i * pitch + q];
        s = s - t;
        self[i * pitch + q] = 0.25 * s;
    }
}

__device__ __forceinline__ double cw_residual(const MgCoarseLevel& L, int64_t i, int64_t j) {
    const int64_t pitch = L.pitch;
    double s = split_at(L.u_red, L.u_black, i + 1, j, pitch) +
               split_at(L.u_red, L.u_black, i - 1, j, pitch);
    s = s + split_at(L.u_red, L.u_black, i, j + 1, pitch);
    s = s + split_at(L.u_red, L.u_black, i, j - 1, pitch);
    const double lap = (s - 4.0 * split_at(L.u_red, L.u_black, i, j, pitch)) * L.inv_h2;
    return split_at(L.f_red, L.f_black, i, j, pitch) - lap;
}

__device__ void cw_restrict(const MgCoarseLevel& F, const MgCoarseLevel& C) {
    const int nc = C.n;
    for (int idx = threadIdx.x; idx < nc * nc; idx += kCoarseThreads) {
        const int64_t I = idx / nc + 1, J = idx % nc + 1;
        double row[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int64_t i = 2 * I - 1 + a;
            row[a] = weight_row(cw_residual(F, i, 2 * J - 1), cw_residual(F, i, 2 * J),
                                cw_residual(F, i, 2 * J + 1));
        }
        double* fdst = ((I + J) & 1) ? C.f_black : C.f_red;
        double* udst = ((I + J) & 1) ? C.u_black : C.u_red;
        fdst[I * C.pitch + (J >> 1)] = ((row[0] + 2.0 * row[1]) + row[2]) * 0.0625;
        udst[I * C.pitch + (J >> 1)] = 0.0;
    }
}

__device__ void cw_prolong_add(const MgCoarseLevel& C, const MgCoarseLevel& F) {
    const int nf = F.n;
    for (int idx = threadIdx.x; idx < nf * nf; idx += kCoarseThreads) {
        const int64_t i = idx / nf + 1, j = idx % nf + 1;
        const int64_t I = i >> 1, J = j >> 1;
        const double e00 = split_at(C.u_red, C.u_black, I, J, C.pitch);
        double v;
        if ((i & 1) == 0 && (j & 1) == 0) {
            v = e00;
        } else if ((i & 1) == 1 && (j & 1) == 0) {
            v = (e00 + split_at(C.u_red, C.u_black, I + 1, J, C.pitch)) * 0.5;
        } else if ((i & 1) == 0) {
            v = (e00 + split_at(C.u_red, C.u_black, I, J + 1, C.pitch)) * 0.5;
        } else {
            const double e01 = split_at(C.u_red, C.u_black, I, J + 1, C.pitch);
            const double e10 = split_at(C.u_red, C.u_black, I + 1, J, C.pitch);
            const double e11 = split_at(C.u_red, C.u_black, I + 1, J + 1, C.pitch);
            v = ((e00 + e01) + (e10 + e11)) * 0.25;
        }
        double* dst = (((i + j) & 1) ? F.u_black : F.u_red) + i * F.pitch + (j >> 1);
        *dst = *dst + v;
    }
}

__device__ void cw_sweeps(const MgCoarseLevel& L, int count) {
    for (int s = 0; s < count; ++s) {
        cw_half_sweep(L, 0);
        __syncthreads();
        cw_half_sweep(L, 1);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kCoarseThreads) void k_mg_coarse_vcycle(MgCoarseLevels lv, int nu1,
                                                                    int nu2, int coarse_sweeps,
                                                                    const int* stop) {
    if (stop && *stop) return;
    const int m = lv.count;
    for (int l = 0; l + 1 < m; ++l) {
        cw_sweeps(lv.level[l], nu1);
        cw_restrict(lv.level[l], lv.level[l + 1]);
        __syncthreads();
    }
    cw_sweeps(lv.level[m - 1], coarse_sweeps);
    for (int l = m - 2; l >= 0; --l) {
        cw_prolong_add(lv.level[l + 1], lv.level[l]);
        __syncthreads();
        cw_sweeps(lv.level[l], nu2);
    }
}

}  // namespace

hipError_t launch_mg_coarse_vcycle(const MgCoarseLevels& levels, int nu1, int nu2,
                                   int coarse_sweeps, const int* stop, hipStream_t s) {
    if (levels.count < 1 || levels.count > kMgMaxCoarseLevels) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mg_coarse_vcycle, dim3(1), dim3(kCoarseThreads), 0, s, levels, nu1, nu2,
                       coarse_sweeps, stop);
    return hipGetLastError();
}

hipError_t launch_mg_prolong_red(double* u_red, const double* u_black, const double* f_red,
                                 int64_t pitch, int nf, double h2, const double* e_red,
                                 const double* e_black, int64_t cpitch, const int* stop,
                                 hipStream_t s) {
    if (nf < 3) return hipSuccess;
    const int64_t qs = int64_t(nf) / 2 + 1;
    const dim3 grid(unsigned((qs + kMgThreads - 1) / kMgThreads), unsigned(nf));
    hipLaunchKernelGGL(k_mg_prolong_red, grid, dim3(kMgThreads), 0, s, u_red, u_black, f_red,
                       pitch, nf, h2, e_red, e_black, cpitch, stop);
    return hipGetLastError();
}

hipError_t launch_mg_restrict(const double* u_red, const double* u_black, const double* f_red,
                              const double* f_black, int64_t pitch, double inv_h2,
                              double* fc_red, double* fc_black, double* uc_red, double* uc_black,
                              int nc, int64_t cpitch, const int* stop, hipStream_t s) {
    if (nc < 1) return hipSuccess;
    const dim3 grid(unsigned((cpitch + kMgThreads - 1) / kMgThreads),
                    unsigned((nc + kRestrictRows - 1) / kRestrictRows));
    hipLaunchKernelGGL(k_mg_restrict, grid, dim3(kMgThreads), 0, s, u_red, u_black, f_red,
                       f_black, pitch, inv_h2, fc_red, fc_black, uc_red, uc_black, nc, cpitch,
                       stop);
    return hipGetLastError();
}

hipError_t launch_mg_prolong_add(double* u_red, double* u_black, int64_t pitch, int nf,
                                 const double* e_red, const double* e_black, int64_t cpitch,
                                 const int* stop, hipStream_t s) {
    if (nf < 3) return hipSuccess;
    const int64_t qs = int64_t(nf) / 2 + 1;  // q = 0 .. n_c
    const dim3 grid(unsigned((qs + kMgThreads - 1) / kMgThreads), unsigned(nf));
    hipLaunchKernelGGL(k_mg_prolong_add, grid, dim3(kMgThreads), 0, s, u_red, u_black, pitch, nf,
                       e_red, e_black, cpitch, stop);
    return hipGetLastError();
}

}  // namespace rbgs
