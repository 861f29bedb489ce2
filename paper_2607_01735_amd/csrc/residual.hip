// Residual kernels.  For every interior point
//   s   = ((u[i+1][j] + u[i-1][j]) + u[i][j+1]) + u[i][j-1]
//   r   = f - (s - 4 u[i][j]) * (1/h^2)
//   sb  = the same sum with interior neighbours replaced by 0 (ring only)
//   b   = f - sb * (1/h^2)
// all in FP64 (FP32 data is widened first).  ||r||^2 and ||b||^2 are summed
// in a fixed order: each thread sequentially over its points, then a fixed
// binary tree in each workgroup, then one workgroup over the per-workgroup
// partials in slot order.  No floating-point atomics, so the result is
// bitwise reproducible for a given grid size.
#include <mutex>

#include "rbgs_internal.h"

namespace rbgs {
namespace {

constexpr int kRows = 8;  // rows marched per workgroup

__device__ __forceinline__ float round_to_bf16(float x) {
    // bfloat16 keeps the top 16 bits of binary32; round to nearest, ties to
    // even, by adding 0x7fff plus the lowest kept bit before truncation.
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu) != 0u) {
        b |= 0x00400000u;
    } else {
        b += 0x7fffu + ((b >> 16) & 1u);
    }
    return __uint_as_float(b & 0xffff0000u);
}

template <int BT>
__device__ __forceinline__ void block_reduce_store(double r2, double b2, double* partials,
                                                   int slot) {
    __shared__ double sr[BT];
    __shared__ double sb[BT];
    const int t = threadIdx.x;
    sr[t] = r2;
    sb[t] = b2;
    __syncthreads();
#pragma unroll
    for (int stride = BT / 2; stride > 0; stride >>= 1) {
        if (t < stride) {
            sr[t] = sr[t] + sr[t + stride];
            sb[t] = sb[t] + sb[t + stride];
        }
        __syncthreads();
    }
    if (t == 0) {
        partials[2 * slot] = sr[0];
        partials[2 * slot + 1] = sb[0];
    }
}

// Split layout: one thread = one split column q (one point of each colour
// per row), marching kRows rows with the column's red and black values of
// rows i-1, i, i+1 in registers, so u and f are each read once (16 B per
// point in FP64); the other in-row neighbour is the next or previous
// column's value (a cache hit).  Per row the red point's terms are added
// before the black point's.  Blocks of 256 threads.
template <typename T>
__global__ __launch_bounds__(256) void k_residual_split(
    const T* __restrict__ u_red, const T* __restrict__ u_black, const T* __restrict__ f_red,
    const T* __restrict__ f_black, int n, int64_t pitch, double inv_h2, double* partials,
    int col_blocks, float* __restrict__ r_red, float* __restrict__ r_black, int64_t r_pitch,
    int rhs_bf16, int* __restrict__ overflow, T* __restrict__ nat, int64_t ld) {
    const int strip = blockIdx.x / col_blocks;
    const int cb = blockIdx.x - strip * col_blocks;
    const int64_t q = int64_t(cb) * 256 + threadIdx.x;
    const int i0 = 1 + strip * kRows;
    const int i1 = min(n, i0 + kRows - 1);
    double r2 = 0.0, b2 = 0.0;
    if (q <= (n >> 1)) {
        // [colour][row i-1, i, i+1] of column q
        double col[2][3];
        col[0][0] = double(u_red[int64_t(i0 - 1) * pitch + q]);
        col[1][0] = double(u_black[int64_t(i0 - 1) * pitch + q]);
        col[0][1] = double(u_red[int64_t(i0) * pitch + q]);
        col[1][1] = double(u_black[int64_t(i0) * pitch + q]);
        for (int i = i0; i <= i1; ++i) {
            col[0][2] = double(u_red[int64_t(i + 1) * pitch + q]);
            col[1][2] = double(u_black[int64_t(i + 1) * pitch + q]);
#pragma unroll
            for (int colour = 0; colour < 2; ++colour) {
                const int p = (i + colour) & 1;
                const int64_t q_lo = 1 - p, q_hi = (int64_t(n) - p) >> 1;
                if (q < q_lo || q > q_hi) continue;
                const T* other = colour ? u_red : u_black;
                const double(&o)[3] = col[1 - colour];
                const int64_t j = p + 2 * q;
                const double dn = o[2];
                const double up = o[0];
                // in-row neighbours: other[i][q + p] and other[i][q - 1 + p]
                const double right = p ? double(other[int64_t(i) * pitch + q + 1]) : o[1];
                const double left = p ? o[1] : double(other[int64_t(i) * pitch + q - 1]);
                const double c = col[colour][1];
                // the unpack of a fixed-count solve rides along: this point's
                // value into the natural array (interior only, as the unpack)
                if (nat) nat[int64_t(i) * ld + j] = T(c);  // exact: c is a widened T
                // f is read once (streaming, non-temporal)
                const double f = double(__builtin_nontemporal_load(
                    (colour ? f_black : f_red) + int64_t(i) * pitch + q));
                double s = dn + up;
                s = s + right;
                s = s + left;
                double r = f - (s - 4.0 * c) * inv_h2;
                double sbv = (i + 1 == n + 1 ? dn : 0.0) + (i - 1 == 0 ? up : 0.0);
                sbv = sbv + (j + 1 == n + 1 ? right : 0.0);
                sbv = sbv + (j - 1 == 0 ? left : 0.0);
                double b = f - sbv * inv_h2;
                r2 = r2 + r * r;
                b2 = b2 + b * b;
                float* r_out = colour ? r_black : r_red;
                if (r_out) {
                    float r32 = float(r);
                    if (rhs_bf16) r32 = round_to_bf16(r32);
                    r_out[int64_t(i) * r_pitch + q] = r32;
                    // a finite residual that its binary32 / bfloat16 form
                    // cannot hold (every writer stores the same 1)
                    if (overflow && isinf(r32) && isfinite(r)) *overflow = 1;
                }
            }
#pragma unroll
            for (int colour = 0; colour < 2; ++colour) {
                col[colour][0] = col[colour][1];
                col[colour][1] = col[colour][2];
            }
        }
    }
    block_reduce_store<256>(r2, b2, partials, blockIdx.x);
}

// Natural layout: one thread = one column j, marching kRows rows.
template <typename T>
__global__ __launch_bounds__(256) void k_residual_natural(const T* __restrict__ u,
                                                          const T* __restrict__ fn, int n,
                                                          int64_t ld, double inv_h2,
                                                          double* partials, int col_blocks) {
    const int strip = blockIdx.x / col_blocks;
    const int cb = blockIdx.x - strip * col_blocks;
    const int64_t j = int64_t(cb) * 256 + threadIdx.x + 1;
    const int i0 = 1 + strip * kRows;
    const int i1 = min(n, i0 + kRows - 1);
    double r2 = 0.0, b2 = 0.0;
    if (j <= n) {
        for (int i = i0; i <= i1; ++i) {
            const T* row = u + int64_t(i) * ld;
            double dn = double(u[int64_t(i + 1) * ld + j]);
            double up = double(u[int64_t(i - 1) * ld + j]);
            double right = double(row[j + 1]);
            double left = double(row[j - 1]);
            double c = double(row[j]);
            double f = double(fn[int64_t(i) * ld + j]);
            double s = dn + up;
            s = s + right;
            s = s + left;
            double r = f - (s - 4.0 * c) * inv_h2;
            double sbv = (i + 1 == n + 1 ? dn : 0.0) + (i - 1 == 0 ? up : 0.0);
            sbv = sbv + (j + 1 == n + 1 ? right : 0.0);
            sbv = sbv + (j - 1 == 0 ? left : 0.0);
            double b = f - sbv * inv_h2;
            r2 = r2 + r * r;
            b2 = b2 + b * b;
        }
    }
    block_reduce_store<256>(r2, b2, partials, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ partials,
                                                         int slots, double* __restrict__ out) {
    double r2 = 0.0, b2 = 0.0;
    for (int k = threadIdx.x; k < slots; k += 256) {
        r2 = r2 + partials[2 * k];
        b2 = b2 + partials[2 * k + 1];
    }
    __shared__ double sr[256];
    __shared__ double sb[256];
    const int t = threadIdx.x;
    sr[t] = r2;
    sb[t] = b2;
    __syncthreads();
    for (int stride = 128; stride > 0; stride >>= 1) {
        if (t < stride) {
            sr[t] = sr[t] + sr[t + stride];
            sb[t] = sb[t] + sb[t + stride];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = sr[0];
        out[1] = sb[0];
    }
}

int split_col_blocks(int n) { return int(((int64_t(n) >> 1) + 1 + 255) / 256); }
int natural_col_blocks(int n) { return (n + 255) / 256; }
int strips(int n) { return (n + kRows - 1) / kRows; }

}  // namespace

int residual_partial_slots(int n, int64_t, size_t) { return split_col_blocks(n) * strips(n); }
int residual_natural_partial_slots(int n) { return natural_col_blocks(n) * strips(n); }

// ---------------------------------------------------------------------------
// Scratch for the entry point that allocates nothing (rbgs_residual_noalloc):
// the natural-layout residual's partial sums and final sums live in this
// file-scope device array instead of a caller workspace.  Each device holds
// its own copy at its own address, looked up once per device with
// hipGetSymbolAddress (the array's name is not a device address in host
// code).  Every call on a device shares that device's array.
// ---------------------------------------------------------------------------
namespace {
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t static_scratch(void** ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

size_t residual_noalloc_bytes(int n) {
    return 256 + size_t(residual_natural_partial_slots(n)) * 2 * sizeof(double);
}

template <typename T>
hipError_t launch_residual_split(const T* u_red, const T* u_black, const T* f_red,
                                 const T* f_black, int n, int64_t pitch, double inv_h2,
                                 double* partials, double* out, float* r_out_red,
                                 float* r_out_black, int64_t r_pitch, int rhs_bf16,
                                 hipStream_t s, int* overflow, T* nat, int64_t ld) {
    const int cb = split_col_blocks(n);
    dim3 grid(unsigned(cb * strips(n)));
    hipLaunchKernelGGL((k_residual_split<T>), grid, dim3(256), 0, s, u_red, u_black, f_red,
                       f_black, n, pitch, inv_h2, partials, cb, r_out_red, r_out_black, r_pitch,
                       rhs_bf16, overflow, nat, ld);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, partials,
                       int(grid.x * grid.y), out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_residual_natural(const T* u, const T* f, int n, int64_t ld, double inv_h2,
                                   double* partials, double* out, hipStream_t s) {
    const int cb = natural_col_blocks(n);
    dim3 grid(unsigned(cb * strips(n)));
    hipLaunchKernelGGL((k_residual_natural<T>), grid, dim3(256), 0, s, u, f, n, ld, inv_h2,
                       partials, cb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, partials, int(grid.x), out);
    return hipGetLastError();
}

namespace {
// The convergence test of a graph-captured solve, after each round's
// residual: rel = ||r|| / ||b|| (||r|| when b = 0), formed exactly as the
// host forms it; the flag stops the later rounds' sweeps.  state = {flag,
// rounds done, overflow, stall, previous rel (double at byte 16)}; cap =
// rounds the sweep budget allows.  With watch (a refinement that may widen
// its inner precision) the rounds also stop when the residual kernel found
// a value its right-hand-side format cannot hold (state[2]), or when round
// first_check or a later one leaves rel no lower than the round before
// (init_prev before the first round; state[3] = 1): the host then widens
// the precision.
__global__ __launch_bounds__(64) void k_judge(const double* __restrict__ sums, double rel_tol,
                                              int* __restrict__ state, int cap, int watch,
                                              int first_check, double init_prev) {
    if (threadIdx.x != 0 || state[0] != 0) return;
    const double rn = sqrt(sums[0]);
    const double bn = sqrt(sums[1]);
    const double rel = bn > 0.0 ? rn / bn : rn;
    const int rounds = state[1] + 1;
    state[1] = rounds;
    bool stop = rel <= rel_tol || !isfinite(rel) || rounds >= cap;
    if (watch) {
        double* prev = reinterpret_cast<double*>(state + 4);
        const double before = rounds == 1 ? init_prev : *prev;
        if (state[2] != 0) stop = true;
        if (rounds >= first_check && rel >= before) {
            state[3] = 1;
            stop = true;
        }
        *prev = rel;
    }
    if (stop) state[0] = 1;
}
}  // namespace

hipError_t launch_judge(const double* sums, double rel_tol, int* state, int cap, hipStream_t s,
                        int watch, int first_check, double init_prev) {
    hipLaunchKernelGGL(k_judge, dim3(1), dim3(64), 0, s, sums, rel_tol, state, cap, watch,
                       first_check, init_prev);
    return hipGetLastError();
}

template hipError_t launch_residual_split<double>(const double*, const double*, const double*,
                                                  const double*, int, int64_t, double, double*,
                                                  double*, float*, float*, int64_t, int,
                                                  hipStream_t, int*, double*, int64_t);
template hipError_t launch_residual_split<float>(const float*, const float*, const float*,
                                                 const float*, int, int64_t, double, double*,
                                                 double*, float*, float*, int64_t, int,
                                                 hipStream_t, int*, float*, int64_t);
template hipError_t launch_residual_natural<double>(const double*, const double*, int, int64_t,
                                                    double, double*, double*, hipStream_t);
template hipError_t launch_residual_natural<float>(const float*, const float*, int, int64_t,
                                                   double, double*, double*, hipStream_t);

}  // namespace rbgs
