// Layout kernels: natural <-> split colour layout, FP64 -> FP32 packing,
// the FP64 correction u <- u + e of iterative refinement, a copy of the
// Dirichlet ring between split grids, and a zero fill.
// All are single streaming passes; one thread handles one (row, q) pair,
// i.e. the two natural elements (i, 2q) and (i, 2q+1).
#include "rbgs_internal.h"

namespace rbgs {
namespace {

constexpr int kThreads = 256;

template <typename W>
__global__ __launch_bounds__(kThreads) void k_pack(const W* __restrict__ nat, int64_t ld,
                                                   W* __restrict__ red, W* __restrict__ black,
                                                   int n, int64_t pitch) {
    int64_t q = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    int64_t i = blockIdx.y;
    if (q >= pitch) return;
    // (i, 2q) has colour i & 1; (i, 2q + 1) has the other colour.
    W* even_dst = (i & 1) ? black : red;
    W* odd_dst = (i & 1) ? red : black;
    int64_t j0 = 2 * q, j1 = 2 * q + 1;
    const W* row = nat + i * ld;
    even_dst[i * pitch + q] = (j0 <= n + 1) ? row[j0] : W(0);
    odd_dst[i * pitch + q] = (j1 <= n + 1) ? row[j1] : W(0);
}

// The Dirichlet ring of a split grid, both colours: rows 0 and n+1 whole,
// and in every other row the q-columns 0 and (n+1)/2, which hold j = 0 and
// j = n+1 in one of the two colours (the other colour's interior point at
// those q comes along, harmlessly).  One workgroup per row.
template <typename W>
__global__ __launch_bounds__(64) void k_copy_ring(W* __restrict__ dst_red, W* __restrict__ dst_black,
                                                  const W* __restrict__ src_red,
                                                  const W* __restrict__ src_black, int n,
                                                  int64_t pitch) {
    const int64_t i = blockIdx.x;
    const int64_t at = i * pitch;
    if (i == 0 || i == int64_t(n) + 1) {
        for (int64_t q = threadIdx.x; q < pitch; q += 64) {
            dst_red[at + q] = src_red[at + q];
            dst_black[at + q] = src_black[at + q];
        }
    } else if (threadIdx.x < 2) {
        const int64_t q = threadIdx.x == 0 ? 0 : (int64_t(n) + 1) >> 1;
        dst_red[at + q] = src_red[at + q];
        dst_black[at + q] = src_black[at + q];
    }
}

template <typename W>
__global__ __launch_bounds__(kThreads) void k_unpack(W* __restrict__ nat, int64_t ld,
                                                     const W* __restrict__ red,
                                                     const W* __restrict__ black, int n,
                                                     int64_t pitch) {
    int64_t q = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    int64_t i = int64_t(blockIdx.y) + 1;  // interior rows only: the ring is never written
    if (q >= pitch) return;
    const W* even_src = (i & 1) ? black : red;
    const W* odd_src = (i & 1) ? red : black;
    int64_t j0 = 2 * q, j1 = 2 * q + 1;
    W* row = nat + i * ld;
    if (j0 >= 1 && j0 <= n) row[j0] = even_src[i * pitch + q];
    if (j1 >= 1 && j1 <= n) row[j1] = odd_src[i * pitch + q];
}

__global__ __launch_bounds__(kThreads) void k_pack_f64_to_f32(const double* __restrict__ nat,
                                                              int64_t ld, float* __restrict__ red,
                                                              float* __restrict__ black, int n,
                                                              int64_t pitch) {
    int64_t q = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    int64_t i = blockIdx.y;
    if (q >= pitch) return;
    float* even_dst = (i & 1) ? black : red;
    float* odd_dst = (i & 1) ? red : black;
    int64_t j0 = 2 * q, j1 = 2 * q + 1;
    const double* row = nat + i * ld;
    even_dst[i * pitch + q] = (j0 <= n + 1) ? float(row[j0]) : 0.0f;
    odd_dst[i * pitch + q] = (j1 <= n + 1) ? float(row[j1]) : 0.0f;
}

// u <- u + e at the interior points of row i = blockIdx.y + 1, both colours.
__global__ __launch_bounds__(kThreads) void k_add_correction(double* __restrict__ u_red,
                                                             double* __restrict__ u_black,
                                                             int64_t pitch,
                                                             const float* __restrict__ e_red,
                                                             const float* __restrict__ e_black,
                                                             int64_t e_pitch, int n,
                                                             const int* __restrict__ stop) {
    if (stop != nullptr && *stop != 0) return;  // a converged graph-captured solve
    int64_t q = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    int64_t i = int64_t(blockIdx.y) + 1;
#pragma unroll
    for (int colour = 0; colour < 2; ++colour) {
        int p = int((i + colour) & 1);
        int64_t q_lo = 1 - p, q_hi = (int64_t(n) - p) >> 1;
        if (q < q_lo || q > q_hi) continue;
        double* u = colour ? u_black : u_red;
        const float* e = colour ? e_black : e_red;
        u[i * pitch + q] = u[i * pitch + q] + double(e[i * e_pitch + q]);
    }
}

__global__ __launch_bounds__(kThreads) void k_zero(uint32_t* __restrict__ p, size_t words) {
    size_t k = size_t(blockIdx.x) * kThreads + threadIdx.x;
    size_t stride = size_t(gridDim.x) * kThreads;
    for (; k < words; k += stride) p[k] = 0u;
}

}  // namespace

hipError_t launch_pack(const void* nat, int64_t ld, void* red, void* black, int n, int64_t pitch,
                       int elem_bytes, hipStream_t s) {
    dim3 grid(unsigned((pitch + kThreads - 1) / kThreads), unsigned(n + 2));
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_pack<uint64_t>, grid, dim3(kThreads), 0, s,
                           static_cast<const uint64_t*>(nat), ld, static_cast<uint64_t*>(red),
                           static_cast<uint64_t*>(black), n, pitch);
    else
        hipLaunchKernelGGL(k_pack<uint32_t>, grid, dim3(kThreads), 0, s,
                           static_cast<const uint32_t*>(nat), ld, static_cast<uint32_t*>(red),
                           static_cast<uint32_t*>(black), n, pitch);
    return hipGetLastError();
}

hipError_t launch_unpack(void* nat, int64_t ld, const void* red, const void* black, int n,
                         int64_t pitch, int elem_bytes, hipStream_t s) {
    dim3 grid(unsigned((pitch + kThreads - 1) / kThreads), unsigned(n));
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_unpack<uint64_t>, grid, dim3(kThreads), 0, s,
                           static_cast<uint64_t*>(nat), ld, static_cast<const uint64_t*>(red),
                           static_cast<const uint64_t*>(black), n, pitch);
    else
        hipLaunchKernelGGL(k_unpack<uint32_t>, grid, dim3(kThreads), 0, s,
                           static_cast<uint32_t*>(nat), ld, static_cast<const uint32_t*>(red),
                           static_cast<const uint32_t*>(black), n, pitch);
    return hipGetLastError();
}

hipError_t launch_pack_f64_to_f32(const double* nat, int64_t ld, float* red, float* black, int n,
                                  int64_t pitch, hipStream_t s) {
    dim3 grid(unsigned((pitch + kThreads - 1) / kThreads), unsigned(n + 2));
    hipLaunchKernelGGL(k_pack_f64_to_f32, grid, dim3(kThreads), 0, s, nat, ld, red, black, n,
                       pitch);
    return hipGetLastError();
}

hipError_t launch_add_correction(double* u_red, double* u_black, int64_t pitch,
                                 const float* e_red, const float* e_black, int64_t e_pitch, int n,
                                 hipStream_t s, const int* stop) {
    dim3 grid(unsigned((pitch + kThreads - 1) / kThreads), unsigned(n));
    hipLaunchKernelGGL(k_add_correction, grid, dim3(kThreads), 0, s, u_red, u_black, pitch, e_red,
                       e_black, e_pitch, n, stop);
    return hipGetLastError();
}

hipError_t launch_copy_ring(void* dst_red, void* dst_black, const void* src_red,
                            const void* src_black, int n, int64_t pitch, int elem_bytes,
                            hipStream_t s) {
    const dim3 grid(unsigned(n + 2));
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_copy_ring<uint64_t>, grid, dim3(64), 0, s,
                           static_cast<uint64_t*>(dst_red), static_cast<uint64_t*>(dst_black),
                           static_cast<const uint64_t*>(src_red),
                           static_cast<const uint64_t*>(src_black), n, pitch);
    else
        hipLaunchKernelGGL(k_copy_ring<uint32_t>, grid, dim3(64), 0, s,
                           static_cast<uint32_t*>(dst_red), static_cast<uint32_t*>(dst_black),
                           static_cast<const uint32_t*>(src_red),
                           static_cast<const uint32_t*>(src_black), n, pitch);
    return hipGetLastError();
}

namespace {
__global__ __launch_bounds__(256) void k_copy_unless(uint4* __restrict__ dst,
                                                     const uint4* __restrict__ src, size_t n,
                                                     const int* __restrict__ stop) {
    if (stop != nullptr && *stop != 0) return;
    for (size_t k = size_t(blockIdx.x) * 256 + threadIdx.x; k < n; k += size_t(gridDim.x) * 256)
        dst[k] = src[k];
}
}  // namespace

hipError_t launch_copy_unless(void* dst, const void* src, size_t bytes, const int* stop,
                              hipStream_t s) {
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_copy_unless, dim3(unsigned(blocks)), dim3(256), 0, s,
                       static_cast<uint4*>(dst), static_cast<const uint4*>(src), n, stop);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    size_t words = bytes / 4;
    if (words == 0) return hipSuccess;
    size_t blocks = (words + kThreads - 1) / kThreads;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero, dim3(unsigned(blocks)), dim3(kThreads), 0, s,
                       static_cast<uint32_t*>(p), words);
    return hipGetLastError();
}

}  // namespace rbgs
