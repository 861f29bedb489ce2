// Grid transfers between vertex-centred levels (fine N_f = 2 N_c + 1), used to
// generate converged solutions by nested iteration: solve the coarsest level,
// prolong, sweep the next level, and so on.  Coarse point (I, J) sits on fine
// point (2I, 2J) in natural indexing (ring rows/columns are index 0 and N+1 on
// both levels, and 2(N_c + 1) = N_f + 1).  Both kernels are HBM streams with
// one thread per output point; a batch of equally sized grids is laid out at a
// constant element stride.
#include <hip/hip_runtime.h>

#include "rbgs_internal.h"

namespace rbgs {
namespace {

constexpr int kTransferThreads = 256;
constexpr int kMaxGridZ = 1024;

// Full weighting, (1,2,1) x (1,2,1) / 16, of the fine interior onto the coarse
// interior.  Every fine point read, 2I - 1 .. 2I + 1 with 1 <= I <= N_c, is a
// fine interior point, so the fine ring is never read.
template <typename T>
__global__ void __launch_bounds__(kTransferThreads)
k_restrict(const T* __restrict__ fine, int64_t fine_ld, int64_t fine_stride,
           T* __restrict__ coarse, int64_t coarse_ld, int64_t coarse_stride, int nc, int batch) {
    const int J = blockIdx.x * kTransferThreads + threadIdx.x + 1;
    const int I = blockIdx.y + 1;
    if (J > nc) return;
    for (int b = blockIdx.z; b < batch; b += gridDim.z) {
        const T* x = fine + int64_t(b) * fine_stride + int64_t(2 * I) * fine_ld + 2 * J;
        const T* up = x - fine_ld;
        const T* dn = x + fine_ld;
        const T top = (up[-1] + T(2) * up[0]) + up[1];
        const T mid = (x[-1] + T(2) * x[0]) + x[1];
        const T bot = (dn[-1] + T(2) * dn[0]) + dn[1];
        coarse[int64_t(b) * coarse_stride + int64_t(I) * coarse_ld + J] =
            ((top + T(2) * mid) + bot) * T(0.0625);
    }
}

// Bilinear interpolation of the coarse grid (ring included) onto the fine
// interior; the fine ring is left as it is.
template <typename T>
__global__ void __launch_bounds__(kTransferThreads)
k_prolong(const T* __restrict__ coarse, int64_t coarse_ld, int64_t coarse_stride,
          T* __restrict__ fine, int64_t fine_ld, int64_t fine_stride, int nf, int batch) {
    const int j = blockIdx.x * kTransferThreads + threadIdx.x + 1;
    const int i = blockIdx.y + 1;
    if (j > nf) return;
    const int I0 = i >> 1, J0 = j >> 1;
    const bool oi = i & 1, oj = j & 1;
    for (int b = blockIdx.z; b < batch; b += gridDim.z) {
        const T* c = coarse + int64_t(b) * coarse_stride + int64_t(I0) * coarse_ld + J0;
        T v;
        if (!oi && !oj) {
            v = c[0];
        } else if (oi && !oj) {
            v = (c[0] + c[coarse_ld]) * T(0.5);
        } else if (!oi && oj) {
            v = (c[0] + c[1]) * T(0.5);
        } else {
            v = ((c[0] + c[1]) + (c[coarse_ld] + c[coarse_ld + 1])) * T(0.25);
        }
        fine[int64_t(b) * fine_stride + int64_t(i) * fine_ld + j] = v;
    }
}

dim3 transfer_grid(int cols, int rows, int batch) {
    return dim3((cols + kTransferThreads - 1) / kTransferThreads, rows,
                batch < kMaxGridZ ? batch : kMaxGridZ);
}

}  // namespace

template <typename T>
hipError_t launch_restrict(const T* fine, int64_t fine_ld, int64_t fine_stride, T* coarse,
                           int64_t coarse_ld, int64_t coarse_stride, int nc, int batch,
                           hipStream_t s) {
    if (batch <= 0 || nc <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_restrict<T>, transfer_grid(nc, nc, batch), dim3(kTransferThreads), 0, s,
                       fine, fine_ld, fine_stride, coarse, coarse_ld, coarse_stride, nc, batch);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(const T* coarse, int64_t coarse_ld, int64_t coarse_stride, T* fine,
                          int64_t fine_ld, int64_t fine_stride, int nf, int batch,
                          hipStream_t s) {
    if (batch <= 0 || nf <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prolong<T>, transfer_grid(nf, nf, batch), dim3(kTransferThreads), 0, s,
                       coarse, coarse_ld, coarse_stride, fine, fine_ld, fine_stride, nf, batch);
    return hipGetLastError();
}

template hipError_t launch_restrict<double>(const double*, int64_t, int64_t, double*, int64_t,
                                            int64_t, int, int, hipStream_t);
template hipError_t launch_restrict<float>(const float*, int64_t, int64_t, float*, int64_t,
                                           int64_t, int, int, hipStream_t);
template hipError_t launch_prolong<double>(const double*, int64_t, int64_t, double*, int64_t,
                                           int64_t, int, int, hipStream_t);
template hipError_t launch_prolong<float>(const float*, int64_t, int64_t, float*, int64_t,
                                          int64_t, int, int, hipStream_t);

}  // namespace rbgs
