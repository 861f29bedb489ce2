// Device-memory bandwidth probe: the copy and triad kernels of the STREAM
// benchmark, which the paper uses to measure attainable memory bandwidth
// (Section 3).  16-byte vector accesses, grid-stride loop, FP64 elements.
#include "rbgs.h"
#include "rbgs_internal.h"

namespace rbgs {
namespace {

// One 16-byte vector per thread and no loop: measured fastest on MI355X
// (grid-stride loops and deeper unrolling both streamed more slowly).
__global__ __launch_bounds__(256) void k_copy(const double2* __restrict__ a,
                                              double2* __restrict__ b, int64_t n2) {
    int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k < n2) b[k] = a[k];
}

__global__ __launch_bounds__(256) void k_triad(double2* __restrict__ a,
                                               const double2* __restrict__ b,
                                               const double2* __restrict__ c, double s,
                                               int64_t n2) {
    int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k < n2) {
        double2 x = b[k], y = c[k];
        double2 r;
        r.x = x.x + s * y.x;
        r.y = x.y + s * y.y;
        a[k] = r;
    }
}

}  // namespace
}  // namespace rbgs

extern "C" int rbgs_stream_probe(int32_t kind, double* a, double* b, double* c, int64_t n_elems,
                                 double s, void* stream) {
    using namespace rbgs;
    if (kind != 0 && kind != 1) return RBGS_EINVAL;
    if (n_elems <= 0 || n_elems % 2 != 0) return RBGS_EINVAL;
    if (!a || !b || (kind == 1 && !c)) return RBGS_EINVAL;
    if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
         reinterpret_cast<uintptr_t>(c)) % 16 != 0)
        return RBGS_EINVAL;
    const int64_t n2 = n_elems / 2;
    const int64_t blocks = (n2 + 255) / 256;
    if (blocks > 0x7fffffff) return RBGS_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (kind == 0)
        hipLaunchKernelGGL(k_copy, dim3(unsigned(blocks)), dim3(256), 0, st,
                           reinterpret_cast<const double2*>(a), reinterpret_cast<double2*>(b), n2);
    else
        hipLaunchKernelGGL(k_triad, dim3(unsigned(blocks)), dim3(256), 0, st,
                           reinterpret_cast<double2*>(a), reinterpret_cast<const double2*>(b),
                           reinterpret_cast<const double2*>(c), s, n2);
    return hipGetLastError() == hipSuccess ? RBGS_OK : RBGS_EHIP;
}
