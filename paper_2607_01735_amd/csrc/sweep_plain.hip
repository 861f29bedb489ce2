// Plain half-sweep kernel: one launch updates every interior point of one
// colour (Eq. (1)), so consecutive launches play the role of the barriers
// after each colour in Algorithm 1.  A variant over-relaxes the update
// (red-black SOR); it also reads the colour it writes, 4 words per update.
//
// Data: split colour layout (rbgs_internal.h).  A workgroup owns a column
// band of BT*V q-columns and a strip of R interior rows; each thread owns V
// consecutive q-columns (one 16-byte vector) and marches down the strip,
// keeping rows i-1, i, i+1 of the other colour in registers, so the other
// colour is read from HBM about once ((R+2)/R times), the own right-hand side
// once, and the own colour written once: 3 words per point update.  The
// horizontal neighbour that lies outside the thread's vector (q-1 or q+V)
// comes from the neighbouring lane through DPP.
//
// Term order (no FMA contraction, -ffp-contract=off):
//   s = O[i+1][q] + O[i-1][q]; s += right; s += left; s -= h2*f; u = 0.25*s
// which is u_{i+1,j} + u_{i-1,j} + u_{i,j+1} + u_{i,j-1} - h^2 f_ij of Eq. (1).
#include "rbgs_internal.h"

namespace rbgs {
namespace {

// Whole-wave DPP shifts: lane i receives lane i+1's value (wave_shl:1) or
// lane i-1's (wave_shr:1); a lane with no source keeps its own value.
template <int CTRL>
__device__ __forceinline__ int dpp_int(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_val(double v) {
    return __hiloint2double(dpp_int<CTRL>(__double2hiint(v)), dpp_int<CTRL>(__double2loint(v)));
}
template <int CTRL>
__device__ __forceinline__ float dpp_val(float v) {
    return __int_as_float(dpp_int<CTRL>(__float_as_int(v)));
}
template <typename T>
__device__ __forceinline__ T lane_from_next(T v) { return dpp_val<0x130>(v); }
template <typename T>
__device__ __forceinline__ T lane_from_prev(T v) { return dpp_val<0x138>(v); }

template <typename T, int V>
struct alignas(sizeof(T) * V) Pack {
    T v[V];
};

template <typename T, int V>
__device__ __forceinline__ Pack<T, V> load_pack(const T* p) {
    return *reinterpret_cast<const Pack<T, V>*>(p);
}

// The right-hand side is read exactly once per launch and the updated
// colour is not read again within it: both go through non-temporal
// accesses so they do not displace the other colour's rows, which the
// workgroups of neighbouring strips re-read from L2.
template <typename T, int V>
__device__ __forceinline__ Pack<T, V> load_pack_nt(const T* p) {
    typedef T VT __attribute__((ext_vector_type(V)));
    VT x = __builtin_nontemporal_load(reinterpret_cast<const VT*>(p));
    Pack<T, V> r;
#pragma unroll
    for (int e = 0; e < V; ++e) r.v[e] = x[e];
    return r;
}

template <typename T, int V>
__device__ __forceinline__ void store_pack_nt(T* p, const Pack<T, V>& v) {
    typedef T VT __attribute__((ext_vector_type(V)));
    VT x;
#pragma unroll
    for (int e = 0; e < V; ++e) x[e] = v.v[e];
    __builtin_nontemporal_store(x, reinterpret_cast<VT*>(p));
}

// Update row i whose parity p = (i + colour) & 1 is a compile-time value.
// up/mid/dn: other colour, rows i-1, i, i+1 at q0..q0+V-1.
// SOR: the Gauss-Seidel value g relaxes the old value, u + omega (g - u),
// each operation rounded once (red-black SOR, the over-relaxed method).
template <typename T, int V, int P, bool SOR>
__device__ __forceinline__ void update_row(T* __restrict__ self_row, const T* __restrict__ mid_row,
                                           const Pack<T, V>& up, const Pack<T, V>& mid,
                                           const Pack<T, V>& dn, const Pack<T, V>& fc, T h2,
                                           int64_t q0, int n, T omega) {
    // P = 1: right neighbour of q is q+1, left is q; P = 0: right q, left q-1.
    // The value outside the thread's vector is the neighbouring lane's first
    // (or last) element, taken through a DPP whole-wave shift; only the lanes
    // at a wave edge, or next to the last active lane, read it from memory.
    // This halves the load instructions the texture units see per row.
    const int lane = threadIdx.x & 63;
    T extra;
    if constexpr (P) {
        extra = lane_from_next(mid.v[0]);
        if (lane == 63 || q0 + V > (n >> 1)) extra = mid_row[q0 + V];
    } else {
        extra = lane_from_prev(mid.v[V - 1]);
        if (lane == 0) extra = mid_row[q0 - 1];
    }
    Pack<T, V> out;
    Pack<T, V> old;
    if constexpr (SOR) old = load_pack<T, V>(self_row + q0);
#pragma unroll
    for (int e = 0; e < V; ++e) {
        T right = P ? (e + 1 < V ? mid.v[e + 1] : extra) : mid.v[e];
        T left = P ? mid.v[e] : (e > 0 ? mid.v[e - 1] : extra);
        T s = dn.v[e] + up.v[e];
        s = s + right;
        s = s + left;
        T t = h2 * fc.v[e];
        s = s - t;
        const T g = T(0.25) * s;
        if constexpr (SOR) {
            const T d = g - old.v[e];
            const T w = omega * d;
            out.v[e] = old.v[e] + w;
        } else {
            out.v[e] = g;
        }
    }
    const int64_t q_lo = 1 - P, q_hi = (int64_t(n) - P) >> 1;
    if (q0 >= q_lo && q0 + V - 1 <= q_hi) {
        store_pack_nt<T, V>(self_row + q0, out);
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e)
            if (q0 + e >= q_lo && q0 + e <= q_hi) self_row[q0 + e] = out.v[e];
    }
}

// Rows i0..i1 of one strip, first row parity P0; two rows per step so both
// parities are compile-time constants.
template <typename T, int V, int P0, bool SOR>
__device__ __forceinline__ void march(T* __restrict__ self, const T* __restrict__ other,
                                      const T* __restrict__ f_self, int n, int64_t pitch, T h2,
                                      int64_t q0, int i0, int i1, T omega) {
    const T* o = other + q0;
    Pack<T, V> up = load_pack<T, V>(o + int64_t(i0 - 1) * pitch);
    Pack<T, V> mid = load_pack<T, V>(o + int64_t(i0) * pitch);
    int i = i0;
    for (; i + 1 <= i1; i += 2) {
        Pack<T, V> dn0 = load_pack<T, V>(o + int64_t(i + 1) * pitch);
        Pack<T, V> dn1 = load_pack<T, V>(o + int64_t(i + 2) * pitch);
        Pack<T, V> f0 = load_pack_nt<T, V>(f_self + int64_t(i) * pitch + q0);
        Pack<T, V> f1 = load_pack_nt<T, V>(f_self + int64_t(i + 1) * pitch + q0);
        update_row<T, V, P0, SOR>(self + int64_t(i) * pitch, other + int64_t(i) * pitch, up, mid,
                                  dn0, f0, h2, q0, n, omega);
        update_row<T, V, 1 - P0, SOR>(self + int64_t(i + 1) * pitch,
                                      other + int64_t(i + 1) * pitch, mid, dn0, dn1, f1, h2, q0, n,
                                      omega);
        up = dn0;
        mid = dn1;
    }
    if (i <= i1) {
        Pack<T, V> dn0 = load_pack<T, V>(o + int64_t(i + 1) * pitch);
        Pack<T, V> f0 = load_pack_nt<T, V>(f_self + int64_t(i) * pitch + q0);
        update_row<T, V, P0, SOR>(self + int64_t(i) * pitch, other + int64_t(i) * pitch, up, mid,
                                  dn0, f0, h2, q0, n, omega);
    }
}

template <typename T, int V, bool SOR>
__global__ __launch_bounds__(256) void k_half_sweep(T* __restrict__ self,
                                                    const T* __restrict__ other,
                                                    const T* __restrict__ f_self, int n,
                                                    int64_t pitch, T h2, int colour,
                                                    int rows_per_block, int col_blocks,
                                                    int nblocks, const int* __restrict__ stop,
                                                    T omega) {
    // a solve captured in a graph stops sweeping once its residual check
    // has raised the converged flag (set by an earlier kernel of the stream)
    if (stop != nullptr && *stop != 0) return;
    const int L = xcd_logical_block(blockIdx.x, nblocks);
    const int strip = L / col_blocks;
    const int cb = L - strip * col_blocks;
    const int64_t q0 = (int64_t(cb) * blockDim.x + threadIdx.x) * V;
    if (q0 > (n >> 1)) return;  // beyond the last interior q of either parity
    const int i0 = 1 + strip * rows_per_block;
    const int i1 = min(n, i0 + rows_per_block - 1);
    if (((i0 + colour) & 1) == 0)
        march<T, V, 0, SOR>(self, other, f_self, n, pitch, h2, q0, i0, i1, omega);
    else
        march<T, V, 1, SOR>(self, other, f_self, n, pitch, h2, q0, i0, i1, omega);
}

struct PlainConfig {
    int threads, col_blocks, rows, strips, blocks;
};

template <int V>
PlainConfig plain_config(int n, int rows_per_block) {
    PlainConfig c;
    int64_t qcols = int64_t(n >> 1) + 1;  // q = 0 .. n>>1
    int64_t vecs = (qcols + V - 1) / V;
    c.threads = vecs >= 256 ? 256 : (vecs > 128 ? 256 : (vecs > 64 ? 128 : 64));
    c.col_blocks = int((vecs + c.threads - 1) / c.threads);
    // Short strips (4 rows by default, measured best on MI355X at 8191^2)
    // give many workgroups in flight; the extra reads of the two halo rows
    // per strip are served by L2 because consecutive strips run on the same
    // XCD (xcd_logical_block).
    int r = rows_per_block > 0 ? rows_per_block : 4;
    c.rows = r;
    c.strips = (n + r - 1) / r;
    c.blocks = c.col_blocks * c.strips;
    return c;
}

}  // namespace

template <typename T>
hipError_t launch_half_sweep(T* self, const T* other, const T* f_self, int n, int64_t pitch, T h2,
                             int colour, int rows_per_block, hipStream_t s, const int* stop,
                             T omega) {
    constexpr int V = 16 / sizeof(T);
    PlainConfig c = plain_config<V>(n, rows_per_block);
    if (omega == T(1))
        hipLaunchKernelGGL((k_half_sweep<T, V, false>), dim3(c.blocks), dim3(c.threads), 0, s, self,
                           other, f_self, n, pitch, h2, colour, c.rows, c.col_blocks, c.blocks, stop,
                           omega);
    else
        hipLaunchKernelGGL((k_half_sweep<T, V, true>), dim3(c.blocks), dim3(c.threads), 0, s, self,
                           other, f_self, n, pitch, h2, colour, c.rows, c.col_blocks, c.blocks, stop,
                           omega);
    return hipGetLastError();
}

template hipError_t launch_half_sweep<double>(double*, const double*, const double*, int, int64_t,
                                              double, int, int, hipStream_t, const int*, double);
template hipError_t launch_half_sweep<float>(float*, const float*, const float*, int, int64_t,
                                             float, int, int, hipStream_t, const int*, float);

}  // namespace rbgs
