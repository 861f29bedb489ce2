// Internal declarations shared by the host API and the kernel files of
// librbgs.so.  Nothing here is part of the public ABI (include/rbgs.h).
//
// Split colour layout (the paper stores red and black values separately,
// Section 2.1): colour C of point (i, j) is (i + j) & 1 (0 = red, 1 = black)
// and the point is stored at C[i][j >> 1] of that colour's array, which has
// n+2 rows (ring rows included) of `pitch` elements.  In row i the points of
// colour C sit at j = p + 2q with p = p_C(i) = (i + C) & 1, so j >> 1 == q.
// Neighbours of C[i][q] (all of the other colour O):
//     (i+1, j) -> O[i+1][q]     (i-1, j) -> O[i-1][q]
//     (i, j+1) -> O[i][q + p]   (i, j-1) -> O[i][q - 1 + p]
// Interior points of colour C in row i: q in [1 - p, (n - p) >> 1].
// A half-sweep therefore streams the other colour once (three rows reused
// from registers), its own right-hand side once and writes its own colour
// once: 3 words per point update instead of the 6 of the natural layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rbgs {

constexpr int kWaveSize = 64;
constexpr int kNumXcd = 8;  // MI355X: 8 accelerator complex dies, round-robin dispatch

// Elements per colour row: ceil((n+2)/2) rounded up to 256 bytes.
inline int64_t split_pitch(int n, size_t elem_bytes) {
    int64_t half = (int64_t(n) + 3) / 2;
    int64_t align = int64_t(256 / elem_bytes);
    return (half + align - 1) / align * align;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workgroup id remapping so that each XCD (die with its own L2) receives a
// contiguous range of logical block ids.  Hardware dispatches workgroup b to
// XCD b % 8; we give XCD x the logical range starting at
// x * (nb / 8) + min(x, nb % 8), in the order the XCD receives its blocks.
__device__ __forceinline__ int xcd_logical_block(int b, int nb) {
    int x = b % kNumXcd;
    int k = b / kNumXcd;
    int base = nb / kNumXcd;
    int rem = nb % kNumXcd;
    return x * base + (x < rem ? x : rem) + k;
}

// ----- kernel launchers (defined in the .hip files) -----------------------

// natural <-> split permutation (pure data movement; elem_bytes is 4 or 8).
hipError_t launch_pack(const void* nat, int64_t ld, void* red, void* black, int n,
                       int64_t pitch, int elem_bytes, hipStream_t s);
hipError_t launch_unpack(void* nat, int64_t ld, const void* red, const void* black, int n,
                         int64_t pitch, int elem_bytes, hipStream_t s);
// Convert a natural FP64 array to split FP32 (round to nearest even).
hipError_t launch_pack_f64_to_f32(const double* nat, int64_t ld, float* red, float* black,
                                  int n, int64_t pitch, hipStream_t s);

// One half-sweep of colour `colour` (0 red, 1 black) in the split layout.
// stop (device, optional): the kernel does nothing when *stop != 0 (the
// converged flag of a graph-captured solve).  omega != 1: red-black SOR,
// u <- u + omega (g - u) with g the Gauss-Seidel value.
template <typename T>
hipError_t launch_half_sweep(T* self, const T* other, const T* f_self, int n, int64_t pitch,
                             T h2, int colour, int rows_per_block, hipStream_t s,
                             const int* stop = nullptr, T omega = T(1));

// Number of partial-sum slots the residual kernels need for grid size n.
int residual_partial_slots(int n, int64_t pitch, size_t elem_bytes);

// Residual norms of a split-layout iterate.  partials: residual_partial_slots
// * 2 doubles; out: 2 doubles (sum r^2, sum b^2) in device memory.
// r_out_red/black (optional): store r rounded to FP32 (or bfloat16 when
// rhs_bf16) in a split FP32 array of pitch r_pitch, for refinement;
// overflow (optional) is set to 1 when a finite r becomes infinite there.
// nat (optional): also unpack the interior of u into this natural array of
// row pitch ld (the same values the unpack kernel writes), in the same pass.
template <typename T>
hipError_t launch_residual_split(const T* u_red, const T* u_black, const T* f_red,
                                 const T* f_black, int n, int64_t pitch, double inv_h2,
                                 double* partials, double* out, float* r_out_red,
                                 float* r_out_black, int64_t r_pitch, int rhs_bf16,
                                 hipStream_t s, int* overflow = nullptr, T* nat = nullptr,
                                 int64_t ld = 0);

// Convergence test of a graph-captured solve round (device-side): from the
// residual kernel's sums, sets state[0] (the converged flag the sweep
// kernels' `stop` reads) when rel <= rel_tol, rel is not finite or
// state[1] (rounds done, incremented here) reaches cap.  watch != 0 (a
// refinement with the precision fallback): also when state[2] (the residual
// kernel's overflow flag) is set, or when round first_check or later leaves
// rel no lower than the previous rel (init_prev before the first round, then
// a double at state + 4; state[3] = 1).
hipError_t launch_judge(const double* sums, double rel_tol, int* state, int cap, hipStream_t s,
                        int watch = 0, int first_check = 0, double init_prev = 0.0);

// Residual norms of a natural-layout iterate (no packing).
template <typename T>
hipError_t launch_residual_natural(const T* u, const T* f, int n, int64_t ld, double inv_h2,
                                   double* partials, double* out, hipStream_t s);
int residual_natural_partial_slots(int n);

// Static scratch of the no-allocation residual: a file-scope device array
// of kStaticScratchBytes per device.  static_scratch gives the current
// device's address of it (looked up once per device); residual_noalloc_bytes
// is what a grid of size n needs there (sums, then the partial sums).
constexpr size_t kStaticScratchBytes = size_t(4) << 20;
hipError_t static_scratch(void** ptr);
size_t residual_noalloc_bytes(int n);

// u <- u + e at the interior points (split layouts; u FP64, e FP32);
// nothing when stop != nullptr and *stop != 0.
hipError_t launch_add_correction(double* u_red, double* u_black, int64_t pitch,
                                 const float* e_red, const float* e_black, int64_t e_pitch,
                                 int n, hipStream_t s, const int* stop = nullptr);

// Vertex-centred grid transfers over `batch` grids at constant strides
// (natural layout): full-weighting restriction onto the nc x nc coarse
// interior, bilinear prolongation onto the nf x nf fine interior.
template <typename T>
hipError_t launch_restrict(const T* fine, int64_t fine_ld, int64_t fine_stride, T* coarse,
                           int64_t coarse_ld, int64_t coarse_stride, int nc, int batch,
                           hipStream_t s);
template <typename T>
hipError_t launch_prolong(const T* coarse, int64_t coarse_ld, int64_t coarse_stride, T* fine,
                          int64_t fine_ld, int64_t fine_stride, int nf, int batch,
                          hipStream_t s);

// Multigrid transfers on split FP64 arrays (fine n_f = 2 n_c + 1, pitch /
// cpitch the fine / coarse split pitches).  restrict: coarse f <- full
// weighting of the fine residual f - A_h u (inv_h2 = 1 / h_f^2), coarse u
// interior rows <- 0.  prolong_add: fine u += bilinear interpolation of the
// coarse iterate.  Both do nothing when stop != nullptr and *stop != 0.
hipError_t launch_mg_restrict(const double* u_red, const double* u_black, const double* f_red,
                              const double* f_black, int64_t pitch, double inv_h2,
                              double* fc_red, double* fc_black, double* uc_red, double* uc_black,
                              int nc, int64_t cpitch, const int* stop, hipStream_t s);
hipError_t launch_mg_prolong_add(double* u_red, double* u_black, int64_t pitch, int nf,
                                 const double* e_red, const double* e_black, int64_t cpitch,
                                 const int* stop, hipStream_t s);
// The interpolant's correction fused into the red half-sweep that follows
// it (h2 = h * h of the fine level): red <- Gauss-Seidel with the corrected
// black neighbours; black is left uncorrected, for a black half-sweep that
// overwrites it next.
hipError_t launch_mg_prolong_red(double* u_red, const double* u_black, const double* f_red,
                                 int64_t pitch, int nf, double h2, const double* e_red,
                                 const double* e_black, int64_t cpitch, const int* stop,
                                 hipStream_t s);

// The coarse end of a multigrid cycle in one workgroup: levels[0] (at most
// kMgCoarseN points per side) down to the coarsest, each with its split u
// and f arrays; pre/post smoothing counts nu1/nu2 and the coarsest level's
// sweeps; nothing when stop != nullptr and *stop != 0.
constexpr int kMgCoarseN = 127;
constexpr int kMgMaxCoarseLevels = 8;
struct MgCoarseLevel {
    double* u_red;
    double* u_black;
    double* f_red;
    double* f_black;
    int64_t pitch;
    int n;
    double h2;      // h * h (the smoother's)
    double inv_h2;  // 1 / (h * h) (the residual's)
};
struct MgCoarseLevels {
    MgCoarseLevel level[kMgMaxCoarseLevels];
    int count;
};
hipError_t launch_mg_coarse_vcycle(const MgCoarseLevels& levels, int nu1, int nu2,
                                   int coarse_sweeps, const int* stop, hipStream_t s);

// Four-colour 9-point Gauss-Seidel on one array per colour (colour
// (i & 1) + 2 (j & 1), point (i, j) at [i >> 1][j >> 1]; mc9_rows(n) rows of
// mc9_pitch(n) doubles each).  quarter: one colour's update, c6 = 6 (h h);
// nothing when stop != nullptr and *stop != 0.  residual: sums of r^2 and
// b^2 into out[0..1] through mc9_residual_blocks(n) partial pairs.
int mc9_rows(int n);
int64_t mc9_pitch(int n);
int mc9_residual_blocks(int n);
hipError_t launch_mc9_pack(const double* nat, int64_t ld, double* const colours[4], int n,
                           hipStream_t s);
hipError_t launch_mc9_unpack(double* nat, int64_t ld, double* const colours[4], int n,
                             hipStream_t s);
hipError_t launch_mc9_quarter(double* const u[4], double* const f[4], int n, double c6,
                              int colour, const int* stop, hipStream_t s);
hipError_t launch_mc9_residual(double* const u[4], double* const f[4], int n, double inv6h2,
                               double* partials, double* out, hipStream_t s);
// The flag-driven 9-point form: `levels` quarter-sweeps (colour 0 first) in
// one launch (levels x mc9_flags_blocks(n, capacity) < 2^31).  capacity:
// resident workgroups of the kernel (mc9_flags_capacity()); ticket and
// progress: a zeroed counter and mc9_flags_blocks(n, capacity) zeroed block
// counters; error: a zeroed word, raised when a bounded wait expires.
constexpr int kMc9MaxBlocks = 65536;
int mc9_flags_capacity();
int mc9_flags_blocks(int n, int capacity);
hipError_t launch_mc9_flags(double* const u[4], double* const f[4], int n, double c6, int levels,
                            int capacity, int* ticket, int* progress, int* error, int spin_limit,
                            int delay, int stall_block, hipStream_t s);

// Red-black Gauss-Seidel in 3D (7-point): split arrays with a row per (i, j)
// pair, (n+2)^2 rows of `pitch` (split_pitch(n, 8)) doubles.  half: colour
// `colour`'s update with h2 = h h; nothing when stop != nullptr and *stop
// != 0.  residual: sums of r^2 and b^2 into out[0..1] through
// rb3_residual_blocks(n) partial pairs.
int rb3_residual_blocks(int n);
hipError_t launch_rb3_pack(const double* nat, int64_t ld, double* red, double* black, int n,
                           int64_t pitch, hipStream_t s);
hipError_t launch_rb3_unpack(double* nat, int64_t ld, const double* red, const double* black,
                             int n, int64_t pitch, hipStream_t s);
hipError_t launch_rb3_half(double* self, const double* other, const double* f, int n,
                           int64_t pitch, double h2, int colour, const int* stop, hipStream_t s);
// The flag-driven 3D form: `levels` half-sweeps (red first) of the split
// iterate in one launch (levels x rb3_flags_blocks(n, capacity) < 2^31).
// capacity: resident one-wave workgroups (rb3_flags_capacity(n)); ticket
// and progress: a zeroed counter and rb3_flags_blocks(n, capacity) zeroed
// block counters; error: a zeroed word, raised when a bounded wait
// (spin_limit polls) expires.
constexpr int kRb3MaxBlocks = 65536;
int rb3_flags_capacity(int n);
int rb3_flags_blocks(int n, int capacity);
hipError_t launch_rb3_flags(double* red, double* black, const double* f_red,
                            const double* f_black, int n, int64_t pitch, double h2, int levels,
                            int capacity, int* ticket, int* progress, int* error, int spin_limit,
                            int delay, int stall_block, const int* stop, hipStream_t s);
hipError_t launch_rb3_residual(const double* ur, const double* ub, const double* fr,
                               const double* fb, int n, int64_t pitch, double inv_h2,
                               double* partials, double* out, hipStream_t s);

// Copies the Dirichlet ring (and nothing that a pass would not overwrite
// before reading) of split grid src into dst; n + 2 rows of `pitch` elements.
hipError_t launch_copy_ring(void* dst_red, void* dst_black, const void* src_red,
                            const void* src_black, int n, int64_t pitch, int elem_bytes,
                            hipStream_t s);

// Zero a device range with a kernel (usable inside graph capture).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// dst <- src for `bytes` (a multiple of 16, 16-byte aligned buffers) unless
// stop != nullptr and *stop != 0.
hipError_t launch_copy_unless(void* dst, const void* src, size_t bytes, const int* stop,
                              hipStream_t s);

}  // namespace rbgs
