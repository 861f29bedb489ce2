/*
 * Oracle for red-black Gauss-Seidel on the 5-point 2D Poisson stencil.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU definition that the GPU library is checked against.  Only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * GPU library neither links nor calls it, and it shares no code with the GPU
 * library.
 *
 * What it computes (paper: Section 2, Eq. (1) and Algorithm 1):
 *   - the Poisson problem  laplace(u) = f  on the unit square with Dirichlet
 *     data g on the boundary, discretised on a uniform grid of N x N interior
 *     points with spacing h = 1/(N+1);
 *   - the Gauss-Seidel point update of Eq. (1),
 *         u_ij <- 1/4 (u_{i+1,j} + u_{i-1,j} + u_{i,j+1} + u_{i,j-1} - h^2 f_ij),
 *     where neighbours on the boundary ring take the Dirichlet value g;
 *   - red-black ordering: red points have i+j even, black points i+j odd
 *     (Section 2); one sweep (one "iteration" of Algorithms 1 and 2) is all
 *     red points, then all black points.
 *
 * Storage: natural row-major layout with the boundary ring included.  The
 * grid has n+2 rows of ld >= n+2 elements; element (i, j), 0 <= i, j <= n+1,
 * is a[i*ld + j]; i is the row (x, the outer loop of Algorithm 1) and j the
 * column (y, the inner loop).  Row 0, row n+1, column 0 and column n+1 hold g
 * in u and are read, never written; the ring entries of f are never read.
 *
 * Floating point (the paper states no term order; this is the reading used
 * throughout): the four neighbours are summed left to right in the order of
 * Eq. (1), h^2 is the product h*h rounded once in the working precision, the
 * product h^2*f is subtracted, the result is scaled by 1/4, and nothing is
 * contracted into FMA (build with -ffp-contract=off).  Points of one colour
 * never read each other (Section 2), so the loop order inside a colour and
 * the OpenMP split of its rows cannot change a single bit.
 *
 * Precision: FP64 (the paper's workload; its arithmetic intensity of about
 * 0.29 FLOP/B in Section 3 corresponds to 8-byte words).  The _f32 functions
 * are the same algorithm with every value held and every operation rounded
 * in IEEE binary32; they exist to check the FP32 forms of the GPU sweep.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RBGS_REF_OK 0
#define RBGS_REF_EINVAL (-1)
#define RBGS_REF_ENOCONV (-3)
#define RBGS_REF_ENOMEM (-7)

#define AT(a, i, j) ((a)[(size_t)(i) * (size_t)ld + (size_t)(j)])

static int bad_grid(int32_t n, int64_t ld, double h)
{
    return n < 1 || ld < (int64_t)n + 2 || !(h > 0.0) || !isfinite(h);
}

/* Colour of point (i, j): 0 = red (i+j even), 1 = black (i+j odd). */
static int colour_of(int64_t i, int64_t j) { return (int)((i + j) & 1); }

/* ------------------------------------------------------------------------- */
/* FP64 half-sweep: Eq. (1) on every interior point of one colour.            */
/* Row x starts at column 2 or 1 by the parity rule of Algorithm 1 and steps  */
/* by two, so it visits exactly the points of the requested colour.           */
/* ------------------------------------------------------------------------- */
int rbgs_ref_half_sweep_f64(int32_t n, int64_t ld, double h, double *u,
                            const double *f, int32_t colour)
{
    if (bad_grid(n, ld, h) || !u || !f || (colour != 0 && colour != 1))
        return RBGS_REF_EINVAL;
    const double h2 = h * h;
#pragma omp parallel for schedule(static)
    for (int64_t i = 1; i <= n; ++i) {
        /* red: even rows start at column 2, odd rows at 1; black the reverse */
        int64_t j_start = (i % 2 == 0) ? (colour == 0 ? 2 : 1) : (colour == 0 ? 1 : 2);
        for (int64_t j = j_start; j <= n; j += 2) {
            double s = AT(u, i + 1, j) + AT(u, i - 1, j);
            s = s + AT(u, i, j + 1);
            s = s + AT(u, i, j - 1);
            double t = h2 * AT(f, i, j);
            s = s - t;
            AT(u, i, j) = 0.25 * s;
        }
    }
    return RBGS_REF_OK;
}

/* nsweeps full sweeps: red half-sweep, then black half-sweep (Algorithm 2's
 * loop runs exactly num_iterations times; the bound one lower in Algorithm 1
 * is read as a typo). */
int rbgs_ref_sweep_f64(int32_t n, int64_t ld, double h, double *u,
                       const double *f, int32_t nsweeps)
{
    if (bad_grid(n, ld, h) || !u || !f || nsweeps < 0) return RBGS_REF_EINVAL;
    for (int32_t it = 0; it < nsweeps; ++it) {
        rbgs_ref_half_sweep_f64(n, ld, h, u, f, 0);
        rbgs_ref_half_sweep_f64(n, ld, h, u, f, 1);
    }
    return RBGS_REF_OK;
}

/* ------------------------------------------------------------------------- */
/* FP32 emulation of the same sweep.  h^2 is h*h formed in double and rounded  */
/* once to binary32; every other value and operation is binary32.            */
/* ------------------------------------------------------------------------- */
int rbgs_ref_half_sweep_f32(int32_t n, int64_t ld, double h, float *u,
                            const float *f, int32_t colour)
{
    if (bad_grid(n, ld, h) || !u || !f || (colour != 0 && colour != 1))
        return RBGS_REF_EINVAL;
    const float h2 = (float)(h * h);
#pragma omp parallel for schedule(static)
    for (int64_t i = 1; i <= n; ++i) {
        int64_t j_start = (i % 2 == 0) ? (colour == 0 ? 2 : 1) : (colour == 0 ? 1 : 2);
        for (int64_t j = j_start; j <= n; j += 2) {
            float s = AT(u, i + 1, j) + AT(u, i - 1, j);
            s = s + AT(u, i, j + 1);
            s = s + AT(u, i, j - 1);
            float t = h2 * AT(f, i, j);
            s = s - t;
            AT(u, i, j) = 0.25f * s;
        }
    }
    return RBGS_REF_OK;
}

int rbgs_ref_sweep_f32(int32_t n, int64_t ld, double h, float *u,
                       const float *f, int32_t nsweeps)
{
    if (bad_grid(n, ld, h) || !u || !f || nsweeps < 0) return RBGS_REF_EINVAL;
    for (int32_t it = 0; it < nsweeps; ++it) {
        rbgs_ref_half_sweep_f32(n, ld, h, u, f, 0);
        rbgs_ref_half_sweep_f32(n, ld, h, u, f, 1);
    }
    return RBGS_REF_OK;
}

/* ------------------------------------------------------------------------- */
/* Residual.  The paper runs a fixed iteration count and defines no residual; */
/* the reading used here is the residual of the discrete system A_h u = f     */
/* whose Jacobi-form solution step is Eq. (1):                                */
/*   (A_h u)_ij = (u_{i+1,j} + u_{i-1,j} + u_{i,j+1} + u_{i,j-1} - 4 u_ij)/h^2 */
/*   r_ij = f_ij - (A_h u)_ij,            over the interior points,           */
/* and the scale b = r evaluated with the interior of u set to zero (b = f    */
/* when g = 0).  rel = ||r||_2 / ||b||_2, or ||r||_2 when ||b||_2 = 0.        */
/* Per point: s = ((u[i+1][j] + u[i-1][j]) + u[i][j+1]) + u[i][j-1];          */
/* r = f - (s - 4u) * (1/(h*h)), all in FP64.  Sums of squares use Neumaier's */
/* compensated summation in row-major order.                                  */
/* ------------------------------------------------------------------------- */
static void neumaier_add(double *sum, double *comp, double x)
{
    double t = *sum + x;
    if (fabs(*sum) >= fabs(x))
        *comp += (*sum - t) + x;
    else
        *comp += (x - t) + *sum;
    *sum = t;
}

static int on_ring(int32_t n, int64_t i, int64_t j)
{
    return i == 0 || j == 0 || i == (int64_t)n + 1 || j == (int64_t)n + 1;
}

/* The value of neighbour (i, j) as seen by b: the ring keeps g, the interior
 * counts as zero. */
#define RING_ONLY(a, i, j) (on_ring(n, (i), (j)) ? (double)AT(a, i, j) : 0.0)

#define RESIDUAL_BODY(T)                                                        \
    const double inv_h2 = 1.0 / (h * h);                                        \
    double rs = 0.0, rc = 0.0, bs = 0.0, bc = 0.0;                              \
    for (int64_t i = 1; i <= n; ++i) {                                          \
        for (int64_t j = 1; j <= n; ++j) {                                      \
            double s = (double)AT(u, i + 1, j) + (double)AT(u, i - 1, j);       \
            s = s + (double)AT(u, i, j + 1);                                    \
            s = s + (double)AT(u, i, j - 1);                                    \
            double lap = (s - 4.0 * (double)AT(u, i, j)) * inv_h2;              \
            double r = (double)AT(f, i, j) - lap;                               \
            double sb = RING_ONLY(u, i + 1, j) + RING_ONLY(u, i - 1, j);        \
            sb = sb + RING_ONLY(u, i, j + 1);                                   \
            sb = sb + RING_ONLY(u, i, j - 1);                                   \
            double b = (double)AT(f, i, j) - sb * inv_h2;                       \
            if (r_out) AT(r_out, i, j) = r;                                     \
            neumaier_add(&rs, &rc, r * r);                                      \
            neumaier_add(&bs, &bc, b * b);                                      \
        }                                                                       \
    }                                                                           \
    double rn = sqrt(rs + rc), bn = sqrt(bs + bc);                              \
    if (abs_norm) *abs_norm = rn;                                               \
    if (rel_norm) *rel_norm = (bn > 0.0) ? rn / bn : rn;                        \
    return RBGS_REF_OK;

/* r_out (optional, may be NULL): natural-layout array receiving r_ij at the
 * interior points; its ring is left untouched. */
int rbgs_ref_residual_f64(int32_t n, int64_t ld, double h, const double *u,
                          const double *f, double *abs_norm, double *rel_norm,
                          double *r_out)
{
    if (bad_grid(n, ld, h) || !u || !f) return RBGS_REF_EINVAL;
    RESIDUAL_BODY(double)
}

/* Same residual of a binary32 iterate: every value is widened to FP64 first
 * and the arithmetic is the FP64 arithmetic above. */
int rbgs_ref_residual_f32(int32_t n, int64_t ld, double h, const float *u,
                          const float *f, double *abs_norm, double *rel_norm,
                          double *r_out)
{
    if (bad_grid(n, ld, h) || !u || !f) return RBGS_REF_EINVAL;
    RESIDUAL_BODY(float)
}

/* ------------------------------------------------------------------------- */
/* Solve to a relative residual: the residual is checked before the first    */
/* sweep and after every check_every sweeps (the last group may be shorter   */
/* so that exactly max_sweeps can be reached).  rel_tol <= 0 means "run       */
/* exactly max_sweeps sweeps", with one residual at the end.                 */
/* Returns 0 when rel <= rel_tol was reached (or rel_tol <= 0), else          */
/* RBGS_REF_ENOCONV with u holding the last iterate.                          */
/* ------------------------------------------------------------------------- */
int rbgs_ref_solve_f64(int32_t n, int64_t ld, double h, double *u,
                       const double *f, int32_t max_sweeps, double rel_tol,
                       int32_t check_every, int32_t *sweeps_done,
                       double *rel_out)
{
    if (bad_grid(n, ld, h) || !u || !f || max_sweeps < 0 || check_every < 1)
        return RBGS_REF_EINVAL;
    int32_t done = 0;
    double rel = 0.0;
    if (rel_tol <= 0.0) {
        rbgs_ref_sweep_f64(n, ld, h, u, f, max_sweeps);
        done = max_sweeps;
        rbgs_ref_residual_f64(n, ld, h, u, f, NULL, &rel, NULL);
        if (sweeps_done) *sweeps_done = done;
        if (rel_out) *rel_out = rel;
        return RBGS_REF_OK;
    }
    rbgs_ref_residual_f64(n, ld, h, u, f, NULL, &rel, NULL);
    while (!(rel <= rel_tol) && done < max_sweeps) {
        int32_t k = max_sweeps - done < check_every ? max_sweeps - done : check_every;
        rbgs_ref_sweep_f64(n, ld, h, u, f, k);
        done += k;
        rbgs_ref_residual_f64(n, ld, h, u, f, NULL, &rel, NULL);
    }
    if (sweeps_done) *sweeps_done = done;
    if (rel_out) *rel_out = rel;
    return rel <= rel_tol ? RBGS_REF_OK : RBGS_REF_ENOCONV;
}

/* ------------------------------------------------------------------------- */
/* Red-black SOR, the first extension beyond the paper's method (successive  */
/* over-relaxation of the same red-black Gauss-Seidel): at each point the    */
/* Gauss-Seidel value g of Eq. (1), formed exactly as above, relaxes the old */
/* value,                                                                    */
/*     u_ij <- u_ij + omega * (g - u_ij),                                    */
/* the difference, the product and the sum each rounded once (no FMA).       */
/* omega = 1 is Gauss-Seidel in exact arithmetic but not bit for bit (the    */
/* functions above are the Gauss-Seidel definition); 1 < omega < 2 over-     */
/* relaxes.  Red then black per sweep, as for Gauss-Seidel.                  */
/* ------------------------------------------------------------------------- */
int rbgs_ref_sor_half_sweep_f64(int32_t n, int64_t ld, double h, double omega, double *u,
                                const double *f, int32_t colour)
{
    if (bad_grid(n, ld, h) || !u || !f || (colour != 0 && colour != 1) ||
        !(omega > 0.0 && omega < 2.0))
        return RBGS_REF_EINVAL;
    const double h2 = h * h;
#pragma omp parallel for schedule(static)
    for (int64_t i = 1; i <= n; ++i) {
        int64_t j_start = (i % 2 == 0) ? (colour == 0 ? 2 : 1) : (colour == 0 ? 1 : 2);
        for (int64_t j = j_start; j <= n; j += 2) {
            double s = AT(u, i + 1, j) + AT(u, i - 1, j);
            s = s + AT(u, i, j + 1);
            s = s + AT(u, i, j - 1);
            double t = h2 * AT(f, i, j);
            s = s - t;
            const double g = 0.25 * s;
            const double old = AT(u, i, j);
            const double d = g - old;
            const double w = omega * d;
            AT(u, i, j) = old + w;
        }
    }
    return RBGS_REF_OK;
}

int rbgs_ref_sor_sweep_f64(int32_t n, int64_t ld, double h, double omega, double *u,
                           const double *f, int32_t nsweeps)
{
    if (bad_grid(n, ld, h) || !u || !f || nsweeps < 0 || !(omega > 0.0 && omega < 2.0))
        return RBGS_REF_EINVAL;
    for (int32_t it = 0; it < nsweeps; ++it) {
        rbgs_ref_sor_half_sweep_f64(n, ld, h, omega, u, f, 0);
        rbgs_ref_sor_half_sweep_f64(n, ld, h, omega, u, f, 1);
    }
    return RBGS_REF_OK;
}

/* The solve loop of rbgs_ref_solve_f64 around SOR sweeps. */
int rbgs_ref_sor_solve_f64(int32_t n, int64_t ld, double h, double omega, double *u,
                           const double *f, int32_t max_sweeps, double rel_tol,
                           int32_t check_every, int32_t *sweeps_done, double *rel_out)
{
    if (bad_grid(n, ld, h) || !u || !f || max_sweeps < 0 || check_every < 1 ||
        !(omega > 0.0 && omega < 2.0))
        return RBGS_REF_EINVAL;
    int32_t done = 0;
    double rel = 0.0;
    rbgs_ref_residual_f64(n, ld, h, u, f, NULL, &rel, NULL);
    while (!(rel <= rel_tol) && done < max_sweeps) {
        int32_t k = max_sweeps - done < check_every ? max_sweeps - done : check_every;
        rbgs_ref_sor_sweep_f64(n, ld, h, omega, u, f, k);
        done += k;
        rbgs_ref_residual_f64(n, ld, h, u, f, NULL, &rel, NULL);
    }
    if (sweeps_done) *sweeps_done = done;
    if (rel_out) *rel_out = rel;
    return rel <= rel_tol ? RBGS_REF_OK : RBGS_REF_ENOCONV;
}

/* Threads an OpenMP region of the oracle uses (1 without OpenMP); the
 * timing harness reports it beside the oracle's throughput. */
int rbgs_ref_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Round a binary32 value to bfloat16 (8 significand bits, round to nearest, */
/* ties to even) and widen it back to binary32.  NaN stays NaN.               */
/* ------------------------------------------------------------------------- */
float rbgs_ref_round_bf16(float x)
{
    uint32_t bits;
    memcpy(&bits, &x, sizeof bits);
    if ((bits & 0x7f800000u) == 0x7f800000u && (bits & 0x007fffffu) != 0u) {
        bits |= 0x00400000u; /* quiet NaN */
    } else {
        uint32_t lsb = (bits >> 16) & 1u;
        bits += 0x7fffu + lsb;
    }
    bits &= 0xffff0000u;
    float y;
    memcpy(&y, &bits, sizeof y);
    return y;
}

/* ------------------------------------------------------------------------- */
/* Mixed-precision iterative refinement (not in the paper; the outer loop is  */
/* classical iterative refinement around the FP32 sweep above):               */
/*   repeat: r = f - A_h u in FP64 (the residual above), stop when            */
/*           rel <= rel_tol; round r to binary32 (rhs_bf16 != 0: then further */
/*           to bfloat16); e = 0 with a zero ring; inner_sweeps FP32 sweeps   */
/*           of A_h e = r; u <- u + e in FP64 at the interior points.          */
/* The residual is checked before each outer step; the ring of u is g and is  */
/* never written.  Returns 0 when converged, RBGS_REF_ENOCONV otherwise.      */
/* ------------------------------------------------------------------------- */
int rbgs_ref_ir_solve(int32_t n, int64_t ld, double h, double *u,
                      const double *f, int32_t rhs_bf16, int32_t inner_sweeps,
                      int32_t max_outer, double rel_tol, int32_t *outer_done,
                      double *rel_out)
{
    if (bad_grid(n, ld, h) || !u || !f || inner_sweeps < 1 || max_outer < 0)
        return RBGS_REF_EINVAL;
    size_t cells = (size_t)(n + 2) * (size_t)ld;
    double *r = (double *)calloc(cells, sizeof(double));
    float *r32 = (float *)calloc(cells, sizeof(float));
    float *e = (float *)calloc(cells, sizeof(float));
    if (!r || !r32 || !e) {
        free(r); free(r32); free(e);
        return RBGS_REF_ENOMEM;
    }
    int32_t outer = 0;
    double rel = 0.0;
    rbgs_ref_residual_f64(n, ld, h, u, f, NULL, &rel, r);
    while (!(rel <= rel_tol) && outer < max_outer) {
        for (int64_t i = 1; i <= n; ++i)
            for (int64_t j = 1; j <= n; ++j) {
                float v = (float)AT(r, i, j);
                AT(r32, i, j) = rhs_bf16 ? rbgs_ref_round_bf16(v) : v;
            }
        memset(e, 0, cells * sizeof(float));
        rbgs_ref_sweep_f32(n, ld, h, e, r32, inner_sweeps);
        for (int64_t i = 1; i <= n; ++i)
            for (int64_t j = 1; j <= n; ++j)
                AT(u, i, j) = AT(u, i, j) + (double)AT(e, i, j);
        ++outer;
        rbgs_ref_residual_f64(n, ld, h, u, f, NULL, &rel, r);
    }
    free(r); free(r32); free(e);
    if (outer_done) *outer_done = outer;
    if (rel_out) *rel_out = rel;
    return rel <= rel_tol ? RBGS_REF_OK : RBGS_REF_ENOCONV;
}


/* ------------------------------------------------------------------------- */
/* Refinement with a precision fallback (not in the paper; the build's own    */
/* rule).  The outer steps are those of rbgs_ref_ir_solve, with a budget of    */
/* max_sweeps sweeps in all, and the inner precision widens when it stops     */
/* helping:                                                                   */
/*   - range: when the FP64 residual holds a value that the inner right-hand  */
/*     side format cannot hold (binary32 or bfloat16 rounding gives an        */
/*     infinity), the solve switches to FP64 sweeps of u at once;             */
/*   - stall: when an outer step after the first leaves the relative residual */
/*     no lower than before it (the first step of a solve from a smooth start */
/*     raises it: Gauss-Seidel's first sweep leaves the residual on one       */
/*     colour), a bfloat16 right-hand side becomes binary32, and binary32    */
/*     inner sweeps become FP64 sweeps of u.                                  */
/* In FP64 the sweeps run inner_sweeps at a time with the residual after      */
/* each group.  *prec_out: the precision in use at the end (0 = FP64 sweeps,  */
/* 1 = binary32 inner, 2 = bfloat16 right-hand side).                         */
/* ------------------------------------------------------------------------- */
static int ir_residual_rounded(int32_t n, int64_t ld, double h, const double *u,
                               const double *f, double *r, float *r32, int32_t prec,
                               double *rel)
{
    rbgs_ref_residual_f64(n, ld, h, u, f, NULL, rel, r);
    int overflow = 0;
    for (int64_t i = 1; i <= n; ++i)
        for (int64_t j = 1; j <= n; ++j) {
            double x = AT(r, i, j);
            float v = (float)x;
            if (prec == 2) v = rbgs_ref_round_bf16(v);
            if (isinf(v) && isfinite(x)) overflow = 1;
            AT(r32, i, j) = v;
        }
    return overflow;
}

int rbgs_ref_ir_solve_fallback(int32_t n, int64_t ld, double h, double *u, const double *f,
                               int32_t rhs_bf16, int32_t inner_sweeps, int32_t max_sweeps,
                               double rel_tol, int32_t *outer_done, int32_t *sweeps_done,
                               double *rel_out, int32_t *prec_out)
{
    if (bad_grid(n, ld, h) || !u || !f || inner_sweeps < 1 || max_sweeps < 0)
        return RBGS_REF_EINVAL;
    size_t cells = (size_t)(n + 2) * (size_t)ld;
    double *r = (double *)calloc(cells, sizeof(double));
    float *r32 = (float *)calloc(cells, sizeof(float));
    float *e = (float *)calloc(cells, sizeof(float));
    if (!r || !r32 || !e) {
        free(r); free(r32); free(e);
        return RBGS_REF_ENOMEM;
    }
    int32_t prec = rhs_bf16 ? 2 : 1, outer = 0, done = 0;
    double rel = 0.0;
    if (ir_residual_rounded(n, ld, h, u, f, r, r32, prec, &rel)) prec = 0;
    while (!(rel <= rel_tol) && done < max_sweeps && isfinite(rel)) {
        int32_t k = max_sweeps - done < inner_sweeps ? max_sweeps - done : inner_sweeps;
        if (prec == 0) {
            rbgs_ref_sweep_f64(n, ld, h, u, f, k);
            done += k;
            rbgs_ref_residual_f64(n, ld, h, u, f, NULL, &rel, NULL);
            continue;
        }
        memset(e, 0, cells * sizeof(float));
        rbgs_ref_sweep_f32(n, ld, h, e, r32, k);
        for (int64_t i = 1; i <= n; ++i)
            for (int64_t j = 1; j <= n; ++j)
                AT(u, i, j) = AT(u, i, j) + (double)AT(e, i, j);
        done += k;
        ++outer;
        const double before = rel;
        int overflow = ir_residual_rounded(n, ld, h, u, f, r, r32, prec, &rel);
        if (outer >= 2 && rel >= before) {
            prec = prec == 2 ? 1 : 0;
            if (prec == 1) overflow = ir_residual_rounded(n, ld, h, u, f, r, r32, prec, &rel);
        }
        if (overflow) prec = 0;
    }
    free(r); free(r32); free(e);
    if (outer_done) *outer_done = outer;
    if (sweeps_done) *sweeps_done = done;
    if (rel_out) *rel_out = rel;
    if (prec_out) *prec_out = prec;
    if (!isfinite(rel)) return RBGS_REF_ENOCONV;
    return rel <= rel_tol ? RBGS_REF_OK : RBGS_REF_ENOCONV;
}

/* ------------------------------------------------------------------------- */
/* Multigrid with red-black Gauss-Seidel as the smoother (an extension: the   */
/* conclusion, Section 5, names odd-even and related multilevel techniques as  */
/* future work; the paper itself runs Gauss-Seidel alone).  The textbook       */
/* V-cycle for the vertex-centred grid hierarchy:                               */
/*   - level sizes n_0 = n and n_{l+1} = (n_l - 1) / 2 while n_l is odd and   */
/*     n_l >= 3 (and fewer than max_levels levels, if max_levels > 0);         */
/*     h_{l+1} = 2 h_l; coarse point (I, J) lies on fine point (2I, 2J);       */
/*   - the coarse problems are the same 5-point Poisson system on the coarser  */
/*     grid (rediscretised, not Galerkin), for the error, with a zero ring;    */
/*   - on a level above the coarsest: nu1 sweeps; the residual field r of the  */
/*     residual function above; coarse right-hand side = full weighting of r;  */
/*     coarse iterate = 0; the cycle on the coarser level; u += bilinear        */
/*     prolongation of the coarse iterate; nu2 sweeps;                          */
/*   - on the coarsest level: coarse_sweeps sweeps (one sweep is exact when    */
/*     n = 1: the single point is red and its neighbours are ring values).     */
/* Rounding order of the transfers (each + and * rounded once, no FMA):        */
/*   full weighting, per fine row a in {2I-1, 2I, 2I+1}:                       */
/*       row_a = (r[a][2J-1] + 2 r[a][2J]) + r[a][2J+1],                       */
/*       f_c[I][J] = ((row_{2I-1} + 2 row_{2I}) + row_{2I+1}) * 0.0625;        */
/*   bilinear prolongation at fine (i, j), e = coarse iterate (ring included), */
/*   I = i >> 1, J = j >> 1:                                                   */
/*       i, j even: v = e[I][J];                                               */
/*       i odd, j even: v = (e[I][J] + e[I+1][J]) * 0.5;                       */
/*       i even, j odd: v = (e[I][J] + e[I][J+1]) * 0.5;                       */
/*       i, j odd: v = ((e[I][J] + e[I][J+1]) + (e[I+1][J] + e[I+1][J+1])) * 0.25; */
/*       u[i][j] = u[i][j] + v.                                                */
/* ------------------------------------------------------------------------- */

#define RBGS_REF_MG_MAX_LEVELS 32

/* Level sizes of the hierarchy for grid size n; returns the level count and  */
/* writes the sizes to `sizes` (capacity RBGS_REF_MG_MAX_LEVELS) if given.     */
int32_t rbgs_ref_mg_levels(int32_t n, int32_t max_levels, int32_t *sizes)
{
    if (n < 1 || max_levels < 0) return 0;
    int32_t cnt = 1;
    int32_t m = n;
    if (sizes) sizes[0] = m;
    while (m >= 3 && (m % 2) == 1 && cnt < RBGS_REF_MG_MAX_LEVELS &&
           (max_levels == 0 || cnt < max_levels)) {
        m = (m - 1) / 2;
        if (sizes) sizes[cnt] = m;
        ++cnt;
    }
    return cnt;
}

/* Full weighting of the fine interior field r (n_f = 2 nc + 1 points per      */
/* side, natural layout, row length ld) onto the interior of fc (row length    */
/* ldc); the ring of fc is left as it is.                                      */
int rbgs_ref_mg_restrict_f64(int32_t nc, const double *r, int64_t ld, double *fc, int64_t ldc)
{
    if (nc < 1 || !r || !fc || ld < 2 * (int64_t)nc + 3 || ldc < (int64_t)nc + 2)
        return RBGS_REF_EINVAL;
    for (int64_t I = 1; I <= nc; ++I) {
        for (int64_t J = 1; J <= nc; ++J) {
            double row[3];
            for (int a = 0; a < 3; ++a) {
                const int64_t i = 2 * I - 1 + a;
                row[a] = (AT(r, i, 2 * J - 1) + 2.0 * AT(r, i, 2 * J)) + AT(r, i, 2 * J + 1);
            }
            fc[(size_t)I * (size_t)ldc + (size_t)J] = ((row[0] + 2.0 * row[1]) + row[2]) * 0.0625;
        }
    }
    return RBGS_REF_OK;
}

/* u += bilinear prolongation of ec (nc interior points per side, ring        */
/* included, row length ldc) at the interior points of u (n_f = 2 nc + 1,     */
/* row length ld); the ring of u is not written.                               */
int rbgs_ref_mg_prolong_add_f64(int32_t nc, const double *ec, int64_t ldc, double *u, int64_t ld)
{
    if (nc < 1 || !ec || !u || ld < 2 * (int64_t)nc + 3 || ldc < (int64_t)nc + 2)
        return RBGS_REF_EINVAL;
    const int64_t nf = 2 * (int64_t)nc + 1;
#define EC(I, J) ec[(size_t)(I) * (size_t)ldc + (size_t)(J)]
    for (int64_t i = 1; i <= nf; ++i) {
        for (int64_t j = 1; j <= nf; ++j) {
            const int64_t I = i >> 1, J = j >> 1;
            double v;
            if (i % 2 == 0 && j % 2 == 0)
                v = EC(I, J);
            else if (i % 2 == 1 && j % 2 == 0)
                v = (EC(I, J) + EC(I + 1, J)) * 0.5;
            else if (i % 2 == 0 && j % 2 == 1)
                v = (EC(I, J) + EC(I, J + 1)) * 0.5;
            else
                v = ((EC(I, J) + EC(I, J + 1)) + (EC(I + 1, J) + EC(I + 1, J + 1))) * 0.25;
            AT(u, i, j) = AT(u, i, j) + v;
        }
    }
#undef EC
    return RBGS_REF_OK;
}

typedef struct {
    int32_t n;
    int64_t ld;
    double h;
    double *u, *f, *r;
} mg_level;

static void mg_cycle(mg_level *lv, int32_t l, int32_t nlev, int32_t nu1, int32_t nu2,
                     int32_t coarse_sweeps)
{
    mg_level *a = &lv[l];
    if (l == nlev - 1) {
        rbgs_ref_sweep_f64(a->n, a->ld, a->h, a->u, a->f, coarse_sweeps);
        return;
    }
    mg_level *c = &lv[l + 1];
    rbgs_ref_sweep_f64(a->n, a->ld, a->h, a->u, a->f, nu1);
    rbgs_ref_residual_f64(a->n, a->ld, a->h, a->u, a->f, NULL, NULL, a->r);
    rbgs_ref_mg_restrict_f64(c->n, a->r, a->ld, c->f, c->ld);
    memset(c->u, 0, (size_t)(c->n + 2) * (size_t)c->ld * sizeof(double));
    mg_cycle(lv, l + 1, nlev, nu1, nu2, coarse_sweeps);
    rbgs_ref_mg_prolong_add_f64(c->n, c->u, c->ld, a->u, a->ld);
    rbgs_ref_sweep_f64(a->n, a->ld, a->h, a->u, a->f, nu2);
}

/* V-cycles until rel <= rel_tol or max_cycles cycles; the residual is checked */
/* before the first cycle and after each (rel_tol <= 0: exactly max_cycles     */
/* cycles, one residual at the end), as in rbgs_ref_solve_f64.  u, f: the      */
/* finest level in the natural layout with ring g; coarse levels are held      */
/* here.  Returns 0, RBGS_REF_ENOCONV or an error.                             */
int rbgs_ref_mg_solve_f64(int32_t n, int64_t ld, double h, double *u, const double *f,
                          int32_t nu1, int32_t nu2, int32_t max_levels, int32_t coarse_sweeps,
                          int32_t max_cycles, double rel_tol, int32_t *cycles_done,
                          double *rel_out)
{
    if (bad_grid(n, ld, h) || !u || !f || nu1 < 0 || nu2 < 0 || max_levels < 0 ||
        coarse_sweeps < 0 || max_cycles < 0)
        return RBGS_REF_EINVAL;
    int32_t sizes[RBGS_REF_MG_MAX_LEVELS];
    const int32_t nlev = rbgs_ref_mg_levels(n, max_levels, sizes);
    mg_level lv[RBGS_REF_MG_MAX_LEVELS];
    int ok = 1;
    for (int32_t l = 0; l < nlev; ++l) {
        lv[l].n = sizes[l];
        lv[l].ld = l == 0 ? ld : (int64_t)sizes[l] + 2;
        lv[l].h = l == 0 ? h : 2.0 * lv[l - 1].h;
        const size_t cells = (size_t)(lv[l].n + 2) * (size_t)lv[l].ld;
        lv[l].u = l == 0 ? u : (double *)calloc(cells, sizeof(double));
        lv[l].f = l == 0 ? (double *)f : (double *)calloc(cells, sizeof(double));
        lv[l].r = l + 1 < nlev ? (double *)calloc(cells, sizeof(double)) : NULL;
        if (!lv[l].u || !lv[l].f || (l + 1 < nlev && !lv[l].r)) ok = 0;
    }
    int32_t cycles = 0;
    double rel = 0.0;
    if (ok) {
        if (rel_tol <= 0.0) {
            for (; cycles < max_cycles; ++cycles) mg_cycle(lv, 0, nlev, nu1, nu2, coarse_sweeps);
        } else {
            rbgs_ref_residual_f64(n, ld, h, u, f, NULL, &rel, NULL);
            while (!(rel <= rel_tol) && cycles < max_cycles) {
                mg_cycle(lv, 0, nlev, nu1, nu2, coarse_sweeps);
                ++cycles;
                rbgs_ref_residual_f64(n, ld, h, u, f, NULL, &rel, NULL);
            }
        }
        if (rel_tol <= 0.0) rbgs_ref_residual_f64(n, ld, h, u, f, NULL, &rel, NULL);
    }
    for (int32_t l = 0; l < nlev; ++l) {
        if (l > 0) { free(lv[l].u); free(lv[l].f); }
        free(lv[l].r);
    }
    if (!ok) return RBGS_REF_ENOMEM;
    if (cycles_done) *cycles_done = cycles;
    if (rel_out) *rel_out = rel;
    return (rel_tol <= 0.0 || rel <= rel_tol) ? RBGS_REF_OK : RBGS_REF_ENOCONV;
}

/* ------------------------------------------------------------------------- */
/* Multi-colour Gauss-Seidel for a wider stencil (an extension: the           */
/* conclusion, Section 5, names multi-colour variants, whose extra colours     */
/* add synchronisation, as future work).  The 9-point Laplacian               */
/*     lap9(u)_ij = (4 e_ij + c_ij - 20 u_ij) / (6 h^2),                       */
/* e = sum of the four edge neighbours, c = sum of the four corner neighbours, */
/* couples diagonal neighbours, which red-black colouring puts in one colour,  */
/* so four colours are needed: colour (i & 1) + 2 (j & 1); no two points of    */
/* one colour are neighbours.  The Gauss-Seidel update solves point (i, j)'s   */
/* equation lap9(u) = f for u_ij:                                             */
/*     u_ij <- (4 e + c - 6 h^2 f) / 20,                                       */
/* with, in this order (each operation rounded once, no FMA):                  */
/*     e = ((u[i+1][j] + u[i-1][j]) + u[i][j+1]) + u[i][j-1],                  */
/*     c = ((u[i+1][j+1] + u[i+1][j-1]) + u[i-1][j+1]) + u[i-1][j-1],          */
/*     s = 4 e + c;  s = s - (6 (h h)) f;  u = s / 20.                          */
/* One sweep updates colours 0, 1, 2, 3 in turn.                               */
/* ------------------------------------------------------------------------- */
int32_t rbgs_ref_mc9_colour(int64_t i, int64_t j) { return (int32_t)((i & 1) + 2 * (j & 1)); }

int rbgs_ref_mc9_quarter_sweep_f64(int32_t n, int64_t ld, double h, double *u, const double *f,
                                   int32_t colour)
{
    if (bad_grid(n, ld, h) || !u || !f || colour < 0 || colour > 3) return RBGS_REF_EINVAL;
    const double c6 = 6.0 * (h * h);
    const int64_t i0 = (colour & 1) ? 1 : 2, j0 = (colour & 2) ? 1 : 2;
#pragma omp parallel for schedule(static)
    for (int64_t i = i0; i <= n; i += 2) {
        for (int64_t j = j0; j <= n; j += 2) {
            double e = AT(u, i + 1, j) + AT(u, i - 1, j);
            e = e + AT(u, i, j + 1);
            e = e + AT(u, i, j - 1);
            double c = AT(u, i + 1, j + 1) + AT(u, i + 1, j - 1);
            c = c + AT(u, i - 1, j + 1);
            c = c + AT(u, i - 1, j - 1);
            double s = 4.0 * e + c;
            const double t = c6 * AT(f, i, j);
            s = s - t;
            AT(u, i, j) = s / 20.0;
        }
    }
    return RBGS_REF_OK;
}

int rbgs_ref_mc9_sweep_f64(int32_t n, int64_t ld, double h, double *u, const double *f,
                           int32_t nsweeps)
{
    if (bad_grid(n, ld, h) || !u || !f || nsweeps < 0) return RBGS_REF_EINVAL;
    for (int32_t it = 0; it < nsweeps; ++it)
        for (int32_t colour = 0; colour < 4; ++colour)
            rbgs_ref_mc9_quarter_sweep_f64(n, ld, h, u, f, colour);
    return RBGS_REF_OK;
}

/* Residual of the 9-point system: r = f - lap9(u) over the interior with    */
/* lap9(u) = ((4 e + c) - 20 u) * (1 / (6 h h)) in FP64 (e, c summed as in    */
/* the update), b = f - (4 e_g + c_g) * (1 / (6 h h)) with only the ring's    */
/* values (b = f for g = 0); ||r||_2 and ||r||_2/||b||_2 with compensated     */
/* sums, as rbgs_ref_residual_f64.                                            */
int rbgs_ref_mc9_residual_f64(int32_t n, int64_t ld, double h, const double *u, const double *f,
                              double *abs_norm, double *rel_norm, double *r_out)
{
    if (bad_grid(n, ld, h) || !u || !f) return RBGS_REF_EINVAL;
    const double inv6h2 = 1.0 / (6.0 * (h * h));
    double rs = 0.0, rc = 0.0, bs = 0.0, bc = 0.0;
    for (int64_t i = 1; i <= n; ++i) {
        for (int64_t j = 1; j <= n; ++j) {
            double e = AT(u, i + 1, j) + AT(u, i - 1, j);
            e = e + AT(u, i, j + 1);
            e = e + AT(u, i, j - 1);
            double c = AT(u, i + 1, j + 1) + AT(u, i + 1, j - 1);
            c = c + AT(u, i - 1, j + 1);
            c = c + AT(u, i - 1, j - 1);
            const double lap = ((4.0 * e + c) - 20.0 * AT(u, i, j)) * inv6h2;
            const double r = AT(f, i, j) - lap;
            double eb = RING_ONLY(u, i + 1, j) + RING_ONLY(u, i - 1, j);
            eb = eb + RING_ONLY(u, i, j + 1);
            eb = eb + RING_ONLY(u, i, j - 1);
            double cb = RING_ONLY(u, i + 1, j + 1) + RING_ONLY(u, i + 1, j - 1);
            cb = cb + RING_ONLY(u, i - 1, j + 1);
            cb = cb + RING_ONLY(u, i - 1, j - 1);
            const double b = AT(f, i, j) - (4.0 * eb + cb) * inv6h2;
            if (r_out) AT(r_out, i, j) = r;
            neumaier_add(&rs, &rc, r * r);
            neumaier_add(&bs, &bc, b * b);
        }
    }
    const double rn = sqrt(rs + rc), bn = sqrt(bs + bc);
    if (abs_norm) *abs_norm = rn;
    if (rel_norm) *rel_norm = (bn > 0.0) ? rn / bn : rn;
    return RBGS_REF_OK;
}

/* The solve loop of rbgs_ref_solve_f64 around 4-colour 9-point sweeps. */
int rbgs_ref_mc9_solve_f64(int32_t n, int64_t ld, double h, double *u, const double *f,
                           int32_t max_sweeps, double rel_tol, int32_t check_every,
                           int32_t *sweeps_done, double *rel_out)
{
    if (bad_grid(n, ld, h) || !u || !f || max_sweeps < 0 || check_every < 1)
        return RBGS_REF_EINVAL;
    int32_t done = 0;
    double rel = 0.0;
    if (rel_tol <= 0.0) {
        rbgs_ref_mc9_sweep_f64(n, ld, h, u, f, max_sweeps);
        done = max_sweeps;
        rbgs_ref_mc9_residual_f64(n, ld, h, u, f, NULL, &rel, NULL);
    } else {
        rbgs_ref_mc9_residual_f64(n, ld, h, u, f, NULL, &rel, NULL);
        while (!(rel <= rel_tol) && done < max_sweeps) {
            int32_t k = max_sweeps - done < check_every ? max_sweeps - done : check_every;
            rbgs_ref_mc9_sweep_f64(n, ld, h, u, f, k);
            done += k;
            rbgs_ref_mc9_residual_f64(n, ld, h, u, f, NULL, &rel, NULL);
        }
    }
    if (sweeps_done) *sweeps_done = done;
    if (rel_out) *rel_out = rel;
    return (rel_tol <= 0.0 || rel <= rel_tol) ? RBGS_REF_OK : RBGS_REF_ENOCONV;
}

/* ------------------------------------------------------------------------- */
/* Red-black Gauss-Seidel in three dimensions (an extension: the conclusion,  */
/* Section 5, names higher dimensions as future work).  Poisson's equation    */
/* lap(u) = f on the unit cube, N^3 interior points, h = 1/(N+1), the 7-point */
/* Laplacian (sum of the six neighbours - 6 u) / h^2; red points have i+j+k   */
/* even.  The point update solves point (i, j, k)'s equation for u_ijk:       */
/*     s = ((((u[i+1] + u[i-1]) + u[j+1]) + u[j-1]) + u[k+1]) + u[k-1],       */
/*     s = s - (h h) f,  u_ijk = s / 6                                         */
/* (each operation rounded once, no FMA; u[i+1] means u[i+1][j][k], etc.).   */
/* Storage: (n+2) planes (index i) of (n+2) rows (index j) of ld >= n+2       */
/* elements (index k); element (i, j, k) is a[(i (n+2) + j) ld + k]; the      */
/* ring (any index 0 or n+1) holds the Dirichlet data g.                       */
/* ------------------------------------------------------------------------- */
#define AT3(a, i, j, k) ((a)[((size_t)(i) * (size_t)(n + 2) + (size_t)(j)) * (size_t)ld + (size_t)(k)])

static int on_ring3(int32_t n, int64_t i, int64_t j, int64_t k)
{
    return i == 0 || j == 0 || k == 0 || i == (int64_t)n + 1 || j == (int64_t)n + 1 ||
           k == (int64_t)n + 1;
}

int rbgs_ref_rb3_half_sweep_f64(int32_t n, int64_t ld, double h, double *u, const double *f,
                                int32_t colour)
{
    if (bad_grid(n, ld, h) || !u || !f || (colour != 0 && colour != 1)) return RBGS_REF_EINVAL;
    const double h2 = h * h;
#pragma omp parallel for schedule(static)
    for (int64_t i = 1; i <= n; ++i) {
        for (int64_t j = 1; j <= n; ++j) {
            /* first k >= 1 with (i + j + k) & 1 == colour */
            const int64_t k0 = ((i + j + 1) & 1) == colour ? 1 : 2;
            for (int64_t k = k0; k <= n; k += 2) {
                double s = AT3(u, i + 1, j, k) + AT3(u, i - 1, j, k);
                s = s + AT3(u, i, j + 1, k);
                s = s + AT3(u, i, j - 1, k);
                s = s + AT3(u, i, j, k + 1);
                s = s + AT3(u, i, j, k - 1);
                const double t = h2 * AT3(f, i, j, k);
                s = s - t;
                AT3(u, i, j, k) = s / 6.0;
            }
        }
    }
    return RBGS_REF_OK;
}

int rbgs_ref_rb3_sweep_f64(int32_t n, int64_t ld, double h, double *u, const double *f,
                           int32_t nsweeps)
{
    if (bad_grid(n, ld, h) || !u || !f || nsweeps < 0) return RBGS_REF_EINVAL;
    for (int32_t it = 0; it < nsweeps; ++it) {
        rbgs_ref_rb3_half_sweep_f64(n, ld, h, u, f, 0);
        rbgs_ref_rb3_half_sweep_f64(n, ld, h, u, f, 1);
    }
    return RBGS_REF_OK;
}

/* r = f - (s6 - 6 u) * (1 / (h h)) with s6 summed as in the update; b = f -  */
/* (ring-only s6) * (1 / (h h)); norms with compensated sums.                 */
int rbgs_ref_rb3_residual_f64(int32_t n, int64_t ld, double h, const double *u, const double *f,
                              double *abs_norm, double *rel_norm, double *r_out)
{
    if (bad_grid(n, ld, h) || !u || !f) return RBGS_REF_EINVAL;
    const double inv_h2 = 1.0 / (h * h);
    double rs = 0.0, rc = 0.0, bs = 0.0, bc = 0.0;
#define R3(i, j, k) (on_ring3(n, (i), (j), (k)) ? AT3(u, i, j, k) : 0.0)
    for (int64_t i = 1; i <= n; ++i) {
        for (int64_t j = 1; j <= n; ++j) {
            for (int64_t k = 1; k <= n; ++k) {
                double s = AT3(u, i + 1, j, k) + AT3(u, i - 1, j, k);
                s = s + AT3(u, i, j + 1, k);
                s = s + AT3(u, i, j - 1, k);
                s = s + AT3(u, i, j, k + 1);
                s = s + AT3(u, i, j, k - 1);
                const double lap = (s - 6.0 * AT3(u, i, j, k)) * inv_h2;
                const double r = AT3(f, i, j, k) - lap;
                double sb = R3(i + 1, j, k) + R3(i - 1, j, k);
                sb = sb + R3(i, j + 1, k);
                sb = sb + R3(i, j - 1, k);
                sb = sb + R3(i, j, k + 1);
                sb = sb + R3(i, j, k - 1);
                const double b = AT3(f, i, j, k) - sb * inv_h2;
                if (r_out) AT3(r_out, i, j, k) = r;
                neumaier_add(&rs, &rc, r * r);
                neumaier_add(&bs, &bc, b * b);
            }
        }
    }
#undef R3
    const double rn = sqrt(rs + rc), bn = sqrt(bs + bc);
    if (abs_norm) *abs_norm = rn;
    if (rel_norm) *rel_norm = (bn > 0.0) ? rn / bn : rn;
    return RBGS_REF_OK;
}

/* The solve loop of rbgs_ref_solve_f64 around 3D red-black sweeps. */
int rbgs_ref_rb3_solve_f64(int32_t n, int64_t ld, double h, double *u, const double *f,
                           int32_t max_sweeps, double rel_tol, int32_t check_every,
                           int32_t *sweeps_done, double *rel_out)
{
    if (bad_grid(n, ld, h) || !u || !f || max_sweeps < 0 || check_every < 1)
        return RBGS_REF_EINVAL;
    int32_t done = 0;
    double rel = 0.0;
    if (rel_tol <= 0.0) {
        rbgs_ref_rb3_sweep_f64(n, ld, h, u, f, max_sweeps);
        done = max_sweeps;
        rbgs_ref_rb3_residual_f64(n, ld, h, u, f, NULL, &rel, NULL);
    } else {
        rbgs_ref_rb3_residual_f64(n, ld, h, u, f, NULL, &rel, NULL);
        while (!(rel <= rel_tol) && done < max_sweeps) {
            int32_t kk = max_sweeps - done < check_every ? max_sweeps - done : check_every;
            rbgs_ref_rb3_sweep_f64(n, ld, h, u, f, kk);
            done += kk;
            rbgs_ref_rb3_residual_f64(n, ld, h, u, f, NULL, &rel, NULL);
        }
    }
    if (sweeps_done) *sweeps_done = done;
    if (rel_out) *rel_out = rel;
    return (rel_tol <= 0.0 || rel <= rel_tol) ? RBGS_REF_OK : RBGS_REF_ENOCONV;
}
#undef AT3

/* Colour query used by the tests to check the colouring convention. */
int32_t rbgs_ref_colour(int64_t i, int64_t j) { return colour_of(i, j); }
