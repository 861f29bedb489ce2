/*
 * rbgs.h - red-black Gauss-Seidel for the 5-point 2D Poisson stencil on
 * AMD Instinct MI355X (gfx950).  C ABI of librbgs.so.
 *
 * The method (paper, Section 2): laplace(u) = f on the unit square with
 * Dirichlet data u = g on the boundary, N x N interior points, spacing
 * h = 1/(N+1), point update Eq. (1)
 *     u_ij <- 1/4 (u_{i+1,j} + u_{i-1,j} + u_{i,j+1} + u_{i,j-1} - h^2 f_ij),
 * red points (i+j even) first, then black points (i+j odd); one red and one
 * black half-sweep form one full sweep (one iteration of Algorithms 1 and 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid arrays (u, f) are DEVICE pointers owned by the caller, in the natural
 * row-major layout with the boundary ring included: n+2 rows of ld >= n+2
 * elements, element (i, j) at a[i*ld + j], 0 <= i, j <= n+1; i is the row
 * (the outer loop of Algorithm 1), j the column.  In u the ring (row 0, row
 * n+1, column 0, column n+1) holds g and is read, never written; the ring of
 * f is never read.  u is in/out.
 *
 * Arithmetic: the four neighbours are summed in the order written in Eq. (1)
 * (i+1, i-1, j+1, j-1), then h^2*f is subtracted and the sum scaled by 1/4;
 * h^2 = h*h is formed in FP64 and rounded once to the working precision; no
 * FMA contraction.  With these rules the FP64 sweep reproduces, bit for bit,
 * any correct sequential red-black Gauss-Seidel that uses the same order.
 *
 * Scratch: the library never allocates device memory.  Entry points that
 * need scratch take a caller-owned device workspace of at least the size
 * returned by the matching *_workspace_size call, 256-byte aligned.
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  All
 * device work is enqueued on it.  Entry points that return host values
 * (residual norms, solve statistics) synchronise that stream; rbgs_sweep
 * and rbgs_sweep_batched do not.
 *
 * Errors: every entry point returns RBGS_OK (0) or a negative rbgs_status.
 * Argument checks run before any device work, so RBGS_EINVAL and
 * RBGS_EWORKSPACE leave every buffer untouched.  rbgs_last_error() gives a
 * human-readable message for the calling thread's last failure.
 * Calls on different streams with disjoint buffers are independent.
 */
#ifndef RBGS_H
#define RBGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RBGS_OK = 0,
    RBGS_EINVAL = -1,       /* bad argument (size, pointer, h, count, ...) */
    RBGS_EHIP = -2,         /* a HIP runtime call or kernel launch failed  */
    RBGS_ENOCONV = -3,      /* tolerance not reached within the sweep cap  */
    RBGS_ETIMEOUT = -4,     /* a bounded wait in the persistent kernel expired */
    RBGS_ENONFINITE = -5,   /* the residual became NaN or infinite         */
    RBGS_EUNSUPPORTED = -6, /* valid but not implemented (e.g. SOR in FP32)  */
    RBGS_EWORKSPACE = -8,   /* workspace missing, too small or misaligned  */
    RBGS_EORDER = -9        /* debug_stamp_check: a persistent-kernel work item
                               saw a neighbour tile more than one pass ahead
                               (the dependency rule of Algorithm 2 broken)  */
} rbgs_status;

typedef enum {
    RBGS_F64 = 0, /* IEEE binary64 storage and arithmetic */
    RBGS_F32 = 1  /* IEEE binary32 storage and arithmetic */
} rbgs_dtype;

typedef enum {
    RBGS_KERNEL_AUTO = 0,    /* library choice, from measured time per sweep:
                                PLAIN below 8 sweeps; else RESIDENT up to
                                n = 384 (FP64) / 768 (FP32), PLAIN for FP32
                                n < 1536, BLOCKED otherwise                    */
    RBGS_KERNEL_PLAIN = 1,   /* one kernel launch per half-sweep (Algorithm 1's
                                barrier after every colour)                     */
    RBGS_KERNEL_BLOCKED = 2, /* persistent, temporally blocked kernel: several
                                half-sweeps per pass over HBM, tiles ordered by
                                per-tile progress flags instead of grid-wide
                                barriers (the dependency idea of Algorithm 2)   */
    RBGS_KERNEL_RESIDENT = 3 /* small grids (n <= 512 in FP64, n <= 1024 in
                                FP32): Algorithm 2's stripes as co-resident
                                workgroups that keep their rows in registers
                                for all sweeps of the call and trade boundary
                                rows with their two neighbours every 4 sweeps;
                                RBGS_EUNSUPPORTED for larger n              */
} rbgs_kernel;

typedef enum {
    RBGS_PREC_F64 = 0,        /* plain sweeps in the storage precision          */
    RBGS_PREC_F32_IR = 1,     /* FP64 residual + correction, FP32 inner sweeps  */
    RBGS_PREC_BF16RHS_IR = 2  /* as above with the inner rhs rounded to bfloat16 */
} rbgs_precision;

/* One grid: N = n interior points per side, row pitch ld (elements), h. */
typedef struct {
    int32_t n;   /* interior points per side, 1 <= n <= 65533         */
    int64_t ld;  /* row pitch in elements, ld >= n + 2                */
    double h;    /* grid spacing, finite and > 0 (1/(n+1) on [0,1]^2) */
} rbgs_grid;

/* Optional per-call timing, filled when rbgs_sweep_opts.timing != NULL
 * (in rbgs_sweep, or in rbgs_solve through rbgs_solve_opts.sweep).  The
 * library then brackets its kernel groups with HIP events on `stream` and
 * synchronises the stream before returning; in a solve, sweep_ms sums the
 * sweep groups between residual checks. */
typedef struct {
    float pack_ms;          /* natural -> split packing of u and f            */
    float sweep_ms;         /* all sweep kernels (half-sweeps or blocked passes) */
    float unpack_ms;        /* split -> natural unpacking of u                */
    int32_t sweep_launches; /* kernel launches inside sweep_ms                */
    float persistent_ms;    /* BLOCKED: the launch(es) of the deeper passes
                               alone (no ring copies, no passes one sweep
                               shallower); RESIDENT: its launches             */
    int32_t persistent_launches; /* launches inside persistent_ms             */
    int32_t passes;         /* BLOCKED: passes those launches ran             */
    int32_t fuse;           /* BLOCKED: sweeps per pass in those launches     */
} rbgs_timing;

/* Kernel selection for sweeps.  Zero-initialise for the library defaults. */
typedef struct {
    int32_t kernel;     /* rbgs_kernel                                         */
    int32_t fuse;       /* BLOCKED: most sweeps per pass (1..10), 0 = default;
                           nsweeps runs as ceil(nsweeps / fuse) passes whose
                           depths differ by at most one                      */
    int32_t tile_rows;  /* BLOCKED: interior rows per tile, 8..65536, 0 = default */
    int32_t tile_cols;  /* BLOCKED: interior columns per tile, 0 = default     */
    int32_t rows_per_block; /* PLAIN: rows each workgroup marches, 0 = default */
    int32_t debug_delay;    /* BLOCKED: >0 injects pseudo-random per-tile delays
                               (schedule stress); results must not change      */
    int32_t debug_spin_limit; /* BLOCKED: >0 bounds each flag wait to this many
                               polls (watchdog tests); 0 = default bound       */
    int32_t debug_stall_tile; /* BLOCKED: t+1 > 0 makes tile t never publish its
                               progress, so its neighbours' bounded waits expire
                               and the call returns RBGS_ETIMEOUT (watchdog
                               test; every wave still exits)                   */
    rbgs_timing *timing;    /* HOST pointer or NULL (see rbgs_timing)          */
    int32_t lds_max_n;      /* BATCHED: grids with n <= lds_max_n whose iterate
                               and h^2 f fit in one workgroup's LDS are swept
                               there, one workgroup per grid, for all sweeps
                               of the call; the others go through the
                               persistent tiles.  0 = the autotuner's choice
                               for this batch shape (127 FP32 / 63 FP64, or
                               never), else never; -1 = never.  Ignored
                               elsewhere.                                       */
    /* Verification modes of the single-grid persistent (BLOCKED) kernel, for
     * tests of the dependency rule (Section 2.3, Algorithm 2); results must
     * not change.  RBGS_EUNSUPPORTED in batched sweeps.                     */
    int32_t debug_tile_order;  /* order of the tiles within a pass: 0 as
                                  numbered, 1 reversed, 2 a permutation per
                                  pass drawn from debug_seed (tickets stay
                                  pass-major, so no order can deadlock)      */
    uint32_t debug_seed;       /* seed of debug_tile_order 2                  */
    int32_t debug_stamp_check; /* 1: before and after each work item (pass p,
                                  tile t), every tile of t's 3 x 3
                                  neighbourhood must have completed p or p + 1
                                  passes (p + 2 would mean it overwrote the
                                  buffer t reads); else RBGS_EORDER          */
    int32_t debug_trace_items; /* records debug_trace holds (0: no trace)      */
    uint64_t *debug_trace;     /* DEVICE array of debug_trace_items records of
                                  4 words, or NULL: for the work items of the
                                  deeper passes (those rbgs_timing's
                                  persistent_ms covers), record k = ticket k
                                  of those launches in order (pass-major):
                                  {start, end, (pass << 32) | tile,
                                  (workgroup << 32) | ticket within its
                                  launch}; start and end read the device's
                                  constant-rate real-time counter (100 MHz)
                                  after the dependency wait and after the
                                  item's writes were released.  Records past
                                  debug_trace_items are dropped; the caller
                                  zero-fills the array to spot unwritten ones.
                                  The array is owned by the caller.          */
} rbgs_sweep_opts;

/* Solve options.  Zero-initialise, then set what is needed. */
typedef struct {
    int32_t max_sweeps;    /* cap on full sweeps (all inner sweeps in IR modes) */
    double rel_tol;        /* stop at ||r||_2/||b||_2 <= rel_tol; <= 0: run
                              exactly max_sweeps sweeps                       */
    int32_t check_every;   /* full sweeps between residual checks, >= 1        */
    int32_t precision;     /* rbgs_precision; IR modes need RBGS_F64 storage   */
    int32_t inner_sweeps;  /* IR: FP32 sweeps per outer step (0 = check_every) */
    double omega;          /* relaxation: 1.0 = Gauss-Seidel (the paper's method);
                              in (0, 2) = red-black SOR, u <- u + omega (g - u)
                              with g the Gauss-Seidel value (an extension: FP64,
                              plain, resident or blocked kernel (the blocked
                              one reads and writes red every pass), no
                              refinement, no sweep verification modes; else
                              RBGS_EUNSUPPORTED); 0.0 = the model problem's
                              optimum 2 / (1 + sin(pi h)) for this grid's h   */
    rbgs_sweep_opts sweep; /* kernel choice for the (inner) sweeps             */
    int32_t fallback;      /* IR: 1 = widen the inner precision when it stops
                              helping (not in the paper; the build's rule): a
                              value of r that the inner right-hand-side format
                              cannot hold switches to FP64 sweeps of u at once;
                              an outer step after the first that leaves rel no
                              lower turns a bfloat16 right-hand side into FP32,
                              FP32 inner sweeps into FP64 sweeps of u
                              (inner_sweeps at a time, residual after each).
                              info->precision reports where it ended.  0 = off.
                              Not available for batches (RBGS_EUNSUPPORTED).  */
} rbgs_solve_opts;

typedef struct {
    int32_t sweeps;        /* full sweeps performed (inner sweeps in IR)       */
    int32_t outer_iters;   /* IR outer steps performed (0 for plain solves)    */
    double rel_residual;   /* final ||r||_2/||b||_2 (||r||_2 if ||b||_2 = 0)   */
    double abs_residual;   /* final ||r||_2                                    */
    int32_t status;        /* same value as the return code                    */
    int32_t precision;     /* rbgs_precision of the sweeps at the end: the
                              requested one, or a wider one after a fallback
                              (RBGS_PREC_F64 for plain solves)                */
} rbgs_solve_info;

/* Size in bytes of the workspace that rbgs_sweep, rbgs_residual and
 * rbgs_solve need for grid g and storage type dt: the red and black arrays
 * of u and f (the separate colour arrays of Section 2.1), the persistent
 * kernels' second buffer and state, the residual's partial sums, and for
 * the IR modes the FP32 right-hand side and correction (mixed precision
 * read as FP64 refinement around narrower inner sweeps).  `opts` (may be NULL)
 * selects the solve mode.  Returns 0 for invalid arguments. */
size_t rbgs_workspace_size(const rbgs_grid *g, rbgs_dtype dt,
                           const rbgs_solve_opts *opts);

/* nsweeps full red-black sweeps of u in place (Eq. (1); red half-sweep then
 * black half-sweep, Algorithms 1 and 2).  u, f: device arrays as above, of
 * type dt.  nsweeps >= 0 (0 is a no-op).  opts may be NULL (defaults).
 * Every kernel choice gives the same bits.  Asynchronous on `stream`. */
int rbgs_sweep(const rbgs_grid *g, rbgs_dtype dt, void *u, const void *f,
               int32_t nsweeps, const rbgs_sweep_opts *opts, void *workspace,
               size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------
 * Split colour layout at the boundary, for callers that keep u and f in
 * it between calls (the paper stores the colours apart, Section 2.1):
 * colour C of point (i, j) is (i + j) & 1 (0 = red) and the point sits at
 * element (i * pitch + (j >> 1)) of that colour's array of n + 2 rows,
 * pitch = rbgs_split_pitch(g, dt) = ceil((n + 2) / 2) rounded up to 256
 * bytes.  Every sweep call otherwise packs u and f into this layout and
 * unpacks u, one pass each.
 * --------------------------------------------------------------------- */

/* Elements per row of a colour array; 0 for invalid arguments. */
int64_t rbgs_split_pitch(const rbgs_grid *g, rbgs_dtype dt);

/* natural (n+2) x ld array -> red and black arrays (DEVICE, each (n+2) x
 * pitch elements; entries past column n+1 are set to 0).  Asynchronous. */
int rbgs_pack(const rbgs_grid *g, rbgs_dtype dt, const void *nat, void *red,
              void *black, void *stream);

/* red and black arrays -> the interior of the natural array (its ring is
 * not written).  Asynchronous. */
int rbgs_unpack(const rbgs_grid *g, rbgs_dtype dt, void *nat, const void *red,
                const void *black, void *stream);

/* nsweeps sweeps of the split iterate (u_red, u_black) in place with the
 * split right-hand side (f_red, f_black): the same kernels and the same
 * bits as rbgs_sweep, without its pack and unpack.  The workspace
 * (rbgs_workspace_size) holds the persistent kernels' second buffer and
 * state.  opts->timing must be NULL.  Synchronises `stream` when a
 * persistent kernel ran (its error word is read), else asynchronous. */
int rbgs_sweep_split(const rbgs_grid *g, rbgs_dtype dt, void *u_red,
                     void *u_black, const void *f_red, const void *f_black,
                     int32_t nsweeps, const rbgs_sweep_opts *opts,
                     void *workspace, size_t workspace_bytes, void *stream);

/* Residual of the discrete system whose Gauss-Seidel step is Eq. (1):
 *   r_ij = f_ij - (u_{i+1,j} + u_{i-1,j} + u_{i,j+1} + u_{i,j-1} - 4 u_ij)/h^2
 * over the interior, and b = r evaluated with the interior of u set to zero
 * (b = f for g = 0).  Writes ||r||_2 to *abs_norm and ||r||_2/||b||_2 (or
 * ||r||_2 when ||b||_2 = 0) to *rel_norm, both HOST pointers (either may be
 * NULL).  All arithmetic in FP64 (FP32 data is widened); the sums of squares
 * are reduced in a fixed order, so repeated calls give identical bits.
 * Synchronises `stream`. */
int rbgs_residual(const rbgs_grid *g, rbgs_dtype dt, const void *u,
                  const void *f, double *abs_norm, double *rel_norm,
                  void *workspace, size_t workspace_bytes, void *stream);

/* rbgs_residual for callers that cannot allocate device memory or pass a
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same kernels, the same results bit for bit,
 * but the partial sums live in a static device array of 4 MiB that the
 * library holds on each GPU it runs on until the process ends, so no
 * workspace argument.  Grids whose partial sums do not fit (n above about
 * 23 000; 256 + 16 * ceil(n/256) * ceil(n/8) bytes) return RBGS_EINVAL
 * before any device work.  Calls no hipMalloc, hipFree or allocating
 * library routine.  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (different streams or host threads) race and
 * must be serialised by the caller.  u, f, abs_norm, rel_norm as for
 * rbgs_residual; synchronises `stream`. */
int rbgs_residual_noalloc(const rbgs_grid *g, rbgs_dtype dt, const void *u,
                          const void *f, double *abs_norm, double *rel_norm,
                          void *stream);

/* Sweeps until rel <= opts->rel_tol or opts->max_sweeps sweeps.
 * Algorithms 1 and 2 repeat Eq. (1)'s sweep a given number of times and
 * return the converged solution; the paper states no stopping test, so the
 * residual, norm and test are this library's choice, the ones
 * rbgs_residual computes (rel = ||r||_2 / ||b||_2), and max_sweeps with rel_tol <= 0 is the
 * paper's fixed iteration count.  The
 * residual is evaluated before the first sweep and after every check_every
 * sweeps (the last group is shortened to end exactly at max_sweeps).
 * RBGS_PREC_F64: plain sweeps in dt.  IR modes (dt must be RBGS_F64): each
 * outer step computes r = f - A_h u in FP64, stops if rel <= rel_tol, rounds
 * r to FP32 (or bfloat16), runs inner_sweeps FP32 sweeps of A_h e = r from
 * e = 0 with a zero ring, and adds e to u in FP64.  The whole rounds (sweeps
 * or an outer step, the residual, a device-side convergence test) run as
 * replays of a captured HIP graph, four per host poll; rounds of more than
 * 65536 launches, the sweeps after the last whole round and calls with
 * timing requested run launch by launch instead (same results).  info
 * (HOST, may be NULL) receives the statistics.  Returns RBGS_OK,
 * RBGS_ENOCONV (u holds the last iterate), RBGS_ENONFINITE, or an error.
 * Synchronises `stream`. */
int rbgs_solve(const rbgs_grid *g, rbgs_dtype dt, void *u, const void *f,
               const rbgs_solve_opts *opts, rbgs_solve_info *info,
               void *workspace, size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------
 * Batches of independent grids (one persistent launch for all of them).
 * Grid g has its own size grids[g], device arrays u[g] and f[g] (natural
 * layout, type dt; the HOST arrays u and f hold the device pointers).  Work
 * items are (pass, grid, tile) of the persistent blocked kernel, handed out
 * pass by pass with the largest grids first; each grid's tiles follow the
 * same dependency rule as a single grid, so every grid's result is bitwise
 * what rbgs_sweep gives it alone.  Small grids (opts->lds_max_n) are instead
 * swept entirely in one workgroup's LDS, with the same operations in the
 * same order, hence the same bits.  count in [1, 65535].
 * opts: kernel must be AUTO or BLOCKED; fuse/tile_rows 0 take the values
 * rbgs_autotune_batched stored for this batch shape (else the defaults).
 * --------------------------------------------------------------------- */

/* Workspace bytes for a batch (0 for invalid arguments). */
size_t rbgs_batch_workspace_size(int32_t count, const rbgs_grid *grids,
                                 rbgs_dtype dt);

/* nsweeps sweeps of every grid of the batch, in place.  Uploads its tables
 * and reads the kernel's error word, so it synchronises `stream`.  Returns
 * RBGS_ETIMEOUT if a bounded dependency wait expired. */
int rbgs_sweep_batched(int32_t count, const rbgs_grid *grids, rbgs_dtype dt,
                       void *const *u, const void *const *f, int32_t nsweeps,
                       const rbgs_sweep_opts *opts, void *workspace,
                       size_t workspace_bytes, void *stream);

/* A batched sweep captured once into a HIP graph (pack, persistent
 * kernel(s), unpack; flags and tickets are cleared by kernels inside the
 * graph, so every replay starts clean).  The plan keeps the pointers given
 * here: u, f and the workspace must stay allocated while it is used.  Each
 * rbgs_batch_plan_launch advances every grid by nsweeps sweeps,
 * asynchronously on `stream`; rbgs_batch_plan_check synchronises `stream`
 * and returns RBGS_ETIMEOUT if a wait expired in any replay since the last
 * check (RBGS_OK otherwise). */
typedef struct rbgs_batch_plan rbgs_batch_plan;
int rbgs_batch_plan_create(rbgs_batch_plan **plan, int32_t count,
                           const rbgs_grid *grids, rbgs_dtype dt,
                           void *const *u, const void *const *f,
                           int32_t nsweeps, const rbgs_sweep_opts *opts,
                           void *workspace, size_t workspace_bytes);
int rbgs_batch_plan_launch(rbgs_batch_plan *plan, void *stream);
int rbgs_batch_plan_check(rbgs_batch_plan *plan, void *stream);
int rbgs_batch_plan_destroy(rbgs_batch_plan *plan);

/* Autotuner: times the persistent kernel on this batch for fusion depths
 * {4, 5, 6, 7} and tile heights {64, 128, 256} (two passes each after a
 * warm-up pass; the workspace copies are swept, u and f are only read),
 * then, for the best of those, the LDS-resident threshold (lds_max_n: none,
 * or 127 FP32 / 63 FP64), and stores the fastest choice for the batch shape
 * (dtype, CU count and the
 * multiset of grid sizes) in a process-wide table, appends it to the file
 * named by the environment variable RBGS_TUNE_CACHE if set (and reads that
 * file on first use), and returns it in *best (HOST, may be NULL) with its
 * time per sweep in *best_ms_per_sweep (HOST, may be NULL).  Synchronises. */
int rbgs_autotune_batched(int32_t count, const rbgs_grid *grids,
                          rbgs_dtype dt, void *const *u, const void *const *f,
                          void *workspace, size_t workspace_bytes,
                          void *stream, rbgs_sweep_opts *best,
                          float *best_ms_per_sweep);

/* Batched solve to a tolerance: every grid of the batch (FP64 u and f,
 * natural layout, HOST arrays of device pointers as above) is solved as
 * rbgs_solve solves it alone, in one of two modes.
 *   precision F64: the solve loop around Eq. (1)'s sweeps (the paper
 *     fixes no stopping test; the norms are rbgs_residual's): the relative
 *     residual, then check_every FP64 sweeps (inner_sweeps when check_every
 *     is 0; the last round of a grid near max_sweeps takes the remainder),
 *     until rel <= rel_tol or max_sweeps.  outer_iters is 0.
 *   precision F32_IR or BF16RHS_IR (the mixed-precision refinement the
 *     build adds to the paper's method): an FP64 residual, r rounded to
 *     FP32 (or bfloat16), inner_sweeps FP32 sweeps of A e = r from e = 0
 *     with a zero ring (check_every when inner_sweeps is 0), u <- u + e in
 *     FP64, until rel <= rel_tol or max_sweeps.
 * The sweeps of all grids still iterating run as one batched persistent
 * launch per round (opts->sweep selects its tuning; the autotuner's table
 * applies); a converged grid is left alone, so each grid's result is
 * bitwise that of rbgs_solve on it alone.  Needs rel_tol > 0 and fallback
 * = 0 (RBGS_EUNSUPPORTED).  omega: 1 = Gauss-Seidel; with precision F64
 * also red-black SOR (an extension, as in rbgs_solve), omega in (0, 2)
 * for every grid or 0 for each grid's own optimum 2 / (1 + sin(pi h)),
 * every grid swept by the tiled kernel (none LDS-resident); SOR with the
 * IR precisions is RBGS_EUNSUPPORTED, omega outside [0, 2) RBGS_EINVAL.  infos (HOST, count entries, may be NULL)
 * receives each grid's sweeps, outer steps, norms, status and precision.
 * Returns RBGS_OK when every grid converged, else the first failing grid's
 * status (RBGS_ENOCONV, RBGS_ENONFINITE).  The workspace
 * (rbgs_batch_solve_workspace_size bytes, 256-byte aligned) serves both
 * modes.  Synchronises `stream`. */
size_t rbgs_batch_solve_workspace_size(int32_t count, const rbgs_grid *grids);
int rbgs_solve_batched(int32_t count, const rbgs_grid *grids, double *const *u,
                       const double *const *f, const rbgs_solve_opts *opts,
                       rbgs_solve_info *infos, void *workspace,
                       size_t workspace_bytes, void *stream);

/* Message for the calling thread's last failure in a batched call. */
const char *rbgs_batch_last_error(void);

/* ---------------------------------------------------------------------
 * Learned initial guess (not in the paper): a small U-Net f -> u0 trained
 * on (f, u*) pairs that this library's solver produced, run and trained by
 * the library's own BF16/FP32 kernels.  Four levels N_l = (N_{l-1}+1)/F - 1
 * with coarsening factor F = 2 (N = 2^k - 1 in [63, 8191]) or F = 4 (N + 1
 * a multiple of 64, N in [127, 8191]; the coarsest level's convolutions then
 * see the whole grid); input f/rms(f), output u0 = net(f/rms(f)) * rms(f).  Batched arrays are `batch` natural-layout grids
 * of (n+2) x ld doubles stored back to back.  Parameters: one FP32 vector of
 * rbgs_unet_param_count() values, per conv layer its weight (cout, cin,
 * 3, 3) then bias (cout), in the order enc0.0, enc0.1, ..., enc3.1,
 * dec2.0, dec2.1, dec1.0, dec1.1, dec0.0, dec0.1, then the 1x1 head's 16
 * weights and 1 bias.  All state (master weights, Adam moments, BF16
 * copies, activations) lives in the caller's workspace.
 * --------------------------------------------------------------------- */
typedef struct rbgs_unet rbgs_unet;
size_t rbgs_unet_param_count(void);
size_t rbgs_unet_workspace_size(int32_t n, int32_t batch, int32_t factor);
int rbgs_unet_create(rbgs_unet **net, int32_t n, int32_t batch,
                     int32_t factor, void *workspace, size_t workspace_bytes);
int rbgs_unet_destroy(rbgs_unet *net);
/* HOST vector in; resets the Adam state.  Synchronises. */
int rbgs_unet_set_params(rbgs_unet *net, const float *params, size_t count,
                         void *stream);
/* HOST vectors out.  Synchronise. */
int rbgs_unet_get_params(rbgs_unet *net, float *params, size_t count,
                         void *stream);
int rbgs_unet_get_grads(rbgs_unet *net, float *grads, size_t count,
                        void *stream);
/* Adam's state, to save and resume a training run (the optimiser of Kingma
 * and Ba that the learned part is trained with; not in the paper): the
 * first and second moment estimates m and v, count = rbgs_unet_param_count()
 * FP32 values each in the parameter order (HOST arrays), and *step / step,
 * the number of Adam steps taken (its bias corrections use it).  get copies
 * them out; set restores them, after rbgs_unet_set_params (which restarts
 * Adam), so that the next update continues the saved run bit for bit.
 * RBGS_EINVAL on a NULL array, a wrong count or step < 0.  Synchronise. */
int rbgs_unet_get_adam(rbgs_unet *net, float *m, float *v, size_t count,
                       int32_t *step, void *stream);
int rbgs_unet_set_adam(rbgs_unet *net, const float *m, const float *v,
                       size_t count, int32_t step, void *stream);
/* u0 (device) interior <- network guess for f (device); u0's ring is left
 * untouched.  batch <= the batch given at creation.  Asynchronous. */
int rbgs_unet_forward(rbgs_unet *net, int32_t batch, const double *f,
                      int64_t ld, double *u0, void *stream);
/* One training step on a batch: forward, mean squared error against
 * u_target/rms(f) on the interior, backward into the gradient vector, and
 * (update != 0) one Adam step with learning rate lr (beta 0.9/0.999,
 * eps 1e-8).  *loss (HOST, may be NULL) receives the loss before the
 * update; passing it synchronises. */
int rbgs_unet_train_step(rbgs_unet *net, int32_t batch, const double *f,
                         const double *u_target, int64_t ld, float lr,
                         int32_t update, float *loss, void *stream);
/* Solve with the learned guess.  The network's guess and the caller's start
 * u (same Dirichlet ring) are both given compare_after sweeps (0: none);
 * the guess replaces the start only if its relative residual is then lower
 * (the plain start is both fallback and judge), and rbgs_solve continues
 * for the remaining max_sweeps - compare_after sweeps (max_sweeps bounds the
 * sweeps applied to the returned iterate).  info->sweeps counts every sweep
 * run: 2 * compare_after comparison sweeps (both starts) plus the solve's.
 * *used_guess and *rel_start (HOST, may be NULL) report the choice.  Needs
 * ld = n + 2. */
int rbgs_solve_learned(rbgs_unet *net, const rbgs_grid *g, double *u,
                       const double *f, const rbgs_solve_opts *opts,
                       int32_t compare_after, rbgs_solve_info *info,
                       int32_t *used_guess, double *rel_start,
                       void *workspace, size_t workspace_bytes,
                       void *stream);
const char *rbgs_unet_last_error(void);

/* ---------------------------------------------------------------------
 * Grid transfers for nested iteration (not in the paper): the learned
 * guess's training targets are converged by solving a coarse grid first,
 * interpolating, and sweeping the next finer grid.  Levels are vertex-
 * centred: fine n_f = 2 n_c + 1, and coarse point (I, J) sits on fine point
 * (2I, 2J) in natural indexing (rings at index 0 and n+1 on both levels).
 * `batch` >= 1 grids per level, stored at a constant element stride of at
 * least (n+2) * ld of that level; input and output must not overlap.  Only
 * n and ld of each rbgs_grid are used (h must still be valid).
 * Asynchronous on `stream`.
 * --------------------------------------------------------------------- */

/* Coarse interior <- full weighting, (1,2,1) x (1,2,1) / 16, of the fine
 * interior.  The fine ring is not read and the coarse ring not written. */
int rbgs_restrict(int32_t batch, rbgs_dtype dt, const rbgs_grid *fine,
                  const void *x_fine, int64_t fine_stride,
                  const rbgs_grid *coarse, void *x_coarse,
                  int64_t coarse_stride, void *stream);

/* Fine interior <- bilinear interpolation of the coarse grid (its ring
 * included: fine points next to the ring interpolate towards it).  The fine
 * ring is not written. */
int rbgs_prolong(int32_t batch, rbgs_dtype dt, const rbgs_grid *coarse,
                 const void *x_coarse, int64_t coarse_stride,
                 const rbgs_grid *fine, void *x_fine, int64_t fine_stride,
                 void *stream);

/* ---------------------------------------------------------------------
 * Multigrid with red-black Gauss-Seidel as the smoother (an extension: the
 * conclusion, Section 5, names multilevel odd-even techniques as future
 * work).  The textbook V-cycle on the vertex-centred hierarchy
 *   n_0 = n, n_{l+1} = (n_l - 1) / 2 while n_l is odd and >= 3
 *   (and fewer than max_levels levels when max_levels > 0), h_{l+1} = 2 h_l;
 * each coarse level is the same 5-point system (rediscretised) for the error
 * of the level above, with a zero ring.  On a level above the coarsest:
 * pre_sweeps sweeps (Eq. (1), red then black), r = f - A_h u, coarse
 * right-hand side = full weighting (1,2,1) x (1,2,1) / 16 of r, coarse
 * iterate = 0, the cycle on the coarser level, u += bilinear interpolation
 * of the coarse iterate, post_sweeps sweeps.  On the coarsest level:
 * coarse_sweeps sweeps (0 = 1 when it is a single point, which one sweep
 * solves exactly, else 2 (n_L + 1)^2).  The transfers' rounding order is
 * fixed (see the multigrid kernels' source), so the iterate after any
 * number of cycles is bitwise that of the CPU definition.  FP64 only.
 * --------------------------------------------------------------------- */
typedef struct {
    int32_t max_cycles;    /* cap on V-cycles, >= 0                            */
    double rel_tol;        /* stop at ||r||_2/||b||_2 <= rel_tol, checked before
                              the first cycle and after each; <= 0: run
                              exactly max_cycles cycles                       */
    int32_t pre_sweeps;    /* sweeps before the coarse correction, >= 0       */
    int32_t post_sweeps;   /* sweeps after it, >= 0; pre + post >= 1          */
    int32_t max_levels;    /* 0 = coarsen as far as the sizes allow, else at
                              most this many levels (1 = plain sweeps)         */
    int32_t coarse_sweeps; /* sweeps on the coarsest level; 0 = the default    */
    rbgs_sweep_opts sweep; /* kernel for every level's sweeps: AUTO picks per
                              level; RESIDENT needs every level to fit it;
                              timing is not supported (must be NULL)          */
} rbgs_mg_opts;

typedef struct {
    int32_t cycles;        /* V-cycles performed                              */
    int32_t levels;        /* levels of the hierarchy                         */
    int32_t coarsest_n;    /* size of the coarsest level                      */
    int32_t coarse_sweeps; /* sweeps used on it                               */
    double rel_residual;   /* final ||r||_2/||b||_2 (||r||_2 if ||b||_2 = 0)  */
    double abs_residual;   /* final ||r||_2                                   */
    int32_t graph;         /* 1 if the cycles ran as replays of a captured
                              graph, 0 if launched one by one                 */
    int32_t status;        /* same value as the return code                   */
} rbgs_mg_info;

/* Workspace bytes for rbgs_mg_solve (all levels' split arrays and kernel
 * state); 0 for invalid arguments.  opts may be NULL (max_levels = 0). */
size_t rbgs_mg_workspace_size(const rbgs_grid *g, rbgs_dtype dt,
                              const rbgs_mg_opts *opts);

/* V-cycles until rel <= opts->rel_tol or opts->max_cycles cycles.  u, f:
 * DEVICE arrays in the natural layout (as rbgs_solve); the ring of u is the
 * Dirichlet data and is not written.  dt must be RBGS_F64 (else
 * RBGS_EUNSUPPORTED).  The cycles run as replays of a captured HIP graph
 * (cycle, residual and a device-side convergence test), with a launch-by-
 * launch fallback (also taken when a cycle has more than 65536 launches,
 * e.g. tens of thousands of sweeps on a large coarsest level; info->graph
 * says which ran).  info (HOST, may be NULL) receives the statistics.
 * Returns RBGS_OK, RBGS_ENOCONV (u holds the last iterate), RBGS_ENONFINITE,
 * RBGS_ETIMEOUT (a persistent smoother's bounded wait expired) or an error.
 * Synchronises `stream`. */
int rbgs_mg_solve(const rbgs_grid *g, rbgs_dtype dt, void *u, const void *f,
                  const rbgs_mg_opts *opts, rbgs_mg_info *info,
                  void *workspace, size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------
 * Four-colour Gauss-Seidel for the 9-point Laplacian (an extension: the
 * conclusion, Section 5, names multi-colour variants for wider stencils).
 * The system is lap9(u) = f with
 *   lap9(u)_ij = (4 e_ij + c_ij - 20 u_ij) / (6 h^2),
 * e = sum of the four edge neighbours, c = sum of the four corner
 * neighbours; points are coloured (i & 1) + 2 (j & 1), which separates all
 * eight neighbours, and one sweep updates colours 0, 1, 2, 3 in turn, each
 * point by u_ij = ((4 e + c) - 6 (h h) f_ij) / 20 (e and c summed in the
 * order N, S, E, W and NE, NW, SE, SW; no FMA): bitwise the CPU definition.
 * FP64 only.  u, f: DEVICE arrays in the natural layout (as rbgs_sweep);
 * the ring of u is the Dirichlet data.  The residual is r = f - lap9(u),
 * b = r with the interior of u set to zero (b = f for g = 0).
 * --------------------------------------------------------------------- */

/* Workspace bytes (four colour arrays each of u and f, reduction space);
 * 0 for an invalid grid. */
size_t rbgs_mc9_workspace_size(const rbgs_grid *g);

/* nsweeps sweeps of u in place.  kernel: RBGS_KERNEL_AUTO or
 * RBGS_KERNEL_PLAIN = one launch per colour (a device-wide barrier between
 * colours, Algorithm 1's structure); RBGS_KERNEL_RESIDENT = the
 * flag-driven form, the dependency rule of Algorithm 2 (Section 2.3)
 * carried to four colours: all quarter-sweeps of the call in one launch,
 * the (i >> 1, j >> 1) index grid cut into blocks whose quarter-sweep h
 * waits only until the block and its eight neighbours have completed h
 * quarter-sweeps (a counter per block; bounded waits), same result bit
 * for bit; this form reads its error word at the end, so it synchronises
 * `stream` and may return RBGS_ETIMEOUT; nsweeps <= 2^29.
 * RBGS_KERNEL_BLOCKED: RBGS_EUNSUPPORTED.  Asynchronous on `stream` with
 * PLAIN. */
int rbgs_mc9_sweep(const rbgs_grid *g, double *u, const double *f,
                   int32_t nsweeps, int32_t kernel, void *workspace,
                   size_t workspace_bytes, void *stream);

/* ||r||_2 and ||r||_2/||b||_2 (HOST pointers, may be NULL), FP64, fixed
 * reduction order.  Synchronises `stream`. */
int rbgs_mc9_residual(const rbgs_grid *g, const double *u, const double *f,
                      double *abs_norm, double *rel_norm, void *workspace,
                      size_t workspace_bytes, void *stream);

/* Sweeps until rel <= rel_tol (checked before the first sweep and after
 * every check_every sweeps; rel_tol <= 0: exactly max_sweeps sweeps), as
 * rbgs_solve, with the rounds captured in a HIP graph (PLAIN) or one
 * flag-driven launch per round (RESIDENT); kernel as for rbgs_mc9_sweep.  info (HOST, may be NULL): sweeps, rel_residual,
 * abs_residual, status (outer_iters = 0).  Returns RBGS_OK, RBGS_ENOCONV,
 * RBGS_ENONFINITE or an error.  Synchronises `stream`. */
int rbgs_mc9_solve(const rbgs_grid *g, double *u, const double *f,
                   int32_t max_sweeps, double rel_tol, int32_t check_every,
                   int32_t kernel, rbgs_solve_info *info, void *workspace,
                   size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------
 * Red-black Gauss-Seidel in three dimensions (an extension: the
 * conclusion, Section 5, names higher dimensions as future work).  Poisson's
 * equation on the unit cube with the 7-point Laplacian (six neighbours - 6
 * u) / h^2; red points have i + j + k even; one sweep is red then black,
 * each point by u = (((((u[i+1] + u[i-1]) + u[j+1]) + u[j-1]) + u[k+1])
 * + u[k-1] - (h h) f) / 6 (no FMA): bitwise the CPU definition.  FP64 only.
 * u, f: DEVICE arrays of (n+2) planes (index i) of (n+2) rows (index j) of
 * ld >= n+2 elements (index k), element (i, j, k) at (i (n+2) + j) ld + k;
 * the ring (any index 0 or n+1) of u is the Dirichlet data.  1 <= n <= 4094
 * (memory bounds it far lower: 1023^3 FP64 is 8.6 GB per array).  The
 * residual is r = f - lap(u), b = r with the interior of u set to zero.
 * --------------------------------------------------------------------- */

/* Workspace bytes (split u and f, reduction space); 0 for an invalid grid. */
size_t rbgs_rb3_workspace_size(const rbgs_grid *g);

/* nsweeps sweeps of u in place, one launch per half-sweep.  Asynchronous
 * on `stream`. */
int rbgs_rb3_sweep(const rbgs_grid *g, double *u, const double *f,
                   int32_t nsweeps, void *workspace, size_t workspace_bytes,
                   void *stream);

/* ||r||_2 and ||r||_2/||b||_2 (HOST pointers, may be NULL), FP64, fixed
 * reduction order.  Synchronises `stream`. */
int rbgs_rb3_residual(const rbgs_grid *g, const double *u, const double *f,
                      double *abs_norm, double *rel_norm, void *workspace,
                      size_t workspace_bytes, void *stream);

/* Sweeps until rel <= rel_tol, as rbgs_mc9_solve (graph-captured rounds;
 * rel_tol <= 0: exactly max_sweeps sweeps).  Synchronises `stream`. */
int rbgs_rb3_solve(const rbgs_grid *g, double *u, const double *f,
                   int32_t max_sweeps, double rel_tol, int32_t check_every,
                   rbgs_solve_info *info, void *workspace,
                   size_t workspace_bytes, void *stream);

/* Kernel choice for the 3D calls (zero-initialise; NULL = all zero).
 * kernel: RBGS_KERNEL_AUTO or RBGS_KERNEL_PLAIN = one launch per half-sweep
 * (a device-wide barrier between colours, Algorithm 1's structure);
 * RBGS_KERNEL_RESIDENT = the flag-driven form, the dependency rule of
 * Algorithm 2 (Section 2.3) carried to 3D: all half-sweeps of a call in one
 * cooperative launch of co-resident one-wave workgroups, the interior cut
 * into blocks whose half-sweep h waits only until the block and its six
 * face neighbours have completed h half-sweeps (a counter per block), so
 * colours and sweeps overlap instead of waiting at barriers; same result,
 * bit for bit.  RBGS_KERNEL_BLOCKED: RBGS_EUNSUPPORTED (no temporally
 * blocked 3D kernel).  The debug fields apply to RESIDENT only. */
typedef struct {
    int32_t kernel;
    int32_t debug_delay;       /* > 0: pseudo-random stall of up to debug_delay
                                  sleeps per block and half-sweep (schedule
                                  stress); results must not change            */
    int32_t debug_spin_limit;  /* > 0: polls per dependency wait before the
                                  call fails with RBGS_ETIMEOUT; 0 = 2^22      */
    int32_t debug_stall_block; /* b + 1 > 0: block b never publishes its
                                  progress, so the waits on it expire and the
                                  call returns RBGS_ETIMEOUT (watchdog test;
                                  every wave still exits); at most the block
                                  count, else RBGS_EINVAL                     */
} rbgs_rb3_opts;

/* rbgs_rb3_sweep with a kernel choice.  With RESIDENT the call reads the
 * kernel's error word at the end and so synchronises `stream`; on
 * RBGS_ETIMEOUT u holds a partly swept iterate.  nsweeps <= 2^29. */
int rbgs_rb3_sweep_ex(const rbgs_grid *g, double *u, const double *f,
                      int32_t nsweeps, const rbgs_rb3_opts *opts,
                      void *workspace, size_t workspace_bytes, void *stream);

/* rbgs_rb3_solve with a kernel choice.  RESIDENT runs each group of
 * check_every sweeps as one launch (host-driven rounds, no graph); same
 * sweeps, residuals and result as the plain kernel. */
int rbgs_rb3_solve_ex(const rbgs_grid *g, double *u, const double *f,
                      int32_t max_sweeps, double rel_tol, int32_t check_every,
                      const rbgs_rb3_opts *opts, rbgs_solve_info *info,
                      void *workspace, size_t workspace_bytes, void *stream);

/* Device-memory bandwidth probe: the copy (kind 0: b = a) and triad
 * (kind 1: a = b + s*c) kernels of the STREAM benchmark, which the paper
 * uses for the attainable memory bandwidth in its roofline (Section 3,
 * Eq. (2)).  a, b, c: DEVICE arrays of n_elems FP64 values, 16-byte
 * aligned, n_elems even and > 0 (c unused for copy).  Asynchronous on
 * `stream`; time it with events around the call. */
int rbgs_stream_probe(int32_t kind, double *a, double *b, double *c,
                      int64_t n_elems, double s, void *stream);

/* Human-readable name of a status code (static string; the codes are the
 * library's, not the paper's).  Unknown codes give "unknown rbgs status". */
const char *rbgs_strerror(int status);

/* Message describing the calling thread's last failure (static per thread). */
const char *rbgs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RBGS_H */
