// Host side of librbgs.so: argument validation, workspace carving, kernel
// dispatch and the solve drivers.  The public contract is include/rbgs.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <functional>
#include <vector>
#include <cstdio>
#include <cstring>
#include <string>

#include "rbgs.h"
#include "rbgs_internal.h"
#include "rbgs_blocked.h"
#include "rbgs_resident.h"

using namespace rbgs;

namespace {

thread_local std::string g_last_error = "no error";

int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(RBGS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t _e = (expr);                      \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

constexpr int kMaxN = 65533;  // n + 2 rows must fit a grid dimension

bool valid_grid(const rbgs_grid* g, std::string* why) {
    if (!g) { *why = "grid is NULL"; return false; }
    if (g->n < 1 || g->n > kMaxN) { *why = "n must be in [1, 65533]"; return false; }
    if (g->ld < int64_t(g->n) + 2) { *why = "ld must be >= n + 2"; return false; }
    if (!(g->h > 0.0) || !std::isfinite(g->h)) { *why = "h must be finite and > 0"; return false; }
    return true;
}

size_t elem_size(rbgs_dtype dt) { return dt == RBGS_F64 ? 8 : 4; }
bool valid_dtype(int dt) { return dt == RBGS_F64 || dt == RBGS_F32; }

// The device allocation that contains [p, p + bytes) must exist.
int check_device_range(const void* p, size_t bytes, const char* name) {
    if (!p) return fail(RBGS_EINVAL, std::string(name) + " is NULL");
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof attr);
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RBGS_EINVAL, std::string(name) + " is not a device pointer");
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(RBGS_EINVAL, std::string(name) + " is not device memory");
    void* base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(reinterpret_cast<hipDeviceptr_t*>(&base), &size,
                              const_cast<void*>(p));
    if (e == hipSuccess && base) {
        size_t off = size_t(static_cast<const char*>(p) - static_cast<const char*>(base));
        if (off + bytes > size)
            return fail(RBGS_EINVAL, std::string(name) + " allocation is smaller than the grid");
    } else {
        (void)hipGetLastError();
    }
    return RBGS_OK;
}

size_t grid_bytes(const rbgs_grid* g, rbgs_dtype dt) {
    return (size_t(g->n + 1) * size_t(g->ld) + size_t(g->n) + 2) * elem_size(dt);
}

// Workspace carving.  All pieces 256-byte aligned.
struct Workspace {
    int64_t pitch = 0;      // split pitch of the storage type
    int64_t pitch32 = 0;    // split pitch of FP32 refinement arrays
    void* u_red = nullptr;
    void* u_black = nullptr;
    void* u2_red = nullptr;   // second buffer of the persistent kernel's ping-pong
    void* u2_black = nullptr;
    void* f_red = nullptr;
    void* f_black = nullptr;
    double* partials = nullptr;
    double* sums = nullptr;  // 2 doubles: sum r^2, sum b^2
    float* e_red = nullptr;  // refinement: correction and its right-hand side
    float* e_black = nullptr;
    float* r_red = nullptr;
    float* r_black = nullptr;
    float* e2_red = nullptr;  // second buffer for blocked inner sweeps
    float* e2_black = nullptr;
    void* blocked = nullptr;  // persistent-kernel state (flags, ticket, error word)
    size_t blocked_bytes = 0;
    void* resident = nullptr;  // resident-kernel state (error word, band flags, exchange rows)
    size_t resident_bytes = 0;
    size_t total = 0;
};

bool is_ir(const rbgs_solve_opts* o) {
    return o && (o->precision == RBGS_PREC_F32_IR || o->precision == RBGS_PREC_BF16RHS_IR);
}

Workspace plan_workspace(const rbgs_grid* g, rbgs_dtype dt, bool ir, char* base) {
    Workspace w;
    const int n = g->n;
    const size_t es = elem_size(dt);
    w.pitch = split_pitch(n, es);
    const size_t colour = align256(size_t(n + 2) * size_t(w.pitch) * es);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align256(bytes);
        return static_cast<void*>(p);
    };
    w.u_red = take(colour);
    w.u_black = take(colour);
    w.u2_red = take(colour);
    w.u2_black = take(colour);
    w.f_red = take(colour);
    w.f_black = take(colour);
    int slots = residual_partial_slots(n, w.pitch, es);
    int nslots = residual_natural_partial_slots(n);
    if (nslots > slots) slots = nslots;
    w.partials = static_cast<double*>(take(size_t(slots) * 2 * sizeof(double)));
    w.sums = static_cast<double*>(take(256));
    w.blocked_bytes = blocked_state_bytes(n, dt == RBGS_F64 ? 8 : 4);
    w.blocked = take(w.blocked_bytes);
    w.resident_bytes = resident::state_bytes(n, es);
    if (w.resident_bytes) w.resident = take(w.resident_bytes);
    if (ir) {
        w.pitch32 = split_pitch(n, 4);
        const size_t c32 = align256(size_t(n + 2) * size_t(w.pitch32) * 4);
        w.e_red = static_cast<float*>(take(c32));
        w.e_black = static_cast<float*>(take(c32));
        w.r_red = static_cast<float*>(take(c32));
        w.r_black = static_cast<float*>(take(c32));
        w.e2_red = static_cast<float*>(take(c32));
        w.e2_black = static_cast<float*>(take(c32));
    }
    w.total = off;
    return w;
}

int check_workspace(void* ws, size_t ws_bytes, size_t need) {
    if (!ws) return fail(RBGS_EWORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return fail(RBGS_EWORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(RBGS_EWORKSPACE, "workspace too small: need " + std::to_string(need) +
                                         " bytes, got " + std::to_string(ws_bytes));
    return check_device_range(ws, need, "workspace");
}

int validate_sweep_opts(const rbgs_sweep_opts* o) {
    if (!o) return RBGS_OK;
    if (o->kernel < RBGS_KERNEL_AUTO || o->kernel > RBGS_KERNEL_RESIDENT)
        return fail(RBGS_EINVAL, "unknown kernel");
    if (o->fuse < 0 || o->tile_rows < 0 || o->tile_cols < 0 || o->rows_per_block < 0 ||
        o->debug_delay < 0 || o->debug_spin_limit < 0 || o->debug_stall_tile < 0)
        return fail(RBGS_EINVAL, "sweep options must be >= 0");
    if (o->rows_per_block > 4096) return fail(RBGS_EINVAL, "rows_per_block must be <= 4096");
    if (o->debug_delay > 1000) return fail(RBGS_EINVAL, "debug_delay must be <= 1000");
    int rc = validate_blocked_opts(o->fuse, o->tile_rows, o->tile_cols, &g_last_error);
    if (rc != RBGS_OK) return rc;
    if ((rc = validate_blocked_debug(o, &g_last_error)) != RBGS_OK) return rc;
    if (o->debug_trace)
        return check_device_range(o->debug_trace, size_t(o->debug_trace_items) * 32, "debug_trace");
    return RBGS_OK;
}

struct EventTimer {
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool on = false;
    hipError_t init(bool enable) {
        on = enable;
        if (!on) return hipSuccess;
        for (auto& e : ev) {
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    }
    hipError_t mark(int k, hipStream_t s) { return on ? hipEventRecord(ev[k], s) : hipSuccess; }
    ~EventTimer() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// Times the persistent launches alone (the blocked kernel's passes or the
// resident kernel), accumulated over the sweep groups of a call.
struct PersistentTimer {
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool on = false, armed = false;
    float ms = 0.f;
    int launches = 0, passes = 0, fuse = 0;
    hipError_t init(bool enable) {
        on = enable;
        if (!on) return hipSuccess;
        for (auto& e : ev) {
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    }
    // after a group whose events were recorded: add their interval
    hipError_t collect() {
        if (!on || !armed) return hipSuccess;
        armed = false;
        hipError_t e = hipEventSynchronize(ev[1]);
        if (e != hipSuccess) return e;
        float t = 0.f;
        e = hipEventElapsedTime(&t, ev[0], ev[1]);
        ms += t;
        return e;
    }
    void fill(rbgs_timing* t) const {
        t->persistent_ms = ms;
        t->persistent_launches = launches;
        t->passes = passes;
        t->fuse = fuse;
    }
    ~PersistentTimer() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// Accumulates the time of sweep groups inside a solve (events on the stream;
// every group is followed by a synchronising residual fetch).
struct GroupTimer {
    EventTimer t;
    rbgs_timing acc{};
    hipError_t begin(hipStream_t s) { return t.mark(1, s); }
    hipError_t end(hipStream_t s) { return t.mark(2, s); }
    hipError_t collect(int launches) {
        if (!t.on) return hipSuccess;
        hipError_t e = hipEventSynchronize(t.ev[2]);
        if (e != hipSuccess) return e;
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, t.ev[1], t.ev[2]);
        acc.sweep_ms += ms;
        acc.sweep_launches += launches;
        return e;
    }
};

// Half-sweeps on the split arrays already in the workspace.  *err_state is
// set to the state of the persistent kernel that ran (blocked or resident),
// whose error word must be checked.
template <typename T>
int run_sweeps(const rbgs_grid* g, const Workspace& w, int32_t nsweeps, const rbgs_sweep_opts* o,
               hipStream_t s, int* launches, void** err_state, PersistentTimer* pt,
               const int* stop = nullptr, double omega = 1.0, int start = 0) {
    const int n = g->n;
    const T h2 = T(g->h * g->h);
    T* ur = static_cast<T*>(w.u_red);
    T* ub = static_cast<T*>(w.u_black);
    const T* fr = static_cast<const T*>(w.f_red);
    const T* fb = static_cast<const T*>(w.f_black);
    int kernel = o ? o->kernel : RBGS_KERNEL_AUTO;
    if (kernel == RBGS_KERNEL_AUTO) kernel = auto_kernel(n, sizeof(T), nsweeps);
    *launches = 0;
    if (start != 0 && kernel != RBGS_KERNEL_BLOCKED)
        return fail(RBGS_EINVAL, "internal: only the blocked kernel starts in the second buffer");
    if (kernel == RBGS_KERNEL_BLOCKED) {
        BlockedParams bp = blocked_params(n, sizeof(T), o);
        bp.stop = stop;
        bp.keep_error = stop != nullptr;
        // start = 1: the caller packed u into the second buffer, so that an
        // odd number of passes ends in the first without a copy back
        T* const u2r = static_cast<T*>(w.u2_red);
        T* const u2b = static_cast<T*>(w.u2_black);
        T* const bred[2] = {start ? u2r : ur, start ? ur : u2r};
        T* const bblack[2] = {start ? u2b : ub, start ? ub : u2b};
        const bool timed = pt && pt->on;
        int plaunches = 0, passes = 0, depth = 0;
        HIP_TRY(run_blocked<T>(bred, bblack, fr, fb, n, w.pitch, h2, nsweeps, bp, w.blocked,
                               w.blocked_bytes, s, launches, timed ? pt->ev[0] : nullptr,
                               timed ? pt->ev[1] : nullptr, &plaunches, &passes, &depth,
                               T(omega), start != 0),
                "blocked sweep");
        if (timed && plaunches > 0) {
            pt->armed = true;
            pt->launches += plaunches;
            pt->passes += passes;
            pt->fuse = depth;
        }
        *err_state = w.blocked;
        return RBGS_OK;
    }
    if (kernel == RBGS_KERNEL_RESIDENT) {
        if (n > resident::max_n<T>() || !w.resident)
            return fail(RBGS_EUNSUPPORTED, "the resident kernel takes n <= " +
                                               std::to_string(resident::max_n<T>()) +
                                               " for this precision");
        if (resident::bands_for(n) > resident::max_resident_bands<T>(n))
            return fail(RBGS_EUNSUPPORTED, "the resident kernel's bands do not fit on the device");
        const int spin = (o && o->debug_spin_limit > 0) ? o->debug_spin_limit : (1 << 22);
        const bool timed = pt && pt->on && nsweeps > 0;
        if (timed) HIP_TRY(hipEventRecord(pt->ev[0], s), "event record");
        HIP_TRY(resident::run<T>(ur, ub, fr, fb, n, w.pitch, h2, nsweeps, spin,
                                 o ? o->debug_delay : 0, o ? o->debug_stall_tile : 0, w.resident,
                                 s, stop, stop != nullptr, T(omega)),
                "resident sweep");
        if (timed) {
            HIP_TRY(hipEventRecord(pt->ev[1], s), "event record");
            pt->armed = true;
            pt->launches += 1;
        }
        *launches = nsweeps > 0 ? 1 : 0;
        *err_state = w.resident;
        return RBGS_OK;
    }
    const int rows = o ? o->rows_per_block : 0;
    for (int32_t it = 0; it < nsweeps; ++it) {
        HIP_TRY(launch_half_sweep<T>(ur, ub, fr, n, w.pitch, h2, 0, rows, s, stop, T(omega)),
                "red half-sweep");
        HIP_TRY(launch_half_sweep<T>(ub, ur, fb, n, w.pitch, h2, 1, rows, s, stop, T(omega)),
                "black half-sweep");
        *launches += 2;
    }
    return RBGS_OK;
}

int run_sweeps_dt(rbgs_dtype dt, const rbgs_grid* g, const Workspace& w, int32_t nsweeps,
                  const rbgs_sweep_opts* o, hipStream_t s, int* launches, void** err_state,
                  PersistentTimer* pt, const int* stop = nullptr, double omega = 1.0,
                  int start = 0) {
    return dt == RBGS_F64
               ? run_sweeps<double>(g, w, nsweeps, o, s, launches, err_state, pt, stop, omega, start)
               : run_sweeps<float>(g, w, nsweeps, o, s, launches, err_state, pt, stop, omega, start);
}

// Where a call that sweeps nsweeps times straight after packing should pack
// u: the second buffer (1) when the persistent kernel will run an odd number
// of passes, whose result then lands in the first buffer with no copy back;
// else the first (0).
int pack_buffer(const rbgs_grid* g, rbgs_dtype dt, int32_t nsweeps, const rbgs_sweep_opts* o) {
    int kernel = o ? o->kernel : RBGS_KERNEL_AUTO;
    if (kernel == RBGS_KERNEL_AUTO) kernel = auto_kernel(g->n, elem_size(dt), nsweeps);
    if (kernel != RBGS_KERNEL_BLOCKED) return 0;
    return blocked_pass_parity(g->n, elem_size(dt), nsweeps, o);
}

// Reads the two device sums, synchronising the stream.
int fetch_norms(const Workspace& w, hipStream_t s, double* abs_norm, double* rel_norm) {
    double host[2] = {0.0, 0.0};
    HIP_TRY(hipMemcpyAsync(host, w.sums, sizeof host, hipMemcpyDeviceToHost, s), "norm copy");
    HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
    double rn = std::sqrt(host[0]);
    double bn = std::sqrt(host[1]);
    if (abs_norm) *abs_norm = rn;
    if (rel_norm) *rel_norm = bn > 0.0 ? rn / bn : rn;
    return RBGS_OK;
}

// The graph rounds' device state: {converged flag, rounds, overflow flag,
// stall flag, previous rel (double)}, 64 bytes after the residual sums.
int* round_state(const Workspace& w) {
    return reinterpret_cast<int*>(reinterpret_cast<char*>(w.sums) + 64);
}

template <typename T>
int split_residual(const rbgs_grid* g, const Workspace& w, hipStream_t s, float* r_red,
                   float* r_black, int rhs_bf16, int* overflow = nullptr, void* nat = nullptr) {
    HIP_TRY(launch_residual_split<T>(static_cast<const T*>(w.u_red),
                                     static_cast<const T*>(w.u_black),
                                     static_cast<const T*>(w.f_red),
                                     static_cast<const T*>(w.f_black), g->n, w.pitch,
                                     1.0 / (g->h * g->h), w.partials, w.sums, r_red, r_black,
                                     w.pitch32, rhs_bf16, s, overflow, static_cast<T*>(nat),
                                     g->ld),
            "residual");
    return RBGS_OK;
}

// nat (optional): the caller's natural u, unpacked in the same pass.
int split_residual_dt(rbgs_dtype dt, const rbgs_grid* g, const Workspace& w, hipStream_t s,
                      void* nat = nullptr) {
    return dt == RBGS_F64 ? split_residual<double>(g, w, s, nullptr, nullptr, 0, nullptr, nat)
                          : split_residual<float>(g, w, s, nullptr, nullptr, 0, nullptr, nat);
}

// The residual-cadence loop of a solve, run as a captured graph: one round
// is k sweeps, the FP64 residual and a device-side test that raises a
// converged flag (rel <= rel_tol, rel not finite, or `cap` rounds done); the
// sweep kernels of later rounds see the flag and do nothing, so the iterate
// and the sweep count are those of the host loop.  The host launches a few
// rounds at a time and reads the flag once per batch.  *used = false when
// the graph could not be built (e.g. a launch that cannot be captured); the
// caller then runs the host loop.  *rounds_done: rounds whose sweeps ran.
// body(stream, stop, &err_state) enqueues one round's work up to and
// including the residual (sums in w.sums); the judge follows it.
using RoundBody = std::function<int(hipStream_t, const int*, void**)>;

// Rounds of more launches than this are not captured (a graph holds one
// node per launch); the caller's launch-by-launch loop runs them instead.
constexpr int64_t kGraphMaxLaunchesPerRound = int64_t(1) << 16;

// watch, first_check, prev_rel: a refinement with the precision fallback
// (launch_judge); *flags (optional) receives the overflow and stall flags.
int solve_rounds_graph(const Workspace& w, const RoundBody& body_fn, int cap, double rel_tol,
                       hipStream_t s, void** err_state, int* rounds_done, bool* used,
                       int64_t launches_per_round, int watch = 0, int first_check = 0,
                       double prev_rel = 0.0, int* flags = nullptr) {
    *used = false;
    *rounds_done = 0;
    if (launches_per_round > kGraphMaxLaunchesPerRound) return RBGS_OK;
    int* state = round_state(w);
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto cleanup = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cs) (void)hipStreamDestroy(cs);
    };
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return RBGS_OK;
    }
    void* es = nullptr;
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        const std::string saved = g_last_error;
        bool body = body_fn(cs, state, &es) == RBGS_OK;
        body = body && launch_judge(w.sums, rel_tol, state, cap, cs, watch, first_check,
                                    prev_rel) == hipSuccess;
        const bool ended = hipStreamEndCapture(cs, &graph) == hipSuccess;
        ok = body && ended &&
             hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (!ok) g_last_error = saved;  // a launch that cannot be captured is not a failure
    }
    if (!ok) {
        (void)hipGetLastError();
        cleanup();
        return RBGS_OK;
    }
    *used = true;
    *err_state = es;
    // the error word of a persistent kernel is cleared once here, not per round
    hipError_t e = launch_zero(state, 16, s);
    if (e == hipSuccess && es) e = launch_zero(static_cast<char*>(es) + 64, 4, s);
    const int per_poll = cap < 4 ? cap : 4;
    int host[4] = {0, 0, 0, 0};
    while (e == hipSuccess) {
        for (int r = 0; r < per_poll && e == hipSuccess; ++r) e = hipGraphLaunch(exec, s);
        if (e == hipSuccess) e = hipMemcpyAsync(host, state, sizeof host, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess || host[0] != 0) break;
        if (es) {  // a timed-out dependency wait ends the solve at once
            int err = 0;
            e = hipMemcpyAsync(&err, static_cast<char*>(es) + 64, sizeof err,
                               hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e == hipSuccess && err != 0) break;
        }
    }
    cleanup();
    if (e != hipSuccess) return fail(RBGS_EHIP, std::string("solve graph: ") + hipGetErrorString(e));
    *rounds_done = host[1];
    if (flags) {
        flags[0] = host[2];
        flags[1] = host[3];
    }
    return RBGS_OK;
}


// Shared argument checks of the grid transfers: coarse/fine sizes related by
// n_f = 2 n_c + 1, strides covering a grid, and device ranges that hold all
// `batch` grids of each level.
int check_transfer(int32_t batch, rbgs_dtype dt, const rbgs_grid* coarse, const void* xc,
                   int64_t cstride, const rbgs_grid* fine, const void* xf, int64_t fstride) {
    std::string why;
    if (batch < 1) return fail(RBGS_EINVAL, "batch must be >= 1");
    if (!valid_dtype(dt)) return fail(RBGS_EINVAL, "unknown dtype");
    if (!valid_grid(coarse, &why)) return fail(RBGS_EINVAL, "coarse: " + why);
    if (!valid_grid(fine, &why)) return fail(RBGS_EINVAL, "fine: " + why);
    if (int64_t(fine->n) != 2 * int64_t(coarse->n) + 1)
        return fail(RBGS_EINVAL, "fine n must be 2 * coarse n + 1");
    const int64_t cext = int64_t(coarse->n + 2) * coarse->ld;
    const int64_t fext = int64_t(fine->n + 2) * fine->ld;
    if (cstride < cext || fstride < fext)
        return fail(RBGS_EINVAL, "grid stride must be >= (n + 2) * ld");
    const size_t es = elem_size(dt);
    int rc;
    if ((rc = check_device_range(xc, (size_t(batch - 1) * size_t(cstride) + size_t(cext)) * es,
                                 "coarse array")))
        return rc;
    if ((rc = check_device_range(xf, (size_t(batch - 1) * size_t(fstride) + size_t(fext)) * es,
                                 "fine array")))
        return rc;
    return RBGS_OK;
}

// ----- multigrid (red-black Gauss-Seidel as the smoother) ----------------

constexpr int kMgMaxLevels = 32;

// Level sizes n_0 = n, n_{l+1} = (n_l - 1) / 2 while n_l is odd and >= 3
// (and fewer than max_levels levels when max_levels > 0).
int mg_level_sizes(int n, int max_levels, int* sizes) {
    int cnt = 1, m = n;
    sizes[0] = m;
    while (m >= 3 && (m & 1) && cnt < kMgMaxLevels && (max_levels == 0 || cnt < max_levels)) {
        m = (m - 1) / 2;
        sizes[cnt++] = m;
    }
    return cnt;
}

// One Workspace per level, back to back: level 0 holds the caller's grid
// (packed), the others the coarse iterate and right-hand side; h doubles
// from level to level (exactly, a power-of-two scaling).
struct MgPlan {
    int levels = 0;
    rbgs_grid g[kMgMaxLevels];
    Workspace w[kMgMaxLevels];
    size_t total = 0;
};

MgPlan plan_mg(const rbgs_grid* g, int max_levels, char* base) {
    MgPlan p;
    int sizes[kMgMaxLevels];
    p.levels = mg_level_sizes(g->n, max_levels, sizes);
    size_t off = 0;
    double h = g->h;
    for (int l = 0; l < p.levels; ++l) {
        p.g[l] = l == 0 ? *g : rbgs_grid{sizes[l], int64_t(sizes[l]) + 2, h};
        p.w[l] = plan_workspace(&p.g[l], RBGS_F64, false, base ? base + off : nullptr);
        off += p.w[l].total;
        h = 2.0 * h;
    }
    p.total = off;
    return p;
}

int mg_default_coarse_sweeps(int nc) { return nc == 1 ? 1 : 2 * (nc + 1) * (nc + 1); }

struct MgParams {
    int nu1, nu2, coarse_sweeps;
    rbgs_sweep_opts sweep;
};

// Enqueues one V-cycle from level l down; *states collects the persistent
// kernels' state blocks whose error words must be checked.
// Launches one V-cycle enqueues (an upper bound: the plain smoother's two
// per sweep), for the decision to capture the cycles as a graph.
int64_t mg_launches_per_cycle(const MgPlan& p, const MgParams& mp) {
    int64_t total = 0;
    for (int l = 0; l < p.levels; ++l) {
        if (p.g[l].n <= kMgCoarseN && p.levels - l <= kMgMaxCoarseLevels) return total + 1;
        if (l == p.levels - 1) return total + 2 * int64_t(mp.coarse_sweeps);
        total += 2 * (int64_t(mp.nu1) + mp.nu2) + 2;
    }
    return total;
}

int mg_cycle(const MgPlan& p, int l, const MgParams& mp, hipStream_t s, const int* stop,
             std::vector<void*>* states) {
    const Workspace& a = p.w[l];
    if (p.g[l].n <= kMgCoarseN && p.levels - l <= kMgMaxCoarseLevels) {
        // this level and all below: one workgroup, one launch
        MgCoarseLevels lv;
        lv.count = p.levels - l;
        for (int k = 0; k < lv.count; ++k) {
            const Workspace& wk = p.w[l + k];
            const double h = p.g[l + k].h;
            lv.level[k] = MgCoarseLevel{static_cast<double*>(wk.u_red),
                                        static_cast<double*>(wk.u_black),
                                        static_cast<double*>(wk.f_red),
                                        static_cast<double*>(wk.f_black), wk.pitch, p.g[l + k].n,
                                        h * h, 1.0 / (h * h)};
        }
        HIP_TRY(launch_mg_coarse_vcycle(lv, mp.nu1, mp.nu2, mp.coarse_sweeps, stop, s),
                "multigrid coarse cycle");
        return RBGS_OK;
    }
    auto smooth = [&](int k) -> int {
        if (k <= 0) return RBGS_OK;
        int launches = 0;
        void* es = nullptr;
        int rc = run_sweeps<double>(&p.g[l], a, k, &mp.sweep, s, &launches, &es, nullptr, stop);
        if (rc) return rc;
        if (es && std::find(states->begin(), states->end(), es) == states->end())
            states->push_back(es);
        return RBGS_OK;
    };
    if (l == p.levels - 1) return smooth(mp.coarse_sweeps);
    int rc = smooth(mp.nu1);
    if (rc) return rc;
    const Workspace& c = p.w[l + 1];
    const double hl = p.g[l].h;
    HIP_TRY(launch_mg_restrict(static_cast<const double*>(a.u_red),
                               static_cast<const double*>(a.u_black),
                               static_cast<const double*>(a.f_red),
                               static_cast<const double*>(a.f_black), a.pitch, 1.0 / (hl * hl),
                               static_cast<double*>(c.f_red), static_cast<double*>(c.f_black),
                               static_cast<double*>(c.u_red), static_cast<double*>(c.u_black),
                               p.g[l + 1].n, c.pitch, stop, s),
            "multigrid restriction");
    if ((rc = mg_cycle(p, l + 1, mp, s, stop, states))) return rc;
    if (mp.nu2 >= 1) {
        // the first post-smoothing sweep: interpolant fused into its red
        // half, then its black half; the other nu2 - 1 sweeps as usual
        const double h2 = hl * hl;
        HIP_TRY(launch_mg_prolong_red(static_cast<double*>(a.u_red),
                                      static_cast<const double*>(a.u_black),
                                      static_cast<const double*>(a.f_red), a.pitch, p.g[l].n, h2,
                                      static_cast<const double*>(c.u_red),
                                      static_cast<const double*>(c.u_black), c.pitch, stop, s),
                "multigrid prolongation");
        HIP_TRY(launch_half_sweep<double>(static_cast<double*>(a.u_black),
                                          static_cast<const double*>(a.u_red),
                                          static_cast<const double*>(a.f_black), p.g[l].n,
                                          a.pitch, h2, 1, 0, s, stop),
                "black half-sweep");
        return smooth(mp.nu2 - 1);
    }
    HIP_TRY(launch_mg_prolong_add(static_cast<double*>(a.u_red), static_cast<double*>(a.u_black),
                                  a.pitch, p.g[l].n, static_cast<const double*>(c.u_red),
                                  static_cast<const double*>(c.u_black), c.pitch, stop, s),
            "multigrid prolongation");
    return smooth(mp.nu2);
}

// ----- four-colour Gauss-Seidel for the 9-point Laplacian -----------------

struct Mc9Workspace {
    double* u[4] = {nullptr, nullptr, nullptr, nullptr};
    double* f[4] = {nullptr, nullptr, nullptr, nullptr};
    double* partials = nullptr;
    double* sums = nullptr;  // sum r^2, sum b^2; the graph rounds' state at +64 bytes
    int* state = nullptr;    // flag-driven form: error word, ticket at +32 ints, block
                             // counters from +64 ints
    size_t total = 0;
};

Mc9Workspace plan_mc9(const rbgs_grid* g, char* base) {
    Mc9Workspace w;
    const size_t colour = align256(size_t(mc9_rows(g->n)) * size_t(mc9_pitch(g->n)) * 8);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align256(bytes);
        return reinterpret_cast<double*>(p);
    };
    for (auto& c : w.u) c = take(colour);
    for (auto& c : w.f) c = take(colour);
    w.partials = take(size_t(mc9_residual_blocks(g->n)) * 2 * sizeof(double));
    w.sums = take(256);
    w.state = reinterpret_cast<int*>(take(256 + size_t(kMc9MaxBlocks) * sizeof(int)));
    w.total = off;
    return w;
}

// Four-colour kernel choice: AUTO or PLAIN (a launch per colour), RESIDENT
// (the flag-driven form, one launch for all quarter-sweeps); no temporally
// blocked form.
int mc9_check_kernel(int kernel) {
    if (kernel == RBGS_KERNEL_BLOCKED)
        return fail(RBGS_EUNSUPPORTED, "the 9-point sweep has no temporally blocked kernel: use "
                                       "PLAIN or RESIDENT (the flag-driven form)");
    if (kernel < RBGS_KERNEL_AUTO || kernel > RBGS_KERNEL_RESIDENT)
        return fail(RBGS_EINVAL, "unknown kernel");
    return RBGS_OK;
}

// nsweeps sweeps as flag-driven launches (the caller cleared the error
// word): one launch unless the ticket count would leave the int range.
int mc9_sweeps_flags(const rbgs_grid* g, const Mc9Workspace& w, int nsweeps, int capacity,
                     hipStream_t s) {
    const int nb = mc9_flags_blocks(g->n, capacity);
    const int per_launch = int(((int64_t(1) << 30) / nb) / 4);  // levels x nb < 2^31
    for (int done = 0; done < nsweeps;) {
        const int k = std::min(nsweeps - done, per_launch);
        HIP_TRY(launch_zero(w.state + 32, size_t(32 + nb) * sizeof(int), s),
                "clear ticket and block counters");
        HIP_TRY(launch_mc9_flags(w.u, w.f, g->n, 6.0 * (g->h * g->h), 4 * k, capacity,
                                 w.state + 32, w.state + 64, w.state, 1 << 22, 0, 0, s),
                "9-point flag-driven sweeps");
        done += k;
    }
    return RBGS_OK;
}

int mc9_flags_error(const Mc9Workspace& w, hipStream_t s) {
    int err = 0;
    HIP_TRY(hipMemcpyAsync(&err, w.state, sizeof err, hipMemcpyDeviceToHost, s), "read error word");
    HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
    if (err) return fail(RBGS_ETIMEOUT, "a block dependency wait of the 9-point flag-driven sweep "
                                        "timed out");
    return RBGS_OK;
}

int mc9_flags_setup(const Mc9Workspace& w, hipStream_t s, int* capacity) {
    *capacity = mc9_flags_capacity();
    if (*capacity < 64) return fail(RBGS_EHIP, "occupancy query for the 9-point flag-driven kernel");
    HIP_TRY(launch_zero(w.state, 256, s), "clear error word");
    return RBGS_OK;
}

int mc9_prepare(const rbgs_grid* g, const void* u, const void* f, void* ws, size_t ws_bytes,
                Mc9Workspace* w) {
    std::string why;
    if (!valid_grid(g, &why)) return fail(RBGS_EINVAL, why);
    Mc9Workspace plan = plan_mc9(g, nullptr);
    int rc;
    if ((rc = check_workspace(ws, ws_bytes, plan.total))) return rc;
    if ((rc = check_device_range(u, grid_bytes(g, RBGS_F64), "u"))) return rc;
    if ((rc = check_device_range(f, grid_bytes(g, RBGS_F64), "f"))) return rc;
    *w = plan_mc9(g, static_cast<char*>(ws));
    return RBGS_OK;
}

int mc9_sweeps(const rbgs_grid* g, const Mc9Workspace& w, int nsweeps, hipStream_t s,
               const int* stop) {
    const double c6 = 6.0 * (g->h * g->h);
    for (int it = 0; it < nsweeps; ++it)
        for (int colour = 0; colour < 4; ++colour)
            HIP_TRY(launch_mc9_quarter(w.u, w.f, g->n, c6, colour, stop, s), "quarter-sweep");
    return RBGS_OK;
}

int mc9_residual_sums(const rbgs_grid* g, const Mc9Workspace& w, hipStream_t s) {
    HIP_TRY(launch_mc9_residual(w.u, w.f, g->n, 1.0 / (6.0 * (g->h * g->h)), w.partials, w.sums, s),
            "9-point residual");
    return RBGS_OK;
}

int mc9_fetch(const Mc9Workspace& w, hipStream_t s, double* abs_norm, double* rel_norm) {
    Workspace v;
    v.sums = w.sums;
    return fetch_norms(v, s, abs_norm, rel_norm);
}

// ----- red-black Gauss-Seidel in 3D -----------------------------------------

constexpr int kMaxN3 = 4094;  // (n+2) planes and rows must fit the grid's y and z

struct Rb3Workspace {
    int64_t pitch = 0;
    double* u_red = nullptr;
    double* u_black = nullptr;
    double* f_red = nullptr;
    double* f_black = nullptr;
    double* partials = nullptr;
    double* sums = nullptr;  // sum r^2, sum b^2; the graph rounds' state at +64 bytes
    int* state = nullptr;    // flag-driven form: error word, ticket at +32 ints, block
                             // counters from +64 ints
    size_t total = 0;
};

bool valid_grid3(const rbgs_grid* g, std::string* why) {
    if (!g) { *why = "grid is NULL"; return false; }
    if (g->n < 1 || g->n > kMaxN3) { *why = "3D n must be in [1, 4094]"; return false; }
    if (g->ld < int64_t(g->n) + 2) { *why = "ld must be >= n + 2"; return false; }
    if (!(g->h > 0.0) || !std::isfinite(g->h)) { *why = "h must be finite and > 0"; return false; }
    return true;
}

size_t grid3_bytes(const rbgs_grid* g) {
    return size_t(g->n + 2) * size_t(g->n + 2) * size_t(g->ld) * sizeof(double);
}

Rb3Workspace plan_rb3(const rbgs_grid* g, char* base) {
    Rb3Workspace w;
    w.pitch = split_pitch(g->n, 8);
    const size_t colour = align256(size_t(g->n + 2) * size_t(g->n + 2) * size_t(w.pitch) * 8);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align256(bytes);
        return reinterpret_cast<double*>(p);
    };
    w.u_red = take(colour);
    w.u_black = take(colour);
    w.f_red = take(colour);
    w.f_black = take(colour);
    w.partials = take(size_t(rb3_residual_blocks(g->n)) * 2 * sizeof(double));
    w.sums = take(256);
    w.state = reinterpret_cast<int*>(take(256 + size_t(kRb3MaxBlocks) * sizeof(int)));
    w.total = off;
    return w;
}

int rb3_prepare(const rbgs_grid* g, const void* u, const void* f, void* ws, size_t ws_bytes,
                Rb3Workspace* w) {
    std::string why;
    if (!valid_grid3(g, &why)) return fail(RBGS_EINVAL, why);
    Rb3Workspace plan = plan_rb3(g, nullptr);
    int rc;
    if ((rc = check_workspace(ws, ws_bytes, plan.total))) return rc;
    if ((rc = check_device_range(u, grid3_bytes(g), "u"))) return rc;
    if ((rc = check_device_range(f, grid3_bytes(g), "f"))) return rc;
    *w = plan_rb3(g, static_cast<char*>(ws));
    return RBGS_OK;
}

int rb3_pack_both(const rbgs_grid* g, const Rb3Workspace& w, const double* u, const double* f,
                  hipStream_t s) {
    HIP_TRY(launch_rb3_pack(u, g->ld, w.u_red, w.u_black, g->n, w.pitch, s), "pack u");
    HIP_TRY(launch_rb3_pack(f, g->ld, w.f_red, w.f_black, g->n, w.pitch, s), "pack f");
    return RBGS_OK;
}

int rb3_sweeps(const rbgs_grid* g, const Rb3Workspace& w, int nsweeps, hipStream_t s,
               const int* stop) {
    const double h2 = g->h * g->h;
    for (int it = 0; it < nsweeps; ++it) {
        HIP_TRY(launch_rb3_half(w.u_red, w.u_black, w.f_red, g->n, w.pitch, h2, 0, stop, s),
                "red half-sweep");
        HIP_TRY(launch_rb3_half(w.u_black, w.u_red, w.f_black, g->n, w.pitch, h2, 1, stop, s),
                "black half-sweep");
    }
    return RBGS_OK;
}

// Options of the 3D calls: plain (one launch per half-sweep) or the
// flag-driven form (kernel RESIDENT).
int rb3_check_opts(const rbgs_rb3_opts* o) {
    if (!o) return RBGS_OK;
    if (o->kernel == RBGS_KERNEL_BLOCKED)
        return fail(RBGS_EUNSUPPORTED, "3D sweeps have no temporally blocked kernel: use PLAIN or "
                                       "RESIDENT (the flag-driven form)");
    if (o->kernel < RBGS_KERNEL_AUTO || o->kernel > RBGS_KERNEL_RESIDENT)
        return fail(RBGS_EINVAL, "unknown kernel");
    if (o->debug_delay < 0 || o->debug_spin_limit < 0 || o->debug_stall_block < 0)
        return fail(RBGS_EINVAL, "debug options must be >= 0");
    return RBGS_OK;
}

bool rb3_flag_driven(const rbgs_rb3_opts* o) { return o && o->kernel == RBGS_KERNEL_RESIDENT; }

// nsweeps sweeps as flag-driven launches (the caller cleared the error
// word once for the call): one launch unless the ticket count would leave
// the int range, each starting from zeroed ticket and block counters.
int rb3_sweeps_flags(const rbgs_grid* g, const Rb3Workspace& w, int nsweeps,
                     const rbgs_rb3_opts* o, int capacity, hipStream_t s) {
    const int nb = rb3_flags_blocks(g->n, capacity);
    const int per_launch = int(((int64_t(1) << 30) / nb) / 2);  // sweeps, so levels x nb < 2^31
    for (int done = 0; done < nsweeps;) {
        const int k = std::min(nsweeps - done, per_launch);
        HIP_TRY(launch_zero(w.state + 32, size_t(32 + nb) * sizeof(int), s),
                "clear ticket and block counters");
        HIP_TRY(launch_rb3_flags(w.u_red, w.u_black, w.f_red, w.f_black, g->n, w.pitch,
                                 g->h * g->h, 2 * k, capacity, w.state + 32, w.state + 64,
                                 w.state, o->debug_spin_limit > 0 ? o->debug_spin_limit : (1 << 22),
                                 o->debug_delay, o->debug_stall_block, nullptr, s),
                "3D flag-driven sweeps");
        done += k;
    }
    return RBGS_OK;
}

int rb3_flags_error(const Rb3Workspace& w, hipStream_t s) {
    int err = 0;
    HIP_TRY(hipMemcpyAsync(&err, w.state, sizeof err, hipMemcpyDeviceToHost, s), "read error word");
    HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
    if (err) return fail(RBGS_ETIMEOUT, "a block dependency wait of the 3D flag-driven sweep "
                                        "timed out");
    return RBGS_OK;
}

int rb3_flags_setup(const rbgs_grid* g, const rbgs_rb3_opts* o, const Rb3Workspace& w,
                    hipStream_t s, int* capacity) {
    *capacity = rb3_flags_capacity(g->n);
    if (*capacity < 64) return fail(RBGS_EHIP, "occupancy query for the 3D flag-driven kernel");
    if (o->debug_stall_block > rb3_flags_blocks(g->n, *capacity))
        return fail(RBGS_EINVAL, "debug_stall_block beyond the block count");
    HIP_TRY(launch_zero(w.state, 256, s), "clear error word");
    return RBGS_OK;
}

int rb3_residual_sums(const rbgs_grid* g, const Rb3Workspace& w, hipStream_t s) {
    HIP_TRY(launch_rb3_residual(w.u_red, w.u_black, w.f_red, w.f_black, g->n, w.pitch,
                                1.0 / (g->h * g->h), w.partials, w.sums, s),
            "3D residual");
    return RBGS_OK;
}

}  // namespace

extern "C" {

const char* rbgs_strerror(int status) {
    switch (status) {
        case RBGS_OK: return "RBGS_OK";
        case RBGS_EINVAL: return "RBGS_EINVAL: invalid argument";
        case RBGS_EHIP: return "RBGS_EHIP: HIP runtime error";
        case RBGS_ENOCONV: return "RBGS_ENOCONV: tolerance not reached";
        case RBGS_ETIMEOUT: return "RBGS_ETIMEOUT: dependency wait timed out";
        case RBGS_ENONFINITE: return "RBGS_ENONFINITE: non-finite residual";
        case RBGS_EUNSUPPORTED: return "RBGS_EUNSUPPORTED: unsupported option";
        case RBGS_EWORKSPACE: return "RBGS_EWORKSPACE: bad workspace";
        case RBGS_EORDER: return "RBGS_EORDER: dependency stamp check failed";
        default: return "unknown rbgs status";
    }
}

const char* rbgs_last_error(void) { return g_last_error.c_str(); }

size_t rbgs_workspace_size(const rbgs_grid* g, rbgs_dtype dt, const rbgs_solve_opts* opts) {
    std::string why;
    if (!valid_grid(g, &why) || !valid_dtype(dt)) return 0;
    return plan_workspace(g, dt, is_ir(opts) && dt == RBGS_F64, nullptr).total;
}

int64_t rbgs_split_pitch(const rbgs_grid* g, rbgs_dtype dt) {
    std::string why;
    if (!valid_grid(g, &why) || !valid_dtype(dt)) return 0;
    return split_pitch(g->n, elem_size(dt));
}

int rbgs_pack(const rbgs_grid* g, rbgs_dtype dt, const void* nat, void* red, void* black,
              void* stream) {
    std::string why;
    if (!valid_grid(g, &why)) return fail(RBGS_EINVAL, why);
    if (!valid_dtype(dt)) return fail(RBGS_EINVAL, "unknown dtype");
    const int64_t pitch = split_pitch(g->n, elem_size(dt));
    const size_t colour = size_t(g->n + 2) * size_t(pitch) * elem_size(dt);
    int rc;
    if ((rc = check_device_range(nat, grid_bytes(g, dt), "natural array"))) return rc;
    if ((rc = check_device_range(red, colour, "red array"))) return rc;
    if ((rc = check_device_range(black, colour, "black array"))) return rc;
    HIP_TRY(launch_pack(nat, g->ld, red, black, g->n, pitch, int(elem_size(dt)),
                        static_cast<hipStream_t>(stream)),
            "pack");
    return RBGS_OK;
}

int rbgs_unpack(const rbgs_grid* g, rbgs_dtype dt, void* nat, const void* red, const void* black,
                void* stream) {
    std::string why;
    if (!valid_grid(g, &why)) return fail(RBGS_EINVAL, why);
    if (!valid_dtype(dt)) return fail(RBGS_EINVAL, "unknown dtype");
    const int64_t pitch = split_pitch(g->n, elem_size(dt));
    const size_t colour = size_t(g->n + 2) * size_t(pitch) * elem_size(dt);
    int rc;
    if ((rc = check_device_range(nat, grid_bytes(g, dt), "natural array"))) return rc;
    if ((rc = check_device_range(red, colour, "red array"))) return rc;
    if ((rc = check_device_range(black, colour, "black array"))) return rc;
    HIP_TRY(launch_unpack(nat, g->ld, red, black, g->n, pitch, int(elem_size(dt)),
                          static_cast<hipStream_t>(stream)),
            "unpack");
    return RBGS_OK;
}

int rbgs_sweep_split(const rbgs_grid* g, rbgs_dtype dt, void* u_red, void* u_black,
                     const void* f_red, const void* f_black, int32_t nsweeps,
                     const rbgs_sweep_opts* opts, void* workspace, size_t workspace_bytes,
                     void* stream) {
    std::string why;
    if (!valid_grid(g, &why)) return fail(RBGS_EINVAL, why);
    if (!valid_dtype(dt)) return fail(RBGS_EINVAL, "unknown dtype");
    if (nsweeps < 0) return fail(RBGS_EINVAL, "nsweeps must be >= 0");
    int rc = validate_sweep_opts(opts);
    if (rc) return fail(rc, g_last_error);
    if (opts && opts->timing) return fail(RBGS_EUNSUPPORTED, "the split-layout sweep takes no timing");
    Workspace plan = plan_workspace(g, dt, false, nullptr);
    if ((rc = check_workspace(workspace, workspace_bytes, plan.total))) return rc;
    const size_t colour = size_t(g->n + 2) * size_t(plan.pitch) * elem_size(dt);
    if ((rc = check_device_range(u_red, colour, "u_red"))) return rc;
    if ((rc = check_device_range(u_black, colour, "u_black"))) return rc;
    if ((rc = check_device_range(f_red, colour, "f_red"))) return rc;
    if ((rc = check_device_range(f_black, colour, "f_black"))) return rc;
    if (nsweeps == 0) return RBGS_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the caller's colour arrays take the place of the packed copies; the
    // workspace still holds the persistent kernels' second buffer and state
    Workspace w = plan_workspace(g, dt, false, static_cast<char*>(workspace));
    w.u_red = u_red;
    w.u_black = u_black;
    w.f_red = const_cast<void*>(f_red);
    w.f_black = const_cast<void*>(f_black);
    int launches = 0;
    void* err_state = nullptr;
    if ((rc = run_sweeps_dt(dt, g, w, nsweeps, opts, s, &launches, &err_state, nullptr))) return rc;
    if (err_state) return blocked_check_error(err_state, s, &g_last_error);
    return RBGS_OK;
}

int rbgs_sweep(const rbgs_grid* g, rbgs_dtype dt, void* u, const void* f, int32_t nsweeps,
               const rbgs_sweep_opts* opts, void* workspace, size_t workspace_bytes,
               void* stream) {
    std::string why;
    if (!valid_grid(g, &why)) return fail(RBGS_EINVAL, why);
    if (!valid_dtype(dt)) return fail(RBGS_EINVAL, "unknown dtype");
    if (nsweeps < 0) return fail(RBGS_EINVAL, "nsweeps must be >= 0");
    int rc = validate_sweep_opts(opts);
    if (rc) return fail(rc, g_last_error);
    Workspace plan = plan_workspace(g, dt, false, nullptr);
    if ((rc = check_workspace(workspace, workspace_bytes, plan.total))) return rc;
    if ((rc = check_device_range(u, grid_bytes(g, dt), "u"))) return rc;
    if ((rc = check_device_range(f, grid_bytes(g, dt), "f"))) return rc;
    if (nsweeps == 0) {
        if (opts && opts->timing) *opts->timing = rbgs_timing{};
        return RBGS_OK;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace w = plan_workspace(g, dt, false, static_cast<char*>(workspace));
    const int es = int(elem_size(dt));
    EventTimer tm;
    HIP_TRY(tm.init(opts && opts->timing), "event create");
    PersistentTimer pt;
    HIP_TRY(pt.init(opts && opts->timing), "event create");
    const int start = pack_buffer(g, dt, nsweeps, opts);
    HIP_TRY(tm.mark(0, s), "event record");
    HIP_TRY(launch_pack(u, g->ld, start ? w.u2_red : w.u_red, start ? w.u2_black : w.u_black, g->n,
                        w.pitch, es, s),
            "pack u");
    HIP_TRY(launch_pack(f, g->ld, w.f_red, w.f_black, g->n, w.pitch, es, s), "pack f");
    HIP_TRY(tm.mark(1, s), "event record");
    int launches = 0;
    void* err_state = nullptr;
    if ((rc = run_sweeps_dt(dt, g, w, nsweeps, opts, s, &launches, &err_state, &pt, nullptr, 1.0,
                            start)))
        return rc;
    HIP_TRY(tm.mark(2, s), "event record");
    HIP_TRY(launch_unpack(u, g->ld, w.u_red, w.u_black, g->n, w.pitch, es, s), "unpack u");
    HIP_TRY(tm.mark(3, s), "event record");
    if (tm.on) {
        HIP_TRY(hipEventSynchronize(tm.ev[3]), "event synchronise");
        rbgs_timing t{};
        t.sweep_launches = launches;
        HIP_TRY(hipEventElapsedTime(&t.pack_ms, tm.ev[0], tm.ev[1]), "event time");
        HIP_TRY(hipEventElapsedTime(&t.sweep_ms, tm.ev[1], tm.ev[2]), "event time");
        HIP_TRY(hipEventElapsedTime(&t.unpack_ms, tm.ev[2], tm.ev[3]), "event time");
        HIP_TRY(pt.collect(), "event time");
        pt.fill(&t);
        *opts->timing = t;
    }
    return err_state ? blocked_check_error(err_state, s, &g_last_error) : RBGS_OK;
}

int rbgs_residual(const rbgs_grid* g, rbgs_dtype dt, const void* u, const void* f,
                  double* abs_norm, double* rel_norm, void* workspace, size_t workspace_bytes,
                  void* stream) {
    std::string why;
    if (!valid_grid(g, &why)) return fail(RBGS_EINVAL, why);
    if (!valid_dtype(dt)) return fail(RBGS_EINVAL, "unknown dtype");
    Workspace plan = plan_workspace(g, dt, false, nullptr);
    int rc;
    if ((rc = check_workspace(workspace, workspace_bytes, plan.total))) return rc;
    if ((rc = check_device_range(u, grid_bytes(g, dt), "u"))) return rc;
    if ((rc = check_device_range(f, grid_bytes(g, dt), "f"))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace w = plan_workspace(g, dt, false, static_cast<char*>(workspace));
    const double inv_h2 = 1.0 / (g->h * g->h);
    if (dt == RBGS_F64)
        HIP_TRY(launch_residual_natural<double>(static_cast<const double*>(u),
                                                static_cast<const double*>(f), g->n, g->ld,
                                                inv_h2, w.partials, w.sums, s),
                "residual");
    else
        HIP_TRY(launch_residual_natural<float>(static_cast<const float*>(u),
                                               static_cast<const float*>(f), g->n, g->ld, inv_h2,
                                               w.partials, w.sums, s),
                "residual");
    return fetch_norms(w, s, abs_norm, rel_norm);
}

int rbgs_residual_noalloc(const rbgs_grid* g, rbgs_dtype dt, const void* u, const void* f,
                          double* abs_norm, double* rel_norm, void* stream) {
    std::string why;
    if (!valid_grid(g, &why)) return fail(RBGS_EINVAL, why);
    if (!valid_dtype(dt)) return fail(RBGS_EINVAL, "unknown dtype");
    const size_t need = residual_noalloc_bytes(g->n);
    if (need > kStaticScratchBytes)
        return fail(RBGS_EINVAL, "grid too large for the static scratch of rbgs_residual_noalloc (" +
                                     std::to_string(need) + " bytes needed, " +
                                     std::to_string(kStaticScratchBytes) + " available)");
    int rc;
    if ((rc = check_device_range(u, grid_bytes(g, dt), "u"))) return rc;
    if ((rc = check_device_range(f, grid_bytes(g, dt), "f"))) return rc;
    void* base = nullptr;
    HIP_TRY(static_scratch(&base), "static scratch address");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* sums = static_cast<double*>(base);
    double* partials = reinterpret_cast<double*>(static_cast<char*>(base) + 256);
    const double inv_h2 = 1.0 / (g->h * g->h);
    if (dt == RBGS_F64)
        HIP_TRY(launch_residual_natural<double>(static_cast<const double*>(u),
                                                static_cast<const double*>(f), g->n, g->ld,
                                                inv_h2, partials, sums, s),
                "residual");
    else
        HIP_TRY(launch_residual_natural<float>(static_cast<const float*>(u),
                                               static_cast<const float*>(f), g->n, g->ld, inv_h2,
                                               partials, sums, s),
                "residual");
    Workspace w;
    w.sums = sums;
    return fetch_norms(w, s, abs_norm, rel_norm);
}

int rbgs_solve(const rbgs_grid* g, rbgs_dtype dt, void* u, const void* f,
               const rbgs_solve_opts* o, rbgs_solve_info* info, void* workspace,
               size_t workspace_bytes, void* stream) {
    std::string why;
    if (!valid_grid(g, &why)) return fail(RBGS_EINVAL, why);
    if (!valid_dtype(dt)) return fail(RBGS_EINVAL, "unknown dtype");
    if (!o) return fail(RBGS_EINVAL, "solve options are NULL");
    if (o->max_sweeps < 0) return fail(RBGS_EINVAL, "max_sweeps must be >= 0");
    if (o->check_every < 1) return fail(RBGS_EINVAL, "check_every must be >= 1");
    if (std::isnan(o->rel_tol)) return fail(RBGS_EINVAL, "rel_tol is NaN");
    if (o->precision < RBGS_PREC_F64 || o->precision > RBGS_PREC_BF16RHS_IR)
        return fail(RBGS_EINVAL, "unknown precision");
    if (o->inner_sweeps < 0) return fail(RBGS_EINVAL, "inner_sweeps must be >= 0");
    if (o->fallback != 0 && o->fallback != 1) return fail(RBGS_EINVAL, "fallback must be 0 or 1");
    const bool ir = is_ir(o);
    // omega: 1 = Gauss-Seidel; (0, 2) = red-black SOR; 0 = the model
    // problem's optimum 2 / (1 + sin(pi h)) for this grid's h
    const double omega = o->omega == 0.0 ? 2.0 / (1.0 + std::sin(M_PI * g->h)) : o->omega;
    if (omega != 1.0) {
        if (!(omega > 0.0 && omega < 2.0))
            return fail(RBGS_EINVAL, "omega must be in (0, 2), or 0 for the optimum");
        if (dt != RBGS_F64 || ir)
            return fail(RBGS_EUNSUPPORTED, "SOR (omega != 1) runs in FP64 without refinement");
        if (o->sweep.debug_tile_order != 0 || o->sweep.debug_stamp_check != 0 ||
            o->sweep.debug_trace != nullptr)
            return fail(RBGS_EUNSUPPORTED, "SOR (omega != 1) runs without the verification modes");
    }
    if (ir && dt != RBGS_F64)
        return fail(RBGS_EINVAL, "refinement modes need FP64 storage of u and f");
    int rc = validate_sweep_opts(&o->sweep);
    if (rc) return rc;
    Workspace plan = plan_workspace(g, dt, ir, nullptr);
    if ((rc = check_workspace(workspace, workspace_bytes, plan.total))) return rc;
    if ((rc = check_device_range(u, grid_bytes(g, dt), "u"))) return rc;
    if ((rc = check_device_range(f, grid_bytes(g, dt), "f"))) return rc;

    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace w = plan_workspace(g, dt, ir, static_cast<char*>(workspace));
    const int es = int(elem_size(dt));
    GroupTimer gt;
    HIP_TRY(gt.t.init(o->sweep.timing != nullptr), "event create");
    PersistentTimer pt;
    HIP_TRY(pt.init(o->sweep.timing != nullptr), "event create");
    // Timing never waits for the device on its own: every interval is read
    // after a synchronisation the solve makes anyway (a residual readback or
    // the final one), so a timed solve keeps the GPU as busy as an untimed one.
    // a fixed sweep count (no refinement) packs u where its sweeps end
    const int start = (!ir && o->rel_tol <= 0.0) ? pack_buffer(g, dt, o->max_sweeps, &o->sweep) : 0;
    HIP_TRY(gt.t.mark(0, s), "event record");
    HIP_TRY(launch_pack(u, g->ld, start ? w.u2_red : w.u_red, start ? w.u2_black : w.u_black, g->n,
                        w.pitch, es, s),
            "pack u");
    HIP_TRY(launch_pack(f, g->ld, w.f_red, w.f_black, g->n, w.pitch, es, s), "pack f");
    HIP_TRY(gt.t.mark(3, s), "event record");

    rbgs_solve_info out{0, 0, 0.0, 0.0, RBGS_OK, RBGS_PREC_F64};
    int launches = 0;
    void* err_state = nullptr;
    rbgs_sweep_opts sw = o->sweep;
    sw.timing = nullptr;
    // a fixed sweep count reads its norms back only after the unpack is
    // enqueued (one synchronisation for the whole call)
    bool norms_pending = false;
    int pending_launches = 0;
    if (!ir) {
        double rel = 0.0, ab = 0.0;
        int32_t done = 0;
        if (o->rel_tol <= 0.0) {
            HIP_TRY(gt.begin(s), "event record");
            if ((rc = run_sweeps_dt(dt, g, w, o->max_sweeps, &sw, s, &launches, &err_state, &pt,
                                    nullptr, omega, start)))
                return rc;
            HIP_TRY(gt.end(s), "event record");
            done = o->max_sweeps;
            // the last read of u: its residual and its unpack in one pass
            if ((rc = split_residual_dt(dt, g, w, s, u))) return rc;
            norms_pending = true;
            pending_launches = launches;
        } else {
            if ((rc = split_residual_dt(dt, g, w, s))) return rc;
            if ((rc = fetch_norms(w, s, &ab, &rel))) return rc;
            const int cap = o->max_sweeps / o->check_every;
            if (!gt.t.on && !(rel <= o->rel_tol) && std::isfinite(rel) && cap > 0) {
                // whole rounds as a captured graph; the sweeps beyond the last
                // whole round (if still needed) in the host loop below
                int rounds = 0;
                bool used = false;
                const int k = o->check_every;
                RoundBody body = [&](hipStream_t cs, const int* stop, void** es) -> int {
                    int l = 0;
                    int r = run_sweeps_dt(dt, g, w, k, &sw, cs, &l, es, nullptr, stop, omega);
                    return r ? r : split_residual_dt(dt, g, w, cs);
                };
                if ((rc = solve_rounds_graph(w, body, cap, o->rel_tol, s, &err_state, &rounds,
                                             &used, 2 * int64_t(k) + 3)))
                    return rc;
                if (used) {
                    done = rounds * o->check_every;
                    if ((rc = fetch_norms(w, s, &ab, &rel))) return rc;
                    if (err_state && (rc = blocked_check_error(err_state, s, &g_last_error)))
                        return rc;
                }
            }
            while (!(rel <= o->rel_tol) && done < o->max_sweeps && std::isfinite(rel)) {
                int32_t k = o->max_sweeps - done < o->check_every ? o->max_sweeps - done
                                                                  : o->check_every;
                HIP_TRY(gt.begin(s), "event record");
                if ((rc = run_sweeps_dt(dt, g, w, k, &sw, s, &launches, &err_state, &pt, nullptr,
                                        omega)))
                    return rc;
                HIP_TRY(gt.end(s), "event record");
                done += k;
                if ((rc = split_residual_dt(dt, g, w, s))) return rc;
                if ((rc = fetch_norms(w, s, &ab, &rel))) return rc;
                HIP_TRY(gt.collect(launches), "event time");
                HIP_TRY(pt.collect(), "event time");
                if (err_state && (rc = blocked_check_error(err_state, s, &g_last_error)))
                    return rc;
            }
        }
        out.sweeps = done;
        out.rel_residual = rel;
        out.abs_residual = ab;
        if (!std::isfinite(rel))
            out.status = RBGS_ENONFINITE;
        else
            out.status = (o->rel_tol <= 0.0 || rel <= o->rel_tol) ? RBGS_OK : RBGS_ENOCONV;
    } else {
        // Iterative refinement: FP64 residual and correction, FP32 inner
        // sweeps (bfloat16 right-hand side in the BF16RHS mode).  With
        // opts.fallback the inner precision widens when it stops helping: a
        // value of r that its format cannot hold switches to FP64 sweeps at
        // once; an outer step after the first that leaves rel no lower turns
        // a bfloat16 right-hand side into FP32, and FP32 inner sweeps into
        // FP64 sweeps of u (inner_sweeps at a time, residual after each).
        const int inner = o->inner_sweeps > 0 ? o->inner_sweeps : o->check_every;
        const bool fb = o->fallback != 0;
        int prec = o->precision;
        Workspace inner_w = w;  // FP32 view: e is the iterate, r the right-hand side
        inner_w.pitch = w.pitch32;
        inner_w.u_red = w.e_red;
        inner_w.u_black = w.e_black;
        inner_w.f_red = w.r_red;
        inner_w.f_black = w.r_black;
        inner_w.u2_red = w.e2_red;
        inner_w.u2_black = w.e2_black;
        const size_t c32 = align256(size_t(g->n + 2) * size_t(w.pitch32) * 4);
        rbgs_grid gi = *g;
        double rel = 0.0, ab = 0.0;
        int32_t done = 0, outer = 0;
        int* state = round_state(w);
        int* ovf = fb ? state + 2 : nullptr;  // set by the residual kernel
        if (fb) HIP_TRY(launch_zero(state, 16, s), "zero flags");
        // the overflow flag of the last residual (0 without the fallback)
        auto overflowed = [&](int* flag) -> int {
            *flag = 0;
            if (!fb) return RBGS_OK;
            HIP_TRY(hipMemcpyAsync(flag, ovf, sizeof *flag, hipMemcpyDeviceToHost, s), "flag copy");
            HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
            return RBGS_OK;
        };
        // r rounded to the current right-hand-side format, rel, and the switch
        // to FP64 sweeps when a value does not fit
        auto residual_now = [&]() -> int {
            int r = split_residual<double>(g, w, s, w.r_red, w.r_black,
                                           prec == RBGS_PREC_BF16RHS_IR, ovf);
            if (r || (r = fetch_norms(w, s, &ab, &rel))) return r;
            int flag = 0;
            if ((r = overflowed(&flag))) return r;
            if (flag) prec = RBGS_PREC_F64;
            return RBGS_OK;
        };
        // after an outer step from rel `before`: widen on a stall
        auto after_step = [&](double before) -> int {
            int flag = 0;
            int r = overflowed(&flag);
            if (r) return r;
            if (flag) {
                prec = RBGS_PREC_F64;
            } else if (fb && outer >= 2 && rel >= before) {
                prec = prec == RBGS_PREC_BF16RHS_IR ? RBGS_PREC_F32_IR : RBGS_PREC_F64;
                if (prec == RBGS_PREC_F32_IR) return residual_now();
            }
            return RBGS_OK;
        };
        if ((rc = residual_now())) return rc;
        while (!(rel <= o->rel_tol) && done < o->max_sweeps && std::isfinite(rel)) {
            const int32_t k = o->max_sweeps - done < inner ? o->max_sweeps - done : inner;
            if (prec == RBGS_PREC_F64) {  // after a fallback: FP64 sweeps of u
                HIP_TRY(gt.begin(s), "event record");
                if ((rc = run_sweeps<double>(g, w, k, &sw, s, &launches, &err_state, &pt))) return rc;
                HIP_TRY(gt.end(s), "event record");
                done += k;
                if ((rc = split_residual<double>(g, w, s, nullptr, nullptr, 0))) return rc;
                if ((rc = fetch_norms(w, s, &ab, &rel))) return rc;
                HIP_TRY(gt.collect(launches), "event time");
                HIP_TRY(pt.collect(), "event time");
                if (err_state && (rc = blocked_check_error(err_state, s, &g_last_error)))
                    return rc;
                continue;
            }
            const int bf16 = prec == RBGS_PREC_BF16RHS_IR;
            const int cap = (o->max_sweeps - done) / inner;
            if (!gt.t.on && cap > 0) {
                // whole outer steps as a captured graph (zero e, inner sweeps,
                // correction, residual with r for the next step, the judge)
                RoundBody body = [&, bf16](hipStream_t cs, const int* stop, void** es) -> int {
                    int l = 0;
                    HIP_TRY(launch_zero(w.e_red, c32, cs), "zero correction");
                    HIP_TRY(launch_zero(w.e_black, c32, cs), "zero correction");
                    int r = run_sweeps<float>(&gi, inner_w, inner, &sw, cs, &l, es, nullptr, stop);
                    if (r) return r;
                    HIP_TRY(launch_add_correction(static_cast<double*>(w.u_red),
                                                  static_cast<double*>(w.u_black), w.pitch,
                                                  w.e_red, w.e_black, w.pitch32, g->n, cs, stop),
                            "correction");
                    return split_residual<double>(g, w, cs, w.r_red, w.r_black, bf16, ovf);
                };
                int rounds = 0, flags[2] = {0, 0};
                bool used = false;
                if ((rc = solve_rounds_graph(w, body, cap, o->rel_tol, s, &err_state, &rounds,
                                             &used, 2 * int64_t(inner) + 6, fb ? 1 : 0,
                                             outer >= 1 ? 1 : 2, rel, flags)))
                    return rc;
                if (used) {
                    done += rounds * inner;
                    outer += rounds;
                    if ((rc = fetch_norms(w, s, &ab, &rel))) return rc;
                    if (err_state && (rc = blocked_check_error(err_state, s, &g_last_error)))
                        return rc;
                    if (flags[0]) {
                        prec = RBGS_PREC_F64;
                    } else if (flags[1]) {
                        prec = bf16 ? RBGS_PREC_F32_IR : RBGS_PREC_F64;
                        if (prec == RBGS_PREC_F32_IR && (rc = residual_now())) return rc;
                    }
                    continue;
                }
            }
            HIP_TRY(launch_zero(w.e_red, c32, s), "zero correction");
            HIP_TRY(launch_zero(w.e_black, c32, s), "zero correction");
            HIP_TRY(gt.begin(s), "event record");
            if ((rc = run_sweeps<float>(&gi, inner_w, k, &sw, s, &launches, &err_state, &pt))) return rc;
            HIP_TRY(gt.end(s), "event record");
            const int step_launches = launches;
            HIP_TRY(launch_add_correction(static_cast<double*>(w.u_red),
                                          static_cast<double*>(w.u_black), w.pitch, w.e_red,
                                          w.e_black, w.pitch32, g->n, s),
                    "correction");
            done += k;
            ++outer;
            const double before = rel;
            if ((rc = split_residual<double>(g, w, s, w.r_red, w.r_black, bf16, ovf))) return rc;
            if ((rc = fetch_norms(w, s, &ab, &rel))) return rc;
            HIP_TRY(gt.collect(step_launches), "event time");
            HIP_TRY(pt.collect(), "event time");
            if (err_state && (rc = blocked_check_error(err_state, s, &g_last_error)))
                return rc;
            if ((rc = after_step(before))) return rc;
        }
        out.sweeps = done;
        out.outer_iters = outer;
        out.rel_residual = rel;
        out.abs_residual = ab;
        out.precision = prec;
        if (!std::isfinite(rel))
            out.status = RBGS_ENONFINITE;
        else
            out.status = rel <= o->rel_tol ? RBGS_OK : RBGS_ENOCONV;
    }
    HIP_TRY(gt.t.mark(4, s), "event record");
    if (!norms_pending)  // a fixed count unpacked u with its residual
        HIP_TRY(launch_unpack(u, g->ld, w.u_red, w.u_black, g->n, w.pitch, es, s), "unpack u");
    HIP_TRY(gt.t.mark(5, s), "event record");
    if (norms_pending) {
        double rel = 0.0, ab = 0.0;
        if ((rc = fetch_norms(w, s, &ab, &rel))) return rc;
        HIP_TRY(gt.collect(pending_launches), "event time");
        HIP_TRY(pt.collect(), "event time");
        out.rel_residual = rel;
        out.abs_residual = ab;
        out.status = std::isfinite(rel) ? RBGS_OK : RBGS_ENONFINITE;
    }
    HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
    if (gt.t.on) {
        HIP_TRY(hipEventElapsedTime(&gt.acc.pack_ms, gt.t.ev[0], gt.t.ev[3]), "event time");
        HIP_TRY(hipEventElapsedTime(&gt.acc.unpack_ms, gt.t.ev[4], gt.t.ev[5]), "event time");
        pt.fill(&gt.acc);
        *o->sweep.timing = gt.acc;
    }
    if (err_state && (rc = blocked_check_error(err_state, s, &g_last_error))) out.status = rc;
    if (info) *info = out;
    if (out.status == RBGS_ENONFINITE) g_last_error = "residual is not finite";
    if (out.status == RBGS_ENOCONV) g_last_error = "tolerance not reached";
    return out.status;
}

size_t rbgs_mg_workspace_size(const rbgs_grid* g, rbgs_dtype dt, const rbgs_mg_opts* o) {
    std::string why;
    if (!valid_grid(g, &why) || dt != RBGS_F64) return 0;
    const int ml = o ? o->max_levels : 0;
    if (ml < 0) return 0;
    return plan_mg(g, ml, nullptr).total;
}

int rbgs_mg_solve(const rbgs_grid* g, rbgs_dtype dt, void* u, const void* f,
                  const rbgs_mg_opts* o, rbgs_mg_info* info, void* workspace,
                  size_t workspace_bytes, void* stream) {
    std::string why;
    if (!valid_grid(g, &why)) return fail(RBGS_EINVAL, why);
    if (!valid_dtype(dt)) return fail(RBGS_EINVAL, "unknown dtype");
    if (dt != RBGS_F64) return fail(RBGS_EUNSUPPORTED, "multigrid runs in FP64");
    if (!o) return fail(RBGS_EINVAL, "multigrid options are NULL");
    if (o->max_cycles < 0) return fail(RBGS_EINVAL, "max_cycles must be >= 0");
    if (std::isnan(o->rel_tol)) return fail(RBGS_EINVAL, "rel_tol is NaN");
    if (o->pre_sweeps < 0 || o->post_sweeps < 0)
        return fail(RBGS_EINVAL, "pre_sweeps and post_sweeps must be >= 0");
    if (int64_t(o->pre_sweeps) + o->post_sweeps < 1)
        return fail(RBGS_EINVAL, "pre_sweeps + post_sweeps must be >= 1");
    if (o->max_levels < 0) return fail(RBGS_EINVAL, "max_levels must be >= 0");
    if (o->coarse_sweeps < 0) return fail(RBGS_EINVAL, "coarse_sweeps must be >= 0");
    int rc = validate_sweep_opts(&o->sweep);
    if (rc) return rc;
    if (o->sweep.timing) return fail(RBGS_EUNSUPPORTED, "multigrid does not take sweep timing");
    MgPlan plan = plan_mg(g, o->max_levels, nullptr);
    if ((rc = check_workspace(workspace, workspace_bytes, plan.total))) return rc;
    if ((rc = check_device_range(u, grid_bytes(g, dt), "u"))) return rc;
    if ((rc = check_device_range(f, grid_bytes(g, dt), "f"))) return rc;

    hipStream_t s = static_cast<hipStream_t>(stream);
    MgPlan p = plan_mg(g, o->max_levels, static_cast<char*>(workspace));
    const Workspace& w0 = p.w[0];
    MgParams mp;
    mp.nu1 = o->pre_sweeps;
    mp.nu2 = o->post_sweeps;
    const int nL = p.g[p.levels - 1].n;
    mp.coarse_sweeps = o->coarse_sweeps > 0 ? o->coarse_sweeps : mg_default_coarse_sweeps(nL);
    mp.sweep = o->sweep;
    HIP_TRY(launch_pack(u, g->ld, w0.u_red, w0.u_black, g->n, w0.pitch, 8, s), "pack u");
    HIP_TRY(launch_pack(f, g->ld, w0.f_red, w0.f_black, g->n, w0.pitch, 8, s), "pack f");
    for (int l = 0; l < p.levels; ++l) {
        const Workspace& wl = p.w[l];
        if (l > 0) {  // coarse iterates: zero ring (and interior, rewritten per cycle)
            const size_t colour = align256(size_t(p.g[l].n + 2) * size_t(wl.pitch) * 8);
            HIP_TRY(launch_zero(wl.u_red, colour, s), "zero coarse iterate");
            HIP_TRY(launch_zero(wl.u_black, colour, s), "zero coarse iterate");
        }
        // persistent smoothers' error words start clear once per solve
        HIP_TRY(launch_zero(static_cast<char*>(wl.blocked) + 64, 4, s), "clear error word");
        if (wl.resident)
            HIP_TRY(launch_zero(static_cast<char*>(wl.resident) + 64, 4, s), "clear error word");
    }

    rbgs_mg_info out{0, p.levels, nL, mp.coarse_sweeps, 0.0, 0.0, 0, RBGS_OK};
    std::vector<void*> states;
    double rel = 0.0, ab = 0.0;
    int32_t cycles = 0;
    const bool fixed = o->rel_tol <= 0.0;  // exactly max_cycles cycles
    if (!fixed) {
        if ((rc = split_residual<double>(&p.g[0], w0, s, nullptr, nullptr, 0))) return rc;
        if ((rc = fetch_norms(w0, s, &ab, &rel))) return rc;
    }
    if ((fixed || (!(rel <= o->rel_tol) && std::isfinite(rel))) && o->max_cycles > 0) {
        RoundBody body = [&](hipStream_t cs, const int* stop, void** es) -> int {
            states.clear();
            int r = mg_cycle(p, 0, mp, cs, stop, &states);
            if (r) return r;
            *es = states.empty() ? nullptr : states[0];
            return split_residual<double>(&p.g[0], w0, cs, nullptr, nullptr, 0);
        };
        int rounds = 0;
        bool used = false;
        void* es = nullptr;
        if ((rc = solve_rounds_graph(w0, body, o->max_cycles, fixed ? -1.0 : o->rel_tol, s, &es,
                                     &rounds, &used, mg_launches_per_cycle(p, mp) + 3)))
            return rc;
        if (used) {
            out.graph = 1;
            cycles = rounds;
            if ((rc = fetch_norms(w0, s, &ab, &rel))) return rc;
        } else {
            states.clear();
            while (cycles < o->max_cycles && (fixed || (!(rel <= o->rel_tol) && std::isfinite(rel)))) {
                if ((rc = mg_cycle(p, 0, mp, s, nullptr, &states))) return rc;
                ++cycles;
                if (!fixed || cycles == o->max_cycles) {
                    if ((rc = split_residual<double>(&p.g[0], w0, s, nullptr, nullptr, 0)))
                        return rc;
                    if ((rc = fetch_norms(w0, s, &ab, &rel))) return rc;
                }
            }
        }
    } else if (fixed) {  // zero cycles: the residual of the start
        if ((rc = split_residual<double>(&p.g[0], w0, s, nullptr, nullptr, 0))) return rc;
        if ((rc = fetch_norms(w0, s, &ab, &rel))) return rc;
    }
    HIP_TRY(launch_unpack(u, g->ld, w0.u_red, w0.u_black, g->n, w0.pitch, 8, s), "unpack u");
    HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
    out.cycles = cycles;
    out.rel_residual = rel;
    out.abs_residual = ab;
    if (!std::isfinite(rel))
        out.status = RBGS_ENONFINITE;
    else
        out.status = (fixed || rel <= o->rel_tol) ? RBGS_OK : RBGS_ENOCONV;
    for (void* st : states)
        if ((rc = blocked_check_error(st, s, &g_last_error))) out.status = rc;
    if (info) *info = out;
    if (out.status == RBGS_ENONFINITE) g_last_error = "residual is not finite";
    if (out.status == RBGS_ENOCONV) g_last_error = "tolerance not reached";
    return out.status;
}

size_t rbgs_mc9_workspace_size(const rbgs_grid* g) {
    std::string why;
    if (!valid_grid(g, &why)) return 0;
    return plan_mc9(g, nullptr).total;
}

int rbgs_mc9_sweep(const rbgs_grid* g, double* u, const double* f, int32_t nsweeps,
                   int32_t kernel, void* workspace, size_t workspace_bytes, void* stream) {
    if (nsweeps < 0) return fail(RBGS_EINVAL, "nsweeps must be >= 0");
    if (kernel < RBGS_KERNEL_AUTO || kernel > RBGS_KERNEL_RESIDENT)
        return fail(RBGS_EINVAL, "unknown kernel");
    Mc9Workspace w;
    int rc = mc9_prepare(g, u, f, workspace, workspace_bytes, &w);
    if (rc) return rc;
    if ((rc = mc9_check_kernel(kernel))) return rc;
    if (nsweeps > (1 << 29)) return fail(RBGS_EINVAL, "nsweeps must be <= 2^29");
    if (nsweeps == 0) return RBGS_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool flags = kernel == RBGS_KERNEL_RESIDENT;
    int capacity = 0;
    if (flags && (rc = mc9_flags_setup(w, s, &capacity))) return rc;
    HIP_TRY(launch_mc9_pack(u, g->ld, w.u, g->n, s), "pack u");
    HIP_TRY(launch_mc9_pack(f, g->ld, w.f, g->n, s), "pack f");
    rc = flags ? mc9_sweeps_flags(g, w, nsweeps, capacity, s) : mc9_sweeps(g, w, nsweeps, s, nullptr);
    if (rc) return rc;
    HIP_TRY(launch_mc9_unpack(u, g->ld, w.u, g->n, s), "unpack u");
    return flags ? mc9_flags_error(w, s) : RBGS_OK;
}

int rbgs_mc9_residual(const rbgs_grid* g, const double* u, const double* f, double* abs_norm,
                      double* rel_norm, void* workspace, size_t workspace_bytes, void* stream) {
    Mc9Workspace w;
    int rc = mc9_prepare(g, u, f, workspace, workspace_bytes, &w);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(launch_mc9_pack(u, g->ld, w.u, g->n, s), "pack u");
    HIP_TRY(launch_mc9_pack(f, g->ld, w.f, g->n, s), "pack f");
    if ((rc = mc9_residual_sums(g, w, s))) return rc;
    return mc9_fetch(w, s, abs_norm, rel_norm);
}

int rbgs_mc9_solve(const rbgs_grid* g, double* u, const double* f, int32_t max_sweeps,
                   double rel_tol, int32_t check_every, int32_t kernel, rbgs_solve_info* info,
                   void* workspace, size_t workspace_bytes, void* stream) {
    if (max_sweeps < 0) return fail(RBGS_EINVAL, "max_sweeps must be >= 0");
    if (check_every < 1) return fail(RBGS_EINVAL, "check_every must be >= 1");
    if (std::isnan(rel_tol)) return fail(RBGS_EINVAL, "rel_tol is NaN");
    if (kernel < RBGS_KERNEL_AUTO || kernel > RBGS_KERNEL_RESIDENT)
        return fail(RBGS_EINVAL, "unknown kernel");
    Mc9Workspace w;
    int rc = mc9_prepare(g, u, f, workspace, workspace_bytes, &w);
    if (rc) return rc;
    if ((rc = mc9_check_kernel(kernel))) return rc;
    const bool flags = kernel == RBGS_KERNEL_RESIDENT;
    if (flags && max_sweeps > (1 << 29))
        return fail(RBGS_EINVAL, "the flag-driven form runs at most 2^29 sweeps per call");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int capacity = 0;
    if (flags && (rc = mc9_flags_setup(w, s, &capacity))) return rc;
    HIP_TRY(launch_mc9_pack(u, g->ld, w.u, g->n, s), "pack u");
    HIP_TRY(launch_mc9_pack(f, g->ld, w.f, g->n, s), "pack f");
    double rel = 0.0, ab = 0.0;
    int32_t done = 0;
    // k sweeps of the asked-for form; the flag-driven form checks its error
    // word after each group (one launch per group of sweeps)
    auto sweeps = [&](int k) -> int {
        if (!flags) return mc9_sweeps(g, w, k, s, nullptr);
        int r = mc9_sweeps_flags(g, w, k, capacity, s);
        return r ? r : mc9_flags_error(w, s);
    };
    if (rel_tol <= 0.0) {
        if ((rc = sweeps(max_sweeps))) return rc;
        done = max_sweeps;
        if ((rc = mc9_residual_sums(g, w, s))) return rc;
        if ((rc = mc9_fetch(w, s, &ab, &rel))) return rc;
    } else {
        if ((rc = mc9_residual_sums(g, w, s))) return rc;
        if ((rc = mc9_fetch(w, s, &ab, &rel))) return rc;
        const int cap = max_sweeps / check_every;
        if (!flags && !(rel <= rel_tol) && std::isfinite(rel) && cap > 0) {
            Workspace v;
            v.sums = w.sums;
            RoundBody body = [&](hipStream_t cs, const int* stop, void** es) -> int {
                *es = nullptr;
                int r = mc9_sweeps(g, w, check_every, cs, stop);
                return r ? r : mc9_residual_sums(g, w, cs);
            };
            int rounds = 0;
            bool used = false;
            void* es = nullptr;
            if ((rc = solve_rounds_graph(v, body, cap, rel_tol, s, &es, &rounds, &used,
                                         4 * int64_t(check_every) + 3)))
                return rc;
            if (used) {
                done = rounds * check_every;
                if ((rc = mc9_fetch(w, s, &ab, &rel))) return rc;
            }
        }
        while (!(rel <= rel_tol) && done < max_sweeps && std::isfinite(rel)) {
            const int32_t k = max_sweeps - done < check_every ? max_sweeps - done : check_every;
            if ((rc = sweeps(k))) return rc;
            done += k;
            if ((rc = mc9_residual_sums(g, w, s))) return rc;
            if ((rc = mc9_fetch(w, s, &ab, &rel))) return rc;
        }
    }
    HIP_TRY(launch_mc9_unpack(u, g->ld, w.u, g->n, s), "unpack u");
    HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
    rbgs_solve_info out{done, 0, rel, ab, RBGS_OK};
    if (!std::isfinite(rel))
        out.status = RBGS_ENONFINITE;
    else
        out.status = (rel_tol <= 0.0 || rel <= rel_tol) ? RBGS_OK : RBGS_ENOCONV;
    if (info) *info = out;
    if (out.status == RBGS_ENONFINITE) g_last_error = "residual is not finite";
    if (out.status == RBGS_ENOCONV) g_last_error = "tolerance not reached";
    return out.status;
}

size_t rbgs_rb3_workspace_size(const rbgs_grid* g) {
    std::string why;
    if (!valid_grid3(g, &why)) return 0;
    return plan_rb3(g, nullptr).total;
}

int rbgs_rb3_sweep(const rbgs_grid* g, double* u, const double* f, int32_t nsweeps,
                   void* workspace, size_t workspace_bytes, void* stream) {
    return rbgs_rb3_sweep_ex(g, u, f, nsweeps, nullptr, workspace, workspace_bytes, stream);
}

int rbgs_rb3_sweep_ex(const rbgs_grid* g, double* u, const double* f, int32_t nsweeps,
                      const rbgs_rb3_opts* opts, void* workspace, size_t workspace_bytes,
                      void* stream) {
    if (nsweeps < 0 || nsweeps > (1 << 29)) return fail(RBGS_EINVAL, "nsweeps must be in [0, 2^29]");
    int rc = rb3_check_opts(opts);
    if (rc) return rc;
    Rb3Workspace w;
    if ((rc = rb3_prepare(g, u, f, workspace, workspace_bytes, &w))) return rc;
    if (nsweeps == 0) return RBGS_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool flags = rb3_flag_driven(opts);
    int capacity = 0;
    if (flags && (rc = rb3_flags_setup(g, opts, w, s, &capacity))) return rc;
    if ((rc = rb3_pack_both(g, w, u, f, s))) return rc;
    if (flags)
        rc = rb3_sweeps_flags(g, w, nsweeps, opts, capacity, s);
    else
        rc = rb3_sweeps(g, w, nsweeps, s, nullptr);
    if (rc) return rc;
    HIP_TRY(launch_rb3_unpack(u, g->ld, w.u_red, w.u_black, g->n, w.pitch, s), "unpack u");
    return flags ? rb3_flags_error(w, s) : RBGS_OK;
}

int rbgs_rb3_residual(const rbgs_grid* g, const double* u, const double* f, double* abs_norm,
                      double* rel_norm, void* workspace, size_t workspace_bytes, void* stream) {
    Rb3Workspace w;
    int rc = rb3_prepare(g, u, f, workspace, workspace_bytes, &w);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = rb3_pack_both(g, w, u, f, s))) return rc;
    if ((rc = rb3_residual_sums(g, w, s))) return rc;
    Workspace v;
    v.sums = w.sums;
    return fetch_norms(v, s, abs_norm, rel_norm);
}

int rbgs_rb3_solve(const rbgs_grid* g, double* u, const double* f, int32_t max_sweeps,
                   double rel_tol, int32_t check_every, rbgs_solve_info* info, void* workspace,
                   size_t workspace_bytes, void* stream) {
    return rbgs_rb3_solve_ex(g, u, f, max_sweeps, rel_tol, check_every, nullptr, info, workspace,
                             workspace_bytes, stream);
}

int rbgs_rb3_solve_ex(const rbgs_grid* g, double* u, const double* f, int32_t max_sweeps,
                      double rel_tol, int32_t check_every, const rbgs_rb3_opts* opts,
                      rbgs_solve_info* info, void* workspace, size_t workspace_bytes,
                      void* stream) {
    if (max_sweeps < 0) return fail(RBGS_EINVAL, "max_sweeps must be >= 0");
    if (check_every < 1) return fail(RBGS_EINVAL, "check_every must be >= 1");
    if (std::isnan(rel_tol)) return fail(RBGS_EINVAL, "rel_tol is NaN");
    int rc = rb3_check_opts(opts);
    if (rc) return rc;
    const bool flags = rb3_flag_driven(opts);
    if (flags && (max_sweeps > (1 << 29)))
        return fail(RBGS_EINVAL, "the flag-driven form runs at most 2^29 sweeps per call");
    Rb3Workspace w;
    if ((rc = rb3_prepare(g, u, f, workspace, workspace_bytes, &w))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int capacity = 0;
    if (flags && (rc = rb3_flags_setup(g, opts, w, s, &capacity))) return rc;
    if ((rc = rb3_pack_both(g, w, u, f, s))) return rc;
    Workspace v;
    v.sums = w.sums;
    double rel = 0.0, ab = 0.0;
    int32_t done = 0;
    // k sweeps of whichever form was asked for; the flag-driven form checks
    // its error word after each group (one launch per group of sweeps)
    auto sweeps = [&](int k) -> int {
        if (!flags) return rb3_sweeps(g, w, k, s, nullptr);
        int r = rb3_sweeps_flags(g, w, k, opts, capacity, s);
        return r ? r : rb3_flags_error(w, s);
    };
    if (rel_tol <= 0.0) {
        if ((rc = sweeps(max_sweeps))) return rc;
        done = max_sweeps;
        if ((rc = rb3_residual_sums(g, w, s))) return rc;
        if ((rc = fetch_norms(v, s, &ab, &rel))) return rc;
    } else {
        if ((rc = rb3_residual_sums(g, w, s))) return rc;
        if ((rc = fetch_norms(v, s, &ab, &rel))) return rc;
        const int cap = max_sweeps / check_every;
        if (!flags && !(rel <= rel_tol) && std::isfinite(rel) && cap > 0) {
            RoundBody body = [&](hipStream_t cs, const int* stop, void** es) -> int {
                *es = nullptr;
                int r = rb3_sweeps(g, w, check_every, cs, stop);
                return r ? r : rb3_residual_sums(g, w, cs);
            };
            int rounds = 0;
            bool used = false;
            void* es = nullptr;
            if ((rc = solve_rounds_graph(v, body, cap, rel_tol, s, &es, &rounds, &used,
                                         2 * int64_t(check_every) + 3)))
                return rc;
            if (used) {
                done = rounds * check_every;
                if ((rc = fetch_norms(v, s, &ab, &rel))) return rc;
            }
        }
        while (!(rel <= rel_tol) && done < max_sweeps && std::isfinite(rel)) {
            const int32_t k = max_sweeps - done < check_every ? max_sweeps - done : check_every;
            if ((rc = sweeps(k))) return rc;
            done += k;
            if ((rc = rb3_residual_sums(g, w, s))) return rc;
            if ((rc = fetch_norms(v, s, &ab, &rel))) return rc;
        }
    }
    HIP_TRY(launch_rb3_unpack(u, g->ld, w.u_red, w.u_black, g->n, w.pitch, s), "unpack u");
    HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
    rbgs_solve_info out{done, 0, rel, ab, RBGS_OK};
    if (!std::isfinite(rel))
        out.status = RBGS_ENONFINITE;
    else
        out.status = (rel_tol <= 0.0 || rel <= rel_tol) ? RBGS_OK : RBGS_ENOCONV;
    if (info) *info = out;
    if (out.status == RBGS_ENONFINITE) g_last_error = "residual is not finite";
    if (out.status == RBGS_ENOCONV) g_last_error = "tolerance not reached";
    return out.status;
}

int rbgs_restrict(int32_t batch, rbgs_dtype dt, const rbgs_grid* fine, const void* x_fine,
                  int64_t fine_stride, const rbgs_grid* coarse, void* x_coarse,
                  int64_t coarse_stride, void* stream) {
    int rc = check_transfer(batch, dt, coarse, x_coarse, coarse_stride, fine, x_fine, fine_stride);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dt == RBGS_F64)
        HIP_TRY(launch_restrict<double>(static_cast<const double*>(x_fine), fine->ld, fine_stride,
                                        static_cast<double*>(x_coarse), coarse->ld,
                                        coarse_stride, coarse->n, batch, s),
                "restrict");
    else
        HIP_TRY(launch_restrict<float>(static_cast<const float*>(x_fine), fine->ld, fine_stride,
                                       static_cast<float*>(x_coarse), coarse->ld, coarse_stride,
                                       coarse->n, batch, s),
                "restrict");
    return RBGS_OK;
}

int rbgs_prolong(int32_t batch, rbgs_dtype dt, const rbgs_grid* coarse, const void* x_coarse,
                 int64_t coarse_stride, const rbgs_grid* fine, void* x_fine, int64_t fine_stride,
                 void* stream) {
    int rc = check_transfer(batch, dt, coarse, x_coarse, coarse_stride, fine, x_fine, fine_stride);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dt == RBGS_F64)
        HIP_TRY(launch_prolong<double>(static_cast<const double*>(x_coarse), coarse->ld,
                                       coarse_stride, static_cast<double*>(x_fine), fine->ld,
                                       fine_stride, fine->n, batch, s),
                "prolong");
    else
        HIP_TRY(launch_prolong<float>(static_cast<const float*>(x_coarse), coarse->ld,
                                      coarse_stride, static_cast<float*>(x_fine), fine->ld,
                                      fine_stride, fine->n, batch, s),
                "prolong");
    return RBGS_OK;
}

}  // extern "C"
