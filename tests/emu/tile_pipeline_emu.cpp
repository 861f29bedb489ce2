// Runs the persistent tile pipeline of the blocked sweep (the device code in
// paper_2607_01735_amd/csrc/blocked_pipeline.h, unchanged) on the CPU.  Each
// emulated workgroup (one wave: 64 lanes as fibers) runs on its own host
// thread and takes (pass, tile) tickets from the shared counter exactly
// as a workgroup of the persistent kernel would; the progress flags,
// tickets and grid arrays are shared between the threads through the same
// atomic operations and fences the device code uses.  Every array the
// pipeline touches is its own heap block of exactly the size the library
// allocates, so an AddressSanitizer build reports any access outside them;
// a ThreadSanitizer build reports any grid access that the dependency
// protocol does not order.  Test infrastructure only:
// tests/test_tile_pipeline_emu.py builds it and compares the result with the
// oracle bit for bit.
//
// Build: g++ -std=c++17 -DEMU_T=double -DEMU_FUSE=7 -I tests/emu
//            -I paper_2607_01735_amd/csrc -I include ...
// Run:   emu n rows passes h in.bin out.bin [workgroups [yield_every]]
//   in.bin  = u then f, natural (n+2) x (n+2) arrays of EMU_T, row major
//   out.bin = u after passes x fuse full sweeps, same layout
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>

#include <thread>
#include <vector>

#include "blocked_pipeline.h"
#include "rbgs_blocked.h"

namespace emu {
thread_local int nthreads = kLanes;
thread_local int current = 0;
thread_local jmp_buf lane_jmp[kMaxThreads];
thread_local bool lane_done[kMaxThreads];
thread_local uint64_t lane_slot[kMaxThreads];
thread_local int bar_arrived = 0, bar_generation = 0;
int yield_every = 0;
thread_local unsigned switches = 0;
thread_local int workgroup = 0;
#ifdef EMU_TSAN
thread_local void* lane_fiber[kMaxThreads];
thread_local void* host_fiber;
#endif
}  // namespace emu

// Fibers: each lane's stack is entered once through makecontext/swapcontext
// (lane_start parks it with _setjmp and returns to the host); from then on
// lanes switch with _setjmp/_longjmp.
static thread_local ucontext_t g_host_ctx, g_start_ctx[emu::kMaxThreads];
static thread_local jmp_buf g_host_jmp;

using namespace rbgs;
using namespace rbgs::blocked;
typedef EMU_T T;
constexpr int kFuse = EMU_FUSE;
constexpr int kL = 2 * kFuse;
constexpr int kV = 16 / int(sizeof(T));

static GridDesc<T> g_grid;
static Queue g_queue;
static DebugModes g_debug;  // tile order / stamp check (environment EMU_TILE_ORDER,
                            // EMU_SEED, EMU_STAMP_CHECK), as the verification kernel runs them
static bool g_debug_on = false;
static T g_omega = T(1);  // != 1: the SOR pipeline (environment EMU_OMEGA)
static int g_split = 1 << 30;  // EMU_MERGED: passes from g_split on run one sweep shallower
                               // (environment EMU_SPLIT), as the merged launch does

static void to_host() {
#ifdef EMU_TSAN
    __tsan_switch_to_fiber(emu::host_fiber, 0);
#endif
    _longjmp(g_host_jmp, 1);
}

// The body of the persistent kernel for one workgroup, run by every lane
// fiber; a finished lane hands over to the next live one, the last to the
// host.
static void lane_start(int lane) {
    if (_setjmp(emu::lane_jmp[lane]) == 0) {
#ifdef EMU_TSAN
        __tsan_switch_to_fiber(emu::host_fiber, 0);
#endif
        swapcontext(&g_start_ctx[lane], &g_host_ctx);
    }
    const int total = g_queue.passes * g_grid.ntiles;
    for (;;) {
        const int tk = next_ticket(g_queue);
        if (tk >= total) break;
        const int pass = tk / g_grid.ntiles;
#ifdef EMU_MERGED
        if (pass >= g_split) {  // the shallower passes of a merged launch
            if (!run_item<T, kV, kL - 2>(g_grid, g_queue, pass, tk - pass * g_grid.ntiles)) break;
            continue;
        }
#endif
        if (g_omega != T(1)) {
            if (!run_item<T, kV, kL, false, true>(g_grid, g_queue, pass, tk - pass * g_grid.ntiles,
                                                  DebugModes(), 0, g_omega))
                break;
        } else if (g_debug_on) {
            const int tile = tile_of_ticket(g_debug, g_grid.ntiles, pass, tk - pass * g_grid.ntiles);
            if (!run_item<T, kV, kL, true>(g_grid, g_queue, pass, tile, g_debug, tk)) break;
        } else if (!run_item<T, kV, kL>(g_grid, g_queue, pass, tk - pass * g_grid.ntiles)) {
            break;
        }
    }
    emu::lane_done[lane] = true;
    for (int k = 1; k < emu::nthreads; ++k) {
        const int nx = (lane + k) % emu::nthreads;
        if (!emu::lane_done[nx]) emu::jump_to_lane(nx);
    }
    to_host();
}

// One workgroup on this host thread: park every lane, then run them.
static void run_workgroup(int wg) {
    emu::workgroup = wg;
    emu::nthreads = emu::kLanes;
    emu::current = 0;
    emu::bar_arrived = emu::bar_generation = 0;
#ifdef EMU_TSAN
    emu::host_fiber = __tsan_get_current_fiber();
#endif
    const size_t stack_bytes = size_t(1) << 20;
    std::vector<char*> stacks(emu::nthreads);
    for (int l = 0; l < emu::nthreads; ++l) {
        stacks[l] = static_cast<char*>(malloc(stack_bytes));
        if (!stacks[l] || getcontext(&g_start_ctx[l]) != 0) abort();
        g_start_ctx[l].uc_stack.ss_sp = stacks[l];
        g_start_ctx[l].uc_stack.ss_size = stack_bytes;
        g_start_ctx[l].uc_link = nullptr;
        makecontext(&g_start_ctx[l], reinterpret_cast<void (*)()>(lane_start), 1, l);
        emu::lane_done[l] = false;
#ifdef EMU_TSAN
        emu::lane_fiber[l] = __tsan_create_fiber(0);
        __tsan_switch_to_fiber(emu::lane_fiber[l], 0);
#endif
        if (swapcontext(&g_host_ctx, &g_start_ctx[l]) != 0) abort();  // parks lane l
    }
    if (_setjmp(g_host_jmp) == 0) emu::jump_to_lane(0);
    for (int l = 0; l < emu::nthreads; ++l) free(stacks[l]);
}

static T* block_of(size_t count) {
    T* p = static_cast<T*>(malloc(count * sizeof(T)));
    if (!p) abort();
    for (size_t k = 0; k < count; ++k) p[k] = T(-12345);
    return p;
}

int main(int argc, char** argv) {
    if (argc < 7 || argc > 9) {
        fprintf(stderr, "usage: %s n rows passes h in.bin out.bin [workgroups [yield_every]]\n",
                argv[0]);
        return 2;
    }
    const int n = atoi(argv[1]), rows = atoi(argv[2]), passes = atoi(argv[3]);
    const double h = atof(argv[4]);
    const Geometry geo = geometry(n, int(sizeof(T)), kFuse, rows < kL ? kL : rows);
    if (geo.ntiles > max_tiles(n)) {
        fprintf(stderr, "tile count %d above the state bound %d\n", geo.ntiles, max_tiles(n));
        return 3;
    }
    const size_t W = size_t(n) + 2;
    std::vector<T> u(W * W), f(W * W);
    FILE* fin = fopen(argv[5], "rb");
    if (!fin || fread(u.data(), sizeof(T), u.size(), fin) != u.size() ||
        fread(f.data(), sizeof(T), f.size(), fin) != f.size()) {
        fprintf(stderr, "cannot read %s\n", argv[5]);
        return 2;
    }
    fclose(fin);
    // split colour layout: point (i, j) of colour (i + j) & 1 at C[i][j >> 1]
    const int64_t P = split_pitch(n, sizeof(T));
    const size_t cells = W * size_t(P);
    T* red[2] = {block_of(cells), block_of(cells)};
    T* black[2] = {block_of(cells), block_of(cells)};
    T* f_red = block_of(cells);
    T* f_black = block_of(cells);
    // buffer 0 holds the packed iterate; buffer 1 only what the library
    // copies into it (the Dirichlet ring) and NaN elsewhere, so that a read
    // of anything else would show in the result
    const T nan = T(__builtin_nan(""));
    for (size_t k = 0; k < cells; ++k) red[1][k] = black[1][k] = nan;
    for (size_t i = 0; i < W; ++i)
        for (size_t j = 0; j < W; ++j) {
            const size_t at = i * size_t(P) + (j >> 1);
            const bool is_red = ((i + j) & 1) == 0;
            (is_red ? red[0] : black[0])[at] = u[i * W + j];
            (is_red ? f_red : f_black)[at] = f[i * W + j];
        }
    for (size_t i = 0; i < W; ++i)  // rows 0 and n+1; q-columns 0 and (n+1)/2
        for (size_t q = 0; q < size_t(P); ++q)
            if (i == 0 || i == W - 1 || q == 0 || q == size_t(n + 1) / 2) {
                red[1][i * P + q] = red[0][i * P + q];
                black[1][i * P + q] = black[0][i * P + q];
            }
    GridDesc<T>& g = g_grid;
    g.red[0] = red[0];
    g.red[1] = red[1];
    g.black[0] = black[0];
    g.black[1] = black[1];
    g.f_red = f_red;
    g.f_black = f_black;
    g.n = n;
    g.pitch = P;
    g.h2 = T(h * h);
    g.rows = geo.rows;
    g.halo_q = geo.halo_q;
    g.q_core = geo.q_core;
    g.strips = geo.strips;
    g.bands = geo.bands;
    g.ntiles = geo.ntiles;
    g.flag_base = 0;
    g.omega = T(1);
    Queue& qu = g_queue;
    qu.passes = passes;
    qu.progress = static_cast<int*>(calloc(size_t(geo.ntiles), sizeof(int)));
    qu.ticket = static_cast<int*>(calloc(1, sizeof(int)));
    qu.error = static_cast<int*>(calloc(1, sizeof(int)));
    qu.spin_limit = 1 << 20;
    qu.delay = 0;
    qu.stall_tile = 0;
    qu.buf_offset = 0;
    qu.stop = nullptr;
    if (const char* e = getenv("EMU_TILE_ORDER")) g_debug.order = atoi(e);
    if (const char* e = getenv("EMU_SEED")) g_debug.seed = uint32_t(strtoul(e, nullptr, 10));
    if (const char* e = getenv("EMU_STAMP_CHECK")) g_debug.stamp_check = atoi(e);
    g_debug_on = g_debug.order != 0 || g_debug.stamp_check != 0;
    if (const char* e = getenv("EMU_OMEGA")) g_omega = T(atof(e));
    if (const char* e = getenv("EMU_SPLIT")) g_split = atoi(e);
#ifdef EMU_MERGED
    {  // the merged launch needs the same tiles at both depths
        const Geometry lo = geometry(n, int(sizeof(T)), kFuse - 1, rows < kL ? kL : rows);
        if (lo.halo_q != geo.halo_q || lo.q_core != geo.q_core || lo.ntiles != geo.ntiles) {
            fprintf(stderr, "depths %d and %d give different tiles\n", kFuse, kFuse - 1);
            return 3;
        }
    }
#endif
    const int workgroups = argc > 7 ? atoi(argv[7]) : 1;
    emu::yield_every = argc > 8 ? atoi(argv[8]) : 0;
    if (workgroups > 1) qu.spin_limit = 1 << 28;
    if (workgroups <= 1) {
        run_workgroup(0);  // on the main thread
    } else {
        std::vector<std::thread> threads;
        for (int w = 0; w < workgroups; ++w) threads.emplace_back(run_workgroup, w);
        for (auto& t : threads) t.join();
    }
    if (*qu.error != 0) {
        fprintf(stderr, "the pipeline raised its error word (%d)\n", *qu.error);
        return 4;
    }
    const int out = passes & 1;
    for (size_t i = 0; i < W; ++i)
        for (size_t j = 0; j < W; ++j) {
            const size_t at = i * size_t(P) + (j >> 1);
            u[i * W + j] = (((i + j) & 1) == 0 ? red[out] : black[out])[at];
        }
    FILE* fout = fopen(argv[6], "wb");
    if (!fout || fwrite(u.data(), sizeof(T), u.size(), fout) != u.size()) return 2;
    fclose(fout);
    printf("n=%d rows=%d passes=%d fuse=%d workgroups=%d tiles=%d halo_q=%d q_core=%d order=%d "
           "stamp_check=%d\n", n, geo.rows, passes, kFuse, workgroups, geo.ntiles, geo.halo_q,
           geo.q_core, g_debug.order, g_debug.stamp_check);
    for (int b = 0; b < 2; ++b) {
        free(red[b]);
        free(black[b]);
    }
    free(f_red);
    free(f_black);
    free(qu.progress);
    free(qu.ticket);
    free(qu.error);
    return 0;
}
