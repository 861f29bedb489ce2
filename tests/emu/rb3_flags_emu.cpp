// Runs the flag-driven 3D sweep (the device code in
// paper_2607_01735_amd/csrc/rb3_flags.h, unchanged) on the CPU.  Each
// emulated workgroup (one wave: 64 lanes as fibers) runs on its own host
// thread and takes (level, block) tickets from the shared counter as a
// workgroup of the persistent kernel would; the ticket, the block counters,
// the error word and the grid arrays are shared between the threads
// through the same atomic operations and fences the device code uses.  Every array is its own heap block of
// exactly the size the library allocates, so an AddressSanitizer build
// reports any access outside them; a ThreadSanitizer build reports any grid
// access that the block dependencies do not order.  Test infrastructure
// only: tests/test_rb3_flags_emu.py builds it and compares the result with
// the oracle bit for bit.
//
// Build: g++ -std=c++17 -I tests/emu -I paper_2607_01735_amd/csrc ...
// Run:   emu n sweeps h in.bin out.bin max_blocks workgroups [delay [stall_block]]
//        (EMU_CHUNK=lean in the environment: the lean plane chunk, else the deep one)
//   in.bin  = u then f, natural (n+2)^3 arrays of doubles, index (i, j, k)
//   out.bin = u after the sweeps, same layout
// Exit status 4 when the kernel raised its error word (a wait expired).
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>

#include <thread>
#include <vector>

#include "rb3_flags.h"

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

static thread_local ucontext_t g_host_ctx, g_start_ctx[emu::kMaxThreads];
static thread_local jmp_buf g_host_jmp;
static rbgs::rb3f::Args g_args;
static bool g_lean = false;  // the kernel with the lean plane chunk (EMU_CHUNK=lean)

static void to_host() {
#ifdef EMU_TSAN
    __tsan_switch_to_fiber(emu::host_fiber, 0);
#endif
    _longjmp(g_host_jmp, 1);
}

static void lane_start(int lane) {
    if (_setjmp(emu::lane_jmp[lane]) == 0) {
#ifdef EMU_TSAN
        __tsan_switch_to_fiber(emu::host_fiber, 0);
#endif
        swapcontext(&g_start_ctx[lane], &g_host_ctx);
    }
    if (g_lean)
        rbgs::rb3f::run<rbgs::rb3f::kLeanChunk>(g_args);
    else
        rbgs::rb3f::run<rbgs::rb3f::kDeepChunk>(g_args);
    emu::lane_done[lane] = true;
    for (int k = 1; k < emu::nthreads; ++k) {
        const int nx = (lane + k) % emu::nthreads;
        if (!emu::lane_done[nx]) emu::jump_to_lane(nx);
    }
    to_host();
}

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
        if (swapcontext(&g_host_ctx, &g_start_ctx[l]) != 0) abort();
    }
    if (_setjmp(g_host_jmp) == 0) emu::jump_to_lane(0);
    for (int l = 0; l < emu::nthreads; ++l) free(stacks[l]);
}

int main(int argc, char** argv) {
    if (argc < 8 || argc > 10) {
        fprintf(stderr,
                "usage: %s n sweeps h in.bin out.bin max_blocks workgroups [delay [stall]]\n",
                argv[0]);
        return 2;
    }
    const int n = atoi(argv[1]), sweeps = atoi(argv[2]);
    const double h = atof(argv[3]);
    const int max_blocks = atoi(argv[6]), workgroups = atoi(argv[7]);
    const char* chunk = getenv("EMU_CHUNK");
    g_lean = chunk && chunk[0] == 'l';
    const rbgs::rb3f::Geometry geo = rbgs::rb3f::geometry(n, max_blocks);
    const size_t W = size_t(n) + 2;
    const size_t cells_nat = W * W * W;
    std::vector<double> u(cells_nat), f(cells_nat);
    FILE* fin = fopen(argv[4], "rb");
    if (!fin || fread(u.data(), 8, cells_nat, fin) != cells_nat ||
        fread(f.data(), 8, cells_nat, fin) != cells_nat) {
        fprintf(stderr, "cannot read %s\n", argv[4]);
        return 2;
    }
    fclose(fin);
    // the library's split layout: (i, j, k) of colour (i + j + k) & 1 at
    // C[(i (n+2) + j) pitch + (k >> 1)], pitch = (n + 3) / 2 rounded up to
    // 256 bytes; the padding holds NaN, so a read of it would show
    const int64_t P = ((int64_t(n) + 3) / 2 + 31) / 32 * 32;
    const size_t cells = W * W * size_t(P);
    auto block_of = [&]() {
        double* p = static_cast<double*>(malloc(cells * sizeof(double)));
        if (!p) abort();
        for (size_t k = 0; k < cells; ++k) p[k] = __builtin_nan("");
        return p;
    };
    double *red = block_of(), *black = block_of(), *f_red = block_of(), *f_black = block_of();
    for (size_t i = 0; i < W; ++i)
        for (size_t j = 0; j < W; ++j)
            for (size_t k = 0; k < W; ++k) {
                const size_t at = (i * W + j) * size_t(P) + (k >> 1);
                const bool is_red = ((i + j + k) & 1) == 0;
                (is_red ? red : black)[at] = u[(i * W + j) * W + k];
                (is_red ? f_red : f_black)[at] = f[(i * W + j) * W + k];
            }
    rbgs::rb3f::Args& a = g_args;
    a.red = red;
    a.black = black;
    a.f_red = f_red;
    a.f_black = f_black;
    a.n = n;
    a.pitch = P;
    a.h2 = h * h;
    a.qw = geo.qw;
    a.rj = geo.rj;
    a.rz = geo.rz;
    a.qblocks = geo.qblocks;
    a.jblocks = geo.jblocks;
    a.zblocks = geo.zblocks;
    a.nblocks = geo.nblocks;
    a.levels = 2 * sweeps;
    a.ticket = static_cast<int*>(calloc(1, sizeof(int)));
    a.progress = static_cast<int*>(calloc(size_t(geo.nblocks), sizeof(int)));
    a.error = static_cast<int*>(calloc(1, sizeof(int)));
    a.spin_limit = 1 << 26;
    a.delay = argc > 8 ? atoi(argv[8]) : 0;
    a.stall_block = argc > 9 ? atoi(argv[9]) : 0;
    if (a.stall_block) a.spin_limit = 1 << 12;
    a.stop = nullptr;
    if (workgroups <= 1) {
        run_workgroup(0);
    } else {
        std::vector<std::thread> threads;
        for (int w = 0; w < workgroups; ++w) threads.emplace_back(run_workgroup, w);
        for (auto& t : threads) t.join();
    }
    printf("n=%d sweeps=%d qw=%d rj=%d rz=%d blocks=%d (%d x %d x %d) workgroups=%d chunk=%s\n", n,
           sweeps, geo.qw, geo.rj, geo.rz, geo.nblocks, geo.qblocks, geo.jblocks, geo.zblocks,
           workgroups, g_lean ? "lean" : "deep");
    if (*a.error != 0) {
        fprintf(stderr, "the kernel raised its error word (%d)\n", *a.error);
        return 4;
    }
    for (size_t i = 0; i < W; ++i)
        for (size_t j = 0; j < W; ++j)
            for (size_t k = 0; k < W; ++k) {
                const size_t at = (i * W + j) * size_t(P) + (k >> 1);
                u[(i * W + j) * W + k] = (((i + j + k) & 1) == 0 ? red : black)[at];
            }
    FILE* fout = fopen(argv[5], "wb");
    if (!fout || fwrite(u.data(), 8, cells_nat, fout) != cells_nat) return 2;
    fclose(fout);
    free(red);
    free(black);
    free(f_red);
    free(f_black);
    free(a.progress);
    free(a.ticket);
    free(a.error);
    return 0;
}
