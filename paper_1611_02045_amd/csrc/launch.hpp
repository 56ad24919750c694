// Host-side launch helpers for directional passes.
#pragma once

#include <atomic>
#include <mutex>

#include <algorithm>

#include <hip/hip_ext.h>

#include "passes.hpp"

namespace gpe {

// Compute units of the current device (queried once per device).
inline int device_cus() {
    static std::atomic<int> cached[16] = {};  // solves may run on several host threads
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return 256;
    int n = cached[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cached[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

// Optional start/stop events a launch records around its own execution (per-kernel timing).
struct LaunchEvents {
    hipEvent_t start, stop;
};

// hipLaunchKernelGGL, or its event-recording form when timing.
template <typename K, typename... Args>
inline void launch_timed(const LaunchEvents* ev, K kern, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                         Args... args) {
    if (ev)
        hipExtLaunchKernelGGL(kern, grid, block, lds, s, ev->start, ev->stop, 0, args...);
    else
        hipLaunchKernelGGL(kern, grid, block, lds, s, args...);
}

constexpr size_t kPassLdsBudget = 96 * 1024;
// Workgroup size cap of the passes: with 256 threads (one wave per SIMD) every kernel may keep up
// to 256 VGPRs per lane without scratch spills.
constexpr int kMaxPassThreads = 256;

inline size_t pass_lds_bytes_cb(int cb, int M, int C, int threads, int K, int axis) {
    size_t b = (size_t)cb * ((size_t)M + (size_t)C * line_stride(M, cb, axis, C));
    b = (b + 15) & ~(size_t)15;
    b += sizeof(double) * (size_t)((((threads + 63) / 64) + 1) * (K > 0 ? K : 1) + 4);
    return b;
}

// Lines per workgroup for a pass along AX over B instances.  x passes pack up to 256 threads of
// whole lines; strided passes take enough adjacent lines for 128-byte row segments, capped by
// the thread and LDS budgets and by n_x.  When the whole launch would have few workgroups (small
// single grids) the groups are made smaller so that every CU gets work: these launches are bound
// by latency, not bandwidth.
// Lines per workgroup chosen by measurement (gpe_autotune) for a grid, axis, point size and batch
// size, or 0 when none was recorded; recording replaces the rule below for every later launch.
int tuned_lines(const Geo& g, int AX, int complex_bytes, int B);
void record_tuned_lines(const Geo& g, int AX, int complex_bytes, int B, int C);

// Whether C lines per workgroup is a valid tile for a pass along AX (whole lines, at most 256
// threads, C dividing the lines of a field, strided groups within n_x, LDS within budget).
inline bool valid_lines(const Geo& g, int AX, int complex_bytes, int C) {
    const int TPL = g.n[AX] / 8;
    if (C < 1 || (C & (C - 1)) != 0 || C * TPL > 256) return false;
    if (lines_per_field(g, AX) % C != 0) return false;
    if (AX != 0 && C > g.n[0]) return false;
    return pass_lds_bytes_cb(complex_bytes, g.n[AX], C, C * TPL, 32, AX) <= kPassLdsBudget;
}

// Largest power of two <= x (x >= 1).
inline int floor_pow2(int x) {
    int p = 1;
    while (2 * p <= x) p *= 2;
    return p;
}

inline int pass_lines_rule(const Geo& g, int AX, int complex_bytes, int B) {
    const int TPL = g.n[AX] / 8;
    const int64_t lpf = lines_per_field(g, AX);
    const int64_t lines = lpf * (int64_t)B;
    int C;
    if (AX == 0) {
        C = floor_pow2(std::max(1, 256 / TPL));
    } else {
        C = std::max(1, 128 / complex_bytes);
        C = std::min(C, floor_pow2(std::max(1, 256 / TPL)));
        C = std::min(C, floor_pow2(g.n[0]));
    }
    // keep at least 64 workgroups so that small grids still spread over the chip, but never less
    // than one full wave per workgroup: a partial wave leaves lanes idle and takes the slow
    // partial-row reduction; larger groups keep the per-instance partial rows (which every
    // consumer workgroup reduces) few.  (Lines of 5 * 2^k points give partial waves regardless.)
    const int Cmin = floor_pow2(std::max(1, 64 / TPL));
    while (C > Cmin && lines / C < 64) C >>= 1;
    while (C > 1 && (lpf % C) != 0) C >>= 1;
    // keep the LDS footprint (twiddles + lines + reduction scratch) within budget
    while (C > 1 && pass_lds_bytes_cb(complex_bytes, g.n[AX], C, C * TPL, 32, AX) > kPassLdsBudget) C >>= 1;
    return C;
}

// Lines per workgroup of a launch: operator passes take a measured tile when one was recorded;
// solver passes (which absorb their producers' partial rows, one per workgroup) always take the
// rule: tiles measured on the operator pass favour more, smaller workgroups, which made the
// solver's passes up to 30% slower.
inline int pass_lines_per_block(const Geo& g, int AX, int complex_bytes, int B, bool solver) {
    if (!solver)
        if (const int t = tuned_lines(g, AX, complex_bytes, B)) return t;
    return pass_lines_rule(g, AX, complex_bytes, B);
}

inline int pass_blocks_per_field(const Geo& g, int AX, int complex_bytes, int B, bool solver) {
    return (int)(lines_per_field(g, AX) / pass_lines_per_block(g, AX, complex_bytes, B, solver));
}

// Launch one pass over B instances.  `pr` receives nb (blocks per instance) if the Op reduces.
template <typename T, int AX, class Op>
hipError_t launch_pass(const Geo& g, int B, const void* tw, const Op& op, Partials pr, hipStream_t s,
                       const LaunchEvents* ev = nullptr, int C_force = 0) {
    const int cb = (int)sizeof(C2<T>);
    const int C = C_force > 0 ? C_force : pass_lines_per_block(g, AX, cb, B, Op::SCALARS);
    const int TPL = g.n[AX] / 8;
    const int threads = C * TPL;
    const int nb = (int)(lines_per_field(g, AX) / C);
    pr.nb = nb;
    if (pr.stride == 0) pr.stride = nb;
    // reduction scratch sized for the pass's own sums and for absorbing up to 16 sums of its predecessor
    const size_t lds = pass_lds_bytes<T>(g.n[AX], C, threads, Op::K > 16 ? Op::K : 16, AX);
    if (threads > kMaxPassThreads) return hipErrorInvalidConfiguration;
    const int64_t blocks = nb * (int64_t)(g.bl > 0 ? g.bl : B);  // instances [g.b0, g.b0 + g.bl) only
    // one workgroup per CU or fewer: fetch everything ahead of the scalar logic (see pass_kernel)
    const bool early = blocks <= device_cus();
    // lines of 64, 128, 256, 512 and 640 points (the common sizes and the paper's) take the
    // compile-time transform (measured 18% less time per iteration than the run-time one on 256^2,
    // 22-27% on 64^2 and 64^3); other sizes the run-time one
    constexpr int kMaxT = kMaxPassThreads;
    const int lg = g.lg[AX];
    const int ct = g.f5[AX] ? (lg == 7 ? 4 : 0) : (lg == 9 ? 3 : lg == 8 ? 2 : lg == 7 ? 1 : lg == 6 ? 5 : 0);
    using K = decltype(&pass_kernel<T, AX, Op, kMaxT, true, 0>);
    const K variants[12] = {pass_kernel<T, AX, Op, kMaxT, false, 0>,   pass_kernel<T, AX, Op, kMaxT, true, 0>,
                            pass_kernel<T, AX, Op, kMaxT, false, 7>,   pass_kernel<T, AX, Op, kMaxT, true, 7>,
                            pass_kernel<T, AX, Op, kMaxT, false, 8>,   pass_kernel<T, AX, Op, kMaxT, true, 8>,
                            pass_kernel<T, AX, Op, kMaxT, false, 9>,   pass_kernel<T, AX, Op, kMaxT, true, 9>,
                            pass_kernel<T, AX, Op, kMaxT, false, 107>, pass_kernel<T, AX, Op, kMaxT, true, 107>,
                            pass_kernel<T, AX, Op, kMaxT, false, 6>,   pass_kernel<T, AX, Op, kMaxT, true, 6>};
    const K kern = variants[2 * ct + (early ? 1 : 0)];
    static std::once_flag attr_once;  // one attribute call per instantiation set (thread-safe)
    std::call_once(attr_once, [&] {
        // Raise the dynamic-LDS cap once; a runtime that does not need it may refuse harmlessly.
        for (K k : variants)
            if (hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPassLdsBudget) !=
                hipSuccess)
                (void)hipGetLastError();
    });
    launch_timed(ev, kern, dim3((unsigned)blocks), dim3(threads), lds, s, g, C, (const C2<T>*)tw, op, pr);
    return hipGetLastError();
}

}  // namespace gpe
