// Generic directional pass: one workgroup transforms C grid lines along one axis.
//
// Every hot operator of the solver is a chain of such passes (Section 3: the discrete
// operators act as 1-D transforms along x at fixed y, along y at fixed x, ...).  A pass is
//   decode line -> Op::load (prologue, fills the 8 registers) -> forward FFT (optional)
//   -> Op::spectral (multiplier and spectral reductions) -> inverse FFT (optional)
//   -> Op::store (epilogue: combine, write, pointwise reductions)
//   -> deterministic block reduction of Op::K sums into per-block partials.
// Solver passes (Op::SCALARS) first build the instance's FP64 scalar state in LDS with Op::begin:
// every block reduces the partials of the previous pass in the same fixed order and runs the same
// scalar logic, so all blocks agree without atomics or fences (the kernel boundary makes the
// previous pass's partials visible), and one block per instance publishes the new state.
// Field layout: x fastest; a batch of B equally sized instances is stored back to back.  For the
// x axis consecutive lanes walk along one line (stride 1, coalesced); for y and z consecutive
// lanes walk across C adjacent lines (adjacent x, coalesced), and each thread keeps its 8
// points strided along the line.
#pragma once

#include <type_traits>

#include "fft.hpp"

namespace gpe {

struct LineCtx {
    int t;          // position of this thread within its line, [0, TPL)
    int c;          // line within the block
    int b;          // instance (batch) index
    int i1, i2;     // indices of the line along the other axes (x-pass: y,z; y-pass: x,z; z-pass: x,y)
    int lg, M, TPL;
    int64_t base;   // offset of point 0 of the line in the batched field
    int64_t stride; // distance between consecutive points of the line
    int64_t off_b;  // b * N
    const Scal* sc; // the instance's scalar state in LDS (solver passes only)
    bool wave;      // every line of the workgroup lies within one wave (x passes, M <= 512)
    __device__ __forceinline__ int64_t at(int s) const { return base + (int64_t)(t + s * TPL) * stride; }
    __device__ __forceinline__ int k(int s) const { return t + s * TPL; }
};

// Number of lines of one instance for a pass along axis AX.
__host__ __device__ inline int64_t lines_per_field(const Geo& g, int AX) {
    return g.N / g.n[AX];
}

// Compile-time line sizes of the pass kernels: LG in 1..10 stands for 2^LG points, LG >= 100 for
// 5 * 2^(LG - 100) points; 0 means the size is taken at run time.
__host__ __device__ constexpr bool ct_f5(int LG) { return LG >= 100; }
__host__ __device__ constexpr int ct_lg(int LG) { return LG >= 100 ? LG - 100 : LG; }
__host__ __device__ constexpr int ct_points(int LG) { return ct_f5(LG) ? 5 << ct_lg(LG) : 1 << ct_lg(LG); }

// When every extent is a power of two the decomposition of the launch into lines uses shifts and
// masks only (64-bit integer division is a long software sequence on the GPU); grids with an axis
// of 5 * 2^k points take 32-bit divisions (line counts stay far below 2^32).  blk receives the
// workgroup's index within its instance.  C (lines per workgroup) is always a power of two.
template <int AX, int LG = 0>
__device__ __forceinline__ LineCtx decode_line(const Geo& g, int C, int& blk) {
    LineCtx lc;
    lc.lg = LG > 0 ? ct_lg(LG) : g.lg[AX];  // a compile-time size folds every index below
    const bool f5 = LG > 0 ? ct_f5(LG) : g.f5[AX] != 0;
    lc.M = f5 ? 5 << lc.lg : 1 << lc.lg;
    lc.TPL = lc.M >> 3;
    // x lines take consecutive lanes, TPL of them per line; lines of 5 * 2^k points can straddle
    // waves
    lc.wave = AX == 0 && !f5 && lc.TPL <= 64;
    const int lgC = __ffs(C) - 1;
    const int tid = threadIdx.x;
    if (AX == 0 && f5) {
        lc.c = tid / lc.TPL;
        lc.t = tid - lc.c * lc.TPL;
    } else if (AX == 0) {
        lc.c = tid >> (lc.lg - 3);
        lc.t = tid & (lc.TPL - 1);
    } else {
        lc.c = tid & (C - 1);
        lc.t = tid >> lgC;
    }
    const int lg_lpf = g.lg[0] + g.lg[1] + g.lg[2] - lc.lg;  // log2 of the lines per field
    // Workgroups are dealt to the 8 XCDs round robin (workgroup i to XCD i mod 8), each with its
    // own L2.  A strided pass's workgroup reads C adjacent columns, a fraction of each 128-byte
    // line, so neighbouring column groups are given to workgroups on the same XCD: logical group
    // x * G/8 + j runs as workgroup 8 j + x, and the XCD's L2 serves each line to all of them.
    unsigned grp = blockIdx.x;
    if (AX != 0 && (gridDim.x & 7u) == 0) grp = (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    const int nx = g.n[0], ny = g.n[1];
    if (!g.pow2) {
        const unsigned lpf = (unsigned)(g.N / lc.M);
        const unsigned line = (grp << lgC) + (unsigned)lc.c;
        const unsigned bi = line / lpf;  // instance within the launch
        lc.b = g.imap ? g.imap[bi] : g.b0 + (int)bi;
        const unsigned lf = line - bi * lpf;
        blk = (int)(lf >> lgC);
        lc.off_b = (int64_t)lc.b * g.N;
        const unsigned q = lf / (unsigned)(AX == 0 ? ny : nx);
        const int r = (int)(lf - q * (unsigned)(AX == 0 ? ny : nx));
        lc.i1 = r;
        lc.i2 = (int)q;
        if (AX == 0) {
            lc.base = lc.off_b + (int64_t)lf * nx;
            lc.stride = 1;
        } else if (AX == 1) {
            lc.base = lc.off_b + (int64_t)q * nx * ny + r;
            lc.stride = nx;
        } else {
            lc.base = lc.off_b + (int64_t)q * nx + r;
            lc.stride = (int64_t)nx * ny;
        }
        return lc;
    }
    const int64_t line = ((int64_t)grp << lgC) + lc.c;
    lc.b = g.imap ? g.imap[line >> lg_lpf] : g.b0 + (int)(line >> lg_lpf);
    const int64_t lf = line & (((int64_t)1 << lg_lpf) - 1);
    blk = (int)(lf >> lgC);
    lc.off_b = (int64_t)lc.b * g.N;
    if (AX == 0) {
        lc.i1 = (int)(lf & (ny - 1));
        lc.i2 = (int)(lf >> g.lg[1]);
        lc.base = lc.off_b + (lf << g.lg[0]);
        lc.stride = 1;
    } else if (AX == 1) {
        lc.i1 = (int)(lf & (nx - 1));
        lc.i2 = (int)(lf >> g.lg[0]);
        lc.base = lc.off_b + ((int64_t)lc.i2 << (g.lg[0] + g.lg[1])) + lc.i1;
        lc.stride = nx;
    } else {
        lc.i1 = (int)(lf & (nx - 1));
        lc.i2 = (int)(lf >> g.lg[0]);
        lc.base = lc.off_b + ((int64_t)lc.i2 << g.lg[0]) + lc.i1;
        lc.stride = (int64_t)nx * ny;
    }
    return lc;
}

// The line transform of a pass: the compile-time form for LG > 0, else the run-time one.
template <typename T, int DIR, int AX, int LG>
__device__ __forceinline__ void line_fft(C2<T> (&v)[8], C2<T>* buf, const C2<T>* tw, const LineCtx& lc) {
    if constexpr (LG > 0)
        fft_line_ct<T, DIR, ct_lg(LG), AX == 0 && !ct_f5(LG) && ct_lg(LG) <= 9, ct_f5(LG)>(v, buf, tw, lc.t);
    else
        fft_line<T, DIR>(v, buf, tw, lc.t, lc.lg, lc.M, lc.wave);
}

// Dynamic LDS layout of a pass: [twiddles M][lines C * line_stride(M)][reduction scratch].
template <typename T>
__host__ __device__ inline size_t pass_lds_bytes(int M, int C, int threads, int K, int axis) {
    size_t b = sizeof(C2<T>) * ((size_t)M + (size_t)C * line_stride(M, (int)sizeof(C2<T>), axis, C));
    b = (b + 15) & ~(size_t)15;
    b += sizeof(double) * (size_t)((((threads + 63) / 64) + 1) * (K > 0 ? K : 1) + 4);
    return b;
}

// Partial-sum buffers for reducing passes: parts[b][block][K] (FP64) and one ticket counter per
// instance.  `nb` is the number of blocks per instance.
// A region of per-block partial rows (K doubles each).  A producing pass writes its block blk of
// instance b to row b * stride + off + blk (several passes can share a region, at different
// offsets); a consumer reduces rows [b * stride, b * stride + nb).  stride 0 means nb.
struct Partials {
    double* parts;
    int nb;
    int stride;
    int off;
    __host__ __device__ int row_stride() const { return stride > 0 ? stride : nb; }
};

// Sum K partials of instance b over its nb blocks with all threads of the (last) block, in a
// fixed order.  `red` is block_reduce scratch; `out` (LDS, K doubles) receives the totals.
template <int K>
__device__ __forceinline__ void reduce_partials(const double* parts, int nb, double* red, double* out,
                                                unsigned maxmask) {
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = ((maxmask >> k) & 1u) ? -1e300 : 0.0;
    for (int blk = threadIdx.x; blk < nb; blk += blockDim.x) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double p = parts[(size_t)blk * K + k];
            acc[k] = ((maxmask >> k) & 1u) ? fmax(acc[k], p) : acc[k] + p;
        }
    }
    block_reduce<K>(acc, red, out, maxmask);
}

// Loads a solver pass issues before everything else (state, partial rows of its producers).
template <class Op, bool = Op::SCALARS>
struct IntakeOf {
    struct type {};
};
template <class Op>
struct IntakeOf<Op, true> {
    using type = typename Op::Intake;
};

// Whether launches of an Op run without the occupancy cap (see pass_kernel): Op::WIDE, and for the
// run-time-size transform (LG = 0) Op::WIDE_RT when the Op defines it.
template <class Op, class = void>
struct WideRt {
    static constexpr bool value = Op::WIDE;
};
template <class Op>
struct WideRt<Op, std::void_t<decltype(Op::WIDE_RT)>> {
    static constexpr bool value = Op::WIDE_RT;
};
template <class Op, int LG>
constexpr bool kWideAt = LG == 0 || ct_f5(LG) ? WideRt<Op>::value : Op::WIDE;

// Whether a late launch of an Op fetches its transform input (Op::prefetch) before begin(), with
// the state intake: Op::PREFETCH_EARLY when the Op defines it (Ops whose prefetch is light enough
// to hold in registers through begin()).
template <class Op, class = void>
struct PrefetchEarly {
    static constexpr bool value = false;
};
template <class Op>
struct PrefetchEarly<Op, std::void_t<decltype(Op::PREFETCH_EARLY)>> {
    static constexpr bool value = Op::PREFETCH_EARLY;
};

// Twiddles per thread fetched into registers ahead of the scalar logic (more go straight to LDS).
constexpr int kTwiddleRegs = 4;  // tw0..tw3 in pass_kernel

// The pass kernel.  Op must provide:
//   static constexpr bool FWD, INV;  static constexpr int K;  static constexpr unsigned MAXMASK;
//   static constexpr bool SCALARS;   (bit k of MAXMASK set: sum k is a max-reduction)
//   static constexpr bool PREFETCH;
//   static constexpr bool WIDE;      (register-heavy: no occupancy target, see below)
//   struct State;
//   __device__ void prefetch(const Geo&, const LineCtx&, State&) const;       // if PREFETCH: load()'s inputs
//   __device__ void prefetch_tail(const Geo&, const LineCtx&, State&) const;  // if PREFETCH: store()'s inputs
//   struct Intake;                                                                         // if SCALARS
//   __device__ void intake(int b, int blk_in_inst, Intake&) const;                         // if SCALARS
//   __device__ void begin(const Geo&, int b, int blk_in_inst, double* red, Scal* s, Intake&) const;  // if SCALARS
//   __device__ void load(const Geo&, const LineCtx&, State&, C2<T>(&)[8], double(&)[K]) const;
//   __device__ void spectral(const Geo&, const LineCtx&, State&, C2<T>(&)[8], double(&)[K],
//                            C2<T>* buf, const C2<T>* tw) const;   (buf/tw: to transform more lines)
//   __device__ void store(const Geo&, const LineCtx&, State&, C2<T>(&)[8], double(&)[K]) const;
// K sums are accumulated per thread in FP64 and reduced deterministically into pr.parts.
// Launches with several workgroups per CU (!EARLY) ask the register allocator for the occupancy
// the LDS footprint allows: four 4-wave workgroups per CU for 8-byte points, three for 16-byte
// points (their line buffers take about 45 KB of the 160 KB).  A WIDE Op keeps more live state than
// that budget and would spill, so it is left unconstrained (WIDE_RT: only with the run-time-size
// transform, whose index arithmetic needs more registers).
// LG > 0: the kernel is specialised for lines of ct_points(LG) points (2^LG, or 5 * 2^(LG - 100)
// for LG >= 100), so the transform's stages, strides and LDS offsets are compile-time constants;
// LG = 0 takes the size at run time.
template <typename T, int AX, class Op, int MAXT, bool EARLY, int LG>
__global__ __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(EARLY || kWideAt<Op, LG> ? 1 : (sizeof(T) == 4 ? 4 : 3))))
void pass_kernel(Geo g, int C, const C2<T>* __restrict__ twg, Op op, Partials pr) {
    extern __shared__ double4 smem_raw[];
    int blk_in_inst;
    LineCtx lc = decode_line<AX, LG>(g, C, blk_in_inst);
    C2<T>* tw = reinterpret_cast<C2<T>*>(smem_raw);
    constexpr int kPB = (int)sizeof(C2<T>);
    const int stride_pts = line_stride(lc.M, kPB, AX, C);
    C2<T>* buf = tw + lc.M + (size_t)lc.c * stride_pts;
    size_t off = sizeof(C2<T>) * ((size_t)lc.M + (size_t)C * stride_pts);
    off = (off + 15) & ~(size_t)15;
    double* red = reinterpret_cast<double*>(reinterpret_cast<char*>(smem_raw) + off);
    lc.sc = nullptr;
    typename Op::State st;
    // The loads of the scalar state and of the producers' partial rows go first, then every load
    // that does not depend on the state (twiddles, fields): all complete in one round trip, and
    // begin() waits for the first group only (memory counters retire in issue order).
    // EARLY (launches too small to fill the chip, bound by latency): twiddles and every field,
    // epilogue inputs included, are fetched before begin().  Otherwise (many workgroups per CU,
    // bound by bandwidth) they are fetched when needed, which keeps the register footprint and
    // hence the occupancy that hides the latency.
    typename IntakeOf<Op>::type in;
    if constexpr (Op::SCALARS) op.intake(lc.b, blk_in_inst, in);
    // (four named registers rather than an array, which the compiler may demote to scratch)
    auto tw_at = [&](int j) { return min((int)(threadIdx.x + j * blockDim.x), lc.M - 1); };
    C2<T> tw0, tw1, tw2, tw3;
    // A fixed-size transform in a launch too small to fill the chip reads its few twiddles per
    // stage straight from the global table (cached), sparing the table's copy into LDS; otherwise
    // the table is staged in LDS, whose latency the transform's dependent reads need.
    constexpr bool kTwGlobal = LG > 0 && EARLY;
    if constexpr (EARLY && !kTwGlobal) {
        tw0 = twg[tw_at(0)];
        tw1 = twg[tw_at(1)];
        tw2 = twg[tw_at(2)];
        tw3 = twg[tw_at(3)];
    }
    if constexpr (EARLY && Op::PREFETCH) {
        op.prefetch(g, lc, st);
        op.prefetch_tail(g, lc, st);
    }
    // Late launches stage the twiddle table (and fetch a light transform input) before begin(), so
    // that these loads share one memory round trip with the state intake.
    constexpr bool kEarlyInput = !EARLY && Op::PREFETCH && PrefetchEarly<Op>::value;
    if constexpr (!EARLY) {
        for (int i = threadIdx.x; i < lc.M; i += blockDim.x) tw[i] = twg[i];
        if constexpr (kEarlyInput) op.prefetch(g, lc, st);
    }
    if constexpr (Op::SCALARS) {
        __shared__ Scal s_local;
        op.begin(g, lc.b, blk_in_inst, red, &s_local, in);  // all threads; ends with a barrier
        if (s_local.done) return;                       // uniform per block (one instance per block)
        lc.sc = &s_local;
    }
    if constexpr (EARLY && !kTwGlobal) {
        auto tw_put = [&](int j, C2<T> x) {
            const int i = threadIdx.x + j * blockDim.x;
            if (i < lc.M) tw[i] = x;
        };
        tw_put(0, tw0);
        tw_put(1, tw1);
        tw_put(2, tw2);
        tw_put(3, tw3);
        for (int i = threadIdx.x + kTwiddleRegs * blockDim.x; i < lc.M; i += blockDim.x) tw[i] = twg[i];
    } else if constexpr (!EARLY && !kEarlyInput) {
        if constexpr (Op::PREFETCH) op.prefetch(g, lc, st);
    }
    if constexpr (!kTwGlobal) __syncthreads();  // the LDS twiddle table is complete

    C2<T> v[8];
    double acc[Op::K > 0 ? Op::K : 1];
#pragma unroll
    for (int k = 0; k < (Op::K > 0 ? Op::K : 1); ++k) acc[k] = ((Op::MAXMASK >> k) & 1u) ? 0.0 : 0.0;

    const C2<T>* twx = kTwGlobal ? twg : tw;
    op.load(g, lc, st, v, acc);
    if (Op::FWD) line_fft<T, -1, AX, LG>(v, buf, twx, lc);
    op.template spectral<LG>(g, lc, st, v, acc, buf, twx);
    if (Op::INV) line_fft<T, +1, AX, LG>(v, buf, twx, lc);
    if constexpr (!EARLY && Op::PREFETCH) op.prefetch_tail(g, lc, st);
    op.store(g, lc, st, v, acc);

    if constexpr (Op::K > 0) {
        const int nw = (blockDim.x + 63) >> 6;
        double* outK = red + (size_t)nw * Op::K;
        block_reduce<Op::K>(acc, red, outK, Op::MAXMASK);
        double* P = pr.parts + ((size_t)lc.b * pr.row_stride() + pr.off + blk_in_inst) * Op::K;
        for (int k = threadIdx.x; k < Op::K; k += blockDim.x) P[k] = outK[k];
    }
}

}  // namespace gpe
