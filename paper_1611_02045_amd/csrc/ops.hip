// Standalone operators of the solver as chains of directional passes:
//   * H_phi phi and L f = (T + V - omega L_z) f            (Sections 2-3)
//   * the energy E(phi) and its parts                     (Section 2)
//   * the preconditioners P_Delta, P_V, P_C, P_C1, P_C2   (Section 5.5)
#include <cmath>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"

namespace gpe {

// Rotation coefficient of the directional symbol along AX for the line (i1, i2):
// R = -omega L_z = i omega (x d_y - y d_x) acts as +omega y xi along x and -omega x mu along y.
template <int AX>
__device__ __forceinline__ double rot_coef(const Geo& g, const LineCtx& lc, double omega) {
    if (g.dim < 2 || omega == 0.0) return 0.0;
    if (AX == 0) return omega * coord_of(lc.i1, g.L[1], g.h[1]);
    if (AX == 1) return -omega * coord_of(lc.i1, g.L[0], g.h[0]);
    return 0.0;
}

// ---------------------------------------------------------------------------------------------
// Directional part of L (and H): out = acc + F_a^{-1}[sigma_a F_a f], sigma_a = xi^2/2 + rot*xi,
// and on the pass with `pointwise` set also + (V + beta|f|^2) f (beta term only for the
// nonlinear H).  The pointwise part goes with the x pass, where V is read contiguously; the
// strided passes then read only f and the running sum.
// ---------------------------------------------------------------------------------------------
template <typename T, int AX>
struct OpApply {
    static constexpr bool FWD = true, INV = true, SCALARS = false, PREFETCH = false, WIDE = false;
    static constexpr int K = 0;
    static constexpr unsigned MAXMASK = 0;
    const C2<T>* f;
    const C2<T>* acc;  // nullable
    C2<T>* out;
    const T* V;        // used by the pass with `pointwise` set
    double beta, omega;
    int pointwise, nonlinear;
    double kin = 1.0;  // weight of the kinetic symbol (0: rotation part only)
    // only the x pass carries the pointwise part: the strided passes keep no copy of f
    static constexpr bool PW = AX == 0;
    struct State { C2<T> f0[PW ? 8 : 1]; };
    __device__ void load(const Geo&, const LineCtx& lc, State& st, C2<T> (&v)[8], double (&acc)[K > 0 ? K : 1]) const {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            v[s] = f[lc.at(s)];
            if constexpr (PW) st.f0[s] = v[s];
        }
    }
    template <int LG>
    __device__ void spectral(const Geo& g, const LineCtx& lc, State&, C2<T> (&v)[8], double (&)[1], C2<T>*,
                             const C2<T>*) const {
        const double rot = rot_coef<AX>(g, lc, omega);
        const double inv = 1.0 / lc.M;  // 1/M (exact for M = 2^k)
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const double xi = freq_of(lc.k(s), lc.M, g.dk[AX]);
            v[s] = scl(v[s], (T)((0.5 * kin * xi * xi + rot * xi) * inv));
        }
    }
    __device__ void store(const Geo&, const LineCtx& lc, State& st, C2<T> (&v)[8], double (&)[1]) const {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int64_t i = lc.at(s);
            C2<T> o = v[s];
            if (acc) o = add(o, acc[i]);
            if constexpr (PW) {
                if (pointwise && V) {
                    T w = V[i - lc.off_b];
                    if (nonlinear) w += (T)beta * abs2(st.f0[s]);
                    o = add(o, scl(st.f0[s], w));
                }
            }
            out[i] = o;
        }
    }
};

template <typename T>
static hipError_t apply_t(const Geo& g, int B, const Twiddles& tw, const void* f, const void* V, void* out,
                          void* tmp, double beta, double omega, bool nl, hipStream_t s) {
    const bool f64 = sizeof(T) == 8;
    const C2<T>* F = (const C2<T>*)f;
    Partials none{nullptr, 0, 0, 0};
    hipError_t e;
    if (g.dim == 1) {
        OpApply<T, 0> op{F, nullptr, (C2<T>*)out, (const T*)V, beta, omega, 1, nl};
        return launch_pass<T, 0>(g, B, tw.get(0, f64), op, none, s);
    }
    if (plane_preferred(g, f64, B)) {
        // whole xy-planes in LDS: all of H f in 2-D; in 3-D the xy-part into tmp, then the z pass
        if (g.dim == 2) return op_apply_plane(g, f64, B, tw, f, V, out, beta, omega, nl, s);
        if ((e = op_apply_plane(g, f64, B, tw, f, V, tmp, beta, omega, nl, s)) != hipSuccess) return e;
        OpApply<T, 2> oz{F, (const C2<T>*)tmp, (C2<T>*)out, nullptr, beta, omega, 0, nl};
        return launch_pass<T, 2>(g, B, tw.get(2, f64), oz, none, s);
    }
    // x-pass (with the pointwise part) into tmp, then the y (and z) passes accumulate.
    OpApply<T, 0> ox{F, nullptr, (C2<T>*)tmp, (const T*)V, beta, omega, 1, nl};
    if ((e = launch_pass<T, 0>(g, B, tw.get(0, f64), ox, none, s)) != hipSuccess) return e;
    if (g.dim == 2) {
        OpApply<T, 1> oy{F, (const C2<T>*)tmp, (C2<T>*)out, nullptr, beta, omega, 0, nl};
        return launch_pass<T, 1>(g, B, tw.get(1, f64), oy, none, s);
    }
    OpApply<T, 1> oy{F, (const C2<T>*)tmp, (C2<T>*)tmp, nullptr, beta, omega, 0, nl};
    if ((e = launch_pass<T, 1>(g, B, tw.get(1, f64), oy, none, s)) != hipSuccess) return e;
    OpApply<T, 2> oz{F, (const C2<T>*)tmp, (C2<T>*)out, nullptr, beta, omega, 0, nl};
    return launch_pass<T, 2>(g, B, tw.get(2, f64), oz, none, s);
}

// out = R f with R = -L_z (rotation symbol with omega = 1, no kinetic, no potential); dim >= 2.
template <typename T>
static hipError_t rotation_t(const Geo& g, const Twiddles& tw, const void* f, void* out, void* tmp, hipStream_t s) {
    const bool f64 = sizeof(T) == 8;
    const C2<T>* F = (const C2<T>*)f;
    Partials none{nullptr, 0, 0, 0};
    hipError_t e;
    OpApply<T, 0> ox{F, nullptr, (C2<T>*)tmp, nullptr, 0.0, 1.0, 0, 0, 0.0};
    if ((e = launch_pass<T, 0>(g, 1, tw.get(0, f64), ox, none, s)) != hipSuccess) return e;
    // the y pass completes R (no z part in 3-D: L_z acts in the xy-planes)
    OpApply<T, 1> oy{F, (const C2<T>*)tmp, (C2<T>*)out, nullptr, 0.0, 1.0, 1, 0, 0.0};
    return launch_pass<T, 1>(g, 1, tw.get(1, f64), oy, none, s);
}

hipError_t op_rotation(const Geo& g, bool f64, const Twiddles& tw, const void* f, void* out, void* tmp, hipStream_t s) {
    return f64 ? rotation_t<double>(g, tw, f, out, tmp, s) : rotation_t<float>(g, tw, f, out, tmp, s);
}

hipError_t op_apply(const Geo& g, bool f64, int B, const Twiddles& tw, const void* f, const void* V, void* out,
                    void* tmp, double beta, double omega, bool nonlinear, hipStream_t s) {
    return f64 ? apply_t<double>(g, B, tw, f, V, out, tmp, beta, omega, nonlinear, s)
               : apply_t<float>(g, B, tw, f, V, out, tmp, beta, omega, nonlinear, s);
}

// ---------------------------------------------------------------------------------------------
// Interpolation onto the grid with twice the points per axis and the same box (the nested grids
// of Section 6), one axis per pass, by the trigonometric interpolant of the discretisation with
// the Nyquist coefficient split evenly between the frequencies -M/2 and +M/2.  At the coarse
// points the interpolant is the input itself; at the midpoints x_j + h/2 it is the input shifted
// by half a cell, F^{-1}[e^{i pi p / M} F f] over -M/2 < p < M/2, the split Nyquist pair adding
// cos(pi/2) = 0 there.  The pass writes both: out[2j] = f[j], out[2j + 1] = the shifted value.
// The pass geometry is the source's (axes before AX already doubled); out has twice its points.
// ---------------------------------------------------------------------------------------------
template <typename T, int AX>
struct OpProlong {
    static constexpr bool FWD = true, INV = true, SCALARS = false, PREFETCH = false, WIDE = false;
    static constexpr int K = 0;
    static constexpr unsigned MAXMASK = 0;
    const C2<T>* f;
    C2<T>* out;
    double hr, hi;  // e^{i pi / M} (host FP64) for the pass's line length M
    struct State {};
    __device__ void load(const Geo&, const LineCtx& lc, State&, C2<T> (&v)[8], double (&)[1]) const {
#pragma unroll
        for (int s = 0; s < 8; ++s) v[s] = f[lc.at(s)];
    }
    // e^{i pi p / M} from the transform's table tw[e] = e^{-2 pi i e / M}: conj(tw[floor(p/2) mod M]),
    // times e^{i pi / M} for odd p.
    template <int LG>
    __device__ void spectral(const Geo&, const LineCtx& lc, State&, C2<T> (&v)[8], double (&)[1], C2<T>*,
                             const C2<T>* tw) const {
        const T inv = (T)(1.0 / lc.M);  // 1/M (exact for M = 2^k)
        const C2<T> half{(T)hr, (T)hi};
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int j = lc.k(s);
            const int p = j < (lc.M >> 1) ? j : j - lc.M;
            if (2 * p == -lc.M) {
                v[s] = C2<T>{(T)0, (T)0};
            } else {
                const int q = (p - (p & 1)) >> 1;
                const C2<T> t = tw[q < 0 ? q + lc.M : q];
                C2<T> m{t.x, -t.y};
                if (p & 1) m = mul(m, half);
                v[s] = scl(mul(v[s], m), inv);
            }
        }
    }
    __device__ void store(const Geo& g, const LineCtx& lc, State&, C2<T> (&v)[8], double (&)[1]) const {
        // source offset s (within its instance) -> even output offset: x: 2s; y: 2s - x;
        // z: 2s - (y n_x + x); the odd neighbour is one output step further along AX.
        const int64_t nx = g.n[0], nxy = (int64_t)g.n[0] * g.n[1];
        const int64_t keep = AX == 0 ? 0 : (AX == 1 ? (int64_t)lc.i1 : (int64_t)lc.i2 * nx + lc.i1);
        const int64_t step = AX == 0 ? 1 : (AX == 1 ? nx : nxy);
        C2<T>* o = out + 2 * lc.off_b;
        const int64_t e0 = 2 * (lc.at(0) - lc.off_b) - keep;  // the points of a thread are TPL apart
        const int64_t de = 2 * (int64_t)lc.TPL * lc.stride;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            o[e0 + s * de] = f[lc.at(s)];  // re-read (cached): keeping the inputs across the transforms
            o[e0 + s * de + step] = v[s];  // put them in scratch memory in FP64
        }
    }
};

// g with axes [0, upto) doubled (the geometry of the source of the pass along `upto`).
static Geo doubled_upto(const Geo& g, int upto) {
    Geo d = g;
    for (int a = 0; a < upto; ++a) {
        d.n[a] *= 2;
        d.lg[a] += 1;
        d.N *= 2;
        d.h[a] *= 0.5;
        d.cell *= 0.5;
    }
    return d;
}

template <typename T, int AX>
static OpProlong<T, AX> prolong_op(const Geo& g, const C2<T>* src, C2<T>* dst) {
    const double a = 3.141592653589793238462643383279502884 / g.n[AX];
    return OpProlong<T, AX>{src, dst, std::cos(a), std::sin(a)};
}

template <typename T>
static hipError_t prolong_t(const Geo& g, const Twiddles& tw, const void* in, void* out, void* tmp, hipStream_t s) {
    const bool f64 = sizeof(T) == 8;
    Partials none{nullptr, 0, 0, 0};
    hipError_t e;
    const C2<T>* src = (const C2<T>*)in;
    C2<T>* dst = (C2<T>*)out;
    C2<T>* t = (C2<T>*)tmp;
    if (g.dim == 1) return launch_pass<T, 0>(g, 1, tw.get(0, f64), prolong_op<T, 0>(g, src, dst), none, s);
    // 2-D: x into tmp (2N), y into out.  3-D: x into the last quarter of out, y into tmp (4N),
    // z into out (the x result is dead by then; passes on one stream run in order).
    C2<T>* xo = g.dim == 2 ? t : dst + 6 * g.N;
    if ((e = launch_pass<T, 0>(g, 1, tw.get(0, f64), prolong_op<T, 0>(g, src, xo), none, s)) != hipSuccess) return e;
    const Geo g1 = doubled_upto(g, 1);
    if (g.dim == 2) return launch_pass<T, 1>(g1, 1, tw.get(1, f64), prolong_op<T, 1>(g1, xo, dst), none, s);
    if ((e = launch_pass<T, 1>(g1, 1, tw.get(1, f64), prolong_op<T, 1>(g1, xo, t), none, s)) != hipSuccess) return e;
    const Geo g2 = doubled_upto(g, 2);
    return launch_pass<T, 2>(g2, 1, tw.get(2, f64), prolong_op<T, 2>(g2, t, dst), none, s);
}

hipError_t op_prolong(const Geo& g, bool f64, const Twiddles& tw, const void* in, void* out, void* tmp, hipStream_t s) {
    return f64 ? prolong_t<double>(g, tw, in, out, tmp, s) : prolong_t<float>(g, tw, in, out, tmp, s);
}

// ---------------------------------------------------------------------------------------------
// Tile measurement: for each axis, the directional pass (forward transform, kinetic multiplier,
// inverse transform, store) over B fields is timed for every valid number of lines per workgroup,
// and the fastest is recorded for the grid, point size and batch size.
// ---------------------------------------------------------------------------------------------
template <typename T, int AX>
static hipError_t tune_axis(const Geo& g, int B, const Twiddles& tw, const C2<T>* f, C2<T>* out, hipStream_t s,
                            int& best_C, double& best_us) {
    const int cb = (int)sizeof(C2<T>);
    const int TPL = g.n[AX] / 8;
    OpApply<T, AX> op{f, nullptr, out, nullptr, 0.0, 0.0, 0, 0};
    Partials none{nullptr, 0, 0, 0};
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) return e;
    best_C = 0;
    best_us = 0.0;
    // whole waves where the grid allows it (a partial wave idles lanes)
    int Cmin = 1;
    while (Cmin * TPL < 64 && valid_lines(g, AX, cb, 2 * Cmin)) Cmin *= 2;
    for (int C = Cmin; C * TPL <= 256 && e == hipSuccess; C *= 2) {
        if (!valid_lines(g, AX, cb, C)) continue;
        constexpr int kWarm = 2, kReps = 10;
        for (int r = 0; r < kWarm && e == hipSuccess; ++r) e = launch_pass<T, AX>(g, B, tw.get(AX, sizeof(T) == 8), op, none, s, nullptr, C);
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < kReps && e == hipSuccess; ++r) e = launch_pass<T, AX>(g, B, tw.get(AX, sizeof(T) == 8), op, none, s, nullptr, C);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        const double us = 1e3 * ms / kReps;
        if (e == hipSuccess && (best_C == 0 || us < best_us)) {
            best_C = C;
            best_us = us;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e == hipSuccess && best_C > 0) record_tuned_lines(g, AX, cb, B, best_C);
    return e;
}

template <typename T>
static hipError_t autotune_t(const Geo& g, int B, const Twiddles& tw, void* f, void* out, hipStream_t s, int tiles[3],
                             double us[3]) {
    const C2<T>* F = (const C2<T>*)f;
    C2<T>* O = (C2<T>*)out;
    hipError_t e = tune_axis<T, 0>(g, B, tw, F, O, s, tiles[0], us[0]);
    if (e == hipSuccess && g.dim > 1) e = tune_axis<T, 1>(g, B, tw, F, O, s, tiles[1], us[1]);
    if (e == hipSuccess && g.dim > 2) e = tune_axis<T, 2>(g, B, tw, F, O, s, tiles[2], us[2]);
    return e;
}

hipError_t op_autotune(const Geo& g, bool f64, int B, const Twiddles& tw, void* f, void* out, hipStream_t s,
                       int tiles[3], double us[3]) {
    return f64 ? autotune_t<double>(g, B, tw, f, out, s, tiles, us) : autotune_t<float>(g, B, tw, f, out, s, tiles, us);
}

// ---------------------------------------------------------------------------------------------
// Energy: forward transforms only; Parseval turns <phi, F^{-1} sigma F phi> into
// (1/M) sum sigma |F phi|^2 per line.  Sums: {kinetic, rotation, potential, quartic}.
// ---------------------------------------------------------------------------------------------
template <typename T, int AX>
struct OpEnergy {
    static constexpr bool FWD = true, INV = false, SCALARS = false, PREFETCH = false, WIDE = false;
    static constexpr int K = 4;
    static constexpr unsigned MAXMASK = 0;
    const C2<T>* phi;
    const T* V;
    double omega;
    struct State { C2<T> f0[8]; };
    __device__ void load(const Geo&, const LineCtx& lc, State& st, C2<T> (&v)[8], double (&acc)[K > 0 ? K : 1]) const {
#pragma unroll
        for (int s = 0; s < 8; ++s) st.f0[s] = v[s] = phi[lc.at(s)];
    }
    template <int LG>
    __device__ void spectral(const Geo& g, const LineCtx& lc, State&, C2<T> (&v)[8], double (&acc)[4], C2<T>*,
                             const C2<T>*) const {
        const double rot = rot_coef<AX>(g, lc, omega);
        const double inv = 1.0 / lc.M;  // 1/M (exact for M = 2^k)
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const double xi = freq_of(lc.k(s), lc.M, g.dk[AX]);
            const double w = (double)abs2(v[s]) * inv;
            acc[0] += 0.5 * xi * xi * w;
            acc[1] += rot * xi * w;
        }
    }
    __device__ void store(const Geo&, const LineCtx& lc, State& st, C2<T> (&)[8], double (&acc)[4]) const {
        if (AX != 0) return;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int64_t i = lc.at(s);
            const double r = (double)abs2(st.f0[s]);
            acc[2] += (double)V[i] * r;
            acc[3] += r * r;
        }
    }
};

// Sum the per-block partials of up to three passes and scale into {kin, pot, inter, rot}.
__global__ void k_energy_collect(const double* p0, int n0, const double* p1, int n1, const double* p2, int n2,
                                 double cell, double beta, double* dst) {
    __shared__ double red[16 * 4 + 8];
    double v[4] = {0, 0, 0, 0};
    const double* ps[3] = {p0, p1, p2};
    const int ns[3] = {n0, n1, n2};
    for (int q = 0; q < 3; ++q) {
        if (!ps[q]) continue;
        for (int blk = threadIdx.x; blk < ns[q]; blk += blockDim.x)
            for (int k = 0; k < 4; ++k) v[k] += ps[q][(size_t)blk * 4 + k];
    }
    __shared__ double T4[4];
    block_reduce<4>(v, red, T4, 0u);
    if (threadIdx.x == 0) {
        dst[0] = cell * T4[0];               // <phi, T phi>
        dst[1] = cell * T4[2];               // <phi, V phi>
        dst[2] = 0.5 * beta * cell * T4[3];  // beta/2 h^d sum |phi|^4
        dst[3] = cell * T4[1];               // <phi, R phi> = -omega Re<phi, L_z phi>
    }
}

template <typename T>
static hipError_t energy_t(const Geo& g, const Twiddles& tw, const void* phi, const void* V, double beta,
                           double omega, Reduce& red, double* dst, hipStream_t s) {
    const bool f64 = sizeof(T) == 8;
    const int cb = (int)sizeof(C2<T>);
    const C2<T>* P = (const C2<T>*)phi;
    double* parts = (double*)red.parts.ptr;
    size_t off = 0;
    const double* pp[3] = {nullptr, nullptr, nullptr};
    int nn[3] = {0, 0, 0};
    hipError_t e;
    for (int ax = 0; ax < g.dim; ++ax) {
        Partials pr{parts + off, 0, 0, 0};
        const int nb = pass_blocks_per_field(g, ax, cb, 1, false);
        if (ax == 0) e = launch_pass<T, 0>(g, 1, tw.get(0, f64), OpEnergy<T, 0>{P, (const T*)V, omega}, pr, s);
        else if (ax == 1) e = launch_pass<T, 1>(g, 1, tw.get(1, f64), OpEnergy<T, 1>{P, (const T*)V, omega}, pr, s);
        else e = launch_pass<T, 2>(g, 1, tw.get(2, f64), OpEnergy<T, 2>{P, (const T*)V, omega}, pr, s);
        if (e != hipSuccess) return e;
        pp[ax] = parts + off;
        nn[ax] = nb;
        off += (size_t)nb * 4;
    }
    hipLaunchKernelGGL(k_energy_collect, dim3(1), dim3(256), 0, s, pp[0], nn[0], pp[1], nn[1], pp[2], nn[2],
                       g.cell, beta, dst);
    return hipGetLastError();
}

hipError_t op_energy(const Geo& g, bool f64, const Twiddles& tw, const void* phi, const void* V, double beta,
                     double omega, Reduce& red, double* dst, hipStream_t s) {
    return f64 ? energy_t<double>(g, tw, phi, V, beta, omega, red, dst, s)
               : energy_t<float>(g, tw, phi, V, beta, omega, red, dst, s);
}

__global__ void k_lambda_tilde(const double* parts, double* dst) {
    if (threadIdx.x == 0) *dst = parts[0] + parts[1] + 2.0 * parts[2];
}

hipError_t op_lambda_tilde(const double* parts, double* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_lambda_tilde, dim3(1), dim3(64), 0, s, parts, dst);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Preconditioners.  Scaling kinds: 0 none, 1 by (alpha + V + beta|phi|^2)^{-1/2}, 2 by its inverse.
// The spectral multiplier 1/(alpha + |k|^2/2) (with the 1/N of the inverse transforms) is applied
// in the pass that does both the forward and the inverse transform (the last axis).
// ---------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T pv_scale(int kind, double alpha, T V, T rho, double beta) {
    const double d = alpha + (double)V + beta * (double)rho;
    return kind == 1 ? (T)(1.0 / sqrt(d)) : (T)(1.0 / d);
}

template <typename T, int AX, bool F, bool I>
struct OpPre {
    static constexpr bool FWD = F, INV = I, SCALARS = false, PREFETCH = false, WIDE = false;
    static constexpr int K = 0;
    static constexpr unsigned MAXMASK = 0;
    const C2<T>* in;
    C2<T>* out;
    const C2<T>* phi;
    const T* V;
    const double* alpha;
    double beta;
    int pre, post;
    struct State {};
    __device__ void load(const Geo&, const LineCtx& lc, State&, C2<T> (&v)[8], double (&acc)[K > 0 ? K : 1]) const {
        const double a = *alpha;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int64_t i = lc.at(s);
            v[s] = in[i];
            if (pre) v[s] = scl(v[s], pv_scale<T>(pre, a, V[i], abs2(phi[i]), beta));
        }
    }
    template <int LG>
    __device__ void spectral(const Geo& g, const LineCtx& lc, State&, C2<T> (&v)[8], double (&)[1], C2<T>*,
                             const C2<T>*) const {
        if (!(F && I)) return;
        const double a = *alpha;
        // frequencies of the other (already transformed) axes
        double ko = 0.0;
        if (AX == 1) {
            const double xi = freq_of(lc.i1, g.n[0], g.dk[0]);
            ko = xi * xi;
        } else if (AX == 2) {
            const double xi = freq_of(lc.i1, g.n[0], g.dk[0]);
            const double mu = freq_of(lc.i2, g.n[1], g.dk[1]);
            ko = xi * xi + mu * mu;
        }
        const double invN = 1.0 / (double)g.N;  // 1/N (exact for powers of two)
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const double k = freq_of(lc.k(s), lc.M, g.dk[AX]);
            v[s] = scl(v[s], (T)(invN / (a + 0.5 * (ko + k * k))));
        }
    }
    __device__ void store(const Geo&, const LineCtx& lc, State&, C2<T> (&v)[8], double (&)[1]) const {
        const double a = post ? *alpha : 0.0;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int64_t i = lc.at(s);
            C2<T> o = v[s];
            if (post) o = scl(o, pv_scale<T>(post, a, V[i], abs2(phi[i]), beta));
            out[i] = o;
        }
    }
};

template <typename T>
__global__ void k_precond_diag(const C2<T>* r, C2<T>* out, const C2<T>* phi, const T* V, const double* alpha,
                               double beta, int kind, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    C2<T> v = r[i];
    if (kind == GPE_P_POTENTIAL) v = scl(v, pv_scale<T>(2, *alpha, V[i], abs2(phi[i]), beta));
    out[i] = v;
}

// Full multi-dimensional P_Delta with pre/post scalings: x forward, middle axes, x inverse.
template <typename T>
static hipError_t kinetic_chain(const Geo& g, const Twiddles& tw, const C2<T>* r, C2<T>* out, C2<T>* tmp,
                                const C2<T>* phi, const T* V, const double* alpha, double beta, int pre,
                                int post, hipStream_t s) {
    const bool f64 = sizeof(T) == 8;
    Partials none{nullptr, 0, 0, 0};
    hipError_t e;
    if (g.dim == 1) {
        OpPre<T, 0, true, true> op{r, out, phi, V, alpha, beta, pre, post};
        return launch_pass<T, 0>(g, 1, tw.get(0, f64), op, none, s);
    }
    OpPre<T, 0, true, false> x1{r, tmp, phi, V, alpha, beta, pre, 0};
    if ((e = launch_pass<T, 0>(g, 1, tw.get(0, f64), x1, none, s)) != hipSuccess) return e;
    if (g.dim == 2) {
        OpPre<T, 1, true, true> y{tmp, tmp, phi, V, alpha, beta, 0, 0};
        if ((e = launch_pass<T, 1>(g, 1, tw.get(1, f64), y, none, s)) != hipSuccess) return e;
    } else {
        OpPre<T, 1, true, false> y1{tmp, tmp, phi, V, alpha, beta, 0, 0};
        if ((e = launch_pass<T, 1>(g, 1, tw.get(1, f64), y1, none, s)) != hipSuccess) return e;
        OpPre<T, 2, true, true> z{tmp, tmp, phi, V, alpha, beta, 0, 0};
        if ((e = launch_pass<T, 2>(g, 1, tw.get(2, f64), z, none, s)) != hipSuccess) return e;
        OpPre<T, 1, false, true> y2{tmp, tmp, phi, V, alpha, beta, 0, 0};
        if ((e = launch_pass<T, 1>(g, 1, tw.get(1, f64), y2, none, s)) != hipSuccess) return e;
    }
    OpPre<T, 0, false, true> x2{tmp, out, phi, V, alpha, beta, 0, post};
    return launch_pass<T, 0>(g, 1, tw.get(0, f64), x2, none, s);
}

template <typename T>
static hipError_t precond_t(const Geo& g, const Twiddles& tw, int kind, const void* phi, const void* V,
                            const double* alpha, double beta, const void* r, void* out, void* tmp, hipStream_t s) {
    const C2<T>* R = (const C2<T>*)r;
    C2<T>* O = (C2<T>*)out;
    const C2<T>* P = (const C2<T>*)phi;
    const T* Vt = (const T*)V;
    if (kind == GPE_P_NONE || kind == GPE_P_POTENTIAL) {
        const int64_t N = g.N;
        hipLaunchKernelGGL(k_precond_diag<T>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, R, O, P, Vt, alpha,
                           beta, kind, N);
        return hipGetLastError();
    }
    int pre = 0, post = 0;
    if (kind == GPE_P_COMBINED) pre = post = 1;  // P_V^{1/2} P_Delta P_V^{1/2}
    if (kind == GPE_P_C1) post = 2;              // P_V P_Delta
    if (kind == GPE_P_C2) pre = 2;               // P_Delta P_V
    return kinetic_chain<T>(g, tw, R, O, (C2<T>*)tmp, P, Vt, alpha, beta, pre, post, s);
}

hipError_t op_precond(const Geo& g, bool f64, const Twiddles& tw, int kind, const void* phi, const void* V,
                      const double* alpha_dev, double beta, const void* r, void* out, void* tmp, hipStream_t s) {
    return f64 ? precond_t<double>(g, tw, kind, phi, V, alpha_dev, beta, r, out, tmp, s)
               : precond_t<float>(g, tw, kind, phi, V, alpha_dev, beta, r, out, tmp, s);
}

// Minimum of alpha + V + beta |phi|^2 (SPD check of P_V), two-level deterministic reduction.
template <typename T>
__global__ void k_min_diag(const C2<T>* phi, const T* V, const double* alpha, double beta, int64_t N,
                           double* parts) {
    __shared__ double red[16 + 4];
    double m[1] = {1e300};
    const double a = *alpha;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        m[0] = fmin(m[0], a + (double)V[i] + beta * (double)abs2(phi[i]));
    m[0] = -m[0];
    __shared__ double o1[1];
    block_reduce<1>(m, red, o1, 1u);
    if (threadIdx.x == 0) parts[blockIdx.x] = -o1[0];
}

__global__ void k_min_collect(const double* parts, int n, double* dst) {
    if (threadIdx.x == 0) {
        double m = parts[0];
        for (int i = 1; i < n; ++i) m = fmin(m, parts[i]);
        *dst = m;
    }
}

hipError_t op_min_diag(const Geo& g, bool f64, const void* phi, const void* V, const double* alpha_dev,
                       double beta, Reduce& red, double* dst, hipStream_t s) {
    const int blocks = 256;
    double* parts = (double*)red.parts.ptr;
    if (f64)
        hipLaunchKernelGGL(k_min_diag<double>, dim3(blocks), dim3(256), 0, s, (const C2<double>*)phi,
                           (const double*)V, alpha_dev, beta, g.N, parts);
    else
        hipLaunchKernelGGL(k_min_diag<float>, dim3(blocks), dim3(256), 0, s, (const C2<float>*)phi,
                           (const float*)V, alpha_dev, beta, g.N, parts);
    hipLaunchKernelGGL(k_min_collect, dim3(1), dim3(64), 0, s, parts, blocks, dst);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Small pointwise helpers.
// ---------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_scale_complex(C2<T>* x, T s, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = scl(x[i], s);
}

template <typename T>
__global__ void k_density(const C2<T>* phi, T* out, T scale, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = scale * abs2(phi[i]);
}

hipError_t op_scale_complex(const Geo&, bool f64, void* x, double s, int64_t count, hipStream_t st) {
    const unsigned blocks = (unsigned)((count + 255) / 256);
    if (f64) hipLaunchKernelGGL(k_scale_complex<double>, dim3(blocks), dim3(256), 0, st, (C2<double>*)x, s, count);
    else hipLaunchKernelGGL(k_scale_complex<float>, dim3(blocks), dim3(256), 0, st, (C2<float>*)x, (float)s, count);
    return hipGetLastError();
}

hipError_t op_density(const Geo& g, bool f64, const void* phi, void* out, double scale, hipStream_t s) {
    const unsigned blocks = (unsigned)((g.N + 255) / 256);
    if (f64)
        hipLaunchKernelGGL(k_density<double>, dim3(blocks), dim3(256), 0, s, (const C2<double>*)phi, (double*)out,
                           scale, g.N);
    else
        hipLaunchKernelGGL(k_density<float>, dim3(blocks), dim3(256), 0, s, (const C2<float>*)phi, (float*)out,
                           (float)scale, g.N);
    return hipGetLastError();
}

}  // namespace gpe
