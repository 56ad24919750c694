// Shared device/host definitions of libgpe: complex arithmetic, grid geometry, per-instance
// solver scalars and the deterministic block reduction used by every reducing kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpe {

// ------------------------------------------------------------------------------------------------
// Complex numbers stored interleaved (re, im); alignment gives 8/16-byte vector loads.
// ------------------------------------------------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) C2 {
    T x, y;
};

template <typename T> __host__ __device__ __forceinline__ C2<T> mk(T a, T b) { C2<T> r; r.x = a; r.y = b; return r; }
template <typename T> __host__ __device__ __forceinline__ C2<T> add(C2<T> a, C2<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T> __host__ __device__ __forceinline__ C2<T> sub(C2<T> a, C2<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T> __host__ __device__ __forceinline__ C2<T> scl(C2<T> a, T s) { return mk(a.x * s, a.y * s); }
template <typename T> __host__ __device__ __forceinline__ C2<T> mul(C2<T> a, C2<T> b) {
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T> __host__ __device__ __forceinline__ C2<T> mulc(C2<T> a, C2<T> b) {
    return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T> __host__ __device__ __forceinline__ T abs2(C2<T> a) { return a.x * a.x + a.y * a.y; }
// Re(conj(a) b)
template <typename T> __host__ __device__ __forceinline__ T redot(C2<T> a, C2<T> b) { return a.x * b.x + a.y * b.y; }
// a * (i s): multiplication by a purely imaginary number
template <typename T> __host__ __device__ __forceinline__ C2<T> muli(C2<T> a, T s) { return mk(-a.y * s, a.x * s); }

// ------------------------------------------------------------------------------------------------
// Grid geometry of one problem (Section 3).
// ------------------------------------------------------------------------------------------------
struct Geo {
    int dim;
    int n[3];       // points per axis (1 for unused axes)
    int lg[3];      // log2 of the power-of-two part of n (n = 2^lg, or 5 * 2^lg when f5)
    int f5[3];      // 1 when n = 5 * 2^lg (a radix-5 stage ends the line transform)
    int pow2;       // every axis is a power of two (the line decomposition uses shifts only)
    int b0, bl;     // a launch covers instances [b0, b0 + bl) of the B laid out (bl = 0: all of them),
                    // or, when imap is set, the bl instances imap[0 .. bl) (device, each < B); tiles and
                    // partial-row strides always follow the full B
    const int* imap;
    double L[3];    // half-widths
    double h[3];    // spacings 2L/n
    double dk[3];   // frequency spacings pi/L
    double cell;    // h^d
    int64_t N;      // points per field
};

// Frequency xi of transform index j on an axis of n points and half-width L (Nyquist kept), given
// the spacing dk = pi/L.
__device__ __forceinline__ double freq_of(int j, int n, double dk) {
    int p = (j < (n >> 1)) ? j : j - n;
    return (double)p * dk;
}
// Grid coordinate x_k = -L + k h.
__device__ __forceinline__ double coord_of(int k, double L, double h) { return -L + (double)k * h; }

// ------------------------------------------------------------------------------------------------
// Per-instance solver state (FP64).  One struct per instance, resident in device memory.
// ------------------------------------------------------------------------------------------------
struct alignas(16) Scal {
    // problem parameters (per instance: batched solves mix boxes, beta and omega)
    double beta, omega, cell;
    double L[3], h[3], dk[3];  // dk = pi/L
    // scalars of the current iterate phi_n
    double a;          // <phi, L phi>, L = T + V - omega L_z (tracked field)
    double aR;         // <phi, R phi>, R = -omega L_z
    double q4;         // h^d sum |phi|^4
    double nrm2;       // ||phi||^2
    double lam;        // lambda_n
    double lamt;       // lambda~_n (preconditioner shift)
    double E;          // E(phi_n)
    double E_prev;     // E(phi_{n-1})
    double res;        // ||r_n||_inf
    double dphi;       // ||phi_n - phi_{n-1}||_inf
    // conjugate-gradient memory
    double rPr_prev;   // <r_{n-1}, P_{n-1} r_{n-1}>
    // direction (after the preconditioner reductions)
    double beta_cg, rho, pnorm, d1, d2, rPr_cur;
    double aR_next;    // <phi_{n+1}, R phi_{n+1}> predicted by the step
    int32_t restarted, dim;
    // step (after the line search)
    double theta, c_phi, c_p, c_L, c_Lp, dE;
    // counters and flags
    int64_t n, restarts, halvings, iters_fp32;
    int32_t done, status, have_prev, linesearch_fail;  // linesearch_fail: consecutive failures
    int32_t stagnant, nonfinite, b_phase, precision;   // b_phase: direction partials are pending
    // options copied per instance
    double tol_res, tol_energy, theta_default;
    int32_t method, beta_rule, max_halvings, precond;
    int64_t max_iter;
    // stagnation tracking (mixed precision)
    double best_res, best_E;
    int64_t best_n;
    double switch_res;
    int32_t stall_window, has_step;   // has_step: a retraction step is pending (applied by phase A)
    int32_t line_search, pad0;        // 0 decrease test, 1 Armijo test, 2 full line search
    // history
    double* hist;      // device ring of rows of 8 doubles, nullable
    int64_t hist_cap;
};

enum : int { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_LINESEARCH = -5, ST_NONFINITE = -4 };

// ------------------------------------------------------------------------------------------------
// Deterministic block reduction of K doubles.  Entry k is summed, or max-reduced when bit k of
// `maxmask` is set.  Inside a full wave the K entries are reduced by a transposing butterfly: at
// each of the first log2(K') exchanges (K' = K rounded up to a power of two) a lane keeps half of
// its entries and trades the other half with its partner; after log2(64 / K') plain xor steps
// lane l holds entry l / (64 / K') summed over the wave, for K' - 1 + log2(64 / K') exchanges in
// total instead of 6 K.  Blocks whose size is not a multiple of 64 take a masked xor tree per entry (lanes beyond
// the block's last thread contribute the identity).  The waves are then combined in a fixed order.
// `red` is LDS scratch of at least (blockDim/64 + 1) * K doubles; `out` is an LDS array of K
// doubles that holds the totals for every thread on return; v is clobbered.  Must be called by
// every thread of the block, in uniform control flow.
// ------------------------------------------------------------------------------------------------
// One exchange of the transposing butterfly (HALF entries traded with the lane at distance OFF),
// then the next; template recursion keeps every register index a compile-time constant.
template <int HALF, int OFF, int KP>
__device__ __forceinline__ void butterfly_round(double (&u)[KP], int lane, int& base, unsigned maxmask) {
    if constexpr (HALF >= 1) {
        const bool up = (lane & OFF) != 0;
#pragma unroll
        for (int j = 0; j < HALF; ++j) {
            const double keep = up ? u[j + HALF] : u[j];
            const double send = up ? u[j] : u[j + HALF];
            const double recv = __shfl_xor(send, OFF, 64);
            const bool mx = (maxmask >> (base + (up ? HALF : 0) + j)) & 1u;
            u[j] = mx ? fmax(keep, recv) : keep + recv;
        }
        base += up ? HALF : 0;
        butterfly_round<HALF / 2, OFF / 2, KP>(u, lane, base, maxmask);
    }
}

template <int K>
__device__ __forceinline__ void block_reduce(double (&v)[K], double* red, double* out, unsigned maxmask) {
    static_assert(K >= 1 && K <= 64, "block_reduce handles 1..64 entries");
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    if ((blockDim.x & 63u) == 0) {
        constexpr int KP = K <= 1 ? 1 : K <= 2 ? 2 : K <= 4 ? 4 : K <= 8 ? 8 : K <= 16 ? 16 : K <= 32 ? 32 : 64;
        double u[KP];
#pragma unroll
        for (int k = 0; k < KP; ++k) u[k] = k < K ? v[k] : 0.0;  // padding entries are sums of zeros
        int base = 0;  // first entry index still held by this lane
        butterfly_round<KP / 2, 32>(u, lane, base, maxmask);
        const bool mx = (maxmask >> base) & 1u;
#pragma unroll
        for (int off = 32 / KP; off >= 1; off >>= 1) {
            const double o = __shfl_xor(u[0], off, 64);
            u[0] = mx ? fmax(u[0], o) : u[0] + o;
        }
        __syncthreads();
        if ((lane & (64 / KP - 1)) == 0 && base < K) red[wave * K + base] = u[0];
    } else {
        const int nact = min(64, (int)blockDim.x - wave * 64);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = v[k];
            const bool mx = (maxmask >> k) & 1u;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                double o = __shfl_xor(s, off, 64);
                if ((lane ^ off) >= nact) o = mx ? -1e300 : 0.0;
                s = mx ? fmax(s, o) : s + o;
            }
            v[k] = s;
        }
        __syncthreads();
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) red[wave * K + k] = v[k];
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const bool mx = (maxmask >> k) & 1u;
        double s = red[k];
        for (int w = 1; w < nw; ++w) {
            const double o = red[w * K + k];
            s = mx ? fmax(s, o) : s + o;
        }
        out[k] = s;
    }
    __syncthreads();
}

// "Last block done" ticket: every block calls this after writing its partials.  Returns true in
// exactly one block (the last to arrive), after resetting the counter for the next launch, so
// the pattern survives graph replays.  All threads of the block get the same answer.
__device__ __forceinline__ bool last_block(unsigned int* counter, unsigned int nblocks, int* lds_flag) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int ticket = atomicAdd(counter, 1u);
        int last = (ticket == nblocks - 1u);
        if (last) atomicExch(counter, 0u);
        *lds_flag = last;
    }
    __syncthreads();
    bool last = *lds_flag != 0;
    if (last) __threadfence();
    return last;
}

}  // namespace gpe
