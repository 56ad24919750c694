// Field linear algebra shared by the linear solvers (implicit adjoint, backward Euler): inner
// products with a fixed reduction order (deterministic), copies, zeroing.
#pragma once

#include "internal.hpp"

namespace gpe {

constexpr int kDotBlocks = 256;

// Partial sums (kDotBlocks per request) of up to 4 products Re or Im of conj(a_k) b_k.
template <typename T>
struct DotReq {
    const C2<T>* a[4];
    const C2<T>* b[4];
    int imag[4];
};

template <typename T>
__global__ __launch_bounds__(256) void k_dots(DotReq<T> q, int nq, int64_t N, double* parts) {
    __shared__ double red[4 * 4];
    __shared__ double out[4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k < nq) {
                const C2<T> x = q.a[k][i], y = q.b[k][i];
                acc[k] += q.imag[k] ? (double)(x.x * y.y - x.y * y.x) : (double)(x.x * y.x + x.y * y.y);
            }
        }
    }
    block_reduce<4>(acc, red, out, 0u);
    if (threadIdx.x < 4) parts[blockIdx.x * 4 + threadIdx.x] = out[threadIdx.x];
}

// dst[k] = scale * sum over blocks (fixed order) of parts[.][k], k < 4.
static __global__ void k_dots_final(const double* parts, int nb, double scale, double* dst) {
    __shared__ double red[4 * 4];
    __shared__ double out[4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
        for (int k = 0; k < 4; ++k) acc[k] += parts[b * 4 + k];
    block_reduce<4>(acc, red, out, 0u);
    if (threadIdx.x < 4) dst[threadIdx.x] = scale * out[threadIdx.x];
}

template <typename T>
__global__ void k_copy_c(const C2<T>* a, C2<T>* b, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) b[i] = a[i];
}

template <typename T>
__global__ void k_zero_c(C2<T>* a, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) a[i] = mk((T)0, (T)0);
}

// Device state of a preconditioned linear CG (every scalar stays on the device; the host polls
// `done`).  lam, beta, cell, nphi2 are parameters of the operator of the solver using it.
struct CgS {
    double lam, beta, cell, nphi2;  // chemical potential, nonlinearity, h^d, ||phi||^2
    double rz, pq, rr, rr0, a, b;
    double tol2;
    int64_t it, max_it;
    int32_t done, status;
};

static __global__ void k_cg_alpha(CgS* S, const double* pq) {
    if (threadIdx.x != 0 || S->done) return;
    S->pq = pq[0];
    if (!(S->pq > 0.0)) {
        S->status = -1;  // the operator is not positive definite
        S->done = 1;
        return;
    }
    S->a = S->rz / S->pq;
}

template <typename T>
__global__ void k_cg_update(C2<T>* x, C2<T>* r, const C2<T>* p, const C2<T>* q, const CgS* S, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || S->done) return;
    const T a = (T)S->a;
    x[i] = add(x[i], scl(p[i], a));
    r[i] = sub(r[i], scl(q[i], a));
}

// dots = {<r, z>, <r, r>}: convergence test ||r||^2 <= tol2 * rr0 (rr0: the reference norm the
// solver set), then the CG coefficient.
static __global__ void k_cg_beta(CgS* S, const double* dots) {
    if (threadIdx.x != 0 || S->done) return;
    S->it += 1;
    S->rr = dots[1];
    if (!(dots[0] == dots[0]) || !(dots[1] == dots[1])) {
        S->status = -4;
        S->done = 1;
        return;
    }
    if (S->rr <= S->tol2 * S->rr0) {
        S->status = 0;
        S->done = 1;
        return;
    }
    if (S->it >= S->max_it) {
        S->status = 1;
        S->done = 1;
        return;
    }
    S->b = dots[0] / S->rz;
    S->rz = dots[0];
}

template <typename T>
__global__ void k_cg_dir(C2<T>* p, const C2<T>* z, const CgS* S, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || S->done) return;
    p[i] = add(z[i], scl(p[i], (T)S->b));
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// dst[k] = h^d sum conj(a_k) b_k (real part, or imaginary part where i_k), k < nq <= 2, over N points.
template <typename T>
hipError_t field_dots(int64_t N, double cell, double* parts, int nq, const C2<T>* a0, const C2<T>* b0, int i0,
                      const C2<T>* a1, const C2<T>* b1, int i1, double* dst, hipStream_t s) {
    DotReq<T> q{};
    q.a[0] = a0; q.b[0] = b0; q.imag[0] = i0;
    q.a[1] = a1 ? a1 : a0; q.b[1] = b1 ? b1 : b0; q.imag[1] = i1;
    q.a[2] = a0; q.b[2] = b0; q.a[3] = a0; q.b[3] = b0;
    hipLaunchKernelGGL(k_dots<T>, dim3(kDotBlocks), dim3(256), 0, s, q, nq, N, parts);
    hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(256), 0, s, parts, kDotBlocks, cell, dst);
    return hipGetLastError();
}

}  // namespace gpe
