// Implicit adjoint of a converged ground state (second-order conditions of Section 2).
//
// At a ground state phi* (H phi* = lambda phi*, ||phi*|| = 1) the tangent linearisation of the
// stationarity condition is A dphi = -Pi (d_theta H) phi* dtheta with
//   A = Pi (1/2 nabla^2 E(phi*) - lambda) Pi,   1/2 nabla^2 E[f] = H f + 2 beta Re(conj(phi) f) phi,
// on {phi*, i phi*}^perp in the real inner product Re<.,.> (the sphere's normal and the global
// phase, a null direction of the Hessian, are projected out; A is SPD there at a local minimum).
// For a loss with d l = Re<g, d phi>, the adjoint state mu solves A mu = Pi g and
// d l / d theta = -Re<mu, (d_theta H) phi*> (plus the loss's own explicit dependence).
// The solve is linear preconditioned CG with the projected combined preconditioner Pi P_C Pi;
// every CG scalar lives in device memory, so iterations are queued without host round trips
// and the host only polls a convergence flag.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>

#include "internal.hpp"
#include "plan.hpp"
#include "linear.hpp"

namespace gpe {


// f <- f - (c0 phi + c1 i phi) / ||phi||^2 with c = {Re<phi,f>, Re<i phi,f>} (device).
template <typename T>
__global__ void k_project(C2<T>* f, const C2<T>* phi, const double* c, const CgS* S, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const T c0 = (T)(c[0] / S->nphi2), c1 = (T)(c[1] / S->nphi2);
    const C2<T> p = phi[i];
    // c0 phi + c1 (i phi) = (c0 p.x - c1 p.y, c0 p.y + c1 p.x)
    f[i] = mk(f[i].x - (c0 * p.x - c1 * p.y), f[i].y - (c0 * p.y + c1 * p.x));
}

// q <- q + beta |phi|^2 p + 2 beta Re(conj(phi) p) phi - lambda p  (q holds L p on entry).
template <typename T>
__global__ void k_hessian(C2<T>* q, const C2<T>* p, const C2<T>* phi, const CgS* S, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const C2<T> ph = phi[i], pv = p[i];
    const T beta = (T)S->beta, lam = (T)S->lam;
    const T w = beta * abs2(ph) - lam;
    const T re2 = (T)2 * beta * redot(ph, pv);
    q[i] = add(add(q[i], scl(pv, w)), scl(ph, re2));
}





__global__ void k_adj_init(CgS* S, const double* dots, const double* nphi) {
    if (threadIdx.x != 0) return;
    S->rz = dots[0];
    S->rr0 = dots[1];
    S->rr = dots[1];
    S->nphi2 = nphi[0];
    if (!(S->rr0 > 0.0)) S->done = 1;  // zero right-hand side: mu = 0
}

// grad_V = -h^d Re(conj(mu) phi) (the adjoint part of dl/dV_k).
template <typename T>
__global__ void k_grad_V(const C2<T>* mu, const C2<T>* phi, T* gV, T cell, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) gV[i] = -cell * redot(mu[i], phi[i]);
}

// v = |phi|^2 phi (the field (d_beta H) phi).
template <typename T>
__global__ void k_cubic(const C2<T>* phi, C2<T>* v, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) v[i] = scl(phi[i], abs2(phi[i]));
}


template <typename T>
struct AdjCtx {
    const Geo* g;
    const Twiddles* tw;
    const C2<T>* phi;
    const T* V;
    double beta, omega;
    CgS* S;
    double* parts;  // kDotBlocks * 4
    double* sc;     // device scalars: [0..3] dots, [4..7] projection coefficients, [8] alpha, [9] ||phi||^2
    C2<T>*x, *r, *z, *p, *q, *w;
    hipStream_t s;
};

template <typename T>
static hipError_t dots(AdjCtx<T>& c, int nq, const C2<T>* a0, const C2<T>* b0, int i0, const C2<T>* a1,
                       const C2<T>* b1, int i1, double* dst) {
    return field_dots<T>(c.g->N, c.g->cell, c.parts, nq, a0, b0, i0, a1, b1, i1, dst, c.s);
}

// f <- Pi f: remove the components along phi and i phi.
template <typename T>
static hipError_t project(AdjCtx<T>& c, C2<T>* f) {
    hipError_t e = dots<T>(c, 2, c.phi, f, 0, c.phi, f, 1, c.sc + 4);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_project<T>, dim3(nblk(c.g->N)), dim3(256), 0, c.s, f, c.phi, c.sc + 4, c.S, c.g->N);
    return hipGetLastError();
}

// z <- Pi P_C Pi r (r is already in the tangent space).
template <typename T>
static hipError_t precondition(AdjCtx<T>& c, const C2<T>* rin, C2<T>* zout) {
    hipError_t e = op_precond(*c.g, sizeof(T) == 8, *c.tw, GPE_P_COMBINED, c.phi, c.V, c.sc + 8, c.beta, rin, zout, c.w,
                              c.s);
    if (e != hipSuccess) return e;
    return project<T>(c, zout);
}

template <typename T>
static hipError_t adjoint_run(AdjCtx<T>& c, const C2<T>* rhs, int check_every, int64_t max_it, CgS& hostS) {
    const int64_t N = c.g->N;
    hipError_t e;
    // r = Pi rhs, x = 0, z = Pi P Pi r, p = z
    hipLaunchKernelGGL(k_copy_c<T>, dim3(nblk(N)), dim3(256), 0, c.s, rhs, c.r, N);
    hipLaunchKernelGGL(k_zero_c<T>, dim3(nblk(N)), dim3(256), 0, c.s, c.x, N);
    if ((e = project<T>(c, c.r)) != hipSuccess) return e;
    if ((e = precondition<T>(c, c.r, c.z)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_copy_c<T>, dim3(nblk(N)), dim3(256), 0, c.s, c.z, c.p, N);
    if ((e = dots<T>(c, 2, c.r, c.z, 0, c.r, c.r, 0, c.sc)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_init, dim3(1), dim3(64), 0, c.s, c.S, c.sc, c.sc + 9);
    for (int64_t it = 0; it <= max_it; it += check_every) {
        for (int k = 0; k < check_every; ++k) {
            // q = Pi (1/2 nabla^2 E - lambda) p
            if ((e = op_apply(*c.g, sizeof(T) == 8, 1, *c.tw, c.p, c.V, c.q, c.w, c.beta, c.omega, false, c.s)) !=
                hipSuccess)
                return e;
            hipLaunchKernelGGL(k_hessian<T>, dim3(nblk(N)), dim3(256), 0, c.s, c.q, c.p, c.phi, c.S, N);
            if ((e = project<T>(c, c.q)) != hipSuccess) return e;
            if ((e = dots<T>(c, 1, c.p, c.q, 0, nullptr, nullptr, 0, c.sc)) != hipSuccess) return e;
            hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(64), 0, c.s, c.S, c.sc);
            hipLaunchKernelGGL(k_cg_update<T>, dim3(nblk(N)), dim3(256), 0, c.s, c.x, c.r, c.p, c.q, c.S, N);
            if ((e = precondition<T>(c, c.r, c.z)) != hipSuccess) return e;
            if ((e = dots<T>(c, 2, c.r, c.z, 0, c.r, c.r, 0, c.sc)) != hipSuccess) return e;
            hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(64), 0, c.s, c.S, c.sc);
            hipLaunchKernelGGL(k_cg_dir<T>, dim3(nblk(N)), dim3(256), 0, c.s, c.p, c.z, c.S, N);
        }
        if ((e = hipMemcpyAsync(&hostS, c.S, sizeof(CgS), hipMemcpyDeviceToHost, c.s)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(c.s)) != hipSuccess) return e;
        if (hostS.done) break;
    }
    return hipSuccess;
}

}  // namespace gpe

using namespace gpe;

#define HIPCHK(expr)                                                                    \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess) {                                                         \
            set_error(std::string("HIP error in " #expr ": ") + hipGetErrorString(_e)); \
            return GPE_EHIP;                                                            \
        }                                                                               \
    } while (0)

template <typename T>
static int adjoint_impl(gpe_plan_t* plan, const void* phi_star, const void* V, const void* rhs, void* mu,
                        const gpe_pcg_opts_t* o, gpe_pcg_report_t* report, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const Geo& g = plan->g;
    const int64_t N = g.N;
    const size_t cf = sizeof(C2<T>) * (size_t)N;
    HIPCHK(plan->tmp.ensure(6 * cf + sizeof(CgS) + 64 * sizeof(double) + kDotBlocks * 4 * sizeof(double) + 256));
    char* base = (char*)plan->tmp.ptr;
    AdjCtx<T> c;
    c.g = &g;
    c.tw = &plan->tw;
    c.phi = (const C2<T>*)phi_star;
    c.V = (const T*)V;
    c.beta = plan->prob.beta;
    c.omega = plan->prob.omega;
    c.x = (C2<T>*)mu;
    c.r = (C2<T>*)(base + 0 * cf);
    c.z = (C2<T>*)(base + 1 * cf);
    c.p = (C2<T>*)(base + 2 * cf);
    c.q = (C2<T>*)(base + 3 * cf);
    c.w = (C2<T>*)(base + 4 * cf);
    C2<T>* hphi = (C2<T>*)(base + 5 * cf);
    c.S = (CgS*)(base + 6 * cf);
    c.sc = (double*)(base + 6 * cf + sizeof(CgS));
    c.parts = c.sc + 64;
    c.s = s;
    // lambda and ||phi||^2 (fresh), lambda~ for the preconditioner
    HIPCHK(op_apply(g, sizeof(T) == 8, 1, plan->tw, phi_star, V, hphi, c.w, c.beta, c.omega, true, s));
    HIPCHK(dots<T>(c, 2, c.phi, hphi, 0, c.phi, c.phi, 0, c.sc + 12));
    HIPCHK(op_energy(g, sizeof(T) == 8, plan->tw, phi_star, V, c.beta, c.omega, plan->red, c.sc + 16, s));
    HIPCHK(op_lambda_tilde(c.sc + 16, c.sc + 8, s));
    double h2[2];
    HIPCHK(hipMemcpyAsync(h2, c.sc + 12, sizeof(h2), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    CgS hs;
    std::memset(&hs, 0, sizeof(hs));
    hs.lam = h2[0] / h2[1];
    hs.beta = c.beta;
    hs.cell = g.cell;
    hs.nphi2 = h2[1];
    hs.tol2 = o->tol_res_inf * o->tol_res_inf;
    hs.max_it = o->max_iter;
    HIPCHK(hipMemcpyAsync(c.S, &hs, sizeof(CgS), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c.sc + 9, &h2[1], sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(adjoint_run<T>(c, (const C2<T>*)rhs, std::max(1, o->check_every), o->max_iter, hs));
    const auto t1 = std::chrono::steady_clock::now();
    int st = hs.status == 0 ? GPE_OK : hs.status == 1 ? GPE_NOT_CONVERGED : hs.status == -4 ? GPE_ENONFINITE : GPE_EINVAL;
    if (report) {
        std::memset(report, 0, sizeof(*report));
        report->status = st;
        report->iters = hs.it;
        report->lambda = hs.lam;
        report->res_inf = hs.rr0 > 0.0 ? std::sqrt(hs.rr / hs.rr0) : 0.0;
        report->seconds = std::chrono::duration<double>(t1 - t0).count();
    }
    if (st == GPE_EINVAL) set_error("the projected Hessian is not positive definite (phi_star is not a local minimum)");
    if (st == GPE_ENONFINITE) set_error("non-finite value in the adjoint iteration");
    return st;
}

extern "C" int gpe_adjoint_solve(gpe_plan_t* plan, const void* phi_star, const void* V, const void* rhs, void* mu,
                                 const gpe_pcg_opts_t* opts, gpe_pcg_report_t* report, void* stream) {
    if (!plan || !phi_star || !V || !rhs || !mu || !opts) { set_error("NULL argument"); return GPE_EINVAL; }
    if (mu == rhs || mu == phi_star) { set_error("mu must not alias rhs or phi_star"); return GPE_EINVAL; }
    if (!(opts->tol_res_inf > 0.0) || opts->max_iter < 1) { set_error("need tol > 0 and max_iter >= 1"); return GPE_EINVAL; }
    return plan->f64() ? adjoint_impl<double>(plan, phi_star, V, rhs, mu, opts, report, (hipStream_t)stream)
                       : adjoint_impl<float>(plan, phi_star, V, rhs, mu, opts, report, (hipStream_t)stream);
}

// Parameter gradients of the adjoint part: grad_V = -h^d Re(conj(mu) phi) (device, nullable),
// *dl_dbeta = -Re<mu, |phi|^2 phi>, *dl_domega = +Re<mu, L_z phi> (host, nullable).
template <typename T>
static int param_grads_impl(gpe_plan_t* plan, const void* phi, const void* mu, void* grad_V, double* dl_dbeta,
                            double* dl_domega, hipStream_t s) {
    const Geo& g = plan->g;
    const int64_t N = g.N;
    const size_t cf = sizeof(C2<T>) * (size_t)N;
    HIPCHK(plan->tmp.ensure(2 * cf + 64 * sizeof(double) + kDotBlocks * 4 * sizeof(double) + 256));
    char* base = (char*)plan->tmp.ptr;
    AdjCtx<T> c{};
    c.g = &g;
    c.s = s;
    c.sc = (double*)(base + 2 * cf);
    c.parts = c.sc + 64;
    C2<T>* v = (C2<T>*)base;
    C2<T>* w = (C2<T>*)(base + cf);
    if (grad_V)
        hipLaunchKernelGGL(k_grad_V<T>, dim3(nblk(N)), dim3(256), 0, s, (const C2<T>*)mu, (const C2<T>*)phi, (T*)grad_V,
                           (T)g.cell, N);
    double h[2] = {0.0, 0.0};
    if (dl_dbeta) {
        hipLaunchKernelGGL(k_cubic<T>, dim3(nblk(N)), dim3(256), 0, s, (const C2<T>*)phi, v, N);
        HIPCHK(dots<T>(c, 1, (const C2<T>*)mu, v, 0, nullptr, nullptr, 0, c.sc));
        HIPCHK(hipMemcpyAsync(&h[0], c.sc, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (dl_domega && g.dim >= 2) {
        HIPCHK(op_rotation(g, sizeof(T) == 8, plan->tw, phi, v, w, s));  // v = -L_z phi
        HIPCHK(dots<T>(c, 1, (const C2<T>*)mu, v, 0, nullptr, nullptr, 0, c.sc + 4));
        HIPCHK(hipMemcpyAsync(&h[1], c.sc + 4, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    if (dl_dbeta) *dl_dbeta = -h[0];
    if (dl_domega) *dl_domega = g.dim >= 2 ? -h[1] : 0.0;
    return GPE_OK;
}

extern "C" int gpe_adjoint_param_grads(gpe_plan_t* plan, const void* phi_star, const void* mu, void* grad_V,
                                       double* dl_dbeta, double* dl_domega, void* stream) {
    if (!plan || !phi_star || !mu) { set_error("NULL argument"); return GPE_EINVAL; }
    return plan->f64() ? param_grads_impl<double>(plan, phi_star, mu, grad_V, dl_dbeta, dl_domega, (hipStream_t)stream)
                       : param_grads_impl<float>(plan, phi_star, mu, grad_V, dl_dbeta, dl_domega, (hipStream_t)stream);
}
