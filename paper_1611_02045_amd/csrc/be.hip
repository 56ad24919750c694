// Backward Euler discretisation of the normalised gradient flow (the BESP schemes of Section 4, run
// in Section 6 as BE_nu with a preconditioned Krylov inner solver).
//
// Outer step n (||phi_n|| = 1): lambda_n = <phi_n, H_{phi_n} phi_n>; stop when
// ||H_{phi_n} phi_n - lambda_n phi_n||_inf <= tol; otherwise solve
//   (I/dt + H_{phi_n} - s lambda_n) phit = phi_n / dt,   H_{phi_n} = L + beta |phi_n|^2 (frozen),
// with s = 1 for the scheme with the Lagrange multiplier (the multiplier on the new iterate, the
// reading under which the scheme is the plain one with the effective step dt / (1 - dt lambda_n))
// and s = 0 for the plain scheme, then phi_{n+1} = phit / ||phit||.  The inner solve is
// preconditioned linear CG from phit = phi_n (the operator is Hermitian, and positive definite
// when 1/dt > s (lambda_n - lambda_1)); the preconditioner is P_nu of Section 5.5 with the shift
// 1/dt of the BESP literature the paper cites.  Every CG scalar stays on the device; the host
// polls the inner state every `check_every` iterations and reads two scalars per outer step.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>

#include "internal.hpp"
#include "linear.hpp"
#include "plan.hpp"

namespace gpe {

// q <- q + (1/dt - shift + beta |phi|^2) x  (q holds L x on entry).
template <typename T>
__global__ void k_be_op(C2<T>* q, const C2<T>* x, const C2<T>* phi, const double* invdt_shift, double beta, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const T w = (T)invdt_shift[0] + (T)beta * abs2(phi[i]);
    q[i] = add(q[i], scl(x[i], w));
}

// r = phi / dt - q  (q = A phi: the residual of the initial guess phit = phi).
template <typename T>
__global__ void k_be_rhs_resid(C2<T>* r, const C2<T>* phi, const C2<T>* q, double invdt, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    r[i] = sub(scl(phi[i], (T)invdt), q[i]);
}

// Per-block maxima of |Hphi - lambda phi| (lambda = sc[0] / sc[1]).
template <typename T>
__global__ __launch_bounds__(256) void k_be_resmax(const C2<T>* hphi, const C2<T>* phi, const double* sc, double* parts,
                                                   int64_t N) {
    __shared__ double red[4];
    __shared__ double out[1];
    const T lam = (T)(sc[0] / sc[1]);
    double m[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const C2<T> r = sub(hphi[i], scl(phi[i], lam));
        m[0] = fmax(m[0], (double)abs2(r));
    }
    block_reduce<1>(m, red, out, 1u);
    if (threadIdx.x == 0) parts[blockIdx.x] = out[0];
}

// sc[4] = sqrt(max of the parts); sc[5] = lambda = sc[0] / sc[1]; sc[6] = 1/dt - s lambda.
__global__ void k_be_scalars(const double* parts, int nb, double* sc, double invdt, int lambda_term) {
    __shared__ double red[4];
    __shared__ double out[1];
    double m[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x) m[0] = fmax(m[0], parts[b]);
    block_reduce<1>(m, red, out, 1u);
    if (threadIdx.x == 0) {
        sc[4] = sqrt(out[0]);
        sc[5] = sc[0] / sc[1];
        sc[6] = invdt - (lambda_term ? sc[5] : 0.0);
    }
}

// CG start: rz = <r, z>, reference norm ||b||^2 = ||phi||^2 / dt^2 (the relative residual test of
// the inner solve is ||r|| <= tol ||b||).
__global__ void k_be_cg_init(CgS* S, const double* dots, const double* nphi2, double invdt, double tol2, int64_t max_it) {
    if (threadIdx.x != 0) return;
    S->rz = dots[0];
    S->rr = dots[1];
    S->rr0 = nphi2[0] * invdt * invdt;
    S->tol2 = tol2;
    S->it = 0;
    S->max_it = max_it;
    S->done = 0;
    S->status = 0;
    if (S->rr <= tol2 * S->rr0) S->done = 1;  // the initial guess already solves the system
}

// phi = x / sqrt(nx2[0]).
template <typename T>
__global__ void k_be_normalise(C2<T>* phi, const C2<T>* x, const double* nx2, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) phi[i] = scl(x[i], (T)(1.0 / sqrt(nx2[0])));
}

template <typename T>
struct BeCtx {
    const Geo* g;
    const Twiddles* tw;
    const T* V;
    double beta, omega, invdt;
    int kind;
    CgS* S;
    double* parts;  // kDotBlocks * 4
    double* sc;     // [0..1] <phi,H phi>, <phi,phi>; [4] ||r||_inf; [5] lambda; [6] 1/dt - s lambda;
                    // [8..9] CG dots; [12] <x,x>; [16] preconditioner shift 1/dt (an inner product
                    // request writes 4 consecutive slots)
    C2<T>*phi, *hphi, *x, *r, *z, *p, *q, *w;
    hipStream_t s;
};

// q = A v = L v + (1/dt - s lambda + beta |phi|^2) v.
template <typename T>
static hipError_t be_apply(BeCtx<T>& c, const C2<T>* v, C2<T>* q) {
    hipError_t e = op_apply(*c.g, sizeof(T) == 8, 1, *c.tw, v, c.V, q, c.w, c.beta, c.omega, false, c.s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_be_op<T>, dim3(nblk(c.g->N)), dim3(256), 0, c.s, q, v, c.phi, c.sc + 6, c.beta, c.g->N);
    return hipGetLastError();
}

template <typename T>
static hipError_t be_precond(BeCtx<T>& c, const C2<T>* rin, C2<T>* zout) {
    if (c.kind == GPE_P_NONE) {
        hipLaunchKernelGGL(k_copy_c<T>, dim3(nblk(c.g->N)), dim3(256), 0, c.s, rin, zout, c.g->N);
        return hipGetLastError();
    }
    return op_precond(*c.g, sizeof(T) == 8, *c.tw, c.kind, c.phi, c.V, c.sc + 16, c.beta, rin, zout, c.w, c.s);
}

// One inner solve (phi_n in c.phi, lambda and the shift in c.sc): c.x <- phit.  Returns the CG
// state in hostS.
template <typename T>
static hipError_t be_inner(BeCtx<T>& c, double tol, int64_t max_it, int check_every, CgS& hostS) {
    const int64_t N = c.g->N;
    hipError_t e;
    hipLaunchKernelGGL(k_copy_c<T>, dim3(nblk(N)), dim3(256), 0, c.s, c.phi, c.x, N);
    if ((e = be_apply<T>(c, c.x, c.q)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_be_rhs_resid<T>, dim3(nblk(N)), dim3(256), 0, c.s, c.r, c.phi, c.q, c.invdt, N);
    if ((e = be_precond<T>(c, c.r, c.z)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_copy_c<T>, dim3(nblk(N)), dim3(256), 0, c.s, c.z, c.p, N);
    if ((e = field_dots<T>(N, c.g->cell, c.parts, 2, c.r, c.z, 0, c.r, c.r, 0, c.sc + 8, c.s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_be_cg_init, dim3(1), dim3(64), 0, c.s, c.S, c.sc + 8, c.sc + 1, c.invdt, tol * tol, max_it);
    for (int64_t it = 0; it <= max_it; it += check_every) {
        for (int k = 0; k < check_every; ++k) {
            if ((e = be_apply<T>(c, c.p, c.q)) != hipSuccess) return e;
            if ((e = field_dots<T>(N, c.g->cell, c.parts, 1, c.p, c.q, 0, nullptr, nullptr, 0, c.sc + 8, c.s)) !=
                hipSuccess)
                return e;
            hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(64), 0, c.s, c.S, c.sc + 8);
            hipLaunchKernelGGL(k_cg_update<T>, dim3(nblk(N)), dim3(256), 0, c.s, c.x, c.r, c.p, c.q, c.S, N);
            if ((e = be_precond<T>(c, c.r, c.z)) != hipSuccess) return e;
            if ((e = field_dots<T>(N, c.g->cell, c.parts, 2, c.r, c.z, 0, c.r, c.r, 0, c.sc + 8, c.s)) != hipSuccess)
                return e;
            hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(64), 0, c.s, c.S, c.sc + 8);
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

constexpr int64_t kBeInnerMax = 10000;

template <typename T>
static int be_impl(gpe_plan_t* plan, const void* V, void* phi_inout, double dt, int lambda_term,
                   const gpe_pcg_opts_t* o, double inner_tol, int64_t* inner_total, gpe_pcg_report_t* report,
                   hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const Geo& g = plan->g;
    const int64_t N = g.N;
    const size_t cf = sizeof(C2<T>) * (size_t)N;
    HIPCHK(plan->tmp.ensure(7 * cf + sizeof(CgS) + 64 * sizeof(double) + kDotBlocks * 4 * sizeof(double) + 256));
    char* base = (char*)plan->tmp.ptr;
    BeCtx<T> c;
    c.g = &g;
    c.tw = &plan->tw;
    c.V = (const T*)V;
    c.beta = plan->prob.beta;
    c.omega = plan->prob.omega;
    c.invdt = 1.0 / dt;
    c.kind = o->precond;
    c.phi = (C2<T>*)phi_inout;
    c.hphi = (C2<T>*)(base + 0 * cf);
    c.x = (C2<T>*)(base + 1 * cf);
    c.r = (C2<T>*)(base + 2 * cf);
    c.z = (C2<T>*)(base + 3 * cf);
    c.p = (C2<T>*)(base + 4 * cf);
    c.q = (C2<T>*)(base + 5 * cf);
    c.w = (C2<T>*)(base + 6 * cf);
    c.S = (CgS*)(base + 7 * cf);
    c.sc = (double*)(base + 7 * cf + sizeof(CgS));
    c.parts = c.sc + 64;
    c.s = s;
    const double pshift = c.invdt;
    HIPCHK(hipMemcpyAsync(c.sc + 16, &pshift, sizeof(double), hipMemcpyHostToDevice, s));
    // normalise the start
    HIPCHK(field_dots<T>(N, g.cell, c.parts, 1, c.phi, c.phi, 0, nullptr, nullptr, 0, c.sc + 12, s));
    hipLaunchKernelGGL(k_be_normalise<T>, dim3(nblk(N)), dim3(256), 0, s, c.phi, c.phi, c.sc + 12, N);
    HIPCHK(hipGetLastError());
    int64_t inner = 0, n = 0;
    int st = GPE_NOT_CONVERGED;
    double hs[2] = {0.0, 0.0};  // ||r||_inf, lambda
    for (n = 0;; ++n) {
        // lambda_n and the residual of phi_n
        HIPCHK(op_apply(g, sizeof(T) == 8, 1, plan->tw, c.phi, V, c.hphi, c.w, c.beta, c.omega, true, s));
        HIPCHK(field_dots<T>(N, g.cell, c.parts, 2, c.phi, c.hphi, 0, c.phi, c.phi, 0, c.sc, s));
        hipLaunchKernelGGL(k_be_resmax<T>, dim3(kDotBlocks), dim3(256), 0, s, c.hphi, c.phi, c.sc, c.parts, N);
        hipLaunchKernelGGL(k_be_scalars, dim3(1), dim3(256), 0, s, c.parts, kDotBlocks, c.sc, c.invdt, lambda_term);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(hs, c.sc + 4, sizeof(hs), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (!std::isfinite(hs[0]) || !std::isfinite(hs[1])) {
            st = GPE_ENONFINITE;
            set_error("non-finite value in the backward Euler iteration");
            break;
        }
        if (hs[0] <= o->tol_res_inf) {
            st = GPE_OK;
            break;
        }
        if (n >= o->max_iter) break;
        CgS cs;
        HIPCHK(be_inner<T>(c, inner_tol, kBeInnerMax, std::max(1, o->check_every), cs));
        inner += cs.it;
        if (cs.status == -1) {
            st = GPE_EINVAL;
            set_error("the backward Euler operator is not positive definite (reduce dt)");
            break;
        }
        if (cs.status == -4) {
            st = GPE_ENONFINITE;
            set_error("non-finite value in the inner solve");
            break;
        }
        // phi_{n+1} = phit / ||phit||
        HIPCHK(field_dots<T>(N, g.cell, c.parts, 1, c.x, c.x, 0, nullptr, nullptr, 0, c.sc + 12, s));
        hipLaunchKernelGGL(k_be_normalise<T>, dim3(nblk(N)), dim3(256), 0, s, c.phi, c.x, c.sc + 12, N);
        HIPCHK(hipGetLastError());
    }
    if (inner_total) *inner_total = inner;
    if (report) {
        std::memset(report, 0, sizeof(*report));
        report->status = st;
        report->iters = n;
        report->res_inf = hs[0];
        report->lambda = hs[1];
        double* ed = (double*)plan->red.scalars.ptr;
        double h[4] = {0.0, 0.0, 0.0, 0.0};
        HIPCHK(op_energy(g, sizeof(T) == 8, plan->tw, c.phi, V, c.beta, c.omega, plan->red, ed, s));
        HIPCHK(hipMemcpyAsync(h, ed, sizeof(h), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        report->E = h[0] + h[1] + h[2] + h[3];
        report->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return st;
}

extern "C" int gpe_be_solve(gpe_plan_t* plan, const void* V, void* phi_inout, double dt, int lambda_term,
                            const gpe_pcg_opts_t* opts, double inner_tol, int64_t* inner_iters,
                            gpe_pcg_report_t* report, void* stream) {
    if (!plan || !V || !phi_inout || !opts) { set_error("NULL argument"); return GPE_EINVAL; }
    if (!(dt > 0.0) || !std::isfinite(dt)) { set_error("dt must be positive"); return GPE_EINVAL; }
    if (!(inner_tol > 0.0) || !(opts->tol_res_inf > 0.0) || opts->max_iter < 0) {
        set_error("need inner_tol > 0, tol_res_inf > 0 and max_iter >= 0");
        return GPE_EINVAL;
    }
    if (opts->precond < GPE_P_NONE || opts->precond > GPE_P_COMBINED) {
        set_error("the inner CG needs a symmetric preconditioner (none, kinetic, potential or combined)");
        return GPE_EINVAL;
    }
    return plan->f64() ? be_impl<double>(plan, V, phi_inout, dt, lambda_term, opts, inner_tol, inner_iters, report,
                                         (hipStream_t)stream)
                       : be_impl<float>(plan, V, phi_inout, dt, lambda_term, opts, inner_tol, inner_iters, report,
                                        (hipStream_t)stream);
}
