// C ABI of libgpe: argument validation, plans, error reporting, and the operator entry points.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "internal.hpp"
#include "plan.hpp"

namespace gpe {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

Geo make_geo(const gpe_problem_t& p) {
    Geo g;
    std::memset(&g, 0, sizeof(g));
    g.dim = p.dim;
    g.cell = 1.0;
    g.N = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < p.dim) {
            g.n[a] = p.n[a];
            const int f5 = p.n[a] % 5 == 0 ? 1 : 0;
            const int m = f5 ? p.n[a] / 5 : p.n[a];
            int lg = 0;
            while ((1 << lg) < m) ++lg;
            g.lg[a] = lg;
            g.f5[a] = f5;
            g.L[a] = p.L[a];
            g.h[a] = 2.0 * p.L[a] / p.n[a];
            g.dk[a] = 3.141592653589793238462643383279502884 / p.L[a];
            g.cell *= g.h[a];
            g.N *= p.n[a];
        } else {
            g.n[a] = 1;
            g.lg[a] = 0;
            g.L[a] = 1.0;
            g.h[a] = 1.0;
            g.dk[a] = 3.141592653589793238462643383279502884;
        }
    }
    g.pow2 = !(g.f5[0] || g.f5[1] || g.f5[2]);
    return g;
}

std::mutex& capture_mutex() {
    static std::mutex m;
    return m;
}

namespace {
using TileKey = std::tuple<int, int, int, int, int, int, int>;  // dim, n0, n1, n2, axis, point bytes, batch
std::mutex g_tiles_mutex;
std::map<TileKey, int> g_tiles;
TileKey tile_key(const Geo& g, int AX, int cb, int B) { return TileKey{g.dim, g.n[0], g.n[1], g.n[2], AX, cb, B}; }
}  // namespace

int tuned_lines(const Geo& g, int AX, int complex_bytes, int B) {
    std::lock_guard<std::mutex> lock(g_tiles_mutex);
    if (g_tiles.empty()) return 0;
    const auto it = g_tiles.find(tile_key(g, AX, complex_bytes, B));
    return it == g_tiles.end() ? 0 : it->second;
}

void record_tuned_lines(const Geo& g, int AX, int complex_bytes, int B, int C) {
    std::lock_guard<std::mutex> lock(g_tiles_mutex);
    g_tiles[tile_key(g, AX, complex_bytes, B)] = C;
}

hipError_t build_twiddles(const Geo& g, Twiddles& tw) {
    for (int a = 0; a < g.dim; ++a) {
        const int M = g.n[a];
        std::vector<double> t64(2 * M);
        std::vector<float> t32(2 * M);
        for (int e = 0; e < M; ++e) {
            const double ang = -2.0 * M_PI * (double)e / (double)M;
            t64[2 * e] = std::cos(ang);
            t64[2 * e + 1] = std::sin(ang);
            t32[2 * e] = (float)t64[2 * e];
            t32[2 * e + 1] = (float)t64[2 * e + 1];
        }
        hipError_t e;
        if ((e = tw.t64[a].ensure(sizeof(double) * 2 * M)) != hipSuccess) return e;
        if ((e = tw.t32[a].ensure(sizeof(float) * 2 * M)) != hipSuccess) return e;
        std::lock_guard<std::mutex> lock(capture_mutex());
        if ((e = hipMemcpy(tw.t64[a].ptr, t64.data(), sizeof(double) * 2 * M, hipMemcpyHostToDevice)) != hipSuccess)
            return e;
        if ((e = hipMemcpy(tw.t32[a].ptr, t32.data(), sizeof(float) * 2 * M, hipMemcpyHostToDevice)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t reduce_init(Reduce& r, int instances, int slots, size_t part_doubles) {
    hipError_t e;
    if ((e = r.parts.ensure(sizeof(double) * part_doubles)) != hipSuccess) return e;
    const size_t cbytes = sizeof(unsigned int) * (size_t)instances * slots;
    if (cbytes > r.counters.bytes) {
        if ((e = r.counters.ensure(cbytes)) != hipSuccess) return e;
        std::lock_guard<std::mutex> lock(capture_mutex());
        if ((e = hipMemset(r.counters.ptr, 0, r.counters.bytes)) != hipSuccess) return e;
        if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
    }
    r.counter_slots = slots;
    if ((e = r.scalars.ensure(sizeof(double) * 64)) != hipSuccess) return e;
    return hipSuccess;
}

__global__ void k_set_scalar(double* dst, double v) {
    if (threadIdx.x == 0) *dst = v;
}

// Validation of a problem description against the supported grids.
int validate_problem(const gpe_problem_t* p) {
    if (!p) { set_error("problem is NULL"); return GPE_EINVAL; }
    if (p->dim < 1 || p->dim > 3) { set_error("dim must be 1, 2 or 3"); return GPE_EINVAL; }
    for (int a = 0; a < p->dim; ++a) {
        const int n = p->n[a];
        if (n < 2 || (n & 1)) { set_error("grid sizes must be even and >= 2"); return GPE_EINVAL; }
        const bool pow2 = (n & (n - 1)) == 0 && n >= 8 && n <= 1024;
        const int m = n / 5;
        const bool five = n % 5 == 0 && (m & (m - 1)) == 0 && n >= 40 && n <= 640;
        if (!pow2 && !five) {
            set_error("grid sizes must be 2^k (8 to 1024) or 5 * 2^k (40 to 640)");
            return GPE_EUNSUPPORTED;
        }
        if (!(p->L[a] > 0.0) || !std::isfinite(p->L[a])) { set_error("half-widths L must be positive"); return GPE_EINVAL; }
    }
    if (!std::isfinite(p->beta) || !std::isfinite(p->omega)) { set_error("beta and omega must be finite"); return GPE_EINVAL; }
    if (p->dim == 1 && p->omega != 0.0) { set_error("rotation needs dim >= 2 (omega must be 0 in 1-D)"); return GPE_EINVAL; }
    return GPE_OK;
}

}  // namespace gpe

using namespace gpe;

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess) {                                                             \
            set_error(std::string("HIP error in " #expr ": ") + hipGetErrorString(_e));     \
            return GPE_EHIP;                                                                \
        }                                                                                   \
    } while (0)

#define NEEDPTR(p, name)                                   \
    do {                                                   \
        if (!(p)) {                                        \
            set_error(std::string(name) + " is NULL");     \
            return GPE_EINVAL;                             \
        }                                                  \
    } while (0)

extern "C" {

const char* gpe_last_error(void) { return g_last_error.c_str(); }

const char* gpe_version(void) { return "libgpe 0.1 (gfx950)"; }

int gpe_plan_create(const gpe_problem_t* prob, int dtype, gpe_plan_t** out) {
    if (!out) { set_error("out is NULL"); return GPE_EINVAL; }
    *out = nullptr;
    int st = validate_problem(prob);
    if (st != GPE_OK) return st;
    if (dtype != GPE_F64 && dtype != GPE_F32) { set_error("dtype must be GPE_F64 or GPE_F32"); return GPE_EINVAL; }
    gpe_plan* p = new gpe_plan();
    p->prob = *prob;
    p->dtype = dtype;
    p->g = make_geo(*prob);
    hipError_t e = build_twiddles(p->g, p->tw);
    if (e == hipSuccess) e = reduce_init(p->red, 1, 16, 1 << 18);
    if (e == hipSuccess) e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        set_error(std::string("plan creation failed: ") + hipGetErrorString(e));
        p->release();
        delete p;
        return GPE_EHIP;
    }
    *out = p;
    return GPE_OK;
}

int gpe_plan_destroy(gpe_plan_t* plan) {
    if (!plan) return GPE_OK;
    {
        std::lock_guard<std::mutex> lock(capture_mutex());
        (void)hipDeviceSynchronize();
    }
    plan->release();
    delete plan;
    return GPE_OK;
}

int gpe_energy(gpe_plan_t* plan, const void* phi, const void* V, double* E, double* parts, void* stream) {
    NEEDPTR(plan, "plan");
    NEEDPTR(phi, "phi");
    NEEDPTR(V, "V");
    NEEDPTR(E, "E");
    hipStream_t s = (hipStream_t)stream;
    double* dst = (double*)plan->red.scalars.ptr;
    HIPCHK(op_energy(plan->g, plan->f64(), plan->tw, phi, V, plan->prob.beta, plan->prob.omega, plan->red, dst, s));
    double h[4];
    HIPCHK(hipMemcpyAsync(h, dst, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *E = h[0] + h[1] + h[2] + h[3];
    if (parts) std::memcpy(parts, h, sizeof(h));
    if (!std::isfinite(*E)) { set_error("energy is not finite"); return GPE_ENONFINITE; }
    return GPE_OK;
}

int gpe_apply_H_batched(gpe_plan_t* plan, int count, const void* phi, const void* V, void* Hphi, void* stream) {
    NEEDPTR(plan, "plan");
    NEEDPTR(phi, "phi");
    NEEDPTR(V, "V");
    NEEDPTR(Hphi, "Hphi");
    if (count < 1) { set_error("count must be >= 1"); return GPE_EINVAL; }
    if (phi == Hphi) { set_error("Hphi must not alias phi"); return GPE_EINVAL; }
    const size_t cb = plan->f64() ? 16 : 8;
    HIPCHK(plan->tmp.ensure(cb * (size_t)plan->g.N * count));
    HIPCHK(op_apply(plan->g, plan->f64(), count, plan->tw, phi, V, Hphi, plan->tmp.ptr, plan->prob.beta,
                    plan->prob.omega, true, (hipStream_t)stream));
    return GPE_OK;
}

int gpe_apply_H(gpe_plan_t* plan, const void* phi, const void* V, void* Hphi, void* stream) {
    return gpe_apply_H_batched(plan, 1, phi, V, Hphi, stream);
}

int gpe_set_apply_kernel(int kind) {
    if (kind < GPE_APPLY_AUTO || kind > GPE_APPLY_PLANE) {
        set_error("unknown apply kernel kind");
        return GPE_EINVAL;
    }
    set_apply_kind(kind);
    return GPE_OK;
}

int gpe_apply_kernel_for(gpe_plan_t* plan, int count, int* kind) {
    NEEDPTR(plan, "plan");
    NEEDPTR(kind, "kind");
    if (count < 1) { set_error("count must be >= 1"); return GPE_EINVAL; }
    *kind = plane_preferred(plan->g, plan->f64(), count) ? GPE_APPLY_PLANE : GPE_APPLY_PASSES;
    return GPE_OK;
}

int gpe_precond(gpe_plan_t* plan, int kind, const void* phi, const void* V, double alpha, const void* r, void* Pr,
                void* stream) {
    NEEDPTR(plan, "plan");
    NEEDPTR(phi, "phi");
    NEEDPTR(V, "V");
    NEEDPTR(r, "r");
    NEEDPTR(Pr, "Pr");
    if (kind < GPE_P_NONE || kind > GPE_P_C2) { set_error("unknown preconditioner kind"); return GPE_EINVAL; }
    if (Pr == r || Pr == phi) { set_error("Pr must not alias r or phi"); return GPE_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    double* sc = (double*)plan->red.scalars.ptr;
    double* alpha_dev = sc + 8;
    if (std::isnan(alpha)) {
        HIPCHK(op_energy(plan->g, plan->f64(), plan->tw, phi, V, plan->prob.beta, plan->prob.omega, plan->red, sc, s));
        HIPCHK(op_lambda_tilde(sc, alpha_dev, s));
    } else {
        if (!std::isfinite(alpha)) { set_error("alpha must be finite or NaN"); return GPE_EINVAL; }
        hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(64), 0, s, alpha_dev, alpha);
        HIPCHK(hipGetLastError());
    }
    if (kind != GPE_P_NONE) {
        // P_Delta needs alpha > 0 (its symbol 1/(alpha + |k|^2/2) must be positive at k = 0);
        // the others need alpha + V + beta|phi|^2 > 0 pointwise.
        double hmin[2];
        HIPCHK(op_min_diag(plan->g, plan->f64(), phi, V, alpha_dev, plan->prob.beta, plan->red, sc + 9, s));
        HIPCHK(hipMemcpyAsync(hmin, sc + 8, sizeof(hmin), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (!std::isfinite(hmin[0]) || !std::isfinite(hmin[1])) { set_error("non-finite shift or field"); return GPE_ENONFINITE; }
        if (kind == GPE_P_KINETIC ? !(hmin[0] > 0.0) : !(hmin[1] > 0.0)) {
            set_error("preconditioner is not positive definite (alpha + V + beta|phi|^2 <= 0 or alpha <= 0)");
            return GPE_EINVAL;
        }
    }
    const size_t cb = plan->f64() ? 16 : 8;
    HIPCHK(plan->tmp.ensure(cb * (size_t)plan->g.N));
    HIPCHK(op_precond(plan->g, plan->f64(), plan->tw, kind, phi, V, alpha_dev, plan->prob.beta, r, Pr, plan->tmp.ptr, s));
    return GPE_OK;
}

int gpe_autotune(gpe_plan_t* plan, int count, int* tiles, double* us, void* stream) {
    NEEDPTR(plan, "plan");
    if (count < 1) { set_error("count must be >= 1"); return GPE_EINVAL; }
    const size_t cb = plan->f64() ? 16 : 8;
    const size_t bytes = cb * (size_t)plan->g.N * count;
    HIPCHK(plan->tmp.ensure(2 * bytes));
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipMemsetAsync(plan->tmp.ptr, 0, 2 * bytes, s));
    int t[3] = {0, 0, 0};
    double u[3] = {0.0, 0.0, 0.0};
    HIPCHK(op_autotune(plan->g, plan->f64(), count, plan->tw, plan->tmp.ptr, (char*)plan->tmp.ptr + bytes, s, t, u));
    HIPCHK(hipStreamSynchronize(s));
    for (int a = 0; a < 3; ++a) {
        if (tiles) tiles[a] = t[a];
        if (us) us[a] = u[a];
    }
    return GPE_OK;
}

int gpe_prolong(gpe_plan_t* plan, const void* in, void* out, void* stream) {
    NEEDPTR(plan, "plan");
    NEEDPTR(in, "in");
    NEEDPTR(out, "out");
    if (in == out) { set_error("out must not alias in"); return GPE_EINVAL; }
    for (int a = 0; a < plan->g.dim; ++a)
        if (2 * plan->g.n[a] > 1024) { set_error("the refined grid exceeds 1024 points per axis"); return GPE_EUNSUPPORTED; }
    const size_t cb = plan->f64() ? 16 : 8;
    if (plan->g.dim > 1) HIPCHK(plan->tmp.ensure(cb * (size_t)plan->g.N * (plan->g.dim == 2 ? 2 : 4)));
    HIPCHK(op_prolong(plan->g, plan->f64(), plan->tw, in, out, plan->tmp.ptr, (hipStream_t)stream));
    return GPE_OK;
}

int gpe_energy_grad(gpe_plan_t* plan, const void* phi, const void* V, void* grad_phi, void* grad_V, double* dE_dbeta,
                    double* dE_domega, void* stream) {
    NEEDPTR(plan, "plan");
    NEEDPTR(phi, "phi");
    NEEDPTR(V, "V");
    NEEDPTR(grad_phi, "grad_phi");
    if (grad_phi == phi) { set_error("grad_phi must not alias phi"); return GPE_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    const size_t cb = plan->f64() ? 16 : 8;
    HIPCHK(plan->tmp.ensure(cb * (size_t)plan->g.N));
    // dE/dphi (conjugate Wirtinger, real loss) = 2 h^d H_phi phi: apply H then scale.
    HIPCHK(op_apply(plan->g, plan->f64(), 1, plan->tw, phi, V, grad_phi, plan->tmp.ptr, plan->prob.beta,
                    plan->prob.omega, true, s));
    HIPCHK(op_scale_complex(plan->g, plan->f64(), grad_phi, 2.0 * plan->g.cell, plan->g.N, s));
    if (grad_V) HIPCHK(op_density(plan->g, plan->f64(), phi, grad_V, plan->g.cell, s));
    if (dE_dbeta || dE_domega) {
        // With beta = omega = 1 the energy parts are exactly 1/2 h^d sum|phi|^4 = dE/dbeta and
        // <phi, (-L_z) phi> = dE/domega (E is affine in beta and in omega).
        double* dst = (double*)plan->red.scalars.ptr;
        HIPCHK(op_energy(plan->g, plan->f64(), plan->tw, phi, V, 1.0, plan->g.dim >= 2 ? 1.0 : 0.0, plan->red, dst, s));
        double h[4];
        HIPCHK(hipMemcpyAsync(h, dst, sizeof(h), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (dE_dbeta) *dE_dbeta = h[2];
        if (dE_domega) *dE_domega = h[3];
    }
    return GPE_OK;
}

}  // extern "C"
