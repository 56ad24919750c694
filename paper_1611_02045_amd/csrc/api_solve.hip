// C ABI of the solver: options, single solves, history.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"
#include "plan.hpp"
#include "solver.hpp"

using namespace gpe;

#define HIPCHK(expr)                                                                    \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess) {                                                         \
            set_error(std::string("HIP error in " #expr ": ") + hipGetErrorString(_e)); \
            return GPE_EHIP;                                                            \
        }                                                                               \
    } while (0)

namespace {

// Run one phase with precision T on fields f, then return the host scalars.
template <typename T>
int phase(gpe_plan* plan, IterFields<T> f, std::vector<Scal>& hs, const gpe_pcg_opts_t& o, hipStream_t s) {
    PhaseArgs pa;
    pa.g = plan->g;
    pa.B = 1;
    pa.tw = &plan->tw;
    pa.S = (Scal*)plan->scal.ptr;
    pa.red = &plan->red;
    pa.region_doubles = region_doubles_for(plan->g, 1);
    pa.precond = o.precond;
    pa.check_every = o.check_every;
    pa.refresh_every = o.refresh_every;
    pa.final_f_r_is_rp = false;
    HIPCHK(run_phase<T>(pa, f, hs, s));
    return GPE_OK;
}

}  // namespace

extern "C" {

void gpe_pcg_opts_default(gpe_pcg_opts_t* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->method = 1;
    o->precond = GPE_P_COMBINED;
    o->tol_res_inf = 1e-8;
    o->tol_energy = 0.0;
    o->max_iter = 20000;
    o->precision = 0;
    o->beta_rule = 0;
    o->switch_res = 1e-6;
    o->theta_default = 0.1;
    o->max_halvings = 30;
    o->refresh_every = 50;
    o->check_every = 16;
    o->record_history = 0;
}

int gpe_pcg_solve(gpe_plan_t* plan, const void* V, void* phi_inout, const gpe_pcg_opts_t* opts,
                  gpe_pcg_report_t* report, void* stream) {
    if (!plan) { set_error("plan is NULL"); return GPE_EINVAL; }
    if (!V || !phi_inout) { set_error("V and phi_inout must be device pointers"); return GPE_EINVAL; }
    if (!report) { set_error("report is NULL"); return GPE_EINVAL; }
    int st = validate_opts(opts);
    if (st != GPE_OK) return st;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    const gpe_pcg_opts_t& o = *opts;
    const Geo& g = plan->g;
    const int64_t N = g.N;
    std::memset(report, 0, sizeof(*report));

    HIPCHK(reduce_init(plan->red, 1, R_COUNT, std::max<size_t>(1 << 18, R_COUNT * region_doubles_for(g, 1))));
    HIPCHK(plan->scal.ensure(sizeof(Scal)));
    Scal base = make_scal(plan->prob, g, o);
    int64_t cap = 0;
    if (o.record_history) {
        cap = std::min<int64_t>(o.max_iter + 1, 1 << 20);
        HIPCHK(plan->hist.ensure(sizeof(double) * 8 * (size_t)cap));
        HIPCHK(hipMemsetAsync(plan->hist.ptr, 0, sizeof(double) * 8 * (size_t)cap, s));
        base.hist = (double*)plan->hist.ptr;
        base.hist_cap = cap;
    }
    std::vector<Scal> hs(1, base);
    hipError_t e = hipSuccess;
    const bool mixed = o.precision == 1 && plan->f64();

    void* final_phi = nullptr;  // solver-owned final iterate (plan precision or FP64)
    bool final_is_64 = plan->f64();
    if (!plan->f64()) {
        IterFields<float> f = carve_fields<float>(plan->solver, N, &e);
        HIPCHK(e);
        HIPCHK(copy_bytes(phi_inout, f.phi, sizeof(float) * 2 * N, s));
        HIPCHK(copy_bytes(V, f.V, sizeof(float) * N, s));
        if ((st = phase<float>(plan, f, hs, o, s)) != GPE_OK) return st;
        final_phi = f.phi;
        report->iters_fp32 = hs[0].n;
    } else {
        IterFields<double> f = carve_fields<double>(plan->solver, N, &e);
        HIPCHK(e);
        if (mixed) {
            IterFields<float> f32 = carve_fields<float>(plan->solver32, N, &e);
            HIPCHK(e);
            HIPCHK(convert_complex(false, phi_inout, f32.phi, N, s));
            HIPCHK(convert_real(false, V, f32.V, N, s));
            hs[0].precision = 1;
            hs[0].tol_res = std::max(o.tol_res_inf, o.switch_res);
            hs[0].stall_window = 100;
            if ((st = phase<float>(plan, f32, hs, o, s)) != GPE_OK) return st;
            report->iters_fp32 = hs[0].n;
            report->switched = 1;
            HIPCHK(convert_complex(true, f32.phi, f.phi, N, s));
            const bool failed = hs[0].status == ST_NONFINITE;
            hs[0].precision = 0;
            hs[0].tol_res = o.tol_res_inf;
            hs[0].stall_window = 0;
            hs[0].stagnant = 0;
            hs[0].linesearch_fail = 0;
            if (!failed && hs[0].n < o.max_iter) {
                hs[0].done = 0;
                hs[0].status = ST_OK;
            }
        } else {
            HIPCHK(copy_bytes(phi_inout, f.phi, sizeof(double) * 2 * N, s));
        }
        HIPCHK(copy_bytes(V, f.V, sizeof(double) * N, s));
        if (!hs[0].done) {
            // FP64 phase; resume if the tracked residual met tol while the fresh one did not
            for (int attempt = 0; attempt < 4; ++attempt) {
                if ((st = phase<double>(plan, f, hs, o, s)) != GPE_OK) return st;
                if (hs[0].status != ST_OK || hs[0].n >= o.max_iter) break;
                double chk[3];
                HIPCHK(verify_field<double>(g, plan->tw, f.phi, f.V, f.lp, f.w, plan->prob.beta, plan->prob.omega,
                                            plan->red, chk, s));
                if (chk[2] <= o.tol_res_inf || o.tol_energy > 0.0) break;
                hs[0].done = 0;
            }
        }
        final_phi = f.phi;
    }
    // copy the iterate back and verify it
    const size_t cbytes = (plan->f64() ? sizeof(double) : sizeof(float)) * 2 * (size_t)N;
    HIPCHK(copy_bytes(final_phi, phi_inout, cbytes, s));
    (void)final_is_64;
    HIPCHK(plan->tmp.ensure(2 * cbytes));
    double chk[3];
    if (plan->f64())
        HIPCHK(verify_field<double>(g, plan->tw, phi_inout, V, plan->tmp.ptr, (char*)plan->tmp.ptr + cbytes,
                                    plan->prob.beta, plan->prob.omega, plan->red, chk, s));
    else
        HIPCHK(verify_field<float>(g, plan->tw, phi_inout, V, plan->tmp.ptr, (char*)plan->tmp.ptr + cbytes,
                                   plan->prob.beta, plan->prob.omega, plan->red, chk, s));
    const auto t1 = std::chrono::steady_clock::now();
    report->status = status_of(hs[0].status);
    report->iters = hs[0].n;
    report->restarts = hs[0].restarts;
    report->halvings = hs[0].halvings;
    report->E = chk[0];
    report->lambda = chk[1];
    report->res_inf = chk[2];
    report->dE = std::fabs(hs[0].E - hs[0].E_prev);
    report->dphi_inf = hs[0].dphi;
    report->seconds = std::chrono::duration<double>(t1 - t0).count();
    plan->hist_rows = o.record_history ? std::min<int64_t>(hs[0].n + 1, cap) : 0;
    if (report->status < 0) {
        set_error(report->status == GPE_ENONFINITE ? "non-finite value during the iteration"
                                                   : "line search found no energy decrease");
    }
    return report->status;
}

int gpe_pcg_history(gpe_plan_t* plan, double* hist, int cap) {
    if (!plan || !hist || cap < 0) { set_error("invalid arguments"); return GPE_EINVAL; }
    const int64_t rows = std::min<int64_t>(plan->hist_rows, cap);
    if (rows > 0) HIPCHK(hipMemcpy(hist, plan->hist.ptr, sizeof(double) * 8 * (size_t)rows, hipMemcpyDeviceToHost));
    return (int)rows;
}

int gpe_pcg_profile(gpe_plan_t* plan, const void* V, const void* phi, const gpe_pcg_opts_t* opts, int iters, int cap,
                    double* avg_ms, double* bytes, char* names, void* stream) {
    if (!plan || !V || !phi || !avg_ms || !bytes || !names) { set_error("NULL argument"); return GPE_EINVAL; }
    int st = validate_opts(opts);
    if (st != GPE_OK) return st;
    if (iters < 1 || cap < 1) { set_error("iters and cap must be >= 1"); return GPE_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    const Geo& g = plan->g;
    const int64_t N = g.N;
    HIPCHK(reduce_init(plan->red, 1, R_COUNT, std::max<size_t>(1 << 18, R_COUNT * region_doubles_for(g, 1))));
    HIPCHK(plan->scal.ensure(sizeof(Scal)));
    gpe_pcg_opts_t o = *opts;
    o.tol_res_inf = 0.0;
    o.tol_energy = 0.0;
    o.max_iter = (int64_t)iters + 1000;
    std::vector<Scal> hs(1, make_scal(plan->prob, g, o));
    PhaseArgs pa;
    pa.g = g;
    pa.B = 1;
    pa.tw = &plan->tw;
    pa.S = (Scal*)plan->scal.ptr;
    pa.red = &plan->red;
    pa.region_doubles = region_doubles_for(g, 1);
    pa.precond = o.precond;
    pa.check_every = 1;
    pa.refresh_every = 0;
    pa.final_f_r_is_rp = false;
    KernelTimer timer;
    hipError_t e = timer.init();
    const bool fp32 = !plan->f64() || o.precision == 1;
    if (e == hipSuccess) {
        if (fp32) {
            IterFields<float> f = carve_fields<float>(plan->f64() ? plan->solver32 : plan->solver, N, &e);
            if (e == hipSuccess) {
                if (plan->f64()) {
                    e = convert_complex(false, phi, f.phi, N, s);
                    if (e == hipSuccess) e = convert_real(false, V, f.V, N, s);
                } else {
                    e = copy_bytes(phi, f.phi, sizeof(float) * 2 * N, s);
                    if (e == hipSuccess) e = copy_bytes(V, f.V, sizeof(float) * N, s);
                }
            }
            if (e == hipSuccess) e = profile_phase<float>(pa, f, hs, iters, timer, s);
        } else {
            IterFields<double> f = carve_fields<double>(plan->solver, N, &e);
            if (e == hipSuccess) e = copy_bytes(phi, f.phi, sizeof(double) * 2 * N, s);
            if (e == hipSuccess) e = copy_bytes(V, f.V, sizeof(double) * N, s);
            if (e == hipSuccess) e = profile_phase<double>(pa, f, hs, iters, timer, s);
        }
    }
    int n = 0;
    if (e == hipSuccess) {
        n = std::min(timer.slots, cap);
        for (int k = 0; k < n; ++k) {
            avg_ms[k] = timer.launches[k] ? timer.total_ms[k] / (double)timer.launches[k] : 0.0;
            bytes[k] = timer.bytes[k];
            std::memset(names + 32 * k, 0, 32);
            std::strncpy(names + 32 * k, timer.names[k] ? timer.names[k] : "?", 31);
        }
    }
    timer.destroy();
    HIPCHK(e);
    if (hs[0].done) { set_error("the instrumented iteration finished early (non-finite or line search)"); return GPE_ENONFINITE; }
    return n;
}

int gpe_pcg_solve_batched(int, const gpe_problem_t*, int, void* const*, void* const*, const gpe_pcg_opts_t*,
                          gpe_pcg_report_t*, void*) {
    set_error("gpe_pcg_solve_batched: not implemented yet");
    return GPE_EUNSUPPORTED;
}

int gpe_adjoint_solve(gpe_plan_t*, const void*, const void*, const void*, void*, const gpe_pcg_opts_t*,
                      gpe_pcg_report_t*, void*) {
    set_error("gpe_adjoint_solve: not implemented yet");
    return GPE_EUNSUPPORTED;
}

}  // extern "C"
