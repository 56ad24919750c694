// C ABI of the solver: options, single solves, history.
#include <algorithm>
#include <tuple>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
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

// Iterations without progress after which an instance leaves the FP32 phase of a mixed-precision
// solve (neither ||r||_inf down by 10% nor E down by 1e-9 relative).  When the tolerance is below
// switch_res the FP32 phase cannot end the solve and only prepares the FP64 phase: a short window
// (kFp32WarmupWindow).  When the tolerance is at or above switch_res (coarse nested levels) the FP32
// phase may meet it alone, and a longer window (kFp32FinishWindow) lets it ride out plateaus of
// vortex rearrangement instead of handing them to the costlier FP64 phase.
constexpr int kFp32WarmupWindow = 100;
constexpr int kFp32FinishWindow = 400;

// Device workspace of one batch of equally sized instances.
struct BatchWork {
    Geo g;                 // shared grid (n); box, beta and omega are per instance in the scalars
    const Twiddles* tw;
    Reduce* red;
    DevBuf* scal;          // B solver scalars
    DevBuf* f64;           // FP64 fields (B instances)
    DevBuf* f32;           // FP32 fields (B instances)
    DevBuf* tmp;           // verification scratch (2 fields of one instance)
};

template <typename T>
int run(BatchWork& w, int B, IterFields<T> f, std::vector<Scal>& hs, const gpe_pcg_opts_t& o, hipStream_t s) {
    PhaseArgs pa;
    pa.g = w.g;
    pa.B = B;
    pa.tw = w.tw;
    pa.S = (Scal*)w.scal->ptr;
    pa.red = w.red;
    pa.region_doubles = region_doubles_for(w.g, B);
    pa.precond = o.precond;
    pa.check_every = o.check_every;
    pa.refresh_every = o.refresh_every;
    pa.use_graph = o.use_graph != 0;
    pa.final_f_r_is_rp = false;
    HIPCHK(run_phase<T>(pa, f, hs, s));
    return GPE_OK;
}

// Workspace of an instrumented run.
struct ProfileWork {
    Geo g;
    const Twiddles* tw;
    Reduce* red;
    DevBuf* scal;
    DevBuf* f64;   // FP64 fields
    DevBuf* f32;   // FP32 fields
};

// `iters` instrumented iterations of B instances of one grid at the precision of o (FP32 fields
// for an FP32 input or a mixed solve), from copies of phi[b]; the kernel durations of an iteration
// are averaged over the iterations.  Returns the number of kernels per iteration or an error.
int profile_group(ProfileWork& w, int B, const gpe_problem_t* probs, bool in_f64, const void* const* V,
                  const void* const* phi, const gpe_pcg_opts_t& opts, int iters, int cap, double* avg_ms,
                  double* bytes, char* names, hipStream_t s) {
    const Geo& g = w.g;
    const int64_t N = g.N;
    HIPCHK(reduce_init(*w.red, B, R_COUNT, std::max<size_t>(1 << 18, R_COUNT * region_doubles_for(g, B))));
    HIPCHK(w.scal->ensure(3 * sizeof(Scal) * (size_t)B));
    gpe_pcg_opts_t o = opts;
    o.tol_res_inf = 0.0;
    o.tol_energy = 0.0;
    o.max_iter = (int64_t)iters + 1000;
    std::vector<Scal> hs(B);
    for (int b = 0; b < B; ++b) hs[b] = make_scal(probs[b], make_geo(probs[b]), o);
    PhaseArgs pa;
    pa.g = g;
    pa.B = B;
    pa.tw = w.tw;
    pa.S = (Scal*)w.scal->ptr;
    pa.red = w.red;
    pa.region_doubles = region_doubles_for(g, B);
    pa.precond = o.precond;
    pa.check_every = 1;
    pa.refresh_every = 0;
    pa.final_f_r_is_rp = false;
    KernelTimer timer;
    hipError_t e = timer.init();
    const bool fp32 = !in_f64 || o.precision == 1;
    const size_t cb = in_f64 ? 16 : 8, rb = in_f64 ? 8 : 4;
    if (e == hipSuccess) {
        if (fp32) {
            IterFields<float> f = carve_fields<float>(*w.f32, (int64_t)B * N, &e);
            for (int b = 0; b < B && e == hipSuccess; ++b) {
                if (in_f64) {
                    e = convert_complex(false, phi[b], f.phi + (int64_t)b * N, N, s);
                    if (e == hipSuccess) e = convert_real(false, V[b], f.V + (int64_t)b * N, N, s);
                } else {
                    e = copy_bytes(phi[b], f.phi + (int64_t)b * N, cb * N, s);
                    if (e == hipSuccess) e = copy_bytes(V[b], f.V + (int64_t)b * N, rb * N, s);
                }
            }
            if (e == hipSuccess) e = profile_phase<float>(pa, f, hs, iters, timer, s);
        } else {
            IterFields<double> f = carve_fields<double>(*w.f64, (int64_t)B * N, &e);
            for (int b = 0; b < B && e == hipSuccess; ++b) {
                e = copy_bytes(phi[b], f.phi + (int64_t)b * N, cb * N, s);
                if (e == hipSuccess) e = copy_bytes(V[b], f.V + (int64_t)b * N, rb * N, s);
            }
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
    for (int b = 0; b < B; ++b)
        if (hs[b].done) {
            set_error("the instrumented iteration finished early (non-finite or line search)");
            return GPE_ENONFINITE;
        }
    return n;
}

Geo instance_geo(const Geo&, const gpe_problem_t& p) { return make_geo(p); }

// Solve B instances of one grid.  Inputs phi[b], V[b] are device fields in the caller's type
// (FP64 when in_f64); phi[b] receives the final iterate.  hist (device) only for B == 1.
int solve_batch(BatchWork& w, int B, const gpe_problem_t* probs, bool in_f64, const void* const* V, void* const* phi,
                const gpe_pcg_opts_t& o, double* hist, int64_t hist_cap, gpe_pcg_report_t* reports, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const Geo& g = w.g;
    const int64_t N = g.N;
    HIPCHK(reduce_init(*w.red, B, R_COUNT, std::max<size_t>(1 << 18, R_COUNT * region_doubles_for(g, B))));
    HIPCHK(w.scal->ensure(3 * sizeof(Scal) * (size_t)B));
    std::vector<Scal> hs(B);
    for (int b = 0; b < B; ++b) {
        hs[b] = make_scal(probs[b], instance_geo(g, probs[b]), o);
        if (hist && b == 0) {
            hs[b].hist = hist;
            hs[b].hist_cap = hist_cap;
        }
    }
    hipError_t e = hipSuccess;
    int st;
    const bool mixed = o.precision == 1 && in_f64;
    const size_t cb = in_f64 ? 16 : 8, rb = in_f64 ? 8 : 4;
    std::vector<int64_t> iters32(B, 0);
    auto verify_b = [&](int b, const void* ph, const void* Vb, double out[3]) -> hipError_t {
        const Geo gb = instance_geo(g, probs[b]);
        hipError_t ee = w.tmp->ensure(2 * cb * (size_t)N);
        if (ee != hipSuccess) return ee;
        return in_f64 ? verify_field<double>(gb, *w.tw, ph, Vb, w.tmp->ptr, (char*)w.tmp->ptr + cb * N, probs[b].beta,
                                             probs[b].omega, *w.red, out, s)
                      : verify_field<float>(gb, *w.tw, ph, Vb, w.tmp->ptr, (char*)w.tmp->ptr + cb * N, probs[b].beta,
                                            probs[b].omega, *w.red, out, s);
    };
    if (!in_f64) {
        IterFields<float> f = carve_fields<float>(*w.f32, (int64_t)B * N, &e);
        HIPCHK(e);
        for (int b = 0; b < B; ++b) {
            HIPCHK(copy_bytes(phi[b], f.phi + (int64_t)b * N, cb * N, s));
            HIPCHK(copy_bytes(V[b], f.V + (int64_t)b * N, rb * N, s));
        }
        if ((st = run<float>(w, B, f, hs, o, s)) != GPE_OK) return st;
        for (int b = 0; b < B; ++b) {
            iters32[b] = hs[b].n;
            HIPCHK(copy_bytes(f.phi + (int64_t)b * N, phi[b], cb * N, s));
        }
    } else {
        IterFields<double> f = carve_fields<double>(*w.f64, (int64_t)B * N, &e);
        HIPCHK(e);
        if (mixed) {
            IterFields<float> f32 = carve_fields<float>(*w.f32, (int64_t)B * N, &e);
            HIPCHK(e);
            for (int b = 0; b < B; ++b) {
                HIPCHK(convert_complex(false, phi[b], f32.phi + (int64_t)b * N, N, s));
                HIPCHK(convert_real(false, V[b], f32.V + (int64_t)b * N, N, s));
                hs[b].precision = 1;
                hs[b].tol_res = std::max(o.tol_res_inf, o.switch_res);
                hs[b].stall_window = o.tol_res_inf < o.switch_res ? kFp32WarmupWindow : kFp32FinishWindow;
            }
            if ((st = run<float>(w, B, f32, hs, o, s)) != GPE_OK) return st;
            HIPCHK(convert_complex(true, f32.phi, f.phi, (int64_t)B * N, s));
            for (int b = 0; b < B; ++b) {
                iters32[b] = hs[b].n;
                const bool failed = hs[b].status == ST_NONFINITE;
                hs[b].precision = 0;
                hs[b].tol_res = o.tol_res_inf;
                hs[b].stall_window = 0;
                hs[b].stagnant = 0;
                hs[b].linesearch_fail = 0;
                if (!failed && hs[b].n < o.max_iter) {
                    hs[b].done = 0;
                    hs[b].status = ST_OK;
                }
            }
        } else {
            for (int b = 0; b < B; ++b) HIPCHK(copy_bytes(phi[b], f.phi + (int64_t)b * N, cb * N, s));
        }
        for (int b = 0; b < B; ++b) HIPCHK(copy_bytes(V[b], f.V + (int64_t)b * N, rb * N, s));
        // FP64 phase.  An instance whose tracked residual met tol but whose fresh one did not
        // resumes (from L phi recomputed, CG memory cleared) with an internal target lowered by a
        // tenth per attempt, so that it iterates past the rounding gap between the two; the report
        // below turns any instance still above tol into GPE_NOT_CONVERGED.
        for (int attempt = 0; attempt < 8; ++attempt) {
            bool any = false;
            for (int b = 0; b < B; ++b) any = any || !hs[b].done;
            if (!any) break;
            if ((st = run<double>(w, B, f, hs, o, s)) != GPE_OK) return st;
            bool again = false;
            for (int b = 0; b < B; ++b) {
                if (hs[b].status != ST_OK || hs[b].n >= o.max_iter || o.tol_energy > 0.0) continue;
                double chk[3];
                HIPCHK(verify_b(b, f.phi + (int64_t)b * N, f.V + (int64_t)b * N, chk));
                if (chk[2] > o.tol_res_inf) {
                    hs[b].done = 0;
                    hs[b].tol_res = o.tol_res_inf * (0.9 - 0.1 * attempt);
                    again = true;
                }
            }
            if (!again) break;
        }
        for (int b = 0; b < B; ++b) HIPCHK(copy_bytes(f.phi + (int64_t)b * N, phi[b], cb * N, s));
    }
    const auto t1 = std::chrono::steady_clock::now();
    const double secs = std::chrono::duration<double>(t1 - t0).count();
    int worst = GPE_OK;
    for (int b = 0; b < B; ++b) {
        double chk[3];
        HIPCHK(verify_b(b, phi[b], V[b], chk));
        gpe_pcg_report_t& r = reports[b];
        std::memset(&r, 0, sizeof(r));
        r.status = status_of(hs[b].status);
        // success means the fresh FP64 residual of the returned state meets the residual tolerance
        if (r.status == GPE_OK && o.tol_energy == 0.0 && !(chk[2] <= o.tol_res_inf)) r.status = GPE_NOT_CONVERGED;
        r.switched = mixed ? 1 : 0;
        r.iters = hs[b].n;
        r.iters_fp32 = in_f64 ? (mixed ? iters32[b] : 0) : hs[b].n;
        r.restarts = hs[b].restarts;
        r.halvings = hs[b].halvings;
        r.E = chk[0];
        r.lambda = chk[1];
        r.res_inf = chk[2];
        r.dE = std::fabs(hs[b].E - hs[b].E_prev);
        r.dphi_inf = hs[b].dphi;
        r.seconds = secs;
        worst = worse_status(worst, r.status);
    }
    return worst;
}

// One grid group on one stream: twiddles, workspace, the solve, release.
int solve_group(int B, const gpe_problem_t* gp, bool in_f64, const void* const* gV, void* const* gphi,
                const gpe_pcg_opts_t& o, gpe_pcg_report_t* rep, hipStream_t s) {
    Geo g = make_geo(gp[0]);
    Twiddles tw;
    Reduce red;
    DevBuf scal, f64, f32, tmp;
    int st;
    hipError_t e = build_twiddles(g, tw);
    if (e == hipSuccess) {
        BatchWork w{g, &tw, &red, &scal, &f64, &f32, &tmp};
        st = solve_batch(w, B, gp, in_f64, gV, gphi, o, nullptr, 0, rep, s);
    } else {
        set_error(std::string("twiddle tables: ") + hipGetErrorString(e));
        st = GPE_EHIP;
    }
    (void)hipStreamSynchronize(s);
    for (int a = 0; a < 3; ++a) {
        tw.t64[a].release();
        tw.t32[a].release();
    }
    red.parts.release();
    red.counters.release();
    red.scalars.release();
    scal.release();
    f64.release();
    f32.release();
    tmp.release();
    return st;
}

// Runs task(k, stream_k) for k = 0 .. n-1 concurrently: task 0 on the caller's thread and stream,
// the others each on a stream (default priority) and host thread of their own, after the work
// already queued on the caller's stream.  Returns a HIP or argument error of any task, else the
// worst status, with the message moved to the caller's thread.
template <class F>
int run_concurrent(int n, hipStream_t s, F task) {
    if (n < 2) return task(0, s);
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    std::vector<hipStream_t> ss(n, s);
    int created = 1;
    hipError_t e = hipEventRecord(ev, s);  // the inputs are ready on the caller's stream
    {
        std::lock_guard<std::mutex> lock(capture_mutex());
        for (int k = 1; k < n && e == hipSuccess; ++k) {
            e = hipStreamCreateWithFlags(&ss[k], hipStreamNonBlocking);
            if (e == hipSuccess) {
                created = k + 1;
                e = hipStreamWaitEvent(ss[k], ev, 0);
            }
        }
    }
    std::vector<int> st(n, GPE_OK);
    std::vector<std::string> err(n);
    if (e == hipSuccess) {
        auto run = [&](int k) {
            st[k] = task(k, ss[k]);
            if (st[k] < 0) err[k] = gpe_last_error();  // the message is thread-local
        };
        std::vector<std::thread> th;
        for (int k = 1; k < n; ++k) {
            try {
                th.emplace_back([&, k] {
                    (void)hipSetDevice(dev);  // the current device is per host thread
                    run(k);
                });
            } catch (...) {
                run(k);  // no thread: this task runs before the caller's instead of beside it
            }
        }
        run(0);
        for (auto& t : th) t.join();
    }
    for (int k = 1; k < created; ++k) (void)hipStreamSynchronize(ss[k]);
    {
        std::lock_guard<std::mutex> lock(capture_mutex());
        for (int k = 1; k < created; ++k) (void)hipStreamDestroy(ss[k]);
        (void)hipEventDestroy(ev);
    }
    HIPCHK(e);
    // a HIP or argument error first (the tasks' outputs are then unreliable), else the worst status
    // (per-instance reports stay valid for the others), with the message of the task that set it
    for (int k = 0; k < n; ++k)
        if (st[k] == GPE_EHIP || st[k] == GPE_EINVAL) {
            set_error(err[k]);
            return st[k];
        }
    int worst = GPE_OK, from = -1;
    for (int k = 0; k < n; ++k)
        if (worse_status(worst, st[k]) != worst) {
            worst = worse_status(worst, st[k]);
            from = k;
        }
    if (worst < 0 && from >= 0) set_error(err[from]);
    return worst;
}

// Instances of one grid solved as kSolveStreams independent parts, each on its own stream driven by
// its own host thread.  A part's kernels then run while another part's are in a different phase
// (one loading fields, the other transforming), which a single batched launch cannot do: every
// workgroup of a launch passes through the same phases at the same time.  Each instance's
// arithmetic does not depend on how the instances are grouped, so results are bit-identical to a
// single batch.  Measured on the eight-start 512^2 step: one batch 1.14 s (mixed) / 3.01 s (FP64),
// two parts 0.97 / 2.45 s, four 0.98 / 2.50 s, eight 1.11 / 2.72 s.
constexpr int kSolveStreams = 2;

int solve_group_split(int B, const gpe_problem_t* gp, bool in_f64, const void* const* gV, void* const* gphi,
                      const gpe_pcg_opts_t& o, gpe_pcg_report_t* rep, hipStream_t s) {
    const int P = std::min(B, kSolveStreams);
    std::vector<int> b0(P + 1);
    for (int k = 0; k <= P; ++k) b0[k] = (int)((int64_t)B * k / P);
    return run_concurrent(P, s, [&](int k, hipStream_t sk) {
        return solve_group(b0[k + 1] - b0[k], gp + b0[k], in_f64, gV + b0[k], gphi + b0[k], o, rep + b0[k], sk);
    });
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
    o->use_graph = 1;
    o->line_search = 0;
}

int gpe_pcg_solve(gpe_plan_t* plan, const void* V, void* phi_inout, const gpe_pcg_opts_t* opts,
                  gpe_pcg_report_t* report, void* stream) {
    if (!plan) { set_error("plan is NULL"); return GPE_EINVAL; }
    if (!V || !phi_inout) { set_error("V and phi_inout must be device pointers"); return GPE_EINVAL; }
    if (!report) { set_error("report is NULL"); return GPE_EINVAL; }
    int st = validate_opts(opts);
    if (st != GPE_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const gpe_pcg_opts_t& o = *opts;
    int64_t cap = 0;
    double* hist = nullptr;
    if (o.record_history) {
        cap = std::min<int64_t>(o.max_iter + 1, 1 << 20);
        HIPCHK(plan->hist.ensure(sizeof(double) * 8 * (size_t)cap));
        HIPCHK(hipMemsetAsync(plan->hist.ptr, 0, sizeof(double) * 8 * (size_t)cap, s));
        hist = (double*)plan->hist.ptr;
    }
    BatchWork w{plan->g, &plan->tw, &plan->red, &plan->scal, &plan->solver, plan->f64() ? &plan->solver32 : &plan->solver,
                &plan->tmp};
    const void* Vs[1] = {V};
    void* phis[1] = {phi_inout};
    st = solve_batch(w, 1, &plan->prob, plan->f64(), Vs, phis, o, hist, cap, report, s);
    plan->hist_rows = o.record_history ? std::min<int64_t>(report->iters + 1, cap) : 0;
    if (st < 0 && st != GPE_EHIP) {
        set_error(st == GPE_ENONFINITE ? "non-finite value during the iteration" : "line search found no energy decrease");
    }
    return st;
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
    const void* Vs[1] = {V};
    const void* phis[1] = {phi};
    ProfileWork w{plan->g, &plan->tw, &plan->red, &plan->scal, &plan->solver, &plan->solver32};
    return profile_group(w, 1, &plan->prob, plan->f64(), Vs, phis, *opts, iters, cap, avg_ms, bytes, names,
                         (hipStream_t)stream);
}

int gpe_pcg_profile_batched(int count, const gpe_problem_t* probs, int dtype, const void* const* V,
                            const void* const* phi, const gpe_pcg_opts_t* opts, int iters, int cap, double* avg_ms,
                            double* bytes, char* names, void* stream) {
    if (count < 1 || !probs || !V || !phi || !avg_ms || !bytes || !names) {
        set_error("invalid batch arguments");
        return GPE_EINVAL;
    }
    if (dtype != GPE_F64 && dtype != GPE_F32) { set_error("dtype must be GPE_F64 or GPE_F32"); return GPE_EINVAL; }
    int st = validate_opts(opts);
    if (st != GPE_OK) return st;
    if (iters < 1 || cap < 1) { set_error("iters and cap must be >= 1"); return GPE_EINVAL; }
    for (int i = 0; i < count; ++i) {
        if ((st = validate_problem(&probs[i])) != GPE_OK) return st;
        if (!V[i] || !phi[i]) { set_error("NULL field in batch"); return GPE_EINVAL; }
        for (int a = 0; a < 3; ++a)
            if (probs[i].dim != probs[0].dim || (a < probs[0].dim && probs[i].n[a] != probs[0].n[a])) {
                set_error("a profiled batch must share one grid");
                return GPE_EINVAL;
            }
    }
    const Geo g = make_geo(probs[0]);
    Twiddles tw;
    Reduce red;
    DevBuf scal, f64, f32;
    hipError_t e = build_twiddles(g, tw);
    if (e != hipSuccess) {
        set_error(std::string("twiddle tables: ") + hipGetErrorString(e));
        return GPE_EHIP;
    }
    ProfileWork w{g, &tw, &red, &scal, &f64, &f32};
    st = profile_group(w, count, probs, dtype == GPE_F64, V, phi, *opts, iters, cap, avg_ms, bytes, names,
                       (hipStream_t)stream);
    (void)hipStreamSynchronize((hipStream_t)stream);
    for (int a = 0; a < 3; ++a) {
        tw.t64[a].release();
        tw.t32[a].release();
    }
    red.parts.release();
    red.counters.release();
    red.scalars.release();
    scal.release();
    f64.release();
    f32.release();
    return st;
}

int gpe_pcg_solve_batched(int count, const gpe_problem_t* probs, int dtype, void* const* V, void* const* phi_inout,
                          const gpe_pcg_opts_t* opts, gpe_pcg_report_t* reports, void* stream) {
    if (count < 1 || !probs || !V || !phi_inout || !reports) { set_error("invalid batch arguments"); return GPE_EINVAL; }
    if (dtype != GPE_F64 && dtype != GPE_F32) { set_error("dtype must be GPE_F64 or GPE_F32"); return GPE_EINVAL; }
    int st = validate_opts(opts);
    if (st != GPE_OK) return st;
    for (int i = 0; i < count; ++i) {
        if ((st = validate_problem(&probs[i])) != GPE_OK) return st;
        if (!V[i] || !phi_inout[i]) { set_error("NULL field in batch"); return GPE_EINVAL; }
    }
    hipStream_t s = (hipStream_t)stream;
    // group the instances by grid (dim, n): one batch of fused launches per group
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    auto key = [&](int i) {
        const gpe_problem_t& p = probs[i];
        return std::make_tuple(p.dim, p.n[0], p.dim > 1 ? p.n[1] : 1, p.dim > 2 ? p.n[2] : 1);
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
    // grid groups [first[g], first[g+1]) of `order`, solved concurrently (a latency-bound group of
    // small grids then runs beside a bandwidth-bound group of large ones)
    std::vector<size_t> first{0};
    for (size_t i = 1; i < order.size(); ++i)
        if (key(order[i]) != key(order[i - 1])) first.push_back(i);
    first.push_back(order.size());
    const int G = (int)first.size() - 1;
    const bool in_f64 = dtype == GPE_F64;
    std::vector<gpe_problem_t> gp(count);
    std::vector<const void*> gV(count);
    std::vector<void*> gphi(count);
    std::vector<gpe_pcg_report_t> rep(count);
    for (int i = 0; i < count; ++i) {
        gp[i] = probs[order[i]];
        gV[i] = V[order[i]];
        gphi[i] = phi_inout[order[i]];
    }
    const gpe_pcg_opts_t& o = *opts;
    const int worst = run_concurrent(G, s, [&](int g, hipStream_t sg) {
        const size_t a = first[g];
        return solve_group_split((int)(first[g + 1] - a), gp.data() + a, in_f64, gV.data() + a, gphi.data() + a,
                                 o, rep.data() + a, sg);
    });
    if (worst == GPE_EHIP || worst == GPE_EINVAL) return worst;
    for (int i = 0; i < count; ++i) reports[order[i]] = rep[i];
    return worst;
}

int gpe_pcg_solve_nested(int count, int levels, const gpe_problem_t* coarsest, int dtype, void* const* V,
                         void* const* phi_coarse, void* const* phi_fine, const gpe_pcg_opts_t* opts, double tol_coarse,
                         gpe_pcg_report_t* reports, void* stream) {
    if (count < 1 || levels < 1 || !coarsest || !V || !phi_coarse || !phi_fine || !reports) {
        set_error("invalid nested-solve arguments");
        return GPE_EINVAL;
    }
    if (dtype != GPE_F64 && dtype != GPE_F32) { set_error("dtype must be GPE_F64 or GPE_F32"); return GPE_EINVAL; }
    if (!(tol_coarse > 0.0) || !std::isfinite(tol_coarse)) { set_error("tol_coarse must be positive"); return GPE_EINVAL; }
    if (levels > 8) { set_error("at most 8 nested levels (grids of 8 to 1024 points per axis)"); return GPE_EUNSUPPORTED; }
    int st = validate_opts(opts);
    if (st != GPE_OK) return st;
    // level l: the coarsest problem with 2^l times the points per axis, same box
    std::vector<std::vector<gpe_problem_t>> probs(levels, std::vector<gpe_problem_t>(coarsest, coarsest + count));
    for (int l = 0; l < levels; ++l)
        for (int i = 0; i < count; ++i) {
            for (int a = 0; a < probs[l][i].dim; ++a) probs[l][i].n[a] = coarsest[i].n[a] << l;
            if ((st = validate_problem(&probs[l][i])) != GPE_OK) return st;
            if (!V[(size_t)l * count + i]) { set_error("NULL potential in nested solve"); return GPE_EINVAL; }
        }
    for (int i = 0; i < count; ++i)
        if (!phi_coarse[i] || !phi_fine[i]) { set_error("NULL field in nested solve"); return GPE_EINVAL; }
    struct Owned {  // device memory of the call, released on every return path
        std::vector<DevBuf> bufs;
        Twiddles tw;
        ~Owned() {
            for (DevBuf& b : bufs) b.release();
            for (int a = 0; a < 3; ++a) {
                tw.t64[a].release();
                tw.t32[a].release();
            }
        }
    } own;
    own.bufs.resize((size_t)levels + 1);  // one field set per coarse level, plus interpolation scratch
    hipStream_t s = (hipStream_t)stream;
    const size_t cb = dtype == GPE_F64 ? 16 : 8;
    std::vector<std::vector<void*>> phis(levels, std::vector<void*>(count));
    for (int l = 0; l < levels; ++l)
        for (int i = 0; i < count; ++i) {
            if (l == levels - 1) {
                phis[l][i] = phi_fine[i];
                continue;
            }
            size_t off = 0, total = 0;
            for (int j = 0; j < count; ++j) total += cb * (size_t)make_geo(probs[l][j]).N;
            HIPCHK(own.bufs[l].ensure(total));
            for (int j = 0; j < i; ++j) off += cb * (size_t)make_geo(probs[l][j]).N;
            phis[l][i] = (char*)own.bufs[l].ptr + off;
        }
    for (int i = 0; i < count; ++i)
        HIPCHK(hipMemcpyAsync(phis[0][i], phi_coarse[i], cb * (size_t)make_geo(probs[0][i]).N, hipMemcpyDeviceToDevice, s));
    int worst = GPE_OK;
    for (int l = 0; l < levels; ++l) {
        gpe_pcg_opts_t o = *opts;
        if (l < levels - 1) o.tol_res_inf = tol_coarse;
        std::vector<void*> Vl(V + (size_t)l * count, V + (size_t)(l + 1) * count);
        st = gpe_pcg_solve_batched(count, probs[l].data(), dtype, Vl.data(), phis[l].data(), &o,
                                   reports + (size_t)l * count, stream);
        if (st < 0 && st != GPE_ELINESEARCH) return st;
        if (l == levels - 1) {
            worst = st;
            break;
        }
        // interpolate every instance onto the next grid (the solver renormalises its start)
        for (int i = 0; i < count; ++i) {
            const Geo g = make_geo(probs[l][i]);
            HIPCHK(build_twiddles(g, own.tw));
            if (g.dim > 1) HIPCHK(own.bufs[levels].ensure(cb * (size_t)g.N * (g.dim == 2 ? 2 : 4)));
            HIPCHK(op_prolong(g, dtype == GPE_F64, own.tw, phis[l][i], phis[l + 1][i], own.bufs[levels].ptr, s));
            HIPCHK(hipStreamSynchronize(s));  // the tables are rebuilt for the next instance
        }
    }
    return worst;
}

}  // extern "C"
