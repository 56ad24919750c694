// Host driver of the PG / PCG ground-state solver (Algorithms 1-2) and its C ABI entry points.
//
// A solve runs one or two phases.  FP64 mode: one FP64 phase to tol.  Mixed mode: an FP32 phase
// (fields and transforms in FP32, every scalar in FP64) until ||r||_inf <= switch_res, a
// stagnation of the residual, or a failed line search; then the iterate is promoted to FP64,
// L phi is recomputed from it, the CG memory is reset and an FP64 phase finishes to tol.
// Within a phase, iterations are queued in chunks of `check_every`; the host polls the
// per-instance scalars between chunks (kernels of a finished instance return immediately).
// Every `refresh_every` iterations L phi and its scalars are recomputed from phi, bounding the
// drift of the linearity update.  The reported E, lambda and ||r||_inf are recomputed in FP64
// from the final iterate.
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"
#include "pcg.hpp"
#include "plan.hpp"
#include "solver.hpp"

namespace gpe {

// ---------------------------------------------------------------------------------------------
// Small kernels of the driver
// ---------------------------------------------------------------------------------------------
template <typename TI, typename TO>
__global__ void k_convert(const TI* in, TO* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (TO)in[i];
}

template <typename T>
__global__ void k_zero(T* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (T)0;
}

// Per-instance sum of |phi|^2 over fixed chunks (deterministic partials: nbpi per instance).
template <typename T>
__global__ __launch_bounds__(256) void k_norm_partial(const C2<T>* phi, int64_t N, int nbpi, double* parts) {
    __shared__ double red[8];
    const int b = blockIdx.x / nbpi, blk = blockIdx.x - b * nbpi;
    const int64_t chunk = (N + nbpi - 1) / nbpi, lo = (int64_t)blk * chunk, hi = min(N, lo + chunk);
    double v[1] = {0.0};
    for (int64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) v[0] += (double)abs2(phi[(int64_t)b * N + j]);
    __shared__ double o1[1];
    block_reduce<1>(v, red, o1, 0u);
    if (threadIdx.x == 0) parts[blockIdx.x] = o1[0];
}

// Scale instance b by 1/||phi||, each block reducing the instance's partials itself (same order).
template <typename T>
__global__ __launch_bounds__(256) void k_norm_apply(C2<T>* phi, int64_t N, int nbpi, const double* parts,
                                                    const Scal* S) {
    __shared__ double red[8];
    __shared__ double inv;
    const int b = blockIdx.x / nbpi, blk = blockIdx.x - b * nbpi;
    double v[1] = {0.0};
    for (int k = threadIdx.x; k < nbpi; k += blockDim.x) v[0] += parts[(size_t)b * nbpi + k];
    __shared__ double o1[1];
    block_reduce<1>(v, red, o1, 0u);
    if (threadIdx.x == 0) inv = 1.0 / sqrt(S[b].cell * o1[0]);
    __syncthreads();
    const int64_t chunk = (N + nbpi - 1) / nbpi, lo = (int64_t)blk * chunk, hi = min(N, lo + chunk);
    for (int64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) {
        const int64_t i = (int64_t)b * N + j;
        phi[i] = scl(phi[i], (T)inv);
    }
}

// Fill the scalars of a (re)started iterate from the energy parts computed with beta = 1:
// parts = {<phi,T phi>, <phi,V phi>, 1/2 h^d sum|phi|^4, <phi,R phi>}.
__global__ void k_scal_from_parts(Scal* S, const double* parts, int restart_cg) {
    if (threadIdx.x != 0) return;
    Scal& s = *S;
    const double kin = parts[0], pot = parts[1], q4 = 2.0 * parts[2], rot = parts[3];
    s.a = kin + pot + rot;
    s.aR = rot;
    s.q4 = q4;
    s.lam = s.a + s.beta * q4;
    s.lamt = kin + pot + s.beta * q4;
    const double E = s.a + 0.5 * s.beta * q4;
    if (restart_cg) {
        s.nrm2 = 1.0;
        s.have_prev = 0;
        s.has_step = 0;
        s.E_prev = E;
        s.best_res = 1e300;
        s.best_E = 1e300;
        s.best_n = s.n;
    }
    s.E = E;
}

// Fresh FP64 check of a final iterate: lambda = Re<phi, H phi>/||phi||^2, ||H phi - lambda phi||_inf.
template <typename T>
__global__ __launch_bounds__(256) void k_verify_dot(const C2<T>* phi, const C2<T>* hphi, int64_t N, double* parts) {
    __shared__ double red[16];
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        v[0] += (double)redot(phi[i], hphi[i]);
        v[1] += (double)abs2(phi[i]);
    }
    __shared__ double o2[2];
    block_reduce<2>(v, red, o2, 0u);
    if (threadIdx.x < 2) parts[blockIdx.x * 2 + threadIdx.x] = o2[threadIdx.x];
}

template <typename T>
__global__ __launch_bounds__(256) void k_verify_res(const C2<T>* phi, const C2<T>* hphi, int64_t N, const double* dots,
                                                    int ndot, double* maxparts, double* lam_out) {
    __shared__ double red[16];
    __shared__ double lam_s;
    double v[2] = {0.0, 0.0};
    for (int k = threadIdx.x; k < ndot; k += blockDim.x) {
        v[0] += dots[2 * k];
        v[1] += dots[2 * k + 1];
    }
    __shared__ double t2[2];
    block_reduce<2>(v, red, t2, 0u);
    if (threadIdx.x == 0) {
        lam_s = t2[0] / t2[1];
        if (blockIdx.x == 0) *lam_out = lam_s;
    }
    __syncthreads();
    const double lam = lam_s;
    double m[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const C2<T> p = phi[i], h = hphi[i];
        const double rx = (double)h.x - lam * (double)p.x, ry = (double)h.y - lam * (double)p.y;
        m[0] = fmax(m[0], sqrt(rx * rx + ry * ry));
    }
    __shared__ double o1[1];
    block_reduce<1>(m, red, o1, 1u);
    if (threadIdx.x == 0) maxparts[blockIdx.x] = o1[0];
}

__global__ void k_max_collect(const double* parts, int n, double* dst) {
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int i = 0; i < n; ++i) m = fmax(m, parts[i]);
        *dst = m;
    }
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename TI, typename TO>
static hipError_t convert(const void* in, void* out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((k_convert<TI, TO>), dim3(blocks_for(n)), dim3(256), 0, s, (const TI*)in, (TO*)out, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Workspace of one precision: 8 complex fields + V for B instances.
// ---------------------------------------------------------------------------------------------
template <typename T>
static IterFields<T> carve(DevBuf& buf, int64_t BN, hipError_t* err) {
    const size_t cf = sizeof(C2<T>) * (size_t)BN;
    const size_t need = 8 * cf + sizeof(T) * (size_t)BN + 256;
    *err = buf.ensure(need);
    IterFields<T> f{};
    if (*err != hipSuccess) return f;
    char* p = (char*)buf.ptr;
    C2<T>** slots[8] = {&f.phi, &f.Lphi, &f.r, &f.rp, &f.pp, &f.pr, &f.lp, &f.w};
    for (int k = 0; k < 8; ++k) *slots[k] = (C2<T>*)(p + k * cf);
    f.V = (T*)(p + 8 * cf);
    return f;
}

// Recompute L phi and the scalars of the current iterate (instance-wise, B = 1 per call).
template <typename T>
static hipError_t refresh_instance(const Geo& g, const Twiddles& tw, IterFields<T>& f, int64_t off, Scal* Sd,
                                   double beta, double omega, Reduce& red, bool restart_cg, hipStream_t s) {
    const bool f64 = sizeof(T) == 8;
    hipError_t e;
    // L phi into Lphi (w as the transform intermediate)
    if ((e = op_apply(g, f64, 1, tw, f.phi + off, f.V + off, f.Lphi + off, f.w + off, beta, omega, false, s)) !=
        hipSuccess)
        return e;
    // Mid-phase refreshes stop here: the scalars already describe the iterate that the pending
    // step produces, and L phi (fresh) is only combined linearly by that step.
    if (!restart_cg) return hipSuccess;
    double* parts = (double*)red.scalars.ptr + 16;
    if ((e = op_energy(g, f64, tw, f.phi + off, f.V + off, 1.0, omega, red, parts, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scal_from_parts, dim3(1), dim3(64), 0, s, Sd, parts, 1);
    return hipGetLastError();
}

template <typename T>
static hipError_t normalize_all(IterFields<T>& f, int B, int64_t N, Scal* Sd, Reduce& red, hipStream_t s) {
    const int nbpi = (int)std::max<int64_t>(1, std::min<int64_t>(256, N / 2048));
    double* parts = (double*)red.parts.ptr;
    hipLaunchKernelGGL(k_norm_partial<T>, dim3(nbpi * B), dim3(256), 0, s, f.phi, N, nbpi, parts);
    hipLaunchKernelGGL(k_norm_apply<T>, dim3(nbpi * B), dim3(256), 0, s, f.phi, N, nbpi, parts, Sd);
    return hipGetLastError();
}

template <typename T>
static hipError_t zero_cg_memory(IterFields<T>& f, int64_t BN, hipStream_t s) {
    hipLaunchKernelGGL(k_zero<T>, dim3(blocks_for(2 * BN)), dim3(256), 0, s, (T*)f.rp, 2 * BN);
    hipLaunchKernelGGL(k_zero<T>, dim3(blocks_for(2 * BN)), dim3(256), 0, s, (T*)f.pp, 2 * BN);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// One phase for B instances of one grid.
// ---------------------------------------------------------------------------------------------
// A non-blocking stream of default priority ordered after the work queued on another stream;
// synchronised and destroyed with the object.
struct PrivateStream {
    hipStream_t s = nullptr;
    hipError_t create_after(hipStream_t other) {
        std::lock_guard<std::mutex> lock(capture_mutex());
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) {
            s = nullptr;
            return e;
        }
        hipEvent_t ev;
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
        e = hipEventRecord(ev, other);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
        (void)hipEventDestroy(ev);
        return e;
    }
    ~PrivateStream() {
        if (s) {
            (void)hipStreamSynchronize(s);
            std::lock_guard<std::mutex> lock(capture_mutex());
            (void)hipStreamDestroy(s);
        }
    }
};

// An instantiated graph captured from work queued on one stream.  Every graph call of the library
// (capture and instantiation, launch, destruction) holds capture_mutex: instantiating a graph and
// destroying its executable allocate and free the device memory that holds the graph's kernel
// arguments, which the mutex keeps out of other host threads' capture windows like every other
// allocation and free, and no two host threads run graph calls at once.  Captures only kernel
// launches: no memory-set or copy nodes.
struct GraphExec {
    hipGraphExec_t exec = nullptr;
    template <class F>
    hipError_t capture(hipStream_t s, F enqueue) {
        std::lock_guard<std::mutex> lock(capture_mutex());
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        hipError_t qe = enqueue();
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(s, &g);
        if (qe != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return qe != hipSuccess ? qe : e;
        }
        e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) exec = nullptr;
        return e;
    }
    hipError_t launch(hipStream_t s) {
        std::lock_guard<std::mutex> lock(capture_mutex());
        return hipGraphLaunch(exec, s);
    }
    void reset() {
        if (exec) {
            std::lock_guard<std::mutex> lock(capture_mutex());
            (void)hipGraphExecDestroy(exec);
        }
        exec = nullptr;
    }
    ~GraphExec() { reset(); }
};

template <typename T>
hipError_t run_phase(PhaseArgs& pa, IterFields<T> f, std::vector<Scal>& host_S, hipStream_t s_caller) {
    const Geo& g = pa.g;
    const int B = pa.B;
    const int64_t N = g.N;
    hipError_t e;
    // Graph capture is not possible on the legacy default stream (the usual caller's stream): with
    // graphs the phase runs on a private stream that first waits for the caller's queued work; the
    // loop below ends with a synchronisation of that stream, so nothing is left queued on it.
    const bool want_graph = pa.use_graph && pa.check_every % 2 == 0;
    PrivateStream own;
    hipStream_t s = s_caller;
    if (want_graph) {
        if ((e = own.create_after(s_caller)) != hipSuccess) return e;
        s = own.s;
    }
    // scalars to the device
    // three versioned state slots (after the step, after the convergence test, after the direction);
    // an iteration starts from S_dir
    Scal* S_dir = pa.S + 2 * B;
    for (int k = 0; k < 3; ++k)
        if ((e = hipMemcpyAsync(pa.S + k * B, host_S.data(), sizeof(Scal) * B, hipMemcpyHostToDevice, s)) != hipSuccess)
            return e;
    if ((e = normalize_all<T>(f, B, N, S_dir, *pa.red, s)) != hipSuccess) return e;
    if ((e = zero_cg_memory<T>(f, (int64_t)B * N, s)) != hipSuccess) return e;
    for (int b = 0; b < B; ++b) {
        Geo gb = g;
        for (int a = 0; a < 3; ++a) {
            gb.L[a] = host_S[b].L[a];
            gb.h[a] = host_S[b].h[a];
            gb.dk[a] = host_S[b].dk[a];
        }
        gb.cell = host_S[b].cell;
        if ((e = refresh_instance<T>(gb, *pa.tw, f, (int64_t)b * N, S_dir + b, host_S[b].beta, host_S[b].omega,
                                     *pa.red, true, s)) != hipSuccess)
            return e;
    }
    IterCtx<T> c;
    c.g = g;
    c.B = B;
    c.tw = pa.tw;
    c.f = f;
    c.S = pa.S;
    c.parts = (double*)pa.red->parts.ptr;
    c.region_doubles = pa.region_doubles;
    c.counters = (unsigned int*)pa.red->counters.ptr;
    c.precond = pa.precond;
    c.pointwise_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, N / 1024));
    int64_t since_refresh = 0;
    int64_t queued = 0;
    int64_t max_iter = 0;
    for (int b = 0; b < B; ++b) max_iter = std::max<int64_t>(max_iter, host_S[b].max_iter);
    // A chunk of check_every iterations launches the same kernels with the same arguments every
    // time (the r / r_{n-1} roles swap each iteration, so an even chunk ends where it started): after
    // one chunk ran eagerly, the next is captured into a graph and every later chunk replays it.
    GraphExec graph;
    int64_t chunks = 0;
    // device list of the unfinished instances (used when they are not contiguous), owned by the phase
    struct OwnedBuf : DevBuf {
        ~OwnedBuf() { release(); }
    } imap;
    std::vector<int> imap_host;
    if ((e = imap.ensure(sizeof(int) * (size_t)B)) != hipSuccess) return e;
    for (;;) {
        // host-side guard: every queued iteration either advances n or finishes the instance
        if (queued > 2 * max_iter + 4 * (int64_t)pa.check_every + 64) return hipErrorUnknown;
        queued += pa.check_every;
        if (!graph.exec && want_graph && chunks >= 1) {
            if ((e = graph.capture(s, [&] {
                     for (int k = 0; k < pa.check_every; ++k) {
                         hipError_t ee = enqueue_iteration<T>(c, s);
                         if (ee != hipSuccess) return ee;
                         std::swap(c.f.r, c.f.rp);
                     }
                     return hipSuccess;
                 })) != hipSuccess)
                return e;
        }
        if (graph.exec) {
            if ((e = graph.launch(s)) != hipSuccess) return e;
        } else {
            for (int k = 0; k < pa.check_every; ++k) {
                if ((e = enqueue_iteration<T>(c, s)) != hipSuccess) return e;
                std::swap(c.f.r, c.f.rp);
            }
        }
        ++chunks;
        since_refresh += pa.check_every;
        if ((e = hipMemcpyAsync(host_S.data(), S_dir, sizeof(Scal) * B, hipMemcpyDeviceToHost, s)) != hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        bool all_done = true;
        for (int b = 0; b < B; ++b) all_done = all_done && host_S[b].done;
        if (all_done) break;
        // Converged instances are left out of later launches (a masked instance still costs its
        // workgroups' state and row reads in every pass): a contiguous run of unfinished instances is
        // launched as a range, any other set through the device list of their indices.  Tiles and row
        // layout keep following all B instances.  The stream is idle here, so the list can be
        // rewritten and the graph holding the old launches can go; the next chunk captures anew.
        {
            std::vector<int> run;
            for (int b = 0; b < B; ++b)
                if (!host_S[b].done) run.push_back(b);
            const int nl = (int)run.size();
            const bool contiguous = run.back() - run.front() + 1 == nl;
            const bool same = contiguous ? (!c.g.imap && c.g.b0 == run.front() && (c.g.bl > 0 ? c.g.bl : B) == nl)
                                         : (c.g.imap && c.g.bl == nl && run == imap_host);
            if (!same) {
                if (contiguous) {
                    c.g.imap = nullptr;
                    c.g.b0 = run.front();
                } else {
                    imap_host = run;
                    if ((e = hipMemcpyAsync(imap.ptr, imap_host.data(), sizeof(int) * nl, hipMemcpyHostToDevice, s)) !=
                        hipSuccess)
                        return e;
                    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
                    c.g.imap = (const int*)imap.ptr;
                    c.g.b0 = 0;
                }
                c.g.bl = nl;
                graph.reset();
            }
        }
        // Every queued iteration of an unfinished instance ran, so r/rp roles are in sync.
        if (pa.refresh_every > 0 && since_refresh >= pa.refresh_every) {
            since_refresh = 0;
            for (int b = 0; b < B; ++b) {
                if (host_S[b].done) continue;
                Geo gb = g;
                for (int a = 0; a < 3; ++a) {
                    gb.L[a] = host_S[b].L[a];
                    gb.h[a] = host_S[b].h[a];
                    gb.dk[a] = host_S[b].dk[a];
                }
                gb.cell = host_S[b].cell;
                if ((e = refresh_instance<T>(gb, *pa.tw, c.f, (int64_t)b * N, S_dir + b, host_S[b].beta,
                                             host_S[b].omega, *pa.red, false, s)) != hipSuccess)
                    return e;
            }
        }
    }
    pa.final_f_r_is_rp = false;
    return hipSuccess;
}

// Instrumented iterations: initialise like run_phase, then run exactly `iters` iterations with
// every launch bracketed by events (the solver must not finish meanwhile: tol = 0 is expected).
template <typename T>
hipError_t profile_phase(PhaseArgs& pa, IterFields<T> f, std::vector<Scal>& host_S, int iters, KernelTimer& timer,
                         hipStream_t s) {
    const Geo& g = pa.g;
    const int64_t N = g.N;
    hipError_t e;
    Scal* S_dir = pa.S + 2 * pa.B;
    for (int k = 0; k < 3; ++k)
        if ((e = hipMemcpyAsync(pa.S + k * pa.B, host_S.data(), sizeof(Scal) * pa.B, hipMemcpyHostToDevice, s)) !=
            hipSuccess)
            return e;
    if ((e = normalize_all<T>(f, pa.B, N, S_dir, *pa.red, s)) != hipSuccess) return e;
    if ((e = zero_cg_memory<T>(f, (int64_t)pa.B * N, s)) != hipSuccess) return e;
    for (int b = 0; b < pa.B; ++b) {
        if ((e = refresh_instance<T>(g, *pa.tw, f, (int64_t)b * N, S_dir + b, host_S[b].beta, host_S[b].omega,
                                     *pa.red, true, s)) != hipSuccess)
            return e;
    }
    IterCtx<T> c;
    c.g = g;
    c.B = pa.B;
    c.tw = pa.tw;
    c.f = f;
    c.S = pa.S;
    c.parts = (double*)pa.red->parts.ptr;
    c.region_doubles = pa.region_doubles;
    c.counters = (unsigned int*)pa.red->counters.ptr;
    c.precond = pa.precond;
    c.pointwise_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, N / 1024));
    c.timer = &timer;
    for (int k = 0; k < iters; ++k) {
        if ((e = enqueue_iteration<T>(c, s)) != hipSuccess) return e;
        if ((e = timer.collect()) != hipSuccess) return e;
        std::swap(c.f.r, c.f.rp);
    }
    return hipMemcpy(host_S.data(), S_dir, sizeof(Scal) * pa.B, hipMemcpyDeviceToHost);
}

template hipError_t profile_phase<double>(PhaseArgs&, IterFields<double>, std::vector<Scal>&, int, KernelTimer&,
                                          hipStream_t);
template hipError_t profile_phase<float>(PhaseArgs&, IterFields<float>, std::vector<Scal>&, int, KernelTimer&,
                                         hipStream_t);

template hipError_t run_phase<double>(PhaseArgs&, IterFields<double>, std::vector<Scal>&, hipStream_t);
template hipError_t run_phase<float>(PhaseArgs&, IterFields<float>, std::vector<Scal>&, hipStream_t);

// Fresh FP64 (or FP32 plan) energy, lambda and residual of one field.
template <typename T>
hipError_t verify_field(const Geo& g, const Twiddles& tw, const void* phi, const void* V, void* hphi, void* tmp,
                        double beta, double omega, Reduce& red, double out[3], hipStream_t s) {
    const bool f64 = sizeof(T) == 8;
    hipError_t e;
    if ((e = op_apply(g, f64, 1, tw, phi, V, hphi, tmp, beta, omega, true, s)) != hipSuccess) return e;
    double* sc = (double*)red.scalars.ptr;
    double* parts = (double*)red.parts.ptr;
    const int nb = 256;
    hipLaunchKernelGGL(k_verify_dot<T>, dim3(nb), dim3(256), 0, s, (const C2<T>*)phi, (const C2<T>*)hphi, g.N, parts);
    hipLaunchKernelGGL(k_verify_res<T>, dim3(nb), dim3(256), 0, s, (const C2<T>*)phi, (const C2<T>*)hphi, g.N, parts, nb,
                       parts + 2 * nb, sc + 32);
    hipLaunchKernelGGL(k_max_collect, dim3(1), dim3(64), 0, s, parts + 2 * nb, nb, sc + 33);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = op_energy(g, f64, tw, phi, V, beta, omega, red, sc + 36, s)) != hipSuccess) return e;
    double h[8];
    if ((e = hipMemcpyAsync(h, sc + 32, sizeof(h), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    out[0] = h[4] + h[5] + h[6] + h[7];  // E
    out[1] = h[0];                        // lambda
    out[2] = h[1];                        // ||r||_inf
    return hipSuccess;
}

template hipError_t verify_field<double>(const Geo&, const Twiddles&, const void*, const void*, void*, void*, double,
                                         double, Reduce&, double*, hipStream_t);
template hipError_t verify_field<float>(const Geo&, const Twiddles&, const void*, const void*, void*, void*, double,
                                        double, Reduce&, double*, hipStream_t);

hipError_t convert_complex(bool to64, const void* in, void* out, int64_t n, hipStream_t s) {
    return to64 ? convert<float, double>(in, out, 2 * n, s) : convert<double, float>(in, out, 2 * n, s);
}
hipError_t convert_real(bool to64, const void* in, void* out, int64_t n, hipStream_t s) {
    return to64 ? convert<float, double>(in, out, n, s) : convert<double, float>(in, out, n, s);
}
hipError_t copy_bytes(const void* in, void* out, size_t bytes, hipStream_t s) {
    return hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, s);
}

template <typename T>
IterFields<T> carve_fields(DevBuf& buf, int64_t BN, hipError_t* err) {
    return carve<T>(buf, BN, err);
}
template IterFields<double> carve_fields<double>(DevBuf&, int64_t, hipError_t*);
template IterFields<float> carve_fields<float>(DevBuf&, int64_t, hipError_t*);

// Host template of the per-instance scalars.
Scal make_scal(const gpe_problem_t& p, const Geo& g, const gpe_pcg_opts_t& o) {
    Scal s;
    std::memset(&s, 0, sizeof(s));
    s.beta = p.beta;
    s.omega = p.omega;
    s.cell = g.cell;
    s.dim = p.dim;
    for (int a = 0; a < 3; ++a) {
        s.L[a] = g.L[a];
        s.dk[a] = g.dk[a];
        s.h[a] = g.h[a];
    }
    s.tol_res = o.tol_res_inf;
    s.tol_energy = o.tol_energy;
    s.theta_default = o.theta_default;
    s.method = o.method;
    s.beta_rule = o.beta_rule;
    s.line_search = o.line_search;
    s.max_halvings = o.max_halvings;
    s.precond = o.precond;
    s.max_iter = o.max_iter;
    s.switch_res = o.switch_res;
    s.best_res = 1e300;
    s.best_E = 1e300;
    return s;
}

int validate_opts(const gpe_pcg_opts_t* o) {
    if (!o) { set_error("opts is NULL"); return GPE_EINVAL; }
    if (o->method != 0 && o->method != 1) { set_error("method must be 0 (PG) or 1 (PCG)"); return GPE_EINVAL; }
    if (o->precond < GPE_P_NONE || o->precond > GPE_P_C2) { set_error("unknown preconditioner"); return GPE_EINVAL; }
    if (!(o->tol_res_inf >= 0.0) || !(o->tol_energy >= 0.0)) { set_error("tolerances must be >= 0"); return GPE_EINVAL; }
    if (o->max_iter < 0) { set_error("max_iter must be >= 0"); return GPE_EINVAL; }
    if (o->precision != 0 && o->precision != 1) { set_error("precision must be 0 (FP64) or 1 (mixed)"); return GPE_EINVAL; }
    if (o->beta_rule != 0 && o->beta_rule != 1) { set_error("beta_rule must be 0 (PR) or 1 (FR)"); return GPE_EINVAL; }
    if (o->line_search < 0 || o->line_search > 3) {
        set_error("line_search must be 0 (decrease test), 1 (Armijo), 2 (full) or 3 (strong Wolfe)");
        return GPE_EINVAL;
    }
    if (o->max_halvings < 0 || o->max_halvings > 60) { set_error("max_halvings must be in [0, 60]"); return GPE_EINVAL; }
    if (!(o->theta_default > 0.0)) { set_error("theta_default must be positive"); return GPE_EINVAL; }
    if (o->check_every < 1) { set_error("check_every must be >= 1"); return GPE_EINVAL; }
    if (o->refresh_every < 0) { set_error("refresh_every must be >= 0"); return GPE_EINVAL; }
    return GPE_OK;
}

int status_of(int st) {
    switch (st) {
        case ST_OK: return GPE_OK;
        case ST_NOT_CONVERGED: return GPE_NOT_CONVERGED;
        case ST_LINESEARCH: return GPE_ELINESEARCH;
        case ST_NONFINITE: return GPE_ENONFINITE;
        default: return GPE_EHIP;
    }
}

}  // namespace gpe
