// Shared declarations of the PCG iteration (pcg.hip) and its host driver (solve.hip).
#pragma once

#include "internal.hpp"
#include "launch.hpp"

namespace gpe {

// Fields of one iteration (B instances back to back, N points each).
template <typename T>
struct IterFields {
    C2<T>* phi;   // phi_n
    C2<T>* Lphi;  // L phi_n, L = T + V - omega L_z (carried by linearity)
    C2<T>* r;     // r_n
    C2<T>* rp;    // r_{n-1}
    C2<T>* pp;    // p_{n-1}, overwritten by p_n
    C2<T>* pr;    // P r_n
    C2<T>* lp;    // L phat_n
    C2<T>* w;     // transform intermediate
    T* V;         // potential
};

// Partial-sum regions of the reducing passes, and their collapsed counterparts (one row per
// instance) used when a pass has more workgroups per instance than a consumer should re-reduce.
enum : int {
    R_A1 = 0, R_A3, R_B, R_A1C = R_B + 3, R_A3C, R_BC, R_COUNT  // R_B spans three regions (x, y, z passes)
};
constexpr int kAbsorbRows = 256;

// Optional per-kernel timing of an iteration (gpe_pcg_profile): every launch of the iteration
// records a start/stop event pair with the launch itself, which brackets that kernel's execution
// alone (the dispatch gaps between kernels are not counted).
struct KernelTimer {
    static constexpr int MAX = 16;
    int n = 0;
    hipEvent_t ev0[MAX] = {}, ev1[MAX] = {};
    const char* names[MAX] = {};
    double bytes[MAX] = {};
    double total_ms[MAX] = {};
    int64_t launches[MAX] = {};
    int slots = 0;
    hipError_t init() {
        for (int k = 0; k < MAX; ++k) {
            hipError_t e = hipEventCreate(&ev0[k]);
            if (e == hipSuccess) e = hipEventCreate(&ev1[k]);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    void destroy() {
        for (int k = 0; k < MAX; ++k) {
            if (ev0[k]) (void)hipEventDestroy(ev0[k]);
            if (ev1[k]) (void)hipEventDestroy(ev1[k]);
        }
    }
    // the start/stop event pair the next launch records (its own execution interval), or null
    const LaunchEvents* next(const char* name, double b) {
        if (n >= MAX) return nullptr;
        names[n] = name;
        bytes[n] = b;
        pair = LaunchEvents{ev0[n], ev1[n]};
        ++n;
        return &pair;
    }
    // after an iteration: wait, and accumulate the launch durations
    hipError_t collect() {
        if (n == 0) return hipSuccess;
        hipError_t e = hipEventSynchronize(ev1[n - 1]);
        if (e != hipSuccess) return e;
        for (int k = 0; k < n; ++k) {
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, ev0[k], ev1[k]);
            if (e != hipSuccess) return e;
            total_ms[k] += ms;
            launches[k] += 1;
        }
        slots = n;
        n = 0;
        return hipSuccess;
    }
    LaunchEvents pair{};
};

template <typename T>
struct IterCtx {
    KernelTimer* timer = nullptr;
    Geo g;
    int B;
    const Twiddles* tw;
    IterFields<T> f;
    Scal* S;
    double* parts;
    size_t region_doubles;
    unsigned int* counters;
    int precond;
    int pointwise_blocks;
};

// Phase A sums: residual maximum, non-finite flag, the inner products of the CG update, and the
// fresh scalars of the (just updated) iterate: <phi, L phi>, sum|phi|^4, ||phi||^2,
// ||phi_n - phi_{n-1}||_inf.
enum : int {
    A_RES = 0, A_NF, A_RPR, A_RPPR, A_PRPHI, A_PRPR, A_PRPP, A_RPP, A_PPPHI, A_PPPP, A_RPHI, A_PHIPHI,
    A_A, A_Q4, A_N2, A_DPHI, A_K = 16
};
constexpr unsigned A_MAXMASK = (1u << A_RES) | (1u << A_NF) | (1u << A_DPHI);

// Phase B sums: rotation forms, <phat, L phat>, <phi, L phat>, and the line-search polynomials.
enum : int {
    B_CR = 0, B_AR, B_BR, B_C, B_B, B_AA, B_AB, B_ACA, B_CACA, B_CAB, B_BB, B_AC, B_SB, B_SC, B_NF,
    B_K = 15
};
constexpr unsigned B_MAXMASK = 1u << B_NF;


// Pending retraction step of the previous iteration, applied pointwise at the start of phase A:
// phi <- c_phi phi + c_p p, L phi <- c_L L phi + c_Lp L phat (linearity of L), with the fresh
// sums of the new iterate.  ph and lph hold the loaded values and receive the updated ones; pp and
// lpv are p and L phat at the same point (read only when has_step).
template <typename T>
__device__ __forceinline__ void apply_step_pref(const IterFields<T>& f, const Scal& s, int64_t i, C2<T>& ph,
                                                C2<T>& lph, C2<T> pp, C2<T> lpv, double* acc) {
    if (s.has_step) {
        const C2<T> np = add(scl(ph, (T)s.c_phi), scl(pp, (T)s.c_p));
        const C2<T> nl = add(scl(lph, (T)s.c_L), scl(lpv, (T)s.c_Lp));
        acc[A_DPHI] = fmax(acc[A_DPHI], (double)abs2(sub(np, ph)));  // squared; the root is taken once
        f.phi[i] = np;
        f.Lphi[i] = nl;
        ph = np;
        lph = nl;
    }
    const double r2 = abs2(ph);
    acc[A_A] += (double)redot(ph, lph);
    acc[A_Q4] += r2 * r2;
    acc[A_N2] += r2;
}

// As apply_step_pref, loading p and L phat itself.
template <typename T>
__device__ __forceinline__ void apply_step(const IterFields<T>& f, const Scal& s, int64_t i, C2<T>& ph, C2<T>& lph,
                                           double* acc) {
    apply_step_pref<T>(f, s, i, ph, lph, s.has_step ? f.pp[i] : C2<T>{}, s.has_step ? f.lp[i] : C2<T>{}, acc);
}

template <typename T>
__device__ __forceinline__ void res_sums(double* acc, C2<T> r) {
    const double m2 = (double)abs2(r);  // max of |r|^2; the root of the maximum is taken once
    acc[A_RES] = fmax(acc[A_RES], m2);
    if (!isfinite(m2)) acc[A_NF] = 1.0;
}

template <typename T>
__device__ __forceinline__ void cg_sums(double* acc, C2<T> r, C2<T> pr, C2<T> rp, C2<T> pp, C2<T> ph) {
    acc[A_RPR] += (double)redot(r, pr);
    acc[A_RPPR] += (double)redot(rp, pr);
    acc[A_PRPHI] += (double)redot(pr, ph);
    acc[A_PRPR] += (double)abs2(pr);
    acc[A_PRPP] += (double)redot(pr, pp);
    acc[A_RPP] += (double)redot(r, pp);
    acc[A_PPPHI] += (double)redot(pp, ph);
    acc[A_PPPP] += (double)abs2(pp);
    acc[A_RPHI] += (double)redot(r, ph);
    acc[A_PHIPHI] += (double)abs2(ph);
}

template <typename T>
hipError_t enqueue_iteration(const IterCtx<T>& c, hipStream_t s);

}  // namespace gpe
