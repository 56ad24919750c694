// Shared declarations of the PCG iteration (pcg.hip) and its host driver (solve.hip).
#pragma once

#include "internal.hpp"
#include "passes.hpp"

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

// Partial-sum regions (one per reducing kernel) and their ticket counters.
enum : int { R_A1 = 0, R_A3 = 1, R_B0 = 2, R_B1 = 3, R_B2 = 4, R_C = 5, R_COUNT = 6 };

template <typename T>
struct IterCtx {
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

// Phase A sums: residual maximum, non-finite flag, and the inner products of the CG update.
enum : int {
    A_RES = 0, A_NF, A_RPR, A_RPPR, A_PRPHI, A_PRPR, A_PRPP, A_RPP, A_PPPHI, A_PPPP, A_RPHI, A_PHIPHI,
    A_K = 12
};
constexpr unsigned A_MAXMASK = (1u << A_RES) | (1u << A_NF);

// Phase B sums: rotation forms, <phat, L phat>, <phi, L phat>, and the line-search polynomials.
enum : int {
    B_CR = 0, B_AR, B_BR, B_C, B_B, B_AA, B_AB, B_ACA, B_CACA, B_CAB, B_BB, B_AC, B_SB, B_SC, B_NF,
    B_K = 15
};
constexpr unsigned B_MAXMASK = 1u << B_NF;

// Phase C sums: <phi, L phi>, sum|phi|^4, ||phi||^2, ||phi_{n+1} - phi_n||_inf, non-finite flag.
enum : int { C_A = 0, C_Q4, C_N2, C_DPHI, C_NF, C_K = 5 };
constexpr unsigned C_MAXMASK = (1u << C_DPHI) | (1u << C_NF);

template <typename T>
__device__ __forceinline__ void res_sums(double* acc, C2<T> r) {
    const double m = sqrt((double)abs2(r));
    acc[A_RES] = fmax(acc[A_RES], m);
    if (!isfinite(m)) acc[A_NF] = 1.0;
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
