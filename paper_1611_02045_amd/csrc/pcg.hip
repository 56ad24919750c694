// One iteration of the projected preconditioned gradient / conjugate gradient method on the
// unit sphere (Algorithms 1-2 with the step control of Sections 5.1-5.2), as a short chain of
// fused passes over the fields of B independent instances of one grid:
//
//   A  r = L phi + beta|phi|^2 phi - lambda phi, ||r||_inf, preconditioner (Section 5.5)
//        [x pass: residual + P_V^{1/2} prologue + forward x]  [middle passes: y (z), multiplier
//        1/(lambda~ + |k|^2/2)]  [x pass: inverse x + P_V^{1/2} epilogue + CG reductions]
//   B  p = -P r + beta_cg p_{n-1} - Re<d, phi> phi, phat = p/||p||, L phat  (Section 5.2)
//        [x pass, y/z passes; the last one also forms every line-search sum]
//   The retraction phi <- (cos t phi + sin t phat)/nu, L phi <- (cos t L phi + sin t L phat)/nu
//        (linearity of L: no transform of phi_{n+1} is needed) is applied pointwise at the start
//        of the next iteration's phase A, which also reduces the fresh <phi, L phi>, sum|phi|^4
//        and ||phi||^2 of the new iterate.
//
// Scalar logic (FP64) runs at the start of the pass that consumes a reduction: every workgroup
// reduces the previous pass's per-block partials in the same fixed order and runs the same
// logic, so all workgroups agree bit for bit without atomics, fences or a serial tail; one
// workgroup per instance publishes the state into a versioned slot (S_step after the step, S_res
// after the convergence test, S_dir after the CG direction), so no pass writes a slot it reads.
// The convergence test runs at the start of the first middle pass, beta_cg and the descent test
// at the start of the direction pass, and the step at the start of the next iteration.  lambda, lambda~ and E of the next iterate follow exactly from the line-search sums
// (they are quadratic and quartic forms in (cos t, sin t)), so the residual of iteration n+1 can
// be formed in the same pass that applies the step.  Every kernel returns at once for instances
// whose `done` flag is set, so surplus iterations queued after convergence are no-ops.
//
// Line search: E(cos t phi + sin t phat) - E(phi) is a trigonometric polynomial in t whose
// coefficients are the reductions <phat, L phat>, <phi, L phat>, <phi, L phi> and sums of
// A = |phi|^2, B = Re(conj(phi) phat), C = |phat|^2 products; the trial steps of the paper's
// heuristic are therefore evaluated exactly, for any number of trials, from one pass.
#include <cmath>

#include "internal.hpp"
#include "launch.hpp"
#include "pcg.hpp"

namespace gpe {

// ---------------------------------------------------------------------------------------------
// Shared pieces
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double pv_diag(const Scal& S, double V, double rho) {
    return S.lamt + V + S.beta * rho;
}

// Pointwise factor of the diagonal preconditioner: P_V^{1/2} (kind 1), P_V (kind 2) or 1, in the
// field precision.
template <typename T>
__device__ __forceinline__ T pscale(int kind, double d) {
    if constexpr (sizeof(T) == 8) {
        return kind == 1 ? rsqrt(d) : kind == 2 ? 1.0 / d : 1.0;
    } else {
        const float df = (float)d;
        return kind == 1 ? rsqrtf(df) : kind == 2 ? 1.0f / df : 1.0f;
    }
}

// Rotation coefficient of the directional symbol (see ops.hip) from per-instance geometry.
template <int AX>
__device__ __forceinline__ double rot_coef_s(const Scal& S, const LineCtx& lc) {
    if (S.dim < 2 || S.omega == 0.0) return 0.0;
    if (AX == 0) return S.omega * coord_of(lc.i1, S.L[1], S.h[1]);
    if (AX == 1) return -S.omega * coord_of(lc.i1, S.L[0], S.h[0]);
    return 0.0;
}

__device__ __forceinline__ void hist_row(Scal& S, int col, double v) {
    if (S.hist && S.n < S.hist_cap) S.hist[S.n * 8 + col] = v;
}

// Convergence test at the top of iteration n (Section 5.3; reading: ||r_n||_inf <= tol).
__device__ __forceinline__ void fin_residual(Scal& S, const double* t) {
    {
        const double res = sqrt(t[A_RES]), nonfinite = t[A_NF];  // the sums hold squared maxima
        // fresh scalars of phi_n (the step of the previous iteration has just been applied)
        S.a = S.cell * t[A_A];
        S.q4 = S.cell * t[A_Q4];
        S.nrm2 = S.cell * t[A_N2];
        S.dphi = sqrt(t[A_DPHI]);
        S.E = S.a + 0.5 * S.beta * S.q4;
        S.has_step = 0;
        S.res = res;
        hist_row(S, 0, (double)S.n);
        hist_row(S, 1, S.E);
        hist_row(S, 2, S.lam);
        hist_row(S, 3, res);
        if (nonfinite > 0.0 || !isfinite(res) || !isfinite(S.E)) {
            S.status = ST_NONFINITE;
            S.nonfinite = 1;
            S.done = 1;
        } else if (res <= S.tol_res) {
            S.status = ST_OK;
            S.done = 1;
        } else if (S.tol_energy > 0.0 && S.n > 0 && fabs(S.E - S.E_prev) <= S.tol_energy) {
            S.status = ST_OK;
            S.done = 1;
        } else if (S.n >= S.max_iter) {
            S.status = ST_NOT_CONVERGED;
            S.done = 1;
        } else if (S.stall_window > 0) {
            // mixed precision: leave the FP32 phase once neither the residual (by 10%) nor the
            // energy (by 1e-9 relative) has improved for stall_window iterations.  The residual
            // alone plateaus for hundreds of iterations while vortices still move; the energy
            // keeps falling then, and stops only at the FP32 floor.
            const bool better_res = res < 0.9 * S.best_res;
            const bool better_E = S.E < S.best_E - 1e-9 * fabs(S.E);
            if (better_res) S.best_res = res;
            if (better_E) S.best_E = S.E;
            if (better_res || better_E) {
                S.best_n = S.n;
            } else if (S.n - S.best_n >= S.stall_window) {
                S.stagnant = 1;
                S.status = ST_OK;
                S.done = 1;
            }
        }
    }
}

// CG direction from the A-phase sums (Section 5.2, readings: beta_0 = 0, PR+ with the stored
// denominator, restart when Re<r, p> >= 0).
__device__ __forceinline__ void fin_direction(Scal& S, const double* t) {
    if (!S.done) {
        const double w = S.cell;
        const double rPr = w * t[A_RPR], rpPr = w * t[A_RPPR], Prphi = w * t[A_PRPHI], PrPr = w * t[A_PRPR];
        const double Prpp = w * t[A_PRPP], rpp = w * t[A_RPP], ppphi = w * t[A_PPPHI], pppp = w * t[A_PPPP];
        const double rphi = w * t[A_RPHI], phiphi = w * t[A_PHIPHI];
        double beta = 0.0;
        if (S.method == 1 && S.have_prev && S.rPr_prev > 0.0) {
            beta = S.beta_rule == 1 ? rPr / S.rPr_prev : fmax((rPr - rpPr) / S.rPr_prev, 0.0);
        }
        double rho = -Prphi + beta * ppphi;                 // Re<d, phi>
        double rp = -rPr + beta * rpp - rho * rphi;         // Re<r, p>
        S.restarted = 0;
        if (!(rp < 0.0)) {  // not a descent direction: gradient step
            beta = 0.0;
            rho = -Prphi;
            rp = -rPr - rho * rphi;
            S.restarted = 1;
            S.restarts += 1;
        }
        const double dd = PrPr - 2.0 * beta * Prpp + beta * beta * pppp;
        const double pp = dd - 2.0 * rho * rho + rho * rho * phiphi;
        S.beta_cg = beta;
        S.rho = rho;
        S.pnorm = sqrt(fmax(pp, 0.0));
        S.rPr_cur = rPr;
        S.d1 = rp;
        if (!(S.pnorm > 0.0) || !isfinite(S.pnorm) || !isfinite(rPr)) {
            S.status = ST_NONFINITE;
            S.nonfinite = 1;
            S.done = 1;
        }
        hist_row(S, 5, beta);
        hist_row(S, 7, (double)S.restarted);
    }
}

// Energy change along the great circle, from the B-phase sums (see the file comment).
// q0..q4 = sum A B, sum A (C - A), sum B^2, sum (C - A) B, sum (C - A)^2 (times h^d).
__device__ __forceinline__ double delta_energy(double c, double s, double a, double b, double cc, double beta,
                                               double q0, double q1, double q2, double q3, double q4) {
    const double quad = s * s * (cc - a) + 2.0 * c * s * b;
    const double quart = 4.0 * c * s * q0 + 2.0 * s * s * q1 + 4.0 * c * c * s * s * q2 + 4.0 * c * s * s * s * q3 +
                         s * s * s * s * q4;
    return quad + 0.5 * beta * quart;
}

// Slope and curvature of delta_energy in t.  In double angles (C2, S2 = cos 2t, sin 2t; C4, S4 =
// cos 4t, sin 4t): s^2 = (1 - C2)/2, 2cs = S2, 4c^2s^2 = (1 - C4)/2, 4cs^3 = S2 - S4/2 and
// s^4 = 3/8 - C2/2 + C4/8, which differentiate term by term.
__device__ __forceinline__ void delta_slope(double t, double a, double b, double cc, double beta, double q0,
                                            double q1, double q2, double q3, double q4, double* g, double* gg) {
    double S2, C2;
    sincos(2.0 * t, &S2, &C2);
    const double C4 = C2 * C2 - S2 * S2, S4 = 2.0 * S2 * C2;
    const double dq = cc - a;
    *g = dq * S2 + 2.0 * b * C2 +
         0.5 * beta * (4.0 * C2 * q0 + 2.0 * S2 * q1 + 2.0 * S4 * q2 + 2.0 * (C2 - C4) * q3 + (S2 - 0.5 * S4) * q4);
    *gg = 2.0 * dq * C2 - 4.0 * b * S2 +
          0.5 * beta * (-8.0 * S2 * q0 + 4.0 * C2 * q1 + 8.0 * C4 * q2 + (8.0 * S4 - 4.0 * S2) * q3 +
                        2.0 * (C2 - C4) * q4);
}

// Full line search of Section 5.1: the global minimiser of the energy along the great circle.
// E(t) has period pi (u -> -u keeps E), so [0, pi) is scanned at kFullSamples angles (the first
// lowest sample wins); the slope's zero bracketed between the best angle and the neighbour
// towards which E falls is then found by Newton steps kept inside the shrinking bracket
// (bisection when a step leaves it), to the last few ulps.  The result is reduced into [0, pi).
// The scan runs one angle per lane of the first wave when the workgroup has one (full_scan_wave,
// `kb` >= 0), else serially here.
constexpr int kFullSamples = 64;
constexpr double kFullStep = 3.141592653589793 / kFullSamples;
__device__ double theta_full(int kb, double a, double b, double cc, double beta, double q0, double q1, double q2,
                             double q3, double q4) {
    const double step = kFullStep;
    if (kb < 0) {
        kb = 0;
        double eb = 0.0;  // t = 0 changes nothing
        for (int k = 1; k < kFullSamples; ++k) {
            double s, c;
            sincos(k * step, &s, &c);
            const double e = delta_energy(c, s, a, b, cc, beta, q0, q1, q2, q3, q4);
            if (e < eb) {
                eb = e;
                kb = k;
            }
        }
    }
    double t = kb * step, g, gg;
    delta_slope(t, a, b, cc, beta, q0, q1, q2, q3, q4, &g, &gg);
    double lo = g < 0.0 ? t : t - step, hi = g < 0.0 ? t + step : t;
    double glo, ghi, unused;
    delta_slope(lo, a, b, cc, beta, q0, q1, q2, q3, q4, &glo, &unused);
    delta_slope(hi, a, b, cc, beta, q0, q1, q2, q3, q4, &ghi, &unused);
    if (g != 0.0 && glo < 0.0 && ghi > 0.0) {
        for (int it = 0; it < 80; ++it) {
            if (g == 0.0) break;
            if (g < 0.0)
                lo = t;
            else
                hi = t;
            double tn = t - g / gg;
            if (!(gg > 0.0) || !(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
            if (tn == t || !(hi - lo > 4.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)))) break;
            t = tn;
            delta_slope(t, a, b, cc, beta, q0, q1, q2, q3, q4, &g, &gg);
        }
    }
    t = fmod(t, 3.141592653589793);
    return t < 0.0 ? t + 3.141592653589793 : t;
}

// Sufficient-decrease constant of the Armijo test (the customary value).
constexpr double kArmijoC1 = 1e-4;
// Curvature constant of the strong Wolfe conditions (the usual nonlinear-CG value, below 1/2).
constexpr double kWolfeC2 = 0.1;

// A step satisfying the strong Wolfe conditions f(t) <= c1 t f'(0), |f'(t)| <= -c2 f'(0) for the
// energy change f along the great circle: bracketing from the heuristic's trial (doubled while it
// is too short, up to pi/2, where a step that still descends is taken), then a zoom that bisects
// the bracket; at most max_steps evaluations in each phase.  Returns the step, or -1 when none was
// found; *nev receives the number of evaluations.
__device__ double theta_wolfe(double th, double d1, int max_steps, int* nev, double a, double b, double cc,
                              double beta, double q0, double q1, double q2, double q3, double q4) {
    const double half_pi = 1.5707963267948966;
    auto f = [&](double t) {
        double s, c;
        sincos(t, &s, &c);
        return delta_energy(c, s, a, b, cc, beta, q0, q1, q2, q3, q4);
    };
    auto g = [&](double t) {
        double gv, unused;
        delta_slope(t, a, b, cc, beta, q0, q1, q2, q3, q4, &gv, &unused);
        return gv;
    };
    const double curv = -kWolfeC2 * d1;
    int n = 0;
    double result = -1.0, lo = 0.0, f_lo = 0.0, hi = 0.0;
    bool zoom = false;
    double t_prev = 0.0, f_prev = 0.0, t = fmin(th, half_pi);
    for (int i = 0; i < max_steps; ++i) {
        ++n;
        const double ft = f(t);
        if (!(ft <= kArmijoC1 * t * d1) || (i > 0 && ft >= f_prev)) {
            lo = t_prev;
            f_lo = f_prev;
            hi = t;
            zoom = true;
            break;
        }
        const double gt = g(t);
        if (fabs(gt) <= curv) {
            result = t;
            break;
        }
        if (gt >= 0.0) {
            lo = t;
            f_lo = ft;
            hi = t_prev;
            zoom = true;
            break;
        }
        if (t >= half_pi) {
            result = t;
            break;
        }
        t_prev = t;
        f_prev = ft;
        t = fmin(2.0 * t, half_pi);
    }
    if (zoom) {
        for (int k = 0; k < max_steps; ++k) {
            const double tm = 0.5 * (lo + hi);
            ++n;
            const double fm = f(tm);
            if (!(fm <= kArmijoC1 * tm * d1) || fm >= f_lo) {
                hi = tm;
            } else {
                const double gm = g(tm);
                if (fabs(gm) <= curv) {
                    result = tm;
                    break;
                }
                if (gm * (hi - lo) >= 0.0) hi = lo;
                lo = tm;
                f_lo = fm;
            }
        }
    }
    *nev = n;
    return result;
}

// Step selection (Section 5.1 heuristic; readings: theta_opt = -E'(0)/E''(0) when E''(0) > 0,
// else theta_default; clamp to (0, pi/2]; halve until E decreases, at most max_halvings times).
// line_search 1 asks each trial for the Armijo decrease as well; 2 takes the full line search; 3
// the strong Wolfe search (its evaluations are counted as halvings).
__device__ __forceinline__ void fin_step(Scal& S, const double* t, int kb) {
    if (!S.done) {
        const double w = S.cell;
        const double cR = w * t[B_CR], aR = w * t[B_AR], bR = w * t[B_BR];
        const double cc = w * t[B_C], b = w * t[B_B];
        const double SAA = w * t[B_AA], SAB = w * t[B_AB], SACA = w * t[B_ACA], SCACA = w * t[B_CACA];
        const double SCAB = w * t[B_CAB], SBB = w * t[B_BB], SAC = w * t[B_AC], SB = w * t[B_SB], SC = w * t[B_SC];
        const double nonfinite = t[B_NF];
        const double beta = S.beta;
        // E'(0) = 2 Re<H phi, phat>, E''(0) = 2 (<phat, H phat> + 2 beta sum (Re conj(phi) phat)^2 - lambda)
        const double d1 = 2.0 * (b + beta * SAB);
        const double d2 = 2.0 * (cc + beta * SAC + 2.0 * beta * SBB - S.lam);
        double th = d2 > 0.0 ? -d1 / d2 : S.theta_default;
        th = fmin(fmax(th, 0.0), 1.5707963267948966);
        double acc_t = -1.0, dE = 0.0, c = 1.0, s = 0.0;
        int j = 0;
        if (S.line_search == 2 || S.line_search == 3) {
            const double tf = S.line_search == 2
                                  ? theta_full(kb, S.a, b, cc, beta, SAB, SACA, SBB, SCAB, SCACA)
                                  : theta_wolfe(th, d1, S.max_halvings, &j, S.a, b, cc, beta, SAB, SACA, SBB, SCAB,
                                                SCACA);
            double sf, cf;
            sincos(tf, &sf, &cf);
            const double e = delta_energy(cf, sf, S.a, b, cc, beta, SAB, SACA, SBB, SCAB, SCACA);
            if (tf >= 0.0 && (S.line_search == 3 || e < 0.0)) {
                acc_t = tf;
                dE = e;
                c = cf;
                s = sf;
            }
        } else {
            for (; j <= S.max_halvings; ++j) {
                const double tj = th * ldexp(1.0, -j);
                if (!(tj > 0.0)) break;
                double sj, cj;
                sincos(tj, &sj, &cj);
                const double e = delta_energy(cj, sj, S.a, b, cc, beta, SAB, SACA, SBB, SCAB, SCACA);
                if (e < 0.0 && (S.line_search != 1 || e <= kArmijoC1 * tj * d1)) {
                    acc_t = tj;
                    dE = e;
                    c = cj;
                    s = sj;
                    break;
                }
            }
        }
        S.d2 = d2;
        if (nonfinite > 0.0 || !isfinite(d1) || !isfinite(d2)) {
            S.status = ST_NONFINITE;
            S.nonfinite = 1;
            S.done = 1;
        } else if (acc_t < 0.0) {
            // No trial decreased the energy.  In FP64 this is an error.  In FP32 the first failure
            // is retried from a steepest-descent direction (no step, CG memory dropped); a second
            // one in a row ends the phase (switch to FP64).
            S.linesearch_fail += 1;
            if (S.precision == 1 && S.linesearch_fail < 2) {
                S.have_prev = 0;
                S.n += 1;
                S.iters_fp32 += 1;
            } else {
                if (S.precision == 1) {
                    S.stagnant = 1;
                    S.status = ST_OK;
                } else {
                    S.status = ST_LINESEARCH;
                }
                S.done = 1;
            }
        } else {
            S.linesearch_fail = 0;
            const double n2 = c * c * S.nrm2 + 2.0 * c * s * SB + s * s * SC;
            const double nu = 1.0 / sqrt(n2);
            S.theta = acc_t;
            S.dE = dE;
            S.halvings += j;
            S.c_phi = nu * c;
            S.c_p = nu * s / S.pnorm;
            S.c_L = nu * c;
            S.c_Lp = nu * s;
            S.aR_next = nu * nu * (c * c * aR + 2.0 * c * s * bR + s * s * cR);
            hist_row(S, 4, acc_t);
            hist_row(S, 6, (double)j);
            // scalars of phi_{n+1} = nu (c phi + s phat), exact in (c, s):
            //   <phi', L phi'> = nu^2 (c^2 a + 2 c s b + s^2 <phat, L phat>)
            //   h^d sum|phi'|^4 = nu^4 (sum|phi|^4 + the quartic change of the line search)
            const double a1 = nu * nu * (c * c * S.a + 2.0 * c * s * b + s * s * cc);
            const double dq = 4.0 * c * s * SAB + 2.0 * s * s * SACA + 4.0 * c * c * s * s * SBB +
                              4.0 * c * s * s * s * SCAB + s * s * s * s * SCACA;
            const double q41 = nu * nu * nu * nu * (SAA + dq);
            S.E_prev = S.E;
            S.aR = S.aR_next;
            S.lam = a1 + beta * q41;
            S.lamt = a1 - S.aR + beta * q41;
            S.E = a1 + 0.5 * beta * q41;
            S.rPr_prev = S.rPr_cur;
            S.have_prev = 1;
            S.has_step = 1;
            S.n += 1;
            if (S.precision == 1) S.iters_fp32 += 1;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Scalar-state helpers for the passes
// ---------------------------------------------------------------------------------------------
// The state of instance b travels as 16-byte chunks, one per thread, so that a block fetches it
// in one round trip.
constexpr int kScalChunks = (int)(sizeof(Scal) / sizeof(uint4));
static_assert(sizeof(Scal) % sizeof(uint4) == 0, "Scal is copied in 16-byte chunks");

// The state of instance b, fetched by the first threads (one chunk each) at the start of a pass
// and stored into LDS in begin().
struct StateChunk {
    uint4 ch;
    __device__ __forceinline__ void issue(const Scal* in, int b) {
        if (threadIdx.x < kScalChunks) ch = reinterpret_cast<const uint4*>(in + b)[threadIdx.x];
    }
    __device__ __forceinline__ void store(const Scal* in, int b, Scal* s) const {
        uint4* dst = reinterpret_cast<uint4*>(s);
        if (threadIdx.x < kScalChunks) dst[threadIdx.x] = ch;
        for (int c = threadIdx.x + blockDim.x; c < kScalChunks; c += blockDim.x)  // blocks < 28 threads
            dst[c] = reinterpret_cast<const uint4*>(in + b)[c];
    }
};

// The partial rows (K <= 16 sums) of instance b in a region, fetched at the start of a pass in an
// (entry, row group) layout: thread t reads entry k = t % 16 of rows t / 16 + j G (G = blockDim / 16,
// j < NV) into registers.  reduce() folds them (and any rows beyond NV G), combines the four row
// groups of each wave by two exchanges and the waves through LDS, in a fixed order.  Blocks that
// are not whole waves fetch nothing early and reduce row by row.  Rows may be stale (a region
// whose sums are not pending), never out of bounds.
template <int K, int NV>
struct RowFetch {
    static_assert(K >= 1 && K <= 16, "up to 16 sums per row");
    double v[NV];
    __device__ __forceinline__ static bool fast() { return (blockDim.x & 63u) == 0; }
    __device__ __forceinline__ void issue(const Partials& P, int b, unsigned mask) {
        if (!fast() || !P.parts || P.nb <= 0) return;
        const int k = threadIdx.x & 15, grp = threadIdx.x >> 4, G = blockDim.x >> 4;
        const double id = ((mask >> k) & 1u) ? -1e300 : 0.0;
        const double* rows = P.parts + (size_t)b * P.row_stride() * K;
        const int kc = k < K ? k : K - 1;
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int r = grp + j * G;
            const double x = rows[(size_t)min(r, P.nb - 1) * K + kc];  // clamped: always in bounds
            v[j] = (k < K && r < P.nb) ? x : id;
        }
    }
    __device__ __forceinline__ void reduce(const Partials& P, int b, unsigned mask, double* red, double* tot) const {
        if (!P.parts || P.nb <= 0) {
            for (int k = threadIdx.x; k < K; k += blockDim.x) tot[k] = ((mask >> k) & 1u) ? -1e300 : 0.0;
            __syncthreads();
            return;
        }
        const double* rows = P.parts + (size_t)b * P.row_stride() * K;
        if (!fast()) {
            reduce_partials<K>(rows, P.nb, red, tot, mask);
            return;
        }
        const int k = threadIdx.x & 15, grp = threadIdx.x >> 4, G = blockDim.x >> 4;
        const bool mx = (mask >> k) & 1u;
        double a = v[0];
#pragma unroll
        for (int j = 1; j < NV; ++j) a = mx ? fmax(a, v[j]) : a + v[j];
        if (k < K)
            for (int r = grp + NV * G; r < P.nb; r += G) a = mx ? fmax(a, rows[(size_t)r * K + k]) : a + rows[(size_t)r * K + k];
        double o = __shfl_xor(a, 16, 64);
        a = mx ? fmax(a, o) : a + o;
        o = __shfl_xor(a, 32, 64);
        a = mx ? fmax(a, o) : a + o;
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
        if (lane < 16) red[wave * 16 + lane] = a;
        __syncthreads();
        if (threadIdx.x < K) {
            double t = red[threadIdx.x];
            for (int w = 1; w < nw; ++w) t = mx ? fmax(t, red[w * 16 + threadIdx.x]) : t + red[w * 16 + threadIdx.x];
            tot[threadIdx.x] = t;
        }
        __syncthreads();
    }
};

// What a pass that only reads the state fetches early.
struct IntakeState {
    StateChunk st;
};
// What a pass that absorbs a region of K-sum rows fetches early (NV rows per thread in registers).
template <int K, int NV>
struct IntakeAbsorb {
    StateChunk st;
    RowFetch<K, NV> rows;
};

// Copy the fetched state into LDS and barrier.
__device__ __forceinline__ void state_copy(const Scal* in, int b, Scal* s, const StateChunk& ch) {
    ch.store(in, b, s);
    __syncthreads();
}

// Thread 0 runs the scalar logic `fn(S, totals)` on the LDS state, with the totals copied into
// registers first (so that stores to the state cannot force reloads of them), then barrier.  Only
// the publishing block (blk 0) keeps the history pointer.
template <int K, class F>
__device__ __forceinline__ void finish(Scal* s, const double* tot, int blk, F fn) {
    if (threadIdx.x == 0) {
        double t[K];
#pragma unroll
        for (int k = 0; k < K; ++k) t[k] = tot[k];
        if (blk != 0) s->hist = nullptr;
        fn(*s, t);
    }
    __syncthreads();
}

// Start of an absorbing pass: the fetched state into LDS, the fetched rows reduced into `tot`
// (LDS, K doubles; the reduction's barriers also publish the state), then `fn` on thread 0.
template <int K, int NV, class F>
__device__ __forceinline__ void absorb_finish(const Scal* in, int b, int blk, Scal* s, const IntakeAbsorb<K, NV>& it,
                                              const Partials& P, unsigned mask, double* red, double* tot, F fn) {
    it.st.store(in, b, s);
    it.rows.reduce(P, b, mask, red, tot);
    finish<K>(s, tot, blk, fn);
}

// Block 0 of the instance writes the LDS state to out[b] (after a barrier that made it final).
__device__ __forceinline__ void state_publish(Scal* out, int b, int blk, const Scal* s) {
    if (blk != 0) return;
    const uint4* src = reinterpret_cast<const uint4*>(s);
    uint4* dst = reinterpret_cast<uint4*>(out + b);
    for (int c = threadIdx.x; c < kScalChunks; c += blockDim.x) dst[c] = src[c];
}

// The scan of the full line search on the first wave: lane k evaluates the energy change at
// k pi / 64 from the same coefficients as fin_step, and an xor butterfly over (change, k) keeps
// the lowest change, the lowest k among equal ones (what the serial scan keeps).
__device__ __forceinline__ int full_scan_wave(const Scal& S, const double* t) {
    static_assert(kFullSamples == 64, "one angle per lane");
    const int k = threadIdx.x & 63;
    const double w = S.cell;
    const double cc = w * t[B_C], b = w * t[B_B];
    const double SAB = w * t[B_AB], SACA = w * t[B_ACA], SBB = w * t[B_BB], SCAB = w * t[B_CAB],
                 SCACA = w * t[B_CACA];
    double s, c;
    sincos(k * kFullStep, &s, &c);
    double e = k == 0 ? 0.0 : delta_energy(c, s, S.a, b, cc, S.beta, SAB, SACA, SBB, SCAB, SCACA);
    int kk = k;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double eo = __shfl_xor(e, off, 64);
        const int ko = __shfl_xor(kk, off, 64);
        if (eo < e || (eo == e && ko < kk)) {
            e = eo;
            kk = ko;
        }
    }
    return kk;
}

// The step at the start of phase A, from the direction sums of every pass of phase B (one region,
// B sums), when they are pending: the line search and the predicted scalars of the new iterate.
constexpr int kStepRowsPerThread = 16;   // 256 rows with 256-thread blocks
using IntakeStep = IntakeAbsorb<B_K, kStepRowsPerThread>;
__device__ __forceinline__ void intake_step(const Scal* in, const Partials& pb, int b, IntakeStep& it) {
    it.st.issue(in, b);
    it.rows.issue(pb, b, B_MAXMASK);
}
__device__ __forceinline__ void begin_step(const Scal* in, Scal* out, const Partials& pb, int b, int blk, double* red,
                                           Scal* s, const IntakeStep& it) {
    __shared__ double tot[B_K];
    it.st.store(in, b, s);
    it.rows.reduce(pb, b, B_MAXMASK, red, tot);  // ends with a barrier: s and tot are visible
    int kb = -1;
    if (s->line_search == 2 && !s->done && s->b_phase && blockDim.x >= 64 && threadIdx.x < 64)
        kb = full_scan_wave(*s, tot);  // the whole first wave takes this branch (s is uniform)
    finish<B_K>(s, tot, blk, [kb](Scal& S, const double* t) {
        if (!S.done && S.b_phase) {
            fin_step(S, t, kb);
            S.b_phase = 0;
        }
    });
    state_publish(out, b, blk, s);
}

// Passes that absorb the phase-A sums (A_K per row, one region of at most 128 rows per thread
// group's registers).
constexpr int kARowsPerThread = 8;
using IntakeA = IntakeAbsorb<A_K, kARowsPerThread>;

// ---------------------------------------------------------------------------------------------
// Phase A, first pass (x): [step from the direction sums], the pending retraction applied to
// phi and L phi, residual, ||r||_inf, fresh scalars, P_V^{1/2} (or P_V) prologue, forward x.
// With ONE (1-D) the pass also applies the multiplier, the inverse and the epilogue, i.e. the
// whole preconditioner and the CG reductions.
// ---------------------------------------------------------------------------------------------
template <typename T, bool ONE>
struct OpResid {
    // FP32 2-D/3-D: capped at four workgroups per CU despite a small spill (measured faster than the
    // second round of workgroups the unconstrained allocation leaves on the batched 512^2 step);
    // the run-time-size transform would spill 208 bytes under the cap and runs unconstrained
    // (measured 15% faster on 640^2)
    static constexpr bool FWD = true, INV = ONE, SCALARS = true, PREFETCH = true, WIDE = sizeof(T) == 8 || ONE;
    static constexpr bool WIDE_RT = true;
    static constexpr int K = A_K;
    static constexpr unsigned MAXMASK = A_MAXMASK;
    IterFields<T> f;
    const Scal* Sin;  // S_dir
    Scal* Sout;       // S_step
    Partials pb;      // the direction passes' rows (consumer view)
    int pre, post;
    using Intake = IntakeStep;
    __device__ void intake(int b, int, Intake& it) const { intake_step(Sin, pb, b, it); }
    struct State {
        C2<T> ph[8], lph[8], pp[8], lp[8];
        T V[8];
        C2<T> r[ONE ? 8 : 1];
        double d[ONE ? 8 : 1];
    };
    __device__ void prefetch(const Geo&, const LineCtx& lc, State& st) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = lc.at(q);
            st.ph[q] = f.phi[i];
            st.lph[q] = f.Lphi[i];
            st.pp[q] = f.pp[i];
            st.lp[q] = f.lp[i];
            st.V[q] = f.V[i];
        }
    }
    __device__ void prefetch_tail(const Geo&, const LineCtx&, State&) const {}
    __device__ void begin(const Geo&, int b, int blk, double* red, Scal* s, Intake& it) const {
        begin_step(Sin, Sout, pb, b, blk, red, s, it);
    }
    __device__ void load(const Geo&, const LineCtx& lc, State& st, C2<T> (&v)[8], double (&acc)[K]) const {
        const Scal& s = *lc.sc;
        const T lam = (T)s.lam, beta = (T)s.beta;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = lc.at(q);
            C2<T> ph = st.ph[q];
            C2<T> lp = st.lph[q];
            apply_step_pref<T>(f, s, i, ph, lp, st.pp[q], st.lp[q], acc);
            const T V = st.V[q];
            const T rho = abs2(ph);
            const C2<T> r = add(lp, scl(ph, beta * rho - lam));
            f.r[i] = r;
            res_sums<T>(acc, r);
            const double d = pv_diag(s, (double)V, (double)rho);
            v[q] = scl(r, pscale<T>(pre, d));
            if constexpr (ONE) {
                st.ph[q] = ph;
                st.r[q] = r;
                st.d[q] = d;
            }
        }
    }
    template <int LG>
    __device__ void spectral(const Geo&, const LineCtx& lc, State&, C2<T> (&v)[8], double (&)[K], C2<T>*,
                             const C2<T>*) const {
        if constexpr (ONE) {
            const Scal& s = *lc.sc;
            const double invN = 1.0 / lc.M;  // 1/M (exact for M = 2^k)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double k = freq_of(lc.k(q), lc.M, s.dk[0]);
                v[q] = scl(v[q], (T)(invN / (s.lamt + 0.5 * k * k)));
            }
        }
    }
    __device__ void store(const Geo&, const LineCtx& lc, State& st, C2<T> (&v)[8], double (&acc)[K]) const {
        if constexpr (!ONE) {
#pragma unroll
            for (int q = 0; q < 8; ++q) f.w[lc.at(q)] = v[q];
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int64_t i = lc.at(q);
                const C2<T> pr = scl(v[q], pscale<T>(post, st.d[q]));
                f.pr[i] = pr;
                cg_sums<T>(acc, st.r[q], pr, f.rp[i], f.pp[i], st.ph[q]);
            }
        }
    }
};

// ---------------------------------------------------------------------------------------------
// Phase A, middle passes (y, z): forward and/or inverse transform with the kinetic multiplier
// 1/(lambda~ + |k|^2/2) (with the 1/N of the inverse transforms) on the pass that does both.
// The first middle pass (ABS) runs the convergence test on the first pass's sums, in the block
// that publishes the instance's state (blk 0) only: the multiplier needs lambda~ alone, which the
// step already put in S_step, so the other blocks start their transforms without waiting for the
// reduction.  They also transform the lines of an instance that the test finds converged (their
// output is never read).
// ---------------------------------------------------------------------------------------------
template <typename T, int AX, bool F, bool I, bool ABS>
struct OpPMid {
    static constexpr bool FWD = F, INV = I, SCALARS = true, PREFETCH = true, WIDE = false;
    static constexpr bool PREFETCH_EARLY = true;  // w only: eight points per thread
    static constexpr int K = 0;
    static constexpr unsigned MAXMASK = 0;
    C2<T>* w;
    const Scal* Sin;  // ABS: S_step; otherwise S_res
    Scal* Sout;       // ABS: S_res
    Partials pa1;
    using Intake = std::conditional_t<ABS, IntakeA, IntakeState>;
    __device__ void intake(int b, int blk, Intake& it) const {
        it.st.issue(Sin, b);
        if constexpr (ABS)
            if (blk == 0) it.rows.issue(pa1, b, A_MAXMASK);
    }
    struct State {
        C2<T> w[8];
    };
    __device__ void prefetch(const Geo&, const LineCtx& lc, State& st) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) st.w[q] = w[lc.at(q)];
    }
    __device__ void prefetch_tail(const Geo&, const LineCtx&, State&) const {}
    __device__ void begin(const Geo&, int b, int blk, double* red, Scal* s, Intake& it) const {
        if constexpr (ABS) {
            if (blk == 0) {
                __shared__ double tot[A_K];
                absorb_finish(Sin, b, blk, s, it, pa1, A_MAXMASK, red, tot, [](Scal& S, const double* t) {
                    if (!S.done) fin_residual(S, t);
                });
                state_publish(Sout, b, blk, s);
                return;
            }
        }
        state_copy(Sin, b, s, it.st);
    }
    __device__ void load(const Geo&, const LineCtx&, State& st, C2<T> (&v)[8], double (&)[1]) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = st.w[q];
    }
    template <int LG>
    __device__ void spectral(const Geo& g, const LineCtx& lc, State&, C2<T> (&v)[8], double (&)[1], C2<T>*,
                             const C2<T>*) const {
        if constexpr (F && I) {
            const Scal& s = *lc.sc;
            double ko;
            if (AX == 1) {
                const double xi = freq_of(lc.i1, g.n[0], s.dk[0]);
                ko = xi * xi;
            } else {
                const double xi = freq_of(lc.i1, g.n[0], s.dk[0]);
                const double mu = freq_of(lc.i2, g.n[1], s.dk[1]);
                ko = xi * xi + mu * mu;
            }
            const double invN = 1.0 / (double)g.N;  // 1/N (exact for powers of two)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double k = freq_of(lc.k(q), lc.M, s.dk[AX]);
                v[q] = scl(v[q], (T)(invN / (s.lamt + 0.5 * (ko + k * k))));
            }
        }
    }
    __device__ void store(const Geo&, const LineCtx& lc, State&, C2<T> (&v)[8], double (&)[1]) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) w[lc.at(q)] = v[q];
    }
};

// ---------------------------------------------------------------------------------------------
// Phase A, last pass (x): inverse x, epilogue scaling -> P r, and the CG reductions.
// ---------------------------------------------------------------------------------------------
template <typename T>
struct OpPLast {
    static constexpr bool FWD = false, INV = true, SCALARS = true, PREFETCH = true, WIDE = sizeof(T) == 8;
    static constexpr int K = A_K;
    static constexpr unsigned MAXMASK = A_MAXMASK;
    IterFields<T> f;
    const Scal* Sin;  // S_res
    int post;
    // w for the transform; the tail: what the epilogue and the CG sums read
    struct State {
        C2<T> w[8], ph[8], r[8], rp[8], pp[8];
        T V[8];
    };
    __device__ void prefetch(const Geo&, const LineCtx& lc, State& st) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) st.w[q] = f.w[lc.at(q)];
    }
    __device__ void prefetch_tail(const Geo&, const LineCtx& lc, State& st) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = lc.at(q);
            st.ph[q] = f.phi[i];
            st.V[q] = f.V[i];
            st.r[q] = f.r[i];
            st.rp[q] = f.rp[i];
            st.pp[q] = f.pp[i];
        }
    }
    using Intake = IntakeState;
    __device__ void intake(int b, int, Intake& it) const { it.st.issue(Sin, b); }
    __device__ void begin(const Geo&, int b, int, double*, Scal* s, Intake& it) const { state_copy(Sin, b, s, it.st); }
    __device__ void load(const Geo&, const LineCtx&, State& st, C2<T> (&v)[8], double (&)[K]) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = st.w[q];
    }
    template <int LG>
    __device__ void spectral(const Geo&, const LineCtx&, State&, C2<T> (&)[8], double (&)[K], C2<T>*,
                             const C2<T>*) const {}
    __device__ void store(const Geo&, const LineCtx& lc, State& st, C2<T> (&v)[8], double (&acc)[K]) const {
        const Scal& s = *lc.sc;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = lc.at(q);
            const C2<T> ph = st.ph[q];
            C2<T> pr = v[q];
            if (post) pr = scl(pr, pscale<T>(post, pv_diag(s, (double)st.V[q], (double)abs2(ph))));
            f.pr[i] = pr;
            cg_sums<T>(acc, st.r[q], pr, st.rp[q], st.pp[q], ph);
        }
    }
};

// ---------------------------------------------------------------------------------------------
// Phase B: p = -P r + beta_cg p_{n-1} - rho phi (written over p_{n-1}), phat = p/||p||, and
// L phat = sum_a F_a^{-1}[sigma_a F_a phat] + V phat (V phat with the x part).  When omega != 0 the passes along x and y
// also transform phi (forward only) to accumulate <phi, R phi>, Re<phi, R phat>, <phat, R phat>
// (Parseval per line), which keeps lambda~ exact without a separate rotation field.  The first
// pass runs the CG direction logic (and, on the one-pass paths, the convergence test).
// ---------------------------------------------------------------------------------------------
template <typename T, int AX, bool FIRST, bool LAST>
struct OpLp {
    static constexpr bool FWD = true, INV = true, SCALARS = true, PREFETCH = true, WIDE = true;
    static constexpr bool PHI = FIRST || LAST || AX < 2;  // phi is read (x, y: for the rotation sums when omega != 0)
    static constexpr int K = B_K;
    static constexpr unsigned MAXMASK = B_MAXMASK;
    IterFields<T> f;
    const Scal* Sin;   // FIRST: S_res (or S_step on the one-pass paths); otherwise S_dir
    Scal* Sout;        // FIRST: S_dir
    Partials pres;     // FIRST: set (to pdir's region) when the convergence test runs here (one-pass paths)
    Partials pdir;     // FIRST: sums for the CG direction
    using Intake = std::conditional_t<FIRST, IntakeA, IntakeState>;
    __device__ void intake(int b, int, Intake& it) const {
        it.st.issue(Sin, b);
        if constexpr (FIRST) it.rows.issue(pdir, b, A_MAXMASK);
    }
    struct State {
        C2<T> ph[8];
        C2<T> p[8];
        C2<T> w[FIRST ? 1 : 8];
        T V[FIRST ? 8 : 1];
    };
    // phi (when read) and P r (FIRST, from which load() builds the new direction) or p; the tail:
    // what the epilogue adds, the previous passes' partial L phat (w), or V (the first pass, along
    // x, adds V phat: a contiguous read there rather than one more strided stream later)
    __device__ void prefetch(const Geo&, const LineCtx& lc, State& st) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = lc.at(q);
            if constexpr (PHI) st.ph[q] = f.phi[i];
            st.p[q] = FIRST ? f.pr[i] : f.pp[i];
        }
    }
    __device__ void prefetch_tail(const Geo&, const LineCtx& lc, State& st) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = lc.at(q);
            if constexpr (!FIRST) st.w[q] = f.w[i];
            if constexpr (FIRST) st.V[q] = f.V[i];
        }
    }
    __device__ void begin(const Geo&, int b, int blk, double* red, Scal* s, Intake& it) const {
        if constexpr (FIRST) {
            // on the one-pass paths the convergence test reads the same region as the direction
            __shared__ double tot[A_K];
            it.st.store(Sin, b, s);
            it.rows.reduce(pdir, b, A_MAXMASK, red, tot);
            auto direction = [](Scal& S, const double* t) {
                if (!S.done) {
                    fin_direction(S, t);
                    if (!S.done) S.b_phase = 1;
                }
            };
            if (pres.parts) {
                finish<A_K>(s, tot, blk, [direction](Scal& S, const double* t) {
                    if (!S.done) fin_residual(S, t);
                    direction(S, t);
                });
            } else {
                finish<A_K>(s, tot, blk, direction);
            }
            state_publish(Sout, b, blk, s);
        } else {
            state_copy(Sin, b, s, it.st);
        }
    }
    __device__ void load(const Geo&, const LineCtx& lc, State& st, C2<T> (&v)[8], double (&)[K]) const {
        const Scal& s = *lc.sc;
        const T inv = (T)(1.0 / s.pnorm);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = lc.at(q);
            C2<T> p;
            if constexpr (FIRST) {
                const C2<T> ph = st.ph[q];
                p = sub(scl(f.pp[i], (T)s.beta_cg), add(st.p[q], scl(ph, (T)s.rho)));
                f.pp[i] = p;
            } else {
                p = st.p[q];
            }
            st.p[q] = v[q] = scl(p, inv);
        }
    }
    template <int LG>
    __device__ void spectral(const Geo&, const LineCtx& lc, State& st, C2<T> (&v)[8], double (&acc)[K],
                             C2<T>* buf, const C2<T>* tw) const {
        const Scal& s = *lc.sc;
        const double rot = rot_coef_s<AX>(s, lc);
        const double invM = 1.0 / lc.M;  // 1/M (exact for M = 2^k)
        if (AX < 2 && s.omega != 0.0 && s.dim >= 2) {
            C2<T> u[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) u[q] = st.ph[q];
            line_fft<T, -1, AX, LG>(u, buf, tw, lc);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double xi = freq_of(lc.k(q), lc.M, s.dk[AX]);
                const double wr = rot * xi * invM;
                acc[B_CR] += wr * (double)abs2(v[q]);
                acc[B_AR] += wr * (double)abs2(u[q]);
                acc[B_BR] += wr * (double)redot(u[q], v[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double xi = freq_of(lc.k(q), lc.M, s.dk[AX]);
            v[q] = scl(v[q], (T)((0.5 * xi * xi + rot * xi) * invM));
        }
    }
    __device__ void store(const Geo&, const LineCtx& lc, State& st, C2<T> (&v)[8], double (&acc)[K]) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = lc.at(q);
            C2<T> o = v[q];
            if constexpr (!FIRST) o = add(o, st.w[q]);
            if constexpr (FIRST) o = add(o, scl(st.p[q], st.V[q]));
            if constexpr (!LAST) {
                f.w[i] = o;
            } else {
                const C2<T> ph = st.ph[q], p = st.p[q];
                f.lp[i] = o;
                // line-search sums (A = |phi|^2, B = Re conj(phi) phat, C = |phat|^2)
                const double A = abs2(ph), Bq = redot(ph, p), Cq = abs2(p);
                acc[B_C] += (double)redot(p, o);
                acc[B_B] += (double)redot(ph, o);
                acc[B_AA] += A * A;
                acc[B_AB] += A * Bq;
                acc[B_ACA] += A * (Cq - A);
                acc[B_CACA] += (Cq - A) * (Cq - A);
                acc[B_CAB] += (Cq - A) * Bq;
                acc[B_BB] += Bq * Bq;
                acc[B_AC] += A * Cq;
                acc[B_SB] += Bq;
                acc[B_SC] += Cq;
                if (!isfinite((double)o.x) || !isfinite((double)o.y)) acc[B_NF] = 1.0;
            }
        }
    }
};

// ---------------------------------------------------------------------------------------------
// Diagonal preconditioners (identity, P_V): [step], the pending retraction, residual, P r and all
// phase-A sums in one pointwise sweep (fixed chunks per block: deterministic partials).
// ---------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_resid_diag(IterFields<T> f, const Scal* Sin, Scal* Sout, int64_t N, int nbpi,
                                                   int pre, Partials pb, Partials pr, int b0, const int* imap) {
    __shared__ double red[(256 / 64 + 1) * 16 + 8];
    __shared__ Scal s;
    const int bi = blockIdx.x / nbpi;  // instance within the launch
    const int b = imap ? imap[bi] : b0 + bi;
    const int blk = blockIdx.x - bi * nbpi;
    IntakeStep it;
    intake_step(Sin, pb, b, it);
    begin_step(Sin, Sout, pb, b, blk, red, &s, it);
    if (s.done) return;
    double acc[A_K];
#pragma unroll
    for (int k = 0; k < A_K; ++k) acc[k] = 0.0;
    const T lam = (T)s.lam, beta = (T)s.beta;
    const int64_t chunk = (N + nbpi - 1) / nbpi;
    const int64_t lo = (int64_t)blk * chunk, hi = min(N, lo + chunk);
    const int64_t off = (int64_t)b * N;
    for (int64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) {
        const int64_t i = off + j;
        C2<T> ph = f.phi[i];
        C2<T> lph = f.Lphi[i];
        apply_step<T>(f, s, i, ph, lph, acc);
        const T rho = abs2(ph);
        const C2<T> r = add(lph, scl(ph, beta * rho - lam));
        f.r[i] = r;
        const C2<T> prv = scl(r, pscale<T>(pre, pv_diag(s, (double)f.V[i], (double)rho)));
        f.pr[i] = prv;
        res_sums<T>(acc, r);
        cg_sums<T>(acc, r, prv, f.rp[i], f.pp[i], ph);
    }
    __shared__ double totals[A_K];
    block_reduce<A_K>(acc, red, totals, A_MAXMASK);
    double* P = pr.parts + ((size_t)b * pr.row_stride() + pr.off + blk) * A_K;
    for (int k = threadIdx.x; k < A_K; k += blockDim.x) P[k] = totals[k];
}

// ---------------------------------------------------------------------------------------------
// Collapse the per-block partial rows of each instance into one row (one workgroup per instance,
// fixed order), so that the consuming pass's workgroups reduce a single row.
// ---------------------------------------------------------------------------------------------
template <int K>
__global__ __launch_bounds__(256) void k_collapse(const double* parts, int nb, int stride, double* out, unsigned mask,
                                                 int b0, const int* imap) {
    __shared__ double red[(256 / 64 + 1) * K];
    __shared__ double tot[K];
    const int b = imap ? imap[blockIdx.x] : b0 + (int)blockIdx.x;
    reduce_partials<K>(parts + (size_t)b * stride * K, nb, red, tot, mask);
    for (int k = threadIdx.x; k < K; k += blockDim.x) out[(size_t)b * K + k] = tot[k];
}

// ---------------------------------------------------------------------------------------------
// Host: enqueue one iteration for B instances.
// ---------------------------------------------------------------------------------------------
template <typename T>
hipError_t enqueue_iteration(const IterCtx<T>& c, hipStream_t s) {
    const Geo& g = c.g;
    const bool f64 = sizeof(T) == 8;
    const int cb = (int)sizeof(C2<T>);
    const IterFields<T>& f = c.f;
    Scal* S_step = c.S;
    Scal* S_res = c.S + c.B;
    Scal* S_dir = c.S + 2 * c.B;
    // launched instances: [g.b0, g.b0 + Bl), or g.imap[0 .. Bl) (converged instances are not launched)
    const int Bl = g.bl > 0 ? g.bl : c.B;
    hipError_t e;
    auto region = [&](int r, int ax) {
        const int nb = pass_blocks_per_field(g, ax, cb, c.B, true);
        return Partials{c.parts + (size_t)r * c.region_doubles, nb, nb, 0};
    };
    // the view a consumer absorbs: the region itself, or its one-row collapse for many rows
    auto consumable = [&](const Partials& p, int rc, int K, unsigned mask) -> Partials {
        if (p.nb <= kAbsorbRows) return p;
        const Partials q{c.parts + (size_t)rc * c.region_doubles, 1, 1, 0};
        if (K == A_K)
            hipLaunchKernelGGL(k_collapse<A_K>, dim3((unsigned)Bl), dim3(256), 0, s, p.parts, p.nb, p.row_stride(),
                               q.parts, mask, g.b0, g.imap);
        else
            hipLaunchKernelGGL(k_collapse<B_K>, dim3((unsigned)Bl), dim3(256), 0, s, p.parts, p.nb, p.row_stride(),
                               q.parts, mask, g.b0, g.imap);
        return q;
    };
    const Partials none{nullptr, 0, 0, 0};
    // algorithmic bytes of a launch: `reals` real numbers of sizeof(T) per grid point and instance
    const double unit = (double)sizeof(T) * (double)g.N * (double)c.B;
    auto tick = [&](const char* name, double reals) -> const LaunchEvents* {
        return c.timer ? c.timer->next(name, reals * unit) : nullptr;
    };
    // The direction passes (x, y, z) share one region of B-sum rows, each pass at its own offset
    // within an instance's rows; the step absorbs them at the next iteration's start, through their
    // one-row collapse when they are many.
    const int nbx = pass_blocks_per_field(g, 0, cb, c.B, true);
    const int nby = g.dim >= 2 ? pass_blocks_per_field(g, 1, cb, c.B, true) : 0;
    const int nbz = g.dim >= 3 ? pass_blocks_per_field(g, 2, cb, c.B, true) : 0;
    const int nbB = nbx + nby + nbz;
    double* const partsB = c.parts + (size_t)R_B * c.region_doubles;
    const Partials pb0{partsB, nbx, nbB, 0}, pb1{partsB, nby, nbB, nbx}, pb2{partsB, nbz, nbB, nbx + nby};
    const Partials pbAll{partsB, nbB, nbB, 0};
    const Partials sb = nbB <= kAbsorbRows ? pbAll : Partials{c.parts + (size_t)R_BC * c.region_doubles, 1, 1, 0};
    // ---- phase A ----
    int pre = 0, post = 0;
    const bool spectral_p = c.precond == GPE_P_KINETIC || c.precond == GPE_P_COMBINED || c.precond == GPE_P_C1 ||
                            c.precond == GPE_P_C2;
    if (c.precond == GPE_P_COMBINED) pre = post = 1;
    if (c.precond == GPE_P_C1) post = 2;
    if (c.precond == GPE_P_C2 || c.precond == GPE_P_POTENTIAL) pre = 2;
    Partials pres = none, pdir;
    const Scal* dir_in;
    if (!spectral_p) {
        // diagonal P (identity or P_V): one pointwise kernel for residual, P r and every sum
        const int nbpi = c.pointwise_blocks;
        const Partials pr{c.parts + (size_t)R_A1 * c.region_doubles, nbpi, nbpi, 0};
        launch_timed(tick("step_resid_diag", 21), k_resid_diag<T>, dim3((unsigned)(nbpi * Bl)), dim3(256), 0, s, f,
                     S_dir, S_step, g.N, nbpi, pre, sb, pr, g.b0, g.imap);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        pres = consumable(pr, R_A1C, A_K, A_MAXMASK);
        pdir = pres;
        dir_in = S_step;
    } else if (g.dim == 1) {
        OpResid<T, true> op{f, S_dir, S_step, sb, pre, post};
        const Partials pa = region(R_A1, 0);
        if ((e = launch_pass<T, 0>(g, c.B, c.tw->get(0, f64), op, pa, s,
                tick("step_resid_precond_x", 21))) != hipSuccess)
            return e;
        pres = consumable(pa, R_A1C, A_K, A_MAXMASK);
        pdir = pres;
        dir_in = S_step;
    } else {
        OpResid<T, false> op{f, S_dir, S_step, sb, pre, post};
        const Partials pa1r = region(R_A1, 0);
        if ((e = launch_pass<T, 0>(g, c.B, c.tw->get(0, f64), op, pa1r, s,
                tick("step_resid_fwd_x", 17))) != hipSuccess)
            return e;
        const Partials pa1 = consumable(pa1r, R_A1C, A_K, A_MAXMASK);
        if (g.dim == 2) {
            OpPMid<T, 1, true, true, true> y{f.w, S_step, S_res, pa1};
            if ((e = launch_pass<T, 1>(g, c.B, c.tw->get(1, f64), y, none, s,
                    tick("resid_test_precond_y", 4))) != hipSuccess)
                return e;
        } else {
            OpPMid<T, 1, true, false, true> y1{f.w, S_step, S_res, pa1};
            if ((e = launch_pass<T, 1>(g, c.B, c.tw->get(1, f64), y1, none, s,
                    tick("resid_test_precond_fwd_y", 4))) != hipSuccess)
                return e;
            OpPMid<T, 2, true, true, false> z{f.w, S_res, nullptr, none};
            if ((e = launch_pass<T, 2>(g, c.B, c.tw->get(2, f64), z, none, s,
                    tick("precond_z", 4))) != hipSuccess)
                return e;
            OpPMid<T, 1, false, true, false> y2{f.w, S_res, nullptr, none};
            if ((e = launch_pass<T, 1>(g, c.B, c.tw->get(1, f64), y2, none, s,
                    tick("precond_inv_y", 4))) != hipSuccess)
                return e;
        }
        OpPLast<T> op3{f, S_res, post};
        const Partials pa3 = region(R_A3, 0);
        if ((e = launch_pass<T, 0>(g, c.B, c.tw->get(0, f64), op3, pa3, s,
                tick("precond_inv_x", 13))) != hipSuccess)
            return e;
        pdir = consumable(pa3, R_A3C, A_K, A_MAXMASK);
        dir_in = S_res;
    }
    // ---- phase B ----
    if (g.dim == 1) {
        OpLp<T, 0, true, true> op{f, dir_in, S_dir, pres, pdir};
        if ((e = launch_pass<T, 0>(g, c.B, c.tw->get(0, f64), op, pb0, s,
                tick("dir_Lp_x_linesearch", 11))) != hipSuccess)
            return e;
    } else if (g.dim == 2) {
        OpLp<T, 0, true, false> ox{f, dir_in, S_dir, pres, pdir};
        if ((e = launch_pass<T, 0>(g, c.B, c.tw->get(0, f64), ox, pb0, s,
                tick("dir_Lp_x", 11))) != hipSuccess)
            return e;
        OpLp<T, 1, false, true> oy{f, S_dir, nullptr, none, none};
        if ((e = launch_pass<T, 1>(g, c.B, c.tw->get(1, f64), oy, pb1, s,
                tick("Lp_y_linesearch", 8))) != hipSuccess)
            return e;
    } else {
        OpLp<T, 0, true, false> ox{f, dir_in, S_dir, pres, pdir};
        if ((e = launch_pass<T, 0>(g, c.B, c.tw->get(0, f64), ox, pb0, s,
                tick("dir_Lp_x", 11))) != hipSuccess)
            return e;
        OpLp<T, 1, false, false> oy{f, S_dir, nullptr, none, none};
        if ((e = launch_pass<T, 1>(g, c.B, c.tw->get(1, f64), oy, pb1, s, tick("Lp_y", 8))) != hipSuccess) return e;
        OpLp<T, 2, false, true> oz{f, S_dir, nullptr, none, none};
        if ((e = launch_pass<T, 2>(g, c.B, c.tw->get(2, f64), oz, pb2, s,
                tick("Lp_z_linesearch", 8))) != hipSuccess)
            return e;
    }
    (void)consumable(pbAll, R_BC, B_K, B_MAXMASK);
    return hipGetLastError();
}

template hipError_t enqueue_iteration<double>(const IterCtx<double>&, hipStream_t);
template hipError_t enqueue_iteration<float>(const IterCtx<float>&, hipStream_t);

}  // namespace gpe
