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

template <typename T>
__device__ __forceinline__ T pscale(int kind, double d) {
    return kind == 1 ? (T)(1.0 / sqrt(d)) : kind == 2 ? (T)(1.0 / d) : (T)1;
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
__device__ void fin_residual(Scal& S, const double* t) {
    if (threadIdx.x == 0) {
        const double res = t[A_RES], nonfinite = t[A_NF];
        // fresh scalars of phi_n (the step of the previous iteration has just been applied)
        S.a = S.cell * t[A_A];
        S.q4 = S.cell * t[A_Q4];
        S.nrm2 = S.cell * t[A_N2];
        S.dphi = t[A_DPHI];
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
            // mixed precision: leave the FP32 phase when the residual stops improving
            if (res < S.best_res * (1.0 - 1e-3)) {
                S.best_res = res;
                S.best_n = S.n;
            } else if (S.n - S.best_n >= S.stall_window) {
                S.stagnant = 1;
                S.status = ST_OK;
                S.done = 1;
            }
        }
    }
    __syncthreads();
}

// CG direction from the A-phase sums (Section 5.2, readings: beta_0 = 0, PR+ with the stored
// denominator, restart when Re<r, p> >= 0).
__device__ void fin_direction(Scal& S, const double* t) {
    if (threadIdx.x == 0 && !S.done) {
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
    __syncthreads();
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

// Step selection (Section 5.1 heuristic; readings: theta_opt = -E'(0)/E''(0) when E''(0) > 0,
// else theta_default; clamp to (0, pi/2]; halve until E decreases, at most max_halvings times).
__device__ void fin_step(Scal& S, const double* t) {
    if (threadIdx.x == 0 && !S.done) {
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
        double acc_t = -1.0, dE = 0.0;
        int j = 0;
        for (; j <= S.max_halvings; ++j) {
            const double tj = th * ldexp(1.0, -j);
            if (!(tj > 0.0)) break;
            const double e = delta_energy(cos(tj), sin(tj), S.a, b, cc, beta, SAB, SACA, SBB, SCAB, SCACA);
            if (e < 0.0) {
                acc_t = tj;
                dE = e;
                break;
            }
        }
        S.d2 = d2;
        if (nonfinite > 0.0 || !isfinite(d1) || !isfinite(d2)) {
            S.status = ST_NONFINITE;
            S.nonfinite = 1;
            S.done = 1;
        } else if (acc_t < 0.0) {
            // no trial decreased the energy: in FP32 this ends the phase (switch to FP64)
            S.linesearch_fail = 1;
            if (S.precision == 1) {
                S.stagnant = 1;
                S.status = ST_OK;
            } else {
                S.status = ST_LINESEARCH;
            }
            S.done = 1;
        } else {
            const double c = cos(acc_t), s = sin(acc_t);
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
    __syncthreads();
}

// ---------------------------------------------------------------------------------------------
// Scalar-state helpers for the passes
// ---------------------------------------------------------------------------------------------
// Copy the instance's state into LDS; only the publishing block keeps the history pointer.
__device__ __forceinline__ void state_load(const Scal* in, int b, int blk, Scal* s) {
    if (threadIdx.x == 0) {
        *s = in[b];
        if (blk != 0) s->hist = nullptr;
    }
    __syncthreads();
}

__device__ __forceinline__ void state_publish(Scal* out, int b, int blk, const Scal* s) {
    __syncthreads();
    if (blk == 0 && threadIdx.x == 0) {
        Scal c = *s;
        c.hist = out[b].hist;  // keep the instance's history pointer
        out[b] = c;
    }
}

// Totals of K sums of instance b over the producing pass's blocks (LDS `out`, K doubles).
template <int K>
__device__ __forceinline__ void absorb(const Partials& P, int b, unsigned mask, double* red, double* out) {
    reduce_partials<K>(P.parts + (size_t)b * P.nb * K, P.nb, red, out, mask);
}

// The step: totals of the direction passes (x, y, z partial regions, B sums).
__device__ void absorb_step(const Partials& p0, const Partials& p1, const Partials& p2, int b, double* red,
                            Scal* s) {
    __shared__ double tot[B_K];
    __shared__ double part[B_K];
    for (int k = threadIdx.x; k < B_K; k += blockDim.x) tot[k] = 0.0;
    __syncthreads();
    auto merge = [&](const Partials& P) {
        if (!P.parts) return;
        absorb<B_K>(P, b, B_MAXMASK, red, part);
        for (int k = threadIdx.x; k < B_K; k += blockDim.x) {
            const bool mx = (B_MAXMASK >> k) & 1u;
            tot[k] = mx ? fmax(tot[k], part[k]) : tot[k] + part[k];
        }
        __syncthreads();
    };
    merge(p0);
    merge(p1);
    merge(p2);
    fin_step(*s, tot);
    if (threadIdx.x == 0) s->b_phase = 0;
    __syncthreads();
}

// ---------------------------------------------------------------------------------------------
// Phase A, first pass (x): [step from the direction sums], the pending retraction applied to
// phi and L phi, residual, ||r||_inf, fresh scalars, P_V^{1/2} (or P_V) prologue, forward x.
// With ONE (1-D) the pass also applies the multiplier, the inverse and the epilogue, i.e. the
// whole preconditioner and the CG reductions.
// ---------------------------------------------------------------------------------------------
template <typename T, bool ONE>
struct OpResid {
    static constexpr bool FWD = true, INV = ONE, SCALARS = true, PREFETCH = true;
    static constexpr int K = A_K;
    static constexpr unsigned MAXMASK = A_MAXMASK;
    IterFields<T> f;
    const Scal* Sin;  // S_dir
    Scal* Sout;       // S_step
    Partials pb0, pb1, pb2;
    int pre, post;
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
    __device__ void begin(const Geo&, int b, int blk, double* red, Scal* s) const {
        state_load(Sin, b, blk, s);
        if (!s->done && s->b_phase) absorb_step(pb0, pb1, pb2, b, red, s);
        state_publish(Sout, b, blk, s);
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
    __device__ void spectral(const Geo&, const LineCtx& lc, State&, C2<T> (&v)[8], double (&)[K], C2<T>*,
                             const C2<T>*) const {
        if constexpr (ONE) {
            const Scal& s = *lc.sc;
            const double invN = 1.0 / lc.M;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double k = freq_of(lc.k(q), lc.M, s.L[0]);
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
// The first middle pass (ABS) runs the convergence test on the first pass's sums.
// ---------------------------------------------------------------------------------------------
template <typename T, int AX, bool F, bool I, bool ABS>
struct OpPMid {
    static constexpr bool FWD = F, INV = I, SCALARS = true, PREFETCH = true;
    static constexpr int K = 0;
    static constexpr unsigned MAXMASK = 0;
    C2<T>* w;
    const Scal* Sin;  // ABS: S_step; otherwise S_res
    Scal* Sout;       // ABS: S_res
    Partials pa1;
    struct State {
        C2<T> w[8];
    };
    __device__ void prefetch(const Geo&, const LineCtx& lc, State& st) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) st.w[q] = w[lc.at(q)];
    }
    __device__ void begin(const Geo&, int b, int blk, double* red, Scal* s) const {
        state_load(Sin, b, blk, s);
        if constexpr (ABS) {
            if (!s->done) {
                __shared__ double tot[A_K];
                absorb<A_K>(pa1, b, A_MAXMASK, red, tot);
                fin_residual(*s, tot);
            }
            state_publish(Sout, b, blk, s);
        }
    }
    __device__ void load(const Geo&, const LineCtx&, State& st, C2<T> (&v)[8], double (&)[1]) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = st.w[q];
    }
    __device__ void spectral(const Geo& g, const LineCtx& lc, State&, C2<T> (&v)[8], double (&)[1], C2<T>*,
                             const C2<T>*) const {
        if constexpr (F && I) {
            const Scal& s = *lc.sc;
            double ko;
            if (AX == 1) {
                const double xi = freq_of(lc.i1, g.n[0], s.L[0]);
                ko = xi * xi;
            } else {
                const double xi = freq_of(lc.i1, g.n[0], s.L[0]);
                const double mu = freq_of(lc.i2, g.n[1], s.L[1]);
                ko = xi * xi + mu * mu;
            }
            const double invN = 1.0 / (double)g.N;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double k = freq_of(lc.k(q), lc.M, s.L[AX]);
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
    static constexpr bool FWD = false, INV = true, SCALARS = true, PREFETCH = false;
    static constexpr int K = A_K;
    static constexpr unsigned MAXMASK = A_MAXMASK;
    IterFields<T> f;
    const Scal* Sin;  // S_res
    int post;
    struct State {};
    __device__ void begin(const Geo&, int b, int blk, double*, Scal* s) const { state_load(Sin, b, blk, s); }
    __device__ void load(const Geo&, const LineCtx& lc, State&, C2<T> (&v)[8], double (&)[K]) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = f.w[lc.at(q)];
    }
    __device__ void spectral(const Geo&, const LineCtx&, State&, C2<T> (&)[8], double (&)[K], C2<T>*,
                             const C2<T>*) const {}
    __device__ void store(const Geo&, const LineCtx& lc, State&, C2<T> (&v)[8], double (&acc)[K]) const {
        const Scal& s = *lc.sc;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = lc.at(q);
            const C2<T> ph = f.phi[i];
            C2<T> pr = v[q];
            if (post) pr = scl(pr, pscale<T>(post, pv_diag(s, (double)f.V[i], (double)abs2(ph))));
            f.pr[i] = pr;
            cg_sums<T>(acc, f.r[i], pr, f.rp[i], f.pp[i], ph);
        }
    }
};

// ---------------------------------------------------------------------------------------------
// Phase B: p = -P r + beta_cg p_{n-1} - rho phi (written over p_{n-1}), phat = p/||p||, and
// L phat = sum_a F_a^{-1}[sigma_a F_a phat] + V phat.  When omega != 0 the passes along x and y
// also transform phi (forward only) to accumulate <phi, R phi>, Re<phi, R phat>, <phat, R phat>
// (Parseval per line), which keeps lambda~ exact without a separate rotation field.  The first
// pass runs the CG direction logic (and, on the one-pass paths, the convergence test).
// ---------------------------------------------------------------------------------------------
template <typename T, int AX, bool FIRST, bool LAST>
struct OpLp {
    static constexpr bool FWD = true, INV = true, SCALARS = true, PREFETCH = FIRST;
    static constexpr int K = B_K;
    static constexpr unsigned MAXMASK = B_MAXMASK;
    IterFields<T> f;
    const Scal* Sin;   // FIRST: S_res (or S_step on the one-pass paths); otherwise S_dir
    Scal* Sout;        // FIRST: S_dir
    Partials pres;     // FIRST: sums for the convergence test (one-pass paths), else empty
    Partials pdir;     // FIRST: sums for the CG direction
    struct State {
        C2<T> ph[8];
        C2<T> p[8];
    };
    // FIRST: phi and the preconditioned residual P r (into p, where load() builds the new direction)
    __device__ void prefetch(const Geo&, const LineCtx& lc, State& st) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = lc.at(q);
            st.ph[q] = f.phi[i];
            st.p[q] = f.pr[i];
        }
    }
    __device__ void begin(const Geo&, int b, int blk, double* red, Scal* s) const {
        state_load(Sin, b, blk, s);
        if constexpr (FIRST) {
            __shared__ double tot[A_K];
            if (!s->done && pres.parts) {
                absorb<A_K>(pres, b, A_MAXMASK, red, tot);
                fin_residual(*s, tot);
            }
            if (!s->done) {
                absorb<A_K>(pdir, b, A_MAXMASK, red, tot);
                fin_direction(*s, tot);
                if (threadIdx.x == 0 && !s->done) s->b_phase = 1;
            }
            state_publish(Sout, b, blk, s);
        }
    }
    __device__ void load(const Geo&, const LineCtx& lc, State& st, C2<T> (&v)[8], double (&)[K]) const {
        const Scal& s = *lc.sc;
        const T inv = (T)(1.0 / s.pnorm);
        const bool need_phi = LAST || (s.omega != 0.0 && AX < 2);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = lc.at(q);
            C2<T> p;
            if constexpr (FIRST) {
                const C2<T> ph = st.ph[q];
                p = sub(scl(f.pp[i], (T)s.beta_cg), add(st.p[q], scl(ph, (T)s.rho)));
                f.pp[i] = p;
            } else {
                p = f.pp[i];
                if (need_phi) st.ph[q] = f.phi[i];
            }
            st.p[q] = v[q] = scl(p, inv);
        }
    }
    __device__ void spectral(const Geo&, const LineCtx& lc, State& st, C2<T> (&v)[8], double (&acc)[K],
                             C2<T>* buf, const C2<T>* tw) const {
        const Scal& s = *lc.sc;
        const double rot = rot_coef_s<AX>(s, lc);
        const double invM = 1.0 / lc.M;
        if (AX < 2 && s.omega != 0.0 && s.dim >= 2) {
            C2<T> u[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) u[q] = st.ph[q];
            fft_line<T, -1>(u, buf, tw, lc.t, lc.lg);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double xi = freq_of(lc.k(q), lc.M, s.L[AX]);
                const double wr = rot * xi * invM;
                acc[B_CR] += wr * (double)abs2(v[q]);
                acc[B_AR] += wr * (double)abs2(u[q]);
                acc[B_BR] += wr * (double)redot(u[q], v[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double xi = freq_of(lc.k(q), lc.M, s.L[AX]);
            v[q] = scl(v[q], (T)((0.5 * xi * xi + rot * xi) * invM));
        }
    }
    __device__ void store(const Geo&, const LineCtx& lc, State& st, C2<T> (&v)[8], double (&acc)[K]) const {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = lc.at(q);
            C2<T> o = v[q];
            if constexpr (!FIRST) o = add(o, f.w[i]);
            if constexpr (!LAST) {
                f.w[i] = o;
            } else {
                const C2<T> ph = st.ph[q], p = st.p[q];
                o = add(o, scl(p, f.V[i]));
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
                                                   int pre, Partials pb0, Partials pb1, Partials pb2, Partials pr) {
    __shared__ double red[(256 / 64 + 1) * 16 + 8];
    __shared__ Scal s;
    const int b = blockIdx.x / nbpi;
    const int blk = blockIdx.x - b * nbpi;
    state_load(Sin, b, blk, &s);
    if (!s.done && s.b_phase) absorb_step(pb0, pb1, pb2, b, red, &s);
    state_publish(Sout, b, blk, &s);
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
    double* P = pr.parts + ((size_t)b * nbpi + blk) * A_K;
    for (int k = threadIdx.x; k < A_K; k += blockDim.x) P[k] = totals[k];
}

// ---------------------------------------------------------------------------------------------
// Collapse the per-block partial rows of each instance into one row (one workgroup per instance,
// fixed order), so that the consuming pass's workgroups reduce a single row.
// ---------------------------------------------------------------------------------------------
template <int K>
__global__ __launch_bounds__(256) void k_collapse(const double* parts, int nb, double* out, unsigned mask) {
    __shared__ double red[(256 / 64) * K];
    __shared__ double tot[K];
    const int b = blockIdx.x;
    reduce_partials<K>(parts + (size_t)b * nb * K, nb, red, tot, mask);
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
    hipError_t e;
    auto region = [&](int r, int ax) {
        Partials p;
        p.parts = c.parts + (size_t)r * c.region_doubles;
        p.counters = nullptr;
        p.nb = pass_blocks_per_field(g, ax, cb, c.B);
        return p;
    };
    // the view a consumer absorbs: the region itself, or its one-row collapse for many rows
    auto consumable = [&](const Partials& p, int rc, int K, unsigned mask) -> Partials {
        if (p.nb <= kAbsorbRows) return p;
        Partials q{c.parts + (size_t)rc * c.region_doubles, nullptr, 1};
        if (K == A_K)
            hipLaunchKernelGGL(k_collapse<A_K>, dim3((unsigned)c.B), dim3(256), 0, s, p.parts, p.nb, q.parts, mask);
        else
            hipLaunchKernelGGL(k_collapse<B_K>, dim3((unsigned)c.B), dim3(256), 0, s, p.parts, p.nb, q.parts, mask);
        return q;
    };
    const Partials none{nullptr, nullptr, 0};
    // algorithmic bytes of a launch: `reals` real numbers of sizeof(T) per grid point and instance
    const double unit = (double)sizeof(T) * (double)g.N * (double)c.B;
    auto tick = [&](const char* name, double reals) {
        if (c.timer) c.timer->mark(s, name, reals * unit);
    };
    // partial regions of the direction passes (absorbed by the step at the next iteration's start,
    // through their collapsed rows when they have many)
    const Partials pb0 = region(R_B0, 0);
    const Partials pb1 = g.dim >= 2 ? region(R_B1, 1) : none;
    const Partials pb2 = g.dim >= 3 ? region(R_B2, 2) : none;
    auto view = [&](const Partials& p, int rc) -> Partials {
        if (!p.parts || p.nb <= kAbsorbRows) return p;
        return Partials{c.parts + (size_t)rc * c.region_doubles, nullptr, 1};
    };
    const Partials sb0 = view(pb0, R_B0C), sb1 = view(pb1, R_B1C), sb2 = view(pb2, R_B2C);
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
        Partials pr{c.parts + (size_t)R_A1 * c.region_doubles, nullptr, nbpi};
        tick("step_resid_diag", 21);
        hipLaunchKernelGGL(k_resid_diag<T>, dim3((unsigned)(nbpi * c.B)), dim3(256), 0, s, f, S_dir, S_step, g.N, nbpi,
                           pre, sb0, sb1, sb2, pr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        pres = consumable(pr, R_A1C, A_K, A_MAXMASK);
        pdir = pres;
        dir_in = S_step;
    } else if (g.dim == 1) {
        OpResid<T, true> op{f, S_dir, S_step, sb0, sb1, sb2, pre, post};
        tick("step_resid_precond_x", 21);
        const Partials pa = region(R_A1, 0);
        if ((e = launch_pass<T, 0>(g, c.B, c.tw->get(0, f64), op, pa, s)) != hipSuccess) return e;
        pres = consumable(pa, R_A1C, A_K, A_MAXMASK);
        pdir = pres;
        dir_in = S_step;
    } else {
        OpResid<T, false> op{f, S_dir, S_step, sb0, sb1, sb2, pre, post};
        tick("step_resid_fwd_x", 17);
        const Partials pa1r = region(R_A1, 0);
        if ((e = launch_pass<T, 0>(g, c.B, c.tw->get(0, f64), op, pa1r, s)) != hipSuccess) return e;
        const Partials pa1 = consumable(pa1r, R_A1C, A_K, A_MAXMASK);
        if (g.dim == 2) {
            OpPMid<T, 1, true, true, true> y{f.w, S_step, S_res, pa1};
            tick("resid_test_precond_y", 4);
            if ((e = launch_pass<T, 1>(g, c.B, c.tw->get(1, f64), y, none, s)) != hipSuccess) return e;
        } else {
            OpPMid<T, 1, true, false, true> y1{f.w, S_step, S_res, pa1};
            tick("resid_test_precond_fwd_y", 4);
            if ((e = launch_pass<T, 1>(g, c.B, c.tw->get(1, f64), y1, none, s)) != hipSuccess) return e;
            OpPMid<T, 2, true, true, false> z{f.w, S_res, nullptr, none};
            tick("precond_z", 4);
            if ((e = launch_pass<T, 2>(g, c.B, c.tw->get(2, f64), z, none, s)) != hipSuccess) return e;
            OpPMid<T, 1, false, true, false> y2{f.w, S_res, nullptr, none};
            tick("precond_inv_y", 4);
            if ((e = launch_pass<T, 1>(g, c.B, c.tw->get(1, f64), y2, none, s)) != hipSuccess) return e;
        }
        OpPLast<T> op3{f, S_res, post};
        tick("precond_inv_x", 13);
        const Partials pa3 = region(R_A3, 0);
        if ((e = launch_pass<T, 0>(g, c.B, c.tw->get(0, f64), op3, pa3, s)) != hipSuccess) return e;
        pdir = consumable(pa3, R_A3C, A_K, A_MAXMASK);
        dir_in = S_res;
    }
    // ---- phase B ----
    if (g.dim == 1) {
        OpLp<T, 0, true, true> op{f, dir_in, S_dir, pres, pdir};
        tick("dir_Lp_x_linesearch", 11);
        if ((e = launch_pass<T, 0>(g, c.B, c.tw->get(0, f64), op, pb0, s)) != hipSuccess) return e;
    } else if (g.dim == 2) {
        OpLp<T, 0, true, false> ox{f, dir_in, S_dir, pres, pdir};
        tick("dir_Lp_x", 10);
        if ((e = launch_pass<T, 0>(g, c.B, c.tw->get(0, f64), ox, pb0, s)) != hipSuccess) return e;
        OpLp<T, 1, false, true> oy{f, S_dir, nullptr, none, none};
        tick("Lp_y_linesearch", 9);
        if ((e = launch_pass<T, 1>(g, c.B, c.tw->get(1, f64), oy, pb1, s)) != hipSuccess) return e;
    } else {
        OpLp<T, 0, true, false> ox{f, dir_in, S_dir, pres, pdir};
        tick("dir_Lp_x", 10);
        if ((e = launch_pass<T, 0>(g, c.B, c.tw->get(0, f64), ox, pb0, s)) != hipSuccess) return e;
        OpLp<T, 1, false, false> oy{f, S_dir, nullptr, none, none};
        tick("Lp_y", 8);
        if ((e = launch_pass<T, 1>(g, c.B, c.tw->get(1, f64), oy, pb1, s)) != hipSuccess) return e;
        OpLp<T, 2, false, true> oz{f, S_dir, nullptr, none, none};
        tick("Lp_z_linesearch", 9);
        if ((e = launch_pass<T, 2>(g, c.B, c.tw->get(2, f64), oz, pb2, s)) != hipSuccess) return e;
    }
    (void)consumable(pb0, R_B0C, B_K, B_MAXMASK);
    if (pb1.parts) (void)consumable(pb1, R_B1C, B_K, B_MAXMASK);
    if (pb2.parts) (void)consumable(pb2, R_B2C, B_K, B_MAXMASK);
    return hipGetLastError();
}

template hipError_t enqueue_iteration<double>(const IterCtx<double>&, hipStream_t);
template hipError_t enqueue_iteration<float>(const IterCtx<float>&, hipStream_t);

}  // namespace gpe
