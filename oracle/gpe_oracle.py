"""Plain FP64 CPU oracle for the ground state of the rotating Gross-Pitaevskii energy.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the benchmark's CPU-baseline
leg may import or run this module; the GPU library never does.  It shares no code with the GPU
path: numpy in float64 / complex128 throughout, with numpy.fft as the transform primitive.

It follows X. Antoine, A. Levitt, Q. Tang, "Efficient spectral computation of the stationary
states of rotating Bose-Einstein condensates by the preconditioned nonlinear conjugate gradient
method" (arXiv:1611.02045).  Citations below name the paper's sections, equations and
algorithms.  Where the paper is silent or garbled, the reading taken is stated next to the code
(the "reading:" notes); all of them are also listed in the design notes.

Discrete conventions (Section 3):
  * axis a spans [-L_a, L_a) periodically with M_a (even) points, h_a = 2 L_a / M_a and
    x_k = -L_a + k h_a (reading: the phase e^{i xi_p (x_k + L)} of the paper's expansions puts the
    first grid point at -L);
  * frequencies xi_p = p pi / L_a for -M/2 <= p <= M/2 - 1, stored in FFT order (p = j or j - M);
    the Nyquist mode p = -M/2 is kept in odd derivatives exactly as written (reading);
  * forward transforms are unnormalised, the inverse carries 1/M (the paper's expansions);
  * inner product <f, g> = h^d sum conj(f) g and unit sphere h^d sum |phi|^2 = 1 (reading: the
    quadrature-weighted form is the one under which the paper's tabulated energies hold).
Arrays use numpy shape (n_x,), (n_y, n_x) or (n_z, n_y, n_x): axis a lives on numpy axis -1-a.

Parity status: every function here is pinned by a CPU test against closed forms, brute-force
sums, library eigensolvers, finite differences, the asymptotic rates and condition numbers the
paper states (Sections 4, 5.2, 5.5) or the paper's printed energies, except:
  * the iteration-by-iteration trajectory of PCG at Omega > 0: the paper shows its iteration
    counts only in figures that are not available, so no external value fixes it (parity
    unpinned for trajectories).  pcg itself is pinned through its results: the paper's printed
    energies, the exact beta = 0 ground states, the dense eigensolver, the conjugate-gradient
    contraction rate, energy decrease and norm conservation along the iterates;
  * the shift of the potential preconditioner, alpha_V = lambda~: definitional (eq. PV with the
    adaptive shift of Section 5.5), checked by reading (parity unpinned).  Its diagonal
    V + eta |phi|^2 is pinned: it equals the multiplicative part of H_phi (on constant fields,
    where T and L_z vanish, H_phi phi = (V + eta |phi|^2) phi), and the Section 5.5 scaling of
    kappa_V needs the V in it.
The Polak-Ribiere coefficient is pinned by the properties that set it apart (it vanishes when the
residual repeats, the automatic restart; it equals Fletcher-Reeves for P-orthogonal successive
residuals; it is cut at zero) and by the conjugate-gradient contraction rate.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

EPS64 = np.finfo(np.float64).eps


# ----------------------------------------------------------------------------------------------
# Grid (Section 3)
# ----------------------------------------------------------------------------------------------

def _axis_shape(dim: int, a: int, m: int) -> list:
    s = [1] * dim
    s[dim - 1 - a] = m
    return s


def coordinates(prob) -> list:
    """Grid coordinates x_{k} = -L + k h per axis, broadcastable (Section 3, uniform grid)."""
    out = []
    for a in range(prob.dim):
        M, L = prob.n[a], prob.L[a]
        x = -L + (2.0 * L / M) * np.arange(M, dtype=np.float64)
        out.append(x.reshape(_axis_shape(prob.dim, a, M)))
    return out


def frequencies(prob) -> list:
    """Discrete Fourier frequencies xi_p = p pi / L, -M/2 <= p < M/2, in transform index order
    (index j carries p = j for j < M/2 and p = j - M otherwise) (Section 3)."""
    out = []
    for a in range(prob.dim):
        M, L = prob.n[a], prob.L[a]
        j = np.arange(M)
        p = np.where(j < M // 2, j, j - M).astype(np.float64)
        out.append((p * math.pi / L).reshape(_axis_shape(prob.dim, a, M)))
    return out


def cell(prob) -> float:
    """Quadrature weight h^d."""
    return float(np.prod([2.0 * prob.L[a] / prob.n[a] for a in range(prob.dim)]))


def inner(prob, f, g) -> complex:
    """<f, g> = h^d sum conj(f) g (Section 3 inner product, quadrature-weighted reading)."""
    return cell(prob) * complex(np.vdot(f.ravel(), g.ravel()))


def norm(prob, f) -> float:
    return math.sqrt(inner(prob, f, f).real)


# ----------------------------------------------------------------------------------------------
# Pseudo-spectral operators (Section 3, the matrices [[d^2_x]], [[d^2_y]], x[[d_y]], y[[d_x]])
# ----------------------------------------------------------------------------------------------

def along_axis(prob, f, a: int, symbol) -> np.ndarray:
    """1-D transform along axis a, multiply by symbol(xi), inverse transform (the directional
    expansions of Section 3: forward sum with e^{-i xi_p (x_k + L)}, inverse with 1/M)."""
    ax = -1 - a
    fh = np.fft.fft(f, axis=ax)
    return np.fft.ifft(symbol * fh, axis=ax)


def second_derivative(prob, f, a: int) -> np.ndarray:
    """[[d^2_a]] f: symbol -xi^2."""
    xi = frequencies(prob)[a]
    return along_axis(prob, f, a, -(xi ** 2))


def first_derivative(prob, f, a: int) -> np.ndarray:
    """[[d_a]] f: symbol i xi (Nyquist kept as written)."""
    xi = frequencies(prob)[a]
    return along_axis(prob, f, a, 1j * xi)


def laplacian(prob, f) -> np.ndarray:
    """[[Delta]] = sum_a [[d^2_a]]."""
    out = np.zeros_like(f, dtype=np.complex128)
    for a in range(prob.dim):
        out = out + second_derivative(prob, f, a)
    return out


def kinetic(prob, f) -> np.ndarray:
    """T f = -(1/2) [[Delta]] f."""
    return -0.5 * laplacian(prob, f)


def angular_momentum(prob, f) -> np.ndarray:
    """[[L_z]] f = -i (x [[d_y]] f - y [[d_x]] f) (Section 3; Section 2 defines
    L_z = i (y d_x - x d_y)).  Requires dim >= 2."""
    if prob.dim < 2:
        raise ValueError("L_z needs at least two dimensions")
    X = coordinates(prob)
    return -1j * (X[0] * first_derivative(prob, f, 1) - X[1] * first_derivative(prob, f, 0))


def linear_part(prob, V, f) -> np.ndarray:
    """L f = (T + V - Omega L_z) f: the phi-independent part of the Hamiltonian."""
    out = kinetic(prob, f) + V * f
    if prob.omega != 0.0:
        out = out - prob.omega * angular_momentum(prob, f)
    return out


def hamiltonian(prob, V, phi) -> np.ndarray:
    """H_phi phi = -1/2 [[Delta]] phi + [[V]] phi + eta [[|phi|^2]] phi - Omega [[L_z]] phi
    (Section 2 mean-field Hamiltonian, discretised in Section 3)."""
    return linear_part(prob, V, phi) + prob.beta * np.abs(phi) ** 2 * phi


# ----------------------------------------------------------------------------------------------
# Energy and scalars (Section 2)
# ----------------------------------------------------------------------------------------------

@dataclass
class EnergyParts:
    kinetic: float
    potential: float
    interaction: float
    rotation: float

    @property
    def total(self) -> float:
        return self.kinetic + self.potential + self.interaction + self.rotation


def energy_parts(prob, V, phi) -> EnergyParts:
    """E(phi) = int 1/2 |grad phi|^2 + V |phi|^2 + eta/2 |phi|^4 - Omega phi^* L_z phi (Section 2),
    with the gradient term written as <phi, T phi>."""
    w = cell(prob)
    kin = inner(prob, phi, kinetic(prob, phi)).real
    rho = np.abs(phi) ** 2
    pot = w * float(np.sum(V * rho))
    inter = 0.5 * prob.beta * w * float(np.sum(rho * rho))
    rot = 0.0
    if prob.omega != 0.0:
        rot = -prob.omega * inner(prob, phi, angular_momentum(prob, phi)).real
    return EnergyParts(kin, pot, inter, rot)


def energy(prob, V, phi) -> float:
    return energy_parts(prob, V, phi).total


def chemical_potential(prob, V, phi) -> float:
    """lambda = <H_phi phi, phi> (Section 2, Euler-Lagrange multiplier)."""
    return inner(prob, phi, hamiltonian(prob, V, phi)).real


def characteristic_energy(prob, V, phi) -> float:
    """lambda~ = int 1/2 |grad phi|^2 + V |phi|^2 + eta |phi|^4 (Section 5.5, adaptive shift;
    no rotation term, eta rather than eta/2)."""
    p = energy_parts(prob, V, phi)
    return p.kinetic + p.potential + 2.0 * p.interaction


def residual(prob, V, phi):
    """r = H_phi phi - lambda phi with lambda = <H_phi phi, phi> (Algorithm 1)."""
    Hphi = hamiltonian(prob, V, phi)
    lam = inner(prob, phi, Hphi).real
    return Hphi - lam * phi, lam


def project(prob, phi, h) -> np.ndarray:
    """M_phi h = h - Re<phi, h> phi: projection on the tangent space of the sphere (Section 2)."""
    return h - inner(prob, phi, h).real * phi


def hessian_form(prob, V, phi, f) -> float:
    """(1/2) nabla^2 E(phi)[f, f] = <f, H_phi f> + 2 eta int (Re conj(phi) f)^2.
    Reading: the Section 2 formula omits eta int |phi|^2 |f|^2; this is the second-order
    coefficient of E(phi + t f) in t (pinned by finite differences)."""
    w = cell(prob)
    q = (np.conj(phi) * f).real
    Hf = linear_part(prob, V, f) + prob.beta * np.abs(phi) ** 2 * f   # H_phi applied to f
    return inner(prob, f, Hf).real + 2.0 * prob.beta * w * float(np.sum(q * q))


# ----------------------------------------------------------------------------------------------
# Preconditioners (Section 5.5)
# ----------------------------------------------------------------------------------------------

PRECONDITIONERS = ("none", "kinetic", "potential", "combined", "c1", "c2")


def kinetic_preconditioner(prob, f, alpha: float) -> np.ndarray:
    """P_Delta f = (alpha - Delta/2)^{-1} f: Fourier-diagonal with symbol 1/(alpha + |xi|^2/2)."""
    k2 = np.zeros(prob.shape)
    for xi in frequencies(prob):
        k2 = k2 + xi ** 2
    axes = tuple(range(-prob.dim, 0))
    return np.fft.ifftn(np.fft.fftn(f, axes=axes) / (alpha + 0.5 * k2), axes=axes)


def potential_diagonal(prob, V, phi, alpha: float) -> np.ndarray:
    """alpha + V + eta |phi|^2, the inverse of P_V as a real diagonal (Section 5.5)."""
    d = alpha + V + prob.beta * np.abs(phi) ** 2
    if not np.all(d > 0.0):
        raise ValueError("alpha + V + eta|phi|^2 must be positive for an SPD preconditioner")
    return d


def apply_preconditioner(prob, kind: str, V, phi, r, alpha: float | None = None) -> np.ndarray:
    """P r for P in {I, P_Delta, P_V, P_C = P_V^{1/2} P_Delta P_V^{1/2}, P_C1 = P_V P_Delta,
    P_C2 = P_Delta P_V}, with alpha = lambda~(phi) unless given (Section 5.5)."""
    if alpha is None:
        alpha = characteristic_energy(prob, V, phi)
    if kind == "none":
        return r.copy()
    if kind == "kinetic":
        return kinetic_preconditioner(prob, r, alpha)
    d = potential_diagonal(prob, V, phi, alpha)
    if kind == "potential":
        return r / d
    if kind == "combined":
        s = 1.0 / np.sqrt(d)
        return s * kinetic_preconditioner(prob, s * r, alpha)
    if kind == "c1":
        return kinetic_preconditioner(prob, r, alpha) / d
    if kind == "c2":
        return kinetic_preconditioner(prob, r / d, alpha)
    raise ValueError(f"unknown preconditioner {kind!r}")


# ----------------------------------------------------------------------------------------------
# Line search pieces (Section 5.1)
# ----------------------------------------------------------------------------------------------

def energy_along(prob, V, phi, phat, theta: float) -> float:
    """E(cos(theta) phi + sin(theta) phat) by the plain definition."""
    return energy(prob, V, math.cos(theta) * phi + math.sin(theta) * phat)


def energy_change(prob, phi, phat, Lphi, Lphat, theta: float) -> float:
    """E(cos t phi + sin t phat) - E(phi), written without cancellation of O(1) terms.
    Reading of the paper's acceptance test ("the energy is decreased"): both energies are
    quadratic + quartic in the field, so the difference is expanded exactly:
      quadratic: s^2 (<phat, L phat> - <phi, L phi>) + 2 c s Re<phi, L phat>,
      quartic:   (eta/2) h^d sum D (2 |phi|^2 + D),  D = s^2 (|phat|^2 - |phi|^2) + 2 c s Re(conj(phi) phat),
    which equals the plain difference up to rounding but resolves decreases far below eps*|E|."""
    c, s = math.cos(theta), math.sin(theta)
    w = cell(prob)
    a = inner(prob, phi, Lphi).real
    b = inner(prob, phi, Lphat).real
    cc = inner(prob, phat, Lphat).real
    quad = s * s * (cc - a) + 2.0 * c * s * b
    rho = np.abs(phi) ** 2
    D = s * s * (np.abs(phat) ** 2 - rho) + 2.0 * c * s * (np.conj(phi) * phat).real
    quart = 0.5 * prob.beta * w * float(np.sum(D * (2.0 * rho + D)))
    return quad + quart


def theta_derivatives(prob, V, phi, phat, lam: float):
    """E'(0) and E''(0) of theta -> E(cos theta phi + sin theta phat) for unit phat orthogonal to
    phi.  Reading of the garbled expansion of Section 5.1: E'(0) = Re<nabla E, phat> =
    2 Re<H_phi phi, phat>, E''(0) = nabla^2 E[phat, phat] - 2 lambda."""
    d1 = 2.0 * inner(prob, hamiltonian(prob, V, phi), phat).real
    d2 = 2.0 * (hessian_form(prob, V, phi, phat) - lam)
    return d1, d2


def energy_slope(prob, V, phi, phat, theta: float) -> float:
    """dE/dtheta of theta -> E(u), u = cos(theta) phi + sin(theta) phat, by the chain rule on the
    Section 2 gradient: E'(u)[u'] = 2 Re<H_u u, u'>, u' = -sin(theta) phi + cos(theta) phat."""
    c, s = math.cos(theta), math.sin(theta)
    u = c * phi + s * phat
    du = -s * phi + c * phat
    return 2.0 * inner(prob, hamiltonian(prob, V, u), du).real


# Samples of the period [0, pi) that locate the global minimiser of the full line search.
FULL_SEARCH_SAMPLES = 64
# Sufficient-decrease constant of the Armijo test (the paper names the test, not the constant;
# reading: the customary 1e-4).
ARMIJO_C1 = 1e-4
# Curvature constant of the strong Wolfe conditions (reading: 0.1, the usual choice for nonlinear
# conjugate gradients, below the 1/2 that keeps their directions descent directions).
WOLFE_C2 = 0.1


def theta_full(prob, V, phi, phat, Lphi, Lphat, samples: int = FULL_SEARCH_SAMPLES) -> float:
    """The full line search of Section 5.1: theta = argmin E(cos theta phi + sin theta phat).
    E along the great circle has period pi (u -> -u leaves E unchanged), so the minimiser is
    sought in [0, pi).  Readings: the global minimiser is taken; it is located on `samples` equally
    spaced angles (the energy change of each, see energy_change), then refined to a zero of the
    slope (energy_slope) bracketed between the best angle and the neighbour towards which the
    energy falls, by Brent's method to a few ulps.  The result is reduced into [0, pi)."""
    from scipy.optimize import brentq

    step = math.pi / samples
    vals = [energy_change(prob, phi, phat, Lphi, Lphat, k * step) for k in range(samples)]
    k = int(np.argmin(vals))
    t0 = k * step
    g0 = energy_slope(prob, V, phi, phat, t0)
    lo, hi = (t0, t0 + step) if g0 < 0.0 else (t0 - step, t0)
    glo, ghi = energy_slope(prob, V, phi, phat, lo), energy_slope(prob, V, phi, phat, hi)
    if g0 == 0.0 or not (glo < 0.0 < ghi):
        t = t0
    else:
        t = brentq(lambda x: energy_slope(prob, V, phi, phat, x), lo, hi, xtol=1e-300, rtol=4 * EPS64,
                   maxiter=200)
    return t % math.pi


def trial_ladder(prob, phi, phat, Lphi, Lphat, theta: float, d1: float, max_halvings: int,
                 armijo: bool = False):
    """Step control of Section 5.1: the trials theta, theta/2, theta/4, ... (at most max_halvings
    halvings); the first whose energy change is negative is accepted (with armijo=True, the first
    that also satisfies E(t) - E(0) <= ARMIJO_C1 t E'(0), E'(0) = d1).  Returns (t, halvings), or
    (None, max_halvings) when no trial passes."""
    for j in range(max_halvings + 1):
        t = theta * 0.5 ** j
        if not t > 0.0:
            continue
        dE = energy_change(prob, phi, phat, Lphi, Lphat, t)
        if dE < 0.0 and (not armijo or dE <= ARMIJO_C1 * t * d1):
            return t, j
    return None, max_halvings


def wolfe_search(prob, V, phi, phat, Lphi, Lphat, theta: float, d1: float, max_steps: int):
    """A step satisfying the strong Wolfe conditions (named in Section 5.1 as an acceptance rule):
        f(t) <= ARMIJO_C1 t f'(0)  and  |f'(t)| <= -WOLFE_C2 f'(0),   f(t) = E(t) - E(0),
    by the textbook bracketing search (readings: start at the heuristic's trial theta, double the
    step while it is too short, at most up to pi/2, where a step that still descends is taken) and
    a zoom by bisection of the bracket (the midpoint of the two ends each time), at most max_steps
    evaluations in each phase.  f is energy_change, f' is energy_slope.  Returns (t, evaluations)
    or (None, evaluations)."""
    half_pi = 0.5 * math.pi
    f = lambda t: energy_change(prob, phi, phat, Lphi, Lphat, t)
    g = lambda t: energy_slope(prob, V, phi, phat, t)
    armijo = lambda t, ft: ft <= ARMIJO_C1 * t * d1
    curv = lambda gt: abs(gt) <= -WOLFE_C2 * d1

    def zoom(lo, f_lo, hi, n):
        for _ in range(max_steps):
            t = 0.5 * (lo + hi)
            n += 1
            ft = f(t)
            if not armijo(t, ft) or ft >= f_lo:
                hi = t
            else:
                gt = g(t)
                if curv(gt):
                    return t, n
                if gt * (hi - lo) >= 0.0:
                    hi = lo
                lo, f_lo = t, ft
        return None, n

    t_prev, f_prev = 0.0, 0.0
    t = min(theta, half_pi)
    n = 0
    for i in range(max_steps):
        n += 1
        ft = f(t)
        if not armijo(t, ft) or (i > 0 and ft >= f_prev):
            return zoom(t_prev, f_prev, t, n)
        gt = g(t)
        if curv(gt):
            return t, n
        if gt >= 0.0:
            return zoom(t, ft, t_prev, n)
        if t >= half_pi:
            return t, n
        t_prev, f_prev = t, ft
        t = min(2.0 * t, half_pi)
    return None, n


# ----------------------------------------------------------------------------------------------
# PG / PCG on the sphere (Algorithms 1 and 2, Sections 5.1-5.3)
# ----------------------------------------------------------------------------------------------

@dataclass
class SolveResult:
    phi: np.ndarray
    status: str
    iters: int
    E: float
    lam: float
    res_inf: float
    restarts: int = 0
    halvings: int = 0
    history: list = field(default_factory=list)


def cg_coefficient(prob, r, Pr, r_prev, rPr_prev: float, rule: str = "pr") -> float:
    """The conjugate-gradient coefficient of Section 5.2 (eq. CG:PR) from the current residual r_n,
    its preconditioned form P_n r_n, the previous residual r_{n-1} and the stored
    <r_{n-1}, P_{n-1} r_{n-1}>: Polak-Ribiere, kept non-negative,
    max((<r_n, P_n r_n> - Re<r_{n-1}, P_n r_n>) / <r_{n-1}, P_{n-1} r_{n-1}>, 0), or with
    rule="fr" the Fletcher-Reeves ratio <r_n, P_n r_n> / <r_{n-1}, P_{n-1} r_{n-1}>."""
    rPr = inner(prob, r, Pr).real
    if rule == "fr":
        return rPr / rPr_prev
    return max((rPr - inner(prob, r_prev, Pr).real) / rPr_prev, 0.0)


def pcg(prob, V, phi0, *, method: str = "pcg", precond: str = "combined", tol_res: float = 1e-8,
        tol_energy: float = 0.0, max_iter: int = 10_000, theta_default: float = 0.1,
        max_halvings: int = 30, beta_rule: str = "pr", line_search: str = "heuristic",
        record: bool = False) -> SolveResult:
    """Projected preconditioned gradient (method="pg", Algorithm 1) or conjugate gradient
    (method="pcg", Algorithm 2) minimisation of E on the unit sphere, with the step control of
    Sections 5.1-5.2 and the residual stopping rule of Section 5.3.

    Readings (the paper is silent on these):
      * beta at n = 0 is 0; beta = max(beta^PR, 0) with numerator <r_n, P_n r_n> -
        Re<r_{n-1}, P_n r_n> and the stored denominator <r_{n-1}, P_{n-1} r_{n-1}>;
        beta_rule="fr" uses the Fletcher-Reeves ratio instead;
      * p_{n-1} is used as stored (no transport between tangent spaces);
      * not a descent direction <=> Re<r_n, p_n> >= 0, then the gradient direction is used;
      * trial step theta_opt = -E'(0)/E''(0) when E''(0) > 0, else theta_default; clamped to
        (0, pi/2]; halved until the energy decreases (at most max_halvings times, after which the
        run stops with status "linesearch");
      * line_search="armijo" accepts a trial only when E(theta) - E(0) <= ARMIJO_C1 theta E'(0)
        (the Armijo test the section names as an alternative), halving as above;
        line_search="full" takes theta_full (the full line search of the section), accepted
        when it decreases the energy, else the run stops with status "linesearch";
        line_search="wolfe" takes wolfe_search from the same trial (max_halvings bounds each of
        its phases; halvings records its evaluations);
      * phi is renormalised after every step;
      * stop when ||r_n||_inf <= tol_res at the top of iteration n (or, when tol_energy > 0,
        when |E_{n+1} - E_n| <= tol_energy).
    """
    if method not in ("pg", "pcg"):
        raise ValueError("method must be 'pg' or 'pcg'")
    if line_search not in ("heuristic", "armijo", "full", "wolfe"):
        raise ValueError("line_search must be 'heuristic', 'armijo', 'full' or 'wolfe'")
    phi = np.array(phi0, dtype=np.complex128, copy=True)
    phi /= norm(prob, phi)
    r_prev = p_prev = None
    rPr_prev = 0.0
    hist = []
    restarts = halvings = 0
    status = "not_converged"
    E_prev = None
    n = 0
    for n in range(max_iter + 1):
        # lambda_n, r_n
        r, lam = residual(prob, V, phi)
        res = float(np.max(np.abs(r)))
        E = energy(prob, V, phi)
        if record:
            hist.append({"n": n, "E": E, "lam": lam, "res": res})
        if res <= tol_res:
            status = "converged"
            break
        if tol_energy > 0.0 and E_prev is not None and abs(E - E_prev) <= tol_energy:
            status = "converged"
            break
        if n == max_iter:
            break
        E_prev = E
        # preconditioned residual, alpha = lambda~_n (Section 5.5)
        Pr = apply_preconditioner(prob, precond, V, phi, r)
        rPr = inner(prob, r, Pr).real
        # CG coefficient (Section 5.2)
        beta = 0.0
        if method == "pcg" and p_prev is not None and rPr_prev > 0.0:
            beta = cg_coefficient(prob, r, Pr, r_prev, rPr_prev, beta_rule)
        d = -Pr + beta * p_prev if beta != 0.0 else -Pr
        p = project(prob, phi, d)
        restarted = False
        if inner(prob, r, p).real >= 0.0:
            # not a descent direction: revert to the gradient step (Section 5.2)
            p = project(prob, phi, -Pr)
            beta = 0.0
            restarted = True
            restarts += 1
        pn = norm(prob, p)
        phat = p / pn
        # trial step (Section 5.1): minimiser of the second-order model
        d1, d2 = theta_derivatives(prob, V, phi, phat, lam)
        theta = -d1 / d2 if d2 > 0.0 else theta_default
        theta = min(max(theta, 0.0), 0.5 * math.pi)
        Lphi = linear_part(prob, V, phi)
        Lphat = linear_part(prob, V, phat)
        j = 0
        if line_search == "full":
            t = theta_full(prob, V, phi, phat, Lphi, Lphat)
            accepted = t if energy_change(prob, phi, phat, Lphi, Lphat, t) < 0.0 else None
        elif line_search == "wolfe":
            accepted, j = wolfe_search(prob, V, phi, phat, Lphi, Lphat, theta, d1, max_halvings)
            if accepted is not None:
                halvings += j
        else:
            accepted, j = trial_ladder(prob, phi, phat, Lphi, Lphat, theta, d1, max_halvings,
                                       armijo=line_search == "armijo")
            if accepted is not None:
                halvings += j
        if accepted is None:
            status = "linesearch"
            break
        if record:
            hist[-1].update(theta=accepted, beta=beta, restarted=restarted, d1=d1, d2=d2,
                            halvings=j)
        new = math.cos(accepted) * phi + math.sin(accepted) * phat
        new /= norm(prob, new)
        r_prev, p_prev, rPr_prev = r, p, rPr
        phi = new
    E = energy(prob, V, phi)
    r, lam = residual(prob, V, phi)
    return SolveResult(phi, status, n, E, lam, float(np.max(np.abs(r))), restarts, halvings, hist)


# ----------------------------------------------------------------------------------------------
# Nested grids (Section 6, the multigrid preparation of initial data)
# ----------------------------------------------------------------------------------------------

def refined(prob):
    """The same box with twice the points per axis (level p -> p + 1 of the nested grids)."""
    import dataclasses
    n = tuple(2 * int(prob.n[a]) if a < prob.dim else int(prob.n[a]) for a in range(len(prob.n)))
    return dataclasses.replace(prob, n=n)


def prolong(prob, f) -> np.ndarray:
    """Interpolate a grid function of `prob` onto the grid with twice the points per axis and the
    same box, axis by axis, by its trigonometric interpolant (the interpolation step of the nested
    grids of Section 6; reading: the paper does not name the interpolation, and the spectral one
    matches its Fourier discretisation).  Along an axis of M points the coefficients X_p,
    -M/2 < p < M/2, are kept; the Nyquist coefficient X_{-M/2} is split evenly between the
    frequencies -M/2 and +M/2 of the fine grid (reading: the symmetric split keeps real data real
    and is the interpolant of least norm); the fine grid's other coefficients are zero.  Coarse
    points are fine points 0, 2, 4, ...; there the result equals the input."""
    out = np.asarray(f, dtype=np.complex128)
    for a in range(prob.dim):
        ax = prob.dim - 1 - a
        M = out.shape[ax]
        X = np.fft.fft(out, axis=ax)
        shape = list(out.shape)
        shape[ax] = 2 * M
        Y = np.zeros(shape, dtype=np.complex128)

        def put(dst, src, scale):
            sl_d = [slice(None)] * out.ndim
            sl_s = [slice(None)] * out.ndim
            sl_d[ax], sl_s[ax] = dst, src
            Y[tuple(sl_d)] += scale * X[tuple(sl_s)]

        # fine inverse transform carries 1/(2M): coefficients double to evaluate the same sum
        put(slice(0, M // 2), slice(0, M // 2), 2.0)                      # p = 0 .. M/2 - 1
        put(slice(2 * M - M // 2 + 1, 2 * M), slice(M // 2 + 1, M), 2.0)  # p = -M/2 + 1 .. -1
        put(slice(M // 2, M // 2 + 1), slice(M // 2, M // 2 + 1), 1.0)    # Nyquist, at +M/2 ...
        put(slice(2 * M - M // 2, 2 * M - M // 2 + 1), slice(M // 2, M // 2 + 1), 1.0)  # ... and -M/2
        out = np.fft.ifft(Y, axis=ax)
    return out


def pcg_nested(probs, Vs, phi0, *, tol_coarse: float = 1e-6, tol_res: float = 1e-8, max_iter: int = 20_000,
               **kw):
    """Ground state on nested grids (Section 6): solve on the coarsest grid from phi0, interpolate
    the converged state onto the next grid (prolong), renormalise it and solve again, up to the
    finest grid.  probs[l], Vs[l]: the problem and potential of level l (each grid twice the
    previous one per axis, same box); the coarse levels stop at ||r||_inf <= tol_coarse, the finest
    at tol_res.  Returns the finest level's SolveResult and the list of all levels' results."""
    results = []
    phi = phi0
    for lvl, (prob, V) in enumerate(zip(probs, Vs)):
        if lvl > 0:
            phi = prolong(probs[lvl - 1], results[-1].phi)
        last = lvl == len(probs) - 1
        results.append(pcg(prob, V, phi, tol_res=tol_res if last else tol_coarse, max_iter=max_iter, **kw))
    return results[-1], results


# ----------------------------------------------------------------------------------------------
# Backward Euler imaginary-time scheme (Section 4), used as an independent check of PCG
# ----------------------------------------------------------------------------------------------

def conjugate_gradient(prob, apply, rhs, x0, tol: float = 1e-10, max_iter: int = 10_000):
    """Linear CG for a Hermitian positive definite operator in the <.,.> inner product."""
    x = x0.copy()
    r = rhs - apply(x)
    p = r.copy()
    rr = inner(prob, r, r).real
    b2 = inner(prob, rhs, rhs).real
    it = 0
    for it in range(max_iter):
        if rr <= tol * tol * b2:
            break
        Ap = apply(p)
        pAp = inner(prob, p, Ap).real
        if pAp <= 0.0:
            raise ValueError("operator is not positive definite")
        a = rr / pAp
        x = x + a * p
        r = r - a * Ap
        rr_new = inner(prob, r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, it


def backward_euler(prob, V, phi0, *, dt: float = 0.01, lambda_term: bool = True,
                   inner_tol: float = 1e-10, tol_res: float = 1e-8, max_iter: int = 100_000,
                   record: bool = False):
    """BE discretisation of the normalised gradient flow (Section 4), H = H_{phi_n} frozen at the
    current iterate (semi-implicit nonlinearity), followed by phi_{n+1} = phi~ / ||phi~||.
    Without the lambda term: (phi~ - phi_n)/dt = -H phi~.  With it (reading): the multiplier acts
    on the new iterate, (I/dt + H - lambda_n) phi~ = phi_n / dt.  Section 4 states that this
    scheme equals the plain one with the effective step dt/(1 - dt lambda) and that it needs the
    system (H - lambda) phi~ = phi_n; placing lambda_n on phi_n instead would make the term a
    scalar factor that the normalisation removes.  The linear solve is matrix-free CG (the
    operator is SPD for the traps used here when 1/dt > lambda_n - lambda_1)."""
    phi = np.array(phi0, dtype=np.complex128, copy=True)
    phi /= norm(prob, phi)
    hist = []
    inner_total = 0
    status = "not_converged"
    n = 0
    for n in range(max_iter + 1):
        r, lam = residual(prob, V, phi)
        res = float(np.max(np.abs(r)))
        if record:
            hist.append({"n": n, "E": energy(prob, V, phi), "lam": lam, "res": res})
        if res <= tol_res:
            status = "converged"
            break
        if n == max_iter:
            break
        rho = np.abs(phi) ** 2

        shift = lam if lambda_term else 0.0

        def op(x, rho=rho, shift=shift):
            return (1.0 / dt - shift) * x + linear_part(prob, V, x) + prob.beta * rho * x

        phit, k = conjugate_gradient(prob, op, phi / dt, phi, tol=inner_tol)
        inner_total += k
        phi = phit / norm(prob, phit)
    r, lam = residual(prob, V, phi)
    out = SolveResult(phi, status, n, energy(prob, V, phi), lam, float(np.max(np.abs(r))), history=hist)
    out.inner_iterations = inner_total
    return out


def backward_euler_step(prob, V, phi, dt: float, lambda_term: bool = True,
                        inner_tol: float = 1e-13) -> np.ndarray:
    """One BE step of Section 4 (same reading as ``backward_euler``) and normalisation."""
    Hphi = hamiltonian(prob, V, phi)
    shift = inner(prob, phi, Hphi).real if lambda_term else 0.0
    rho = np.abs(phi) ** 2

    def op(x):
        return (1.0 / dt - shift) * x + linear_part(prob, V, x) + prob.beta * rho * x

    phit, _ = conjugate_gradient(prob, op, phi / dt, phi, tol=inner_tol)
    return phit / norm(prob, phit)


def forward_euler_step(prob, V, phi, dt: float, lambda_term: bool = True) -> np.ndarray:
    """One FE step of Section 4 followed by the normalisation step."""
    Hphi = hamiltonian(prob, V, phi)
    if lambda_term:
        lam = inner(prob, phi, Hphi).real
        new = phi - dt * (Hphi - lam * phi)
    else:
        new = phi - dt * Hphi
    return new / norm(prob, new)


# ----------------------------------------------------------------------------------------------
# Dense assembly for tiny grids (tests)
# ----------------------------------------------------------------------------------------------

def dense_operator(prob, apply) -> np.ndarray:
    """Matrix of a linear map on C^N, assembled column by column on the grid basis."""
    N = int(np.prod(prob.shape))
    A = np.zeros((N, N), dtype=np.complex128)
    for k in range(N):
        e = np.zeros(N, dtype=np.complex128)
        e[k] = 1.0
        A[:, k] = apply(e.reshape(prob.shape)).ravel()
    return A


# ----------------------------------------------------------------------------------------------
# Implicit differentiation of the ground state (second-order conditions of Section 2)
# ----------------------------------------------------------------------------------------------

def hessian_apply(prob, V, phi, f) -> np.ndarray:
    """(1/2) nabla^2 E(phi)[f] = H_phi f + 2 eta Re(conj(phi) f) phi: the real-linear second
    derivative whose quadratic form is ``hessian_form`` (Section 2, completed interaction term)."""
    return (linear_part(prob, V, f) + prob.beta * np.abs(phi) ** 2 * f
            + 2.0 * prob.beta * (np.conj(phi) * f).real * phi)


def project_gauge(prob, phi, f) -> np.ndarray:
    """Projection onto {phi, i phi}^perp in the real inner product Re<.,.>: removes the sphere's
    normal direction and the global-phase (gauge) null direction of the Hessian.  phi is unit."""
    iphi = 1j * phi
    return f - inner(prob, phi, f).real * phi - inner(prob, iphi, f).real * iphi


@dataclass
class CurvatureCheck:
    """Outcome of ``second_order_check``.  ``negative`` is True when a tangent direction h with
    (1/2) nabla^2 E[h, h] - lambda ||h||^2 <= 0 was met (then ``direction`` holds it and
    ``rayleigh`` its value of that form over ||h||^2: a certificate that phi is not a strict local
    minimum); otherwise ``min_ritz`` is the smallest Ritz value of the preconditioned operator P A
    on the Krylov space explored, ``iters`` the CG steps and ``rel_res`` the final relative
    residual."""
    negative: bool
    min_ritz: float
    max_ritz: float
    rayleigh: float
    iters: int
    rel_res: float
    direction: np.ndarray | None = None


def second_order_check(prob, V, phi, rhs, *, tol: float = 1e-6, max_iter: int = 3000,
                       precond: str = "combined", shift: float = 0.0, progress=None) -> CurvatureCheck:
    """Second-order condition of Section 2 at a stationary state phi: for every tangent h,
    (1/2) nabla^2 E(phi)[h, h] - lambda ||h||^2 >= 0, strictly on {phi, i phi}^perp for a strict
    local minimum (the global phase i phi is a null direction of every state).

    Preconditioned linear CG on A mu = Pi rhs, A = Pi ((1/2) nabla^2 E(phi) - lambda) Pi, in the
    real inner product Re<.,.> (the system of ``adjoint_solve``).  CG meets a direction p with
    <p, A p> <= 0 exactly when the Lanczos matrix of the run stops being positive definite; a run
    that reaches ``tol`` with every curvature positive has resolved every eigen-component of the
    right-hand side above that level.  The Lanczos matrix T of the run (diagonal 1/a_k +
    b_{k-1}/a_{k-1}, off-diagonal sqrt(b_k)/a_k from the CG step lengths a_k and ratios b_k)
    gives the Ritz values of P A.  precond="none" gives those of A itself.

    shift > 0 checks A + shift instead, i.e. the weaker condition that no tangent curvature lies
    below -shift: directions of curvature in [-shift, 0] count as flat.  (Degenerate families of
    minima, such as the rotations of a vortex lattice in an isotropic trap, leave curvatures at
    rounding level of either sign.)  The reported Ritz values are those of P (A + shift);
    ``rayleigh`` is always that of A.  progress, if given, is called as progress(step, relative
    residual) every 100 steps."""
    lam = chemical_potential(prob, V, phi)
    alpha = characteristic_energy(prob, V, phi)

    def A(f):
        return project_gauge(prob, phi, hessian_apply(prob, V, phi, f) - (lam - shift) * f)

    def P(f):
        f = project_gauge(prob, phi, f)
        if precond != "none":
            f = project_gauge(prob, phi, apply_preconditioner(prob, precond, V, phi, f, alpha=alpha))
        return f

    b = project_gauge(prob, phi, rhs)
    r = b.copy()
    z = P(r)
    p = z.copy()
    rz = inner(prob, r, z).real
    b2 = math.sqrt(inner(prob, b, b).real)
    steps, ratios = [], []
    rel = 1.0
    for k in range(max_iter):
        q = A(p)
        pq = inner(prob, p, q).real
        if pq <= 0.0:
            return CurvatureCheck(True, float("nan"), float("nan"), pq / inner(prob, p, p).real - shift, k, rel, p)
        a = rz / pq
        steps.append(a)
        r = r - a * q
        rel = math.sqrt(inner(prob, r, r).real) / b2
        if rel <= tol:
            break
        if progress is not None and (k + 1) % 100 == 0:
            progress(k + 1, rel)
        z = P(r)
        rz_new = inner(prob, r, z).real
        ratios.append(rz_new / rz)
        p = z + ratios[-1] * p
        rz = rz_new
    m = len(steps)
    diag = np.array([1.0 / steps[0]] + [1.0 / steps[i] + ratios[i - 1] / steps[i - 1] for i in range(1, m)])
    off = np.array([math.sqrt(ratios[i]) / steps[i] for i in range(m - 1)])
    ritz = np.linalg.eigvalsh(np.diag(diag) + np.diag(off, 1) + np.diag(off, -1))
    return CurvatureCheck(False, float(ritz[0]), float(ritz[-1]), float("nan"), m, rel)


def adjoint_solve(prob, V, phi, rhs, *, tol: float = 1e-10, max_iter: int = 5000, precond: str = "combined"):
    """Solve A mu = Pi rhs with A = Pi ((1/2) nabla^2 E(phi) - lambda) Pi on {phi, i phi}^perp by
    preconditioned linear CG in the real inner product (A is SPD there at a local minimum:
    the second-order condition of Section 2).  The preconditioner is Pi P Pi with the solver's P
    at phi.  Returns (mu, iterations, final relative residual)."""
    lam = chemical_potential(prob, V, phi)
    alpha = characteristic_energy(prob, V, phi)

    def A(f):
        return project_gauge(prob, phi, hessian_apply(prob, V, phi, f) - lam * f)

    def P(f):
        return project_gauge(prob, phi, apply_preconditioner(prob, precond, V, phi, project_gauge(prob, phi, f),
                                                             alpha=alpha))

    b = project_gauge(prob, phi, rhs)
    x = np.zeros_like(b)
    r = b.copy()
    z = P(r)
    p = z.copy()
    rz = inner(prob, r, z).real
    b2 = math.sqrt(inner(prob, b, b).real)
    it = 0
    rel = 0.0 if b2 == 0 else 1.0
    for it in range(max_iter):
        rel = math.sqrt(inner(prob, r, r).real) / b2 if b2 > 0 else 0.0
        if rel <= tol:
            break
        q = A(p)
        pq = inner(prob, p, q).real
        if pq <= 0.0:
            raise ValueError("the projected Hessian is not positive definite (not a local minimum)")
        a = rz / pq
        x = x + a * p
        r = r - a * q
        z = P(r)
        rz_new = inner(prob, r, z).real
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, rel


def density_loss(prob, phi, rho_target) -> float:
    """h^d sum (|phi|^2 - rho_target)^2."""
    return cell(prob) * float(np.sum((np.abs(phi) ** 2 - rho_target) ** 2))


def density_loss_gradient(prob, phi, rho_target) -> np.ndarray:
    """g with d(density_loss) = Re<g, d phi>: g = 4 (|phi|^2 - rho_target) phi."""
    return 4.0 * (np.abs(phi) ** 2 - rho_target) * phi


def implicit_gradient(prob, V, phi, g, dV_list, *, tol: float = 1e-11):
    """Gradient of  l(theta) = E(phi*; theta) + G(phi*)  at a converged ground state phi*, where
    d G = Re<g, d phi>.  By the envelope property the energy contributes its partial derivatives
    only; G contributes -Re<mu, (d_theta H) phi*> with A mu = Pi g.  dV_list holds dV/dtheta for
    the potential parameters; the last two entries of the result are d/d eta and d/d Omega."""
    mu, _, _ = adjoint_solve(prob, V, phi, g, tol=tol)
    w = cell(prob)
    rho = np.abs(phi) ** 2
    out = []
    for dV in dV_list:
        out.append(w * float(np.sum(dV * rho)) - inner(prob, mu, dV * phi).real)
    out.append(0.5 * w * float(np.sum(rho * rho)) - inner(prob, mu, rho * phi).real)
    if prob.dim >= 2:
        lz = angular_momentum(prob, phi)
        out.append(-inner(prob, phi, lz).real - inner(prob, mu, -lz).real)
    else:
        out.append(0.0)
    return np.array(out), mu
