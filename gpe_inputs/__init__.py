"""Seeded synthetic inputs for the rotating Gross-Pitaevskii ground-state solver.

This module only *generates* problem data -- grid coordinates, trap potentials and initial
wave functions -- from numpy seeds.  It holds none of the solver's arithmetic (no transforms,
no energies, no Hamiltonian).  Both the GPU library's tests/bench and the CPU oracle draw their
inputs from here, so that the two sides see bit-identical arrays.

Conventions (the paper's Section 3 grid): axis a spans the periodic box [-L_a, L_a) with M_a
points, h_a = 2 L_a / M_a, x_k = -L_a + k h_a.  Arrays are C-ordered with x fastest, i.e. numpy
shape (n_x,), (n_y, n_x) or (n_z, n_y, n_x).  Wave functions are complex128, potentials float64;
callers cast to complex64/float32 for the single-precision path.

Every generated wave function is scaled so that h^d * sum |phi|^2 = 1 (the quadrature-weighted
unit sphere).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Seeds of the named workloads.
SEED_1D = 101
SEED_2D_256 = 102
SEED_2D_512 = 103
SEED_3D = 104
SEED_PINS = 105
SEED_THETA_TARGET = 106
SEED_BATCH_BASE = 2000
# seeded vortex-seed starts of the 2-D 512^2 time-to-tolerance workload (the first is SEED_2D_512)
SEEDS_2D_512_SET = (103, 107, 109, 113, 127, 131, 137, 139)


@dataclass(frozen=True)
class Problem:
    """Discrete problem description: dimension, points and half-widths per axis (x, y, z),
    nonlinearity strength ``beta`` (the paper's eta) and rotation speed ``omega``."""

    dim: int
    n: tuple
    L: tuple
    beta: float
    omega: float

    def __post_init__(self):
        if self.dim not in (1, 2, 3):
            raise ValueError("dim must be 1, 2 or 3")
        if len(self.n) < self.dim or len(self.L) < self.dim:
            raise ValueError("n and L need one entry per axis")

    @property
    def shape(self) -> tuple:
        return tuple(int(self.n[a]) for a in reversed(range(self.dim)))

    @property
    def h(self) -> tuple:
        return tuple(2.0 * self.L[a] / self.n[a] for a in range(self.dim))

    @property
    def cell(self) -> float:
        return float(np.prod(self.h))

    @property
    def size(self) -> int:
        return int(np.prod(self.shape))


def axis_points(M: int, L: float) -> np.ndarray:
    """Grid points x_k = -L + k (2L/M), k = 0..M-1 of one axis."""
    return -L + (2.0 * L / M) * np.arange(M, dtype=np.float64)


def mesh(prob: Problem) -> list:
    """Broadcastable coordinate arrays [x, y, (z)] for the array layout of ``prob``."""
    out = []
    for a in range(prob.dim):
        shape = [1] * prob.dim
        shape[prob.dim - 1 - a] = prob.n[a]
        out.append(axis_points(prob.n[a], prob.L[a]).reshape(shape))
    return out


def _unit(phi: np.ndarray, prob: Problem) -> np.ndarray:
    s = math.sqrt(prob.cell * float(np.sum(np.abs(phi) ** 2)))
    return (phi / s).astype(np.complex128)


def harmonic_potential(prob: Problem, gammas=(1.0, 1.0, 1.0)) -> np.ndarray:
    """V = sum_a gamma_a^2 x_a^2 / 2 on the grid (float64, full array)."""
    X = mesh(prob)
    V = np.zeros(prob.shape)
    for a in range(prob.dim):
        V = V + 0.5 * (gammas[a] ** 2) * X[a] ** 2
    return np.ascontiguousarray(V, dtype=np.float64)


def pinned_centres(seed: int = SEED_PINS, count: int = 9, radius: float = 6.0) -> np.ndarray:
    """``count`` points drawn area-uniformly in the disc r < radius."""
    rng = np.random.default_rng(seed)
    r = radius * np.sqrt(rng.uniform(0.0, 1.0, count))
    t = rng.uniform(0.0, 2.0 * math.pi, count)
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=1)


def pinned_potential(prob: Problem, gamma_y: float, amp: float, centres: np.ndarray,
                     width: float = 0.5) -> np.ndarray:
    """V_theta = (x^2 + gamma_y^2 y^2)/2 + amp * sum_j exp(-|r - r_j|^2 / (2 width^2)) (2-D)."""
    if prob.dim != 2:
        raise ValueError("pinned potential is two-dimensional")
    x, y = mesh(prob)
    V = 0.5 * (x ** 2 + (gamma_y ** 2) * y ** 2)
    for cx, cy in centres:
        V = V + amp * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * width ** 2))
    return np.ascontiguousarray(V, dtype=np.float64)


def gaussian(prob: Problem, gammas=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Normalised exp(-sum gamma_a x_a^2 / 2): the harmonic-trap ground state at beta = 0."""
    X = mesh(prob)
    e = np.zeros(prob.shape)
    for a in range(prob.dim):
        e = e + 0.5 * gammas[a] * X[a] ** 2
    return _unit(np.exp(-e).astype(np.complex128), prob)


def noisy_gaussian_1d(prob: Problem, seed: int = SEED_1D, amp: float = 0.1) -> np.ndarray:
    """1-D start: G(x) (1 + amp xi), xi ~ U[-1, 1) real, normalised."""
    rng = np.random.default_rng(seed)
    (x,) = mesh(prob)
    xi = rng.uniform(-1.0, 1.0, prob.shape)
    return _unit(np.exp(-0.5 * x ** 2) * (1.0 + amp * xi), prob)


def vortex_seed_2d(prob: Problem, seed: int, radius: float = 4.0) -> np.ndarray:
    """2-D start: phi_a + e^{i chi} ((x - x0) + i (y - y0)) phi_a, with phi_a the unit Gaussian,
    chi ~ U[0, 2 pi) and (x0, y0) area-uniform in r < radius; normalised."""
    rng = np.random.default_rng(seed)
    chi = rng.uniform(0.0, 2.0 * math.pi)
    r0 = radius * math.sqrt(rng.uniform(0.0, 1.0))
    t0 = rng.uniform(0.0, 2.0 * math.pi)
    x0, y0 = r0 * math.cos(t0), r0 * math.sin(t0)
    x, y = mesh(prob)
    pa = np.exp(-0.5 * (x ** 2 + y ** 2)) / math.sqrt(math.pi)
    phi = pa + np.exp(1j * chi) * ((x - x0) + 1j * (y - y0)) * pa
    return _unit(phi, prob)


def noisy_gaussian_3d(prob: Problem, seed: int = SEED_3D, amp: float = 0.1) -> np.ndarray:
    """3-D start: exp(-(x^2 + y^2)/2 - z^2) (1 + amp (xi_r + i xi_i)), xi ~ U[-1, 1); normalised."""
    rng = np.random.default_rng(seed)
    x, y, z = mesh(prob)
    g = np.exp(-0.5 * (x ** 2 + y ** 2) - z ** 2)
    xr = rng.uniform(-1.0, 1.0, prob.shape)
    xi = rng.uniform(-1.0, 1.0, prob.shape)
    return _unit(g * (1.0 + amp * (xr + 1j * xi)), prob)


def random_field(prob: Problem, seed: int, envelope: float = 0.0) -> np.ndarray:
    """Complex field with U[-1,1) real and imaginary parts (times an optional Gaussian envelope
    exp(-envelope |x|^2)); normalised.  Used for operator parity at arbitrary inputs."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(-1.0, 1.0, prob.shape) + 1j * rng.uniform(-1.0, 1.0, prob.shape)
    if envelope > 0.0:
        r2 = sum(X ** 2 for X in mesh(prob))
        f = f * np.exp(-envelope * r2)
    return _unit(f, prob)


def paper_initial(prob: Problem, kind: str, omega: float = 0.0) -> np.ndarray:
    """The 2-D initial data (a), (b), (b2), (c), (c2), (d), (d2), (e), (e2) of the paper's
    initial-data experiment (Section 6.2): phi_a = e^{-(x^2+y^2)/2}/sqrt(pi), phi_b = (x+iy) phi_a,
    (c) the normalised mean of the two, (d) (1-Omega) phi_a + Omega phi_b, (e) Omega phi_a +
    (1-Omega) phi_b; a trailing 2 denotes the complex conjugate.  Returned normalised on the grid."""
    x, y = mesh(prob)
    pa = np.exp(-0.5 * (x ** 2 + y ** 2)) / math.sqrt(math.pi)
    pb = (x + 1j * y) * pa
    base = kind.rstrip("2")
    if base == "a":
        phi = pa + 0j
    elif base == "b":
        phi = pb
    elif base == "c":
        phi = 0.5 * (pa + pb)
    elif base == "d":
        phi = (1.0 - omega) * pa + omega * pb
    elif base == "e":
        phi = omega * pa + (1.0 - omega) * pb
    else:
        raise ValueError(f"unknown initial datum {kind!r}")
    if kind.endswith("2"):
        phi = np.conj(phi)
    return _unit(phi, prob)


# ----------------------------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------------------------

def lattice_potential(prob: Problem, gammas=(1.0, 1.0, 1.0), kappas=(25.0, 25.0, 25.0),
                      qs=(math.pi / 4, math.pi / 4, math.pi / 4)) -> np.ndarray:
    """Harmonic plus optical-lattice trap of the paper's numerical section:
    sum_a gamma_a^2 x_a^2 / 2 + kappa_a sin^2(q_a x_a) (reading: the harmonic part in the 1/2 form of
    the paper's harmonic examples, and the lattice term periodic in x_a)."""
    X = mesh(prob)
    V = np.zeros(prob.shape)
    for a in range(prob.dim):
        V = V + 0.5 * (gammas[a] ** 2) * X[a] ** 2 + kappas[a] * np.sin(qs[a] * X[a]) ** 2
    return np.ascontiguousarray(V, dtype=np.float64)


def quartic_potential(prob: Problem, alpha: float = 1.2, kappa: float = 0.3, gamma_z: float = 3.0) -> np.ndarray:
    """Harmonic plus quartic trap of the paper's numerical section (dim 2 or 3):
    (1 - alpha) (x^2 + y^2) / 2 + kappa (x^2 + y^2)^2 / 4 (+ gamma_z^2 z^2 / 2 in 3-D).  With
    alpha > 1 the quadratic part is repulsive and the quartic term confines, so rotations
    Omega > 1 remain bound."""
    if prob.dim < 2:
        raise ValueError("the quartic trap is defined for dim 2 and 3")
    X = mesh(prob)
    r2 = X[0] ** 2 + X[1] ** 2
    V = 0.5 * (1.0 - alpha) * r2 + 0.25 * kappa * r2 ** 2
    if prob.dim == 3:
        V = V + 0.5 * gamma_z ** 2 * X[2] ** 2
    return np.ascontiguousarray(np.broadcast_to(V, prob.shape), dtype=np.float64)


def thomas_fermi(prob: Problem, V: np.ndarray, gammas=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Thomas-Fermi initial data of the paper's numerical section: sqrt(max(mu - V, 0) / beta),
    normalised, with mu = (3 beta g_x)^{2/3} / 2 (1-D), (4 beta g_x g_y)^{1/2} / 2 (2-D),
    (15 beta g_x g_y g_z)^{2/5} / 2 (3-D) for trap frequencies g (the harmonic-trap formula the paper
    uses for every trap).  Needs beta > 0."""
    b = prob.beta
    if not b > 0.0:
        raise ValueError("Thomas-Fermi data needs beta > 0")
    g = gammas
    mu = {1: 0.5 * (3.0 * b * g[0]) ** (2.0 / 3.0), 2: 0.5 * (4.0 * b * g[0] * g[1]) ** 0.5,
          3: 0.5 * (15.0 * b * g[0] * g[1] * g[2]) ** 0.4}[prob.dim]
    phi = np.sqrt(np.maximum(mu - V, 0.0) / b).astype(np.complex128)
    return _unit(phi, prob)


def workload_quartic_2d(M: int = 512, omega: float = 2.0, beta: float = 1000.0, L: float = 20.0):
    """The paper's fast-rotation example in 2-D: harmonic plus quartic trap (alpha = 1.2,
    kappa = 0.3), Thomas-Fermi start, on [-L, L]^2 with M^2 points (the paper: L = 20, h = 1/16,
    i.e. M = 640)."""
    prob = Problem(2, (M, M), (L, L), beta, omega)
    V = quartic_potential(prob)
    return prob, V, thomas_fermi(prob, V)


def workload_1d():
    """1-D, V = x^2/2 on [-16, 16], 256 points, beta = 250, Omega = 0."""
    prob = Problem(1, (256,), (16.0,), 250.0, 0.0)
    return prob, harmonic_potential(prob), noisy_gaussian_1d(prob)


def workload_2d(M: int = 512, seed: int | None = None, beta: float = 1000.0, omega: float = 0.9):
    """2-D fast rotation, V = (x^2 + y^2)/2 on [-16, 16]^2, M x M points."""
    prob = Problem(2, (M, M), (16.0, 16.0), beta, omega)
    if seed is None:
        seed = SEED_2D_512 if M == 512 else SEED_2D_256
    return prob, harmonic_potential(prob), vortex_seed_2d(prob, seed)


def workload_2d_set(M: int = 512, seeds=SEEDS_2D_512_SET):
    """The 2-D fast-rotation problem with several seeded vortex-seed starts (same V, beta, Omega)."""
    prob, V, _ = workload_2d(M, seeds[0])
    return prob, V, [vortex_seed_2d(prob, s) for s in seeds]


def workload_3d(M: int = 128):
    """3-D rotation, V = (x^2 + y^2 + 4 z^2)/2 on [-8, 8]^3, M^3 points, beta = 5000, Omega = 0.8."""
    prob = Problem(3, (M, M, M), (8.0, 8.0, 8.0), 5000.0, 0.8)
    return prob, harmonic_potential(prob, (1.0, 1.0, 2.0)), noisy_gaussian_3d(prob)


def thomas_fermi_radius(beta: float, omega: float) -> float:
    """Thomas-Fermi radius of a 2-D harmonic trap softened by rotation, used to size boxes."""
    return (4.0 * beta / math.pi) ** 0.25 * (1.0 - omega ** 2) ** (-0.25)


@dataclass
class BatchInstance:
    prob: Problem
    V: np.ndarray
    phi0: np.ndarray
    seed: int


def batch_instances(count: int = 64, base_seed: int = SEED_BATCH_BASE, sizes=(128, 256, 512),
                    betas=(100.0, 500.0, 1000.0, 2000.0), omega_max: float = 0.95):
    """Independent 2-D instances: Omega ~ U[0, omega_max], beta ~ U{betas}, M ~ U{sizes},
    harmonic trap, half-width L = clamp(1.5 R_TF, 12, 20), vortex-seed start."""
    out = []
    for i in range(count):
        seed = base_seed + i
        rng = np.random.default_rng(seed)
        omega = float(rng.uniform(0.0, omega_max))
        beta = float(betas[int(rng.integers(0, len(betas)))])
        M = int(sizes[int(rng.integers(0, len(sizes)))])
        L = float(min(20.0, max(12.0, 1.5 * thomas_fermi_radius(beta, omega))))
        prob = Problem(2, (M, M), (L, L), beta, omega)
        out.append(BatchInstance(prob, harmonic_potential(prob), vortex_seed_2d(prob, seed + 10_000), seed))
    return out


def differentiation_workload(gamma_y: float = 1.05, amp: float = 2.0, M: int = 256):
    """2-D 256^2 on [-16, 16]^2, beta = 1000, Omega = 0.85, pinned potential with 9 centres."""
    prob = Problem(2, (M, M), (16.0, 16.0), 1000.0, 0.85)
    centres = pinned_centres()
    return prob, centres, pinned_potential(prob, gamma_y, amp, centres), vortex_seed_2d(prob, SEED_PINS)


def target_parameters(seed: int = SEED_THETA_TARGET):
    """theta' = (gamma_y', A') with gamma_y' ~ U[1.0, 1.1], A' ~ U[1.5, 2.5]."""
    rng = np.random.default_rng(seed)
    return float(rng.uniform(1.0, 1.1)), float(rng.uniform(1.5, 2.5))
