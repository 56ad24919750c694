"""Pins of the oracle's implicit differentiation: the adjoint gradient of
l(theta) = E(phi*(theta)) + h^d sum (|phi*|^2 - rho_t)^2 against central finite differences of
full (warm-started) oracle solves, and algebraic properties of the projected Hessian."""
from dataclasses import replace

import numpy as np
import pytest

from gpe_inputs import Problem, mesh, pinned_centres, pinned_potential, vortex_seed_2d, random_field
from oracle import gpe_oracle as O


def _setup():
    prob = Problem(2, (32, 32), (7.0, 7.0), 60.0, 0.4)
    cent = pinned_centres(105, 3, 3.0)
    return prob, cent


def test_hessian_apply_matches_quadratic_form_and_is_symmetric():
    prob, cent = _setup()
    V = pinned_potential(prob, 1.05, 2.0, cent)
    phi = random_field(prob, 3, envelope=0.1)
    f, g = random_field(prob, 4, envelope=0.1), random_field(prob, 5, envelope=0.1)
    Hf, Hg = O.hessian_apply(prob, V, phi, f), O.hessian_apply(prob, V, phi, g)
    assert abs(O.inner(prob, f, Hf).real - O.hessian_form(prob, V, phi, f)) < 1e-12 * abs(O.hessian_form(prob, V, phi, f))
    # real-linear and self-adjoint in Re<.,.>
    assert abs(O.inner(prob, g, Hf).real - O.inner(prob, f, Hg).real) < 1e-11
    np.testing.assert_allclose(O.hessian_apply(prob, V, phi, 2.5 * f), 2.5 * Hf, atol=1e-12)


def test_gauge_direction_is_in_the_kernel_at_a_critical_point():
    """(1/2 nabla^2 E - lambda)(i phi*) = i (H phi* - lambda phi*) = 0 at a ground state."""
    prob, cent = _setup()
    V = pinned_potential(prob, 1.05, 2.0, cent)
    res = O.pcg(prob, V, vortex_seed_2d(prob, 5), tol_res=1e-12, max_iter=5000)
    lam = res.lam
    v = O.hessian_apply(prob, V, res.phi, 1j * res.phi) - lam * 1j * res.phi
    assert np.max(np.abs(v)) < 1e-10


def test_adjoint_gradient_matches_finite_differences():
    prob, cent = _setup()

    def Vof(gy, A):
        return pinned_potential(prob, gy, A, cent)

    gy, A = 1.05, 2.0
    V = Vof(gy, A)
    res = O.pcg(prob, V, vortex_seed_2d(prob, 5), tol_res=1e-12, max_iter=5000)
    assert res.status == "converged"
    rho_t = np.abs(O.pcg(prob, Vof(1.08, 1.7), res.phi, tol_res=1e-10).phi) ** 2
    x, y = mesh(prob)
    dVg = gy * y ** 2
    dVA = sum(np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * 0.25)) for cx, cy in cent)
    g = O.density_loss_gradient(prob, res.phi, rho_t)
    grad, _ = O.implicit_gradient(prob, V, res.phi, g, [dVg, dVA])

    def loss_at(gy_, A_, beta, om):
        pr = replace(prob, beta=beta, omega=om)
        V_ = Vof(gy_, A_)
        r = O.pcg(pr, V_, res.phi, tol_res=1e-12, max_iter=5000)
        return O.energy(pr, V_, r.phi) + O.density_loss(pr, r.phi, rho_t)

    d = 1e-4
    fd = np.array([
        (loss_at(gy * (1 + d), A, 60, .4) - loss_at(gy * (1 - d), A, 60, .4)) / (2 * d * gy),
        (loss_at(gy, A * (1 + d), 60, .4) - loss_at(gy, A * (1 - d), 60, .4)) / (2 * d * A),
        (loss_at(gy, A, 60 * (1 + d), .4) - loss_at(gy, A, 60 * (1 - d), .4)) / (2 * d * 60),
        (loss_at(gy, A, 60, .4 * (1 + d)) - loss_at(gy, A, 60, .4 * (1 - d))) / (2 * d * .4),
    ])
    np.testing.assert_allclose(grad, fd, rtol=1e-6)
