import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")


def load_table(name):
    """Rows of a whitespace table under tests/golden (comment lines start with '#')."""
    path = os.path.join(ROOT, "tests", "golden", name)
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return rows


def residual_bound(tol):
    """Largest oracle-evaluated ||r||_inf accepted for a state the library reports at ||r||_inf <= tol:
    the two FP64 evaluations of the same residual differ only by rounding (about 1e-13 here)."""
    return tol * (1.0 + 1e-9) + 1e-12


def assert_state(prob, V, phi, rep, tol, *, E_rel=1e-11, lam_rel=1e-10):
    """A state the library returned as converged: the report keeps its contract (status OK means
    the fresh residual meets tol), and the oracle's FP64 re-evaluation of the returned field gives
    unit norm, ||r||_inf within FP64 rounding of tol, and the reported E and lambda."""
    import numpy as np
    from oracle import gpe_oracle as O
    assert rep["status"] == 0 and rep["res_inf"] <= tol, rep
    assert abs(O.norm(prob, phi) - 1.0) < 1e-12
    r, lam = O.residual(prob, V, phi)
    assert float(np.max(np.abs(r))) <= residual_bound(tol)
    E = O.energy(prob, V, phi)
    assert abs(E - rep["E"]) < E_rel * abs(E)
    assert abs(lam - rep["lam"]) < lam_rel * abs(lam)
    return E, lam


# Grids up to this many points run the second-order check to convergence; larger ones for a fixed
# number of Lanczos steps (the CG run of the check), enough to expose a negative curvature of
# size ~1e-4 of the preconditioned operator's largest eigenvalue, or larger.
FULL_CHECK_POINTS = 256 * 256
CHECK_BUDGET = 500
# Curvatures (of (1/2) nabla^2 E - lambda on unit tangent vectors) above -FLAT_CURVATURE count as
# flat.  At ||r||_inf <= 1e-8 on these boxes (area <= 1600) the energy's slope along a unit tangent
# direction is up to 2 ||r||_2 <= 8e-7, so a curvature of -1e-9 cannot lower E by more than ~1e-9 over
# any move on the sphere:
# such a direction is the flat valley of a degenerate family of minima (rotations of a lattice in
# an isotropic trap, curvature ~1e-11 of either sign), not a saddle, whose unstable curvatures
# are many orders larger (-1e-4 and below).
FLAT_CURVATURE = 1e-9


def _second_order_job(args):
    prob, V, phi, seed, tol, max_iter = args
    import time
    from gpe_inputs import random_field
    from oracle import gpe_oracle as O
    t0 = time.time()
    rhs = random_field(prob, seed, envelope=1.0 / prob.L[0] ** 2)
    shape = prob.n[:prob.dim]

    def progress(k, rel):
        print(f"  second-order check {shape}: step {k}, rel. residual {rel:.1e}", flush=True)

    chk = O.second_order_check(prob, V, phi, rhs, tol=tol, max_iter=max_iter, shift=FLAT_CURVATURE,
                               progress=progress)
    chk.direction = None
    print(f"  second-order check {prob.n[:prob.dim]}: {chk.iters} CG steps in {time.time() - t0:.0f} s", flush=True)
    return chk


def second_order_checks(items, *, tol=1e-6, workers=8):
    """The oracle's second-order (local minimum) check of Section 2 for each (prob, V, phi), run
    in parallel worker processes (each only uses numpy); returns the CurvatureCheck results."""
    import concurrent.futures as cf
    import multiprocessing as mp
    jobs = [(prob, V, phi, 700 + k, tol, 8000 if prob.size <= FULL_CHECK_POINTS else CHECK_BUDGET)
            for k, (prob, V, phi) in enumerate(items)]
    if len(jobs) == 1:
        return [_second_order_job(jobs[0])]
    # one thread per worker: the oracle's small BLAS calls (inner products) slow down by an order
    # of magnitude when several processes each start a full thread pool
    import os
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    os.environ.update({k: "1" for k in keys})
    try:
        with cf.ProcessPoolExecutor(max_workers=min(workers, len(jobs)), mp_context=mp.get_context("spawn")) as ex:
            return list(ex.map(_second_order_job, jobs))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def assert_local_minima(items, *, tol=1e-6):
    """Every state of items passes the second-order check of Section 2: CG on the projected
    Hessian shifted by FLAT_CURVATURE meets positive curvature only and its smallest Ritz value is
    positive (no tangent curvature below -FLAT_CURVATURE); on grids up to
    FULL_CHECK_POINTS points the run also converges (every eigen-component of a random right-hand
    side resolved), on larger ones it runs CHECK_BUDGET steps."""
    for (prob, _, _), chk in zip(items, second_order_checks(items, tol=tol)):
        print(f"  {prob.n[:prob.dim]}: min Ritz {chk.min_ritz:.3e}, max {chk.max_ritz:.3e}, {chk.iters} steps, "
              f"rel. residual {chk.rel_res:.1e}", flush=True)
        assert not chk.negative, chk.rayleigh
        assert chk.min_ritz > 0.0
        if prob.size <= FULL_CHECK_POINTS:
            assert chk.rel_res <= tol
