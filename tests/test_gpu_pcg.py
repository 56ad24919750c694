"""GPU parity of the PG / PCG solver against the FP64 oracle through the C ABI.

Same seeded inputs on both sides; the GPU path's per-iteration record (energy, chemical potential,
residual, step) is compared with the oracle's for the first iterations, the final state is
compared in energy (1e-10 relative in FP64 mode, 1e-6 in mixed mode) and density, and the
closed-form ground state (beta = 0: E = d/2) pins the end-to-end path."""
import math

import numpy as np
import pytest

from conftest import assert_local_minima, assert_state
from gpe_inputs import (Problem, gaussian, harmonic_potential, noisy_gaussian_1d, paper_initial, random_field,
                        vortex_seed_2d)
from oracle import gpe_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_02045_amd import gpe
    gpe.lib()
    return torch


def _dev(torch, x, f64=True):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if np.iscomplexobj(x):
        return t.to("cuda", torch.complex128 if f64 else torch.complex64)
    return t.to("cuda", torch.float64 if f64 else torch.float32)


def _gpu_solve(torch, prob, V, phi0, dtype="f64", **opts):
    from paper_1611_02045_amd import gpe
    plan = gpe.Plan.from_problem(prob, dtype)
    phi = _dev(torch, phi0, dtype == "f64")
    rep = plan.pcg_solve(_dev(torch, V, dtype == "f64"), phi, **opts)
    hist = plan.history() if opts.get("record_history") else None
    return rep, phi.cpu().numpy().astype(np.complex128), hist


CASES = {
    "1d": (Problem(1, (256,), (16.0,), 250.0, 0.0), "1d"),
    "2d": (Problem(2, (64, 64), (8.0, 8.0), 100.0, 0.5), "2d"),
    "2d-aniso": (Problem(2, (64, 32), (8.0, 6.0), 60.0, 0.3), "2d"),
    "3d": (Problem(3, (16, 16, 16), (5.0, 5.0, 5.0), 40.0, 0.4), "3d"),
    # lines of 5 * 2^k points (radix-5 stage in every transform)
    "1d-640": (Problem(1, (640,), (16.0,), 250.0, 0.0), "1d"),
    "2d-80x40": (Problem(2, (80, 40), (8.0, 6.0), 100.0, 0.5), "2d"),
    "3d-40": (Problem(3, (40, 16, 40), (5.0, 5.0, 5.0), 40.0, 0.4), "3d"),
}


def _inputs(key):
    prob, kind = CASES[key]
    V = harmonic_potential(prob)
    if kind == "1d":
        phi0 = noisy_gaussian_1d(prob)
    elif kind == "2d":
        phi0 = vortex_seed_2d(prob, 7)
    else:
        phi0 = random_field(prob, 9, envelope=0.1)
    return prob, V, phi0


@pytest.mark.parametrize("key", list(CASES))
def test_trajectory_matches_oracle(torch_gpu, key):
    """First iterations: E_n, lambda_n, ||r_n||_inf and the accepted step agree with the oracle."""
    prob, V, phi0 = _inputs(key)
    print(f"trajectory {key}", flush=True)
    ref = O.pcg(prob, V, phi0, tol_res=1e-30, max_iter=12, record=True)
    rep, _, hist = _gpu_solve(torch_gpu, prob, V, phi0, tol_res=1e-30, max_iter=12, record_history=1,
                              check_every=4)
    assert rep["iters"] == 12 and rep["status"] == 1
    for h_ref, h in zip(ref.history, hist):
        assert int(h["n"]) == h_ref["n"]
        assert abs(h["E"] - h_ref["E"]) < 1e-11 * abs(h_ref["E"])
        assert abs(h["lam"] - h_ref["lam"]) < 1e-11 * abs(h_ref["lam"])
        assert abs(h["res"] - h_ref["res"]) < 1e-8 * h_ref["res"] + 1e-13
        if "theta" in h_ref:
            assert abs(h["theta"] - h_ref["theta"]) < 1e-7 * h_ref["theta"]
            assert int(h["restarted"]) == int(h_ref["restarted"])


@pytest.mark.parametrize("key", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_converged_state_matches_oracle(torch_gpu, key, precision):
    prob, V, phi0 = _inputs(key)
    tol = 1e-9
    print(f"solve {key} {precision}", flush=True)
    ref = O.pcg(prob, V, phi0, tol_res=tol, max_iter=3000)
    rep, phi, _ = _gpu_solve(torch_gpu, prob, V, phi0, tol_res=tol, max_iter=3000, precision=precision)
    assert ref.status == "converged"
    assert rep["status"] == 0, rep
    assert rep["res_inf"] <= tol
    rel = 1e-10 if precision == "fp64" else 1e-6
    assert abs(rep["E"] - ref.E) < rel * abs(ref.E)
    # the oracle's own evaluation of the GPU state
    assert abs(O.energy(prob, V, phi) - ref.E) < rel * abs(ref.E)
    gap = float(np.max(np.abs(np.abs(phi) ** 2 - np.abs(ref.phi) ** 2)))
    print(f"  iters gpu={rep['iters']} oracle={ref.iters} density Linf gap={gap:.3e}")
    assert gap < 1e-6


@pytest.mark.parametrize("method,precond", [("pg", "combined"), ("pcg", "kinetic"), ("pcg", "potential"),
                                            ("pcg", "none"), ("pcg", "c1"), ("pcg", "c2")])
def test_methods_and_preconditioners(torch_gpu, method, precond):
    prob, V, phi0 = _inputs("2d")
    print(f"method {method} {precond}", flush=True)
    ref = O.pcg(prob, V, phi0, method=method, precond=precond, tol_res=1e-30, max_iter=8, record=True)
    rep, _, hist = _gpu_solve(torch_gpu, prob, V, phi0, method=method, precond=precond, tol_res=1e-30,
                              max_iter=8, record_history=1)
    for h_ref, h in zip(ref.history, hist):
        assert abs(h["E"] - h_ref["E"]) < 1e-11 * abs(h_ref["E"])
        assert abs(h["res"] - h_ref["res"]) < 1e-8 * h_ref["res"]


@pytest.mark.parametrize("key", ["1d", "2d", "3d"])
@pytest.mark.parametrize("line_search,beta_rule", [("armijo", "pr"), ("full", "pr"), ("wolfe", "pr"),
                                                   ("heuristic", "fr"), ("full", "fr"), ("wolfe", "fr")])
def test_step_rules_trajectory_matches_oracle(torch_gpu, key, line_search, beta_rule):
    """The Armijo test, the full and the strong Wolfe line searches and the Fletcher-Reeves
    coefficient: the first iterations agree with the oracle's (energy, chemical potential,
    residual, accepted angle, halvings or evaluations)."""
    prob, V, phi0 = _inputs(key)
    print(f"step rules {key} {line_search} {beta_rule}", flush=True)
    ref = O.pcg(prob, V, phi0, tol_res=1e-30, max_iter=12, record=True, line_search=line_search,
                beta_rule=beta_rule)
    rep, _, hist = _gpu_solve(torch_gpu, prob, V, phi0, tol_res=1e-30, max_iter=12, record_history=1,
                              check_every=4, line_search=line_search, beta_rule=beta_rule)
    assert rep["iters"] == 12 and rep["status"] == 1
    assert len(hist) >= 12
    for h_ref, h in zip(ref.history, hist):
        assert abs(h["E"] - h_ref["E"]) < 1e-11 * abs(h_ref["E"])
        assert abs(h["lam"] - h_ref["lam"]) < 1e-11 * abs(h_ref["lam"])
        assert abs(h["res"] - h_ref["res"]) < 1e-8 * h_ref["res"] + 1e-13
        if "theta" in h_ref:
            assert abs(h["theta"] - h_ref["theta"]) < 1e-7 * h_ref["theta"]
            assert int(h["halvings"]) == h_ref["halvings"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("line_search", ["armijo", "full", "wolfe"])
def test_step_rules_converge_to_oracle_state(torch_gpu, precision, line_search):
    prob, V, phi0 = _inputs("2d")
    tol = 1e-9
    print(f"step rules solve {line_search} {precision}", flush=True)
    ref = O.pcg(prob, V, phi0, tol_res=tol, max_iter=3000, line_search=line_search)
    rep, phi, _ = _gpu_solve(torch_gpu, prob, V, phi0, tol_res=tol, max_iter=3000, precision=precision,
                             line_search=line_search)
    assert ref.status == "converged"
    assert rep["status"] == 0, rep
    rel = 1e-10 if precision == "fp64" else 1e-6
    assert abs(rep["E"] - ref.E) < rel * abs(ref.E)
    assert abs(O.energy(prob, V, phi) - ref.E) < rel * abs(ref.E)
    print(f"  iters gpu={rep['iters']} oracle={ref.iters}")


def test_beta0_gives_exact_ground_state(torch_gpu):
    """1-D harmonic trap, beta = 0, seeded noisy start: E = 1/2 to 1e-10."""
    prob = Problem(1, (256,), (16.0,), 0.0, 0.0)
    V = harmonic_potential(prob)
    rep, phi, _ = _gpu_solve(torch_gpu, prob, V, noisy_gaussian_1d(prob), tol_res=1e-10)
    assert rep["status"] == 0
    assert abs(rep["E"] - 0.5) < 1e-10
    g = gaussian(prob)
    ov = abs(O.inner(prob, g, phi))
    assert abs(ov - 1.0) < 1e-10


def test_2d_beta0_rotating_ground_state(torch_gpu):
    """2-D harmonic trap, beta = 0, Omega = 0.6: the minimum is E = 1 (m = 0 Gaussian)."""
    prob = Problem(2, (64, 64), (8.0, 8.0), 0.0, 0.6)
    V = harmonic_potential(prob)
    rep, _, _ = _gpu_solve(torch_gpu, prob, V, random_field(prob, 3, envelope=0.05), tol_res=1e-10)
    assert rep["status"] == 0 and abs(rep["E"] - 1.0) < 1e-10


def test_paper_sector_energy(torch_gpu):
    """Start (b) at Omega = 0.5, beta = 500 on 256^2: the printed 8.2606 = 8.7606 - Omega."""
    prob = Problem(2, (256, 256), (16.0, 16.0), 500.0, 0.5)
    V = harmonic_potential(prob)
    rep, _, _ = _gpu_solve(torch_gpu, prob, V, paper_initial(prob, "b", 0.5), tol_res=1e-7)
    assert rep["status"] == 0
    assert abs(rep["E"] - 8.2606) < 6e-5


def test_max_iter_reports_not_converged(torch_gpu):
    prob, V, phi0 = _inputs("2d")
    rep, _, _ = _gpu_solve(torch_gpu, prob, V, phi0, tol_res=1e-14, max_iter=5)
    assert rep["status"] == 1 and rep["iters"] == 5


def test_nonfinite_input_is_reported(torch_gpu):
    from paper_1611_02045_amd import gpe
    prob, V, phi0 = _inputs("2d")
    phi0 = phi0.copy()
    phi0[3, 5] = np.nan
    with pytest.raises(gpe.GpeError) as ei:
        _gpu_solve(torch_gpu, prob, V, phi0)
    assert ei.value.status == -4


def test_zero_start_is_reported_not_iterated(torch_gpu):
    """A start with no norm cannot be normalised: the solve ends with GPE_ENONFINITE at once (no
    iteration runs on the NaN field)."""
    from paper_1611_02045_amd import gpe
    prob, V, phi0 = _inputs("2d")
    print("zero start", flush=True)
    with pytest.raises(gpe.GpeError) as ei:
        _gpu_solve(torch_gpu, prob, V, np.zeros_like(phi0))
    assert ei.value.status == -4


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_start_at_the_ground_state_takes_no_iteration(torch_gpu, precision):
    """beta = 0, harmonic trap in 2-D: the Gaussian start is already the discrete ground state to
    spectral accuracy (E = 1/2 per axis), so in FP64 the convergence test passes at n = 0 and the
    field comes back unchanged; in mixed precision the start is rounded to FP32 first, and the FP64
    phase restores the state in a few iterations."""
    from gpe_inputs import gaussian
    prob = Problem(2, (64, 64), (8.0, 8.0), 0.0, 0.0)
    V = harmonic_potential(prob)
    phi0 = gaussian(prob)
    print(f"ground-state start {precision}", flush=True)
    rep, phi, _ = _gpu_solve(torch_gpu, prob, V, phi0, tol_res=1e-8, precision=precision)
    assert rep["status"] == 0
    assert abs(rep["E"] - 1.0) < 1e-10
    if precision == "fp64":
        assert rep["iters"] == 0
        np.testing.assert_allclose(phi, phi0, atol=1e-13)
    else:
        assert rep["iters"] <= 50
        np.testing.assert_allclose(np.abs(phi), np.abs(phi0), atol=1e-7)


def test_zero_max_iter_reports_the_start(torch_gpu):
    """max_iter = 0: no step is taken; the report carries the start's energy and residual."""
    prob, V, phi0 = _inputs("2d")
    print("max_iter 0", flush=True)
    rep, phi, _ = _gpu_solve(torch_gpu, prob, V, phi0, tol_res=1e-12, max_iter=0)
    assert rep["status"] == 1 and rep["iters"] == 0
    unit = phi0 / O.norm(prob, phi0)
    np.testing.assert_allclose(phi, unit, atol=1e-13)
    assert abs(rep["E"] - O.energy(prob, V, unit)) < 1e-11 * abs(rep["E"])
    r, _ = O.residual(prob, V, unit)
    assert abs(rep["res_inf"] - np.max(np.abs(r))) < 1e-9 * np.max(np.abs(r))


def test_trajectory_large_grid_collapsed_partials(torch_gpu):
    """1024^2 (512 partial rows per pass, reduced through the one-row collapse): the first
    iterations agree with the oracle."""
    prob = Problem(2, (1024, 1024), (16.0, 16.0), 500.0, 0.6)
    V = harmonic_potential(prob)
    phi0 = vortex_seed_2d(prob, 21)
    print("trajectory 1024^2", flush=True)
    ref = O.pcg(prob, V, phi0, tol_res=1e-30, max_iter=6, record=True)
    rep, _, hist = _gpu_solve(torch_gpu, prob, V, phi0, tol_res=1e-30, max_iter=6, record_history=1,
                              check_every=2)
    assert rep["iters"] == 6
    for h_ref, h in zip(ref.history, hist):
        assert abs(h["E"] - h_ref["E"]) < 1e-11 * abs(h_ref["E"])
        assert abs(h["res"] - h_ref["res"]) < 1e-8 * h_ref["res"]


@pytest.mark.timeout(600)
def test_3d_rotating_workload_mixed(torch_gpu):
    """3-D 128^3 on [-8,8]^3, V = (x^2 + y^2 + 4 z^2)/2, beta = 5000, Omega = 0.8, mixed precision to
    ||r||_inf <= 1e-8; the oracle re-evaluates the GPU state (energy and residual)."""
    from gpe_inputs import workload_3d
    prob, V, phi0 = workload_3d(128)
    print("3d 128^3 mixed solve", flush=True)
    rep, phi, _ = _gpu_solve(torch_gpu, prob, V, phi0, tol_res=1e-8, max_iter=100000, precision="mixed")
    print(f"  iters {rep['iters']} (fp32 {rep['iters_fp32']}), E = {rep['E']:.10f}, {rep['seconds']:.2f} s", flush=True)
    assert_state(prob, V, phi, rep, 1e-8, E_rel=1e-10)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_2d_256_workload(torch_gpu, precision):
    """2-D 256^2 on [-16,16]^2, V = r^2/2, beta = 1000, Omega = 0.9 from the seeded vortex-seed start
    (seed 102), to ||r||_inf <= 1e-8 in FP64 and in mixed precision.  The oracle re-evaluates the
    returned state (norm, residual, E, lambda), checks that it is a local minimum (second-order
    condition of Section 2), and that the oracle's own PCG started from it stays put."""
    from gpe_inputs import workload_2d
    prob, V, phi0 = workload_2d(256)
    print(f"2d 256^2 {precision} solve", flush=True)
    rep, phi, _ = _gpu_solve(torch_gpu, prob, V, phi0, tol_res=1e-8, max_iter=100000, precision=precision)
    print(f"  iters {rep['iters']} (fp32 {rep['iters_fp32']}), E = {rep['E']:.10f}", flush=True)
    E, _ = assert_state(prob, V, phi, rep, 1e-8)
    assert 6.35 < E < 6.37
    stay = O.pcg(prob, V, phi, tol_res=1e-8, max_iter=200)
    assert stay.status == "converged" and stay.iters <= 5 and abs(stay.E - E) <= 1e-12 * abs(E)
    assert_local_minima([(prob, V, phi)])


def test_trajectory_512_lines_single_and_batched(torch_gpu):
    """512^2 (lines of 512 points: the compile-time transform): the first iterations of a single
    solve (few workgroups: fields fetched early) and of three instances solved together (many
    workgroups: fields fetched late) agree with the oracle."""
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob = Problem(2, (512, 512), (16.0, 16.0), 1000.0, 0.9)
    V = harmonic_potential(prob)
    starts = [vortex_seed_2d(prob, s) for s in (103, 107, 109)]
    iters = 6
    print("trajectory 512^2", flush=True)
    refs = [O.pcg(prob, V, p0, tol_res=1e-30, max_iter=iters, record=True) for p0 in starts]
    rep, _, hist = _gpu_solve(torch, prob, V, starts[0], tol_res=1e-30, max_iter=iters, record_history=1,
                              check_every=2)
    assert rep["iters"] == iters
    for h_ref, h in zip(refs[0].history, hist):
        assert abs(h["E"] - h_ref["E"]) < 1e-11 * abs(h_ref["E"])
        assert abs(h["res"] - h_ref["res"]) < 1e-8 * h_ref["res"]
    Vd = _dev(torch, V)
    phis = [_dev(torch, p0) for p0 in starts]
    _, reps = gpe.pcg_solve_batched([prob] * 3, [Vd] * 3, phis, "f64", tol=1e-30, max_iter=iters)
    for r, ref in zip(reps, refs):
        assert r["status"] == 1 and r["iters"] == iters
        assert abs(r["E"] - ref.E) < 1e-11 * abs(ref.E)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("key", sorted(CASES))
def test_graph_replay_matches_eager_launches(torch_gpu, key, precision):
    """Chunks of iterations replayed from a captured HIP graph (with the solver's own host polls,
    drift refreshes and precision switch between the replays) give the very same trajectory as
    launching every kernel: identical iteration counts, energies and final fields, bit for bit."""
    prob, V, phi0 = _inputs(key)
    print(f"graph replay {key} {precision}", flush=True)
    runs = {}
    for g in (0, 1):
        runs[g] = _gpu_solve(torch_gpu, prob, V, phi0, tol=1e-10, max_iter=3000, precision=precision,
                             use_graph=g, refresh_every=48)
    (r0, f0, _), (r1, f1, _) = runs[0], runs[1]
    assert r0["status"] == 0 and r1["status"] == 0
    assert r0["iters"] == r1["iters"] and r0["iters_fp32"] == r1["iters_fp32"]
    assert r0["E"] == r1["E"]
    assert np.array_equal(f0, f1)


def test_graph_option_batched_matches_eager(torch_gpu):
    """The batched solve (two parts on two streams and threads, each capturing and replaying its own
    graph) gives identical per-instance results with the graph option on and off."""
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    probs, Vs, starts = [], [], []
    for i, (beta, om) in enumerate([(50.0, 0.2), (100.0, 0.5), (200.0, 0.6), (80.0, 0.0)]):
        p = Problem(2, (64, 64), (8.0, 8.0), beta, om)
        probs.append(p)
        Vs.append(_dev(torch, harmonic_potential(p)))
        starts.append(vortex_seed_2d(p, 11 + i))
    out = {}
    for g in (0, 1):
        phis = [_dev(torch, s) for s in starts]
        st, reps = gpe.pcg_solve_batched(probs, Vs, phis, "f64", tol=1e-10, max_iter=5000, precision="mixed",
                                         use_graph=g)
        assert st == 0
        out[g] = (reps, [p.cpu().numpy() for p in phis])
    for a, b in zip(out[0][0], out[1][0]):
        assert a["iters"] == b["iters"] and a["E"] == b["E"]
    for a, b in zip(out[0][1], out[1][1]):
        assert np.array_equal(a, b)
