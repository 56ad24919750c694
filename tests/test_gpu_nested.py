"""GPU parity of the nested-grid path (the multigrid preparation of initial data, Section 6.2)
against the FP64 oracle, through the C ABI: the interpolation onto the doubled grid (gpe_prolong)
on every dimension and transform size, and ground states on nested grids
(gpe_pcg_solve_nested), single and batched, FP64 and mixed, up to the 512^2 workload."""
import numpy as np
import pytest

from conftest import assert_state
from gpe_inputs import Problem, harmonic_potential, paper_initial, random_field, workload_2d_set
from oracle import gpe_oracle as O

pytestmark = pytest.mark.gpu

SHAPES = [
    (1, (8,), (2.0,)),
    (1, (256,), (16.0,)),
    (1, (512,), (16.0,)),
    (2, (8, 8), (3.0, 3.0)),
    (2, (16, 64), (4.0, 6.0)),
    (2, (64, 16), (6.0, 4.0)),
    (2, (8, 512), (2.0, 12.0)),
    (2, (512, 8), (12.0, 2.0)),
    (2, (256, 256), (16.0, 16.0)),
    (2, (512, 512), (16.0, 16.0)),
    (3, (8, 8, 8), (3.0, 3.0, 3.0)),
    (3, (16, 32, 8), (4.0, 5.0, 3.0)),
    (3, (64, 64, 64), (8.0, 8.0, 8.0)),
    # 5 * 2^k points: 40 -> 80, 320 -> 640 (the paper's finest grid), mixed with powers of two
    (1, (40,), (4.0,)),
    (1, (320,), (16.0,)),
    (2, (320, 320), (20.0, 20.0)),
    (2, (40, 64), (4.0, 6.0)),
    (3, (40, 16, 80), (4.0, 3.0, 5.0)),
]
IDS = ["x".join(map(str, s[1])) for s in SHAPES]
TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_02045_amd import gpe
    gpe.lib()
    return torch


def _to(torch, x, dtype):
    real = {"f64": torch.float64, "f32": torch.float32}[dtype]
    cplx = {"f64": torch.complex128, "f32": torch.complex64}[dtype]
    t = torch.from_numpy(np.ascontiguousarray(x))
    return t.to(device="cuda", dtype=cplx if np.iscomplexobj(x) else real)


def _relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("dim,n,L", SHAPES, ids=IDS)
def test_prolong_matches_oracle(torch_gpu, dim, n, L, dtype):
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob = Problem(dim, n, L, 0.0, 0.0)
    f = random_field(prob, 9, envelope=0.5 / max(L) ** 2)
    print(f"prolong {dim}D n={n} {dtype}", flush=True)
    plan = gpe.Plan.from_problem(prob, dtype)
    fin = _to(torch, f, dtype)
    out = plan.prolong(fin).cpu().numpy()
    ref = O.prolong(prob, f)
    assert out.shape == ref.shape
    assert _relerr(out, ref) < TOL[dtype]
    # the coarse points are written from the input itself (bit-exact)
    even = out[tuple(slice(None, None, 2) for _ in range(dim))]
    assert np.array_equal(even, fin.cpu().numpy())


def test_prolong_rejects_bad_arguments(torch_gpu):
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob = Problem(2, (1024, 8), (8.0, 2.0), 0.0, 0.0)
    plan = gpe.Plan.from_problem(prob, "f64")
    f = torch.zeros(prob.shape, dtype=torch.complex128, device="cuda")
    with pytest.raises(gpe.GpeError) as e:
        plan.prolong(f, out=torch.empty((16, 2048), dtype=torch.complex128, device="cuda"))
    assert e.value.status == -2
    plan2 = gpe.Plan.from_problem(Problem(1, (16,), (2.0,), 0.0, 0.0), "f64")
    buf = torch.zeros(32, dtype=torch.complex128, device="cuda")
    with pytest.raises(gpe.GpeError) as e:  # out aliasing in
        gpe._check(gpe.lib().gpe_prolong(plan2._h, buf.data_ptr(), buf.data_ptr(), gpe._stream()))
    assert e.value.status == -1


def _levels(m0, nlev, L, beta, omega):
    probs = [Problem(2, (m0 << l, m0 << l), (L, L), beta, omega) for l in range(nlev)]
    return probs, [harmonic_potential(p) for p in probs]


@pytest.mark.parametrize("precision,tol_E", [("fp64", 1e-10), ("mixed", 1e-6)])
@pytest.mark.parametrize("coarsest", [16, 40])
def test_nested_solve_matches_oracle(torch_gpu, precision, tol_E, coarsest):
    """16^2 -> 32^2 -> 64^2 (and 40^2 -> 80^2 -> 160^2, the 5 * 2^k hierarchy of the paper's 640
    grids) at beta = 100, Omega = 0.4 from start (d): every level converges and the finest state has
    the oracle's nested-solve energy and density."""
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    probs, Vs = _levels(coarsest, 3, 8.0, 100.0, 0.4)
    start = paper_initial(probs[0], "d", 0.4)
    ref, ref_levels = O.pcg_nested(probs, Vs, start, tol_coarse=1e-6, tol_res=1e-9, max_iter=5000)
    assert ref.status == "converged"
    print(f"nested {precision} from {coarsest}^2", flush=True)
    st, outs, reps = gpe.pcg_solve_nested([probs[0]], [[_to(torch, V, "f64")] for V in Vs], [_to(torch, start, "f64")],
                                          "f64", tol_coarse=1e-6, tol=1e-9, max_iter=5000, precision=precision)
    assert st == 0
    assert [r[0]["status_name"] for r in reps] == ["ok"] * 3
    phi = outs[0].cpu().numpy()
    assert phi.shape == probs[-1].shape
    E = O.energy(probs[-1], Vs[-1], phi)
    assert abs(E - ref.E) / abs(ref.E) < tol_E
    assert abs(reps[-1][0]["E"] - ref.E) / abs(ref.E) < tol_E
    assert np.max(np.abs(np.abs(phi) ** 2 - np.abs(ref.phi) ** 2)) < (1e-7 if precision == "fp64" else 1e-4)


def test_nested_batched_equals_one_at_a_time(torch_gpu):
    """Three instances (different beta, Omega) solved together on nested grids end where each one
    solved alone ends (FP64)."""
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    cases = [(50.0, 0.0), (100.0, 0.3), (200.0, 0.5)]
    probs0, Vs_lv, starts = [], [[], [], []], []
    for beta, om in cases:
        probs, Vs = _levels(16, 3, 8.0, beta, om)
        probs0.append(probs[0])
        for l in range(3):
            Vs_lv[l].append(_to(torch, Vs[l], "f64"))
        starts.append(_to(torch, paper_initial(probs[0], "c", om), "f64"))
    st, outs, reps = gpe.pcg_solve_nested(probs0, Vs_lv, starts, "f64", tol_coarse=1e-6, tol=1e-9, max_iter=5000)
    assert st == 0
    for i in range(3):
        st1, out1, rep1 = gpe.pcg_solve_nested([probs0[i]], [[Vs_lv[l][i]] for l in range(3)], [starts[i]], "f64",
                                               tol_coarse=1e-6, tol=1e-9, max_iter=5000)
        assert abs(reps[-1][i]["E"] - rep1[-1][0]["E"]) < 1e-10 * abs(rep1[-1][0]["E"])
        assert reps[-1][i]["res_inf"] <= 1e-9


def test_nested_workload_512_reaches_tolerance(torch_gpu):
    """The 512^2, Omega = 0.9, beta = 1000 workload on nested grids 64^2 -> 512^2 from the bench's
    first two starts (generated on the coarsest grid), mixed precision: the oracle, re-evaluating the
    returned states, finds unit norm, ||r||_inf within FP64 rounding of 1e-8 and the
    reported energy and chemical potential."""
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob0, V0, starts = workload_2d_set(64)
    starts = starts[:2]
    probs, Vs = _levels(64, 4, prob0.L[0], prob0.beta, prob0.omega)
    assert np.allclose(Vs[0], V0)
    print("nested 512^2 mixed", flush=True)
    st, outs, reps = gpe.pcg_solve_nested([prob0] * 2, [[_to(torch, V, "f64")] * 2 for V in Vs],
                                          [_to(torch, s, "f64") for s in starts], "f64", tol_coarse=1e-6,
                                          tol=1e-8, max_iter=100000, precision="mixed")
    assert st == 0
    for i in range(2):
        phi = outs[i].cpu().numpy()
        assert_state(probs[-1], Vs[-1], phi, reps[-1][i], 1e-8, E_rel=1e-12)
