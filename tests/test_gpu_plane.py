"""GPU parity of the whole-plane H apply (one workgroup holds an xy-plane in LDS and applies both
directions of the Section 3 operator in one pass) against the FP64 oracle and against the
directional passes, through the C ABI, on seeded inputs: square and anisotropic planes, the largest
plane of each dtype (two rounds of rows per thread), 2-D and 3-D (the z pass after the planes, also
with 5 * 2^k points along z), single and batched fields, rotation and the cubic term on.  Which
kernel runs is forced through gpe_set_apply_kernel and checked with gpe_apply_kernel_for."""
import numpy as np
import pytest

from gpe_inputs import Problem, harmonic_potential, random_field
from oracle import gpe_oracle as O

pytestmark = pytest.mark.gpu

# (dim, n, L, dtypes)
PLANE_SHAPES = [
    (2, (32, 32), (4.0, 4.0), ("f64", "f32")),
    (2, (64, 64), (8.0, 8.0), ("f64", "f32")),
    (2, (128, 128), (12.0, 12.0), ("f32",)),  # the largest complex64 plane (147 KiB of LDS)
    (2, (128, 64), (10.0, 6.0), ("f64", "f32")),  # the largest complex128 planes
    (2, (64, 128), (6.0, 10.0), ("f64", "f32")),
    (2, (256, 64), (16.0, 6.0), ("f32",)),
    (2, (32, 256), (4.0, 16.0), ("f64", "f32")),
    (2, (256, 32), (16.0, 4.0), ("f64", "f32")),
    (3, (64, 64, 16), (8.0, 8.0, 3.0), ("f64", "f32")),
    (3, (128, 128, 8), (12.0, 12.0, 3.0), ("f32",)),
    (3, (32, 64, 40), (4.0, 6.0, 5.0), ("f64", "f32")),
]
CASES = [(d, n, L, t) for d, n, L, ts in PLANE_SHAPES for t in ts]
IDS = ["x".join(map(str, n)) + "-" + t for _, n, _, t in CASES]
TOL = {"f64": 2e-12, "f32": 2e-5}
# plane kernel vs passes: the same transforms and additions, possibly contracted into FMAs
# differently (and the passes take the run-time transform for 32-point lines), so they agree to a
# few units in the last place of the largest value
AGREE = {"f64": 1e-14, "f32": 5e-6}


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_02045_amd import gpe
    gpe.lib()  # fails loudly if the library is missing
    yield torch
    gpe.set_apply_kernel("auto")


def _setup(dim, n, L, beta=300.0, omega=0.7, seed=5):
    prob = Problem(dim, n, L, beta, omega)
    V = harmonic_potential(prob, (1.0, 1.3, 0.8))
    phi = random_field(prob, seed, envelope=0.5 / max(L) ** 2)
    return prob, V, phi


def _to(torch, x, dtype):
    real = {"f64": torch.float64, "f32": torch.float32}[dtype]
    cplx = {"f64": torch.complex128, "f32": torch.complex64}[dtype]
    t = torch.from_numpy(np.ascontiguousarray(x))
    return t.to(device="cuda", dtype=cplx if np.iscomplexobj(x) else real)


def _relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _apply(torch, plan, kind, phi, V, count=None):
    from paper_1611_02045_amd import gpe
    gpe.set_apply_kernel(kind)
    try:
        assert plan.apply_kernel_for(count or 1) == kind
        out = plan.apply_H_batched(phi, V) if count else plan.apply_H(phi, V)
        torch.cuda.synchronize()
    finally:
        gpe.set_apply_kernel("auto")
    return out


@pytest.mark.parametrize("dim,n,L,dtype", CASES, ids=IDS)
def test_plane_apply_matches_oracle_and_passes(torch_gpu, dim, n, L, dtype):
    """One field: the whole-plane kernel against the oracle's H phi, and against the directional
    passes to rounding."""
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob, V, phi = _setup(dim, n, L)
    print(f"plane apply {dim}D n={n} {dtype}", flush=True)
    plan = gpe.Plan.from_problem(prob, dtype)
    phi_d, V_d = _to(torch, phi, dtype), _to(torch, V, dtype)
    out_plane = _apply(torch, plan, "plane", phi_d, V_d)
    out_pass = _apply(torch, plan, "passes", phi_d, V_d)
    ref = O.hamiltonian(prob, V, phi)
    got, alt = out_plane.cpu().numpy(), out_pass.cpu().numpy()
    print(f"  vs oracle {_relerr(got, ref):.2e}, vs passes {_relerr(got, alt):.2e}, "
          f"{np.count_nonzero(got != alt)} of {got.size} values differ", flush=True)
    assert _relerr(got, ref) < TOL[dtype]
    assert _relerr(got, alt) < AGREE[dtype]


@pytest.mark.parametrize("dim,n,L,dtype,count", [
    (2, (64, 64), (8.0, 8.0), "f64", 5),
    (2, (128, 128), (12.0, 12.0), "f32", 7),
    (3, (64, 64, 16), (8.0, 8.0, 3.0), "f32", 3),
], ids=["64x64-f64-x5", "128x128-f32-x7", "64x64x16-f32-x3"])
def test_plane_apply_batched(torch_gpu, dim, n, L, dtype, count):
    """Batched fields (one workgroup per plane of every field, V shared): every field against the
    oracle, and the whole batch against the passes to rounding."""
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob, V, _ = _setup(dim, n, L)
    phis = [random_field(prob, 40 + k, envelope=0.5 / max(L) ** 2) for k in range(count)]
    print(f"plane apply batched {dim}D n={n} {dtype} x{count}", flush=True)
    plan = gpe.Plan.from_problem(prob, dtype)
    phi_d = torch.stack([_to(torch, p, dtype) for p in phis])
    V_d = _to(torch, V, dtype)
    out_plane = _apply(torch, plan, "plane", phi_d, V_d, count)
    out_pass = _apply(torch, plan, "passes", phi_d, V_d, count)
    got = out_plane.cpu().numpy()
    assert _relerr(got, out_pass.cpu().numpy()) < AGREE[dtype]
    for k in range(count):
        assert _relerr(got[k], O.hamiltonian(prob, V, phis[k])) < TOL[dtype], k


def test_plane_kernel_applicability(torch_gpu):
    """Where the whole-plane kernel runs: planes within its sizes and the LDS budget (128^2 in FP32,
    not in FP64; no 5 * 2^k axis in the plane; not 1-D), and never under "passes"."""
    from paper_1611_02045_amd import gpe
    cases = [
        ((2, (128, 128), (8.0, 8.0)), "f32", "plane"),
        ((2, (128, 128), (8.0, 8.0)), "f64", "passes"),
        ((2, (64, 64), (8.0, 8.0)), "f64", "plane"),
        ((2, (512, 512), (8.0, 8.0)), "f32", "passes"),
        ((2, (80, 40), (5.0, 4.0)), "f64", "passes"),
        ((2, (16, 64), (4.0, 6.0)), "f64", "passes"),
        ((3, (64, 64, 40), (8.0, 8.0, 5.0)), "f64", "plane"),
        ((1, (128,), (8.0,)), "f32", "passes"),
    ]
    try:
        for (dim, n, L), dtype, want in cases:
            plan = gpe.Plan.from_problem(Problem(dim, n, L, 100.0, 0.5 if dim > 1 else 0.0), dtype)
            gpe.set_apply_kernel("plane")
            assert plan.apply_kernel_for(4) == want, (n, dtype)
            gpe.set_apply_kernel("passes")
            assert plan.apply_kernel_for(4) == "passes", (n, dtype)
    finally:
        gpe.set_apply_kernel("auto")


def test_automatic_kernel_choice(torch_gpu):
    """The default choice: planes of up to 4096 points always take the plane kernel; larger ones
    (a CU per plane) only once a launch has a plane for every CU."""
    from paper_1611_02045_amd import gpe
    cus = torch_gpu.cuda.get_device_properties(0).multi_processor_count
    small = gpe.Plan.from_problem(Problem(2, (64, 64), (8.0, 8.0), 100.0, 0.5), "f64")
    big = gpe.Plan.from_problem(Problem(2, (128, 128), (8.0, 8.0), 100.0, 0.5), "f32")
    cube = gpe.Plan.from_problem(Problem(3, (128, 128, 128), (8.0, 8.0, 8.0), 100.0, 0.5), "f32")
    assert small.apply_kernel_for(1) == "plane"
    assert big.apply_kernel_for(1) == "passes"
    assert big.apply_kernel_for(cus - 1) == "passes"
    assert big.apply_kernel_for(cus) == "plane"
    assert cube.apply_kernel_for(1) == ("plane" if 128 >= cus else "passes")
    assert cube.apply_kernel_for(-(-cus // 128)) == "plane"


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_solvers_with_either_apply_kernel(torch_gpu, dtype):
    """The solvers' own H applies (L phi refreshes, the final FP64 check, the backward-Euler inner
    operator) run through whichever kernel is set: a 64^2 rotating problem solved by PCG and
    advanced by backward-Euler steps with the plane kernel and with the passes reaches the same
    state (energy and the oracle's residual) either way."""
    from paper_1611_02045_amd import gpe
    from conftest import residual_bound
    torch = torch_gpu
    prob = Problem(2, (64, 64), (8.0, 8.0), 200.0, 0.4)
    V = harmonic_potential(prob)
    phi0 = random_field(prob, 9, envelope=0.08)
    plan = gpe.Plan.from_problem(prob, dtype)
    tol = 1e-8 if dtype == "f64" else 1e-4
    out = {}
    try:
        for kind in ("plane", "passes"):
            gpe.set_apply_kernel(kind)
            assert plan.apply_kernel_for(1) == kind
            phi = _to(torch, phi0, dtype)
            rep = plan.pcg_solve(_to(torch, V, dtype), phi, tol=tol, max_iter=20000)
            assert rep["status"] == 0, (kind, rep)
            be = phi.clone()
            rb = plan.be_solve(_to(torch, V, dtype), be, 0.05, inner_tol=1e-10, tol=1e-300, max_iter=3)
            out[kind] = (rep, phi.cpu().numpy(), rb, be.cpu().numpy())
            print(f"  {kind}: {rep['iters']} iterations, E = {rep['E']:.12f}, BE E = {rb['E']:.12f}", flush=True)
    finally:
        gpe.set_apply_kernel("auto")
    (ra, pa, ba, bea), (rp, pp, bp, bep) = out["plane"], out["passes"]
    e_tol = 1e-9 if dtype == "f64" else 1e-5
    assert abs(ra["E"] - rp["E"]) < e_tol * abs(rp["E"])
    for rep, phi in ((ra, pa), (rp, pp)):
        r, lam = O.residual(prob, V, phi.astype(np.complex128) / O.norm(prob, phi.astype(np.complex128)))
        if dtype == "f64":
            assert float(np.max(np.abs(r))) <= residual_bound(tol)
        assert abs(lam - rep["lam"]) < (1e-9 if dtype == "f64" else 1e-4) * abs(lam)
    # three backward-Euler steps from each converged state stay at it (energies agree)
    assert abs(ba["E"] - bp["E"]) < e_tol * abs(bp["E"])
