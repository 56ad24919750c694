"""GPU parity of the operators (H apply, energy, preconditioners) against the FP64 oracle, through
the C ABI, on seeded inputs: shapes cover every supported dimension, anisotropic grids, several
lines per workgroup and the smallest/largest transform sizes."""
import math

import numpy as np
import pytest

from gpe_inputs import Problem, harmonic_potential, random_field
from oracle import gpe_oracle as O

pytestmark = pytest.mark.gpu

SHAPES = [
    (1, (8,), (2.0,)),
    (1, (256,), (16.0,)),
    (1, (1024,), (20.0,)),
    (1, (512,), (16.0,)),
    (2, (8, 8), (3.0, 3.0)),
    (2, (16, 64), (4.0, 6.0)),
    (2, (64, 16), (6.0, 4.0)),
    (2, (8, 1024), (2.0, 12.0)),
    (2, (1024, 8), (12.0, 2.0)),
    (2, (256, 256), (16.0, 16.0)),
    (2, (512, 512), (16.0, 16.0)),
    (2, (512, 32), (16.0, 6.0)),
    (2, (32, 512), (6.0, 16.0)),
    (3, (8, 8, 8), (3.0, 3.0, 3.0)),
    (3, (16, 32, 8), (4.0, 5.0, 3.0)),
    (3, (64, 64, 64), (8.0, 8.0, 8.0)),
    # lines of 5 * 2^k points (radix-5 stage): smallest, largest, mixed with powers of two
    (1, (40,), (4.0,)),
    (1, (640,), (20.0,)),
    (2, (640, 640), (20.0, 20.0)),
    (2, (80, 40), (5.0, 4.0)),
    (2, (640, 32), (16.0, 6.0)),
    (2, (32, 640), (6.0, 16.0)),
    (2, (512, 160), (16.0, 8.0)),
    (3, (40, 80, 40), (4.0, 5.0, 4.0)),
    (3, (160, 16, 320), (8.0, 3.0, 10.0)),
]
IDS = ["x".join(map(str, s[1])) for s in SHAPES]
TOL = {"f64": 2e-12, "f32": 2e-5}


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_02045_amd import gpe  # noqa: F401  (fails loudly if the library is missing)
    gpe.lib()
    return torch


def _setup(dim, n, L, beta=300.0, omega=0.7, seed=5):
    prob = Problem(dim, n, L, beta, omega if dim > 1 else 0.0)
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


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("dim,n,L", SHAPES, ids=IDS)
def test_apply_H_matches_oracle(torch_gpu, dim, n, L, dtype):
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob, V, phi = _setup(dim, n, L)
    print(f"apply_H {dim}D n={n} {dtype}", flush=True)
    ref = O.hamiltonian(prob, V, phi)
    plan = gpe.Plan.from_problem(prob, dtype)
    out = plan.apply_H(_to(torch, phi, dtype), _to(torch, V, dtype)).cpu().numpy()
    assert _relerr(out, ref) < TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("dim,n,L", SHAPES, ids=IDS)
def test_energy_matches_oracle(torch_gpu, dim, n, L, dtype):
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob, V, phi = _setup(dim, n, L)
    print(f"energy {dim}D n={n} {dtype}", flush=True)
    ref = O.energy_parts(prob, V, phi)
    plan = gpe.Plan.from_problem(prob, dtype)
    E, parts = plan.energy(_to(torch, phi, dtype), _to(torch, V, dtype), parts=True)
    scale = abs(ref.kinetic) + abs(ref.potential) + abs(ref.interaction) + abs(ref.rotation)
    assert abs(E - ref.total) < TOL[dtype] * scale
    for key, val in (("kinetic", ref.kinetic), ("potential", ref.potential), ("interaction", ref.interaction),
                     ("rotation", ref.rotation)):
        assert abs(parts[key] - val) < TOL[dtype] * scale, key


PRECOND_SHAPES = {"1d": (1, (256,), (16.0,)), "2d-aniso": (2, (16, 64), (4.0, 6.0)), "2d": (2, (256, 256), (16.0, 16.0)),
                  "2d-512x": (2, (512, 32), (16.0, 6.0)), "2d-512y": (2, (32, 512), (6.0, 16.0)),
                  "3d": (3, (16, 32, 8), (4.0, 5.0, 3.0)), "2d-640": (2, (640, 640), (20.0, 20.0)),
                  "2d-5x": (2, (80, 40), (5.0, 4.0)), "3d-5": (3, (40, 80, 40), (4.0, 5.0, 4.0))}


@pytest.mark.parametrize("kind", ["none", "kinetic", "potential", "combined", "c1", "c2"])
@pytest.mark.parametrize("dim,n,L", list(PRECOND_SHAPES.values()), ids=list(PRECOND_SHAPES))
def test_preconditioners_match_oracle(torch_gpu, dim, n, L, kind):
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob, V, phi = _setup(dim, n, L)
    r = random_field(prob, 77)
    print(f"precond {kind} {dim}D n={n}", flush=True)
    plan = gpe.Plan.from_problem(prob, "f64")
    P, Vg, R = _to(torch, phi, "f64"), _to(torch, V, "f64"), _to(torch, r, "f64")
    # adaptive shift lambda~ computed on the device
    ref = O.apply_preconditioner(prob, kind, V, phi, r)
    out = plan.precond(kind, P, Vg, R).cpu().numpy()
    assert _relerr(out, ref) < 1e-12
    # explicit shift
    ref = O.apply_preconditioner(prob, kind, V, phi, r, alpha=2.5)
    out = plan.precond(kind, P, Vg, R, alpha=2.5).cpu().numpy()
    assert _relerr(out, ref) < 1e-12


def test_preconditioner_rejects_non_spd(torch_gpu):
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob, V, phi = _setup(2, (16, 16), (4.0, 4.0))
    plan = gpe.Plan.from_problem(prob, "f64")
    with pytest.raises(gpe.GpeError) as ei:
        plan.precond("combined", _to(torch, phi, "f64"), _to(torch, V - 1e3, "f64"), _to(torch, phi, "f64"), alpha=1.0)
    assert ei.value.status == -1
    with pytest.raises(gpe.GpeError):
        plan.precond("kinetic", _to(torch, phi, "f64"), _to(torch, V, "f64"), _to(torch, phi, "f64"), alpha=-1.0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_apply_H_batched(torch_gpu, dtype):
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob, V, _ = _setup(2, (128, 64), (10.0, 8.0))
    phis = np.stack([random_field(prob, s, envelope=0.01) for s in range(5)])
    plan = gpe.Plan.from_problem(prob, dtype)
    out = plan.apply_H_batched(_to(torch, phis, dtype), _to(torch, V, dtype)).cpu().numpy()
    for b in range(5):
        assert _relerr(out[b], O.hamiltonian(prob, V, phis[b])) < TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_apply_H_batch32_at_512(torch_gpu, dtype):
    """The bench's apply configuration: 32 fields of 512^2 (Omega = 0.9, beta = 1000) in one batched
    apply; sampled instances (first, middle, last) against the oracle."""
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob = Problem(2, (512, 512), (16.0, 16.0), 1000.0, 0.9)
    V = harmonic_potential(prob)
    base = random_field(prob, 21, envelope=0.02)
    phis = np.stack([base * (1.0 + 0.01 * k) * np.exp(0.1j * k) for k in range(32)])
    print(f"apply batch 32 at 512^2 {dtype}", flush=True)
    plan = gpe.Plan.from_problem(prob, dtype)
    out = plan.apply_H_batched(_to(torch, phis, dtype), _to(torch, V, dtype)).cpu().numpy()
    for b in (0, 15, 31):
        assert _relerr(out[b], O.hamiltonian(prob, V, phis[b])) < TOL[dtype]


def test_apply_H_beyond_the_mall(torch_gpu):
    """The bench's above-MALL apply configuration: 64 FP32 fields of 512^2 in one batched apply
    (phi, H phi and the intermediate: 384 MiB); sampled instances (first, middle, last) against the
    oracle."""
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob = Problem(2, (512, 512), (16.0, 16.0), 1000.0, 0.9)
    V = harmonic_potential(prob)
    base = random_field(prob, 23, envelope=0.02)
    print("apply batch 64 at 512^2 f32", flush=True)
    phis = torch.stack([_to(torch, base * (1.0 + 0.01 * k) * np.exp(0.1j * k), "f32") for k in range(64)])
    plan = gpe.Plan.from_problem(prob, "f32")
    out = plan.apply_H_batched(phis, _to(torch, V, "f32"))
    for b in (0, 31, 63):
        ref = O.hamiltonian(prob, V, phis[b].cpu().numpy().astype(np.complex128))
        assert _relerr(out[b].cpu().numpy(), ref) < TOL["f32"]


def test_energy_grad(torch_gpu):
    """grad_phi = 2 h^d H phi, grad_V = h^d |phi|^2, dE/dbeta, dE/domega against the oracle."""
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob, V, phi = _setup(2, (64, 32), (6.0, 5.0))
    plan = gpe.Plan.from_problem(prob, "f64")
    gphi, gV, db, do = plan.energy_grad(_to(torch, phi, "f64"), _to(torch, V, "f64"))
    w = O.cell(prob)
    assert _relerr(gphi.cpu().numpy(), 2 * w * O.hamiltonian(prob, V, phi)) < 1e-12
    assert _relerr(gV.cpu().numpy(), w * np.abs(phi) ** 2) < 1e-14
    assert abs(db - 0.5 * w * np.sum(np.abs(phi) ** 4)) < 1e-12 * abs(db)
    lz = O.inner(prob, phi, O.angular_momentum(prob, phi)).real
    assert abs(do + lz) < 1e-12 * max(1.0, abs(lz))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_apply_H_replayed_from_a_captured_graph(torch_gpu, dtype):
    """The H apply captured into a graph (after an eager call sized the plan's scratch) and replayed
    three times, with other eager applies and synchronisations between the replays: every replay
    gives the eager result bit for bit (the graph holds kernel nodes only)."""
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob, V, phi = _setup(2, (64, 128), (6.0, 8.0))
    plan = gpe.Plan.from_problem(prob, dtype)
    f, Vd = _to(torch, phi, dtype), _to(torch, V, dtype)
    other = _to(torch, random_field(prob, 77, envelope=0.02), dtype)
    ref = plan.apply_H(f, Vd)
    out = torch.empty_like(f)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            plan.apply_H(f, Vd, out, stream=side)
    torch.cuda.synchronize()
    for k in range(3):
        out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {k}"
        plan.apply_H(other, Vd)  # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_autotuned_tiles_keep_parity(torch_gpu, dtype):
    """After tile measurement on a grid, every pass launches with the recorded tiles: the H apply
    and a full solve still match the oracle."""
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob, V, phi = _setup(2, (128, 64), (8.0, 6.0))
    plan = gpe.Plan.from_problem(prob, dtype)
    tiles, us = plan.autotune(1)
    print(f"tiles {tiles} us {us}", flush=True)
    assert all(t >= 1 for t in tiles) and all(u > 0.0 for u in us)
    out = plan.apply_H(_to(torch, phi, dtype), _to(torch, V, dtype)).cpu().numpy()
    ref = O.hamiltonian(prob, V, phi)
    assert _relerr(out, ref) < TOL[dtype]
    if dtype == "f64":
        ph = _to(torch, phi, dtype)
        rep = plan.pcg_solve(_to(torch, V, dtype), ph, tol=1e-9, max_iter=5000)
        assert rep["status"] == 0
        E = O.energy(prob, V, ph.cpu().numpy())
        assert abs(E - rep["E"]) < 1e-12 * abs(E)
