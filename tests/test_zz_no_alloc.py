"""gpe_apply_H_batched_noalloc (the batched H apply whose intermediate lives in the library's static
device scratch) against gpe_apply_H_batched (the same kernels with the plan's workspace), through
the C ABI: two calls in a row on each grid, the second with a smaller input, and a request beyond
the scratch size rejected before any launch."""
import numpy as np
import pytest

from gpe_inputs import Problem, harmonic_potential, random_field

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_02045_amd import gpe
    gpe.lib()
    return torch


def _fields(torch, prob, count, seed, dtype):
    ct = torch.complex128 if dtype == "f64" else torch.complex64
    rt = torch.float64 if dtype == "f64" else torch.float32
    phi = np.stack([random_field(prob, seed + k, envelope=0.05) for k in range(count)])
    return torch.from_numpy(phi).to("cuda", ct), torch.from_numpy(harmonic_potential(prob)).to("cuda", rt)


@pytest.mark.parametrize("prob,dtype,counts", [
    (Problem(2, (512, 512), (16.0, 16.0), 1000.0, 0.9), "f64", (8, 3)),
    (Problem(2, (512, 512), (16.0, 16.0), 1000.0, 0.9), "f32", (16, 5)),
    (Problem(3, (64, 64, 64), (8.0, 8.0, 8.0), 500.0, 0.6), "f64", (4, 1)),
    (Problem(1, (1024,), (16.0,), 250.0, 0.0), "f64", (32, 7)),
])
def test_noalloc_apply_equals_the_allocating_apply(torch_gpu, prob, dtype, counts):
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    plan = gpe.Plan.from_problem(prob, dtype)
    for call, count in enumerate(counts):
        print(f"noalloc apply {prob.shape} {dtype} count {count} (call {call + 1})", flush=True)
        phi, V = _fields(torch, prob, count, 50 + 10 * call, dtype)
        ref = plan.apply_H_batched(phi, V)
        out = torch.full_like(phi, float("nan"))
        plan.apply_H_batched_noalloc(phi, V, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


def test_noalloc_apply_rejects_a_batch_beyond_the_scratch(torch_gpu):
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob = Problem(2, (512, 512), (16.0, 16.0), 1000.0, 0.9)
    plan = gpe.Plan.from_problem(prob, "f64")
    count = 17  # 17 fields of 4 MiB: above the 64 MiB scratch
    phi = torch.zeros((count, 512, 512), dtype=torch.complex128, device="cuda")
    V = torch.zeros((512, 512), dtype=torch.float64, device="cuda")
    out = torch.full_like(phi, 7.0)
    with pytest.raises(gpe.GpeError) as ei:
        plan.apply_H_batched_noalloc(phi, V, out)
    assert ei.value.status == -1 and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())  # nothing was launched


def test_noalloc_apply_replayed_from_a_captured_graph(torch_gpu):
    """The callers the entry point is for: a batched apply captured into a graph (on a side
    stream) and replayed three times, with eager work and synchronisations between the replays;
    every replay equals the eager allocating apply."""
    from paper_1611_02045_amd import gpe
    torch = torch_gpu
    prob = Problem(2, (256, 256), (16.0, 16.0), 1000.0, 0.9)
    plan = gpe.Plan.from_problem(prob, "f64")
    phi, V = _fields(torch, prob, 4, 90, "f64")
    ref = plan.apply_H_batched(phi, V)
    out = torch.zeros_like(phi)
    plan.apply_H_batched_noalloc(phi, V, out)  # first call on the device outside the capture
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            plan.apply_H_batched_noalloc(phi, V, out, stream=side)
    torch.cuda.synchronize()
    for rep in range(3):
        out.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
        plan.apply_H_batched(phi, V)  # eager work between the replays
        torch.cuda.synchronize()
