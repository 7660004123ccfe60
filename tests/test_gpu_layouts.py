"""The one-stream layout of a solve's middle part (cols_type2 and nodes in
their own launches, then the type-1 window columns and every I1 spectrum
column in one launch; the default on padded sides up to 1024 in both
precisions and 2048 in FP32) against the two-stream layout of separate
launches (PHI_TWO_STREAMS): bit-identical results, forward and transposed, on
padded sides from 16 to 4096 (where both flags give the two-stream layout the
test still checks the flag), for every multiplier, at exact and general grid
bounds, on repeated calls and under graph replay.  Both layouts also stay
within the solve's bars of the FP64 oracle (checked by the parity tests; here
one small case per layout closes the loop)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOLS = {torch.float64: 1e-12, torch.float32: 1e-7}


@pytest.fixture(scope="module")
def ps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_2014_amd as ps
    return ps


def density(n, half, seed):
    spec = W.draw_mixture(seed, 8, 0.375 * half, (0.5, 2.0))
    if half > 16:
        spec = W.MixtureSpec(spec.cx, spec.cy, spec.wx * half / 16, spec.wy * half / 16, spec.phase)
    return W.mixture_density(n, half, spec)


CASES = [(8, 4.0), (16, 4.0), (64, 8.0), (96, 4.0), (200, 8.0), (256, 8.0), (300, 8.0), (512, 8.0),
         (600, 12.0), (1024, 16.0), (2048, 16.0)]


@pytest.mark.parametrize("n,half", CASES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_default_layout_equals_two_streams(ps, n, half, dtype):
    print(f"case: default layout vs two streams N={n} {dtype}", flush=True)
    h = 2 * half / n
    rho = torch.as_tensor(density(n, half, 500 + n), dtype=dtype, device="cuda")
    plan = ps.Plan(n, h, dtype=dtype, tol=TOLS[dtype])
    split = ps.Plan(n, h, dtype=dtype, tol=TOLS[dtype], two_streams=True)
    a1 = plan.solve(rho)
    b1 = split.solve(rho)
    assert torch.equal(a1, b1)
    for _ in range(3):
        assert torch.equal(plan.solve(rho), a1)
    a2 = plan.solve_adjoint(a1)
    b2 = split.solve_adjoint(b1)
    assert torch.equal(a2, b2)
    plan.close()
    split.close()


@pytest.mark.parametrize("n,half", [(64, 8.0), (200, 8.0), (512, 8.0)])
@pytest.mark.parametrize("component", ["y", "xy", "coulomb"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_one_stream_layout_other_multipliers(ps, n, half, component, dtype):
    print(f"case: one-stream layout vs two streams N={n} {component} {dtype}", flush=True)
    h = 2 * half / n
    rho = torch.as_tensor(density(n, half, 41), dtype=dtype, device="cuda")
    a = ps.Plan(n, h, dtype=dtype, tol=TOLS[dtype], component=component)
    b = ps.Plan(n, h, dtype=dtype, tol=TOLS[dtype], component=component, two_streams=True)
    fa = a.solve(rho)
    assert torch.equal(fa, b.solve(rho))
    assert torch.equal(a.solve_adjoint(fa), b.solve_adjoint(fa))
    a.close()
    b.close()


@pytest.mark.parametrize("n,half", [(256, 8.0), (1024, 16.0)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_default_layout_under_graph_replay(ps, n, half, dtype):
    """Ten replays of a captured forward + transposed pair, with eager solves
    between them: every replay equals the eager result (the one-stream layout
    at 256^2, and at 1024^2 in FP32)."""
    h = 2 * half / n
    print(f"case: graph replay N={n} {dtype}", flush=True)
    plan = ps.Plan(n, h, dtype=dtype, tol=TOLS[dtype])
    rho = torch.as_tensor(density(n, half, 77), dtype=dtype, device="cuda")
    ref_f = plan.solve(rho)
    ref_b = plan.solve_adjoint(ref_f)
    out_f = torch.empty_like(rho)
    out_b = torch.empty_like(rho)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.solve(rho, out_f)
        plan.solve_adjoint(out_f, out_b)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.solve(rho, out_f)
        plan.solve_adjoint(out_f, out_b)
    for i in range(10):
        out_f.zero_()
        out_b.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out_f, ref_f), f"replay {i}"
        assert torch.equal(out_b, ref_b), f"replay {i}"
        assert torch.equal(plan.solve(rho), ref_f)
    plan.close()


@pytest.mark.parametrize("n,half", [(96, 4.0), (300, 8.0)])
def test_default_layout_matches_oracle(ps, n, half):
    h = 2 * half / n
    print(f"case: default layout vs oracle N={n} FP64", flush=True)
    rho = density(n, half, 9)
    plan = ps.Plan(n, h, dtype=torch.float64, tol=1e-12)
    got = plan.solve(torch.as_tensor(rho, device="cuda")).cpu().numpy()
    fine = plan.info["n_fine"]
    plan.close()
    ref = O.phi(rho, O.SplitParams(n=n, h=h, n_r=64, n_theta=128, pad_side=fine))
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,half,dtype,one_stream", [
    (64, 8.0, torch.float64, True), (256, 8.0, torch.float32, True), (512, 8.0, torch.float64, True),
    (1024, 16.0, torch.float32, True), (1024, 16.0, torch.float64, False), (2048, 16.0, torch.float32, False)])
def test_layout_choice_by_size(ps, n, half, dtype, one_stream):
    """The plan's layout, read off the kernels a timed solve reports: the
    one-stream layout on padded sides up to 1024 and on 2048 in FP32 (its last
    launch holds the type-1 window columns and the I1 columns), the two-stream
    layout beyond; PHI_TWO_STREAMS always gives the two-stream one."""
    print(f"case: layout choice N={n} {dtype}", flush=True)
    h = 2 * half / n
    rho = torch.as_tensor(density(n, half, 7), dtype=dtype, device="cuda")
    out = torch.empty_like(rho)
    plan = ps.Plan(n, h, dtype=dtype, tol=TOLS[dtype])
    names = [name for name, _ in plan.solve_timed(rho, out)]
    plan.close()
    expect = (["rows_forward", "cols_type2", "nodes", "type1_highfreq", "rows_inverse"] if one_stream else
              ["rows_forward", "cols_type2", "nodes", "cols_type1", "cols_highfreq", "rows_inverse"])
    assert sorted(names) == sorted(expect), names
    split = ps.Plan(n, h, dtype=dtype, tol=TOLS[dtype], two_streams=True)
    names = [name for name, _ in split.solve_timed(rho, out)]
    split.close()
    assert "type1_highfreq" not in names and "cols_highfreq" in names
