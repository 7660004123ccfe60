"""GPU parity of the standard periodic FFT potential solver (the paper's
baseline, Sec. 3.1 Tables 1 and 4) against its oracle, the printed table
errors, and its exact invariant.

Bars: rel L-inf <= 1e-12 (FP64; FFT rounding only) and <= 1e-6 (FP32) against
the oracle on the same input; the printed errors of Tables 1 and 4 to their
three digits (FP64)."""
import math

import numpy as np
import pytest

from oracle import closed_forms as C
from oracle import periodic as OP
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_2014_amd as ps
    return ps


def rel_linf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("n", [16, 32, 128, 512, 2048, 4096])
@pytest.mark.parametrize("dtype,bar", [(torch.float64, 1e-12), (torch.float32, 1e-6)])
def test_periodic_solver_matches_oracle(ps, n, dtype, bar):
    print(f"case: periodic {n}^2 {dtype}", flush=True)
    half = 8.0
    rho = W.mixture_density(n, half, W.draw_mixture(20 + n % 97, 8, 4.0, (0.5, 1.5)))
    plan = ps.Plan(n, 2 * half / n, dtype=dtype, n_r=16, n_theta=32)
    r = torch.as_tensor(rho, dtype=dtype, device="cuda")
    got = plan.periodic(r).double().cpu().numpy()
    ref = OP.phi_periodic(r.double().cpu().numpy(), 2 * half / n)
    assert rel_linf(got, ref) <= bar
    plan.close()


def test_component_y_and_the_invariant(ps):
    print("case: periodic xx + yy", flush=True)
    n, half = 256, 8.0
    rho = W.mixture_density(n, half, W.draw_mixture(5, 8, 4.0, (0.5, 1.5)))
    r = torch.as_tensor(rho, dtype=torch.float64, device="cuda")
    px = ps.Plan(n, 2 * half / n, dtype=torch.float64, n_r=16, n_theta=32)
    py = ps.Plan(n, 2 * half / n, dtype=torch.float64, n_r=16, n_theta=32, component="y")
    fx = px.periodic(r).cpu().numpy()
    fy = py.periodic(r).cpu().numpy()
    assert rel_linf(fy, OP.phi_periodic(rho, 2 * half / n, "yy")) <= 1e-12
    assert np.max(np.abs(fx + fy + (rho - rho.mean()))) <= 1e-13 * rho.max()
    px.close()
    py.close()


@pytest.mark.parametrize("table,kind", [("table1_gaussian_periodic_fft.txt", "gaussian"),
                                        ("table4_arkadiev_periodic_fft.txt", "arkadiev")])
def test_printed_table_errors(ps, golden, table, kind):
    print(f"case: periodic {table}", flush=True)
    for half, h, printed in golden(table):
        n = int(round(2 * half / h))
        x, y, _ = W.grid_2d(n, half)
        if kind == "gaussian":
            rho = W.paper_gaussian_density(n, half)
            exact = C.phi_isotropic_gaussian(x, y, math.pi, math.pi ** 2)
        else:
            rho = W.arkadiev_density(n, half)
            exact = C.phi_arkadiev(x, y)
        plan = ps.Plan(n, h, dtype=torch.float64, n_r=16, n_theta=32)
        got = plan.periodic(torch.as_tensor(rho, dtype=torch.float64, device="cuda")).cpu().numpy()
        err = rel_linf(got, exact)
        assert abs(err - printed) <= 0.006 * printed, (half, h, err, printed)
        plan.close()


def test_periodic_argument_errors(ps):
    from paper_1409_2014_amd import _binding as B
    print("case: periodic argument errors", flush=True)
    plan = ps.Plan(8, 1.0, dtype=torch.float64, n_r=8, n_theta=16)
    with pytest.raises(B.PhiError, match="PHI_ERR_UNSUPPORTED"):
        plan.periodic(torch.zeros(8, 8, dtype=torch.float64, device="cuda"))
    plan.close()
    bp = ps.BatchPlan([dict(n=128, h=1 / 32), dict(n=256, h=1 / 32)], dtype=torch.float32)
    src = torch.zeros(bp.total, dtype=torch.float32, device="cuda")
    with pytest.raises(B.PhiError, match="PHI_ERR_UNSUPPORTED"):
        bp._call(B.lib().phi_solve_periodic, src, None)
    bp.close()


def test_periodic_graph_replay_matches_eager(ps):
    """The periodic solve captured into a HIP graph gives the eager result on
    every replay, with other eager work on the plan between replays."""
    print("case: periodic graph replay 1024^2 FP32", flush=True)
    n, half = 1024, 16.0
    rho = W.mixture_density(n, half, W.draw_mixture(21, 8, 6.0, (0.5, 1.5)))
    other = W.mixture_density(n, half, W.draw_mixture(22, 8, 6.0, (0.5, 1.5)))
    plan = ps.Plan(n, 2 * half / n, dtype=torch.float32, n_r=16, n_theta=32)
    r = torch.as_tensor(rho, dtype=torch.float32, device="cuda")
    o = torch.as_tensor(other, dtype=torch.float32, device="cuda")
    eager = plan.periodic(r).cpu().numpy()
    out = torch.empty_like(r)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.periodic(r, out)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.periodic(r, out)
    for rep in range(4):
        out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), f"replay {rep}"
        plan.periodic(o)
        plan.solve(o)
        torch.cuda.synchronize()
    plan.close()
