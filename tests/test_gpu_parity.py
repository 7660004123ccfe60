"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Bars: rel L-inf and L2 <= 1e-10 (FP64 data path) and
<= 1e-6 (FP32 data path, oracle run on the FP32-rounded input promoted to
FP64); each NUFFT stage alone within 10x its tolerance in relative l2, on a
smooth density and on white noise."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel_linf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def ps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_2014_amd as ps
    return ps


def to_dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def run_solve(ps, rho64, n, h, dtype, **kw):
    plan = ps.Plan(n, h, dtype=dtype, **kw)
    rho_dev = to_dev(rho64, dtype)
    out = plan.solve(rho_dev)
    torch.cuda.synchronize()
    rho_used = rho_dev.double().cpu().numpy()
    return plan, rho_used, out.double().cpu().numpy()


# --------------------------------------------------------------------------
# the small FP64 case: 64 x 64 over [-8, 8)^2, exp(-r^2), 32 x 64 nodes, tol 1e-12
# --------------------------------------------------------------------------

def test_small_gaussian_fp64_matches_oracle(ps):
    print("case: 64x64 Gaussian FP64", flush=True)
    rho = W.gaussian_density(64, 8.0)
    plan, rho_used, got = run_solve(ps, rho, 64, 0.25, torch.float64, n_r=32, n_theta=64, tol=1e-12)
    ref = O.phi(rho_used, O.SplitParams(n=64, h=0.25, n_r=32, n_theta=64))
    assert rel_linf(got, ref) <= 1e-10
    assert rel_l2(got, ref) <= 1e-10


def test_highfreq_and_lowfreq_parts_fp64(ps):
    print("case: parts 128x128 mixture FP64", flush=True)
    n, half = 128, 8.0
    rho = W.mixture_density(n, half, W.draw_mixture(3, 8, 4.0, (0.5, 1.5)))
    plan = ps.Plan(n, 2 * half / n, dtype=torch.float64, tol=1e-12)
    r = to_dev(rho, torch.float64)
    i1 = plan.highfreq(r).cpu().numpy()
    i2 = plan.lowfreq(r).cpu().numpy()
    parts = O.phi_parts(rho, O.SplitParams(n=n, h=2 * half / n, n_r=64, n_theta=128))
    scale = np.max(np.abs(parts["phi"]))
    # I1 is an exact FFT chain: rounding only
    assert np.max(np.abs(i1 - parts["i1"])) <= 1e-13 * scale
    assert np.max(np.abs(i2 - parts["i2"])) <= 1e-11 * scale


# Stage bars: 10 tol in relative l2 (the NUFFT tolerance is a relative l2 target
# for each transform), on two inputs.  "smooth": the mixture density of the
# workloads (for type 1: the coefficients a_j = q_j rho_hat_j of that density,
# the values the solve spreads).  "noise": independent standard normal grid
# values (type 2) or coefficients (type 1).  Measured on MI355X: FP32 at tol
# 1e-7 gives 0.5e-7 .. 3e-7 (smooth) and 2.4e-7 .. 4.3e-7 (noise); FP64 at tol
# 1e-12 stays below 2.6e-12.
STAGE_CASES = [(torch.float64, 1e-12, "smooth", 1e-11), (torch.float64, 1e-12, "noise", 1e-11),
               (torch.float64, 1e-6, "noise", 1e-5), (torch.float32, 1e-7, "smooth", 1e-6),
               (torch.float32, 1e-7, "noise", 1e-6)]


def stage_density(kind, n, half):
    if kind == "noise":
        return np.random.default_rng(21).standard_normal((n, n))
    return W.mixture_density(n, half, W.draw_mixture(23, 8, 0.375 * half, (0.5, 2.0)))


@pytest.mark.parametrize("kernel", ["es", "gaussian"])
@pytest.mark.parametrize("dtype,tol,kind,bar", STAGE_CASES)
def test_type2_stage_against_direct_sums(ps, dtype, tol, kind, bar, kernel):
    print(f"case: type2 {dtype} tol={tol} {kind} kernel={kernel}", flush=True)
    n, half = 256, 8.0
    rho = stage_density(kind, n, half)
    plan = ps.Plan(n, 2 * half / n, dtype=dtype, tol=tol, kernel=kernel)
    r = to_dev(rho, dtype)
    got = plan.type2(r).cpu().numpy().astype(np.complex128)
    kx, ky, _ = plan.nodes()
    ref = O.type2_direct(r.double().cpu().numpy(), 2 * half / n, O.grid_points(O.SplitParams(n, 2 * half / n, 1, 2)),
                         kx, ky)
    err = rel_l2(got, ref)
    print(f"  rel l2 {err:.3e} (bar {bar:.0e})", flush=True)
    assert err <= bar


@pytest.mark.parametrize("kernel", ["es", "gaussian"])
@pytest.mark.parametrize("dtype,tol,kind,bar", [c for c in STAGE_CASES if c[1] != 1e-6])
def test_type1_stage_against_direct_sums(ps, dtype, tol, kind, bar, kernel):
    print(f"case: type1 {dtype} {kind} kernel={kernel}", flush=True)
    n, half = 256, 8.0
    h = 2 * half / n
    plan = ps.Plan(n, h, dtype=dtype, tol=tol, kernel=kernel)
    m = plan.info["n_nodes"]
    kx, ky, q = plan.nodes()
    xs = O.grid_points(O.SplitParams(n, h, 1, 2))
    if kind == "noise":
        rng = np.random.default_rng(22)
        coef = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    else:
        coef = q * O.type2_direct(stage_density("smooth", n, half), h, xs, kx, ky)
    cdt = torch.complex128 if dtype == torch.float64 else torch.complex64
    c = torch.as_tensor(coef, dtype=cdt, device="cuda")
    got = plan.type1(c).double().cpu().numpy()
    ref = O.type1_direct(c.cpu().numpy().astype(np.complex128), xs, kx, ky).real
    err = rel_l2(got, ref)
    print(f"  rel l2 {err:.3e} (bar {bar:.0e})", flush=True)
    assert err <= bar


# --------------------------------------------------------------------------
# sizes spanning several tiles, both precisions
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512, 1024])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_mixture_sizes_match_oracle(ps, n, dtype):
    print(f"case: mixture n={n} {dtype}", flush=True)
    half = max(4.0, n / 64.0)
    h = 2 * half / n
    spec = W.draw_mixture(100 + n, 8, 0.375 * half, (0.5, 2.0))
    spec = W.MixtureSpec(spec.cx, spec.cy, spec.wx * half / 16, spec.wy * half / 16, spec.phase) \
        if half > 16 else spec
    rho = W.mixture_density(n, half, spec)
    kw = dict(tol=1e-12) if dtype == torch.float64 else dict(tol=1e-7)
    # tiny grids: the default disk reaches past the Nyquist frequency, shrink it
    if n <= 16:
        kw.update(sigma=0.35 / half, cutoff=1.6 / half)
    plan, rho_used, got = run_solve(ps, rho, n, h, dtype, **kw)
    ref = O.phi(rho_used, O.SplitParams(n=n, h=h, n_r=64, n_theta=128, sigma=kw.get("sigma"),
                                        cutoff=kw.get("cutoff")))
    bar = 1e-10 if dtype == torch.float64 else 1e-6
    assert rel_linf(got, ref) <= bar, (rel_linf(got, ref), rel_l2(got, ref))
    assert rel_l2(got, ref) <= bar


def test_tiny_grid_brute_size(ps):
    print("case: 8x8 FP64", flush=True)
    n, h = 8, 0.5
    rho = np.random.default_rng(9).standard_normal((n, n))
    kw = dict(n_r=3, n_theta=4, sigma=0.4, cutoff=0.9, tol=1e-12)
    plan, rho_used, got = run_solve(ps, rho, n, h, torch.float64, **kw)
    ref = O.phi(rho_used, O.SplitParams(n=n, h=h, n_r=3, n_theta=4, sigma=0.4, cutoff=0.9))
    assert rel_linf(got, ref) <= 1e-10


@pytest.mark.parametrize("n_r,n_theta,sub_nodes", [(5, 6, 8), (7, 10, 9), (1, 2, 64)])
def test_odd_node_counts_and_ragged_subproblems(ps, n_r, n_theta, sub_nodes):
    """Node counts that are not multiples of 4 (no x <-> y symmetry of the node
    set; N_theta even keeps it closed under k -> -k), a single radial node, and
    subproblem sizes that leave ragged last runs in every bin."""
    print(f"case: 64x64 n_r={n_r} n_theta={n_theta} sub_nodes={sub_nodes}", flush=True)
    n, half = 64, 8.0
    rho = W.mixture_density(n, half, W.draw_mixture(41, 6, 3.0, (0.6, 1.5)))
    plan, rho_used, got = run_solve(ps, rho, n, 2 * half / n, torch.float64, n_r=n_r, n_theta=n_theta, tol=1e-12,
                                    sub_nodes=sub_nodes)
    ref = O.phi(rho_used, O.SplitParams(n=n, h=2 * half / n, n_r=n_r, n_theta=n_theta))
    assert rel_linf(got, ref) <= 1e-10
    assert rel_l2(got, ref) <= 1e-10
    plan.close()


def test_zero_density_gives_zero(ps):
    plan = ps.Plan(128, 0.125, dtype=torch.float32)
    out = plan.solve(torch.zeros(128, 128, dtype=torch.float32, device="cuda"))
    assert torch.count_nonzero(out).item() == 0


# --------------------------------------------------------------------------
# full-size single solve: 2048^2 over [-16, 16)^2, 64 x 128 nodes
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def big_case():
    spec = W.draw_mixture(0)
    rho = W.mixture_density(2048, 16.0, spec)
    return rho


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_full_size_single_solve(ps, big_case, dtype):
    print(f"case: 2048x2048 {dtype}", flush=True)
    tol = 1e-7 if dtype == torch.float32 else 1e-12
    plan, rho_used, got = run_solve(ps, big_case, 2048, 1 / 64, dtype, tol=tol)
    ref = O.phi(rho_used, O.SplitParams(n=2048, h=1 / 64, n_r=64, n_theta=128))
    bar = 1e-10 if dtype == torch.float64 else 1e-6
    print(f"  rel_linf={rel_linf(got, ref):.3e} rel_l2={rel_l2(got, ref):.3e}", flush=True)
    assert rel_linf(got, ref) <= bar
    assert rel_l2(got, ref) <= bar


# --------------------------------------------------------------------------
# transposed solve, second component, invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_adjoint_against_oracle_transpose(ps, dtype):
    print(f"case: adjoint {dtype}", flush=True)
    n, half = 256, 8.0
    h = 2 * half / n
    rng = np.random.default_rng(31)
    g = rng.standard_normal((n, n))
    rho = W.mixture_density(n, half, W.draw_mixture(5, 8, 3.0, (0.5, 1.5)))
    plan = ps.Plan(n, h, dtype=dtype, tol=1e-12 if dtype == torch.float64 else 1e-7)
    gd = to_dev(g, dtype)
    rd = to_dev(rho, dtype)
    at_g = plan.solve_adjoint(gd).double().cpu().numpy()
    a_r = plan.solve(rd).double().cpu().numpy()
    ref = O.phi_transpose(gd.double().cpu().numpy(), O.SplitParams(n=n, h=h, n_r=64, n_theta=128))
    bar = 1e-10 if dtype == torch.float64 else 1e-6
    assert rel_l2(at_g, ref) <= bar
    lhs = float(np.vdot(a_r, gd.double().cpu().numpy()))
    rhs = float(np.vdot(rd.double().cpu().numpy(), at_g))
    assert abs(lhs - rhs) <= (1e-12 if dtype == torch.float64 else 1e-5) * abs(lhs)


def test_components_sum_to_minus_rho(ps):
    print("case: xx + yy", flush=True)
    n, half = 256, 8.0
    rho = W.mixture_density(n, half, W.draw_mixture(6, 8, 3.0, (0.5, 1.5)))
    px = ps.Plan(n, 2 * half / n, dtype=torch.float64)
    py = ps.Plan(n, 2 * half / n, dtype=torch.float64, component="y")
    r = to_dev(rho, torch.float64)
    total = (px.solve(r) + py.solve(r)).cpu().numpy()
    assert np.max(np.abs(total + rho)) <= 1e-11 * rho.max()


def test_transposed_density_swaps_components(ps):
    n, half = 256, 8.0
    rho = W.mixture_density(n, half, W.draw_mixture(7, 8, 3.0, (0.5, 1.5)))
    px = ps.Plan(n, 2 * half / n, dtype=torch.float64)
    py = ps.Plan(n, 2 * half / n, dtype=torch.float64, component="y")
    a = px.solve(to_dev(rho.T, torch.float64)).cpu().numpy()
    b = py.solve(to_dev(rho, torch.float64)).cpu().numpy().T
    assert np.max(np.abs(a - b)) <= 1e-11 * np.max(np.abs(b))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_repeated_solves_are_bitwise_identical(ps, dtype):
    """No atomics anywhere in the chain: the same input gives the same bits."""
    n = 512
    rho = W.mixture_density(n, 8.0, W.draw_mixture(8, 8, 3.0, (0.5, 1.5)))
    plan = ps.Plan(n, 16.0 / n, dtype=dtype)
    r = to_dev(rho, dtype)
    a = plan.solve(r).cpu().numpy()
    b = plan.solve(r).cpu().numpy()
    c = plan.solve_adjoint(r).cpu().numpy()
    d = plan.solve_adjoint(r).cpu().numpy()
    assert np.array_equal(a, b)
    assert np.array_equal(c, d)


def test_output_and_overlap_rules(ps):
    """The binding writes results into `out` itself: a non-contiguous `out`
    (which a copy would leave untouched) and an `out` sharing memory with the
    input are refused; a non-contiguous input is copied and solves as usual."""
    print("case: output and overlap rules 128^2 FP64", flush=True)
    n = 128
    rho = W.mixture_density(n, 8.0, W.draw_mixture(8, 5, 3.0, (0.5, 1.5)))
    plan = ps.Plan(n, 16.0 / n, dtype=torch.float64)
    r = to_dev(rho, torch.float64)
    ref = plan.solve(r).cpu().numpy()
    wide = torch.zeros((n, 2 * n), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError, match="contiguous"):
        plan.solve(r, wide[:, :n])
    with pytest.raises(ValueError, match="overlap"):
        plan.solve(r, r)
    with pytest.raises(ValueError, match="overlap"):
        plan.solve_adjoint(r, r)
    wide[:, 1::2] = r
    assert np.array_equal(plan.solve(wide[:, 1::2]).cpu().numpy(), ref)
    assert float(wide[:, ::2].abs().max()) == 0.0
    plan.close()
    bp = ps.BatchPlan([dict(n=128, h=1 / 16), dict(n=256, h=1 / 16)], dtype=torch.float32)
    src = torch.zeros(bp.total, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError, match="overlap"):
        bp.solve(src, src)
    two = torch.zeros(2 * bp.total, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError, match="contiguous"):
        bp.solve(src, two[::2])
    bp.close()


def test_autograd_backward_is_the_adjoint(ps):
    n, half = 128, 8.0
    rho = W.mixture_density(n, half, W.draw_mixture(9, 8, 3.0, (0.5, 1.5)))
    plan = ps.Plan(n, 2 * half / n, dtype=torch.float64)
    r = to_dev(rho, torch.float64).requires_grad_(True)
    target = to_dev(np.random.default_rng(4).standard_normal((n, n)) * 0.01, torch.float64)
    phi = ps.phi_solve(r, plan)
    loss = ((phi - target) ** 2).sum()
    loss.backward()
    g = 2 * (phi.detach() - target)
    ref = plan.solve_adjoint(g)
    assert torch.allclose(r.grad, ref, rtol=0, atol=1e-14 * ref.abs().max().item())


def test_graph_replay_matches_eager(ps):
    """A solve captured into a HIP graph (through torch's capture stream; the
    node-side chain joins the capture through the plan's fork/join events)
    gives the eager result on every replay, with other eager work between."""
    print("case: graph replay 512^2 FP32", flush=True)
    n = 512
    rho = W.mixture_density(n, 8.0, W.draw_mixture(12, 8, 3.0, (0.5, 1.5)))
    other = W.mixture_density(n, 8.0, W.draw_mixture(13, 8, 3.0, (0.5, 1.5)))
    plan = ps.Plan(n, 16.0 / n, dtype=torch.float32)
    r = to_dev(rho, torch.float32)
    o = to_dev(other, torch.float32)
    eager = plan.solve(r).cpu().numpy()
    out = torch.empty_like(r)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.solve(r, out)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.solve(r, out)
    for rep in range(4):
        out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), f"replay {rep}"
        # unrelated eager work on the same plan between replays
        plan.solve(o)
        torch.cuda.synchronize()


# --------------------------------------------------------------------------
# node sort parameters and the plan-time autotuner
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dtype,bin_side,sub_nodes", [
    (torch.float64, 4, 32), (torch.float64, 16, 64), (torch.float64, 16, 8),
    (torch.float32, 4, 64), (torch.float32, 16, 32)])
def test_node_sort_parameters_match_oracle(ps, dtype, bin_side, sub_nodes):
    print(f"case: 256x256 mixture {dtype} bin={bin_side} sub={sub_nodes}", flush=True)
    n, half = 256, 8.0
    rho = W.mixture_density(n, half, W.draw_mixture(11, 8, 4.0, (0.5, 1.5)))
    tol = 1e-12 if dtype == torch.float64 else 1e-7
    plan, rho_used, got = run_solve(ps, rho, n, 2 * half / n, dtype, tol=tol, bin=bin_side, sub_nodes=sub_nodes)
    assert plan.info["bin"] == bin_side and plan.info["sub_nodes"] == sub_nodes
    ref = O.phi(rho_used, O.SplitParams(n=n, h=2 * half / n, n_r=64, n_theta=128))
    bar = 1e-10 if dtype == torch.float64 else 1e-6
    assert rel_linf(got, ref) <= bar
    assert rel_l2(got, ref) <= bar


def test_autotuned_plan_matches_oracle(ps):
    print("case: 512x512 mixture FP32 autotune", flush=True)
    n, half = 512, 8.0
    rho = W.mixture_density(n, half, W.draw_mixture(12, 8, 4.0, (0.5, 1.5)))
    plan, rho_used, got = run_solve(ps, rho, n, 2 * half / n, torch.float32, tol=1e-7, autotune=True)
    assert plan.info["bin"] in (4, 8, 16) and plan.info["sub_nodes"] in (32, 64)
    print(f"autotuned bin={plan.info['bin']} sub_nodes={plan.info['sub_nodes']}", flush=True)
    ref = O.phi(rho_used, O.SplitParams(n=n, h=2 * half / n, n_r=64, n_theta=128))
    assert rel_linf(got, ref) <= 1e-6
    assert rel_l2(got, ref) <= 1e-6


@pytest.mark.parametrize("dtype,bar", [(torch.float64, 1e-10), (torch.float32, 1e-6)])
def test_jacobi_radial_rule_and_the_papers_node_counts(ps, dtype, bar):
    """The paper's own variant of the quadrature: Gauss-Jacobi radial rule and
    60 x 60 polar nodes (Sec. 2.1), against the oracle with the same rule."""
    print(f"case: Gauss-Jacobi 60x60 256^2 {dtype}", flush=True)
    n, half = 256, 8.0
    rho = W.mixture_density(n, half, W.draw_mixture(13, 8, 4.0, (0.5, 1.5)))
    tol = 1e-12 if dtype == torch.float64 else 1e-7
    plan, rho_used, got = run_solve(ps, rho, n, 2 * half / n, dtype, n_r=60, n_theta=60, tol=tol, radial="jacobi")
    ref = O.phi(rho_used, O.SplitParams(n=n, h=2 * half / n, n_r=60, n_theta=60, radial="jacobi"))
    assert rel_linf(got, ref) <= bar
    assert rel_l2(got, ref) <= bar


@pytest.mark.parametrize("dtype,bar", [(torch.float64, 1e-10), (torch.float32, 1e-6)])
def test_the_papers_exact_variant(ps, dtype, bar, golden):
    """Everything as the paper states it (Sec. 2.1): Gauss-Jacobi radial rule,
    60 x 60 polar nodes and Greengard-Lee Gaussian gridding for both NUFFTs,
    against the oracle with the same quadrature; and Example 1 on [-8, 8)^2 at
    h = 1/8 against its closed form: the error must reproduce the value Table 2
    prints for that grid (read from the golden table) within 2 %, the band the
    oracle's own pin uses, and equal the oracle's error on the same grid and
    rule to within 0.1 % of it (the GPU and oracle results differ by rounding,
    about 1e-14, against an error of 1.6e-10)."""
    print(f"case: paper variant 256^2 {dtype}", flush=True)
    n, half = 256, 8.0
    rho = W.mixture_density(n, half, W.draw_mixture(14, 8, 4.0, (0.5, 1.5)))
    tol = 1e-12 if dtype == torch.float64 else 1e-7
    kw = dict(n_r=60, n_theta=60, tol=tol, radial="jacobi", kernel="gaussian")
    plan, rho_used, got = run_solve(ps, rho, n, 2 * half / n, dtype, **kw)
    ref = O.phi(rho_used, O.SplitParams(n=n, h=2 * half / n, n_r=60, n_theta=60, radial="jacobi"))
    assert rel_linf(got, ref) <= bar
    assert rel_l2(got, ref) <= bar
    if dtype == torch.float64:
        n = 128
        x, y, _ = W.grid_2d(n, half)
        plan, _, got = run_solve(ps, W.paper_gaussian_density(n, half), n, 2 * half / n, dtype, **kw)
        ex = O.closed_forms.phi_isotropic_gaussian(x, y, math.pi, math.pi ** 2)
        err = rel_linf(got, ex)
        printed = [row[2] for row in golden("table2_gaussian_nufft.txt") if row[0] == 8 and row[1] == 0.125]
        assert len(printed) == 1
        p = O.SplitParams(n=n, h=2 * half / n, n_r=60, n_theta=60, radial="jacobi")
        err_oracle = rel_linf(O.phi(W.paper_gaussian_density(n, half), p), ex)
        print(f"  Example 1, L = 8, h = 1/8: {err:.4e} (oracle {err_oracle:.4e}, Table 2 {printed[0]:.2e})",
              flush=True)
        assert abs(err - printed[0]) <= 0.02 * printed[0]
        assert abs(err - err_oracle) <= 1e-3 * err_oracle


# --------------------------------------------------------------------------
# the largest grid the plans take: 4096^2 (fine grid 8192)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def max_case():
    """A mixture density at N = 4096 over [-16, 16)^2, rounded to FP32 so that
    both data paths see the same input, and the oracle at 256 sampled points
    (I1 by the padded FFT everywhere, I2 by direct sums evaluated at the
    samples only)."""
    n, half = 4096, 16.0
    h = 2 * half / n
    rho = W.mixture_density(n, half, W.draw_mixture(0)).astype(np.float32).astype(np.float64)
    p = O.SplitParams(n=n, h=h, n_r=64, n_theta=128)
    idx = np.random.default_rng(17).integers(0, n, size=(256, 2))
    i1 = O.i1_padded_fft(rho, p)[idx[:, 0], idx[:, 1]]
    kx, ky, q = O.polar_rule(p)
    xs = O.grid_points(p)
    rho_hat = O.type2_direct(rho, h, xs, kx, ky)
    phase = np.exp(2j * np.pi * (np.outer(xs[idx[:, 1]], kx) + np.outer(xs[idx[:, 0]], ky)))
    i2 = (phase @ (q * rho_hat)).real
    return rho, idx, i1 + i2


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_largest_grid_against_sampled_oracle(ps, max_case, dtype):
    print(f"case: 4096x4096 {dtype}", flush=True)
    rho, idx, ref = max_case
    n = rho.shape[0]
    tol = 1e-12 if dtype == torch.float64 else 1e-7
    plan, _, got = run_solve(ps, rho, n, 32.0 / n, dtype, tol=tol)
    assert plan.info["n_fine"] == 8192
    g = got[idx[:, 0], idx[:, 1]]
    bar = 1e-10 if dtype == torch.float64 else 1e-6
    err = float(np.max(np.abs(g - ref)) / np.max(np.abs(got)))
    print(f"  sampled rel err {err:.3e}", flush=True)
    assert err <= bar
    plan.close()
