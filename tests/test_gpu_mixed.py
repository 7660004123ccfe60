"""GPU parity of the mixed component, multiplier -kx ky/|k|^2 (the Remark of
Sec. 2.1: another potential through the same split), through the C ABI, against
the FP64 oracle on the same seeded inputs.

Bars as for the DS component: rel L-inf and L2 <= 1e-10 (FP64 data path) and
<= 1e-6 (FP32 data path, oracle on the FP32-rounded input); the periodic
solver <= 1e-12 / 1e-6 (FFT rounding only); batch members bitwise equal to
their single-plan solves."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import closed_forms as C
from oracle import periodic as OP
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BARS = {torch.float64: 1e-10, torch.float32: 1e-6}
TOLS = {torch.float64: 1e-12, torch.float32: 1e-7}


@pytest.fixture(scope="module")
def ps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_2014_amd as ps
    return ps


def rel_linf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("n", [16, 64, 128, 256, 512])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_mixed_solve_matches_oracle(ps, n, dtype):
    print(f"case: mixed n={n} {dtype}", flush=True)
    half = max(4.0, n / 64.0)
    h = 2 * half / n
    rho = W.mixture_density(n, half, W.draw_mixture(200 + n, 8, 0.375 * half, (0.5, 2.0)))
    kw = dict(tol=TOLS[dtype])
    if n <= 16:            # the default disk reaches past the Nyquist frequency: shrink it
        kw.update(sigma=0.35 / half, cutoff=1.6 / half)
    plan = ps.Plan(n, h, dtype=dtype, component="xy", **kw)
    r = dev(rho, dtype)
    got = plan.solve(r).double().cpu().numpy()
    ref = O.phi(r.double().cpu().numpy(), O.SplitParams(n=n, h=h, n_r=64, n_theta=128, component="xy",
                                                         sigma=kw.get("sigma"), cutoff=kw.get("cutoff")))
    assert rel_linf(got, ref) <= BARS[dtype], (rel_linf(got, ref), rel_l2(got, ref))
    assert rel_l2(got, ref) <= BARS[dtype]
    plan.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_mixed_transposed_solve_and_random_input(ps, dtype):
    # random input: every bin of the padded grid, the Nyquist lines included, is
    # populated, so the Nyquist reading is exercised
    print(f"case: mixed adjoint {dtype}", flush=True)
    n, half = 128, 6.0
    h = 2 * half / n
    g = np.random.default_rng(41).standard_normal((n, n))
    plan = ps.Plan(n, h, dtype=dtype, component="xy", tol=TOLS[dtype])
    gd = dev(g, dtype)
    used = gd.double().cpu().numpy()
    p = O.SplitParams(n=n, h=h, n_r=64, n_theta=128, component="xy")
    got_t = plan.solve_adjoint(gd).double().cpu().numpy()
    got = plan.solve(gd).double().cpu().numpy()
    assert rel_l2(got_t, O.phi_transpose(used, p)) <= BARS[dtype]
    assert rel_l2(got, O.phi(used, p)) <= BARS[dtype]
    plan.close()


def test_mixed_example1_against_closed_form(ps):
    print("case: mixed Example 1 closed form", flush=True)
    n, half = 256, 8.0
    x, y, _ = W.grid_2d(n, half)
    plan = ps.Plan(n, 2 * half / n, dtype=torch.float64, tol=1e-12, component="xy")
    got = plan.solve(dev(W.paper_gaussian_density(n, half), torch.float64)).cpu().numpy()
    ex = C.phi_xy_isotropic_gaussian(x, y, math.pi, math.pi ** 2)
    assert rel_linf(got, ex) <= 1e-11
    plan.close()


@pytest.mark.parametrize("n", [16, 128, 1024])
@pytest.mark.parametrize("dtype,bar", [(torch.float64, 1e-12), (torch.float32, 1e-6)])
def test_mixed_periodic_matches_oracle(ps, n, dtype, bar):
    print(f"case: mixed periodic {n} {dtype}", flush=True)
    h = 16.0 / n
    g = np.random.default_rng(50 + n).standard_normal((n, n))
    plan = ps.Plan(n, h, dtype=dtype, n_r=16, n_theta=32, component="xy")
    r = dev(g, dtype)
    got = plan.periodic(r).double().cpu().numpy()
    ref = OP.phi_periodic(r.double().cpu().numpy(), h, "xy")
    assert rel_linf(got, ref) <= bar
    plan.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_with_mixed_members_matches_single_plans(ps, dtype):
    print(f"case: batch with mixed members {dtype}", flush=True)
    specs = [(256, "xy", 3), (128, "x", 4), (512, "xy", 5), (128, "xy", 6)]
    members, params = [], []
    for n, comp, seed in specs:
        half = n / 64.0
        members.append(W.mixture_density(n, half, W.draw_mixture(seed, 8, 0.375 * half, (0.5 * half / 16, 2 * half / 16))))
        params.append(dict(n=n, h=2 * half / n, n_r=64, n_theta=128, tol=TOLS[dtype], component=comp))
    bp = ps.BatchPlan(params, dtype=dtype)
    packed = bp.pack(members)
    got = [g.cpu().numpy() for g in bp.unpack(bp.solve(packed))]
    used = [g.double().cpu().numpy() for g in bp.unpack(packed)]
    for i, kw in enumerate(params):
        single = ps.Plan(kw["n"], kw["h"], dtype=dtype, n_r=64, n_theta=128, tol=kw["tol"], component=kw["component"])
        ref_single = single.solve(dev(used[i], dtype)).cpu().numpy()
        assert np.array_equal(got[i], ref_single), f"member {i}"
        comp = "xx" if kw["component"] == "x" else "xy"
        ref = O.phi(used[i], O.SplitParams(n=kw["n"], h=kw["h"], n_r=64, n_theta=128, component=comp))
        assert rel_linf(got[i], ref) <= BARS[dtype], f"member {i}"
        single.close()
    bp.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_with_gaussian_gridding_members(ps, dtype):
    """Members with the Gaussian gridding kernel (wider taps, window 128) next to
    ES members: the batch's node blocks take the wide tap store; every member
    equals its single-plan solve bit for bit and the oracle within the bar."""
    print(f"case: batch with Gaussian gridding members {dtype}", flush=True)
    specs = [(256, "gaussian", 7), (512, "es", 8), (128, "gaussian", 9)]
    members, params = [], []
    for n, kernel, seed in specs:
        half = n / 64.0
        members.append(W.mixture_density(n, half, W.draw_mixture(seed, 8, 0.375 * half, (0.5 * half / 16, 2 * half / 16))))
        params.append(dict(n=n, h=2 * half / n, n_r=64, n_theta=128, tol=TOLS[dtype], kernel=kernel))
    bp = ps.BatchPlan(params, dtype=dtype)
    packed = bp.pack(members)
    got = [g.cpu().numpy() for g in bp.unpack(bp.solve(packed))]
    used = [g.double().cpu().numpy() for g in bp.unpack(packed)]
    for i, kw in enumerate(params):
        single = ps.Plan(kw["n"], kw["h"], dtype=dtype, n_r=64, n_theta=128, tol=kw["tol"], kernel=kw["kernel"])
        assert np.array_equal(got[i], single.solve(dev(used[i], dtype)).cpu().numpy()), f"member {i}"
        ref = O.phi(used[i], O.SplitParams(n=kw["n"], h=kw["h"], n_r=64, n_theta=128))
        assert rel_linf(got[i], ref) <= BARS[dtype], f"member {i}"
        single.close()
    bp.close()
