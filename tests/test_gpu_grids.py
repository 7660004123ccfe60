"""GPU parity on grids of any even side and with padding factors kappa > 2
(Sec. 2.1: kappa >= 2; Sec. 3: N even), against the FP64 oracle on the same
seeded inputs and the same padded box.

The plan pads the I1 box (and the NUFFT fine grid) to the smallest power of
two F >= kappa N; the oracle is given that side as pad_side, so both compute
the same discrete quadrature (the oracle's pins show the potential does not
depend on the padded side beyond rounding).  Bars as for every solve: rel L-inf
and L2 <= 1e-10 (FP64), <= 1e-6 (FP32, the oracle on the FP32-rounded input);
the largest grid against a sampled oracle."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BARS = {torch.float64: 1e-10, torch.float32: 1e-6}
TOLS = {torch.float64: 1e-12, torch.float32: 1e-7}


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


def density(n, half, seed):
    spec = W.draw_mixture(seed, 8, 0.375 * half, (0.5, 2.0))
    if half > 16:
        spec = W.MixtureSpec(spec.cx, spec.cy, spec.wx * half / 16, spec.wy * half / 16, spec.phase)
    return W.mixture_density(n, half, spec)


@pytest.mark.parametrize("n,pad,fine", [(96, 2, 256), (100, 2, 256), (384, 2, 1024), (1536, 2, 4096),
                                        (200, 3, 1024), (320, 3, 1024), (256, 4, 1024), (1024, 3, 4096)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_grid_side_and_padding_match_oracle(ps, n, pad, fine, dtype):
    half = max(4.0, n / 64.0)
    h = 2 * half / n
    print(f"case: N={n} kappa={pad} {dtype}", flush=True)
    rho = density(n, half, 300 + n + pad)
    plan = ps.Plan(n, h, dtype=dtype, tol=TOLS[dtype], pad=pad)
    assert plan.info["n_fine"] == fine
    r = torch.as_tensor(rho, dtype=dtype, device="cuda")
    got = plan.solve(r).double().cpu().numpy()
    used = r.double().cpu().numpy()
    ref = O.phi(used, O.SplitParams(n=n, h=h, n_r=64, n_theta=128, kappa=pad, pad_side=fine))
    e_inf, e_2 = rel_linf(got, ref), rel_l2(got, ref)
    print(f"  rel L-inf {e_inf:.3e}, L2 {e_2:.3e}", flush=True)
    assert e_inf <= BARS[dtype]
    assert e_2 <= BARS[dtype]
    # the transposed solve against the oracle's literal transpose
    g = np.random.default_rng(n + pad).standard_normal((n, n))
    gt = torch.as_tensor(g, dtype=dtype, device="cuda")
    back = plan.solve_adjoint(gt).double().cpu().numpy()
    ref_t = O.phi_transpose(gt.double().cpu().numpy(),
                            O.SplitParams(n=n, h=h, n_r=64, n_theta=128, kappa=pad, pad_side=fine))
    assert rel_l2(back, ref_t) <= BARS[dtype]
    plan.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_grid_of_3072_against_sampled_oracle(ps, dtype):
    """N = 3072 over [-24, 24)^2 (padded side 8192): I1 by the oracle's padded
    FFT everywhere, I2 by direct sums at 256 sampled points."""
    n, half = 3072, 24.0
    h = 2 * half / n
    print(f"case: N=3072 {dtype}", flush=True)
    rho = density(n, half, 17).astype(np.float32).astype(np.float64)
    plan = ps.Plan(n, h, dtype=dtype, tol=TOLS[dtype])
    assert plan.info["n_fine"] == 8192
    got = plan.solve(torch.as_tensor(rho, dtype=dtype, device="cuda")).double().cpu().numpy()
    plan.close()
    p = O.SplitParams(n=n, h=h, n_r=64, n_theta=128, pad_side=8192)
    idx = np.random.default_rng(18).integers(0, n, size=(256, 2))
    i1 = O.i1_padded_fft(rho, p)[idx[:, 0], idx[:, 1]]
    kx, ky, q = O.polar_rule(p)
    xs = O.grid_points(p)
    rho_hat = O.type2_direct(rho, h, xs, kx, ky)
    phase = np.exp(2j * np.pi * (np.outer(xs[idx[:, 1]], kx) + np.outer(xs[idx[:, 0]], ky)))
    ref = i1 + (phase @ (q * rho_hat)).real
    g = got[idx[:, 0], idx[:, 1]]
    err = float(np.max(np.abs(g - ref)) / np.max(np.abs(got)))
    print(f"  sampled rel err {err:.3e}", flush=True)
    assert err <= BARS[dtype]


def test_batch_of_uneven_non_power_of_two_members(ps):
    """A batch whose members have sides 96, 200, 384 and 640 (padded sides 256,
    512, 1024, 2048): every member bitwise equal to its single-plan solve and
    within the FP32 bar of the oracle."""
    dtype = torch.float32
    sizes = [384, 96, 640, 200]
    print(f"case: batch of sides {sizes}", flush=True)
    members = [(n, n / 64.0, density(n, n / 64.0, 40 + n)) for n in sizes]
    params = [dict(n=n, h=2 * half / n, n_r=64, n_theta=128, tol=TOLS[dtype]) for n, half, _ in members]
    bp = ps.BatchPlan(params, dtype=dtype)
    packed = bp.pack([m[2] for m in members])
    got = [g.cpu().numpy() for g in bp.unpack(bp.solve(packed))]
    used = [g.double().cpu().numpy() for g in bp.unpack(packed)]
    for i, (n, half, _) in enumerate(members):
        h = 2 * half / n
        plan = ps.Plan(n, h, dtype=dtype, tol=TOLS[dtype])
        single = plan.solve(torch.as_tensor(used[i], dtype=dtype, device="cuda")).cpu().numpy()
        fine = plan.info["n_fine"]
        plan.close()
        assert np.array_equal(got[i], single), f"member {i} (N={n})"
        ref = O.phi(used[i], O.SplitParams(n=n, h=h, n_r=64, n_theta=128, pad_side=fine))
        assert rel_linf(got[i], ref) <= BARS[dtype], f"member {i} N={n}"
        assert rel_l2(got[i], ref) <= BARS[dtype], f"member {i} N={n}"
    bp.close()


def test_periodic_solver_and_stepper_refuse_non_power_of_two_grids(ps):
    """The periodic FFT solver and the DS stepper transform the unpadded grid
    itself, so they take power-of-two sides only, and say so."""
    from paper_1409_2014_amd import _binding as B
    print("case: periodic / stepper refusals", flush=True)
    plan = ps.Plan(96, 0.125, dtype=torch.float64)
    r = torch.zeros((96, 96), dtype=torch.float64, device="cuda")
    with pytest.raises(B.PhiError, match="PHI_ERR_UNSUPPORTED"):
        plan.periodic(r)
    plan.close()
    with pytest.raises(B.PhiError, match="PHI_ERR_UNSUPPORTED"):
        ps.DSStepper(96, 0.125, alpha=1.0, beta=1.0, tau=1e-3, dtype=torch.float64)
