"""GPU parity of the 2-D Coulomb solve (multiplier 1/|k|, PHI_COMPONENT_COULOMB;
Sec. 2.1, Remark) against the FP64 oracle on the same seeded inputs, with both
partitions: erfc(|k|/sigma) (the default, smooth integrands) and the paper's
Gaussian (a cone in the I1 integrand at k = 0).

Bars as for every solve: rel L-inf and L2 <= 1e-10 (FP64), <= 1e-6 (FP32, the
oracle on the FP32-rounded input); the full 2048^2 case against the oracle's
padded FFT for I1 everywhere and direct sums for I2 at sampled points.  The
closed form of a Gaussian density is met to the NUFFT tolerance with the erfc
partition, and the Gaussian partition's cone error reproduces the oracle's."""
import numpy as np
import pytest

import oracle as O
from oracle import closed_forms as C
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


@pytest.mark.parametrize("n,half", [(64, 8.0), (96, 6.0), (256, 8.0)])
@pytest.mark.parametrize("partition", ["erfc", "gauss"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_coulomb_solve_and_transpose_match_oracle(ps, n, half, partition, dtype):
    h = 2 * half / n
    print(f"case: coulomb N={n} {partition} {dtype}", flush=True)
    rho = density(n, half, 600 + n)
    plan = ps.Plan(n, h, dtype=dtype, tol=TOLS[dtype], component="coulomb", partition=partition)
    fine = plan.info["n_fine"]
    r = torch.as_tensor(rho, dtype=dtype, device="cuda")
    got = plan.solve(r).double().cpu().numpy()
    p = O.SplitParams(n=n, h=h, n_r=64, n_theta=128, component="coulomb", partition=partition, pad_side=fine)
    ref = O.phi(r.double().cpu().numpy(), p)
    print(f"  rel L-inf {rel_linf(got, ref):.3e}, L2 {rel_l2(got, ref):.3e}", flush=True)
    assert rel_linf(got, ref) <= BARS[dtype]
    assert rel_l2(got, ref) <= BARS[dtype]
    g = torch.as_tensor(np.random.default_rng(n).standard_normal((n, n)), dtype=dtype, device="cuda")
    back = plan.solve_adjoint(g).double().cpu().numpy()
    ref_t = O.phi_transpose(g.double().cpu().numpy(), p)
    assert rel_l2(back, ref_t) <= BARS[dtype]
    assert rel_linf(back, ref_t) <= BARS[dtype]
    plan.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_coulomb_closed_form_of_a_gaussian(ps, dtype):
    """rho = e^{-r^2} on [-8, 8)^2, h = 1/4: Phi = pi^{3/2} e^{-r^2/2} I_0(r^2/2).
    erfc partition: within the NUFFT tolerance (the split itself reaches
    rounding); Gaussian partition: the cone error of the oracle, 3.1e-4."""
    n, half = 64, 8.0
    h = 2 * half / n
    print(f"case: coulomb closed form {dtype}", flush=True)
    x, y, _ = W.grid_2d(n, half)
    rho = torch.as_tensor(np.exp(-(x * x + y * y)), dtype=dtype, device="cuda")
    exact = C.coulomb_isotropic_gaussian(x, y)
    plan = ps.Plan(n, h, dtype=dtype, tol=TOLS[dtype], component="coulomb")
    err = rel_linf(plan.solve(rho).double().cpu().numpy(), exact)
    plan.close()
    print(f"  erfc partition: {err:.3e}", flush=True)
    assert err <= (1e-12 if dtype == torch.float64 else 1e-6)
    plan = ps.Plan(n, h, dtype=dtype, tol=TOLS[dtype], component="coulomb", partition="gauss")
    err_g = rel_linf(plan.solve(rho).double().cpu().numpy(), exact)
    plan.close()
    print(f"  gauss partition: {err_g:.3e}", flush=True)
    assert 2.5e-4 < err_g < 4e-4


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_coulomb_full_size_against_sampled_oracle(ps, dtype):
    """2048^2 over [-16, 16)^2 (the C2 grid and density): I1 by the oracle's padded
    FFT everywhere, I2 by direct sums at 256 sampled points."""
    n, half = 2048, 16.0
    h = 2 * half / n
    print(f"case: coulomb 2048 {dtype}", flush=True)
    rho = W.mixture_density(n, half, W.draw_mixture(0)).astype(np.float32).astype(np.float64)
    plan = ps.Plan(n, h, dtype=dtype, tol=TOLS[dtype], component="coulomb")
    got = plan.solve(torch.as_tensor(rho, dtype=dtype, device="cuda")).double().cpu().numpy()
    plan.close()
    p = O.SplitParams(n=n, h=h, n_r=64, n_theta=128, component="coulomb", partition="erfc")
    idx = np.random.default_rng(31).integers(0, n, size=(256, 2))
    i1 = O.i1_padded_fft(rho, p)[idx[:, 0], idx[:, 1]]
    kx, ky, q = O.polar_rule(p)
    xs = O.grid_points(p)
    rho_hat = O.type2_direct(rho, h, xs, kx, ky)
    phase = np.exp(2j * np.pi * (np.outer(xs[idx[:, 1]], kx) + np.outer(xs[idx[:, 0]], ky)))
    ref = i1 + (phase @ (q * rho_hat)).real
    err = float(np.max(np.abs(got[idx[:, 0], idx[:, 1]] - ref)) / np.max(np.abs(got)))
    print(f"  sampled rel err {err:.3e}", flush=True)
    assert err <= BARS[dtype]


def test_coulomb_is_refused_where_it_is_not_built(ps):
    from paper_1409_2014_amd import _binding as B
    print("case: coulomb refusals", flush=True)
    with pytest.raises(B.PhiError, match="PHI_ERR_UNSUPPORTED"):
        ps.BatchPlan([dict(n=128, h=0.25, component="coulomb")])
    plan = ps.Plan(64, 0.25, dtype=torch.float64, component="coulomb")
    with pytest.raises(B.PhiError, match="PHI_ERR_UNSUPPORTED"):
        plan.periodic(torch.zeros((64, 64), dtype=torch.float64, device="cuda"))
    plan.close()
