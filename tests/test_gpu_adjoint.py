"""The hand-written transposed solve as the gradient of a loss: central finite
differences along 16 random directions and the oracle's literal transpose, at
1024^2 over [-16, 16)^2 (h = 1/32).

L(rho) = sum_n (Phi(rho)_n - Phi_t,n)^2 with Phi_t = Phi(rho_t) from another
seed; dL/drho = 2 A^T (A rho - Phi_t).  L is a quadratic in rho, so a central
difference (L(rho + e v) - L(rho - e v)) / (2 e) equals <dL/drho, v> with no
truncation error: what is left is rounding in the computed Phi, amplified by
1/e.

A rounding error d in Phi moves L by about 2 <Phi - Phi_t, d>, so the FD error
is of order u ||Phi - Phi_t|| ||Phi|| / e (u the data path's relative error),
a fixed fraction of the largest directional derivative ||g|| ||v||.  A random
direction of N^2 independent entries has <g, v> ~ ||g|| ||v|| / N, so the error
relative to |<g, v>| is N times larger: about 1e-7 * 1e2 * 1e3 = 1e-2 in FP32
with e = 1e-2.  The bars therefore compare |FD - <g, v>| with ||g|| ||v||:
<= 1e-10 (FP64, e = 1e-3) and <= 1e-4 (FP32, e = 1e-2); in FP64 the error
relative to |<g, v>| itself is also held to <= 1e-8.  g against the oracle's A^T
applied to the same residual: <= 1e-10 (FP64) / 1e-6 (FP32) in rel L-inf."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N, HALF = 1024, 16.0
H = 2 * HALF / N
# dtype, NUFFT tol, FD step, bar on |FD - <g,v>| / (||g|| ||v||), bar on it / |<g,v>|, adjoint bar
CASES = [(torch.float64, 1e-12, 1e-3, 1e-10, 1e-8, 1e-10), (torch.float32, 1e-7, 1e-2, 1e-4, None, 1e-6)]


@pytest.fixture(scope="module")
def ps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_2014_amd as ps
    return ps


@pytest.mark.parametrize("dtype,tol,eps,fd_bar,fd_rel_bar,grad_bar", CASES)
def test_gradient_by_adjoint_matches_fd_and_oracle_transpose(ps, dtype, tol, eps, fd_bar, fd_rel_bar, grad_bar):
    print(f"case: loss gradient 1024^2 {dtype}", flush=True)
    rho = W.mixture_density(N, HALF, W.draw_mixture(2))
    rho_t = W.mixture_density(N, HALF, W.draw_mixture(3))
    plan = ps.Plan(N, H, dtype=dtype, n_r=64, n_theta=128, tol=tol)
    r = torch.as_tensor(rho, dtype=dtype, device="cuda")
    phi_t = plan.solve(torch.as_tensor(rho_t, dtype=dtype, device="cuda")).double()

    def loss(x):
        d = plan.solve(x).double() - phi_t
        return float(torch.sum(d * d))

    # gradient through autograd: PhiSolve's backward is the transposed solve
    x = r.clone().requires_grad_(True)
    d = ps.phi_solve(x, plan) - phi_t.to(dtype)
    (d * d).sum().backward()
    g = x.grad.double().cpu().numpy()

    # the transposed solve on the same residual, against the oracle's literal A^T
    resid = 2.0 * (plan.solve(r).double() - phi_t)
    resid_used = resid.to(dtype).double().cpu().numpy()
    g_dev = plan.solve_adjoint(resid.to(dtype).contiguous()).double().cpu().numpy()
    ref = O.phi_transpose(resid_used, O.SplitParams(n=N, h=H, n_r=64, n_theta=128))
    err = float(np.max(np.abs(g_dev - ref)) / np.max(np.abs(ref)))
    print(f"adjoint vs oracle transpose: {err:.3e}", flush=True)
    assert err <= grad_bar

    worst, worst_rel = 0.0, 0.0
    gnorm = float(np.linalg.norm(g))
    for v in W.random_directions(N, range(100, 116), like=rho):
        vt = torch.as_tensor(v, dtype=dtype, device="cuda")
        a, b = r + eps * vt, r - eps * vt
        fd = (loss(a) - loss(b)) / (2 * eps)
        # the step actually taken (a - b is exact in FP64 from the rounded points)
        step = ((a.double() - b.double()) / (2 * eps)).cpu().numpy()
        dot = float(np.sum(g * step))
        worst = max(worst, abs(fd - dot) / (gnorm * float(np.linalg.norm(step))))
        worst_rel = max(worst_rel, abs(fd - dot) / abs(dot))
    print(f"16 directions: worst |FD - <g,v>| / (|g| |v|) = {worst:.3e}, / |<g,v>| = {worst_rel:.3e}",
          flush=True)
    assert worst <= fd_bar
    if fd_rel_bar is not None:
        assert worst_rel <= fd_rel_bar
    plan.close()
