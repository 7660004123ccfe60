"""GPU parity of the DS time stepper (split-step passes + one potential solve
per step) against the oracle stepper, closed forms, invariants and finite
differences.

Bars (FP64 data path unless stated):
  * beta = 0 (linear flow only) vs the exact Gaussian evolution: <= 1e-12 abs.
  * steps vs the oracle stepper: rel L-inf <= 1e-10; FP32 <= 1e-5 after 10 steps
    (the single-solve FP32 bar 1e-6 per step, and FFT rounding of the same
    order, accumulated over the steps).
  * mass h^2 sum |u|^2 after 100 steps: relative drift <= 1e-12 (FP32: 1e-5;
    every substep conserves it exactly, so the drift is rounding: in FP32 the
    rotation by e^{i pi/4} inside each radix-16 butterfly has modulus^2
    1 - 3.4e-8 for every float pair, a small systematic loss per transform).
  * checkpointed gradient of h^2 sum |u(T)|^4 vs the oracle's reverse pass:
    rel L-inf <= 1e-9 (FP32: 1e-4).
  * self-consistency: the gradient against central differences of the GPU
    stepper's own loss, relative to |<g, d>|: <= 1e-6 (truncation O(e^2) with
    e = 1e-4, plus the transposed solve's tolerance).
"""
import ctypes

import numpy as np
import pytest

from oracle import ds_stepper as D
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CDT = {torch.float64: torch.complex128, torch.float32: torch.complex64}
TOL = {torch.float64: 1e-12, torch.float32: 1e-7}


@pytest.fixture(scope="module")
def ps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_2014_amd as ps
    return ps


def initial(n, half, kx=0.0, ky=0.0):
    x, y, _ = W.grid_2d(n, half)
    return (np.exp(-(x ** 2 + 2 * y ** 2)) * np.exp(1j * (kx * x + ky * y))).astype(np.complex128)


def dev(u, dtype):
    return torch.as_tensor(u, dtype=CDT[dtype], device="cuda").contiguous()


def rel_linf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_linear_flow_matches_exact_gaussian_evolution(ps):
    print("case: stepper beta=0 128^2 FP64", flush=True)
    n, half, tau, steps = 128, 16.0, 0.05, 4
    st = ps.DSStepper(n, 2 * half / n, alpha=1.0, beta=0.0, tau=tau, dtype=torch.float64,
                      n_r=16, n_theta=32, tol=1e-12)
    x, y, _ = W.grid_2d(n, half)
    u = dev(np.exp(-x ** 2 - y ** 2 / 1.5), torch.float64)
    st.forward(u, steps)
    t = tau * steps
    ax, ay = 1.0 + 4j * t, 1.5 - 4j * t
    ref = np.sqrt(1.0 / ax) * np.exp(-x ** 2 / ax) * np.sqrt(1.5 / ay) * np.exp(-y ** 2 / ay)
    assert np.max(np.abs(u.cpu().numpy() - ref)) < 1e-12
    st.close()


@pytest.mark.parametrize("dtype,bar", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
@pytest.mark.parametrize("alpha", [1.0, -1.0])
def test_steps_match_oracle_stepper(ps, dtype, bar, alpha):
    print(f"case: stepper 64^2 10 steps alpha={alpha} {dtype}", flush=True)
    n, half, steps = 64, 4.0, 10
    p = D.DSParams(n=n, h=2 * half / n, alpha=alpha, beta=1.0, tau=1e-2, n_r=32, n_theta=64)
    u0 = initial(n, half, kx=0.7)
    st = ps.DSStepper(n, p.h, alpha=alpha, beta=1.0, tau=p.tau, dtype=dtype, n_r=32, n_theta=64, tol=TOL[dtype])
    u = dev(u0, dtype)
    u_used = u.cpu().numpy().astype(np.complex128)
    st.forward(u, steps)
    ref = D.evolve(u_used, p, steps)
    err = rel_linf(u.cpu().numpy(), ref)
    print(f"rel L-inf after {steps} steps: {err:.3e}", flush=True)
    assert err <= bar
    st.close()


@pytest.mark.parametrize("scheme,pot,dtype,bar", [
    ("yoshida4", "split", torch.float64, 1e-10), ("yoshida4", "periodic", torch.float64, 1e-10),
    ("strang", "periodic", torch.float64, 1e-10), ("yoshida4", "split", torch.float32, 1e-5)])
def test_other_schemes_match_oracle_stepper(ps, scheme, pot, dtype, bar):
    print(f"case: stepper 64^2 6 steps {scheme} {pot} {dtype}", flush=True)
    n, half, steps = 64, 4.0, 6
    p = D.DSParams(n=n, h=2 * half / n, alpha=-1.0, beta=1.0, tau=1e-2, n_r=32, n_theta=64, scheme=scheme,
                   potential=pot)
    st = ps.DSStepper(n, p.h, alpha=-1.0, beta=1.0, tau=p.tau, dtype=dtype, n_r=32, n_theta=64, tol=TOL[dtype],
                      scheme=scheme, potential=pot)
    assert st.substeps == (3 if scheme == "yoshida4" else 1)
    u = dev(initial(n, half, kx=0.7, ky=-0.3), dtype)
    u_used = u.cpu().numpy().astype(np.complex128)
    st.forward(u, steps)
    err = rel_linf(u.cpu().numpy(), D.evolve(u_used, p, steps))
    print(f"rel L-inf after {steps} steps: {err:.3e}", flush=True)
    assert err <= bar
    st.close()


@pytest.mark.parametrize("dtype,bar", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
def test_largest_grid_step_matches_oracle(ps, dtype, bar):
    """One Strang step at the largest side the stepper takes (4096, transforms of
    length 4096 along both axes), with the periodic potential so that the
    oracle step stays a few full-grid FFTs."""
    print(f"case: stepper 4096^2 1 step periodic {dtype}", flush=True)
    n, half = 4096, 32.0
    p = D.DSParams(n=n, h=2 * half / n, alpha=1.0, beta=1.0, tau=1e-2, n_r=32, n_theta=64, potential="periodic")
    st = ps.DSStepper(n, p.h, alpha=1.0, beta=1.0, tau=p.tau, dtype=dtype, n_r=32, n_theta=64, tol=TOL[dtype],
                      potential="periodic")
    u = dev(initial(n, half, kx=0.5, ky=0.25), dtype)
    u_used = u.cpu().numpy().astype(np.complex128)
    st.forward(u, 1)
    err = rel_linf(u.cpu().numpy(), D.evolve(u_used, p, 1))
    print(f"rel L-inf after 1 step: {err:.3e}", flush=True)
    assert err <= bar
    st.close()


@pytest.mark.parametrize("dtype,bar", [(torch.float64, 1e-10), (torch.float32, 2e-5)])
def test_large_phases_match_oracle(ps, dtype, bar):
    """Nonlinear phases from 0 up to about 1.03 rad: beyond pi/4, so that the
    rotation's argument reduction leaves quadrant 0, with the polynomials
    exercised near the ends of their interval."""
    print(f"case: stepper 64^2 large phases {dtype}", flush=True)
    n, half, steps = 64, 4.0, 2
    p = D.DSParams(n=n, h=2 * half / n, alpha=1.0, beta=1.0, tau=0.2, n_r=32, n_theta=64, c_local=2.0,
                   c_potential=1.0)
    st = ps.DSStepper(n, p.h, alpha=1.0, tau=p.tau, c_local=2.0, c_potential=1.0, dtype=dtype, n_r=32,
                      n_theta=64, tol=TOL[dtype])
    u0 = 1.8 * initial(n, half, kx=0.5, ky=0.2)
    phase = D.nonlinear_phase(u0, p, p.tau)
    assert np.max(np.abs(phase)) > 1.0 and np.min(np.abs(phase)) < 0.1
    u = dev(u0, dtype)
    u_used = u.cpu().numpy().astype(np.complex128)
    st.forward(u, steps)
    err = rel_linf(u.cpu().numpy(), D.evolve(u_used, p, steps))
    print(f"rel L-inf after {steps} steps: {err:.3e}", flush=True)
    assert err <= bar
    st.close()


@pytest.mark.parametrize("c_local,c_potential,bar", [(300.0, 1.0, 1e-10), (-300.0, -1.0, 1e-10),
                                                      (4.0e6, 1.0, 1e-7)])
def test_phases_over_many_quadrants_match_oracle(ps, c_local, c_potential, bar):
    """FP64 nonlinear phases up to about +-200 rad (a hundred quadrants of the
    sine/cosine argument reduction, either sign), and a field whose phases run
    from near 0 through 1e5-1.5e6 up to about 2.6e6 rad.  One step.  The third
    bar allows for the phase itself, a product of FP64 numbers near 1e6,
    differing by a few units in its last place (about 1e-9) between the two
    sides."""
    print(f"case: stepper 64^2 phases c_local={c_local} c_potential={c_potential}", flush=True)
    n, half = 64, 4.0
    p = D.DSParams(n=n, h=2 * half / n, alpha=1.0, beta=1.0, tau=0.2, n_r=32, n_theta=64, c_local=c_local,
                   c_potential=c_potential)
    st = ps.DSStepper(n, p.h, alpha=1.0, tau=p.tau, c_local=c_local, c_potential=c_potential,
                      dtype=torch.float64, n_r=32, n_theta=64, tol=1e-12)
    u0 = 1.8 * initial(n, half, kx=0.5, ky=0.2)
    phase = np.abs(D.nonlinear_phase(u0, p, p.tau))
    if abs(c_local) < 1e3:
        assert 100.0 < np.max(phase) < 300.0
    else:
        assert np.max(phase) > 2.0e6 and np.any((phase > 1e5) & (phase < 1.5e6))
    u = dev(u0, torch.float64)
    u_used = u.cpu().numpy().astype(np.complex128)
    st.forward(u, 1)
    err = rel_linf(u.cpu().numpy(), D.evolve(u_used, p, 1))
    print(f"rel L-inf after one step: {err:.3e}", flush=True)
    assert err <= bar
    st.close()


def test_independent_phase_coefficients_match_oracle(ps):
    """The E-E system's nonlinear substep (c_local = -chi, c_potential = -gamma)."""
    print("case: stepper E-E coefficients 64^2", flush=True)
    n, half, steps = 64, 8.0, 5
    p = D.DSParams(n=n, h=2 * half / n, alpha=-1.0, tau=2e-3, n_r=32, n_theta=64, scheme="yoshida4",
                   c_local=1.0, c_potential=-1.0)
    st = ps.DSStepper(n, p.h, alpha=-1.0, c_local=1.0, c_potential=-1.0, tau=p.tau, dtype=torch.float64,
                      n_r=32, n_theta=64, tol=1e-12, scheme="yoshida4")
    x, y, _ = W.grid_2d(n, half)
    u0 = (4 * np.exp(-(x ** 2 + y ** 2) / 4)).astype(np.complex128)
    u = dev(u0, torch.float64)
    st.forward(u, steps)
    assert rel_linf(u.cpu().numpy(), D.evolve(u0, p, steps)) <= 1e-10
    st.close()


@pytest.mark.parametrize("scheme,pot", [("yoshida4", "split"), ("yoshida4", "periodic")])
def test_gradient_of_other_schemes_matches_oracle(ps, scheme, pot):
    print(f"case: L4 gradient 32^2 {scheme} {pot}", flush=True)
    n, half, steps = 32, 4.0, 4
    p = D.DSParams(n=n, h=2 * half / n, alpha=1.0, beta=1.5, tau=2e-2, n_r=16, n_theta=32, scheme=scheme,
                   potential=pot)
    st = ps.DSStepper(n, p.h, alpha=1.0, beta=1.5, tau=p.tau, dtype=torch.float64, n_r=16, n_theta=32, tol=1e-12,
                      scheme=scheme, potential=pot)
    u = dev(initial(n, half, ky=0.4), torch.float64)
    loss, g, counts = st.loss_and_grad(u, steps, checkpoint_every=3)
    assert counts == {"forward_solves": 12, "recomputed_solves": 9, "adjoint_solves": 12}
    ref_loss, ref_g = D.loss_l4_gradient(u.cpu().numpy(), p, steps)
    assert abs(float(loss) - ref_loss) <= 1e-12 * ref_loss
    assert rel_linf(g.cpu().numpy(), ref_g) <= 1e-9
    st.close()


@pytest.mark.parametrize("dtype,bar", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_mass_is_conserved(ps, dtype, bar):
    print(f"case: mass over 100 steps 256^2 {dtype}", flush=True)
    n, half = 256, 8.0
    st = ps.DSStepper(n, 2 * half / n, alpha=1.0, beta=1.0, tau=1e-3, dtype=dtype, tol=TOL[dtype])
    u = dev(initial(n, half, kx=1.0), dtype)
    m0 = float(st.moments(u)[0])
    st.forward(u, 100)
    m1 = float(st.moments(u)[0])
    ref = 2 * half / n
    exact = ref ** 2 * float(np.sum(np.abs(u.cpu().numpy().astype(np.complex128)) ** 2))
    assert abs(m1 - exact) <= 1e-12 * exact       # the reduction itself
    print(f"mass drift {abs(m1 - m0) / m0:.3e}", flush=True)
    assert abs(m1 - m0) <= bar * m0
    st.close()


@pytest.mark.parametrize("dtype,bar", [(torch.float64, 1e-9), (torch.float32, 1e-4)])
def test_checkpointed_gradient_matches_oracle_reverse_pass(ps, dtype, bar):
    print(f"case: L4 gradient 32^2 6 steps {dtype}", flush=True)
    n, half, steps = 32, 4.0, 6
    p = D.DSParams(n=n, h=2 * half / n, alpha=1.0, beta=1.5, tau=2e-2, n_r=16, n_theta=32)
    u0 = initial(n, half, ky=0.4)
    st = ps.DSStepper(n, p.h, alpha=1.0, beta=1.5, tau=p.tau, dtype=dtype, n_r=16, n_theta=32, tol=TOL[dtype])
    u = dev(u0, dtype)
    u_used = u.cpu().numpy().astype(np.complex128)
    loss, g, counts = st.loss_and_grad(u, steps, checkpoint_every=4)   # segments of 4 and 2 steps
    assert counts == {"forward_solves": 6, "recomputed_solves": 4, "adjoint_solves": 6}
    ref_loss, ref_g = D.loss_l4_gradient(u_used, p, steps)
    lerr = abs(float(loss) - ref_loss) / ref_loss
    gerr = rel_linf(g.cpu().numpy(), ref_g)
    print(f"loss rel err {lerr:.3e}, gradient rel L-inf {gerr:.3e}", flush=True)
    assert lerr <= bar and gerr <= bar
    st.close()


@pytest.mark.parametrize("dtype,bar", [(torch.float64, 1e-13), (torch.float32, 1e-6)])
def test_zero_steps(ps, dtype, bar):
    """The degenerate run of zero steps: the forward leaves the field bit for
    bit, and the loss and gradient are those of the field itself
    (J = h^2 sum |u0|^4, dJ/du0 = 4 h^2 |u0|^2 u0), with no solves counted."""
    print(f"case: stepper zero steps 32^2 {dtype}", flush=True)
    n, half = 32, 4.0
    p = D.DSParams(n=n, h=2 * half / n, alpha=1.0, beta=1.0, tau=1e-2, n_r=16, n_theta=32)
    st = ps.DSStepper(n, p.h, alpha=1.0, beta=1.0, tau=p.tau, dtype=dtype, n_r=16, n_theta=32, tol=TOL[dtype])
    u = dev(initial(n, half, ky=0.4), dtype)
    before = u.clone()
    st.forward(u, 0)
    assert torch.equal(u, before)
    u_used = u.cpu().numpy().astype(np.complex128)
    loss, g, counts = st.loss_and_grad(u, 0, checkpoint_every=4)
    assert counts == {"forward_solves": 0, "recomputed_solves": 0, "adjoint_solves": 0}
    ref_loss, ref_g = D.loss_l4_gradient(u_used, p, 0)
    assert abs(float(loss) - ref_loss) / ref_loss <= bar
    assert rel_linf(g.cpu().numpy(), ref_g) <= bar
    st.close()


def test_gradient_against_central_differences(ps):
    print("case: L4 gradient FD 64^2 FP64", flush=True)
    n, half, steps = 64, 4.0, 5
    st = ps.DSStepper(n, 2 * half / n, alpha=1.0, beta=1.0, tau=1e-2, dtype=torch.float64,
                      n_r=32, n_theta=64, tol=1e-12)
    u0 = dev(initial(n, half, kx=0.5), torch.float64)
    _, g, _ = st.loss_and_grad(u0, steps, checkpoint_every=2)
    gh = g.cpu().numpy()
    rng = np.random.default_rng(31)
    eps = 1e-4

    def loss(u):
        w = u.clone()
        st.forward(w, steps)
        return float(st.moments(w)[1])

    for _ in range(3):
        d = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        dd = dev(d, torch.float64)
        fd = (loss(u0 + eps * dd) - loss(u0 - eps * dd)) / (2 * eps)
        dot = float(np.sum(np.real(np.conj(gh) * d)))
        assert abs(fd - dot) <= 1e-6 * abs(dot), (fd, dot)
    st.close()


def test_autograd_function_matches_loss_and_grad(ps):
    print("case: DSEvolve autograd 64^2 FP64", flush=True)
    n, half, steps = 64, 4.0, 7
    st = ps.DSStepper(n, 2 * half / n, alpha=-1.0, beta=1.0, tau=1e-2, dtype=torch.float64,
                      n_r=32, n_theta=64, tol=1e-12)
    u0 = dev(initial(n, half), torch.float64)
    loss, g, _ = st.loss_and_grad(u0, steps, checkpoint_every=3)
    x = u0.clone().requires_grad_(True)
    u_t = ps.ds_evolve(x, st, steps, 3)
    j = (2 * half / n) ** 2 * torch.sum(torch.abs(u_t) ** 4)
    j.backward()
    assert abs(float(j.detach()) - float(loss)) <= 1e-13 * float(loss)
    # the same kernels; only the final loss gradient 4 h^2 |u|^2 u comes from torch here
    assert rel_linf(x.grad.cpu().numpy(), g.cpu().numpy()) <= 1e-13
    st.close()


def test_graph_replay_of_steps_matches_eager(ps):
    print("case: stepper graph replay 128^2 FP32", flush=True)
    n, half = 128, 8.0
    st = ps.DSStepper(n, 2 * half / n, tau=1e-3, dtype=torch.float32, tol=1e-7)
    u0 = dev(initial(n, half, kx=1.0), torch.float32)
    eager = u0.clone()
    st.forward(eager, 5)
    ref = eager.cpu().numpy()
    u = u0.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        st.forward(u, 5)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        st.forward(u, 5)
    for _ in range(3):
        u.copy_(u0)
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), ref)
        w = u0.clone()
        st.forward(w, 5)
        torch.cuda.synchronize()
    st.close()


def test_stepper_argument_errors(ps):
    from paper_1409_2014_amd import _binding as B
    print("case: stepper argument errors", flush=True)
    with pytest.raises(B.PhiError, match="PHI_ERR_UNSUPPORTED"):
        ps.DSStepper(8, 0.5)
    st = ps.DSStepper(32, 0.25, n_r=16, n_theta=32)
    g = dev(initial(32, 4.0), torch.float64)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = B.lib().phi_ds_backward(st._handle, ctypes.c_void_p(g.data_ptr()), 3, None, None, s)
    assert B.STATUS_NAMES[rc] == "PHI_ERR_INVALID_ARG"
    with pytest.raises(ValueError):
        st.forward(g.to(torch.complex64), 1)
    st.close()


# --------------------------------------------------------------------------
# the full stepper workload: 2048^2 over [-32, 32)^2, u0 = exp(-(x^2 + 2 y^2)),
# alpha = beta = 1, tau = 1e-3, 500 Strang steps, checkpoints every 50
# --------------------------------------------------------------------------

def full_initial():
    x, y, _ = W.grid_2d(2048, 32.0)
    return np.exp(-(x ** 2 + 2 * y ** 2)).astype(np.complex128)


def test_full_size_steps_match_oracle(ps):
    """Two steps at the full size, in the configuration the benchmark times,
    against the oracle stepper (split potential by direct sums)."""
    print("case: stepper 2048^2 2 steps FP64 vs oracle", flush=True)
    n, half = 2048, 32.0
    p = D.DSParams(n=n, h=2 * half / n, alpha=1.0, beta=1.0, tau=1e-3, n_r=64, n_theta=128)
    st = ps.DSStepper(n, p.h, alpha=1.0, beta=1.0, tau=p.tau, dtype=torch.float64, tol=1e-12)
    u = dev(full_initial(), torch.float64)
    u_used = u.cpu().numpy()
    st.forward(u, 2)
    err = rel_linf(u.cpu().numpy(), D.evolve(u_used, p, 2))
    print(f"rel L-inf after 2 steps: {err:.3e}", flush=True)
    assert err <= 1e-10
    st.close()


@pytest.mark.parametrize("dtype,mass_bar", [(torch.float64, 1e-12), (torch.float32, 1e-4)])
def test_full_size_run_invariants(ps, dtype, mass_bar):
    """500 steps at the full size: mass conservation; the checkpointed loss and
    gradient do not depend on the checkpoint interval beyond rounding; and, in
    FP64, the gradient against a central difference of the loss along one
    random direction."""
    print(f"case: stepper 2048^2 500 steps invariants {dtype}", flush=True)
    n, half, steps = 2048, 32.0, 500
    st = ps.DSStepper(n, 2 * half / n, alpha=1.0, beta=1.0, tau=1e-3, dtype=dtype, tol=TOL[dtype])
    u0 = dev(full_initial(), dtype)
    w = u0.clone()
    m0 = float(st.moments(w)[0])
    st.forward(w, steps)
    drift = abs(float(st.moments(w)[0]) - m0) / m0
    print(f"mass drift over {steps} steps: {drift:.3e}", flush=True)
    assert drift <= mass_bar
    loss50, g50, counts = st.loss_and_grad(u0, steps, checkpoint_every=50)
    assert counts["forward_solves"] == 500 and counts["recomputed_solves"] == 450
    assert counts["adjoint_solves"] == 500
    loss100, g100, _ = st.loss_and_grad(u0, steps, checkpoint_every=100)
    # the runs merge the linear substeps of consecutive steps except across
    # segment ends, which differ between the intervals and from the plain
    # forward run: equal to rounding
    lbar, gbar = (1e-12, 1e-9) if dtype == torch.float64 else (1e-5, 1e-3)
    assert abs(float(loss50) - float(loss100)) <= lbar * float(loss50)
    assert rel_linf(g100.cpu().numpy(), g50.cpu().numpy()) <= gbar
    assert abs(float(loss50) - float(st.moments(w)[1])) <= lbar * float(loss50)
    if dtype == torch.float64:
        rng = np.random.default_rng(77)
        d = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        dd = dev(d, dtype)
        eps = 1e-4

        def loss(u):
            v = u.clone()
            st.forward(v, steps)
            return float(st.moments(v)[1])

        fd = (loss(u0 + eps * dd) - loss(u0 - eps * dd)) / (2 * eps)
        dot = float(np.sum(np.real(np.conj(g50.cpu().numpy()) * d)))
        print(f"FD {fd:.10e} adjoint {dot:.10e}", flush=True)
        assert abs(fd - dot) <= 1e-6 * abs(dot)
    st.close()
