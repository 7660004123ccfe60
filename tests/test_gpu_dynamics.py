"""The paper's dynamics comparison (Sec. 3.2 Tables 7-10, Sec. 3.3 Tables 11-12)
reproduced by the GPU stepper: fourth-order splitting with the potential from
the standard periodic FFT solver or from the split (NUFFT) solver, relative l2
errors of u and Phi at the final time against the exact solution (H-E case I)
or against a reference run on [-64, 64)^2 at h = 1/8 (H-E case II, E-E).

Bar: within 1.5 % of every printed error above 1e-12 (three printed digits,
and the runs differ from the paper's in the NUFFT kernel, the radial rule and
the node counts, which move the potential by the last printed digit); at or
below 1e-12 the printed values sit at the paper's NUFFT accuracy, and the GPU
errors must be no larger."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_2014_amd as ps
    return ps


def lump(x, y, t):
    return 2 * np.exp(1j * (2 * y + 4 * t)) / ((x + 1) ** 2 + (y + 4 * t) ** 2 + 1)


def lump_phi(x, y, t):
    s = (x + 1) ** 2 + (y + 4 * t) ** 2 + 1
    return -2 * ((y + 4 * t) ** 2 - x * (x + 2)) / s ** 2


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# H-E: alpha = 1, beta = -1 (c_l = -2, c_p = -4); E-E: alpha = -1, chi = -1, gamma = 1 (c_l = 1, c_p = -1)
SYSTEMS = {"he": dict(alpha=1.0, c_local=-2.0, c_potential=-4.0, t_end=0.4, tau=1e-3),
           "ee": dict(alpha=-1.0, c_local=1.0, c_potential=-1.0, t_end=0.05, tau=1e-4)}


def run(ps, system, u0, half, h, pot):
    cfg = SYSTEMS[system]
    n = int(round(2 * half / h))
    st = ps.DSStepper(n, h, alpha=cfg["alpha"], c_local=cfg["c_local"], c_potential=cfg["c_potential"],
                      tau=cfg["tau"], dtype=torch.float64, scheme="yoshida4", potential=pot, tol=1e-12)
    u = torch.as_tensor(u0, dtype=torch.complex128, device="cuda").contiguous()
    st.forward(u, int(round(cfg["t_end"] / cfg["tau"])))
    rho = (u.real ** 2 + u.imag ** 2).contiguous()
    plan = ps.Plan(n, h, dtype=torch.float64, tol=1e-12)
    phi = (plan.periodic(rho) if pot == "periodic" else plan.solve(rho)).cpu().numpy()
    out = u.cpu().numpy()
    st.close()
    plan.close()
    return out, phi


def check(got, printed, what):
    if printed > 1e-12:
        assert abs(got - printed) <= 0.015 * printed, (what, got, printed)
    else:
        assert got <= printed, (what, got, printed)


@pytest.mark.parametrize("table,pot", [("table7_he_case1_fft.txt", "periodic"),
                                       ("table8_he_case1_nufft.txt", "split")])
def test_he_case1_exact_lump(ps, golden, table, pot):
    print(f"case: {table}", flush=True)
    for half, h, eu, ep in golden(table):
        n = int(round(2 * half / h))
        x, y, _ = W.grid_2d(n, half)
        u, phi = run(ps, "he", lump(x, y, 0.0), half, h, pot)
        check(rel_l2(u, lump(x, y, 0.4)), eu, (half, h, "u"))
        check(rel_l2(phi, lump_phi(x, y, 0.4)), ep, (half, h, "phi"))


@pytest.fixture(scope="module")
def references(ps):
    """Reference runs on [-64, 64)^2 at h = 1/8 with the split solver."""
    half, h = 64.0, 0.125
    n = int(round(2 * half / h))
    x, y, _ = W.grid_2d(n, half)
    return {"he": run(ps, "he", np.exp(-(x ** 2 + y ** 2) / 4), half, h, "split"),
            "ee": run(ps, "ee", 4 * np.exp(-(x ** 2 + y ** 2) / 4), half, h, "split")}


@pytest.mark.parametrize("table,system,amp,pot", [
    ("table9_he_case2_fft.txt", "he", 1.0, "periodic"), ("table10_he_case2_nufft.txt", "he", 1.0, "split"),
    ("table11_ee_fft.txt", "ee", 4.0, "periodic"), ("table12_ee_nufft.txt", "ee", 4.0, "split")])
def test_gaussian_cases_against_reference(ps, golden, references, table, system, amp, pot):
    print(f"case: {table}", flush=True)
    u_ref, phi_ref = references[system]
    for half, h, eu, ep in golden(table):
        n = int(round(2 * half / h))
        x, y, _ = W.grid_2d(n, half)
        u, phi = run(ps, system, amp * np.exp(-(x ** 2 + y ** 2) / 4), half, h, pot)
        # the reference grid (h = 1/8 on [-64, 64)) contains this grid's points
        ix = np.round((x[0] + 64.0) / 0.125).astype(int)
        sel = np.ix_(ix, ix)
        check(rel_l2(u, u_ref[sel]), eu, (half, h, "u"))
        check(rel_l2(phi, phi_ref[sel]), ep, (half, h, "phi"))
