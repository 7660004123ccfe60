"""CPU tests of the C-ABI library: it loads, exports every declared symbol, and
its host-side plan logic (quadrature, kernel transform, parameter readings,
error codes) is right.  No GPU calls."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O

from conftest import ROOT

B = pytest.importorskip("paper_1409_2014_amd._binding")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail(f"library not built: {B.LIB_PATH} (run python -m paper_1409_2014_amd.build_lib)")
    return B.lib()


def declared_functions():
    names = set()
    for header in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if header.endswith(".h"):
            with open(os.path.join(ROOT, "include", header)) as f:
                text = f.read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(phi_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 15
    raw = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing
    assert set(B.exported_symbols()) <= set(names)


def test_status_strings(lib):
    for code, name in B.STATUS_NAMES.items():
        assert lib.phi_status_string(code).decode() == name


def test_gauss_legendre_matches_numpy(lib):
    import paper_1409_2014_amd.solver as S
    for n in (1, 2, 5, 32, 64, 127, 512):
        x, w = S.host_gauss_legendre(n)
        xr, wr = np.polynomial.legendre.leggauss(n)
        assert np.max(np.abs(x - xr)) < 2e-15
        # numpy's endpoint weights drift from the exact ones by up to ~1e-10
        # relative at n = 512 (checked against 40-digit values); the exactness
        # test below pins this rule independently
        assert np.max(np.abs(w - wr) / wr) < 1e-9
    for n in (3, 16, 64):
        x, w = S.host_gauss_legendre(n)
        for k in range(0, 2 * n, 2):
            assert abs(np.sum(w * x ** k) - 2.0 / (k + 1)) < 1e-14


def test_es_transform_against_adaptive_quadrature(lib):
    from scipy import integrate
    import paper_1409_2014_amd.solver as S
    for beta in (2.30 * 8, 2.30 * 13):
        omegas = np.array([0.0, 0.7, 3.1, 9.0])
        got = S.host_es_transform(omegas, beta)
        for om, g in zip(omegas, got):
            # z = sin t removes the square-root endpoints: a smooth integrand on [-pi/2, pi/2]
            ref = integrate.quad(lambda t: math.exp(beta * (math.cos(t) - 1)) * math.cos(om * math.sin(t)) * math.cos(t),
                                 -math.pi / 2, math.pi / 2, limit=200, epsabs=1e-15, epsrel=1e-13)[0]
            assert abs(g - ref) < 1e-13 * max(1.0, abs(ref))
        z = np.array([-1.0, -0.5, 0.0, 0.3, 1.0, 1.5])
        k = S.host_es_kernel(z, beta)
        assert k[2] == 1.0 and k[0] == 0.0 and k[4] == 0.0 and k[5] == 0.0
        assert abs(k[1] - math.exp(beta * (math.sqrt(0.75) - 1))) < 1e-15


def test_plan_nodes_equal_the_oracle_rule(lib):
    import paper_1409_2014_amd.solver as S
    for comp, ocomp in (("x", "xx"), ("y", "yy"), ("xy", "xy")):
        kx, ky, q = S.host_polar_nodes(n=64, h=0.25, n_r=32, n_theta=64, component=comp)
        okx, oky, oq = O.polar_rule(O.SplitParams(n=64, h=0.25, n_r=32, n_theta=64, component=ocomp))
        a = np.stack([kx, ky, q], 1)
        b = np.stack([okx, oky, oq], 1)
        a = a[np.lexsort((a[:, 1], a[:, 0]))]
        b = b[np.lexsort((b[:, 1], b[:, 0]))]
        assert np.max(np.abs(a - b)) < 1e-15


def test_describe_defaults_small_case(lib):
    import paper_1409_2014_amd.solver as S
    d = S.describe(n=64, h=0.25, n_r=32, n_theta=64, tol=1e-12)
    assert d["n_fine"] == 128 and d["n_nodes"] == 2048
    assert abs(d["sigma"] - 0.120753014) < 1e-8
    assert abs(d["cutoff"] - 0.732935599) < 1e-8
    assert d["kernel_width"] == 13 and abs(d["beta"] - 29.9) < 1e-12
    # nodes reach n_fine h c = 23.45 cells; window covers them plus half a kernel
    assert d["patch"] == 64 and d["patch_lo"] == -32
    d = S.describe(n=2048, h=1 / 64, dtype="float32")
    assert d["kernel_width"] == 8 and d["patch"] == 64 and d["n_nodes"] == 8192


def test_describe_gaussian_gridding(lib):
    """Greengard-Lee gridding at oversampling 2: half-width M = ceil(1.5 ln(1/tol)/pi)
    cells, Gaussian exp(-(3 pi/(4 M)) t^2); the wider kernel widens the window."""
    import paper_1409_2014_amd.solver as S
    for tol, m in ((1e-12, 14), (1e-7, 8), (1e-3, 4)):
        d = S.describe(n=256, h=1 / 16, tol=tol, kernel="gaussian")
        assert d["kernel_width"] == 2 * m == 2 * math.ceil(1.5 * math.log(1 / tol) / math.pi)
        assert abs(d["beta"] - 0.75 * math.pi / m) < 1e-15
        assert d["tile"] == d["bin"] + 2 * m - 1
        # the window holds every tap: n_fine h c + M cells from the origin
        assert d["patch"] // 2 >= math.ceil(2 * 256 / 16 * d["cutoff"] + m) + 1
    with pytest.raises(B.PhiError) as exc:
        S.describe(n=256, h=1 / 16, tol=1e-14, kernel="gaussian")
    assert exc.value.status == 2
    with pytest.raises(B.PhiError) as exc:
        S.describe(n=256, h=1 / 16, tol=1e-12, kernel="gaussian", bin=8)
    assert exc.value.status == 2


def test_describe_small_grid_uses_whole_fine_grid(lib):
    import paper_1409_2014_amd.solver as S
    d = S.describe(n=16, h=1.0)
    assert d["patch"] == d["n_fine"] == 32


@pytest.mark.parametrize("kwargs,status", [
    (dict(n=64, h=0.25, n_theta=63), 1),            # odd azimuthal count
    (dict(n=64, h=-1.0), 1),                        # negative spacing
    (dict(n=61, h=0.25), 1),                        # odd grid side
    (dict(n=6, h=0.25), 2),                         # below 8 points per side
    (dict(n=8192, h=0.25), 2),                      # padded side above 8192
    (dict(n=4098, h=0.25), 2),
    (dict(n=2800, h=0.25, pad=3), 2),
    (dict(n=64, h=0.25, tol=1e-9, dtype="float32"), 3),
    (dict(n=64, h=0.25, tol=1e-16), 3),
    (dict(n=64, h=0.25, pad=9), 2),                 # kappa above 8
    (dict(n=64, h=0.25, pad=1), 1),
    (dict(n=64, h=0.25, bin=5), 1),                 # bin side not in {4, 8, 16}
    (dict(n=64, h=0.25, sub_nodes=65), 1),          # more nodes per block than the LDS holds
    (dict(n=64, h=0.25, sub_nodes=4), 1),
])
def test_invalid_parameters_return_documented_codes(lib, kwargs, status):
    import paper_1409_2014_amd.solver as S
    with pytest.raises(B.PhiError) as exc:
        S.describe(**kwargs)
    assert exc.value.status == status


def test_component_flags_exclude_each_other(lib):
    import paper_1409_2014_amd.solver as S
    p = S.make_params(64, 0.25, component="xy")
    p.flags |= B.PHI_COMPONENT_Y
    info = B.PhiPlanInfo()
    assert lib.phi_describe(ctypes.byref(p), ctypes.byref(info)) == 1
    with pytest.raises(ValueError):
        S.make_params(64, 0.25, component="yx")


def test_null_and_destroyed_plans_are_rejected(lib):
    st = lib.phi_solve(None, ctypes.c_void_p(1), ctypes.c_void_p(2), None)
    assert st == 1
    assert lib.phi_destroy(None) == 0
    assert b"plan" in lib.phi_last_error(None)
    info = B.PhiPlanInfo()
    assert lib.phi_plan_get_info(ctypes.c_void_p(12345), ctypes.byref(info)) == 1


def test_nonsquare_grid_is_unsupported(lib):
    p = B.PhiParams()
    assert lib.phi_params_default(ctypes.byref(p), 64, 0.25, 0) == 0
    p.ny = 32
    info = B.PhiPlanInfo()
    assert lib.phi_describe(ctypes.byref(p), ctypes.byref(info)) == 2
    p.ny = 64
    p.hy = 0.5
    assert lib.phi_describe(ctypes.byref(p), ctypes.byref(info)) == 2


@pytest.mark.parametrize("bin_side,sub_nodes", [(4, 32), (8, 64), (16, 64), (16, 8)])
def test_node_sort_follows_the_bin_of_the_first_tap(lib, bin_side, sub_nodes):
    """Plan order groups the nodes by the bin of their first kernel tap (bin
    index non-decreasing), every block holds at most sub_nodes nodes, and the
    spread tile is bin + w - 1 cells wide."""
    import paper_1409_2014_amd.solver as S
    kw = dict(n=256, h=1 / 16, n_r=32, n_theta=64, tol=1e-7, dtype="float32", bin=bin_side,
              sub_nodes=sub_nodes)
    d = S.describe(**kw)
    w, q, lo, nf, h = d["kernel_width"], d["patch"], d["patch_lo"], d["n_fine"], d["h"]
    assert d["bin"] == bin_side and d["sub_nodes"] == sub_nodes
    assert d["tile"] == bin_side + w - 1
    kx, ky, _ = S.host_polar_nodes(**kw)
    cx = np.ceil(nf * h * kx - 0.5 * w).astype(int) - lo
    cy = np.ceil(nf * h * ky - 0.5 * w).astype(int) - lo
    assert cx.min() >= 0 and cx.max() + w <= q and cy.min() >= 0 and cy.max() + w <= q
    nb = q // bin_side
    key = (cy // bin_side) * nb + cx // bin_side
    assert np.all(np.diff(key) >= 0)
    counts = np.bincount(key)
    assert d["n_sub"] == int(np.sum((counts + sub_nodes - 1) // sub_nodes))
    assert d["max_cell_nodes"] == int(counts.max())


def test_plan_creation_without_a_device_fails_with_a_status(lib):
    """Without a usable GPU every constructor returns PHI_ERR_DEVICE and a
    message (never a crash); parameter errors are still found first."""
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    p = B.PhiParams()
    assert lib.phi_params_default(ctypes.byref(p), 128, 0.25, B.PHI_F32) == 0
    h = ctypes.c_void_p()
    assert lib.phi_plan(ctypes.byref(p), None, ctypes.byref(h)) == 5 and not h.value
    assert b"device" in lib.phi_last_error(None)
    arr = (B.PhiParams * 2)(p, p)
    assert lib.phi_plan_batch(arr, 2, None, ctypes.byref(h)) == 5 and not h.value
    assert lib.phi_plan_batch(arr, 0, None, ctypes.byref(h)) == 1
    opts = B.PhiDsOptions(1.0, 2.0, 4.0, 1e-3, 0, 0)
    assert lib.phi_ds_create(ctypes.byref(p), ctypes.byref(opts), None, ctypes.byref(h)) == 5 and not h.value
    small = B.PhiParams()
    assert lib.phi_params_default(ctypes.byref(small), 64, 0.25, B.PHI_F32) == 0
    arr2 = (B.PhiParams * 1)(small)
    assert lib.phi_plan_batch(arr2, 1, None, ctypes.byref(h)) == 2          # side below 128
    bad = B.PhiDsOptions(float("nan"), 2.0, 4.0, 1e-3, 0, 0)
    assert lib.phi_ds_create(ctypes.byref(small), ctypes.byref(bad), None, ctypes.byref(h)) == 1
    bad = B.PhiDsOptions(1.0, 2.0, 4.0, 1e-3, 7, 0)
    assert lib.phi_ds_create(ctypes.byref(small), ctypes.byref(bad), None, ctypes.byref(h)) == 1
    tiny = B.PhiParams()
    assert lib.phi_params_default(ctypes.byref(tiny), 8, 0.25, B.PHI_F64) == 0
    assert lib.phi_ds_create(ctypes.byref(tiny), ctypes.byref(opts), None, ctypes.byref(h)) == 2
    # entry points on handles that were never created
    assert lib.phi_ds_forward(ctypes.c_void_p(4321), ctypes.c_void_p(1), 1, None, None, None) == 1
    assert lib.phi_ds_destroy(None) == 0


@pytest.mark.parametrize("n", [1, 2, 5, 32, 64, 257, 1024])
def test_gauss_jacobi_rule_against_golub_welsch(lib, n):
    """The host Gauss-Jacobi(0, 1) rule against the eigenvalues of the Jacobi
    matrix of its orthogonal polynomials (Golub-Welsch), an independent route,
    and its defining exactness: sum_i w_i P_k(x_i) = int (1 + x) P_k(x) dx
    (2, 2/3, then 0) for every Legendre polynomial of degree k <= 2n - 1."""
    import paper_1409_2014_amd.solver as S
    x, w = S.host_gauss_jacobi01(n)
    # recurrence coefficients of the monic Jacobi(0, 1) polynomials
    k = np.arange(n, dtype=np.float64)
    a, b = 0.0, 1.0
    diag = (b * b - a * a) / ((2 * k + a + b) * (2 * k + a + b + 2))
    kk = np.arange(1, n, dtype=np.float64)
    off = np.sqrt(4 * kk * (kk + a) * (kk + b) * (kk + a + b)
                  / ((2 * kk + a + b) ** 2 * (2 * kk + a + b + 1) * (2 * kk + a + b - 1)))
    ev, vec = np.linalg.eigh(np.diag(diag) + np.diag(off, 1) + np.diag(off, -1))
    wref = 2.0 * vec[0, :] ** 2          # mu_0 = int (1 + x) dx = 2
    assert np.all(np.diff(x) > 0)
    assert np.max(np.abs(x - ev)) < 1e-13
    # eigenvector weights carry an error of a few n eps; the weights near
    # x = -1 vanish like (1 + x)
    big = wref > 1e-6 * np.max(wref)
    assert np.max(np.abs(w - wref)[big] / wref[big]) < 1e-10
    degrees = range(0, 2 * n) if n <= 64 else sorted({*range(8), *range(0, 2 * n, 97), 2 * n - 2, 2 * n - 1})
    for deg in degrees:
        c = np.zeros(deg + 1)
        c[deg] = 1.0
        expect = 2.0 if deg == 0 else (2.0 / 3.0 if deg == 1 else 0.0)
        assert abs(np.sum(w * np.polynomial.legendre.legval(x, c)) - expect) < 1e-13, deg


def test_plan_nodes_with_the_jacobi_rule_equal_the_oracle(lib):
    import paper_1409_2014_amd.solver as S
    kw = dict(n=64, h=0.25, n_r=24, n_theta=48, radial="jacobi")
    kx, ky, q = S.host_polar_nodes(**kw)
    okx, oky, oq = O.polar_rule(O.SplitParams(n=64, h=0.25, n_r=24, n_theta=48, radial="jacobi"))
    a = np.stack([kx, ky, q], axis=1)
    b = np.stack([okx, oky, oq], axis=1)
    # sort on rounded positions: angles evaluated in two ways differ in the last bit
    a = a[np.lexsort((np.round(a[:, 1], 10), np.round(a[:, 0], 10)))]
    b = b[np.lexsort((np.round(b[:, 1], 10), np.round(b[:, 0], 10)))]
    assert np.max(np.abs(a - b)) < 1e-15


@pytest.mark.parametrize("n,pad,fine", [(96, 2, 256), (384, 2, 1024), (1536, 2, 4096), (3072, 2, 8192),
                                        (10, 2, 32), (100, 3, 512), (2048, 3, 8192), (1024, 4, 4096),
                                        (64, 2, 128), (2730, 3, 8192)])
def test_padded_side_is_the_smallest_power_of_two_at_least_kappa_n(lib, n, pad, fine):
    """Any even grid side: the padded box of I1 (and the NUFFT fine grid) is the
    smallest power of two >= kappa N, and the default sigma follows the padding
    factor F / N of that box (Sec. 2.1 with kappa = F / N), as in the oracle."""
    import oracle as O
    import paper_1409_2014_amd.solver as S
    h = 1 / 32
    d = S.describe(n=n, h=h, pad=pad)
    assert d["n_fine"] == fine
    sigma, c = O.split_constants(O.SplitParams(n=n, h=h, n_r=8, n_theta=8, pad_side=fine))
    assert abs(d["sigma"] - sigma) <= 1e-14 * sigma
    assert abs(d["cutoff"] - c) <= 1e-14 * c


@pytest.mark.parametrize("partition", ["erfc", "gauss"])
def test_plan_nodes_for_coulomb_equal_the_oracle(lib, partition):
    """The Coulomb weights q_j = (c/2) w_i (2 pi/N_theta) p(r_i) as the plan builds
    them, against the oracle's rule (Sec. 2.1, Remark)."""
    import paper_1409_2014_amd.solver as S
    kx, ky, q = S.host_polar_nodes(n=64, h=0.25, n_r=24, n_theta=48, component="coulomb", partition=partition)
    okx, oky, oq = O.polar_rule(O.SplitParams(n=64, h=0.25, n_r=24, n_theta=48, component="coulomb",
                                              partition=partition))
    a = np.stack([kx, ky, q], axis=1)
    b = np.stack([okx, oky, oq], axis=1)
    a = a[np.lexsort((np.round(a[:, 1], 10), np.round(a[:, 0], 10)))]
    b = b[np.lexsort((np.round(b[:, 1], 10), np.round(b[:, 0], 10)))]
    assert np.max(np.abs(a - b)) <= 1e-15 * np.max(np.abs(b))


@pytest.mark.parametrize("flags", [
    lambda B: B.PHI_COMPONENT_COULOMB | B.PHI_COMPONENT_Y,
    lambda B: B.PHI_COMPONENT_COULOMB | B.PHI_COMPONENT_XY,
    lambda B: B.PHI_COMPONENT_COULOMB | B.PHI_RADIAL_JACOBI,
    lambda B: B.PHI_PARTITION_GAUSS,
])
def test_coulomb_flag_combinations_are_refused(lib, flags):
    import ctypes
    import paper_1409_2014_amd.solver as S
    from paper_1409_2014_amd import _binding as B
    p = S.make_params(n=64, h=0.25)
    p.flags = flags(B)
    info = B.PhiPlanInfo()
    assert lib.phi_describe(ctypes.byref(p), ctypes.byref(info)) == 1
