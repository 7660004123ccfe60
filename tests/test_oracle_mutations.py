"""The pins must catch plausible mistakes.  Each case plants one mistake in the
oracle (CPU only, via monkeypatch) and checks that at least one pin fails:
the closed form of the small Gaussian case, the printed Arkadiev error of
Table 5 (L = 16, h = 1/4) and the Phi_xx + Phi_yy = -rho invariant."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import closed_forms as C
from oracle import split_solver as S
import workloads as W


def _pins_hold():
    p = O.SplitParams(n=64, h=0.25, n_r=32, n_theta=64)
    x, y, _ = W.grid_2d(64, 8.0)
    ok_gauss = np.max(np.abs(O.phi(W.gaussian_density(64, 8.0), p) - C.phi_isotropic_gaussian(x, y))) < 1e-11

    p = O.SplitParams(n=128, h=0.25, n_r=64, n_theta=128)
    x, y, _ = W.grid_2d(128, 16.0)
    ex = C.phi_arkadiev(x, y)
    err = np.max(np.abs(O.phi(W.arkadiev_density(128, 16.0), p) - ex)) / np.max(np.abs(ex))
    ok_table = abs(err - 4.28e-6) < 0.03 * 4.28e-6

    spec = W.draw_mixture(4, 4, 3.0, (0.6, 1.4))
    rho = W.mixture_density(64, 8.0, spec)
    px = O.SplitParams(n=64, h=0.25, n_r=64, n_theta=128)
    py = O.SplitParams(n=64, h=0.25, n_r=64, n_theta=128, component="yy")
    ok_sum = np.max(np.abs(O.phi(rho, px) + O.phi(rho, py) + rho)) < 1e-12 * rho.max()
    return ok_gauss and ok_table and ok_sum


def test_unmodified_oracle_passes_the_pins():
    assert _pins_hold()


def _drop_i2(monkeypatch):
    monkeypatch.setattr(S, "i2_direct", lambda rho, p, return_imag=False:
                        (np.zeros_like(rho), np.zeros_like(rho)) if return_imag else np.zeros_like(rho))


def _wrong_phase_sign_type2(monkeypatch):
    orig = S.type2_direct
    monkeypatch.setattr(S, "type2_direct", lambda rho, h, xs, kx, ky: orig(rho, h, xs, -kx, -ky))


def _transposed_density_type2(monkeypatch):
    orig = S.type2_direct
    monkeypatch.setattr(S, "type2_direct", lambda rho, h, xs, kx, ky: orig(rho.T, h, xs, kx, ky))


def _missing_h2(monkeypatch):
    orig = S.type2_direct
    monkeypatch.setattr(S, "type2_direct", lambda rho, h, xs, kx, ky: orig(rho, 1.0, xs, kx, ky))


def _dropped_jacobian(monkeypatch):
    orig = S.polar_nodes_weights

    def bad(p):
        r, w_r, th, w_t = orig(p)
        return r, w_r / r, th, w_t
    monkeypatch.setattr(S, "polar_nodes_weights", bad)


def _sin_for_cos(monkeypatch):
    orig = S.polar_rule

    def bad(p):
        flipped = O.SplitParams(p.n, p.h, p.n_r, p.n_theta, p.kappa, p.sigma, p.cutoff,
                                p.eps_split, "yy" if p.component == "xx" else "xx")
        kx, ky, _ = orig(p)
        _, _, q = orig(flipped)
        return kx, ky, q
    monkeypatch.setattr(S, "polar_rule", bad)


def _partition_not_complement(monkeypatch):
    def bad(kx, ky, sigma, component="xx", partition="gauss"):
        k2 = kx * kx + ky * ky
        num = kx * kx if component == "xx" else ky * ky
        out = np.zeros_like(k2)
        nz = k2 > 0
        out[nz] = -(num[nz] / k2[nz]) * np.exp(-k2[nz] / sigma ** 2)
        return out
    monkeypatch.setattr(S, "highfreq_multiplier", bad)


def _wrong_frequency_scale(monkeypatch):
    # frequencies of I1 computed on the unpadded box (k_m = m/(N h))
    def bad(p):
        k = np.fft.fftfreq(p.kappa * p.n, d=p.h) * p.kappa
        ky, kx = np.meshgrid(k, k, indexing="ij")
        return kx, ky
    monkeypatch.setattr(S, "_padded_frequencies", bad)


@pytest.mark.parametrize("plant", [
    _drop_i2, _wrong_phase_sign_type2, _transposed_density_type2, _missing_h2,
    _dropped_jacobian, _sin_for_cos, _partition_not_complement, _wrong_frequency_scale,
])
def test_planted_mistake_is_caught(monkeypatch, plant):
    plant(monkeypatch)
    assert not _pins_hold()
