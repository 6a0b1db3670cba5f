"""Pins of the oracle's domain-size measure (Eq. Cluster_L_eq) against closed
forms and invariants: a single Fourier mode, Parseval's identity, and
invariance under translation and under adding a constant to phi."""
import numpy as np

from oracle import domain as D


def _rho_from_phi(phi):
    # rho_A - rho_B = phi (rho_A + rho_B) with rho_A + rho_B = 2
    return np.stack([1.0 + phi, 1.0 - phi])


def _mode(shape, m):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return 0.5 * np.cos(2 * np.pi * (m[0] * x / nx + m[1] * y / ny + m[2] * z / nz)).ravel()


def test_single_mode_gives_box_over_wavenumber():
    # |m| = 5 (3, 4, 0): one shell, L = 2 pi / k = 40 / 5 = 8 exactly
    shape = (40, 40, 40)
    phi = _mode(shape, (3, 4, 0))
    fluid = np.ones(phi.size, bool)
    L, S = D.domain_size(_rho_from_phi(phi), fluid, shape)
    assert abs(L - 8.0) < 1e-12
    assert np.count_nonzero(S > 1e-20) == 1 and S[5] > 0


def test_parseval():
    shape = (12, 10, 8)
    rng = np.random.default_rng(1)
    phi = 0.3 * rng.standard_normal(np.prod(shape))
    fluid = rng.random(phi.size) > 0.2
    pp = D.order_parameter(_rho_from_phi(np.clip(phi, -0.9, 0.9)), fluid)
    F = np.fft.fftn(pp.reshape(shape[::-1]))
    assert abs((np.abs(F) ** 2).sum() / pp.size - (pp ** 2).sum()) < 1e-10 * (pp ** 2).sum()
    S, counts, _ = D.structure_factor(pp, shape)
    # every mode of the fully populated shells is counted once
    s, _, smax = D.shells(shape)
    assert counts.sum() == np.count_nonzero(s <= smax)
    assert np.allclose((S * counts).sum(), (np.abs(F) ** 2)[s <= smax].sum() / pp.size)


def test_translation_and_offset_invariance():
    shape = (16, 12, 10)
    rng = np.random.default_rng(2)
    phi = np.tanh(3 * rng.standard_normal(np.prod(shape)))
    fluid = np.ones(phi.size, bool)
    L0, S0 = D.domain_size(_rho_from_phi(0.9 * phi), fluid, shape)
    shifted = np.roll((0.9 * phi).reshape(shape[::-1]), (3, 5, 7), axis=(0, 1, 2)).ravel()
    L1, S1 = D.domain_size(_rho_from_phi(shifted), fluid, shape)
    assert abs(L1 - L0) < 1e-12 * L0 and np.allclose(S1, S0, rtol=1e-10, atol=1e-14)
    L2, _ = D.domain_size(_rho_from_phi(0.9 * phi * 0.5 + 0.2), fluid, shape)
    assert abs(L2 - L0) < 1e-10 * L0     # a constant shift and a scale leave L alone


def test_uniform_phase_has_no_structure():
    shape = (8, 8, 8)
    _, S = D.domain_size(_rho_from_phi(np.full(512, 0.3)), np.ones(512, bool), shape)
    assert S.max() < 1e-28   # only the rounding of the mean removal is left


def test_half_integral_radius_rounds_up():
    # 48 x 40 x 36: the mode m = (2, 0, 0) has |k| / dk = 36 * 2 / 48 = 1.5 exactly,
    # m = (0, 0, 5) has 5 and m = (6, 5, 0) has 36 sqrt(1/64 + 1/64) = 6.36...
    s, dk, smax = D.shells((48, 40, 36))
    assert s[0, 0, 2] == 2 and s[0, 0, 46] == 2
    assert s[5, 0, 0] == 5
    assert s[0, 5, 6] == 6
    assert smax == 18 and abs(dk - 2 * np.pi / 36) < 1e-15
