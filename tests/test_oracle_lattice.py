"""Pins of the oracle's lattice tables and equilibrium (Sec. 2.1, Eq. LEQ).

The checks are the textbook moment identities of D3Q19 and of the
second-order equilibrium; a wrong weight, vector or sign in the oracle's
tables or in f_eq breaks one of them.
"""
import itertools

import numpy as np
import pytest

import oracle as O

CS2 = 1.0 / 3.0


def test_d3q19_set_and_weights():
    c, w = O.lattice()
    # 1 rest, 6 of length 1, 12 of length sqrt(2), all distinct
    n2 = (c ** 2).sum(1)
    assert sorted(n2.tolist()) == [0] + [1] * 6 + [2] * 12
    assert len({tuple(v) for v in c}) == 19
    assert np.allclose(w[n2 == 0], 1 / 3) and np.allclose(w[n2 == 1], 1 / 18)
    assert np.allclose(w[n2 == 2], 1 / 36)
    # closed under inversion
    s = {tuple(v) for v in c}
    assert all(tuple(-v) in s for v in c)


def test_lattice_isotropy():
    c, w = O.lattice()
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(w @ c).max() < 1e-16
    M2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(M2, CS2 * np.eye(3), atol=1e-16)
    M3 = np.einsum("i,ia,ib,ic->abc", w, c, c, c)
    assert np.abs(M3).max() < 1e-16
    M4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(M4, iso, atol=1e-16)


@pytest.mark.parametrize("rho,u", [(1.0, (0.0, 0.0, 0.0)), (1.3, (0.05, -0.02, 0.01)),
                                   (0.7, (-0.1, 0.03, 0.08))])
def test_equilibrium_moments(rho, u):
    """sum f_eq = rho, sum f_eq c = rho u, sum f_eq c c = rho cs2 I + rho u u."""
    p = O.Params(1, 1, 1, ncomp=1, tau=(1.0,))
    o = O.Oracle(p, np.array([[rho]]), np.array([u]))
    f = o.f()[0, :, 0]
    c, _ = O.lattice()
    u = np.array(u)
    assert abs(f.sum() - rho) < 1e-15
    assert np.abs(f @ c - rho * u).max() < 1e-16
    P = np.einsum("i,ia,ib->ab", f, c, c)
    assert np.abs(P - (rho * CS2 * np.eye(3) + rho * np.outer(u, u))).max() < 1e-15
