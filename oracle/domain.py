"""Average domain size of the two-fluid phase field (TEST INFRASTRUCTURE ONLY).

Plain numpy FP64 transcription of the paper's domain-size measure (Sec. 4,
Eq. Cluster_L_eq): L(t) = 2 pi int S(k) dk / int k S(k) dk, where S(k) is the
structure factor |phi'(k)|^2 of the order-parameter fluctuations
phi' = phi - <phi>, phi = (rho_A - rho_B) / (rho_A + rho_B), averaged over
spherical shells of radius k = |k|. Only tests may import this module.

Readings (where the paper leaves the discrete form open):
* phi is defined on fluid nodes; <phi> is its mean over them, and phi' is 0
  on solid nodes.
* Wave vectors are k_d = 2 pi m_d / L_d with integer m_d of the discrete
  Fourier transform (|m_d| <= L_d / 2). Shells have width dk = 2 pi / min(L)
  and shell s collects the modes with round(|k| / dk) = s, halves rounded
  up; the integrals run over the fully populated shells 1 <= s <= min(L) // 2,
  as sums with the shell means S(s) = mean of |phi'(k)|^2 / N over the modes
  of shell s.
* In boxes of unequal sides |k| / dk can be exactly half-integral, so the
  rounding is decided in integers (see shells), not in floating point.
"""
from __future__ import annotations

import math

import numpy as np


def order_parameter(rho: np.ndarray, fluid: np.ndarray) -> np.ndarray:
    """phi' = phi - <phi>_fluid on fluid nodes, 0 on solid nodes (node order
    x fastest); rho is [2][N]."""
    phi = np.zeros(rho.shape[1])
    phi[fluid] = (rho[0, fluid] - rho[1, fluid]) / (rho[0, fluid] + rho[1, fluid])
    out = np.zeros_like(phi)
    out[fluid] = phi[fluid] - phi[fluid].mean()
    return out


def shells(shape):
    """(shell index of every mode [nz][ny][nx], dk, s_max) for a box (nx, ny, nz).

    With A = lcm(L_d) and a_d = A / L_d, |k| / dk = Lmin sqrt(Q) / A where
    Q = sum_d (m_d a_d)^2 is an integer, and round-half-up of |k| / dk is the
    largest s >= 0 with (2s - 1)^2 A^2 <= 4 Lmin^2 Q, checked in exact
    integers around a floating-point first guess."""
    nx, ny, nz = shape
    A = math.lcm(nx, ny, nz)
    Lmin = min(shape)
    m = [np.rint(np.fft.fftfreq(n) * n).astype(np.int64) for n in (nx, ny, nz)]
    mz, my, mx = np.meshgrid(m[2], m[1], m[0], indexing="ij")
    Q = ((mx * (A // nx)).astype(object) ** 2 + (my * (A // ny)).astype(object) ** 2
         + (mz * (A // nz)).astype(object) ** 2)
    s = np.floor(Lmin * np.sqrt(Q.astype(np.float64)) / A + 0.5).astype(np.int64)
    rhs = 4 * Lmin * Lmin * Q
    so = s.astype(object)
    up = (2 * so + 1) ** 2 * (A * A) <= rhs          # s + 1 still satisfies the bound
    so = np.where(up, so + 1, so)
    down = (so > 0) & ((2 * so - 1) ** 2 * (A * A) > rhs)
    so = np.where(down, so - 1, so)
    return so.astype(np.int64), 2 * np.pi / Lmin, Lmin // 2


def structure_factor(phi_prime: np.ndarray, shape):
    """Shell means S(s) of |phi'(k)|^2 / N for s = 0..s_max, and the mode
    counts of each shell."""
    nx, ny, nz = shape
    F = np.fft.fftn(phi_prime.reshape(nz, ny, nx))
    S = (F.real ** 2 + F.imag ** 2) / phi_prime.size
    s, dk, smax = shells(shape)
    sums = np.bincount(s.ravel(), weights=S.ravel(), minlength=smax + 1)[:smax + 1]
    counts = np.bincount(s.ravel(), minlength=smax + 1)[:smax + 1]
    mean = np.where(counts > 0, sums / np.maximum(counts, 1), 0.0)
    return mean, counts, dk


def domain_size(rho: np.ndarray, fluid: np.ndarray, shape):
    """(L, S(s) for s = 0..s_max) of Eq. Cluster_L_eq; L is nan when phi' = 0."""
    S, counts, dk = structure_factor(order_parameter(rho, fluid), shape)
    s = np.arange(S.size)
    use = (s >= 1) & (counts > 0)
    num = S[use].sum()
    den = (s[use] * dk * S[use]).sum()
    return (2 * np.pi * num / den if den > 0 else float("nan")), S
