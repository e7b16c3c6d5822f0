"""Tiny dense brute-force SHT -- TEST INFRASTRUCTURE ONLY.

Builds the synthesis and analysis of Schaeffer (arXiv 1202.6522, Sec. 2.2 and
2.3) as explicit dense real matrices from scipy's spherical harmonics
(``scipy.special.sph_harm_y``, Condon-Shortley phase included, as in the
paper's definition of P_n^m, Sec. 2.1) and numpy's Gauss-Legendre rule.  It
shares nothing with the C oracle (different nodes, different P_n^m, no
recurrence, no DFT tables) and so pins it at small degree (L <= 8 or so).

Real parametrisation of a spectrum: v = [Re Q (nlm), Im Q (nlm)].
  - S (nlat*nphi x 2 nlm): f = Re(Q_n^0) Y_n^0 + 2 Re(Q_n^m Y_n^m) summed
    (real-field Hermitian symmetry, Sec. 2.2); Im Q_n^0 has no effect.
  - A (2 nlm x nlat*nphi): Q_n^m = sum_i w_i sum_k (2 pi/nphi) f_ik conj(Y_n^m)
    (eq. gauss with the trapezoidal phi integral); the Im Q_n^0 row is 0.
"""
from __future__ import annotations

import numpy as np
from scipy.special import sph_harm_y


def nodes(nlat):
    x, w = np.polynomial.legendre.leggauss(nlat)
    order = np.argsort(-x)
    return x[order], w[order]


def modes(L, M):
    out = []
    for m in range(M + 1):
        for n in range(m, L + 1):
            out.append((n, m))
    return out


def matrices(L, M, nlat, nphi):
    x, w = nodes(nlat)
    theta = np.arccos(np.clip(x, -1.0, 1.0))
    phi = 2.0 * np.pi * np.arange(nphi) / nphi
    md = modes(L, M)
    nl = len(md)
    S = np.zeros((nlat * nphi, 2 * nl))
    A = np.zeros((2 * nl, nlat * nphi))
    scale = (2.0 * np.pi / nphi) * np.repeat(w, nphi)
    for j, (n, m) in enumerate(md):
        Y = sph_harm_y(n, m, theta[:, None], phi[None, :]).reshape(-1)
        if m == 0:
            S[:, j] = Y.real
        else:
            S[:, j] = 2.0 * Y.real
            S[:, nl + j] = -2.0 * Y.imag
        A[j, :] = scale * Y.real
        if m > 0:
            A[nl + j, :] = -scale * Y.imag
    return S, A


def to_real(Q):
    Q = np.asarray(Q)
    return np.concatenate([Q.real, Q.imag], axis=-1)


def to_complex(v):
    v = np.asarray(v)
    n = v.shape[-1] // 2
    return v[..., :n] + 1j * v[..., n:]
