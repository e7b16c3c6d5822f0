"""Vector (spheroidal / toroidal) spherical harmonic transforms -- TEST
INFRASTRUCTURE ONLY (same rules as the rest of ``oracle/``).

The paper names vector transforms among the uses of the library but gives no
formulas for them.  This module states the usual definition and computes it
plainly, in numpy float64, from the scalar oracle's Gauss nodes and P_n^m
(both pinned by tests/test_oracle_pins.py):

A tangent vector field on the unit sphere is written with a spheroidal
potential S and a toroidal potential T,

    V_theta = dS/dtheta - (1/sin theta) dT/dphi,
    V_phi   = (1/sin theta) dS/dphi + dT/dtheta,

S = sum S_n^m Y_n^m and T likewise, real fields (Hermitian symmetry, Im of
the m = 0 coefficients ignored, as for scalars).  Per order m:

    Vt_m(theta) = sum_n [ S_n^m dP_n^m/dtheta - i m T_n^m P_n^m / sin theta ],
    Vp_m(theta) = sum_n [ i m S_n^m P_n^m / sin theta + T_n^m dP_n^m/dtheta ],

and each component on the grid is Re V_0 + 2 Re sum_{m>=1} V_m e^{i m phi}
(direct DFT, no FFT).  The analysis projects on the two basis fields of each
(n, m), (dP, i m P/sin) e^{i m phi} and (-i m P/sin, dP) e^{i m phi}, whose
squared norm is n(n+1):

    S_n^m = 1/(n(n+1)) sum_i w_i [ Ft_m dP_n^m/dtheta - i m Fp_m P_n^m / sin theta ],
    T_n^m = 1/(n(n+1)) sum_i w_i [ i m Ft_m P_n^m / sin theta + Fp_m dP_n^m/dtheta ],

with F_m = (2 pi / nphi) sum_k f_ik e^{-i m phi_k} as for scalars.  The
degree 0 coefficients are 0.
dP_n^m/dtheta comes from the identity (orthonormal P, x = cos theta)

    sin theta dP_n^m/dtheta = n x P_n^m - c_n P_{n-1}^m,
    c_n = sqrt((2n+1)(n^2-m^2)/(2n-1)),

checked against finite differences of P_n^m in the pins.  sin theta is taken
as sqrt((1-x)(1+x)) of the node x actually used for P_n^m.
"""
from __future__ import annotations

import numpy as np

from . import gauss, lm_index, nlm, plm


def _sin(x):
    x = np.asarray(x, dtype=np.float64)
    return np.sqrt((1.0 - x) * (1.0 + x))


def dplm(L: int, M: int, x):
    """dP_n^m/dtheta at x = cos theta, [nlm, len(x)] in m-major order."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    P = plm(L, M, x)
    s = _sin(x)
    D = np.zeros_like(P)
    for m in range(M + 1):
        for n in range(m, L + 1):
            i = lm_index(L, n, m)
            v = n * x * P[i]
            if n > m:
                c = np.sqrt((2.0 * n + 1) * (n * n - m * m) / (2.0 * n - 1))
                v = v - c * P[lm_index(L, n - 1, m)]
            D[i] = v / s
    return D


def _dft_tables(M, nphi):
    k = np.arange(nphi)
    j = (np.arange(M + 1)[:, None] * k[None, :]) % nphi  # exact integer reduction
    ang = 2.0 * np.pi * j / nphi
    return np.cos(ang), np.sin(ang)


def _grid_from_orders(V, M, nphi, cs, sn):
    """V [nf, M+1, nlat] complex -> [nf, nlat, nphi] real."""
    g = np.einsum("fi,k->fik", V[:, 0, :].real, np.ones(nphi))
    for m in range(1, M + 1):
        g += 2.0 * (V[:, m, :].real[:, :, None] * cs[m][None, None, :]
                    - V[:, m, :].imag[:, :, None] * sn[m][None, None, :])
    return g


def _orders_from_grid(g, M, nphi, cs, sn):
    """[nf, nlat, nphi] -> F [nf, M+1, nlat] complex, F_m = (2 pi/nphi) sum_k f e^{-i m phi_k}."""
    sc = 2.0 * np.pi / nphi
    re = np.einsum("fik,mk->fmi", g, cs) * sc
    im = -np.einsum("fik,mk->fmi", g, sn) * sc
    return re + 1j * im


def vec_synth(S, T, L, M, nlat, nphi):
    """(S, T) [..., nlm] complex -> (V_theta, V_phi) [..., nlat, nphi]."""
    S = np.asarray(S, dtype=np.complex128)
    T = np.asarray(T, dtype=np.complex128)
    lead = S.shape[:-1]
    S = S.reshape(-1, nlm(L, M))
    T = T.reshape(-1, nlm(L, M))
    x, _ = gauss(nlat)
    s = _sin(x)
    P = plm(L, M, x)
    D = dplm(L, M, x)
    nf = S.shape[0]
    Vt = np.zeros((nf, M + 1, nlat), dtype=np.complex128)
    Vp = np.zeros((nf, M + 1, nlat), dtype=np.complex128)
    for m in range(M + 1):
        a, b = lm_index(L, m, m), lm_index(L, L, m) + 1
        Sm, Tm = S[:, a:b].copy(), T[:, a:b].copy()
        if m == 0:
            Sm = Sm.real.astype(np.complex128)
            Tm = Tm.real.astype(np.complex128)
        Pm, Dm = P[a:b], D[a:b]
        Vt[:, m] = Sm @ Dm - 1j * m * (Tm @ Pm) / s
        Vp[:, m] = 1j * m * (Sm @ Pm) / s + Tm @ Dm
    cs, sn = _dft_tables(M, nphi)
    gt = _grid_from_orders(Vt, M, nphi, cs, sn)
    gp = _grid_from_orders(Vp, M, nphi, cs, sn)
    return gt.reshape(lead + (nlat, nphi)), gp.reshape(lead + (nlat, nphi))


def vec_analys(Vt, Vp, L, M, nlat, nphi):
    """(V_theta, V_phi) [..., nlat, nphi] -> (S, T) [..., nlm] complex."""
    Vt = np.asarray(Vt, dtype=np.float64)
    Vp = np.asarray(Vp, dtype=np.float64)
    lead = Vt.shape[:-2]
    Vt = Vt.reshape(-1, nlat, nphi)
    Vp = Vp.reshape(-1, nlat, nphi)
    x, w = gauss(nlat)
    s = _sin(x)
    P = plm(L, M, x)
    D = dplm(L, M, x)
    cs, sn = _dft_tables(M, nphi)
    Ft = _orders_from_grid(Vt, M, nphi, cs, sn)
    Fp = _orders_from_grid(Vp, M, nphi, cs, sn)
    nf = Vt.shape[0]
    S = np.zeros((nf, nlm(L, M)), dtype=np.complex128)
    T = np.zeros((nf, nlm(L, M)), dtype=np.complex128)
    for m in range(M + 1):
        a, b = lm_index(L, m, m), lm_index(L, L, m) + 1
        n = np.arange(m, L + 1)
        Pm, Dm = P[a:b] * w, D[a:b] * w  # [n, lat], weights folded in
        # projections on the conjugated basis fields (dP, -i m P/s) and (i m P/s, dP)
        s_val = Ft[:, m] @ Dm.T - 1j * m * (Fp[:, m] / s) @ Pm.T
        t_val = 1j * m * (Ft[:, m] / s) @ Pm.T + Fp[:, m] @ Dm.T
        nn = n * (n + 1.0)
        with np.errstate(divide="ignore", invalid="ignore"):
            S[:, a:b] = np.where(n > 0, s_val / nn, 0.0)
            T[:, a:b] = np.where(n > 0, t_val / nn, 0.0)
        if m == 0:
            S[:, a:b] = S[:, a:b].real
            T[:, a:b] = T[:, a:b].real
    return S.reshape(lead + (nlm(L, M),)), T.reshape(lead + (nlm(L, M),))
