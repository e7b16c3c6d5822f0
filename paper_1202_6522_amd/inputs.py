"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no transform arithmetic: it only draws random spectra and
lays them out in the library's m-major triangular order
idx(n,m) = m(2L+1-m)/2 + n.  The recipe follows the paper's accuracy protocol
(random coefficients, Sec. 3.5) with a power-law spectrum:

  rng = numpy.random.default_rng(12026522 + case)
  re = rng.standard_normal(nlm); im = rng.standard_normal(nlm)   (m-major)
  Q = (re + i im) * (n+1)^(-slope);  Im Q = 0 where m = 0

Workloads (all FP64; nlat Gauss nodes, nphi equispaced longitudes):
  case 0: L=M=31,   nlat=32,   nphi=64,   1 field,  slope 1
  case 1: L=M=255,  nlat=256,  nphi=512,  1 field,  slope 1.5
  case 2: L=M=1023, nlat=1024, nphi=2048, 1 field,  slope 1.5
  case 3: 64 fields, L drawn from {63,127,255,511} (first draw of the rng),
          nlat=L+1, nphi=2(L+1), then each field's spectrum in field order
  case 4: 16 fields, L=M=511, nlat=512, nphi=1024: target spectra Q_T
          (16 fields) then starting spectra Q_0 (16 fields)
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 12026522

SCALAR_CASES = {
    0: dict(L=31, M=31, nlat=32, nphi=64, slope=1.0),
    1: dict(L=255, M=255, nlat=256, nphi=512, slope=1.5),
    2: dict(L=1023, M=1023, nlat=1024, nphi=2048, slope=1.5),
}


def nlm(L: int, M: int) -> int:
    return (M + 1) * (L + 1) - M * (M + 1) // 2


def degree_order(L: int, M: int):
    """Arrays (n, m) of every coefficient in m-major order."""
    ns, ms = [], []
    for m in range(M + 1):
        ns.append(np.arange(m, L + 1))
        ms.append(np.full(L + 1 - m, m))
    return np.concatenate(ns), np.concatenate(ms)


def draw_spectrum(rng, L: int, M: int, slope: float, nfields: int = 1, dist: str = "normal"):
    """nfields spectra [nfields, nlm] complex128, drawn field by field."""
    n, m = degree_order(L, M)
    k = nlm(L, M)
    out = np.empty((nfields, k), dtype=np.complex128)
    for f in range(nfields):
        if dist == "normal":
            re = rng.standard_normal(k)
            im = rng.standard_normal(k)
        elif dist == "uniform":  # the paper's accuracy protocol: each part in [-1, 1]
            re = rng.uniform(-1.0, 1.0, k)
            im = rng.uniform(-1.0, 1.0, k)
        else:
            raise ValueError(dist)
        amp = (n + 1.0) ** (-slope)
        q = (re + 1j * im) * amp
        q[m == 0] = q[m == 0].real
        out[f] = q
    return out


def scalar_case(case: int):
    """(shape dict, Q [1, nlm]) for the single-field workloads 0, 1, 2."""
    p = SCALAR_CASES[case]
    rng = np.random.default_rng(SEED_BASE + case)
    return dict(p), draw_spectrum(rng, p["L"], p["M"], p["slope"], 1)


def batch_case(case: int = 3, nfields: int = 64):
    """Mixed-degree batch: list of (L, M, nlat, nphi) and list of spectra."""
    rng = np.random.default_rng(SEED_BASE + case)
    Ls = rng.choice([63, 127, 255, 511], nfields)
    shapes = [(int(L), int(L), int(L) + 1, 2 * (int(L) + 1)) for L in Ls]
    specs = [draw_spectrum(rng, L, M, 1.5, 1)[0] for (L, M, _, _) in shapes]
    return shapes, specs


def grad_case(case: int = 4, nfields: int = 16, L: int = 511):
    """Target spectra Q_T then starting spectra Q_0, [nfields, nlm] each."""
    rng = np.random.default_rng(SEED_BASE + case)
    QT = draw_spectrum(rng, L, L, 1.5, nfields)
    Q0 = draw_spectrum(rng, L, L, 1.5, nfields)
    return dict(L=L, M=L, nlat=L + 1, nphi=2 * (L + 1)), QT, Q0


def random_grid(seed: int, nfields: int, nlat: int, nphi: int):
    """Non-band-limited grid values, N(0,1)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nfields, nlat, nphi))
