"""Reference (oracle) spherical harmonic transform -- TEST INFRASTRUCTURE ONLY.

A plain, slow CPU implementation of the Gauss-Legendre spherical harmonic
transform of Schaeffer (arXiv 1202.6522), used to check the GPU library.  Only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the GPU library.

The arithmetic lives in ``shtn_oracle.c`` (double and long-double
instantiations); this module only marshals numpy arrays through ctypes.
``dense.py`` holds an independent tiny dense brute force built on scipy, used
to pin the C oracle itself.  ``vector.py`` holds the vector (spheroidal /
toroidal) transforms in plain numpy on top of this module's nodes and P_n^m.

Conventions: spectra are complex128 arrays in m-major triangular order
idx(n,m) = m(2L+1-m)/2 + n; grids are float64 [nlat, nphi] with row i the
colatitude theta_i increasing and column k the longitude 2 pi k / nphi.

Parity status: every function here is pinned by tests/test_oracle_pins.py
(closed forms, identities, scipy brute force, quadrature exactness), and
those of vector.py by tests/test_oracle_vector_pins.py.  The long-double
instantiation (precision="ld", the reference where P_m^m falls below the
range of double) is pinned by tests/test_oracle_ld_pins.py against 40-digit
mpmath: its unrounded P_n^m (``plm_raw``) and its rounded ones at lmax 2047
and 4095, its Gauss nodes, and its synthesis.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "shtn_oracle.c"), os.path.join(_HERE, "shtn_oracle_body.h")]
_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc -O2 -fopenmp (no fast-math)."""
    newest = max(os.path.getmtime(p) for p in _SRC)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < newest:
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
             "-o", tmp, _SRC[0], "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    i = ctypes.c_int
    for sfx in ("_d", "_ld"):
        getattr(lib, "oracle_gauss" + sfx).argtypes = [i, dp, dp]
        getattr(lib, "oracle_plm" + sfx).argtypes = [i, i, i, dp, dp]
        getattr(lib, "oracle_synth" + sfx).argtypes = [i, i, i, i, i, dp, dp, i, ip, i, ip, i]
        getattr(lib, "oracle_analys_adj" + sfx).argtypes = [i, i, i, i, i, dp, dp, i, ip, i, ip, i]
        getattr(lib, "oracle_analys" + sfx).argtypes = [i, i, i, i, i, dp, dp, i, ip, i]
        getattr(lib, "oracle_synth_adj" + sfx).argtypes = [i, i, i, i, i, dp, dp, i, ip, i]
        for name in ("oracle_gauss", "oracle_plm", "oracle_synth", "oracle_analys",
                     "oracle_synth_adj", "oracle_analys_adj"):
            getattr(lib, name + sfx).restype = ctypes.c_int
    lib.oracle_plm_raw_d.argtypes = [i, i, ip, i, dp, dp]
    lib.oracle_plm_raw_d.restype = ctypes.c_int
    lib.oracle_plm_raw_ld.argtypes = [i, i, ip, i, dp, ctypes.POINTER(ctypes.c_longdouble)]
    lib.oracle_plm_raw_ld.restype = ctypes.c_int
    lib.oracle_nlm.argtypes = [i, i]
    lib.oracle_nlm.restype = ctypes.c_long
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _sfx(precision):
    if precision in ("double", "d", np.float64):
        return "_d"
    if precision in ("long double", "ld", "longdouble"):
        return "_ld"
    raise ValueError(precision)


def _threads(nthreads):
    if nthreads is None:
        return max(1, min(16, os.cpu_count() or 1))
    return int(nthreads)


def nlm(L: int, M: int) -> int:
    return (M + 1) * (L + 1) - M * (M + 1) // 2


def lm_index(L: int, n, m):
    """m-major triangular index of (n, m)."""
    return m * (2 * L + 1 - m) // 2 + n


def gauss(nlat: int, precision="double"):
    """Gauss-Legendre nodes x (decreasing) and weights w."""
    x = np.zeros(nlat)
    w = np.zeros(nlat)
    rc = getattr(_load(), "oracle_gauss" + _sfx(precision))(nlat, _dp(x), _dp(w))
    if rc:
        raise ValueError("oracle_gauss failed")
    return x, w


def plm(L: int, M: int, x, precision="double"):
    """P_n^m(x_j) as an array [nlm, len(x)] in m-major order."""
    x = np.ascontiguousarray(np.atleast_1d(x), dtype=np.float64)
    out = np.zeros((nlm(L, M), x.size))
    rc = getattr(_load(), "oracle_plm" + _sfx(precision))(L, M, x.size, _dp(x), _dp(out))
    if rc:
        raise ValueError("oracle_plm failed")
    return out


def plm_raw(L: int, mlist, x, precision="ld"):
    """P_n^m(x_j) in the oracle's working type, without the final rounding to
    double: an array [len(mlist), L+1, len(x)] (entries n < m are 0) of
    numpy.longdouble for precision "ld" (float64 for "double")."""
    x = np.ascontiguousarray(np.atleast_1d(x), dtype=np.float64)
    ml = np.ascontiguousarray(np.atleast_1d(mlist), dtype=np.int32)
    sfx = _sfx(precision)
    dt = np.longdouble if sfx == "_ld" else np.float64
    out = np.zeros((ml.size, L + 1, x.size), dtype=dt)
    ptr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_longdouble if sfx == "_ld" else ctypes.c_double))
    rc = getattr(_load(), "oracle_plm_raw" + sfx)(L, ml.size, _ip(ml), x.size, _dp(x), ptr)
    if rc:
        raise ValueError("oracle_plm_raw failed")
    return out


def _mlist(mlist):
    if mlist is None:
        return 0, None
    a = np.ascontiguousarray(mlist, dtype=np.int32)
    return a.size, a


def _prep_spec(Q, L, M):
    Q = np.ascontiguousarray(Q, dtype=np.complex128)
    n = nlm(L, M)
    if Q.shape[-1] != n:
        raise ValueError("spectrum length %d != nlm %d" % (Q.shape[-1], n))
    return Q.reshape(-1, n)


def _prep_grid(g, nlat, nphi):
    g = np.ascontiguousarray(g, dtype=np.float64)
    if g.shape[-2:] != (nlat, nphi):
        raise ValueError("grid shape")
    return g.reshape(-1, nlat, nphi)


def _to_grid(name, Q, L, M, nlat, nphi, mlist, rows, precision, nthreads):
    lead = np.shape(Q)[:-1]
    Qf = _prep_spec(Q, L, M)
    nf = Qf.shape[0]
    nm, ml = _mlist(mlist)
    if rows is None:
        nr, ra = nlat, None
    else:
        ra = np.ascontiguousarray(rows, dtype=np.int32)
        nr = ra.size
    out = np.zeros((nf, nr, nphi))
    rc = getattr(_load(), name + _sfx(precision))(
        L, M, nlat, nphi, nf, _dp(Qf.view(np.float64)), _dp(out), nm, _ip(ml),
        nr, _ip(ra), _threads(nthreads))
    if rc:
        raise ValueError(name + " failed (bad arguments)")
    return out.reshape(lead + (nr, nphi))


def _to_spec(name, g, L, M, nlat, nphi, mlist, precision, nthreads):
    lead = np.shape(g)[:-2]
    gf = _prep_grid(g, nlat, nphi)
    nf = gf.shape[0]
    nm, ml = _mlist(mlist)
    out = np.zeros((nf, nlm(L, M)), dtype=np.complex128)
    rc = getattr(_load(), name + _sfx(precision))(
        L, M, nlat, nphi, nf, _dp(gf), _dp(out.view(np.float64)), nm, _ip(ml), _threads(nthreads))
    if rc:
        raise ValueError(name + " failed (bad arguments)")
    return out.reshape(lead + (nlm(L, M),))


def synth(Q, L, M, nlat, nphi, mlist=None, rows=None, precision="double", nthreads=None):
    """Synthesis f = S Q (Sec. 2.2).  Q [..., nlm] complex -> [..., nrows, nphi]."""
    return _to_grid("oracle_synth", Q, L, M, nlat, nphi, mlist, rows, precision, nthreads)


def analys(grid, L, M, nlat, nphi, mlist=None, precision="double", nthreads=None):
    """Analysis Q = A f (Sec. 2.3, eq. gauss).  [..., nlat, nphi] -> [..., nlm]."""
    return _to_spec("oracle_analys", grid, L, M, nlat, nphi, mlist, precision, nthreads)


def synth_adj(grid, L, M, nlat, nphi, mlist=None, precision="double", nthreads=None):
    """Adjoint of the synthesis S^T (grid -> spectrum shape)."""
    return _to_spec("oracle_synth_adj", grid, L, M, nlat, nphi, mlist, precision, nthreads)


def analys_adj(h, L, M, nlat, nphi, mlist=None, rows=None, precision="double", nthreads=None):
    """Adjoint of the analysis A^T (spectrum shape -> grid)."""
    return _to_grid("oracle_analys_adj", h, L, M, nlat, nphi, mlist, rows, precision, nthreads)
