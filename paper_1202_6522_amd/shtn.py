"""ctypes binding of libshtn (include/shtn.h): argument marshalling only.

The functions below carry the C names and signatures; every transform step
runs in the HIP kernels of the library.  `Plan` adds torch plumbing (device
buffers for the plan tables and the workspace, the current HIP stream).

Importing this module does not load the library; the first call does, and it
raises if libshtn.so has not been built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libshtn.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "shtn.h")

SHTN_OK = 0
SHTN_EINVAL = -1
SHTN_EUNSUPPORTED = -2
SHTN_ESTATE = -3
SHTN_EHIP = -4
SHTN_ENOMEM = -5
SHTN_MAX_FIELDS = 65535      # fields per scalar call (include/shtn.h)
SHTN_MAX_VEC_FIELDS = 16383  # fields per vector call
SHTN_ALGO_ONTHEFLY = 0
SHTN_ALGO_STORED = 1
SHTN_ALGO_STORED_SYNTH = 2
SHTN_ALGO_STORED_ANALYS = 3
ALGORITHMS = {"onthefly": SHTN_ALGO_ONTHEFLY, "stored": SHTN_ALGO_STORED,
              "stored_synth": SHTN_ALGO_STORED_SYNTH, "stored_analys": SHTN_ALGO_STORED_ANALYS}

_lib = None

_c = ctypes
_vp = _c.c_void_p
_dp = _c.POINTER(_c.c_double)
_sz = _c.c_size_t
_SIGS = {
    "shtn_plan": (_vp, [_c.c_int, _c.c_int, _c.c_int, _c.c_int]),
    "shtn_plan_destroy": (None, [_vp]),
    "shtn_plan_device_bytes": (_sz, [_vp]),
    "shtn_plan_upload": (_c.c_int, [_vp, _vp, _vp]),
    "shtn_work_bytes": (_sz, [_vp, _c.c_int]),
    "shtn_synth": (_c.c_int, [_vp, _vp, _vp, _c.c_int, _vp, _vp]),
    "shtn_synth_noalloc": (_c.c_int, [_vp, _vp, _vp, _c.c_int, _vp]),
    "shtn_analys": (_c.c_int, [_vp, _vp, _vp, _c.c_int, _vp, _vp]),
    "shtn_synth_adj": (_c.c_int, [_vp, _vp, _vp, _c.c_int, _vp, _vp]),
    "shtn_analys_adj": (_c.c_int, [_vp, _vp, _vp, _c.c_int, _vp, _vp]),
    "shtn_nlm": (_c.c_long, [_vp]),
    "shtn_lm_index": (_c.c_long, [_vp, _c.c_int, _c.c_int]),
    "shtn_get_grid": (_c.c_int, [_vp, _dp, _dp]),
    "shtn_legendre_flops": (_c.c_double, [_vp]),
    "shtn_plan_table": (_c.c_long, [_vp, _c.c_int, _vp, _sz]),
    "shtn_plan_set_tiling": (_c.c_int, [_vp] + [_c.c_int] * 7),
    "shtn_plan_set_polar": (_c.c_int, [_vp, _c.c_int]),
    "shtn_batch": (_vp, [_c.c_int, _c.POINTER(_vp)]),
    "shtn_batch_destroy": (None, [_vp]),
    "shtn_batch_offsets": (_c.c_int, [_vp, _c.POINTER(_sz), _c.POINTER(_sz)]),
    "shtn_batch_device_bytes": (_sz, [_vp]),
    "shtn_batch_work_bytes": (_sz, [_vp]),
    "shtn_batch_upload": (_c.c_int, [_vp, _vp, _vp]),
    "shtn_batch_synth": (_c.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "shtn_batch_analys": (_c.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "shtn_batch_set_tiling": (_c.c_int, [_vp, _c.c_int, _c.c_int, _c.c_int, _c.c_int]),
    "shtn_batch_get_tiling": (_c.c_int, [_vp, _c.POINTER(_c.c_int)]),
    "shtn_batch_set_algorithm": (_c.c_int, [_vp, _c.c_int]),
    "shtn_batch_get_algorithm": (_c.c_int, [_vp]),
    "shtn_batch_capture": (_c.c_int, [_vp, _c.c_int, _vp, _vp, _vp]),
    "shtn_batch_replay": (_c.c_int, [_vp, _c.c_int, _vp]),
    "shtn_batch_tune": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _c.c_int, _c.c_char_p,
                                   _c.POINTER(_c.c_float)]),
    "shtn_vec_work_bytes": (_sz, [_vp, _c.c_int]),
    "shtn_vec_synth": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _c.c_int, _vp, _vp]),
    "shtn_vec_analys": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _c.c_int, _vp, _vp]),
    "shtn_vec_synth_adj": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _c.c_int, _vp, _vp]),
    "shtn_vec_analys_adj": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _c.c_int, _vp, _vp]),
    "shtn_ptable_bytes": (_c.c_long, [_vp]),
    "shtn_ptable_build": (_c.c_int, [_vp, _vp, _sz, _vp]),
    "shtn_ptable_release": (_c.c_int, [_vp]),
    "shtn_ptable_set_tiling": (_c.c_int, [_vp, _c.c_int, _c.c_int, _c.c_int, _c.c_int]),
    "shtn_ptable_get_tiling": (_c.c_int, [_vp, _c.POINTER(_c.c_int)]),
    "shtn_plan_set_algorithm": (_c.c_int, [_vp, _c.c_int]),
    "shtn_plan_get_algorithm": (_c.c_int, [_vp]),
    "shtn_plan_tune_algorithm": (_c.c_int, [_vp, _vp, _vp, _vp, _c.c_int, _vp, _vp, _c.c_int,
                                            _c.POINTER(_c.c_float)]),
    "shtn_fp64_probe_tflops": (_c.c_double, [_vp]),
    "shtn_profile_enable": (_c.c_int, [_c.c_int]),
    "shtn_profile_select": (_c.c_int, [_c.c_uint]),
    "shtn_profile_read": (_c.c_int, [_c.c_int, _c.POINTER(_c.c_double), _c.POINTER(_c.c_long)]),
    "shtn_profile_reset": (None, []),
    "shtn_strerror": (_c.c_char_p, [_c.c_int]),
    "shtn_last_error_detail": (_c.c_char_p, []),
}


class ShtnError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        lib = load_library()
        msg = "%s: %s (%s)" % (where, lib.shtn_strerror(code).decode(),
                               lib.shtn_last_error_detail().decode())
        super().__init__(msg)


def load_library():
    """Loads libshtn.so (built by paper_1202_6522_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libshtn.so is not built: run `python -m paper_1202_6522_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def declared_functions():
    """Names of the functions declared in include/shtn.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(shtn_\w+)\s*\(", text)))


def check(code, where):
    if code != SHTN_OK:
        raise ShtnError(code, where)
    return code


# --- thin wrappers with the C names ---------------------------------------

def shtn_plan(lmax, mmax, nlat, nphi):
    lib = load_library()
    h = lib.shtn_plan(lmax, mmax, nlat, nphi)
    if not h:
        raise ValueError("shtn_plan(%d, %d, %d, %d): %s" % (
            lmax, mmax, nlat, nphi, lib.shtn_last_error_detail().decode()))
    return h


def shtn_plan_destroy(h):
    load_library().shtn_plan_destroy(h)


def shtn_plan_device_bytes(h):
    return load_library().shtn_plan_device_bytes(h)


def shtn_plan_upload(h, dev_ptr, stream):
    return check(load_library().shtn_plan_upload(h, dev_ptr, stream), "shtn_plan_upload")


def shtn_work_bytes(h, nfields):
    return load_library().shtn_work_bytes(h, nfields)


def shtn_synth(h, Q, grid, nfields, work, stream):
    return check(load_library().shtn_synth(h, Q, grid, nfields, work, stream), "shtn_synth")


def shtn_synth_noalloc(h, Q, grid, nfields, stream):
    return check(load_library().shtn_synth_noalloc(h, Q, grid, nfields, stream), "shtn_synth_noalloc")


SHTN_NOALLOC_MAX_BYTES = 32 << 20  # static workspace of shtn_synth_noalloc (include/shtn.h)


def shtn_analys(h, grid, Q, nfields, work, stream):
    return check(load_library().shtn_analys(h, grid, Q, nfields, work, stream), "shtn_analys")


def shtn_synth_adj(h, grid, Q, nfields, work, stream):
    return check(load_library().shtn_synth_adj(h, grid, Q, nfields, work, stream), "shtn_synth_adj")


def shtn_analys_adj(h, Q, grid, nfields, work, stream):
    return check(load_library().shtn_analys_adj(h, Q, grid, nfields, work, stream),
                 "shtn_analys_adj")


def shtn_nlm(h):
    return load_library().shtn_nlm(h)


def shtn_lm_index(h, n, m):
    return load_library().shtn_lm_index(h, n, m)


def shtn_get_grid(h, nlat):
    x = np.zeros(nlat)
    w = np.zeros(nlat)
    check(load_library().shtn_get_grid(h, x.ctypes.data_as(_dp), w.ctypes.data_as(_dp)),
          "shtn_get_grid")
    return x, w


def shtn_legendre_flops(h):
    return load_library().shtn_legendre_flops(h)


_TABLE_DTYPES = {0: np.float64, 1: np.float64, 2: np.float64, 3: np.float64, 4: np.float64,
                 5: np.float64, 6: np.int32, 7: np.int32, 8: np.int32, 9: np.float64,
                 10: np.int32, 11: np.int32, 12: np.int32, 13: np.int32, 14: np.int32,
                 15: np.int32, 16: np.float64, 17: np.int32, 18: np.uint32}

UNIT_INTS = 12  # ints per work unit in tables 11 and 12


def shtn_plan_table(h, which):
    lib = load_library()
    n = lib.shtn_plan_table(h, which, None, 0)
    if n < 0:
        raise ShtnError(int(n), "shtn_plan_table")
    dt = _TABLE_DTYPES[which]
    out = np.zeros(n // np.dtype(dt).itemsize, dtype=dt)
    if n:
        lib.shtn_plan_table(h, which, out.ctypes.data, n)
    return out


def shtn_fp64_probe_tflops(stream):
    v = load_library().shtn_fp64_probe_tflops(stream)
    if v < 0:
        raise RuntimeError("shtn_fp64_probe_tflops: HIP error")
    return v


def shtn_vec_work_bytes(h, nfields):
    return load_library().shtn_vec_work_bytes(h, nfields)


def shtn_vec_synth(h, S, T, Vt, Vp, nfields, work, stream):
    return check(load_library().shtn_vec_synth(h, S, T, Vt, Vp, nfields, work, stream), "shtn_vec_synth")


def shtn_vec_analys(h, Vt, Vp, S, T, nfields, work, stream):
    return check(load_library().shtn_vec_analys(h, Vt, Vp, S, T, nfields, work, stream), "shtn_vec_analys")


def shtn_vec_synth_adj(h, Vt, Vp, S, T, nfields, work, stream):
    return check(load_library().shtn_vec_synth_adj(h, Vt, Vp, S, T, nfields, work, stream), "shtn_vec_synth_adj")


def shtn_vec_analys_adj(h, S, T, Vt, Vp, nfields, work, stream):
    return check(load_library().shtn_vec_analys_adj(h, S, T, Vt, Vp, nfields, work, stream), "shtn_vec_analys_adj")


def shtn_ptable_bytes(h):
    v = load_library().shtn_ptable_bytes(h)
    if v < 0:
        raise ShtnError(v, "shtn_ptable_bytes")
    return v


def shtn_ptable_build(h, dev_ptr, nbytes, stream):
    return check(load_library().shtn_ptable_build(h, dev_ptr, nbytes, stream), "shtn_ptable_build")


def shtn_ptable_release(h):
    return check(load_library().shtn_ptable_release(h), "shtn_ptable_release")


def shtn_ptable_set_tiling(h, synth_rt, synth_ct, analys_jt, analys_ct):
    return check(load_library().shtn_ptable_set_tiling(h, synth_rt, synth_ct, analys_jt, analys_ct),
                 "shtn_ptable_set_tiling")


def shtn_ptable_get_tiling(h):
    t = (_c.c_int * 4)()
    check(load_library().shtn_ptable_get_tiling(h, t), "shtn_ptable_get_tiling")
    return list(t)


def shtn_plan_set_algorithm(h, algo):
    return check(load_library().shtn_plan_set_algorithm(h, algo), "shtn_plan_set_algorithm")


def shtn_plan_get_algorithm(h):
    v = load_library().shtn_plan_get_algorithm(h)
    if v < 0:
        raise ShtnError(v, "shtn_plan_get_algorithm")
    return v


def shtn_plan_tune_algorithm(h, Q, grid, Qout, nfields, work, stream, reps=5):
    """Mean microseconds [synthesis on-the-fly, synthesis stored, analysis
    on-the-fly, analysis stored] (-1 where not timed)."""
    t = (_c.c_float * 4)()
    check(load_library().shtn_plan_tune_algorithm(h, Q, grid, Qout, nfields, work, stream, reps, t),
          "shtn_plan_tune_algorithm")
    return [float(v) for v in t]


def shtn_plan_set_polar(h, log2_threshold):
    return check(load_library().shtn_plan_set_polar(h, log2_threshold), "shtn_plan_set_polar")


def shtn_plan_set_tiling(h, synth_lp, analys_lp, analys_waves, fw, m_pairing, split=0, fft_rows=0):
    return check(load_library().shtn_plan_set_tiling(h, synth_lp, analys_lp, analys_waves, fw,
                                                     m_pairing, split, fft_rows),
                 "shtn_plan_set_tiling")


def shtn_batch(plan_handles):
    lib = load_library()
    arr = (_vp * len(plan_handles))(*plan_handles)
    h = lib.shtn_batch(len(plan_handles), arr)
    if not h:
        raise ValueError("shtn_batch: %s" % lib.shtn_last_error_detail().decode())
    return h


def shtn_batch_destroy(h):
    load_library().shtn_batch_destroy(h)


def shtn_batch_offsets(h, nfields):
    q = (_sz * (nfields + 1))()
    g = (_sz * (nfields + 1))()
    check(load_library().shtn_batch_offsets(h, q, g), "shtn_batch_offsets")
    return list(q), list(g)


def shtn_batch_device_bytes(h):
    return load_library().shtn_batch_device_bytes(h)


def shtn_batch_work_bytes(h):
    return load_library().shtn_batch_work_bytes(h)


def shtn_batch_upload(h, dev_ptr, stream):
    return check(load_library().shtn_batch_upload(h, dev_ptr, stream), "shtn_batch_upload")


def shtn_batch_synth(h, Q, grid, work, stream):
    return check(load_library().shtn_batch_synth(h, Q, grid, work, stream), "shtn_batch_synth")


def shtn_batch_analys(h, grid, Q, work, stream):
    return check(load_library().shtn_batch_analys(h, grid, Q, work, stream), "shtn_batch_analys")


def shtn_batch_set_tiling(h, synth_lp, fw, m_pairing, analys_merge):
    return check(load_library().shtn_batch_set_tiling(h, synth_lp, fw, m_pairing, analys_merge),
                 "shtn_batch_set_tiling")


def shtn_batch_get_tiling(h):
    t = (_c.c_int * 4)()
    check(load_library().shtn_batch_get_tiling(h, t), "shtn_batch_get_tiling")
    return list(t)


def shtn_batch_capture(h, which, inp, out, work):
    return check(load_library().shtn_batch_capture(h, which, inp, out, work), "shtn_batch_capture")


def shtn_batch_replay(h, which, stream):
    return check(load_library().shtn_batch_replay(h, which, stream), "shtn_batch_replay")


def shtn_batch_tune(h, Q, grid, Qout, work, stream, reps=10, cache_path=None):
    best = _c.c_float(0.0)
    cp = cache_path.encode() if cache_path else None
    check(load_library().shtn_batch_tune(h, Q, grid, Qout, work, stream, reps, cp, _c.byref(best)),
          "shtn_batch_tune")
    return best.value


PROFILE_KINDS = {0: "prescale", 1: "legendre_synth", 2: "legendre_analys", 3: "c2r", 4: "r2c"}


def shtn_profile_enable(on):
    return check(load_library().shtn_profile_enable(1 if on else 0), "shtn_profile_enable")


def shtn_profile_read(kind):
    ms = _c.c_double()
    n = _c.c_long()
    check(load_library().shtn_profile_read(kind, _c.byref(ms), _c.byref(n)), "shtn_profile_read")
    return ms.value, n.value


def shtn_profile_select(kinds):
    """Time only these kernel kinds (keys of PROFILE_KINDS) while enabled."""
    mask = 0
    for k in kinds:
        mask |= 1 << int(k)
    return check(load_library().shtn_profile_select(mask), "shtn_profile_select")


def shtn_profile_reset():
    load_library().shtn_profile_reset()


def shtn_strerror(code):
    return load_library().shtn_strerror(code).decode()


def shtn_last_error_detail():
    return load_library().shtn_last_error_detail().decode()


# --- torch plumbing --------------------------------------------------------

def _stream_ptr(torch, device):
    return torch.cuda.current_stream(device).cuda_stream


class Plan:
    """A transform plan whose tables live in a torch-owned device buffer."""

    def __init__(self, lmax, mmax=None, nlat=None, nphi=None, device="cuda", tiling=None, polar_log2=None):
        import torch
        self.lmax = int(lmax)
        self.mmax = int(lmax if mmax is None else mmax)
        self.nlat = int(self.lmax + 1 if nlat is None else nlat)
        self.nphi = int(2 * (self.lmax + 1) if nphi is None else nphi)
        self.device = torch.device(device)
        self.handle = shtn_plan(self.lmax, self.mmax, self.nlat, self.nphi)
        self.nlm = int(shtn_nlm(self.handle))
        self.npair = (self.nlat + 1) // 2
        self._work = {}
        self._vwork = {}
        self._dev = None
        self._ptab = None
        if polar_log2 is not None:
            shtn_plan_set_polar(self.handle, int(polar_log2))
        if tiling is not None:
            self.set_tiling(**tiling)
        else:
            self._upload()

    def _upload(self):
        import torch
        nbytes = shtn_plan_device_bytes(self.handle)
        self._dev = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self._dev.data_ptr()
        off = (-ptr) % 256
        shtn_plan_upload(self.handle, ptr + off, _stream_ptr(torch, self.device))

    def set_tiling(self, synth_lp, analys_lp, analys_waves=1, fw=1, m_pairing=0, split=0, fft_rows=0):
        shtn_plan_set_tiling(self.handle, synth_lp, analys_lp, analys_waves, fw, m_pairing, split,
                             fft_rows)
        self._upload()

    def set_polar(self, log2_threshold):
        """Polar threshold exponent (see shtn_plan_set_polar); re-uploads and
        rebuilds the stored-P table if the plan has one."""
        algo = shtn_plan_get_algorithm(self.handle)
        shtn_plan_set_polar(self.handle, int(log2_threshold))
        self._upload()
        if self._ptab is not None:
            self.build_ptable()
            shtn_plan_set_algorithm(self.handle, algo)

    # --- stored-P Legendre stage (Sec. 3.1) and the runtime choice (Sec. 3.2) ---
    def build_ptable(self):
        """Allocates and builds the stored-P table (shtn_ptable_bytes of device memory)."""
        import torch
        nb = shtn_ptable_bytes(self.handle)
        if self._ptab is None or self._ptab.numel() < nb + 256:
            self._ptab = None
            self._ptab = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        ptr = self._ptab.data_ptr()
        shtn_ptable_build(self.handle, ptr + ((-ptr) % 256), nb, _stream_ptr(torch, self.device))

    def release_ptable(self):
        """Drops the table (and selects the on-the-fly algorithm)."""
        shtn_ptable_release(self.handle)
        self._ptab = None

    def ptable_bytes(self):
        return shtn_ptable_bytes(self.handle)

    def set_algorithm(self, algo):
        """'onthefly', 'stored', 'stored_synth' or 'stored_analys' (the
        passes that read the table; builds it if the plan has none)."""
        a = ALGORITHMS.get(algo, algo)
        if a != SHTN_ALGO_ONTHEFLY and self._ptab is None:
            self.build_ptable()
        shtn_plan_set_algorithm(self.handle, int(a))

    def algorithm(self):
        v = shtn_plan_get_algorithm(self.handle)
        return next(k for k, a in ALGORITHMS.items() if a == v)

    def set_ptable_tiling(self, synth_rt=4, synth_ct=2, analys_jt=4, analys_ct=2):
        shtn_ptable_set_tiling(self.handle, synth_rt, synth_ct, analys_jt, analys_ct)

    def ptable_tiling(self):
        t = shtn_ptable_get_tiling(self.handle)
        return dict(synth_rt=t[0], synth_ct=t[1], analys_jt=t[2], analys_ct=t[3])

    def tune_algorithm(self, nfields, reps=5, keep_table=False):
        """Runtime choice between the two Legendre algorithms for calls of
        nfields fields (Sec. 3.2): builds the table, times both on random
        data, keeps the faster (the table is dropped when the on-the-fly
        algorithm wins, unless keep_table)."""
        import torch
        if self._ptab is None:
            self.build_ptable()
        g = torch.Generator(device=self.device).manual_seed(12026522)
        Q = torch.randn((nfields, self.nlm), dtype=torch.complex128, device=self.device, generator=g)
        grid = torch.empty((nfields, self.nlat, self.nphi), dtype=torch.float64, device=self.device)
        Qout = torch.empty_like(Q)
        t = shtn_plan_tune_algorithm(self.handle, Q.data_ptr(), grid.data_ptr(), Qout.data_ptr(),
                                     nfields, self.workspace(nfields), _stream_ptr(torch, self.device), reps)
        algo = self.algorithm()
        if algo == "onthefly" and not keep_table:
            self.release_ptable()
        return dict(algorithm=algo, synth_onthefly_us=t[0], synth_stored_us=t[1],
                    analys_onthefly_us=t[2], analys_stored_us=t[3])

    def polar_log2(self):
        return int(shtn_plan_table(self.handle, 13)[8])

    def tiling(self):
        t = shtn_plan_table(self.handle, 13)
        return dict(synth_lp=int(t[0]), analys_lp=int(t[1]), analys_waves=int(t[6]), fw=int(t[2]),
                    m_pairing=int(t[3]), split=int(t[4]), fft_rows=int(t[5]))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                shtn_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    def grid(self):
        return shtn_get_grid(self.handle, self.nlat)

    def legendre_flops(self):
        return shtn_legendre_flops(self.handle)

    def lm_index(self, n, m):
        return shtn_lm_index(self.handle, n, m)

    def workspace(self, nfields):
        import torch
        w = self._work.get(nfields)
        if w is None:
            nb = shtn_work_bytes(self.handle, nfields)
            w = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
            self._work[nfields] = w
        return w.data_ptr() + ((-w.data_ptr()) % 256)

    # shape checks + calls
    def _spec_in(self, Q):
        import torch
        if Q.dtype != torch.complex128 or Q.device.type != "cuda" or Q.shape[-1] != self.nlm:
            raise ValueError("spectrum must be a complex128 CUDA tensor [..., %d]" % self.nlm)
        return Q.contiguous()

    def _grid_in(self, g):
        import torch
        if g.dtype != torch.float64 or g.device.type != "cuda" or \
                tuple(g.shape[-2:]) != (self.nlat, self.nphi):
            raise ValueError("grid must be a float64 CUDA tensor [..., %d, %d]" % (self.nlat, self.nphi))
        return g.contiguous()

    def _to_grid(self, fn, Q):
        import torch
        Q = self._spec_in(Q)
        lead = Q.shape[:-1]
        nf = int(np.prod(lead)) if len(lead) else 1
        out = torch.empty(lead + (self.nlat, self.nphi), dtype=torch.float64, device=Q.device)
        fn(self.handle, Q.data_ptr(), out.data_ptr(), nf, self.workspace(nf),
           _stream_ptr(torch, Q.device))
        return out

    def _to_spec(self, fn, g):
        import torch
        g = self._grid_in(g)
        lead = g.shape[:-2]
        nf = int(np.prod(lead)) if len(lead) else 1
        out = torch.empty(lead + (self.nlm,), dtype=torch.complex128, device=g.device)
        fn(self.handle, g.data_ptr(), out.data_ptr(), nf, self.workspace(nf),
           _stream_ptr(torch, g.device))
        return out

    def vec_workspace(self, nfields):
        import torch
        w = self._vwork.get(nfields)
        if w is None:
            nb = shtn_vec_work_bytes(self.handle, nfields)
            w = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
            self._vwork[nfields] = w
        return w.data_ptr() + ((-w.data_ptr()) % 256)

    def vec_synth(self, S, T):
        """Vector synthesis (spheroidal S, toroidal T spectra [..., nlm]
        complex128) -> (V_theta, V_phi), each [..., nlat, nphi] float64."""
        return self._vec_to_grid(shtn_vec_synth, S, T)

    def vec_analys_adj(self, S, T):
        """Adjoint of the vector analysis: spectra -> grids."""
        return self._vec_to_grid(shtn_vec_analys_adj, S, T)

    def vec_analys(self, vt, vp):
        """Vector analysis (V_theta, V_phi) [..., nlat, nphi] -> (S, T) [..., nlm]."""
        return self._vec_to_spec(shtn_vec_analys, vt, vp)

    def vec_synth_adj(self, vt, vp):
        """Adjoint of the vector synthesis: grids -> spectra."""
        return self._vec_to_spec(shtn_vec_synth_adj, vt, vp)

    def _vec_to_grid(self, fn, S, T):
        import torch
        S = self._spec_in(S)
        T = self._spec_in(T)
        if S.shape != T.shape:
            raise ValueError("S and T must have the same shape")
        lead = S.shape[:-1]
        nf = int(np.prod(lead)) if len(lead) else 1
        vt = torch.empty(lead + (self.nlat, self.nphi), dtype=torch.float64, device=S.device)
        vp = torch.empty_like(vt)
        fn(self.handle, S.data_ptr(), T.data_ptr(), vt.data_ptr(), vp.data_ptr(), nf,
           self.vec_workspace(nf), _stream_ptr(torch, S.device))
        return vt, vp

    def _vec_to_spec(self, fn, vt, vp):
        import torch
        vt = self._grid_in(vt)
        vp = self._grid_in(vp)
        if vt.shape != vp.shape:
            raise ValueError("V_theta and V_phi must have the same shape")
        lead = vt.shape[:-2]
        nf = int(np.prod(lead)) if len(lead) else 1
        S = torch.empty(lead + (self.nlm,), dtype=torch.complex128, device=vt.device)
        T = torch.empty_like(S)
        fn(self.handle, vt.data_ptr(), vp.data_ptr(), S.data_ptr(), T.data_ptr(), nf,
           self.vec_workspace(nf), _stream_ptr(torch, vt.device))
        return S, T

    def synth(self, Q):
        """Synthesis S Q: [..., nlm] complex128 -> [..., nlat, nphi] float64."""
        return self._to_grid(shtn_synth, Q)

    def analys(self, g):
        """Analysis A g: [..., nlat, nphi] float64 -> [..., nlm] complex128."""
        return self._to_spec(shtn_analys, g)

    def synth_adj(self, g):
        """Adjoint of the synthesis S^T g (gradient convention dRe + i dIm)."""
        return self._to_spec(shtn_synth_adj, g)

    def analys_adj(self, h):
        """Adjoint of the analysis A^T h."""
        return self._to_grid(shtn_analys_adj, h)


class Batch:
    """Fields of different truncations transformed together (shtn_batch_*).

    shapes: list of (lmax, mmax, nlat, nphi), one per field.  Fields sharing a
    shape share one Plan.  Packed buffers: spectra [total_q // 2] complex128,
    grids [total_grid] float64, fields back to back in the given order.
    """

    def __init__(self, shapes, device="cuda"):
        import torch
        self.device = torch.device(device)
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.plans = {}
        for s in self.shapes:
            if s not in self.plans:
                self.plans[s] = Plan(*s, device=self.device)
        self.handle = shtn_batch([self.plans[s].handle for s in self.shapes])
        self.q_off, self.g_off = shtn_batch_offsets(self.handle, len(self.shapes))
        self._dev = torch.empty(shtn_batch_device_bytes(self.handle) + 256, dtype=torch.uint8,
                                device=self.device)
        self._work = torch.empty(shtn_batch_work_bytes(self.handle) + 256, dtype=torch.uint8,
                                 device=self.device)
        self._captured = {}
        self.upload()

    @staticmethod
    def _aligned(t):
        return t.data_ptr() + ((-t.data_ptr()) % 256)

    def _stream(self):
        import torch
        return _stream_ptr(torch, self.device)

    def upload(self):
        shtn_batch_upload(self.handle, self._aligned(self._dev), self._stream())

    def set_tiling(self, synth_lp=1, fw=1, m_pairing=0, analys_merge=0):
        shtn_batch_set_tiling(self.handle, synth_lp, fw, m_pairing, analys_merge)
        self.upload()

    def tiling(self):
        t = shtn_batch_get_tiling(self.handle)
        return dict(synth_lp=t[0], fw=t[1], m_pairing=t[2], analys_merge=t[3])

    def build_ptables(self):
        """Builds the stored-P table of every plan of the batch (see
        Plan.build_ptable), then uploads the batch again (a plan that changed
        makes the batch's copies stale until then)."""
        for p in self.plans.values():
            p.build_ptable()
        self.upload()

    def set_algorithm(self, algo):
        """'onthefly' or 'stored' (the plans with a table use the stored kernels); re-uploads."""
        a = {"onthefly": SHTN_ALGO_ONTHEFLY, "stored": SHTN_ALGO_STORED}.get(algo, algo)
        check(load_library().shtn_batch_set_algorithm(self.handle, int(a)), "shtn_batch_set_algorithm")
        self.upload()

    def algorithm(self):
        v = load_library().shtn_batch_get_algorithm(self.handle)
        if v < 0:
            raise ShtnError(v, "shtn_batch_get_algorithm")
        return "stored" if v == SHTN_ALGO_STORED else "onthefly"

    @property
    def work(self):
        return self._aligned(self._work)

    def new_spectra(self):
        import torch
        return torch.zeros(self.q_off[-1] // 2, dtype=torch.complex128, device=self.device)

    def new_grids(self):
        import torch
        return torch.zeros(self.g_off[-1], dtype=torch.float64, device=self.device)

    def pack_spectra(self, specs):
        """List of per-field [nlm] complex arrays/tensors -> packed tensor."""
        import torch
        out = self.new_spectra()
        for f, q in enumerate(specs):
            q = torch.as_tensor(q).to(self.device)
            out[self.q_off[f] // 2:self.q_off[f + 1] // 2] = q.reshape(-1)
        return out

    def field_spectrum(self, Qp, f):
        return Qp[self.q_off[f] // 2:self.q_off[f + 1] // 2]

    def field_grid(self, gp, f):
        _, _, nlat, nphi = self.shapes[f]
        return gp[self.g_off[f]:self.g_off[f + 1]].view(nlat, nphi)

    def _check(self, t, n, dtype):
        import torch
        if t.dtype != dtype or t.device.type != "cuda" or t.numel() != n or not t.is_contiguous():
            raise ValueError("expected a contiguous %s CUDA tensor of %d elements" % (dtype, n))

    def synth(self, Qp, out=None):
        import torch
        self._check(Qp, self.q_off[-1] // 2, torch.complex128)
        out = self.new_grids() if out is None else out
        self._check(out, self.g_off[-1], torch.float64)
        shtn_batch_synth(self.handle, Qp.data_ptr(), out.data_ptr(), self.work, self._stream())
        return out

    def analys(self, gp, out=None):
        import torch
        self._check(gp, self.g_off[-1], torch.float64)
        out = self.new_spectra() if out is None else out
        self._check(out, self.q_off[-1] // 2, torch.complex128)
        shtn_batch_analys(self.handle, gp.data_ptr(), out.data_ptr(), self.work, self._stream())
        return out

    def capture(self, which, inp, out):
        """Captures one direction (0 synthesis, 1 analysis) for these buffers
        (kept referenced while the graph exists)."""
        shtn_batch_capture(self.handle, which, inp.data_ptr(), out.data_ptr(), self.work)
        self._captured[which] = (inp, out)

    def replay(self, which):
        shtn_batch_replay(self.handle, which, self._stream())

    def tune(self, Qp, gp, Qout, reps=10, cache_path=None):
        """Autotunes the tiling on these buffers; leaves both graphs captured
        (the buffers kept referenced).  Returns the best round-trip time in
        microseconds, or -1 when the tiling came from the cache."""
        us = shtn_batch_tune(self.handle, Qp.data_ptr(), gp.data_ptr(), Qout.data_ptr(),
                             self.work, self._stream(), reps, cache_path)
        self._captured = {0: (Qp, gp), 1: (gp, Qout)}
        return us

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                shtn_batch_destroy(h)
            except Exception:
                pass
            self.handle = None
