"""Memory ranges of a call: every buffer a call writes (outputs, workspace)
must share no byte with any other buffer it touches (inputs, the other
outputs, the plan's or batch's device buffers); buffers that are only read
may overlap. Overlaps are refused with SHTN_EINVAL before any launch, and
buffers that merely touch are accepted: transforms through them match the
oracle to the parity bar (max |gpu - oracle| / max |oracle| <= 1e-12).
"""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import vector as V
from paper_1202_6522_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

L, NLAT, NPHI = 31, 32, 64  # nlm * 16 and nlat * nphi * 8 are multiples of 256


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1202_6522_amd import shtn
    shtn.load_library()
    return torch.device("cuda:0")


def aligned(t):
    return t.data_ptr() + ((-t.data_ptr()) % 256)


class Arena:
    """One device allocation; views at byte offsets from a 256-aligned base."""

    def __init__(self, nbytes, dev):
        self.buf = torch.zeros(nbytes + 256, dtype=torch.uint8, device=dev)
        self.base = aligned(self.buf)
        self.off0 = self.base - self.buf.data_ptr()

    def f64(self, off, n):
        o = self.off0 + off
        assert o % 8 == 0 and o + 8 * n <= self.buf.numel()
        return self.buf[o:o + 8 * n].view(torch.float64)

    def ptr(self, off):
        return self.base + off


def test_scalar_ranges(dev):
    from paper_1202_6522_amd import shtn as S
    lib = S.load_library()
    plan = S.Plan(L, L, NLAT, NPHI, device=dev)
    h = plan.handle
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    sb, gb, wb = plan.nlm * 16, NLAT * NPHI * 8, S.shtn_work_bytes(h, 1)
    assert sb % 256 == 0 and gb % 256 == 0
    a = Arena(sb + gb + wb, dev)
    q_off, g_off, w_off = 0, sb, sb + gb
    rng = np.random.default_rng(2024)
    Q = inputs.draw_spectrum(rng, L, L, 1.0, 1)[0]
    a.f64(q_off, 2 * plan.nlm).copy_(torch.from_numpy(Q.view(np.float64)))
    p = lambda off: ctypes.c_void_p(a.ptr(off))

    # touching ranges are accepted
    assert lib.shtn_synth(h, p(q_off), p(g_off), 1, p(w_off), stream) == S.SHTN_OK
    torch.cuda.synchronize(dev)
    g = a.f64(g_off, NLAT * NPHI).cpu().numpy().reshape(NLAT, NPHI)
    assert rel(g, oracle.synth(Q[None], L, L, NLAT, NPHI)[0]) <= 1e-12
    assert lib.shtn_analys(h, p(g_off), p(q_off), 1, p(w_off), stream) == S.SHTN_OK
    torch.cuda.synchronize(dev)
    A = a.f64(q_off, 2 * plan.nlm).cpu().numpy().view(np.complex128)
    assert rel(A, oracle.analys(g[None], L, L, NLAT, NPHI)[0]) <= 1e-12

    def refused(rc, words):
        assert rc == S.SHTN_EINVAL
        detail = lib.shtn_last_error_detail().decode()
        assert "overlaps" in detail and all(w in detail for w in words), detail

    # output over the input's last element, both directions
    refused(lib.shtn_synth(h, p(q_off), p(g_off - 8), 1, p(w_off), stream), ["input", "output"])
    refused(lib.shtn_analys(h, p(g_off), p(g_off - sb + 8), 1, p(w_off), stream), ["input", "output"])
    refused(lib.shtn_synth_adj(h, p(g_off), p(g_off + gb - 16), 1, p(w_off), stream), ["input", "output"])
    # workspace over the output's last element, and over the input
    refused(lib.shtn_synth(h, p(q_off), p(g_off), 1, p(w_off - 256), stream), ["workspace", "output"])
    refused(lib.shtn_analys(h, p(g_off), p(q_off), 1, p(q_off + sb - 256), stream), ["workspace"])
    # output inside the plan's own device buffer
    refused(lib.shtn_synth(h, p(q_off), ctypes.c_void_p(aligned(plan._dev) + 256), 1, p(w_off), stream),
            ["plan's device buffer"])
    # tuning: Qout over Q
    us4 = (ctypes.c_float * 4)()
    refused(lib.shtn_plan_tune_algorithm(h, p(q_off), p(g_off), p(q_off), 1, p(w_off), stream, 1, us4),
            ["Q", "Qout"])
    torch.cuda.synchronize(dev)
    # nothing above launched: the arena still holds the analysis result
    assert np.array_equal(a.f64(q_off, 2 * plan.nlm).cpu().numpy().view(np.complex128), A)


def test_vector_ranges(dev):
    from paper_1202_6522_amd import shtn as S
    lib = S.load_library()
    plan = S.Plan(L, L, NLAT, NPHI, device=dev)
    h = plan.handle
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    sb, gb, wb = plan.nlm * 16, NLAT * NPHI * 8, S.shtn_vec_work_bytes(h, 1)
    a = Arena(sb + 2 * gb + wb, dev)
    s_off, t_off, p_off, w_off = 0, sb, sb + gb, sb + 2 * gb
    rng = np.random.default_rng(2025)
    Sp = inputs.draw_spectrum(rng, L, L, 1.0, 1)[0]
    a.f64(s_off, 2 * plan.nlm).copy_(torch.from_numpy(Sp.view(np.float64)))
    p = lambda off: ctypes.c_void_p(a.ptr(off))

    # S and T the same buffer (read-only ranges may overlap), outputs touching
    assert lib.shtn_vec_synth(h, p(s_off), p(s_off), p(t_off), p(p_off), 1, p(w_off), stream) == S.SHTN_OK
    torch.cuda.synchronize(dev)
    et, ep = V.vec_synth(Sp[None], Sp[None], L, L, NLAT, NPHI)
    assert rel(a.f64(t_off, NLAT * NPHI).cpu().numpy().reshape(NLAT, NPHI), et[0]) <= 1e-12
    assert rel(a.f64(p_off, NLAT * NPHI).cpu().numpy().reshape(NLAT, NPHI), ep[0]) <= 1e-12

    def refused(rc, words):
        assert rc == S.SHTN_EINVAL
        detail = lib.shtn_last_error_detail().decode()
        assert "overlaps" in detail and all(w in detail for w in words), detail

    refused(lib.shtn_vec_synth(h, p(s_off), p(s_off), p(t_off), p(t_off + gb - 8), 1, p(w_off), stream),
            ["first output", "second output"])
    refused(lib.shtn_vec_synth(h, p(s_off), p(t_off - 16), p(t_off), p(p_off), 1, p(w_off), stream),
            ["second input", "first output"])
    refused(lib.shtn_vec_analys(h, p(t_off), p(p_off), p(s_off), p(p_off + gb - 16), 1, p(w_off), stream),
            ["second input", "second output"])
    refused(lib.shtn_vec_synth(h, p(s_off), p(s_off), p(t_off), p(p_off), 1, p(w_off - 8), stream),
            ["second output", "workspace"])


def test_batch_ranges(dev):
    from paper_1202_6522_amd import shtn as S
    lib = S.load_library()
    b = S.Batch([(L, L, NLAT, NPHI), (15, 15, 16, 32)], device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    Q, G = b.new_spectra(), b.new_grids()
    qb, gb = Q.numel() * 16, G.numel() * 8
    p = ctypes.c_void_p
    assert lib.shtn_batch_synth(b.handle, p(Q.data_ptr()), p(G.data_ptr()), p(b.work), stream) == S.SHTN_OK

    def refused(rc, words):
        assert rc == S.SHTN_EINVAL
        detail = lib.shtn_last_error_detail().decode()
        assert "overlaps" in detail and all(w in detail for w in words), detail

    refused(lib.shtn_batch_synth(b.handle, p(Q.data_ptr()), p(Q.data_ptr() + qb - 8), p(b.work), stream),
            ["input", "output"])
    refused(lib.shtn_batch_analys(b.handle, p(G.data_ptr()), p(Q.data_ptr()), p(G.data_ptr() + gb - 256), stream),
            ["input", "workspace"])
    refused(lib.shtn_batch_synth(b.handle, p(Q.data_ptr()), p(aligned(b._dev) + 8), p(b.work), stream),
            ["batch's device buffer"])
    refused(lib.shtn_batch_capture(b.handle, 1, p(G.data_ptr()), p(G.data_ptr() + 8), p(b.work)),
            ["input", "output"])
    torch.cuda.synchronize(dev)


def test_noalloc_ranges(dev):
    # the static-workspace synthesis checks its input and output the same way
    from paper_1202_6522_amd import shtn as S
    lib = S.load_library()
    plan = S.Plan(L, L, NLAT, NPHI, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    sb, gb = plan.nlm * 16, NLAT * NPHI * 8
    a = Arena(sb + gb, dev)
    p = lambda off: ctypes.c_void_p(a.ptr(off))
    assert lib.shtn_synth_noalloc(plan.handle, p(0), p(sb), 1, stream) == S.SHTN_OK
    assert lib.shtn_synth_noalloc(plan.handle, p(0), p(sb - 16), 1, stream) == S.SHTN_EINVAL
    detail = lib.shtn_last_error_detail().decode()
    assert "overlaps" in detail and "input" in detail and "output" in detail, detail
    torch.cuda.synchronize(dev)
