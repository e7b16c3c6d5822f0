"""shtn_synth_noalloc (synthesis with the library's static device workspace)
against shtn_synth (caller workspace) through the C interface.

Two calls in a row, the second smaller (fewer fields of a smaller plan), each
bitwise equal to shtn_synth on the same input (the same kernels run on the
same data; only the workspace differs); the second also after the first
left its larger contents in the static array.  A call needing more than the
static workspace is refused with SHTN_EINVAL.
"""
import numpy as np
import pytest

from paper_1202_6522_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1202_6522_amd import shtn
    shtn.load_library()
    return torch.device("cuda:0")


def _pair(plan, Q, dev):
    from paper_1202_6522_amd import shtn as S
    stream = torch.cuda.current_stream(dev).cuda_stream
    nf = Q.shape[0]
    g_ref = torch.empty((nf, plan.nlat, plan.nphi), dtype=torch.float64, device=dev)
    g_new = torch.full_like(g_ref, float("nan"))
    S.shtn_synth(plan.handle, Q.data_ptr(), g_ref.data_ptr(), nf, plan.workspace(nf), stream)
    S.shtn_synth_noalloc(plan.handle, Q.data_ptr(), g_new.data_ptr(), nf, stream)
    torch.cuda.synchronize(dev)
    return g_ref, g_new


def test_noalloc_matches_workspace_call_twice(dev):
    from paper_1202_6522_amd.shtn import Plan
    rng = np.random.default_rng(inputs.SEED_BASE + 70)
    big = Plan(511, 511, 512, 1024, device=dev)
    Qb = torch.from_numpy(inputs.draw_spectrum(rng, 511, 511, 1.5, 4)).to(dev)
    g_ref, g_new = _pair(big, Qb, dev)
    assert torch.equal(g_new, g_ref)
    small = Plan(100, 80, 101, 256, device=dev)
    Qs = torch.from_numpy(inputs.draw_spectrum(rng, 100, 80, 1.0, 2)).to(dev)
    g_ref, g_new = _pair(small, Qs, dev)
    assert torch.equal(g_new, g_ref)
    # and the larger call once more, after the smaller one
    g_ref, g_new = _pair(big, Qb, dev)
    assert torch.equal(g_new, g_ref)


def test_noalloc_lmax1023_and_limit(dev):
    from paper_1202_6522_amd import shtn as S
    from paper_1202_6522_amd.shtn import Plan
    p, Qh = inputs.scalar_case(2)
    plan = Plan(p["L"], p["M"], p["nlat"], p["nphi"], device=dev)
    Q = torch.from_numpy(Qh).to(dev)
    g_ref, g_new = _pair(plan, Q, dev)
    assert torch.equal(g_new, g_ref)
    # two lmax-1023 fields need 48 MiB: refused, nothing launched
    assert S.shtn_work_bytes(plan.handle, 2) > S.SHTN_NOALLOC_MAX_BYTES
    Q2 = torch.cat([Q, Q])
    out = torch.zeros((2, plan.nlat, plan.nphi), dtype=torch.float64, device=dev)
    lib = S.load_library()
    rc = lib.shtn_synth_noalloc(plan.handle, Q2.data_ptr(), out.data_ptr(), 2,
                                torch.cuda.current_stream(dev).cuda_stream)
    assert rc == S.SHTN_EINVAL
    torch.cuda.synchronize(dev)
    assert torch.count_nonzero(out) == 0
