"""Largest field counts per call: SHTN_MAX_FIELDS (65535) scalar fields and
SHTN_MAX_VEC_FIELDS (16383) vector fields, at tiny shapes. The longitude and
Legendre launches put the field (group) index in the grid's y extent, which
reaches HIP's limit here; every transform still matches the oracle, and one
field more is refused before any launch.

Bars as for the other parity tests: max |gpu - oracle| / max |oracle| <= 1e-12.
"""
import numpy as np
import pytest

import oracle
from oracle import vector as V
from paper_1202_6522_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1202_6522_amd import shtn
    shtn.load_library()
    return torch.device("cuda:0")


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("algo", ["onthefly", "stored"])
def test_max_scalar_fields(algo, dev):
    from paper_1202_6522_amd import shtn
    L, M, nlat, nphi = 2, 2, 3, 8
    nf = shtn.SHTN_MAX_FIELDS
    rng = np.random.default_rng(65535)
    Q = inputs.draw_spectrum(rng, L, M, 1.0, nf)
    grid = rng.standard_normal((nf, nlat, nphi))
    plan = shtn.Plan(L, M, nlat, nphi, device=dev)
    if algo == "stored":
        plan.build_ptable()
        plan.set_algorithm("stored")
    g = plan.synth(to_dev(Q, dev)).cpu().numpy()
    assert rel(g, oracle.synth(Q, L, M, nlat, nphi)) <= 1e-12
    A = plan.analys(to_dev(grid, dev)).cpu().numpy()
    assert rel(A, oracle.analys(grid, L, M, nlat, nphi)) <= 1e-12
    St = plan.synth_adj(to_dev(grid, dev)).cpu().numpy()
    assert rel(St, oracle.synth_adj(grid, L, M, nlat, nphi)) <= 1e-12
    At = plan.analys_adj(to_dev(Q, dev)).cpu().numpy()
    assert rel(At, oracle.analys_adj(Q, L, M, nlat, nphi)) <= 1e-12
    with pytest.raises(shtn.ShtnError):
        plan.synth(to_dev(np.zeros((nf + 1, plan.nlm), complex), dev))


def test_max_vector_fields(dev):
    from paper_1202_6522_amd import shtn
    L, M, nlat, nphi = 3, 3, 4, 8
    nf = shtn.SHTN_MAX_VEC_FIELDS
    rng = np.random.default_rng(16383)
    S = inputs.draw_spectrum(rng, L, M, 1.0, nf)
    T = inputs.draw_spectrum(rng, L, M, 1.0, nf)
    plan = shtn.Plan(L, M, nlat, nphi, device=dev)
    vt, vp = plan.vec_synth(to_dev(S, dev), to_dev(T, dev))
    et, ep = V.vec_synth(S, T, L, M, nlat, nphi)
    assert rel(vt.cpu().numpy(), et) <= 1e-12
    assert rel(vp.cpu().numpy(), ep) <= 1e-12
    gt, gp = rng.standard_normal((2, nf, nlat, nphi))
    S2, T2 = plan.vec_analys(to_dev(gt, dev), to_dev(gp, dev))
    eS, eT = V.vec_analys(gt, gp, L, M, nlat, nphi)
    assert rel(S2.cpu().numpy(), eS) <= 1e-12
    assert rel(T2.cpu().numpy(), eT) <= 1e-12
    with pytest.raises(shtn.ShtnError):
        z = to_dev(np.zeros((nf + 1, plan.nlm), complex), dev)
        plan.vec_synth(z, z)
