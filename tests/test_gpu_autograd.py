"""Differentiable SHT on the GPU: autograd through the hand-written adjoints.

Workload of the differentiable case: 16 fields, lmax = mmax = 511, nlat = 512,
nphi = 1024, spectra N(0,1) (n+1)^-1.5 (target Q_T, then start Q_0).  Loss
L = sum_b sum_{i,k} w_i (S Q_b - T_b)_{ik}^2 with T = S Q_T.

Bars (written per test):
  - central finite differences, h = 1e-6, on 200 seeded real coordinates of
    Q_0, in the residual form L+ - L- = sum w (r+ - r-)(r+ + r-) of each
    field's own loss: per-coordinate |g_FD - g| / |g| <= 1e-6;
  - the gradient against the oracle's transpose, 2 S^T (w (S Q_0 - T)) computed
    entirely by the oracle: max |diff| / max |oracle| <= 1e-10 (lmax 511);
  - torch.autograd.gradcheck of all four Functions at small sizes.
"""
import numpy as np
import pytest

import oracle
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


@pytest.fixture(scope="module")
def grad_setup(dev):
    from paper_1202_6522_amd.shtn import Plan
    from paper_1202_6522_amd.autograd import synth
    p, QT, Q0 = inputs.grad_case()
    plan = Plan(p["L"], p["M"], p["nlat"], p["nphi"], device=dev)
    _, w = plan.grid()
    wd = torch.from_numpy(w).to(dev).view(1, -1, 1)
    T = plan.synth(torch.from_numpy(QT).to(dev))
    Q = torch.from_numpy(Q0).to(dev).requires_grad_(True)
    loss = (wd * (synth(Q, plan) - T) ** 2).sum()
    loss.backward()
    return dict(p=p, QT=QT, Q0=Q0, plan=plan, wd=wd, T=T, grad=Q.grad.detach().clone())


def test_gradient_finite_differences(grad_setup, dev):
    s = grad_setup
    p, plan, wd, T, G = s["p"], s["plan"], s["wd"], s["T"], s["grad"]
    L, M = p["L"], p["M"]
    nf, nlm = s["Q0"].shape
    _, m_all = inputs.degree_order(L, M)
    rng = np.random.default_rng(inputs.SEED_BASE + 40)
    coords = []
    while len(coords) < 200:
        b = int(rng.integers(nf))
        i = int(rng.integers(nlm))
        part = int(rng.integers(2))
        if part == 1 and m_all[i] == 0:
            continue  # Im Q_n^0 is not a coordinate of the transform
        coords.append((b, i, part))
    h = 1e-6
    Q0 = torch.from_numpy(s["Q0"]).to(dev)
    worst = 0.0
    for c0 in range(0, len(coords), 50):
        chunk = coords[c0:c0 + 50]
        Qp = Q0[[b for b, _, _ in chunk]].clone()
        Qm = Qp.clone()
        for r, (b, i, part) in enumerate(chunk):
            d = h if part == 0 else 1j * h
            Qp[r, i] += d
            Qm[r, i] -= d
        Tb = T[[b for b, _, _ in chunk]]
        rp = plan.synth(Qp) - Tb
        rm = plan.synth(Qm) - Tb
        dL = (wd * (rp - rm) * (rp + rm)).sum(dim=(1, 2))
        fd = (dL / (2 * h)).cpu().numpy()
        for r, (b, i, part) in enumerate(chunk):
            g = G[b, i].item()
            g = g.real if part == 0 else g.imag
            err = abs(fd[r] - g) / abs(g)
            worst = max(worst, err)
            assert err <= 1e-6, (b, i, part, fd[r], g)
    print("finite differences: worst per-coordinate relative error %.3e" % worst)


def test_gradient_vs_oracle_transpose(grad_setup):
    s = grad_setup
    p = s["p"]
    L, M, nlat, nphi = p["L"], p["M"], p["nlat"], p["nphi"]
    fields = list(range(16))
    _, w = oracle.gauss(nlat)
    Q0 = s["Q0"][fields]
    QT = s["QT"][fields]
    r = oracle.synth(Q0, L, M, nlat, nphi) - oracle.synth(QT, L, M, nlat, nphi)
    gref = oracle.synth_adj(2.0 * w[None, :, None] * r, L, M, nlat, nphi)
    g = s["grad"][fields].cpu().numpy()
    err = np.max(np.abs(g - gref)) / np.max(np.abs(gref))
    print("gradient vs oracle transpose: %.3e" % err)
    assert err <= 1e-10


def test_analysis_gradient(dev):
    # loss |A g - h|^2 over the spectrum; the gradient is 2 A^T (A g - h)
    from paper_1202_6522_amd.shtn import Plan
    from paper_1202_6522_amd.autograd import analys
    L, nlat, nphi = 63, 64, 128
    plan = Plan(L, L, nlat, nphi, device=dev)
    rng = np.random.default_rng(5)
    g0 = rng.standard_normal((2, nlat, nphi))
    hq = inputs.draw_spectrum(rng, L, L, 1.0, 2)
    g = torch.from_numpy(g0).to(dev).requires_grad_(True)
    hd = torch.from_numpy(hq).to(dev)
    loss = (analys(g, plan) - hd).abs().pow(2).sum()
    loss.backward()
    R = oracle.analys(g0, L, L, nlat, nphi) - hq
    R[:, :L + 1] = R[:, :L + 1].real  # Im Q_n^0 is not an output of the analysis
    gref = oracle.analys_adj(2.0 * R, L, L, nlat, nphi)
    err = np.max(np.abs(g.grad.cpu().numpy() - gref)) / np.max(np.abs(gref))
    assert err <= 1e-11


def test_gradcheck_small(dev):
    from paper_1202_6522_amd.shtn import Plan
    from paper_1202_6522_amd import autograd as AG
    L, nlat, nphi = 6, 7, 16
    plan = Plan(L, L, nlat, nphi, device=dev)
    rng = np.random.default_rng(9)
    Q = torch.from_numpy(inputs.draw_spectrum(rng, L, L, 0.0, 2)).to(dev).requires_grad_(True)
    g = torch.from_numpy(rng.standard_normal((2, nlat, nphi))).to(dev).requires_grad_(True)
    # Im Q_n^0 is ignored by the transforms: its derivative is 0 on both sides
    assert torch.autograd.gradcheck(lambda q: AG.SynthFn.apply(q, plan), (Q,), eps=1e-6, atol=1e-9)
    assert torch.autograd.gradcheck(lambda x: AG.AnalysFn.apply(x, plan), (g,), eps=1e-6, atol=1e-9)
    assert torch.autograd.gradcheck(lambda x: AG.SynthAdjFn.apply(x, plan), (g,), eps=1e-6, atol=1e-9)
    assert torch.autograd.gradcheck(lambda q: AG.AnalysAdjFn.apply(q, plan), (Q,), eps=1e-6, atol=1e-9)
