"""GPU parity: the HIP path (through the C interface) against the CPU oracle.

Bar (written per test): max |gpu - oracle| / max |oracle| over each output
array <= 1e-11 for lmax <= 255.  The full-array comparisons at lmax 1023 and
the long-double ones at lmax 4095 are in test_gpu_parity_full.py.
"""
import numpy as np
import pytest

import oracle
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


def make_plan(L, M, nlat, nphi, dev, **tiling):
    from paper_1202_6522_amd.shtn import Plan
    return Plan(L, M, nlat, nphi, device=dev, tiling=tiling or None)


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("case", [0, 1])
def test_scalar_cases_full(case, dev):
    p, Q = inputs.scalar_case(case)
    L, M, nlat, nphi = p["L"], p["M"], p["nlat"], p["nphi"]
    plan = make_plan(L, M, nlat, nphi, dev)
    g = plan.synth(to_dev(Q, dev)).cpu().numpy()
    gref = oracle.synth(Q, L, M, nlat, nphi)
    assert rel(g, gref) <= 1e-11
    # analysis of the oracle's grid
    R = plan.analys(to_dev(gref, dev)).cpu().numpy()
    Rref = oracle.analys(gref, L, M, nlat, nphi)
    assert rel(R, Rref) <= 1e-11
    assert np.all(R[:, :L + 1].imag == 0)
    # round trip on the GPU
    R2 = plan.analys(plan.synth(to_dev(Q, dev))).cpu().numpy()
    assert rel(R2, Q) <= 1e-11


EDGE = [
    (0, 0, 1, 2),
    (1, 1, 2, 4),
    (1, 0, 3, 2),
    (5, 3, 7, 16),
    (12, 12, 13, 32),
    (40, 33, 51, 128),
    (64, 64, 65, 256),
    (30, 30, 45, 64),
    (100, 20, 101, 64),
    (127, 127, 128, 256),
    (255, 200, 256, 1024),
]


@pytest.mark.parametrize("shape", EDGE)
def test_edge_shapes_all_transforms(shape, dev):
    L, M, nlat, nphi = shape
    rng = np.random.default_rng(sum(shape))
    nf = 3
    Q = inputs.draw_spectrum(rng, L, M, 1.0, nf)
    Q[:, :L + 1] += 0.25j  # must be ignored
    plan = make_plan(L, M, nlat, nphi, dev)
    g = plan.synth(to_dev(Q, dev)).cpu().numpy()
    assert rel(g, oracle.synth(Q, L, M, nlat, nphi)) <= 1e-11
    grid = rng.standard_normal((nf, nlat, nphi))
    A = plan.analys(to_dev(grid, dev)).cpu().numpy()
    assert rel(A, oracle.analys(grid, L, M, nlat, nphi)) <= 1e-11
    St = plan.synth_adj(to_dev(grid, dev)).cpu().numpy()
    assert rel(St, oracle.synth_adj(grid, L, M, nlat, nphi)) <= 1e-11
    At = plan.analys_adj(to_dev(Q, dev)).cpu().numpy()
    assert rel(At, oracle.analys_adj(Q, L, M, nlat, nphi)) <= 1e-11


@pytest.mark.parametrize("tiling", [
    dict(synth_lp=1, analys_lp=4, fw=1, m_pairing=0),
    dict(synth_lp=2, analys_lp=8, fw=1, m_pairing=1, split=64),
    dict(synth_lp=4, analys_lp=4, fw=2, m_pairing=1),
    dict(synth_lp=1, analys_lp=4, fw=2, m_pairing=0, split=32),
    dict(synth_lp=4, analys_lp=8, fw=1, m_pairing=1, split=96),
    dict(synth_lp=1, analys_lp=2, analys_waves=2, fw=1, m_pairing=0, split=64),
    dict(synth_lp=2, analys_lp=4, analys_waves=2, fw=2, m_pairing=1),
    dict(synth_lp=1, analys_lp=4, analys_waves=4, fw=1, m_pairing=0, split=32),
    # FFT workgroups of one row (one wave) and of three rows (a ragged last block)
    dict(synth_lp=1, analys_lp=4, fw=1, m_pairing=0, fft_rows=1),
    dict(synth_lp=1, analys_lp=4, fw=2, m_pairing=0, fft_rows=3),
    dict(synth_lp=1, analys_lp=2, analys_waves=2, fw=4, m_pairing=0),
    dict(synth_lp=2, analys_lp=2, fw=4, m_pairing=1, split=64),
    dict(synth_lp=2, analys_lp=2, fw=4, m_pairing=0, fft_rows=1),
    dict(synth_lp=1, analys_lp=8, fw=4, m_pairing=1),
])
def test_tilings_agree(tiling, dev):
    L, M, nlat, nphi = 255, 255, 256, 512
    rng = np.random.default_rng(3)
    Q = inputs.draw_spectrum(rng, L, M, 1.5, 3)
    base = make_plan(L, M, nlat, nphi, dev)
    plan = make_plan(L, M, nlat, nphi, dev, **tiling)
    Qd = to_dev(Q, dev)
    g0 = base.synth(Qd).cpu().numpy()
    g1 = plan.synth(Qd).cpu().numpy()
    # the per-lane synthesis arithmetic does not depend on the tiling
    np.testing.assert_array_equal(g0, g1)
    gd = to_dev(g0, dev)
    a0 = base.analys(gd).cpu().numpy()
    a1 = plan.analys(gd).cpu().numpy()
    assert rel(a1, a0) <= 1e-13
    assert rel(a1, Q) <= 1e-11


def test_adjoint_dot_products(dev):
    L, M, nlat, nphi = 200, 180, 211, 512
    rng = np.random.default_rng(12)
    plan = make_plan(L, M, nlat, nphi, dev)
    Q = inputs.draw_spectrum(rng, L, M, 0.5, 2)
    h = inputs.draw_spectrum(rng, L, M, 0.5, 2)
    g = rng.standard_normal((2, nlat, nphi))
    f = rng.standard_normal((2, nlat, nphi))
    SQ = plan.synth(to_dev(Q, dev)).cpu().numpy()
    Stg = plan.synth_adj(to_dev(g, dev)).cpu().numpy()
    lhs = np.sum(SQ * g)
    rhs = np.sum(Q.real * Stg.real + Q.imag * Stg.imag)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(SQ * g))
    Af = plan.analys(to_dev(f, dev)).cpu().numpy()
    Ath = plan.analys_adj(to_dev(h, dev)).cpu().numpy()
    lhs = np.sum(Af.real * h.real + Af.imag * h.imag)
    rhs = np.sum(f * Ath)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(f * Ath))


def test_lmax2047_underflow_guard_and_wide_analysis(dev):
    # lmax 2047: P_m^m underflows double precision near the poles for large m
    # although P_n^m later matters (the plan-time guard), and an analysis unit
    # spans 1024 latitude pairs (two waves of 8 pairs per lane).  Synthesis on
    # selected orders against the long-double oracle; round trip in full.
    L, nlat, nphi = 2047, 2048, 4096
    plan = make_plan(L, L, nlat, nphi, dev)
    assert plan.tiling()["analys_waves"] == 2
    rng = np.random.default_rng(2047)
    ms = [0, 700, 1200, 1600, 2000, 2047]
    Q = np.zeros((1, plan.nlm), complex)
    n_all, m_all = inputs.degree_order(L, L)
    sel = np.isin(m_all, ms)
    Q[0, sel] = (rng.standard_normal(sel.sum()) + 1j * rng.standard_normal(sel.sum())) \
        * (n_all[sel] + 1.0) ** -1.0
    Q[0, m_all == 0] = Q[0, m_all == 0].real
    g = plan.synth(to_dev(Q, dev))
    rows = np.array([0, 1, 5, 40, 200, 600, 1023, 1024, 1500, 2040, 2047])
    gref = oracle.synth(Q, L, L, nlat, nphi, mlist=ms, rows=rows, precision="ld")
    assert rel(g.cpu().numpy()[0][rows], gref[0]) <= 1e-10
    R = plan.analys(g).cpu().numpy()
    err = np.max(np.abs(R - Q)) / np.max(np.abs(Q))
    print("lmax 2047 round trip: %.3e" % err)
    assert err <= 1e-10


def test_paper_accuracy_protocol(dev):
    # Sec. 3.5: coefficients uniform in [-1, 1], backward then forward
    # transform; eps_max < 1e-11 for N < 2048.
    for L in (255, 1023):
        rng = np.random.default_rng(L)
        Q = inputs.draw_spectrum(rng, L, L, 0.0, 1, dist="uniform")
        plan = make_plan(L, L, L + 1, 2 * (L + 1), dev)
        R = plan.analys(plan.synth(to_dev(Q, dev))).cpu().numpy()
        eps_max = np.max(np.abs(R - Q))
        eps_rms = np.sqrt(2.0 / ((L + 1) * (L + 2)) * np.sum(np.abs(R - Q) ** 2))
        print("paper protocol L=%d: eps_max %.3e eps_rms %.3e" % (L, eps_max, eps_rms))
        assert eps_max < 1e-11


def test_deterministic_repeats(dev):
    p, Q = inputs.scalar_case(1)
    plan = make_plan(p["L"], p["M"], p["nlat"], p["nphi"], dev)
    Qd = to_dev(Q, dev)
    g0 = plan.synth(Qd)
    a0 = plan.analys(g0)
    for _ in range(5):
        assert torch.equal(plan.synth(Qd), g0)
        assert torch.equal(plan.analys(g0), a0)


def test_nan_propagates(dev):
    L = 31
    plan = make_plan(L, L, 32, 64, dev)
    Q = inputs.draw_spectrum(np.random.default_rng(0), L, L, 1.0)
    Q[0, oracle.lm_index(L, 5, 3)] = np.nan
    g = plan.synth(to_dev(Q, dev)).cpu().numpy()
    assert np.isnan(g).any()
    torch.cuda.synchronize()


def test_bad_calls_raise(dev):
    from paper_1202_6522_amd import shtn as S
    plan = make_plan(31, 31, 32, 64, dev)
    with pytest.raises(ValueError):
        plan.synth(torch.zeros(10, dtype=torch.complex128, device=dev))
    with pytest.raises(ValueError):
        plan.analys(torch.zeros(32, 64, dtype=torch.float32, device=dev))
    # analysis units cover at most 4096 latitudes (2048 pairs)
    big = make_plan(4200, 100, 4201, 256, dev)
    with pytest.raises(S.ShtnError):
        big.analys(torch.zeros(4201, 256, dtype=torch.float64, device=dev))


def test_polar_threshold_error_bound(dev):
    # Sec. 3.1 polar optimisation with a raised threshold 2^-30: every
    # dropped term has |P_n^m| < 2^-30, so the synthesis moves by at most
    # 2 2^-30 sum|Q| (F_m enters the grid with weight <= 2) and the analysis
    # by at most 2^-30 sum_i w_i |F_m| <= 2^-30 (sum w = 2) (2 pi max|f|).
    # The default threshold must not move at all relative to itself.
    from paper_1202_6522_amd import shtn as S
    L = 511
    rng = np.random.default_rng(inputs.SEED_BASE + 40)
    Qh = inputs.draw_spectrum(rng, L, L, 1.5, 1)
    Q = torch.from_numpy(Qh).to(dev)
    exact = S.Plan(L, L, L + 1, 2 * (L + 1), device=dev)
    cut = S.Plan(L, L, L + 1, 2 * (L + 1), device=dev, polar_log2=-30)
    assert cut.polar_log2() == -30 and exact.polar_log2() == -200
    g0 = exact.synth(Q)
    g1 = cut.synth(Q)
    dg = float((g1 - g0).abs().max())
    bound_s = 2.0 * 2.0**-30 * float(np.abs(Qh).sum())
    assert 0.0 < dg <= bound_s, (dg, bound_s)
    a0 = exact.analys(g0)
    a1 = cut.analys(g0)
    da = float((a1 - a0).abs().max())
    bound_a = 2.0**-30 * 2.0 * 2.0 * np.pi * float(g0.abs().max())
    assert 0.0 < da <= bound_a, (da, bound_a)
    # back to the default: identical to the plan that never changed
    cut.set_polar(-200)
    assert torch.equal(cut.synth(Q), g0)
    assert torch.equal(cut.analys(g0), a0)
