"""Host-side tests of libshtn: exported symbols, argument validation and the
plan tables, with a numpy emulation of the kernels' algorithm (rescaled
recurrence, lanes starting from plan-time states) checked against the oracle.
No GPU is needed: plan construction is host code and no transform is called
here.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1202_6522_amd import inputs
from paper_1202_6522_amd import shtn as S

T_XP, T_SP, T_WQ, T_BETA, T_GAMMA, T_STY, T_STK, T_SEGE, T_SEGO, T_RSTY, T_RSTK, T_AU, T_SU, T_TIL, T_FIRST, \
    T_INJJ, T_INJY = range(17)
UI = S.UNIT_INTS
# unit fields
U_M, U_JS, U_JW, U_PB, U_J1, U_RST, U_ZERO = 3, 4, 5, 6, 7, 8, 9


@pytest.fixture(scope="module")
def lib():
    return S.load_library()


def test_exports_every_declared_symbol(lib):
    names = S.declared_functions()
    assert len(names) >= 25
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("args,why", [
    ((-1, 0, 4, 8), "lmax<0"),
    ((4, 5, 5, 16), "mmax>lmax"),
    ((4, 4, 0, 16), "nlat<1"),
    ((4, 4, 5, 8), "nphi<=2mmax"),
    ((4, 4, 5, 12), "nphi not a power of two"),
    ((0, 0, 1, 1), "nphi<2"),
])
def test_plan_rejects_bad_arguments(lib, args, why):
    assert not lib.shtn_plan(*args), why
    assert S.shtn_last_error_detail()


def test_calls_before_upload_and_null_pointers(lib):
    h = S.shtn_plan(8, 8, 9, 32)
    try:
        one = ctypes.c_void_p(16)
        assert lib.shtn_synth(h, one, ctypes.c_void_p(32), 1, one, None) == S.SHTN_ESTATE
        assert lib.shtn_synth(None, one, one, 1, one, None) == S.SHTN_EINVAL
        # field counts past one launch row per field are refused before anything else
        for fn in (lib.shtn_synth, lib.shtn_analys, lib.shtn_synth_adj, lib.shtn_analys_adj):
            assert fn(h, one, ctypes.c_void_p(32), 0, one, None) == S.SHTN_EINVAL
            assert fn(h, one, ctypes.c_void_p(32), 65536, one, None) == S.SHTN_EINVAL
            assert fn(h, one, ctypes.c_void_p(32), 65535, one, None) == S.SHTN_ESTATE
        v = [ctypes.c_void_p(16 * k) for k in range(1, 5)]
        for fn in (lib.shtn_vec_synth, lib.shtn_vec_analys, lib.shtn_vec_synth_adj, lib.shtn_vec_analys_adj):
            assert fn(h, *v, 16384, one, None) == S.SHTN_EINVAL
            assert fn(h, *v, 16383, one, None) == S.SHTN_ESTATE
        assert lib.shtn_work_bytes(h, 0) == 0
        assert lib.shtn_lm_index(h, 3, 4) == -1
        assert lib.shtn_lm_index(h, 8, 8) == S.shtn_nlm(h) - 1
        assert lib.shtn_plan_set_tiling(h, 3, 1, 1, 1, 1, 0, 0) == S.SHTN_EINVAL
        assert lib.shtn_plan_set_tiling(h, 1, 1, 1, 1, 1, 40, 0) == S.SHTN_EINVAL
        assert lib.shtn_plan_set_tiling(h, 1, 1, 3, 1, 0, 0, 0) == S.SHTN_EINVAL
        assert lib.shtn_plan_set_tiling(h, 1, 1, 2, 1, 0, 0, 0) == S.SHTN_EINVAL  # lp 1 x 2 waves: not built
        assert lib.shtn_plan_set_tiling(h, 1, 2, 2, 1, 0, 0, 0) == S.SHTN_OK
        assert lib.shtn_plan_set_tiling(h, 1, 1, 1, 3, 0, 0, 0) == S.SHTN_EINVAL  # fw 3
        assert lib.shtn_plan_set_tiling(h, 4, 1, 1, 4, 0, 0, 0) == S.SHTN_EINVAL  # fw 4 needs synth_lp <= 2
        # fw 4: the analysis takes fewer fields per wave (two, or one for analys_lp 8)
        assert lib.shtn_plan_set_tiling(h, 2, 8, 1, 4, 0, 0, 0) == S.SHTN_OK
        assert S.shtn_strerror(S.SHTN_EUNSUPPORTED) == "unsupported configuration"
    finally:
        S.shtn_plan_destroy(h)


@pytest.mark.parametrize("nlat", [2, 7, 32, 255, 1024])
def test_plan_grid_matches_oracle(nlat):
    h = S.shtn_plan(nlat - 1, nlat - 1, nlat, 1 << int(np.ceil(np.log2(2 * nlat))))
    try:
        x, w = S.shtn_get_grid(h, nlat)
        xo, wo = oracle.gauss(nlat, precision="ld")
        # the plan's long-double Newton in theta and the oracle's long-double
        # Newton in x agree to rounding
        assert np.max(np.abs(x - xo)) <= 2.3e-16
        assert np.max(np.abs(w / wo - 1)) < 1e-14
        sp = S.shtn_plan_table(h, T_SP)
        npair = (nlat + 1) // 2
        xs = x[:npair]
        tol = 1.2e-16 / (1 - np.abs(xs)) + 1e-15  # sin from rounded x vs the exact node
        assert np.all(np.abs(sp / np.sqrt((1 - xs) * (1 + xs)) - 1) < tol)
        assert abs(S.shtn_legendre_flops(h) - 8 * npair * S.shtn_nlm(h)) == 0
    finally:
        S.shtn_plan_destroy(h)


def _tables(h):
    return {k: S.shtn_plan_table(h, k) for k in range(17)}


def test_beta_gamma_tables():
    L, M = 70, 60
    h = S.shtn_plan(L, M, L + 1, 256)
    try:
        t = _tables(h)
        n_all, m_all = inputs.degree_order(L, M)
        j = n_all - m_all
        beta = t[T_BETA]
        assert np.all(beta[j == 0] == 1) and np.all(beta[j == 1] == 0)
        sel = j >= 2
        n, m = n_all[sel], m_all[sel]
        ref = -((n - 1.0) ** 2 - m**2) / ((2 * n - 1.0) * (2 * n - 3.0))
        np.testing.assert_allclose(beta[sel], ref, rtol=2e-16)
        # gamma_n = alpha_n 2^{-E}: gamma_n / gamma_{n-1} = a_n^m within a segment
        g = t[T_GAMMA]
        a = np.sqrt(np.abs(4.0 * n_all**2 - 1) / np.maximum(n_all**2 - m_all**2, 1))
        inseg = (j >= 1) & (j % 32 != 0)
        idx = np.nonzero(inseg)[0]
        np.testing.assert_allclose(g[idx] / g[idx - 1], a[idx], rtol=1e-15)
        assert np.all(g[j == 0] == 1)
        assert np.all(g >= 1) and np.max(g) < 2.0**200
    finally:
        S.shtn_plan_destroy(h)


def test_start_values_scaled_exponents():
    # P_m^m(x) = w 2^{-256 k}: compare with log2 of the closed form
    L, nlat = 2047, 2048
    h = S.shtn_plan(L, L, nlat, 4096)
    try:
        t = _tables(h)
        npair = nlat // 2
        sy = t[T_STY].reshape(L + 1, npair)
        sk = t[T_STK].reshape(L + 1, npair)
        sp = t[T_SP]
        m = np.arange(L + 1)[:, None]
        logamm = 0.5 * (np.concatenate([[0.0], np.cumsum(np.log2((2 * np.arange(1, L + 1) + 1) /
                                                                (2.0 * np.arange(1, L + 1))))])
                        - np.log2(4 * np.pi))
        ref = logamm[:, None] + m * np.log2(sp)[None, :]
        kept = np.ones_like(sk, dtype=bool)
        got = np.log2(np.abs(sy)) - 256.0 * sk
        err = np.abs(got - ref) / np.maximum(1, np.abs(ref))
        assert np.max(err[kept]) < 1e-12
        assert np.all(np.sign(sy[kept]) == np.broadcast_to((-1.0) ** m, sy.shape)[kept])
        pos = sk > 0
        assert np.all(np.abs(sy[pos]) < 1) and np.all(np.abs(sy[pos]) >= 2.0**-256)
        assert np.all(np.abs(sy[kept & ~pos]) >= 2.0**-256)
        # small-m values are plain doubles that match the oracle
        # (the oracle takes sin(theta) from its rounded x, which near the pole
        # carries ~1e-16/(1-x) relative error per power of sin)
        x = S.shtn_plan_table(h, T_XP)[:8]
        P = oracle.plm(4, 4, x)
        for mm in range(5):
            tol = mm * 1.2e-16 / (1 - x) + 1e-14
            assert np.all(np.abs(sy[mm, :8] / P[oracle.lm_index(4, mm, mm)] - 1) < tol)
    finally:
        S.shtn_plan_destroy(h)


def _lane_walk(t, L, M, npair, m, upto=None):
    """Yields (j, ua or ub, parity) along the kernels' per-lane recurrence for
    order m: every lane holds 0 until its start step (a multiple of 8), where
    it takes the state stored by the plan; segment shifts at multiples of 32.
    Vectorised over latitude pairs."""
    xp, beta = t[T_XP], t[T_BETA]
    sege, sego = t[T_SEGE], t[T_SEGO]
    sj = t[T_INJJ].reshape(M + 1, npair)[m]
    sy = t[T_INJY].reshape(M + 1, npair, 2)[m]
    base = oracle.lm_index(L, m, m)
    nj = L - m + 1 if upto is None else upto
    ua = np.zeros(npair)
    ub = np.zeros(npair)
    for j in range(0, nj, 2):
        if j > 0 and j % 32 == 0:
            sc = 2.0 ** sege[sego[m] + j // 32]
            ua *= sc
            ub *= sc
        if j % 8 == 0:
            go = sj == j
            ua = np.where(go, sy[:, 0], ua)
            ub = np.where(go, sy[:, 1], ub)
        ua = xp * ub + beta[base + j] * ua
        yield j, ua
        if j + 1 < L - m + 1 and j + 1 < nj:
            ub = xp * ua + beta[base + j + 1] * ub
            yield j + 1, ub


def emulate_legendre(t, L, M, nlat, Q=None, F=None):
    """numpy emulation of the kernels' per-lane algorithm: rescaled recurrence,
    segment rescaling, lanes starting from the plan's stored states, mirror
    fold.  Synthesis if Q is given (returns F[m][lat]), analysis if F is given
    (returns Q)."""
    npair = (nlat + 1) // 2
    wq, gamma = t[T_WQ], t[T_GAMMA]
    nlm = len(t[T_BETA])
    out = np.zeros((M + 1, nlat), complex) if Q is not None else np.zeros(nlm, complex)
    pairs = np.arange(npair)
    south = nlat - 1 - pairs
    for m in range(M + 1):
        base = oracle.lm_index(L, m, m)
        if Q is not None:
            E = np.zeros(npair, complex)
            O = np.zeros(npair, complex)
            for j, u in _lane_walk(t, L, M, npair, m):
                if j % 2 == 0:
                    E += gamma[base + j] * Q[base + j] * u
                else:
                    O += gamma[base + j] * Q[base + j] * u
            out[m, pairs] = E + O
            out[m, south] = E - O
        else:
            fe = wq * (F[m, pairs] + F[m, south])
            fo = wq * (F[m, pairs] - F[m, south])
            for j, u in _lane_walk(t, L, M, npair, m):
                out[base + j] = gamma[base + j] * np.sum((fe if j % 2 == 0 else fo) * u)
            if m == 0:
                out[base:base + L + 1] = out[base:base + L + 1].real
    return out


@pytest.mark.parametrize("L,M,nlat", [(40, 40, 41), (63, 50, 70), (30, 30, 33)])
def test_emulated_recurrence_matches_oracle(L, M, nlat):
    h = S.shtn_plan(L, M, nlat, 256)
    try:
        t = _tables(h)
        x, w = S.shtn_get_grid(h, nlat)
        rng = np.random.default_rng(L + M)
        Q = inputs.draw_spectrum(rng, L, M, 1.0)[0]
        F = emulate_legendre(t, L, M, nlat, Q=Q)
        P = oracle.plm(L, M, x)
        n_all, m_all = inputs.degree_order(L, M)
        ref = np.zeros((M + 1, nlat), complex)
        np.add.at(ref, m_all, Q[:, None] * P)
        assert np.max(np.abs(F - ref)) < 1e-13 * np.max(np.abs(ref))
        # analysis: Q_n^m = sum_i w_i P_n^m(x_i) F_m(theta_i)
        G = rng.standard_normal((M + 1, nlat)) + 1j * rng.standard_normal((M + 1, nlat))
        got = emulate_legendre(t, L, M, nlat, F=G)
        refq = np.sum(P * w[None, :] * G[m_all], axis=1)
        refq[m_all == 0] = refq[m_all == 0].real
        assert np.max(np.abs(got - refq)) < 1e-13 * np.max(np.abs(refq))
    finally:
        S.shtn_plan_destroy(h)


def test_emulated_guard_at_high_degree():
    # At L = 2047 some starts underflow double precision although the
    # functions later reach significant values: the guard must recover them.
    # Reference: the long-double oracle restricted to a few orders.
    L, nlat, nphi = 2047, 2048, 4096
    h = S.shtn_plan(L, L, nlat, nphi)
    try:
        t = _tables(h)
        x, _ = S.shtn_get_grid(h, nlat)
        ms = [900, 1100, 1500]
        Mx = max(ms)
        # emulate only the listed orders: zero spectrum elsewhere
        rng = np.random.default_rng(1)
        Q = np.zeros(S.shtn_nlm(h), complex)
        n_all, m_all = inputs.degree_order(L, L)
        sel = np.isin(m_all, ms)
        Q[sel] = (rng.standard_normal(sel.sum()) + 1j * rng.standard_normal(sel.sum()))
        t2 = dict(t)
        F = _emulate_orders(t2, L, L, nlat, Q, ms)
        rows = np.arange(0, nlat // 2, 7)
        gref = oracle.synth(Q, L, L, nlat, nphi, mlist=ms, rows=rows, precision="ld")
        phi = 2 * np.pi * np.arange(nphi) / nphi
        g = np.zeros((rows.size, nphi))
        for m in ms:
            g += 2 * np.real(F[m][rows][:, None] * np.exp(1j * m * phi)[None, :])
        assert np.max(np.abs(g - gref)) < 1e-11 * np.max(np.abs(gref))
        # and double precision without rescaling loses the rows whose starts underflow
        sk = t[T_STK].reshape(L + 1, nlat // 2)
        assert np.any(sk[ms][:, rows] > 0)
    finally:
        S.shtn_plan_destroy(h)


def _emulate_orders(t, L, M, nlat, Q, ms):
    """emulate_legendre restricted to a few orders (returns {m: F_m[lat]})."""
    npair = (nlat + 1) // 2
    gamma = t[T_GAMMA]
    pairs = np.arange(npair)
    out = {}
    for m in ms:
        base = oracle.lm_index(L, m, m)
        E = np.zeros(npair, complex)
        O = np.zeros(npair, complex)
        for j, u in _lane_walk(t, L, M, npair, m):
            if j % 2 == 0:
                E += gamma[base + j] * Q[base + j] * u
            else:
                O += gamma[base + j] * Q[base + j] * u
        F = np.zeros(nlat, complex)
        F[pairs] = E + O
        F[nlat - 1 - pairs] = E - O
        out[m] = F
    return out


def test_emulated_values_stay_in_range():
    # once started, the carried values stay far from under- and overflow:
    # lanes start from states of at least 2^-900 (the block start rule), and
    # the recurrence dips at most a few binary orders below its start
    L = 1023
    h = S.shtn_plan(L, L, L + 1, 2048)
    try:
        t = _tables(h)
        npair = (L + 2) // 2
        for m in [0, 1, 300, 700, 1000, 1023]:
            lo, hi = np.inf, 0.0
            for j, u in _lane_walk(t, L, L, npair, m):
                v = np.abs(u[u != 0])
                if v.size:
                    lo, hi = min(lo, v.min()), max(hi, v.max())
            assert hi < 1e3, (m, hi)
            assert lo > 2.0**-960, (m, lo)
    finally:
        S.shtn_plan_destroy(h)


@pytest.mark.parametrize("thr", [-200, -40])
def test_lane_starts_against_long_double_oracle(thr):
    # Sec. 3.5 guard and Sec. 3.1 polar threshold at plan time, checked with
    # the long-double oracle (its exponent range covers these values at
    # lmax 1023).  A lane's own start is the checkpoint (multiple of 8) that
    # opens the first block of 8 steps in which |P_n^m| reaches 2^thr; a
    # block of 64 latitude pairs starts at the earliest own start of its
    # lanes, and its lanes start there too when their state is a normal
    # double of at least 2^-900, else later (never after their own start).
    # So: no dropped term reaches the threshold, each started block's first
    # start is where one of its lanes first reaches it, a later start in a
    # block only follows a negligible state, and the stored state continues
    # the recurrence onto the true P_n^m.  thr = -200 is the default; -40 a
    # raised threshold set with shtn_plan_set_polar.
    L, nlat = 1023, 1024
    h = S.shtn_plan(L, L, nlat, 2048)
    if thr != -200:
        S.shtn_plan_set_polar(h, thr)
    try:
        t = _tables(h)
        npair = nlat // 2
        x = t[T_XP]
        sj = t[T_INJJ].reshape(L + 1, npair)
        sy = t[T_INJY].reshape(L + 1, npair, 2)
        for m in (0, 5, 200, 512, 800, 1000, 1023):
            nj = L - m + 1
            base = oracle.lm_index(L, m, m)
            assert np.all((sj[m] % 8 == 0) | (sj[m] == nj))
            Pall = np.abs(oracle.plm_raw(L, [m], x, precision="ld")[0, m:, :]).astype(np.float64)
            # the 8-step block maxima of |P| per checkpoint and pair
            nck = (nj + 7) // 8
            pad = np.zeros((nck * 8, npair))
            pad[:nj] = Pall
            bmax = pad.reshape(nck, 8, npair).max(axis=1)
            for b in range(npair // 64):
                lanes = slice(64 * b, 64 * b + 64)
                own = np.array([np.argmax(bmax[:, i] >= 2.0**(thr - 1)) * 8 if np.any(bmax[:, i] >= 2.0**(thr - 1))
                                else nj for i in range(64 * b, 64 * b + 64)])
                starts = sj[m, lanes]
                if starts.min() >= nj:
                    # a block that never starts: no lane of it reaches the threshold
                    assert np.all(bmax[:, lanes] < 2.0**thr), (m, b)
                    continue
                b0 = starts.min()
                # (the plan compares binary exponents: the threshold is met
                # from 2^(thr-1) on; the oracle may differ by a rounding there)
                assert abs(b0 - own.min()) <= 8, (m, b, b0, own.min())
                for i in range(64 * b, 64 * b + 64):
                    j = int(sj[m, i])
                    if j < nj:
                        assert np.all(Pall[:j, i] < 2.0**thr), (m, i)
                    else:
                        assert np.all(Pall[:, i] < 2.0**thr), (m, i)
                    if j > b0:
                        assert Pall[b0, i] < 2.0**-800, (m, i, j, b0, Pall[b0, i])
            # two steps from the stored state, at a few lanes of each kind
            for i in sorted({int(np.argmin(sj[m])), npair - 1, npair // 2, int(np.argmax(np.where(sj[m] < nj, sj[m], -1)))}):
                j = int(sj[m, i])
                if j >= nj:
                    continue
                P = oracle.plm_raw(L, [m], np.array([x[i]]), precision="ld")[0, m:, 0].astype(np.float64)
                ua, ub = sy[m, i]
                ua = x[i] * ub + t[T_BETA][base + j] * ua
                got = [ua * t[T_GAMMA][base + j]]
                if j + 1 < nj:
                    ub = x[i] * ua + t[T_BETA][base + j + 1] * ub
                    got.append(ub * t[T_GAMMA][base + j + 1])
                ref = P[j:j + len(got)]
                # Near the pole |P| grows slowly with n, so the next value is
                # the difference of two nearly equal terms and the rounding of
                # the stored pair is amplified (up to ~1e-10 relative for a
                # lane that starts at ~2^-890); a wrong state is off by O(1).
                np.testing.assert_allclose(got, ref, rtol=1e-9)
    finally:
        S.shtn_plan_destroy(h)


def _check_analysis_units(h, t, L, npair):
    """Pieces cover every order's degrees once, start where they may, hold
    the right restart slots; workgroup b runs on XCD b % 8, every order stays
    on one XCD, each XCD runs its pieces longest first (by the plan's time
    model) and the XCDs carry about equal work."""
    til = t[T_TIL]
    au = t[T_AU].reshape(-1, UI)
    sj = t[T_INJJ].reshape(L + 1, npair)
    lp, waves, nb = int(til[1]), int(til[6]), (npair + 63) // 64
    bf = S.shtn_plan_table(h, 17).reshape(L + 1, nb)
    ck = S.shtn_plan_table(h, 18).reshape(L + 1, -1, 2)
    bfw = np.full((L + 1, waves * lp), 1 << 30)
    bfw[:, :min(nb, waves * lp)] = bf[:, :waves * lp]
    bfw = bfw.reshape(L + 1, waves, lp)

    def unit_cost(u):
        # ns: 4600 set-up, per half pass of 8 steps 320 + 100 per pair slot
        # whose 64-pair block has started + 460 if start states are injected
        # (the busiest of the unit's waves of analys_lp slots each)
        m, js, j1 = int(u[U_M]), int(u[U_JS]), int(u[U_J1])
        if js >= j1:
            return 0
        tot = 4600
        for c in range(js, j1, 8):
            k = np.sum(bfw[m] <= c, axis=1)
            inj = np.array([(int(ck[m, c // 8, 0]) >> (w * lp)) & ((1 << lp) - 1) != 0 for w in range(waves)])
            tot += int(np.max(320 + 100 * k + 460 * inj))
        return tot

    xcd = np.arange(len(au)) % 8
    real = au[:, U_M] >= 0
    load = np.zeros(8)
    for x in range(8):
        q = au[(xcd == x) & real]
        cost = np.array([unit_cost(u) for u in q])
        assert np.all(np.diff(cost) <= 0), "units are ordered longest first"
        load[x] = cost.sum()
    # orders dealt largest first to the least loaded XCD: within one order's
    # cost of each other
    mcost = np.zeros(L + 1)
    for u in au[real]:
        mcost[int(u[U_M])] += unit_cost(u)
    assert load.max() - load.min() <= mcost.max() + 1
    assert np.all(au[~real][:, U_M] == -1)
    xcd = xcd[real]
    au = au[real]
    for m in range(L + 1):
        assert len(set(xcd[au[:, U_M] == m])) == 1
    cover = {}
    for u in au:
        m, js, jw, j0, j1, r = (int(v) for v in u[[U_M, U_JS, U_JW, U_PB, U_J1, U_RST]])
        cover.setdefault(m, []).append((j0, j1))
        assert (r < 0) == (j0 == 0)
        assert j0 % 32 == 0
        # the unit starts at a segment boundary no later than its first
        # started lane, and its window covers every start inside it
        assert j0 <= js <= j1 and (js - j0) % 32 == 0
        lanes = sj[m]
        assert not np.any((lanes >= j0) & (lanes < js)) or js == j0
        inside = lanes[(lanes >= js) & (lanes < j1)]
        if inside.size:
            assert jw >= inside.max()
        if js > j0:
            assert not np.any(lanes < js)
    for m in range(L + 1):
        segs = sorted(cover[m])
        assert segs[0][0] == 0 and segs[-1][1] == L - m + 1
        assert all(a[1] == b[0] for a, b in zip(segs, segs[1:]))
    return au


@pytest.mark.parametrize("split", [0, 128])
def test_restart_states_match_recurrence(split):
    L = 255
    npair = 128
    h = S.shtn_plan(L, L, 256, 512)
    try:
        if split:
            S.shtn_plan_set_tiling(h, 1, 2, 1, 1, 0, split, 0)
        t = _tables(h)
        # (0: automatic, 64-degree pieces at lmax 255)
        assert int(t[T_TIL][4]) == (split or 64)
        au = _check_analysis_units(h, t, L, npair)
        sj = t[T_INJJ].reshape(L + 1, npair)
        # a restart state equals the recurrence run from the lane starts
        ry = t[T_RSTY].reshape(-1, npair, 2)
        assert t[T_RSTK].size == 0
        assert au[au[:, U_RST] >= 0].shape[0] > 0
        for u in au[au[:, U_RST] >= 0][:6]:
            m, j0, r = int(u[U_M]), int(u[U_PB]), int(u[U_RST])
            last = {}
            for j, v in _lane_walk(t, L, L, npair, m, upto=j0):
                last[j % 2] = v
            sc = 2.0 ** t[T_SEGE][t[T_SEGO][m] + j0 // 32]
            live = sj[m] < j0
            # (numpy rounds the products separately; the host uses fused multiply-adds)
            for k in (0, 1):
                want = np.where(live, last[k] * sc, 0.0)
                np.testing.assert_allclose(ry[r, :, k], want, rtol=0,
                                           atol=1e-12 * max(np.max(np.abs(want)), 1e-300))
    finally:
        S.shtn_plan_destroy(h)


@pytest.mark.parametrize("shape", [(1023, 1023, 1024, 2048), (511, 511, 512, 1024)])
def test_analysis_units_at_workload_sizes(shape):
    # automatic pieces (256 degrees at lmax 1023), coverage, order per XCD
    L, M, nlat, nphi = shape
    h = S.shtn_plan(L, M, nlat, nphi)
    try:
        t = _tables(h)
        _check_analysis_units(h, t, L, (nlat + 1) // 2)
    finally:
        S.shtn_plan_destroy(h)


def test_synthesis_units_cover_all_work():
    for (L, M, nlat, pairing) in [(31, 31, 32, 1), (40, 33, 51, 1), (40, 33, 51, 0), (300, 300, 301, 1)]:
        h = S.shtn_plan(L, M, nlat, 1024)
        try:
            S.shtn_plan_set_tiling(h, 1, 8 if nlat > 256 else 1, 1, 1, pairing, 0, 0)
            t = _tables(h)
            su = t[T_SU].reshape(-1, UI)
            npair = (nlat + 1) // 2
            sj = t[T_INJJ].reshape(M + 1, npair)
            seen = np.zeros((M + 1, npair), int)
            for u in su:
                m = u[U_M]
                if m < 0:
                    continue
                pb = u[U_PB]
                blk = sj[m, pb:min(pb + 64, npair)]
                seen[m, pb:min(pb + 64, npair)] += 1
                started = blk[blk < L - m + 1]
                if u[U_ZERO]:
                    assert started.size == 0
                else:
                    assert u[U_JS] == started.min() and u[U_JW] == started.max()
            assert np.all(seen == 1)
        finally:
            S.shtn_plan_destroy(h)


@pytest.mark.parametrize("thr", [-200, -40])
def test_polar_cut_drops_only_negligible_latitudes(thr):
    # Sec. 3.1 polar optimisation: the first kept pair per order is where
    # max_n |P_n^m| first reaches 2^thr; checked with the long-double oracle,
    # whose range (1e-4951) covers these values.
    L, nlat = 1023, 1024
    h = S.shtn_plan(L, L, nlat, 2048)
    if thr != -200:
        S.shtn_plan_set_polar(h, thr)
    try:
        first = S.shtn_plan_table(h, T_FIRST)
        x = S.shtn_plan_table(h, T_XP)
        assert first[0] == 0 and np.all(np.diff(first) >= 0)
        for m in (200, 512, 800, 1000):
            i0 = int(first[m])
            assert 0 < i0 < nlat // 2
            xs = np.array([x[i0 - 1], x[i0]])
            P = oracle.plm(L, m, xs, precision="ld")
            rows = slice(oracle.lm_index(L, m, m), oracle.lm_index(L, L, m) + 1)
            Pm = np.abs(P[rows])
            assert Pm[:, 0].max() < 2.0**thr, m        # dropped pair: negligible
            assert Pm[:, 1].max() >= 2.0**(thr - 1), m # first kept pair: at the threshold
    finally:
        S.shtn_plan_destroy(h)


def test_batch_layout_and_state_errors(lib):
    shapes = [(63, 63, 64, 128), (31, 31, 32, 64), (63, 63, 64, 128), (20, 10, 25, 32)]
    hs = {}
    for s in shapes:
        if s not in hs:
            hs[s] = S.shtn_plan(*s)
    try:
        b = S.shtn_batch([hs[s] for s in shapes])
        try:
            q, g = S.shtn_batch_offsets(b, len(shapes))
            nq = [2 * inputs.nlm(L, M) for (L, M, _, _) in shapes]
            ng = [nlat * nphi for (_, _, nlat, nphi) in shapes]
            assert q == [0] + list(np.cumsum(nq))
            assert g == [0] + list(np.cumsum(ng))
            assert S.shtn_batch_device_bytes(b) > 0
            assert S.shtn_batch_work_bytes(b) >= 8 * (q[-1] + sum(
                2 * (M + 1) * nlat for (_, M, nlat, _) in shapes))
            assert S.shtn_batch_get_tiling(b) == [1, 1, 0, 0]
            # nothing uploaded: every device call is refused before any HIP call
            fake = ctypes.c_void_p(4096)
            assert lib.shtn_batch_synth(b, fake, ctypes.c_void_p(8192), fake, None) == S.SHTN_ESTATE
            assert lib.shtn_batch_analys(b, fake, ctypes.c_void_p(8192), fake, None) == S.SHTN_ESTATE
            assert lib.shtn_batch_capture(b, 0, fake, ctypes.c_void_p(8192), fake) == S.SHTN_ESTATE
            assert lib.shtn_batch_replay(b, 0, None) == S.SHTN_ESTATE
            assert lib.shtn_batch_upload(b, ctypes.c_void_p(4097), None) == S.SHTN_EINVAL
            for bad in [(3, 1, 0, 0), (1, 3, 0, 0), (1, 1, 2, 0), (1, 1, 0, 2), (4, 4, 0, 0)]:
                assert lib.shtn_batch_set_tiling(b, *bad) == S.SHTN_EINVAL
            assert lib.shtn_batch_get_algorithm(b) == S.SHTN_ALGO_ONTHEFLY
            assert lib.shtn_batch_set_algorithm(b, 2) == S.SHTN_EINVAL
            assert lib.shtn_batch_set_algorithm(b, S.SHTN_ALGO_STORED) == S.SHTN_OK  # no table yet: all on the fly
            assert lib.shtn_batch_get_algorithm(b) == S.SHTN_ALGO_STORED
            S.shtn_batch_set_tiling(b, 2, 4, 0, 0)
            assert lib.shtn_batch_get_algorithm(b) == S.SHTN_ALGO_STORED  # the tiling keeps the algorithm
            assert lib.shtn_batch_set_algorithm(b, S.SHTN_ALGO_ONTHEFLY) == S.SHTN_OK
            assert S.shtn_batch_get_tiling(b) == [2, 4, 0, 0]
            S.shtn_batch_set_tiling(b, 2, 2, 1, 1)
            assert S.shtn_batch_get_tiling(b) == [2, 2, 1, 1]
        finally:
            S.shtn_batch_destroy(b)
        assert not lib.shtn_batch(0, None)
        with pytest.raises(ValueError):
            S.shtn_batch([hs[shapes[0]], None])
    finally:
        for h in hs.values():
            S.shtn_plan_destroy(h)


def test_polar_threshold_setting():
    # shtn_plan_set_polar: range check, the plan reports the exponent, a
    # raised threshold only delays lane starts (never advances one) and cuts
    # at least as many polar latitudes, and the default restores the tables.
    L = 255
    h = S.shtn_plan(L, L, 256, 512)
    try:
        base = _tables(h)
        assert int(base[T_TIL][8]) == -200
        for bad in (-1001, 0, 5):
            with pytest.raises(S.ShtnError):
                S.shtn_plan_set_polar(h, bad)
        S.shtn_plan_set_polar(h, -30)
        t = _tables(h)
        assert int(t[T_TIL][8]) == -30
        assert np.all(t[T_INJJ] >= base[T_INJJ]) and np.any(t[T_INJJ] > base[T_INJJ])
        assert np.all(t[T_FIRST] >= base[T_FIRST])
        # units still cover every order's degrees once
        au = t[T_AU].reshape(-1, UI)
        au = au[au[:, U_M] >= 0]
        for m in (0, 100, 255):
            segs = sorted((int(u[U_PB]), int(u[U_J1])) for u in au if u[U_M] == m)
            assert segs[0][0] == 0 and segs[-1][1] == L - m + 1
        S.shtn_plan_set_polar(h, -200)
        again = _tables(h)
        for k in (T_INJJ, T_INJY, T_FIRST, T_AU, T_SU, T_RSTY):
            assert np.array_equal(again[k], base[k]), k
    finally:
        S.shtn_plan_destroy(h)


@pytest.mark.parametrize("shape", [(63, 40, 65, 128), (255, 255, 256, 512), (1023, 1023, 1024, 2048),
                                   (300, 300, 2100, 1024)])
def test_block_start_tables(shape):
    # Tables 17 and 18 summarise the lane starts (table 15) per block of 64
    # latitude pairs: the first start step of each block, and per checkpoint
    # (every 8 steps) the blocks with a lane starting there and the blocks
    # with a lane started by then.  The analysis kernel runs only the pair
    # slots of started blocks and injects start states only where a bit is
    # set, so these must agree exactly with the lane starts.
    L, M, nlat, nphi = shape
    h = S.shtn_plan(L, M, nlat, nphi)
    try:
        npair = (nlat + 1) // 2
        nb = (npair + 63) // 64
        inj = S.shtn_plan_table(h, 15).reshape(M + 1, npair)
        bf = S.shtn_plan_table(h, 17).reshape(M + 1, nb)
        ck = S.shtn_plan_table(h, 18).reshape(M + 1, -1, 2)
        nck = ck.shape[1]
        assert nck == (L + 32) // 8 + 2
        for m in range(M + 1):
            nj = L - m + 1
            for b in range(nb):
                js = inj[m, 64 * b:64 * (b + 1)]
                started = js[js < nj]
                assert bf[m, b] == (started.min() if started.size else nj)
                if b >= 32:
                    continue
                bit = np.uint32(1 << b)
                starts_at = np.zeros(nck, bool)
                starts_at[np.unique(started // 8)] = True
                assert np.all(started % 8 == 0)
                assert np.array_equal((ck[m, :, 0] & bit) != 0, starts_at)
                k = np.arange(nck)
                assert np.array_equal((ck[m, :, 1] & bit) != 0, (8 * k >= bf[m, b]) & (bf[m, b] < nj))
    finally:
        S.shtn_plan_destroy(h)


def test_polar_threshold_keeps_start_states_normal(lib):
    # A very low threshold (lanes start far into the evanescent region)
    # would store start states below DBL_MIN, denormals that have lost bits;
    # shtn_plan_set_polar refuses such a threshold and leaves the plan as it
    # was.  At lmax 1023 the lowest accepted one is about -900; every stored
    # state there is 0 or a normal double.
    L = 1023
    h = S.shtn_plan(L, L, L + 1, 2 * (L + 1))
    try:
        base = _tables(h)
        for t in (-1000, -960, -920):
            assert lib.shtn_plan_set_polar(h, t) == S.SHTN_EINVAL, t
            now = _tables(h)
            assert int(now[T_TIL][8]) == -200
            for k in (T_INJJ, T_INJY, T_AU, T_SU, T_RSTY):
                assert np.array_equal(now[k], base[k]), (t, k)
        S.shtn_plan_set_polar(h, -900)
        y = _tables(h)[T_INJY]
        nz = np.abs(y[y != 0])
        assert nz.size and nz.min() >= np.finfo(np.float64).tiny
        # lanes start earlier than at the default threshold, never later
        assert np.all(_tables(h)[T_INJJ] <= base[T_INJJ])
    finally:
        S.shtn_plan_destroy(h)


@pytest.mark.parametrize("shape", [(0, 0, 1, 2), (31, 31, 32, 64), (63, 40, 65, 128), (1023, 1023, 1024, 2048)])
def test_ptable_geometry_and_states(lib, shape):
    """Stored-P table size: per order m (nj = lmax - m + 1) ceil(nj/2) even and
    floor(nj/2) odd degree rows, each parity in block rows of 16 x ceil(npair/16)
    blocks of 16 x 16 doubles, after the block offsets padded to 256 bytes."""
    L, M, nlat, nphi = shape
    h = S.shtn_plan(L, M, nlat, nphi)
    try:
        npt = ((nlat + 1) // 2 + 15) // 16
        nblocks = sum(((L - m + 2) // 2 + 15) // 16 * npt + ((L - m + 1) // 2 + 15) // 16 * npt
                      for m in range(M + 1))
        head = ((M + 1) * 2 * 8 + 255) // 256 * 256
        assert S.shtn_ptable_bytes(h) == head + nblocks * 2048
        if shape[0] == 1023:
            assert abs(S.shtn_ptable_bytes(h) / 2.2e9 - 1) < 0.05
        # no table yet: the stored algorithm is refused, building needs an upload
        assert lib.shtn_plan_set_algorithm(h, S.SHTN_ALGO_STORED) == S.SHTN_ESTATE
        assert lib.shtn_plan_set_algorithm(h, 4) == S.SHTN_EINVAL
        assert lib.shtn_plan_set_algorithm(h, S.SHTN_ALGO_STORED_SYNTH) == S.SHTN_ESTATE
        assert S.shtn_plan_get_algorithm(h) == S.SHTN_ALGO_ONTHEFLY
        assert lib.shtn_ptable_build(h, ctypes.c_void_p(4096), 1 << 40, None) == S.SHTN_ESTATE
        assert S.shtn_ptable_get_tiling(h) == [4, 2, 4, 2]
        for bad in [(3, 1, 1, 1), (1, 4, 1, 1), (1, 1, 8, 1), (1, 1, 1, 0)]:
            assert lib.shtn_ptable_set_tiling(h, *bad) == S.SHTN_EINVAL
        S.shtn_ptable_set_tiling(h, 2, 1, 4, 2)
        assert S.shtn_ptable_get_tiling(h) == [2, 1, 4, 2]
        S.shtn_ptable_release(h)
        assert S.shtn_plan_get_algorithm(h) == S.SHTN_ALGO_ONTHEFLY
        one = ctypes.c_void_p(16)
        assert lib.shtn_plan_tune_algorithm(h, one, ctypes.c_void_p(32), ctypes.c_void_p(48), 1, one, None,
                                            1, None) == S.SHTN_ESTATE
    finally:
        S.shtn_plan_destroy(h)
