"""Pins of the long-double instantiation of the oracle against 40-digit mpmath.

The long-double oracle is the reference of the GPU tests at lmax 2047 and
4095, where the P_m^m that start the recurrence of Sec. 3.2 (eq. rec) fall
below the range of double although P_n^m later reaches O(1) (the case the
scaled-exponent guard of Sec. 3.5 exists for).  These tests pin it to an
independent high-precision reference:

- the mpmath reference itself: the recurrence of Sec. 3.2 run in 40-digit
  arithmetic, checked against the closed form of the definition of Sec. 2.1
  (the m-th derivative of P_n, a terminating hypergeometric polynomial in
  (1-x)/2, times (-1)^m sin^m(theta) and the orthonormal factor) at spots far
  outside the double range, and that closed form against mpmath's own
  Ferrers function ``mpmath.legenp`` at ordinary spots;
- ``oracle.plm_raw(..., "ld")`` (long double, before any rounding to double)
  against that reference at lmax 2047 and 4095 for m in {700, 1200, 1600,
  2000, 3000, 4000} (those <= lmax), at the three most polar Gauss nodes, one
  mid-latitude node, and the node nearest the pole at which P_m^m underflows
  double while P_n^m still reaches O(1) by n = lmax.  Bar: 2e-16 of the
  column's largest |P|.  The long-double rounding over a few thousand steps
  stays below 8e-17; a copy of the oracle with its long-double square root
  bound to the double one (a slip in the macro block of shtn_oracle.c) misses
  by 1e-15 to 2e-13 on these columns.  A column whose start P_m^m lies below
  even the long-double range must stay below 1e-300 throughout;
- ``oracle.plm(..., "ld")`` (the values rounded to double) on the same
  columns to 3e-16 of the largest |P|; at the underflow node the double
  instantiation is off by more than a tenth of the largest |P| (its start
  flushes to 0 or to a denormal of a few bits), which is why the long double
  one serves as the reference;
- the Gauss nodes of nlat 2048 and 4096 against a 40-digit Newton iteration;
- ``oracle.synth(..., precision="ld")`` at lmax 2047 on the spectrum of the GPU
  guard test (orders {0, 700, 1200, 1600, 2000, 2047}) against a 40-digit
  synthesis at sampled latitudes and longitudes, to 1e-15 of max |f|.
"""
import math

import numpy as np
import pytest

import oracle

mp = pytest.importorskip("mpmath")
DPS = 40


@pytest.fixture(autouse=True)
def _precision():
    with mp.workdps(DPS):
        yield


def ld_to_mp(v):
    """Exact value of a numpy longdouble (its shortest round-trip decimal)."""
    return mp.mpf(np.format_float_scientific(np.longdouble(v), unique=True))


def mp_coeffs(L, m):
    """a_n^m and b_n^m of Sec. 3.2 for n = m+2..L, and a_m^m, a_{m+1}^m."""
    amm = mp.sqrt(mp.fprod([mp.mpf(2 * k + 1) / (2 * k) for k in range(1, m + 1)]) / (4 * mp.pi))
    a1 = mp.sqrt(mp.mpf(2 * m + 3))
    a, b = [], []
    for n in range(m + 2, L + 1):
        nn, mm, n1 = mp.mpf(n) ** 2, mp.mpf(m) ** 2, mp.mpf(n - 1) ** 2
        a.append(mp.sqrt((4 * nn - 1) / (nn - mm)))
        b.append(-mp.sqrt(mp.mpf(2 * n + 1) / (2 * n - 3) * (n1 - mm) / (nn - mm)))
    return amm, a1, a, b


def mp_column(L, m, x, co):
    """[P_m^m(x), ..., P_L^m(x)] by the recurrence of Sec. 3.2 in mpmath."""
    amm, a1, a, b = co
    x = mp.mpf(x)
    s = mp.sqrt((1 - x) * (1 + x))
    p0 = (-1) ** m * amm * s ** m
    col = [p0]
    if m + 1 <= L:
        col.append(a1 * x * p0)
    for k in range(len(a)):
        col.append(a[k] * x * col[-1] + b[k] * col[-2])
    return col


def mp_closed_form(n, m, x):
    """P_n^m of Sec. 2.1 (orthonormal, with the (-1)^m factor) in closed form:
    (-1)^m sin^m(theta) d^m P_n/dx^m, where
    d^m P_n/dx^m = (n+m)! / (2^m m! (n-m)!) 2F1(m-n, n+m+1; m+1; (1-x)/2)
    is a polynomial (the series terminates), times sqrt((2n+1)/(4 pi)
    (n-m)!/(n+m)!)."""
    x = mp.mpf(x)
    s = mp.sqrt((1 - x) * (1 + x))
    c = mp.sqrt((2 * n + 1) / (4 * mp.pi) * mp.factorial(n + m) / mp.factorial(n - m)) \
        / (2 ** m * mp.factorial(m))
    return (-1) ** m * c * s ** m * mp.hyp2f1(m - n, n + m + 1, m + 1, (1 - x) / 2)


def test_mp_reference_against_closed_forms():
    # the closed form against mpmath's Ferrers function where that converges
    for n, m, x in [(5, 3, 0.3), (300, 150, 0.3), (900, 400, -0.7), (2047, 700, 0.95)]:
        ferrers = mp.sqrt((2 * n + 1) / (4 * mp.pi) * mp.factorial(n - m) / mp.factorial(n + m)) \
            * mp.legenp(n, m, mp.mpf(x), type=2)
        assert abs(mp_closed_form(n, m, x) - ferrers) <= mp.mpf(10) ** (-(DPS - 8)) * abs(ferrers)
    # the 40-digit recurrence against the closed form, far below the double
    # range (first four spots) and at ordinary ones
    spots = [(2047, 700, 0.9999), (2047, 1600, 0.99), (4095, 2000, 0.999), (4095, 4000, 0.999),
             (4095, 1200, 0.7071), (300, 150, 0.3), (900, 400, -0.7)]
    for n, m, x in spots:
        rec = mp_column(n, m, x, mp_coeffs(n, m))[-1]
        ref = mp_closed_form(n, m, x)
        assert abs(rec - ref) <= mp.mpf(10) ** (-(DPS - 10)) * abs(ref), (n, m, x, rec, ref)
    assert abs(mp_closed_form(2047, 700, 0.9999)) < mp.mpf(10) ** -800


def critical_node(L, m, x):
    """Index of the node nearest the north pole at which P_m^m underflows
    double (|P_m^m| < 2^-1074) while the recurrence is past its turning point
    well before n = L (sin(theta) >= 1.05 m / L), or None."""
    s = np.sqrt((1 - x) * (1 + x))
    lamm = 0.5 * (sum(math.log((2 * k + 1) / (2 * k)) for k in range(1, m + 1)) - math.log(4 * math.pi))
    for i in range(len(x) // 2):
        if s[i] >= 1.05 * m / L:
            return i if lamm + m * math.log(s[i]) < -1074 * math.log(2) else None
    return None


CASES = [(2047, m) for m in (700, 1200, 1600, 2000)] + [(4095, m) for m in (700, 1200, 1600, 2000, 3000, 4000)]


@pytest.mark.parametrize("L,m", CASES)
def test_plm_long_double_against_mpmath(L, m):
    nlat = L + 1
    x, _ = oracle.gauss(nlat, precision="ld")
    nodes = [0, 1, 2, nlat // 4]
    crit = critical_node(L, m, x)
    if crit is not None:
        nodes.append(crit)
    raw = oracle.plm_raw(L, [m], x[nodes], precision="ld")[0]      # [L+1, nodes] long double
    dbl = oracle.plm(L, L, x[nodes], precision="ld")               # rounded to double
    dbl_plain = oracle.plm(L, L, x[nodes], precision="double")
    co = mp_coeffs(L, m)
    base = oracle.lm_index(L, m, m)
    for j, i in enumerate(nodes):
        ref = mp_column(L, m, x[i], co)
        big = max(abs(v) for v in ref)
        err = max(abs(ld_to_mp(raw[m + k, j]) - ref[k]) for k in range(len(ref)))
        if abs(ref[0]) >= mp.mpf(10) ** -4900:
            # the start P_m^m lies inside the long-double range
            assert err <= mp.mpf(2e-16) * big, (L, m, i, float(err / big))
        else:
            # it underflows long double too: allowed only for a column that
            # stays negligible next to anything double can hold
            assert big < mp.mpf(10) ** -300, (L, m, i)
            assert np.all(np.abs(raw[m:, j]) < np.longdouble(1e-300)), (L, m, i)
        col = dbl[base:base + L + 1 - m, j]
        refd = np.array([float(v) for v in ref])   # 0 below the double range
        scale = max(float(big), 1e-300)
        assert np.max(np.abs(col - refd)) <= 3e-16 * scale, (L, m, i)
        if i == crit:
            # the case the guard exists for: O(1) values by n = L, yet the
            # double recurrence has lost its start (flushed to 0, or left as
            # a denormal of a few bits that the recurrence then amplifies)
            assert big >= 1e-3, (L, m, i, float(big))
            assert np.max(np.abs(dbl_plain[base:base + L + 1 - m, j] - refd)) > 0.1 * float(big)


def mp_gauss_node(N, i):
    """The i-th Gauss node of order N (decreasing) by Newton's method on the
    Bonnet recurrence of Sec. 2.1, in mpmath."""
    x = mp.cos(mp.pi * (i + mp.mpf(3) / 4) / (N + mp.mpf(1) / 2))
    for _ in range(100):
        p0, p1 = mp.mpf(1), x
        for n in range(2, N + 1):
            p0, p1 = p1, ((2 * n - 1) * x * p1 - (n - 1) * p0) / n
        dp = N * (x * p1 - p0) / ((x - 1) * (x + 1))
        dx = p1 / dp
        x -= dx
        if abs(dx) < mp.mpf(10) ** (-(DPS - 5)):
            break
    return x


@pytest.mark.parametrize("nlat", [2048, 4096])
def test_gauss_long_double_against_mpmath(nlat):
    x, _ = oracle.gauss(nlat, precision="ld")
    for i in (0, 1, 2, nlat // 4, nlat // 2 - 1):
        ref = mp_gauss_node(nlat, i)
        assert abs(mp.mpf(float(x[i])) - ref) <= mp.mpf(2.0 ** -53) * abs(ref), (nlat, i)


def test_synth_long_double_against_mpmath():
    # the spectrum of the GPU guard test at lmax 2047, on a few latitudes
    from paper_1202_6522_amd import inputs
    L, nlat, nphi = 2047, 2048, 4096
    ms = [0, 700, 1200, 1600, 2000, 2047]
    rng = np.random.default_rng(2047)
    Q = np.zeros((1, oracle.nlm(L, L)), complex)
    n_all, m_all = inputs.degree_order(L, L)
    sel = np.isin(m_all, ms)
    Q[0, sel] = (rng.standard_normal(sel.sum()) + 1j * rng.standard_normal(sel.sum())) * (n_all[sel] + 1.0) ** -1.0
    Q[0, m_all == 0] = Q[0, m_all == 0].real
    x, _ = oracle.gauss(nlat, precision="ld")
    rows = [0, 5, 200, 1023, 2047]
    ks = [0, 1, 777, 2048, 4095]
    got = oracle.synth(Q, L, L, nlat, nphi, mlist=ms, rows=rows, precision="ld")[0]
    F = {}
    for m in ms:
        co = mp_coeffs(L, m)
        base = oracle.lm_index(L, m, m)
        for i in rows:
            col = mp_column(L, m, x[i], co)
            re = mp.fsum(mp.mpf(Q[0, base + k].real) * col[k] for k in range(len(col)))
            im = mp.fsum(mp.mpf(Q[0, base + k].imag) * col[k] for k in range(len(col)))
            F[m, i] = (re, 0 if m == 0 else im)
    ref = np.zeros((len(rows), len(ks)))
    for r, i in enumerate(rows):
        for c, k in enumerate(ks):
            acc = F[0, i][0]
            for m in ms[1:]:
                ph = 2 * mp.pi * m * k / nphi
                acc += 2 * (F[m, i][0] * mp.cos(ph) - F[m, i][1] * mp.sin(ph))
            ref[r, c] = float(acc)
    big = np.max(np.abs(ref))
    assert big > 1e-3
    assert np.max(np.abs(got[:, ks] - ref)) <= 1e-15 * big
