"""Pins of the oracle's RK7(8) integrator (the paper's RK78, Sec. 3) and the
library's srp_rk78 against it (host code, no GPU).

The tableau is pinned by the order conditions it must satisfy (row sums equal
the nodes; the quadrature conditions sum_i b_i c_i^(q-1) = 1/q for q <= 8 for
the 8th-order weights and q <= 7 for the embedded 7th-order ones; the
conditions sum_i b_i a_ij c_j^(q-1) = 1/(q (q + 1)) for q <= 7), the
integrator by order-8 convergence on an eccentric Kepler orbit, the step
control by the accuracy it reaches on the paper's reference orbit (a = 0.557 AU,
e = 0.682, Sec. 5.1), and the two-body + cannonball SRP closed form."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import propagate as OP
from test_propagator import AU, MU, kepler_state, two_body


def _exact_tableau():
    """The same coefficients as exact fractions (from the float tableau)."""
    A = [[Fr(x).limit_denominator(10000) for x in row] for row in OP.A78]
    C = [Fr(x).limit_denominator(10000) for x in OP.C78]
    B8 = [Fr(x).limit_denominator(10000) for x in OP.B78]
    w = Fr(OP.ERR_W).limit_denominator(10000)
    # the 7th-order weights: b7 = b8 + err weights (err = b7 - b8 with the sign of k0 + k10 - k11 - k12)
    B7 = list(B8)
    B7[0] += w
    B7[10] += w
    B7[11] -= w
    B7[12] -= w
    return A, C, B8, B7


def test_tableau_order_conditions():
    A, C, B8, B7 = _exact_tableau()
    for i, row in enumerate(A):
        assert sum(row, Fr(0)) == C[i], i
    for q in range(1, 9):
        assert sum(b * c ** (q - 1) for b, c in zip(B8, C)) == Fr(1, q), q
    for q in range(1, 8):
        assert sum(b * c ** (q - 1) for b, c in zip(B7, C)) == Fr(1, q), q
    for B, qmax in ((B8, 7), (B7, 6)):
        for q in range(1, qmax + 1):
            s = sum(B[i] * sum(A[i][j] * C[j] ** (q - 1) for j in range(len(A[i]))) for i in range(13))
            assert s == Fr(1, q * (q + 1)), q
    # the 8th-order solution differs from the 7th-order one
    assert B8 != B7


def test_rk78_is_eighth_order():
    a, e = 0.557 * AU, 0.682
    T = 2 * np.pi * np.sqrt(a ** 3 / MU)
    y0 = kepler_state(MU, a, e, 0.0)
    exact = kepler_state(MU, a, e, 0.5 * T)
    errs = []
    for n in (60, 120):
        tr, ev = OP.rk78(two_body(MU), y0, 0.0, 0.5 * T, 0.5 * T / n)
        assert ev == 13 * n and len(tr) == n + 1
        errs.append(np.linalg.norm(tr[-1, 1:4] - exact[:3]) / a)
    assert errs[1] < 1e-9
    assert 150 < errs[0] / errs[1] < 450, errs      # 2^8 = 256


def test_adaptive_rk78_meets_its_tolerance():
    """One revolution of the paper's reference orbit from perihelion: the
    final position error shrinks with the tolerance; at rtol 1e-10 (position
    atol 1e-10 AU) it is below 2 km of a 0.56 AU orbit; rejected steps are
    retried, so every accepted step satisfied the test."""
    a, e = 0.557 * AU, 0.682
    T = 2 * np.pi * np.sqrt(a ** 3 / MU)
    y0 = kepler_state(MU, a, e, 0.0)
    res = {}
    for tol in (1e-9, 1e-11):
        tr, ev = OP.rk78(two_body(MU), y0, 0.0, T, T / 100, rtol=tol, atol=[tol * AU] * 3 + [tol * 1e4] * 3,
                         adaptive=True)
        assert tr[-1, 0] == T and np.all(np.diff(tr[:, 0]) > 0)
        res[tol] = (np.linalg.norm(tr[-1, 1:4] - y0[:3]), len(tr) - 1, ev)
    assert res[1e-9][0] < 2e4 and res[1e-11][0] < res[1e-9][0] / 20, res
    assert res[1e-11][1] > res[1e-9][1]


def test_rk78_cannonball_closed_form():
    R, rd, m, P0 = 2.0, 0.4, 50.0, 4.56e-6
    k = P0 * AU ** 2 * np.pi * R * R * (1 + 4 * rd / 9) / m
    mu_eff = MU - k

    def f(t, y):
        r = y[:3]
        rn = np.linalg.norm(r)
        return np.concatenate([y[3:], -MU * r / rn ** 3 + k * r / rn ** 3])

    a, e = AU, 0.1
    y0 = kepler_state(mu_eff, a, e, 0.0)
    T = 2 * np.pi * np.sqrt(a ** 3 / mu_eff)
    tr, _ = OP.rk78(f, y0, 0.0, 0.3 * T, 0.3 * T / 40)
    exact = kepler_state(mu_eff, a, e, 0.3 * T)
    assert np.linalg.norm(tr[-1, 1:4] - exact[:3]) / a < 1e-12


@pytest.fixture(scope="module")
def srp():
    import paper_2608_07307_amd as m
    from paper_2608_07307_amd import _lib as L
    L.load()
    return m


def _accel(k):
    def acc(t, r, v):
        rn = np.linalg.norm(r)
        return -MU * r / rn ** 3 + k * r / rn ** 3 + 1e-8 * np.array([np.cos(t * 2e-7), 0.3, 0.0])
    return acc


def test_library_rk78_fixed_matches_oracle(srp):
    a, e = 0.388 * AU, 0.881
    y0 = kepler_state(MU, a, e, 0.0)
    T = 2 * np.pi * np.sqrt(a ** 3 / MU)
    acc = _accel(2e9)
    f = lambda t, y: np.concatenate([y[3:], acc(t, y[:3], y[3:])])  # noqa: E731
    h0 = T / 333.3
    tr, ev = srp.rk78(y0, 50.0, 50.0 + 0.4 * T, acc, srp.rk78_opts(h0))
    ref, rev = OP.rk78(f, y0, 50.0, 50.0 + 0.4 * T, h0)
    assert ev == rev and tr.shape == ref.shape
    np.testing.assert_array_equal(tr[:, 0], ref[:, 0])
    np.testing.assert_allclose(tr[:, 1:4], ref[:, 1:4], rtol=1e-12, atol=1e-3)
    np.testing.assert_allclose(tr[:, 4:], ref[:, 4:], rtol=1e-11, atol=1e-9)


@pytest.mark.parametrize("atol_zero", [False, True])
def test_library_rk78_adaptive_matches_oracle(srp, atol_zero):
    """Same accepted steps and states as the oracle; with atol_zero the planar
    orbit's z components have zero error and zero tolerance scale."""
    a, e = 0.557 * AU, 0.682
    y0 = kepler_state(MU, a, e, 0.0)
    T = 2 * np.pi * np.sqrt(a ** 3 / MU)
    acc = (lambda t, r, v: -MU * r / np.linalg.norm(r) ** 3) if atol_zero else _accel(-1e9)
    f = lambda t, y: np.concatenate([y[3:], acc(t, y[:3], y[3:])])  # noqa: E731
    atol = [0.0] * 6 if atol_zero else [1e-10 * AU] * 3 + [1e-6] * 3
    tr, ev = srp.rk78(y0, 0.0, 2 * T, acc, srp.rk78_opts(T / 50, True, 1e-10, atol))
    ref, rev = OP.rk78(f, y0, 0.0, 2 * T, T / 50, rtol=1e-10, atol=atol, adaptive=True)
    assert ev == rev and tr.shape == ref.shape, (ev, rev, tr.shape, ref.shape)
    np.testing.assert_allclose(tr[:, 0], ref[:, 0], rtol=1e-13)
    np.testing.assert_allclose(tr[:, 1:4], ref[:, 1:4], rtol=1e-11, atol=1e-2)


def test_library_rk78_errors(srp):
    from paper_2608_07307_amd import SrpError
    y0 = kepler_state(MU, AU, 0.1, 0.0)
    acc = _accel(0.0)
    with pytest.raises(SrpError):
        srp.rk78(y0, 0.0, 1e6, acc, srp.rk78_opts(1e5, True, 0.0, 0.0))       # no tolerance
    with pytest.raises(SrpError):
        srp.rk78(y0, 0.0, 1e6, acc, srp.rk78_opts(-1.0))
    with pytest.raises(SrpError):
        srp.rk78(y0, 0.0, 1e7, acc, srp.rk78_opts(1e4), max_rows=10)          # more steps than rows
    with pytest.raises(ZeroDivisionError):                                   # the callback's error comes back
        srp.rk78(y0, 0.0, 1e6, lambda t, r, v: 1 / 0, srp.rk78_opts(1e5))


def test_library_spad_rk78_matches_oracle(srp):
    """SPAD propagation with RK7(8): fixed steps give the oracle's states to
    rounding; adaptive steps agree to the integration accuracy only, since the
    bilinear table makes the right-hand side kinked at cell boundaries and the
    step sizes then depend on rounding-level differences of the error
    estimate (one revolution of E(M), a = 0.437 AU, e = 0.786)."""
    from oracle import spad as OS
    deg = np.pi / 180
    g = (20, 10, -175 * deg, -85 * deg, 18 * deg, 18 * deg)
    tab = np.random.default_rng(41).normal(size=(10, 20, 6)) * 3e-4
    a, e = 0.437 * AU, 0.786
    y0 = kepler_state(MU, a, e, 0.0)
    T = 2 * np.pi * np.sqrt(a ** 3 / MU)

    def f(t, y):
        rn = np.linalg.norm(y[:3])
        F = OS.interp(g, tab, -y[:3] / rn)[:3] * (4.56e-6 * (AU / rn) ** 2 / 2.0)
        return np.concatenate([y[3:], -MU * y[:3] / rn ** 3 + F / 700.0])

    G = srp.spad_grid(*g)
    tr = srp.propagate_spad_rk78(G, tab, 2.0, y0, 0.0, T, srp.rk78_opts(T / 300), MU, 700.0, 4.56e-6, AU)
    ref, _ = OP.rk78(f, y0, 0.0, T, T / 300)
    assert tr.shape == ref.shape == (301, 7)
    np.testing.assert_allclose(tr[:, 1:4], ref[:, 1:4], rtol=1e-11, atol=1e-2)
    atol = [1e-11 * AU] * 3 + [1e-7] * 3
    tr = srp.propagate_spad_rk78(G, tab, 2.0, y0, 0.0, T, srp.rk78_opts(T / 40, True, 1e-11, atol), MU, 700.0,
                                 4.56e-6, AU)
    ref, _ = OP.rk78(f, y0, 0.0, T, T / 40, rtol=1e-11, atol=atol, adaptive=True)
    assert tr[-1, 0] == ref[-1, 0] == T
    assert np.linalg.norm(tr[-1, 1:4] - ref[-1, 1:4]) / a < 2e-6
