"""Pins of the oracle's position-only spline variants (the spline ablation of
Sec. V: cubic and quadratic splines whose velocity targets are zero, against
the cubic Hermite parameterization): the natural cubic spline against scipy's
CubicSpline, the quadratic spline against pieces built one by one from their
own interpolation and continuity conditions, and the variants' sampling,
zero velocity targets and warm-start shift."""
import numpy as np
import pytest
from scipy.interpolate import CubicSpline

import oracle as O
from paper_2511_19204_amd import synth


def _knots(rng, nk, nu):
    return np.concatenate([rng.normal(size=nk * nu), np.zeros(nk * nu)])


def _eval(kn, nk, nu, H, dt, j):
    """Values and slopes of joint j at the H fine steps of the horizon (Hermite form)."""
    q = np.array([O.hermite(kn, nk, nu, H, dt, h, j)[0] for h in range(H + 1)])
    v = np.array([O.hermite(kn, nk, nu, H, dt, h, j)[1] for h in range(H + 1)])
    return q, v


@pytest.mark.parametrize("nk", [2, 3, 4, 8, 10])
def test_natural_cubic_matches_scipy(nk):
    nu, H, dt = 3, 60, 0.01
    T = H * dt
    delta = T / (nk - 1)
    kn = O.spline_slopes(1, _knots(np.random.default_rng(nk), nk, nu), nk, nu, delta)
    tk = np.linspace(0, T, nk)
    th = np.arange(H + 1) * dt
    for j in range(nu):
        Q = kn[: nk * nu].reshape(nk, nu)[:, j]
        cs = CubicSpline(tk, Q, bc_type="natural")
        assert np.allclose(kn[nk * nu:].reshape(nk, nu)[:, j], cs(tk, 1), atol=1e-10, rtol=1e-10)
        q, v = _eval(kn, nk, nu, H, dt, j)
        assert np.allclose(q, cs(th), atol=1e-10, rtol=1e-10)
        assert np.allclose(v, cs(th, 1), atol=1e-9, rtol=1e-9)


def _quadratic_pieces(Q, delta):
    """Pieces a + b tau + c tau^2 on [0, Delta]: each through its two knots with a
    slope that continues the previous piece's (zero at the start), solved as a
    3x3 system per piece."""
    pieces, slope = [], 0.0
    for k in range(len(Q) - 1):
        A = np.array([[1.0, 0.0, 0.0], [1.0, delta, delta ** 2], [0.0, 1.0, 0.0]])
        a, b, c = np.linalg.solve(A, [Q[k], Q[k + 1], slope])
        pieces.append((a, b, c))
        slope = b + 2 * c * delta
    return pieces


@pytest.mark.parametrize("nk", [2, 4, 8])
def test_quadratic_matches_pieces_built_from_their_conditions(nk):
    nu, H, dt = 2, 56, 0.01
    T = H * dt
    delta = T / (nk - 1)
    kn = O.spline_slopes(2, _knots(np.random.default_rng(10 + nk), nk, nu), nk, nu, delta)
    for j in range(nu):
        Q = kn[: nk * nu].reshape(nk, nu)[:, j]
        pieces = _quadratic_pieces(Q, delta)
        q, v = _eval(kn, nk, nu, H, dt, j)
        for h in range(H + 1):
            t = h * dt
            k = min(int(np.floor(t / delta + 1e-12)), nk - 2)
            tau = t - k * delta
            a, b, c = pieces[k]
            assert abs(q[h] - (a + b * tau + c * tau * tau)) <= 1e-9
            assert abs(v[h] - (b + 2 * c * tau)) <= 1e-8
        assert kn[nk * nu + j] == 0.0  # zero initial slope


@pytest.mark.parametrize("mode", [1, 2])
def test_variant_sampling_perturbs_positions_only(mode):
    m, p, s = synth.config("quadruped", n_samples=8)
    nk, nu = p["n_knots"], m["n_u"]
    nom = synth.nominal_knots(m, nk)
    delta = p["horizon"] * p["dt"] / (nk - 1)
    pv = dict(p)
    pv["spline_mode"] = mode
    for n in (0, 3):
        a = O.sample_knots(m, p, nom, s, 5, 1, n)      # cubic Hermite
        b = O.sample_knots(m, pv, nom, s, 5, 1, n)     # variant: same position noise
        assert np.array_equal(a[: nk * nu], b[: nk * nu])
        assert np.allclose(b, O.spline_slopes(mode, b, nk, nu, delta), atol=1e-12, rtol=0)


@pytest.mark.parametrize("mode", [1, 2])
def test_variant_velocity_targets_are_zero(mode):
    """One control step of a variant equals the physics step tracking the spline
    position with a zero velocity target."""
    m, p, s = synth.config("chain", n_samples=4)
    p = dict(p)
    p["spline_mode"] = mode
    nk, nu = p["n_knots"], m["n_u"]
    delta = p["horizon"] * p["dt"] / (nk - 1)
    rng = np.random.default_rng(mode)
    kn = O.spline_slopes(mode, np.concatenate([rng.uniform(-0.5, 0.5, nk * nu), np.zeros(nk * nu)]),
                         nk, nu, delta)
    x0 = np.concatenate([rng.uniform(-0.5, 0.5, nu), rng.uniform(-0.5, 0.5, nu)])
    qr = np.array([O.hermite(kn, nk, nu, p["horizon"], p["dt"], 0, j)[0] for j in range(nu)])
    q, v = O.euler_step(m, p["dt"], x0[:nu], x0[nu:], qr, np.zeros(nu))
    assert np.allclose(O.predict(m, p, x0, kn, 1), np.concatenate([q, v]), atol=1e-13, rtol=1e-13)


@pytest.mark.parametrize("mode", [1, 2])
def test_variant_shift_defines_a_new_spline_of_the_same_kind(mode):
    nk, nu, H, dt = 8, 3, 100, 0.005
    T = H * dt
    delta = T / (nk - 1)
    kn = O.spline_slopes(mode, _knots(np.random.default_rng(20 + mode), nk, nu), nk, nu, delta)
    n = 9
    out = O.shift_knots(kn, nk, nu, H, dt, n, spline_mode=mode)
    tk = np.linspace(0, T, nk)
    t = np.minimum(tk + n * dt, T)
    for j in range(nu):
        Q = kn[: nk * nu].reshape(nk, nu)[:, j]
        if mode == 1:
            ref = CubicSpline(tk, Q, bc_type="natural")(t)
        else:
            pieces = _quadratic_pieces(Q, delta)
            ref = []
            for tt in t:
                k = min(int(np.floor(tt / delta + 1e-12)), nk - 2)
                a, b, c = pieces[k]
                tau = tt - k * delta
                ref.append(a + b * tau + c * tau * tau)
            ref = np.array(ref)
        assert np.allclose(out[: nk * nu].reshape(nk, nu)[:, j], ref, atol=1e-10, rtol=1e-10)
    assert np.allclose(out, O.spline_slopes(mode, out, nk, nu, delta), atol=1e-12, rtol=0)
