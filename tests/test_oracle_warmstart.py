"""Pins of the oracle's state prediction and warm-start shift (Sec. III-E):
closed forms of the shift (identity, the repeated final action, a shift by one
knot spacing), an independent Hermite evaluator (scipy), and the prediction's
rest equilibrium and one-step agreement with the physics step."""
import numpy as np
import pytest
from scipy.interpolate import CubicHermiteSpline

import oracle as O
from paper_2511_19204_amd import synth


def _random_knots(rng, nk, nu):
    return rng.normal(size=2 * nk * nu)


@pytest.mark.parametrize("nk,nu,H,dt", [(4, 3, 50, 0.01), (8, 12, 100, 0.005), (10, 21, 150, 0.004)])
def test_shift_by_zero_is_the_identity(nk, nu, H, dt):
    kn = _random_knots(np.random.default_rng(0), nk, nu)
    # k Delta / Delta need not round back to k exactly: equal up to rounding
    assert np.allclose(O.shift_knots(kn, nk, nu, H, dt, 0), kn, atol=1e-12, rtol=0)


@pytest.mark.parametrize("n", [100, 101, 250])
def test_shift_past_the_horizon_repeats_the_final_action(n):
    nk, nu, H, dt = 8, 12, 100, 0.005
    kn = _random_knots(np.random.default_rng(1), nk, nu)
    out = O.shift_knots(kn, nk, nu, H, dt, n)
    Q, V = kn[: nk * nu].reshape(nk, nu), kn[nk * nu:].reshape(nk, nu)
    oq, ov = out[: nk * nu].reshape(nk, nu), out[nk * nu:].reshape(nk, nu)
    assert np.allclose(oq, Q[-1], atol=1e-12, rtol=0) and np.allclose(ov, V[-1], atol=1e-12, rtol=0)


def test_shift_by_one_knot_spacing_moves_the_knots_down():
    """H = m (K - 1): shifting by m steps moves every knot to the previous index;
    the last knot repeats."""
    nk, nu, m, dt = 6, 4, 20, 0.01
    H = m * (nk - 1)
    kn = _random_knots(np.random.default_rng(2), nk, nu)
    out = O.shift_knots(kn, nk, nu, H, dt, m)
    for blk in (slice(0, nk * nu), slice(nk * nu, 2 * nk * nu)):
        a, b = kn[blk].reshape(nk, nu), out[blk].reshape(nk, nu)
        assert np.allclose(b[:-1], a[1:], atol=1e-12, rtol=0)
        assert np.allclose(b[-1], a[-1], atol=1e-12, rtol=0)


@pytest.mark.parametrize("n", [1, 3, 7, 13, 42])
def test_shift_matches_an_independent_hermite_evaluator(n):
    """The shifted knots are the old spline's value and slope at t_k + n dt
    (clamped to T), evaluated here with scipy's CubicHermiteSpline."""
    nk, nu, H, dt = 8, 5, 100, 0.005
    T = H * dt
    kn = _random_knots(np.random.default_rng(3), nk, nu)
    out = O.shift_knots(kn, nk, nu, H, dt, n)
    tk = np.linspace(0.0, T, nk)
    Q, V = kn[: nk * nu].reshape(nk, nu), kn[nk * nu:].reshape(nk, nu)
    t = np.minimum(tk + n * dt, T)
    for j in range(nu):
        sp = CubicHermiteSpline(tk, Q[:, j], V[:, j])
        assert np.allclose(out[: nk * nu].reshape(nk, nu)[:, j], sp(t), atol=1e-12, rtol=1e-12)
        assert np.allclose(out[nk * nu:].reshape(nk, nu)[:, j], sp(t, 1), atol=1e-11, rtol=1e-11)


def test_prediction_of_zero_steps_is_the_state():
    m, p, s = synth.config("quadruped", n_samples=4)
    kn = synth.nominal_knots(m, p["n_knots"])
    assert np.array_equal(O.predict(m, p, m["x0"], kn, 0), m["x0"].astype(np.float64))


def test_prediction_stays_at_rest_without_gravity():
    """Arm at rest, no gravity, knots holding the current pose with zero velocity:
    every torque is zero and the predicted state is the initial one."""
    m, p, s = synth.config("chain", n_samples=4)
    m = dict(m)
    m["gravity"] = 0.0
    x0 = np.array([0.3, -0.4, 0.2, 0.0, 0.0, 0.0])
    nk = p["n_knots"]
    kn = np.concatenate([np.tile(x0[:3], nk), np.zeros(3 * nk)])
    x = O.predict(m, p, x0, kn, 17)
    assert np.allclose(x, x0, atol=1e-15, rtol=0)


def test_one_step_prediction_is_one_physics_step():
    """One control step of the prediction equals the physics step tracking the
    Hermite reference at t = 0 (arm, no contact, one substep)."""
    m, p, s = synth.config("chain", n_samples=4)
    rng = np.random.default_rng(4)
    nk, nu = p["n_knots"], m["n_u"]
    kn = np.concatenate([rng.uniform(-0.5, 0.5, nk * nu), rng.uniform(-1, 1, nk * nu)])
    x0 = np.concatenate([rng.uniform(-0.5, 0.5, nu), rng.uniform(-0.5, 0.5, nu)])
    qr = np.array([O.hermite(kn, nk, nu, p["horizon"], p["dt"], 0, j)[0] for j in range(nu)])
    vr = np.array([O.hermite(kn, nk, nu, p["horizon"], p["dt"], 0, j)[1] for j in range(nu)])
    q, v = O.euler_step(m, p["dt"], x0[:nu], x0[nu:], qr, vr)
    x1 = O.predict(m, p, x0, kn, 1)
    assert np.allclose(x1, np.concatenate([q, v]), atol=1e-13, rtol=1e-13)
