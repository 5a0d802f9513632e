"""Pins of the oracle's spline path: cubic Hermite segments (eq. hermite_segment),
the bound-aware derivative clamp (eq. vel-clamp), feasibility of the weighted
update, and equality of the knot-space update with the paper's dense route."""
import numpy as np
import pytest

import oracle as O
from paper_2511_19204_amd import synth


def _knots(nk, nu, rng):
    return np.concatenate([rng.normal(0, 1, nk * nu), rng.normal(0, 3, nk * nu)])


@pytest.mark.parametrize("nk,H", [(4, 48), (8, 140), (10, 135)])
def test_hermite_interpolates_positions_and_derivatives_at_nodes(nk, H):
    """P1: q(t_k) = theta^q_k and dq/dt(t_k) = theta^v_k; node k sits at step k H/(nk-1)."""
    rng = np.random.default_rng(nk)
    nu, dt = 3, 0.01
    kn = _knots(nk, nu, rng)
    for k in range(nk):
        h = k * H // (nk - 1)
        for j in range(nu):
            qr, vr = O.hermite(kn, nk, nu, H, dt, h, j)
            assert qr == pytest.approx(kn[k * nu + j], abs=1e-12)
            assert vr == pytest.approx(kn[nk * nu + k * nu + j], abs=1e-10)


def test_hermite_reproduces_any_cubic_and_partition_of_unity():
    """A cubic P(t) sampled as (P(t_k), P'(t_k)) is reproduced exactly at every step;
    constant position knots with zero slopes give that constant (h00 + h01 = 1)."""
    nk, nu, H, dt = 6, 1, 100, 0.005
    T = H * dt
    delta = T / (nk - 1)
    c = np.array([0.3, -1.2, 4.0, -7.5])
    P = lambda t: c[0] + c[1] * t + c[2] * t**2 + c[3] * t**3  # noqa: E731
    dP = lambda t: c[1] + 2 * c[2] * t + 3 * c[3] * t**2  # noqa: E731
    tk = np.arange(nk) * delta
    kn = np.concatenate([P(tk), dP(tk)])
    for h in range(H + 1):
        qr, vr = O.hermite(kn, nk, nu, H, dt, h, 0)
        assert qr == pytest.approx(P(h * dt), abs=1e-12)
        assert vr == pytest.approx(dP(h * dt), abs=1e-10)
    const = np.concatenate([np.full(nk, 0.7), np.zeros(nk)])
    for h in range(H + 1):
        assert O.hermite(const, nk, nu, H, dt, h, 0) == pytest.approx((0.7, 0.0), abs=1e-14)


def _wide_params(model, nk, H):
    p = synth.params(model, 64, H, 0.005, nk, 2, ("linear", 2.0, 4.0), "walking")
    return p


def test_clamp_bounds_every_sample_and_its_whole_trajectory():
    """P2: after the position clip and the velocity clamp with factor 2/Delta, the
    reference of every sample stays inside [q_min, q_max] at every step (a provable
    property of the factor-2 clamp), under very large noise."""
    m = synth.quadruped_model(0)
    nk, H = 8, 140
    p = _wide_params(m, nk, H)
    nom = synth.nominal_knots(m, nk)
    nu = m["n_u"]
    delta = H * p["dt"] / (nk - 1)
    worst = -np.inf
    for n in range(1, 65):
        th = O.sample_knots(m, p, nom, 99, 4, 1, n)
        Q, V = th[: nk * nu].reshape(nk, nu), th[nk * nu:].reshape(nk, nu)
        lim = 2 * np.minimum(m["q_max"] - Q, Q - m["q_min"]) / delta
        assert np.all(Q >= m["q_min"]) and np.all(Q <= m["q_max"])
        assert np.all(np.abs(V) <= lim + 1e-12)
        for h in range(0, H + 1, 2):
            for j in range(nu):
                qr, _ = O.hermite(th, nk, nu, H, p["dt"], h, j)
                worst = max(worst, qr - m["q_max"][j], m["q_min"][j] - qr)
    assert worst <= 1e-12


def test_sample_zero_is_the_clipped_nominal_and_noise_scales_with_sigma():
    """Sample 0 carries no noise; sample n >= 1 is nominal + sigma_k z (before the clip)."""
    m = synth.chain_model(0)
    p = synth.params(m, 4, 50, 0.01, 4, 1, ("linear", 1e-3, 2e-3), "ee")
    nom = synth.nominal_knots(m, 4)
    assert np.array_equal(O.sample_knots(m, p, nom, 5, 0, 0, 0), nom)
    th = O.sample_knots(m, p, nom, 5, 0, 0, 3)
    zq, zv = O.normals(5, 0, 0, 3, 12)
    sig = O.sigma_table(p)[0]
    delta = 50 * p["dt"] / 3
    sq = np.repeat(sig, 3)
    assert np.allclose(th[:12], nom[:12] + sq * zq, atol=1e-15)
    assert np.allclose(th[12:], nom[12:] + sq / delta * zv, atol=1e-12)


def test_weighted_update_preserves_the_clamp_set():
    """P3: the clamp set is convex (four half-planes per knot), so the weighted average
    of clamped samples satisfies the clamp again."""
    m = synth.quadruped_model(1)
    nk, H = 8, 140
    p = _wide_params(m, nk, H)
    nom = synth.nominal_knots(m, nk)
    nu = m["n_u"]
    delta = H * p["dt"] / (nk - 1)
    smp = np.stack([O.sample_knots(m, p, nom, 11, 0, 0, n) for n in range(64)])
    w = np.random.default_rng(0).dirichlet(np.ones(64))
    avg = O.weighted_average(w, smp)
    Q, V = avg[: nk * nu].reshape(nk, nu), avg[nk * nu:].reshape(nk, nu)
    lim = 2 * np.minimum(m["q_max"] - Q, Q - m["q_min"]) / delta
    assert np.all(np.abs(V) <= lim + 1e-9)


def test_knot_update_equals_dense_route():
    """P9: Hermite evaluation is linear in the knots, so resampling the weighted dense
    average at the node times (the paper's route) equals the weighted knot average."""
    m = synth.humanoid_model(0)
    nk, H = 10, 150
    p = synth.params(m, 32, H, 0.004, nk, 1, ("exp", 0.4, 1.0, 1.0), "bipedal")
    nom = synth.nominal_knots(m, nk)
    smp = np.stack([O.sample_knots(m, p, nom, 3, 1, 0, n) for n in range(32)])
    w = np.random.default_rng(2).dirichlet(np.ones(32))
    a = O.weighted_average(w, smp)
    b = O.dense_route_update(w, smp, nk, m["n_u"], H, p["dt"])
    assert np.max(np.abs(a - b)) < 1e-12
