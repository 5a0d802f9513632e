"""Pins of the oracle's MPPI layer: importance weights (eq. omega-weights and the
min-max form eq. softmax_minmax), the weighted update, best-sample tracking
(Sec. III-D), the sigma = 0 fixed point and a brute-force two-sample case."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2511_19204_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_cost_weight_table_matches_paper():
    ref = json.load(open(os.path.join(GOLDEN, "cost_weights.json")))["rows"]
    assert set(ref) == set(synth.COST_WEIGHTS)
    for k, row in ref.items():
        assert tuple(row) == synth.COST_WEIGHTS[k]


def test_weights_basic_properties():
    rng = np.random.default_rng(0)
    S = rng.normal(100, 20, 257)
    w, nstar, nf = O.weights(S, 1.0)
    assert nf == 257 and nstar == int(np.argmin(S))
    assert abs(w.sum() - 1) < 1e-14 and np.all(w > 0)
    order = np.argsort(S)
    assert np.all(np.diff(w[order]) <= 0)
    Sh = (S - S.min()) / (S.max() - S.min())
    ref = np.exp(-Sh) / np.exp(-Sh).sum()
    assert np.allclose(w, ref, rtol=1e-14)


def test_weights_minmax_invariant_to_affine_costs():
    """P8: min-max normalisation makes the weights invariant to S -> a S + b, a > 0."""
    rng = np.random.default_rng(1)
    S = rng.exponential(50, 64)
    w0, _, _ = O.weights(S, 0.7)
    for a, b in ((3.0, -1e3), (1e-3, 7.0), (1e4, 1e6)):
        w1, _, _ = O.weights(a * S + b, 0.7)
        assert np.allclose(w0, w1, rtol=1e-9, atol=1e-15)


def test_weights_temperature_limits():
    """P8: lambda -> 0 concentrates all mass on the unique minimum; equal costs give
    uniform weights (so the update returns the plain mean)."""
    S = np.array([5.0, 3.0, 3.5, 9.0])
    w, nstar, _ = O.weights(S, 1e-4)
    assert nstar == 1 and w[1] == pytest.approx(1.0, abs=1e-12)
    w, _, _ = O.weights(np.full(10, 2.5), 1.0)
    assert np.allclose(w, 0.1, rtol=1e-15)
    samples = np.random.default_rng(2).normal(size=(10, 7))
    assert np.allclose(O.weighted_average(w, samples), samples.mean(axis=0), rtol=1e-13)


def test_weights_raw_mode_is_plain_softmax():
    S = np.array([1.0, 2.0, 0.5, 4.0])
    w, _, _ = O.weights(S, 2.0, mode=1)
    ref = np.exp(-S / 2.0) / np.exp(-S / 2.0).sum()
    assert np.allclose(w, ref, rtol=1e-14)


def test_weights_non_finite_costs():
    """Non-finite costs get zero weight and do not enter min/max; none finite -> 0."""
    S = np.array([np.inf, 4.0, np.nan, 2.0, 6.0])
    w, nstar, nf = O.weights(S, 1.0)
    assert nf == 3 and nstar == 3
    assert w[0] == 0 and w[2] == 0
    ref = O.weights(np.array([4.0, 2.0, 6.0]), 1.0)[0]
    assert np.allclose(w[[1, 3, 4]], ref, rtol=1e-15)
    w, nstar, nf = O.weights(np.array([np.inf, np.nan]), 1.0)
    assert nf == 0 and nstar == -1 and np.all(w == 0)
    # a tie for the minimum resolves to the lowest index
    assert O.weights(np.array([3.0, 1.0, 1.0]), 1.0)[1] == 1


def test_zero_noise_is_a_fixed_point():
    """P10: sigma = 0 makes every sample equal the (feasible) nominal, so all costs are
    equal and the update returns the nominal knots."""
    m, p, seed = synth.config("chain")
    p["sigma_lo"] = p["sigma_hi"] = 0.0
    p["n_iters"] = 2
    kn = synth.nominal_knots(m, p["n_knots"])
    kn[12:] = 0.0
    kn[:12] = np.repeat([0.3, 0.1, -0.2, 0.4], 3)
    r = O.step(m, p, m["x0"], kn, seed, 0)
    assert np.all(r["costs"] == r["costs"][0, 0])
    assert np.max(np.abs(r["knots"] - kn)) < 1e-14


def _pendulum():
    t = synth._Tree()
    t.body(-1, (0, 1, 0), (0, 0, 0), 1.3, (0.15, 0, 0), (0.3, 0.04, 0.04),
           joint=(-2.0, 2.0, 30.0, 20.0, 0.5, 0.0))
    m = t.finish("pend", False, [], np.zeros((0, 3)), ee_body=0, ee_pos=(0.3, 0, 0))
    m["n_substeps"] = 1
    m["x0"] = synth.f32([0.2, -0.4])
    return m


def test_brute_force_two_samples_one_step():
    """P11: one link, N_s = 2, H = 1: costs, weights and the update by hand.
    At h = 0 the reference is knot 0; one implicit step (I_o + g) qdd = tau + m g l cos q,
    v1 = v0 + dt qdd, q1 = q0 + dt v1; end-effector height z = -L sin q."""
    m = _pendulum()
    p = synth.params(m, 2, 1, 0.02, 2, 1, ("linear", 0.3, 0.6), "ee")
    nom = synth.f32([0.1, 0.5, 0.2, -1.0])
    seed = 77
    r = O.step(m, p, m["x0"], nom, seed, 5)
    q0, v0 = m["x0"]
    L, lc, mass = m["ee_pos"][0], m["com"][0][0], m["mass"][0]
    Io = m["inertia"][0][1] + mass * lc * lc
    dt = p["dt"]
    costs, thetas = [], []
    for n in range(2):
        th = O.sample_knots(m, p, nom, seed, 5, 0, n)
        thetas.append(th)
        tau = np.clip(20.0 * (th[0] - q0) + 0.5 * (th[2] - v0), -30, 30)
        g = dt * (0.5 + dt * 20.0) if abs(tau) < 30 else 0.0
        qdd = (tau + mass * 9.81 * lc * np.cos(q0)) / (Io + g)
        v1 = v0 + dt * qdd
        q1 = q0 + dt * v1
        z0, z1 = -L * np.sin(q0), -L * np.sin(q1)
        S = 1e2 * (z0 - 0.5) ** 2 + 1e-3 * tau * tau + 1e2 * (z1 - 0.5) ** 2
        costs.append(S)
    assert np.allclose(r["costs"][0], costs, rtol=1e-12)
    lo = int(np.argmin(costs))
    w = np.array([1.0, np.exp(-1.0)]) if lo == 0 else np.array([np.exp(-1.0), 1.0])
    w /= w.sum()
    assert np.allclose(r["knots"], w[0] * thetas[0] + w[1] * thetas[1], rtol=1e-12, atol=1e-14)
    assert r["S_best"] == pytest.approx(min(costs), rel=1e-14)
    assert np.array_equal(r["best_knots"], thetas[lo])


def test_step_costs_match_single_rollouts_and_best_tracking():
    """Iteration 0's costs equal stand-alone rollouts of the sampled knots; S_best is the
    running minimum with strict improvement and the lowest index among ties."""
    m, p, seed = synth.config("chain")
    p["n_iters"] = 4
    kn = synth.nominal_knots(m, p["n_knots"])
    r = O.step(m, p, m["x0"], kn, seed, 3)
    for n in (0, 1, 17, 31):
        th = O.sample_knots(m, p, kn, seed, 3, 0, n)
        assert r["costs"][0, n] == pytest.approx(O.rollout(m, p, m["x0"], th), rel=1e-15)
    per_iter_min = r["costs"].min(axis=1)
    assert r["S_best"] == per_iter_min.min()
    assert r["best_iter"] == int(np.argmin(per_iter_min))
    assert r["n_nonfinite"] == 0


def test_step_is_deterministic_and_thread_independent():
    m, p, seed = synth.config("quadruped")
    p["n_samples"] = 16
    kn = synth.nominal_knots(m, p["n_knots"])
    a = O.step(m, p, m["x0"], kn, seed, 9, threads=1)
    b = O.step(m, p, m["x0"], kn, seed, 9, threads=4)
    for k in ("knots", "best_knots", "costs"):
        assert np.array_equal(a[k], b[k])


def test_mppi_iterations_reduce_the_chain_cost():
    """Behavioural sanity (not a paper number): ten iterations lower the cost of the
    nominal knots on the end-effector-height task."""
    m, p, seed = synth.config("chain")
    kn = synth.nominal_knots(m, p["n_knots"])
    before = O.rollout(m, p, m["x0"], kn)
    r = O.step(m, p, m["x0"], kn, seed, 0)
    after = O.rollout(m, p, m["x0"], r["knots"])
    assert after < 0.8 * before
    assert r["S_best"] <= before
