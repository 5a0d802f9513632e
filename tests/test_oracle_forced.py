"""The oracle's trajectory-forced steps (one control step of the Alg. 1 simulate
step from a given state), which the GPU's per-step parity checks use: fed the
oracle's own trajectory they reproduce it, its stage costs and masks exactly,
and their accelerations equal the separately exposed step dynamics at that
state with the Hermite reference of that step."""
import numpy as np
import pytest

import oracle as O
from paper_2511_19204_amd import synth


@pytest.mark.parametrize("kind", ["chain", "quadruped", "humanoid"])
def test_forced_steps_reproduce_the_rollout(kind):
    m, p, seed = synth.config(kind, n_samples=4)
    p = dict(p)
    p["horizon"] = 30
    H, K, nu = p["horizon"], p["n_knots"], m["n_u"]
    kn = synth.nominal_knots(m, K)
    samples = np.stack([O.sample_knots(m, p, kn, seed, 0, 0, n) for n in range(3)])
    trajs, stages, masks = [], [], []
    for s in samples:
        S, traj, mk, st = O.rollout(m, p, m["x0"], s, debug=True)
        trajs.append(traj); stages.append(st); masks.append(mk)
    trajs = np.stack(trajs)
    out = O.forced_steps(m, p, m["x0"], samples, trajs)
    assert np.array_equal(out["next"], trajs[:, 1:])
    assert np.array_equal(out["cost"], np.stack(stages))
    assert np.array_equal(out["masks"], np.stack(masks))
    nq = m["n_q"]
    for r in range(3):
        for h in (0, 7, H - 1):
            qr = np.zeros(nu); vr = np.zeros(nu)
            for j in range(nu):
                qr[j], vr[j] = O.hermite(samples[r], K, nu, H, p["dt"], h, j)
            x = trajs[r, h]
            qdd, _, _, cf = O.step_dynamics(m, x[:nq], x[nq:], qr, vr, p["dt"])
            assert np.allclose(out["qdd"][r, h], qdd, rtol=0, atol=1e-9 * max(1.0, np.abs(qdd).max()))
            if m["contact_body"].size:
                assert np.allclose(out["fn"][r, h], cf[:, 2], rtol=0, atol=1e-9)


def test_forced_steps_float_evaluation_is_close_to_fp64():
    m, p, seed = synth.config("quadruped", n_samples=4)
    p = dict(p)
    p["horizon"] = 20
    kn = synth.nominal_knots(m, p["n_knots"])
    s = O.sample_knots(m, p, kn, seed, 0, 0, 1)[None]
    _, traj, _, _ = O.rollout(m, p, m["x0"], s[0], debug=True)
    a = O.forced_steps(m, p, m["x0"], s, traj[None])
    b = O.forced_steps(m, p, m["x0"], s, traj[None], f32=True)
    scale = np.maximum(1.0, np.abs(a["qdd"]).max(axis=2, keepdims=True))
    assert np.max(np.abs(a["qdd"] - b["qdd"]) / scale) < 1e-3
    assert not np.array_equal(a["qdd"], b["qdd"])


@pytest.mark.parametrize("kind", ["chain", "quadruped"])
def test_integrate_alone_reproduces_the_step(kind):
    """The integration step applied to the step's own accelerations gives the
    next state of the rollout bit for bit (one physics substep per control step)."""
    m, p, seed = synth.config(kind, n_samples=4)
    p = dict(p)
    p["horizon"] = 12
    kn = synth.nominal_knots(m, p["n_knots"])
    s = O.sample_knots(m, p, kn, seed, 0, 0, 2)
    _, traj, _, _ = O.rollout(m, p, m["x0"], s, debug=True)
    out = O.forced_steps(m, p, m["x0"], s[None], traj[None])
    nxt = O.integrate(m, p["dt"], traj[:-1], out["qdd"][0])
    assert np.array_equal(nxt, traj[1:])


def test_integrate_free_flight_closed_form():
    """Zero acceleration: joints and base position move by dt v (base linear
    velocity rotated to the world); a base spinning about z at rate w turns its
    quaternion by dt w."""
    m, p, seed = synth.config("quadruped", n_samples=4)
    nq, nv = m["n_q"], m["n_v"]
    x = np.array(m["x0"], float)
    x[nq + 2] = 1.5                 # yaw rate
    x[nq + 3:nq + 6] = [0.2, -0.1, 0.3]
    x[nq + 6:] = np.linspace(-1, 1, m["n_u"])
    dt = 0.01
    out = O.integrate(m, dt, x[None], np.zeros((1, nv)))[0]
    assert np.allclose(out[7:nq], x[7:nq] + dt * x[nq + 6:], rtol=0, atol=1e-15)
    assert np.allclose(out[:3], x[:3] + dt * x[nq + 3:nq + 6], rtol=0, atol=1e-15)  # identity orientation
    half = 0.5 * 1.5 * dt
    assert np.allclose(out[3:7], [np.cos(half), 0, 0, np.sin(half)], rtol=0, atol=1e-15)
    assert np.array_equal(out[nq:], x[nq:])


def test_clip_flip_classifier():
    """The torque-clip flip classification of the GPU per-step check: a step
    whose joint torque sits at its limit within rounding is accepted when its
    accelerations are those of the other clip branch, and only then."""
    from forced_parity import ACC_TOL, _clip_flips
    m, p, seed = synth.config("quadruped", n_samples=4)
    p = dict(p)
    p["horizon"] = 20
    H, K, nu, nq, dt = p["horizon"], p["n_knots"], m["n_u"], m["n_q"], p["dt"]
    kn = synth.nominal_knots(m, K)
    s = O.sample_knots(m, p, kn, seed, 0, 0, 1)
    _, traj, _, _ = O.rollout(m, p, m["x0"], s, debug=True)
    h, j = 9, 4
    qr = np.array([O.hermite(s, K, nu, H, dt, h, i)[0] for i in range(nu)])
    vr = np.array([O.hermite(s, K, nu, H, dt, h, i)[1] for i in range(nu)])
    kp, kd, tm = m["kp"][j], m["kd"][j], m["tau_max"][j]

    def at(frac):
        """Trajectory copy whose joint-j torque at step h is frac * tau_max."""
        X = traj.copy()
        t = kp * (qr[j] - X[h, 7 + j]) + kd * (vr[j] - X[h, nq + 6 + j])
        X[h, 7 + j] -= (frac * tm - t) / kp
        return X

    X = at(1 + 1e-9)                      # FP64 saturates, at the limit within rounding
    a_sat = O.step_dynamics(m, X[h, :nq], X[h, nq:], qr, vr, dt)[0]
    qr_in = qr.copy()
    qr_in[j] -= 2e-9 * tm / kp            # the same step below the limit
    a_lin = O.step_dynamics(m, X[h, :nq], X[h, nq:], qr_in, vr, dt)[0]
    scale = max(np.abs(a_sat).max(), 1.0)
    assert np.abs(a_sat - a_lin).max() / scale > 100 * ACC_TOL  # the branches differ by a finite step
    cand = np.zeros((1, H), dtype=bool)
    cand[0, h] = True

    def classify(X, a):
        A = np.zeros((1, H, m["n_v"]))
        A[0, h] = a
        return bool(_clip_flips(m, p, s[None], X[None], A, cand)[0, h])

    assert classify(X, a_lin)                 # other branch: a clip flip
    assert not classify(X, a_lin * (1 + 1e-3))  # other branch, wrong values
    assert not classify(X, a_sat * (1 + 1e-3))  # own branch, wrong values
    Xf = at(0.9)                               # far from the limit: never a flip
    a_far = O.step_dynamics(m, Xf[h, :nq], Xf[h, nq:], qr, vr, dt)[0]
    assert not classify(Xf, a_far * (1 + 1e-3))
