"""Pins of the oracle's running and terminal cost terms (Sec. IV-A cost function,
Tab. cost-weights, plus the effort term w_eff ||tau||^2 of the workloads).

Each test switches on ONE weight, rolls out a horizon of one (or a few) control
steps, and recomputes that term by hand from the state, the contact outputs
(positions, velocities, forces, activity) and the PD law written out here:

  running:  w_h |p_z - z_des|                 base height
            w_q ||q_j - q_j0||^2              posture
            w_cv sum_{c: f_n > 0} ||v_c||_1   contact velocity, active points only
            w_cf sum_c ||f_c - f0_c||_1       contact force about f0 = (0, 0, f0z_c)
            w_eff ||tau||^2                   effort (clipped PD torques)
  terminal: w_H ||p(x_H) - (p(x0) + v_des H dt)||_1

The states have some feet pressed into the ground and one lifted and moving, so
summing the velocity term over every point, dropping f0, using an L2 norm or
flipping the sign of the terminal target each changes a value checked here.
The end-effector task of the fixed-base arm (w_ee (z_ee - z_des)^2 + w_tau
||tau||^2, terminal w_ee (z_ee(x_H) - z_des)^2) is pinned the same way.
"""
import numpy as np
import pytest

import oracle as O
from paper_2511_19204_amd import synth

WEIGHTS = ("w_h", "w_or", "w_q", "w_cv", "w_cf", "w_eff", "w_H", "w_ee", "w_tau")


def _only(p, horizon=1, **w):
    p = dict(p)
    for k in WEIGHTS:
        p[k] = 0.0
    p.update(w)
    p["horizon"] = horizon
    return p


def _lifted_state(m, seed, lift_leg=0):
    """Quadruped state: leg `lift_leg` folded so its foot is off the ground, the
    base lowered so the other feet press in, random joint and base velocities."""
    rng = np.random.default_rng(seed)
    x = np.array(m["x0"], float)
    nq = m["n_q"]
    x[2] -= 0.01
    x[7 + 3 * lift_leg + 2] = -2.5                 # knee folded
    x[7 + 3 * lift_leg + 1] = 1.4                  # hip raised
    x[3:7] = [1.0, 0.02, -0.01, 0.03]
    x[3:7] /= np.linalg.norm(x[3:7])
    x[7:nq] += rng.normal(0, 0.03, nq - 7) * (np.arange(nq - 7) // 3 != lift_leg)
    x[nq:nq + 6] = rng.normal(0, 0.2, 6)
    x[nq + 6:] = rng.normal(0, 1.0, m["n_u"])
    return x


def _humanoid_state(m, seed):
    rng = np.random.default_rng(seed)
    x = np.array(m["x0"], float)
    nq = m["n_q"]
    x[2] -= 0.004
    x[7:nq] += rng.normal(0, 0.05, nq - 7)
    x[7:nq] = np.clip(x[7:nq], m["q_min"], m["q_max"])
    x[nq:] = rng.normal(0, 0.3, m["n_v"])
    return x


def _knots(m, p, seed):
    rng = np.random.default_rng(seed + 100)
    kn = synth.nominal_knots(m, p["n_knots"]).copy()
    kn += rng.normal(0, 0.2, kn.size)
    return kn


def _tau0(m, p, x, kn):
    """Clipped PD torques of control step 0 (eq. pd-controller): the Hermite
    reference at t = 0 is knot 0 (position) and its velocity knot."""
    nu, K = m["n_u"], p["n_knots"]
    off_q = 7 if m["floating_base"] else 0
    off_v = 6 if m["floating_base"] else 0
    nq = m["n_q"]
    q = x[off_q:off_q + nu]
    v = x[nq + off_v:nq + off_v + nu]
    qr = kn[:nu]
    vr = kn[K * nu:K * nu + nu]
    t = m["kp"] * (qr - q) + m["kd"] * (vr - v)
    return np.clip(t, -m["tau_max"], m["tau_max"])


def _split(m, x):
    nq = m["n_q"]
    return x[:nq], x[nq:]


def _cases():
    out = []
    for seed in range(3):
        out.append(("quadruped", seed))
    out.append(("humanoid", 0))
    return out


def _setup(kind, seed):
    m, p, _ = synth.config(kind, n_samples=4)
    if kind == "quadruped":
        x = _lifted_state(m, seed, lift_leg=seed % 4)
    else:
        x = _humanoid_state(m, seed)
    kn = _knots(m, p, seed)
    q, v = _split(m, x)
    pos, vel, f, mask = O.contacts(m, q, v)
    active = f[:, 2] > 0
    return m, p, x, kn, pos, vel, f, active, mask


@pytest.mark.parametrize("kind,seed", _cases())
def test_states_have_active_and_lifted_points(kind, seed):
    """The fixtures exercise both branches of every contact term: some points
    press into the ground with f_n > 0, some are off it with nonzero velocity."""
    m, p, x, kn, pos, vel, f, active, mask = _setup(kind, seed)
    assert active.any() and (~active).any()
    assert np.all(np.abs(vel[~active]).sum(axis=1) > 1e-3)
    assert np.all(pos[active, 2] < 0)
    assert mask == sum(1 << i for i in np.flatnonzero(active))


def _stage0(m, p, x, kn):
    S, traj, masks, stage = O.rollout(m, p, x, kn, debug=True)
    assert abs(S - stage.sum()) <= 1e-12 * max(1.0, abs(S))
    return stage


@pytest.mark.parametrize("kind,seed", _cases())
def test_height_term(kind, seed):
    m, p, x, kn, *_ = _setup(kind, seed)
    p = _only(p, w_h=7.0)
    p["z_des"] = float(x[2]) + 0.123
    st = _stage0(m, p, x, kn)
    assert st[0] == pytest.approx(7.0 * abs(x[2] - p["z_des"]), rel=1e-13)
    assert st[1] == 0.0


@pytest.mark.parametrize("kind,seed", _cases())
def test_posture_term(kind, seed):
    m, p, x, kn, *_ = _setup(kind, seed)
    p = _only(p, w_q=0.3)
    rng = np.random.default_rng(seed + 7)
    p["q0_cost"] = np.asarray(m["q0"]) + rng.normal(0, 0.1, m["n_u"])
    st = _stage0(m, p, x, kn)
    e = x[7:m["n_q"]] - p["q0_cost"]
    assert st[0] == pytest.approx(0.3 * float(np.sum(e * e)), rel=1e-12)


@pytest.mark.parametrize("kind,seed", _cases())
def test_contact_velocity_term_counts_active_points_only(kind, seed):
    m, p, x, kn, pos, vel, f, active, mask = _setup(kind, seed)
    p = _only(p, w_cv=0.5)
    st = _stage0(m, p, x, kn)
    ref = 0.5 * float(np.sum(np.abs(vel[active])))
    every = 0.5 * float(np.sum(np.abs(vel)))
    assert st[0] == pytest.approx(ref, rel=1e-12)
    assert abs(every - ref) > 1e-3 * ref      # the lifted points would change it


@pytest.mark.parametrize("kind,seed", _cases())
def test_contact_force_term_is_l1_about_f0(kind, seed):
    m, p, x, kn, pos, vel, f, active, mask = _setup(kind, seed)
    p = _only(p, w_cf=0.05)
    # a different reference force per point (a shared f0 can make sum|f - f0|
    # equal sum|f| by accident when as many points are lifted as exceed f0)
    p["f0z"] = np.asarray(p["f0z"]) * np.random.default_rng(seed).uniform(0.5, 1.5, len(p["f0z"]))
    f0 = np.zeros_like(f)
    f0[:, 2] = p["f0z"]
    st = _stage0(m, p, x, kn)
    ref = 0.05 * float(np.sum(np.abs(f - f0)))
    assert st[0] == pytest.approx(ref, rel=1e-12)
    # the L1 norm about f0, not about zero and not the L2 norm
    assert abs(0.05 * float(np.sum(np.abs(f))) - ref) > 1e-3 * ref
    assert abs(0.05 * float(np.sum(np.linalg.norm(f - f0, axis=1))) - ref) > 1e-3 * ref
    # every point enters, lifted ones with |0 - f0|
    assert np.all(f[~active] == 0.0)


@pytest.mark.parametrize("kind,seed", _cases())
def test_effort_term_uses_the_clipped_pd_torques(kind, seed):
    m, p, x, kn, *_ = _setup(kind, seed)
    p = _only(p, w_eff=1e-3)
    tau = _tau0(m, p, x, kn)
    st = _stage0(m, p, x, kn)
    assert st[0] == pytest.approx(1e-3 * float(np.sum(tau * tau)), rel=1e-12)
    # the oracle's own step reports the same torques
    q, v = _split(m, x)
    nu, K = m["n_u"], p["n_knots"]
    _, tau_o, _, _ = O.step_dynamics(m, q, v, kn[:nu], kn[K * nu:K * nu + nu], p["dt"])
    assert np.allclose(tau_o, tau, rtol=0, atol=1e-12)


def test_effort_fixture_saturates_some_joints():
    m, p, x, kn, *_ = _setup("quadruped", 0)
    tau = _tau0(m, p, x, kn)
    sat = np.abs(tau) == m["tau_max"]
    assert sat.any() and (~sat).any()


@pytest.mark.parametrize("kind,seed", _cases())
@pytest.mark.parametrize("horizon", (1, 4))
def test_terminal_target_is_l1_about_p0_plus_vdes_T(kind, seed, horizon):
    m, p, x, kn, *_ = _setup(kind, seed)
    p = _only(p, horizon=horizon, w_H=2.5e3)
    p["v_des"] = [0.5, -0.3, 0.1]
    S, traj, masks, stage = O.rollout(m, p, x, kn, debug=True)
    T = horizon * p["dt"]
    target = x[:3] + np.asarray(p["v_des"]) * T
    err = traj[horizon][:3] - target
    ref = 2.5e3 * float(np.sum(np.abs(err)))
    assert np.all(stage[:horizon] == 0.0)
    assert stage[horizon] == pytest.approx(ref, rel=1e-12)
    assert S == pytest.approx(ref, rel=1e-12)
    # sign of the velocity offset and the L1 norm both matter here
    flipped = 2.5e3 * float(np.sum(np.abs(traj[horizon][:3] - (x[:3] - np.asarray(p["v_des"]) * T))))
    l2 = 2.5e3 * float(np.linalg.norm(err))
    assert abs(flipped - ref) > 1e-3 * ref and abs(l2 - ref) > 1e-3 * ref


def _orientation_angle(qb):
    """Rotation angle of a unit quaternion (identity target): 2 atan2(|v|, |w|)."""
    return 2.0 * np.arctan2(np.linalg.norm(qb[1:4]), abs(qb[0]))


def _stage_by_hand(m, p, x, x0, kn, h):
    """Running cost of control step h at state x (all locomotion terms)."""
    nu, K, H = m["n_u"], p["n_knots"], p["horizon"]
    nq = m["n_q"]
    q, v = x[:nq], x[nq:]
    qr = np.zeros(nu); vr = np.zeros(nu)
    for j in range(nu):
        qr[j], vr[j] = O.hermite(kn, K, nu, H, p["dt"], h, j)
    tau = np.clip(m["kp"] * (qr - q[7:]) + m["kd"] * (vr - v[6:]), -m["tau_max"], m["tau_max"])
    pos, vel, f, mask = O.contacts(m, q, v)
    act = f[:, 2] > 0
    f0 = np.zeros_like(f)
    f0[:, 2] = p["f0z"]
    phi = _orientation_angle(q[3:7])
    c = (p["w_h"] * abs(q[2] - p["z_des"]) + p["w_or"] * phi * phi
         + p["w_q"] * float(np.sum((q[7:] - p["q0_cost"]) ** 2))
         + p["w_cv"] * float(np.sum(np.abs(vel[act])))
         + p["w_cf"] * float(np.sum(np.abs(f - f0)))
         + p["w_eff"] * float(np.sum(tau * tau)))
    return c, mask


@pytest.mark.parametrize("kind,seed", _cases())
def test_all_terms_together_over_a_short_horizon(kind, seed):
    """Every weight of the task's row on, H = 5: each stage cost equals the sum of
    the terms at the state the step starts from (not the integrated one), the
    terminal cost follows, and the rollout cost is their plain sum (no dt)."""
    m, p, x, kn, *_ = _setup(kind, seed)
    p = dict(p)
    p["horizon"] = 5
    p["v_des"] = [0.5, 0.2, 0.0]
    p["w_q"] = 0.3
    S, traj, masks, stage = O.rollout(m, p, x, kn, debug=True)
    for h in range(5):
        c, mk = _stage_by_hand(m, p, traj[h], x, kn, h)
        assert stage[h] == pytest.approx(c, rel=1e-11), h
        assert masks[h] == mk
    T = 5 * p["dt"]
    cT = p["w_H"] * float(np.sum(np.abs(traj[5][:3] - (x[:3] + np.asarray(p["v_des"]) * T))))
    assert stage[5] == pytest.approx(cT, rel=1e-11)
    assert S == pytest.approx(float(np.sum(stage)), rel=1e-13)


def _ee_height(m, q):
    R, pw = O.body_poses(m, q)
    b = m["ee_body"]
    return float((R[b] @ np.asarray(m["ee_pos"]) + pw[b])[2])


@pytest.mark.parametrize("seed", range(3))
def test_end_effector_terms(seed):
    """Fixed-base arm: running w_ee (z_ee - z_des)^2 + w_tau ||tau||^2 at the
    step's start state, terminal w_ee (z_ee(x_H) - z_des)^2."""
    m, p, _ = synth.config("chain", seed=seed)
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.uniform(-1, 1, 3), rng.normal(0, 1, 3)])
    kn = _knots(m, p, seed)
    pa = _only(p, w_ee=1e2)
    S, traj, _, stage = O.rollout(m, pa, x, kn, debug=True)
    z0, z1 = _ee_height(m, traj[0][:3]), _ee_height(m, traj[1][:3])
    assert stage[0] == pytest.approx(1e2 * (z0 - p["z_des"]) ** 2, rel=1e-12)
    assert stage[1] == pytest.approx(1e2 * (z1 - p["z_des"]) ** 2, rel=1e-12)
    pb = _only(p, w_tau=1e-3)
    _, _, _, stage = O.rollout(m, pb, x, kn, debug=True)
    tau = _tau0(m, pb, x, kn)
    assert stage[0] == pytest.approx(1e-3 * float(np.sum(tau * tau)), rel=1e-12)
    assert stage[1] == 0.0
