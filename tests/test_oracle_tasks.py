"""Pins of the oracle's task targets (Sec. IV-A: the orientation residual
||log3(R_base^T R_des)|| with a task-specific R_des, and the terminal target of
the jumping task given as an absolute base height): closed forms of the rotation
angle, the identity target, and the terminal term's special case and slope."""
import numpy as np
import pytest

import oracle as O
from paper_2511_19204_amd import synth


def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _axis_angle(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    return np.concatenate([[np.cos(ang / 2)], np.sin(ang / 2) * axis])


def _only(p, **w):
    p = dict(p)
    for k in ("w_h", "w_or", "w_q", "w_cv", "w_cf", "w_eff", "w_H"):
        p[k] = 0.0
    p.update(w)
    p["horizon"] = 1
    return p


@pytest.mark.parametrize("seed", range(6))
def test_orientation_residual_is_the_relative_rotation_angle(seed):
    """Base orientation q_des * exp(alpha axis / 2), either quaternion sign: the
    stage cost with only w_orient is w_orient * alpha^2 for alpha <= pi and
    w_orient * (2 pi - alpha)^2 beyond (the shorter rotation)."""
    rng = np.random.default_rng(seed)
    m, p, s = synth.config("quadruped", n_samples=4)
    q_des = _axis_angle(rng.normal(size=3), rng.uniform(0, np.pi))
    p = _only(p, w_or=3.0)
    p["q_des"] = list(q_des)
    kn = synth.nominal_knots(m, p["n_knots"])
    for alpha in (0.0, 0.3, 1.7, np.pi - 1e-3, np.pi + 0.4, 2 * np.pi - 0.2):
        qb = _qmul(q_des, _axis_angle(rng.normal(size=3), alpha))
        for sign in (1.0, -1.0):
            x0 = np.array(m["x0"], float)
            x0[3:7] = sign * qb
            _, _, _, stage = O.rollout(m, p, x0, kn, debug=True)
            ref = min(alpha, 2 * np.pi - alpha) ** 2
            assert abs(stage[0] - 3.0 * ref) <= 1e-11 * max(1.0, ref), (alpha, sign, stage[0], 3.0 * ref)


def test_identity_target_is_the_default():
    m, p, s = synth.config("quadruped", n_samples=4)
    kn = synth.nominal_knots(m, p["n_knots"]) + np.random.default_rng(1).normal(0, 0.05, 2 * 8 * 12)
    a = O.rollout(m, p, m["x0"], kn)
    p1 = dict(p)
    p1["q_des"] = [1.0, 0.0, 0.0, 0.0]
    p0 = dict(p)
    p0["q_des"] = [0.0, 0.0, 0.0, 0.0]
    assert O.rollout(m, p1, m["x0"], kn) == a == O.rollout(m, p0, m["x0"], kn)
    # a rotated target changes the cost
    p2 = dict(p)
    p2["q_des"] = list(_axis_angle([0, 1, 0], np.pi / 4))
    assert O.rollout(m, p2, m["x0"], kn) > a


def test_absolute_terminal_height_reduces_to_the_default():
    """z_terminal = p_z(x0) with v_des,z = 0 is the default terminal target."""
    m, p, s = synth.config("quadruped", n_samples=4)
    kn = synth.nominal_knots(m, p["n_knots"])
    p = dict(p)
    p["v_des"] = [0.5, 0.0, 0.0]
    a = O.rollout(m, p, m["x0"], kn)
    p["terminal_z_abs"] = 1
    p["z_terminal"] = float(m["x0"][2])
    assert O.rollout(m, p, m["x0"], kn) == a


def test_absolute_terminal_height_has_slope_minus_w_H_below_the_final_height():
    """For targets below the final base height, raising the target by dz lowers
    the terminal cost by w_H dz (the L1 terminal term of Sec. IV-A)."""
    m, p, s = synth.config("quadruped", n_samples=4)
    kn = synth.nominal_knots(m, p["n_knots"])
    p = _only(p, w_H=7.0)
    p["horizon"] = 20
    p["terminal_z_abs"] = 1
    p["z_terminal"] = -1.0
    S1, traj, _, _ = O.rollout(m, p, m["x0"], kn, debug=True)
    zH = traj[-1][2]
    assert zH > -0.5
    p["z_terminal"] = -0.5
    S2 = O.rollout(m, p, m["x0"], kn)
    assert abs((S1 - S2) - 7.0 * 0.5) <= 1e-9
