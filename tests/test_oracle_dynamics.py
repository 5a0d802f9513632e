"""Pins of the oracle's rigid-body dynamics, contact and integrator.

The articulated-body algorithm is checked against the composite-rigid-body mass
matrix with a Cholesky solve (textbook route), the mass matrix itself against
kinetic energy from an independent numpy forward kinematics written here, the
bias terms against energy and momentum conservation, and against closed forms
(free fall, a single pendulum).  The linearly implicit step is checked against
its dense joint-space definition."""
import numpy as np
import pytest
from scipy.linalg import cho_factor, cho_solve, expm

import oracle as O
from paper_2511_19204_amd import synth


# ---------------------------------------------------------------- independent kinematics
def _rot(axis, q):
    a = np.asarray(axis, float)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return expm(K * q)


def _quat_R(w, x, y, z):
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _fk(m, base_R, base_p, joints):
    """World rotation and origin of every body, straight from the model's definition."""
    Rs, ps = [], []
    fb = m["floating_base"]
    for i, lam in enumerate(m["parent"]):
        if fb and i == 0:
            Rs.append(base_R); ps.append(base_p); continue
        j = i - (1 if fb else 0)
        C = m["R_tree"][i] @ _rot(m["axis"][i], joints[j])
        Rl, pl = (Rs[lam], ps[lam]) if lam >= 0 else (np.eye(3), np.zeros(3))
        Rs.append(Rl @ C); ps.append(pl + Rl @ m["p_tree"][i])
    return Rs, ps


def _kinetic_energy(m, q, v, eps=1e-6):
    """T = sum 1/2 m |v_com|^2 + 1/2 w^T I_world w with velocities from central
    differences of the configuration moved along v (base twist in base coordinates)."""
    fb = m["floating_base"]
    def pose(e):
        if fb:
            R0 = _quat_R(*q[3:7])
            Rb = R0 @ expm(e * np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]]))
            pb = q[:3] + e * R0 @ v[3:6]
            return _fk(m, Rb, pb, q[7:] + e * v[6:])
        return _fk(m, None, None, q + e * v)
    Rp, pp = pose(eps)
    Rm, pm = pose(-eps)
    T = 0.0
    for i in range(len(m["parent"])):
        cp = pp[i] + Rp[i] @ m["com"][i]
        cm = pm[i] + Rm[i] @ m["com"][i]
        vc = (cp - cm) / (2 * eps)
        R0 = 0.5 * (Rp[i] + Rm[i])
        W = (Rp[i] - Rm[i]) / (2 * eps) @ R0.T
        w = np.array([W[2, 1], W[0, 2], W[1, 0]])
        I = m["inertia"][i]
        Ib = np.array([[I[0], I[3], I[4]], [I[3], I[1], I[5]], [I[4], I[5], I[2]]])
        T += 0.5 * m["mass"][i] * vc @ vc + 0.5 * w @ (R0 @ Ib @ R0.T) @ w
    return T


def _tiny_floating(n_links):
    """Free base + a chain of n_links revolute bodies with skewed axes."""
    rng = np.random.default_rng(n_links)
    t = synth._Tree()
    t.body(-1, (0, 0, 1), (0, 0, 0), 3.0, (0.01, -0.02, 0.03), (0.3, 0.2, 0.1))
    prev = 0
    for k in range(n_links):
        ax = rng.normal(size=3); ax /= np.linalg.norm(ax)
        prev = t.body(prev, ax, rng.normal(0, 0.1, 3), 0.5 + k, rng.normal(0, 0.05, 3),
                      (0.1, 0.05, 0.2), joint=(-2, 2, 50, 10, 1, 0))
    m = t.finish("tiny", True, [prev], [(0, 0, -0.1)])
    # exact (float64) unit axes and rotations: this tree only feeds the FP64 oracle
    m["axis"] = np.array(t.axis) / np.linalg.norm(np.array(t.axis), axis=1, keepdims=True)
    m["R_tree"] = np.array([_rot(rng.normal(size=3) / 2, 0.7) for _ in range(len(m["parent"]))])
    m["n_substeps"] = 1
    m["x0"] = synth.f32(np.concatenate([[0, 0, 1, 1, 0, 0, 0], np.zeros(n_links), np.zeros(6 + n_links)]))
    return m


MODELS = {
    "chain": lambda: synth.chain_model(3),
    "tiny1": lambda: _tiny_floating(1),
    "tiny2": lambda: _tiny_floating(2),
    "quadruped": lambda: synth.quadruped_model(2),
    "humanoid": lambda: synth.humanoid_model(1),
}


def _random_state(m, rng, vel=1.0):
    nq, nv = m["n_q"], m["n_v"]
    q = m["x0"][:nq] + rng.normal(0, 0.2, nq)
    if m["floating_base"]:
        q[3:7] /= np.linalg.norm(q[3:7])
    return q, rng.normal(0, vel, nv)


@pytest.mark.parametrize("name", list(MODELS))
def test_fk_matches_independent_kinematics(name):
    m = MODELS[name]()
    rng = np.random.default_rng(0)
    q, _ = _random_state(m, rng)
    R, p = O.body_poses(m, q)
    Rs, ps = _fk(m, _quat_R(*q[3:7]) if m["floating_base"] else None,
                 q[:3] if m["floating_base"] else None, q[7:] if m["floating_base"] else q)
    assert np.allclose(R, np.array(Rs), atol=1e-12)
    assert np.allclose(p, np.array(ps), atol=1e-12)


@pytest.mark.parametrize("name", list(MODELS))
def test_mass_matrix_equals_kinetic_energy_hessian(name):
    """M(q) from the CRBA equals the Hessian of kinetic energy in v, the energy coming
    from the independent kinematics above (polarisation over basis vectors)."""
    m = MODELS[name]()
    rng = np.random.default_rng(1)
    q, _ = _random_state(m, rng)
    Hm = O.crba(m, q)
    nv = m["n_v"]
    E = np.eye(nv)
    T1 = [_kinetic_energy(m, q, E[i]) for i in range(nv)]
    ref = np.zeros((nv, nv))
    for i in range(nv):
        ref[i, i] = 2 * T1[i]
        for j in range(i):
            ref[i, j] = ref[j, i] = _kinetic_energy(m, q, E[i] + E[j]) - T1[i] - T1[j]
    # rotor (armature) kinetic energy 1/2 I_a qd_j^2 adds to the joint diagonal
    off = 6 if m["floating_base"] else 0
    ref[off:, off:] += np.diag(np.asarray(m.get("armature", np.zeros(m["n_u"]))))
    assert np.allclose(Hm, Hm.T, atol=1e-14)
    assert np.max(np.abs(Hm - ref)) < 1e-7 * np.max(np.abs(ref))


@pytest.mark.parametrize("name", list(MODELS))
def test_aba_equals_crba_cholesky(name):
    """P7: ABA(q, v, tau, f) = M^-1 (tau_full - C(q, v, f)), with C from the RNEA at
    zero acceleration and M factorised by Cholesky."""
    m = MODELS[name]()
    rng = np.random.default_rng(2)
    for trial in range(3):
        q, v = _random_state(m, rng)
        tau = rng.normal(0, 5, m["n_u"])
        a = O.forward_dynamics(m, q, v, tau, with_contacts=True)
        Hm = O.crba(m, q)
        C = O.rnea(m, q, v, np.zeros(m["n_v"]), with_contacts=True)
        full = np.concatenate([np.zeros(6), tau]) if m["floating_base"] else tau
        ref = cho_solve(cho_factor(Hm), full - C)
        assert np.max(np.abs(a - ref)) < 1e-10 * max(1.0, np.max(np.abs(ref)))
        # round trip through inverse dynamics
        back = O.rnea(m, q, v, a, with_contacts=True)
        assert np.max(np.abs(back - full)) < 1e-9 * max(1.0, np.max(np.abs(full)))


@pytest.mark.parametrize("name", ["quadruped", "humanoid", "tiny2"])
def test_free_fall(name):
    """Zero velocity, zero torque, no contact: every body falls with g, joints stay."""
    m = MODELS[name]()
    rng = np.random.default_rng(3)
    q, _ = _random_state(m, rng)
    a = O.forward_dynamics(m, q, np.zeros(m["n_v"]), np.zeros(m["n_u"]), with_contacts=False)
    R = _quat_R(*q[3:7])
    assert np.allclose(a[:3], 0, atol=1e-12)
    assert np.allclose(a[3:6], R.T @ np.array([0, 0, -9.81]), atol=1e-12)
    assert np.allclose(a[6:], 0, atol=1e-11)


def test_single_pendulum_closed_form():
    """Fixed-base single link about y with its com at distance l along x:
    (I_c + m l^2) qdd = tau + m g l cos q, plus an implicit gain on qdd."""
    t = synth._Tree()
    mass, l = 1.7, 0.23
    t.body(-1, (0, 1, 0), (0, 0, 0), mass, (l, 0, 0), (0.5, 0.05, 0.05), joint=(-3, 3, 1e3, 40.0, 2.0, 0))
    m = t.finish("pend", False, [], np.zeros((0, 3)), ee_body=0, ee_pos=(2 * l, 0, 0))
    m["n_substeps"] = 1
    l = m["com"][0][0]
    Io = m["inertia"][0][1] + m["mass"][0] * l**2
    for q in (-1.0, 0.0, 0.4, 2.0):
        for tau in (0.0, 3.0):
            a = O.forward_dynamics(m, [q], [0.7], [tau], with_contacts=False)
            assert a[0] == pytest.approx((tau + m["mass"][0] * 9.81 * l * np.cos(q)) / Io, rel=1e-12)
    # implicit PD: (Io + dt (Kd + dt Kp)) qdd = Kp (qr - q) + Kd (vr - v) + m g l cos q
    dt, q, v, qr, vr = 0.01, 0.3, -0.2, 0.5, 0.1
    a, tau, g, _ = O.step_dynamics(m, [q], [v], [qr], [vr], dt)
    gain = dt * (2.0 + dt * 40.0)
    tref = 40.0 * (qr - q) + 2.0 * (vr - v)
    assert tau[0] == pytest.approx(tref, rel=1e-14) and g[0] == pytest.approx(gain, rel=1e-14)
    assert a[0] == pytest.approx((tref + m["mass"][0] * 9.81 * l * np.cos(q)) / (Io + gain), rel=1e-12)


@pytest.mark.parametrize("name", ["chain", "tiny2", "quadruped"])
def test_energy_conserved_without_torque_and_contact(name):
    """P7: E = 1/2 v^T M v + V is constant along RK4 (dt = 1e-4, 1 s) with tau = 0."""
    m = MODELS[name]()
    rng = np.random.default_rng(4)
    q, v = _random_state(m, rng, vel=1.5)
    E0 = O.energy(m, q, v)
    scale = abs(E0) + 0.5 * v @ O.crba(m, q) @ v
    q1, v1 = O.rk4(m, 1e-4, 10_000, q, v, np.zeros(m["n_u"]))
    assert abs(O.energy(m, q1, v1) - E0) < 1e-8 * scale


def test_momentum_conserved_without_gravity():
    """P7: with g = 0 and only internal joint torques, the total spatial momentum of a
    free-floating tree is constant."""
    m = synth.quadruped_model(5)
    m["gravity"] = 0.0
    rng = np.random.default_rng(5)
    q, v = _random_state(m, rng)
    q[2] = 5.0
    h0 = O.momentum(m, q, v)
    q1, v1 = O.rk4(m, 1e-4, 5_000, q, v, rng.normal(0, 0.2, m["n_u"]))
    assert np.max(np.abs(O.momentum(m, q1, v1) - h0)) < 1e-9 * np.max(np.abs(h0))


def _contact_jacobians(m, q):
    nv = m["n_v"]
    J = np.zeros((len(m["contact_body"]), 3, nv))
    for i in range(nv):
        e = np.zeros(nv); e[i] = 1.0
        _, vel, _, _ = O.contacts(m, q, e)
        J[:, :, i] = vel
    return J


@pytest.mark.parametrize("name", ["quadruped", "humanoid", "tiny1"])
def test_implicit_step_equals_dense_definition(name):
    """The step's accelerations solve (M + dt sum J_c^T D_c J_c + diag(g)) qdd =
    tau_full - C(q, v, f_explicit), with D_c the closed-form velocity Jacobian of the
    soft contact law (tangential-normal coupling dropped) and g = dt (Kd + dt Kp) on
    unsaturated joints."""
    m = MODELS[name]()
    rng = np.random.default_rng(6)
    dt = 0.005
    nq, nv, nu = m["n_q"], m["n_v"], m["n_u"]
    for trial in range(4):
        q = m["x0"][:nq] + rng.normal(0, 0.02, nq)
        q[2] = m["x0"][2] - 0.01  # push the feet into the ground
        q[3:7] /= np.linalg.norm(q[3:7])
        v = rng.normal(0, 0.3, nv)
        off = 7
        qr = q[off:] + rng.normal(0, 0.2, nu)
        vr = rng.normal(0, 1, nu)
        a, tau, g, f = O.step_dynamics(m, q, v, qr, vr, dt)
        t = m["kp"] * (qr - q[off:]) + m["kd"] * (vr - v[6:])
        sat = np.abs(t) >= m["tau_max"]
        assert np.allclose(tau, np.clip(t, -m["tau_max"], m["tau_max"]), atol=1e-12)
        assert np.allclose(g, np.where(sat, 0.0, dt * (m["kd"] + dt * m["kp"])), atol=1e-15)
        Hm = O.crba(m, q)
        C = O.rnea(m, q, v, np.zeros(nv), with_contacts=True)
        J = _contact_jacobians(m, q)
        _, vel, force, _ = O.contacts(m, q, v)
        A = Hm.copy()
        A[6:, 6:] += np.diag(g)
        for c in range(len(m["contact_body"])):
            fn = force[c, 2]
            if fn <= 0:
                continue
            vx, vy = vel[c, 0], vel[c, 1]
            n2 = vx * vx + vy * vy + m["eps_fric"] ** 2
            s = m["mu"] * fn / np.sqrt(n2)
            D = np.array([[s * (1 - vx * vx / n2), -s * vx * vy / n2, 0],
                          [-s * vx * vy / n2, s * (1 - vy * vy / n2), 0],
                          [0, 0, m["d_contact"]]])
            A += dt * J[c].T @ D @ J[c]
        ref = np.linalg.solve(A, np.concatenate([np.zeros(6), tau]) - C)
        assert np.max(np.abs(a - ref)) < 1e-9 * max(1.0, np.max(np.abs(ref)))


def test_contact_law_closed_form():
    """Penalty normal force max(0, -k z - d v_z) below the ground only, smoothed Coulomb
    friction -mu f_n v_t / sqrt(|v_t|^2 + eps^2)."""
    m = synth.quadruped_model(0)
    nq, nv = m["n_q"], m["n_v"]
    q = m["x0"][:nq].copy()
    rng = np.random.default_rng(8)
    v = rng.normal(0, 0.5, nv)
    pos, vel, f, mask = O.contacts(m, q, v)
    for c in range(4):
        z, vz = pos[c, 2], vel[c, 2]
        fn = max(0.0, -m["k_contact"] * z - m["d_contact"] * vz) if z < 0 else 0.0
        nrm = np.sqrt(vel[c, 0] ** 2 + vel[c, 1] ** 2 + m["eps_fric"] ** 2)
        assert f[c, 2] == pytest.approx(fn, rel=1e-13, abs=1e-12)
        assert np.allclose(f[c, :2], -m["mu"] * fn * vel[c, :2] / nrm, rtol=1e-13, atol=1e-12)
        assert bool(mask & (1 << c)) == (fn > 0)
    q[2] += 0.1
    _, _, f, mask = O.contacts(m, q, v)
    assert mask == 0 and np.all(f == 0)


def test_contact_statics_after_settling():
    """P12: a quadruped holding its stance settles; over the last second the mean total
    normal force equals the weight (vertical momentum balance) within 1e-3."""
    for seed in (0, 1, 2):
        m, p, _ = synth.config("quadruped", seed=seed)
        p["horizon"] = 600  # 3 s
        kn = synth.nominal_knots(m, p["n_knots"])
        _, traj, _, _ = O.rollout(m, p, m["x0"], kn, debug=True)
        nq = m["n_q"]
        fz = [O.contacts(m, x[:nq], x[nq:])[2][:, 2].sum() for x in traj[400:]]
        W = m["mass"].sum() * 9.81
        assert abs(np.mean(fz) / W - 1) < 1e-3
        assert np.abs(traj[-1][nq:]).max() < 0.05


def test_orientation_angle_closed_form():
    """P13: a rotation by alpha about any axis has |log3| = alpha (alpha in [0, pi]),
    for either sign of the quaternion."""
    rng = np.random.default_rng(9)
    for alpha in np.linspace(0, np.pi, 13):
        ax = rng.normal(size=3); ax /= np.linalg.norm(ax)
        qt = np.concatenate([[np.cos(alpha / 2)], np.sin(alpha / 2) * ax])
        assert O.orientation_angle(qt) == pytest.approx(alpha, abs=1e-12)
        assert O.orientation_angle(-qt) == pytest.approx(alpha, abs=1e-12)


def test_integrator_quaternion_stays_unit_and_base_position_follows_rotation():
    """One step: base position advances by dt R(quat) v_lin with the updated velocity and
    the quaternion stays unit."""
    m = synth.quadruped_model(3)
    nq, nv = m["n_q"], m["n_v"]
    rng = np.random.default_rng(10)
    q = m["x0"][:nq].copy(); q[2] += 1.0
    q[3:7] = rng.normal(size=4); q[3:7] /= np.linalg.norm(q[3:7])
    v = rng.normal(0, 1, nv)
    qr = q[7:].copy(); vr = np.zeros(m["n_u"])
    dt = 0.005
    a, _, _, _ = O.step_dynamics(m, q, v, qr, vr, dt)
    q1, v1 = O.euler_step(m, dt, q, v, qr, vr)
    assert np.allclose(v1, v + dt * a, atol=1e-12)
    assert np.allclose(q1[:3], q[:3] + dt * _quat_R(*q[3:7]) @ v1[3:6], atol=1e-12)
    assert np.allclose(q1[7:], q[7:] + dt * v1[6:], atol=1e-12)
    assert abs(np.linalg.norm(q1[3:7]) - 1) < 1e-14
    R1 = _quat_R(*q1[3:7])
    w = v1[:3]
    Rref = _quat_R(*q[3:7]) @ expm(dt * np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]))
    assert np.allclose(R1, Rref, atol=1e-12)
