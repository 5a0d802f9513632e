"""Seeded synthetic workloads: kinematic trees, initial states, nominal knots and
controller parameters.

This module makes inputs only.  It holds none of the controller's arithmetic
(no sampling, spline, dynamics, cost or weighting code) and is the one module
shared by the HIP path's tests and the CPU oracle.  The paper's robots (a 12-joint
quadruped and a humanoid) and its simulator are not available, so seeded trees
of the same shape stand in for them:

* ``chain_model``      fixed-base planar 3R arm (links 0.3 m / 1 kg, +-10 %);
* ``quadruped_model``  free base + 4 legs x (abduction x, hip y, knee y), point feet;
* ``humanoid_model``   free pelvis + 2 legs x 6 + torso yaw + 2 arms x 4,
                       4 sole corners per foot and one point per hand.

Every inertia comes from a solid box, so it is physically valid by
construction.  All floating values are rounded to float32 so that the FP32
device path and the FP64 oracle start from identical numbers.

Model dict keys: floating_base, parent[nb], axis[nb,3], R_tree[nb,3,3],
p_tree[nb,3], mass[nb], com[nb,3], inertia[nb,6] (xx yy zz xy xz yz about the
com), q_min/q_max/tau_max/kp/kd/q0[n_u], contact_body[nc], contact_pos[nc,3],
k_contact, d_contact, mu, eps_fric, gravity, ee_body, ee_pos[3], n_substeps,
armature[n_u] (reflected rotor inertia per joint), x0[nq+nv].
"""
import numpy as np

GRAVITY = 9.81

# Cost weights of the paper's Table (cost-weights): w_h, w_orient, w_q, w_c_vel, w_c_force, w_H.
COST_WEIGHTS = {
    "walking": (1e2, 10.0, 0.0, 0.5, 5e-2, 2.5e3),
    "jumping": (1.0, 0.5, 0.3, 1.0, 5e-4, 2e3),
    "handstand": (50.0, 10.0, 0.3, 1.0, 5e-4, 0.0),
    "backflip": (1.0, 0.5, 0.3, 1.0, 5e-4, 2e3),
    "bipedal": (10.0, 1.0, 0.3, 1.0, 5e-4, 2e2),
}


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def _box_inertia(m, a, b, c):
    """Solid box of mass m and edge lengths a, b, c along x, y, z about its centre."""
    return np.array([m * (b * b + c * c) / 12.0, m * (a * a + c * c) / 12.0,
                     m * (a * a + b * b) / 12.0, 0.0, 0.0, 0.0])


class _Tree:
    def __init__(self):
        self.parent, self.axis, self.R, self.p, self.mass, self.com, self.inertia = \
            [], [], [], [], [], [], []
        self.q_min, self.q_max, self.tau_max, self.kp, self.kd, self.q0 = [], [], [], [], [], []

    def body(self, parent, axis, p, mass, com, box, joint=None):
        """Append a body; `joint` = (q_min, q_max, tau_max, kp, kd, q0) for a revolute body."""
        self.parent.append(parent)
        self.axis.append(np.asarray(axis, float))
        self.R.append(np.eye(3))
        self.p.append(np.asarray(p, float))
        self.mass.append(mass)
        self.com.append(np.asarray(com, float))
        self.inertia.append(_box_inertia(mass, *box))
        if joint is not None:
            for lst, val in zip((self.q_min, self.q_max, self.tau_max, self.kp, self.kd, self.q0),
                                joint):
                lst.append(val)
        return len(self.parent) - 1

    def finish(self, name, floating, contact_body, contact_pos, ee_body=-1, ee_pos=(0, 0, 0)):
        nc = len(contact_body)
        m = {
            "name": name,
            "floating_base": bool(floating),
            "parent": np.asarray(self.parent, np.int32),
            "axis": f32(self.axis),
            "R_tree": f32(self.R),
            "p_tree": f32(self.p),
            "mass": f32(self.mass),
            "com": f32(self.com),
            "inertia": f32(self.inertia),
            "q_min": f32(self.q_min),
            "q_max": f32(self.q_max),
            "tau_max": f32(self.tau_max),
            "kp": f32(self.kp),
            "kd": f32(self.kd),
            "q0": f32(self.q0),
            "contact_body": np.asarray(contact_body, np.int32).reshape(nc),
            "contact_pos": f32(np.asarray(contact_pos, float).reshape(nc, 3)),
            "k_contact": 2e4,
            "d_contact": 200.0,
            "mu": 0.8,
            "eps_fric": 0.01,
            "gravity": GRAVITY,
            "ee_body": int(ee_body),
            "ee_pos": f32(ee_pos),
        }
        m["n_u"] = len(m["q0"])
        m["n_q"] = m["n_u"] + (7 if floating else 0)
        m["n_v"] = m["n_u"] + (6 if floating else 0)
        return m


def chain_model(seed=0):
    """Fixed-base planar 3R arm: links along +x at q = 0, joint axes along y, no contact."""
    rng = np.random.default_rng(seed)
    L = 0.3 * (1 + rng.uniform(-0.1, 0.1, 3))
    mass = 1.0 * (1 + rng.uniform(-0.1, 0.1, 3))
    t = _Tree()
    prev = -1
    for i in range(3):
        p = (0.0, 0.0, 0.0) if i == 0 else (L[i - 1], 0.0, 0.0)
        prev = t.body(prev, (0, 1, 0), p, mass[i], (L[i] / 2, 0, 0), (L[i], 0.04, 0.04),
                      joint=(-2.5, 2.5, 30.0, 30.0, 0.3, 0.0))
    m = t.finish("chain3", False, [], np.zeros((0, 3)), ee_body=2, ee_pos=(L[2], 0, 0))
    m["n_substeps"] = 1
    m["armature"] = f32(np.zeros(3))
    m["x0"] = f32(np.zeros(6))
    return m


def quadruped_model(seed=0):
    """Free base + 4 legs of (abduction about x, hip about y, knee about y), point feet.

    Base 6-15 kg, every link 0.3-1.5 kg (drawn per link type, shared by the legs).
    The initial state stands on the four feet with the static spring compression.
    """
    rng = np.random.default_rng(seed)
    jit = lambda v: v * (1 + rng.uniform(-0.1, 0.1))  # noqa: E731
    m_base = rng.uniform(6.0, 15.0)
    m_abd, m_thigh, m_shank = rng.uniform(0.3, 1.5, 3)
    bx, by, bz = jit(0.45), jit(0.25), jit(0.12)
    hx, hy, off = jit(0.19), jit(0.05), jit(0.08)
    L = jit(0.21)
    hip0, knee0 = 0.8, -1.6
    t = _Tree()
    t.body(-1, (0, 0, 1), (0, 0, 0), m_base, (0, 0, 0), (bx, by, bz))
    feet = []
    for sx, sy in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
        a = t.body(0, (1, 0, 0), (sx * hx, sy * hy, 0), m_abd, (0, sy * 0.03, 0), (0.08, 0.06, 0.06),
                   joint=(-0.8, 0.8, 25.0, 150.0, 3.0, 0.0))
        h = t.body(a, (0, 1, 0), (0, sy * off, 0), m_thigh, (0, 0, -L / 2), (0.04, 0.04, L),
                   joint=(-1.0, 2.6, 25.0, 150.0, 3.0, hip0))
        k = t.body(h, (0, 1, 0), (0, 0, -L), m_shank, (0, 0, -L / 2), (0.03, 0.03, L),
                   joint=(-2.7, -0.5, 45.0, 150.0, 3.0, knee0))
        feet.append(k)
    cpos = [(0.0, 0.0, -L)] * 4
    m = t.finish("quadruped18", True, feet, cpos)
    m["n_substeps"] = 1
    m["armature"] = f32(np.full(m["n_u"], 0.01))
    m_tot = float(np.sum(m["mass"]))
    sink = m_tot * GRAVITY / (4 * m["k_contact"])
    z0 = 2 * L * np.cos(hip0) - sink
    q = np.concatenate([[0.0, 0.0, z0, 1.0, 0.0, 0.0, 0.0], np.tile([0.0, hip0, knee0], 4)])
    m["x0"] = f32(np.concatenate([q, np.zeros(m["n_v"])]))
    m["support"] = np.ones(4, bool)
    return m


def hexapod_model(seed=0):
    """Free base + 6 legs of (abduction about x, hip about y, knee about y), point feet:
    a legged tree of six three-body chains (19 bodies), built like the quadruped.

    Base 8-20 kg, every link 0.2-1.0 kg (drawn per link type, shared by the legs).
    The initial state stands on the six feet with the static spring compression.
    """
    rng = np.random.default_rng(seed)
    jit = lambda v: v * (1 + rng.uniform(-0.1, 0.1))  # noqa: E731
    m_base = rng.uniform(8.0, 20.0)
    m_abd, m_thigh, m_shank = rng.uniform(0.2, 1.0, 3)
    bx, by, bz = jit(0.60), jit(0.30), jit(0.10)
    hx, hy, off = jit(0.25), jit(0.12), jit(0.06)
    L = jit(0.18)
    hip0, knee0 = 0.8, -1.6
    t = _Tree()
    t.body(-1, (0, 0, 1), (0, 0, 0), m_base, (0, 0, 0), (bx, by, bz))
    feet = []
    for sx, sy in ((1, 1), (1, -1), (0, 1), (0, -1), (-1, 1), (-1, -1)):
        a = t.body(0, (1, 0, 0), (sx * hx, sy * hy, 0), m_abd, (0, sy * 0.03, 0), (0.07, 0.05, 0.05),
                   joint=(-0.8, 0.8, 20.0, 120.0, 2.5, 0.0))
        h = t.body(a, (0, 1, 0), (0, sy * off, 0), m_thigh, (0, 0, -L / 2), (0.04, 0.04, L),
                   joint=(-1.0, 2.6, 20.0, 120.0, 2.5, hip0))
        k = t.body(h, (0, 1, 0), (0, 0, -L), m_shank, (0, 0, -L / 2), (0.03, 0.03, L),
                   joint=(-2.7, -0.5, 35.0, 120.0, 2.5, knee0))
        feet.append(k)
    cpos = [(0.0, 0.0, -L)] * 6
    m = t.finish("hexapod24", True, feet, cpos)
    m["n_substeps"] = 1
    m["armature"] = f32(np.full(m["n_u"], 0.01))
    m_tot = float(np.sum(m["mass"]))
    sink = m_tot * GRAVITY / (6 * m["k_contact"])
    z0 = 2 * L * np.cos(hip0) - sink
    q = np.concatenate([[0.0, 0.0, z0, 1.0, 0.0, 0.0, 0.0], np.tile([0.0, hip0, knee0], 6)])
    m["x0"] = f32(np.concatenate([q, np.zeros(m["n_v"])]))
    m["support"] = np.ones(6, bool)
    return m


def humanoid_model(seed=0):
    """Free pelvis + 2 legs x 6 + torso yaw + 2 arms x 4 (27 DoF), 10 contact points.

    Masses per link type drawn inside 0.5-20 kg.  Feet are boxes with a contact
    point at each sole corner (+-0.1 x +-0.04 m); each forearm end is a hand point.
    """
    rng = np.random.default_rng(seed)
    jit = lambda v: v * (1 + rng.uniform(-0.1, 0.1))  # noqa: E731
    m_pelvis = rng.uniform(5.0, 12.0)
    m_torso = rng.uniform(10.0, 20.0)
    m_hipy, m_hipr = rng.uniform(0.5, 2.0, 2)
    m_thigh, m_shank = rng.uniform(2.0, 6.0), rng.uniform(1.5, 4.0)
    m_ankle, m_foot = rng.uniform(0.5, 1.0), rng.uniform(0.5, 1.5)
    m_sp, m_sr, m_ua, m_fa = rng.uniform(0.5, 2.5, 4)
    Lt = jit(0.35)
    La, Lf = jit(0.25), jit(0.25)
    hf = 0.05
    bend = 0.3
    big, small, foot_g = (400.0, 8.0), (60.0, 1.5), (1000.0, 10.0)
    t = _Tree()
    t.body(-1, (0, 0, 1), (0, 0, 0), m_pelvis, (0, 0, 0), (0.2, 0.3, 0.15))
    feet, cpos = [], []
    for s in (1, -1):
        a = t.body(0, (0, 0, 1), (0, s * 0.09, -0.06), m_hipy, (0, 0, -0.03), (0.06, 0.06, 0.06),
                   joint=(-0.8, 0.8, 80.0, *big, 0.0))
        b = t.body(a, (1, 0, 0), (0, 0, -0.05), m_hipr, (0, 0, -0.03), (0.06, 0.06, 0.06),
                   joint=(-0.6, 0.6, 80.0, *big, 0.0))
        c = t.body(b, (0, 1, 0), (0, 0, -0.05), m_thigh, (0, 0, -Lt / 2), (0.1, 0.1, Lt),
                   joint=(-2.0, 1.0, 120.0, *big, -bend))
        d = t.body(c, (0, 1, 0), (0, 0, -Lt), m_shank, (0, 0, -Lt / 2), (0.08, 0.08, Lt),
                   joint=(0.0, 2.4, 150.0, *big, 2 * bend))
        e = t.body(d, (0, 1, 0), (0, 0, -Lt), m_ankle, (0, 0, -0.02), (0.05, 0.05, 0.04),
                   joint=(-0.9, 0.6, 40.0, *foot_g, -bend))
        f = t.body(e, (1, 0, 0), (0, 0, -0.04), m_foot, (0.02, 0, -0.03), (0.22, 0.1, 0.04),
                   joint=(-0.4, 0.4, 40.0, *foot_g, 0.0))
        for cx in (0.12, -0.08):
            for cy in (0.04, -0.04):
                feet.append(f)
                cpos.append((cx, cy, -hf))
    torso = t.body(0, (0, 0, 1), (0, 0, 0.1), m_torso, (0, 0, 0.2), (0.25, 0.3, 0.4),
                   joint=(-1.0, 1.0, 100.0, *big, 0.0))
    hands = []
    for s in (1, -1):
        a = t.body(torso, (0, 1, 0), (0, s * 0.2, 0.35), m_sp, (0, 0, 0), (0.06, 0.06, 0.06),
                   joint=(-2.5, 2.5, 40.0, *small, 0.0))
        b = t.body(a, (1, 0, 0), (0, 0, 0), m_sr, (0, 0, -0.03), (0.06, 0.06, 0.06),
                   joint=(-1.5, 1.5, 40.0, *small, 0.0))
        c = t.body(b, (0, 0, 1), (0, 0, -0.05), m_ua, (0, 0, -La / 2), (0.06, 0.06, La),
                   joint=(-1.5, 1.5, 40.0, *small, 0.0))
        d = t.body(c, (0, 1, 0), (0, 0, -La), m_fa, (0, 0, -Lf / 2), (0.05, 0.05, Lf),
                   joint=(-2.5, 0.0, 40.0, *small, -0.3))
        hands.append(d)
    cbody = feet + hands
    cpos = cpos + [(0.0, 0.0, -Lf)] * 2
    m = t.finish("humanoid27", True, cbody, cpos)
    m["n_substeps"] = 1
    m["armature"] = f32(np.full(m["n_u"], 0.02))
    m_tot = float(np.sum(m["mass"]))
    sink = m_tot * GRAVITY / (8 * m["k_contact"])
    depth = 0.06 + 0.05 + 0.05 + 2 * Lt * np.cos(bend) + 0.04 + hf
    q = np.concatenate([[0.0, 0.0, depth - sink, 1.0, 0.0, 0.0, 0.0], m["q0"]])
    m["x0"] = f32(np.concatenate([q, np.zeros(m["n_v"])]))
    m["support"] = np.array([True] * 8 + [False] * 2)
    return m


MODELS = {"chain": chain_model, "quadruped": quadruped_model, "humanoid": humanoid_model}


def nominal_knots(model, n_knots):
    """Warm start: every position knot at the stance q0, every velocity knot at zero."""
    nu = model["n_u"]
    kq = np.tile(model["q0"], (n_knots, 1))
    return f32(np.concatenate([kq.reshape(-1), np.zeros(n_knots * nu)]))


def params(model, n_samples, horizon, dt, n_knots, n_iters, noise, cost, lam=1.0):
    """Controller parameters.  noise = ("exp", scale_q, beta1, beta2) or ("linear", lo, hi);
    cost = "ee" (end-effector height, fixed base) or a row name of COST_WEIGHTS."""
    p = {
        "n_samples": int(n_samples), "horizon": int(horizon), "n_knots": int(n_knots),
        "n_iters": int(n_iters), "dt": float(np.float32(dt)), "lambda": float(lam),
        "weight_mode": 0, "noise_mode": 0, "scale_q": 0.0, "beta1": 1.0, "beta2": 1.0,
        "sigma_lo": 0.0, "sigma_hi": 0.0, "cost_kind": 0,
        "w_h": 0.0, "w_or": 0.0, "w_q": 0.0, "w_cv": 0.0, "w_cf": 0.0, "w_eff": 0.0, "w_H": 0.0,
        "w_ee": 0.0, "w_tau": 0.0, "z_des": 0.0, "v_des": [0.0, 0.0, 0.0],
        "q0_cost": model["q0"].copy(), "f0z": np.zeros(max(len(model["contact_body"]), 0)),
    }
    if noise[0] == "exp":
        p["noise_mode"] = 0
        p["scale_q"], p["beta1"], p["beta2"] = map(float, noise[1:])
    else:
        p["noise_mode"] = 1
        p["sigma_lo"], p["sigma_hi"] = map(float, noise[1:])
    if cost == "ee":
        p["cost_kind"] = 0
        p["w_ee"], p["w_tau"], p["z_des"] = 1e2, 1e-3, 0.5
    else:
        p["cost_kind"] = 1
        w = COST_WEIGHTS[cost]
        p["w_h"], p["w_or"], p["w_q"], p["w_cv"], p["w_cf"], p["w_H"] = w
        p["w_eff"] = 1e-3
        p["z_des"] = float(model["x0"][2])
        p["v_des"] = [0.5, 0.0, 0.0]
        support = model.get("support", np.ones(len(model["contact_body"]), bool))
        m_tot = float(np.sum(model["mass"]))
        p["f0z"] = f32(np.where(support, m_tot * GRAVITY / max(int(np.sum(support)), 1), 0.0))
    return p


def ytree_model(seed=0):
    """Fixed-base branching arm: a yaw root joint carrying a 2-link branch and a
    3-link branch (the shorter one hangs off the root joint body, so its chain
    attaches to a joint, not to a floating base)."""
    rng = np.random.default_rng(seed)
    L = 0.25 * (1 + rng.uniform(-0.1, 0.1, 5))
    ms = 1.0 * (1 + rng.uniform(-0.2, 0.2, 6))
    jt = (-2.5, 2.5, 30.0, 30.0, 0.3, 0.0)
    t = _Tree()
    r = t.body(-1, (0, 0, 1), (0, 0, 0), ms[0], (0, 0, 0.05), (0.1, 0.1, 0.1), joint=jt)
    a = t.body(r, (0, 1, 0), (0, 0.1, 0.1), ms[1], (L[0] / 2, 0, 0), (L[0], 0.04, 0.04), joint=jt)
    b = t.body(a, (0, 1, 0), (L[0], 0, 0), ms[2], (L[1] / 2, 0, 0), (L[1], 0.04, 0.04), joint=jt)
    c = t.body(b, (1, 0, 0), (L[1], 0, 0), ms[3], (L[2] / 2, 0, 0), (L[2], 0.04, 0.04), joint=jt)
    d = t.body(r, (0, 1, 0), (0, -0.1, 0.1), ms[4], (L[3] / 2, 0, 0), (L[3], 0.04, 0.04), joint=jt)
    t.body(d, (0, 1, 0), (L[3], 0, 0), ms[5], (L[4] / 2, 0, 0), (L[4], 0.04, 0.04), joint=jt)
    m = t.finish("ytree6", False, [], np.zeros((0, 3)), ee_body=c, ee_pos=(L[2], 0, 0))
    m["n_substeps"] = 1
    m["armature"] = f32(np.full(6, 0.01))
    m["x0"] = f32(np.zeros(12))
    return m


# Targets of the tasks of Sec. IV-B (the paper gives the weights, Tab. cost-weights,
# and describes the targets in words; the numbers below are this synthetic stand-in's):
#   walking   commanded forward velocity 0.5 m/s, level base;
#   jumping   terminal base height raised by JUMP_RISE (the paper's 0.325 -> 0.7 m step);
#   handstand base pitched 45 degrees nose down;
#   backflip  base pitched 180 degrees;
#   bipedal   humanoid walking at 0.5 m/s, level pelvis.
JUMP_RISE = 0.375
TASKS = ("walking", "jumping", "handstand", "backflip", "bipedal")
# Sampling of the closed-loop task runs on the synthetic robots (the paper gives no
# temperature; with 64 samples and the 0.4 rad kernel no sample ever beats the held
# stance on these models, so the runs use more samples, a smaller noise scale and a
# sharper softmax).
TASK_SAMPLING = {"n_samples": 1024, "scale_q": 0.1, "lambda": 0.1}


def pitch_quaternion(deg):
    """Unit quaternion (w, x, y, z) of a rotation by deg about the base y axis
    (positive: nose down for x forward, z up)."""
    h = np.deg2rad(deg) / 2
    return [float(np.float32(np.cos(h))), 0.0, float(np.float32(np.sin(h))), 0.0]


def task_params(model, p, name):
    """Parameters p with the weights of the task's row of the cost-weights table and
    the task's targets."""
    p = dict(p)
    p["cost_kind"] = 1
    p["w_h"], p["w_or"], p["w_q"], p["w_cv"], p["w_cf"], p["w_H"] = COST_WEIGHTS[name]
    z0 = float(model["x0"][2])
    p["z_des"] = z0
    p["v_des"] = [0.0, 0.0, 0.0]
    p["q_des"] = [0.0, 0.0, 0.0, 0.0]
    p["terminal_z_abs"], p["z_terminal"] = 0, 0.0
    if name in ("walking", "bipedal"):
        p["v_des"] = [0.5, 0.0, 0.0]
    elif name == "jumping":
        p["terminal_z_abs"], p["z_terminal"] = 1, float(np.float32(z0 + JUMP_RISE))
    elif name == "handstand":
        p["q_des"] = pitch_quaternion(45.0)
    elif name == "backflip":
        p["q_des"] = pitch_quaternion(180.0)
    else:
        raise KeyError(name)
    return p


# The five workloads: shapes, sizes and noise/cost settings of each configuration.
def config(name, n_samples=None, seed=0):
    """(model, params, seed) of a named workload.

    chain        3R arm, K=32, H=50, dt=0.01, 4 knots, 10 iterations, linear std 0.1->0.3
    quadruped    18 DoF, K=64, H=100, dt=0.005, 8 knots, 3 iterations, exp kernel 0.4
    quadruped_tp 18 DoF at throughput scale, K in {256,1024,4096}, H=200, 1 iteration,
                 linear std 0.05->0.4
    humanoid     27 DoF, K=256, H=150, dt=0.004, 10 knots, 3 iterations, exp kernel 0.4
    hexapod      24 DoF (six three-joint legs), K=64, H=100, as quadruped
    """
    if name == "chain":
        m = chain_model(seed)
        p = params(m, n_samples or 32, 50, 0.01, 4, 10, ("linear", 0.1, 0.3), "ee")
    elif name == "quadruped":
        m = quadruped_model(seed)
        p = params(m, n_samples or 64, 100, 0.005, 8, 3, ("exp", 0.4, 1.0, 1.0), "walking")
    elif name == "quadruped_tp":
        m = quadruped_model(seed)
        p = params(m, n_samples or 4096, 200, 0.005, 8, 1, ("linear", 0.05, 0.4), "walking")
    elif name == "humanoid":
        m = humanoid_model(seed)
        p = params(m, n_samples or 256, 150, 0.004, 10, 3, ("exp", 0.4, 1.0, 1.0), "bipedal")
    elif name == "hexapod":
        m = hexapod_model(seed)
        p = params(m, n_samples or 64, 100, 0.005, 8, 3, ("exp", 0.4, 1.0, 1.0), "walking")
    else:
        raise KeyError(name)
    return m, p, 1000 + seed


def serving_mix(n_robots=64, seed=0):
    """Robots of the serving workload: model kind uniform over chain / quadruped / humanoid,
    K uniform over multiples of 32 in [32, 1024], H uniform in [50, 200], 3 iterations;
    Poisson ticks at 50 Hz per robot.  Returns a list of (model, params, seed) triples."""
    rng = np.random.default_rng(10_000 + seed)
    out = []
    kinds = ("chain", "quadruped", "humanoid")
    for r in range(n_robots):
        kind = kinds[int(rng.integers(0, 3))]
        K = 32 * int(rng.integers(1, 33))
        H = int(rng.integers(50, 201))
        mseed = int(rng.integers(0, 10))
        if kind == "chain":
            m = chain_model(mseed)
            p = params(m, K, H, 0.01, 4, 3, ("linear", 0.1, 0.3), "ee")
        elif kind == "quadruped":
            m = quadruped_model(mseed)
            p = params(m, K, H, 0.005, 8, 3, ("exp", 0.4, 1.0, 1.0), "walking")
        else:
            m = humanoid_model(mseed)
            p = params(m, K, H, 0.004, 10, 3, ("exp", 0.4, 1.0, 1.0), "bipedal")
        out.append((m, p, 20_000 + r))
    return out


def poisson_ticks(n_robots, duration_s, rate_hz=50.0, seed=0):
    """Arrival times (s) per robot: exponential inter-arrival with mean 1/rate."""
    rng = np.random.default_rng(30_000 + seed)
    ticks = []
    for r in range(n_robots):
        t, ts = 0.0, []
        while True:
            t += rng.exponential(1.0 / rate_hz)
            if t >= duration_s:
                break
            ts.append(t)
        ticks.append(np.asarray(ts))
    return ticks


def perturbed_states(model, count, seed=0, scale=0.05):
    """States near x0 (joint angles, base pose and all velocities jittered) for
    teacher-forced dynamics checks.  Quaternions are renormalised."""
    rng = np.random.default_rng(seed)
    nq, nv = model["n_q"], model["n_v"]
    X = np.tile(model["x0"], (count, 1))
    X[:, :nq] += rng.normal(0, scale, (count, nq))
    X[:, nq:] += rng.normal(0, 10 * scale, (count, nv))
    if model["floating_base"]:
        X[:, 3:7] /= np.linalg.norm(X[:, 3:7], axis=1, keepdims=True)
    lo, hi = model["q_min"], model["q_max"]
    off = 7 if model["floating_base"] else 0
    X[:, off:off + model["n_u"]] = np.clip(X[:, off:off + model["n_u"]], lo, hi)
    return f32(X)
