"""CPU oracle for the reference-free MPPI step -- TEST INFRASTRUCTURE ONLY.

This package wraps ``liboracle.so`` (plain scalar C++, FP64) with ctypes.  It is
imported only by ``tests/``, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of ``bench.py``; the product library never loads it and
shares no code with it.  Models and parameters arrive as the plain dicts made by
``paper_2511_19204_amd.synth`` (inputs only, no method arithmetic).

Each function names the part of Schramm et al. (arXiv 2511.19204) it follows:
  philox / normals ........ counter-based noise for Alg. 1's sampling step
  sigma_table ............. eq. overall-noise-kernel (Sec. III-B), or linear
  hermite ................. eq. hermite_segment with its basis (Sec. III-A)
  sample_knots ............ Alg. 1 sampling step + eq. vel-clamp
  forward_dynamics ........ articulated-body algorithm (the simulator's dynamics)
  rollout ................. Alg. 1 simulate step with the Sec. IV-A costs
  forced_steps ............ one control step of that simulate step from given states
  weights ................. eq. omega-weights / eq. softmax_minmax
  weighted_average ........ eq. update-nominal carried to the knots
  step .................... Alg. 1 inner loop with Sec. III-D best tracking
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_ip = C.POINTER(C.c_int32)
_up = C.POINTER(C.c_uint32)


class OrcModel(C.Structure):
    _fields_ = [
        ("n_bodies", C.c_int32), ("floating_base", C.c_int32), ("parent", _ip),
        ("axis", _dp), ("R_tree", _dp), ("p_tree", _dp), ("mass", _dp), ("com", _dp),
        ("inertia", _dp), ("q_min", _dp), ("q_max", _dp), ("tau_max", _dp), ("kp", _dp),
        ("kd", _dp), ("n_contacts", C.c_int32), ("contact_body", _ip), ("contact_pos", _dp),
        ("k_contact", C.c_double), ("d_contact", C.c_double), ("mu", C.c_double),
        ("eps_fric", C.c_double), ("gravity", C.c_double), ("ee_body", C.c_int32),
        ("ee_pos", C.c_double * 3), ("n_substeps", C.c_int32), ("armature", _dp),
    ]


class OrcParams(C.Structure):
    _fields_ = [
        ("n_samples", C.c_int32), ("horizon", C.c_int32), ("n_knots", C.c_int32),
        ("n_iters", C.c_int32), ("dt", C.c_double), ("lam", C.c_double),
        ("weight_mode", C.c_int32), ("noise_mode", C.c_int32), ("scale_q", C.c_double),
        ("beta1", C.c_double), ("beta2", C.c_double), ("sigma_lo", C.c_double),
        ("sigma_hi", C.c_double), ("cost_kind", C.c_int32), ("w_h", C.c_double),
        ("w_or", C.c_double), ("w_q", C.c_double), ("w_cv", C.c_double), ("w_cf", C.c_double),
        ("w_eff", C.c_double), ("w_H", C.c_double), ("w_ee", C.c_double), ("w_tau", C.c_double),
        ("z_des", C.c_double), ("v_des", C.c_double * 3), ("f0z", _dp),
        ("q0_cost", _dp), ("spline_mode", C.c_int32), ("q_des", C.c_double * 4),
        ("terminal_z_abs", C.c_int32), ("z_terminal", C.c_double),
    ]


def lib():
    global _lib
    if _lib is None:
        # ORACLE_LIB: another build of the same source (the sanitizer build)
        path = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        _lib = C.CDLL(path)
        _lib.orc_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_int, C.c_int, C.c_int, _dp, _dp]
        _lib.orc_sample_knots.argtypes = [C.c_void_p, C.c_void_p, _dp, C.c_uint64, C.c_uint32,
                                          C.c_int, C.c_int, _dp]
        _lib.orc_rollouts.argtypes = [C.c_void_p, C.c_void_p, _dp, _dp, C.c_uint64, C.c_uint32,
                                      C.c_int, C.c_int, C.c_int, _dp, _dp, C.c_int]
        _lib.orc_step.argtypes = [C.c_void_p, C.c_void_p, _dp, _dp, C.c_uint64, C.c_uint32, _dp,
                                  _dp, _dp, _ip, _dp, _ip, _ip, C.c_int]
        _lib.orc_step_f32.argtypes = _lib.orc_step.argtypes
        _lib.orc_rollout_f32_traj.argtypes = [C.c_void_p, C.c_void_p, _dp, _dp, _dp]
        _lib.orc_shift_knots.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, _dp]
        _lib.orc_spline_slopes.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, _dp]
        _lib.orc_hermite.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                     _dp, _dp]
        _lib.orc_weights.argtypes = [C.c_int, _dp, C.c_double, C.c_int, _dp, _ip]
        _lib.orc_euler_step.argtypes = [C.c_void_p, C.c_double, _dp, _dp, _dp, _dp]
        _lib.orc_step_dynamics.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp,
                                           _dp, _dp]
        _lib.orc_rk4.argtypes = [C.c_void_p, C.c_double, C.c_int, _dp, _dp, _dp]
        _lib.orc_dense_route_update.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                                _dp, _dp, _dp]
        _lib.orc_count_selftest.argtypes = [_dp]
        _lib.orc_count_ops.argtypes = [C.c_void_p, C.c_void_p, _dp, _dp, C.c_uint64, C.c_int, _dp]
        _lib.orc_integrate_batch.argtypes = [C.c_void_p, C.c_double, C.c_int, _dp, _dp, _dp]
        _lib.orc_forced_steps.argtypes = [C.c_void_p, C.c_void_p, _dp, C.c_int, _dp, _dp, _dp, _dp, _up,
                                          _dp, _dp, C.c_int, C.c_int]
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


class _Model:
    """orc_model view of a synth model dict (keeps the arrays alive)."""

    def __init__(self, m):
        self.keep = []
        s = OrcModel()
        nb = int(len(m["parent"]))
        s.n_bodies = nb
        s.floating_base = 1 if m["floating_base"] else 0
        for name in ("parent",):
            a, p = _i(m[name]); self.keep.append(a); setattr(s, name, p)
        for name in ("axis", "R_tree", "p_tree", "mass", "com", "inertia", "q_min", "q_max",
                     "tau_max", "kp", "kd"):
            a, p = _d(np.asarray(m[name]).reshape(-1)); self.keep.append(a); setattr(s, name, p)
        nc = int(len(m["contact_body"]))
        s.n_contacts = nc
        a, p = _i(m["contact_body"] if nc else np.zeros(1, np.int32)); self.keep.append(a)
        s.contact_body = p
        a, p = _d(np.asarray(m["contact_pos"]).reshape(-1) if nc else np.zeros(3)); self.keep.append(a)
        s.contact_pos = p
        s.k_contact = float(m["k_contact"]); s.d_contact = float(m["d_contact"])
        s.mu = float(m["mu"]); s.eps_fric = float(m["eps_fric"]); s.gravity = float(m["gravity"])
        s.ee_body = int(m["ee_body"])
        for k in range(3):
            s.ee_pos[k] = float(m["ee_pos"][k])
        s.n_substeps = int(m.get("n_substeps", 1))
        arm = np.asarray(m.get("armature", np.zeros(self_nu := nb - (1 if m["floating_base"] else 0))),
                         dtype=np.float64)
        a, s.armature = _d(arm); self.keep.append(a)
        self.s = s
        self.nu = nb - (1 if m["floating_base"] else 0)
        self.nq = self.nu + (7 if m["floating_base"] else 0)
        self.nv = self.nu + (6 if m["floating_base"] else 0)
        self.nc = nc

    @property
    def ptr(self):
        return C.addressof(self.s)


class _Params:
    def __init__(self, p, nu, nc=None):
        # the C oracle reads f0z per contact point and q0_cost per joint
        if nc is not None and "f0z" in p and len(p["f0z"]) != nc:
            raise ValueError(f"f0z has {len(p['f0z'])} entries for {nc} contact points")
        if nc is not None and "q0_cost" in p and len(p["q0_cost"]) != nu:
            raise ValueError(f"q0_cost has {len(p['q0_cost'])} entries for {nu} joints")
        s = OrcParams()
        for name in ("n_samples", "horizon", "n_knots", "n_iters", "weight_mode", "noise_mode",
                     "cost_kind"):
            setattr(s, name, int(p[name]))
        for name in ("dt", "scale_q", "beta1", "beta2", "sigma_lo", "sigma_hi", "w_h", "w_or",
                     "w_q", "w_cv", "w_cf", "w_eff", "w_H", "w_ee", "w_tau", "z_des"):
            setattr(s, name, float(p[name]))
        s.lam = float(p["lambda"])
        for k in range(3):
            s.v_des[k] = float(p["v_des"][k])
        q0 = np.asarray(p.get("q0_cost", np.zeros(nu)), dtype=np.float64)
        self.q0, s.q0_cost = _d(q0)
        f0 = np.asarray(p.get("f0z", np.zeros(1)), dtype=np.float64).reshape(-1)
        self.f0, s.f0z = _d(f0 if f0.size else np.zeros(1))
        s.spline_mode = int(p.get("spline_mode", 0))
        qd = p.get("q_des", (0.0, 0.0, 0.0, 0.0))
        for k in range(4):
            s.q_des[k] = float(qd[k])
        s.terminal_z_abs = int(p.get("terminal_z_abs", 0))
        s.z_terminal = float(p.get("z_terminal", 0.0))
        self.s = s

    @property
    def ptr(self):
        return C.addressof(self.s)


def _check(rc, what):
    if rc < 0:
        raise ValueError(f"oracle rejected the arguments of {what}")
    return rc


# ----------------------------------------------------------------------------------------------
def philox(ctr, key):
    """Philox4x32-10 block function: 4 counter words, 2 key words -> 4 words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox(c.ctypes.data_as(_up), k.ctypes.data_as(_up), out.ctypes.data_as(_up))
    return out


def normals(seed, tick, iota, n, count):
    """(z_q, z_v) standard normals of knot slots 0..count-1 of sample n."""
    zq = np.zeros(count); zv = np.zeros(count)
    lib().orc_normals(seed, tick, iota, n, count, zq.ctypes.data_as(_dp), zv.ctypes.data_as(_dp))
    return zq, zv


def sigma_table(params):
    p = _Params(params, 1)
    out = np.zeros((params["n_iters"], params["n_knots"]))
    _check(lib().orc_sigma_table(C.c_void_p(p.ptr), out.ctypes.data_as(_dp)), "sigma_table")
    return out


def hermite(knots, nk, nu, H, dt, h, j):
    k, kp = _d(knots)
    qr = C.c_double(); vr = C.c_double()
    _check(lib().orc_hermite(kp, nk, nu, H, dt, h, j, C.byref(qr), C.byref(vr)), "hermite")
    return qr.value, vr.value


def shift_knots(knots, nk, nu, H, dt, n_steps, spline_mode=0):
    """Warm-start shift of the best trajectory's knots by n_steps control steps
    (Sec. III-E): the old spline at t_k + n_steps dt, clamped to the horizon end
    (position-only variants: new knot slopes from the shifted positions)."""
    k, kp = _d(knots)
    out = np.zeros(2 * nk * nu)
    _check(lib().orc_shift_knots(kp, nk, nu, H, dt, int(n_steps), int(spline_mode), out.ctypes.data_as(_dp)),
           "shift_knots")
    return out


def spline_slopes(mode, knots, nk, nu, delta):
    """Knots with the velocity block replaced by the slopes of the position-only
    spline variant `mode` (1 natural cubic, 2 quadratic) through the positions."""
    out = np.array(knots, dtype=np.float64)
    _check(lib().orc_spline_slopes(int(mode), nk, nu, float(delta), out.ctypes.data_as(_dp)), "spline_slopes")
    return out


def predict(model, params, x0, knots, n_steps):
    """State prediction (Sec. III-E): the state after simulating n_steps control
    steps of the trajectory the knots define, from x0 (the rollout's own
    dynamics along the horizon's timeline)."""
    H = params["horizon"]
    if not 0 <= n_steps <= H:
        raise ValueError("n_steps must be in 0..horizon")
    _, traj, _, _ = rollout(model, params, x0, knots, debug=True)
    return traj[n_steps]


def predict_f32(model, params, x0, knots, n_steps):
    """predict() in the oracle's float instantiation (rounding reference only)."""
    M = _Model(model); P = _Params(params, M.nu, M.nc)
    xa, xp = _d(x0); ka, kp = _d(knots)
    traj = np.zeros((params["horizon"] + 1, M.nq + M.nv))
    _check(lib().orc_rollout_f32_traj(C.c_void_p(M.ptr), C.c_void_p(P.ptr), xp, kp, traj.ctypes.data_as(_dp)),
           "rollout_f32_traj")
    return traj[n_steps]


def sample_knots(model, params, nominal, seed, tick, iota, n):
    M = _Model(model); P = _Params(params, M.nu, M.nc)
    nom, npt = _d(nominal)
    out = np.zeros(2 * params["n_knots"] * M.nu)
    _check(lib().orc_sample_knots(M.ptr, P.ptr, npt, seed, tick, iota, n, out.ctypes.data_as(_dp)),
           "sample_knots")
    return out


def forward_dynamics(model, q, v, tau, with_contacts=True, return_forces=False):
    M = _Model(model)
    qa, qp = _d(q); va, vp = _d(v); ta, tp = _d(tau)
    qdd = np.zeros(M.nv); cf = np.zeros(max(M.nc, 1) * 3)
    _check(lib().orc_forward_dynamics(C.c_void_p(M.ptr), qp, vp, tp, int(with_contacts),
                                      qdd.ctypes.data_as(_dp), cf.ctypes.data_as(_dp)), "fd")
    if return_forces:
        return qdd, cf[:M.nc * 3].reshape(M.nc, 3)
    return qdd


def forward_dynamics_f32(model, q, v, tau, with_contacts=True):
    M = _Model(model)
    qa = np.ascontiguousarray(q, np.float32); va = np.ascontiguousarray(v, np.float32)
    ta = np.ascontiguousarray(tau, np.float32)
    qdd = np.zeros(M.nv, np.float32)
    _check(lib().orc_forward_dynamics_f32(C.c_void_p(M.ptr), qa.ctypes.data_as(_fp),
                                          va.ctypes.data_as(_fp), ta.ctypes.data_as(_fp),
                                          int(with_contacts), qdd.ctypes.data_as(_fp)), "fd32")
    return qdd


def step_dynamics_f32(model, q, v, qr, vr, dt):
    """step_dynamics in float arithmetic (FP32-vs-FP64 diagnosis only)."""
    M = _Model(model)
    f = lambda a: np.ascontiguousarray(a, np.float32)  # noqa: E731
    qa, va, ra, sa = f(q), f(v), f(qr), f(vr)
    qdd = np.zeros(M.nv, np.float32)
    L = lib()
    L.orc_step_dynamics_f32.argtypes = [C.c_void_p, _fp, _fp, _fp, _fp, C.c_float, _fp]
    _check(L.orc_step_dynamics_f32(M.ptr, qa.ctypes.data_as(_fp), va.ctypes.data_as(_fp),
                                   ra.ctypes.data_as(_fp), sa.ctypes.data_as(_fp), dt,
                                   qdd.ctypes.data_as(_fp)), "step_dynamics_f32")
    return qdd


def crba(model, q):
    M = _Model(model)
    qa, qp = _d(q)
    H = np.zeros((M.nv, M.nv))
    _check(lib().orc_crba(C.c_void_p(M.ptr), qp, H.ctypes.data_as(_dp)), "crba")
    return H


def rnea(model, q, v, qdd, with_contacts=True):
    M = _Model(model)
    qa, qp = _d(q); va, vp = _d(v); aa, ap = _d(qdd)
    tau = np.zeros(M.nv)
    _check(lib().orc_rnea(C.c_void_p(M.ptr), qp, vp, ap, int(with_contacts),
                          tau.ctypes.data_as(_dp)), "rnea")
    return tau


def body_poses(model, q):
    M = _Model(model)
    qa, qp = _d(q)
    nb = len(model["parent"])
    R = np.zeros((nb, 3, 3)); p = np.zeros((nb, 3))
    _check(lib().orc_body_poses(C.c_void_p(M.ptr), qp, R.ctypes.data_as(_dp),
                                p.ctypes.data_as(_dp)), "poses")
    return R, p


def euler_step(model, dt, q, v, qr, vr):
    """One rollout physics step tracking the joint reference (qr, vr)."""
    M = _Model(model)
    q = np.array(q, dtype=np.float64); v = np.array(v, dtype=np.float64)
    ra, rp = _d(qr); sa, sp = _d(vr)
    _check(lib().orc_euler_step(M.ptr, dt, q.ctypes.data_as(_dp), v.ctypes.data_as(_dp), rp, sp),
           "euler")
    return q, v


def step_dynamics(model, q, v, qr, vr, dt):
    """Accelerations of one rollout physics step: PD on (qr, vr), contact, and the
    linearly implicit terms of step dt (dt = 0: fully explicit).
    Returns (qdd, tau, g, contact_forces)."""
    M = _Model(model)
    qa, qp = _d(q); va, vp = _d(v); ra, rp = _d(qr); sa, sp = _d(vr)
    qdd = np.zeros(M.nv); tau = np.zeros(M.nu); g = np.zeros(M.nu)
    cf = np.zeros((max(M.nc, 1), 3))
    _check(lib().orc_step_dynamics(M.ptr, qp, vp, rp, sp, dt, qdd.ctypes.data_as(_dp),
                                   tau.ctypes.data_as(_dp), g.ctypes.data_as(_dp),
                                   cf.ctypes.data_as(_dp)), "step_dynamics")
    return qdd, tau, g, cf[:M.nc]


def rk4(model, dt, steps, q, v, tau):
    M = _Model(model)
    q = np.array(q, dtype=np.float64); v = np.array(v, dtype=np.float64)
    ta, tp = _d(tau)
    _check(lib().orc_rk4(M.ptr, dt, steps, q.ctypes.data_as(_dp), v.ctypes.data_as(_dp), tp), "rk4")
    return q, v


def energy(model, q, v):
    M = _Model(model)
    qa, qp = _d(q); va, vp = _d(v)
    E = C.c_double()
    _check(lib().orc_energy(C.c_void_p(M.ptr), qp, vp, C.byref(E)), "energy")
    return E.value


def momentum(model, q, v):
    M = _Model(model)
    qa, qp = _d(q); va, vp = _d(v)
    h = np.zeros(6)
    _check(lib().orc_momentum(C.c_void_p(M.ptr), qp, vp, h.ctypes.data_as(_dp)), "momentum")
    return h


def contacts(model, q, v):
    M = _Model(model)
    qa, qp = _d(q); va, vp = _d(v)
    n = max(M.nc, 1)
    pos = np.zeros((n, 3)); vel = np.zeros((n, 3)); f = np.zeros((n, 3)); mask = C.c_uint32()
    _check(lib().orc_contacts(C.c_void_p(M.ptr), qp, vp, pos.ctypes.data_as(_dp),
                              vel.ctypes.data_as(_dp), f.ctypes.data_as(_dp), C.byref(mask)),
           "contacts")
    return pos[:M.nc], vel[:M.nc], f[:M.nc], mask.value


def rollout(model, params, x0, knots, debug=False):
    M = _Model(model); P = _Params(params, M.nu, M.nc)
    xa, xp = _d(x0); ka, kp = _d(knots)
    S = C.c_double()
    H = params["horizon"]
    if debug:
        traj = np.zeros((H + 1, M.nq + M.nv)); masks = np.zeros(H, np.uint32); stage = np.zeros(H + 1)
        _check(lib().orc_rollout(C.c_void_p(M.ptr), C.c_void_p(P.ptr), xp, kp, C.byref(S),
                                 traj.ctypes.data_as(_dp), masks.ctypes.data_as(_up),
                                 stage.ctypes.data_as(_dp)), "rollout")
        return S.value, traj, masks, stage
    _check(lib().orc_rollout(C.c_void_p(M.ptr), C.c_void_p(P.ptr), xp, kp, C.byref(S), None, None,
                             None), "rollout")
    return S.value


def forced_steps(model, params, x0, knots, traj, f32=False, threads=None):
    """Trajectory-forced steps of the Alg. 1 simulate step: for rollout r (knots
    [n, E], every rollout starting from x0) and each control step h < H, one
    control step from the GIVEN state traj[r, h] (traj [n, H+1, nq+nv]).
    Returns a dict of
      qdd   [n, H, nv]      accelerations of the step's first physics substep
      cost  [n, H+1]        running cost of step h; cost[:, H] = terminal cost at traj[:, H]
      masks [n, H]          contact-activity mask (bit c: f_n > 0 at point c)
      fn    [n, H, nc]      normal force of every contact point
      next  [n, H, nq+nv]   the state the step reaches
    f32=True evaluates in float (rounding reference only)."""
    M = _Model(model); P = _Params(params, M.nu, M.nc)
    H = int(params["horizon"])
    kn = np.ascontiguousarray(knots, dtype=np.float64)
    tr = np.ascontiguousarray(traj, dtype=np.float64)
    n = kn.shape[0]
    nx = M.nq + M.nv
    if kn.shape != (n, 2 * params["n_knots"] * M.nu) or tr.shape != (n, H + 1, nx):
        raise ValueError("knots must be [n, E] and traj [n, H+1, nq+nv]")
    xa, xp = _d(x0)
    out = {"qdd": np.zeros((n, H, M.nv)), "cost": np.zeros((n, H + 1)), "masks": np.zeros((n, H), np.uint32),
           "next": np.zeros((n, H, nx)), "fn": np.zeros((n, H, max(M.nc, 1)))}
    th = threads or os.cpu_count() or 1
    _check(lib().orc_forced_steps(M.ptr, P.ptr, xp, n, kn.ctypes.data_as(_dp), tr.ctypes.data_as(_dp),
                                  out["qdd"].ctypes.data_as(_dp), out["cost"].ctypes.data_as(_dp),
                                  out["masks"].ctypes.data_as(_up), out["next"].ctypes.data_as(_dp),
                                  out["fn"].ctypes.data_as(_dp), int(bool(f32)), th), "forced_steps")
    out["fn"] = out["fn"][:, :, :M.nc]
    return out


def integrate(model, dt, X, A):
    """The rollout's integration step alone: states X [n, nq+nv] advanced by dt
    with accelerations A [n, nv] (joints and base twist: v += dt a; joints
    q += dt v; base p += dt R v_lin, quaternion times exp(dt w / 2))."""
    M = _Model(model)
    Xa = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, M.nq + M.nv)
    Aa = np.ascontiguousarray(A, dtype=np.float64).reshape(-1, M.nv)
    out = np.zeros_like(Xa)
    _check(lib().orc_integrate_batch(M.ptr, float(dt), Xa.shape[0], Xa.ctypes.data_as(_dp), Aa.ctypes.data_as(_dp),
                                     out.ctypes.data_as(_dp)), "integrate")
    return out


OP_KINDS = ("add", "mul", "div", "sqrt", "trans", "cmp", "nt_add", "nt_mul", "nt_div")


def count_ops(model, params, x0, nominal, seed, n=1):
    """Arithmetic of one rollout (sample n drawn around `nominal`, H control steps
    from x0, terminal cost) counted by the oracle's operation-counting scalar:
    {"rollout": {kind: count}, "sampling": {kind: count}} with kinds add (incl.
    subtraction), mul, div, sqrt, trans (sin, cos, exp, log, atan2), cmp
    (comparisons, fabs, floor) and the non-trivial nt_add, nt_mul, nt_div
    (operations not involving an exact 0, or 1 for products and divisors)."""
    M = _Model(model); P = _Params(params, M.nu, M.nc)
    xa, xp = _d(x0); na, npt = _d(nominal)
    out = np.zeros(18)
    _check(lib().orc_count_ops(M.ptr, P.ptr, xp, npt, seed, int(n), out.ctypes.data_as(_dp)), "count_ops")
    return {"rollout": dict(zip(OP_KINDS, out[:9])), "sampling": dict(zip(OP_KINDS, out[9:]))}


def count_selftest():
    """Counts of y = A x (3x3) with the counting scalar: (general A, identity A)."""
    out = np.zeros(18)
    lib().orc_count_selftest(out.ctypes.data_as(_dp))
    return dict(zip(OP_KINDS, out[:9])), dict(zip(OP_KINDS, out[9:]))


def rollout_f32(model, params, x0, knots):
    M = _Model(model); P = _Params(params, M.nu, M.nc)
    xa, xp = _d(x0); ka, kp = _d(knots)
    S = C.c_double()
    masks = np.zeros(params["horizon"], np.uint32)
    _check(lib().orc_rollout_f32(C.c_void_p(M.ptr), C.c_void_p(P.ptr), xp, kp, C.byref(S),
                                 masks.ctypes.data_as(_up)), "rollout_f32")
    return S.value, masks


def rollouts(model, params, x0, nominal, seed, tick, iota, n0, count, threads=None, samples=False):
    """Costs of samples n0..n0+count-1 of iteration iota (and their knots)."""
    M = _Model(model); P = _Params(params, M.nu, M.nc)
    xa, xp = _d(x0); na, npt = _d(nominal)
    S = np.zeros(count)
    E = 2 * params["n_knots"] * M.nu
    smp = np.zeros((count, E)) if samples else None
    th = threads or os.cpu_count() or 1
    _check(lib().orc_rollouts(M.ptr, P.ptr, xp, npt, seed, tick, iota, n0, count,
                              S.ctypes.data_as(_dp),
                              smp.ctypes.data_as(_dp) if samples else None, th), "rollouts")
    return (S, smp) if samples else S


def orientation_angle(quat):
    qa, qp = _d(quat)
    f = lib().orc_orientation_angle
    f.restype = C.c_double
    f.argtypes = [_dp]
    return f(qp)


def weights(S, lam, mode=0):
    Sa, Sp = _d(S)
    w = np.zeros(len(Sa)); nstar = C.c_int32()
    nf = lib().orc_weights(len(Sa), Sp, lam, mode, w.ctypes.data_as(_dp), C.byref(nstar))
    if nf < 0:
        raise ValueError("bad weights arguments")
    return w, nstar.value, nf


def weighted_average(w, samples):
    wa, wp = _d(w); sa, sp = _d(samples)
    n, E = sa.shape
    out = np.zeros(E)
    lib().orc_weighted_average(n, E, wp, sp, out.ctypes.data_as(_dp))
    return out


def dense_route_update(w, samples, nk, nu, H, dt):
    wa, wp = _d(w); sa, sp = _d(samples)
    out = np.zeros(2 * nk * nu)
    lib().orc_dense_route_update(len(wa), nk, nu, H, dt, wp, sp, out.ctypes.data_as(_dp))
    return out


def step(model, params, x0, knots_in, seed, tick, threads=None, f32=False):
    """Full MPC step; returns a dict with knots, best_knots, S_best, best_iter, costs, ...
    f32=True runs sampling and rollouts in float (FP32 divergence diagnosis only)."""
    M = _Model(model); P = _Params(params, M.nu, M.nc)
    xa, xp = _d(x0); ka, kp = _d(knots_in)
    E = 2 * params["n_knots"] * M.nu
    out = np.zeros(E); best = np.zeros(E); sb = C.c_double(); bi = C.c_int32()
    costs = np.zeros((params["n_iters"], params["n_samples"]))
    nnf = C.c_int32(); anf = C.c_int32()
    th = threads or os.cpu_count() or 1
    fn = lib().orc_step_f32 if f32 else lib().orc_step
    _check(fn(M.ptr, P.ptr, xp, kp, seed, tick, out.ctypes.data_as(_dp),
                          best.ctypes.data_as(_dp), C.byref(sb), C.byref(bi),
                          costs.ctypes.data_as(_dp), C.byref(nnf), C.byref(anf), th), "step")
    return {"knots": out, "best_knots": best, "S_best": sb.value, "best_iter": bi.value,
            "costs": costs, "n_nonfinite": nnf.value, "all_nonfinite_iters": anf.value}
