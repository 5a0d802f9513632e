"""ctypes binding of libmppi.so (the C ABI declared in include/mppi.h).

Argument marshalling only: every step of the controller runs in the HIP
kernels of the library.  Device buffers are torch CUDA (HIP) tensors; streams
are torch streams.  The library is loaded on first use and a missing or
unloadable library raises -- there is no CPU fallback.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MPPI_LIB: another build of the same sources (the host-sanitizer build)
LIB_PATH = os.environ.get("MPPI_LIB") or os.path.join(_HERE, "libmppi.so")
_lib = None

MPPI_OK = 0


class MppiError(RuntimeError):
    pass


class ModelDesc(C.Structure):
    _fields_ = [
        ("n_bodies", C.c_int32), ("floating_base", C.c_int32), ("parent", C.POINTER(C.c_int32)),
        ("axis", C.POINTER(C.c_float)), ("R_tree", C.POINTER(C.c_float)),
        ("p_tree", C.POINTER(C.c_float)), ("mass", C.POINTER(C.c_float)),
        ("com", C.POINTER(C.c_float)), ("inertia", C.POINTER(C.c_float)),
        ("q_min", C.POINTER(C.c_float)), ("q_max", C.POINTER(C.c_float)),
        ("tau_max", C.POINTER(C.c_float)), ("kp", C.POINTER(C.c_float)),
        ("kd", C.POINTER(C.c_float)), ("n_contacts", C.c_int32),
        ("contact_body", C.POINTER(C.c_int32)), ("contact_pos", C.POINTER(C.c_float)),
        ("k_contact", C.c_float), ("d_contact", C.c_float), ("mu", C.c_float),
        ("eps_fric", C.c_float), ("gravity", C.c_float), ("ee_body", C.c_int32),
        ("ee_pos", C.c_float * 3), ("n_substeps", C.c_int32),
        ("armature", C.POINTER(C.c_float)),
    ]


class Params(C.Structure):
    _fields_ = [
        ("n_samples", C.c_int32), ("horizon", C.c_int32), ("n_knots", C.c_int32),
        ("n_iters", C.c_int32), ("dt", C.c_float), ("lam", C.c_float),
        ("weight_mode", C.c_int32), ("noise_mode", C.c_int32), ("scale_q", C.c_float),
        ("beta1", C.c_float), ("beta2", C.c_float), ("sigma_lo", C.c_float),
        ("sigma_hi", C.c_float), ("cost_kind", C.c_int32), ("w_h", C.c_float),
        ("w_or", C.c_float), ("w_q", C.c_float), ("w_cv", C.c_float), ("w_cf", C.c_float),
        ("w_eff", C.c_float), ("w_H", C.c_float), ("w_ee", C.c_float), ("w_tau", C.c_float),
        ("z_des", C.c_float), ("v_des", C.c_float * 3), ("f0z", C.POINTER(C.c_float)),
        ("q0_cost", C.POINTER(C.c_float)), ("spline_mode", C.c_int32),
        ("q_des", C.c_float * 4), ("terminal_z_abs", C.c_int32), ("z_terminal", C.c_float),
    ]


class Targets(C.Structure):
    _fields_ = [("z_des", C.c_float), ("v_des", C.c_float * 3), ("q_des", C.c_float * 4),
                ("terminal_z_abs", C.c_int32), ("z_terminal", C.c_float)]


class StepInfo(C.Structure):
    _fields_ = [("S_best", C.c_float), ("best_iter", C.c_int32), ("n_nonfinite", C.c_int32),
                ("all_nonfinite_iters", C.c_int32), ("best_sample", C.c_int32)]


INFO_INTS = 5  # mppi_step_info as int32 words


EXPORTS = [
    "mppi_model_create", "mppi_model_destroy", "mppi_create", "mppi_destroy", "mppi_set_tick",
    "mppi_get_tick", "mppi_set_schedule", "mppi_get_schedule", "mppi_set_lanes_per_rollout",
    "mppi_get_lanes_per_rollout", "mppi_set_targets", "mppi_step", "mppi_predict", "mppi_shift_knots", "mppi_tick",
    "mppi_step_batch", "mppi_debug_philox", "mppi_debug_samples", "mppi_debug_dynamics",
    "mppi_debug_rollouts", "mppi_debug_trace", "mppi_debug_update", "mppi_profile_enable", "mppi_profile_read",
    "mppi_set_batch_options", "mppi_graph_create", "mppi_graph_launch", "mppi_graph_destroy",
    "mppi_autotune", "mppi_server_create", "mppi_server_submit", "mppi_server_submit_tick", "mppi_server_poll",
    "mppi_server_drain", "mppi_server_stats", "mppi_server_destroy", "mppi_update_noalloc",
    "mppi_last_error", "mppi_version",
]


class BatchOpts(C.Structure):
    _fields_ = [("persistent", C.c_int32)]


class ServerCfg(C.Structure):
    _fields_ = [("max_pending", C.c_int32), ("n_streams", C.c_int32), ("max_batch", C.c_int32),
                ("mode", C.c_int32), ("persistent", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MppiError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        vp, i32, u32, u64 = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64
        L.mppi_model_create.argtypes = [C.POINTER(ModelDesc), C.POINTER(vp)]
        L.mppi_model_destroy.argtypes = [vp]
        L.mppi_create.argtypes = [vp, C.POINTER(Params), u64, C.POINTER(vp)]
        L.mppi_destroy.argtypes = [vp]
        L.mppi_set_tick.argtypes = [vp, u32]
        L.mppi_get_tick.argtypes = [vp, C.POINTER(u32)]
        L.mppi_set_schedule.argtypes = [vp, i32]
        L.mppi_get_schedule.argtypes = [vp, C.POINTER(i32)]
        L.mppi_set_lanes_per_rollout.argtypes = [vp, i32]
        L.mppi_get_lanes_per_rollout.argtypes = [vp, C.POINTER(i32)]
        L.mppi_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.mppi_set_targets.argtypes = [vp, C.POINTER(Targets), vp]
        L.mppi_predict.argtypes = [vp, vp, vp, i32, vp, vp]
        L.mppi_shift_knots.argtypes = [vp, vp, i32, vp, vp]
        L.mppi_tick.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp]
        L.mppi_step_batch.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp]
        L.mppi_debug_philox.argtypes = [vp, vp, vp, i32, vp]
        L.mppi_debug_samples.argtypes = [vp, vp, i32, u32, vp, vp]
        L.mppi_debug_dynamics.argtypes = [vp, i32, vp, vp, vp, vp, C.c_float, vp, vp]
        L.mppi_debug_rollouts.argtypes = [vp, vp, vp, vp, vp, vp]
        L.mppi_debug_trace.argtypes = [vp, vp, vp, i32, u32, vp, vp, vp, vp, vp, vp]
        L.mppi_debug_update.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.mppi_profile_enable.argtypes = [vp, i32]
        L.mppi_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(i32),
                                        C.POINTER(C.c_double), C.POINTER(i32)]
        L.mppi_set_batch_options.argtypes = [C.POINTER(BatchOpts)]
        L.mppi_graph_create.argtypes = [i32, vp, vp, vp, vp, vp, vp, C.POINTER(vp)]
        L.mppi_graph_launch.argtypes = [vp, vp]
        L.mppi_graph_destroy.argtypes = [vp]
        L.mppi_autotune.argtypes = [vp, vp, vp, i32, vp, C.POINTER(i32)]
        L.mppi_server_create.argtypes = [C.POINTER(ServerCfg), C.POINTER(vp)]
        L.mppi_server_submit.argtypes = [vp, vp, vp, vp, vp, C.POINTER(u64)]
        L.mppi_server_submit_tick.argtypes = [vp, vp, vp, i32, vp, vp, vp, C.POINTER(u64)]
        L.mppi_server_poll.argtypes = [vp, u64, C.POINTER(i32), C.POINTER(C.c_double)]
        L.mppi_server_drain.argtypes = [vp, C.c_double]
        L.mppi_server_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.mppi_server_destroy.argtypes = [vp]
        L.mppi_update_noalloc.argtypes = [i32, i32, C.c_float, i32, vp, vp, vp, vp, vp, vp]
        L.mppi_last_error.restype = C.c_char_p
        L.mppi_version.restype = C.c_char_p
        for name in EXPORTS[:-2]:
            getattr(L, name).restype = C.c_int32
        L.mppi_last_error.restype = C.c_char_p
        L.mppi_version.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc, what):
    if rc != MPPI_OK:
        raise MppiError(f"{what} failed ({rc}): {lib().mppi_last_error().decode()}")


def _addr(t):
    """Address of a torch tensor's data after the checks every buffer of the C ABI
    needs: contiguous, of a 32-bit element type (float32 values, int32 words)."""
    import torch
    if t.dtype not in (torch.float32, torch.int32):
        raise TypeError(f"tensors passed to the library must be float32 or int32, not {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensors passed to the library must be contiguous")
    return t.data_ptr()


def _ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    return C.c_void_p(_addr(t))


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _farr(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1))
    return a, a.ctypes.data_as(C.POINTER(C.c_float))


def _iarr(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1))
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


class Model:
    """Device-resident kinematic tree built from a synth model dict."""

    def __init__(self, m):
        keep = []
        d = ModelDesc()
        nb = len(m["parent"])
        d.n_bodies = nb
        d.floating_base = 1 if m["floating_base"] else 0
        a, d.parent = _iarr(m["parent"]); keep.append(a)
        for name in ("axis", "R_tree", "p_tree", "mass", "com", "inertia", "q_min", "q_max",
                     "tau_max", "kp", "kd"):
            a, p = _farr(m[name]); keep.append(a); setattr(d, name, p)
        nc = len(m["contact_body"])
        d.n_contacts = nc
        a, d.contact_body = _iarr(m["contact_body"] if nc else [0]); keep.append(a)
        a, d.contact_pos = _farr(m["contact_pos"] if nc else [0, 0, 0]); keep.append(a)
        d.k_contact, d.d_contact = m["k_contact"], m["d_contact"]
        d.mu, d.eps_fric, d.gravity = m["mu"], m["eps_fric"], m["gravity"]
        d.ee_body = int(m["ee_body"])
        for k in range(3):
            d.ee_pos[k] = float(m["ee_pos"][k])
        d.n_substeps = int(m.get("n_substeps", 1))
        a, d.armature = _farr(m.get("armature", np.zeros(m["n_u"]))); keep.append(a)
        h = C.c_void_p()
        _check(lib().mppi_model_create(C.byref(d), C.byref(h)), "mppi_model_create")
        self.h = h
        self.nb = nb
        self.nu = m["n_u"]
        self.nq = m["n_q"]
        self.nv = m["n_v"]
        self.nc = nc

    def close(self):
        if self.h:
            _check(lib().mppi_model_destroy(self.h), "mppi_model_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dynamics(self, q, v, qref, vref, dt, out, stream=None):
        """Accelerations of one physics step for a batch of states (device tensors)."""
        n = q.shape[0]
        _check(lib().mppi_debug_dynamics(self.h, n, _ptr(q), _ptr(v), _ptr(qref), _ptr(vref),
                                         float(dt), _ptr(out), _stream(stream)),
               "mppi_debug_dynamics")


def _check_param_lengths(p, nc, nu):
    """The library reads f0z for every contact point and q0_cost for every joint
    from the caller's arrays; shorter arrays would be read past their end."""
    if len(p["f0z"]) != nc:
        raise MppiError(f"f0z has {len(p['f0z'])} entries for {nc} contact points")
    if len(p["q0_cost"]) != nu:
        raise MppiError(f"q0_cost has {len(p['q0_cost'])} entries for {nu} joints")


def make_params(p):
    s = Params()
    for name in ("n_samples", "horizon", "n_knots", "n_iters", "weight_mode", "noise_mode",
                 "cost_kind"):
        setattr(s, name, int(p[name]))
    for name in ("dt", "scale_q", "beta1", "beta2", "sigma_lo", "sigma_hi", "w_h", "w_or",
                 "w_q", "w_cv", "w_cf", "w_eff", "w_H", "w_ee", "w_tau", "z_des"):
        setattr(s, name, float(p[name]))
    s.lam = float(p["lambda"])
    for k in range(3):
        s.v_des[k] = float(p["v_des"][k])
    f0, s.f0z = _farr(p["f0z"] if len(p["f0z"]) else [0.0])
    q0, s.q0_cost = _farr(p["q0_cost"])
    s.spline_mode = int(p.get("spline_mode", 0))
    qd = p.get("q_des", (0.0, 0.0, 0.0, 0.0))
    for k in range(4):
        s.q_des[k] = float(qd[k])
    s.terminal_z_abs = int(p.get("terminal_z_abs", 0))
    s.z_terminal = float(p.get("z_terminal", 0.0))
    return s, (f0, q0)


SCHEDULES = {"body": 0, "chain": 1, "team": 2}


class Controller:
    """One MPC instance (mppi_ctx).  schedule: "body" (one lane per body, with
    `lanes` lanes per rollout) or "chain" (one lane per kinematic chain); None
    keeps the library's default (the body schedule)."""

    def __init__(self, model, params, seed, lanes=0, schedule=None):
        self.model = model
        self.params = dict(params)
        _check_param_lengths(params, model.nc, model.nu)
        s, self._keep = make_params(params)
        h = C.c_void_p()
        _check(lib().mppi_create(model.h, C.byref(s), C.c_uint64(seed), C.byref(h)), "mppi_create")
        self.h = h
        self.N, self.H, self.K, self.I = (params["n_samples"], params["horizon"],
                                          params["n_knots"], params["n_iters"])
        self.E = 2 * self.K * model.nu
        if schedule is not None:
            self.set_schedule(schedule)
        if lanes:
            self.set_lanes(lanes)

    def close(self):
        if self.h:
            _check(lib().mppi_destroy(self.h), "mppi_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def tick(self):
        t = C.c_uint32()
        _check(lib().mppi_get_tick(self.h, C.byref(t)), "mppi_get_tick")
        return t.value

    @tick.setter
    def tick(self, value):
        _check(lib().mppi_set_tick(self.h, C.c_uint32(value)), "mppi_set_tick")

    @property
    def lanes(self):
        g = C.c_int32()
        _check(lib().mppi_get_lanes_per_rollout(self.h, C.byref(g)), "mppi_get_lanes_per_rollout")
        return g.value

    def set_targets(self, z_des=None, v_des=None, q_des=None, terminal_z_abs=None, z_terminal=None, stream=None):
        """mppi_set_targets: change the task targets (fields left None keep their
        values), ordered on `stream` (torch's current stream by default)."""
        for k, v in (("z_des", z_des), ("v_des", v_des), ("q_des", q_des), ("terminal_z_abs", terminal_z_abs),
                     ("z_terminal", z_terminal)):
            if v is not None:
                self.params[k] = list(v) if k in ("v_des", "q_des") else v
        t = Targets()
        t.z_des = float(self.params["z_des"])
        for k in range(3):
            t.v_des[k] = float(self.params["v_des"][k])
        qd = self.params.get("q_des", (0.0, 0.0, 0.0, 0.0))
        for k in range(4):
            t.q_des[k] = float(qd[k])
        t.terminal_z_abs = int(self.params.get("terminal_z_abs", 0))
        t.z_terminal = float(self.params.get("z_terminal", 0.0))
        _check(lib().mppi_set_targets(self.h, C.byref(t), _stream(stream)), "mppi_set_targets")

    def set_lanes(self, lanes):
        """Body schedule with `lanes` lanes per rollout."""
        _check(lib().mppi_set_lanes_per_rollout(self.h, int(lanes)), "mppi_set_lanes_per_rollout")

    @property
    def schedule(self):
        s = C.c_int32()
        _check(lib().mppi_get_schedule(self.h, C.byref(s)), "mppi_get_schedule")
        return {v: k for k, v in SCHEDULES.items()}[s.value]

    def set_schedule(self, schedule):
        _check(lib().mppi_set_schedule(self.h, SCHEDULES[schedule]), "mppi_set_schedule")

    def step(self, state, knots_in, knots_out, best_knots=None, info=None, costs=None, stream=None):
        _check(lib().mppi_step(self.h, _ptr(state), _ptr(knots_in), _ptr(knots_out),
                               _ptr(best_knots), _ptr(info), _ptr(costs), _stream(stream)),
               "mppi_step")

    def predict(self, state_in, knots, n_steps, state_out, stream=None):
        """State reached after n_steps control steps along the knots' trajectory."""
        _check(lib().mppi_predict(self.h, _ptr(state_in), _ptr(knots), int(n_steps), _ptr(state_out),
                                  _stream(stream)), "mppi_predict")

    def shift_knots(self, knots_in, n_steps, knots_out, stream=None):
        """Warm-start shift of a trajectory's knots by n_steps control steps."""
        _check(lib().mppi_shift_knots(self.h, _ptr(knots_in), int(n_steps), _ptr(knots_out), _stream(stream)),
               "mppi_shift_knots")

    def run_tick(self, state_meas, n_delay, best, knots_out=None, info=None, state_pred=None, stream=None):
        """mppi_tick: one control step (predict, shift tau_best, iterate); `best` is updated in place."""
        _check(lib().mppi_tick(self.h, _ptr(state_meas), int(n_delay), _ptr(best), _ptr(knots_out), _ptr(info),
                               _ptr(state_pred), _stream(stream)), "mppi_tick")

    def profile(self, on=True):
        """Record HIP events around this instance's kernel launches."""
        _check(lib().mppi_profile_enable(self.h, 1 if on else 0), "mppi_profile_enable")

    def profile_read(self):
        """(rollout ms, rollout launches, update ms, update launches) since the last read."""
        tr, tu = C.c_double(), C.c_double()
        nr, nu = C.c_int32(), C.c_int32()
        _check(lib().mppi_profile_read(self.h, C.byref(tr), C.byref(nr), C.byref(tu), C.byref(nu)),
               "mppi_profile_read")
        return tr.value, nr.value, tu.value, nu.value

    def samples(self, knots_in, iteration, tick, out, stream=None):
        _check(lib().mppi_debug_samples(self.h, _ptr(knots_in), int(iteration), C.c_uint32(tick),
                                        _ptr(out), _stream(stream)), "mppi_debug_samples")

    def rollouts(self, state, samples, costs, masks=None, stream=None):
        _check(lib().mppi_debug_rollouts(self.h, _ptr(state), _ptr(samples), _ptr(costs),
                                         _ptr(masks), _stream(stream)), "mppi_debug_rollouts")

    def trace(self, state, knots_in, iteration, tick, trace_map, trace, samples, costs, masks, stream=None):
        """mppi_debug_trace: iteration `iteration` of a step at `tick`, with per-step
        records [slots][H+1][nq + 2 nv + 2] of the samples whose trace_map entry >= 0."""
        _check(lib().mppi_debug_trace(self.h, _ptr(state), _ptr(knots_in), int(iteration), C.c_uint32(tick),
                                      _ptr(trace_map), _ptr(trace), _ptr(samples), _ptr(costs), _ptr(masks),
                                      _stream(stream)), "mppi_debug_trace")

    def update(self, costs, samples, knots_in, knots_out, weights=None, stream=None):
        _check(lib().mppi_debug_update(self.h, _ptr(costs), _ptr(samples), _ptr(knots_in),
                                       _ptr(knots_out), _ptr(weights), _stream(stream)),
               "mppi_debug_update")


def update_noalloc(n_samples, n_elems, lam, weight_mode, costs, samples, knots_in, knots_out, weights=None,
                   stream=None):
    """mppi_update_noalloc: weights and weighted knot update with the library's
    fixed scratch (no device allocation)."""
    _check(lib().mppi_update_noalloc(int(n_samples), int(n_elems), float(lam), int(weight_mode), _ptr(costs),
                                     _ptr(samples), _ptr(knots_in), _ptr(knots_out), _ptr(weights),
                                     _stream(stream)), "mppi_update_noalloc")


def step_batch(ctrls, states, knots_in, knots_out, best_knots=None, infos=None, stream=None):
    """Fused step of several controllers (lists of equal length)."""
    n = len(ctrls)
    arr = lambda xs: (C.c_void_p * n)(*[x.h if isinstance(x, Controller) else (_addr(x) if x is not None else None) for x in xs])  # noqa: E731
    hs = arr(ctrls)
    st = arr(states)
    ki = arr(knots_in)
    ko = arr(knots_out)
    bk = arr(best_knots) if best_knots is not None else None
    inf = arr(infos) if infos is not None else None
    _check(lib().mppi_step_batch(n, hs, st, ki, ko, bk, inf, _stream(stream)), "mppi_step_batch")


def _ptr_array(xs):
    n = len(xs)
    return (C.c_void_p * n)(*[(x.h if isinstance(x, Controller) else _addr(x)) if x is not None else None
                              for x in xs])


def set_batch_options(persistent):
    o = BatchOpts(1 if persistent else 0)
    _check(lib().mppi_set_batch_options(C.byref(o)), "mppi_set_batch_options")


class Graph:
    """A fixed batch captured into a hipGraph; launch() = one step of every instance."""

    def __init__(self, ctrls, states, knots_in, knots_out, best_knots=None, infos=None):
        self._keep = (ctrls, states, knots_in, knots_out, best_knots, infos)
        h = C.c_void_p()
        _check(lib().mppi_graph_create(len(ctrls), _ptr_array(ctrls), _ptr_array(states),
                                       _ptr_array(knots_in), _ptr_array(knots_out),
                                       _ptr_array(best_knots) if best_knots is not None else None,
                                       _ptr_array(infos) if infos is not None else None, C.byref(h)),
               "mppi_graph_create")
        self.h = h

    def launch(self, stream=None):
        _check(lib().mppi_graph_launch(self.h, _stream(stream)), "mppi_graph_launch")

    def close(self):
        if self.h:
            _check(lib().mppi_graph_destroy(self.h), "mppi_graph_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(ctrl, state, knots, reps=3, stream=None):
    g = C.c_int32()
    _check(lib().mppi_autotune(ctrl.h, _ptr(state), _ptr(knots), int(reps), _stream(stream), C.byref(g)),
           "mppi_autotune")
    return g.value


class Server:
    """Continuous-batching server of MPC ticks: mode "batched" (a batch runs all
    iterations of the ticks it took), "plain" (per-instance launches) or
    "iteration" (every round runs one iteration of each admitted tick; ticks join
    at round boundaries; with several streams each robot type has its own).
    Each stream should have a hardware queue of its own: GPU_MAX_HW_QUEUES (four
    by default) must be set before the process first touches the GPU to at least
    n_streams plus the caller's busy streams."""

    MODES = {"batched": 0, "plain": 1, "iteration": 2}

    def __init__(self, n_streams=3, max_batch=256, max_pending=100000, mode="iteration", persistent=False):
        if mode not in self.MODES:
            raise MppiError(f"unknown server mode {mode!r}; one of {sorted(self.MODES)}")
        cfg = ServerCfg(int(max_pending), int(n_streams), int(max_batch), self.MODES[mode],
                        1 if persistent else 0)
        h = C.c_void_p()
        _check(lib().mppi_server_create(C.byref(cfg), C.byref(h)), "mppi_server_create")
        self.h = h

    def submit(self, ctrl, state, knots_in, knots_out):
        t = C.c_uint64()
        _check(lib().mppi_server_submit(self.h, ctrl.h, _ptr(state), _ptr(knots_in), _ptr(knots_out),
                                        C.byref(t)), "mppi_server_submit")
        return t.value

    def submit_tick(self, ctrl, state, n_delay, best, knots_out=None, info=None):
        """A tick as Controller.run_tick (prediction by n_delay control steps along
        best, warm-start shift, iterations; best updated in place), served."""
        t = C.c_uint64()
        _check(lib().mppi_server_submit_tick(self.h, ctrl.h, _ptr(state), int(n_delay), _ptr(best),
                                             _ptr(knots_out) if knots_out is not None else None,
                                             _ptr(info) if info is not None else None, C.byref(t)),
               "mppi_server_submit_tick")
        return t.value

    def poll(self, ticket):
        """None while running, else the submit-to-completion latency in seconds."""
        done = C.c_int32()
        lat = C.c_double()
        _check(lib().mppi_server_poll(self.h, C.c_uint64(ticket), C.byref(done), C.byref(lat)),
               "mppi_server_poll")
        return lat.value if done.value else None

    def drain(self, timeout_s=60.0):
        _check(lib().mppi_server_drain(self.h, float(timeout_s)), "mppi_server_drain")

    def stats(self):
        b, r = C.c_int64(), C.c_int64()
        _check(lib().mppi_server_stats(self.h, C.byref(b), C.byref(r)), "mppi_server_stats")
        return b.value, r.value

    def close(self):
        if self.h:
            _check(lib().mppi_server_destroy(self.h), "mppi_server_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def philox(ctr, key, out, stream=None):
    n = ctr.shape[0]
    _check(lib().mppi_debug_philox(_ptr(ctr), _ptr(key), _ptr(out), n, _stream(stream)),
           "mppi_debug_philox")


def version():
    return lib().mppi_version().decode()
