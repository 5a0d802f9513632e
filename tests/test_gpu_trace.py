"""Trajectory-forced, element-wise parity of the simulate step of Alg. 1 at the
configurations' own horizons, through the C ABI.

A full rollout of a contact configuration is chaotic in float: a rounding
difference decides a contact event or a stick/slip transition and the two
rollouts part ways (the oracle's own float build does the same).  So the check
is made step by step along the GPU's own trajectory.  mppi_debug_trace runs an
iteration of mppi_step with the step's own kernel and launch shape and records,
for chosen rollouts, the state at the start of every control step, the
accelerations, the running cost and the contact mask.  For every recorded step
h the FP64 oracle starts from the GPU's float state x_h and computes one control
step.  The bars, per step:
  accelerations  |a_gpu - a|_inf <= 1e-5 max(|a|_inf, 1), unless the step is
                 ill-conditioned in float: then within 2x of what plain float
                 evaluations of the same step reach (the oracle in float, at the
                 inputs and at eight copies of them perturbed at float rounding,
                 2^-24 relative: the state, the knots and the model constants
                 that the device stores in derived float forms; worst of them),
                 or within 10x of the step's rounding sensitivity (how far the
                 exact accelerations move under those perturbations).  Stiff
                 contact makes many trajectory states like that; the counts are
                 printed
  integration    x_{h+1} from x_h and the GPU's own accelerations within
                 1e-5 max(|x|_inf, 1)
  contact masks  may differ only on points whose normal force is within
                 rounding of zero (|f_n| <= 0.05 N); the soft-contact model is
                 discontinuous there (the implicit damping switches on at
                 f_n > 0), so such steps skip the acceleration and cost bars
                 and are counted
  torque clip    a step beyond the acceleration bar with a joint whose
                 unclipped PD torque lies within its float rounding of the
                 actuator limit passes if its accelerations match the FP64 step
                 on the other branch of the clip within 1e-5 (the implicit PD
                 gain exists only below the limit, so the branches differ by a
                 finite step); counted
  running cost   1e-3 relative, unless the cost is ill-conditioned the same
                 way (a term like |f - f0| cancels at a settled stance): then
                 within 10x of its rounding sensitivity
  terminal cost  1e-3 relative at the GPU's final state
  rollout cost   the GPU's cost within 1e-3 of the oracle's costs summed along
                 the GPU's trajectory (rollouts without a mask flip)
The iterations of a step are run one at a time (trace, then the update kernel on
the GPU's own costs and samples), which must give mppi_step's costs, nominal,
best knots and step info bit for bit; the update of each iteration is checked
against the oracle's weights and weighted average at 1e-4, the sampled knots
against the oracle's sampler, and the best iteration against the oracle's rule.
"""
import numpy as np
import pytest

from paper_2511_19204_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2511_19204_amd import mppi
    from forced_parity import check_forced, check_iterations, fused_step, traced_iterations


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    mppi.lib()


def _run(name, select, n_samples=None, tick=3, seed=0):
    m, p, s = synth.config(name, n_samples=n_samples, seed=seed)
    model = mppi.Model(m)
    c = mppi.Controller(model, p, s)
    kn = synth.nominal_knots(m, p["n_knots"])
    x0 = np.asarray(m["x0"], np.float64)
    its = traced_iterations(c, m, p, tick, x0, kn, [select(p)] * p["n_iters"])
    fused = fused_step(c, m, p, tick, x0, kn)
    return m, p, s, c, kn, x0, its, fused


@pytest.mark.parametrize("name", ["chain", "quadruped", "humanoid"])
def test_step_iterations_forced_parity(name):
    """chain: K=32, H=50, 10 iterations; quadruped: K=64, H=100, 3 iterations;
    humanoid: K=256, H=150, 3 iterations.  Every rollout of every iteration is
    recorded and checked step by step; the iterations and the update follow the
    oracle and equal the fused step."""
    m, p, s, c, kn, x0, its, fused = _run(name, lambda p: np.arange(p["n_samples"]))
    tot = {"acc_esc_f32": 0, "acc_esc_sens": 0, "steps": 0, "mask_flips": 0}
    for it, d in enumerate(its):
        st = check_forced(m, p, x0, d["samples"][d["idx"]].astype(np.float64), d["trace"], d["costs"][d["idx"]],
                          f"{name} it{it}")
        for k in tot:
            tot[k] += st[k]
    check_iterations(c, m, p, s, 3, x0, kn, its, fused, name)
    print(f"{name} total: {tot}")
    assert tot["mask_flips"] <= 1e-3 * tot["steps"]
    assert fused["n_nonfinite"] == 0


def _tp_select(p):
    N = p["n_samples"]
    return np.unique(np.r_[np.arange(0, N, 16), np.arange(1, 4), np.arange(N - 20, N)])


def test_full_size_forced_parity():
    """Quadruped at throughput scale, K = 4096, H = 200, one iteration, in the
    launch the bench times: 275 rollouts spread over the grid, the last
    wavefronts included, checked step by step; every cost of the traced launch
    equals mppi_step's."""
    m, p, s, c, kn, x0, its, fused = _run("quadruped_tp", _tp_select, tick=1)
    d = its[0]
    st = check_forced(m, p, x0, d["samples"][d["idx"]].astype(np.float64), d["trace"], d["costs"][d["idx"]],
                      "quadruped_tp K=4096")
    assert st["mask_flips"] <= 1e-3 * st["steps"]
    check_iterations(c, m, p, s, 1, x0, kn, its, fused, "quadruped_tp", n_sample_check=48)


def test_trace_records_match_their_rollout():
    """The records of a traced rollout add up to its cost (running costs plus the
    terminal cost, float sums in another order), and the untraced slots of the
    map leave the record buffer untouched."""
    m, p, s, c, kn, x0, its, fused = _run("quadruped", lambda p: np.array([0, 5, 63]))
    d = its[0]
    nx, nv, H = m["n_q"] + m["n_v"], m["n_v"], p["horizon"]
    C = d["trace"][:, :, nx + nv]
    S = d["costs"][d["idx"]]
    assert np.all(np.abs(C.sum(axis=1) - S) <= 1e-5 * np.abs(S))
    assert np.array_equal(d["trace"][:, H, nx:nx + nv], np.zeros((3, nv)))
    MK = d["trace"][:, :H, nx + nv + 1].view(np.uint32)
    assert np.array_equal(MK, d["masks"][d["idx"]])
