"""Trajectory-forced parity (the protocol of tests/test_gpu_trace.py) for the
spline variants of the ablation (natural cubic and quadratic position splines,
zero velocity targets) and for every task preset of Tab. cost-weights
(orientation targets, the jumping task's absolute terminal height), at the
configurations' own horizons: every rollout of every iteration checked step by
step against the FP64 oracle, and the iterations run one at a time equal to
mppi_step bit for bit."""
import numpy as np
import pytest

from paper_2511_19204_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2511_19204_amd import mppi
    from forced_parity import check_forced, fused_step, traced_iterations


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    mppi.lib()


def _run_and_check(m, p, s, label, tick=2):
    model = mppi.Model(m)
    c = mppi.Controller(model, p, s)
    kn = synth.nominal_knots(m, p["n_knots"])
    x0 = np.asarray(m["x0"], np.float64)
    its = traced_iterations(c, m, p, tick, x0, kn, [np.arange(p["n_samples"])] * p["n_iters"])
    fused = fused_step(c, m, p, tick, x0, kn)
    for it, d in enumerate(its):
        assert np.array_equal(d["costs"], fused["costs"][it]), (label, it)
        check_forced(m, p, x0, d["samples"][d["idx"]].astype(np.float64), d["trace"], d["costs"][d["idx"]],
                     f"{label} it{it}")
    assert np.array_equal(its[-1]["next"], fused["knots"]), label


@pytest.mark.parametrize("mode", [1, 2])
def test_spline_variant_forced_parity(mode):
    """Quadruped, K = 64, H = 100, 3 iterations, position-only spline `mode`."""
    m, p, s = synth.config("quadruped")
    p = dict(p, spline_mode=mode)
    _run_and_check(m, p, s, f"spline mode {mode}")


@pytest.mark.parametrize("name", synth.TASKS)
def test_task_preset_forced_parity(name):
    """Each task preset on its robot at the configuration's horizon (quadruped
    H = 100, humanoid H = 150), K = 64, 3 iterations."""
    base = "humanoid" if name == "bipedal" else "quadruped"
    m, p, s = synth.config(base, n_samples=64)
    p = synth.task_params(m, p, name)
    _run_and_check(m, p, s, name)
