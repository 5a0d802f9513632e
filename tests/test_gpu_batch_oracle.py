"""The multi-instance forms -- one fused batched step, the same batch with the
persistent rollout launch, and the batch captured in a hipGraph -- against the
oracle, not only against plain steps.

A batch holds a chain (K = 32, H = 50, 10 iterations), a quadruped (K = 64,
H = 100, 3 iterations) and a humanoid (K = 64, H = 150, 3 iterations) instance.
Each instance's outputs (nominal, best knots, step info) must equal its own
iterations run one at a time with the trace entry point, bit for bit; those
are checked against the FP64 oracle with the trajectory-forced protocol of
tests/test_gpu_trace.py (every rollout, every control step), and each
iteration's sampling, weights, update and best tracking with the oracle's.
The chain instance (smooth, no contact) is also compared free-running with
the oracle's whole step: costs within 1e-3 relative, knots within 1e-4."""
import numpy as np
import pytest

import oracle as O
from paper_2511_19204_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2511_19204_amd import mppi
    from forced_parity import _np, _t, check_forced, check_iterations, traced_iterations

CFG = [("chain", 32), ("quadruped", 64), ("humanoid", 64)]
TICK = 7


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    mppi.lib()


def _made():
    out = []
    for i, (name, n) in enumerate(CFG):
        m, p, s = synth.config(name, n_samples=n, seed=i)
        model = mppi.Model(m)
        out.append((name, m, p, s, model, mppi.Controller(model, p, s)))
    return out


@pytest.mark.parametrize("form", ["batch", "persistent", "graph"])
def test_multi_instance_launch_against_oracle(form):
    made = _made()
    ctrls = [c for (*_, c) in made]
    states = [_t(m["x0"]) for (_, m, *_r) in made]
    kin = [_t(synth.nominal_knots(m, p["n_knots"])) for (_, m, p, *_r) in made]
    kout = [torch.zeros(c.E, device="cuda") for c in ctrls]
    best = [torch.zeros(c.E, device="cuda") for c in ctrls]
    infos = [torch.zeros(mppi.INFO_INTS, dtype=torch.int32, device="cuda") for _ in ctrls]
    for c in ctrls:
        c.tick = TICK
    if form == "graph":
        g = mppi.Graph(ctrls, states, kin, kout, best, infos)
        g.launch()
        torch.cuda.synchronize()
        g.close()
    else:
        mppi.set_batch_options(persistent=(form == "persistent"))
        try:
            mppi.step_batch(ctrls, states, kin, kout, best, infos)
            torch.cuda.synchronize()
        finally:
            mppi.set_batch_options(persistent=False)
    for i, (name, m, p, s, model, c) in enumerate(made):
        assert c.tick == TICK + 1, name
        x0 = np.asarray(m["x0"], np.float64)
        kn = synth.nominal_knots(m, p["n_knots"])
        # the same instance's iterations one at a time, every rollout recorded
        ref = mppi.Controller(model, p, s)
        its = traced_iterations(ref, m, p, TICK, x0, kn, [np.arange(p["n_samples"])] * p["n_iters"])
        inf = _np(infos[i])
        fused = {"knots": _np(kout[i]), "best": _np(best[i]),
                 "costs": np.stack([d["costs"] for d in its]), "S_best": inf[:1].view(np.float32)[0],
                 "best_iter": int(inf[1]), "n_nonfinite": int(inf[2]), "best_sample": int(inf[4])}
        assert np.array_equal(fused["knots"], its[-1]["next"]), (form, name, "nominal")
        check_iterations(ref, m, p, s, TICK, x0, kn, its, fused, f"{form} {name}")
        for it, d in enumerate(its):
            check_forced(m, p, x0, d["samples"][d["idx"]].astype(np.float64), d["trace"], d["costs"][d["idx"]],
                         f"{form} {name} it{it}")
        assert fused["n_nonfinite"] == 0
        if name == "chain":
            r = O.step(m, p, x0, kn, s, TICK)
            rel = np.abs(fused["costs"] - r["costs"]) / np.abs(r["costs"])
            kerr = np.abs(fused["knots"] - r["knots"]) / np.maximum(1.0, np.abs(r["knots"]))
            print(f"{form} chain vs oracle step: costs {rel.max():.2e}, knots {kerr.max():.2e}")
            assert rel.max() <= 1e-3 and kerr.max() <= 1e-4
            assert fused["best_iter"] == r["best_iter"]
