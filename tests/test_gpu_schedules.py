"""The two rollout schedules (one lane per body swept level by level, and one
lane per kinematic chain) run the same per-body arithmetic in the same order,
so every output must be bit-identical between them: rollout costs of every
iteration, contact masks, updated and best knots, step info.  Also checks the
chain schedule on a fixed-base branching tree (a chain hanging off a joint
body) against the FP64 oracle, ragged sample counts, batches that mix the two
schedules, and the fallback for trees the chain schedule does not take."""
import numpy as np
import pytest

import oracle as O
from paper_2511_19204_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2511_19204_amd import mppi


def _t(x, dtype=torch.float32):
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    mppi.lib()


def _cfg(name, n_samples, seed=0, **over):
    if name == "ytree":
        m = synth.ytree_model(seed)
        p = synth.params(m, n_samples, 50, 0.01, 5, 2, ("linear", 0.1, 0.3), "ee")
        s = 3000 + seed
    else:
        m, p, s = synth.config(name, n_samples=n_samples, seed=seed)
    p.update(over)
    return m, p, s


def _step(c, m, p, knots, tick):
    E = c.E
    st, ki = _t(m["x0"]), _t(knots)
    ko = torch.zeros(E, device="cuda")
    best = torch.zeros(E, device="cuda")
    info = torch.zeros(5, dtype=torch.int32, device="cuda")
    costs = torch.zeros((p["n_iters"], p["n_samples"]), device="cuda")
    c.tick = tick
    c.step(st, ki, ko, best, info, costs)
    return {"knots": _np(ko), "best": _np(best), "info": _np(info), "costs": _np(costs)}


CASES = [("chain", 32), ("chain", 37), ("quadruped", 64), ("quadruped", 1), ("quadruped", 50),
         ("humanoid", 40), ("quadruped_tp", 256), ("ytree", 45)]


@pytest.mark.parametrize("name,n", CASES)
def test_chain_schedule_equals_body_schedule(name, n):
    m, p, s = _cfg(name, n)
    model = mppi.Model(m)
    body = mppi.Controller(model, p, s, schedule="body")
    chain = mppi.Controller(model, p, s, schedule="chain")
    assert body.schedule == "body" and chain.schedule == "chain"
    kn = synth.nominal_knots(m, p["n_knots"])
    for tick in (0, 7):
        a = _step(body, m, p, kn, tick)
        b = _step(chain, m, p, kn, tick)
        print(f"{name} N={n} tick {tick}: costs[0][:3] {a['costs'][0][:3]}")
        for k in a:
            assert np.array_equal(a[k], b[k], equal_nan=True), (name, n, tick, k)


@pytest.mark.parametrize("name,n", [("quadruped", 40), ("humanoid", 24), ("ytree", 20)])
def test_chain_schedule_masks_and_debug_rollouts_equal(name, n):
    m, p, s = _cfg(name, n, horizon=60)
    model = mppi.Model(m)
    body = mppi.Controller(model, p, s, schedule="body")
    chain = mppi.Controller(model, p, s, schedule="chain")
    smp = np.stack([synth.f32(O.sample_knots(m, p, synth.nominal_knots(m, p["n_knots"]), s, 0, 0, k))
                    for k in range(n)])
    out = []
    for c in (body, chain):
        costs = torch.zeros(n, device="cuda")
        masks = torch.zeros((n, p["horizon"]), dtype=torch.int32, device="cuda")
        c.rollouts(_t(m["x0"]), _t(smp), costs, masks)
        out.append((_np(costs), _np(masks)))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    if len(m["contact_body"]):
        assert out[0][1].any()  # contacts were exercised


def test_branching_fixed_base_tree_against_oracle():
    """A chain attached to a joint body: costs of oracle-made knots within 1e-3
    (smooth dynamics, no contact), and the full step's knots within 1e-4."""
    m, p, s = _cfg("ytree", 48)
    model = mppi.Model(m)
    c = mppi.Controller(model, p, s, schedule="chain")
    kn = synth.nominal_knots(m, p["n_knots"])
    smp = np.stack([synth.f32(O.sample_knots(m, p, kn, s, 0, 0, k)) for k in range(48)])
    costs = torch.zeros(48, device="cuda")
    c.rollouts(_t(m["x0"]), _t(smp), costs, None)
    ref = np.array([O.rollout(m, p, m["x0"], smp[k]) for k in range(48)])
    rel = np.abs(_np(costs) - ref) / np.abs(ref)
    print(f"ytree rollout costs: max rel err {rel.max():.2e}")
    assert rel.max() <= 1e-3
    g = _step(c, m, p, kn, 0)
    r = O.step(m, p, m["x0"], kn, s, 0)
    kerr = np.abs(g["knots"] - r["knots"]) / np.maximum(1.0, np.abs(r["knots"]))
    print(f"ytree step: knot err {kerr.max():.2e}")
    assert kerr.max() <= 1e-4


@pytest.mark.parametrize("persistent", [False, True])
def test_batch_mixing_schedules_equals_plain(persistent):
    cfgs = [("chain", 32, "body"), ("quadruped", 48, "chain"), ("humanoid", 40, "chain"),
            ("quadruped", 16, "body"), ("ytree", 30, "chain")]
    made = []
    for i, (nm, k, sch) in enumerate(cfgs):
        m, p, s = _cfg(nm, k, seed=i)
        model = mppi.Model(m)
        made.append((m, p, s, model, mppi.Controller(model, p, s, schedule=sch)))
    plain = [_step(c, m, p, synth.nominal_knots(m, p["n_knots"]), 4) for (m, p, s, model, c) in made]
    states = [_t(m["x0"]) for (m, p, s, model, c) in made]
    kin = [_t(synth.nominal_knots(m, p["n_knots"])) for (m, p, s, model, c) in made]
    kout = [torch.zeros(c.E, device="cuda") for (*_, c) in made]
    for (*_, c) in made:
        c.tick = 4
    mppi.set_batch_options(persistent)
    try:
        mppi.step_batch([c for (*_, c) in made], states, kin, kout)
    finally:
        mppi.set_batch_options(False)
    for i in range(len(made)):
        assert np.array_equal(_np(kout[i]), plain[i]["knots"]), i


def test_deep_tree_falls_back_to_body_schedule():
    """A 17-link serial arm is deeper than the chain schedule's level table: the
    default is the body schedule and asking for chains fails cleanly."""
    t = synth._Tree()
    prev = -1
    for i in range(17):
        prev = t.body(prev, (0, 1, 0), (0.0, 0, 0) if i == 0 else (0.1, 0, 0), 0.5, (0.05, 0, 0),
                      (0.1, 0.03, 0.03), joint=(-2.0, 2.0, 10.0, 10.0, 0.1, 0.0))
    m = t.finish("arm17", False, [], np.zeros((0, 3)), ee_body=16, ee_pos=(0.1, 0, 0))
    m["n_substeps"] = 1
    m["armature"] = synth.f32(np.full(17, 0.01))
    m["x0"] = synth.f32(np.zeros(34))
    p = synth.params(m, 8, 10, 0.01, 4, 1, ("linear", 0.1, 0.2), "ee")
    model = mppi.Model(m)
    c = mppi.Controller(model, p, 1)
    assert c.schedule == "body" and c.lanes == 32
    with pytest.raises(mppi.MppiError):
        c.set_schedule("chain")
    g = _step(c, m, p, synth.nominal_knots(m, p["n_knots"]), 0)
    assert np.all(np.isfinite(g["costs"]))
