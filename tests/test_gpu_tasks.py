"""Task presets (Sec. IV-B with the weights of Tab. cost-weights) on the GPU:
orientation targets and the absolute terminal height against the FP64 oracle,
and changing targets between calls.

Bars as for the other rollouts: over oracle-made samples, at least 90 % of the
rollouts with contact sequences identical to the oracle's, and on those the
relative cost error at most 1e-3; mppi_set_targets equals an instance created
with the same targets bit for bit, is ordered on its stream, and cached plans
and graphs use the targets current when they run."""
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


def _task(name, n_samples, **over):
    base = "humanoid" if name == "bipedal" else "quadruped"
    m, p, s = synth.config(base, n_samples=n_samples)
    p = synth.task_params(m, p, name)
    p.update(over)
    return m, p, s


@pytest.mark.parametrize("name", synth.TASKS)
def test_task_rollout_costs_match_oracle(name):
    count, H = 40, 40
    m, p, s = _task(name, count, horizon=H)
    model = mppi.Model(m)
    c = mppi.Controller(model, p, s)
    nom = synth.nominal_knots(m, p["n_knots"])
    smp = np.stack([synth.f32(O.sample_knots(m, p, nom, s, 0, 0, n)) for n in range(count)])
    # from the level stance the handstand and backflip targets are 45 and 180 degrees away
    x0 = np.array(m["x0"], float)
    costs = torch.zeros(count, device="cuda")
    masks = torch.zeros((count, H), dtype=torch.int32, device="cuda")
    c.rollouts(_t(x0), _t(smp), costs, masks)
    got, gm = _np(costs), _np(masks).view(np.uint32)
    ref, rm = np.zeros(count), np.zeros((count, H), np.uint32)
    for n in range(count):
        ref[n], _, rm[n], _ = O.rollout(m, p, x0, smp[n], debug=True)
    same = np.all(gm == rm, axis=1)
    rel = np.abs(got - ref) / np.abs(ref)
    print(f"{name}: identical contact sequences {same.sum()}/{count}, max rel err {rel[same].max():.2e}")
    assert same.mean() >= 0.9 and rel[same].max() <= 1e-3


def test_set_targets_equals_creating_with_them():
    m, p0, s = _task("walking", 64)
    model = mppi.Model(m)
    kn = _t(synth.nominal_knots(m, p0["n_knots"]))
    x = _t(m["x0"])
    outs = {}
    for name in ("handstand", "jumping"):
        p = synth.task_params(m, p0, name)
        fresh = mppi.Controller(model, p, s)
        a = torch.zeros_like(kn)
        costs_a = torch.zeros((p["n_iters"], p["n_samples"]), device="cuda")
        fresh.tick = 3
        fresh.step(x, kn, a, None, None, costs_a)
        # an instance made for walking, retargeted (weights are part of the task: keep them equal)
        q = dict(p)
        q.update(q_des=[0.0] * 4, terminal_z_abs=0, z_terminal=0.0, v_des=[0.5, 0.0, 0.0])
        moved = mppi.Controller(model, q, s)
        moved.set_targets(z_des=p["z_des"], v_des=p["v_des"], q_des=p["q_des"], terminal_z_abs=p["terminal_z_abs"],
                          z_terminal=p["z_terminal"])
        b = torch.zeros_like(kn)
        costs_b = torch.zeros_like(costs_a)
        moved.tick = 3
        moved.step(x, kn, b, None, None, costs_b)
        assert np.array_equal(_np(a), _np(b)) and np.array_equal(_np(costs_a), _np(costs_b)), name
        outs[name] = _np(costs_a)
    assert not np.array_equal(outs["handstand"], outs["jumping"])
    with pytest.raises(mppi.MppiError):
        moved.set_targets(q_des=[1.0, 1.0, 0.0, 0.0])
    with pytest.raises(mppi.MppiError):
        p = synth.task_params(m, p0, "walking")
        p["q_des"] = [0.5, 0.0, 0.0, 0.0]
        mppi.Controller(model, p, s)


def test_set_targets_is_stream_ordered_and_plans_and_graphs_follow():
    """mppi_set_targets is one kernel on the stream: a step enqueued before it
    scores the old targets and one enqueued after it the new ones, with no
    synchronisation in between; a cached batch plan and a captured graph made
    before the change score the targets current when they run."""
    m, p0, s = _task("walking", 64)
    model = mppi.Model(m)
    kn = _t(synth.nominal_knots(m, p0["n_knots"]))
    x = _t(m["x0"])
    ph = synth.task_params(m, p0, "handstand")
    pw = dict(ph)
    pw.update(q_des=[0.0] * 4, terminal_z_abs=0, z_terminal=0.0, v_des=list(p0["v_des"]))

    def fresh(p, tick):
        c = mppi.Controller(model, p, s)
        c.tick = tick
        o = torch.zeros_like(kn)
        c.step(x, kn, o)
        return _np(o)

    ref_w, ref_h, ref_h6 = fresh(pw, 5), fresh(ph, 5), fresh(ph, 6)
    assert not np.array_equal(ref_w, ref_h)
    c = mppi.Controller(model, pw, s)
    stream = torch.cuda.Stream()
    a, b = torch.zeros_like(kn), torch.zeros_like(kn)
    torch.cuda.synchronize()
    c.tick = 5
    with torch.cuda.stream(stream):
        c.step(x, kn, a, stream=stream)             # tick 5, then the tick advances to 6 on the device
        c.set_targets(q_des=ph["q_des"], stream=stream)
        c.step(x, kn, b, stream=stream)             # tick 6
    stream.synchronize()
    assert np.array_equal(_np(a), ref_w) and np.array_equal(_np(b), ref_h6)
    # a cached plan (batched step) and a graph made under the handstand targets
    c.tick = 5
    o = torch.zeros_like(kn)
    mppi.step_batch([c], [x], [kn], [o])
    assert np.array_equal(_np(o), ref_h)
    g = mppi.Graph([c], [x], [kn], [o])
    c.set_targets(q_des=[0.0] * 4)
    c.tick = 5
    mppi.step_batch([c], [x], [kn], [o])
    assert np.array_equal(_np(o), ref_w)
    c.tick = 5
    g.launch()
    assert np.array_equal(_np(o), ref_w)
    c.set_targets(q_des=ph["q_des"])
    c.tick = 5
    g.launch()
    assert np.array_equal(_np(o), ref_h)


def test_batch_of_different_tasks_equals_plain_steps():
    made = []
    for i, name in enumerate(synth.TASKS):
        m, p, s = _task(name, 48)
        model = mppi.Model(m)
        made.append((m, p, model, mppi.Controller(model, p, s + i)))
    plain = []
    for (m, p, model, c) in made:
        c.tick = 1
        o = torch.zeros(c.E, device="cuda")
        c.step(_t(m["x0"]), _t(synth.nominal_knots(m, p["n_knots"])), o)
        plain.append(_np(o))
    for (*_, c) in made:
        c.tick = 1
    kout = [torch.zeros(c.E, device="cuda") for (*_, c) in made]
    mppi.step_batch([c for (*_, c) in made], [_t(m["x0"]) for (m, *_r) in made],
                    [_t(synth.nominal_knots(m, p["n_knots"])) for (m, p, *_r) in made], kout)
    for i in range(len(made)):
        assert np.array_equal(_np(kout[i]), plain[i]), synth.TASKS[i]
