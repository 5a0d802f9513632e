"""The team schedule (each kinematic chain on a block of lanes; the sweeps split
by spatial coordinate over the block's first three lanes) against the FP64
oracle, its determinism, batching, and the trees it does not take.

It evaluates the body schedule's formulas with sums in another order, so it is
compared with the oracle by the same bars as the other schedules (short
horizons: at least 90 % of the rollouts with the oracle's contact sequences and
on those a relative cost error of at most 1e-3; the arm's full step: costs 1e-3,
knots 1e-4), and with itself bit for bit."""
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


def _cfg(name, n, **over):
    if name == "ytree":
        m = synth.ytree_model()
        p = synth.params(m, n, 50, 0.01, 5, 2, ("linear", 0.1, 0.3), "ee")
        s = 3000
    else:
        m, p, s = synth.config(name, n_samples=n)
    p.update(over)
    return m, p, s


@pytest.mark.parametrize("name,count,H", [("chain", 32, 50), ("quadruped", 48, 20), ("humanoid", 32, 40),
                                          ("ytree", 40, 50), ("quadruped", 21, 20), ("hexapod", 40, 20)])
def test_team_rollout_costs_match_oracle(name, count, H):
    m, p, s = _cfg(name, count, horizon=H)
    model = mppi.Model(m)
    c = mppi.Controller(model, p, s, schedule="team")
    assert c.schedule == "team"
    nom = synth.nominal_knots(m, p["n_knots"])
    smp = np.stack([synth.f32(O.sample_knots(m, p, nom, s, 0, 0, n)) for n in range(count)])
    costs = torch.zeros(count, device="cuda")
    masks = torch.zeros((count, H), dtype=torch.int32, device="cuda")
    c.rollouts(_t(m["x0"]), _t(smp), costs, masks)
    got, gm = _np(costs), _np(masks).view(np.uint32)
    ref, rm = np.zeros(count), np.zeros((count, H), np.uint32)
    for n in range(count):
        ref[n], _, rm[n], _ = O.rollout(m, p, m["x0"], smp[n], debug=True)
    same = np.all(gm == rm, axis=1)
    rel = np.abs(got - ref) / np.abs(ref)
    print(f"team {name} H={H}: identical contact sequences {same.sum()}/{count}, max rel err {rel[same].max():.2e}")
    assert same.mean() >= 0.9 and rel[same].max() <= 1e-3


def test_team_full_step_arm_matches_oracle():
    m, p, s = _cfg("chain", 32)
    c = mppi.Controller(mppi.Model(m), p, s, schedule="team")
    kn = synth.nominal_knots(m, p["n_knots"])
    c.tick = 0
    ko, best = torch.zeros(c.E, device="cuda"), torch.zeros(c.E, device="cuda")
    costs = torch.zeros((p["n_iters"], p["n_samples"]), device="cuda")
    c.step(_t(m["x0"]), _t(kn), ko, best, None, costs)
    r = O.step(m, p, m["x0"], kn, s, 0)
    rel = np.abs(_np(costs) - r["costs"]) / np.abs(r["costs"])
    kerr = np.abs(_np(ko) - r["knots"]) / np.maximum(1.0, np.abs(r["knots"]))
    print(f"team arm step: cost {rel.max():.2e} knots {kerr.max():.2e}")
    assert rel.max() <= 1e-3 and kerr.max() <= 1e-4


def test_team_close_to_body_on_the_smooth_arm():
    """No contact: the two schedules differ by the rounding of reordered sums only."""
    m, p, s = _cfg("chain", 64)
    model = mppi.Model(m)
    out = {}
    for sch in ("body", "team"):
        c = mppi.Controller(model, p, s, schedule=sch)
        c.tick = 2
        costs = torch.zeros((p["n_iters"], p["n_samples"]), device="cuda")
        ko = torch.zeros(c.E, device="cuda")
        c.step(_t(m["x0"]), _t(synth.nominal_knots(m, p["n_knots"])), ko, None, None, costs)
        out[sch] = _np(costs)
    rel = np.abs(out["team"] - out["body"]) / np.abs(out["body"])
    assert rel.max() <= 1e-5, rel.max()


@pytest.mark.parametrize("name,n", [("quadruped", 64), ("humanoid", 40), ("ytree", 45), ("quadruped", 37),
                                    ("hexapod", 33)])
def test_team_is_deterministic_and_batches_bit_identically(name, n):
    m, p, s = _cfg(name, n)
    model = mppi.Model(m)
    c = mppi.Controller(model, p, s, schedule="team")
    runs = []
    for _ in range(2):
        c.tick = 5
        ko = torch.zeros(c.E, device="cuda")
        costs = torch.zeros((p["n_iters"], p["n_samples"]), device="cuda")
        c.step(_t(m["x0"]), _t(synth.nominal_knots(m, p["n_knots"])), ko, None, None, costs)
        runs.append((_np(ko), _np(costs)))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    for persistent in (False, True):
        c.tick = 5
        ko = torch.zeros(c.E, device="cuda")
        mppi.set_batch_options(persistent)
        try:
            mppi.step_batch([c], [_t(m["x0"])], [_t(synth.nominal_knots(m, p["n_knots"]))], [ko])
        finally:
            mppi.set_batch_options(False)
        assert np.array_equal(_np(ko), runs[0][0]), persistent


def test_batch_mixing_team_and_body_instances():
    cfgs = [("chain", 32, "team"), ("quadruped", 48, "body"), ("humanoid", 40, "team"), ("quadruped", 16, "team"),
            ("ytree", 30, "body")]
    made = []
    for i, (nm, k, sch) in enumerate(cfgs):
        m, p, s = _cfg(nm, k)
        model = mppi.Model(m)
        made.append((m, p, model, mppi.Controller(model, p, s + i, schedule=sch)))
    plain = []
    for (m, p, model, c) in made:
        c.tick = 4
        o = torch.zeros(c.E, device="cuda")
        c.step(_t(m["x0"]), _t(synth.nominal_knots(m, p["n_knots"])), o)
        plain.append(_np(o))
    for (*_, c) in made:
        c.tick = 4
    kout = [torch.zeros(c.E, device="cuda") for (*_, c) in made]
    mppi.step_batch([c for (*_, c) in made], [_t(m["x0"]) for (m, *_r) in made],
                    [_t(synth.nominal_knots(m, p["n_knots"])) for (m, p, *_r) in made], kout)
    for i in range(len(made)):
        assert np.array_equal(_np(kout[i]), plain[i]), i


def test_team_with_spline_variant_and_task_target():
    m, p, s = _cfg("quadruped", 32, horizon=20)
    p = synth.task_params(m, p, "handstand")
    p["spline_mode"] = 1
    c = mppi.Controller(mppi.Model(m), p, s, schedule="team")
    nom = synth.nominal_knots(m, p["n_knots"])
    smp = np.stack([synth.f32(O.sample_knots(m, p, nom, s, 0, 0, n)) for n in range(32)])
    costs = torch.zeros(32, device="cuda")
    masks = torch.zeros((32, 20), dtype=torch.int32, device="cuda")
    c.rollouts(_t(m["x0"]), _t(smp), costs, masks)
    got, gm = _np(costs), _np(masks).view(np.uint32)
    ref, rm = np.zeros(32), np.zeros((32, 20), np.uint32)
    for n in range(32):
        ref[n], _, rm[n], _ = O.rollout(m, p, m["x0"], smp[n], debug=True)
    same = np.all(gm == rm, axis=1)
    rel = np.abs(got - ref) / np.abs(ref)
    assert same.mean() >= 0.9 and rel[same].max() <= 1e-3


def test_trees_the_team_schedule_does_not_take():
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
    c = mppi.Controller(mppi.Model(m), p, 1)
    with pytest.raises(mppi.MppiError):
        c.set_schedule("team")
    assert c.schedule == "body"
