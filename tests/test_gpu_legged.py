"""Legged trees other than the quadruped's four chains of three, which the body
schedule runs with the legged-tree rollout kernel (every joint body's parent is
the body before it or the base, bodies kept in registers across steps, the
whole tree folded by lane moves): a hexapod (19 bodies, 32 lanes per rollout)
and the quadruped with a second contact point on every shank (two contacts on a
body, so not the four-by-three kernel).  The body schedule must equal the chain
schedule bit for bit, and the step must meet the oracle step by step along the
GPU's own trajectories (the bars of the forced-parity tests).  The hexapod's
knot count first showed the update's two sample forms (drawn again, stored)
summing in different orders past one chunk of element blocks; the last test
pins them equal at such sizes."""
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


def _quadruped_two_contacts(n_samples, seed=0):
    """Each shank carries its foot point and a second point 3 cm ahead of it."""
    m = dict(synth.quadruped_model(seed))
    cb = np.asarray(m["contact_body"])
    cp = np.asarray(m["contact_pos"])
    m["contact_body"] = np.concatenate([cb, cb]).astype(cb.dtype)
    m["contact_pos"] = np.concatenate([cp, cp + np.array([0.03, 0.0, 0.0], cp.dtype)]).astype(cp.dtype)
    m["support"] = np.concatenate([np.asarray(m["support"]), np.zeros(len(cb), bool)])
    p = synth.params(m, n_samples, 100, 0.005, 8, 3, ("exp", 0.4, 1.0, 1.0), "walking")
    return m, p, 4100 + seed


def _cfg(name, n_samples):
    if name == "quadruped2c":
        return _quadruped_two_contacts(n_samples)
    return synth.config(name, n_samples=n_samples)


def _step(c, m, p, knots, tick):
    E = c.E
    ko = torch.zeros(E, device="cuda")
    best = torch.zeros(E, device="cuda")
    info = torch.zeros(5, dtype=torch.int32, device="cuda")
    costs = torch.zeros((p["n_iters"], p["n_samples"]), device="cuda")
    c.tick = tick
    c.step(torch.tensor(np.asarray(m["x0"], np.float32), device="cuda"),
           torch.tensor(np.asarray(knots, np.float32), device="cuda"), ko, best, info, costs)
    torch.cuda.synchronize()
    return {"knots": ko.cpu().numpy(), "best": best.cpu().numpy(), "info": info.cpu().numpy(),
            "costs": costs.cpu().numpy()}


@pytest.mark.parametrize("name,n,lanes", [("hexapod", 64, 32), ("hexapod", 45, 32),
                                          ("quadruped2c", 64, 16), ("quadruped2c", 37, 16),
                                          ("quadruped2c", 40, 32)])
def test_legged_kernel_equals_chain_schedule(name, n, lanes):
    m, p, s = _cfg(name, n)
    model = mppi.Model(m)
    body = mppi.Controller(model, p, s, lanes=lanes, schedule="body")
    chain = mppi.Controller(model, p, s, schedule="chain")
    assert body.schedule == "body" and body.lanes == lanes and chain.schedule == "chain"
    kn = synth.nominal_knots(m, p["n_knots"])
    for tick in (0, 5):
        a = _step(body, m, p, kn, tick)
        b = _step(chain, m, p, kn, tick)
        print(f"{name} N={n} lanes={lanes} tick {tick}: costs[0][:3] {a['costs'][0][:3]}")
        assert np.all(np.isfinite(a["costs"]))
        for k in a:
            assert np.array_equal(a[k], b[k], equal_nan=True), (name, n, lanes, tick, k)


@pytest.mark.parametrize("name", ["hexapod", "quadruped2c"])
def test_legged_kernel_forced_parity(name):
    """K=64, H=100, 3 iterations: every rollout of every iteration is recorded by
    the legged kernel's trace form and checked step by step against the oracle;
    the iterations and the update follow the oracle and equal the fused step."""
    m, p, s = _cfg(name, 64)
    model = mppi.Model(m)
    c = mppi.Controller(model, p, s)
    assert c.schedule == "body" and c.lanes == (32 if name == "hexapod" else 16)
    kn = synth.nominal_knots(m, p["n_knots"])
    x0 = np.asarray(m["x0"], np.float64)
    its = traced_iterations(c, m, p, 3, x0, kn, [np.arange(p["n_samples"])] * p["n_iters"])
    fused = fused_step(c, m, p, 3, x0, kn)
    tot = {"acc_esc_f32": 0, "acc_esc_sens": 0, "steps": 0, "mask_flips": 0}
    for it, d in enumerate(its):
        st = check_forced(m, p, x0, d["samples"][d["idx"]].astype(np.float64), d["trace"], d["costs"][d["idx"]],
                          f"{name} it{it}")
        for k in tot:
            tot[k] += st[k]
    check_iterations(c, m, p, s, 3, x0, kn, its, fused, name)
    print(f"{name} total: {tot}")
    masks = np.concatenate([d["trace"][:, :p["horizon"], m["n_q"] + 2 * m["n_v"] + 1].view(np.uint32)
                            for d in its])
    nc = len(m["contact_body"])
    seen = np.bitwise_or.reduce(masks.ravel())
    print(f"{name}: contact points touching at some step {bin(seen)}")
    assert seen == (1 << nc) - 1, "every contact point, the second shank points included, was exercised"
    assert tot["mask_flips"] <= 1e-3 * tot["steps"]
    assert fused["n_nonfinite"] == 0


@pytest.mark.parametrize("persistent", [False, True])
def test_batches_that_widen_the_kernel_equal_plain_steps(persistent):
    """A batched launch takes the most general kernel its instances share: a
    hexapod beside a humanoid (32 lanes each) runs the general kernel, the
    two-contact quadruped beside the plain one (16 lanes) the legged-tree kernel
    instead of the four-by-three one.  Every instance must still equal its plain
    step bit for bit."""
    made = []
    for i, (name, n) in enumerate([("hexapod", 40), ("humanoid", 24), ("hexapod", 7),
                                   ("quadruped2c", 33), ("quadruped", 48)]):
        m, p, s = _cfg(name, n)
        model = mppi.Model(m)
        c = mppi.Controller(model, p, s + i, schedule="body")
        made.append((m, p, c))
    assert [c.lanes for (_, _, c) in made] == [32, 32, 32, 16, 16]
    plain = [_step(c, m, p, synth.nominal_knots(m, p["n_knots"]), 2) for (m, p, c) in made]
    states = [torch.tensor(np.asarray(m["x0"], np.float32), device="cuda") for (m, p, c) in made]
    kin = [torch.tensor(synth.nominal_knots(m, p["n_knots"]).astype(np.float32), device="cuda")
           for (m, p, c) in made]
    kout = [torch.zeros(c.E, device="cuda") for (m, p, c) in made]
    for (m, p, c) in made:
        c.tick = 2
    mppi.set_batch_options(persistent)
    try:
        mppi.step_batch([c for (m, p, c) in made], states, kin, kout)
    finally:
        mppi.set_batch_options(False)
    torch.cuda.synchronize()
    for i in range(len(made)):
        assert np.array_equal(kout[i].cpu().numpy(), plain[i]["knots"]), i


@pytest.mark.parametrize("n_samples,n_knots", [(2048, 48), (600, 40), (4096, 8)])
def test_update_drawn_again_equals_update_of_stored_samples(n_samples, n_knots):
    """The fused step draws every sample's knots again in the update; the traced
    iterations store them and update from the stored rows.  The two must agree bit
    for bit whatever the element count: 12 joints x 48 knots is 288 element blocks
    for 256 update threads, 40 knots 240 blocks for 64 threads (a chunk of blocks
    beyond the first), 8 knots the throughput shape."""
    m = synth.quadruped_model(0)
    p = synth.params(m, n_samples, 20, 0.005, n_knots, 2, ("exp", 0.4, 1.0, 1.0), "walking")
    s = 4200 + n_knots
    model = mppi.Model(m)
    c = mppi.Controller(model, p, s)
    kn = synth.nominal_knots(m, p["n_knots"])
    x0 = np.asarray(m["x0"], np.float64)
    its = traced_iterations(c, m, p, 1, x0, kn, [np.arange(2)] * p["n_iters"])
    fused = fused_step(c, m, p, 1, x0, kn)
    for it, d in enumerate(its):
        assert np.array_equal(d["costs"], fused["costs"][it]), it
    assert np.array_equal(its[-1]["next"], fused["knots"])
    assert np.all(np.isfinite(fused["knots"]))
