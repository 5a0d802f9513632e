"""State prediction, warm-start shift and the control tick (Sec. III-E, Alg. 1)
on the GPU, through the C ABI, against the FP64 oracle.

Bars: shifted knots within 1e-5 max(1, |x|) (float evaluation of the spline:
the velocity knots carry the 1/Delta scaling); predicted states, per block
(positions, velocities) over eight trajectories, with median and maximum error
against FP64 within 3x and 10x those of the oracle's own float build, plus
1e-6 (soft contact amplifies the per-step rounding of the forces); the tick equals
predict -> shift -> step bit for bit, and its step info reports the best
sample consistently with the costs."""
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


def _ctrl(name, n_samples=32, seed=0, **over):
    m, p, s = synth.config(name, n_samples=n_samples, seed=seed)
    p.update(over)
    model = mppi.Model(m)
    return m, p, s, model, mppi.Controller(model, p, s)


def _perturbed_knots(m, p, seed):
    """Nominal knots moved inside the joint limits (a non-trivial spline)."""
    rng = np.random.default_rng(seed)
    nk, nu = p["n_knots"], m["n_u"]
    kn = synth.nominal_knots(m, p["n_knots"]).astype(np.float64)
    lo, hi = m["q_min"].astype(np.float64), m["q_max"].astype(np.float64)
    q = kn[: nk * nu].reshape(nk, nu) + rng.normal(scale=0.05, size=(nk, nu))
    q = np.clip(q, lo + 0.02, hi - 0.02)
    v = rng.normal(scale=0.3, size=(nk, nu))
    return synth.f32(np.concatenate([q.ravel(), v.ravel()]))


@pytest.mark.parametrize("name", ["chain", "quadruped", "humanoid"])
def test_shift_knots_matches_oracle(name):
    m, p, s, model, c = _ctrl(name)
    kn = _perturbed_knots(m, p, 1)
    H = p["horizon"]
    for n in [0, 1, 3, H // 3, H - 1, H, H + 7]:
        out = torch.zeros(c.E, device="cuda")
        c.shift_knots(_t(kn), n, out)
        ref = O.shift_knots(kn, p["n_knots"], m["n_u"], H, p["dt"], n)
        err = np.abs(_np(out) - ref) / np.maximum(1.0, np.abs(ref))
        assert err.max() <= 1e-5, (name, n, err.max())
    # the final knot pair is reproduced exactly whatever the shift
    out = torch.zeros(c.E, device="cuda")
    c.shift_knots(_t(kn), H + 7, out)
    nk, nu = p["n_knots"], m["n_u"]
    got = _np(out)
    assert np.array_equal(got[: nk * nu].reshape(nk, nu)[-1], kn[: nk * nu].reshape(nk, nu)[-1])


def test_shift_in_place():
    m, p, s, model, c = _ctrl("quadruped")
    kn = _perturbed_knots(m, p, 2)
    a = torch.zeros(c.E, device="cuda")
    c.shift_knots(_t(kn), 9, a)
    b = _t(kn)
    c.shift_knots(b, 9, b)
    assert np.array_equal(_np(a), _np(b))


@pytest.mark.parametrize("name,n", [("chain", 10), ("chain", 50), ("quadruped", 4), ("quadruped", 12),
                                    ("humanoid", 6)])
def test_predict_matches_oracle(name, n):
    """Over eight trajectories, per state block (positions, velocities): the
    GPU's distance to the FP64 oracle has a median at most 3x, and a maximum at
    most 10x, that of the oracle's own float build (plus 1e-6).  One trajectory
    through stiff contact is a noisy sample of rounding, hence the statistics."""
    m, p, s, model, c = _ctrl(name)
    x0 = m["x0"]
    nq = m["n_q"]
    eg, ef = [[], []], [[], []]
    for trial in range(8):
        kn = _perturbed_knots(m, p, 30 + trial)
        out = torch.zeros(len(x0), device="cuda")
        c.predict(_t(x0), _t(kn), n, out)
        got = _np(out)
        ref = O.predict(m, p, x0, kn, n)
        f32 = O.predict_f32(m, p, x0, kn, n)
        for i, blk in enumerate((slice(0, nq), slice(nq, None))):
            eg[i].append(np.abs(got[blk] - ref[blk]).max())
            ef[i].append(np.abs(f32[blk] - ref[blk]).max())
    for i, name_b in enumerate(("positions", "velocities")):
        g, f = np.array(eg[i]), np.array(ef[i])
        print(f"{name} n={n} {name_b}: median gpu {np.median(g):.2e} oracle-f32 {np.median(f):.2e}; "
              f"max gpu {g.max():.2e} oracle-f32 {f.max():.2e}")
        assert np.median(g) <= 3 * np.median(f) + 1e-6
        assert g.max() <= 10 * f.max() + 1e-6


def test_predict_zero_steps_and_in_place():
    m, p, s, model, c = _ctrl("quadruped")
    kn = _t(_perturbed_knots(m, p, 4))
    x = _t(m["x0"])
    out = torch.zeros_like(x)
    c.predict(x, kn, 0, out)
    assert np.array_equal(_np(out), _np(x))
    a = torch.zeros_like(x)
    c.predict(x, kn, 7, a)
    c.predict(x, kn, 7, x)  # in place
    assert np.array_equal(_np(a), _np(x))


@pytest.mark.parametrize("name,delay", [("chain", 0), ("chain", 4), ("quadruped", 3), ("humanoid", 2)])
def test_tick_equals_predict_shift_step(name, delay):
    m, p, s, model, c = _ctrl(name)
    best0 = _perturbed_knots(m, p, 5)
    x = _t(m["x0"])
    # composed from the separate entry points
    c.tick = 3
    xp = torch.zeros_like(x)
    c.predict(x, _t(best0), delay, xp)
    k0 = torch.zeros(c.E, device="cuda")
    c.shift_knots(_t(best0), delay, k0)
    ko_a, best_a = torch.zeros(c.E, device="cuda"), torch.zeros(c.E, device="cuda")
    info_a = torch.zeros(mppi.INFO_INTS, dtype=torch.int32, device="cuda")
    costs = torch.zeros((p["n_iters"], p["n_samples"]), device="cuda")
    c.step(xp, k0, ko_a, best_a, info_a, costs)
    # one tick
    c.tick = 3
    best_b = _t(best0)
    ko_b = torch.zeros(c.E, device="cuda")
    info_b = torch.zeros(mppi.INFO_INTS, dtype=torch.int32, device="cuda")
    xp_b = torch.zeros_like(x)
    c.run_tick(x, delay, best_b, ko_b, info_b, xp_b)
    assert np.array_equal(_np(xp_b), _np(xp))
    assert np.array_equal(_np(ko_b), _np(ko_a))
    assert np.array_equal(_np(best_b), _np(best_a))
    assert np.array_equal(_np(info_b), _np(info_a))
    assert c.tick == 4
    # the reported best sample is the lowest index attaining the minimum of its iteration
    inf = _np(info_b)
    cs = _np(costs)
    it, n = int(inf[1]), int(inf[4])
    assert 0 <= it < p["n_iters"] and n == int(np.argmin(cs[it]))
    assert inf[:1].view(np.float32)[0] == cs[it, n]


def test_tick_against_oracle_smooth_arm():
    """Arm (no contact): the tick's nominal and best knots against the oracle's
    predict -> shift -> step within 1e-4 max(1, |x|)."""
    m, p, s, model, c = _ctrl("chain")
    best0 = _perturbed_knots(m, p, 6)
    delay = 5
    c.tick = 0
    best = _t(best0)
    ko = torch.zeros(c.E, device="cuda")
    info = torch.zeros(mppi.INFO_INTS, dtype=torch.int32, device="cuda")
    c.run_tick(_t(m["x0"]), delay, best, ko, info)
    xpred = O.predict(m, p, m["x0"], best0, delay)
    k0 = O.shift_knots(best0, p["n_knots"], m["n_u"], p["horizon"], p["dt"], delay)
    r = O.step(m, p, xpred, k0, s, 0)
    for got, ref in ((_np(ko), r["knots"]), (_np(best), r["best_knots"])):
        err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
        print(f"tick vs oracle: max err {err.max():.2e}")
        assert err.max() <= 1e-4
    inf = _np(info)
    assert inf[1] == r["best_iter"]
    assert inf[4] == int(np.argmin(r["costs"][r["best_iter"]]))


def _oracle_tick(m, p, s, tick, x_meas, best, delay):
    """One control step of Alg. 1 with Sec. III-E's prediction and warm start:
    x_t = predict(x_meas, best, delay), tau_0 = best shifted by delay, then the
    I iterations; returns the predicted state and the step's results."""
    xpred = O.predict(m, p, x_meas, best, delay)
    k0 = O.shift_knots(best, p["n_knots"], m["n_u"], p["horizon"], p["dt"], delay)
    r = O.step(m, p, xpred, k0, s, tick)
    r["best_sample"] = int(np.argmin(r["costs"][r["best_iter"]])) if r["best_iter"] >= 0 else -1
    return xpred, r


def test_best_trajectory_carried_across_ticks_against_oracle():
    """Twelve chained ticks of the arm task (Sec. III-D/III-E: tau_best carried
    from tick to tick, predicted, shifted, refined; the robot follows the plan,
    so the next measurement is this tick's prediction), on the GPU with the best
    trajectory kept on the device and in the oracle, each side running its own
    chain.  After every tick: tau_best, the nominal and the predicted state
    within 1e-4 max(1, |x|) (the two chains run free, so the float rounding of
    earlier ticks carries into the state; a tick's own prediction is held to
    the per-step bars of the trajectory-forced tests), the same best iteration
    and sample, and so
    the same "failed to improve" flag (the best is sample 0 of iteration 0, the
    shifted previous solution) and the same count over the run."""
    m, p, s, model, c = _ctrl("chain", n_samples=32)
    delay, ticks = 2, 12
    best_o = synth.nominal_knots(m, p["n_knots"]).astype(np.float64)
    x_o = np.asarray(m["x0"], np.float64)
    best = _t(best_o)
    x = _t(x_o)
    c.tick = 0
    failed_gpu = failed_orc = 0
    for t in range(ticks):
        info = torch.zeros(mppi.INFO_INTS, dtype=torch.int32, device="cuda")
        xp = torch.zeros_like(x)
        ko = torch.zeros(c.E, device="cuda")
        c.run_tick(x, delay, best, ko, info, xp)
        x_o, r = _oracle_tick(m, p, s, t, x_o, best_o, delay)
        best_o = r["best_knots"]
        inf = _np(info)
        eb = np.max(np.abs(_np(best) - best_o) / np.maximum(1.0, np.abs(best_o)))
        ek = np.max(np.abs(_np(ko) - r["knots"]) / np.maximum(1.0, np.abs(r["knots"])))
        ex = np.max(np.abs(_np(xp) - x_o) / np.maximum(1.0, np.abs(x_o)))
        print(f"tick {t}: best err {eb:.2e}, nominal err {ek:.2e}, state err {ex:.2e}, "
              f"best (iter, sample) gpu ({inf[1]}, {inf[4]}) oracle ({r['best_iter']}, {r['best_sample']})")
        assert eb <= 1e-4 and ek <= 1e-4 and ex <= 1e-4, t
        assert (int(inf[1]), int(inf[4])) == (r["best_iter"], r["best_sample"]), t
        assert abs(inf[:1].view(np.float32)[0] - r["S_best"]) <= 1e-3 * abs(r["S_best"])
        failed_gpu += int(inf[1] == 0 and inf[4] == 0)
        failed_orc += int(r["best_iter"] == 0 and r["best_sample"] == 0)
        x = xp
    print(f"failed to improve: gpu {failed_gpu}/{ticks}, oracle {failed_orc}/{ticks}")
    assert failed_gpu == failed_orc
    assert c.tick == ticks
