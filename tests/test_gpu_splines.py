"""Spline variants of the ablation (natural cubic and quadratic position splines
with zero velocity targets) on the GPU against the FP64 oracle.

Bars: sampled position knots as in the cubic Hermite case (2e-6 relative); knot
slopes within the position tolerance carried through the positions -> slopes
map plus 1e-5 max(1, |x|) of their own float rounding; short-horizon rollout
costs of oracle-made knots within 1e-3 relative; the arm's full ten-iteration
step within 1e-3 on costs and 1e-4 on knots (no contact); shifted knots within
1e-5 max(1, |x|); the tick equal to predict -> shift -> step bit for bit."""
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


def _ctrl(name, mode, n_samples=None, seed=0, **over):
    m, p, s = synth.config(name, n_samples=n_samples, seed=seed)
    p["spline_mode"] = mode
    p.update(over)
    model = mppi.Model(m)
    return m, p, s, model, mppi.Controller(model, p, s)


def _nominal(m, p, seed=1):
    nom = synth.nominal_knots(m, p["n_knots"])
    return synth.f32(nom + np.random.default_rng(seed).normal(0, 0.05, nom.size))


def _slope_map(mode, K, delta):
    """|L| of the linear map positions -> knot slopes of the variant (same for every
    joint), from the oracle's slopes of unit position vectors."""
    L = np.zeros((K, K))
    for i in range(K):
        e = np.zeros(2 * K)
        e[i] = 1.0
        L[:, i] = O.spline_slopes(mode, e, K, 1, delta)[K:]
    return np.abs(L)


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("name", ["chain", "quadruped", "humanoid"])
def test_variant_sampled_knots_match_oracle(name, mode):
    """Positions as in the Hermite case; a slope inherits the position knots'
    tolerance through the positions -> slopes map (the quadratic recurrence
    carries every earlier error forward, scaled by 2 / Delta), plus its own
    float rounding, 1e-5 max(1, |x|)."""
    m, p, s, model, c = _ctrl(name, mode, n_samples=21)
    nom = _nominal(m, p)
    K, nu = p["n_knots"], m["n_u"]
    delta = p["horizon"] * p["dt"] / (K - 1)
    L = _slope_map(mode, K, delta)
    out = torch.zeros((21, c.E), device="cuda")
    for it in range(p["n_iters"]):
        c.samples(_t(nom), it, 5, out)
        got = _np(out)
        for n in range(21):
            ref = O.sample_knots(m, p, nom, s, 5, it, n)
            tolq = 2e-6 * np.maximum(1.0, np.abs(ref[: K * nu])).reshape(K, nu)
            tolv = L @ tolq + 1e-5 * np.maximum(1.0, np.abs(ref[K * nu:])).reshape(K, nu)
            dq = np.abs(got[n, : K * nu] - ref[: K * nu]).reshape(K, nu)
            dv = np.abs(got[n, K * nu:] - ref[K * nu:]).reshape(K, nu)
            assert np.all(dq <= tolq) and np.all(dv <= tolv), (name, mode, it, n, (dq / tolq).max(), (dv / tolv).max())


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("name,count,H", [("chain", 32, 50), ("quadruped", 48, 20), ("humanoid", 32, 40)])
def test_variant_rollout_costs_strict(name, mode, count, H):
    m, p, s, model, c = _ctrl(name, mode, n_samples=count, horizon=H)
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
    print(f"{name} mode {mode} H={H}: identical contact sequences {same.sum()}/{count}, max rel err {rel[same].max():.2e}")
    assert same.mean() >= 0.9 and rel[same].max() <= 1e-3


@pytest.mark.parametrize("mode", [1, 2])
def test_variant_full_step_arm(mode):
    m, p, s, model, c = _ctrl("chain", mode)
    kn = O.spline_slopes(mode, synth.nominal_knots(m, p["n_knots"]), p["n_knots"], m["n_u"],
                         p["horizon"] * p["dt"] / (p["n_knots"] - 1))
    c.tick = 0
    E = c.E
    ko, best = torch.zeros(E, device="cuda"), torch.zeros(E, device="cuda")
    costs = torch.zeros((p["n_iters"], p["n_samples"]), device="cuda")
    c.step(_t(m["x0"]), _t(kn), ko, best, None, costs)
    r = O.step(m, p, m["x0"], kn, s, 0)
    rel = np.abs(_np(costs) - r["costs"]) / np.abs(r["costs"])
    kerr = np.abs(_np(ko) - r["knots"]) / np.maximum(1.0, np.abs(r["knots"]))
    berr = np.abs(_np(best) - r["best_knots"]) / np.maximum(1.0, np.abs(r["best_knots"]))
    print(f"arm mode {mode}: cost {rel.max():.2e} knots {kerr.max():.2e} best {berr.max():.2e}")
    assert rel.max() <= 1e-3 and kerr.max() <= 1e-4 and berr.max() <= 1e-4


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("name", ["chain", "quadruped"])
def test_variant_shift_matches_oracle(name, mode):
    m, p, s, model, c = _ctrl(name, mode)
    K, nu, H = p["n_knots"], m["n_u"], p["horizon"]
    kn = synth.f32(O.spline_slopes(mode, _nominal(m, p, 3).astype(np.float64), K, nu, H * p["dt"] / (K - 1)))
    for n in [0, 1, 5, H // 2, H + 3]:
        out = torch.zeros(c.E, device="cuda")
        c.shift_knots(_t(kn), n, out)
        ref = O.shift_knots(kn, K, nu, H, p["dt"], n, spline_mode=mode)
        err = np.abs(_np(out) - ref) / np.maximum(1.0, np.abs(ref))
        assert err.max() <= 1e-5, (name, mode, n, err.max())


@pytest.mark.parametrize("mode", [1, 2])
def test_variant_tick_equals_predict_shift_step(mode):
    m, p, s, model, c = _ctrl("quadruped", mode, n_samples=32)
    K, nu, H = p["n_knots"], m["n_u"], p["horizon"]
    best0 = synth.f32(O.spline_slopes(mode, _nominal(m, p, 4).astype(np.float64), K, nu, H * p["dt"] / (K - 1)))
    x = _t(m["x0"])
    c.tick = 2
    xp = torch.zeros_like(x)
    c.predict(x, _t(best0), 3, xp)
    k0 = torch.zeros(c.E, device="cuda")
    c.shift_knots(_t(best0), 3, k0)
    ko_a, best_a = torch.zeros(c.E, device="cuda"), torch.zeros(c.E, device="cuda")
    c.step(xp, k0, ko_a, best_a)
    c.tick = 2
    best_b = _t(best0)
    ko_b = torch.zeros(c.E, device="cuda")
    c.run_tick(x, 3, best_b, ko_b)
    assert np.array_equal(_np(ko_b), _np(ko_a)) and np.array_equal(_np(best_b), _np(best_a))


def test_spline_mode_is_validated():
    m, p, s = synth.config("chain", n_samples=8)
    p["spline_mode"] = 3
    with pytest.raises(mppi.MppiError):
        mppi.Controller(mppi.Model(m), p, s)
