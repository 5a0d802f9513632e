"""mppi_update_noalloc -- the weights and weighted knot update with the library's
fixed device scratch, for callers that cannot allocate -- against
mppi_debug_update, the same update with a context's own buffers.  Two calls in a
row, the second with a smaller input (fewer samples, a shorter knot vector that
is not a multiple of four floats, raw weights): weights within 1e-6 and knots
within 1e-4 max(1, |x|) of the context's update, and of the oracle's."""
import numpy as np
import pytest

import oracle as O
from paper_2511_19204_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2511_19204_amd import mppi


def _t(x):
    return torch.tensor(np.asarray(x), dtype=torch.float32, device="cuda")


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _case(name, N, n_knots, weight_mode, seed):
    m, p, s = synth.config(name, n_samples=N)
    p = dict(p)
    p["n_knots"] = n_knots
    p["weight_mode"] = weight_mode
    model = mppi.Model(m)
    c = mppi.Controller(model, p, s)
    rng = np.random.default_rng(seed)
    E = c.E
    nom = synth.f32(rng.normal(0.0, 0.3, E))
    smp = synth.f32(rng.normal(0.0, 0.3, (N, E)))
    S = synth.f32(rng.exponential(200.0, N) + 500.0)
    S[N // 3] = np.inf
    S[N - 2] = np.nan
    return m, p, c, model, E, nom, smp, S


def test_noalloc_update_matches_the_context_update_twice():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    mppi.lib()
    cases = [("quadruped", 4097, 8, 0, 1), ("chain", 100, 3, 1, 2)]   # second: smaller, E = 18
    for name, N, K, mode, seed in cases:
        m, p, c, model, E, nom, smp, S = _case(name, N, K, mode, seed)
        d_S, d_smp, d_nom = _t(S), _t(smp), _t(nom)
        ref_k = torch.zeros(E, device="cuda")
        ref_w = torch.zeros(N, device="cuda")
        c.update(d_S, d_smp, d_nom, ref_k, ref_w)
        got_k = torch.full((E,), float("nan"), device="cuda")
        got_w = torch.full((N,), float("nan"), device="cuda")
        mppi.update_noalloc(N, E, p["lambda"], mode, d_S, d_smp, d_nom, got_k, got_w)
        gk, gw, rk, rw = _np(got_k), _np(got_w), _np(ref_k), _np(ref_w)
        assert np.max(np.abs(gw - rw)) <= 1e-6, name
        assert np.max(np.abs(gk - rk) / np.maximum(1.0, np.abs(rk))) <= 1e-4, name
        print(f"{name} N={N} E={E}: bit-identical to the context's update: "
              f"{np.array_equal(gk, rk) and np.array_equal(gw, rw)}")
        wo, nstar, nf = O.weights(S.astype(np.float64), p["lambda"], mode)
        ko = O.weighted_average(wo, smp.astype(np.float64))
        assert np.max(np.abs(gw - wo)) <= 1e-6, name
        assert np.max(np.abs(gk - ko) / np.maximum(1.0, np.abs(ko))) <= 1e-4, name


def test_noalloc_update_keeps_the_nominal_when_no_cost_is_finite():
    torch.cuda.set_device(0)
    m, p, c, model, E, nom, smp, S = _case("quadruped", 300, 8, 0, 3)
    out = torch.zeros(E, device="cuda")
    mppi.update_noalloc(300, E, p["lambda"], 0, _t(np.full(300, np.inf)), _t(smp), _t(nom), out)
    assert np.array_equal(_np(out), nom.astype(np.float32))
