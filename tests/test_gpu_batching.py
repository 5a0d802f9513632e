"""Batching and serving on the GPU: persistent launches, graph replays, the
autotuner and the continuous-batching server.  Every path must reproduce the
instance's own plain mppi_step bit for bit (same kernels, fixed-order
reductions, device-resident ticks)."""
import time

import numpy as np
import pytest

from paper_2511_19204_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2511_19204_amd import mppi


def _t(x):
    return torch.tensor(np.asarray(x), dtype=torch.float32, device="cuda")


def _robots(n, seed=0):
    """A small uneven mix (chain / quadruped / humanoid, K and H vary)."""
    out = []
    for (m, p, s) in synth.serving_mix(n, seed=seed):
        p = dict(p)
        p["n_samples"] = min(p["n_samples"], 96)
        p["horizon"] = min(p["horizon"], 80)
        model = mppi.Model(m)
        out.append((m, p, s, model, mppi.Controller(model, p, s)))
    return out


def _buffers(robots):
    st = [_t(m["x0"]) for (m, p, s, model, c) in robots]
    ki = [_t(synth.nominal_knots(m, p["n_knots"])) for (m, p, s, model, c) in robots]
    ko = [torch.zeros_like(k) for k in ki]
    return st, ki, ko


def _plain_reference(robots, ticks):
    """Per-instance plain steps: knots after each of `ticks` warm-started steps."""
    refs = []
    for (m, p, s, model, c) in robots:
        c.tick = 0
        st = _t(m["x0"])
        k = _t(synth.nominal_knots(m, p["n_knots"]))
        seq = []
        for _ in range(ticks):
            out = torch.zeros_like(k)
            c.step(st, k, out)
            torch.cuda.synchronize()
            seq.append(out.cpu().numpy())
            k = out
        refs.append(seq)
    return refs


@pytest.fixture(scope="module")
def mix():
    robots = _robots(6)
    return robots, _plain_reference(robots, 3)


@pytest.mark.parametrize("persistent", [False, True])
def test_batched_steps_equal_plain_steps(mix, persistent):
    robots, refs = mix
    mppi.set_batch_options(persistent)
    try:
        for (*_, c) in robots:
            c.tick = 0
        st, ki, ko = _buffers(robots)
        ctrls = [c for (*_, c) in robots]
        for t in range(3):
            mppi.step_batch(ctrls, st, ki, ko)
            torch.cuda.synchronize()
            for i in range(len(robots)):
                assert np.array_equal(ko[i].cpu().numpy(), refs[i][t]), (persistent, t, i)
            ki = [k.clone() for k in ko]
    finally:
        mppi.set_batch_options(False)


@pytest.mark.parametrize("persistent", [False, True])
def test_graph_replays_equal_eager_steps(mix, persistent):
    """Replay the captured batch several times, with eager work and syncs between
    replays; every replay must equal the plain step of the same tick."""
    robots, refs = mix
    mppi.set_batch_options(persistent)
    try:
        for (*_, c) in robots:
            c.tick = 0
        st, ki, ko = _buffers(robots)
        ctrls = [c for (*_, c) in robots]
        g = mppi.Graph(ctrls, st, ki, ko)
        for t in range(3):
            g.launch()
            torch.cuda.synchronize()
            _ = torch.ones(1000, device="cuda").sum().item()  # unrelated eager work between replays
            for i in range(len(robots)):
                assert np.array_equal(ko[i].cpu().numpy(), refs[i][t]), (persistent, t, i)
            for i in range(len(robots)):
                ki[i].copy_(ko[i])  # warm start in place: the graph reads the same buffers
            torch.cuda.synchronize()
        g.close()
    finally:
        mppi.set_batch_options(False)


def test_autotune_picks_a_valid_lane_count_without_changing_results():
    m, p, s = synth.config("quadruped", n_samples=256)
    model = mppi.Model(m)
    c = mppi.Controller(model, p, s)
    st, k = _t(m["x0"]), _t(synth.nominal_knots(m, p["n_knots"]))
    c.tick = 5
    a = torch.zeros_like(k)
    c.step(st, k, a)
    c.tick = 5
    g = mppi.autotune(c, st, k, reps=2)
    assert g in (16, 32, 64) and c.lanes == g and c.tick == 5
    b = torch.zeros_like(k)
    c.step(st, k, b)
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


# one stream: the launches fork their rollout groups (one per lane count) onto side
# streams; several streams: no side streams, and in iteration mode each robot type
# owns a stream (with four streams and at most three types, at least one stream
# is owned by none and takes ticks of one type at a time)
SERVER_CASES = [("batched", 1), ("batched", 2), ("plain", 2), ("plain", 6), ("iteration", 1), ("iteration", 3),
                ("iteration", 4), ("iteration", 6)]


@pytest.mark.parametrize("mode,n_streams", SERVER_CASES)
def test_server_result_is_the_same_alone_and_in_the_mix(mix, mode, n_streams):
    """Robot 0 served alone, then in a mix where the other robots' ticks arrive in
    between (continuous batching): its knots after every tick equal the plain
    step's, and so do every other robot's."""
    robots, refs = mix
    assert len({c.lanes for (*_, c) in robots}) >= 2  # several rollout groups per launch
    srv = mppi.Server(n_streams=n_streams, max_batch=64, mode=mode)
    try:
        # alone
        (m0, p0, s0, model0, c0) = robots[0]
        c0.tick = 0
        st0 = _t(m0["x0"])
        k0 = _t(synth.nominal_knots(m0, p0["n_knots"]))
        for t in range(3):
            out = torch.zeros_like(k0)
            tk = srv.submit(c0, st0, k0, out)
            while srv.poll(tk) is None:
                time.sleep(1e-4)
            assert np.array_equal(out.cpu().numpy(), refs[0][t])
            k0 = out
        # in the mix: every robot submits 3 ticks, staggered, at most one outstanding each
        for (*_, c) in robots:
            c.tick = 0
        st, ki, _ = _buffers(robots)
        outs = [[torch.zeros_like(ki[i]) for _ in range(3)] for i in range(len(robots))]
        nxt = [0] * len(robots)
        live = {}
        rng = np.random.default_rng(0)
        while any(n < 3 for n in nxt) or live:
            for i in rng.permutation(len(robots)):
                if i not in live and nxt[i] < 3:
                    src = ki[i] if nxt[i] == 0 else outs[i][nxt[i] - 1]
                    live[i] = srv.submit(robots[i][4], st[i], src, outs[i][nxt[i]])
                    nxt[i] += 1
            for i in list(live):
                if srv.poll(live[i]) is not None:
                    del live[i]
            time.sleep(2e-4)
        srv.drain()
        for i in range(len(robots)):
            for t in range(3):
                assert np.array_equal(outs[i][t].cpu().numpy(), refs[i][t]), (mode, i, t)
        batches, requests = srv.stats()
        assert requests == 3 + 3 * len(robots)
        if mode == "batched":
            assert batches < requests  # ticks were batched together
        if mode == "iteration":  # a round per iteration, shared by the ticks in flight
            n_it = sum(r[1]["n_iters"] for r in robots)
            assert batches < 3 * (robots[0][1]["n_iters"] + n_it)
    finally:
        srv.close()


def test_server_three_streams_many_uneven_batches():
    """Regression: batches of very different sizes on three streams recycle the
    per-call launch-table buffers while earlier batches still run on other
    streams; a buffer may only be reused after the last kernel reading it ends.
    Every result must still equal the plain step."""
    robots = _robots(16, seed=3)
    ticks = 6
    refs = _plain_reference(robots, ticks)
    srv = mppi.Server(n_streams=3, max_batch=5, mode="batched")
    try:
        for (*_, c) in robots:
            c.tick = 0
        st, ki, _ = _buffers(robots)
        outs = [[torch.zeros_like(ki[i]) for _ in range(ticks)] for i in range(len(robots))]
        nxt = [0] * len(robots)
        live = {}
        rng = np.random.default_rng(1)
        while any(n < ticks for n in nxt) or live:
            for i in rng.permutation(len(robots))[: rng.integers(1, len(robots) + 1)]:
                if i not in live and nxt[i] < ticks:
                    src = ki[i] if nxt[i] == 0 else outs[i][nxt[i] - 1]
                    live[i] = srv.submit(robots[i][4], st[i], src, outs[i][nxt[i]])
                    nxt[i] += 1
            for i in list(live):
                if srv.poll(live[i]) is not None:
                    del live[i]
        srv.drain()
        for i in range(len(robots)):
            for t in range(ticks):
                assert np.array_equal(outs[i][t].cpu().numpy(), refs[i][t]), (i, t)
        batches, requests = srv.stats()
        assert requests == ticks * len(robots) and batches > 8
    finally:
        srv.close()


def _tick_reference(robots, ticks, delay):
    """Per-instance mppi_tick: (tau_best, nominal, step info) after each tick, the
    measured state being x0 at every tick."""
    refs = []
    for i, (m, p, s, model, c) in enumerate(robots):
        c.tick = 0
        x = _t(m["x0"])
        best = _t(synth.nominal_knots(m, p["n_knots"]))
        seq = []
        for t in range(ticks):
            ko = torch.zeros_like(best)
            info = torch.zeros(mppi.INFO_INTS, dtype=torch.int32, device="cuda")
            c.run_tick(x, delay(i, t, p), best, ko, info)
            torch.cuda.synchronize()
            seq.append((best.cpu().numpy().copy(), ko.cpu().numpy(), info.cpu().numpy()))
        refs.append(seq)
    return refs


@pytest.mark.parametrize("mode,n_streams", SERVER_CASES)
def test_server_ticks_equal_the_instance_ticks(mode, n_streams):
    """Served ticks (prediction by a per-tick delay, warm-start shift, iterations,
    tau_best carried on the device) of an uneven mix, submitted staggered with at
    most one outstanding per robot: every robot's tau_best, nominal and step info
    after every tick equal its own mppi_tick sequence bit for bit."""
    robots = _robots(10, seed=5)
    ticks = 3
    delay = lambda i, t, p: (i + 2 * t) % 5 if t != 1 else p["horizon"]  # includes 0 and the full horizon
    refs = _tick_reference(robots, ticks, delay)
    srv = mppi.Server(n_streams=n_streams, max_batch=6, mode=mode)
    try:
        for (*_, c) in robots:
            c.tick = 0
        xs = [_t(m["x0"]) for (m, *_rest) in robots]
        bests = [_t(synth.nominal_knots(m, p["n_knots"])) for (m, p, *_r) in robots]
        kos = [[torch.zeros_like(bests[i]) for _ in range(ticks)] for i in range(len(robots))]
        infos = [[torch.zeros(mppi.INFO_INTS, dtype=torch.int32, device="cuda") for _ in range(ticks)]
                 for _ in range(len(robots))]
        got_best = [[None] * ticks for _ in range(len(robots))]
        nxt = [0] * len(robots)
        live = {}
        rng = np.random.default_rng(2)
        while any(n < ticks for n in nxt) or live:
            for i in rng.permutation(len(robots)):
                if i not in live and nxt[i] < ticks:
                    t = nxt[i]
                    p = robots[i][1]
                    live[i] = (t, srv.submit_tick(robots[i][4], xs[i], delay(i, t, p), bests[i], kos[i][t],
                                                  infos[i][t]))
                    nxt[i] += 1
            for i in list(live):
                t, tk = live[i]
                if srv.poll(tk) is not None:
                    got_best[i][t] = bests[i].cpu().numpy().copy()
                    del live[i]
            time.sleep(2e-4)
        srv.drain()
        for i in range(len(robots)):
            for t in range(ticks):
                rb, rk, ri = refs[i][t]
                assert np.array_equal(got_best[i][t], rb), (mode, i, t, "best")
                assert np.array_equal(kos[i][t].cpu().numpy(), rk), (mode, i, t, "nominal")
                assert np.array_equal(infos[i][t].cpu().numpy(), ri), (mode, i, t, "info")
        with pytest.raises(mppi.MppiError):
            srv.submit_tick(robots[0][4], xs[0], robots[0][1]["horizon"] + 1, bests[0])
    finally:
        srv.close()
