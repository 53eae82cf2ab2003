"""The serving scheduler on the CPU: the library's admission rule and arena,
driven by a fake executor (wipes_serve_simulate; no device work)."""
import numpy as np
import pytest

from paper_2508_12615_amd.serve import simulate

MB = 1 << 20


def cfg(**kw):
    c = dict(max_slots=8, max_pending=1000, max_batch=4, persistent=1, hbm_budget_bytes=1024 * MB)
    c.update(kw)
    return c


def test_all_complete_in_fifo_admission_order():
    g = np.random.default_rng(0)
    n = 300
    t = np.cumsum(g.exponential(0.002, n))
    out = simulate(cfg(), t, g.integers(1, 200, n) * MB, np.full(n, 0.0005), g.uniform(0.001, 0.004, n))
    assert np.all(out["t_done"] > out["t_admit"]) and np.all(out["t_admit"] >= t - 1e-12)
    assert np.all(np.diff(out["t_admit"]) >= 0)             # FIFO: admission order = arrival order
    assert np.all(np.diff(out["batch"]) >= 0)


def test_budget_is_never_exceeded_and_binds():
    g = np.random.default_rng(1)
    n = 200
    t = np.zeros(n)                                          # everything arrives at once
    fp = g.integers(100, 400, n) * MB
    out = simulate(cfg(hbm_budget_bytes=1000 * MB, max_slots=64, max_batch=16), t, fp, np.full(n, 1e-3),
                   np.full(n, 2e-3))
    assert out["arena_peak"] <= 1000 * MB
    # with this budget at most a few requests fit at a time, so later ones wait
    assert np.max(np.bincount(out["batch"])) <= 9
    assert out["t_admit"][-1] > 0


def test_slots_limit_concurrency():
    n = 64
    out = simulate(cfg(max_slots=4, max_batch=4), np.zeros(n), np.full(n, MB), np.full(n, 1e-3), np.full(n, 1e-3))
    events = sorted([(a, 1) for a in out["t_admit"]] + [(d, -1) for d in out["t_done"]], key=lambda e: (e[0], e[1]))
    live = np.cumsum([e[1] for e in events])
    assert live.max() <= 4


def test_continuous_batching_admits_during_blend():
    """A request arriving while a long blend runs is admitted before that blend completes
    (its preparation overlaps), instead of waiting for the queue to drain."""
    t = np.array([0.0, 0.001])
    out = simulate(cfg(), t, np.full(2, MB), np.array([0.0005, 0.0005]), np.array([0.05, 0.01]))
    assert out["t_admit"][1] < out["t_done"][0]
    assert out["batch"][1] == 1
    # its blend queues behind the first on the blend stream
    assert out["t_done"][1] >= out["t_done"][0]


def test_head_of_line_request_is_not_starved():
    """A large request at the head waits for memory but is not overtaken by later small ones."""
    t = np.array([0.0, 0.0001, 0.0002, 0.0003])
    fp = np.array([600, 900, 10, 10]) * MB
    out = simulate(cfg(hbm_budget_bytes=1000 * MB, max_batch=1), t, fp, np.full(4, 1e-3), np.full(4, 5e-3))
    assert out["t_admit"][1] >= out["t_done"][0] - 1e-12   # waited for the first to free memory
    assert out["t_admit"][2] >= out["t_admit"][1]           # not overtaken


def test_request_larger_than_budget_is_rejected():
    from paper_2508_12615_amd import binding as B
    with pytest.raises(B.WipesError):
        simulate(cfg(hbm_budget_bytes=100 * MB), np.zeros(1), np.array([200 * MB]), np.ones(1), np.ones(1))
