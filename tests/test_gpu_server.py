"""GPU tests of the continuous-batching server: a request's result does not
depend on what else is in the batch, the batched FP32 path matches the plain
single-system path, requests join a running batch, and cancellation and
budget refusal leave the other requests intact."""
import time

import numpy as np
import pytest

import paper_1310_6143_amd as sl
from spin_systems import sc_request_system, fcc_nanoparticle
from tests.gpu_util import max_angle

pytestmark = pytest.mark.gpu


def _mix():
    return [
        sc_request_system(12, 300.0, [0.0, 0.0, 0.5], 300, 1001),
        sc_request_system(9, 800.0, [0.3, 0.0, 0.0], 170, 1002),
        sc_request_system(20, 100.0, [0.0, 1.0, 0.0], 250, 1003),
        sc_request_system(7, 0.0, [0.0, 0.0, -1.0], 90, 1004),
    ]


def test_result_alone_equals_result_in_mix_bitwise():
    reqs = _mix()
    alone = []
    with sl.Server(hbm_budget=1 << 30, chunk_steps=32) as srv:
        for w in reqs:
            t = srv.submit(w, n_avg=50, record=True)
            r = srv.wait(t, 120)
            assert r["state"] == "done"
            alone.append((r, srv.fetch(t)))
    with sl.Server(hbm_budget=1 << 30, chunk_steps=32) as srv:
        tickets = [srv.submit(w, n_avg=50, record=True) for w in reqs]
        for (ra, (Sa, ma, Ea)), t in zip(alone, tickets):
            r = srv.wait(t, 120)
            S, m, E = srv.fetch(t)
            assert np.array_equal(S, Sa)
            assert np.array_equal(m, ma) and np.array_equal(E, Ea)
            assert r["E"] == ra["E"] and np.array_equal(r["m"], ra["m"])
            assert r["avg"]["m_abs"] == ra["avg"]["m_abs"]


def test_server_matches_single_system_path_bitwise():
    """With the same tiling (the server always uses the largest tile) the
    server and the single-system path give the same result bit for bit.
    Requests carry no lattice declaration, so both take the two-launch step."""
    w = sc_request_system(10, 400.0, [0.1, 0.2, 0.3], 200, 77)
    with sl.Server(hbm_budget=1 << 30, chunk_steps=64) as srv:
        t = srv.submit(w, record=True)
        srv.wait(t, 120)
        S, m, E = srv.fetch(t)
    with sl.from_workload(w, precision=sl.FP32, lattice=False) as g:
        g.set_option("tile_sites", 2048)
        m2, E2 = g.integrate(200)
        S2 = g.get_spins()
    assert np.array_equal(S, S2) and np.array_equal(m, m2) and np.array_equal(E, E2)


def test_batched_fp32_vs_plain_fp64_stated_accuracy():
    """Deterministic (T = 0) requests: FP32 batched serving vs the plain FP64
    single-system path after 1000 steps; bound 1e-4 rad per spin."""
    reqs = [sc_request_system(L, 0.0, H, 1000, 5) for L, H in
            ((8, [0.5, 0.0, -2.0]), (11, [0.0, 1.5, 0.5]), (14, [2.0, 0.0, 0.0]))]
    rng = np.random.default_rng(0)
    starts = []
    for w in reqs:
        S0 = np.tile([0.3, 0.1, 1.0], (w.n, 1)) + 0.2 * rng.standard_normal((w.n, 3))
        starts.append(S0 / np.linalg.norm(S0, axis=1, keepdims=True))
    with sl.Server(hbm_budget=1 << 30, chunk_steps=64) as srv:
        tickets = [srv.submit(w, S0=S0) for w, S0 in zip(reqs, starts)]
        got = []
        for t in tickets:
            srv.wait(t, 120)
            got.append(srv.fetch(t)[0])
    for w, S0, S32 in zip(reqs, starts, got):
        w.S0 = S0
        with sl.from_workload(w, precision=sl.FP64) as g:
            g.integrate(1000, record=False)
            S64 = g.get_spins()
        ang = max_angle(S32, S64)
        print(f"L={round(w.n ** (1 / 3))}: FP32 batched vs FP64 max angle {ang:.2e}")
        assert ang < 1e-4


def test_late_request_joins_running_batch():
    long = sc_request_system(24, 300.0, [0, 0, 0], 6000, 11)
    short = sc_request_system(8, 300.0, [0, 0, 0], 200, 12)
    with sl.Server(hbm_budget=1 << 30, chunk_steps=32) as srv:
        t_long = srv.submit(long)
        time.sleep(0.05)
        assert srv.poll(t_long)["state"] == "running"
        t_short = srv.submit(short)
        rs = srv.wait(t_short, 120)
        rl_mid = srv.poll(t_long)
        rl = srv.wait(t_long, 300)
        assert rs["state"] == "done" and rl["state"] == "done"
        assert rs["t_done"] < rl["t_done"]
        assert rl_mid["state"] == "running"          # short finished while long still ran
        assert rs["t_start"] > rl["t_start"]


def test_cancel_and_budget():
    big = sc_request_system(40, 300.0, [0, 0, 0], 200000, 1)
    small = sc_request_system(8, 300.0, [0, 0, 0], 100, 2)
    with sl.Server(hbm_budget=64 << 20, chunk_steps=32) as srv:
        t_big = srv.submit(big)
        time.sleep(0.05)
        srv.cancel(t_big)
        r = srv.wait(t_big, 60)
        assert r["state"] == "cancelled"
        t_small = srv.submit(small)
        assert srv.wait(t_small, 60)["state"] == "done"
        too_big = sc_request_system(48, 300.0, [0, 0, 0], 100, 3)
        with pytest.raises(sl.SllgError) as e:
            with sl.Server(hbm_budget=2 << 20, chunk_steps=32) as tiny:
                tiny.submit(too_big)
        assert e.value.name == "SLLG_E_BUDGET"
        st = srv.stats()
        assert st["cancelled"] == 1 and st["completed"] == 1


def test_queue_drains_when_budget_admits_one_at_a_time():
    # with a budget of 1.5 requests the requests must run one after another,
    # in arrival order
    reqs = [sc_request_system(40, 200.0, [0, 0, 0], 150, 40 + k) for k in range(4)]
    with sl.Server(hbm_budget=1 << 30, chunk_steps=32) as probe:
        size = probe.wait(probe.submit(reqs[0]), 60)["hbm_bytes"]
    assert size > 1 << 20
    with sl.Server(hbm_budget=int(1.5 * size), chunk_steps=32) as srv:
        tickets = [srv.submit(w) for w in reqs]
        res = [srv.wait(t, 120) for t in tickets]
        assert all(r["state"] == "done" for r in res)
        for k in range(1, len(res)):
            assert res[k]["t_start"] >= res[k - 1]["t_done"] - 1e-6
        assert srv.stats()["hbm_in_use"] == 0


def test_ragged_per_site_request():
    w = fcc_nanoparticle(radius_nm=1.4, temperature=50.0)
    w.n_steps = 120
    with sl.Server(hbm_budget=1 << 30, chunk_steps=16) as srv:
        t = srv.submit(w, record=True)
        srv.wait(t, 60)
        S, m, E = srv.fetch(t)
    with sl.from_workload(w, precision=sl.FP32) as g:
        m2, E2 = g.integrate(120)
        assert np.array_equal(S, g.get_spins()) and np.array_equal(E, E2)


def test_server_tunes_launch_shapes_per_composition():
    """Every new batch composition times the launch shapes on its own chunks
    and keeps the fastest; results stay those of the single-system path."""
    reqs = [sc_request_system(14, 300.0, [0.0, 0.0, 0.5], 2000, 3000 + k) for k in range(3)]
    with sl.Server(hbm_budget=1 << 30, chunk_steps=32) as srv:
        tickets = [srv.submit(w, record=True) for w in reqs]
        results = [srv.wait(t, 300) for t in tickets]
        st = srv.stats()
        got = [srv.fetch(t) for t in tickets]
    assert all(r["state"] == "done" for r in results)
    assert st["tuned_compositions"] >= 1
    assert st["last_xcd_remap"] in (0, 1, 2) and st["last_tile_order"] in (0, 1)
    for w, (S, m, E) in zip(reqs, got):
        with sl.from_workload(w, precision=sl.FP32, lattice=False) as g:
            g.set_option("tile_sites", 2048)
            m2, E2 = g.integrate(2000)
            assert np.array_equal(S, g.get_spins())
            assert np.array_equal(m, m2) and np.array_equal(E, E2)
