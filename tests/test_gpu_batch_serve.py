"""GPU: batched stepping and continuous-batching serving.

* A batch of uneven grids (sizes, coefficients, equations, step counts) gives
  every instance exactly its solo result: FP64 equal to the oracle value for
  value, FP32 bit-identical to the solo FP32 run; graph replay and plain
  launches agree.
* Small binary32 instances run LDS-resident (all steps in one workgroup)
  with the same results as the windowed path and the solo run.
* The server returns, for each request of a mixed stream, exactly the result
  of the same request solved alone; admission respects the memory budget and
  a request larger than the budget fails cleanly.
"""
import time

import numpy as np
import pytest

from parity_util import make_solver, rand_state, run_oracle

pytestmark = pytest.mark.gpu

TRT = ((1.0, 0.0, 0.4), (0.0, -0.4, 0.0))


def batch_cases():
    rng = np.random.default_rng(44)
    cases = []
    for i in range(9):
        n = (int(rng.integers(20, 150)), int(rng.integers(12, 90)))
        dx = 1.0 / n[0]
        nu = float(rng.uniform(1e-3, 1e-2))
        dt = 0.5 * min(0.3 * dx * dx / nu, nu / 0.01)
        s = 2 * nu * dt / ((1.0 / 3.0) * dx * dx)
        a = ((s + 1) / 2, 1 - s, (s - 1) / 2)
        cases.append(dict(name="burgers%d" % i, lattice="D2Q9", eq="burgers", n=n, dx=dx, dt=dt, a=a,
                          steps=int(rng.integers(3, 19))))
    cases.append(dict(name="lcde", lattice="D2Q9", eq="lcde", n=(70, 37), u=(0.1, -0.07),
                      K=[[0.3, 0.04], [0.04, 0.2]], lambda_bar=1, a=(1.0, 0.0, 0.0), steps=11))
    cases.append(dict(name="nse-trt", lattice="D2Q9", eq="nse", n=(70, 37), rho0=1.0,
                      kind="three_level", a=TRT[0], ah=TRT[1], steps=9))
    cases.append(dict(name="nse-trt-b", lattice="D2Q9", eq="nse", n=(33, 65), rho0=1.0,
                      kind="three_level", a=TRT[0], ah=TRT[1], steps=4))
    return cases


def _states(cases, seed=3):
    rng = np.random.default_rng(seed)
    return [(rand_state(c, rng), rand_state(c, rng)) for c in cases]


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_fp64_matches_oracle(M, use_graph):
    cases = batch_cases()
    states = _states(cases)
    solvers = []
    b = M.Batch(use_graph=use_graph)
    for c, (cur, prev) in zip(cases, states):
        s = make_solver(M, c, "fp64")
        s.set_state(cur)
        if c.get("kind") == "three_level":
            s.set_state(prev, level=1)
        b.add(s, c["steps"])
        solvers.append(s)
    b.run()
    b.wait()
    b.run()  # a second run continues from the advanced states (graph replay)
    b.wait()
    st = b.stats()
    # one launch per step of each group (burgers, lcde, nse) while any member runs
    groups = {}
    for c in cases:
        groups[c["eq"]] = max(groups.get(c["eq"], 0), c["steps"])
    assert st["launches"] == sum(groups.values())
    for c, (cur, prev), s in zip(cases, states, solvers):
        want = run_oracle(c, cur, prev, 2 * c["steps"])
        got = s.get_state()
        assert np.array_equal(got, want), c["name"]
    b.close()
    for s in solvers:
        s.close()


def test_batch_fp32_equals_solo(M):
    cases = batch_cases()
    states = _states(cases, seed=4)
    solo = []
    for c, (cur, prev) in zip(cases, states):
        s = make_solver(M, c, "fp32")
        s.set_state(cur.astype(np.float32))
        if c.get("kind") == "three_level":
            s.set_state(prev.astype(np.float32), level=1)
        s.step(c["steps"])
        solo.append(s.get_state())
        s.close()
    b = M.Batch()
    solvers = []
    for c, (cur, prev) in zip(cases, states):
        s = make_solver(M, c, "fp32")
        s.set_state(cur.astype(np.float32))
        if c.get("kind") == "three_level":
            s.set_state(prev.astype(np.float32), level=1)
        b.add(s, c["steps"])
        solvers.append(s)
    b.run()
    b.wait()
    for c, s, want in zip(cases, solvers, solo):
        assert np.array_equal(s.get_state(), want), c["name"]
    b.close()
    for s in solvers:
        s.close()


def _resident_cases():
    rng = np.random.default_rng(45)
    cases = []
    for i, n in enumerate([(64, 64), (143, 143), (100, 37), (3, 5), (150, 140), (200, 160)]):
        dx = 1.0 / n[0]
        nu = float(rng.uniform(1e-3, 1e-2))
        dt = 0.5 * min(0.3 * dx * dx / nu, nu / 0.01)
        sp = 2 * nu * dt / ((1.0 / 3.0) * dx * dx)
        a = ((sp + 1) / 2, 1 - sp, (sp - 1) / 2)
        cases.append(dict(name="burgers-%dx%d" % n, lattice="D2Q9", eq="burgers", n=n, dx=dx, dt=dt,
                          a=a, steps=int(rng.integers(5, 40))))
    cases.append(dict(name="lcde-d2q5", lattice="D2Q5", eq="lcde", n=(90, 61), u=(0.1, -0.07),
                      K=[[0.25, 0.0], [0.0, 0.25]], lambda_bar=1, a=(1.0, 0.0, 0.0), steps=17))
    cases.append(dict(name="lcde-d2q9-zero", lattice="D2Q9", eq="lcde", n=(40, 30), u=(0.1, -0.07),
                      K=[[0.3, 0.04], [0.04, 0.2]], lambda_bar=1, a=(1.0, 0.0, 0.0), steps=0))
    return cases


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_resident_equals_solo(M, use_graph):
    """Small binary32 instances (two levels within LDS) run LDS-resident, all
    steps in one workgroup, beside the windowed launches of the large ones:
    every instance's state equals the solo run's bit for bit, with the
    resident path on and off; a resident instance also holds the level one
    step before it, as a run of single steps does (a blocked run holds the
    level its last launch started from)."""
    cases = _resident_cases()
    states = _states(cases, seed=6)
    solo = []
    for c, (cur, _) in zip(cases, states):
        s = make_solver(M, c, "fp32")
        s.set_blocking(1)
        s.set_state(cur.astype(np.float32))
        s.step(c["steps"])
        solo.append((s.get_state(), s.get_state(level=1)))
        s.close()
    for resident in (True, False):
        b = M.Batch(use_graph=use_graph)
        b.set_resident(20480 if resident else 0)
        solvers = []
        for c, (cur, _) in zip(cases, states):
            s = make_solver(M, c, "fp32")
            s.set_state(cur.astype(np.float32))
            b.add(s, c["steps"])
            solvers.append(s)
        b.run()
        b.wait()
        # every instance of at most 20480 nodes with steps to take
        want_res = sum(1 for c in cases if c["steps"] > 0 and c["n"][0] * c["n"][1] <= 20480
                       and min(c["n"]) >= 3)
        assert b.resident() == (want_res if resident else 0)
        for c, s, (w0, w1) in zip(cases, solvers, solo):
            assert np.array_equal(s.get_state(), w0), (c["name"], resident)
            if resident and c["steps"] > 0 and c["n"][0] * c["n"][1] <= 20480:
                assert np.array_equal(s.get_state(level=1), w1), c["name"]
        # a second run continues from the levels the first left
        b.run()
        b.wait()
        b.close()
        for s in solvers:
            s.close()


def _request(M, c, state, out, exclude=False, precision="fp32", prev=None, timeout_s=0.0):
    return M.make_request(c["lattice"], c["eq"], c["n"], c.get("dx", 1.0), c.get("dt", 1.0), c["a"],
                          c["steps"], state, ah=c.get("ah"), kind=c.get("kind", "two_level"),
                          precision=precision, u=c.get("u", ()), K=c.get("K"),
                          lambda_bar=c.get("lambda_bar", 0), rho0=c.get("rho0", 0.0),
                          result_out=out, exclude=exclude, prev0=prev, timeout_s=timeout_s)


def test_server_alone_equals_mixed(M):
    cases = batch_cases()
    states = [s.astype(np.float32) for s, _ in _states(cases, seed=5)]
    # alone: one request at a time through its own server
    alone = []
    for c, st in zip(cases, states):
        srv = M.Server(hbm_budget_bytes=1 << 30, max_slots=4, quantum_steps=5)
        out = np.empty_like(st)
        srv.submit(_request(M, c, st, out), keep=(st, out))
        srv.drain(60)
        alone.append(out)
        srv.close()
    # mixed: all requests, staggered arrivals, small quantum so they overlap
    srv = M.Server(hbm_budget_bytes=1 << 30, max_slots=64, quantum_steps=3)
    outs = []
    tickets = []
    for c, st in zip(cases, states):
        out = np.empty_like(st)
        outs.append(out)
        tickets.append(srv.submit(_request(M, c, st, out), keep=(st, out)))
        time.sleep(0.002)
    srv.drain(60)
    for t in tickets:
        state, lat, rc = srv.poll(t)
        assert state == 2 and rc == 0 and lat > 0
    stats = srv.stats()
    assert stats["completed"] == len(cases) and stats["p99_s"] >= stats["p50_s"] > 0
    srv.close()
    for c, a, m in zip(cases, alone, outs):
        assert np.array_equal(a, m), c["name"]


def test_server_budget(M):
    c = batch_cases()[0]
    st = np.random.default_rng(1).uniform(-0.5, 0.5, c["n"][0] * c["n"][1]).astype(np.float32)
    out0 = np.empty_like(st)
    one = M.server_request_bytes(_request(M, c, st, out0))
    assert one > 3 * st.nbytes
    srv = M.Server(hbm_budget_bytes=2 * one, max_slots=16, quantum_steps=2)
    outs = [np.empty_like(st) for _ in range(6)]
    ts = [srv.submit(_request(M, c, st, o), keep=(st, o)) for o in outs]
    big = dict(c, n=(400, 400))
    bst = np.zeros(400 * 400, dtype=np.float32)
    bout = np.empty_like(bst)
    tb = srv.submit(_request(M, big, bst, bout), keep=(bst, bout))
    srv.drain(60)
    for t in ts:
        assert srv.poll(t)[0] == 2
    state, _, rc = srv.poll(tb)
    assert state == -1 and rc == M.MFD_E_BUDGET
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    srv.close()


@pytest.mark.parametrize("plan", [(4, 32), (6, 48), (2, 128), (3, 32)])
def test_batch_blocked_fp64_matches_oracle(M, plan):
    """Blocked batch launches (Burgers and LCDE groups; NSE groups when the
    window is one of the NSE kernel's, 32 or 64 rows) give every instance its
    oracle result, across two runs (graph replay), with launches = sum over
    groups of ceil(steps / tb) for blocked groups, steps for the others."""
    print("plan", plan, flush=True)
    cases = batch_cases()
    states = _states(cases, seed=9)
    solvers = []
    b = M.Batch(use_graph=True)
    b.set_plan(*plan)
    for c, (cur, prev) in zip(cases, states):
        s = make_solver(M, c, "fp64")
        s.set_state(cur)
        if c.get("kind") == "three_level":
            s.set_state(prev, level=1)
        b.add(s, c["steps"])
        solvers.append(s)
    b.run()
    b.wait()
    b.run()
    b.wait()
    groups = {}
    for c in cases:
        groups[c["eq"]] = max(groups.get(c["eq"], 0), c["steps"])
    tb = plan[0]
    nse_blocked = plan[1] in (32, 64) and 2 * 4 * plan[1] * 64 * 8 <= 160 * 1024

    def launches(eq, m):
        return -(-m // tb) if (eq != "nse" or nse_blocked) else m
    want_launches = sum(launches(eq, m) for eq, m in groups.items())
    assert b.stats()["launches"] == want_launches
    for c, (cur, prev), s in zip(cases, states, solvers):
        want = run_oracle(c, cur, prev, 2 * c["steps"])
        assert np.array_equal(s.get_state(), want), c["name"]
    b.close()
    for s in solvers:
        s.close()


def _lane_cases():
    """Burgers (beta = 1) and LCDE grids from smaller than the 128-column
    window to several windows wide, ragged step counts."""
    cases = batch_cases()[:10]
    rng = np.random.default_rng(46)
    for i, n in enumerate([(300, 140), (129, 200), (64, 64), (257, 33)]):
        dx = 1.0 / n[0]
        nu = float(rng.uniform(1e-3, 1e-2))
        dt = 0.5 * min(0.3 * dx * dx / nu, nu / 0.01)
        sp = 2 * nu * dt / ((1.0 / 3.0) * dx * dx)
        cases.append(dict(name="burgers-w%d" % i, lattice="D2Q9", eq="burgers", n=n, dx=dx, dt=dt,
                          a=((sp + 1) / 2, 1 - sp, (sp - 1) / 2), steps=int(rng.integers(20, 41))))
    cases.append(dict(name="lcde-w", lattice="D2Q9", eq="lcde", n=(260, 150), u=(0.1, -0.07),
                      K=[[0.3, 0.04], [0.04, 0.2]], lambda_bar=1, a=(1.0, 0.0, 0.0), steps=29))
    cases.append(dict(name="lcde-d2q5", lattice="D2Q5", eq="lcde", n=(150, 99), u=(0.1, -0.07),
                      K=[[0.3, 0.0], [0.0, 0.2]], lambda_bar=1, a=(1.0, 0.0, 0.0), steps=17))
    return cases


@pytest.mark.parametrize("plan", [(4, 48, 128), (8, 64, 128), (12, 112, 128), (2, 16, 128),
                                  (16, 128, 128)])
def test_batch_lane_fp32_equals_solo(M, plan):
    """Batched 128-column lane-shared windows (persistent workgroups over the
    tile table, modular wrap for grids narrower than the window) give every
    Burgers and LCDE instance the result of stepping it alone, bit for bit,
    across two runs (graph replay)."""
    print("plan", plan, flush=True)
    cases = _lane_cases()
    states = _states(cases, seed=13)
    solo = []
    for c, (cur, _) in zip(cases, states):
        s = make_solver(M, c, "fp32")
        s.set_blocking(1)
        s.set_state(cur.astype(np.float32))
        s.step(2 * c["steps"])
        solo.append(s.get_state())
        s.close()
    b = M.Batch(use_graph=True)
    b.set_plan(*plan)
    solvers = []
    for c, (cur, _) in zip(cases, states):
        s = make_solver(M, c, "fp32")
        s.set_state(cur.astype(np.float32))
        b.add(s, c["steps"])
        solvers.append(s)
    for _ in range(2):
        b.run()
        b.wait()
    for g in range(2):  # the Burgers and the D2Q9 LCDE groups use the lane kernel
        assert b.plan(g) == plan, (g, b.plan(g))
    for c, s, want in zip(cases, solvers, solo):
        assert np.array_equal(s.get_state(), want), c["name"]
    b.close()
    for s in solvers:
        s.close()


def test_batch_lane_plan_falls_back_for_fp64(M):
    """A 128-column plan asked of binary64 groups runs them in 64-column
    windows; results equal the oracle."""
    cases = _lane_cases()[:3]
    states = _states(cases, seed=14)
    b = M.Batch()
    b.set_plan(4, 48, 128)
    solvers = []
    for c, (cur, _) in zip(cases, states):
        s = make_solver(M, c, "fp64")
        s.set_state(cur)
        b.add(s, c["steps"])
        solvers.append(s)
    b.run()
    b.wait()
    assert b.plan(0) == (4, 48, 64)
    for c, (cur, prev), s in zip(cases, states, solvers):
        assert np.array_equal(s.get_state(), run_oracle(c, cur, prev, c["steps"])), c["name"]
    b.close()
    for s in solvers:
        s.close()
    with pytest.raises(M.MfdError):
        M.Batch().set_plan(4, 48, 96)


def test_batch_autotune_fp32_equals_solo(M):
    """The batch autotuner leaves every state as it was, and the run under the
    plan it picks equals each instance stepped alone, bit for bit."""
    cases = batch_cases()
    states = _states(cases, seed=10)
    solo = []
    for c, (cur, prev) in zip(cases, states):
        s = make_solver(M, c, "fp32")
        s.set_blocking(1)
        s.set_state(cur.astype(np.float32))
        if c.get("kind") == "three_level":
            s.set_state(prev.astype(np.float32), level=1)
        s.step(c["steps"])
        solo.append(s.get_state())
        s.close()
    b = M.Batch()
    solvers = []
    for c, (cur, prev) in zip(cases, states):
        s = make_solver(M, c, "fp32")
        s.set_state(cur.astype(np.float32))
        if c.get("kind") == "three_level":
            s.set_state(prev.astype(np.float32), level=1)
        b.add(s, c["steps"])
        solvers.append(s)
    before = [(s.get_state(), s.reduce()) for s in solvers]
    b.autotune()
    for s, (st, red) in zip(solvers, before):
        assert np.array_equal(s.get_state(), st)
        assert s.reduce() == red
    b.run()
    b.wait()
    for c, s, want in zip(cases, solvers, solo):
        assert np.array_equal(s.get_state(), want), c["name"]
    b.close()
    for s in solvers:
        s.close()


def test_server_concurrent_submitters(M):
    """Requests submitted from four threads at once each come back equal to
    the same request solved alone."""
    import threading
    cases = batch_cases()
    states = [s.astype(np.float32) for s, _ in _states(cases, seed=12)]
    alone = []
    for c, st in zip(cases, states):
        srv = M.Server(hbm_budget_bytes=1 << 30, max_slots=4, quantum_steps=4)
        out = np.empty_like(st)
        srv.submit(_request(M, c, st, out), keep=(st, out))
        srv.drain(60)
        alone.append(out)
        srv.close()
    srv = M.Server(hbm_budget_bytes=1 << 30, max_slots=64, quantum_steps=3)
    outs = [np.empty_like(st) for st in states]
    tickets = [None] * len(cases)

    def submit(idx):
        for i in idx:
            tickets[i] = srv.submit(_request(M, cases[i], states[i], outs[i]), keep=(states[i], outs[i]))

    parts = [list(range(k, len(cases), 4)) for k in range(4)]
    threads = [threading.Thread(target=submit, args=(p,)) for p in parts]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    srv.drain(60)
    for t in tickets:
        assert srv.poll(t)[0] == 2
    srv.close()
    for c, a, m in zip(cases, alone, outs):
        assert np.array_equal(a, m), c["name"]
