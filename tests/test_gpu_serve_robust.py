"""GPU: served results against independent references, failure isolation,
cancellation, timeouts and the memory budget of the continuous-batching
server.

* FP64 requests of a mixed stream (Burgers, linear CDE, NSE three-level)
  come back equal to the FP64 oracle value for value.
* FP32 requests come back bit-identical to a plain solver run of the same
  request.
* A request whose state holds a NaN fails with MFD_E_UNSTABLE (the host-side
  finiteness check at retirement) and frees its slot; every other request of
  the same batches is bit-identical to its plain run.
* Cancelling a queued or a running request fails it with MFD_E_CANCELLED and
  frees its slot for the next request; a request past its timeout fails with
  MFD_E_TIMEOUT.
* A kind the server cannot batch (theta) is refused at submission.
* Under a budget that binds, the device bytes the library holds never exceed
  the budget (mfd_memory_stats).
"""
import time

import numpy as np
import pytest

from parity_util import run_gpu, run_oracle
from test_gpu_batch_serve import _request, _states, batch_cases

pytestmark = pytest.mark.gpu


def _serve(M, cases, states, precision, quantum=3, slots=64, budget=1 << 30, nan_at=None):
    dt = np.float64 if precision == "fp64" else np.float32
    srv = M.Server(hbm_budget_bytes=budget, max_slots=slots, quantum_steps=quantum)
    outs, tickets = [], []
    for i, (c, (cur, prev)) in enumerate(zip(cases, states)):
        st = cur.astype(dt)
        if nan_at is not None and i == nan_at:
            st[st.size // 3] = np.nan
        pv = prev.astype(dt) if c.get("kind") == "three_level" else None
        out = np.empty_like(st)
        outs.append(out)
        tickets.append(srv.submit(_request(M, c, st, out, precision=precision, prev=pv),
                                  keep=(st, pv, out)))
        time.sleep(0.001)
    srv.drain(120)
    polls = [srv.poll(t) for t in tickets]
    srv.close()
    return outs, polls


def test_server_fp64_matches_oracle(M):
    cases = batch_cases()
    states = _states(cases, seed=31)
    outs, polls = _serve(M, cases, states, "fp64")
    for c, (cur, prev), out, (state, _, rc) in zip(cases, states, outs, polls):
        assert state == 2 and rc == 0, c["name"]
        want = run_oracle(c, cur, prev, c["steps"])
        assert np.array_equal(out, want), c["name"]


def test_server_fp32_equals_plain_solver(M):
    cases = batch_cases()
    states = _states(cases, seed=32)
    outs, polls = _serve(M, cases, states, "fp32")
    for c, (cur, prev), out, (state, _, rc) in zip(cases, states, outs, polls):
        assert state == 2 and rc == 0, c["name"]
        want = run_gpu(M, c, cur.astype(np.float32), prev.astype(np.float32), c["steps"], "fp32")
        assert np.array_equal(out.astype(np.float64), want), c["name"]


def test_server_nan_request_fails_alone(M):
    cases = batch_cases()
    states = _states(cases, seed=33)
    bad = 2
    outs, polls = _serve(M, cases, states, "fp32", nan_at=bad)
    for i, (c, (cur, prev), out, (state, _, rc)) in enumerate(zip(cases, states, outs, polls)):
        if i == bad:
            assert state == -1 and rc == M.MFD_E_UNSTABLE, (state, rc)
            continue
        assert state == 2 and rc == 0, c["name"]
        want = run_gpu(M, c, cur.astype(np.float32), prev.astype(np.float32), c["steps"], "fp32")
        assert np.array_equal(out.astype(np.float64), want), c["name"]


def _long_case(steps):
    c = dict(batch_cases()[0])
    c.update(n=(64, 64), steps=steps, dx=1.0 / 64)
    nu = 5e-3
    dt = 0.5 * min(0.3 * c["dx"] ** 2 / nu, nu / 0.01)
    s = 2 * nu * dt / ((1.0 / 3.0) * c["dx"] ** 2)
    c.update(dt=dt, a=((s + 1) / 2, 1 - s, (s - 1) / 2))
    return c


def test_server_cancel_queued_and_running(M):
    rng = np.random.default_rng(7)
    long = _long_case(2_000_000)
    st = rng.uniform(-0.1, 0.1, 64 * 64).astype(np.float32)
    srv = M.Server(hbm_budget_bytes=1 << 30, max_slots=1, quantum_steps=8)
    o1, o2 = np.empty_like(st), np.empty_like(st)
    t1 = srv.submit(_request(M, long, st, o1), keep=(st, o1))
    t2 = srv.submit(_request(M, long, st, o2), keep=(st, o2))
    deadline = time.time() + 20
    while srv.poll(t1)[0] != 1 and time.time() < deadline:
        time.sleep(0.005)
    assert srv.poll(t1)[0] == 1          # running, t2 waits for the slot
    assert srv.poll(t2)[0] == 0
    assert srv.cancel(t2) == 0
    state, _, rc = srv.poll(t2)
    assert state == -1 and rc == M.MFD_E_CANCELLED
    assert srv.cancel(t1) == 0
    # the slot frees up for a new request, which completes normally
    short = dict(long, steps=20)
    o3 = np.empty_like(st)
    t3 = srv.submit(_request(M, short, st, o3), keep=(st, o3))
    srv.drain(30)
    state, _, rc = srv.poll(t1)
    assert state == -1 and rc == M.MFD_E_CANCELLED
    assert srv.poll(t3)[0] == 2
    assert srv.cancel(t3) == M.MFD_E_ORDER  # already done
    srv.close()
    want = run_gpu(M, short, st, st, 20, "fp32")
    assert np.array_equal(o3.astype(np.float64), want)


def test_server_timeout(M):
    rng = np.random.default_rng(8)
    long = _long_case(2_000_000)
    short = dict(long, steps=30)
    st = rng.uniform(-0.1, 0.1, 64 * 64).astype(np.float32)
    srv = M.Server(hbm_budget_bytes=1 << 30, max_slots=4, quantum_steps=8)
    o1, o2 = np.empty_like(st), np.empty_like(st)
    t1 = srv.submit(_request(M, long, st, o1, timeout_s=0.05), keep=(st, o1))
    t2 = srv.submit(_request(M, short, st, o2), keep=(st, o2))
    srv.drain(30)
    state, _, rc = srv.poll(t1)
    assert state == -1 and rc == M.MFD_E_TIMEOUT
    assert srv.poll(t2)[0] == 2
    srv.close()
    assert np.array_equal(o2.astype(np.float64), run_gpu(M, short, st, st, 30, "fp32"))


def test_server_refuses_theta(M):
    c = batch_cases()[9]  # the linear CDE case
    st = np.zeros(c["n"][0] * c["n"][1], dtype=np.float32)
    out = np.empty_like(st)
    srv = M.Server(hbm_budget_bytes=1 << 30, max_slots=4, quantum_steps=4)
    r = _request(M, c, st, out)
    r.kind = M.KINDS["theta"]
    with pytest.raises(M.MfdError) as ei:
        srv.submit(r, keep=(st, out))
    assert ei.value.code == M.MFD_E_UNSUPPORTED
    srv.close()


def test_server_budget_bounds_device_bytes(M):
    """Twelve requests through a budget that holds three at a time: all
    complete, and the library's device bytes stay within the budget."""
    rng = np.random.default_rng(9)
    c = dict(_long_case(40), n=(160, 144))
    N = 160 * 144
    states = [rng.uniform(-0.1, 0.1, N).astype(np.float32) for _ in range(12)]
    outs = [np.empty_like(s) for s in states]
    one = M.server_request_bytes(_request(M, c, states[0], outs[0]))
    budget = 3 * one + one // 2
    base, _ = M.memory_stats(reset_peak=True)
    srv = M.Server(hbm_budget_bytes=budget, max_slots=64, quantum_steps=8)
    ts = [srv.submit(_request(M, c, s, o), keep=(s, o)) for s, o in zip(states, outs)]
    srv.drain(60)
    _, peak = M.memory_stats()
    for t in ts:
        assert srv.poll(t)[0] == 2
    srv.close()
    assert peak - base <= budget, (peak - base, budget)
    assert peak - base > 2 * one  # the budget did bind (several requests at once)
    for s, o in zip(states, outs):
        assert np.array_equal(o.astype(np.float64), run_gpu(M, c, s, s, 40, "fp32"))
