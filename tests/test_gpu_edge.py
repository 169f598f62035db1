"""GPU: checkpoint / resume, degenerate calls and ordering errors.

* A run of N steps equals k steps, a checkpoint of the live levels (and the
  MesoFD populations) into host memory, a fresh solver restored from it, and
  N - k more steps: bit for bit, in every form and level count.
* Zero steps change nothing; empty batches and zero-step batch members run;
  a zero-step request comes back unchanged from the server.
* Calls out of order fail with MFD_E_ORDER, bad sizes with MFD_E_ARG.
* The growth check (mfd_set_check_interval) changes no result and stops a
  solve whose sums are not finite with MFD_E_UNSTABLE.
"""
import numpy as np
import pytest

from parity_util import make_solver, rand_state, run_oracle

pytestmark = pytest.mark.gpu

K2 = [[0.3, 0.04], [0.04, 0.2]]
TRT = ((1.0, 0.0, 0.4), (0.0, -0.4, 0.0))
EX13 = ((0.875, 0.0, 0.125), (0.125, 0.0, -0.125))

CASES = [
    dict(name="lcde-2l-blocked", lattice="D2Q9", n=(150, 77), eq="lcde", u=(0.1, -0.07), K=K2,
         lambda_bar=1, a=(1.0, 0.0, 0.0), plan=(4, 40, 64)),
    dict(name="lcde-3l-blocked", lattice="D2Q9", n=(150, 77), eq="lcde", u=(0.1, -0.07), K=K2,
         lambda_bar=1, kind="three_level", a=EX13[0], ah=EX13[1], plan=(6, 48, 128)),
    dict(name="nse-trt", lattice="D2Q9", n=(70, 37), eq="nse", rho0=1.0, kind="three_level",
         a=TRT[0], ah=TRT[1]),
    dict(name="nse-d3q19", lattice="D3Q19", n=(20, 13, 9), eq="nse", rho0=1.0, kind="three_level",
         a=TRT[0], ah=TRT[1]),
    dict(name="mesofd-nse-3l", lattice="D2Q9", n=(40, 33), eq="nse", rho0=1.0, kind="three_level",
         a=TRT[0], ah=TRT[1], form="mesofd"),
    dict(name="mesofd-lcde", lattice="D2Q9", n=(40, 33), eq="lcde", u=(0.1, -0.07), K=K2,
         lambda_bar=1, a=(1.0, 0.0, 0.0), form="mesofd"),
]


def _new(M, case, precision):
    s = make_solver(M, case, precision)
    if "plan" in case:
        s.set_plan(*case["plan"])
    return s


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: c["name"])
def test_checkpoint_resume(M, case, precision):
    print("case", case["name"], precision, flush=True)
    rng = np.random.default_rng(21)
    dt = np.float64 if precision == "fp64" else np.float32
    cur, prev = rand_state(case, rng).astype(dt), rand_state(case, rng).astype(dt)
    three = case.get("kind") == "three_level"
    meso = case.get("form") == "mesofd"
    N, k = 23, 9
    a = _new(M, case, precision)
    a.set_state(cur)
    if three:
        a.set_state(prev, level=1)
    a.step(N)
    want = a.get_state()
    a.close()
    b = _new(M, case, precision)
    b.set_state(cur)
    if three:
        b.set_state(prev, level=1)
    b.step(k)
    ck0 = b.get_state(populations=meso)
    ck1 = b.get_state(level=1) if three else None
    b.close()
    c = _new(M, case, precision)
    c.set_state(ck0, populations=meso)
    if three:
        c.set_state(ck1, level=1)
    c.step(N - k)
    got = c.get_state()
    c.close()
    assert np.array_equal(got, want)
    if precision == "fp64":
        assert np.array_equal(got, run_oracle(case, cur.astype(np.float64), prev.astype(np.float64), N))


def test_zero_steps_and_order_errors(M):
    case = CASES[0]
    s = make_solver(M, case, "fp64")
    with pytest.raises(M.MfdError) as e:
        s.step(1)
    assert e.value.code == M.MFD_E_ORDER
    with pytest.raises(M.MfdError) as e:
        s.get_state()
    assert e.value.code == M.MFD_E_ORDER
    with pytest.raises(M.MfdError) as e:
        s.set_state(np.zeros(7))
    assert e.value.code == M.MFD_E_ARG
    with pytest.raises(M.MfdError) as e:
        s.set_state(np.zeros(150 * 77), level=1)  # two-level schemes hold one level
    assert e.value.code == M.MFD_E_ARG
    x = np.random.default_rng(3).standard_normal(150 * 77)
    s.set_state(x)
    s.step(0)
    assert np.array_equal(s.get_state(), x)
    with pytest.raises(M.MfdError) as e:
        s.step(-1)
    assert e.value.code == M.MFD_E_ARG
    s.close()


def test_empty_and_zero_step_batches(M):
    b = M.Batch()
    b.run()
    b.autotune()
    b.wait()
    assert b.stats()["launches"] == 0
    case = CASES[0]
    s = make_solver(M, case, "fp32")
    x = np.random.default_rng(4).standard_normal(150 * 77).astype(np.float32)
    s.set_state(x)
    b.add(s, 0)
    b.run()
    b.wait()
    assert np.array_equal(s.get_state(), x)
    assert b.stats()["launches"] == 0
    b.close()
    s.close()


def test_server_zero_step_request(M):
    case = dict(lattice="D2Q9", eq="burgers", n=(40, 30), dx=0.025, dt=0.01, a=(0.6, 0.1, 0.3))
    st = np.random.default_rng(5).uniform(-0.5, 0.5, 1200).astype(np.float32)
    out = np.full_like(st, np.nan)
    srv = M.Server(hbm_budget_bytes=1 << 28, max_slots=4, quantum_steps=8)
    req = M.make_request("D2Q9", "burgers", case["n"], case["dx"], case["dt"], case["a"], 0, st,
                         precision="fp32", result_out=out)
    t = srv.submit(req, keep=(st, out))
    srv.drain(30)
    state, _, rc = srv.poll(t)
    assert state == 2 and rc == 0
    assert np.array_equal(out, st)
    srv.close()


@pytest.mark.parametrize("case", [c for c in CASES if c["name"] in ("lcde-3l-blocked", "nse-trt",
                                                                     "mesofd-lcde")],
                         ids=lambda c: c["name"])
def test_level_ptr_reports_current_storage(M, case):
    """mfd_level_ptr names the buffers that hold the live levels after the
    roles have rotated: a second solver loaded from those device addresses
    (mfd_set_state with on_device = 1) holds the same levels."""
    rng = np.random.default_rng(3)
    cur, prev = rand_state(case, rng), rand_state(case, rng)
    s = _new(M, case, "fp64")
    s.set_state(cur)
    three = case.get("kind") == "three_level"
    if three:
        s.set_state(prev, level=1)
    s.step(7)
    N = int(np.prod(case["n"]))
    nf = 1 if case["eq"] != "nse" else 1 + len(case["n"])
    p0 = [s.level_ptr(0, f) for f in range(nf)]
    assert all(p0[f] - p0[0] == f * N * 8 for f in range(nf))
    t = _new(M, case, "fp64")
    meso = case.get("form") == "mesofd"
    if not meso:  # (MesoFD moments re-initialise the populations; checked below)
        t.set_state_device(p0[0], nf * N * 8)
        assert np.array_equal(t.get_state(), s.get_state())
    if three:
        t.set_state_device(s.level_ptr(1, 0), nf * N * 8, level=1)
        assert np.array_equal(t.get_state(level=1), s.get_state(level=1))
    if meso:
        q = 9
        pp = [s.level_ptr(0, j, populations=True) for j in range(q)]
        assert all(pp[j] - pp[0] == j * N * 8 for j in range(q))
        t.set_state_device(pp[0], q * N * 8, populations=True)
        assert np.array_equal(t.get_state(populations=True), s.get_state(populations=True))
    with pytest.raises(M.MfdError):
        s.level_ptr(0, nf)
    t.close()
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", [c for c in CASES if c["name"] in ("lcde-2l-blocked", "nse-trt",
                                                                      "mesofd-lcde")],
                         ids=lambda c: c["name"])
def test_check_interval_changes_nothing(M, case, precision):
    """Steps taken in runs with the growth check between them equal the same
    steps in one call, bit for bit."""
    print("case", case["name"], precision, flush=True)
    rng = np.random.default_rng(23)
    dt = np.float64 if precision == "fp64" else np.float32
    cur, prev = rand_state(case, rng).astype(dt), rand_state(case, rng).astype(dt)
    three = case.get("kind") == "three_level"
    outs = []
    for every in (0, 7):
        s = _new(M, case, precision)
        s.set_check_interval(every)
        s.set_state(cur)
        if three:
            s.set_state(prev, level=1)
        s.step(30)
        outs.append((s.get_state(), s.get_state(level=1)))
        s.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_check_interval_stops_a_blow_up(M):
    """A NaN in the state (the stand-in for an overflowing unstable run)
    stops the solve at the first check with MFD_E_UNSTABLE; without the
    check the same call returns success."""
    case = CASES[0]
    rng = np.random.default_rng(24)
    st = rand_state(case, rng)
    st[st.size // 2] = np.nan
    s = _new(M, case, "fp64")
    s.set_state(st)
    s.step(5)  # no check: enqueued and done
    s.set_check_interval(4)
    with pytest.raises(M.MfdError) as e:
        s.step(40)
    assert e.value.code == M.MFD_E_UNSTABLE
    s.close()
    t = _new(M, case, "fp64")
    with pytest.raises(M.MfdError) as e:
        t.set_check_interval(-1)
    assert e.value.code == M.MFD_E_ARG
    t.close()
