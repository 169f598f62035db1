"""GPU parity: the HIP library against the FP64 oracle, element by element.

FP64 runs must equal the oracle value for value (signed zeros compare equal);
FP32 runs must stay within a relative L2 error of 1e-5 of the FP64 oracle
(the bound the workloads are held to), and the measured error is printed.
Grids are ragged against every tile shape (1D tiles of 1024 nodes, 2D tiles
of 64 x 16 / 64 x 8, 3D tiles of 32 x 8 x 32-plane chunks) and small enough
for the oracle to finish in seconds.
"""
import numpy as np
import pytest

from parity_util import rand_state, rel_l2, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

TRT = ((1.0, 0.0, 0.4), (0.0, -0.4, 0.0))  # TRT preset, s = 0.6
EX13 = ((0.875, 0.0, 0.125), (0.125, 0.0, -0.125))  # three-level with a t-dt stencil
K2 = [[0.3, 0.04], [0.04, 0.2]]
K3 = [[0.2, 0.02, 0.01], [0.02, 0.15, 0.0], [0.01, 0.0, 0.1]]

CASES = [
    # --- 1D
    dict(name="d1q3-lcde-2l-tiled", lattice="D1Q3", n=(1030,), eq="lcde", u=(0.2,), K=[[0.25]],
         a=(1.25, -0.5, 0.25)),
    dict(name="d1q3-lcde-2l-resident", lattice="D1Q3", n=(1024,), eq="lcde", u=(0.2,), K=[[0.25]],
         a=(1.25, -0.5, 0.25)),
    dict(name="d1q3-lcde-2l-wave64", lattice="D1Q3", n=(64,), eq="lcde", u=(0.2,), K=[[0.25]],
         a=(1.25, -0.5, 0.25)),
    dict(name="d1q3-lcde-mesofd-wave", lattice="D1Q3", n=(512,), eq="lcde", u=(0.2,), K=[[0.25]],
         a=(1.25, -0.5, 0.25), form="mesofd"),
    dict(name="d1q3-burgers-3l", lattice="D1Q3", n=(999,), eq="burgers", dx=0.1, dt=0.02,
         kind="three_level", a=EX13[0], ah=EX13[1]),
    dict(name="d1q3-lcde-mesofd", lattice="D1Q3", n=(1030,), eq="lcde", u=(0.2,), K=[[0.25]],
         a=(1.25, -0.5, 0.25), form="mesofd"),
    dict(name="d1q3-lcde-mesofd-tiled", lattice="D1Q3", n=(5003,), eq="lcde", u=(0.2,), K=[[0.25]],
         a=(1.25, -0.5, 0.25), form="mesofd"),
    dict(name="d1q3-burgers-mesofd-3l", lattice="D1Q3", n=(999,), eq="burgers", dx=0.1, dt=0.02,
         kind="three_level", a=EX13[0], ah=EX13[1], form="mesofd"),
    dict(name="d1q3-burgers-mesofd-trt", lattice="D1Q3", n=(777,), eq="burgers", dx=0.1, dt=0.02,
         kind="three_level", a=(1.0, 0.0, 0.4), ah=(0.0, -0.4, 0.0), form="mesofd"),
    # --- 2D linear
    dict(name="d2q9-lcde-srt", lattice="D2Q9", n=(70, 37), eq="lcde", u=(0.1, -0.07), K=K2,
         lambda_bar=1, a=(1.0, 0.0, 0.0)),
    dict(name="d2q9-lcde-3l-stencil", lattice="D2Q9", n=(70, 37), eq="lcde", u=(0.1, -0.07), K=K2,
         lambda_bar=1, kind="three_level", a=EX13[0], ah=EX13[1]),
    dict(name="d2q9-lcde-trt", lattice="D2Q9", n=(67, 40), eq="lcde", u=(0.05, 0.03), K=K2,
         lambda_bar=1, kind="three_level", a=TRT[0], ah=TRT[1]),
    dict(name="d2q5-lcde", lattice="D2Q5", n=(66, 35), eq="lcde", u=(0.1, 0.05),
         K=[[1.0 / 6.0, 0.0], [0.0, 1.0 / 6.0]], a=(1.0, 0.0, 0.0)),
    dict(name="d2q9-lcde-mesofd", lattice="D2Q9", n=(70, 37), eq="lcde", u=(0.1, -0.07), K=K2,
         lambda_bar=1, a=(1.0, 0.0, 0.0), form="mesofd"),
    dict(name="d2q9-lcde-mesofd-3l", lattice="D2Q9", n=(70, 37), eq="lcde", u=(0.1, -0.07), K=K2,
         lambda_bar=1, kind="three_level", a=EX13[0], ah=EX13[1], form="mesofd"),
    dict(name="d2q9-lcde-theta", lattice="D2Q9", n=(70, 37), eq="lcde", u=(0.05, -0.03), K=K2,
         lambda_bar=1, a=(0.8, -0.2, 0.4), kind="theta", theta=0.5, theta_iters=12),
    dict(name="d2q9-lcde-theta-fused", lattice="D2Q9", n=(150, 77), eq="lcde", u=(0.05, -0.03), K=K2,
         lambda_bar=1, a=(0.8, -0.2, 0.4), kind="theta", theta=0.5, theta_iters=4),
    dict(name="d2q9-lcde-theta-fused-1", lattice="D2Q9", n=(64, 64), eq="lcde", u=(0.05, -0.03), K=K2,
         lambda_bar=1, a=(0.8, -0.2, 0.4), kind="theta", theta=0.25, theta_iters=1),
    dict(name="d2q5-lcde-theta-fused", lattice="D2Q5", n=(100, 70), eq="lcde", u=(0.1, 0.05),
         K=[[0.2, 0.0], [0.0, 0.2]], lambda_bar=0, a=(0.8, -0.2, 0.4), kind="theta", theta=0.75,
         theta_iters=3),
    # --- 2D nonlinear
    dict(name="d2q9-burgers-2l", lattice="D2Q9", n=(70, 37), eq="burgers", dx=0.05, dt=0.01,
         a=(0.8, -0.6, -0.2)),
    dict(name="d2q9-burgers-mesofd", lattice="D2Q9", n=(70, 37), eq="burgers", dx=0.05, dt=0.01,
         a=(0.8, -0.6, -0.2), form="mesofd"),
    dict(name="d2q9-burgers-beta", lattice="D2Q9", n=(70, 37), eq="burgers", dx=0.05, dt=0.01,
         a=(1.0, 0.0, 0.0), beta=0.5),
    dict(name="d2q9-nse-trt", lattice="D2Q9", n=(70, 37), eq="nse", rho0=1.0, kind="three_level",
         a=TRT[0], ah=TRT[1]),
    dict(name="d2q9-nse-3l-stencil-2set", lattice="D2Q9", n=(70, 37), eq="nse", rho0=1.0,
         kind="three_level", a=EX13[0], ah=EX13[1], ab=TRT[0], abh=TRT[1]),
    dict(name="d2q9-nse-plain-rho", lattice="D2Q9", n=(66, 20), eq="nse", rho0=0.0, a=(1.0, 0.0, 0.0)),
    dict(name="d2q9-nse-trt-narrow", lattice="D2Q9", n=(40, 9), eq="nse", rho0=1.0, kind="three_level",
         a=TRT[0], ah=TRT[1]),
    dict(name="d2q9-nse-3l-stencil-small", lattice="D2Q9", n=(7, 5), eq="nse", rho0=1.0,
         kind="three_level", a=EX13[0], ah=EX13[1], ab=TRT[0], abh=TRT[1]),
    dict(name="d2q9-nse-heluo", lattice="D2Q9", n=(66, 20), eq="nse", rho0=1.0, he_luo=1,
         kind="three_level", a=TRT[0], ah=TRT[1]),
    dict(name="d2q9-nse-mesofd-trt", lattice="D2Q9", n=(70, 37), eq="nse", rho0=1.0,
         kind="three_level", a=TRT[0], ah=TRT[1], form="mesofd"),
    # --- the further lattices of Appendix A (single-step kernels; C = 0)
    dict(name="d2q5ii-lcde", lattice="D2Q5II", n=(67, 33), eq="lcde", u=(0.1, -0.05),
         K=[[0.2, 0.0], [0.0, 0.2]], d0=0.4, a=(1.0, 0.0, 0.0)),
    dict(name="d2q5ii-lcde-3l-mesofd", lattice="D2Q5II", n=(40, 31), eq="lcde", u=(0.1, -0.05),
         K=[[0.2, 0.0], [0.0, 0.2]], d0=0.4, kind="three_level", a=EX13[0], ah=EX13[1],
         form="mesofd"),
    dict(name="d2q5ii-burgers", lattice="D2Q5II", n=(70, 37), eq="burgers", dx=0.05, dt=0.01,
         a=(0.8, -0.6, -0.2)),
    dict(name="d2q5ii-nse-trt", lattice="D2Q5II", n=(66, 21), eq="nse", rho0=1.0,
         kind="three_level", a=TRT[0], ah=TRT[1]),
    dict(name="d3q7-lcde-trt", lattice="D3Q7", n=(35, 19, 13), eq="lcde", u=(0.05, 0.02, -0.03),
         K=[[0.1, 0.0, 0.0], [0.0, 0.1, 0.0], [0.0, 0.0, 0.1]], d0=0.25, kind="three_level",
         a=TRT[0], ah=TRT[1]),
    dict(name="d3q7-burgers-mesofd", lattice="D3Q7", n=(20, 13, 9), eq="burgers", dx=0.05,
         dt=0.01, d0=0.25, a=(0.8, -0.6, -0.2), form="mesofd"),
    dict(name="d3q7-nse-trt", lattice="D3Q7", n=(34, 10, 7), eq="nse", rho0=1.0, d0=0.25,
         kind="three_level", a=TRT[0], ah=TRT[1]),
    dict(name="d3q9-lcde", lattice="D3Q9", n=(35, 19, 13), eq="lcde", u=(0.05, 0.02, -0.03),
         K=[[0.15, 0.0, 0.0], [0.0, 0.15, 0.0], [0.0, 0.0, 0.15]], a=(1.1, -0.2, 0.1)),
    dict(name="d3q9-nse-trt", lattice="D3Q9", n=(20, 13, 9), eq="nse", rho0=1.0,
         kind="three_level", a=TRT[0], ah=TRT[1]),
    # --- 3D
    dict(name="d3q19-nse-trt", lattice="D3Q19", n=(35, 19, 13), eq="nse", rho0=1.0,
         kind="three_level", a=TRT[0], ah=TRT[1]),
    dict(name="d3q19-nse-trt-zchunks", lattice="D3Q19", n=(34, 10, 70), eq="nse", rho0=1.0,
         kind="three_level", a=TRT[0], ah=TRT[1]),
    dict(name="d3q19-nse-2l-srt", lattice="D3Q19", n=(9, 7, 5), eq="nse", rho0=1.0, a=(1.0, 0.0, 0.0)),
    dict(name="d3q19-nse-trt-wide", lattice="D3Q19", n=(70, 33, 6), eq="nse", rho0=1.0,
         kind="three_level", a=TRT[0], ah=TRT[1]),
    # the binary32 register march (x >= 64, y >= 16): ragged strips, rows and z chunks
    dict(name="d3q19-nse-trt-strips", lattice="D3Q19", n=(131, 47, 9), eq="nse", rho0=1.0,
         kind="three_level", a=TRT[0], ah=TRT[1]),
    dict(name="d3q19-nse-2l-strips", lattice="D3Q19", n=(66, 16, 3), eq="nse", rho0=1.0,
         a=(1.0, 0.0, 0.0)),
    dict(name="d3q19-nse-3l-stencil", lattice="D3Q19", n=(35, 19, 13), eq="nse", rho0=1.0,
         kind="three_level", a=EX13[0], ah=EX13[1]),
    dict(name="d3q19-nse-mesofd", lattice="D3Q19", n=(35, 19, 13), eq="nse", rho0=1.0,
         kind="three_level", a=TRT[0], ah=TRT[1], form="mesofd"),
    dict(name="d3q19-lcde", lattice="D3Q19", n=(35, 19, 13), eq="lcde", u=(0.05, 0.02, -0.03), K=K3,
         lambda_bar=1, a=(1.0, 0.0, 0.0)),
    dict(name="d3q19-burgers-mesofd", lattice="D3Q19", n=(35, 19, 13), eq="burgers", dx=0.05,
         dt=0.01, a=(0.8, -0.6, -0.2), form="mesofd"),
]

STEPS = 7


def _io(case, seed=12345):
    rng = np.random.default_rng(seed)
    return rand_state(case, rng), rand_state(case, rng)


@pytest.mark.parametrize("case", CASES, ids=lambda c: c["name"])
def test_fp64_bitwise(M, case):
    print("case", case["name"], flush=True)
    cur, prev = _io(case)
    want = run_oracle(case, cur, prev, STEPS)
    got = run_gpu(M, case, cur, prev, STEPS, "fp64", chunks=[1, 2, STEPS - 3])
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, "%d mismatches, first at %d: %r vs %r (max |d| %g)" % (
        bad.size, bad[0], got[bad[0]], want[bad[0]], np.abs(got - want).max())


@pytest.mark.parametrize("case", CASES, ids=lambda c: c["name"])
def test_fp32_tolerance(M, case):
    print("case", case["name"], flush=True)
    cur, prev = _io(case)
    want = run_oracle(case, cur, prev, STEPS)
    # FP32 runs start from the FP32-rounded state; the oracle from the same values
    cur32 = cur.astype(np.float32).astype(np.float64)
    prev32 = prev.astype(np.float32).astype(np.float64)
    want = run_oracle(case, cur32, prev32, STEPS)
    got = run_gpu(M, case, cur32, prev32, STEPS, "fp32")
    err = rel_l2(got, want)
    print("fp32 rel-L2 %s: %.3e" % (case["name"], err))
    assert err <= 1e-5


@pytest.mark.parametrize("n", [64, 128, 256, 512, 1024])
@pytest.mark.parametrize("form", ["mmfd", "mesofd"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_1d_register_run_equals_single_steps(M, n, form, precision):
    """A run of small periodic 1D two-level LCDE grids held in the registers
    of one workgroup (wavefronts joined by DPP shifts and their end nodes)
    equals the same steps taken one launch at a time, bit for bit: the last
    level and, for MesoFD, the populations."""
    from parity_util import make_solver
    case = dict(lattice="D1Q3", n=(n,), eq="lcde", u=(0.2,), K=[[0.25]], a=(1.25, -0.5, 0.25),
                form=form)
    rng = np.random.default_rng(n)
    dt = np.float64 if precision == "fp64" else np.float32
    cur = rand_state(case, rng).astype(dt)
    outs = []
    for chunks in ([23], [1] * 23):
        s = make_solver(M, case, precision)
        s.set_state(cur)
        for k in chunks:
            s.step(k)
        got = [s.get_state()]
        if form == "mesofd":
            got.append(s.get_state(populations=True))
        outs.append(got)
        s.close()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)

