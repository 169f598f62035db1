"""ctypes binding of libmfd.so (include/mfd.h).

Argument marshalling only: every step of the method runs in the HIP library.
The functions keep the C names; `Solver` is a thin owner of one handle.
Importing this module raises if the built library is missing -- there is no
fallback path.

PyTorch, when installed, is imported before the library is loaded: PyTorch
ships its own HIP runtime, and the library must resolve to that same runtime
instance so that torch's streams and device pointers are valid in its calls
(two HIP runtimes in one process do not share stream objects, and whichever
initialises the GPU second may find no device).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

try:  # share PyTorch's HIP runtime (see above)
    import torch  # noqa: F401
except ImportError:  # the library then uses the system HIP runtime
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmfd.so")

MFD_OK = 0
MFD_W_STABILITY_UNPROVEN = 1
MFD_W_INCONSISTENT = 2
MFD_E_ARG = -1
MFD_E_ORDER = -2
MFD_E_UNSUPPORTED = -3
MFD_E_OOM = -4
MFD_E_HIP = -5
MFD_E_UNSTABLE = -6
MFD_E_BUDGET = -7
MFD_E_CANCELLED = -8
MFD_E_TIMEOUT = -9

LATTICES = {"D1Q3": 1, "D2Q5": 2, "D2Q9": 3, "D3Q19": 4, "D2Q5II": 5, "D3Q7": 6, "D3Q9": 7,
            "D3Q27": 8}
DIMS = {"D1Q3": 1, "D2Q5": 2, "D2Q9": 2, "D3Q19": 3, "D2Q5II": 2, "D3Q7": 3, "D3Q9": 3,
        "D3Q27": 3}
QS = {"D1Q3": 3, "D2Q5": 5, "D2Q9": 9, "D3Q19": 19, "D2Q5II": 5, "D3Q7": 7, "D3Q9": 9,
      "D3Q27": 27}
PRECISIONS = {"fp64": 0, "fp32": 1}
FORMS = {"mmfd": 0, "mesofd": 1}
EQS = {"lcde": 0, "burgers": 1, "nse": 2, "wave": 3}
BOUNDARIES = {"periodic": 0, "dirichlet": 1}
KINDS = {"two_level": 0, "theta": 1, "three_level": 2}
PRESETS = {"srt": 0, "trt": 1, "one_stage": 2, "two_level": 3}


class MfdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mfd error %d: %s" % (code, msg))
        self.code = code


class mfd_grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("precision", C.c_int32), ("form", C.c_int32),
                ("boundary", C.c_int32), ("n", C.c_int64 * 3), ("dx", C.c_double)]


class mfd_eq_params(C.Structure):
    _fields_ = [("u", C.c_double * 3), ("K", C.c_double * 9), ("lambda_bar", C.c_int32),
                ("he_luo", C.c_int32), ("beta", C.c_double), ("rho0", C.c_double)]


class mfd_request(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("eq", C.c_int32), ("precision", C.c_int32),
                ("kind", C.c_int32), ("n", C.c_int64 * 2), ("d0", C.c_double), ("dx", C.c_double),
                ("dt", C.c_double), ("ep", mfd_eq_params), ("a", C.c_double * 3),
                ("ah", C.c_double * 3), ("nsteps", C.c_int64), ("state0", C.c_void_p),
                ("prev0", C.c_void_p), ("result_out", C.c_void_p), ("result_bytes", C.c_int64),
                ("exclude_from_stats", C.c_int32), ("reserved", C.c_int32),
                ("timeout_s", C.c_double)]


if not os.path.exists(LIB_PATH):
    raise ImportError("libmfd.so is not built (%s); run paper_2505_17057_amd/build.py" % LIB_PATH)

lib = C.CDLL(LIB_PATH)

_D3 = C.c_double * 3
_PD = C.POINTER(C.c_double)
_VP = C.c_void_p
_H = C.c_void_p

_SIGS = {
    "mfd_create": ([C.POINTER(_H), C.POINTER(mfd_grid)], C.c_int),
    "mfd_destroy": ([_H], C.c_int),
    "mfd_last_error": ([_H], C.c_char_p),
    "mfd_set_lattice": ([_H, C.c_int, C.c_double], C.c_int),
    "mfd_set_equation": ([_H, C.c_int, C.POINTER(mfd_eq_params)], C.c_int),
    "mfd_set_scheme": ([_H, C.c_int, _PD, _PD, _PD, _PD, C.c_double, C.c_int32, C.c_double], C.c_int),
    "mfd_set_stream": ([_H, _VP], C.c_int),
    "mfd_state_size": ([_H, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
    "mfd_set_state": ([_H, C.c_int, _VP, C.c_int64, C.c_int, C.c_int], C.c_int),
    "mfd_get_state": ([_H, C.c_int, _VP, C.c_int64, C.c_int, C.c_int], C.c_int),
    "mfd_step": ([_H, C.c_int64], C.c_int),
    "mfd_synchronize": ([_H], C.c_int),
    "mfd_reduce": ([_H, _PD, _PD], C.c_int),
    "mfd_set_check_interval": ([_H, C.c_int64], C.c_int),
    "mfd_autotune": ([_H, C.POINTER(C.c_int32)], C.c_int),
    "mfd_set_blocking": ([_H, C.c_int32], C.c_int),
    "mfd_set_plan": ([_H, C.c_int32, C.c_int32, C.c_int32], C.c_int),
    "mfd_set_source": ([_H, _PD, C.c_int64, C.c_int, C.c_double, _PD, _PD, _PD], C.c_int),
    "mfd_clear_source": ([_H], C.c_int),
    "mfd_launch_plan": ([_H, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "mfd_coeff_moments": ([_PD, _PD, _PD], C.c_int),
    "mfd_coeffs_from_constraints": ([C.c_double] * 5 + [_PD, _PD], C.c_int),
    "mfd_preset": ([C.c_int, C.c_double, _PD, _PD], C.c_int),
    "mfd_transport_coefficient": ([_PD, _PD, C.c_double, C.c_double, C.c_double, C.c_double, _PD], C.c_int),
    "mfd_max_amplification": ([_H, _PD], C.c_int),
    "mfd_max_stable_dt": ([C.c_int, C.c_double, C.c_double, _PD, C.c_double, C.POINTER(C.c_int64),
                           _PD, _PD], C.c_int),
    "mfd_level_ptr": ([_H, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_void_p)], C.c_int),
    "mfd_set_scheme_sets": ([_H, C.c_int, _PD, _PD, _PD, _PD, _PD, _PD, C.c_double], C.c_int),
    "mfd_set_theta_tolerance": ([_H, C.c_double, C.c_int32], C.c_int),
    "mfd_set_theta_multigrid": ([_H, C.c_int32, C.c_int32, C.c_int32], C.c_int),
    "mfd_set_rectangular": ([_H, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "mfd_general_create": ([C.POINTER(_H), C.POINTER(mfd_grid), C.c_int, _PD, _PD, C.c_int,
                            C.POINTER(mfd_eq_params), C.c_int32, C.c_int32, _PD, _PD,
                            C.c_double], C.c_int),
    "mfd_general_destroy": ([_H], C.c_int),
    "mfd_general_last_error": ([_H], C.c_char_p),
    "mfd_general_set_stream": ([_H, C.c_void_p], C.c_int),
    "mfd_general_set_level": ([_H, C.c_int32, _VP, C.c_int64, C.c_int], C.c_int),
    "mfd_general_get_level": ([_H, C.c_int32, _VP, C.c_int64, C.c_int], C.c_int),
    "mfd_general_step": ([_H, C.c_int64], C.c_int),
    "mfd_general_synchronize": ([_H], C.c_int),
    "mfd_theta_stats": ([_H, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                         C.POINTER(C.c_int32), C.c_int], C.c_int),
    "mfd_step_noalloc": ([_H, _VP, _VP, C.c_int64], C.c_int),
    "mfd_set_boundary": ([_H, _PD, C.c_int64, C.c_int, C.c_double], C.c_int),
    "mfd_wave_start": ([_H, _PD, C.c_int64, C.c_int], C.c_int),
    "mfd_memory_stats": ([C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_int], C.c_int),
    "mfd_batch_create": ([C.POINTER(_H)], C.c_int),
    "mfd_batch_destroy": ([_H], C.c_int),
    "mfd_batch_last_error": ([_H], C.c_char_p),
    "mfd_batch_set_stream": ([_H, _VP], C.c_int),
    "mfd_batch_set_graph": ([_H, C.c_int], C.c_int),
    "mfd_batch_add": ([_H, _H, C.c_int64, C.POINTER(C.c_int32)], C.c_int),
    "mfd_batch_clear": ([_H], C.c_int),
    "mfd_batch_run": ([_H], C.c_int),
    "mfd_batch_wait": ([_H], C.c_int),
    "mfd_batch_stats": ([_H, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
    "mfd_batch_set_plan": ([_H, C.c_int32, C.c_int32, C.c_int32], C.c_int),
    "mfd_batch_set_resident": ([_H, C.c_int32], C.c_int),
    "mfd_batch_resident": ([_H, C.POINTER(C.c_int32)], C.c_int),
    "mfd_batch_autotune": ([_H], C.c_int),
    "mfd_batch_plan": ([_H, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                        C.POINTER(C.c_int32)], C.c_int),
    "mfd_server_create": ([C.POINTER(_H), C.c_int64, C.c_int32, C.c_int64], C.c_int),
    "mfd_server_submit": ([_H, C.POINTER(mfd_request), C.POINTER(C.c_int64)], C.c_int),
    "mfd_server_poll": ([_H, C.c_int64, C.POINTER(C.c_int32), _PD], C.c_int),
    "mfd_server_cancel": ([_H, C.c_int64], C.c_int),
    "mfd_server_request_bytes": ([C.POINTER(mfd_request), C.POINTER(C.c_int64)], C.c_int),
    "mfd_server_drain": ([_H, C.c_double], C.c_int),
    "mfd_server_stats": ([_H, _PD, _PD, _PD, C.POINTER(C.c_int64), _PD], C.c_int),
    "mfd_server_destroy": ([_H], C.c_int),
    "mfd_linear_tables": ([_H, _PD, _PD, _PD], C.c_int),
}

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def _d3(v):
    return _D3(*[float(x) for x in v])


# ------------------------------------------------------- host-side algebra
def mfd_coeff_moments(a, ah):
    out = (C.c_double * 6)()
    rc = lib.mfd_coeff_moments(_d3(a), _d3(ah), out)
    if rc:
        raise MfdError(rc, "mfd_coeff_moments")
    return list(out)


def mfd_coeffs_from_constraints(a0, A10, A11, A21, A22):
    a, ah = _D3(), _D3()
    rc = lib.mfd_coeffs_from_constraints(a0, A10, A11, A21, A22, a, ah)
    if rc:
        raise MfdError(rc, "mfd_coeffs_from_constraints")
    return tuple(a), tuple(ah)


def mfd_preset(preset, param=0.0):
    a, ah = _D3(), _D3()
    rc = lib.mfd_preset(PRESETS.get(preset, preset), float(param), a, ah)
    if rc:
        raise MfdError(rc, "mfd_preset")
    return tuple(a), tuple(ah)


def mfd_transport_coefficient(a, ah, dx, dt, d0=1.0 / 3.0, beta=1.0):
    out = C.c_double()
    rc = lib.mfd_transport_coefficient(_d3(a), _d3(ah), dx, dt, d0, beta, C.byref(out))
    if rc:
        raise MfdError(rc, "mfd_transport_coefficient")
    return out.value


def mfd_max_stable_dt(lattice, dx, u, alpha, n=None, d0=1.0 / 3.0):
    """(dt_sufficient, dt_exact or None) of mfd_max_stable_dt."""
    uu = list(u) + [0.0] * (3 - len(u))
    s, e = C.c_double(), C.c_double()
    nn = None
    if n is not None:
        n3 = list(n) + [1] * (3 - len(n))
        nn = (C.c_int64 * 3)(*[int(v) for v in n3])
    rc = lib.mfd_max_stable_dt(LATTICES[lattice], float(d0), float(dx), _d3(uu), float(alpha), nn,
                               C.byref(s), C.byref(e) if n is not None else None)
    if rc:
        raise MfdError(rc, "mfd_max_stable_dt")
    return s.value, (e.value if n is not None else None)


def _ptr_of(x):
    """(address, on_device, nbytes) of a numpy array or a torch tensor."""
    if isinstance(x, np.ndarray):
        assert x.flags["C_CONTIGUOUS"]
        return x.ctypes.data, 0, x.nbytes
    # torch tensor
    assert x.is_contiguous()
    return x.data_ptr(), 1 if x.is_cuda else 0, x.numel() * x.element_size()


class General:
    """Owner of one mfd_general handle: the MMFD scheme with stencil reach m
    and n time levels for the linear CDE, Burgers' equation or the NSE
    (marshalling only).  a (and the NSE momentum set ab): n rows of 2m + 1
    coefficients (row l: level t - l dt, entry k + m)."""

    def __init__(self, lattice, n, dx, a, dt, u=(), K=None, lambda_bar=0, precision="fp64",
                 d0=1.0 / 3.0, spacing=None, d0v=None, eq="lcde", ab=None, beta=1.0, rho0=0.0,
                 he_luo=0):
        self.lattice = lattice
        self.dim = DIMS[lattice]
        n = tuple(int(v) for v in n)
        assert len(n) == self.dim
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
        assert a.ndim == 2 and a.shape[1] % 2 == 1
        self.nl, self.m = a.shape[0], (a.shape[1] - 1) // 2
        g = mfd_grid()
        g.dim = self.dim
        g.precision = PRECISIONS[precision]
        g.form = FORMS["mmfd"]
        g.boundary = BOUNDARIES["periodic"]
        g.n = (C.c_int64 * 3)(*(list(n) + [1] * (3 - len(n))))
        g.dx = float(dx)
        p = mfd_eq_params()
        p.u = _D3(*(list(u) + [0.0] * (3 - len(u))))
        Kd = np.zeros((3, 3))
        if K is not None:
            K = np.asarray(K, dtype=np.float64)
            Kd[: K.shape[0], : K.shape[1]] = K
        p.K = (C.c_double * 9)(*Kd.ravel().tolist())
        p.lambda_bar = int(lambda_bar)
        p.beta = float(beta)
        p.rho0 = float(rho0)
        p.he_luo = int(he_luo)
        if ab is not None:
            ab = np.ascontiguousarray(np.asarray(ab, dtype=np.float64))
            assert ab.shape == a.shape
        self.nf = 1 + self.dim if eq == "nse" else 1
        dv = list(d0v) if d0v is not None else [d0]
        dv3 = _d3((dv + [dv[0]] * 3)[:3])
        sp = _d3((list(spacing) + [spacing[0]] * 3)[:3]) if spacing is not None else None
        h = _H()
        rc = lib.mfd_general_create(C.byref(h), C.byref(g), LATTICES[lattice], dv3, sp, EQS[eq],
                                    C.byref(p), self.m, self.nl, a.ctypes.data_as(_PD),
                                    ab.ctypes.data_as(_PD) if ab is not None else None,
                                    float(dt))
        if rc < 0:
            raise MfdError(rc, "mfd_general_create")
        self.warnings = [rc] if rc > 0 else []
        self.h = h
        self.n = n
        self.N = self.nf * int(np.prod(n))
        self.dtype = np.float64 if precision == "fp64" else np.float32

    def check(self, rc, what):
        if rc < 0:
            msg = lib.mfd_general_last_error(self.h)
            raise MfdError(rc, "%s: %s" % (what, msg.decode() if msg else ""))
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib.mfd_general_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream_handle):
        return self.check(lib.mfd_general_set_stream(self.h, C.c_void_p(stream_handle)),
                          "mfd_general_set_stream")

    def set_level(self, level, data):
        a = np.ascontiguousarray(data, dtype=self.dtype)
        assert a.size == self.N
        return self.check(lib.mfd_general_set_level(self.h, int(level), a.ctypes.data_as(_VP),
                                                    a.nbytes, 0), "mfd_general_set_level")

    def get_level(self, level=0):
        out = np.empty(self.N, dtype=self.dtype)
        self.check(lib.mfd_general_get_level(self.h, int(level), out.ctypes.data_as(_VP),
                                             out.nbytes, 0), "mfd_general_get_level")
        return out

    def step(self, nsteps=1):
        return self.check(lib.mfd_general_step(self.h, int(nsteps)), "mfd_general_step")

    def synchronize(self):
        return self.check(lib.mfd_general_synchronize(self.h), "mfd_general_synchronize")


class Solver:
    """Owner of one mfd_solver handle (marshalling only)."""

    def __init__(self, lattice, n, dx, precision="fp64", form="mmfd", boundary="periodic",
                 d0=1.0 / 3.0):
        self.lattice = lattice
        self.dim = DIMS[lattice]
        n = tuple(int(v) for v in n)
        assert len(n) == self.dim
        g = mfd_grid()
        g.dim = self.dim
        g.precision = PRECISIONS[precision]
        g.form = FORMS[form]
        g.boundary = BOUNDARIES[boundary]
        g.n = (C.c_int64 * 3)(*(list(n) + [1] * (3 - len(n))))
        g.dx = float(dx)
        h = _H()
        rc = lib.mfd_create(C.byref(h), C.byref(g))
        if rc:
            raise MfdError(rc, "mfd_create")
        self.h = h
        self.n = n
        self.precision = precision
        self.form = form
        self.dtype = np.float64 if precision == "fp64" else np.float32
        self.warnings = []
        self.check(lib.mfd_set_lattice(self.h, LATTICES[lattice], float(d0)), "mfd_set_lattice")

    # -------------------------------------------------------------- plumbing
    def check(self, rc, what):
        if rc < 0:
            msg = lib.mfd_last_error(self.h)
            raise MfdError(rc, "%s: %s" % (what, msg.decode() if msg else ""))
        if rc > 0:
            self.warnings.append((rc, what))
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib.mfd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- configure
    def set_lattice(self, lattice, d0=1.0 / 3.0):
        return self.check(lib.mfd_set_lattice(self.h, LATTICES[lattice], d0), "mfd_set_lattice")

    def set_equation(self, eq, u=(), K=None, lambda_bar=0, beta=1.0, rho0=0.0, he_luo=0):
        p = mfd_eq_params()
        uu = list(u) + [0.0] * (3 - len(u))
        p.u = _D3(*uu)
        Kd = np.zeros((3, 3))
        if K is not None:
            K = np.asarray(K, dtype=np.float64)
            Kd[: K.shape[0], : K.shape[1]] = K
        p.K = (C.c_double * 9)(*Kd.ravel().tolist())
        p.lambda_bar = int(lambda_bar)
        p.he_luo = int(he_luo)
        p.beta = float(beta)
        p.rho0 = float(rho0)
        self.eq = eq
        self.nf = 1 + self.dim if eq == "nse" else 1
        return self.check(lib.mfd_set_equation(self.h, EQS[eq], C.byref(p)), "mfd_set_equation")

    def set_scheme(self, kind, a, ah=None, ab=None, abh=None, theta=1.0, theta_iters=0, dt=1.0):
        self.kind = kind
        return self.check(lib.mfd_set_scheme(
            self.h, KINDS[kind], _d3(a), _d3(ah) if ah is not None else None,
            _d3(ab) if ab is not None else None, _d3(abh) if abh is not None else None,
            float(theta), int(theta_iters), float(dt)), "mfd_set_scheme")

    def set_stream(self, stream_handle):
        return self.check(lib.mfd_set_stream(self.h, C.c_void_p(stream_handle)), "mfd_set_stream")

    def state_size(self):
        m, p, b = C.c_int64(), C.c_int64(), C.c_int64()
        self.check(lib.mfd_state_size(self.h, C.byref(m), C.byref(p), C.byref(b)), "mfd_state_size")
        return m.value, p.value, b.value

    # -------------------------------------------------------------- state
    def set_state(self, x, level=0, populations=False):
        if isinstance(x, np.ndarray):
            x = np.ascontiguousarray(x, dtype=self.dtype)
        addr, dev, nb = _ptr_of(x)
        return self.check(lib.mfd_set_state(self.h, level, C.c_void_p(addr), nb, dev, int(populations)),
                          "mfd_set_state")

    def set_state_device(self, addr, nbytes, level=0, populations=False):
        """mfd_set_state from a raw device address (e.g. mfd_level_ptr)."""
        return self.check(lib.mfd_set_state(self.h, level, C.c_void_p(int(addr)), int(nbytes), 1,
                                            int(populations)), "mfd_set_state")

    def get_state(self, level=0, populations=False, out=None):
        m, p, _ = self.state_size()
        if out is None:
            out = np.empty(p if populations else m, dtype=self.dtype)
        addr, dev, nb = _ptr_of(out)
        self.check(lib.mfd_get_state(self.h, level, C.c_void_p(addr), nb, dev, int(populations)),
                   "mfd_get_state")
        return out

    def step(self, nsteps=1):
        return self.check(lib.mfd_step(self.h, int(nsteps)), "mfd_step")

    def synchronize(self):
        return self.check(lib.mfd_synchronize(self.h), "mfd_synchronize")

    def reduce(self):
        sums = (C.c_double * 4)()
        res = C.c_double()
        self.check(lib.mfd_reduce(self.h, sums, C.byref(res)), "mfd_reduce")
        return list(sums), res.value

    def set_check_interval(self, every):
        return self.check(lib.mfd_set_check_interval(self.h, int(every)), "mfd_set_check_interval")

    def set_blocking(self, depth):
        return self.check(lib.mfd_set_blocking(self.h, int(depth)), "mfd_set_blocking")

    def set_plan(self, tb_depth, window_rows=0, window_cols=64):
        return self.check(lib.mfd_set_plan(self.h, int(tb_depth), int(window_rows), int(window_cols)),
                          "mfd_set_plan")

    def set_source(self, G, lam=0.0, b=(0.0, 1.0, 0.0), bh=(0.0, 0.0, 0.0), v=()):
        """Source term of the linear CDE: S(x, t) = exp(lam t) G(x) (t counted
        from the last set_state), coefficients b (level t) and bh (level
        t - dt) for k = -1, 0, 1, source flux M_1F = v S.  G: float64 array of
        the grid's node count (host)."""
        g = np.ascontiguousarray(np.asarray(G, dtype=np.float64).ravel())
        vv = list(v) + [0.0] * (3 - len(v))
        return self.check(lib.mfd_set_source(self.h, g.ctypes.data_as(_PD), g.size, 0, float(lam),
                                             _d3(b), _d3(bh), _d3(vv)), "mfd_set_source")

    def clear_source(self):
        return self.check(lib.mfd_clear_source(self.h), "mfd_clear_source")

    def launch_plan(self):
        """(time steps per launch, LDS window rows, LDS window columns)."""
        tb, h, w = C.c_int32(), C.c_int32(), C.c_int32()
        self.check(lib.mfd_launch_plan(self.h, C.byref(tb), C.byref(h), C.byref(w)), "mfd_launch_plan")
        return tb.value, h.value, w.value

    def autotune(self):
        d = C.c_int32()
        self.check(lib.mfd_autotune(self.h, C.byref(d)), "mfd_autotune")
        return d.value

    def set_scheme_sets(self, kind, a, ae, ao, ah=None, aeh=None, aoh=None, dt=1.0):
        """Multiple-set scheme of Eq. (2-2-1b) (mfd_set_scheme_sets)."""
        self.kind = kind
        three = kind == "three_level"
        f = (lambda v: _d3(v) if three else None)
        return self.check(lib.mfd_set_scheme_sets(self.h, KINDS[kind], _d3(a), f(ah), _d3(ae), f(aeh),
                                                  _d3(ao), f(aoh), float(dt)), "mfd_set_scheme_sets")

    def set_theta_tolerance(self, tol, chunk=0):
        return self.check(lib.mfd_set_theta_tolerance(self.h, float(tol), int(chunk)),
                          "mfd_set_theta_tolerance")

    def set_rectangular(self, dx, d0):
        """Spacing and d0 per axis (rectangular lattice, linear CDE)."""
        return self.check(lib.mfd_set_rectangular(self.h, _d3((list(dx) + [dx[0]] * 3)[:3]),
                                                  _d3((list(d0) + [d0[0]] * 3)[:3])),
                          "mfd_set_rectangular")

    def set_theta_multigrid(self, levels=-1, pre=2, post=2):
        return self.check(lib.mfd_set_theta_multigrid(self.h, int(levels), int(pre), int(post)),
                          "mfd_set_theta_multigrid")

    def theta_stats(self, reset=False):
        a, b = C.c_int64(), C.c_int64()
        c, d = C.c_int32(), C.c_int32()
        self.check(lib.mfd_theta_stats(self.h, C.byref(a), C.byref(b), C.byref(c), C.byref(d),
                                       1 if reset else 0), "mfd_theta_stats")
        return dict(total_sweeps=a.value, steps=b.value, max_sweeps=c.value, unconverged=d.value)

    def step_noalloc(self, level0_ptr, level1_ptr=None, nsteps=1):
        """mfd_step_noalloc on caller-owned device levels (raw addresses)."""
        return self.check(lib.mfd_step_noalloc(self.h, C.c_void_p(int(level0_ptr)),
                                               C.c_void_p(int(level1_ptr)) if level1_ptr else None,
                                               int(nsteps)), "mfd_step_noalloc")

    def set_boundary(self, G, lam=0.0):
        """Dirichlet values G(x) exp(lam t) of the edge nodes (mfd_set_boundary)."""
        G = np.ascontiguousarray(G, dtype=np.float64).ravel()
        return self.check(lib.mfd_set_boundary(self.h, G.ctypes.data_as(_PD), G.size, 0, float(lam)),
                          "mfd_set_boundary")

    def wave_start(self, phi_t):
        """Special first step of the three-level wave scheme (mfd_wave_start)."""
        v = np.ascontiguousarray(phi_t, dtype=np.float64).ravel()
        return self.check(lib.mfd_wave_start(self.h, v.ctypes.data_as(_PD), v.size, 0),
                          "mfd_wave_start")

    def level_ptr(self, level=0, field=0, populations=False):
        p = C.c_void_p()
        self.check(lib.mfd_level_ptr(self.h, int(level), int(field), 1 if populations else 0,
                                     C.byref(p)), "mfd_level_ptr")
        return p.value

    def max_amplification(self):
        out = C.c_double()
        self.check(lib.mfd_max_amplification(self.h, C.byref(out)), "mfd_max_amplification")
        return out.value

    def linear_tables(self):
        b = QS[self.lattice]
        w = np.zeros(b)
        ub = np.zeros(b)
        p6 = np.zeros(6 * 9)
        self.check(lib.mfd_linear_tables(self.h, w.ctypes.data_as(_PD), ub.ctypes.data_as(_PD),
                                         p6.ctypes.data_as(_PD)), "mfd_linear_tables")
        npair = (b - 1) // 2
        p6 = p6.reshape(6, 9)[:, :npair]
        names = ["ubp", "ubm", "Cp", "Cm", "Chp", "Chm"]
        return w, ub, {k: p6[i].copy() for i, k in enumerate(names)}


class Batch:
    """Owner of one mfd_batch handle (marshalling only)."""

    def __init__(self, stream_handle=None, use_graph=True):
        h = _H()
        rc = lib.mfd_batch_create(C.byref(h))
        if rc:
            raise MfdError(rc, "mfd_batch_create")
        self.h = h
        self.members = []
        if stream_handle:
            self.check(lib.mfd_batch_set_stream(self.h, C.c_void_p(stream_handle)), "mfd_batch_set_stream")
        self.check(lib.mfd_batch_set_graph(self.h, 1 if use_graph else 0), "mfd_batch_set_graph")

    def check(self, rc, what):
        if rc < 0:
            msg = lib.mfd_batch_last_error(self.h)
            raise MfdError(rc, "%s: %s" % (what, msg.decode() if msg else ""))
        return rc

    def add(self, solver, nsteps):
        slot = C.c_int32()
        self.check(lib.mfd_batch_add(self.h, solver.h, int(nsteps), C.byref(slot)), "mfd_batch_add")
        self.members.append(solver)
        return slot.value

    def clear(self):
        self.members = []
        return self.check(lib.mfd_batch_clear(self.h), "mfd_batch_clear")

    def run(self):
        return self.check(lib.mfd_batch_run(self.h), "mfd_batch_run")

    def wait(self):
        return self.check(lib.mfd_batch_wait(self.h), "mfd_batch_wait")

    def stats(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self.check(lib.mfd_batch_stats(self.h, C.byref(a), C.byref(b), C.byref(c)), "mfd_batch_stats")
        return dict(launches=a.value, lups=b.value, tiles=c.value)

    def set_resident(self, max_nodes):
        return self.check(lib.mfd_batch_set_resident(self.h, int(max_nodes)), "mfd_batch_set_resident")

    def resident(self):
        c = C.c_int32()
        self.check(lib.mfd_batch_resident(self.h, C.byref(c)), "mfd_batch_resident")
        return c.value

    def set_plan(self, tb_depth, window_rows=0, window_cols=0):
        return self.check(lib.mfd_batch_set_plan(self.h, int(tb_depth), int(window_rows), int(window_cols)),
                          "mfd_batch_set_plan")

    def autotune(self):
        return self.check(lib.mfd_batch_autotune(self.h), "mfd_batch_autotune")

    def plan(self, group=0):
        tb, h, w = C.c_int32(), C.c_int32(), C.c_int32()
        self.check(lib.mfd_batch_plan(self.h, int(group), C.byref(tb), C.byref(h), C.byref(w)),
                   "mfd_batch_plan")
        return tb.value, h.value, w.value

    def close(self):
        if getattr(self, "h", None):
            lib.mfd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_request(lattice, eq, n, dx, dt, a, nsteps, state0, ah=None, kind="two_level",
                 precision="fp32", u=(), K=None, lambda_bar=0, beta=1.0, rho0=0.0, he_luo=0,
                 result_out=None, prev0=None, exclude=False, d0=1.0 / 3.0, timeout_s=0.0):
    """Fill an mfd_request; the arrays must stay alive until the request is done."""
    r = mfd_request()
    r.lattice = LATTICES[lattice]
    r.eq = EQS[eq]
    r.precision = PRECISIONS[precision]
    r.kind = KINDS[kind]
    r.n = (C.c_int64 * 2)(int(n[0]), int(n[1]))
    r.d0 = d0
    r.dx = float(dx)
    r.dt = float(dt)
    p = mfd_eq_params()
    uu = list(u) + [0.0] * (3 - len(u))
    p.u = _D3(*uu)
    Kd = np.zeros((3, 3))
    if K is not None:
        K = np.asarray(K, dtype=np.float64)
        Kd[: K.shape[0], : K.shape[1]] = K
    p.K = (C.c_double * 9)(*Kd.ravel().tolist())
    p.lambda_bar = int(lambda_bar)
    p.he_luo = int(he_luo)
    p.beta = float(beta)
    p.rho0 = float(rho0)
    r.ep = p
    r.a = _d3(a)
    r.ah = _d3(ah if ah is not None else (0.0, 0.0, 0.0))
    r.nsteps = int(nsteps)
    r.state0 = state0.ctypes.data
    r.prev0 = prev0.ctypes.data if prev0 is not None else None
    r.result_out = result_out.ctypes.data if result_out is not None else None
    r.result_bytes = result_out.nbytes if result_out is not None else 0
    r.exclude_from_stats = 1 if exclude else 0
    r.timeout_s = float(timeout_s)
    return r


def server_request_bytes(req):
    """Device bytes a request holds while admitted (mfd_server_request_bytes)."""
    b = C.c_int64()
    rc = lib.mfd_server_request_bytes(C.byref(req), C.byref(b))
    if rc:
        raise MfdError(rc, "mfd_server_request_bytes")
    return b.value


def memory_stats(reset_peak=False):
    """Device bytes the library holds now and at peak (mfd_memory_stats)."""
    a, b = C.c_int64(), C.c_int64()
    lib.mfd_memory_stats(C.byref(a), C.byref(b), 1 if reset_peak else 0)
    return a.value, b.value


class Server:
    """Owner of one mfd_server handle (marshalling only)."""

    def __init__(self, hbm_budget_bytes, max_slots=256, quantum_steps=50):
        h = _H()
        rc = lib.mfd_server_create(C.byref(h), int(hbm_budget_bytes), int(max_slots), int(quantum_steps))
        if rc:
            raise MfdError(rc, "mfd_server_create")
        self.h = h
        self._keep = {}

    def submit(self, req, keep=()):
        t = C.c_int64()
        rc = lib.mfd_server_submit(self.h, C.byref(req), C.byref(t))
        if rc:
            raise MfdError(rc, "mfd_server_submit")
        self._keep[t.value] = (req, keep)
        return t.value

    def poll(self, ticket):
        st = C.c_int32()
        lat = C.c_double()
        rc = lib.mfd_server_poll(self.h, int(ticket), C.byref(st), C.byref(lat))
        return st.value, lat.value, rc

    def cancel(self, ticket):
        return lib.mfd_server_cancel(self.h, int(ticket))

    def drain(self, timeout_s=600.0):
        rc = lib.mfd_server_drain(self.h, float(timeout_s))
        if rc:
            raise MfdError(rc, "mfd_server_drain")

    def stats(self):
        p50, p99, rps, g = C.c_double(), C.c_double(), C.c_double(), C.c_double()
        n = C.c_int64()
        lib.mfd_server_stats(self.h, C.byref(p50), C.byref(p99), C.byref(rps), C.byref(n), C.byref(g))
        return dict(p50_s=p50.value, p99_s=p99.value, req_per_s=rps.value, completed=n.value,
                    glups=g.value)

    def close(self):
        if getattr(self, "h", None):
            lib.mfd_server_destroy(self.h)
            self.h = None
            self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
