"""ctypes front end of the plain FP64 CPU oracle (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package. The product path never loads it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "maze_oracle.c")
_LIB = os.path.join(_HERE, "libmaze_oracle.so")
# timing build: the same source with -fopenmp, its order-independent loops
# threaded (bitwise the plain build's results)
_LIB_OMP = os.path.join(_HERE, "libmaze_oracle_omp.so")

GUESS_ZERO, GUESS_STATIC, GUESS_TIMEPROP = 0, 1, 2
NORM_REL2, NORM_ABSMAX = 0, 1
OK, NOT_CONVERGED, E_INVALID, E_NOT_NEUTRAL = 0, 1, -1, -2


def _compile(out: str, extra) -> None:
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
           "-fPIC", "-shared"] + list(extra) + ["-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd, cwd=_HERE)
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the oracle with plain gcc (no FMA contraction, no intrinsics),
    and its OpenMP timing build."""
    for out, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            _compile(out, extra)
    return _LIB


class Config(ctypes.Structure):
    _fields_ = [("n_ions", ctypes.c_int32), ("order", ctypes.c_int32),
                ("box", ctypes.c_double), ("grid_spacing", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("residual_norm", ctypes.c_int32), ("coulomb_k", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("grid_n", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("h", ctypes.c_double), ("rel_residual", ctypes.c_double),
                ("max_abs_residual", ctypes.c_double),
                ("net_charge", ctypes.c_double), ("energy", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


_lib = None
_lib_omp = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _load(_LIB)
    return _lib


def lib_omp():
    """The OpenMP timing build (threads from OMP_NUM_THREADS)."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_LIB_OMP) or os.path.getmtime(_LIB_OMP) < os.path.getmtime(_SRC):
            build(force=True)
        _lib_omp = _load(_LIB_OMP)
    return _lib_omp


def _load(path):
    L = ctypes.CDLL(path)
    L.oracle_grid_n.restype = ctypes.c_int
    L.oracle_grid_n.argtypes = [ctypes.c_double, ctypes.c_double]
    L.oracle_axis_weights.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int, _ip, _dp]
    L.oracle_spread_raw.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_int, _dp]
    L.oracle_project_mean.restype = ctypes.c_double
    L.oracle_project_mean.argtypes = [ctypes.c_int, _dp]
    L.oracle_apply_M.argtypes = [ctypes.c_int, _dp, _dp]
    L.oracle_pcg.restype = ctypes.c_int
    L.oracle_pcg.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_int,
                             ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    for name in ("oracle_gather", "oracle_gather_weight_gradient"):
        getattr(L, name).argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int, _dp,
                                     ctypes.c_double, _dp]
    L.oracle_energy.restype = ctypes.c_double
    L.oracle_energy.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double]
    L.oracle_init.restype = ctypes.c_int
    L.oracle_init.argtypes = [ctypes.POINTER(Config), _dp, _dp,
                              ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Stats)]
    L.oracle_step.restype = ctypes.c_int
    L.oracle_step.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp,
                              ctypes.POINTER(Stats)]
    L.oracle_solve.restype = ctypes.c_int
    L.oracle_solve.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp, _dp,
                               ctypes.POINTER(Stats)]
    L.oracle_get_state.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp]
    L.oracle_grid_of.restype = ctypes.c_int
    L.oracle_grid_of.argtypes = [ctypes.c_void_p]
    L.oracle_destroy.argtypes = [ctypes.c_void_p]
    L.oracle_bmh.argtypes = [ctypes.c_int, _dp, _ip, ctypes.c_double, _dp,
                             ctypes.c_double, _dp, _dp]
    L.oracle_md_step.restype = ctypes.c_int
    L.oracle_md_step.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp, _ip,
                                 _dp, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, _dp, _dp, _dp, _dp, _dp,
                                 ctypes.POINTER(Stats)]
    return L


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _i(a):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_ip)


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def grid_n(box, h):
    return lib().oracle_grid_n(box, h)


def axis_weights(order, coord, box, N):
    idx = np.zeros(4, np.int32)
    w = np.zeros(4, np.float64)
    lib().oracle_axis_weights(order, coord, box, N, _i(idx), _d(w))
    return idx[:order].copy(), w[:order].copy()


def spread_raw(pos, Q, box, N, order=2):
    pos, Q = _c(pos), _c(Q)
    q = np.zeros(N ** 3, np.float64)
    lib().oracle_spread_raw(len(Q), _d(pos), _d(Q), box, N, order, _d(q))
    return q.reshape(N, N, N)


def spread(pos, Q, box, N, order=2):
    q = spread_raw(pos, Q, box, N, order).ravel().copy()
    lib().oracle_project_mean(N, _d(q))
    return q.reshape(N, N, N)


def apply_M(x):
    N = x.shape[0]
    x = _c(x).ravel()
    out = np.zeros_like(x)
    lib().oracle_apply_M(N, _d(x), _d(out))
    return out.reshape(N, N, N)


def pcg(b, x0=None, thr=1e-12, norm=NORM_REL2, max_iter=100000):
    N = b.shape[0]
    b = _c(b).ravel()
    x = np.zeros_like(b) if x0 is None else _c(x0).ravel().copy()
    it = ctypes.c_int(0)
    ok = lib().oracle_pcg(N, _d(b), _d(x), thr, norm, max_iter, ctypes.byref(it))
    return x.reshape(N, N, N), int(it.value), bool(ok)


def gather(pos, Q, box, phi, order=2, coulomb_k=1.0, weight_gradient=False):
    N = phi.shape[0]
    pos, Q, phi = _c(pos), _c(Q), _c(phi).ravel()
    F = np.zeros((len(Q), 3), np.float64)
    fn = lib().oracle_gather_weight_gradient if weight_gradient else lib().oracle_gather
    fn(len(Q), _d(pos), _d(Q), box, N, order, _d(phi), coulomb_k, _d(F))
    return F


def energy(phi, q, coulomb_k=1.0):
    N = phi.shape[0]
    return lib().oracle_energy(N, _d(_c(phi).ravel()), _d(_c(q).ravel()), coulomb_k)


def bmh(pos, species, box, table, cutoff=6.0):
    pos = _c(pos)
    F = np.zeros_like(pos)
    e = ctypes.c_double(0.0)
    lib().oracle_bmh(len(pos), _d(pos), _i(_c(species, np.int32)), box,
                     _d(_c(table)), cutoff, _d(F), ctypes.byref(e))
    return F, e.value


class OracleError(RuntimeError):
    pass


class Session:
    """Host-side MaZe session with the same shape as the device C ABI."""

    def __init__(self, charges, pos0, box, grid_spacing, tol=1e-9, order=2,
                 max_iter=100000, residual_norm=NORM_REL2, coulomb_k=1.0, omp=False):
        """omp: run on the OpenMP timing build (bitwise the same results)."""
        self._L = lib_omp() if omp else lib()
        self.charges = _c(charges)
        self.cfg = Config(len(self.charges), order, box, grid_spacing, tol,
                          max_iter, residual_norm, coulomb_k)
        self.box = box
        self.order = order
        self._h = ctypes.c_void_p()
        st = Stats()
        rc = self._L.oracle_init(ctypes.byref(self.cfg), _d(self.charges), _d(_c(pos0)),
                               ctypes.byref(self._h), ctypes.byref(st))
        if rc < 0:
            raise OracleError(f"oracle_init failed with status {rc}")
        self.init_status = rc
        self.init_stats = st.as_dict()
        self.N = self._L.oracle_grid_of(self._h)

    @property
    def n_ions(self):
        return len(self.charges)

    def step(self, pos, want_field=True):
        G = self.N ** 3
        field = np.zeros(G) if want_field else None
        forces = np.zeros((self.n_ions, 3))
        e = np.zeros(1)
        st = Stats()
        rc = self._L.oracle_step(self._h, _d(_c(pos)), _d(field), _d(forces), _d(e),
                               ctypes.byref(st))
        if rc < 0:
            raise OracleError(f"oracle_step failed with status {rc}")
        return dict(status=rc, field=None if field is None else field.reshape((self.N,) * 3),
                    forces=forces, energy=float(e[0]), stats=st.as_dict())

    def solve(self, pos, guess=GUESS_ZERO):
        G = self.N ** 3
        field = np.zeros(G)
        forces = np.zeros((self.n_ions, 3))
        e = np.zeros(1)
        st = Stats()
        rc = self._L.oracle_solve(self._h, guess, _d(_c(pos)), _d(field), _d(forces),
                                _d(e), ctypes.byref(st))
        if rc < 0:
            raise OracleError(f"oracle_solve failed with status {rc}")
        return dict(status=rc, field=field.reshape((self.N,) * 3), forces=forces,
                    energy=float(e[0]), stats=st.as_dict())

    def state(self):
        G = self.N ** 3
        a = [np.zeros(G) for _ in range(5)]
        self._L.oracle_get_state(self._h, *[_d(x) for x in a])
        names = ("phi_k", "phi_km1", "y", "q", "sigma_p")
        return {n: x.reshape((self.N,) * 3) for n, x in zip(names, a)}

    def md_step(self, pos, vel, masses, species, table, cutoff, dt, accel_factor,
                F_es, F_sr, work):
        """One velocity-Verlet step; pos, vel, F_es, F_sr, work updated in place."""
        e_c = ctypes.c_double(0.0)
        v_sr = ctypes.c_double(0.0)
        st = Stats()
        rc = self._L.oracle_md_step(self._h, self.n_ions, _d(pos), _d(vel), _d(masses),
                                  _i(species), _d(_c(table)), cutoff, dt, accel_factor,
                                  _d(F_es), _d(F_sr), _d(work), ctypes.byref(v_sr),
                                  ctypes.byref(e_c), ctypes.byref(st))
        if rc < 0:
            raise OracleError(f"oracle_md_step failed with status {rc}")
        return dict(status=rc, v_sr=v_sr.value, energy_c=e_c.value, stats=st.as_dict())

    def close(self):
        if self._h:
            self._L.oracle_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
