"""Python binding of libmaze.so (argument marshalling only).

Every function named maze_* forwards to the C entry point of the same name
declared in include/maze.h; torch tensors supply device memory and streams.
All numerical work runs in the library's HIP kernels. If the library has
not been built, importing works but every call raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmaze.so")

MAZE_OK, MAZE_NOT_CONVERGED = 0, 1
MAZE_E_INVALID, MAZE_E_NOT_NEUTRAL, MAZE_E_OOM, MAZE_E_DEVICE, MAZE_E_NONFINITE = -1, -2, -3, -4, -5
MAZE_E_CAPACITY = -6
MAZE_FP64, MAZE_MIXED = 0, 1
MAZE_GUESS_ZERO, MAZE_GUESS_STATIC, MAZE_GUESS_TIMEPROP = 0, 1, 2
MAZE_NORM_REL2, MAZE_NORM_ABSMAX = 0, 1
MAZE_FLAG_MULTIGRID, MAZE_FLAG_WEIGHT_GRADIENT_FORCE, MAZE_FLAG_ALLOW_NET_CHARGE = 1, 2, 4
MAZE_FLAG_GRAPH_CHUNKS = 8
MAZE_FLAG_SSTEP = 16
GRID_PHI, GRID_PHI_PREV, GRID_Y, GRID_Q, GRID_SIGMA = 0, 1, 2, 3, 4

EXPORTED = ("maze_abi_version", "maze_strerror", "maze_device_bytes", "maze_init", "maze_step",
            "maze_solve", "maze_step_batch", "maze_step_batch_noalloc", "maze_grid_n",
            "maze_get_grid",
            "maze_state_bytes", "maze_save", "maze_load", "maze_destroy", "maze_md_prime",
            "maze_md_step", "maze_profile_enable", "maze_profile_read", "maze_trace_enable",
            "maze_trace_read", "maze_md_step_batch", "maze_launch_shape", "maze_basis_shape",
            "maze_sstep_layout",
            "maze_langevin_noise",
            "maze_rdf_accumulate", "maze_tcf_create", "maze_tcf_sample", "maze_tcf_read",
            "maze_tcf_destroy", "maze_batch_create", "maze_batch_add", "maze_batch_advance",
            "maze_batch_take", "maze_batch_in_flight", "maze_batch_destroy",
            "maze_stream_copy")


class maze_config(ctypes.Structure):
    _fields_ = [("n_ions", ctypes.c_int32), ("order", ctypes.c_int32),
                ("box", ctypes.c_double), ("grid_spacing", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("residual_norm", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("coulomb_k", ctypes.c_double),
                ("stream", ctypes.c_void_p)]


class maze_stats(ctypes.Structure):
    _fields_ = [("grid_n", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("refinements", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("status", ctypes.c_int32), ("pad", ctypes.c_int32), ("h", ctypes.c_double), ("rel_residual", ctypes.c_double),
                ("max_abs_residual", ctypes.c_double), ("net_charge", ctypes.c_double),
                ("energy", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class maze_md_state(ctypes.Structure):
    _fields_ = [("n_ions", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("pos_dev", ctypes.c_void_p), ("vel_dev", ctypes.c_void_p),
                ("mass_dev", ctypes.c_void_p), ("species_dev", ctypes.c_void_p),
                ("f_es_dev", ctypes.c_void_p), ("f_sr_dev", ctypes.c_void_p),
                ("scratch_dev", ctypes.c_void_p), ("scalars_dev", ctypes.c_void_p),
                ("dt", ctypes.c_double), ("accel", ctypes.c_double),
                ("cutoff", ctypes.c_double), ("bmh_table", ctypes.c_double * 15),
                ("gamma", ctypes.c_double), ("kT", ctypes.c_double), ("seed", ctypes.c_uint64)]


class MazeError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} (status {status})")


_lib = None


def lib():
    """The loaded libmaze.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, i32 = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32
        L.maze_abi_version.restype = ctypes.c_int
        L.maze_strerror.restype = ctypes.c_char_p
        L.maze_strerror.argtypes = [ctypes.c_int]
        L.maze_device_bytes.restype = ctypes.c_size_t
        L.maze_device_bytes.argtypes = [ctypes.POINTER(maze_config)]
        L.maze_init.restype = ctypes.c_int
        L.maze_init.argtypes = [ctypes.POINTER(maze_config), dp, dp, ctypes.POINTER(vp),
                                ctypes.POINTER(maze_stats)]
        L.maze_step.restype = ctypes.c_int
        L.maze_step.argtypes = [vp, dp, dp, dp, dp, ctypes.POINTER(maze_stats)]
        L.maze_solve.restype = ctypes.c_int
        L.maze_solve.argtypes = [vp, ctypes.c_int, dp, dp, dp, dp, ctypes.POINTER(maze_stats)]
        L.maze_step_batch.restype = ctypes.c_int
        L.maze_step_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(dp),
                                      ctypes.POINTER(dp), dp, ctypes.POINTER(maze_stats)]
        L.maze_step_batch_noalloc.restype = ctypes.c_int
        L.maze_step_batch_noalloc.argtypes = L.maze_step_batch.argtypes
        L.maze_batch_create.restype = ctypes.c_int
        L.maze_batch_create.argtypes = [vp, i32, ctypes.POINTER(vp)]
        L.maze_batch_add.restype = ctypes.c_int
        L.maze_batch_add.argtypes = [vp, vp, ctypes.POINTER(maze_md_state), dp, dp, dp,
                                     ctypes.c_uint64]
        L.maze_batch_advance.restype = ctypes.c_int
        L.maze_batch_advance.argtypes = [vp, ctypes.POINTER(i32)]
        L.maze_batch_take.restype = ctypes.c_int
        L.maze_batch_take.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(maze_stats), ctypes.POINTER(i32)]
        L.maze_batch_in_flight.restype = ctypes.c_int
        L.maze_batch_in_flight.argtypes = [vp]
        L.maze_batch_destroy.restype = None
        L.maze_batch_destroy.argtypes = [vp]
        L.maze_stream_copy.restype = ctypes.c_int
        L.maze_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.maze_grid_n.restype = ctypes.c_int
        L.maze_grid_n.argtypes = [vp]
        L.maze_get_grid.restype = ctypes.c_int
        L.maze_get_grid.argtypes = [vp, ctypes.c_int, dp]
        L.maze_state_bytes.restype = ctypes.c_size_t
        L.maze_state_bytes.argtypes = [vp]
        L.maze_save.restype = ctypes.c_int
        L.maze_save.argtypes = [vp, ctypes.c_void_p, ctypes.c_size_t]
        L.maze_load.restype = ctypes.c_int
        L.maze_load.argtypes = [vp, ctypes.c_void_p, ctypes.c_size_t]
        L.maze_destroy.restype = None
        L.maze_destroy.argtypes = [vp]
        L.maze_md_prime.restype = ctypes.c_int
        L.maze_md_prime.argtypes = [vp, ctypes.POINTER(maze_md_state), ctypes.POINTER(maze_stats)]
        L.maze_md_step.restype = ctypes.c_int
        L.maze_md_step.argtypes = [vp, ctypes.POINTER(maze_md_state), ctypes.POINTER(maze_stats)]
        L.maze_profile_enable.restype = ctypes.c_int
        L.maze_profile_enable.argtypes = [vp, ctypes.c_int]
        L.maze_profile_read.restype = ctypes.c_int
        L.maze_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.maze_launch_shape.restype = ctypes.c_int
        L.maze_launch_shape.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
        L.maze_basis_shape.restype = ctypes.c_int
        L.maze_basis_shape.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
        L.maze_sstep_layout.restype = ctypes.c_int
        L.maze_sstep_layout.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
        L.maze_md_step_batch.restype = ctypes.c_int
        L.maze_md_step_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), i32,
                                         ctypes.POINTER(maze_stats)]
        L.maze_trace_enable.restype = ctypes.c_int
        L.maze_trace_enable.argtypes = [vp, ctypes.c_int]
        L.maze_trace_read.restype = ctypes.c_int
        L.maze_trace_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int)]
        L.maze_langevin_noise.restype = ctypes.c_int
        L.maze_langevin_noise.argtypes = [ctypes.c_uint64, ctypes.c_int64, i32, i32, vp, vp]
        L.maze_rdf_accumulate.restype = ctypes.c_int
        L.maze_rdf_accumulate.argtypes = [vp, vp, i32, ctypes.c_double, vp, i32, vp, vp]
        L.maze_tcf_create.restype = ctypes.c_int
        L.maze_tcf_create.argtypes = [i32, vp, i32, i32, vp, ctypes.POINTER(vp)]
        L.maze_tcf_sample.restype = ctypes.c_int
        L.maze_tcf_sample.argtypes = [vp, vp, vp]
        L.maze_tcf_read.restype = ctypes.c_int
        L.maze_tcf_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64)]
        L.maze_tcf_destroy.restype = None
        L.maze_tcf_destroy.argtypes = [vp]
        _lib = L
    return _lib


def strerror(status: int) -> str:
    try:
        return lib().maze_strerror(status).decode()
    except RuntimeError:
        return f"status {status}"


def _ptr(t: Optional[torch.Tensor], dtype=torch.float64, numel: Optional[int] = None):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} device tensor, got {t.dtype} "
                         f"on {t.device} (contiguous={t.is_contiguous()})")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise MazeError(rc, where)
    return rc


# ---- thin functions with the C names ----------------------------------------
def maze_abi_version() -> int:
    return lib().maze_abi_version()


def maze_device_bytes(cfg: maze_config) -> int:
    return int(lib().maze_device_bytes(ctypes.byref(cfg)))


def maze_init(cfg: maze_config, charges: torch.Tensor, pos0: torch.Tensor):
    h = ctypes.c_void_p()
    st = maze_stats()
    rc = lib().maze_init(ctypes.byref(cfg), _ptr(charges, numel=cfg.n_ions),
                         _ptr(pos0, numel=3 * cfg.n_ions), ctypes.byref(h), ctypes.byref(st))
    _check(rc, "maze_init")
    return h, rc, st.as_dict()


def maze_step(handle, pos, field=None, forces=None, energy=None, want_stats=True):
    st = maze_stats() if want_stats else None
    rc = lib().maze_step(handle, _ptr(pos), _ptr(field), _ptr(forces), _ptr(energy),
                         ctypes.byref(st) if st is not None else None)
    _check(rc, "maze_step")
    return rc, (st.as_dict() if st is not None else None)


def maze_solve(handle, guess, pos, field=None, forces=None, energy=None, want_stats=True):
    st = maze_stats() if want_stats else None
    rc = lib().maze_solve(handle, guess, _ptr(pos), _ptr(field), _ptr(forces), _ptr(energy),
                          ctypes.byref(st) if st is not None else None)
    _check(rc, "maze_solve")
    return rc, (st.as_dict() if st is not None else None)


def maze_step_batch(handles: Sequence, pos: Sequence[torch.Tensor],
                    forces: Optional[Sequence[Optional[torch.Tensor]]] = None,
                    energies: Optional[torch.Tensor] = None, want_stats=True):
    """Steps the sessions together. Returns (worst status, per-session stats
    with their own "status"). Raises only for errors of the call as a whole
    (invalid arguments, device or allocation failure); a rejected session is
    reported in its stats entry."""
    n = len(handles)
    H = (ctypes.c_void_p * n)(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    P = (ctypes.c_void_p * n)(*[_ptr(p).value for p in pos])
    F = None
    if forces is not None:
        F = (ctypes.c_void_p * n)(*[(_ptr(f).value if f is not None else None) for f in forces])
    st = (maze_stats * n)() if want_stats else None
    rc = lib().maze_step_batch(H, n, P, F, _ptr(energies, numel=n) if energies is not None else None,
                               st)
    if rc in (MAZE_E_INVALID, MAZE_E_OOM, MAZE_E_DEVICE):
        raise MazeError(rc, "maze_step_batch")
    return rc, ([x.as_dict() for x in st] if st is not None else None)


def maze_step_batch_noalloc(handles: Sequence, pos: Sequence[torch.Tensor],
                            forces: Optional[Sequence[Optional[torch.Tensor]]] = None,
                            energies: Optional[torch.Tensor] = None, want_stats=True):
    """maze_step_batch through the entry point that allocates nothing (its
    batch table is a fixed device array of the library, at most 256
    sessions). Same returns; raises MazeError(MAZE_E_CAPACITY) above 256."""
    n = len(handles)
    H = (ctypes.c_void_p * n)(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    P = (ctypes.c_void_p * n)(*[_ptr(p).value for p in pos])
    F = None
    if forces is not None:
        F = (ctypes.c_void_p * n)(*[(_ptr(f).value if f is not None else None) for f in forces])
    st = (maze_stats * n)() if want_stats else None
    rc = lib().maze_step_batch_noalloc(H, n, P, F,
                                       _ptr(energies, numel=n) if energies is not None else None,
                                       st)
    if rc in (MAZE_E_INVALID, MAZE_E_OOM, MAZE_E_DEVICE, MAZE_E_CAPACITY):
        raise MazeError(rc, "maze_step_batch_noalloc")
    return rc, ([x.as_dict() for x in st] if st is not None else None)


def maze_stream_copy(dst: torch.Tensor, src: torch.Tensor, stream=None):
    """Streaming copy src -> dst (same byte size, a multiple of 16)."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(lib().maze_stream_copy(ctypes.c_void_p(dst.data_ptr()),
                                  ctypes.c_void_p(src.data_ptr()), nbytes,
                                  ctypes.c_void_p(int(stream))), "maze_stream_copy")


def maze_grid_n(handle) -> int:
    return lib().maze_grid_n(handle)


def maze_get_grid(handle, which: int, out: torch.Tensor):
    _check(lib().maze_get_grid(handle, which, _ptr(out)), "maze_get_grid")
    return out


def maze_state_bytes(handle) -> int:
    return int(lib().maze_state_bytes(handle))


def maze_save(handle) -> bytes:
    n = maze_state_bytes(handle)
    buf = ctypes.create_string_buffer(n)
    _check(lib().maze_save(handle, buf, n), "maze_save")
    return buf.raw


def maze_load(handle, blob: bytes):
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(lib().maze_load(handle, buf, len(blob)), "maze_load")


def maze_destroy(handle):
    lib().maze_destroy(handle)


def maze_md_prime(handle, md: maze_md_state, want_stats=True):
    st = maze_stats() if want_stats else None
    rc = _check(lib().maze_md_prime(handle, ctypes.byref(md),
                                    ctypes.byref(st) if st is not None else None), "maze_md_prime")
    return rc, (st.as_dict() if st is not None else None)


def maze_md_step(handle, md: maze_md_state, want_stats=True):
    st = maze_stats() if want_stats else None
    rc = _check(lib().maze_md_step(handle, ctypes.byref(md),
                                   ctypes.byref(st) if st is not None else None), "maze_md_step")
    return rc, (st.as_dict() if st is not None else None)


def maze_md_step_batch(handles: Sequence, mds: Sequence[maze_md_state], want_stats=True):
    """One MD step of several sessions together; (worst status, per-session
    stats). Raises only for errors of the call as a whole."""
    n = len(handles)
    H = (ctypes.c_void_p * n)(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    M = (ctypes.c_void_p * n)(*[ctypes.cast(ctypes.pointer(m), ctypes.c_void_p).value for m in mds])
    st = (maze_stats * n)() if want_stats else None
    rc = lib().maze_md_step_batch(H, M, n, st)
    if rc in (MAZE_E_INVALID, MAZE_E_OOM, MAZE_E_DEVICE):
        raise MazeError(rc, "maze_md_step_batch")
    return rc, ([x.as_dict() for x in st] if st is not None else None)


def maze_profile_enable(handle, on: bool = True):
    _check(lib().maze_profile_enable(handle, int(bool(on))), "maze_profile_enable")


def maze_profile_read(handle) -> dict:
    out = (ctypes.c_double * 8)()
    _check(lib().maze_profile_read(handle, out), "maze_profile_read")
    v = list(out)
    # with MAZE_FLAG_SSTEP a timed unit is a two-iteration outer step, and
    # *_update_ms is the time of its update kernels
    return dict(fp64_sweep=(int(v[0]), v[1]), fp32_sweep=(int(v[2]), v[3]),
                fp64_iters=int(v[4]), fp32_iters=int(v[5]), fp64_update_ms=v[6],
                fp32_update_ms=v[7])


def maze_launch_shape(handle) -> dict:
    """Latency and throughput launch shapes of the session's CG sweep."""
    out = (ctypes.c_int32 * 8)()
    _check(lib().maze_launch_shape(handle, out), "maze_launch_shape")
    return {k: dict(ppt=out[4 * i], cx=out[4 * i + 1], nwg=out[4 * i + 2],
                    segment=out[4 * i + 3])
            for i, k in enumerate(("latency", "throughput"))}


def maze_basis_shape(handle) -> dict:
    """Launch shape of the basis kernel of the two-iteration CG."""
    out = (ctypes.c_int32 * 4)()
    _check(lib().maze_basis_shape(handle, out), "maze_basis_shape")
    return dict(threads=out[0], ppt=out[1], cx=out[2], nwg=out[3])


def maze_sstep_layout(handle) -> dict:
    """Wavefronts per workgroup of the two-iteration kernels' wavefront-row
    layout (0: segment layout), basis and update kernel."""
    out = (ctypes.c_int32 * 2)()
    _check(lib().maze_sstep_layout(handle, out), "maze_sstep_layout")
    return dict(basis=out[0], update=out[1])


def maze_trace_enable(handle, on: bool = True):
    _check(lib().maze_trace_enable(handle, int(bool(on))), "maze_trace_enable")


def maze_trace_read(handle):
    """Rows (pass, iteration, relative residual) of the last solve, as a
    list of tuples; iteration -1 marks an FP64 true residual."""
    n = ctypes.c_int(0)
    _check(lib().maze_trace_read(handle, None, 0, ctypes.byref(n)), "maze_trace_read")
    buf = (ctypes.c_double * (3 * max(n.value, 1)))()
    _check(lib().maze_trace_read(handle, buf, n.value, ctypes.byref(n)), "maze_trace_read")
    v = list(buf)
    return [(int(v[3 * i]), int(v[3 * i + 1]), v[3 * i + 2]) for i in range(n.value)]


# ---- convenience wrapper -------------------------------------------------------
def make_config(n_ions, box, grid_spacing, tol=1e-9, order=2, max_iter=100000,
                precision=MAZE_FP64, residual_norm=MAZE_NORM_REL2, coulomb_k=1.0,
                stream=None, flags=0) -> maze_config:
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    return maze_config(int(n_ions), int(order), float(box), float(grid_spacing), float(tol),
                       int(max_iter), int(precision), int(residual_norm), int(flags),
                       float(coulomb_k), ctypes.c_void_p(int(stream)))


class Session:
    """One MaZe session: owns the device state of one system."""

    def __init__(self, charges: torch.Tensor, pos0: torch.Tensor, box: float,
                 grid_spacing: float, tol: float = 1e-9, order: int = 2,
                 max_iter: int = 100000, precision: int = MAZE_FP64,
                 residual_norm: int = MAZE_NORM_REL2, coulomb_k: float = 1.0,
                 stream=None, flags: int = 0):
        self.cfg = make_config(charges.numel(), box, grid_spacing, tol, order, max_iter,
                               precision, residual_norm, coulomb_k, stream, flags)
        self.device = charges.device
        self.handle, self.init_status, self.init_stats = maze_init(
            self.cfg, charges.contiguous(), pos0.contiguous())
        self.N = maze_grid_n(self.handle)
        self.n_ions = int(charges.numel())

    def _new(self, *shape):
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    def step(self, pos, want_field=False, want_forces=True, want_stats=True):
        field = self._new(self.N, self.N, self.N) if want_field else None
        forces = self._new(self.n_ions, 3) if want_forces else None
        energy = self._new(1)
        rc, st = maze_step(self.handle, pos.contiguous(), field, forces, energy, want_stats)
        return dict(status=rc, field=field, forces=forces, energy=energy, stats=st)

    def solve(self, pos, guess=MAZE_GUESS_ZERO, want_field=True):
        field = self._new(self.N, self.N, self.N) if want_field else None
        forces = self._new(self.n_ions, 3)
        energy = self._new(1)
        rc, st = maze_solve(self.handle, guess, pos.contiguous(), field, forces, energy)
        return dict(status=rc, field=field, forces=forces, energy=energy, stats=st)

    def grid(self, which: int) -> torch.Tensor:
        return maze_get_grid(self.handle, which, self._new(self.N, self.N, self.N))

    def save(self) -> bytes:
        return maze_save(self.handle)

    def load(self, blob: bytes):
        maze_load(self.handle, blob)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            maze_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Continuous batch of steps in flight (maze_batch_*): steps join the
    running batched CG launches when added and leave them when their solve
    ends; each result is bitwise the one the session gets stepped alone."""

    def __init__(self, max_sessions: int = 256, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.handle = ctypes.c_void_p()
        _check(lib().maze_batch_create(ctypes.c_void_p(int(stream)), int(max_sessions),
                                       ctypes.byref(self.handle)), "maze_batch_create")
        self.cap = int(max_sessions)

    def add_md(self, handle, md: "maze_md_state", tag: int):
        """One MD step (maze_md_step) of the session; md's buffers stay in use
        until the step is taken."""
        _check(lib().maze_batch_add(self.handle, handle, ctypes.byref(md), None, None, None,
                                    int(tag)), "maze_batch_add")

    def add(self, handle, pos: torch.Tensor, forces: Optional[torch.Tensor] = None,
            energy: Optional[torch.Tensor] = None, tag: int = 0):
        """One MaZe step (maze_step) at pos; forces and energy are written
        when the step finishes."""
        _check(lib().maze_batch_add(self.handle, handle, None, _ptr(pos), _ptr(forces),
                                    _ptr(energy, numel=1) if energy is not None else None,
                                    int(tag)), "maze_batch_add")

    def advance(self) -> int:
        n = ctypes.c_int32(0)
        _check(lib().maze_batch_advance(self.handle, ctypes.byref(n)), "maze_batch_advance")
        return int(n.value)

    def take(self, max_n: Optional[int] = None):
        """Ready steps, oldest first: list of (tag, stats dict with "status")."""
        m = self.cap if max_n is None else int(max_n)
        tags = (ctypes.c_uint64 * max(m, 1))()
        st = (maze_stats * max(m, 1))()
        n = ctypes.c_int32(0)
        _check(lib().maze_batch_take(self.handle, m, tags, st, ctypes.byref(n)),
               "maze_batch_take")
        return [(int(tags[i]), st[i].as_dict()) for i in range(n.value)]

    def in_flight(self) -> int:
        return int(lib().maze_batch_in_flight(self.handle))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().maze_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
