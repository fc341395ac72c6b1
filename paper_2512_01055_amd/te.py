"""ctypes binding to libte.so (include/te.h). Argument marshalling only: every
step of the (T) evaluation runs in the library's gfx950 kernels.

Arrays may be numpy (host memory) or torch tensors on a HIP device (device
memory); one problem uses one kind. Torch is used for device memory and the
stream handle only.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libte.so")

OK, PENDING, EINVAL, ENOMEM, EDEVICE, EBUSY, ENOTFOUND, ECANCELED, EIO = 0, 1, -1, -2, -3, -4, -5, -6, -7
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x2": 3, "fp16x2": 4}
X_MODES = {"auto": 0, "resident": 1, "on_the_fly": 2}


class TeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"te status {status}: {msg}")
        self.status = status


class Problem(C.Structure):
    _fields_ = [("o", C.c_int32), ("v", C.c_int32), ("naux", C.c_int32), ("mem", C.c_int),
                ("eps_occ", C.c_void_p), ("eps_vir", C.c_void_p), ("t1", C.c_void_p),
                ("t2", C.c_void_p), ("B_oo", C.c_void_p), ("B_ov", C.c_void_p),
                ("B_vv", C.c_void_p), ("ovvv", C.c_void_p), ("ovoo", C.c_void_p),
                ("ovov", C.c_void_p)]


class Config(C.Structure):
    _fields_ = [("device", C.c_int), ("stream", C.c_void_p), ("hbm_budget", C.c_size_t),
                ("validate", C.c_int), ("x_mode", C.c_int), ("x_cache_slices", C.c_int),
                ("t2_host", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("seconds", C.c_double), ("flops", C.c_double), ("tflops", C.c_double),
                ("n_triples", C.c_int64), ("stage_seconds", C.c_double),
                ("assemble_flops", C.c_double), ("w_kernel_seconds", C.c_double),
                ("w_launches", C.c_int64), ("e_kernel_seconds", C.c_double),
                ("e_launches", C.c_int64), ("slices_assembled", C.c_int64),
                ("assemble_seconds", C.c_double), ("cache_slices", C.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerConfig(C.Structure):
    _fields_ = [("device", C.c_int), ("hbm_budget", C.c_size_t),
                ("max_resident_jobs", C.c_int), ("max_queued_jobs", C.c_int),
                ("borrow_inputs", C.c_int), ("staging_threads", C.c_int)]


_lib: Optional[C.CDLL] = None

EXPORTS = ["te_init", "te_energy", "te_energy_triples", "te_energy_triples_noalloc",
           "te_energy_terms",
           "te_energy_checkpointed", "te_checkpoint_scan", "te_free", "te_num_triples",
           "te_triple_list", "te_flops_per_triple", "te_plan_slice_loads", "te_server_create", "te_submit",
           "te_poll", "te_wait", "te_server_destroy", "te_strerror", "te_last_error"]


def lib() -> C.CDLL:
    """Load libte.so; fails loudly when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2512_01055_amd.build` (there is no fallback)")
    # torch ships its own HIP runtime; load it first so that libte.so binds to
    # the same one (one runtime per process: device pointers and streams from
    # torch are then valid in the library)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    S, P = C.c_int, C.c_void_p
    L.te_init.argtypes = [C.POINTER(Problem), C.POINTER(Config), C.POINTER(P)]
    L.te_energy.argtypes = [P, S, C.POINTER(C.c_double), C.c_void_p, C.POINTER(Stats)]
    L.te_energy_triples.argtypes = [P, S, C.c_void_p, C.c_int64, C.POINTER(C.c_double),
                                    C.c_void_p, C.POINTER(Stats)]
    L.te_energy_triples_noalloc.argtypes = L.te_energy_triples.argtypes
    D = C.POINTER(C.c_double)
    L.te_energy_terms.argtypes = [P, S, C.c_void_p, C.c_int64, D, D, C.c_void_p, C.c_void_p,
                                  C.POINTER(Stats)]
    L.te_energy_checkpointed.argtypes = [P, S, C.c_char_p, C.c_uint64, C.c_int64, C.c_int64,
                                         D, D, D, C.POINTER(Stats)]
    L.te_checkpoint_scan.argtypes = [C.c_char_p, C.c_int32, C.c_int32, C.c_int32, S,
                                     C.c_uint64, C.c_int64, C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64)]
    L.te_free.argtypes = [P]
    L.te_num_triples.argtypes = [C.c_int32]
    L.te_num_triples.restype = C.c_int64
    L.te_triple_list.argtypes = [C.c_int32, C.c_void_p]
    L.te_flops_per_triple.argtypes = [C.c_int32, C.c_int32]
    L.te_flops_per_triple.restype = C.c_double
    L.te_plan_slice_loads.argtypes = [C.c_int32, C.c_int32, C.c_int32]
    L.te_plan_slice_loads.restype = C.c_int64
    L.te_mfma_sustained.argtypes = [C.c_int, C.c_int, C.c_double, C.POINTER(C.c_double)]
    L.te_mfma_sustained.restype = C.c_int
    L.te_server_create.argtypes = [C.POINTER(ServerConfig), C.POINTER(P)]
    L.te_submit.argtypes = [P, C.POINTER(Problem), S, C.POINTER(C.c_uint64)]
    L.te_poll.argtypes = [P, C.c_uint64, C.POINTER(C.c_double), C.POINTER(Stats)]
    L.te_wait.argtypes = [P, C.c_uint64, C.POINTER(C.c_double), C.POINTER(Stats)]
    L.te_server_destroy.argtypes = [P]
    L.te_strerror.argtypes = [S]
    L.te_strerror.restype = C.c_char_p
    L.te_last_error.restype = C.c_char_p
    for f in ("te_init", "te_energy", "te_energy_triples", "te_energy_triples_noalloc",
              "te_energy_terms",
              "te_energy_checkpointed", "te_checkpoint_scan", "te_free", "te_triple_list",
              "te_server_create", "te_submit", "te_poll", "te_wait", "te_server_destroy"):
        getattr(L, f).restype = S
    _lib = L
    return L


def _check(status: int) -> int:
    if status not in (OK, PENDING):
        raise TeError(status, lib().te_last_error().decode())
    return status


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


class _Arrays:
    """Holds contiguous FP64 buffers (numpy or device torch) for a problem."""

    NAMES = ("eps_occ", "eps_vir", "t1", "t2", "B_oo", "B_ov", "B_vv", "ovvv", "ovoo", "ovov")

    def __init__(self, src):
        self.keep = {}
        kinds = set()
        for n in self.NAMES:
            x = getattr(src, n, None) if not isinstance(src, dict) else src.get(n)
            if x is None:
                continue
            if _is_torch(x):
                import torch
                if x.device.type != "cuda":
                    x = x.detach().cpu().numpy()
                else:
                    x = x.detach().to(torch.float64).contiguous()
                    kinds.add("device")
            if not _is_torch(x):
                x = np.ascontiguousarray(x, dtype=np.float64)
                kinds.add("host")
            self.keep[n] = x
        if len(kinds) > 1:
            raise ValueError("mix of host and device arrays in one problem")
        self.device = kinds == {"device"}

    def ptr(self, n) -> Optional[int]:
        x = self.keep.get(n)
        if x is None:
            return None
        return x.data_ptr() if self.device else x.ctypes.data


def make_problem_struct(src, o: int, v: int, naux: int):
    arrs = _Arrays(src)
    p = Problem()
    p.o, p.v, p.naux = o, v, naux
    p.mem = 1 if arrs.device else 0
    for n in _Arrays.NAMES:
        setattr(p, n, arrs.ptr(n))
    return p, arrs


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Job:
    """One staged (T) problem (te_init ... te_free)."""

    def __init__(self, prob, *, device: int = 0, stream=None, hbm_budget: int = 0,
                 validate: bool = False, x_mode: str = "auto", x_cache_slices: int = 0,
                 explicit: bool = False, t2_host: bool = False):
        L = lib()
        o, v = int(prob.o), int(prob.v)
        naux = 0 if explicit else int(prob.naux)
        self.o, self.v, self.naux = o, v, naux
        self._p, self._arrays = make_problem_struct(prob, o, v, naux)
        cfg = Config(device, _stream_handle(stream), hbm_budget, int(validate),
                     X_MODES[x_mode], x_cache_slices, int(t2_host))
        h = C.c_void_p()
        _check(L.te_init(C.byref(self._p), C.byref(cfg), C.byref(h)))
        self._h = h
        if not self._arrays.device and not t2_host:
            self._arrays = None      # host arrays were copied (a host t2 is borrowed)

    @property
    def n_triples(self) -> int:
        return int(lib().te_num_triples(self.o))

    def energy(self, precision: str = "fp64", per_triple: bool = False):
        """E(T) over all triples; returns (E, stats[, per-triple partials])."""
        L = lib()
        e = C.c_double()
        st = Stats()
        pt = np.zeros(self.n_triples) if per_triple else None
        _check(L.te_energy(self._h, PRECISIONS[precision], C.byref(e),
                           pt.ctypes.data if pt is not None else None, C.byref(st)))
        return (e.value, st.as_dict(), pt) if per_triple else (e.value, st.as_dict())

    def energy_triples(self, ijk: Sequence, precision: str = "fp64"):
        """Weighted partials of the listed triples; returns (sum, partials, stats)."""
        L = lib()
        t = np.ascontiguousarray(np.asarray(ijk, dtype=np.int32).reshape(-1, 3))
        e = C.c_double()
        st = Stats()
        pt = np.zeros(len(t))
        _check(L.te_energy_triples(self._h, PRECISIONS[precision], t.ctypes.data, len(t),
                                   C.byref(e), pt.ctypes.data, C.byref(st)))
        return e.value, pt, st.as_dict()

    def energy_triples_noalloc(self, ijk: Sequence, precision: str = "fp64"):
        """energy_triples through the entry point that allocates no device
        memory (its scratch is a static device array); same returns."""
        L = lib()
        t = np.ascontiguousarray(np.asarray(ijk, dtype=np.int32).reshape(-1, 3))
        e = C.c_double()
        st = Stats()
        pt = np.zeros(len(t))
        _check(L.te_energy_triples_noalloc(self._h, PRECISIONS[precision], t.ctypes.data,
                                           len(t), C.byref(e), pt.ctypes.data, C.byref(st)))
        return e.value, pt, st.as_dict()

    def energy_terms(self, precision: str = "fp64", triples: Optional[Sequence] = None):
        """E(T) split as (E4, E5, e4, e5, stats): the W Z / D and V Z / D parts,
        summed and per triple (all triples in triple_list order when triples
        is None)."""
        L = lib()
        if triples is None:
            t, n = None, int(L.te_num_triples(self.o))
        else:
            t = np.ascontiguousarray(np.asarray(triples, dtype=np.int32).reshape(-1, 3))
            n = len(t)
        e4, e5 = np.zeros(n), np.zeros(n)
        E4, E5 = C.c_double(), C.c_double()
        st = Stats()
        _check(L.te_energy_terms(self._h, PRECISIONS[precision],
                                 None if t is None else t.ctypes.data, n, C.byref(E4),
                                 C.byref(E5), e4.ctypes.data, e5.ctypes.data, C.byref(st)))
        return E4.value, E5.value, e4, e5, st.as_dict()

    def energy_checkpointed(self, precision: str, path: str, chunk: int, tag: int = 0,
                            max_chunks: int = 0):
        """Whole-job evaluation recorded chunk by chunk in `path` (resumed
        when the file exists). Returns (done, E, E4, E5, stats); done is False
        while chunks remain (max_chunks reached), with the energies None."""
        L = lib()
        E, E4, E5 = C.c_double(), C.c_double(), C.c_double()
        st = Stats()
        s = _check(L.te_energy_checkpointed(self._h, PRECISIONS[precision],
                                            os.fsencode(path), tag, chunk, max_chunks,
                                            C.byref(E), C.byref(E4), C.byref(E5), C.byref(st)))
        if s == PENDING:
            return False, None, None, None, st.as_dict()
        return True, E.value, E4.value, E5.value, st.as_dict()

    def free(self) -> None:
        if getattr(self, "_h", None):
            _check(lib().te_free(self._h))
            self._h = None
            self._arrays = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.free()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def triple_list(o: int) -> np.ndarray:
    n = int(lib().te_num_triples(o))
    out = np.zeros((n, 3), dtype=np.int32)
    if n:
        _check(lib().te_triple_list(o, out.ctypes.data))
    return out


def flops_per_triple(o: int, v: int) -> float:
    return float(lib().te_flops_per_triple(o, v))


def mfma_sustained(precision: str = "fp64", seconds: float = 1.0, device: int = 0) -> float:
    """Sustained MFMA TFLOP/s of the device for the W build's instruction."""
    r = C.c_double()
    _check(lib().te_mfma_sustained(device, PRECISIONS[precision], seconds, C.byref(r)))
    return r.value


class Server:
    """Continuous-batching (T) server (te_server_*)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, max_resident_jobs: int = 0,
                 max_queued_jobs: int = 0, borrow_inputs: bool = False, staging_threads: int = 0):
        L = lib()
        cfg = ServerConfig(device, hbm_budget, max_resident_jobs, max_queued_jobs,
                           int(borrow_inputs), staging_threads)
        h = C.c_void_p()
        _check(L.te_server_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self._borrowed = {}        # ticket -> arrays kept alive while the job runs

    def submit(self, prob, precision: str = "fp64") -> int:
        p, arrs = make_problem_struct(prob, int(prob.o), int(prob.v), int(prob.naux))
        if arrs.device:
            raise ValueError("te_submit takes host arrays")
        t = C.c_uint64()
        _check(lib().te_submit(self._h, C.byref(p), PRECISIONS[precision], C.byref(t)))
        self._borrowed[t.value] = arrs
        return t.value

    def poll(self, ticket: int):
        """None while pending, else (E, stats)."""
        e, st = C.c_double(), Stats()
        try:
            s = _check(lib().te_poll(self._h, ticket, C.byref(e), C.byref(st)))
        except TeError:
            self._borrowed.pop(ticket, None)
            raise
        if s == PENDING:
            return None
        self._borrowed.pop(ticket, None)
        return e.value, st.as_dict()

    def wait(self, ticket: int):
        e, st = C.c_double(), Stats()
        try:
            _check(lib().te_wait(self._h, ticket, C.byref(e), C.byref(st)))
        finally:
            self._borrowed.pop(ticket, None)
        return e.value, st.as_dict()

    def close(self) -> None:
        if getattr(self, "_h", None):
            _check(lib().te_server_destroy(self._h))
            self._h = None
            self._borrowed = {}

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def checkpoint_scan(path: str, o: int, v: int, naux: int, precision: str, chunk: int,
                    tag: int = 0):
    """(chunks recorded intact, chunks in the job) of a checkpoint file; no
    device needed."""
    done, total = C.c_int64(), C.c_int64()
    _check(lib().te_checkpoint_scan(os.fsencode(path), o, v, naux, PRECISIONS[precision], tag,
                                    chunk, C.byref(done), C.byref(total)))
    return done.value, total.value
