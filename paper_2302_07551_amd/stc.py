"""Python binding of the staircase solver's C ABI (include/stc.h).

Argument marshalling only: every step of the method runs in the HIP library
libstc.so.  PyTorch provides the device arena (a uint8 tensor sized by
stc_footprint_bytes) and the stream.  If the library is not built, or no GPU
is visible, the calls raise; there is no fallback implementation.

The functions keep the C names (stc_setup, stc_solve, ...); ``Solver`` wraps
them for convenience.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstc.so")

STC_OK, STC_EINVAL, STC_ENOTGEN, STC_ESINGULAR, STC_EDEGENERATE, STC_EMAXIT, STC_ENOMEM, \
    STC_EDEVICE = range(8)
STC_FP64, STC_FP32, STC_MIXED = 0, 1, 2
STC_STOP_DIFF, STC_STOP_RESIDUAL = 0, 1
STC_MEM_HOST, STC_MEM_DEVICE = 0, 1
STC_DENSE, STC_SPARSE = 0, 1
STC_ANY_PATTERN = -1          # stc_generator.b: a generator of any block pattern
STC_STAIRCASE, STC_JGS = 0, 1   # stc_options.method
METHODS = {"staircase": STC_STAIRCASE, "jgs": STC_JGS}

PRECISIONS = {"fp64": STC_FP64, "fp32": STC_FP32, "mixed": STC_MIXED}
STOPS = {"diff": STC_STOP_DIFF, "residual": STC_STOP_RESIDUAL}

# every symbol include/stc.h declares
EXPORTS = ("stc_footprint_bytes", "stc_setup", "stc_prepare", "stc_setup_prepared",
           "stc_prepared_free", "stc_solve", "stc_solve_gmres", "stc_step",
           "stc_residual", "stc_residual_noalloc",
           "stc_sweeps", "stc_profile_sweeps", "stc_phase_bytes", "stc_variant_count",
           "stc_set_variant", "stc_get_variant", "stc_autotune", "stc_load", "stc_query",
           "stc_store", "stc_promote", "stc_batch_footprint", "stc_batch_create",
           "stc_batch_set", "stc_batch_autotune", "stc_batch_get_tile", "stc_batch_sweeps",
           "stc_batch_query", "stc_batch_sync",
           "stc_batch_destroy",
           "stc_destroy",
           "stc_status_string", "stc_last_error")


class stc_generator(ctypes.Structure):
    _fields_ = [("L", c_int32), ("m", c_int32), ("b", c_int32), ("sizes", POINTER(c_int32)),
                ("blocks", POINTER(c_double)), ("recompute_diagonal", c_int32),
                ("csr_rowptr", c_void_p), ("csr_col", c_void_p), ("csr_val", c_void_p)]


class stc_options(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("stair_type", c_int32), ("stop", c_int32),
                ("check_every", c_int32), ("switch_tol", c_double), ("stream", c_void_p),
                ("arena", c_void_p), ("arena_bytes", c_size_t), ("format", c_int32),
                ("krylov_restart", c_int32), ("krylov_keep_all", c_int32),
                ("method", c_int32), ("jgs_chunks", c_int32)]


class stc_result(ctypes.Structure):
    _fields_ = [("residual_1", c_double), ("diff_1", c_double), ("iters", c_int64),
                ("iters_fp32", c_int64), ("status", c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


_lib = None

# Solvers and batches still open when the interpreter exits are closed by an
# exit handler, in a fixed order (batches, then handles), rather than by
# whatever order the garbage collector finds them in during teardown.
_live_batches: "weakref.WeakSet" = weakref.WeakSet()
_live_solvers: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _close_live():
    for group in (_live_batches, _live_solvers):
        for obj in list(group):
            try:
                obj.close()
            except Exception:
                pass


def load_library(path: str = LIB_PATH):
    """Load libstc.so and declare its signatures; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    H = c_void_p
    dp = POINTER(c_double)
    lib.stc_footprint_bytes.argtypes = [POINTER(stc_generator), POINTER(stc_options)]
    lib.stc_footprint_bytes.restype = c_size_t
    lib.stc_setup.argtypes = [POINTER(stc_generator), POINTER(stc_options), POINTER(H)]
    lib.stc_prepare.argtypes = [POINTER(stc_generator), POINTER(stc_options), POINTER(H)]
    lib.stc_setup_prepared.argtypes = [H, POINTER(stc_options), POINTER(H)]
    lib.stc_prepared_free.argtypes = [H]
    lib.stc_prepared_free.restype = None
    lib.stc_solve.argtypes = [H, c_void_p, c_double, c_int64, c_void_p, POINTER(stc_result),
                              c_int32]
    lib.stc_solve_gmres.argtypes = [H, c_void_p, c_int32, c_double, c_int64, c_void_p,
                                    POINTER(stc_result), c_int32]
    lib.stc_step.argtypes = [H, c_void_p, c_void_p, dp, c_int32]
    lib.stc_residual.argtypes = [H, c_void_p, dp, c_int32]
    lib.stc_residual_noalloc.argtypes = [H, c_void_p, c_void_p]
    lib.stc_sweeps.argtypes = [H, c_int64, c_void_p]
    lib.stc_profile_sweeps.argtypes = [H, c_int64, dp, dp, dp, dp]
    lib.stc_variant_count.argtypes = []
    lib.stc_variant_count.restype = c_int32
    lib.stc_set_variant.argtypes = [H, c_int32, c_int32]
    lib.stc_get_variant.argtypes = [H, c_int32, POINTER(c_int32)]
    lib.stc_autotune.argtypes = [H, c_int32, dp, dp]
    lib.stc_phase_bytes.argtypes = [H, dp, dp]
    lib.stc_load.argtypes = [H, c_void_p, c_int32]
    lib.stc_query.argtypes = [H, POINTER(c_int64), POINTER(c_int32), dp]
    lib.stc_store.argtypes = [H, c_void_p, c_int32]
    lib.stc_promote.argtypes = [H]
    lib.stc_batch_footprint.argtypes = [c_int32, c_int64]
    lib.stc_batch_footprint.restype = c_size_t
    lib.stc_batch_create.argtypes = [c_int32, c_int64, c_int32, c_void_p, c_void_p, c_size_t,
                                     POINTER(H)]
    lib.stc_batch_set.argtypes = [H, POINTER(H), c_int32, c_double, c_int32]
    lib.stc_batch_autotune.argtypes = [H, c_int32, dp]
    lib.stc_batch_get_tile.argtypes = [H, c_int32, c_int32, POINTER(c_int32), POINTER(c_int32),
                                       POINTER(c_int32)]
    lib.stc_batch_sweeps.argtypes = [H, c_int64, c_int32]
    lib.stc_batch_query.argtypes = [H, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.stc_batch_sync.argtypes = [H]
    lib.stc_batch_destroy.argtypes = [H]
    lib.stc_batch_destroy.restype = None
    lib.stc_destroy.argtypes = [H]
    lib.stc_destroy.restype = None
    lib.stc_status_string.argtypes = [c_int32]
    lib.stc_status_string.restype = ctypes.c_char_p
    lib.stc_last_error.argtypes = []
    lib.stc_last_error.restype = ctypes.c_char_p
    for name in ("stc_setup", "stc_prepare", "stc_setup_prepared", "stc_solve", "stc_step", "stc_residual", "stc_sweeps",
                 "stc_profile_sweeps", "stc_phase_bytes", "stc_set_variant", "stc_get_variant",
                 "stc_autotune", "stc_load", "stc_query", "stc_store", "stc_promote",
                 "stc_batch_create", "stc_batch_set", "stc_batch_sweeps", "stc_batch_query",
                 "stc_batch_sync"):
        getattr(lib, name).restype = c_int32
    _lib = lib
    return lib


def _check(status: int, allow=(STC_OK,)):
    if status in allow:
        return status
    lib = load_library()
    raise StcError(status, lib.stc_last_error().decode() or lib.stc_status_string(status).decode())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def make_generator(blocks: np.ndarray, sizes, b: int, recompute_diagonal: bool = False):
    """Marshal [L][2b+1][m][m] blocks (+ sizes) into the C struct; returns
    (struct, keep-alive tuple)."""
    blocks = _f64(blocks)
    L, nb, m, m2 = blocks.shape
    if nb != 2 * b + 1 or m != m2:
        raise ValueError("blocks must have shape [L, 2b+1, m, m]")
    sz = None if sizes is None else np.ascontiguousarray(sizes, dtype=np.int32)
    g = stc_generator(L, m, b,
                      sz.ctypes.data_as(POINTER(c_int32)) if sz is not None else None,
                      blocks.ctypes.data_as(POINTER(c_double)), int(bool(recompute_diagonal)))
    return g, (blocks, sz)


def make_generator_csr(indptr, indices, data, sizes, b: int, m: int | None = None,
                       recompute_diagonal: bool = False):
    """Marshal an N x N generator in CSR form (states numbered level by level,
    level sizes `sizes`) into the C struct; returns (struct, keep-alive)."""
    sz = np.ascontiguousarray(sizes, dtype=np.int32)
    rp = np.ascontiguousarray(indptr, dtype=np.int64)
    col = np.ascontiguousarray(indices, dtype=np.int32)
    val = _f64(data)
    if rp.shape != (int(sz.sum()) + 1,) or col.shape != val.shape:
        raise ValueError("need indptr of length N+1 and matching indices and data")
    L = len(sz)
    m = int(sz.max()) if m is None else int(m)
    g = stc_generator(L, m, b, sz.ctypes.data_as(POINTER(c_int32)), None,
                      int(bool(recompute_diagonal)), rp.ctypes.data, col.ctypes.data,
                      val.ctypes.data)
    return g, (sz, rp, col, val)


FORMATS = {"dense": STC_DENSE, "sparse": STC_SPARSE}


def make_options(precision="fp64", stair_type=1, stop="diff", check_every=1, switch_tol=0.0,
                 stream=0, arena=0, arena_bytes=0, format="dense", krylov_restart=0,
                 krylov_keep_all=False, method="staircase", jgs_chunks=0):
    return stc_options(PRECISIONS[precision] if isinstance(precision, str) else int(precision),
                       int(stair_type), STOPS[stop] if isinstance(stop, str) else int(stop),
                       int(check_every), float(switch_tol), stream or None, arena or None,
                       int(arena_bytes), FORMATS[format] if isinstance(format, str) else int(format),
                       int(krylov_restart), int(bool(krylov_keep_all)),
                       METHODS[method] if isinstance(method, str) else int(method),
                       int(jgs_chunks))


def stc_footprint_bytes(gen: stc_generator, opt: stc_options) -> int:
    return int(load_library().stc_footprint_bytes(byref(gen), byref(opt)))


def stc_setup(gen: stc_generator, opt: stc_options) -> c_void_p:
    h = c_void_p()
    _check(load_library().stc_setup(byref(gen), byref(opt), byref(h)))
    return h


def stc_prepare(gen: stc_generator, opt: stc_options) -> c_void_p:
    """Host half of stc_setup (no HIP call: any thread)."""
    p = c_void_p()
    _check(load_library().stc_prepare(byref(gen), byref(opt), byref(p)))
    return p


def stc_setup_prepared(p, opt: stc_options) -> c_void_p:
    h = c_void_p()
    _check(load_library().stc_setup_prepared(p, byref(opt), byref(h)))
    return h


def stc_prepared_free(p):
    if p:
        load_library().stc_prepared_free(p)


def _vec_arg(x):
    """(pointer, where) for a numpy array (host) or a torch CUDA tensor (device)."""
    if x is None:
        return None, STC_MEM_HOST
    if hasattr(x, "data_ptr") and getattr(x, "is_cuda", False):
        if x.dtype.__repr__() != "torch.float64" or not x.is_contiguous():
            raise ValueError("device vectors must be contiguous float64 tensors")
        return c_void_p(x.data_ptr()), STC_MEM_DEVICE
    if not (isinstance(x, np.ndarray) and x.dtype == np.float64 and x.flags.c_contiguous):
        raise ValueError("host vectors must be contiguous float64 numpy arrays")
    return c_void_p(x.ctypes.data), STC_MEM_HOST


def stc_solve(h, x0, tol: float, maxit: int, pi, allow_maxit: bool = True) -> dict:
    px, w1 = _vec_arg(x0)
    pp, w2 = _vec_arg(pi)
    if x0 is not None and w1 != w2:
        raise ValueError("x0 and pi must both be host or both be device memory")
    res = stc_result()
    allow = (STC_OK, STC_EMAXIT) if allow_maxit else (STC_OK,)
    _check(load_library().stc_solve(h, px, float(tol), int(maxit), pp, byref(res), w2), allow)
    return res.as_dict()


def stc_solve_gmres(h, x0, restart: int, tol: float, max_applies: int, pi,
                    allow_maxit: bool = True) -> dict:
    px, w1 = _vec_arg(x0)
    pp, w2 = _vec_arg(pi)
    if x0 is not None and w1 != w2:
        raise ValueError("x0 and pi must both be host or both be device memory")
    res = stc_result()
    allow = (STC_OK, STC_EMAXIT) if allow_maxit else (STC_OK,)
    _check(load_library().stc_solve_gmres(h, px, int(restart), float(tol), int(max_applies), pp,
                                          byref(res), w2), allow)
    return res.as_dict()


def stc_step(h, x, z) -> float:
    px, w1 = _vec_arg(x)
    pz, w2 = _vec_arg(z)
    if w1 != w2:
        raise ValueError("x and z must both be host or both be device memory")
    d = c_double()
    _check(load_library().stc_step(h, px, pz, byref(d), w1))
    return d.value


def stc_residual(h, x) -> float:
    px, w = _vec_arg(x)
    r = c_double()
    _check(load_library().stc_residual(h, px, byref(r), w))
    return r.value


def stc_residual_noalloc(h, x, res):
    """x: CUDA tensor of N FP64; res: CUDA tensor with room for one FP64
    (written asynchronously on the handle's stream)."""
    _check(load_library().stc_residual_noalloc(h, c_void_p(x.data_ptr()),
                                               c_void_p(res.data_ptr())))


def stc_sweeps(h, nsweeps: int, diffs: np.ndarray | None = None):
    p = None if diffs is None else c_void_p(diffs.ctypes.data)
    _check(load_library().stc_sweeps(h, int(nsweeps), p))


def stc_profile_sweeps(h, nsweeps: int):
    """(ms phase A, ms phase B, ms finalize, ms whole sweep), means per sweep."""
    a, b, f, t = c_double(), c_double(), c_double(), c_double()
    _check(load_library().stc_profile_sweeps(h, int(nsweeps), byref(a), byref(b), byref(f),
                                             byref(t)))
    return a.value, b.value, f.value, t.value


def stc_variant_count() -> int:
    return int(load_library().stc_variant_count())


def stc_set_variant(h, stage: int, variant: int):
    _check(load_library().stc_set_variant(h, int(stage), int(variant)))


def stc_get_variant(h, stage: int) -> int:
    v = c_int32()
    _check(load_library().stc_get_variant(h, int(stage), byref(v)))
    return v.value


def stc_autotune(h, trial_sweeps: int = 20):
    """Returns (best ms per FP64 sweep, best ms per FP32 sweep); NaN for a
    stage the handle does not sweep in."""
    a, b = c_double(float("nan")), c_double(float("nan"))
    _check(load_library().stc_autotune(h, int(trial_sweeps), byref(a), byref(b)))
    return a.value, b.value


def stc_phase_bytes(h):
    a, b = c_double(), c_double()
    _check(load_library().stc_phase_bytes(h, byref(a), byref(b)))
    return a.value, b.value


def stc_load(h, x):
    px, w = _vec_arg(x)
    _check(load_library().stc_load(h, px, w))


def stc_query(h):
    s, f, d = c_int64(), c_int32(), c_double()
    _check(load_library().stc_query(h, byref(s), byref(f), byref(d)))
    return s.value, bool(f.value), d.value


def stc_store(h, pi):
    pp, w = _vec_arg(pi)
    _check(load_library().stc_store(h, pp, w))


def stc_promote(h):
    _check(load_library().stc_promote(h))


def stc_batch_footprint(max_chains: int, max_items: int) -> int:
    return int(load_library().stc_batch_footprint(int(max_chains), int(max_items)))


def stc_batch_create(max_chains: int, max_items: int, b: int, stream: int, arena: int,
                     arena_bytes: int):
    bt = c_void_p()
    _check(load_library().stc_batch_create(int(max_chains), int(max_items), int(b),
                                           stream or None, arena or None, int(arena_bytes),
                                           byref(bt)))
    return bt


def stc_batch_set(bt, handles, tol: float, nontemporal: bool = False):
    arr = (c_void_p * max(len(handles), 1))(*[h.value if isinstance(h, c_void_p) else h
                                             for h in handles])
    _check(load_library().stc_batch_set(bt, arr, len(handles), float(tol), int(bool(nontemporal))))


def stc_batch_autotune(bt, trial_sweeps: int = 20) -> float:
    """Tune the batch's launch shapes on its chains; ms per sweep with them."""
    ms = c_double(float("nan"))
    _check(load_library().stc_batch_autotune(bt, int(trial_sweeps), byref(ms)))
    return ms.value


def stc_batch_get_tile(bt, stage: int, mp: int) -> dict:
    v, per, grid = c_int32(), c_int32(), c_int32()
    _check(load_library().stc_batch_get_tile(bt, int(stage), int(mp), byref(v), byref(per),
                                             byref(grid)))
    return {"variant": v.value, "groups_per_item": per.value, "grid": grid.value}


def stc_batch_sweeps(bt, nsweeps: int, use_graph: bool = True):
    _check(load_library().stc_batch_sweeps(bt, int(nsweeps), int(bool(use_graph))))


def stc_batch_query(bt, count: int):
    """(sweeps, stopped, diff_1, status) arrays over the batch's chains, in
    the order of the last stc_batch_set."""
    sweeps = np.zeros(count, dtype=np.int64)
    stopped = np.zeros(count, dtype=np.int32)
    diffs = np.zeros(count, dtype=np.float64)
    status = np.zeros(count, dtype=np.int32)
    _check(load_library().stc_batch_query(bt, sweeps.ctypes.data, stopped.ctypes.data,
                                          diffs.ctypes.data, status.ctypes.data))
    return sweeps, stopped.astype(bool), diffs, status


def stc_batch_sync(bt):
    _check(load_library().stc_batch_sync(bt))


def stc_batch_destroy(bt):
    if bt:
        load_library().stc_batch_destroy(bt)


class Batch:
    """Many chains swept together (owns the batch tables' torch arena)."""

    def __init__(self, max_chains: int, max_items: int, b: int = 1, device=None, stream=None):
        """stream: a torch stream to launch on, or None for a stream the
        library creates (graphs cannot be captured on the null stream)."""
        import torch
        load_library()
        self.device = torch.device(device if device is not None else "cuda")
        self.stream = stream
        need = stc_batch_footprint(max_chains, max_items)
        self.arena = torch.empty(need, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)   # the arena is ready before other streams use it
        self.bt = stc_batch_create(max_chains, max_items, b,
                                   stream.cuda_stream if stream is not None else 0,
                                   self.arena.data_ptr(), need)
        self.members = []
        _live_batches.add(self)

    def set(self, solvers, tol: float, nontemporal: bool = False):
        solvers = list(solvers)
        try:
            stc_batch_set(self.bt, [s.h for s in solvers], tol, nontemporal)
        except StcError:
            self.members = []      # the library leaves the batch empty
            raise
        self.members = solvers

    def sweeps(self, n: int, use_graph: bool = True):
        stc_batch_sweeps(self.bt, n, use_graph)

    def autotune(self, trial_sweeps: int = 20) -> float:
        """Tune the launch shapes on the chains set (their iterates restart
        from e/N); returns ms per sweep of the batch."""
        return stc_batch_autotune(self.bt, trial_sweeps)

    def tile(self, stage: int, mp: int) -> dict:
        return stc_batch_get_tile(self.bt, stage, mp)

    def query(self):
        """Stopping state of every member: (sweeps, stopped, diff_1, status)."""
        return stc_batch_query(self.bt, len(self.members))

    def sync(self):
        stc_batch_sync(self.bt)

    def close(self):
        if getattr(self, "bt", None):
            stc_batch_destroy(self.bt)
            self.bt = None
        self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stc_destroy(h):
    if h:
        load_library().stc_destroy(h)


class Prepared:
    """The host half of a setup (stc_prepare): the generator validated and
    its blocks packed in the sweep's layout on host threads.  It makes no
    HIP call and touches no torch device state, so any thread may build it
    while another drives the GPU; Solver.from_prepared does the device half.
    Dense storage of block-banded generators only."""

    def __init__(self, blocks: np.ndarray, sizes, b: int, *, precision="fp64", stair_type=1,
                 stop="diff", check_every=1, switch_tol=0.0, recompute_diagonal=False):
        self.p = None
        load_library()
        gen, keep = make_generator(blocks, sizes, b, recompute_diagonal)
        self.opt = make_options(precision, stair_type, stop, check_every, switch_tol)
        self.footprint = stc_footprint_bytes(gen, self.opt)
        if self.footprint == 0:
            raise StcError(STC_EINVAL, "unsupported generator shape or options")
        self.N = int(np.sum(sizes)) if sizes is not None else gen.L * gen.m
        self.p = stc_prepare(gen, self.opt)
        del keep            # the host inputs were read during stc_prepare

    def close(self):
        if getattr(self, "p", None):
            stc_prepared_free(self.p)
        self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """One chain on the current GPU: owns the torch arena and the handle."""

    def __init__(self, blocks: np.ndarray | None, sizes, b: int, *, precision="fp64",
                 stair_type=1, stop="diff", check_every=1, switch_tol=0.0,
                 recompute_diagonal=False, device=None, stream=None, poison=False,
                 format="dense", csr=None, m=None, krylov_restart=0, krylov_keep_all=False,
                 method="staircase", jgs_chunks=0):
        """method "jgs" sweeps Algorithm 1 over jgs_chunks chunks of levels
        instead of the stair splitting.
        blocks: [L][2b+1][m][m] dense blocks, or None with csr = (indptr,
        indices, data) of the N x N generator (sizes then required; m
        defaults to the largest size).  poison: fill the arena with 0xFF
        bytes (a NaN in FP32 and FP64) before setup, so that any read of
        memory the library did not write first shows up as NaN in the
        results (a test aid)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the staircase solver needs a GPU")
        load_library()
        self.device = torch.device(device if device is not None else "cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if blocks is None:
            if csr is None or sizes is None:
                raise ValueError("give blocks, or csr with sizes")
            self.gen, self._keep = make_generator_csr(*csr, sizes, b, m, recompute_diagonal)
        else:
            self.gen, self._keep = make_generator(blocks, sizes, b, recompute_diagonal)
        self.opt = make_options(precision, stair_type, stop, check_every, switch_tol,
                                stream=self.stream.cuda_stream, format=format,
                                krylov_restart=krylov_restart, krylov_keep_all=krylov_keep_all,
                                method=method, jgs_chunks=jgs_chunks)
        need = stc_footprint_bytes(self.gen, self.opt)
        if need == 0:
            raise StcError(STC_EINVAL, "unsupported generator shape or options")
        self.arena = torch.empty(need, dtype=torch.uint8, device=self.device)
        if poison:
            self.arena.fill_(0xFF)
            torch.cuda.synchronize(self.device)
        self.opt.arena = self.arena.data_ptr()
        self.opt.arena_bytes = need
        self.footprint = need
        self.N = int(np.sum(sizes)) if sizes is not None else self.gen.L * self.gen.m
        with torch.cuda.device(self.device):
            self.h = stc_setup(self.gen, self.opt)
        self._keep = None   # host inputs were copied during setup
        _live_solvers.add(self)

    @classmethod
    def from_prepared(cls, prep: "Prepared", device=None, stream=None):
        """The solver of a prepared generator (the device half of the setup:
        upload, inverse, state), on stream (None: the current stream)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the staircase solver needs a GPU")
        if prep.p is None:
            raise ValueError("the prepared setup was released")
        self = cls.__new__(cls)
        self.device = torch.device(device if device is not None else "cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.gen, self._keep = None, None
        self.opt = stc_options.from_buffer_copy(prep.opt)
        self.opt.stream = self.stream.cuda_stream or None
        self.footprint = prep.footprint
        self.N = prep.N
        self.arena = torch.empty(self.footprint, dtype=torch.uint8, device=self.device)
        self.opt.arena = self.arena.data_ptr()
        self.opt.arena_bytes = self.footprint
        self.h = None
        with torch.cuda.device(self.device):
            self.h = stc_setup_prepared(prep.p, self.opt)
        _live_solvers.add(self)
        return self

    @classmethod
    def from_sparse(cls, Q, sizes, b: int, **kw):
        """A solver for a generator given as a scipy.sparse matrix (N x N,
        states numbered level by level); the rows go through the CSR input."""
        Q = Q.tocsr()
        return cls(None, sizes, b, csr=(Q.indptr, Q.indices, Q.data), **kw)

    def solve(self, x0=None, tol=1e-9, maxit=10_000, allow_maxit=True):
        pi = np.empty(self.N)
        x = None if x0 is None else _f64(x0)
        info = stc_solve(self.h, x, tol, maxit, pi, allow_maxit)
        return pi, info

    def solve_gmres(self, x0=None, tol=1e-12, restart=30, max_applies=100_000,
                    allow_maxit=True):
        """Staircase-preconditioned restarted GMRES to ||Q^T pi||_1 <= tol
        (needs krylov_restart >= restart at construction)."""
        pi = np.empty(self.N)
        x = None if x0 is None else _f64(x0)
        info = stc_solve_gmres(self.h, x, restart, tol, max_applies, pi, allow_maxit)
        return pi, info

    def step(self, x):
        z = np.empty(self.N)
        d = stc_step(self.h, _f64(x), z)
        return z, d

    def residual(self, x) -> float:
        return stc_residual(self.h, _f64(x))

    def load(self, x):
        stc_load(self.h, None if x is None else (_f64(x) if isinstance(x, np.ndarray) else x))

    def sweeps(self, n: int, with_diffs: bool = False):
        if with_diffs:
            d = np.empty(max(n - 1, 0))
            stc_sweeps(self.h, n, d)
            return d
        stc_sweeps(self.h, n)
        return None

    def query(self):
        return stc_query(self.h)

    def store(self):
        pi = np.empty(self.N)
        stc_store(self.h, pi)
        return pi

    def promote(self):
        stc_promote(self.h)

    def close(self):
        if getattr(self, "h", None):
            stc_destroy(self.h)
            self.h = None
        self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
