"""ctypes front end of csweep.c (the C/OpenMP Algorithm 2 sweep).

TEST INFRASTRUCTURE ONLY: used by the tests and by the CPU-baseline leg of
the benchmark.  ``build()`` compiles the shared object with gcc; loading
never compiles.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csweep.c")
LIB = os.path.join(HERE, "_csweep.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build() -> str:
    """Compile csweep.c with gcc -O2 -fopenmp (plain C, no tuning)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _load():
    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    lib.cs_factor.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _dp, _dp, _ip]
    lib.cs_factor.restype = ctypes.c_int
    lib.cs_sweep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _dp, _dp, _ip,
                             ctypes.c_int, _dp, _dp, _dp]
    lib.cs_sweep.restype = ctypes.c_int
    _lp = ctypes.POINTER(ctypes.c_longlong)
    lib.cs_gen_factor.argtypes = [ctypes.c_int, ctypes.c_int, _lp, _lp, _ip, _dp, _dp, _ip]
    lib.cs_gen_factor.restype = ctypes.c_int
    lib.cs_gen_sweep.argtypes = [ctypes.c_int, ctypes.c_int, _lp, _lp, _ip, _dp, _dp, _ip,
                                 ctypes.c_int, _dp, _dp, _dp]
    lib.cs_gen_sweep.restype = ctypes.c_int
    lib.cs_threads.argtypes = [ctypes.c_int]
    lib.cs_threads.restype = ctypes.c_int
    lib.cs_mxcsr.argtypes = []
    lib.cs_mxcsr.restype = ctypes.c_uint
    return lib


def _p(a, t):
    return a.ctypes.data_as(t)


class CSweep:
    """Factor once, then run sweeps on padded [L, m] FP64 vectors."""

    def __init__(self, blocks: np.ndarray, sizes, b: int, stair_type: int = 1,
                 threads: int = 0):
        self.lib = _load()
        self.threads = self.lib.cs_threads(int(threads))
        self.blocks = np.ascontiguousarray(blocks, dtype=np.float64)
        self.L, _, self.m, _ = self.blocks.shape
        self.b = int(b)
        self.sizes = np.ascontiguousarray(sizes, dtype=np.int32)
        self.stair_type = int(stair_type)
        self.lu = np.zeros((self.L, self.m, self.m))
        self.piv = np.zeros((self.L, self.m), dtype=np.int32)
        rc = self.lib.cs_factor(self.L, self.m, self.b, _p(self.sizes, _ip),
                                _p(self.blocks, _dp), _p(self.lu, _dp), _p(self.piv, _ip))
        if rc != 0:
            raise np.linalg.LinAlgError("singular diagonal block")

    def sweep(self, x: np.ndarray, z: np.ndarray) -> float:
        err = ctypes.c_double(0.0)
        rc = self.lib.cs_sweep(self.L, self.m, self.b, _p(self.sizes, _ip),
                               _p(self.blocks, _dp), _p(self.lu, _dp), _p(self.piv, _ip),
                               self.stair_type, _p(x, _dp), _p(z, _dp), ctypes.byref(err))
        if rc != 0:
            raise ArithmeticError("e^T z <= 0")
        return err.value


class CGenSweep:
    """The same Algorithm 2 for a generator of any block pattern: A = Q^T as
    compact CSR (a scipy matrix or Q itself, transposed here), level sizes;
    vectors are compact, length N."""

    def __init__(self, Q, sizes, stair_type: int = 1, threads: int = 0):
        import scipy.sparse as sp
        self.lib = _load()
        self.threads = self.lib.cs_threads(int(threads))
        A = sp.csr_matrix(Q).T.tocsr()
        A.sort_indices()
        self.rp = np.ascontiguousarray(A.indptr, dtype=np.int64)
        self.col = np.ascontiguousarray(A.indices, dtype=np.int32)
        self.val = np.ascontiguousarray(A.data, dtype=np.float64)
        sizes = np.asarray(sizes, dtype=np.int64)
        self.off = np.zeros(len(sizes) + 1, dtype=np.int64)
        np.cumsum(sizes, out=self.off[1:])
        self.L = len(sizes)
        self.m = int(sizes.max())
        self.N = int(self.off[-1])
        self.stair_type = int(stair_type)
        self.lu = np.zeros((self.L, self.m, self.m))
        self.piv = np.zeros((self.L, self.m), dtype=np.int32)
        _lp = ctypes.POINTER(ctypes.c_longlong)
        self._lp = _lp
        rc = self.lib.cs_gen_factor(self.L, self.m, _p(self.off, _lp), _p(self.rp, _lp),
                                    _p(self.col, _ip), _p(self.val, _dp), _p(self.lu, _dp),
                                    _p(self.piv, _ip))
        if rc != 0:
            raise np.linalg.LinAlgError("singular diagonal block")

    def sweep(self, x: np.ndarray, z: np.ndarray) -> float:
        err = ctypes.c_double(0.0)
        lp = self._lp
        rc = self.lib.cs_gen_sweep(self.L, self.m, _p(self.off, lp), _p(self.rp, lp),
                                   _p(self.col, _ip), _p(self.val, _dp), _p(self.lu, _dp),
                                   _p(self.piv, _ip), self.stair_type, _p(x, _dp), _p(z, _dp),
                                   ctypes.byref(err))
        if rc != 0:
            raise ArithmeticError("e^T z <= 0")
        return err.value


def ftz_daz() -> dict:
    """Flush-to-zero and denormals-are-zero state of the C sweeps (MXCSR of
    the calling thread, whose setting the OpenMP threads start from)."""
    w = int(_load().cs_mxcsr())
    return {"ftz": bool(w & (1 << 15)), "daz": bool(w & (1 << 6))}
