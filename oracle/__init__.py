"""CPU oracle for the checkerboard Metropolis sweep -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The product (the HIP library and
its binding in ``paper_1209_0296_amd``) never does, and this package never
imports the product.

The arithmetic lives in ``spinlat_oracle.c`` (plain C, OpenMP over rows of one
colour); this module only builds it with gcc and marshals numpy arrays.  See
the C file's header for the model (paper Sec. 3, Eq. 1-3, Alg. I) and the
random-number contract (Philox4x32-10, Salmon et al. SC'11).

Parity-unpinned functions: none.  Every function is pinned by a test in
``tests/test_oracle_*.py`` (rocRAND cross-check of Philox, closed forms,
exact enumeration, deterministic limits, balance of the transition kernel).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spinlat_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ISING = 0
NORTH_EAST = 1
NE_TILES = 2  # North-East model, the paper's random sub-lattice algorithm
NE_BALANCED = 3  # its balanced variant (red, then white sites; four launches per sweep)
NE_COUPLED = 4  # NE constraint on the Ising energy with J, h, T (checkerboard half-sweeps)
INIT_COLD = 0
INIT_RANDOM = 1
RECORD_WORDS = 5  # t, bond_sum, mag, accepted, unflipped


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O3, no fast-math, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "spinlat_oracle.h"))
    ):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32), ("dim", ctypes.c_int32), ("L", ctypes.c_int32),
        ("two_s", ctypes.c_int32), ("init", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("J", ctypes.c_double), ("h", ctypes.c_double), ("T", ctypes.c_double),
        ("c", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("tile", ctypes.c_int32), ("lambda_", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = ctypes.CDLL(path)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_philox4x32_10.restype = None
        L.or_rand.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                              ctypes.c_uint64, ctypes.c_int, ctypes.c_int]
        L.or_rand.restype = ctypes.c_uint32
        L.or_threshold_from_prob.argtypes = [ctypes.c_double]
        L.or_threshold_from_prob.restype = ctypes.c_uint64
        L.or_threshold.argtypes = [ctypes.c_double, ctypes.c_double]
        L.or_threshold.restype = ctypes.c_uint64
        L.or_delta_e.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int]
        L.or_delta_e.restype = ctypes.c_double
        P = ctypes.POINTER(_Params)
        L.or_nsites.argtypes = [P]
        L.or_nsites.restype = ctypes.c_int64
        L.or_init.argtypes = [P, ctypes.c_void_p]
        L.or_init.restype = None
        L.or_half_sweep.argtypes = [P, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32]
        L.or_half_sweep.restype = ctypes.c_int64
        L.or_recount.argtypes = [P, ctypes.c_void_p, ctypes.c_void_p]
        L.or_recount.restype = None
        L.or_reset_persistence.argtypes = [P, ctypes.c_void_p]
        L.or_reset_persistence.restype = None
        L.or_run.argtypes = [P, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                             ctypes.c_void_p, ctypes.c_int]
        L.or_run.restype = ctypes.c_int
        L.or_ne_tiles_launch.argtypes = [P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]
        L.or_ne_tiles_launch.restype = ctypes.c_int64
        L.or_ne_balanced_launch.argtypes = [P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]
        L.or_ne_balanced_launch.restype = ctypes.c_int64
        L.or_threshold_table.argtypes = [P, ctypes.c_void_p, ctypes.c_int64]
        L.or_threshold_table.restype = ctypes.c_int64
        _lib = L
    return _lib


@dataclass
class Params:
    """Model parameters (paper Sec. 3): Ising (J, h, T; spin-1/2 or spin-1,
    2D or 3D) or the North-East model (up-density c, 2D), the latter either by
    checkerboard half-sweeps (NORTH_EAST) or by the paper's random sub-lattice
    algorithm (NE_TILES: side ``tile``, ``lam`` sites per iteration).
    NE_COUPLED moves NE sites with the Ising rates of (J, h, T) over s = 2n - 1;
    c then only sets the initial density."""
    model: int = ISING
    dim: int = 2
    L: int = 64
    two_s: int = 1
    init: int = INIT_RANDOM
    J: float = 1.0
    h: float = 0.0
    T: float = 2.269
    c: float = 0.1
    seed: int = 1
    tile: int = 32   # NE_TILES: side of the sub-lattices
    lam: int = 16    # NE_TILES: sites updated together per iteration

    def c_struct(self) -> _Params:
        return _Params(self.model, self.dim, self.L, self.two_s, self.init, 0,
                       self.J, self.h, self.T, self.c, self.seed, self.tile, self.lam)

    @property
    def nsites(self) -> int:
        return self.L ** self.dim

    @property
    def shape(self):
        return (self.L,) * self.dim


def philox4x32_10(ctr, key):
    """Philox4x32-10 of one 128-bit counter (4 words) under a 64-bit key (2 words)."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def rand_word(seed, tag, t, colour, k, w=1, j=0) -> int:
    return int(lib().or_rand(seed, tag, t, colour, k, w, j))


def threshold(dE: float, T: float) -> int:
    return int(lib().or_threshold(dE, T))


def threshold_from_prob(p: float) -> int:
    return int(lib().or_threshold_from_prob(p))


def threshold_table(p: Params) -> np.ndarray:
    out = np.zeros(128, dtype=np.uint64)
    ps = p.c_struct()
    n = lib().or_threshold_table(ctypes.byref(ps), out.ctypes.data, out.size)
    if n < 0:
        raise ValueError("table capacity")
    return out[:n].copy()


def init_lattice(p: Params) -> np.ndarray:
    """Initial state in natural order (shape (L,L) or (L,L,L) indexed [z][y][x])."""
    s = np.zeros(p.shape, dtype=np.int8)
    ps = p.c_struct()
    lib().or_init(ctypes.byref(ps), s.ctypes.data)
    return s


def half_sweep(p: Params, s: np.ndarray, t: int, colour: int) -> int:
    assert s.dtype == np.int8 and s.flags.c_contiguous and s.size == p.nsites
    ps = p.c_struct()
    return int(lib().or_half_sweep(ctypes.byref(ps), s.ctypes.data, t, colour))


def recount(p: Params, s: np.ndarray):
    out = np.zeros(3, dtype=np.int64)
    ps = p.c_struct()
    lib().or_recount(ctypes.byref(ps), s.ctypes.data, out.ctypes.data)
    return int(out[0]), int(out[1]), int(out[2])


def reset_persistence(p: Params, s: np.ndarray) -> None:
    ps = p.c_struct()
    lib().or_reset_persistence(ctypes.byref(ps), s.ctypes.data)


def run(p: Params, s: np.ndarray, t0: int, nsweeps: int, records: bool = True,
        nthreads: int = 0):
    """Advance ``s`` in place by ``nsweeps`` sweeps starting at sweep index ``t0``.

    Returns an (nsweeps, 5) int64 array of records {t+1, bond_sum, mag,
    accepted, unflipped} (or None when ``records`` is False).
    """
    assert s.dtype == np.int8 and s.flags.c_contiguous and s.size == p.nsites
    rec = np.zeros((nsweeps, RECORD_WORDS), dtype=np.int64) if records else None
    ps = p.c_struct()
    rc = lib().or_run(ctypes.byref(ps), s.ctypes.data, t0, nsweeps,
                      rec.ctypes.data if rec is not None else None, nthreads)
    if rc != 0:
        raise ValueError("invalid parameters for the oracle run")
    return rec


def ne_tiles_launch(p: Params, src: np.ndarray, launch: int):
    """One launch of the paper's NE algorithm: returns (new lattice, accepted)."""
    dst = np.empty_like(src)
    ps = p.c_struct()
    assert src.dtype == np.int8 and src.flags.c_contiguous and src.size == p.nsites
    acc = lib().or_ne_tiles_launch(ctypes.byref(ps), src.ctypes.data, dst.ctypes.data, launch)
    if acc < 0:
        raise ValueError("invalid sub-lattice parameters")
    return dst, int(acc)


def ne_balanced_launch(p: Params, src: np.ndarray, launch: int):
    """One launch of the balanced NE variant: returns (new lattice, accepted)."""
    dst = np.empty_like(src)
    ps = p.c_struct()
    assert src.dtype == np.int8 and src.flags.c_contiguous and src.size == p.nsites
    acc = lib().or_ne_balanced_launch(ctypes.byref(ps), src.ctypes.data, dst.ctypes.data, launch)
    if acc < 0:
        raise ValueError("invalid sub-lattice parameters")
    return dst, int(acc)


def initial_record(p: Params, s: np.ndarray, t: int = 0) -> np.ndarray:
    b, m, u = recount(p, s)
    return np.array([t, b, m, 0, u], dtype=np.int64)
