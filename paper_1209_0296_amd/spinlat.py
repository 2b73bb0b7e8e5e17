"""ctypes binding of the C ABI in ``include/spinlat.h``.

Argument marshalling only: every step of the sweep runs in the HIP kernels of
``libspinlat.so``.  PyTorch provides the device buffer and the stream.  If
the library has not been built the import of this module fails loudly; there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspinlat.so")

ABI_VERSION = 3
BATCH_NO_GRAPH, BATCH_NO_FUSED, BATCH_NO_RESIDENT = 1, 2, 4
ISING, NORTH_EAST, NE_SUBLATTICE, NE_SUBLATTICE_BALANCED, NE_COUPLED = 0, 1, 2, 3, 4
INIT_COLD, INIT_RANDOM, INIT_BUFFER = 0, 1, 2
MODE_AUTO, MODE_SIMPLE, MODE_HALF, MODE_FUSED = 0, 1, 2, 3
MODE_HALF_WINDOW, MODE_FUSED_WINDOW, MODE_RESIDENT, MODE_HALF_ROWS = 4, 5, 6, 7
STATUS = {0: "SL_OK", 1: "SL_E_INVALID", 2: "SL_E_UNSUPPORTED", 3: "SL_E_BUFFER",
          4: "SL_E_HIP", 5: "SL_E_STATE", 6: "SL_E_OVERFLOW"}

# every symbol include/spinlat.h declares
EXPORTS = (
    "sl_query_bytes", "sl_threshold_table", "sl_create_lattice", "sl_set_launch",
    "sl_get_launch", "sl_sweep", "sl_measure", "sl_status_counts", "sl_copy_spins",
    "sl_reset_persistence", "sl_destroy", "sl_status_str", "sl_last_error",
    "sl_record_observables", "sl_batch_job_bytes", "sl_batch_base_bytes", "sl_batch_create",
    "sl_batch_add", "sl_batch_sweep", "sl_batch_job_status", "sl_batch_measure",
    "sl_batch_copy_spins", "sl_batch_remove", "sl_batch_destroy", "sl_batch_drain",
    "sl_record_statistics", "sl_overlap", "sl_autocorrelation", "sl_sweep_static",
)


class SpinlatError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class CParams(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32), ("model", ctypes.c_int32), ("dim", ctypes.c_int32),
        ("L", ctypes.c_int32), ("two_s", ctypes.c_int32), ("init", ctypes.c_int32),
        ("J", ctypes.c_double), ("h", ctypes.c_double), ("T", ctypes.c_double),
        ("c", ctypes.c_double), ("seed", ctypes.c_uint64), ("t0", ctypes.c_uint64),
        ("record_capacity", ctypes.c_uint64), ("init_spins", ctypes.c_void_p),
        ("ne_side", ctypes.c_int32), ("ne_lambda", ctypes.c_int32),
    ]


class CRecord(ctypes.Structure):
    _fields_ = [("t", ctypes.c_uint64), ("bond_sum", ctypes.c_int64), ("mag", ctypes.c_int64),
                ("accepted", ctypes.c_int64), ("unflipped", ctypes.c_int64)]


class CBatchConfig(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("max_jobs", ctypes.c_uint32),
                ("record_capacity", ctypes.c_uint32), ("tile_rows", ctypes.c_int32),
                ("max_workgroups", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class CStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("e", ctypes.c_double), ("e_var", ctypes.c_double),
                ("m", ctypes.c_double), ("m_abs", ctypes.c_double), ("m2", ctypes.c_double),
                ("m4", ctypes.c_double), ("heat_capacity", ctypes.c_double),
                ("susceptibility", ctypes.c_double), ("binder", ctypes.c_double)]


class CLaunch(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("tile_words", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def lib():
    """Load libspinlat.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1209_0296_amd.build` (hipcc, gfx950)")
    # torch's HIP runtime must be the one in the process before the library
    # binds to libamdhip64 (same soname): device buffers and streams come from
    # torch, and a second runtime would not see the device.
    import torch  # noqa: F401

    L = ctypes.CDLL(LIB_PATH)
    P, H = ctypes.POINTER(CParams), ctypes.c_void_p
    sz = ctypes.c_size_t
    L.sl_query_bytes.argtypes = [P, ctypes.POINTER(sz)]
    L.sl_threshold_table.argtypes = [P, ctypes.c_void_p, sz, ctypes.POINTER(sz)]
    L.sl_create_lattice.argtypes = [P, ctypes.c_void_p, sz, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_void_p)]
    L.sl_set_launch.argtypes = [H, ctypes.POINTER(CLaunch)]
    L.sl_get_launch.argtypes = [H, ctypes.POINTER(CLaunch)]
    L.sl_sweep.argtypes = [H, ctypes.c_uint64]
    L.sl_measure.argtypes = [H, ctypes.c_void_p, sz, ctypes.POINTER(sz)]
    L.sl_status_counts.argtypes = [H, ctypes.POINTER(ctypes.c_uint64),
                                   ctypes.POINTER(ctypes.c_uint64)]
    L.sl_copy_spins.argtypes = [H, ctypes.c_void_p, sz]
    L.sl_reset_persistence.argtypes = [H]
    L.sl_destroy.argtypes = [H]
    L.sl_status_str.argtypes = [ctypes.c_int]
    L.sl_status_str.restype = ctypes.c_char_p
    L.sl_last_error.argtypes = []
    L.sl_last_error.restype = ctypes.c_char_p
    L.sl_record_observables.argtypes = [P, ctypes.c_void_p, sz, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]
    B, BC = ctypes.c_void_p, ctypes.POINTER(CBatchConfig)
    L.sl_batch_job_bytes.argtypes = [P, BC, ctypes.POINTER(sz)]
    L.sl_batch_base_bytes.argtypes = [BC, ctypes.POINTER(sz)]
    L.sl_batch_create.argtypes = [BC, ctypes.c_void_p, sz, ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_void_p)]
    L.sl_batch_add.argtypes = [B, P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32)]
    L.sl_batch_sweep.argtypes = [B, ctypes.c_uint64]
    u64p = ctypes.POINTER(ctypes.c_uint64)
    L.sl_batch_job_status.argtypes = [B, ctypes.c_uint32, u64p, u64p, u64p]
    L.sl_batch_measure.argtypes = [B, ctypes.c_uint32, ctypes.c_void_p, sz, ctypes.POINTER(sz)]
    L.sl_batch_copy_spins.argtypes = [B, ctypes.c_uint32, ctypes.c_void_p, sz]
    L.sl_batch_drain.argtypes = [B, ctypes.c_void_p, ctypes.c_void_p, sz, ctypes.POINTER(sz)]
    L.sl_batch_remove.argtypes = [B, ctypes.c_uint32]
    L.sl_batch_destroy.argtypes = [B]
    L.sl_record_statistics.argtypes = [P, ctypes.c_void_p, sz, ctypes.POINTER(CStats)]
    L.sl_overlap.argtypes = [H, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
    L.sl_autocorrelation.argtypes = [P, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
    L.sl_sweep_static.argtypes = [P, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    for name in EXPORTS:
        fn = getattr(L, name)
        if name not in ("sl_status_str", "sl_last_error"):
            fn.restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int) -> None:
    if status != 0:
        raise SpinlatError(status, lib().sl_last_error().decode())


def _count(n) -> int:
    """A sweep count as the C ABI's uint64 (ctypes would wrap a negative one)."""
    n = int(n)
    if n < 0 or n >= 2 ** 64:
        raise ValueError(f"sweep count {n} is outside [0, 2^64)")
    return n


@dataclass
class Params:
    """Model parameters (paper Sec. 3): Ising (J, h, T; spin-1/2 or spin-1; 2D or
    3D) or the North-East model (up-density c; 2D), by checkerboard half-sweeps
    (NORTH_EAST) or by the random sub-lattice algorithm of Sec. 3.2
    (NE_SUBLATTICE: side ``ne_side``, ``ne_lambda`` sites per iteration).
    NE_COUPLED moves NE sites with the Ising rates of (J, h, T) over s = 2n - 1
    (Sec. 3.2, J != 0); c then only sets the initial density."""
    model: int = ISING
    dim: int = 2
    L: int = 64
    two_s: int = 1
    J: float = 1.0
    h: float = 0.0
    T: float = 2.269
    c: float = 0.1
    seed: int = 1
    init: int = INIT_RANDOM
    t0: int = 0
    record_capacity: int = 1024
    ne_side: int = 32
    ne_lambda: int = 16

    def c_struct(self, init_spins_ptr: int = 0) -> CParams:
        return CParams(ABI_VERSION, self.model, self.dim, self.L, self.two_s, self.init,
                       float(self.J), float(self.h), float(self.T), float(self.c),
                       int(self.seed), int(self.t0), int(self.record_capacity),
                       init_spins_ptr or None, int(self.ne_side), int(self.ne_lambda))

    @property
    def nsites(self) -> int:
        return self.L ** self.dim

    @property
    def shape(self):
        return (self.L,) * self.dim


def query_bytes(p: Params) -> int:
    n = ctypes.c_size_t()
    cp = p.c_struct(1 if p.init == INIT_BUFFER else 0)
    _check(lib().sl_query_bytes(ctypes.byref(cp), ctypes.byref(n)))
    return n.value


def threshold_table(p: Params) -> np.ndarray:
    out = np.zeros(64, dtype=np.uint64)
    n = ctypes.c_size_t()
    cp = p.c_struct(1 if p.init == INIT_BUFFER else 0)
    _check(lib().sl_threshold_table(ctypes.byref(cp), out.ctypes.data, out.size, ctypes.byref(n)))
    return out[: n.value].copy()


RECORD_DTYPE = np.dtype([("t", np.uint64), ("bond_sum", np.int64), ("mag", np.int64),
                         ("accepted", np.int64), ("unflipped", np.int64)])


class Lattice:
    """One lattice resident in HBM, advanced by ``sweep`` and read by ``measure``.

    The device buffer is a torch uint8 tensor owned by this object; work goes
    on ``stream`` (default: torch's current stream on ``device``).
    """

    def __init__(self, params: Params, init_spins=None, device="cuda", stream=None):
        import torch

        self.params = params
        self.device = torch.device(device)
        self._torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ptr = 0
        if params.init == INIT_BUFFER:
            if init_spins is None:
                raise ValueError("INIT_BUFFER needs init_spins")
            init_spins = init_spins.to(device=self.device, dtype=torch.int8).contiguous()
            if init_spins.numel() != params.nsites:
                raise ValueError("init_spins has the wrong size")
            self._init_spins = init_spins
            ptr = init_spins.data_ptr()
        nbytes = query_bytes(params)
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        cp = params.c_struct(ptr)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().sl_create_lattice(ctypes.byref(cp), self.buffer.data_ptr(), nbytes,
                                           self.stream.cuda_stream, ctypes.byref(h)))
        self._h = h

    # -- schedule -----------------------------------------------------------
    def set_launch(self, mode: int, tile_rows: int = 0, tile_words: int = 0) -> None:
        _check(lib().sl_set_launch(self._h, ctypes.byref(CLaunch(mode, tile_rows, tile_words, 0))))

    def get_launch(self):
        l = CLaunch()
        _check(lib().sl_get_launch(self._h, ctypes.byref(l)))
        return (l.mode, l.tile_rows, l.tile_words)

    # -- the hot path -------------------------------------------------------
    def sweep(self, n: int) -> None:
        _check(lib().sl_sweep(self._h, _count(n)))

    def counts(self):
        p, t = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().sl_status_counts(self._h, ctypes.byref(p), ctypes.byref(t)))
        return p.value, t.value

    def measure(self) -> np.ndarray:
        """Drain the unread per-sweep records (synchronises the stream)."""
        pending, _ = self.counts()
        out = np.zeros(max(pending, 1), dtype=RECORD_DTYPE)
        n = ctypes.c_size_t()
        _check(lib().sl_measure(self._h, out.ctypes.data, out.size, ctypes.byref(n)))
        return out[: n.value]

    def observables(self, records: np.ndarray):
        """E, M and persistence per record, computed by the library (double)."""
        n = len(records)
        E = np.zeros(n)
        M = np.zeros(n)
        P = np.zeros(n)
        recs = np.ascontiguousarray(records)
        cp = self.params.c_struct(1 if self.params.init == INIT_BUFFER else 0)
        _check(lib().sl_record_observables(ctypes.byref(cp), recs.ctypes.data, n,
                                           E.ctypes.data, M.ctypes.data, P.ctypes.data))
        return E, M, P

    def copy_spins(self):
        """Device int8 tensor of the lattice in natural order, shape (L,)*dim."""
        torch = self._torch
        out = torch.empty(self.params.nsites, dtype=torch.int8, device=self.device)
        _check(lib().sl_copy_spins(self._h, out.data_ptr(), out.numel()))
        return out.view(*self.params.shape)

    def spins(self) -> np.ndarray:
        """Host copy (numpy int8, natural order) -- synchronises."""
        t = self.copy_spins()
        self.stream.synchronize()
        return t.cpu().numpy()

    def reset_persistence(self) -> None:
        _check(lib().sl_reset_persistence(self._h))

    def overlap(self, reference) -> int:
        """sum_i v_i v_i^ref with a device int8 tensor in natural order (synchronises)."""
        ref = reference.to(device=self.device, dtype=self._torch.int8).contiguous()
        if ref.numel() != self.params.nsites:
            raise ValueError("reference has the wrong size")
        out = ctypes.c_int64()
        _check(lib().sl_overlap(self._h, ref.data_ptr(), ctypes.byref(out)))
        return int(out.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            _check(lib().sl_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def record_statistics(p: Params, records) -> dict:
    """Means, heat capacity, susceptibility and Binder cumulant of Ising records,
    or of coupled NE records in their spin variables (structured records or an
    (n, 5) int64 array), computed by the library."""
    recs = np.ascontiguousarray(records)
    if recs.dtype != RECORD_DTYPE:
        a = np.asarray(recs, dtype=np.int64)
        recs = np.zeros(len(a), dtype=RECORD_DTYPE)
        for i, f in enumerate(RECORD_DTYPE.names):
            recs[f] = a[:, i]
    st = CStats()
    cp = p.c_struct(1 if p.init == INIT_BUFFER else 0)
    _check(lib().sl_record_statistics(ctypes.byref(cp), recs.ctypes.data, len(recs),
                                      ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in CStats._fields_}


def autocorrelation(p: Params, overlap: int) -> float:
    """NE spin autocorrelation Phi (Eq. 4) of an overlap, computed by the library."""
    phi = ctypes.c_double()
    cp = p.c_struct(1 if p.init == INIT_BUFFER else 0)
    _check(lib().sl_autocorrelation(ctypes.byref(cp), int(overlap), ctypes.byref(phi)))
    return phi.value


def records_to_array(records: np.ndarray) -> np.ndarray:
    """Structured records -> (n, 5) int64 array {t, bond_sum, mag, accepted, unflipped}."""
    return np.stack([records[f].astype(np.int64) for f in RECORD_DTYPE.names], axis=1)


# ---------------------------------------------------------------------------
# Batches of independent lattices sharing launches

def batch_config(max_jobs: int = 1024, record_capacity: int = 256, tile_rows: int = 0,
                 max_workgroups: int = 0, flags: int = 0) -> CBatchConfig:
    return CBatchConfig(ABI_VERSION, max_jobs, record_capacity, tile_rows, max_workgroups, flags, 0)


def batch_job_bytes(p: Params, cfg: CBatchConfig) -> int:
    n = ctypes.c_size_t()
    cp = p.c_struct(1 if p.init == INIT_BUFFER else 0)
    _check(lib().sl_batch_job_bytes(ctypes.byref(cp), ctypes.byref(cfg), ctypes.byref(n)))
    return n.value


def batch_base_bytes(cfg: CBatchConfig) -> int:
    n = ctypes.c_size_t()
    _check(lib().sl_batch_base_bytes(ctypes.byref(cfg), ctypes.byref(n)))
    return n.value


class Batch:
    """Many lattices (jobs) resident in one device arena, advanced together.

    ``add`` admits a job if its footprint fits the free arena space (returns
    None otherwise), ``sweep(n)`` runs up to n sweeps of every job with sweeps
    left, ``measure(job)`` drains a job's records.
    """

    def __init__(self, arena_bytes: int, max_jobs: int = 1024, record_capacity: int = 256,
                 tile_rows: int = 0, device="cuda", stream=None, max_workgroups: int = 0,
                 flags: int = 0):
        import torch

        self._torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.cfg = batch_config(max_jobs, record_capacity, tile_rows, max_workgroups, flags)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        self._init_refs = {}
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().sl_batch_create(ctypes.byref(self.cfg), self.arena.data_ptr(),
                                         self.arena.numel(), self.stream.cuda_stream,
                                         ctypes.byref(h)))
        self._h = h
        self.params = {}

    def add(self, p: Params, sweeps: int, init_spins=None):
        """Job id, or None when the arena has no room for it or the job table
        is full (both free up as jobs are removed)."""
        torch = self._torch
        ptr = 0
        if p.init == INIT_BUFFER:
            t = init_spins.to(device=self.device, dtype=torch.int8).contiguous()
            ptr = t.data_ptr()
        cp = p.c_struct(ptr)
        jid = ctypes.c_uint32()
        st = lib().sl_batch_add(self._h, ctypes.byref(cp), _count(sweeps), ctypes.byref(jid))
        if st in (3, 5):  # SL_E_BUFFER: no arena room; SL_E_STATE: job table full
            return None
        _check(st)
        self.params[jid.value] = p
        if ptr:
            self._init_refs[jid.value] = t  # the copy runs on the stream later
        return jid.value

    def sweep(self, n: int) -> None:
        _check(lib().sl_batch_sweep(self._h, _count(n)))

    def status(self, job: int):
        d, r, p = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().sl_batch_job_status(self._h, job, ctypes.byref(d), ctypes.byref(r),
                                         ctypes.byref(p)))
        return d.value, r.value, p.value

    def measure(self, job: int) -> np.ndarray:
        _, _, pending = self.status(job)
        out = np.zeros(max(pending, 1), dtype=RECORD_DTYPE)
        n = ctypes.c_size_t()
        _check(lib().sl_batch_measure(self._h, job, out.ctypes.data, out.size, ctypes.byref(n)))
        return out[: n.value]

    def drain(self):
        """All jobs' unread records: {job id: (n, 5) int64 array}."""
        cap = self.cfg.max_jobs * self.cfg.record_capacity
        if not hasattr(self, "_drain_buf") or self._drain_buf.size < cap:
            self._drain_buf = np.zeros(cap, dtype=RECORD_DTYPE)
            self._drain_job = np.zeros(cap, dtype=np.uint32)
        n = ctypes.c_size_t()
        _check(lib().sl_batch_drain(self._h, self._drain_buf.ctypes.data,
                                    self._drain_job.ctypes.data, cap, ctypes.byref(n)))
        n = n.value
        recs = records_to_array(self._drain_buf[:n])
        jobs = self._drain_job[:n]
        out = {}
        if n:
            cuts = np.flatnonzero(np.diff(jobs)) + 1
            starts = np.concatenate([[0], cuts])
            ends = np.concatenate([cuts, [n]])
            for a, e in zip(starts, ends):
                out[int(jobs[a])] = recs[a:e]
        return out

    def spins(self, job: int) -> np.ndarray:
        torch = self._torch
        p = self.params[job]
        out = torch.empty(p.nsites, dtype=torch.int8, device=self.device)
        _check(lib().sl_batch_copy_spins(self._h, job, out.data_ptr(), out.numel()))
        self.stream.synchronize()
        return out.cpu().numpy().reshape(p.shape)

    def remove(self, job: int) -> None:
        _check(lib().sl_batch_remove(self._h, job))
        self.params.pop(job, None)
        self._init_refs.pop(job, None)

    def close(self) -> None:
        if getattr(self, "_h", None):
            _check(lib().sl_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
