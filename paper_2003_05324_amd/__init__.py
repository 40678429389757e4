"""Python binding of libmpgeo, the MI355X mixed-precision Gaussian log-likelihood library.

Argument marshalling only: every step of the computation runs in the HIP library.
The functions named mpgeo_* mirror the C-ABI of include/mpgeo.h one to one; Context
and Dataset are small conveniences around them.  Host inputs are numpy float64
arrays; device inputs are torch tensors on the context's device (their data
pointers are passed with MPGEO_INPUT_DEVICE).  torch is imported first so that the
library binds to the same HIP runtime as torch.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpgeo.so")

(MPGEO_OK, MPGEO_E_ARG, MPGEO_E_NOT_SPD, MPGEO_E_NOMEM, MPGEO_E_DEVICE, MPGEO_E_UNSUPPORTED,
 MPGEO_E_TOO_LARGE) = range(7)
MPGEO_NOALLOC_SCRATCH_BYTES = 320 << 20
MPGEO_ORDER_MORTON = 1
MPGEO_INPUT_DEVICE = 2
MPGEO_TIMING = 4
MPGEO_PROFILE = 8
MPGEO_DIST_GCD = 16
MPGEO_BATCH_QUEUE = 32
MPGEO_ESCALATE = 64
MPGEO_TUNE_BAND = 128
MPGEO_GRAPH = 256

EXPORTED = (
    "mpgeo_ctx_create", "mpgeo_ctx_destroy", "mpgeo_ctx_kernel_stats", "mpgeo_ctx_reset_stats",
    "mpgeo_loglik", "mpgeo_dataset_create", "mpgeo_dataset_destroy", "mpgeo_dataset_loglik",
    "mpgeo_dataset_krige", "mpgeo_dataset_perm", "mpgeo_dataset_covariance",
    "mpgeo_dataset_matrix", "mpgeo_dataset_solution", "mpgeo_factor_dense",
    "mpgeo_footprint_bytes", "mpgeo_plan_tiers", "mpgeo_status_string", "mpgeo_dataset_entries", "mpgeo_dataset_mle",
    "mpgeo_dataset_mle_trace",
    "mpgeo_dataset_simulate", "mpgeo_batch_loglik", "mpgeo_batch_loglik_noalloc", "mpgeo_server_create",
    "mpgeo_server_add_dataset", "mpgeo_server_submit", "mpgeo_server_submit_krige", "mpgeo_server_run",
    "mpgeo_server_destroy",
)


class Theta(ctypes.Structure):
    _fields_ = [("sigma2", ctypes.c_double), ("beta", ctypes.c_double), ("nu", ctypes.c_double)]


class Plan(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("band64", ctypes.c_int32), ("band32", ctypes.c_int32),
                ("lowp", ctypes.c_int32), ("flags", ctypes.c_uint32), ("band0", ctypes.c_int32),
                ("dist64", ctypes.c_double), ("dist32", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("loglik", ctypes.c_double), ("logdet", ctypes.c_double), ("quad", ctypes.c_double),
                ("info", ctypes.c_int64), ("t_covgen", ctypes.c_double),
                ("t_factor", ctypes.c_double), ("t_solve", ctypes.c_double),
                ("t_total", ctypes.c_double), ("band64", ctypes.c_int32), ("band32", ctypes.c_int32),
                ("band0", ctypes.c_int32), ("escalations", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Instance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("locs", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("theta", Theta)]


class Served(ctypes.Structure):
    _fields_ = [("loglik", ctypes.c_double), ("logdet", ctypes.c_double), ("quad", ctypes.c_double),
                ("info", ctypes.c_int64), ("arrival_s", ctypes.c_double), ("start_s", ctypes.c_double),
                ("finish_s", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class PlanTiers(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int64), ("nbp", ctypes.c_int32), ("band64", ctypes.c_int32),
                ("edge", ctypes.c_int32), ("band0", ctypes.c_int32), ("lowp", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("tiles", ctypes.c_int64 * 4),
                ("update_flops", ctypes.c_double * 3), ("trsm_flops", ctypes.c_double * 2),
                ("potrf_flops", ctypes.c_double), ("footprint_bytes", ctypes.c_uint64)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("seconds", ctypes.c_double), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class MpgeoError(RuntimeError):
    def __init__(self, status: int, what: str, info: int = -1):
        self.status = status
        self.info = info
        super().__init__(f"{what}: {status_string(status)} (status {status}, info {info})")


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_2003_05324_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I32, U32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
    sig = {
        "mpgeo_ctx_create": ([ctypes.POINTER(P), ctypes.c_int, P, ctypes.c_size_t], ctypes.c_int),
        "mpgeo_ctx_destroy": ([P], ctypes.c_int),
        "mpgeo_ctx_kernel_stats": ([P, ctypes.POINTER(KernelStat), ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "mpgeo_ctx_reset_stats": ([P], ctypes.c_int),
        "mpgeo_loglik": ([P, I64, P, P, Theta, Plan, ctypes.POINTER(Result)], ctypes.c_int),
        "mpgeo_dataset_create": ([P, I64, P, P, U32, ctypes.POINTER(P)], ctypes.c_int),
        "mpgeo_dataset_destroy": ([P], ctypes.c_int),
        "mpgeo_dataset_loglik": ([P, Theta, Plan, ctypes.POINTER(Result)], ctypes.c_int),
        "mpgeo_dataset_krige": ([P, I64, P, P, P], ctypes.c_int),
        "mpgeo_dataset_perm": ([P, P], ctypes.c_int),
        "mpgeo_dataset_covariance": ([P, Theta, Plan], ctypes.c_int),
        "mpgeo_dataset_matrix": ([P, P, I64], ctypes.c_int),
        "mpgeo_dataset_solution": ([P, P], ctypes.c_int),
        "mpgeo_factor_dense": ([P, I64, P, I64, P, Plan, ctypes.POINTER(Result)], ctypes.c_int),
        "mpgeo_footprint_bytes": ([I64, Plan], ctypes.c_size_t),
        "mpgeo_dataset_entries": ([P, I64, P, P, P], ctypes.c_int),
        "mpgeo_dataset_simulate": ([P, Theta, Plan, P, P], ctypes.c_int),
        "mpgeo_dataset_mle": ([P, Theta, Plan, D, D, I32, ctypes.POINTER(Theta),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I32),
                               ctypes.POINTER(I32)], ctypes.c_int),
        "mpgeo_dataset_mle_trace": ([P, Theta, Plan, D, D, I32, ctypes.POINTER(Theta),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I32),
                                     ctypes.POINTER(I32), ctypes.POINTER(Theta), P], ctypes.c_int),
        "mpgeo_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "mpgeo_plan_tiers": ([I64, Plan, ctypes.POINTER(PlanTiers)], ctypes.c_int),
        "mpgeo_batch_loglik": ([P, I64, ctypes.POINTER(Instance), Plan, ctypes.POINTER(Result),
                                ctypes.POINTER(I32)], ctypes.c_int),
        "mpgeo_batch_loglik_noalloc": ([P, I64, ctypes.POINTER(Instance), Plan, ctypes.POINTER(Result)],
                                       ctypes.c_int),
        "mpgeo_server_create": ([P, ctypes.c_uint64, I32, ctypes.POINTER(P)], ctypes.c_int),
        "mpgeo_server_add_dataset": ([P, I64, P, P, Plan, ctypes.POINTER(I32)], ctypes.c_int),
        "mpgeo_server_submit": ([P, I32, Theta, D, ctypes.POINTER(I64)], ctypes.c_int),
        "mpgeo_server_submit_krige": ([P, I32, Theta, I64, P, P, P, D, ctypes.POINTER(I64)], ctypes.c_int),
        "mpgeo_server_run": ([P, ctypes.POINTER(Served)], ctypes.c_int),
        "mpgeo_server_destroy": ([P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    del I32, D
    return lib


LIB = _load()


def status_string(status: int) -> str:
    return LIB.mpgeo_status_string(status).decode()


def _check(status: int, what: str, info: int = -1) -> None:
    if status != MPGEO_OK:
        raise MpgeoError(status, what, info)


def _host_f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.data_ptr()
    return a.ctypes.data


LOWP = {None: 0, "fp16": 1, "bf16": 2}


def make_plan(tile: int, band64: int, flags: int = 0, band32: int = -1, lowp=None,
              band0: int = -1, dist64: float = 0.0, dist32: float = 0.0) -> Plan:
    """Plan: FP64 within band64 tiles of the diagonal, FP32 beyond; with band32 >= 0 and
    lowp in {"fp16", "bf16"}, 16-bit operands for tiles farther than band64 + band32; with
    band0 >= 0, tiles farther than band0 are dropped (zero).  dist64 > 0: the tiers are drawn
    from the distance between the tiles' blocks of sites instead (FP64 within dist64, FP32
    within dist32 when a 16-bit format is given, 16-bit beyond)."""
    return Plan(tile=tile, band64=band64, band32=band32, lowp=LOWP[lowp], flags=flags,
                band0=band0, dist64=dist64, dist32=dist32)


def mpgeo_footprint_bytes(n: int, tile: int, band64: int, band32: int = -1, lowp=None,
                          band0: int = -1) -> int:
    return int(LIB.mpgeo_footprint_bytes(n, make_plan(tile, band64, 0, band32, lowp, band0)))


def plan_tiers(n: int, tile: int, band64: int, band32: int = -1, lowp=None, band0: int = -1) -> dict:
    """The precision map for n and a plan (host computation): tiers, tile counts, flops."""
    out = PlanTiers()
    _check(LIB.mpgeo_plan_tiers(n, make_plan(tile, band64, 0, band32, lowp, band0), ctypes.byref(out)),
           "mpgeo_plan_tiers")
    return {"p": out.p, "nbp": out.nbp, "band64": out.band64, "edge": out.edge, "band0": out.band0,
            "lowp": out.lowp, "tiles": list(out.tiles), "update_flops": list(out.update_flops),
            "trsm_flops": list(out.trsm_flops), "potrf_flops": out.potrf_flops,
            "footprint_bytes": out.footprint_bytes}


class Context:
    """A library context on one device, ordered on a HIP stream (default: torch's current).
    hbm_budget_bytes > 0 caps the tile memory of one evaluation (MPGEO_E_NOMEM beyond it)."""

    def __init__(self, device: int = 0, stream: Optional["torch.cuda.Stream"] = None,
                 hbm_budget_bytes: int = 0):
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        handle = ctypes.c_void_p()
        _check(LIB.mpgeo_ctx_create(ctypes.byref(handle), device, ctypes.c_void_p(stream.cuda_stream),
                                    int(hbm_budget_bytes)), "mpgeo_ctx_create")
        self.handle = handle

    def close(self) -> None:
        if self.handle:
            LIB.mpgeo_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def loglik(self, locs, z, theta: Sequence[float], tile: int, band64: int,
               morton: bool = True, timing: bool = False, band32: int = -1, lowp=None,
               profile: bool = False, gcd: bool = False, band0: int = -1,
               escalate: bool = False, graph: bool = False) -> dict:
        """One-shot eq. (2) (or the profile likelihood): ordering, covariance tiles, factor,
        solve, reduction.  escalate=True: MPGEO_ESCALATE; graph=True: MPGEO_GRAPH (reserved, rejected)."""
        dev = isinstance(locs, torch.Tensor)
        if not dev:
            locs, z = _host_f64(locs), _host_f64(z)
        flags = (MPGEO_ORDER_MORTON if morton else 0) | (MPGEO_INPUT_DEVICE if dev else 0) | \
                (MPGEO_TIMING if timing else 0) | (MPGEO_PROFILE if profile else 0) | \
                (MPGEO_DIST_GCD if gcd else 0) | (MPGEO_ESCALATE if escalate else 0) | \
                (MPGEO_GRAPH if graph else 0)
        res = Result()
        st = LIB.mpgeo_loglik(self.handle, int(locs.shape[0]), _ptr(locs), _ptr(z), Theta(*theta),
                              make_plan(tile, band64, flags, band32, lowp, band0), ctypes.byref(res))
        _check(st, "mpgeo_loglik", res.info)
        return res.as_dict()

    def factor_dense(self, a, z, tile: int, band64: int, band32: int = -1,
                     lowp=None, band0: int = -1, escalate: bool = False) -> dict:
        """Algorithm 1 on a given symmetric positive-definite matrix (lower triangle read);
        a (and z) may be torch tensors on the device (a column-major: pass the transpose of a
        contiguous row-major tensor's storage, i.e. a symmetric matrix as is)."""
        flags = MPGEO_ESCALATE if escalate else 0
        if isinstance(a, torch.Tensor):
            n = int(a.shape[0])
            zz = z
            flags |= MPGEO_INPUT_DEVICE
        else:
            a = np.asfortranarray(np.asarray(a, dtype=np.float64))
            n = a.shape[0]
            zz = None if z is None else _host_f64(z)
        res = Result()
        st = LIB.mpgeo_factor_dense(self.handle, n, _ptr(a), n, _ptr(zz),
                                    make_plan(tile, band64, flags, band32, lowp, band0), ctypes.byref(res))
        _check(st, "mpgeo_factor_dense", res.info)
        return res.as_dict()

    def batch_loglik(self, problems, tile: int = 0, band64: int = -1, band32: int = -1, lowp=None,
                     profile: bool = False, gcd: bool = False, band0: int = -1,
                     queue: bool = False, tune_band: bool = False, escalate: bool = False) -> tuple:
        """eq. (2) for many independent (locs, z, theta) problems in one call (host arrays).
        tile = 0: tile size chosen per instance by the autotuner; tune_band: the FP64 band too
        (MPGEO_TUNE_BAND; the chosen band is each result's "band64").  queue=True: one
        persistent kernel over a device task queue (two-tier plans, tile 128).  Returns (status,
        results, tiles) without raising on non-positive-definite instances (their info is >= 0)."""
        keep = []
        arr = (Instance * max(1, len(problems)))()
        for q, (locs, z, theta) in enumerate(problems):
            locs, z = _host_f64(locs), _host_f64(z)
            keep.append((locs, z))
            arr[q] = Instance(int(locs.shape[0]), locs.ctypes.data, z.ctypes.data, Theta(*theta))
        res = (Result * max(1, len(problems)))()
        tiles = (ctypes.c_int32 * max(1, len(problems)))()
        flags = ((MPGEO_PROFILE if profile else 0) | (MPGEO_DIST_GCD if gcd else 0) |
                 (MPGEO_BATCH_QUEUE if queue else 0) | (MPGEO_TUNE_BAND if tune_band else 0) |
                 (MPGEO_ESCALATE if escalate else 0))
        st = LIB.mpgeo_batch_loglik(self.handle, len(problems), arr,
                                    make_plan(tile, band64, flags, band32, lowp, band0), res, tiles)
        if st not in (MPGEO_OK, MPGEO_E_NOT_SPD):
            _check(st, "mpgeo_batch_loglik")
        return st, [res[q].as_dict() for q in range(len(problems))], [tiles[q] for q in range(len(problems))]

    def batch_loglik_noalloc(self, problems, band64: int = -1, profile: bool = False,
                             gcd: bool = False) -> tuple:
        """The persistent-queue batch through mpgeo_batch_loglik_noalloc: every work buffer in
        the GPU's fixed device array (tile 128).  Returns (status, results) without raising on
        non-positive-definite instances."""
        keep = []
        arr = (Instance * max(1, len(problems)))()
        for q, (locs, z, theta) in enumerate(problems):
            locs, z = _host_f64(locs), _host_f64(z)
            keep.append((locs, z))
            arr[q] = Instance(int(locs.shape[0]), locs.ctypes.data, z.ctypes.data, Theta(*theta))
        res = (Result * max(1, len(problems)))()
        flags = (MPGEO_PROFILE if profile else 0) | (MPGEO_DIST_GCD if gcd else 0)
        st = LIB.mpgeo_batch_loglik_noalloc(self.handle, len(problems), arr,
                                            make_plan(128, band64, flags), res)
        if st not in (MPGEO_OK, MPGEO_E_NOT_SPD):
            _check(st, "mpgeo_batch_loglik_noalloc")
        return st, [res[q].as_dict() for q in range(len(problems))]

    def kernel_stats(self) -> list:
        arr = (KernelStat * 32)()
        count = ctypes.c_int()
        _check(LIB.mpgeo_ctx_kernel_stats(self.handle, arr, 32, ctypes.byref(count)),
               "mpgeo_ctx_kernel_stats")
        return [{"name": s.name.decode(), "launches": s.launches, "seconds": s.seconds,
                 "flops": s.flops, "bytes": s.bytes} for s in arr[:count.value]]

    def reset_stats(self) -> None:
        _check(LIB.mpgeo_ctx_reset_stats(self.handle), "mpgeo_ctx_reset_stats")


class Dataset:
    """Locations and data resident on the device, Morton-ordered once."""

    def __init__(self, ctx: Context, locs, z=None, morton: bool = True, gcd: bool = False):
        """gcd=True: locations are (longitude, latitude) in degrees and distances are
        great-circle distances in km."""
        self.ctx = ctx
        dev = isinstance(locs, torch.Tensor)
        if not dev:
            locs = _host_f64(locs)
            z = None if z is None else _host_f64(z)
        self.device_io = dev
        self.n = int(locs.shape[0])
        flags = (MPGEO_ORDER_MORTON if morton else 0) | (MPGEO_INPUT_DEVICE if dev else 0) | \
                (MPGEO_DIST_GCD if gcd else 0)
        handle = ctypes.c_void_p()
        _check(LIB.mpgeo_dataset_create(ctx.handle, self.n, _ptr(locs), _ptr(z), flags,
                                        ctypes.byref(handle)), "mpgeo_dataset_create")
        self.handle = handle

    def close(self) -> None:
        if self.handle:
            LIB.mpgeo_dataset_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def loglik(self, theta: Sequence[float], tile: int, band64: int, timing: bool = False,
               band32: int = -1, lowp=None, profile: bool = False, band0: int = -1,
               dist64: float = 0.0, dist32: float = 0.0, escalate: bool = False,
               graph: bool = False) -> dict:
        """eq. (2) at theta on the resident dataset.  graph=True: MPGEO_GRAPH (reserved, rejected)."""
        res = Result()
        flags = (MPGEO_TIMING if timing else 0) | (MPGEO_PROFILE if profile else 0) | \
                (MPGEO_ESCALATE if escalate else 0) | (MPGEO_GRAPH if graph else 0)
        st = LIB.mpgeo_dataset_loglik(self.handle, Theta(*theta),
                                      make_plan(tile, band64, flags, band32, lowp, band0, dist64, dist32),
                                      ctypes.byref(res))
        _check(st, "mpgeo_dataset_loglik", res.info)
        return res.as_dict()

    def try_loglik(self, theta: Sequence[float], tile: int, band64: int, band0: int = -1,
                   band32: int = -1, lowp=None, escalate: bool = False) -> tuple:
        """(status, result dict) without raising (for optimisers that meet non-SPD points)."""
        res = Result()
        st = LIB.mpgeo_dataset_loglik(self.handle, Theta(*theta),
                                      make_plan(tile, band64, MPGEO_ESCALATE if escalate else 0, band32,
                                                lowp, band0), ctypes.byref(res))
        return st, res.as_dict()

    def krige(self, new_locs, variance: bool = False):
        if self.device_io:
            m = int(new_locs.shape[0])
            pred = torch.empty(m, dtype=torch.float64, device=new_locs.device)
            var = torch.empty(m, dtype=torch.float64, device=new_locs.device) if variance else None
        else:
            new_locs = _host_f64(new_locs)
            m = new_locs.shape[0]
            pred = np.empty(m)
            var = np.empty(m) if variance else None
        _check(LIB.mpgeo_dataset_krige(self.handle, m, _ptr(new_locs), _ptr(pred), _ptr(var)),
               "mpgeo_dataset_krige")
        return (pred, var) if variance else pred

    def simulate(self, theta: Sequence[float], eps, tile: int, band64: int = -1):
        """A draw z = P^T L P eps of the Matérn field at the dataset's locations (caller order)."""
        if self.device_io:
            z = torch.empty_like(eps)
        else:
            eps = _host_f64(eps)
            z = np.empty(self.n)
        _check(LIB.mpgeo_dataset_simulate(self.handle, Theta(*theta), make_plan(tile, band64),
                                          _ptr(eps), _ptr(z)), "mpgeo_dataset_simulate")
        return z

    def perm(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int64)
        _check(LIB.mpgeo_dataset_perm(self.handle, out.ctypes.data), "mpgeo_dataset_perm")
        return out

    def covariance(self, theta: Sequence[float], tile: int, band64: int,
                   profile: bool = False, band32: int = -1, lowp=None, dist64: float = 0.0,
                   dist32: float = 0.0) -> np.ndarray:
        """Sigma (the correlation matrix with profile=True) as stored in its tiles
        (tier-rounded), lower triangle, ordered."""
        plan = make_plan(tile, band64, MPGEO_PROFILE if profile else 0, band32, lowp, -1, dist64, dist32)
        _check(LIB.mpgeo_dataset_covariance(self.handle, Theta(*theta), plan),
               "mpgeo_dataset_covariance")
        return self.matrix()

    def matrix(self) -> np.ndarray:
        out = np.zeros((self.n, self.n), order="F")
        _check(LIB.mpgeo_dataset_matrix(self.handle, out.ctypes.data, self.n), "mpgeo_dataset_matrix")
        return out

    def entries(self, rows, cols) -> np.ndarray:
        """Stored lower-triangle entries M[max(r, c), min(r, c)] at ordered indices."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.empty(rows.shape[0])
        _check(LIB.mpgeo_dataset_entries(self.handle, rows.shape[0], rows.ctypes.data,
                                         cols.ctypes.data, out.ctypes.data), "mpgeo_dataset_entries")
        return out

    def mle(self, start: Sequence[float], tile: int, band64: int, xtol: float = 1e-6,
            ftol: float = 0.0, max_evals: int = 1000, band32: int = -1, lowp=None,
            profile: bool = False, escalate: bool = False, graph: bool = False) -> dict:
        """Nelder-Mead maximum-likelihood fit of theta from `start` (eq. (2)); with
        profile=True a two-dimensional search over (theta2, theta3) of the profile likelihood."""
        th = Theta()
        ll = ctypes.c_double()
        ev = ctypes.c_int32()
        it = ctypes.c_int32()
        plan = make_plan(tile, band64, (MPGEO_PROFILE if profile else 0) |
                         (MPGEO_ESCALATE if escalate else 0) | (MPGEO_GRAPH if graph else 0), band32, lowp)
        _check(LIB.mpgeo_dataset_mle(self.handle, Theta(*start), plan, xtol, ftol,
                                     max_evals, ctypes.byref(th), ctypes.byref(ll), ctypes.byref(ev),
                                     ctypes.byref(it)), "mpgeo_dataset_mle")
        return {"theta": (th.sigma2, th.beta, th.nu), "loglik": ll.value, "evals": ev.value,
                "iters": it.value}

    def mle_trace(self, start: Sequence[float], tile: int, band64: int, xtol: float = 1e-6,
                  ftol: float = 0.0, max_evals: int = 1000, band32: int = -1, lowp=None,
                  graph: bool = False) -> dict:
        """mle() that also returns the search's trajectory: every evaluated theta in order and
        its log-likelihood (-inf where the matrix was not positive definite)."""
        th = Theta()
        ll = ctypes.c_double()
        ev = ctypes.c_int32()
        it = ctypes.c_int32()
        trace = (Theta * max_evals)()
        trace_ll = np.empty(max_evals)
        _check(LIB.mpgeo_dataset_mle_trace(self.handle, Theta(*start), make_plan(tile, band64, MPGEO_GRAPH if graph else 0,
                                                                             band32, lowp),
                                           xtol, ftol, max_evals, ctypes.byref(th), ctypes.byref(ll),
                                           ctypes.byref(ev), ctypes.byref(it), trace, trace_ll.ctypes.data),
               "mpgeo_dataset_mle_trace")
        e = ev.value
        return {"theta": (th.sigma2, th.beta, th.nu), "loglik": ll.value, "evals": e, "iters": it.value,
                "trace": [(t.sigma2, t.beta, t.nu) for t in trace[:e]], "trace_loglik": trace_ll[:e].copy()}

    def solution(self) -> np.ndarray:
        out = np.empty(self.n)
        _check(LIB.mpgeo_dataset_solution(self.handle, out.ctypes.data), "mpgeo_dataset_solution")
        return out


class Server:
    """Serving loop: resident datasets, requests with arrival times, continuous dispatch."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, lanes: int = 4):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(LIB.mpgeo_server_create(ctx.handle, int(hbm_budget_bytes), lanes, ctypes.byref(h)),
               "mpgeo_server_create")
        self.handle = h
        self.count = 0
        self._krige = {}   # ticket -> (sites, pred, var) kept alive until run

    def add_dataset(self, locs, z, tile: int, band64: int, band32: int = -1, lowp=None,
                    queue: bool = False) -> int:
        """queue=True: the dataset's likelihood requests run through the persistent task queue,
        batched with the other ready ones (two-tier plans at tile 128, n <= 16,384)."""
        locs, z = _host_f64(locs), _host_f64(z)
        out = ctypes.c_int32()
        flags = MPGEO_BATCH_QUEUE if queue else 0
        _check(LIB.mpgeo_server_add_dataset(self.handle, locs.shape[0], locs.ctypes.data, z.ctypes.data,
                                            make_plan(tile, band64, flags, band32, lowp), ctypes.byref(out)),
               "mpgeo_server_add_dataset")
        return out.value

    def submit(self, dataset: int, theta: Sequence[float], arrival_s: float) -> int:
        t = ctypes.c_int64()
        _check(LIB.mpgeo_server_submit(self.handle, dataset, Theta(*theta), float(arrival_s), ctypes.byref(t)),
               "mpgeo_server_submit")
        self.count += 1
        return t.value

    def submit_krige(self, dataset: int, theta: Sequence[float], new_locs, arrival_s: float,
                     variance: bool = False) -> int:
        """A kriging request: the factor of (dataset, theta), then predictions (and variances)
        at new_locs (m x 2); they appear as "pred" (and "var") in run()'s result."""
        sites = _host_f64(new_locs)
        m = int(sites.shape[0])
        pred = np.empty(m, dtype=np.float64)
        var = np.empty(m, dtype=np.float64) if variance else None
        t = ctypes.c_int64()
        _check(LIB.mpgeo_server_submit_krige(self.handle, dataset, Theta(*theta), m, sites.ctypes.data,
                                             pred.ctypes.data, var.ctypes.data if variance else None,
                                             float(arrival_s), ctypes.byref(t)),
               "mpgeo_server_submit_krige")
        self._krige[t.value] = (sites, pred, var)
        self.count += 1
        return t.value

    def run(self) -> tuple:
        """Replays the submitted requests; returns (status, per-request dicts in ticket order)."""
        out = (Served * max(1, self.count))()
        st = LIB.mpgeo_server_run(self.handle, out)
        if st not in (MPGEO_OK, MPGEO_E_NOT_SPD):
            self._krige = {}
            _check(st, "mpgeo_server_run")
        res = [out[q].as_dict() for q in range(self.count)]
        for t, (_, pred, var) in self._krige.items():
            res[t]["pred"] = pred
            if var is not None:
                res[t]["var"] = var
        self._krige = {}
        self.count = 0
        return st, res

    def close(self) -> None:
        if self.handle:
            LIB.mpgeo_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
