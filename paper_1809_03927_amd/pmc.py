"""Thin ctypes binding of libpmc (include/pmc.h), with the same names.

Argument marshalling only: every step of the transport runs in libpmc's HIP
kernels.  Importing this module loads the in-tree libpmc.so and fails loudly
if it has not been built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

from .workloads import FIELD_DTYPE, SPOT_DTYPE

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmc.so")

PMC_OK = 0
PMC_E_INVAL, PMC_E_NOPHASE, PMC_E_BUDGET, PMC_E_DEVICE, PMC_E_RANGE, PMC_E_STATE = -1, -2, -3, -4, -5, -6
PMC_MAX_HISTORIES = 50_000_000
PMC_MAX_PHASES = 64
PMC_FP32, PMC_FP64 = 0, 1
PMC_NO_STRAGGLING, PMC_NO_MCS, PMC_NO_DELTA, PMC_NO_NUCLEAR, PMC_FROZEN = 1, 2, 4, 8, 16
PMC_ENGINE_PLAIN, PMC_ENGINE_PERSISTENT = 0, 1
PMC_TALLY_AUTO, PMC_TALLY_LANE, PMC_TALLY_CORE = 0, 1, 2
PMC_COUNTERS = 16

ERROR_NAMES = {0: "PMC_OK", -1: "PMC_E_INVAL", -2: "PMC_E_NOPHASE", -3: "PMC_E_BUDGET",
               -4: "PMC_E_DEVICE", -5: "PMC_E_RANGE", -6: "PMC_E_STATE"}

# every symbol declared in include/pmc.h
EXPORTS = ["pmc_create", "pmc_destroy", "pmc_last_error", "pmc_load_phase", "pmc_unload_phase",
           "pmc_load_spots", "pmc_load_plan", "pmc_load_subplans", "pmc_unload_plan", "pmc_request_items", "pmc_request_item_histories", "pmc_launch_shape", "pmc_dose",
           "pmc_dose_device", "pmc_dose_device_notify", "pmc_dose_device_noalloc", "pmc_atomic_log", "pmc_atomic_replay",
           "pmc_balance_from_counters",
           "pmc_convert_device", "pmc_trace", "pmc_split_histories", "pmc_bytes_in_use",
           "pmc_graph_create", "pmc_graph_launch", "pmc_graph_destroy", "pmc_influence_boxes",
           "pmc_influence", "pmc_influence_read", "pmc_influence_device", "pmc_influence_free",
           "pmc_load_dvf", "pmc_unload_dvf", "pmc_dvf_points", "pmc_accumulate", "pmc_accumulate_device",
           "pmc_accumulate_dim", "pmc_accumulate_dim_device", "pmc_delivery_simulate"]


class pmc_config(C.Structure):
    _fields_ = [("device", C.c_int32), ("precision", C.c_int32), ("seed", C.c_uint64),
                ("hbm_budget_bytes", C.c_uint64)]


class pmc_dvf(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("start_mm", C.c_double * 3), ("spacing_mm", C.c_double * 3),
                ("row", C.c_double * 3), ("col", C.c_double * 3), ("delta_mm", C.c_void_p),
                ("pre", C.c_void_p), ("post", C.c_void_p)]


class pmc_param(C.Structure):
    _fields_ = [("central", C.c_double), ("sd", C.c_double)]


class pmc_synchrotron(C.Structure):
    _fields_ = [(name, pmc_param) for name in (
        "layer_switch_s", "layer_switch_per_mev", "discard_s", "spill_rate_mu_s", "spill_rate_per_mev",
        "spot_switch_s", "spot_switch_per_mm", "capacity_mu", "extraction_max_s")]


class pmc_delivery(C.Structure):
    _fields_ = [("n_phases", C.c_int32), ("start_phase", C.c_int32), ("period_s", C.c_double),
                ("period_sd_s", C.c_double), ("period_min_s", C.c_int32), ("period_max_s", C.c_int32),
                ("gate_lo", C.c_int32), ("gate_hi", C.c_int32), ("max_mu", C.c_double),
                ("sync", pmc_synchrotron), ("seed", C.c_uint64), ("n_trials", C.c_int32)]


class pmc_shape(C.Structure):
    _fields_ = [("block_size", C.c_int32), ("chunk", C.c_int32), ("refill_min", C.c_int32),
                ("tally_mode", C.c_int32), ("core_capacity", C.c_int32), ("reserved", C.c_int32 * 3)]


class pmc_request(C.Structure):
    _fields_ = [("request_id", C.c_uint32), ("flags", C.c_uint32), ("n_histories", C.c_uint64),
                ("phases", C.POINTER(C.c_int32)), ("n_phases", C.c_int32), ("engine", C.c_int32),
                ("block_size", C.c_int32), ("chunk", C.c_int32), ("refill_min", C.c_int32),
                ("grid_blocks", C.c_int32), ("plan", C.c_int32), ("tally_mode", C.c_int32),
                ("item_begin", C.c_uint64), ("item_end", C.c_uint64)]


class pmc_balance(C.Structure):
    _fields_ = [("incident", C.c_uint64 * 2), ("deposited", C.c_uint64 * 2),
                ("escaped", C.c_uint64 * 2), ("nuclear", C.c_uint64 * 2), ("cutoff", C.c_uint64 * 2),
                ("histories", C.c_uint64), ("steps", C.c_uint64), ("delta_events", C.c_uint64),
                ("nuclear_events", C.c_uint64), ("escapes", C.c_uint64), ("misses", C.c_uint64)]

    def as_dict(self):
        def w(x):
            return int(x[0]) + (int(x[1]) << 64)
        return {"incident": w(self.incident), "deposited": w(self.deposited),
                "escaped": w(self.escaped), "nuclear": w(self.nuclear), "cutoff": w(self.cutoff),
                "histories": int(self.histories), "steps": int(self.steps),
                "delta_events": int(self.delta_events), "nuclear_events": int(self.nuclear_events),
                "escapes": int(self.escapes), "misses": int(self.misses)}


TRACE_DTYPE = np.dtype([
    ("cause", "<i4"), ("voxel", "<i4"), ("fate", "<i4"), ("block", "<u4"),
    ("s", "<f8"), ("E", "<f8"), ("r", "<f8", 3), ("w", "<f8", 3),
    ("n_delta", "<f8"), ("n_nuc", "<f8"), ("l_acc", "<f8"), ("dep", "<i8"), ("t_delta", "<f8"),
])
assert TRACE_DTYPE.itemsize == 120

BOX_DTYPE = np.dtype([("lo", "<i4", 3), ("hi", "<i4", 3)])  # pmc_box


class PmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1809_03927_amd/build.py "
                              "(or __graft_entry__.build())")
        # One HIP runtime per process: PyTorch ships its own libamdhip64 (same
        # SONAME as the system one libpmc links).  Loading torch first makes
        # libpmc bind to that copy; loading libpmc first would make torch load
        # a second runtime, which then finds no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u32, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
        L.pmc_create.argtypes = [C.POINTER(pmc_config), C.POINTER(vp)]
        L.pmc_destroy.argtypes = [vp]
        L.pmc_destroy.restype = None
        L.pmc_last_error.argtypes = [vp]
        L.pmc_last_error.restype = C.c_char_p
        L.pmc_load_phase.argtypes = [vp, i32, vp, i32, i32, i32, vp, vp, vp, vp, vp, i32, vp]
        L.pmc_unload_phase.argtypes = [vp, i32]
        L.pmc_load_spots.argtypes = [vp, vp, i32, vp, i64]
        L.pmc_load_plan.argtypes = [vp, i32, vp, i32, vp, i64]
        L.pmc_load_subplans.argtypes = [vp, i32, vp, i32, vp, i64, vp, i32, vp, vp]
        L.pmc_unload_plan.argtypes = [vp, i32]
        L.pmc_request_items.argtypes = [vp, C.POINTER(pmc_request), C.POINTER(u64)]
        L.pmc_request_item_histories.argtypes = [vp, C.POINTER(pmc_request), vp, u64, C.POINTER(u64)]
        L.pmc_load_dvf.argtypes = [vp, i32, C.POINTER(pmc_dvf)]
        L.pmc_unload_dvf.argtypes = [vp, i32]
        L.pmc_dvf_points.argtypes = [vp, i32, vp, vp]
        L.pmc_delivery_simulate.argtypes = [vp, C.POINTER(pmc_delivery), vp, i64, i32, vp, vp, vp]
        L.pmc_accumulate.argtypes = [vp, i32, vp, i32, vp, vp, vp, i32, u64, vp, vp]
        L.pmc_accumulate_device.argtypes = [vp, i32, vp, i32, vp, vp, vp, i32, u64, vp, vp, vp]
        L.pmc_accumulate_dim.argtypes = [vp, i32, vp, i32, vp, vp, vp, i32, u64, vp, vp]
        L.pmc_accumulate_dim_device.argtypes = [vp, i32, vp, i32, vp, vp, vp, i32, u64, vp, vp, vp]
        L.pmc_launch_shape.argtypes = [vp, C.POINTER(pmc_request), C.POINTER(pmc_shape)]
        L.pmc_dose.argtypes = [vp, C.POINTER(pmc_request), vp, vp, vp, C.POINTER(pmc_balance)]
        L.pmc_dose_device.argtypes = [vp, C.POINTER(pmc_request), vp, vp, vp]
        L.pmc_dose_device_notify.argtypes = [vp, C.POINTER(pmc_request), vp, vp, vp, vp]
        L.pmc_dose_device_noalloc.argtypes = [vp, C.POINTER(pmc_request), vp, vp, vp]
        L.pmc_atomic_log.argtypes = [vp, C.POINTER(pmc_request), vp, vp, vp, vp, u32, vp]
        L.pmc_atomic_replay.argtypes = [vp, vp, vp, u32, vp, u32]
        L.pmc_balance_from_counters.argtypes = [vp, C.POINTER(pmc_request), vp, vp,
                                                C.POINTER(pmc_balance)]
        L.pmc_convert_device.argtypes = [vp, i32, vp, u64, vp, vp, vp]
        L.pmc_trace.argtypes = [vp, i32, i32, i64, u32, u32, u32, vp, i32, C.POINTER(C.c_int32)]
        L.pmc_split_histories.argtypes = [vp, i64, vp, i32, u64, vp]
        L.pmc_bytes_in_use.argtypes = [vp]
        L.pmc_bytes_in_use.restype = u64
        L.pmc_graph_create.argtypes = [vp, C.POINTER(pmc_request), vp, vp, vp, C.POINTER(vp)]
        L.pmc_graph_launch.argtypes = [vp, vp]
        L.pmc_graph_destroy.argtypes = [vp]
        L.pmc_graph_destroy.restype = None
        L.pmc_influence_boxes.argtypes = [vp, i32, i32, vp, i64]
        L.pmc_influence.argtypes = [vp, C.POINTER(pmc_request), vp, C.c_double, u64, C.POINTER(u64),
                                    C.POINTER(pmc_balance), vp]
        L.pmc_influence_read.argtypes = [vp, vp, vp, vp]
        L.pmc_influence_device.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]
        L.pmc_influence_free.argtypes = [vp]
        _lib = L
    return _lib


def _check(rc: int, ctx=None):
    if rc != PMC_OK:
        msg = lib().pmc_last_error(ctx).decode(errors="replace")
        raise PmcError(rc, msg)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


# ----------------------------------------------------------------------------
# same names as the C ABI
# ----------------------------------------------------------------------------

def pmc_create(device=0, precision=PMC_FP32, seed=0, hbm_budget_bytes=0):
    cfg = pmc_config(device, precision, seed, hbm_budget_bytes)
    h = C.c_void_p()
    _check(lib().pmc_create(C.byref(cfg), C.byref(h)))
    return h


def pmc_destroy(ctx):
    lib().pmc_destroy(ctx)


def pmc_last_error(ctx=None) -> str:
    return lib().pmc_last_error(ctx).decode(errors="replace")


def pmc_load_phase(ctx, phase_id: int, ph) -> None:
    hu = np.ascontiguousarray(ph.hu, dtype=np.int16)
    nz, ny, nx = hu.shape
    sp = np.ascontiguousarray(ph.spacing_mm, dtype=np.float64)
    org = np.ascontiguousarray(ph.origin_mm, dtype=np.float64)
    ch = np.ascontiguousarray(ph.calib_hu, dtype=np.float64)
    cr = np.ascontiguousarray(ph.calib_rho, dtype=np.float64)
    cs = np.ascontiguousarray(ph.calib_rsp, dtype=np.float64)
    mask = None if ph.mask is None else np.ascontiguousarray(ph.mask, dtype=np.uint8)
    if not (len(ch) == len(cr) == len(cs)):
        raise ValueError("calibration arrays differ in length")
    _check(lib().pmc_load_phase(ctx, phase_id, _ptr(hu), nx, ny, nz, _ptr(sp), _ptr(org), _ptr(ch),
                                _ptr(cr), _ptr(cs), len(ch), _ptr(mask)), ctx)


def pmc_unload_phase(ctx, phase_id: int) -> None:
    _check(lib().pmc_unload_phase(ctx, phase_id), ctx)


def pmc_load_spots(ctx, fields: np.ndarray, spots: np.ndarray) -> None:
    f = np.ascontiguousarray(fields, dtype=FIELD_DTYPE)
    s = np.ascontiguousarray(spots, dtype=SPOT_DTYPE)
    _check(lib().pmc_load_spots(ctx, _ptr(f), len(f), _ptr(s), len(s)), ctx)


def pmc_load_plan(ctx, plan_id: int, fields: np.ndarray, spots: np.ndarray) -> None:
    f = np.ascontiguousarray(fields, dtype=FIELD_DTYPE)
    s = np.ascontiguousarray(spots, dtype=SPOT_DTYPE)
    _check(lib().pmc_load_plan(ctx, plan_id, _ptr(f), len(f), _ptr(s), len(s)), ctx)


def pmc_load_subplans(ctx, plan_id: int, fields: np.ndarray, spots: np.ndarray, mu: np.ndarray,
                      phase_ids: Sequence[int]) -> int:
    """mu: (n_spots, n_phases) MU of one delivery trial; returns the number
    of sub-plan spots loaded as plan plan_id."""
    f = np.ascontiguousarray(fields, dtype=FIELD_DTYPE)
    s = np.ascontiguousarray(spots, dtype=SPOT_DTYPE)
    m = np.ascontiguousarray(mu, dtype=np.float64)
    ids = np.ascontiguousarray(phase_ids, dtype=np.int32)
    if m.shape != (len(s), len(ids)):
        raise ValueError("mu must be (n_spots, n_phases)")
    n = C.c_int64(0)
    _check(lib().pmc_load_subplans(ctx, plan_id, _ptr(f), len(f), _ptr(s), len(s), _ptr(m), len(ids),
                                   _ptr(ids), C.byref(n)), ctx)
    return int(n.value)


def pmc_unload_plan(ctx, plan_id: int) -> None:
    _check(lib().pmc_unload_plan(ctx, plan_id), ctx)


class Request:
    """A pmc_request that keeps its phase list alive."""

    def __init__(self, n_histories: int, phases: Sequence[int], request_id=0, flags=0,
                 engine=PMC_ENGINE_PLAIN, block_size=0, chunk=0, refill_min=0, grid_blocks=0,
                 plan=0, item_begin=0, item_end=0, tally_mode=PMC_TALLY_AUTO):
        self.phase_arr = np.ascontiguousarray(phases, dtype=np.int32)
        self.c = pmc_request(request_id, flags, n_histories,
                             self.phase_arr.ctypes.data_as(C.POINTER(C.c_int32)),
                             len(self.phase_arr), engine, block_size, chunk, refill_min, grid_blocks,
                             plan, tally_mode, item_begin, item_end)

    def slice(self, item_begin: int, item_end: int) -> "Request":
        """The same request restricted to work items [item_begin, item_end)."""
        r = Request.__new__(Request)
        r.phase_arr = self.phase_arr
        r.c = pmc_request.from_buffer_copy(self.c)
        r.c.item_begin = item_begin
        r.c.item_end = item_end
        return r

    @property
    def n_phases(self):
        return len(self.phase_arr)


def pmc_dose(ctx, req: Request, nvox: Sequence[int], want_dose=True, want_tally=True,
             want_density=False):
    """Returns (doses, tallies, densities, balance dict); lists per phase."""
    n = req.n_phases
    doses = [np.zeros(v, dtype=np.float64) for v in nvox] if want_dose else None
    tallies = [np.zeros(v, dtype=np.int64) for v in nvox] if want_tally else None
    dens = [np.zeros(v, dtype=np.float64) for v in nvox] if want_density else None
    dp = (C.c_void_p * n)(*[d.ctypes.data for d in doses]) if want_dose else None
    tp = (C.c_void_p * n)(*[t.ctypes.data for t in tallies]) if want_tally else None
    rp = (C.c_void_p * n)(*[d.ctypes.data for d in dens]) if want_density else None
    bal = pmc_balance()
    _check(lib().pmc_dose(ctx, C.byref(req.c), dp, tp, rp, C.byref(bal)), ctx)
    return doses, tallies, dens, bal.as_dict()


def pmc_dose_device(ctx, req: Request, stream: int, dev_tallies: Sequence[int],
                    dev_counters: Optional[int]) -> None:
    tp = (C.c_void_p * req.n_phases)(*[int(p) for p in dev_tallies])
    _check(lib().pmc_dose_device(ctx, C.byref(req.c), C.c_void_p(stream), tp,
                                 None if dev_counters is None else C.c_void_p(dev_counters)), ctx)


def pmc_dose_device_noalloc(ctx, req: Request, stream: int, dev_tallies: Sequence[int],
                            dev_counters: int) -> None:
    """pmc_dose_device without device allocation (the request data goes into
    the library's fixed per-device scratch array)."""
    tp = (C.c_void_p * req.n_phases)(*[int(p) for p in dev_tallies])
    _check(lib().pmc_dose_device_noalloc(ctx, C.byref(req.c), C.c_void_p(stream), tp,
                                         C.c_void_p(dev_counters)), ctx)


def pmc_atomic_log(ctx, req: Request, stream: int, dev_tallies: Sequence[int], dev_counters: int,
                   dev_log: int, per_lane: int, dev_log_count: int) -> None:
    tp = (C.c_void_p * req.n_phases)(*[int(p) for p in dev_tallies])
    _check(lib().pmc_atomic_log(ctx, C.byref(req.c), C.c_void_p(stream), tp, C.c_void_p(dev_counters),
                                C.c_void_p(dev_log), per_lane, C.c_void_p(dev_log_count)), ctx)


def pmc_atomic_replay(ctx, stream: int, dev_log: int, per_lane: int, dev_log_count: int, n_lanes: int) -> None:
    _check(lib().pmc_atomic_replay(ctx, C.c_void_p(stream), C.c_void_p(dev_log), per_lane,
                                   C.c_void_p(dev_log_count), n_lanes), ctx)


def pmc_dose_device_notify(ctx, req: Request, stream: int, dev_tallies: Sequence[int],
                           dev_counters: Optional[int], host_drained: int) -> None:
    """host_drained: address of a pinned host uint32 (set to 0 before)."""
    tp = (C.c_void_p * req.n_phases)(*[int(p) for p in dev_tallies])
    _check(lib().pmc_dose_device_notify(ctx, C.byref(req.c), C.c_void_p(stream), tp,
                                        None if dev_counters is None else C.c_void_p(dev_counters),
                                        C.c_void_p(host_drained)), ctx)


def pmc_balance_from_counters(ctx, req: Request, counters: np.ndarray, deposited: int) -> dict:
    c = np.ascontiguousarray(counters, dtype=np.uint64)
    d = np.array([deposited & (2**64 - 1), deposited >> 64], dtype=np.uint64)
    bal = pmc_balance()
    _check(lib().pmc_balance_from_counters(ctx, C.byref(req.c), _ptr(c), _ptr(d), C.byref(bal)), ctx)
    return bal.as_dict()


def balance_from_words(counters: np.ndarray, deposited: int, incident: int) -> dict:
    """The dict of pmc_balance_from_counters from a counter block read back
    earlier (layout of PMC_COUNTERS in pmc.h) and the request's incident
    energy (pmc_balance_from_counters with the request still loaded)."""
    c = [int(x) for x in np.asarray(counters, dtype=np.uint64)]
    return {"incident": int(incident), "deposited": int(deposited),
            "escaped": c[0] + (c[1] << 64), "nuclear": c[2] + (c[3] << 64),
            "cutoff": c[4] + (c[5] << 64), "histories": c[6], "steps": c[7],
            "delta_events": c[8], "nuclear_events": c[9], "escapes": c[10], "misses": c[11]}


def pmc_convert_device(ctx, phase_id: int, dev_tally: int, n_histories: int, stream: int,
                       dev_dose: Optional[int], dev_density: Optional[int]) -> None:
    _check(lib().pmc_convert_device(ctx, phase_id, C.c_void_p(dev_tally), n_histories,
                                    C.c_void_p(stream), None if dev_dose is None else C.c_void_p(dev_dose),
                                    None if dev_density is None else C.c_void_p(dev_density)), ctx)


def pmc_request_items(ctx, req: Request) -> int:
    n = C.c_uint64(0)
    _check(lib().pmc_request_items(ctx, C.byref(req.c), C.byref(n)), ctx)
    return int(n.value)


def pmc_request_item_histories(ctx, req: Request) -> np.ndarray:
    """Histories of each work item of a persistent-engine request, queue order."""
    n = C.c_uint64(0)
    _check(lib().pmc_request_item_histories(ctx, C.byref(req.c), None, 0, C.byref(n)), ctx)
    out = np.zeros(n.value, dtype=np.uint32)
    _check(lib().pmc_request_item_histories(ctx, C.byref(req.c), _ptr(out), n.value, C.byref(n)), ctx)
    return out


def pmc_load_dvf(ctx, dvf_id: int, dvf) -> None:
    """dvf: a workloads.Dvf (translations (nz, ny, nx, 3), i fastest)."""
    delta = np.ascontiguousarray(dvf.delta_mm, dtype=np.float64)
    if delta.shape != (dvf.n[2], dvf.n[1], dvf.n[0], 3):
        raise ValueError("delta_mm must have shape (n[2], n[1], n[0], 3)")
    mats = []
    for m in (getattr(dvf, "pre", None), getattr(dvf, "post", None)):
        if m is None:
            mats.append(None)
            continue
        a = np.ascontiguousarray(m, dtype=np.float64)
        if a.shape != (4, 4):
            raise ValueError("pre/post must be 4x4 matrices")
        mats.append(a)
    d = pmc_dvf((C.c_int32 * 3)(*dvf.n), (C.c_double * 3)(*dvf.start_mm),
                (C.c_double * 3)(*dvf.spacing_mm), (C.c_double * 3)(*dvf.row),
                (C.c_double * 3)(*dvf.col), delta.ctypes.data,
                None if mats[0] is None else mats[0].ctypes.data,
                None if mats[1] is None else mats[1].ctypes.data)
    _check(lib().pmc_load_dvf(ctx, dvf_id, C.byref(d)), ctx)


def pmc_dvf_points(ctx, dvf_id: int, n):
    """(x0, r_f) of every grid point, each (n[2], n[1], n[0], 3), computed on
    the device (Eqs. (8), (7))."""
    x0 = np.zeros((n[2], n[1], n[0], 3), dtype=np.float64)
    rf = np.zeros_like(x0)
    _check(lib().pmc_dvf_points(ctx, dvf_id, _ptr(x0), _ptr(rf)), ctx)
    return x0, rf


def pmc_unload_dvf(ctx, dvf_id: int) -> None:
    _check(lib().pmc_unload_dvf(ctx, dvf_id), ctx)


def pmc_accumulate(ctx, ref_phase: int, ref_tally: np.ndarray, src_phases: Sequence[int],
                   src_dvfs: Sequence[int], src_tallies: Sequence[np.ndarray], n_sub: int,
                   n_histories: int, nvox_ref: int, want_mask: bool = False):
    """Returns (dose, mask or None) on the reference grid."""
    ref = np.ascontiguousarray(ref_tally, dtype=np.int64)
    srcs = [np.ascontiguousarray(t, dtype=np.int64) for t in src_tallies]
    ph = np.ascontiguousarray(src_phases, dtype=np.int32)
    dv = np.ascontiguousarray(src_dvfs, dtype=np.int32)
    tp = (C.c_void_p * max(len(srcs), 1))(*[t.ctypes.data for t in srcs])
    dose = np.zeros(nvox_ref, dtype=np.float64)
    mask = np.zeros(nvox_ref, dtype=np.uint8) if want_mask else None
    _check(lib().pmc_accumulate(ctx, ref_phase, _ptr(ref), len(srcs), _ptr(ph), _ptr(dv), tp, n_sub,
                                n_histories, _ptr(dose), _ptr(mask)), ctx)
    return dose, mask


def pmc_accumulate_device(ctx, ref_phase: int, ref_tally: int, src_phases: Sequence[int],
                          src_dvfs: Sequence[int], src_tallies: Sequence[int], n_sub: int,
                          n_histories: int, stream: int, dev_dose: int, dev_mask: Optional[int] = None):
    ph = np.ascontiguousarray(src_phases, dtype=np.int32)
    dv = np.ascontiguousarray(src_dvfs, dtype=np.int32)
    tp = (C.c_void_p * max(len(src_tallies), 1))(*[int(t) for t in src_tallies])
    _check(lib().pmc_accumulate_device(ctx, ref_phase, C.c_void_p(ref_tally), len(src_tallies), _ptr(ph),
                                       _ptr(dv), tp, n_sub, n_histories, C.c_void_p(stream),
                                       C.c_void_p(dev_dose), None if dev_mask is None else C.c_void_p(dev_mask)),
           ctx)


def pmc_accumulate_dim(ctx, ref_phase: int, ref_tally: np.ndarray, src_phases: Sequence[int],
                   src_dvfs: Sequence[int], src_tallies: Sequence[np.ndarray], n_sub: int,
                   n_histories: int, nvox_ref: int, want_mask: bool = False):
    """Dose interpolation (Eq. (3)); src_dvfs map the reference phase onto each
    source.  Returns (dose, mask or None) on the reference grid."""
    ref = np.ascontiguousarray(ref_tally, dtype=np.int64)
    srcs = [np.ascontiguousarray(t, dtype=np.int64) for t in src_tallies]
    ph = np.ascontiguousarray(src_phases, dtype=np.int32)
    dv = np.ascontiguousarray(src_dvfs, dtype=np.int32)
    tp = (C.c_void_p * max(len(srcs), 1))(*[t.ctypes.data for t in srcs])
    dose = np.zeros(nvox_ref, dtype=np.float64)
    mask = np.zeros(nvox_ref, dtype=np.uint8) if want_mask else None
    _check(lib().pmc_accumulate_dim(ctx, ref_phase, _ptr(ref), len(srcs), _ptr(ph), _ptr(dv), tp, n_sub,
                                n_histories, _ptr(dose), _ptr(mask)), ctx)
    return dose, mask


def pmc_accumulate_dim_device(ctx, ref_phase: int, ref_tally: int, src_phases: Sequence[int],
                          src_dvfs: Sequence[int], src_tallies: Sequence[int], n_sub: int,
                          n_histories: int, stream: int, dev_dose: int, dev_mask: Optional[int] = None):
    ph = np.ascontiguousarray(src_phases, dtype=np.int32)
    dv = np.ascontiguousarray(src_dvfs, dtype=np.int32)
    tp = (C.c_void_p * max(len(src_tallies), 1))(*[int(t) for t in src_tallies])
    _check(lib().pmc_accumulate_dim_device(ctx, ref_phase, C.c_void_p(ref_tally), len(src_tallies), _ptr(ph),
                                       _ptr(dv), tp, n_sub, n_histories, C.c_void_p(stream),
                                       C.c_void_p(dev_dose), None if dev_mask is None else C.c_void_p(dev_mask)),
           ctx)


def pmc_delivery_simulate(ctx, d, spots: np.ndarray, n_fields: int) -> dict:
    """d: a workloads.Delivery; spots: SPOT_DTYPE array (weight = MU, field)
    in delivery order.  Returns {"mu": (n_trials, n_spots, N), "time":
    (n_trials, n_fields), "fills": (n_trials, n_fields)}."""
    sp = np.ascontiguousarray(spots)
    if sp.dtype != SPOT_DTYPE:
        raise ValueError("spots must use the pmc_spot layout")
    sync = pmc_synchrotron(*[pmc_param(*d.sync[f[0]]) for f in pmc_synchrotron._fields_])
    c = pmc_delivery(d.n_phases, d.start_phase, d.period_s, d.period_sd_s, d.period_min_s, d.period_max_s,
                     d.gate_lo, d.gate_hi, d.max_mu, sync, d.seed, d.n_trials)
    mu = np.zeros((d.n_trials, len(sp), d.n_phases), dtype=np.float64)
    t = np.zeros((d.n_trials, n_fields), dtype=np.float64)
    fills = np.zeros((d.n_trials, n_fields), dtype=np.int32)
    _check(lib().pmc_delivery_simulate(ctx, C.byref(c), _ptr(sp), len(sp), n_fields, _ptr(mu), _ptr(t),
                                       _ptr(fills)), ctx)
    return {"mu": mu, "time": t, "fills": fills}


def pmc_launch_shape(ctx, req: Request) -> dict:
    out = pmc_shape()
    _check(lib().pmc_launch_shape(ctx, C.byref(req.c), C.byref(out)), ctx)
    return {k: getattr(out, k) for k in ("block_size", "chunk", "refill_min", "tally_mode",
                                          "core_capacity")}


def pmc_trace(ctx, phase_id: int, spot: int, history: int, request_id=0, flags=0,
              max_rec=100_000, plan=0) -> np.ndarray:
    rec = np.zeros(max_rec, dtype=TRACE_DTYPE)
    n = C.c_int32(0)
    _check(lib().pmc_trace(ctx, plan, phase_id, spot, history, request_id, flags, _ptr(rec),
                           max_rec, C.byref(n)), ctx)
    if n.value > max_rec:
        raise ValueError(f"trace longer than {max_rec} records")
    return rec[: n.value].copy()


def pmc_split_histories(spots: np.ndarray, phases: Sequence[int], n_histories: int) -> np.ndarray:
    s = np.ascontiguousarray(spots, dtype=SPOT_DTYPE)
    ph = np.ascontiguousarray(phases, dtype=np.int32)
    out = np.zeros(len(s), dtype=np.int64)
    _check(lib().pmc_split_histories(_ptr(s), len(s), _ptr(ph), len(ph), n_histories, _ptr(out)))
    return out


def pmc_bytes_in_use(ctx) -> int:
    return int(lib().pmc_bytes_in_use(ctx))


def pmc_graph_create(ctx, req: Request, dev_tallies: Sequence[int], dev_counters: int,
                     dev_doses: Optional[Sequence[Optional[int]]] = None):
    tp = (C.c_void_p * req.n_phases)(*[int(p) for p in dev_tallies])
    dp = None
    if dev_doses is not None:
        dp = (C.c_void_p * req.n_phases)(*[None if p is None else int(p) for p in dev_doses])
    g = C.c_void_p()
    _check(lib().pmc_graph_create(ctx, C.byref(req.c), tp, C.c_void_p(dev_counters), dp,
                                  C.byref(g)), ctx)
    return g


def pmc_graph_launch(g, stream: int, ctx=None) -> None:
    _check(lib().pmc_graph_launch(g, C.c_void_p(stream)), ctx)


def pmc_graph_destroy(g) -> None:
    lib().pmc_graph_destroy(g)


def pmc_influence_boxes(ctx, plan: int, phase: int, n_spots: int) -> np.ndarray:
    out = np.zeros(n_spots, dtype=BOX_DTYPE)
    _check(lib().pmc_influence_boxes(ctx, plan, phase, _ptr(out), n_spots), ctx)
    return out


def pmc_influence(ctx, req: Request, boxes: Optional[np.ndarray], rel_threshold: float,
                  max_scratch_bytes: int = 0):
    """Compute the influence matrix (kept in the context); returns
    (nnz, balance dict, outside energy in 2^-32 MeV)."""
    b = None if boxes is None else np.ascontiguousarray(boxes, dtype=BOX_DTYPE)
    nnz = C.c_uint64(0)
    bal = pmc_balance()
    out = np.zeros(2, dtype=np.uint64)
    _check(lib().pmc_influence(ctx, C.byref(req.c), _ptr(b), float(rel_threshold),
                               int(max_scratch_bytes), C.byref(nnz), C.byref(bal), _ptr(out)), ctx)
    return int(nnz.value), bal.as_dict(), int(out[0]) + (int(out[1]) << 64)


def pmc_influence_read(ctx, n_spots: int, nnz: int):
    """(row_ptr int64[n_spots + 1], voxel int32[nnz], value float32[nnz])."""
    rows = np.zeros(n_spots + 1, dtype=np.int64)
    vox = np.zeros(nnz, dtype=np.int32)
    val = np.zeros(nnz, dtype=np.float32)
    _check(lib().pmc_influence_read(ctx, _ptr(rows), _ptr(vox), _ptr(val)), ctx)
    return rows, vox, val


def pmc_influence_device(ctx):
    r, v, x = C.c_void_p(), C.c_void_p(), C.c_void_p()
    _check(lib().pmc_influence_device(ctx, C.byref(r), C.byref(v), C.byref(x)), ctx)
    return r.value, v.value, x.value


def pmc_influence_free(ctx) -> None:
    _check(lib().pmc_influence_free(ctx), ctx)


# ----------------------------------------------------------------------------
# convenience wrapper
# ----------------------------------------------------------------------------

class Engine:
    """Owns a context; loads a Workload's phases and plan."""

    def __init__(self, device=0, precision=PMC_FP32, seed=0, hbm_budget_bytes=0):
        self.ctx = pmc_create(device, precision, seed, hbm_budget_bytes)
        self.nvox = {}

    def close(self):
        if self.ctx:
            pmc_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_phase(self, phase_id: int, ph):
        pmc_load_phase(self.ctx, phase_id, ph)
        self.nvox[phase_id] = ph.nvox

    def load_plan(self, plan):
        pmc_load_spots(self.ctx, plan.fields, plan.spots)

    def load_workload(self, wl):
        for i, ph in enumerate(wl.phases):
            self.load_phase(i, ph)
        self.load_plan(wl.plan)

    def dose(self, n_histories: int, phases: Sequence[int], request_id=0, flags=0,
             engine=PMC_ENGINE_PLAIN, want_density=False, **launch):
        req = Request(n_histories, phases, request_id, flags, engine, **launch)
        return pmc_dose(self.ctx, req, [self.nvox[p] for p in phases], want_density=want_density)

    def trace(self, phase_id, spot, history, request_id=0, flags=0, max_rec=100_000):
        return pmc_trace(self.ctx, phase_id, spot, history, request_id, flags, max_rec)
