"""ctypes wrapper of the FP64 oracle (liboracle.so, built from pmc_oracle.c).

TEST INFRASTRUCTURE ONLY.  Imported by tests, by the smoke check and by the
benchmark's CPU-baseline leg; the product package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NO_STRAGGLING, NO_MCS, NO_DELTA, NO_NUCLEAR, FROZEN = 1, 2, 4, 8, 16
CAUSE_STOP, CAUSE_GEO, CAUSE_DELTA, CAUSE_NUCLEAR, CAUSE_PHYS = 0, 1, 2, 3, 4
FATE_ALIVE, FATE_STOPPED, FATE_ESCAPED, FATE_NUCLEAR, FATE_MISSED = 0, 1, 2, 3, 4
Q_SCALE = 2.0 ** 32


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C11, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
               "-o", _LIB, _SRC, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
    return _LIB


class Phase(C.Structure):
    _fields_ = [
        ("hu", C.c_void_p), ("mask", C.c_void_p),
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("spacing_mm", C.c_double * 3), ("origin_mm", C.c_double * 3),
        ("calib_hu", C.c_void_p), ("calib_rho", C.c_void_p), ("calib_rsp", C.c_void_p),
        ("n_nodes", C.c_int32),
    ]


class Balance(C.Structure):
    _fields_ = [
        ("incident", C.c_uint64 * 2), ("deposited", C.c_uint64 * 2), ("escaped", C.c_uint64 * 2),
        ("nuclear", C.c_uint64 * 2), ("cutoff", C.c_uint64 * 2),
        ("histories", C.c_uint64), ("steps", C.c_uint64), ("delta_events", C.c_uint64),
        ("nuclear_events", C.c_uint64), ("escapes", C.c_uint64), ("misses", C.c_uint64),
    ]

    def as_dict(self):
        def w(x):
            return int(x[0]) + (int(x[1]) << 64)
        return {
            "incident": w(self.incident), "deposited": w(self.deposited), "escaped": w(self.escaped),
            "nuclear": w(self.nuclear), "cutoff": w(self.cutoff), "histories": int(self.histories),
            "steps": int(self.steps), "delta_events": int(self.delta_events),
            "nuclear_events": int(self.nuclear_events), "escapes": int(self.escapes),
            "misses": int(self.misses),
        }


TRACE_DTYPE = np.dtype([
    ("cause", "<i4"), ("voxel", "<i4"), ("fate", "<i4"), ("block", "<u4"),
    ("s", "<f8"), ("E", "<f8"), ("r", "<f8", 3), ("w", "<f8", 3),
    ("n_delta", "<f8"), ("n_nuc", "<f8"), ("l_acc", "<f8"), ("dep", "<i8"), ("t_delta", "<f8"),
    ("margin", "<f8"),
])


class Tables(C.Structure):
    _fields_ = [("e", C.c_double * 1024), ("R", C.c_double * 1024),
                ("mu_delta", C.c_double * 1024), ("omega2", C.c_double * 1024),
                ("lnE0", C.c_double), ("dlnE", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        d = C.c_double
        for name in ("orc_stopping_unrestricted", "orc_stopping_restricted", "orc_mu_delta",
                     "orc_omega2", "orc_range", "orc_range_inverse"):
            getattr(L, name).restype = d
            getattr(L, name).argtypes = [d]
        L.orc_highland_theta2.restype = d
        L.orc_highland_theta2.argtypes = [d, d]
        L.orc_interp.restype = d
        L.orc_interp.argtypes = [C.c_void_p, d]
        L.orc_build_tables.argtypes = [C.c_void_p]
        L.orc_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_sample_delta.restype = C.c_int
        L.orc_sample_delta.argtypes = [d, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                       C.c_int32, C.c_void_p]
        L.orc_split_histories.restype = C.c_int
        L.orc_split_histories.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32,
                                          C.c_uint64, C.c_void_p]
        L.orc_dose.restype = C.c_int
        L.orc_dose.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_int64,
                               C.c_void_p, C.c_int32, C.c_uint64, C.c_uint32, C.c_uint64,
                               C.c_uint32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_dose_subset.restype = C.c_int
        L.orc_dose_subset.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                      C.c_int64, C.c_void_p, C.c_int32, C.c_uint64, C.c_uint32,
                                      C.c_uint64, C.c_uint32, C.c_int32, C.c_uint32, C.c_uint32,
                                      C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p]
        L.orc_dose_spots.restype = C.c_int
        L.orc_dose_spots.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                     C.c_int64, C.c_void_p, C.c_int32, C.c_uint64, C.c_uint32,
                                     C.c_uint64, C.c_uint32, C.c_int32, C.c_int64, C.c_int64,
                                     C.c_void_p, C.c_void_p]
        L.orc_dose_spots_batch.restype = C.c_int
        L.orc_dose_spots_batch.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                           C.c_int64, C.c_void_p, C.c_int32, C.c_uint64, C.c_uint32,
                                           C.c_uint64, C.c_uint32, C.c_int32, C.c_int64, C.c_int64,
                                           C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p]
        L.orc_trace.restype = C.c_int
        L.orc_trace.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int64,
                                C.c_int64, C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint32,
                                C.c_void_p, C.c_int32]
        L.orc_convert.restype = C.c_int
        L.orc_convert.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


# ----------------------------------------------------------------------------
# marshalling helpers
# ----------------------------------------------------------------------------

class _PhaseHolder:
    """Keeps the numpy buffers alive for the lifetime of the C struct."""

    def __init__(self, ph):
        self.hu = np.ascontiguousarray(ph.hu, dtype=np.int16)
        self.mask = None if ph.mask is None else np.ascontiguousarray(ph.mask, dtype=np.uint8)
        self.ch = np.ascontiguousarray(ph.calib_hu, dtype=np.float64)
        self.cr = np.ascontiguousarray(ph.calib_rho, dtype=np.float64)
        self.cs = np.ascontiguousarray(ph.calib_rsp, dtype=np.float64)
        nz, ny, nx = self.hu.shape
        self.s = Phase()
        self.s.hu = self.hu.ctypes.data
        self.s.mask = None if self.mask is None else self.mask.ctypes.data
        self.s.nx, self.s.ny, self.s.nz = nx, ny, nz
        self.s.spacing_mm[:] = list(ph.spacing_mm)
        self.s.origin_mm[:] = list(ph.origin_mm)
        self.s.calib_hu = self.ch.ctypes.data
        self.s.calib_rho = self.cr.ctypes.data
        self.s.calib_rsp = self.cs.ctypes.data
        self.s.n_nodes = len(self.ch)


def _phase_array(phases):
    holders = [_PhaseHolder(p) for p in phases]
    arr = (Phase * len(phases))(*[h.s for h in holders])
    return holders, arr


def tables() -> Tables:
    t = Tables()
    lib().orc_build_tables(C.byref(t))
    return t


def philox(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def split_histories(spots: np.ndarray, phase_ids: Sequence[int], n_hist: int) -> np.ndarray:
    ids = np.asarray(phase_ids, dtype=np.int32)
    out = np.zeros(len(spots), dtype=np.int64)
    rc = lib().orc_split_histories(spots.ctypes.data, len(spots), ids.ctypes.data, len(ids),
                                   int(n_hist), out.ctypes.data)
    if rc:
        raise ValueError(f"orc_split_histories failed: {rc}")
    return out


def dose(phases, plan, n_hist: int, seed: int, request_id: int = 0, phase_ids=None,
         flags: int = 0, n_threads: Optional[int] = None, with_dose: bool = True):
    """Run the oracle.  Returns (tallies[list], doses[list or None], balance dict)."""
    if phase_ids is None:
        phase_ids = list(range(len(phases)))
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    holders, parr = _phase_array(phases)
    ids = np.asarray(phase_ids, dtype=np.int32)
    tallies = [np.zeros(phases[i].hu.size, dtype=np.int64) for i in phase_ids]
    doses = [np.zeros(phases[i].hu.size, dtype=np.float64) for i in phase_ids] if with_dose else None
    tp = (C.c_void_p * len(ids))(*[t.ctypes.data for t in tallies])
    dp = (C.c_void_p * len(ids))(*[d.ctypes.data for d in doses]) if with_dose else None
    bal = Balance()
    spots = np.ascontiguousarray(plan.spots)
    fields = np.ascontiguousarray(plan.fields)
    rc = lib().orc_dose(parr, len(phases), fields.ctypes.data, len(fields), spots.ctypes.data,
                        len(spots), ids.ctypes.data, len(ids), int(seed), int(request_id),
                        int(n_hist), int(flags), int(n_threads), tp, dp, C.byref(bal))
    if rc:
        raise ValueError(f"orc_dose failed: {rc}")
    del holders
    return tallies, doses, bal.as_dict()


def dose_subset(phases, plan, n_hist: int, seed: int, h_begin: int, h_end: int, request_id=0,
                phase_ids=None, flags=0, n_threads=None, h_mod=1, h_rem=0):
    """Tallies of only the histories h (index within each spot's share) with
    h_begin <= h < h_end and h % h_mod == h_rem."""
    if phase_ids is None:
        phase_ids = list(range(len(phases)))
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    holders, parr = _phase_array(phases)
    ids = np.asarray(phase_ids, dtype=np.int32)
    tallies = [np.zeros(phases[i].hu.size, dtype=np.int64) for i in phase_ids]
    tp = (C.c_void_p * len(ids))(*[t.ctypes.data for t in tallies])
    bal = Balance()
    spots = np.ascontiguousarray(plan.spots)
    fields = np.ascontiguousarray(plan.fields)
    rc = lib().orc_dose_subset(parr, len(phases), fields.ctypes.data, len(fields),
                               spots.ctypes.data, len(spots), ids.ctypes.data, len(ids), int(seed),
                               int(request_id), int(n_hist), int(flags), int(n_threads),
                               int(h_begin), int(h_end), int(h_mod), int(h_rem), tp,
                               C.byref(bal))
    if rc:
        raise ValueError(f"orc_dose_subset failed: {rc}")
    del holders
    return tallies, bal.as_dict()


def dose_batches(phases, plan, n_hist: int, seed: int, n_batches=10, request_id=0, phase_ids=None,
                 flags=0, n_threads=None):
    """Per-batch tallies, batch = history index mod n_batches; their sum is
    the full run and their spread gives the per-voxel statistical error."""
    out = []
    for b in range(n_batches):
        t, _ = dose_subset(phases, plan, n_hist, seed, 0, 2**32 - 1, request_id, phase_ids, flags,
                           n_threads, h_mod=n_batches, h_rem=b)
        out.append(t)
    return out


def dose_spots(phases, plan, n_hist: int, seed: int, s_begin: int, s_end: int, request_id=0,
               phase_ids=None, flags=0, n_threads=None, h_mod: int = 1, h_rem: int = 0):
    """Tallies of only the histories of spots s_begin <= s < s_end (history
    split of the whole request); with h_mod > 1 only the histories h of
    those spots with h % h_mod == h_rem."""
    if phase_ids is None:
        phase_ids = list(range(len(phases)))
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    holders, parr = _phase_array(phases)
    ids = np.asarray(phase_ids, dtype=np.int32)
    tallies = [np.zeros(phases[i].hu.size, dtype=np.int64) for i in phase_ids]
    tp = (C.c_void_p * len(ids))(*[t.ctypes.data for t in tallies])
    bal = Balance()
    spots = np.ascontiguousarray(plan.spots)
    fields = np.ascontiguousarray(plan.fields)
    rc = lib().orc_dose_spots_batch(parr, len(phases), fields.ctypes.data, len(fields), spots.ctypes.data,
                                    len(spots), ids.ctypes.data, len(ids), int(seed), int(request_id),
                                    int(n_hist), int(flags), int(n_threads), int(s_begin), int(s_end),
                                    int(h_mod), int(h_rem), tp, C.byref(bal))
    if rc:
        raise ValueError(f"orc_dose_spots_batch failed: {rc}")
    del holders
    return tallies, bal.as_dict()


MEV_TO_J = 1.602176634e-13


def influence(phase, plan, n_hist: int, seed: int, boxes, rel_threshold: float, request_id=0,
              flags=0, n_threads=None):
    """Per-spot influence matrix, from its definition: for every spot, the
    tally of that spot's histories alone (same history split and random
    numbers as the whole request), restricted to the spot's voxel box; keep
    the voxels whose tally / density is at least rel_threshold times the
    spot's maximum of it; value = energy / (density x voxel volume) / the
    spot's histories, rounded to float32.  The per-spot dose is what an
    optimiser of spot weights needs (Sec. 1 and Sec. 4.C of the paper).

    boxes: structured array with int32 fields lo[3], hi[3] (voxel index
    ranges [lo, hi) along x, y, z), one per spot.  The plan's spots must all
    be on `phase` (phase index 0).  Returns a dict with row_ptr, voxel,
    value, box_deposited, outside (2^-32 MeV) and the summed balance."""
    per_spot = split_histories(plan.spots, [0], n_hist)
    _, rho = convert(phase, np.zeros(phase.hu.size, dtype=np.int64), 1)
    nx, ny, nz = phase.hu.shape[2], phase.hu.shape[1], phase.hu.shape[0]
    vol = (phase.spacing_mm[0] * 0.1) * (phase.spacing_mm[1] * 0.1) * (phase.spacing_mm[2] * 0.1)
    rows = [0]
    vox, val = [], []
    box_dep, outside = 0, 0
    bal_sum = None
    for s in range(len(plan.spots)):
        if per_spot[s] == 0:
            rows.append(rows[-1])
            continue
        (t,), bal = dose_spots([phase], plan, n_hist, seed, s, s + 1, request_id, [0], flags,
                               n_threads)
        bal_sum = bal if bal_sum is None else {k: bal_sum[k] + bal[k] for k in bal}
        t3 = t.reshape(nz, ny, nx)
        lo, hi = boxes[s]["lo"], boxes[s]["hi"]
        inside = np.zeros_like(t3, dtype=bool)
        inside[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = True
        total = int(np.sum(t, dtype=np.int64))
        t_in = np.where(inside, t3, 0).reshape(-1)
        kept_energy = int(np.sum(t_in, dtype=np.int64))
        box_dep += kept_energy
        outside += total - kept_energy
        ok = (t_in > 0) & (rho > 0)
        score = np.zeros(t_in.size, dtype=np.float64)
        score[ok] = t_in[ok].astype(np.float64) / rho[ok]
        m = score.max() if ok.any() else 0.0
        keep = ok & (score >= rel_threshold * m)
        idx = np.nonzero(keep)[0]  # ascending voxel index
        e_j = t_in[idx].astype(np.float64) / Q_SCALE * MEV_TO_J
        m_kg = rho[idx] * vol * 1e-3
        vox.append(idx.astype(np.int32))
        val.append((e_j / m_kg / float(per_spot[s])).astype(np.float32))
        rows.append(rows[-1] + len(idx))
    return {"row_ptr": np.array(rows, dtype=np.int64),
            "voxel": np.concatenate(vox) if vox else np.zeros(0, np.int32),
            "value": np.concatenate(val) if val else np.zeros(0, np.float32),
            "box_deposited": box_dep, "outside": outside, "balance": bal_sum, "per_spot": per_spot}


def trace(phase, plan, spot: int, h: int, seed: int, request_id: int = 0, flags: int = 0,
          max_rec: int = 100_000) -> np.ndarray:
    holders, parr = _phase_array([phase])
    rec = np.zeros(max_rec, dtype=TRACE_DTYPE)
    spots = np.ascontiguousarray(plan.spots)
    fields = np.ascontiguousarray(plan.fields)
    n = lib().orc_trace(parr, fields.ctypes.data, len(fields), spots.ctypes.data, len(spots),
                        int(spot), int(h), int(seed), int(request_id), int(flags),
                        rec.ctypes.data, max_rec)
    if n < 0:
        raise ValueError(f"orc_trace failed: {n}")
    if n > max_rec:
        raise ValueError(f"trace longer than {max_rec} records")
    del holders
    return rec[:n].copy()


def convert(phase, tally: np.ndarray, n_hist: int):
    holders, parr = _phase_array([phase])
    d = np.zeros(phase.hu.size, dtype=np.float64)
    rho = np.zeros(phase.hu.size, dtype=np.float64)
    t = np.ascontiguousarray(tally, dtype=np.int64)
    rc = lib().orc_convert(parr, t.ctypes.data, int(n_hist), d.ctypes.data, rho.ctypes.data)
    if rc:
        raise ValueError("orc_convert failed")
    del holders
    return d, rho


def sample_delta(E: float, n: int, seed=7, request_id=0, h=0, s=0) -> np.ndarray:
    out = np.zeros(n, dtype=np.float64)
    rc = lib().orc_sample_delta(float(E), seed, request_id, h, s, n, out.ctypes.data)
    if rc:
        raise ValueError("no delta production at this energy")
    return out


def f64(name: str, *args) -> float:
    return float(getattr(lib(), name)(*args))
