"""Voxel box of a spot, for the per-spot influence matrix, plain numpy FP64.

TEST INFRASTRUCTURE ONLY (like the rest of `oracle/`): imported by tests and
by the benchmark's CPU-baseline leg, never by the product package.

The paper's robust optimiser (Sec. 4.C) needs the dose of every spot alone;
it gives no definition of where a spot's dose is kept.  The reading used
here (and documented with pmc_influence_boxes): the spot's central axis is
followed from where it first meets matter (a voxel whose stopping-power
ratio is at least 0.1; the air in front of the body is left out) to
water-equivalent depth R(E) + 3 cm, R the range table of the transport
(or to where the axis leaves the grid).  Across the beam the segment is
widened by 3 sigma_max, sigma_max^2 = sigma_spot^2 + (0.035 L)^2 with L the
geometric length of the segment: a point a u + b v of the disc of that
radius around the axis has |a u_k + b v_k| <= 3 sigma_max (|u_k| + |v_k|)
along axis k, so the box takes that half-width per axis.  Voxel index
ranges [floor(lo / d), floor(hi / d) + 1), clamped to the grid; a spot whose
axis misses the grid or meets no matter gets an empty box.

The axis is cut into voxel segments at every plane crossing of the ray
(all plane parameters sorted; each segment's voxel is that of its
midpoint), not by a voxel-stepping walk, so it shares no arithmetic with
the library's walk.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

BODY_RSP = 0.1        # a voxel with at least this stopping-power ratio is matter
MARGIN_CM = 3.0       # water-equivalent depth beyond the range
SPREAD = 0.035        # lateral spread per unit length of the segment
N_SIGMA = 3.0

BOX_DTYPE = np.dtype([("lo", "<i4", (3,)), ("hi", "<i4", (3,))])


def rsp_grid(phase) -> np.ndarray:
    """Stopping-power ratio per voxel, x fastest (nz, ny, nx): the
    calibration's piecewise-linear map at the integer HU clamped to
    [-1024, 3071], clamped to its end nodes; 0 outside the external mask."""
    hu = np.clip(phase.hu.astype(np.float64), -1024.0, 3071.0)
    r = np.interp(hu, np.asarray(phase.calib_hu, float), np.asarray(phase.calib_rsp, float))
    if phase.mask is not None:
        r = np.where(phase.mask != 0, r, 0.0)
    return r


def segments(c, w, d, n):
    """Voxel segments of the ray c + t w inside the grid box [0, n d):
    (t_a, t_b, (i, j, k)) in order of t, or [] if it misses."""
    t_in, t_out = -math.inf, math.inf
    for k in range(3):
        if w[k] != 0.0:
            t1, t2 = (0.0 - c[k]) / w[k], (n[k] * d[k] - c[k]) / w[k]
            t_in, t_out = max(t_in, min(t1, t2)), min(t_out, max(t1, t2))
        elif not (0.0 <= c[k] < n[k] * d[k]):
            return []
    if not t_in < t_out:
        return []
    ts = [t_in, t_out]
    for k in range(3):
        if w[k] != 0.0:
            for j in range(n[k] + 1):
                t = (j * d[k] - c[k]) / w[k]
                if t_in < t < t_out:
                    ts.append(t)
    ts = sorted(set(ts))
    out = []
    for ta, tb in zip(ts[:-1], ts[1:]):
        tm = 0.5 * (ta + tb)
        ijk = tuple(min(n[k] - 1, max(0, int(math.floor((c[k] + tm * w[k]) / d[k])))) for k in range(3))
        out.append((ta, tb, ijk))
    return out


def spot_box(phase, rsp, field, spot):
    """(lo[3], hi[3], lo_real[3], hi_real[3]) of one spot; the real-valued
    bounds are lo / d and hi / d before the floor (to tell a tie)."""
    nx, ny, nz = phase.hu.shape[2], phase.hu.shape[1], phase.hu.shape[0]
    n = (nx, ny, nz)
    d = tuple(0.1 * float(x) for x in phase.spacing_mm)
    w = np.asarray(field["direction"], float)
    w = w / math.sqrt(float(w @ w))
    u = np.asarray(field["bev_u"], float)
    u = u / math.sqrt(float(u @ u))
    v = np.array([w[1] * u[2] - w[2] * u[1], w[2] * u[0] - w[0] * u[2], w[0] * u[1] - w[1] * u[0]])
    iso = np.asarray(field["isocentre_mm"], float)
    org = np.asarray(phase.origin_mm, float)
    c = 0.1 * (iso - org) + 0.1 * float(spot["x_mm"]) * u + 0.1 * float(spot["y_mm"]) * v
    empty = ((0, 0, 0), (0, 0, 0), None, None)
    segs = segments(c, w, d, n)
    if not segs:
        return empty
    target = oracle.f64("orc_range", float(spot["energy_MeV"])) + MARGIN_CM
    wet, t_body, t_end = 0.0, None, segs[-1][1]
    for ta, tb, (i, j, k) in segs:
        r = float(rsp[k, j, i])
        if t_body is None and r >= BODY_RSP:
            t_body = ta
        if r > 0.0 and wet + r * (tb - ta) >= target:
            t_end = ta + (target - wet) / r
            break
        wet += r * (tb - ta)
    if t_body is None:
        return empty
    L = t_end - t_body
    sig = 0.1 * float(spot["sigma_mm"])
    half_r = N_SIGMA * math.sqrt(sig * sig + (SPREAD * L) ** 2)
    lo, hi, lo_r, hi_r = [], [], [], []
    for k in range(3):
        a, e = c[k] + t_body * w[k], c[k] + t_end * w[k]
        half = half_r * (abs(u[k]) + abs(v[k]))
        xl, xh = (min(a, e) - half) / d[k], (max(a, e) + half) / d[k]
        lo_r.append(xl)
        hi_r.append(xh)
        lo.append(min(n[k], max(0, math.floor(xl))))
        hi.append(min(n[k], max(0, math.floor(xh) + 1)))
    if any(h <= l for l, h in zip(lo, hi)):
        return empty
    return tuple(lo), tuple(hi), lo_r, hi_r


def spot_boxes(phase, plan, phase_id=0):
    """Boxes of every spot of the plan on `phase` (plan phase id phase_id;
    spots of other phases get empty boxes) as BOX_DTYPE, plus the real
    bounds per spot (None for an empty box)."""
    rsp = rsp_grid(phase)
    out = np.zeros(len(plan.spots), dtype=BOX_DTYPE)
    real = []
    for s, sp in enumerate(plan.spots):
        if int(sp["phase"]) != phase_id:
            real.append(None)
            continue
        lo, hi, lr, hr = spot_box(phase, rsp, plan.fields[int(sp["field"])], sp)
        out[s]["lo"] = lo
        out[s]["hi"] = hi
        real.append(None if lr is None else (lr, hr))
    return out, real
