"""Deformable dose accumulation by energy/mass transfer, plain numpy in FP64.

TEST INFRASTRUCTURE ONLY (like the rest of `oracle/`): imported by tests and
by the benchmark's CPU-baseline leg, never by the product package.

Follows Sec. 2.D.2 (Eqs. (2), (4)-(6)) and App. B (Eqs. (7)-(8)) of the
paper; the readings where it is silent are the ones of the library's
documentation of pmc_accumulate (integer accumulators, points outside a DVF
grid, the report mask).

* DVF (App. B): grid point (i, j, k) sits at x0 = start + i dX U + j dY V +
  k dZ W with W = U x V (Eq. (8)) and maps to M_post (M_pre x0 + delta)
  (Eq. (7); the rigid matrices are the identity between 4DCT phases, None
  here).  A point r between grid points maps to M_post (M_pre r + delta(r)),
  delta(r) the trilinear interpolation of the translations of the grid points
  around it (with identity matrices: r plus that interpolation).  Points
  outside the box of grid-point centres are not mapped.
* EMTM (Eqs. (4)-(6)): every voxel j of a source phase is split into n^3
  subvoxels of volume v = V/n^3; subvoxel k carries mass M = rho_j v and
  energy E = M D_j, which for the Monte Carlo dose D_j = E_j / (rho_j V) is
  E_j / n^3.  Each subvoxel centre is mapped to the reference phase; the
  energy and mass of all subvoxels mapped into reference voxel i are summed
  and D_i^S = sum E / sum M.  Sums are kept as exact integers: energy in the
  tally's units (2^-32 MeV) as two halves (sum of tally >> 32, sum of tally &
  (2^32 - 1)), mass as the sum of round-half-even(rho 2^32), each counted
  once per subvoxel; the common factor 1/n^3 cancels in the ratio.
* Eq. (2): D_i = D_i^R (the reference phase's own dose) + sum over sources of
  D_i^S, in source order; reported where the reference voxel centre lies in
  the grid box of every DVF used (else 0).
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence

import numpy as np

MEV_TO_J = 1.602176634e-13


def dvf_axes(dvf):
    """Unit row, column and depth directions (Eq. (8): W = U x V)."""
    u = np.asarray(dvf.row, dtype=np.float64)
    v = np.asarray(dvf.col, dtype=np.float64)
    w = np.array([u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]])
    return u, v, w


def affine(m, pts: np.ndarray) -> np.ndarray:
    """A 4x4 rigid matrix applied to points (..., 3): output axis a is
    m[a,0] x + m[a,1] y + m[a,2] z + m[a,3], summed in that order."""
    m = np.asarray(m, dtype=np.float64)
    out = np.empty_like(pts)
    for a in range(3):
        out[..., a] = m[a, 0] * pts[..., 0] + m[a, 1] * pts[..., 1] + m[a, 2] * pts[..., 2] + m[a, 3]
    return out


def dvf_points(dvf):
    """Eqs. (8) and (7) at every grid point: x0 (the matrix product written
    out per axis: (U_a dX) i + (V_a dY) j + (W_a dZ) k + start_a) and
    r_f = M_post (M_pre x0 + delta); both (n[2], n[1], n[0], 3)."""
    u, v, w = dvf_axes(dvf)
    n = dvf.n
    k, j, i = np.meshgrid(np.arange(n[2], dtype=np.float64), np.arange(n[1], dtype=np.float64),
                          np.arange(n[0], dtype=np.float64), indexing="ij")
    x0 = np.empty(k.shape + (3,))
    for a in range(3):
        x0[..., a] = ((u[a] * dvf.spacing_mm[0]) * i + (v[a] * dvf.spacing_mm[1]) * j
                      + (w[a] * dvf.spacing_mm[2]) * k + dvf.start_mm[a])
    m = x0 if dvf.pre is None else affine(dvf.pre, x0)
    rf = m + np.asarray(dvf.delta_mm, dtype=np.float64)
    if dvf.post is not None:
        rf = affine(dvf.post, rf)
    return x0, rf


def dvf_grid_coords(dvf, pts: np.ndarray) -> np.ndarray:
    """Grid coordinates (i, j, k) of points (mm): projections of r - start
    on U, V, W divided by the grid spacings (the inverse of Eq. (8))."""
    u, v, w = dvf_axes(dvf)
    rel = pts - np.asarray(dvf.start_mm, dtype=np.float64)
    out = np.empty_like(rel)
    for a, ax in enumerate((u, v, w)):
        out[..., a] = (rel[..., 0] * ax[0] + rel[..., 1] * ax[1] + rel[..., 2] * ax[2]) / dvf.spacing_mm[a]
    return out


def dvf_inside(dvf, pts: np.ndarray) -> np.ndarray:
    """Is each point inside the box of grid-point centres?"""
    g = dvf_grid_coords(dvf, pts)
    ok = np.ones(pts.shape[:-1], dtype=bool)
    for a in range(3):
        ok &= (g[..., a] >= 0.0) & (g[..., a] <= dvf.n[a] - 1)
    return ok


def dvf_map(dvf, pts: np.ndarray) -> np.ndarray:
    """T(r) of Eq. (1) for points pts (..., 3) in mm; NaN where r is outside
    the grid.  Trilinear interpolation of the translations, x first, then y,
    then z; then the rigid matrices of Eq. (7), if any."""
    g = dvf_grid_coords(dvf, pts)
    inside = dvf_inside(dvf, pts)
    out = np.full(pts.shape, np.nan)
    if not inside.any():
        return out
    gi = g[inside]
    p = pts[inside]
    i0 = np.empty(gi.shape, dtype=np.int64)
    f = np.empty(gi.shape)
    for a in range(3):
        base = np.floor(gi[:, a]).astype(np.int64)
        base = np.minimum(base, dvf.n[a] - 2)  # a point on the last plane uses the last cell
        i0[:, a] = base
        f[:, a] = gi[:, a] - base
    d = dvf.delta_mm  # (nz, ny, nx, 3) with nx = n[0]

    def corner(di, dj, dk):
        return d[i0[:, 2] + dk, i0[:, 1] + dj, i0[:, 0] + di]

    fx, fy, fz = f[:, 0:1], f[:, 1:2], f[:, 2:3]
    c00 = corner(0, 0, 0) + fx * (corner(1, 0, 0) - corner(0, 0, 0))
    c10 = corner(0, 1, 0) + fx * (corner(1, 1, 0) - corner(0, 1, 0))
    c01 = corner(0, 0, 1) + fx * (corner(1, 0, 1) - corner(0, 0, 1))
    c11 = corner(0, 1, 1) + fx * (corner(1, 1, 1) - corner(0, 1, 1))
    c0 = c00 + fy * (c10 - c00)
    c1 = c01 + fy * (c11 - c01)
    base = p if getattr(dvf, "pre", None) is None else affine(dvf.pre, p)
    q = base + (c0 + fz * (c1 - c0))
    if getattr(dvf, "post", None) is not None:
        q = affine(dvf.post, q)
    out[inside] = q
    return out


def voxel_centres(ph) -> np.ndarray:
    """Centres (mm) of a phase's voxels, (nz, ny, nx, 3)."""
    nz, ny, nx = ph.hu.shape
    o, s = ph.origin_mm, ph.spacing_mm
    x = o[0] + (np.arange(nx) + 0.5) * s[0]
    y = o[1] + (np.arange(ny) + 0.5) * s[1]
    z = o[2] + (np.arange(nz) + 0.5) * s[2]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def mass_units(rho: np.ndarray) -> np.ndarray:
    """round-half-even(rho 2^32) as int64 (the mass accumulator's unit)."""
    return np.rint(np.asarray(rho, dtype=np.float64) * 4294967296.0).astype(np.int64)


def push(src, tally: np.ndarray, rho: np.ndarray, ref, dvf, n: int) -> Dict[str, np.ndarray]:
    """Eqs. (4)-(6) for one source phase: integer energy (hi, lo halves) and
    mass sums per reference voxel of the subvoxels mapped into it."""
    nz, ny, nx = src.hu.shape
    rz, ry, rx = ref.hu.shape
    t = np.asarray(tally, dtype=np.int64).reshape(nz, ny, nx)
    rq = mass_units(rho).reshape(nz, ny, nx)
    has_mass = rq > 0
    zz, yy, xx = np.nonzero(has_mass)
    t_hi = (t[zz, yy, xx] >> 32)
    t_lo = (t[zz, yy, xx] & 0xFFFFFFFF)
    m = rq[zz, yy, xx]
    acc = {k: np.zeros(rz * ry * rx, dtype=np.int64) for k in ("e_hi", "e_lo", "mass")}
    o, s = np.asarray(src.origin_mm), np.asarray(src.spacing_mm)
    ro, rs = np.asarray(ref.origin_mm), np.asarray(ref.spacing_mm)
    idx = np.stack([xx, yy, zz], axis=-1).astype(np.float64)
    for c in range(n):
        for b in range(n):
            for a in range(n):
                sub = np.array([(a + 0.5) / n, (b + 0.5) / n, (c + 0.5) / n])
                r = o + (idx + sub) * s
                q = dvf_map(dvf, r)
                ok = ~np.isnan(q[:, 0])
                tgt = np.floor((q[ok] - ro) / rs).astype(np.int64)
                ok2 = np.all((tgt >= 0) & (tgt < np.array([rx, ry, rz])), axis=1)
                tgt = tgt[ok2]
                lin = tgt[:, 0] + rx * (tgt[:, 1] + ry * tgt[:, 2])
                sel = np.nonzero(ok)[0][ok2]
                np.add.at(acc["e_hi"], lin, t_hi[sel])
                np.add.at(acc["e_lo"], lin, t_lo[sel])
                np.add.at(acc["mass"], lin, m[sel])
    return acc


def phase_dose(tally: np.ndarray, rho: np.ndarray, voxel_cm3: float, n_hist: int) -> np.ndarray:
    """The reference phase's own dose, Eq. (4) with E = the tally: D = E / (rho V)."""
    t = np.asarray(tally, dtype=np.float64)
    out = np.zeros_like(t)
    ok = rho > 0
    out[ok] = t[ok] / 4294967296.0 * MEV_TO_J / (rho[ok] * voxel_cm3 * 1e-3) / n_hist
    return out


def dose_from_sums(acc: Dict[str, np.ndarray], voxel_cm3: float, n_hist: int) -> np.ndarray:
    """Eq. (5): D = sum E / sum M, in Gy per history; 0 where no mass arrived."""
    e = acc["e_hi"].astype(np.float64) * 4294967296.0 + acc["e_lo"].astype(np.float64)
    m = acc["mass"].astype(np.float64)
    out = np.zeros_like(e)
    ok = acc["mass"] > 0
    out[ok] = (e[ok] * MEV_TO_J) / (m[ok] * voxel_cm3 * 1e-3 * n_hist)
    return out


def report_mask(ref, dvfs: Sequence) -> np.ndarray:
    """Reference voxels whose centre lies in the grid box of every DVF."""
    c = voxel_centres(ref).reshape(-1, 3)
    ok = np.ones(c.shape[0], dtype=bool)
    for d in dvfs:
        ok &= dvf_inside(d, c)
    return ok


def emtm(phases: Sequence, tallies: Sequence[np.ndarray], densities: Sequence[np.ndarray],
         ref_index: int, dvfs: Sequence[Optional[object]], n: int, n_hist: int) -> Dict[str, np.ndarray]:
    """Accumulated dose on phase ref_index (Eq. (2)) from the per-phase
    tallies (2^-32 MeV) and densities of a run of n_hist histories; dvfs[s]
    maps phase s to the reference (ignored for the reference itself)."""
    ref = phases[ref_index]
    used = [dvfs[s] for s in range(len(phases)) if s != ref_index]
    mask = report_mask(ref, used)
    v_ref = float(np.prod(np.asarray(ref.spacing_mm) * 0.1))
    dose = phase_dose(tallies[ref_index], np.asarray(densities[ref_index]), v_ref, n_hist)
    sums = {}
    for s in range(len(phases)):
        if s == ref_index:
            continue
        acc = push(phases[s], tallies[s], densities[s], ref, dvfs[s], n)
        sums[s] = acc
        v_s = float(np.prod(np.asarray(phases[s].spacing_mm) * 0.1))
        dose = dose + dose_from_sums(acc, v_s, n_hist)
    dose = np.where(mask, dose, 0.0)
    return {"dose": dose, "mask": mask, "sums": sums}
