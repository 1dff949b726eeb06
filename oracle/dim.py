"""Deformable accumulation by dose interpolation (DIM), plain numpy in FP64.

TEST INFRASTRUCTURE ONLY (like the rest of `oracle/`): imported by tests and
by the benchmark's CPU-baseline leg, never by the product package.

Follows Sec. 2.D.2, Eqs. (2) and (3), with the DVFs of App. B (the mapping
of `oracle.emtm`, here from the reference phase to each source phase); the
readings where the paper is silent are those of the library's documentation
of pmc_accumulate_dim:

* every reference voxel is split into n^3 subvoxels with centres at
  origin + (i + (s + 1/2) / n) spacing per axis;
* each centre is mapped to the source phase, T^{R->S}(r); a centre outside
  the DVF grid box contributes 0;
* the source dose there is the trilinear interpolation of the source phase's
  voxel doses at their voxel centres (x, then y, then z), with the position
  clamped to the box of voxel centres (a 3D texture's clamp-to-edge);
* D^S_i = (sum over the subvoxels, x outermost, then y, then z) / n^3;
* Eq. (2): D_i = D^R_i + sum over sources in source order; reported where the
  reference voxel centre lies in the grid box of every DVF (else 0).
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import numpy as np

from oracle.emtm import dvf_map, report_mask


def dose_sample(dose: np.ndarray, ph, pts: np.ndarray) -> np.ndarray:
    """Trilinear interpolation of a phase's voxel doses (flat, x fastest) at
    points (..., 3) in mm: voxel-centre coordinates u = (p - origin) /
    spacing - 1/2 clamped to [0, n - 1], corners floor(u) and the next one
    (the same one on the last plane), fraction u - floor(u)."""
    nz, ny, nx = ph.hu.shape
    d = np.asarray(dose, dtype=np.float64).reshape(nz, ny, nx)
    dims = (nx, ny, nz)
    lo = []
    hi = []
    fr = []
    for a in range(3):
        u = (pts[..., a] - ph.origin_mm[a]) / ph.spacing_mm[a] - 0.5
        u = np.minimum(np.maximum(u, 0.0), float(dims[a] - 1))
        i0 = np.floor(u).astype(np.int64)
        lo.append(i0)
        hi.append(np.minimum(i0 + 1, dims[a] - 1))
        fr.append(u - i0)
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    fx, fy, fz = fr
    c00 = d[z0, y0, x0] + fx * (d[z0, y0, x1] - d[z0, y0, x0])
    c10 = d[z0, y1, x0] + fx * (d[z0, y1, x1] - d[z0, y1, x0])
    c01 = d[z1, y0, x0] + fx * (d[z1, y0, x1] - d[z1, y0, x0])
    c11 = d[z1, y1, x0] + fx * (d[z1, y1, x1] - d[z1, y1, x0])
    c0 = c00 + fy * (c10 - c00)
    c1 = c01 + fy * (c11 - c01)
    return c0 + fz * (c1 - c0)


def pull(ref, src, dose_src: np.ndarray, dvf, n: int, voxels: Optional[np.ndarray] = None) -> np.ndarray:
    """Eq. (3): D^S on the reference grid (flat, x fastest) from the source
    phase's dose through the reference-to-source DVF; with `voxels` (flat
    indices) only those reference voxels, in that order."""
    nz, ny, nx = ref.hu.shape
    if voxels is None:
        zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        idx = np.stack([xx, yy, zz], axis=-1).reshape(-1, 3).astype(np.float64)
    else:
        v = np.asarray(voxels, dtype=np.int64)
        idx = np.stack([v % nx, (v // nx) % ny, v // (nx * ny)], axis=-1).astype(np.float64)
    o, s = np.asarray(ref.origin_mm, dtype=np.float64), np.asarray(ref.spacing_mm, dtype=np.float64)
    acc = np.zeros(idx.shape[0])
    for a in range(n):
        for b in range(n):
            for c in range(n):
                sub = np.array([(a + 0.5) / n, (b + 0.5) / n, (c + 0.5) / n])
                r = o + (idx + sub) * s
                q = dvf_map(dvf, r)
                ok = ~np.isnan(q[:, 0])
                val = np.zeros(idx.shape[0])
                val[ok] = dose_sample(dose_src, src, q[ok])
                acc = acc + val
    return acc / float(n * n * n)


def dim(phases: Sequence, doses: Sequence[np.ndarray], ref_index: int, dvfs: Sequence[Optional[object]],
        n: int) -> Dict[str, np.ndarray]:
    """Accumulated dose on phase ref_index (Eq. (2)) from the per-phase doses
    (Gy per history, on each phase's grid); dvfs[s] maps the reference phase
    to phase s (ignored for the reference itself)."""
    ref = phases[ref_index]
    used = [dvfs[s] for s in range(len(phases)) if s != ref_index]
    mask = report_mask(ref, used)
    dose = np.asarray(doses[ref_index], dtype=np.float64).copy()
    terms = {}
    for s in range(len(phases)):
        if s == ref_index:
            continue
        terms[s] = pull(ref, phases[s], doses[s], dvfs[s], n)
        dose = dose + terms[s]
    dose = np.where(mask, dose, 0.0)
    return {"dose": dose, "mask": mask, "terms": terms}
