"""Seeded synthetic inputs for the proton dose engine and its oracle.

This module is the only code that both the HIP path and the FP64 oracle see.
It builds phantoms (HU grids), calibrations, beam fields and spot lists and
holds none of the transport arithmetic: no stopping powers, no sampling, no
geometry tracking.  Everything is deterministic given its seed (numpy PCG64).

The paper's workloads are patient 4DCTs (lung, esophagus and liver, Table I)
and their clinical plans, which are not available; the thorax below stands in
for them with grids and voxel sizes of the same order (Table I: 427x246x161 at
1.27x1.27x2.0 mm; here 256x256x160 at 1.5x1.5x2.0 mm) and with the breathing
motion of up to 20 mm quoted in the introduction.  Spots carry a breathing
phase index assigned by a simplified beam-delivery clock (Sec. 2.B: sub-plans
per phase); the full synchrotron timing model of Appendix A is not reproduced.

Conventions (shared with the C ABI):
  * HU grids are int16 numpy arrays of shape (nz, ny, nx), C order, so x is the
    fastest index in memory.
  * origin_mm is the corner of voxel (0, 0, 0); voxel (i, j, k) spans
    [o + i*d, o + (i+1)*d) on each axis.
  * Spot positions are in the beam's-eye-view plane through the isocentre
    along bev_u and bev_v = direction x bev_u.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Layouts identical to the C structs pmc_spot / pmc_field (48 and 72 bytes).
SPOT_DTYPE = np.dtype(
    [
        ("energy_MeV", "<f8"),
        ("x_mm", "<f8"),
        ("y_mm", "<f8"),
        ("sigma_mm", "<f8"),
        ("weight", "<f8"),
        ("phase", "<i4"),
        ("field", "<i4"),
    ]
)
FIELD_DTYPE = np.dtype(
    [("isocentre_mm", "<f8", 3), ("direction", "<f8", 3), ("bev_u", "<f8", 3)]
)
assert SPOT_DTYPE.itemsize == 48 and FIELD_DTYPE.itemsize == 72

# Six-node synthetic CT calibration (HU -> mass density g/cm^3, HU -> RSP).
# Water (HU 0) maps to exactly (1, 1).  Ref 46 of the paper (the clinical
# calibration) is not available; these nodes are a stand-in of the usual shape.
CALIB_HU = np.array([-1000.0, -100.0, 0.0, 100.0, 1000.0, 3000.0])
CALIB_RHO = np.array([0.0012, 0.93, 1.00, 1.09, 1.62, 2.80])
CALIB_RSP = np.array([0.0010, 0.95, 1.00, 1.07, 1.55, 2.45])

# Single-node-pair "all water" calibration: every HU maps to (1, 1).
WATER_CALIB = (np.array([-1024.0, 3071.0]), np.array([1.0, 1.0]), np.array([1.0, 1.0]))


@dataclasses.dataclass
class Phase:
    """One CT phase: HU grid + geometry + calibration (+ optional mask)."""

    hu: np.ndarray  # int16 (nz, ny, nx)
    spacing_mm: Tuple[float, float, float]
    origin_mm: Tuple[float, float, float]
    calib_hu: np.ndarray
    calib_rho: np.ndarray
    calib_rsp: np.ndarray
    mask: Optional[np.ndarray] = None  # uint8 (nz, ny, nx) or None

    @property
    def shape_xyz(self) -> Tuple[int, int, int]:
        nz, ny, nx = self.hu.shape
        return nx, ny, nz

    @property
    def nvox(self) -> int:
        return int(self.hu.size)


@dataclasses.dataclass
class Plan:
    fields: np.ndarray  # FIELD_DTYPE[n_fields]
    spots: np.ndarray  # SPOT_DTYPE[n_spots]


@dataclasses.dataclass
class Workload:
    name: str
    phases: List[Phase]
    plan: Plan
    n_histories: int
    seed: int  # Philox key word 0
    request_id: int = 0


def make_field(iso_mm, direction, bev_u) -> np.ndarray:
    f = np.zeros((), dtype=FIELD_DTYPE)
    f["isocentre_mm"] = iso_mm
    f["direction"] = direction
    f["bev_u"] = bev_u
    return f


def _spots(rows) -> np.ndarray:
    a = np.zeros(len(rows), dtype=SPOT_DTYPE)
    for i, r in enumerate(rows):
        a[i] = r
    return a


# ----------------------------------------------------------------------------
# Phantoms
# ----------------------------------------------------------------------------

def make_box(shape_xyz, spacing_mm, hu_value=0, origin_mm=None, calib=None) -> Phase:
    nx, ny, nz = shape_xyz
    if origin_mm is None:
        origin_mm = (-0.5 * nx * spacing_mm[0], -0.5 * ny * spacing_mm[1], 0.0)
    hu = np.full((nz, ny, nx), hu_value, dtype=np.int16)
    ch, cr, cs = calib if calib is not None else (CALIB_HU, CALIB_RHO, CALIB_RSP)
    return Phase(hu, tuple(map(float, spacing_mm)), tuple(map(float, origin_mm)),
                 ch.copy(), cr.copy(), cs.copy())


def make_water(n=40, spacing=2.5) -> Phase:
    """Homogeneous water cube, n^3 voxels, all HU 0; z from 0, x/y centred."""
    return make_box((n, n, n), (spacing, spacing, spacing), 0)


def make_slabs() -> Phase:
    """128^3 at 2 mm; z slabs: tissue 30 mm, bone 10 mm, lung 60 mm, tissue."""
    p = make_box((128, 128, 128), (2.0, 2.0, 2.0), 40)
    z_mm = (np.arange(128) + 0.5) * 2.0  # voxel centres
    hu_z = np.where(z_mm < 30, 40, np.where(z_mm < 40, 1000, np.where(z_mm < 100, -700, 40)))
    p.hu[:] = hu_z.astype(np.int16)[:, None, None]
    return p


def random_tally(ph: Phase, seed: int, bits: int = 40) -> np.ndarray:
    """Seeded int64 tally (units of 2^-32 MeV) on a phase's grid, for checks
    of the accumulation that must not take their input from the transport
    under test: uniform in [0, 2^bits) on voxels with matter (HU > -1000),
    0 in air."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = rng.integers(0, 2**bits, size=ph.hu.size, dtype=np.int64)
    return np.where(ph.hu.ravel() > -1000, t, 0).astype(np.int64)


THORAX_EXTENT_MM = (384.0, 384.0, 320.0)


def breathing_shift_mm(t_s: float, amplitude=20.0, period=4.0) -> float:
    """Superior-inferior displacement d(t) = A sin^4(pi t / T)."""
    return amplitude * math.sin(math.pi * t_s / period) ** 4


def make_thorax(shape_xyz=(256, 256, 160), phase=0, n_phases=10, period=4.0,
                lung_scale=1.0, tumour_scale=1.0, tumour_offset_mm=(0.0, 0.0, 0.0),
                extent_mm=THORAX_EXTENT_MM) -> Phase:
    """Synthetic thorax phase on a grid centred on the origin.

    Air -1000; body elliptic cylinder (a=160, b=110 mm) HU 40; two lung
    ellipsoids at (+-80, 10, -20) mm, semi-axes (55, 70, 100) HU -750; spine
    cylinder r=15 mm at (0, -75) HU 700; tumour sphere r=20 mm at
    (-80, 20, -10) HU 40.  Painted in that order and sampled at voxel centres.
    Lungs and tumour move +z by d(t) with t = period * phase / n_phases.
    """
    nx, ny, nz = shape_xyz
    sp = (extent_mm[0] / nx, extent_mm[1] / ny, extent_mm[2] / nz)
    org = (-0.5 * extent_mm[0], -0.5 * extent_mm[1], -0.5 * extent_mm[2])
    x = org[0] + (np.arange(nx) + 0.5) * sp[0]
    y = org[1] + (np.arange(ny) + 0.5) * sp[1]
    z = org[2] + (np.arange(nz) + 0.5) * sp[2]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    d = breathing_shift_mm(period * phase / n_phases, period=period)
    hu = np.full((nz, ny, nx), -1000, dtype=np.int16)
    hu[(X / 160.0) ** 2 + (Y / 110.0) ** 2 <= 1.0] = 40
    la = np.array([55.0, 70.0, 100.0]) * lung_scale
    for cx in (-80.0, 80.0):
        m = ((X - cx) / la[0]) ** 2 + ((Y - 10.0) / la[1]) ** 2 + ((Z - (-20.0 + d)) / la[2]) ** 2 <= 1.0
        hu[m] = -750
    hu[(X - 0.0) ** 2 + (Y + 75.0) ** 2 <= 15.0 ** 2] = 700
    tr = 20.0 * tumour_scale
    tc = (-80.0 + tumour_offset_mm[0], 20.0 + tumour_offset_mm[1], -10.0 + d + tumour_offset_mm[2])
    hu[(X - tc[0]) ** 2 + (Y - tc[1]) ** 2 + (Z - tc[2]) ** 2 <= tr * tr] = 40
    return Phase(hu, sp, org, CALIB_HU.copy(), CALIB_RHO.copy(), CALIB_RSP.copy())


def thorax_tumour_mask(shape_xyz=(256, 256, 160), phase=0, n_phases=10, period=4.0,
                       extent_mm=THORAX_EXTENT_MM) -> np.ndarray:
    """Voxels of make_thorax's tumour sphere on that phase (bool, (nz, ny,
    nx)): the region of interest of the dose-volume histograms."""
    nx, ny, nz = shape_xyz
    sp = (extent_mm[0] / nx, extent_mm[1] / ny, extent_mm[2] / nz)
    org = (-0.5 * extent_mm[0], -0.5 * extent_mm[1], -0.5 * extent_mm[2])
    x = org[0] + (np.arange(nx) + 0.5) * sp[0]
    y = org[1] + (np.arange(ny) + 0.5) * sp[1]
    z = org[2] + (np.arange(nz) + 0.5) * sp[2]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    d = breathing_shift_mm(period * phase / n_phases, period=period)
    return (X + 80.0) ** 2 + (Y - 20.0) ** 2 + (Z - (-10.0 + d)) ** 2 <= 20.0 * 20.0


@dataclasses.dataclass
class Dvf:
    """A deformation vector field as a DICOM deformable registration stores
    it (App. B): a grid of points (i, j, k), 0 <= i < n[0] along the row
    direction, ..., at start_mm + i spacing[0] row + j spacing[1] col +
    k spacing[2] (row x col), each with a translation delta_mm (mm, the
    pre/post rigid matrices are the identity between 4DCT phases)."""
    n: Tuple[int, int, int]
    start_mm: Tuple[float, float, float]
    spacing_mm: Tuple[float, float, float]
    row: Tuple[float, float, float]
    col: Tuple[float, float, float]
    delta_mm: np.ndarray  # float64 (n[2], n[1], n[0], 3), i fastest
    # rigid 4x4 matrices applied before and after the translation (Eq. (7));
    # None is the identity (registrations between 4DCT phases)
    pre: Optional[np.ndarray] = None
    post: Optional[np.ndarray] = None


def thorax_dvf(phase: int, ref_phase: int = 0, n_phases=10, period=4.0, spacing_mm=(2.5, 2.5, 2.5),
               half_extent_mm=(170.0, 120.0, 150.0), taper_mm=15.0, lung_scale=1.0) -> Dvf:
    """Source-to-reference DVF of the synthetic thorax (make_thorax): points
    of the lungs (and the tumour in them) on `phase` move back by the
    breathing shift between the two phases along z; the weight falls from 1
    on the lung surface to 0 taper_mm outside it (cosine), so the field is
    smooth; the body, spine and air stay.  The grid covers the body, not the
    whole CT (like a registration's grid)."""
    d_src = breathing_shift_mm(period * phase / n_phases, period=period)
    d_ref = breathing_shift_mm(period * ref_phase / n_phases, period=period)
    n = tuple(int(2 * h / s) + 1 for h, s in zip(half_extent_mm, spacing_mm))
    start = tuple(-h for h in half_extent_mm)
    x = start[0] + np.arange(n[0]) * spacing_mm[0]
    y = start[1] + np.arange(n[1]) * spacing_mm[1]
    z = start[2] + np.arange(n[2]) * spacing_mm[2]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    la = np.array([55.0, 70.0, 100.0]) * lung_scale
    w = np.zeros(Z.shape)
    for cx in (-80.0, 80.0):
        q = np.sqrt(((X - cx) / la[0]) ** 2 + ((Y - 10.0) / la[1]) ** 2 + ((Z - (-20.0 + d_src)) / la[2]) ** 2)
        # distance outside the surface, in mm, along the ellipsoid's smallest axis
        out_mm = np.maximum(q - 1.0, 0.0) * la.min()
        w = np.maximum(w, np.where(out_mm < taper_mm, 0.5 * (1.0 + np.cos(np.pi * out_mm / taper_mm)), 0.0))
    delta = np.zeros(Z.shape + (3,))
    delta[..., 2] = -(d_src - d_ref) * w
    return Dvf(n, start, tuple(spacing_mm), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), delta)


# ----------------------------------------------------------------------------
# Plans and the simplified delivery clock
# ----------------------------------------------------------------------------

def assign_phases(n_spots_per_layer: Sequence[int], start_phase: int, t_spot=0.002,
                  t_layer_switch=1.0, period=4.0, n_phases=10) -> np.ndarray:
    """Breathing phase at each spot's start time (spots in delivery order).

    The clock starts at phase `start_phase`; each spot takes t_spot seconds and
    each change of energy layer t_layer_switch seconds.  A spot is given whole
    to the phase it starts in (no splitting across phases).
    """
    phases = []
    t = 0.0
    for li, n in enumerate(n_spots_per_layer):
        if li > 0:
            t += t_layer_switch
        for _ in range(n):
            ph = (start_phase + int(math.floor(t / period * n_phases))) % n_phases
            phases.append(ph)
            t += t_spot
    return np.array(phases, dtype=np.int32)


# ----------------------------------------------------------------------------
# Beam-delivery simulation inputs (Sec. 2.B, App. A)
# ----------------------------------------------------------------------------

# Synchrotron timing parameters, each (central value, 1-sigma uncertainty),
# in the order the simulation draws them.  The paper takes its values from
# its Ref. 45 (not available here); these are synthetic, of the magnitudes
# App. A describes (layer switch ~2 s, 70 ms of discarded beam, ~8 s
# extraction limit), and stand in for them.
SYNC_PARAMS = ("layer_switch_s", "layer_switch_per_mev", "discard_s", "spill_rate_mu_s",
               "spill_rate_per_mev", "spot_switch_s", "spot_switch_per_mm", "capacity_mu",
               "extraction_max_s")
SYNC_DEFAULT = {
    "layer_switch_s": (1.9, 0.05),        # reset + acceleration to 70 MeV
    "layer_switch_per_mev": (0.002, 0.0),  # s per MeV above 70 MeV
    "discard_s": (0.070, 0.002),          # beam discarded at every extraction start
    "spill_rate_mu_s": (8.0, 0.4),        # MU/s spilled at 70 MeV
    "spill_rate_per_mev": (0.04, 0.0),    # MU/s per MeV above 70 MeV
    "spot_switch_s": (0.002, 0.0002),     # beam off between spots
    "spot_switch_per_mm": (0.0001, 0.0),  # s per mm of the larger axis move
    "capacity_mu": (8.0, 0.3),            # MU one synchrotron fill delivers
    "extraction_max_s": (8.0, 0.0),       # extraction time limit per fill
}


@dataclasses.dataclass
class Delivery:
    """Options of the beam-delivery simulation (Sec. 2.B)."""
    n_phases: int = 10
    start_phase: int = -1          # -1: U{0..N-1} per trial and field
    period_s: float = 4.0          # breathing period mean mu
    period_sd_s: float = 0.0       # sigma: t_ph = N(mu, sigma) / N per phase
    period_min_s: int = 0          # 0 < min <= max: mu ~ U{min..max} s per trial and field
    period_max_s: int = 0
    gate_lo: int = -1              # gated delivery: phases gate_lo..gate_hi; -1: free breathing
    gate_hi: int = -1
    max_mu: float = 0.0            # isolayered repainting: max MU per spot delivery (0: none)
    sync: dict = dataclasses.field(default_factory=lambda: dict(SYNC_DEFAULT))
    seed: int = 1
    n_trials: int = 1


def layer_grid(nu: int, nv: int, pitch: float, serpentine=True):
    """Spot positions (u, v) of one layer on a centred nu x nv grid."""
    us = (np.arange(nu) - 0.5 * (nu - 1)) * pitch
    vs = (np.arange(nv) - 0.5 * (nv - 1)) * pitch
    out = []
    for j, v in enumerate(vs):
        row = us if (not serpentine or j % 2 == 0) else us[::-1]
        for u in row:
            out.append((float(u), float(v)))
    return out


def plan_single(energy=150.0, sigma=5.0, iso=(0.0, 0.0, 50.0), direction=(0, 0, 1),
                bev_u=(1, 0, 0)) -> Plan:
    fields = np.array([make_field(iso, direction, bev_u)], dtype=FIELD_DTYPE)
    spots = _spots([(energy, 0.0, 0.0, sigma, 1.0, 0, 0)])
    return Plan(fields, spots)


def plan_slabs(seed=2) -> Plan:
    rng = np.random.Generator(np.random.PCG64(seed))
    fields = np.array([make_field((0.0, 0.0, 128.0), (0, 0, 1), (1, 0, 0))], dtype=FIELD_DTYPE)
    rows = []
    for l in range(10):
        e = 100.0 + 80.0 * l / 9.0
        sig = 7.0 - 3.0 * (e - 100.0) / 80.0
        for (u, v) in layer_grid(10, 5, 5.0):
            rows.append((e, u, v, sig, 0.0, 0, 0))
    spots = _spots(rows)
    spots["weight"] = rng.lognormal(0.0, 0.5, size=len(spots))
    return Plan(fields, spots)


def plan_thorax(seed=3, n_layers=20, e_lo=90.0, e_hi=200.0, grid=(15, 10), pitch=5.0,
                directions=((0.0, -1.0, 0.0),), spots_per_field=None,
                iso=(-80.0, 20.0, -2.5), start_phase=None, n_phases=10) -> Plan:
    """Thorax plan: layers delivered high -> low energy, serpentine spots.

    sigma falls linearly from 7 mm at e_lo to 4 mm at e_hi.  Each spot gets the
    breathing phase at its start time from `assign_phases`.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if start_phase is None:
        start_phase = int(rng.integers(0, n_phases))
    fields = []
    rows = []
    for fi, dvec in enumerate(directions):
        dvec = np.asarray(dvec, dtype=float)
        dvec = dvec / np.linalg.norm(dvec)
        # bev_u: x axis unless the beam runs along x, then -y-ish
        ref = np.array([0.0, 0.0, 1.0])
        u = np.cross(ref, dvec)
        if np.linalg.norm(u) < 1e-9:
            u = np.array([1.0, 0.0, 0.0])
        u = u / np.linalg.norm(u)
        fields.append(make_field(iso, dvec, u))
        layer_counts = []
        pos = layer_grid(grid[0], grid[1], pitch)
        if spots_per_field is not None:
            per_layer = int(math.ceil(spots_per_field[fi] / n_layers))
        else:
            per_layer = len(pos)
        for l in range(n_layers):
            e = e_hi - (e_hi - e_lo) * l / max(n_layers - 1, 1)
            sig = 7.0 - 3.0 * (e - e_lo) / (e_hi - e_lo)
            take = pos[:per_layer] if per_layer <= len(pos) else [pos[i % len(pos)] for i in range(per_layer)]
            if spots_per_field is not None:
                remaining = spots_per_field[fi] - sum(layer_counts)
                take = take[: max(0, min(len(take), remaining))]
            layer_counts.append(len(take))
            for (pu, pv) in take:
                rows.append((e, pu, pv, sig, 0.0, 0, fi))
        ph = assign_phases(layer_counts, start_phase, n_phases=n_phases)
        base = len(rows) - len(ph)
        for k, p in enumerate(ph):
            r = list(rows[base + k])
            r[5] = int(p)
            rows[base + k] = tuple(r)
    spots = _spots(rows)
    spots["weight"] = rng.lognormal(0.0, 0.5, size=len(spots))
    return Plan(np.array(fields, dtype=FIELD_DTYPE), spots)


# ----------------------------------------------------------------------------
# The benchmark workloads
# ----------------------------------------------------------------------------

def workload_tiny(n_histories=100_000) -> Workload:
    """40^3 water at 2.5 mm, one 150 MeV spot along +z, sigma 5 mm."""
    ph = make_water(40, 2.5)
    ph.origin_mm = (-50.0, -50.0, 0.0)
    return Workload("tiny_water_40", [ph], plan_single(150.0, 5.0, (0.0, 0.0, 50.0)), n_histories, seed=1)


def workload_slabs(n_histories=10_000_000) -> Workload:
    ph = make_slabs()
    ph.origin_mm = (-128.0, -128.0, 0.0)
    return Workload("slabs_128", [ph], plan_slabs(2), n_histories, seed=2)


def workload_influence(n_histories=30_000) -> Workload:
    """Small heterogeneous case for influence matrices: 48 x 48 x 64 voxels
    of 2.5 mm (water, a lung slab at z 20-50 mm, a bone block at x > 15 mm,
    z 60-80 mm); two fields (+z and oblique in x-z), a 3 x 3 spot grid
    (+-15 mm) at 90 and 120 MeV on the +z field, 4 spots on the oblique
    field, one spot that misses the grid and one spot of another phase."""
    ph = make_box((48, 48, 64), (2.5, 2.5, 2.5), 0, origin_mm=(-60.0, -60.0, 0.0))
    z = (np.arange(64) + 0.5) * 2.5
    x = (np.arange(48) + 0.5) * 2.5 - 60.0
    ph.hu[(z >= 20) & (z < 50), :, :] = -700
    bone = ((z >= 60) & (z < 80))[:, None, None] & (x > 15.0)[None, None, :]
    ph.hu[np.broadcast_to(bone, ph.hu.shape)] = 1000
    c = 1.0 / math.sqrt(2.0)
    fields = np.array([make_field((0.0, 0.0, 60.0), (0, 0, 1), (1, 0, 0)),
                       make_field((0.0, 0.0, 60.0), (c, 0.0, c), (c, 0.0, -c))], dtype=FIELD_DTYPE)
    rows = []
    for e in (90.0, 120.0):
        for yy in (-15.0, 0.0, 15.0):
            for xx in (-15.0, 0.0, 15.0):
                rows.append((e, xx, yy, 4.0, 1.0 + 0.1 * len(rows), 0, 0))
    for k, (xx, yy) in enumerate(((-10.0, 0.0), (0.0, 0.0), (10.0, -10.0), (0.0, 12.0))):
        rows.append((100.0 + 10.0 * k, xx, yy, 3.0, 1.5, 0, 1))
    rows.append((100.0, 300.0, 0.0, 3.0, 1.0, 0, 0))  # misses the grid
    rows.append((100.0, 0.0, 0.0, 3.0, 1.0, 1, 0))    # another phase
    return Workload("influence_48x48x64", [ph], Plan(fields, _spots(rows)), n_histories, seed=6)


def workload_thorax4d(n_histories=50_000_000, shape_xyz=(256, 256, 160), n_phases=10) -> Workload:
    phases = [make_thorax(shape_xyz, p, n_phases) for p in range(n_phases)]
    plan = plan_thorax(3, n_phases=n_phases)
    return Workload("thorax4d_256x256x160x10", phases, plan, n_histories, seed=3)


SERVED_GRIDS = [(64, 64, 64), (96, 96, 96), (128, 128, 128), (192, 192, 120), (256, 256, 160)]


@dataclasses.dataclass
class ServedRequest:
    index: int
    arrival_s: float
    grid: Tuple[int, int, int]
    phase_index: int
    phantom_key: tuple
    n_spots: int
    n_histories: int
    seed: int


def served_stream(n_requests=200, rate_hz=1.0, seed=4, h_lo=1e5, h_hi=5e7) -> List[ServedRequest]:
    """Poisson arrivals of single-phase dose requests of mixed size."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(n_requests):
        t += float(rng.exponential(1.0 / rate_hz))
        grid = SERVED_GRIDS[int(rng.integers(0, len(SERVED_GRIDS)))]
        ph = int(rng.integers(0, 10))
        lung = float(rng.uniform(0.9, 1.1))
        tum = float(rng.uniform(0.9, 1.1))
        off = tuple(float(v) for v in rng.uniform(-10.0, 10.0, size=3))
        n_spots = int(round(math.exp(rng.uniform(math.log(50), math.log(3000)))))
        n_hist = int(round(math.exp(rng.uniform(math.log(h_lo), math.log(h_hi)))))
        out.append(ServedRequest(i, t, grid, ph, (grid, ph, round(lung, 6), round(tum, 6), off),
                                 n_spots, n_hist, int(rng.integers(0, 2**31))))
    return out


def served_phantom(req: ServedRequest) -> Phase:
    grid, ph, lung, tum, off = req.phantom_key
    return make_thorax(grid, ph, 10, lung_scale=lung, tumour_scale=tum, tumour_offset_mm=off)


def served_plan(req: ServedRequest) -> Plan:
    n_layers = max(1, int(math.ceil(req.n_spots / 150)))
    per_layer = int(math.ceil(req.n_spots / n_layers))
    nu = int(math.ceil(math.sqrt(per_layer * 1.5)))
    nv = int(math.ceil(per_layer / nu))
    plan = plan_thorax(req.seed % (2**31), n_layers=n_layers, e_lo=90.0, e_hi=200.0,
                       grid=(nu, nv), spots_per_field=[req.n_spots], start_phase=0, n_phases=1)
    plan.spots["phase"] = 0
    return plan


ROBUST_DIRECTIONS = ((0.0, -1.0, 0.0), (1.0, 0.0, 0.0), (1.0 / math.sqrt(2.0), -1.0 / math.sqrt(2.0), 0.0))
ROBUST_SCENARIOS = [
    ("nominal", (0.0, 0.0, 0.0), 1.0),
    ("x+3", (3.0, 0.0, 0.0), 1.0), ("x-3", (-3.0, 0.0, 0.0), 1.0),
    ("y+3", (0.0, 3.0, 0.0), 1.0), ("y-3", (0.0, -3.0, 0.0), 1.0),
    ("z+3", (0.0, 0.0, 3.0), 1.0), ("z-3", (0.0, 0.0, -3.0), 1.0),
    ("rsp+3.5%", (0.0, 0.0, 0.0), 1.035), ("rsp-3.5%", (0.0, 0.0, 0.0), 0.965),
]


def plan_robust(seed=5, shift_mm=(0.0, 0.0, 0.0)) -> Plan:
    """3-field plan, 8000 spots (2667/2667/2666), 20 layers 90-200 MeV each.

    A setup shift is applied as a translation of every field's isocentre.
    """
    iso = tuple(np.array([-80.0, 20.0, -2.5]) + np.asarray(shift_mm))
    return plan_thorax(seed, n_layers=20, e_lo=90.0, e_hi=200.0, grid=(14, 10), pitch=5.0,
                       directions=ROBUST_DIRECTIONS, spots_per_field=[2667, 2667, 2666], iso=iso)


# ----------------------------------------------------------------------------
# Synthetic phantoms shaped like the paper's three patient cases (Table I:
# lung, esophagus and liver; the CT grids, voxel sizes, field counts, tumour
# volumes and motion amplitudes of the table).  The anatomy is synthetic:
# painted geometric structures, sampled at voxel centres, on a grid centred
# on the origin; the breathing moves the listed structures along +z by
# d(t) = A sin^4(pi t / 4 s) with A the table's tumour motion.
# ----------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Case:
    name: str
    grid: Tuple[int, int, int]            # voxels x, y, z (Table I)
    voxel_mm: Tuple[float, float, float]  # (Table I)
    fields: int                           # (Table I)
    motion_mm: float                      # tumour motion amplitude (Table I)
    tumour_cm3: float                     # tumour volume (Table I)
    body_ab_mm: Tuple[float, float]       # body elliptic cylinder semi-axes x, y
    directions: Tuple[Tuple[float, float, float], ...]
    pitch_mm: float                       # spot and layer spacing
    seed: int


CASES = {
    "lung": Case("lung", (427, 246, 161), (1.27, 1.27, 2.00), 3, 5.4, 79.6, (170.0, 115.0),
                 ((0.0, -1.0, 0.0), (1.0, 0.0, 0.0), (1.0 / math.sqrt(2.0), -1.0 / math.sqrt(2.0), 0.0)),
                 5.0, 41),
    "esophagus": Case("esophagus", (430, 272, 235), (1.27, 1.27, 2.00), 2, 5.3, 204.4, (170.0, 120.0),
                      ((0.0, 1.0, 0.0), (-1.0 / math.sqrt(2.0), 1.0 / math.sqrt(2.0), 0.0)), 6.0, 42),
    "liver": Case("liver", (452, 307, 281), (1.27, 1.27, 1.50), 3, 7.5, 581.0, (180.0, 130.0),
                  ((0.0, -1.0, 0.0), (-1.0, 0.0, 0.0), (-1.0 / math.sqrt(2.0), 1.0 / math.sqrt(2.0), 0.0)),
                  7.0, 43),
}


def _case_axes(c: Case):
    nx, ny, nz = c.grid
    sp = c.voxel_mm
    org = tuple(-0.5 * n * d for n, d in zip(c.grid, sp))
    x = org[0] + (np.arange(nx) + 0.5) * sp[0]
    y = org[1] + (np.arange(ny) + 0.5) * sp[1]
    z = org[2] + (np.arange(nz) + 0.5) * sp[2]
    return sp, org, x[None, None, :], y[None, :, None], z[:, None, None]


def case_tumour(c: Case, d: float):
    """Tumour of the case at breathing shift d: ('sphere', centre, r) or
    ('cylinder', (x, y, z centre), r, half-length) along z."""
    if c.name == "esophagus":
        half = 0.5 * c.tumour_cm3 * 1000.0 / (math.pi * 20.0 ** 2)
        return ("cylinder", (0.0, -40.0, 0.0 + d), 20.0, half)
    r = (3.0 * c.tumour_cm3 * 1000.0 / (4.0 * math.pi)) ** (1.0 / 3.0)
    centre = (-85.0, 20.0, -10.0 + d) if c.name == "lung" else (-60.0, 15.0, 10.0 + d)
    return ("sphere", centre, r)


def make_case(name: str, phase: int = 0, n_phases: int = 10, period: float = 4.0) -> Phase:
    """One breathing phase of the named case.

    Every case: air -1000; body elliptic cylinder HU 40; vertebral body
    (cylinder r 15 mm, 0.7 b behind the centre) HU 700.
    * lung: lungs (ellipsoids at (+-85, 10, -20) mm, semi-axes 60, 75, 110)
      HU -750 and a spherical tumour (79.6 cm^3 at (-85, 20, -10)) HU 40,
      both moving;
    * esophagus: lungs at (+-85, 10, 0), semi-axes (60, 75, 160), moving;
      heart (ellipsoid at (20, 45, -60), semi-axes 55, 45, 55) HU 40; a
      tumour cylinder around the esophagus (r 20 mm, 204.4 cm^3, along z at
      (0, -40)) HU 50 with an air lumen (r 5 mm) HU -900, both moving;
    * liver: lung bases at (+-85, 10, 150), semi-axes (60, 75, 80), moving;
      liver (ellipsoid at (-55, 10, 20), semi-axes 110, 85, 95) HU 60 and a
      spherical tumour (581 cm^3 at (-60, 15, 10)) HU 30, both moving.
    """
    c = CASES[name]
    sp, org, X, Y, Z = _case_axes(c)
    nx, ny, nz = c.grid
    d = breathing_shift_mm(period * phase / n_phases, amplitude=c.motion_mm, period=period)
    hu = np.full((nz, ny, nx), -1000, dtype=np.int16)
    a, b = c.body_ab_mm
    body = (X / a) ** 2 + (Y / b) ** 2 <= 1.0
    hu[np.broadcast_to(body, hu.shape)] = 40

    def ellipsoid(cx, cy, cz, ax, ay, az):
        return ((X - cx) / ax) ** 2 + ((Y - cy) / ay) ** 2 + ((Z - cz) / az) ** 2 <= 1.0

    def paint(mask, value):
        hu[np.broadcast_to(mask, hu.shape)] = value

    if name == "lung":
        for cx in (-85.0, 85.0):
            paint(ellipsoid(cx, 10.0, -20.0 + d, 60.0, 75.0, 110.0), -750)
    elif name == "esophagus":
        for cx in (-85.0, 85.0):
            paint(ellipsoid(cx, 10.0, 0.0 + d, 60.0, 75.0, 160.0), -750)
        paint(ellipsoid(20.0, 45.0, -60.0, 55.0, 45.0, 55.0), 40)
    else:
        for cx in (-85.0, 85.0):
            paint(ellipsoid(cx, 10.0, 150.0 + d, 60.0, 75.0, 80.0), -750)
        paint(ellipsoid(-55.0, 10.0, 20.0 + d, 110.0, 85.0, 95.0), 60)
    paint((X ** 2 + (Y + 0.7 * b) ** 2 <= 15.0 ** 2), 700)
    t = case_tumour(c, d)
    if t[0] == "sphere":
        (tx, ty, tz), r = t[1], t[2]
        paint((X - tx) ** 2 + (Y - ty) ** 2 + (Z - tz) ** 2 <= r * r, 40 if name == "lung" else 30)
    else:
        (tx, ty, tz), r, half = t[1], t[2], t[3]
        along = np.abs(Z - tz) <= half
        paint(((X - tx) ** 2 + (Y - ty) ** 2 <= r * r) & along, 50)
        paint(((X - tx) ** 2 + (Y - ty) ** 2 <= 5.0 ** 2) & along, -900)
    return Phase(hu, sp, org, CALIB_HU.copy(), CALIB_RHO.copy(), CALIB_RSP.copy())


def _energy_for_wet_cm(R: float) -> float:
    """Proton energy (MeV) whose range in water is R cm, from the
    Bragg-Kleeman rule R = 0.0022 E^1.77 (a plan-making approximation)."""
    return (R / 0.0022) ** (1.0 / 1.77)


def _wet_to_tumour(ph: Phase, c: Case, direction, iso) -> Tuple[float, float]:
    """Water-equivalent depth (cm) from where the beam axis through `iso`
    enters the grid to the tumour's near and far surfaces (0.5 mm samples of
    the phase's stopping-power ratio along the axis)."""
    w = np.asarray(direction, float) / np.linalg.norm(direction)
    ext = np.array(c.grid) * np.array(c.voxel_mm)
    org = np.array(ph.origin_mm)
    ts = np.arange(-1000.0, 1000.0, 0.5)
    pts = np.asarray(iso)[None, :] + ts[:, None] * w[None, :]
    idx = np.floor((pts - org) / np.array(c.voxel_mm)).astype(int)
    inside = np.all((idx >= 0) & (idx < np.array(c.grid)), axis=1) & np.all(pts - org < ext, axis=1)
    idx, pts = idx[inside], pts[inside]
    hu = ph.hu[idx[:, 2], idx[:, 1], idx[:, 0]].astype(float)
    wet = np.cumsum(np.interp(hu, ph.calib_hu, ph.calib_rsp)) * 0.05
    t = case_tumour(c, 0.0)
    if t[0] == "sphere":
        (tx, ty, tz), r = t[1], t[2]
        intum = np.sum((pts - np.array([tx, ty, tz])) ** 2, axis=1) <= r * r
    else:
        (tx, ty, tz), r, half = t[1], t[2], t[3]
        intum = ((pts[:, 0] - tx) ** 2 + (pts[:, 1] - ty) ** 2 <= r * r) & (np.abs(pts[:, 2] - tz) <= half)
    k = np.nonzero(intum)[0]
    return float(wet[k[0]]), float(wet[k[-1]])


def plan_case(name: str, start_phase: Optional[int] = None, n_phases: int = 10) -> Plan:
    """Plan of a case: per field, spots on a square grid of pitch_mm in the
    beam's eye view covering the tumour's projection plus 5 mm, in energy
    layers pitch_mm of water apart from 5 mm before the tumour's near
    surface to 5 mm beyond its far surface (along the field's central axis,
    high to low energy), serpentine; sigma 7 -> 4 mm with energy; weights
    lognormal(0, 0.5); breathing phases by the simplified delivery clock (2
    ms per spot, 1 s layer switch, 4 s period, random start phase)."""
    c = CASES[name]
    rng = np.random.Generator(np.random.PCG64(c.seed))
    if start_phase is None:
        start_phase = int(rng.integers(0, n_phases))
    ph0 = make_case(name, 0, n_phases)
    t = case_tumour(c, 0.0)
    iso = t[1]
    fields, rows = [], []
    for fi, dvec in enumerate(c.directions[:c.fields]):
        w = np.asarray(dvec, float) / np.linalg.norm(dvec)
        u = np.cross(np.array([0.0, 0.0, 1.0]), w)
        u = u / np.linalg.norm(u)
        v = np.cross(w, u)
        fields.append(make_field(iso, w, u))
        near, far = _wet_to_tumour(ph0, c, w, iso)
        r_lo, r_hi = max(near - 0.5, 0.5), far + 0.5
        step = c.pitch_mm / 10.0
        n_layers = int(math.floor((r_hi - r_lo) / step)) + 1
        # BEV footprint: the tumour's projection on (u, v) plus 5 mm
        if t[0] == "sphere":
            half_u = half_v = t[2] + 5.0
        else:
            half_u = abs(u[2]) * t[3] + t[2] + 5.0
            half_v = abs(v[2]) * t[3] + t[2] + 5.0
        nu = int(2 * half_u // c.pitch_mm) + 1
        nv = int(2 * half_v // c.pitch_mm) + 1
        pos = [(pu, pv) for (pu, pv) in layer_grid(nu, nv, c.pitch_mm)
               if t[0] == "cylinder" or pu * pu + pv * pv <= half_u * half_u]
        counts = []
        for l in range(n_layers):
            R = r_hi - l * step
            e = min(max(_energy_for_wet_cm(R), 70.0), 230.0)
            sig = 7.0 - 3.0 * (e - 70.0) / 160.0
            for (pu, pv) in pos:
                rows.append((e, pu, pv, sig, 0.0, 0, fi))
            counts.append(len(pos))
        phs = assign_phases(counts, start_phase, n_phases=n_phases)
        base = len(rows) - len(phs)
        for k, p in enumerate(phs):
            r = list(rows[base + k])
            r[5] = int(p)
            rows[base + k] = tuple(r)
    spots = _spots(rows)
    spots["weight"] = rng.lognormal(0.0, 0.5, size=len(spots))
    return Plan(np.array(fields, dtype=FIELD_DTYPE), spots)


def workload_case(name: str, n_histories: int = 50_000_000, n_phases: int = 10, workers: int = 0) -> Workload:
    """The 4D dose calculation of a case: its breathing phases and plan.
    workers > 0 generates the phases in forked processes (call it before
    the process touches the GPU)."""
    if workers > 0:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, n_phases)) as pool:
            phases = pool.starmap(make_case, [(name, p, n_phases) for p in range(n_phases)])
    else:
        phases = [make_case(name, p, n_phases) for p in range(n_phases)]
    c = CASES[name]
    plan = plan_case(name, n_phases=n_phases)
    return Workload(f"{name}4d_{c.grid[0]}x{c.grid[1]}x{c.grid[2]}x{n_phases}", phases, plan, n_histories,
                    seed=c.seed)


def scaled_calibration(phase: Phase, rsp_scale: float) -> Phase:
    """Same phase with its HU->RSP calibration scaled (range uncertainty)."""
    return dataclasses.replace(phase, calib_rsp=phase.calib_rsp * rsp_scale)
