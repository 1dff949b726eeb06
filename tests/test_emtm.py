"""Energy/mass-transfer dose accumulation (Sec. 2.D.2, Eqs. (2), (4)-(6);
DVFs per App. B, Eqs. (7)-(8)): the oracle (`oracle.emtm`) against what
fixes it without the method itself — fields that trilinear interpolation
reproduces exactly, identity and rigid one-voxel maps, exact conservation of
the integer energy and mass sums, the paper's first 3D comparison test
(identical phases, identity DVFs -> the static dose), and a pure-Python
brute force on a tiny grid."""
import math

import numpy as np
import pytest

from paper_1809_03927_amd import workloads as W

E = pytest.importorskip("oracle.emtm")


def dvf_on(ph, delta_fn, spacing=None, row=(1.0, 0.0, 0.0), col=(0.0, 1.0, 0.0), pad_mm=0.0):
    """A DVF whose grid points cover the phase's voxel centres (minus pad)."""
    nz, ny, nx = ph.hu.shape
    sp = np.asarray(spacing or ph.spacing_mm, dtype=np.float64)
    o = np.asarray(ph.origin_mm) + 0.5 * np.asarray(ph.spacing_mm) + pad_mm
    ext = np.asarray(ph.spacing_mm) * (np.array([nx, ny, nz]) - 1) - 2 * pad_mm
    n = tuple(int(math.floor(e / s + 1e-9)) + 1 for e, s in zip(ext, sp))
    d = W.Dvf(n, tuple(o), tuple(sp), row, col, np.zeros((n[2], n[1], n[0], 3)))
    u, v, w = E.dvf_axes(d)
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    x0 = o + i[..., None] * sp[0] * u + j[..., None] * sp[1] * v + k[..., None] * sp[2] * w
    d.delta_mm[...] = delta_fn(x0)
    return d


def dvf_cover(ph, delta_fn):
    """A DVF with the phase's spacing whose grid points run one voxel beyond
    the grid on every side, so every subvoxel centre is inside it."""
    nz, ny, nx = ph.hu.shape
    sp = np.asarray(ph.spacing_mm, dtype=np.float64)
    o = np.asarray(ph.origin_mm) - sp
    n = (nx + 2, ny + 2, nz + 2)
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    x0 = o + np.stack([i, j, k], axis=-1) * sp
    return W.Dvf(n, tuple(o), tuple(sp), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), np.asarray(delta_fn(x0), dtype=np.float64))


def small_box(shape=(12, 10, 8), spacing=(2.0, 2.5, 3.0)):
    ph = W.make_box(shape, spacing, 0)
    rng = np.random.default_rng(5)
    ph.hu[...] = rng.integers(-900, 1200, size=ph.hu.shape).astype(np.int16)
    return ph


def density_of(orc, ph):
    _, rho = orc.convert(ph, np.zeros(ph.hu.size, dtype=np.int64), 1)
    return rho


# ----------------------------------------------------------------------------
# the DVF (App. B)
# ----------------------------------------------------------------------------

def test_dvf_reproduces_affine_fields_on_a_rotated_grid():
    """Trilinear interpolation is exact for affine translation fields, so
    T(r) = r + A r + b everywhere inside the grid; the grid's row and column
    directions are rotated, so a transposed axis or a wrong depth direction
    (Eq. (8)) would show."""
    ph = small_box()
    c, s = math.cos(0.3), math.sin(0.3)
    row, col = (c, s, 0.0), (-s, c, 0.0)
    A = np.array([[0.01, -0.02, 0.005], [0.0, 0.015, 0.01], [-0.01, 0.0, 0.02]])
    b = np.array([0.7, -1.1, 2.3])
    d = dvf_on(ph, lambda x: x @ A.T + b, spacing=(3.0, 2.0, 2.5), row=row, col=col, pad_mm=4.0)
    rng = np.random.default_rng(1)
    pts = np.asarray(ph.origin_mm) + rng.uniform(0.2, 0.8, size=(2000, 3)) * np.array(
        [24.0, 25.0, 24.0])
    got = E.dvf_map(d, pts)
    inside = ~np.isnan(got[:, 0])
    assert inside.sum() > 500 and (~inside).sum() > 0
    want = pts + pts @ A.T + b
    assert np.allclose(got[inside], want[inside], rtol=0, atol=1e-9)
    # grid points themselves map to x0 + delta (Eq. (7))
    u, v, w = E.dvf_axes(d)
    x0 = np.asarray(d.start_mm) + 2 * d.spacing_mm[0] * u + 3 * d.spacing_mm[1] * v + 1 * d.spacing_mm[2] * w
    assert np.allclose(E.dvf_map(d, x0[None])[0], x0 + d.delta_mm[1, 3, 2], atol=1e-12)


def test_points_outside_the_grid_are_not_mapped():
    ph = small_box()
    d = dvf_on(ph, lambda x: 0.0 * x, pad_mm=3.0)
    lo = np.asarray(d.start_mm)
    hi = lo + (np.asarray(d.n) - 1) * np.asarray(d.spacing_mm)
    pts = np.array([lo, hi, lo - 1e-9, hi + [0, 0, 1e-9], 0.5 * (lo + hi)])
    got = E.dvf_map(d, pts)
    assert np.array_equal(np.isnan(got[:, 0]), [False, False, True, True, False])
    assert np.array_equal(got[[0, 1, 4]], pts[[0, 1, 4]])


# ----------------------------------------------------------------------------
# EMTM (Eqs. (2), (4)-(6))
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3])
def test_identity_dvf_gives_each_phase_its_own_dose(orc, n):
    """Identity map: every subvoxel lands in its own voxel, so the sums are
    n^3 x (tally, mass units) exactly and Eq. (2) adds the phases' doses."""
    phs = [small_box(), small_box()]
    rng = np.random.default_rng(2)
    tallies = [rng.integers(0, 2**40, size=p.hu.size) for p in phs]
    rhos = [density_of(orc, p) for p in phs]
    ident = dvf_cover(phs[0], lambda x: 0.0 * x)
    out = E.emtm(phs, tallies, rhos, 0, [None, ident], n, 1000)
    acc = out["sums"][1]
    t = tallies[1]
    assert np.array_equal(acc["e_hi"], n ** 3 * (t >> 32))
    assert np.array_equal(acc["e_lo"], n ** 3 * (t & 0xFFFFFFFF))
    assert np.array_equal(acc["mass"], n ** 3 * E.mass_units(rhos[1]))
    v = 0.2 * 0.25 * 0.3
    want = E.phase_dose(tallies[0], rhos[0], v, 1000) + E.phase_dose(tallies[1], rhos[1], v, 1000)
    m = out["mask"]
    assert m.all()  # the grid covers every voxel centre
    assert np.allclose(out["dose"], want, rtol=1e-9, atol=0)


def test_one_voxel_shift_moves_the_sums_by_one_voxel(orc):
    phs = [small_box(), small_box()]
    rng = np.random.default_rng(3)
    tallies = [np.zeros(p.hu.size, dtype=np.int64) for p in phs]
    tallies[1] = rng.integers(0, 2**45, size=phs[1].hu.size)
    rhos = [density_of(orc, p) for p in phs]
    shift = dvf_cover(phs[0], lambda x: np.broadcast_to([-2.0, 0.0, 0.0], x.shape))  # one voxel in -x
    acc = E.emtm(phs, tallies, rhos, 0, [None, shift], 2, 10)["sums"][1]
    nz, ny, nx = phs[1].hu.shape
    t = tallies[1].reshape(nz, ny, nx)
    eh = acc["e_hi"].reshape(nz, ny, nx)
    el = acc["e_lo"].reshape(nz, ny, nx)
    assert np.array_equal(eh[:, :, :-1], 8 * (t[:, :, 1:] >> 32))
    assert np.array_equal(el[:, :, :-1], 8 * (t[:, :, 1:] & 0xFFFFFFFF))
    # nothing maps into the last column (its source would be beyond the grid)
    assert not eh[:, :, -1].any() and not el[:, :, -1].any()


def test_energy_and_mass_are_conserved_exactly(orc):
    """A smooth field that keeps every mapped subvoxel inside the reference
    grid: the integer energy and mass sums equal n^3 x the source totals."""
    ph = small_box((16, 14, 12), (2.0, 2.0, 2.0))
    rng = np.random.default_rng(4)
    t = rng.integers(0, 2**50, size=ph.hu.size)
    rho = density_of(orc, ph)

    def wobble(x):
        return np.stack([0.8 * np.sin(x[..., 1] / 5.0), 0.6 * np.cos(x[..., 2] / 4.0),
                         0.7 * np.sin(x[..., 0] / 6.0)], axis=-1)

    d = dvf_cover(ph, wobble)
    # source voxels at least two voxels inside the grid: the field moves
    # less than one voxel, so all their subvoxels map inside
    n = 3
    nz, ny, nx = ph.hu.shape
    inner = np.zeros((nz, ny, nx), dtype=bool)
    inner[2:-2, 2:-2, 2:-2] = True
    t2 = np.where(inner.ravel(), t, 0)
    rho2 = np.where(inner.ravel(), rho, 0.0)
    acc = E.emtm([ph, ph], [np.zeros_like(t2), t2], [rho, rho2], 0, [None, d], n, 1)["sums"][1]
    tot_e = int(acc["e_hi"].astype(object).sum()) * 2**32 + int(acc["e_lo"].astype(object).sum())
    assert tot_e == n ** 3 * int(t2.astype(object).sum())
    assert int(acc["mass"].astype(object).sum()) == n ** 3 * int(E.mass_units(rho2).astype(object).sum())
    # and the map did move mass between voxels
    assert not np.array_equal(acc["mass"], n ** 3 * E.mass_units(rho2))


def test_paper_identical_phases_reproduce_the_static_dose(orc):
    """Sec. 2.E, first test: the same CT on every phase with identity DVFs;
    the accumulated dose is the static dose of the whole plan (to the
    rounding of the mass units)."""
    wl = W.workload_tiny(n_histories=20_000)
    ph = wl.phases[0]
    plan = W.Plan(wl.plan.fields.copy(), wl.plan.spots.copy())
    n_ph = 3
    spots = np.concatenate([plan.spots] * n_ph)
    spots["phase"] = np.repeat(np.arange(n_ph), len(plan.spots))
    spots["weight"] = spots["weight"] / n_ph
    plan4 = W.Plan(plan.fields, spots)
    tallies, _, _ = orc.dose([ph] * n_ph, plan4, wl.n_histories, wl.seed, with_dose=False)
    (static,), sdose, _ = orc.dose([ph], W.Plan(plan.fields, plan.spots), wl.n_histories, wl.seed)
    rho = density_of(orc, ph)
    ident = dvf_cover(ph, lambda x: 0.0 * x)
    out = E.emtm([ph] * n_ph, tallies, [rho] * n_ph, 1, [ident] * n_ph, 2, wl.n_histories)
    # the three phases' tallies add up to a static run of the same histories
    # only in distribution (different spot indices key different histories):
    # compare the sum of the phase doses instead, and the energy with the
    # static run statistically
    v = float(np.prod(np.asarray(ph.spacing_mm) * 0.1))
    want = sum(E.phase_dose(t, rho, v, wl.n_histories) for t in tallies)
    assert np.allclose(out["dose"], want, rtol=1e-9, atol=0)
    assert abs(out["dose"].sum() / sdose[0].sum() - 1.0) < 0.02


def test_brute_force_tiny_grid(orc):
    """Pure-Python loops over voxels and subvoxels with a weighted-sum
    trilinear interpolation and Python integers."""
    src = W.make_box((4, 3, 3), (2.0, 2.0, 2.0), 0, origin_mm=(0.0, 0.0, 0.0))
    ref = W.make_box((5, 4, 3), (1.8, 1.9, 2.1), 0, origin_mm=(-0.7, -0.4, 0.3))
    rng = np.random.default_rng(8)
    src.hu[...] = rng.integers(-800, 900, size=src.hu.shape).astype(np.int16)
    ref.hu[...] = rng.integers(-800, 900, size=ref.hu.shape).astype(np.int16)
    ts = rng.integers(0, 2**44, size=src.hu.size)
    tr = rng.integers(0, 2**44, size=ref.hu.size)
    rs, rr = density_of(orc, src), density_of(orc, ref)
    dv = W.Dvf((4, 4, 4), (0.5, 0.5, 0.5), (2.5, 2.4, 2.6), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0),
               rng.uniform(-1.5, 1.5, size=(4, 4, 4, 3)))
    n = 2
    out = E.emtm([ref, src], [tr, ts], [rr, rs], 0, [None, dv], n, 7)

    def tmap(p):
        g = [(p[a] - dv.start_mm[a]) / dv.spacing_mm[a] for a in range(3)]
        if any(g[a] < 0 or g[a] > dv.n[a] - 1 for a in range(3)):
            return None
        i0 = [min(int(math.floor(g[a])), dv.n[a] - 2) for a in range(3)]
        f = [g[a] - i0[a] for a in range(3)]
        q = list(p)
        for dk in (0, 1):
            for dj in (0, 1):
                for di in (0, 1):
                    wgt = (f[0] if di else 1 - f[0]) * (f[1] if dj else 1 - f[1]) * (f[2] if dk else 1 - f[2])
                    for a in range(3):
                        q[a] += wgt * dv.delta_mm[i0[2] + dk, i0[1] + dj, i0[0] + di, a]
        return q

    nzr, nyr, nxr = ref.hu.shape
    e_sum = [0] * ref.hu.size
    m_sum = [0] * ref.hu.size
    nz, ny, nx = src.hu.shape
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                j = x + nx * (y + ny * z)
                mq = int(round(rs[j] * 2**32))
                if mq == 0:
                    continue
                for c in range(n):
                    for b in range(n):
                        for a in range(n):
                            p = [(x + (a + 0.5) / n) * 2.0, (y + (b + 0.5) / n) * 2.0, (z + (c + 0.5) / n) * 2.0]
                            q = tmap(p)
                            if q is None:
                                continue
                            t = [math.floor((q[k] - ref.origin_mm[k]) / ref.spacing_mm[k]) for k in range(3)]
                            if not (0 <= t[0] < nxr and 0 <= t[1] < nyr and 0 <= t[2] < nzr):
                                continue
                            i = t[0] + nxr * (t[1] + nyr * t[2])
                            e_sum[i] += int(ts[j])
                            m_sum[i] += mq
    acc = out["sums"][1]
    assert [int(a) * 2**32 + int(b) for a, b in zip(acc["e_hi"], acc["e_lo"])] == e_sum
    assert [int(m) for m in acc["mass"]] == m_sum
    vr = 0.18 * 0.19 * 0.21
    vs = 0.2 ** 3
    want = []
    for i in range(ref.hu.size):
        d = (int(tr[i]) / 2**32) * E.MEV_TO_J / (rr[i] * vr * 1e-3) / 7 if rr[i] > 0 else 0.0
        if m_sum[i]:
            d += e_sum[i] * E.MEV_TO_J / (m_sum[i] * vs * 1e-3 * 7)
        want.append(d)
    mask = out["mask"]
    assert np.allclose(out["dose"][mask], np.array(want)[mask], rtol=1e-12, atol=0)
    assert not out["dose"][~mask].any()


def test_integer_sums_bound_the_plain_ratio(orc):
    """Eq. (5) in plain FP64 against the oracle's integer sums: subvoxel k
    of source voxel j carries mass M_jk = rho_j V / n^3 (kg) and energy
    E_jk = E_j / n^3 (J); D_i = sum E_jk / sum M_jk over the subvoxels
    mapped into reference voxel i, summed in floating point.  The integer
    sums count round-half-even(rho_j 2^32) per subvoxel and the tally units
    exactly, so they differ from the plain ratio only by the mass rounding:
    |D_int / D - 1| <= 0.5 / (2^32 min rho) over the contributing voxels
    (1e-7 in air at 0.0012 g/cm^3), plus FP64 rounding of the plain sums.
    Densities from air to bone, a breathing-like DVF, n = 3."""
    src = small_box()
    ref = small_box()
    rng = np.random.default_rng(17)
    src.hu[:, :, :4] = -1000  # a slab of air
    rho_s = density_of(orc, src)
    t = rng.integers(0, 2**40, size=src.hu.size)
    dv = dvf_cover(src, lambda x0: np.stack([0.4 * np.sin(x0[..., 1] / 7.0), 0.0 * x0[..., 0],
                                             1.3 * np.cos(x0[..., 0] / 9.0)], axis=-1))
    n = 3
    acc = E.push(src, t, rho_s, ref, dv, n)
    v_s = float(np.prod(np.asarray(src.spacing_mm) * 0.1))
    got = E.dose_from_sums(acc, v_s, 1)
    # plain FP64 sums of Eq. (4)
    nz, ny, nx = src.hu.shape
    rz, ry, rx = ref.hu.shape
    zz, yy, xx = np.nonzero(rho_s.reshape(nz, ny, nx) > 0)
    j = xx + nx * (yy + ny * zz)
    e_j = t[j].astype(np.float64) * 2.0 ** -32 * E.MEV_TO_J / n ** 3
    m_j = rho_s[j] * v_s * 1e-3 / n ** 3
    e_sum = np.zeros(ref.hu.size)
    m_sum = np.zeros(ref.hu.size)
    rho_min = np.full(ref.hu.size, np.inf)
    o, s = np.asarray(src.origin_mm), np.asarray(src.spacing_mm)
    for c in range(n):
        for b in range(n):
            for a in range(n):
                r = o + (np.stack([xx, yy, zz], axis=-1) + (np.array([a, b, c]) + 0.5) / n) * s
                q = E.dvf_map(dv, r)
                tgt = np.floor((q - np.asarray(ref.origin_mm)) / np.asarray(ref.spacing_mm)).astype(np.int64)
                ok = np.all((tgt >= 0) & (tgt < np.array([rx, ry, rz])), axis=1) & ~np.isnan(q[:, 0])
                lin = tgt[ok, 0] + rx * (tgt[ok, 1] + ry * tgt[ok, 2])
                np.add.at(e_sum, lin, e_j[ok])
                np.add.at(m_sum, lin, m_j[ok])
                np.minimum.at(rho_min, lin, rho_s[j][ok])
    sel = m_sum > 0
    assert np.array_equal(sel, acc["mass"] > 0)
    want = e_sum[sel] / m_sum[sel]
    rel = np.abs(got[sel] / want - 1.0)
    bound = 0.5 / (2.0 ** 32 * rho_min[sel]) * (1 + 1e-6) + 1e-12
    assert np.all(rel <= bound), float(np.max(rel / bound))
    air = rho_min[sel] < 0.01
    assert air.any() and (~air).any()
    # the rounding is visible in air and far smaller in tissue
    assert rel[air].max() > 1e-9 and rel[~air].max() < 1e-9
