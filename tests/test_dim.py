"""Dose-interpolation accumulation (Sec. 2.D.2, Eqs. (2), (3)) and the DVF
construction of App. B (Eqs. (7), (8)): the oracle (`oracle.dim`,
`oracle.emtm`) against what fixes it without the method itself — closed
forms for the grid points and for rigid pre/post matrices, trilinear sampling
that reproduces affine dose fields and clamps at the grid's edge, identity and
rigid maps, and a pure-Python brute force on a tiny grid."""
import math

import numpy as np
import pytest

from paper_1809_03927_amd import workloads as W

E = pytest.importorskip("oracle.emtm")
D = pytest.importorskip("oracle.dim")


def rot_z(theta, t):
    c, s = math.cos(theta), math.sin(theta)
    m = np.eye(4)
    m[:3, :3] = [[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]]
    m[:3, 3] = t
    return m


def inverse_rigid(m):
    r = m[:3, :3]
    out = np.eye(4)
    out[:3, :3] = r.T
    out[:3, 3] = -r.T @ m[:3, 3]
    return out


def box(shape=(7, 6, 5), spacing=(2.0, 2.5, 3.0), origin=(-7.0, -6.0, 1.0)):
    return W.make_box(shape, spacing, 0, origin_mm=origin)


def centres(ph):
    return E.voxel_centres(ph).reshape(-1, 3)


# ----------------------------------------------------------------------------
# App. B
# ----------------------------------------------------------------------------

def test_grid_points_follow_eq8_and_eq7():
    """x0 = start + i dX U + j dY V + k dZ W on a rotated grid (Python loop),
    r_f = x0 + delta with identity matrices, and with M_pre = [R | t],
    M_post = its inverse: r_f = x0 + R^T delta."""
    c, s = math.cos(0.4), math.sin(0.4)
    row, col = (c, s, 0.0), (-s * 0.6, c * 0.6, 0.8)
    rng = np.random.default_rng(1)
    n = (3, 4, 2)
    delta = rng.uniform(-2, 2, size=(n[2], n[1], n[0], 3))
    d = W.Dvf(n, (10.0, -5.0, 3.0), (2.0, 1.5, 2.5), row, col, delta)
    x0, rf = E.dvf_points(d)
    u = np.array(row)
    v = np.array(col)
    w = np.cross(u, v)
    for k in range(n[2]):
        for j in range(n[1]):
            for i in range(n[0]):
                want = np.array(d.start_mm) + i * 2.0 * u + j * 1.5 * v + k * 2.5 * w
                assert np.allclose(x0[k, j, i], want, rtol=0, atol=1e-12)
    assert np.array_equal(rf, x0 + delta)
    pre = rot_z(0.7, [3.0, -1.0, 2.0])
    d2 = W.Dvf(n, d.start_mm, d.spacing_mm, row, col, delta, pre=pre, post=inverse_rigid(pre))
    _, rf2 = E.dvf_points(d2)
    want2 = x0 + delta @ pre[:3, :3]  # R^T delta, row-vector form
    assert np.allclose(rf2, want2, rtol=0, atol=1e-12)


def test_rigid_matrices_in_the_map():
    """T(r) = M_post (M_pre r + delta(r)): with M_post the inverse of M_pre and
    a constant delta, every inside point moves by R^T delta."""
    ph = box()
    pre = rot_z(-0.5, [1.0, 2.0, -3.0])
    n = (6, 6, 5)
    const = np.array([0.4, -0.9, 1.3])
    d = W.Dvf(n, (-6.0, -5.0, 2.0), (2.0, 2.0, 2.5), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0),
              np.broadcast_to(const, (n[2], n[1], n[0], 3)).copy(), pre=pre, post=inverse_rigid(pre))
    pts = centres(ph)
    q = E.dvf_map(d, pts)
    ok = ~np.isnan(q[:, 0])
    assert ok.sum() > 20
    assert np.allclose(q[ok], pts[ok] + pre[:3, :3].T @ const, rtol=0, atol=1e-12)


# ----------------------------------------------------------------------------
# Eq. (3)
# ----------------------------------------------------------------------------

def affine_dose(ph, a=(0.3, -0.2, 0.5), b=7.0):
    p = centres(ph)
    return b + p @ np.asarray(a)


def test_dose_sample_is_exact_for_affine_fields_and_clamps():
    ph = box()
    dose = affine_dose(ph)
    # voxel centres give the voxel values
    assert np.allclose(D.dose_sample(dose, ph, centres(ph)), dose, rtol=1e-13, atol=0)
    # interior points: trilinear interpolation reproduces affine fields
    lo = np.asarray(ph.origin_mm) + 0.5 * np.asarray(ph.spacing_mm)
    hi = lo + (np.array(ph.shape_xyz) - 1) * np.asarray(ph.spacing_mm)
    rng = np.random.default_rng(2)
    pts = lo + rng.uniform(0, 1, size=(500, 3)) * (hi - lo)
    assert np.allclose(D.dose_sample(dose, ph, pts), 7.0 + pts @ np.array([0.3, -0.2, 0.5]), rtol=1e-12)
    # beyond the outermost centres: the border value (clamp to edge), exactly
    nz, ny, nx = ph.hu.shape
    d3 = dose.reshape(nz, ny, nx)
    far = np.array([[hi[0] + 5.0, lo[1], lo[2]], [lo[0] - 30.0, hi[1] + 0.1, hi[2] + 9.0]])
    got = D.dose_sample(dose, ph, far)
    assert got[0] == d3[0, 0, nx - 1] and got[1] == d3[nz - 1, ny - 1, 0]


def cover(ph, delta_fn):
    """A DVF on the phase's voxel centres extended one voxel on every side."""
    nz, ny, nx = ph.hu.shape
    sp = np.asarray(ph.spacing_mm, dtype=np.float64)
    o = np.asarray(ph.origin_mm) - 0.5 * sp
    n = (nx + 2, ny + 2, nz + 2)
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    x0 = o + np.stack([i, j, k], axis=-1) * sp
    return W.Dvf(n, tuple(o), tuple(sp), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0),
                 np.asarray(delta_fn(x0), dtype=np.float64))


@pytest.mark.parametrize("n", [1, 3])
def test_identity_dvfs_give_the_phase_doses(n):
    """Identity maps on one geometry: every subvoxel samples its own phase's
    dose field at its own position; with n = 1 (voxel centres) D^S is the
    source dose, and Eq. (2) sums the phases' doses (the paper's first
    comparison test with identical CTs, Sec. 2.E)."""
    ph = box()
    rng = np.random.default_rng(3)
    doses = [rng.uniform(0, 1, size=ph.hu.size) for _ in range(3)]
    ident = cover(ph, lambda x: 0.0 * x)
    out = D.dim([ph, ph, ph], doses, 1, [ident, None, ident], n)
    assert out["mask"].all()
    if n == 1:
        assert np.allclose(out["terms"][0], doses[0], rtol=1e-13, atol=0)
        assert np.allclose(out["dose"], doses[0] + doses[1] + doses[2], rtol=1e-13, atol=0)
    else:
        # an affine dose is reproduced exactly by the subvoxel average too
        aff = affine_dose(ph)
        out2 = D.dim([ph, ph], [np.zeros(ph.hu.size), aff], 0, [None, ident], n)
        nz, ny, nx = ph.hu.shape
        inner = np.zeros((nz, ny, nx), bool)
        inner[1:-1, 1:-1, 1:-1] = True
        assert np.allclose(out2["dose"][inner.ravel()], aff[inner.ravel()], rtol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_rigid_shift_of_an_affine_dose(n):
    """A constant reference-to-source shift s: the subvoxel average of an
    affine dose is its value at the shifted voxel centre (the offsets are
    symmetric), away from the clamped border."""
    ph = box((9, 8, 7), (2.0, 2.0, 2.0), (0.0, 0.0, 0.0))
    s = np.array([1.3, -0.7, 0.45])
    dvf = cover(ph, lambda x: np.broadcast_to(s, x.shape))
    dose = affine_dose(ph)
    term = D.dim([ph, ph], [np.zeros(ph.hu.size), dose], 0, [None, dvf], n)["terms"][1]
    nz, ny, nx = ph.hu.shape
    inner = np.zeros((nz, ny, nx), bool)
    inner[2:-2, 2:-2, 2:-2] = True
    want = 7.0 + (centres(ph) + s) @ np.array([0.3, -0.2, 0.5])
    assert np.allclose(term[inner.ravel()], want[inner.ravel()], rtol=1e-12)


def test_pull_of_selected_voxels_equals_the_whole():
    """The voxel selection only picks which reference voxels are evaluated:
    any subset, in any order, equals the same entries of the whole pull."""
    ph = box((9, 8, 7), (2.0, 2.0, 2.0), (0.0, 0.0, 0.0))
    dvf = cover(ph, lambda x: np.broadcast_to(np.array([1.3, -0.7, 0.45]), x.shape))
    dose = affine_dose(ph) + np.random.default_rng(5).random(ph.hu.size)
    whole = D.pull(ph, ph, dose, dvf, 2)
    pick = np.random.default_rng(6).permutation(ph.hu.size)[:100]
    assert np.array_equal(D.pull(ph, ph, dose, dvf, 2, voxels=pick), whole[pick])


def test_brute_force_tiny_grid():
    """Pure-Python loops with weighted-sum trilinear interpolation of the DVF
    and of the dose (clamped), centres outside the DVF grid contributing 0."""
    ref = box((5, 4, 3), (1.8, 1.9, 2.1), (-0.7, -0.4, 0.3))
    src = box((4, 3, 3), (2.0, 2.0, 2.0), (0.0, 0.0, 0.0))
    rng = np.random.default_rng(8)
    dose_r = rng.uniform(0, 1, size=ref.hu.size)
    dose_s = rng.uniform(0, 1, size=src.hu.size)
    dv = W.Dvf((4, 4, 4), (0.5, 0.5, 0.5), (2.5, 2.4, 2.6), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0),
               rng.uniform(-1.5, 1.5, size=(4, 4, 4, 3)))
    n = 2
    out = D.dim([ref, src], [dose_r, dose_s], 0, [None, dv], n)

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

    nzs, nys, nxs = src.hu.shape
    dims = (nxs, nys, nzs)

    def sample(q):
        u = [min(max((q[a] - src.origin_mm[a]) / src.spacing_mm[a] - 0.5, 0.0), dims[a] - 1) for a in range(3)]
        i0 = [int(math.floor(u[a])) for a in range(3)]
        f = [u[a] - i0[a] for a in range(3)]
        tot = 0.0
        for dk in (0, 1):
            for dj in (0, 1):
                for di in (0, 1):
                    x = min(i0[0] + di, nxs - 1)
                    y = min(i0[1] + dj, nys - 1)
                    z = min(i0[2] + dk, nzs - 1)
                    wgt = (f[0] if di else 1 - f[0]) * (f[1] if dj else 1 - f[1]) * (f[2] if dk else 1 - f[2])
                    tot += wgt * dose_s[x + nxs * (y + nys * z)]
        return tot

    nz, ny, nx = ref.hu.shape
    want = np.zeros(ref.hu.size)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                acc = 0.0
                for a in range(n):
                    for b in range(n):
                        for c in range(n):
                            p = [ref.origin_mm[0] + (x + (a + 0.5) / n) * ref.spacing_mm[0],
                                 ref.origin_mm[1] + (y + (b + 0.5) / n) * ref.spacing_mm[1],
                                 ref.origin_mm[2] + (z + (c + 0.5) / n) * ref.spacing_mm[2]]
                            q = tmap(p)
                            if q is not None:
                                acc += sample(q)
                i = x + nx * (y + ny * z)
                want[i] = dose_r[i] + acc / n ** 3
    inside_all = []
    for p in centres(ref):
        g = [(p[a] - dv.start_mm[a]) / dv.spacing_mm[a] for a in range(3)]
        inside_all.append(all(0 <= g[a] <= dv.n[a] - 1 for a in range(3)))
    m = np.array(inside_all)
    assert np.array_equal(out["mask"], m) and m.any() and not m.all()
    want = np.where(m, want, 0.0)
    assert np.allclose(out["dose"], want, rtol=1e-12, atol=1e-15)
