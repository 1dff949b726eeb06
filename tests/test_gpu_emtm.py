"""Energy/mass-transfer dose accumulation on the GPU (pmc_accumulate, through
the C ABI) against the oracle's plain FP64 evaluation of Eqs. (2), (4)-(6)
with the App. B DVFs: same integer sums, same mapping decisions, so the doses
agree to the rounding of the mass units (the two sides compute the densities
independently) and the report masks are identical."""
import sys

import numpy as np
import pytest

from paper_1809_03927_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    from paper_1809_03927_amd import pmc
    return pmc


@pytest.fixture(scope="module")
def E():
    import oracle.emtm as emtm
    return emtm


def densities(orc, phases):
    return [orc.convert(ph, np.zeros(ph.hu.size, dtype=np.int64), 1)[1] for ph in phases]


def compare(got, want, mask_got, mask_want, exact_min=0.999):
    """Masks identical; doses within 1e-9 relative, which no differing
    decision stays within (one subvoxel moved changes a dose by about 1/n^3);
    and mostly bit-identical.  The reference phase's own dose D^R divides by
    densities the two sides interpolate from the calibration independently
    (they may differ in the last bit; the mass units round(rho 2^32) do not),
    so with many distinct HU values fewer doses are bit-identical."""
    assert np.array_equal(mask_got.astype(bool), mask_want)
    exact = np.mean(got == want)
    assert np.allclose(got, want, rtol=1e-9, atol=0), np.max(np.abs(got - want) / np.maximum(want, 1e-300))
    assert exact > exact_min, exact


@pytest.mark.parametrize("n_sub", [1, 3])
def test_accumulation_matches_oracle_random_tallies(P, E, orc, n_sub):
    """Thorax phases 3, 5, 8 accumulated onto phase 0 with the breathing DVFs;
    random integer tallies exercise both 32-bit halves of the energy sums."""
    shape = (64, 64, 40)
    ids = [0, 3, 5, 8]
    phases = [W.make_thorax(shape, p, 10) for p in ids]
    dvfs = [None] + [W.thorax_dvf(p, 0) for p in ids[1:]]
    rng = np.random.default_rng(7)
    tallies = [rng.integers(0, 2**45, size=ph.hu.size) * (ph.hu.ravel() > -1000) for ph in phases]
    rho = densities(orc, phases)
    ctx = P.pmc_create(0, P.PMC_FP32, 1, 0)
    try:
        for k, ph in enumerate(phases):
            P.pmc_load_phase(ctx, k, ph)
        for k in range(1, len(ids)):
            P.pmc_load_dvf(ctx, 10 + k, dvfs[k])
        say("emtm random tallies", shape, "n_sub", n_sub)
        dose, mask = P.pmc_accumulate(ctx, 0, tallies[0], [1, 2, 3], [11, 12, 13], tallies[1:], n_sub,
                                      1000, phases[0].hu.size, want_mask=True)
    finally:
        P.pmc_destroy(ctx)
    ref = E.emtm(phases, tallies, rho, 0, dvfs, n_sub, 1000)
    assert ref["mask"].sum() < ref["mask"].size  # the DVF grids do not cover the whole CT
    compare(dose, ref["dose"], mask, ref["mask"])


def test_accumulation_of_a_4d_transport_run(P, E, orc):
    """Per-phase tallies of a 4D thorax run (the oracle's transport, so that
    no input of the comparison comes from the library), phases 2, 5 and 7
    accumulated onto phase 0 (n_sub 2), host and device entry points, against
    the oracle."""
    import torch
    wl = W.workload_thorax4d(n_histories=300_000, shape_xyz=(64, 64, 40))
    phases = list(range(10))
    say("oracle 4D run for accumulation")
    tallies = orc.dose(wl.phases, wl.plan, wl.n_histories, wl.seed, phase_ids=phases)[0]
    e = P.Engine(device=0, precision=P.PMC_FP32, seed=wl.seed)
    try:
        e.load_workload(wl)
        src = [2, 5, 7]
        dvfs = {p: W.thorax_dvf(p, 0) for p in src}
        for p in src:
            P.pmc_load_dvf(e.ctx, 100 + p, dvfs[p])
        nv = wl.phases[0].hu.size
        dose, mask = P.pmc_accumulate(e.ctx, 0, tallies[0], src, [100 + p for p in src],
                                      [tallies[p] for p in src], 2, wl.n_histories, nv, want_mask=True)
        # device entry point on torch buffers and stream: identical result
        st = torch.cuda.Stream()
        dt = [torch.from_numpy(t).cuda() for t in tallies]
        dd = torch.empty(nv, dtype=torch.float64, device="cuda")
        dm = torch.empty(nv, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        P.pmc_accumulate_device(e.ctx, 0, dt[0].data_ptr(), src, [100 + p for p in src],
                                [dt[p].data_ptr() for p in src], 2, wl.n_histories, st.cuda_stream,
                                dd.data_ptr(), dm.data_ptr())
        st.synchronize()
        assert np.array_equal(dd.cpu().numpy(), dose) and np.array_equal(dm.cpu().numpy(), mask)
    finally:
        e.close()
    sel = [0] + src
    rho = densities(orc, [wl.phases[p] for p in sel])
    ref = E.emtm([wl.phases[p] for p in sel], [tallies[p] for p in sel], rho, 0,
                 [None] + [dvfs[p] for p in src], 2, wl.n_histories)
    compare(dose, ref["dose"], mask, ref["mask"])
    # the energy the DVFs move stays on the grid: the accumulated dose carries
    # (to the mask and the mass-weighting) the run's energy
    assert dose.max() > 0


def test_identity_dvfs_sum_the_phase_doses(P, orc):
    """Identity DVFs covering the grid: each source voxel lands in itself, so
    the accumulated dose is the sum of the phases' own doses (Sec. 2.E's
    first test, with the MC tallies and doses of a 4D run by the oracle)."""
    wl = W.workload_thorax4d(n_histories=200_000, shape_xyz=(64, 64, 40), n_phases=3)
    tallies, doses, _ = orc.dose(wl.phases, wl.plan, wl.n_histories, wl.seed, phase_ids=[0, 1, 2])
    e = P.Engine(device=0, precision=P.PMC_FP32, seed=wl.seed)
    try:
        e.load_workload(wl)
        ph = wl.phases[0]
        nz, ny, nx = ph.hu.shape
        sp = np.asarray(ph.spacing_mm)
        o = np.asarray(ph.origin_mm) - sp
        ident = W.Dvf((nx + 2, ny + 2, nz + 2), tuple(o), tuple(sp), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0),
                      np.zeros((nz + 2, ny + 2, nx + 2, 3)))
        P.pmc_load_dvf(e.ctx, 7, ident)
        for n_sub in (1, 4):
            dose, mask = P.pmc_accumulate(e.ctx, 0, tallies[0], [1, 2], [7, 7], tallies[1:], n_sub,
                                          wl.n_histories, ph.hu.size, want_mask=True)
            assert mask.all()
            want = doses[0] + doses[1] + doses[2]
            # mass counts in units of 2^-32 g/cm^3 per subvoxel: relative
            # rounding up to 0.5 / (rho 2^32), 1e-7 in air
            assert np.allclose(dose, want, rtol=2e-7, atol=0), n_sub
    finally:
        e.close()


def affine_dvf(ph, A, b, spacing, row=(1.0, 0.0, 0.0), col=(0.0, 1.0, 0.0), pad_mm=0.0):
    """DVF with translations A x + b at its grid points, grid points over the
    phase's voxel centres (minus pad), directions row, col, row x col."""
    import math
    nz, ny, nx = ph.hu.shape
    sp = np.asarray(spacing, dtype=np.float64)
    o = np.asarray(ph.origin_mm) + 0.5 * np.asarray(ph.spacing_mm) + pad_mm
    ext = np.asarray(ph.spacing_mm) * (np.array([nx, ny, nz]) - 1) - 2 * pad_mm
    n = tuple(int(math.floor(e / s + 1e-9)) + 1 for e, s in zip(ext, sp))
    u = np.asarray(row, dtype=np.float64)
    v = np.asarray(col, dtype=np.float64)
    w = np.cross(u, v)
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    x0 = o + i[..., None] * sp[0] * u + j[..., None] * sp[1] * v + k[..., None] * sp[2] * w
    return W.Dvf(n, tuple(o), tuple(sp), tuple(row), tuple(col), x0 @ np.asarray(A).T + np.asarray(b))


def random_box(shape, spacing, seed):
    ph = W.make_box(shape, spacing, 0)
    rng = np.random.default_rng(seed)
    ph.hu[...] = rng.integers(-1000, 1500, size=ph.hu.shape).astype(np.int16)
    return ph


@pytest.mark.parametrize("n_sub", [2, 5, 12, 16])
def test_rotated_and_expanding_dvfs(P, E, orc, n_sub):
    """Rotated DVF grids (the general mapping), an aligned DVF that stretches
    the source threefold (subvoxels fall outside the 4x4x4 counting window and
    go straight to the device sums) and n_sub up to 16 (16-bit counts; the
    LDS tables of n_sub 12 and 16 make the library use 128- and 64-thread
    blocks), all against the oracle."""
    import math
    shape = (24, 20, 16) if n_sub < 12 else (12, 10, 8)
    phases = [random_box(shape, (2.0, 2.5, 3.0), 20 + k) for k in range(3)]
    c, s = math.cos(0.3), math.sin(0.3)
    A1 = np.array([[0.01, -0.02, 0.005], [0.0, 0.015, 0.01], [-0.01, 0.0, 0.02]])
    rot = affine_dvf(phases[1], A1, [0.7, -1.1, 2.3], (3.0, 2.0, 2.5), row=(c, s, 0.0), col=(-s, c, 0.0),
                     pad_mm=4.0)
    # x -> x + 2 (x - centre): threefold stretch about the grid centre
    ctr = np.asarray(phases[2].origin_mm) + 0.5 * np.asarray(phases[2].spacing_mm) * np.array(shape)
    grow = affine_dvf(phases[2], 2.0 * np.eye(3), -2.0 * ctr, (2.0, 2.5, 3.0))
    rng = np.random.default_rng(3)
    tallies = [rng.integers(0, 2**40, size=ph.hu.size) for ph in phases]
    rho = densities(orc, phases)
    ctx = P.pmc_create(0, P.PMC_FP32, 1, 0)
    try:
        for k, ph in enumerate(phases):
            P.pmc_load_phase(ctx, k, ph)
        P.pmc_load_dvf(ctx, 1, rot)
        P.pmc_load_dvf(ctx, 2, grow)
        say("emtm rotated + expanding DVFs", shape, "n_sub", n_sub)
        dose, mask = P.pmc_accumulate(ctx, 0, tallies[0], [1, 2], [1, 2], tallies[1:], n_sub, 500,
                                      phases[0].hu.size, want_mask=True)
    finally:
        P.pmc_destroy(ctx)
    ref = E.emtm(phases, tallies, rho, 0, [None, rot, grow], n_sub, 500)
    assert ref["mask"].any() and ref["dose"].max() > 0
    assert ref["sums"][1]["mass"].sum() > 0 and ref["sums"][2]["mass"].sum() > 0
    # random HU over the whole calibration range (~15 % of HU values give
    # last-bit density differences in D^R)
    compare(dose, ref["dose"], mask, ref["mask"], exact_min=0.8)


@pytest.mark.parametrize("n_sub", [1, 2])
def test_centres_on_voxel_faces(P, E, orc, n_sub):
    """A constant shift of half a subvoxel pitch puts every mapped subvoxel
    centre exactly on a reference voxel face (1.5 mm and 2 mm pitch, so the
    reciprocal of the spacing is inexact along x and y): the binning must
    follow the rounded quotient exactly as a plain division does."""
    shape = (20, 18, 12)
    sp = (1.5, 1.5, 2.0)
    phases = [random_box(shape, sp, 40 + k) for k in range(2)]
    shift = -0.5 * np.asarray(sp) / n_sub
    dvf = affine_dvf(phases[1], np.zeros((3, 3)), shift, sp)
    rng = np.random.default_rng(4)
    tallies = [rng.integers(0, 2**36, size=ph.hu.size) for ph in phases]
    rho = densities(orc, phases)
    ctx = P.pmc_create(0, P.PMC_FP32, 1, 0)
    try:
        for k, ph in enumerate(phases):
            P.pmc_load_phase(ctx, k, ph)
        P.pmc_load_dvf(ctx, 1, dvf)
        say("emtm centres on voxel faces, n_sub", n_sub)
        dose, mask = P.pmc_accumulate(ctx, 0, tallies[0], [1], [1], tallies[1:], n_sub, 100,
                                      phases[0].hu.size, want_mask=True)
    finally:
        P.pmc_destroy(ctx)
    ref = E.emtm(phases, tallies, rho, 0, [None, dvf], n_sub, 100)
    assert ref["sums"][1]["mass"].sum() > 0
    compare(dose, ref["dose"], mask, ref["mask"], exact_min=0.8)
