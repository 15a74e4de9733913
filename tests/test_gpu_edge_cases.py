"""Degenerate and edge inputs of the HIP path against the CPU oracle (through the C ABI): a
density image without an interface, a gas with no liquid, many particles in one storage cell,
two particles, positions outside the box, other detection schedules, other smoothing and
removal settings."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_1502_03234_amd import dcm, synth  # noqa: E402
from test_gpu_parity import FORCE_TOL, check_system, make, rc_close, say  # noqa: E402


def test_uniform_lattice_has_no_interface():
    """One particle per box: the smoothed image is constant, two-means has a single level, every
    box is liquid, every distance is the band cap and every cutoff is r_c^min (Eq. 7)."""
    st = synth.lattice(16, 16.0, seed=5)
    p, po = make(st)
    s = check_system(st, p, po, "lattice 16^3")
    det = s.detect()
    torch.cuda.synchronize()
    km = det["km"].cpu().numpy()
    assert km[0] == km[1] == 64.0
    assert not det["label"].cpu().numpy().any()
    assert np.all(det["dist"].cpu().numpy() == p.rc_max + 1.0)
    assert np.all(det["rc"].cpu().numpy() == p.rc_min)
    s.close()


def test_dilute_gas():
    st = synth.gas(500, (20.0, 20.0, 20.0), seed=6)
    p, po = make(st)
    check_system(st, p, po, "gas 500", planar=False).close()


def test_crowded_storage_cell():
    """64 particles inside one half-box storage cell (a 4 x 4 x 4 lattice of spacing 0.1 x 0.2 x
    0.2) among 1,901 gas particles, a count that fills no whole workgroup: the counting sort's
    runs of one key span a whole wave and its ranks come from atomics in no fixed order. Counts,
    labels, distances, cutoffs, forces and pair counts match the oracle, and a second system made
    from the same state gives the same force bits (the in-cell id order fixes the storage order)."""
    box = (16.0, 16.0, 24.0)
    gas = synth.gas(1901, box, seed=78)
    g = np.arange(4, dtype=np.float64)
    Z, Y, X = np.meshgrid(12.15 + 0.2 * g, 8.15 + 0.2 * g, 8.07 + 0.1 * g, indexing="ij")
    crowd = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    m = crowd.shape[1]
    st = synth.State(x=np.ascontiguousarray(np.concatenate([gas.x, crowd], axis=1)),
                     v=np.ascontiguousarray(np.concatenate([gas.v, np.zeros((3, m))], axis=1)),
                     box=box, n_liquid=0, n_vapor=gas.n_vapor + m, temperature=0.7)
    p, po = make(st)
    s = check_system(st, p, po, "crowded cell", planar=False)
    t = dcm.System(p, st.x, st.v)
    fa, fb = s.forces()["f"], t.forces()["f"]
    torch.cuda.synchronize()
    assert torch.equal(fa, fb)
    s.close()
    t.close()


def test_two_particles_closed_form():
    """Two particles 1.5 apart across the periodic x face: F = 24 eps (2 (s/r)^12 - (s/r)^6) / r
    along the line, equal and opposite (both cutoffs exceed r)."""
    r = 1.5
    st = synth.pair(r, 14.0)
    p, po = make(st)
    s = check_system(st, p, po, "pair")
    f = s.forces()["f"].cpu().numpy()
    mag = 24.0 * (2.0 * r ** -12 - r ** -6) / r
    # particle 0 sits at x = L - r/2, its partner's image at L + r/2: the force on 0 points to -x
    # when repulsive (mag > 0)
    assert abs(f[0, 0] - (-mag)) <= 1e-12 * abs(mag) and abs(f[0, 1] - mag) <= 1e-12 * abs(mag)
    assert np.all(f[1:] == 0.0)
    s.close()


def test_positions_outside_the_box_are_wrapped(slab16k):
    """Inputs moved by -1, 0, 1 or 2 box lengths per particle wrap exactly as the oracle wraps
    them (checked bit for bit inside check_system)."""
    k = (np.arange(slab16k.n) % 4 - 1)[None, :]
    st = synth.State(x=np.ascontiguousarray(slab16k.x + k * np.asarray(slab16k.box)[:, None]),
                     v=slab16k.v, box=slab16k.box, n_liquid=slab16k.n_liquid, n_vapor=slab16k.n_vapor,
                     temperature=slab16k.temperature, meta=dict(slab16k.meta))
    assert st.x.min() < 0.0 and st.x.max() > max(slab16k.box)
    p, po = make(st)
    check_system(st, p, po, "slab16k shifted by whole boxes").close()


def test_positions_far_outside_the_box_land_inside():
    """Coordinates of size 1e16 to 1e22, where x - L floor(x / L) keeps no digit of the remainder
    (for -7.3e22 on edges 14 and 28 and 7.3e22 on edge 24 the rounded remainder stays below 0
    even after adding L), still wrap into [0, L) exactly as the oracle wraps them, so the
    binning, the cell starts and the force kernel's cell windows index only cells of the box.
    The moved particles are ones whose wrapped place is at least 1.0 from every other one."""
    box = (14.0, 28.0, 24.0)
    gas = synth.gas(2000, box, seed=91)
    far = [(0, -7.3e22), (1, -7.3e22), (2, 7.3e22), (0, 1e16), (1, -1e16), (2, 3e17),
           (0, -1e20), (1, 1e20), (2, -2.701e22)]
    x = gas.x.copy()
    po = O.params(box)
    L = np.asarray(box)[:, None]
    wrapped = O.wrap(po, x)
    moved = []
    for i in range(gas.n):
        if len(moved) == len(far):
            break
        ax, val = far[len(moved)]
        y = x[:, i].copy()
        y[ax] = val
        yw = O.wrap(po, np.ascontiguousarray(y[:, None]))
        d = wrapped - yw
        d -= L * np.round(d / L)
        r = np.sqrt(np.sum(d * d, axis=0))
        r[i] = np.inf
        if np.all(r >= 1.0):
            x[:, i] = y
            wrapped[:, i] = yw[:, 0]
            moved.append(i)
    assert len(moved) == len(far)
    st = synth.State(x=np.ascontiguousarray(x), v=gas.v, box=box, n_liquid=0,
                     n_vapor=gas.n_vapor, temperature=gas.temperature)
    p, po = make(st)
    s = check_system(st, p, po, "gas with coordinates up to 7.3e22", planar=False)
    xw = s.state()[0].cpu().numpy()
    assert np.all((xw >= 0.0) & (xw < L))
    s.step(4)
    s.check()
    s.close()


@pytest.mark.parametrize("de,detections", [(0, 0), (1, 6), (3, 2)])
def test_other_detection_schedules(slab16k, de, detections):
    p, po = make(slab16k, detect_every=de)
    s = dcm.System(p, slab16k.x, slab16k.v)
    x0, v0, rc0, _ = s.state()
    f0 = s.forces()["f"]
    torch.cuda.synchronize()
    dcm.dcm_set_profiling(s.h, 1)
    s.step(1)
    x1, v1, rc1, _ = s.state()
    torch.cuda.synchronize()
    rs = O.RunState(x0.cpu().numpy(), v0.cpu().numpy(), rc0.cpu().numpy(), f0.cpu().numpy(), 0)
    O.run(po, rs, 1)
    assert np.max(np.abs(x1.cpu().numpy() - rs.x)) < 1e-13
    if de == 1:
        assert rc_close(rc1.cpu().numpy(), rs.rc)        # step 1 re-detects
    else:
        assert np.array_equal(rc1.cpu().numpy(), rs.rc)
    s.step(5)
    c = {k: v[1] for k, v in dcm.dcm_stage_times(s.h).items()}
    say(f"detect_every={de}: stage counts {c}")
    assert c["forces"] == 6 and c["sort"] == 6
    assert c["distance"] == detections and c["cutoffs"] == detections
    s.check()
    s.close()


def test_single_row_wave_at_the_x_faces():
    """A wave whose particles all lie in force row 0, with one particle just past x = r_s and
    one just short of L_x - r_s (r_s the search radius): the x-interval a row gives them reaches
    a little beyond r_s (the enlarged square root of the bounds), so they must leave the
    single-row form, whose intervals may not wrap. Forces and pair counts match the oracle."""
    from test_gpu_parity import force_err
    st = synth.lattice(16, 16.0, seed=17)           # one particle per box: 64 in force row 0
    rc0 = 2.5
    rs = rc0 * (1.0 + 1e-12) + 1e-9
    x = st.x.copy()
    x[0, 2] = rs + 7.5e-7                           # box (2, 0, 0)
    x[0, (1 * 16 + 1) * 16 + 13] = 16.0 - rs - 7.5e-7   # box (13, 1, 1)
    p, po = make(st)
    s = dcm.System(p, x, st.v)
    rc = np.full(st.n, rc0)
    s.set_cutoffs(rc)
    fo = s.forces()
    xg, _, _, _ = s.state()
    torch.cuda.synchronize()
    s.check()
    xw = xg.cpu().numpy()
    assert np.array_equal(xw, O.wrap(po, x))
    ref = O.forces(po, xw, rc)
    assert force_err(fo["f"].cpu().numpy(), ref.f).max() <= FORCE_TOL
    assert np.array_equal(fo["pairs"].cpu().numpy().astype(np.int64), ref.pairs)
    s.close()


@pytest.mark.parametrize("n,box,seed,passes", [
    (3000, (16.0, 16.0, 28.0), 1, 1),      # force rows 1 x 2 boxes (y too short)
    (5617, (14.0, 14.0, 60.0), 2, 0),      # no smoothing: the count image is the smoothed image
    (2800, (20.0, 20.0, 17.0), 5, 2),      # force rows 2 x 1 (z odd), two smoothing passes
    (30000, (41.0, 37.0, 52.0), 3, 1),      # odd x and y
])
def test_steps_with_detection_on_ragged_grids(n, box, seed, passes):
    """Steps that re-detect take the box-count image from the cell scan of the same step (a
    box's storage cells lie in one scan block). On grids whose force rows are 1 box high in y
    or z, with 0, 1 or 2 smoothing passes (the image lands in either smoothing buffer), two
    steps that both re-detect match the oracle: positions, velocities and the new cutoffs."""
    st = synth.small_slab(n, box, seed)
    p, po = make(st, detect_every=1, smooth_passes=passes)
    s = dcm.System(p, st.x, st.v)
    x0, v0, rc0, _ = s.state()
    f0 = s.forces()["f"]
    torch.cuda.synchronize()
    s.step(2)
    x2, v2, rc2, k = s.state()
    torch.cuda.synchronize()
    assert k == 2
    rs = O.RunState(x0.cpu().numpy(), v0.cpu().numpy(), rc0.cpu().numpy(), f0.cpu().numpy(), 0)
    O.run(po, rs, 2)
    say(f"ragged steps n={n} box={box} passes={passes}: max |dx| "
        f"{np.max(np.abs(x2.cpu().numpy() - rs.x)):.2e}")
    assert np.max(np.abs(x2.cpu().numpy() - rs.x)) < 1e-12
    assert np.max(np.abs(v2.cpu().numpy() - rs.v)) < 1e-10
    assert rc_close(rc2.cpu().numpy(), rs.rc)
    s.check()
    s.close()


@pytest.mark.parametrize("kw", [dict(smooth_passes=2, min_component=0),
                                dict(smooth_passes=0, min_component=100)])
def test_smoothing_and_removal_settings(slab16k, kw):
    p, po = make(slab16k, **kw)
    check_system(slab16k, p, po, f"slab16k {kw}").close()


@pytest.mark.parametrize("kw", [dict(vapor_cutoff=1), dict(ms_nu=0.005, ms_iters=20),
                                dict(neighbor_list=1, skin=0.3)])
def test_options_without_an_interface(kw):
    """The options on a density image with no interface: vapor cutoffs, the Mumford-Shah
    segmentation (a constant image has nothing to segment) and neighbour lists all reduce to the
    plain path's labels and cutoffs."""
    st = synth.lattice(16, 16.0, seed=5)
    p, po = make(st, **kw)
    s = check_system(st, p, po, f"lattice 16^3 {kw}")
    det = s.detect()
    torch.cuda.synchronize()
    assert not det["label"].cpu().numpy().any()
    assert np.all(det["rc"].cpu().numpy() == p.rc_min)
    s.close()


def test_tail_without_an_interface():
    """No interface: every particle is deep in the liquid, so the tail force is zero and the
    tail energy is the uniform one, (8/3) pi rho [(1/3) r_c^-9 - r_c^-3] per particle with the
    two-means density."""
    st = synth.lattice(16, 16.0, seed=5)
    p, po = make(st, tail=1)
    s = dcm.System(p, st.x, st.v)
    fo = s.forces()
    x, _, rc, _ = s.state()
    torch.cuda.synchronize()
    xw, rcg = x.cpu().numpy(), rc.cpu().numpy()
    pair = O.forces(po, xw, rcg)
    assert np.max(np.abs(fo["f"].cpu().numpy() - pair.f)) <= FORCE_TOL * np.sqrt(np.mean(np.sum(pair.f ** 2, axis=0))) + 1e-13
    rho = 1.0                                      # one particle per unit box
    share = (8.0 / 3.0) * np.pi * rho * (rcg ** -9 / 3.0 - rcg ** -3)
    e = fo["e"].cpu().numpy()
    assert np.all(np.abs(e - (pair.e + share)) <= 1e-12 * np.maximum(np.abs(pair.e + share), 1.0))
    s.close()


def test_options_on_a_dilute_gas():
    """A gas with no liquid (every box vapor after removal) with the tail correction, vapor
    cutoffs and the Mumford-Shah segmentation at once."""
    st = synth.gas(500, (20.0, 20.0, 20.0), seed=6)
    p, po = make(st, tail=1, vapor_cutoff=1, ms_nu=0.005, ms_iters=20)
    s = dcm.System(p, st.x, st.v)
    det = s.detect()
    fo = s.forces(per_atom=False, thermo=False)
    x, _, rc, _ = s.state()
    torch.cuda.synchronize()
    xw, rcg = x.cpu().numpy(), rc.cpu().numpy()
    od = O.detect(po, xw)
    assert np.array_equal(det["label"].cpu().numpy(), od.label)
    assert rc_close(rcg, od.rc, p.rc_min, p.rc_max, p.alpha, cap=2 * p.rc_max + 1.0, planar=False)
    ref = O.forces(po, xw, rcg).f + O.tail(po, od, xw, rcg)[0]
    frms = np.sqrt(np.mean(np.sum(ref ** 2, axis=0)))
    err = np.linalg.norm(fo["f"].cpu().numpy() - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), frms)
    assert err.max() <= FORCE_TOL
    s.close()


def test_two_particles_with_lists():
    r = 1.5
    st = synth.pair(r, 14.0)
    p, po = make(st, neighbor_list=1, skin=0.5, rc_max=5.0)    # r_c^max + skin fits the 14-box axis
    s = check_system(st, p, po, "pair with lists")
    f = s.forces()["f"].cpu().numpy()
    mag = 24.0 * (2.0 * r ** -12 - r ** -6) / r
    assert abs(f[0, 0] - (-mag)) <= 1e-12 * abs(mag) and abs(f[0, 1] - mag) <= 1e-12 * abs(mag)
    s.close()


@pytest.mark.slow
def test_largest_system_sampled_parity():
    """The largest system the ABI accepts, near n = 2^26 (406^3 = 66,923,416 particles, one per
    box of a density-0.80 lattice): positions are addressed with 32-bit byte offsets, which reach
    within 0.3 % of 2^31 here. Forces under seeded per-particle cutoffs (the detection of a
    uniform lattice finds no interface) are checked against the oracle for particles at the
    highest storage offsets (the top force rows in y and z), the lowest, and a random sample."""
    m = 406
    assert m ** 3 < 1 << 26
    st = synth.lattice(m, 437.0, seed=11)
    p, po = make(st, rc_min=2.5, rc_max=4.0)
    say(f"largest: n={st.n}, workspace {dcm.dcm_workspace_bytes(p, st.n) / 2**30:.1f} GiB")
    s = dcm.System(p, st.x, st.v)
    rc = np.random.default_rng(12).uniform(2.5, 4.0, st.n)
    s.set_cutoffs(rc)
    fo = s.forces()
    x, _, rcg, _ = s.state()
    torch.cuda.synchronize()
    s.check()
    xw = x.cpu().numpy()
    assert np.array_equal(rcg.cpu().numpy(), rc)
    L = st.box[0]
    top = np.nonzero((xw[2] > L - 2.0) & (xw[1] > L - 2.0))[0]
    low = np.nonzero((xw[2] < 2.0) & (xw[1] < 2.0))[0]
    rng = np.random.default_rng(13)
    idx = np.unique(np.concatenate([rng.choice(top, 400, replace=False), rng.choice(low, 200, replace=False),
                                    rng.choice(st.n, 400, replace=False)]))
    say(f"largest: oracle forces on {idx.size} particles")
    ref = O.forces(po, xw, rc, subset=idx)
    f = fo["f"].cpu().numpy()[:, idx]
    frms = np.sqrt(np.mean(np.sum(ref.f ** 2, axis=0)))
    err = np.linalg.norm(f - ref.f, axis=0) / np.maximum(np.linalg.norm(ref.f, axis=0), frms)
    say(f"largest: max sampled force error {err.max():.2e}")
    assert err.max() <= FORCE_TOL
    assert np.array_equal(fo["pairs"].cpu().numpy()[idx].astype(np.int64), ref.pairs)
    s.close()
    del s, fo, x, rcg
    torch.cuda.empty_cache()
