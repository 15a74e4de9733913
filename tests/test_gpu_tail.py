"""Parity of the runtime tail correction (Eq. 21-22), and of the dynamic cutoffs for vapor
particles (Section 3.1) that share its vapor-side distance field, with the CPU oracle.

The oracle's tail (radial quadrature of Eq. 22 and of its force over a planar two-phase model)
is evaluated on the GPU's own wrapped positions and cutoffs, with the oracle's own detection
fields. Bars: the vapor-side box distances within the distance bar of the interface
distances; forces (pair + tail) per atom within 1e-12 of max(|F_i|, F_rms); per-atom energies
within 1e-12; energy sums within 1e-12 of the sum of absolute terms.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_1502_03234_amd import dcm, synth  # noqa: E402

from test_gpu_parity import (FORCE_TOL, _eager, _serve, check_system, dist_ulps, force_err,  # noqa: E402
                             make, rc_close, say, sum_close, ulp_close)


def _tail_case(state, name, **kw):
    p, po = make(state, tail=1, **kw)
    say(f"{name}: n={state.n} {kw}")
    s = dcm.System(p, state.x, state.v)
    det = s.detect()
    fo = s.forces()
    x, _, rc, _ = s.state()
    torch.cuda.synchronize()
    s.check()
    xw, rcg = x.cpu().numpy(), rc.cpu().numpy()
    od = O.detect(po, xw)
    assert np.array_equal(det["label"].cpu().numpy(), od.label)
    assert np.array_equal(det["km"].cpu().numpy(), od.km)
    bar = dist_ulps(2 * p.rc_max + 1.0, 1.0)          # the tail correction's band
    assert ulp_close(det["dist"].cpu().numpy(), od.dist, bar), "interface distances"
    assert ulp_close(det["dist_v"].cpu().numpy(), od.dist_v, bar), "vapor-side distances"
    pair = O.forces(po, xw, rcg)
    ft, du = O.tail(po, od, xw, rcg)
    ref_f = pair.f + ft
    err = force_err(fo["f"].cpu().numpy(), ref_f)
    tail_rms = np.sqrt(np.mean(np.sum(ft ** 2, axis=0)))
    say(f"{name}: max force error {err.max():.2e}; tail force rms {tail_rms:.3e}, "
        f"tail energy {0.5 * du.sum() / state.n:.5f} per particle")
    assert err.max() <= FORCE_TOL
    assert tail_rms > 0.0
    ref_e = pair.e + 0.5 * du
    e = fo["e"].cpu().numpy()
    assert np.all(np.abs(e - ref_e) <= 1e-12 * np.maximum(np.abs(ref_e), 1.0))
    th = dcm.thermo_records(fo["thermo"])[0]
    assert sum_close(th["pe"], ref_e)
    # the virial holds the pair terms only
    for c in range(6):
        assert sum_close(th["virial"][c], pair.w[c])
    return s


@pytest.mark.parametrize("kw", [dict(rc_min=3.0, rc_max=5.0), dict(rc_min=3.0, rc_max=3.0),
                                dict(rc_min=2.5, rc_max=6.0, cutoff_shape=1)])
def test_tail_parity_slab16k(slab16k, kw):
    _tail_case(slab16k, "slab16k tail", **kw).close()


def test_tail_parity_ragged_and_smoothing():
    st = synth.small_slab(3000, (16.0, 16.0, 28.0), 1)
    _tail_case(st, "slab3000 tail", rc_min=2.5, rc_max=4.0).close()
    st = synth.small_slab(40000, (41.0, 37.0, 52.0), 3)
    _tail_case(st, "slab40000 tail 2 passes", rc_min=3.0, rc_max=5.0, smooth_passes=2).close()


def test_tail_removes_the_pair_difference(slab16k):
    """System with and without the correction: the difference of the forces is the oracle's
    tail force alone."""
    p0, _ = make(slab16k, rc_min=3.0, rc_max=5.0)
    p1, po = make(slab16k, rc_min=3.0, rc_max=5.0, tail=1)
    a, b = dcm.System(p0, slab16k.x, slab16k.v), dcm.System(p1, slab16k.x, slab16k.v)
    fa, fb = a.forces()["f"], b.forces()["f"]
    x, _, rc, _ = b.state()
    torch.cuda.synchronize()
    xw, rcg = x.cpu().numpy(), rc.cpu().numpy()
    ft, _ = O.tail(po, O.detect(po, xw), xw, rcg)
    d = (fb - fa).cpu().numpy()
    scale = np.sqrt(np.mean(np.sum(ft ** 2, axis=0)))
    assert np.max(np.linalg.norm(d - ft, axis=0)) <= 1e-9 * scale
    a.close()
    b.close()


def test_tail_steps_match_oracle(slab16k):
    """Three steps with the correction against the oracle's run (detection at step 2)."""
    p, po = make(slab16k, rc_min=3.0, rc_max=5.0, tail=1)
    s = dcm.System(p, slab16k.x, slab16k.v)
    x0, v0, rc0, _ = s.state()
    f0 = s.forces()["f"]
    torch.cuda.synchronize()
    st = O.RunState(x0.cpu().numpy(), v0.cpu().numpy(), rc0.cpu().numpy(), f0.cpu().numpy(), 0)
    # the creation's force (pair + tail) equals the oracle's
    ref0 = O.prepare(po, slab16k.x, slab16k.v)
    assert force_err(st.f, ref0.f).max() <= FORCE_TOL
    th = dcm.thermo_records(s.step(3))
    x1, v1, rc1, k1 = s.state()
    torch.cuda.synchronize()
    ot = O.run(po, st, 3)
    assert k1 == 3
    assert np.max(np.abs(x1.cpu().numpy() - st.x)) < 1e-12
    assert np.max(np.abs(v1.cpu().numpy() - st.v)) < 1e-10
    for a, b in zip(th, ot):
        assert abs(a["pe"] - b["pe"]) < 1e-11 * abs(b["pe"])
        assert a["pairs"] == b["pairs"]
    s.close()


def test_tail_resume_between_detections_matches_oracle(slab16k):
    """A state resumed at an odd step (no detection due) recomputes the distance fields of the
    resumed positions and keeps the cutoffs; the oracle's run does the same at entry."""
    p, po = make(slab16k, rc_min=3.0, rc_max=5.0, tail=1)
    a = dcm.System(p, slab16k.x, slab16k.v)
    a.step(3)
    x, v, rc, k = a.state()
    b = dcm.System(p, x, v, rc=rc, step=k)
    xb, vb, rcb, kb = b.state()
    fb = b.forces()["f"]
    torch.cuda.synchronize()
    assert kb == 3 and torch.equal(rcb, rc)
    xw = xb.cpu().numpy()
    pair = O.forces(po, xw, rcb.cpu().numpy())
    ft, _ = O.tail(po, O.detect(po, xw), xw, rcb.cpu().numpy())
    assert force_err(fb.cpu().numpy(), pair.f + ft).max() <= FORCE_TOL
    st = O.RunState(xw, vb.cpu().numpy(), rcb.cpu().numpy(), fb.cpu().numpy(), 3)
    b.step(2)
    x2, v2, _, _ = b.state()
    torch.cuda.synchronize()
    O.run(po, st, 2)
    assert np.max(np.abs(x2.cpu().numpy() - st.x)) < 1e-12
    assert np.max(np.abs(v2.cpu().numpy() - st.v)) < 1e-10
    a.close()
    b.close()


def test_tail_precision_form(slab16k):
    p, po = make(slab16k, rc_min=3.0, rc_max=5.0, tail=1, precision=dcm.DCM_FP32C)
    s = dcm.System(p, slab16k.x, slab16k.v)
    fo = s.forces()
    x, _, rc, _ = s.state()
    torch.cuda.synchronize()
    xw, rcg = x.cpu().numpy(), rc.cpu().numpy()
    ref = O.forces(po, xw, rcg).f + O.tail(po, O.detect(po, xw), xw, rcg)[0]
    assert force_err(fo["f"].cpu().numpy(), ref).max() <= 1e-5
    s.close()


def test_tail_served_equals_eager():
    """The correction inside the served (recorded, batched) launches gives the eager bits, in a
    batch mixing systems with and without it."""
    reqs = []
    for j, (n, box, ns, tail) in enumerate([(3000, (16.0, 16.0, 28.0), 7, 1), (5617, (14.0, 14.0, 60.0), 6, 0),
                                            (4000, (16.0, 16.0, 32.0), 9, 1)]):
        st = synth.small_slab(n, box, 300 + j)
        reqs.append((dcm.params(st.box, rc_min=2.5, rc_max=4.0, tail=tail), st, ns))
    got, stats = _serve(reqs, budget=1 << 31, pool_bytes=1 << 31)
    assert stats["completed"] == len(reqs)
    for (p, st, ns), (status, x, v, th) in zip(reqs, got):
        ex, ev, eth = _eager(p, st, ns)
        assert np.array_equal(x, ex) and np.array_equal(v, ev)
        assert th["pe"] == eth["pe"]


def test_tail_invalid_combinations(slab16k):
    for kw in (dict(tail=1, pair_rule=dcm.DCM_PAIR_MAX), dict(tail=1, energy_shift=1), dict(tail=2)):
        p = dcm.params(slab16k.box, **kw)
        with pytest.raises(dcm.DcmError) as ei:
            dcm.System(p, slab16k.x, slab16k.v)
        assert ei.value.status == dcm.DCM_E_INVALID
    s = dcm.System(dcm.params(slab16k.box), slab16k.x, slab16k.v)
    G = s.G
    dv = torch.empty(G, dtype=torch.float64, device="cuda")
    with pytest.raises(dcm.DcmError) as ei:
        dcm.dcm_detect_interface(s.h, s.stream, dist_v=dv)
    assert ei.value.status == dcm.DCM_E_INVALID
    s.close()


@pytest.mark.parametrize("kw", [dict(), dict(rc_min=3.0, rc_max=7.0, cutoff_shape=1)])
def test_vapor_cutoffs_parity(slab16k, kw):
    """Vapor particles with dynamic cutoffs: the whole detection and force path against the
    oracle, and the vapor-side distances."""
    p, po = make(slab16k, vapor_cutoff=1, **kw)
    s = check_system(slab16k, p, po, f"slab16k vapor cutoffs {kw}")
    det = s.detect()
    x, _, rc, _ = s.state()
    torch.cuda.synchronize()
    od = O.detect(po, x.cpu().numpy())
    assert ulp_close(det["dist_v"].cpu().numpy(), od.dist_v, dist_ulps(p.rc_max + 1.0, 1.0))
    # some vapor particles got less than r_c^max
    assert (rc.cpu().numpy() < p.rc_max).sum() > (od.d > 0).sum()
    s.close()


def test_vapor_cutoffs_with_tail(slab16k):
    p, po = make(slab16k, rc_min=3.0, rc_max=5.0, vapor_cutoff=1, tail=1)
    s = dcm.System(p, slab16k.x, slab16k.v)
    fo = s.forces(per_atom=False, thermo=False)
    x, _, rc, _ = s.state()
    torch.cuda.synchronize()
    xw, rcg = x.cpu().numpy(), rc.cpu().numpy()
    od = O.detect(po, xw)
    assert rc_close(rcg, od.rc, 3.0, 5.0, -0.5, cap=2 * 5.0 + 1.0, planar=False)   # the tail band
    ref = O.forces(po, xw, rcg).f + O.tail(po, od, xw, rcg)[0]
    assert force_err(fo["f"].cpu().numpy(), ref).max() <= FORCE_TOL
    s.close()
