"""Neighbour-list mode (Verlet lists with a skin, Alg. 3.3) against the CPU oracle and the
direct cell traversal.

The lists hold every slot within r_c[i] + skin at their build and are rebuilt when twice the
largest displacement plus the largest cutoff growth exceeds the skin, so they give the pairs of
the pair rule exactly: pair counts equal the oracle's, forces meet the force bar (the sums run
in list order instead of traversal order).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_1502_03234_amd import dcm, synth  # noqa: E402

from test_gpu_parity import FORCE_TOL, check_system, force_err, make, say  # noqa: E402


@pytest.mark.parametrize("kw", [dict(), dict(rc_min=3.0, rc_max=5.0, energy_shift=1),
                                dict(rc_min=3.0, rc_max=3.0)])
def test_list_parity_slab16k(slab16k, kw):
    p, po = make(slab16k, neighbor_list=1, skin=0.3, **kw)
    s = check_system(slab16k, p, po, f"slab16k lists {kw}")
    assert dcm.dcm_list_builds(s.h) == 1
    s.close()


def test_list_parity_ragged():
    st = synth.small_slab(3000, (16.0, 16.0, 28.0), 1)
    p, po = make(st, neighbor_list=1, skin=0.5)
    check_system(st, p, po, "slab3000 lists").close()


@pytest.mark.parametrize("skin", [0.02, 0.3])
def test_list_steps_match_oracle(slab16k, skin):
    """Steps across list rebuilds (a thin skin rebuilds almost every step) and detections:
    positions and pair counts against the oracle's run."""
    p, po = make(slab16k, neighbor_list=1, skin=skin)
    s = dcm.System(p, slab16k.x, slab16k.v)
    x0, v0, rc0, _ = s.state()
    f0 = s.forces()["f"]
    torch.cuda.synchronize()
    st = O.RunState(x0.cpu().numpy(), v0.cpu().numpy(), rc0.cpu().numpy(), f0.cpu().numpy(), 0)
    th = dcm.thermo_records(s.step(6))
    x, v, rc, k = s.state()
    torch.cuda.synchronize()
    builds = dcm.dcm_list_builds(s.h)
    say(f"lists skin {skin}: {builds} builds in 6 steps")
    ot = O.run(po, st, 6)
    assert np.max(np.abs(x.cpu().numpy() - st.x)) < 1e-11
    assert np.max(np.abs(v.cpu().numpy() - st.v)) < 1e-9
    for a, b in zip(th, ot):
        assert a["pairs"] == b["pairs"]
        assert abs(a["pe"] - b["pe"]) < 1e-10 * abs(b["pe"])
    if skin < 0.05:
        assert builds >= 4
    else:
        # cutoffs change at each detection (every 2nd step) and may outgrow the skin there;
        # between detections the lists hold
        assert builds <= 1 + 6 // 2
    s.close()


def test_list_equals_traversal_over_many_steps(slab16k):
    """40 steps with lists and with the cell traversal from the same state: the same pair
    counts every step and trajectories that agree to rounding growth."""
    pa, _ = make(slab16k)
    pb, _ = make(slab16k, neighbor_list=1, skin=0.3)
    a, b = dcm.System(pa, slab16k.x, slab16k.v), dcm.System(pb, slab16k.x, slab16k.v)
    ta = dcm.thermo_records(a.step(40))
    tb = dcm.thermo_records(b.step(40))
    xa, _, _, _ = a.state()
    xb, _, _, _ = b.state()
    torch.cuda.synchronize()
    builds = dcm.dcm_list_builds(b.h)
    say(f"40 steps: {builds} list builds")
    assert 1 < builds < 40
    assert [r["pairs"] for r in ta] == [r["pairs"] for r in tb]
    assert torch.max(torch.abs(xa - xb)).item() < 1e-9
    a.close()
    b.close()


def test_list_nvt_and_precision_form(slab16k):
    p, po = make(slab16k, neighbor_list=1, skin=0.3, thermostat=dcm.DCM_NOSE_HOOVER, temperature=0.7,
                 tdamp=0.1)
    s = dcm.System(p, slab16k.x, slab16k.v * 1.2)
    x0, v0, rc0, _ = s.state()
    f0 = s.forces()["f"]
    torch.cuda.synchronize()
    st = O.RunState(x0.cpu().numpy(), v0.cpu().numpy(), rc0.cpu().numpy(), f0.cpu().numpy(), 0)
    th = dcm.thermo_records(s.step(3))
    x, _, _, _ = s.state()
    torch.cuda.synchronize()
    ot = O.run(po, st, 3)
    assert np.max(np.abs(x.cpu().numpy() - st.x)) < 1e-12
    assert [r["pairs"] for r in th] == [r["pairs"] for r in ot]
    s.close()
    p, po = make(slab16k, neighbor_list=1, skin=0.3, precision=dcm.DCM_FP32C)
    s = dcm.System(p, slab16k.x, slab16k.v)
    fo = s.forces()
    x, _, rc, _ = s.state()
    torch.cuda.synchronize()
    ref = O.forces(po, x.cpu().numpy(), rc.cpu().numpy())
    assert force_err(fo["f"].cpu().numpy(), ref.f).max() <= 1e-5
    assert np.array_equal(fo["pairs"].cpu().numpy().astype(np.int64), ref.pairs)
    s.close()


def test_list_set_cutoffs_and_tail(slab16k):
    """New cutoffs outgrow the lists, which are rebuilt; with the tail correction on top."""
    p, po = make(slab16k, neighbor_list=1, skin=0.3, tail=1, rc_min=3.0, rc_max=5.0)
    s = dcm.System(p, slab16k.x, slab16k.v)
    rng = np.random.default_rng(3)
    rc = rng.uniform(3.0, 5.0, slab16k.n)
    s.set_cutoffs(rc)
    fo = s.forces()
    x, _, rcg, _ = s.state()
    torch.cuda.synchronize()
    assert dcm.dcm_list_builds(s.h) == 2
    xw = x.cpu().numpy()
    ref = O.forces(po, xw, rc).f + O.tail(po, O.detect(po, xw), xw, rc)[0]
    assert force_err(fo["f"].cpu().numpy(), ref).max() <= FORCE_TOL
    s.close()


def test_list_errors(slab16k):
    p = dcm.params(slab16k.box, neighbor_list=1, skin=0.3, list_capacity=20)
    with pytest.raises(dcm.DcmError) as ei:
        dcm.System(p, slab16k.x, slab16k.v)
    assert ei.value.status == dcm.DCM_E_INVALID and "list_capacity" in str(ei.value)
    for kw in (dict(pair_rule=dcm.DCM_PAIR_MAX), dict(skin=0.0), dict(skin=-1.0), dict(skin=9.0)):
        q = dcm.params(slab16k.box, neighbor_list=1, **{**dict(skin=0.3), **kw})
        with pytest.raises(dcm.DcmError) as ei:
            dcm.System(q, slab16k.x, slab16k.v)
        assert ei.value.status == dcm.DCM_E_INVALID
    pool = dcm.workspace(1 << 28)
    sv = dcm.dcm_server_create(1 << 28, pool)
    with pytest.raises(dcm.DcmError):
        dcm.dcm_submit(sv, dcm.params(slab16k.box, neighbor_list=1), slab16k.x, slab16k.v, 2)
    dcm.dcm_server_destroy(sv)
