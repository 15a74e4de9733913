"""Parity of the Mumford-Shah segmentation (Eq. 13) on the HIP path with the CPU oracle.

The primal-dual iterations are per-box stencils with fused multiply-adds off on both sides, so
the labels before and after component removal are compared bit for bit, and everything
downstream (distances, cutoffs, forces) to the bars of the plain path.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_1502_03234_amd import dcm, synth  # noqa: E402

from test_gpu_parity import _eager, _serve, check_system, make  # noqa: E402


@pytest.mark.parametrize("kw", [dict(ms_nu=0.005, ms_iters=200),
                                dict(ms_nu=0.001, ms_iters=50, smooth_passes=0, bin=2.6, min_component=5,
                                     rc_min=3.0, rc_max=5.0)])
def test_ms_slab16k(slab16k, kw):
    p, po = make(slab16k, **kw)
    check_system(slab16k, p, po, f"slab16k Mumford-Shah {kw}").close()


def test_ms_thesis_geometry_and_ragged():
    st = synth.named("thesis16k")
    p, po = make(st, ms_nu=0.005, ms_iters=150, smooth_passes=0, bin=2.6, min_component=5,
                 rc_min=3.0, rc_max=5.0)
    check_system(st, p, po, "thesis16k Mumford-Shah 2.6-sigma boxes").close()
    st = synth.small_slab(3000, (16.0, 16.0, 28.0), 1)
    p, po = make(st, ms_nu=0.003, ms_iters=77)
    check_system(st, p, po, "slab3000 Mumford-Shah").close()


def test_ms_flattens_the_slab(slab16k):
    """At nu = 0.005 the raw labels of the 16k slab are two flat planes (2 N_x N_y faces)."""
    p, _ = make(slab16k, ms_nu=0.005, ms_iters=200)
    s = dcm.System(p, slab16k.x, slab16k.v)
    det = s.detect()
    torch.cuda.synchronize()
    nx, ny, nz = s.dims
    raw = det["raw"].cpu().numpy().reshape(nz, ny, nx).astype(np.int64)
    faces = sum(int(np.abs(np.roll(raw, -1, ax) - raw).sum()) for ax in range(3))
    assert faces == 2 * nx * ny
    s.close()


def test_ms_steps_and_served_bits():
    """Steps with the segmentation on: served (recorded, batched) launches give the eager bits."""
    reqs = []
    for j, (n, box, ns) in enumerate([(3000, (16.0, 16.0, 28.0), 5), (4000, (16.0, 16.0, 32.0), 4)]):
        st = synth.small_slab(n, box, 500 + j)
        reqs.append((dcm.params(st.box, rc_min=2.5, rc_max=4.0, ms_nu=0.004, ms_iters=40), st, ns))
    got, stats = _serve(reqs, budget=1 << 31, pool_bytes=1 << 31)
    assert stats["completed"] == len(reqs)
    for (p, st, ns), (status, x, v, th) in zip(reqs, got):
        ex, ev, eth = _eager(p, st, ns)
        assert np.array_equal(x, ex) and np.array_equal(v, ev)


def test_ms_invalid(slab16k):
    for kw in (dict(ms_nu=-0.1), dict(ms_nu=0.005, ms_iters=0), dict(ms_nu=float("nan"))):
        p = dcm.params(slab16k.box, **kw)
        with pytest.raises(dcm.DcmError) as ei:
            dcm.System(p, slab16k.x, slab16k.v)
        assert ei.value.status == dcm.DCM_E_INVALID
