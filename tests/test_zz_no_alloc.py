"""dcm_grid_smooth_noalloc (the smoothing stage with its intermediate image in the library's
device array, for callers that cannot allocate) against dcm_grid_smooth with a caller
workspace: the same integers, bit for bit, on two calls in a row (the second on a smaller grid,
after the first left its values in the shared array), and the size limit rejected on the host."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1502_03234_amd import dcm  # noqa: E402


def _smooth_both(dims, passes, seed):
    G = dims[0] * dims[1] * dims[2]
    rng = np.random.default_rng(seed)
    img = torch.from_numpy(rng.integers(0, 1000, G, dtype=np.uint32).view(np.int32)).cuda()
    ref = torch.empty_like(img)
    got = torch.full_like(img, -1)
    ws = dcm.workspace(dcm.dcm_grid_workspace_bytes(dims))
    dcm.dcm_grid_smooth(dims, passes, img, ref, ws)
    dcm.dcm_grid_smooth_noalloc(dims, passes, img, got)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_smoothing_equals_workspace_entry_point():
    for dims, passes, seed in [((64, 48, 40), 2, 1), ((23, 9, 17), 1, 2), ((5, 4, 3), 3, 3)]:
        print(f"[gpu-test] smoothing without allocation dims={dims} passes={passes}", flush=True)
        ref, got = _smooth_both(dims, passes, seed)
        assert np.array_equal(ref, got), dims


def test_noalloc_smoothing_rejects_grids_beyond_the_scratch():
    img = torch.zeros(8, dtype=torch.int32, device="cuda")
    with pytest.raises(dcm.DcmError) as e:
        dcm.dcm_grid_smooth_noalloc((300, 300, 100), 1, img, img)      # 9,000,000 boxes
    assert e.value.status == dcm.DCM_E_INVALID
    with pytest.raises(dcm.DcmError):
        dcm.dcm_grid_smooth_noalloc((8, 8, 8), 5, img, img)
