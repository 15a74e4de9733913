"""The C-ABI library: it loads, exports every entry point include/dcm.h declares, and its
host-only calls (grid dims, workspace sizes, parameter validation) behave. CPU only."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dcm.h")
LIB = os.path.join(ROOT, "paper_1502_03234_amd", "libdcm.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dcm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def dcm():
    if not os.path.exists(LIB):
        from paper_1502_03234_amd import build
        build.build()
    from paper_1502_03234_amd import dcm as mod
    return mod


def test_header_declares_entry_points():
    syms = declared_symbols()
    for required in ("dcm_create", "dcm_detect_interface", "dcm_compute_forces", "dcm_step",
                     "dcm_get_state", "dcm_destroy", "dcm_workspace_bytes"):
        assert required in syms


def test_library_exports_every_declared_symbol(dcm):
    lib = C.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (dcm_[a-z_0-9]+)$", out, flags=re.M))
    assert set(declared_symbols()) <= exported


def test_binding_covers_header(dcm):
    for s in declared_symbols():
        assert hasattr(dcm, s), s


def test_grid_dims_and_workspace(dcm):
    p = dcm.params((320.0, 320.0, 60.0))
    assert dcm.dcm_grid_dims(p) == (320, 320, 60)
    b = dcm.dcm_workspace_bytes(p, 2_048_000)
    assert 400e6 < b < 2e9
    p2 = dcm.params((28.0, 28.0, 60.0))
    assert dcm.dcm_workspace_bytes(p2, 16000) < b
    assert dcm.dcm_version().startswith("dcm-mi355x")


@pytest.mark.parametrize("bad", [
    dict(rc_max=7.0, box=(14.0, 14.0, 60.0)),          # rc_max >= L/2
    dict(rc_min=3.0, rc_max=2.5),                      # rc_min > rc_max
    dict(alpha=0.0),                                   # flat cutoff function
    dict(smooth_passes=5),
    dict(box=(13.0, 28.0, 60.0)),                      # 13 boxes < 2 ceil(6/1) + 2
    dict(dt=0.0),
    dict(precision=7),
    dict(pair_rule=3),
    dict(min_component=-1),
    dict(thermostat=2),
    dict(thermostat=1, temperature=0.0),
    dict(thermostat=1, tdamp=-1.0),
    dict(thermostat=1, tdamp=float("inf")),
    dict(tail=2),                                      # options: flags are 0 or 1
    dict(tail=1, pair_rule=1),                         # the tail needs the r_c[i] rule
    dict(tail=1, energy_shift=1),                      # ... and unshifted energies
    dict(vapor_cutoff=3),
    dict(ms_nu=-0.1),
    dict(ms_nu=float("nan")),
    dict(ms_nu=0.005, ms_iters=0),
    dict(ms_nu=0.005, ms_iters=100001),
    dict(neighbor_list=2),
    dict(neighbor_list=1, skin=0.0),
    dict(neighbor_list=1, skin=float("inf")),
    dict(neighbor_list=1, pair_rule=1),
    dict(neighbor_list=1, list_capacity=-1),
    dict(neighbor_list=1, skin=1.5, box=(14.0, 14.0, 60.0), rc_max=5.0),   # r_c^max + skin >= L/2
])
def test_invalid_parameters_rejected(dcm, bad):
    kw = dict(box=(28.0, 28.0, 60.0))
    kw.update(bad)
    box = kw.pop("box")
    p = dcm.params(box, **kw)
    with pytest.raises(dcm.DcmError) as e:
        dcm.dcm_workspace_bytes(p, 1000)
    assert e.value.status == dcm.DCM_E_INVALID
    assert dcm.dcm_last_error()


def test_option_workspaces(dcm):
    """Each option adds its arrays to the workspace: the vapor-side distance field (8 B per box),
    the Mumford-Shah fields (48 B per box), the neighbour lists (a slot capacity per particle,
    default 1.25 (4/3) pi (r_c^max + skin)^3, plus positions at the build and box counts)."""
    box, n = (28.0, 28.0, 60.0), 16000
    G = 28 * 28 * 60
    base = dcm.dcm_workspace_bytes(dcm.params(box), n)
    tail = dcm.dcm_workspace_bytes(dcm.params(box, tail=1), n)
    vap = dcm.dcm_workspace_bytes(dcm.params(box, vapor_cutoff=1), n)
    ms = dcm.dcm_workspace_bytes(dcm.params(box, ms_nu=0.005), n)
    lists = dcm.dcm_workspace_bytes(dcm.params(box, neighbor_list=1, skin=0.3), n)
    small = dcm.dcm_workspace_bytes(dcm.params(box, neighbor_list=1, skin=0.3, list_capacity=100), n)
    assert tail >= base + 8 * G and vap >= base + 8 * G
    assert ms >= base + 48 * G
    import math
    cap = math.ceil(1.25 * 4.0 / 3.0 * math.pi * 6.3 ** 3)
    assert lists >= base + 4 * cap * n + 4 * n + 32 * n + 4 * G
    assert small < lists and small >= base + 4 * 100 * n


def test_invalid_n_and_workspace(dcm):
    p = dcm.params((28.0, 28.0, 60.0))
    with pytest.raises(dcm.DcmError) as e:
        dcm.dcm_workspace_bytes(p, 1)
    assert e.value.status == dcm.DCM_E_INVALID
    # positions are addressed with 32-bit byte offsets: n stays below 2^26
    assert dcm.dcm_workspace_bytes(p, (1 << 26) - 1) > 0
    with pytest.raises(dcm.DcmError) as e:
        dcm.dcm_workspace_bytes(p, 1 << 26)
    assert e.value.status == dcm.DCM_E_INVALID
    # a missing workspace is rejected before any device work
    h = C.c_void_p()
    st = dcm._lib.dcm_create(C.byref(p), 1000, None, 0, None, None, None, C.byref(h))
    assert st in (dcm.DCM_E_INVALID, dcm.DCM_E_WORKSPACE)
    x = C.c_void_p(256)
    st = dcm._lib.dcm_create(C.byref(p), 1000, x, 10, x, x, None, C.byref(h))
    assert st == dcm.DCM_E_WORKSPACE and h.value is None


def test_grid_stage_argument_checks(dcm):
    with pytest.raises(dcm.DcmError) as e:
        dcm.dcm_grid_workspace_bytes((2, 5, 5))
    assert e.value.status == dcm.DCM_E_INVALID
    assert dcm.dcm_grid_workspace_bytes((5, 5, 5)) > 0
