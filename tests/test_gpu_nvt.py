"""Constant-temperature steps (Nose-Hoover thermostat) of the HIP path against the oracle.

Bars as for the constant-energy steps: after a few steps positions and velocities agree up to
the rounding of the forces, the thermostat state (xi, eta) to 1e-12 relative, the pair counts
exactly. Runs split over several calls, or resumed from a checkpoint through
dcm_get_thermostat / dcm_set_thermostat, give the same bits as one call.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_1502_03234_amd import dcm  # noqa: E402

NVT = dict(thermostat=dcm.DCM_NOSE_HOOVER, temperature=0.7, tdamp=0.1)


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def test_nvt_steps_match_oracle(slab16k):
    say(f"nvt steps vs oracle: n={slab16k.n}")
    p = dcm.params(slab16k.box, **NVT)
    po = O.params(slab16k.box, thermostat=1, temperature=0.7, tdamp=0.1)
    s = dcm.System(p, slab16k.x, slab16k.v * 1.2)
    x0, v0, rc0, _ = s.state()
    f0 = s.forces()["f"]
    torch.cuda.synchronize()
    st = O.RunState(x0.cpu().numpy(), v0.cpu().numpy(), rc0.cpu().numpy(), f0.cpu().numpy(), 0)
    th = dcm.thermo_records(s.step(3))
    x, v, rc, k = s.state()
    xi, eta = s.thermostat()
    torch.cuda.synchronize()
    ot = O.run(po, st, 3)
    assert k == 3
    assert np.max(np.abs(x.cpu().numpy() - st.x)) < 1e-12
    assert np.max(np.abs(v.cpu().numpy() - st.v)) < 1e-10
    for g, o in zip(th, ot):
        assert g["step"] == o["step"] and g["pairs"] == o["pairs"]
        assert rel(g["ke"], o["ke"]) < 1e-11
        assert rel(g["pe"], o["pe"]) < 1e-11
        assert rel(g["xi"], o["xi"]) < 1e-12 and rel(g["eta"], o["eta"]) < 1e-12
    assert ot[-1]["xi"] > 0                      # started hotter than T*: friction switched on
    assert (xi, eta) == (th[-1]["xi"], th[-1]["eta"])
    s.close()


def test_nvt_split_and_resume_bitwise(slab16k):
    p = dcm.params(slab16k.box, **NVT)
    a = dcm.System(p, slab16k.x, slab16k.v)
    tha = a.step(7)
    xa, va, rca, _ = a.state()
    b = dcm.System(p, slab16k.x, slab16k.v)
    b.step(3)
    thb = b.step(4)
    xb, vb, rcb, _ = b.state()
    c0 = dcm.System(p, slab16k.x, slab16k.v)
    c0.step(3)
    x, v, rc, k = c0.state()
    xi, eta = c0.thermostat()
    c = dcm.System(p, x, v, rc=rc, step=k)
    assert c.thermostat() == (0.0, 0.0)
    c.set_thermostat(xi, eta)
    thc = c.step(4)
    xc, vc, rcc, kc = c.state()
    torch.cuda.synchronize()
    assert kc == 7
    for other in ((xb, vb, rcb), (xc, vc, rcc)):
        assert torch.equal(xa, other[0]) and torch.equal(va, other[1]) and torch.equal(rca, other[2])
    last = tha[-dcm.THERMO_DOUBLES:]
    assert torch.equal(last, thb[-dcm.THERMO_DOUBLES:]) and torch.equal(last, thc[-dcm.THERMO_DOUBLES:])
    assert a.thermostat() == b.thermostat() == c.thermostat()
    for s in (a, b, c0, c):
        s.close()


def test_nvt_extended_energy_and_nve_records(slab16k):
    """Static shifted cutoff (no detection) from a hot start: the extended energy stays flat
    while K + U falls; under NVE the records carry xi = eta = 0."""
    kw = dict(rc_min=2.5, rc_max=2.5, detect_every=0, energy_shift=1)
    p = dcm.params(slab16k.box, **kw, **NVT)
    s = dcm.System(p, slab16k.x, slab16k.v * 1.5)
    th = dcm.thermo_records(s.step(100))
    n = slab16k.n
    g = 3 * n - 3
    Q = g * 0.7 * 0.1 ** 2
    E = np.array([t["ke"] + t["pe"] for t in th]) / n
    H = np.array([t["ke"] + t["pe"] + 0.5 * Q * t["xi"] ** 2 + g * 0.7 * t["eta"] for t in th]) / n
    say(f"nvt 100 steps: K+U spread {np.ptp(E):.3e}, extended spread {np.ptp(H):.3e}")
    assert np.ptp(E) > 0.05 and np.max(np.abs(H - H[0])) < 5e-3
    s.close()
    s = dcm.System(dcm.params(slab16k.box, **kw), slab16k.x, slab16k.v)
    th = dcm.thermo_records(s.step(3))
    assert all(t["xi"] == 0.0 and t["eta"] == 0.0 for t in th)
    with pytest.raises(dcm.DcmError):
        s.set_thermostat(float("nan"), 0.0)
    s.close()
