"""Parity of the exact reference forces of the accuracy measure (Eq. 20, Section 6.1.1) with
the oracle's image sum: full Lennard-Jones over every periodic image within R, R beyond half the
box. Bar: per atom |dF_i| / max(|F_i|, F_rms) <= 1e-12 (the force bar of the hot path; both
sides sum the same terms in different orders) and per-atom energies within 1e-12 of max(|e|, 1).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_1502_03234_amd import dcm, synth  # noqa: E402

TOL = 1e-12


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def rel_err(f, ref):
    frms = np.sqrt(np.mean(np.sum(ref ** 2, axis=0)))
    return np.linalg.norm(f - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), frms)


def test_exact_forces_small_slab_all_particles():
    st = synth.small_slab(600, (14.0, 14.0, 18.0), seed=31)
    R = 9.0                                             # beyond half the box: images of j and of i
    say(f"exact forces: small slab n={st.n} R={R}")
    s = dcm.System(dcm.params(st.box, rc_min=2.5, rc_max=5.5), st.x, st.v)
    f, e = s.exact_forces(R, energy=True)
    x, _, _, _ = s.state()
    torch.cuda.synchronize()
    s.check()
    ref_f, ref_e = O.forces_images(O.params(st.box), x.cpu().numpy(), R)
    assert rel_err(f.cpu().numpy(), ref_f).max() <= TOL
    assert np.all(np.abs(e.cpu().numpy() - ref_e) <= TOL * np.maximum(np.abs(ref_e), 1.0))
    s.close()


def test_exact_forces_thesis_geometry_sampled():
    st = synth.named("thesis16k")
    R = 14.0
    say(f"exact forces: thesis16k n={st.n} R={R}, 150 sampled particles")
    s = dcm.System(dcm.params(st.box), st.x, st.v)
    f = s.exact_forces(R)
    x, _, _, _ = s.state()
    torch.cuda.synchronize()
    xw = x.cpu().numpy()
    rng = np.random.default_rng(3)
    # particles of the two interfaces (|z - 44| near 22) and of the bulk
    z = xw[2]
    face = np.nonzero(np.abs(np.abs(z - 44.0) - 22.0) < 2.0)[0]
    idx = np.sort(np.concatenate([rng.choice(st.n, 100, replace=False), rng.choice(face, 50, replace=False)]))
    ref_f, _ = O.forces_images(O.params(st.box), xw, R, subset=idx)
    got = f.cpu().numpy()[:, idx]
    frms = np.sqrt(np.mean(np.sum(ref_f ** 2, axis=0)))
    err = np.linalg.norm(got - ref_f, axis=0) / np.maximum(np.linalg.norm(ref_f, axis=0), frms)
    assert err.max() <= TOL, err.max()
    s.close()


def test_exact_forces_below_half_box_equal_static_cutoff():
    """For R below half the box only nearest images lie within R: the image sum equals the
    static-cutoff force of Alg. 3.2 with r_c = R and unshifted energy (both on the GPU)."""
    st = synth.small_slab(2000, (16.0, 16.0, 24.0), seed=32)
    R = 5.0
    say(f"exact forces vs static cutoff: n={st.n} R={R}")
    s = dcm.System(dcm.params(st.box, rc_min=R, rc_max=R), st.x, st.v)
    f, e = s.exact_forces(R, energy=True)
    fo = s.forces(per_atom=True, thermo=False)
    torch.cuda.synchronize()
    assert rel_err(f.cpu().numpy(), fo["f"].cpu().numpy()).max() <= TOL
    ref_e = fo["e"].cpu().numpy()
    assert np.all(np.abs(e.cpu().numpy() - ref_e) <= TOL * np.maximum(np.abs(ref_e), 1.0))
    s.close()


def test_exact_forces_rejects_bad_radius():
    st = synth.small_slab(600, (14.0, 14.0, 18.0), seed=31)
    s = dcm.System(dcm.params(st.box, rc_min=2.5, rc_max=5.5), st.x, st.v)
    out = torch.empty((3, st.n), dtype=torch.float64, device="cuda")
    for R in (0.0, -1.0, float("nan"), float("inf"), 5000.0):
        with pytest.raises(dcm.DcmError) as ei:
            dcm.dcm_exact_forces(s.h, R, s.stream, f=out)
        assert ei.value.status == dcm.DCM_E_INVALID
    s.close()
