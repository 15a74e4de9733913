"""The seeded input generator: sizes, determinism and the slab/droplet recipe."""
import numpy as np

from paper_1502_03234_amd import synth


def test_slab16k_recipe():
    s = synth.named("slab16k")
    assert s.n == 16000 and s.n_liquid == 15680 and s.n_vapor == 320
    assert s.meta["lattice"] == (16, 16, 31) and s.meta["n_sites"] == 15872
    box = np.array(s.box)[:, None]
    assert np.all((s.x >= 0) & (s.x < box))
    liq, vap = s.x[:, :s.n_liquid], s.x[:, s.n_liquid:]
    assert np.all(np.abs(liq[2] - 30) < 12.5 + 0.05 + 1e-12)
    assert np.all(np.abs(vap[2] - 30) >= 12.5)
    # zero net momentum, exact T* over 3N - 3 degrees of freedom
    assert np.allclose(s.v.sum(axis=1), 0, atol=1e-9)
    assert abs(np.sum(s.v ** 2) / (3 * s.n - 3) - 0.7) < 1e-12


def test_vapor_exclusion_and_determinism():
    from scipy.spatial import cKDTree
    a = synth.small_slab(3000, (18.0, 18.0, 40.0), seed=9)
    b = synth.small_slab(3000, (18.0, 18.0, 40.0), seed=9)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)
    tree = cKDTree(a.x.T, boxsize=np.array(a.box))
    d, _ = tree.query(a.x[:, a.n_liquid:].T, k=2)
    assert np.all(d[:, 1] >= 1.0)
    c = synth.small_slab(3000, (18.0, 18.0, 40.0), seed=10)
    assert not np.array_equal(a.x, c.x)


def test_splitmix64_reference_values():
    # SplitMix64 with state 0: the first outputs of the published generator
    r = synth.SplitMix64(0)
    r.state = 0
    assert [int(v) for v in r.next_u64(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_serving_trace_sizes():
    tr = synth.serving_trace(1)
    ns = np.array([t[0] for t in tr])
    assert len(tr) == 64 and ns.min() >= 4000 and ns.max() <= 200000
    s = synth.serving_system(0, 4000, 0.7)
    assert s.box == (14.0, 14.0, 60.0) and s.n == int(round(0.8 * 196 * 25)) + int(round(0.011662 * 196 * 35))
