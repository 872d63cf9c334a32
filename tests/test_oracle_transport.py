"""Pins of the oracle's photon transport (CPU only).

Closed forms the Monte Carlo must reproduce: isotropic emission, 180-degree
back-to-back photons, narrow-beam attenuation exp(-mu L) through a crystal and
through a phantom slab stack (which exercises the Woodcock majorant and the
real/virtual acceptance), the solid-angle efficiency of a ring of ideal
absorbers, energy conservation per photon, and the paper's split-layer
invariance (one 20 mm layer versus two aligned 10 mm layers, Sec. 3.1).
"""
import math

import numpy as np
import pytest
from scipy import stats

import gpet_inputs as G

V_STEP, V_ENTER_PANEL, V_EXIT, V_ESCAPE, V_DEAD, V_ENTER_PHANTOM, V_EMIT = range(7)


def _z(k, n, p):
    return (k - n * p) / math.sqrt(n * p * (1 - p))


def test_isotropic_back_to_back(oracle_mod):
    s = oracle_mod.OracleScene(G.ring8_scene(n_events=20000))
    v = s.trace(20000)
    em = v[v["kind"] == V_EMIT]
    a = em[em["photon"] == 0]
    b = em[em["photon"] == 1]
    assert len(a) == len(b) == 20000
    da = np.stack([a["dx"], a["dy"], a["dz"]], 1)
    db = np.stack([b["dx"], b["dy"], b["dz"]], 1)
    assert np.array_equal(db, -da)  # exactly opposite
    np.testing.assert_allclose(np.linalg.norm(da, axis=1), 1.0, atol=1e-15)
    assert stats.kstest(da[:, 2], stats.uniform(-1, 2).cdf).pvalue > 0.01
    phi = np.arctan2(da[:, 1], da[:, 0])
    assert stats.kstest(phi, stats.uniform(-math.pi, 2 * math.pi).cdf).pvalue > 0.01


def test_first_hits_collinear_with_source(oracle_mod):
    """Both photons reach their panels along one line through the source."""
    pos = (3.0, -2.0, 1.0)
    sc = G.ring8_scene(n_events=20000, source=G.point_source(pos, 20000))
    v = oracle_mod.OracleScene(sc).trace(20000)
    ent = v[v["kind"] == V_ENTER_PANEL]
    first = {}
    for r in ent:
        first.setdefault((r["event"], r["photon"]), np.array([r["x"], r["y"], r["z"]]))
    x = np.array(pos)
    n = 0
    for ev in range(20000):
        if (ev, 0) in first and (ev, 1) in first:
            pa, pb = first[(ev, 0)] - x, first[(ev, 1)] - x
            assert np.linalg.norm(np.cross(pa, pb)) <= 1e-9 * np.linalg.norm(pa) * np.linalg.norm(pb)
            assert np.dot(pa, pb) < 0
            n += 1
    assert n > 100


def _beam_scene(phantom=None, beam_pos=(0.0, 0.8, 0.8)):
    """Pencil beam along +x through the centre of crystal (4, 4) of panel 0 of
    the 8-panel ring (1.5 mm crystals at 1.6 mm pitch, 10 mm LYSO at 7.1)."""
    sc = G.ring8_scene(n_events=10)
    sc["source"] = G.beam_source(beam_pos, (1.0, 0.0, 0.0))
    if phantom is not None:
        sc["materials"] = sc["materials"] + [G.material("water")]
        sc["phantom"] = phantom
    return sc


def _photon_a_collided(v, region):
    a = v[(v["photon"] == 0) & (v["kind"] == V_STEP) & (v["region"] == region) & (v["accept"] == 1)]
    return np.unique(a["event"])


@pytest.mark.parametrize("analog", [False, True], ids=["woodcock", "analog"])
def test_narrow_beam_crystal_transmission(oracle_mod, analog):
    n = 200_000
    s = oracle_mod.OracleScene(_beam_scene())
    v = s.trace(n, analog=analog)
    coll = _photon_a_collided(v, 1)
    p = math.exp(-s.mu(0, 511.0).sum() * 10.0)
    assert p == pytest.approx(0.45262, abs=5e-5)  # 0.7927 /cm over 10 mm
    assert abs(_z(n - len(coll), n, p)) < 4
    # every first collision sits inside the crystal and picks PE with probability mu_pe/mu
    a = v[(v["photon"] == 0) & (v["kind"] == V_STEP) & (v["region"] == 1) & (v["accept"] == 1)]
    _, first = np.unique(a["event"], return_index=True)
    f = a[first]
    assert np.all(f["mat"] == 0)
    frac = s.mu(0, 511.0)[0] / s.mu(0, 511.0).sum()
    assert abs(_z((f["process"] == 1).sum(), len(f), frac)) < 4


@pytest.mark.parametrize("analog", [False, True], ids=["woodcock", "analog"])
def test_narrow_beam_phantom_slabs(oracle_mod, analog):
    """20 mm water then 5 mm LYSO at 3 g/cm^3: uncollided fraction
    exp(-(mu_w 20 + mu_L 5)); the LYSO slab sets the majorant, so water voxels
    take the virtual-collision branch most of the time (Woodcock); analog
    flights cross the voxel faces instead."""
    ph = G.slab_phantom([2, 0], [20.0, 5.0], [1.0, 3.0])
    s = oracle_mod.OracleScene(_beam_scene(ph, beam_pos=(-1.0, 0.1, 0.1)))
    n = 200_000
    v = s.trace(n, analog=analog)
    coll = _photon_a_collided(v, 0)
    mu_w = s.mu(2, 511.0).sum()                # water at 1.0 g/cm^3
    mu_l = s.mu(0, 511.0).sum() / 7.1 * 3.0    # LYSO scaled to 3 g/cm^3
    p = math.exp(-(mu_w * 20.0 + mu_l * 5.0))
    assert abs(_z(n - len(coll), n, p)) < 4
    virt = v[(v["kind"] == V_STEP) & (v["region"] == 0) & (v["accept"] == 0)]
    assert (len(virt) == 0) if analog else (len(virt) > 0)


@pytest.mark.parametrize("case", ["ring8", "ring12"])
def test_black_ring_solid_angle(oracle_mod, case):
    """Ideal absorbers on a ring, centred point source: for an even panel count
    the pair efficiency equals n * Omega / (4 pi), Omega the solid angle of one
    rectangular face (half-sides a, b at distance D) seen on its axis."""
    if case == "ring8":
        sc = G.black_ring_scene(8, 40.0, 12.8, 12.8, 10.0, density=7.1e4)
        a, b, D, want = 6.4, 6.4, 40.0, 0.0635693
    else:
        sc = G.black_ring_scene(12, 65.0, 24.0, 102.0, 20.0)
        a, b, D, want = 12.0, 51.0, 65.0, 0.428965
    n_pan = sc["scanner"]["n_panels"]
    omega = 4 * math.asin(a * b / math.sqrt((a * a + D * D) * (b * b + D * D)))
    eta = n_pan * omega / (4 * math.pi)
    assert eta == pytest.approx(want, abs=1e-6)
    n = 1_000_000
    s = oracle_mod.OracleScene(sc)
    hits, _ = s.transport(n)
    per_event = np.bincount(hits["event"], minlength=n)
    both = np.zeros(n, bool)
    ph = np.zeros((n, 2), bool)
    ph[hits["event"], hits["photon"]] = True
    both = ph[:, 0] & ph[:, 1]
    assert per_event.max() <= 2
    assert abs(_z(both.sum(), n, eta)) < 4
    # digitizer: both 511 keV singles pass the 350-650 keV window with probability
    # Phi(139/sigma) - Phi(-161/sigma), sigma = 0.16*511/2.3548
    sig = 0.16 * 511.0 / (2 * math.sqrt(2 * math.log(2)))
    acc = stats.norm.cdf(139 / sig) - stats.norm.cdf(-161 / sig)
    assert acc == pytest.approx(0.999967, abs=1e-6)
    if case == "ring8":
        singles, coinc = s.digitize(hits)
        assert abs(_z(len(coinc), n, eta * acc * acc)) < 4


def test_energy_conservation(oracle_mod):
    sc = G.small_animal_scene("C", n_events=5000)
    v = oracle_mod.OracleScene(sc).trace(5000)
    key = v["event"].astype(np.int64) * 2 + v["photon"]
    dep = np.bincount(key, weights=np.where(v["kind"] == V_STEP, v["edep"], 0.0), minlength=10000)
    esc = np.bincount(key, weights=np.where(v["kind"] == V_ESCAPE, v["e"], 0.0), minlength=10000)
    np.testing.assert_allclose(dep + esc, 511.0, atol=1e-9)
    # every photon ends exactly once: escaped or dead
    ends = np.bincount(key, weights=np.isin(v["kind"], [V_ESCAPE, V_DEAD]), minlength=10000)
    assert np.all(ends == 1)


def test_split_layer_invariance(oracle_mod):
    """Design A (one 20 mm layer) and B0 (two aligned 10 mm layers, no gap) hold
    the same material everywhere, so RNG-matched histories are identical and
    only the layer label changes (1CL versus 1CL-split, Sec. 3.1)."""
    n = 20000
    ha, _ = oracle_mod.OracleScene(G.small_animal_scene("A", n_events=n)).transport(n, seed=4)
    hb, _ = oracle_mod.OracleScene(G.small_animal_scene("B0", n_events=n)).transport(n, seed=4)
    assert len(ha) == len(hb) > 1000
    for f in ("event", "photon", "seq", "panel", "module", "crystal", "process", "edep", "tof_ps",
              "depth", "t", "a", "time_ps"):
        assert np.array_equal(ha[f], hb[f]), f
    assert np.all(ha["layer"] == 0)
    assert np.array_equal(hb["layer"], (hb["depth"] >= 10.0).astype(np.uint32))


def test_offset_design_doi_trend(oracle_mod):
    """The offset design's inner layer holds 23x23 instead of 24x24 crystals:
    fewer shallow hits, about the same deep ones (Fig. 3 trend)."""
    n = 100_000
    h = {d: oracle_mod.OracleScene(G.small_animal_scene(d, n_events=n)).transport(n)[0]
         for d in ("A", "C")}
    shallow = (h["C"]["depth"] < 10).sum() / (h["A"]["depth"] < 10).sum()
    deep = (h["C"]["depth"] >= 10).sum() / (h["A"]["depth"] >= 10).sum()
    assert shallow < 0.95
    assert 0.98 < deep < 1.08


def test_chunked_ranges_equal_whole(oracle_mod):
    s = oracle_mod.OracleScene(G.small_animal_scene("C", n_events=4000))
    whole, _ = s.transport(4000, seed=9)
    a, _ = s.transport(1500, seed=9, first=0)
    b, _ = s.transport(2500, seed=9, first=1500)
    cat = np.concatenate([a, b])
    assert np.array_equal(whole, cat)
