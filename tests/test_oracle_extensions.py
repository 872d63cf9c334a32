"""Pins of the oracle's optional physics (CPU only): the effects the paper
switches off or leaves to analytic models (Sec. 2.3: no positron range;
Sec. 4: analytic blurring of the detector response).

* acollinearity: the deviation of photon B from -d, split into two fixed
  transverse components, is normal with the FWHM given per component;
* positron range: each component of the annihilation offset is normal with
  the FWHM given per axis, and both photons start at the same point;
* timing and DOI resolution: time and depth move by a normal deviate of the
  given FWHM (time rounded to the ps);
* light sharing: a moved crystal is an edge neighbour in its layer and
  module, each existing neighbour equally likely, moved with the given
  probability;
* dead time: a brute-force definition on small random inputs, and the
  throughput of a Poisson stream, exp(-rate tau) for the paralyzable and
  1 / (1 + rate tau) for the non-paralyzable model.
"""
import math

import numpy as np
import pytest
from scipy import stats

import gpet_inputs as G

V_EMIT = 6
FWHM = 2.0 * math.sqrt(2.0 * math.log(2.0))


def _emit(oracle_mod, n, **src_extra):
    src = G.point_source((1.0, -2.0, 3.0), n)
    src.update(src_extra)
    v = oracle_mod.OracleScene(G.ring8_scene(n_events=n, source=src)).trace(n)
    em = v[v["kind"] == V_EMIT]
    a, b = em[em["photon"] == 0], em[em["photon"] == 1]
    assert len(a) == len(b) == n
    assert np.array_equal(a["event"], b["event"])
    return a, b


def _dirs(r):
    return np.stack([r["dx"], r["dy"], r["dz"]], 1)


def _pos(r):
    return np.stack([r["x"], r["y"], r["z"]], 1)


def test_acollinearity_zero_is_back_to_back(oracle_mod):
    a, b = _emit(oracle_mod, 2000, acolinearity_fwhm_deg=0.0, positron_range_fwhm_mm=0.0)
    assert np.array_equal(_dirs(b), -_dirs(a))
    assert np.array_equal(_pos(a), _pos(b))
    assert np.all(_pos(a) == np.array([1.0, -2.0, 3.0]))


@pytest.mark.parametrize("fwhm_deg", [0.5, 3.0])
def test_acollinearity_components_are_normal(oracle_mod, fwhm_deg):
    n = 20000
    a, b = _emit(oracle_mod, n, acolinearity_fwhm_deg=fwhm_deg)
    da, db = _dirs(a), _dirs(b)
    np.testing.assert_allclose(np.linalg.norm(db, axis=1), 1.0, atol=1e-14)
    # photon A keeps the isotropic direction; B deviates from -A
    assert stats.kstest(da[:, 2], stats.uniform(-1, 2).cdf).pvalue > 1e-3
    # transverse frame of -A: e1 perpendicular to z, e2 completes it
    m = -da
    e1 = np.cross(np.array([0.0, 0.0, 1.0]), m)
    e1 /= np.linalg.norm(e1, axis=1)[:, None]
    e2 = np.cross(m, e1)
    theta = np.arccos(np.clip(np.sum(db * m, 1), -1.0, 1.0))
    # components of the deviation along e1, e2 (angle times unit direction)
    t = db - np.sum(db * m, 1)[:, None] * m
    tn = np.linalg.norm(t, axis=1)
    c1 = theta * np.sum(t * e1, 1) / tn
    c2 = theta * np.sum(t * e2, 1) / tn
    sig = math.radians(fwhm_deg) / FWHM
    for c in (c1, c2):
        assert stats.kstest(c / sig, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(c1, c2)[0, 1]) < 0.03
    # the deviation angle is Rayleigh distributed
    assert stats.kstest(theta / sig, stats.rayleigh.cdf).pvalue > 1e-3


@pytest.mark.parametrize("fwhm_mm", [0.102, 2.0])
def test_positron_range_offsets_are_normal(oracle_mod, fwhm_mm):
    n = 20000
    a, b = _emit(oracle_mod, n, positron_range_fwhm_mm=fwhm_mm)
    assert np.array_equal(_pos(a), _pos(b))
    assert np.array_equal(_dirs(b), -_dirs(a))  # collinear unless asked
    off = _pos(a) - np.array([1.0, -2.0, 3.0])
    sig = fwhm_mm / FWHM
    for k in range(3):
        assert stats.kstest(off[:, k] / sig, "norm").pvalue > 1e-3
    c = np.corrcoef(off.T)
    assert np.max(np.abs(c - np.eye(3))) < 0.03
    # the radius follows the chi distribution with 3 degrees of freedom
    assert stats.kstest(np.linalg.norm(off, axis=1) / sig, stats.chi(3).cdf).pvalue > 1e-3


def test_positron_range_moves_the_hits(oracle_mod):
    """The offset is the annihilation point: the first panel entries of the
    two photons lie on one line through it, not through the source."""
    n = 4000
    src = G.point_source((0.0, 0.0, 0.0), n)
    src["positron_range_fwhm_mm"] = 4.0
    v = oracle_mod.OracleScene(G.ring8_scene(n_events=n, source=src)).trace(n)
    em = v[(v["kind"] == V_EMIT) & (v["photon"] == 0)]
    x0 = {int(r["event"]): np.array([r["x"], r["y"], r["z"]]) for r in em}
    ent = v[v["kind"] == 1]
    first = {}
    for r in ent:
        first.setdefault((int(r["event"]), int(r["photon"])), np.array([r["x"], r["y"], r["z"]]))
    checked = 0
    for ev in range(n):
        if (ev, 0) in first and (ev, 1) in first:
            pa, pb = first[(ev, 0)] - x0[ev], first[(ev, 1)] - x0[ev]
            assert np.linalg.norm(np.cross(pa, pb)) <= 1e-9 * np.linalg.norm(pa) * np.linalg.norm(pb)
            checked += 1
    assert checked > 100
    moved = np.array([np.linalg.norm(x0[e]) for e in range(n)])
    assert np.median(moved) > 1.0


def _crafted_hits(oracle_mod, n, scene, t0=10**9, spacing=10**7, seed=0):
    """One 511 keV hit per event, each in its own crystal of panel 0 or 6,
    times far apart (no dead time, no coincidences crossing events)."""
    rng = np.random.default_rng(seed)
    h = np.zeros(n, dtype=np.dtype(oracle_mod.Hit))
    h["event"] = np.arange(n)
    cpp = scene.crystals_per_panel
    h["gid"] = rng.integers(0, cpp, n) + cpp * rng.choice([0, 6], n)
    h["edep"] = 511.0
    h["depth"] = rng.uniform(1.0, 9.0, n)
    h["time_ps"] = t0 + np.arange(n, dtype=np.uint64) * spacing
    return h


@pytest.mark.parametrize("fwhm_ps", [200.0, 1000.0])
def test_time_blur_is_rounded_normal(oracle_mod, fwhm_ps):
    s = oracle_mod.OracleScene(G.small_animal_scene("C", n_events=10))
    h = _crafted_hits(oracle_mod, 20000, s)
    s0, _ = s.digitize(h, seed=4)
    s1, _ = s.digitize(h, seed=4, time_fwhm_ps=fwhm_ps)
    assert np.array_equal(s0["energy"], s1["energy"])  # energy deviate unchanged
    d = s1["time_ps"].astype(np.int64) - s0["time_ps"].astype(np.int64)
    sig = fwhm_ps / FWHM
    ks = np.arange(d.min(), d.max() + 1)
    emp = np.searchsorted(np.sort(d), ks, side="right") / len(d)
    model = stats.norm.cdf((ks + 0.5) / sig)  # P(rint(sig z) <= k)
    assert np.max(np.abs(emp - model)) < 1.63 / math.sqrt(len(d))
    assert abs(d.mean()) < 4 * sig / math.sqrt(len(d))


def test_time_blur_stays_non_negative(oracle_mod):
    s = oracle_mod.OracleScene(G.small_animal_scene("C", n_events=10))
    h = _crafted_hits(oracle_mod, 4000, s, t0=0, spacing=1)
    s1, _ = s.digitize(h, seed=1, time_fwhm_ps=5000.0)
    t = s1["time_ps"].astype(np.int64)
    assert t.min() == 0 and np.sum(t == 0) > 100


def test_doi_blur_is_normal(oracle_mod):
    s = oracle_mod.OracleScene(G.small_animal_scene("C", n_events=10))
    h = _crafted_hits(oracle_mod, 20000, s)
    s0, _ = s.digitize(h, seed=5)
    s1, _ = s.digitize(h, seed=5, doi_fwhm_mm=3.0)
    assert np.array_equal(s0["energy"], s1["energy"])
    assert np.array_equal(s0["time_ps"], s1["time_ps"])
    d = (s1["depth"] - s0["depth"]) / (3.0 / FWHM)
    assert stats.kstest(d, "norm").pvalue > 1e-3


def _unit(gid, level, scene):
    return gid // (1 if level == 0 else scene.s.crystals_per_module if level == 1 else scene.crystals_per_panel)


def _brute_lost(singles, unit, tau, mode):
    """Paralyzable: lost iff some earlier single of the unit (in (time, event,
    gid) order) lies less than tau before it.  Non-paralyzable: the kept set
    is built greedily in that order, each single tested against every kept
    single of its unit."""
    order = sorted(range(len(singles)), key=lambda i: (int(singles["time_ps"][i]), int(singles["event"][i]),
                                                       int(singles["gid"][i])))
    lost = np.zeros(len(singles), bool)
    kept = {}
    seen = {}
    for i in order:
        u, t = int(unit[i]), int(singles["time_ps"][i])
        if mode == 1:
            lost[i] = any(t - t2 < tau for t2 in seen.get(u, []))
            seen.setdefault(u, []).append(t)
        else:
            lost[i] = any(t - t2 < tau for t2 in kept.get(u, []))
            if not lost[i]:
                kept.setdefault(u, []).append(t)
    return lost


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("level", [0, 1, 2])
def test_dead_time_brute_force(oracle_mod, mode, level):
    s = oracle_mod.OracleScene(G.small_animal_scene("C", n_events=10))
    rng = np.random.default_rng(10 * mode + level)
    n = 600
    h = np.zeros(n, dtype=np.dtype(oracle_mod.Hit))
    h["event"] = np.arange(n)
    cpm = s.s.crystals_per_module
    # a few crystals of two modules, times on a coarse grid: many ties and
    # close pairs
    h["gid"] = rng.choice([3, 4, 5, cpm + 7, cpm + 8, 6 * s.crystals_per_panel + 1], n)
    h["edep"] = 511.0
    h["time_ps"] = rng.integers(0, 40, n).astype(np.uint64) * 250
    tau = 1000
    singles, _ = s.digitize(h, seed=1, fwhm_511=0.0, dead_ps=tau, dead_mode=mode, dead_level=level)
    ref = _brute_lost(singles, _unit(singles["gid"], level, s), tau, mode)
    assert np.array_equal(singles["lost"].astype(bool), ref)
    assert 0 < ref.sum() < n


@pytest.mark.parametrize("mode", [1, 2])
def test_dead_time_poisson_throughput(oracle_mod, mode):
    """One unit fed by a Poisson stream of rate r: the fraction kept is
    exp(-r tau) (paralyzable) or 1 / (1 + r tau) (non-paralyzable)."""
    s = oracle_mod.OracleScene(G.small_animal_scene("C", n_events=10))
    rng = np.random.default_rng(7 + mode)
    n = 40000
    mean_gap = 100_000.0  # ps
    tau = 50_000          # r tau = 0.5
    t = np.cumsum(rng.exponential(mean_gap, n)).astype(np.uint64) + 1000
    h = np.zeros(n, dtype=np.dtype(oracle_mod.Hit))
    h["event"] = np.arange(n)
    h["gid"] = rng.integers(0, s.s.crystals_per_module, n)  # all in module 0
    h["edep"] = 511.0
    h["time_ps"] = t
    singles, _ = s.digitize(h, seed=1, fwhm_511=0.0, dead_ps=tau, dead_mode=mode, dead_level=1)
    kept = 1.0 - singles["lost"].mean()
    x = tau / mean_gap
    expect = math.exp(-x) if mode == 1 else 1.0 / (1.0 + x)
    assert abs(kept - expect) < 4 * math.sqrt(expect * (1 - expect) / n)
    # the other model is far off: the pin tells the two apart
    other = 1.0 / (1.0 + x) if mode == 1 else math.exp(-x)
    assert abs(kept - other) > 0.03


def test_dead_singles_pass_no_window(oracle_mod):
    s = oracle_mod.OracleScene(G.small_animal_scene("C", n_events=10))
    cpp = s.crystals_per_panel
    # one pair per event in panels 0 and 6, at 0, 20 and 30 ns
    h = np.zeros(6, dtype=np.dtype(oracle_mod.Hit))
    h["event"] = [0, 0, 1, 1, 2, 2]
    h["gid"] = [5, 6 * cpp + 5, 900, 6 * cpp + 900, 7, 6 * cpp + 7]
    h["edep"] = 511.0
    h["time_ps"] = [0, 0, 20000, 20000, 30000, 30000]
    sg, cc = s.digitize(h, seed=1, fwhm_511=0.0, window_ps=3000)
    assert len(cc) == 3
    # panel-level dead time of 15 ns, paralyzable: events 1 (20 ns after 0) keeps,
    # event 2 comes 10 ns after event 1 in the same panels: lost
    sg, cc = s.digitize(h, seed=1, fwhm_511=0.0, window_ps=3000, dead_ps=15000, dead_mode=1, dead_level=2)
    assert sg["lost"].tolist() == [0, 0, 0, 0, 1, 1]
    assert len(cc) == 2
    # a gap of exactly the dead time is not dead (strict comparison)
    for mode in (1, 2):
        sg, cc = s.digitize(h, seed=1, fwhm_511=0.0, window_ps=3000, dead_ps=20000, dead_mode=mode, dead_level=2)
        assert sg["lost"].tolist() == [0, 0, 0, 0, 1, 1]
    sg, cc = s.digitize(h, seed=1, fwhm_511=0.0, window_ps=3000, dead_ps=25000, dead_mode=1, dead_level=2)
    assert sg["lost"].tolist() == [0, 0, 1, 1, 1, 1]
    assert len(cc) == 1
    # non-paralyzable with 25 ns: event 2 is 30 ns after the last kept (event 0)
    sg, cc = s.digitize(h, seed=1, fwhm_511=0.0, window_ps=3000, dead_ps=25000, dead_mode=2, dead_level=2)
    assert sg["lost"].tolist() == [0, 0, 1, 1, 0, 0]
    assert len(cc) == 2


def _place(scene, gid):
    """(module id, layer, i_t, i_a) of crystal ids, from the id layout."""
    S = scene.s
    cpm = S.crystals_per_module
    local = gid % cpm
    bases = [S.layer_base[k] for k in range(S.scan.n_layers)]
    layer = np.searchsorted(bases, local, side="right") - 1
    nt = np.array([S.scan.layer[k].n_t for k in range(S.scan.n_layers)])[layer]
    i = local - np.array(bases)[layer]
    return gid // cpm, layer, i % nt, i // nt


@pytest.mark.parametrize("design", ["A", "C"])
def test_light_sharing_moves_to_a_neighbour(oracle_mod, design):
    s = oracle_mod.OracleScene(G.small_animal_scene(design, n_events=10))
    n = 30000
    rng = np.random.default_rng(11)
    h = np.zeros(n, dtype=np.dtype(oracle_mod.Hit))
    h["event"] = np.arange(n)
    h["gid"] = rng.integers(0, s.n_crystals, n)
    h["edep"] = 511.0
    h["time_ps"] = 10**9 + np.arange(n, dtype=np.uint64) * 10**7
    s0, _ = s.digitize(h, seed=2)
    s1, _ = s.digitize(h, seed=2, light_sharing=1.0)
    assert np.array_equal(s0["energy"], s1["energy"])  # the blur draws follow the true crystal
    g0, g1 = s0["gid"].astype(np.int64), s1["gid"].astype(np.int64)
    m0, l0, t0, a0 = _place(s, g0)
    m1, l1, t1, a1 = _place(s, g1)
    assert np.array_equal(m0, m1) and np.array_equal(l0, l1)
    assert np.all(np.abs(t1 - t0) + np.abs(a1 - a0) == 1)
    # each existing neighbour equally likely: crystals with 4 neighbours
    S = s.s
    nt = np.array([S.scan.layer[k].n_t for k in range(S.scan.n_layers)])[l0]
    na = np.array([S.scan.layer[k].n_a for k in range(S.scan.n_layers)])[l0]
    inner = (t0 > 0) & (t0 < nt - 1) & (a0 > 0) & (a0 < na - 1)
    code = (t1 - t0 + 1) + 3 * (a1 - a0 + 1)  # 3 (t-1), 5 (t+1), 1 (a-1), 7 (a+1)
    counts = np.array([np.sum(code[inner] == c) for c in (3, 5, 1, 7)])
    assert stats.chisquare(counts).pvalue > 1e-3
    # corners have exactly their two neighbours
    corner = (t0 == 0) & (a0 == 0)
    assert set(np.unique(code[corner]).tolist()) <= {5, 7} and corner.sum() > 0
    # partial probability: the moved fraction is binomial
    s3, _ = s.digitize(h, seed=2, light_sharing=0.3)
    moved = np.mean(s3["gid"] != s0["gid"])
    assert abs(moved - 0.3) < 4 * np.sqrt(0.3 * 0.7 / n)
    s4, _ = s.digitize(h, seed=2, light_sharing=0.0)
    assert np.array_equal(s4["gid"], s0["gid"])
