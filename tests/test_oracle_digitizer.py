"""Pins of the oracle's digitizer (CPU only): brute-force adder, Gaussian blur
statistics, exact window filter, and an independent reference of the
coincidence sorter on random and crafted singles."""
import math

import numpy as np
import pytest
from scipy import stats

import gpet_inputs as G


def _hits(oracle_mod, n):
    return np.zeros(n, dtype=np.dtype(oracle_mod.Hit))


def _scene(oracle_mod):
    return oracle_mod.OracleScene(G.small_animal_scene("C", n_events=10))


def test_adder_matches_dictionary(oracle_mod):
    s = oracle_mod.OracleScene(G.small_animal_scene("C", n_events=20000))
    hits, _ = s.transport(20000, seed=2)
    singles, _ = s.digitize(hits, seed=2)
    ref = {}
    for h in hits:
        k = (int(h["event"]), int(h["gid"]))
        e, ed, t = ref.get(k, (0.0, 0.0, 2**64))
        ref[k] = (e + h["edep"], ed + h["edep"] * h["depth"], min(t, int(h["time_ps"])))
    keys = sorted(ref)
    assert [(int(a), int(b)) for a, b in zip(singles["event"], singles["gid"])] == keys
    e = np.array([ref[k][0] for k in keys])
    np.testing.assert_allclose(singles["edep"], e, rtol=1e-12)
    np.testing.assert_allclose(singles["depth"], np.array([ref[k][1] for k in keys]) / e, rtol=1e-10)
    assert np.array_equal(singles["time_ps"], np.array([ref[k][2] for k in keys], np.uint64))


@pytest.mark.parametrize("e0", [511.0, 200.0])
def test_blur_is_gaussian_with_sqrt_e_width(oracle_mod, e0):
    """FWHM(E) = 0.16 sqrt(511 E): 16 % at 511 keV (Sec. 2.3)."""
    s = _scene(oracle_mod)
    n = 100_000
    h = _hits(oracle_mod, n)
    h["event"] = np.arange(n)
    h["gid"] = np.arange(n) % s.n_crystals
    h["edep"] = e0
    h["time_ps"] = np.arange(n, dtype=np.uint64) * 10**7
    singles, _ = s.digitize(h, seed=5)
    sig = 0.16 * math.sqrt(511.0 * e0) / (2 * math.sqrt(2 * math.log(2)))
    assert stats.kstest(singles["energy"], stats.norm(e0, sig).cdf).pvalue > 0.01
    np.testing.assert_array_equal(singles["in_window"],
                                  (singles["energy"] >= 350) & (singles["energy"] <= 650))


def _reference_sorter(t, panel, tau):
    """Coincidences by definition: scan time-ordered singles; each window opens
    at the first single not yet taken and holds every later single within tau
    of the opener; keep it iff it holds exactly two singles in two panels."""
    order = sorted(range(len(t)), key=lambda i: t[i])
    used = [False] * len(t)
    out = []
    for pos, i in enumerate(order):
        if used[i]:
            continue
        members = [j for j in order[pos:] if t[j] - t[i] <= tau]
        for j in members:
            used[j] = True
        if len(members) == 2 and panel[members[0]] != panel[members[1]]:
            out.append(tuple(members))
    return out


def _single_times(oracle_mod, times, gids, edep=511.0, events=None):
    n = len(times)
    h = _hits(oracle_mod, n)
    h["event"] = np.arange(n) if events is None else events
    h["gid"] = gids
    h["edep"] = edep
    h["time_ps"] = np.asarray(times, np.uint64)
    return h


def test_sorter_random_against_reference(oracle_mod):
    s = _scene(oracle_mod)
    rng = np.random.default_rng(8)
    n = 6000
    times = np.sort(rng.integers(0, n * 1500, n))  # mean spacing 1.5 ns: many multiples
    gids = rng.integers(0, s.n_crystals, n)
    singles, coinc = s.digitize(_single_times(oracle_mod, times, gids), fwhm_511=0.0,
                                e_lo=-1e9, e_hi=1e9)
    assert len(singles) == n
    cpp = s.crystals_per_panel
    ref = _reference_sorter(singles["time_ps"].astype(np.int64).tolist(),
                            (singles["gid"] // cpp).tolist(), 3000)
    got = [tuple(int(x) for x in c) for c in coinc]
    assert sorted(got) == sorted(ref)
    assert len(got) > 100


def test_sorter_crafted_cases(oracle_mod):
    s = _scene(oracle_mod)
    cpp = s.crystals_per_panel
    P = lambda p: p * cpp  # noqa: E731  first crystal of panel p
    base = 10**9
    cases = [
        ([0, 3000], [P(0), P(1)], 1),            # exactly tau apart: inside
        ([0, 3001], [P(0), P(1)], 0),            # just outside: two lone singles
        ([0, 1000, 2000], [P(0), P(1), P(2)], 0),  # triple: discarded
        ([0, 10], [P(3), P(3) + 5], 0),          # same panel: rejected
        ([0, 0], [P(1), P(4)], 1),               # equal time stamps
        ([0, 2000, 4000], [P(0), P(1), P(2)], 1),  # window does not retrigger: (0,1) pair, 2 alone
    ]
    for k, (t, g, want) in enumerate(cases):
        times = [base * (k + 1) + x for x in t]
        h = _single_times(oracle_mod, times, g)
        _, coinc = s.digitize(h, fwhm_511=0.0, e_lo=-1e9, e_hi=1e9)
        assert len(coinc) == want, (k, t, g)


def test_window_applies_before_sorting(oracle_mod):
    """A single outside the energy window does not take part in the sorter."""
    s = _scene(oracle_mod)
    cpp = s.crystals_per_panel
    h = _single_times(oracle_mod, [0, 1000, 2000], [0, cpp, 2 * cpp])
    h["edep"] = [511.0, 100.0, 511.0]
    _, coinc = s.digitize(h, fwhm_511=0.0)
    assert len(coinc) == 1


# ---------------------------------------------------------------------------
# single readout levels (Sec. 2.1): crystal, module, panel
# ---------------------------------------------------------------------------
GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def _golden_readout():
    hits, want = [], {"module": [], "panel": []}
    for line in open(f"{GOLDEN}/readout_example.txt"):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        row = (int(f[1]), int(f[2]), float(f[3]), float(f[4]), int(f[5]))
        (hits if f[0] == "hit" else want[f[0]]).append(row)
    return hits, want


@pytest.mark.parametrize("level,code", [("module", 1), ("panel", 2)])
def test_readout_worked_example(oracle_mod, level, code):
    """Module and panel singles of a small hand-worked example: sums, earliest
    times, the crystal and depth of the largest deposit, ties to the lower id."""
    s = _scene(oracle_mod)
    rows, want = _golden_readout()
    h = _hits(oracle_mod, len(rows))
    for k, (ev, gid, e, dep, t) in enumerate(rows):
        h[k]["event"], h[k]["gid"], h[k]["edep"], h[k]["depth"], h[k]["time_ps"] = ev, gid, e, dep, t
    singles, _ = s.digitize(h, fwhm_511=0.0, e_lo=-1e9, e_hi=1e9, readout=code)
    got = [(int(q["event"]), int(q["gid"]), float(q["edep"]), float(q["depth"]), int(q["time_ps"]))
           for q in singles]
    assert len(got) == len(want[level])
    for g, w in zip(got, want[level]):
        assert g[:2] == w[:2] and g[4] == w[4], (g, w)
        assert abs(g[2] - w[2]) < 1e-9 and abs(g[3] - w[3]) < 1e-9, (g, w)


def test_readout_levels_conserve_energy_and_nest(oracle_mod):
    """On transported hits: every level holds the same energy per event, the
    module level has one single per (event, module) the crystal level touches
    and the panel level one per (event, panel), and at the panel level no two
    singles of an event share a panel."""
    s = oracle_mod.OracleScene(G.small_animal_scene("C", n_events=30000))
    hits, _ = s.transport(30000, seed=4)
    levels = [s.digitize(hits, seed=4, fwhm_511=0.0, e_lo=-1e9, e_hi=1e9, readout=r)[0] for r in (0, 1, 2)]
    cpm, cpp = s.s.crystals_per_module, s.s.crystals_per_panel
    per_event = [np.bincount(q["event"], weights=q["edep"], minlength=30000) for q in levels]
    np.testing.assert_allclose(per_event[1], per_event[0], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(per_event[2], per_event[0], rtol=1e-12, atol=1e-9)
    c = levels[0]
    assert len(levels[1]) == len({(int(e), int(g) // cpm) for e, g in zip(c["event"], c["gid"])})
    assert len(levels[2]) == len({(int(e), int(g) // cpp) for e, g in zip(c["event"], c["gid"])})
    assert len(levels[2]) < len(levels[1]) < len(c)
    p = levels[2]
    assert len({(int(e), int(g) // cpp) for e, g in zip(p["event"], p["gid"])}) == len(p)


def test_tallies_worked_example(oracle_mod):
    """Hand-counted tallies (Sec. 2.3 windows, Sec. 3.1 DOI histograms): five
    hits in three crystals of a 20 mm panel read into 4 depth bins of 5 mm,
    four singles of which one lies outside the window and one is dead."""
    h = _hits(oracle_mod, 5)
    h["gid"] = [3, 3, 7, 0, 7]
    h["depth"] = [0.0, 4.999, 5.0, 19.999, 25.0]  # bins 0, 0, 1, 3, past the back face -> 3
    s = np.zeros(4, dtype=np.dtype(oracle_mod.Single))
    s["gid"] = [3, 7, 0, 7]
    s["energy"] = [511.2, 340.0, 699.999, -3.0]
    s["in_window"] = [1, 0, 1, 1]
    s["lost"] = [0, 0, 1, 0]
    t = oracle_mod.tallies(h, s, n_crystals=8, panel_depth=20.0, doi_bins=4)
    assert t["hits_per_crystal"].tolist() == [1, 0, 0, 2, 0, 0, 0, 2]
    assert t["doi"].tolist() == [2, 1, 0, 2]
    assert t["singles_per_crystal"].tolist() == [0, 0, 0, 1, 0, 0, 0, 1]
    spec = np.zeros(700, np.int64)
    spec[511] += 1
    spec[340] += 1
    assert np.array_equal(t["energy_spectrum"], spec)


def test_tallies_conserve_counts(oracle_mod):
    """On a transported run: every hit is in one crystal bin and one depth bin;
    in-window singles and the spectrum count what the single list holds."""
    s = oracle_mod.OracleScene(G.small_animal_scene("C", n_events=20000))
    hits, _ = s.transport(20000, seed=4)
    singles, _ = s.digitize(hits, seed=4)
    t = s.tallies(hits, singles, doi_bins=200)
    assert t["hits_per_crystal"].sum() == len(hits) == t["doi"].sum()
    assert t["singles_per_crystal"].sum() == int(np.sum(singles["in_window"] != 0))
    inside = (singles["energy"] >= 0) & (singles["energy"] < 700)
    assert t["energy_spectrum"].sum() == int(inside.sum())
    # hits per crystal equal the per-crystal sum over the singles' crystals' hits
    assert np.array_equal(np.nonzero(t["hits_per_crystal"])[0], np.unique(singles["gid"]))
    # two 10 mm layers in a 20 mm panel: the DOI histogram has hits on both sides of the layer face
    assert t["doi"][:100].sum() > 0 and t["doi"][100:].sum() > 0
