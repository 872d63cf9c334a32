"""Parity at the benchmark's full size and launch configuration: design C,
1e7 events per launch, source off centre, default launch shape (blocks per
CU from the occupancy, search batch 16, lane schedule 0).

The oracle cannot run 1e7 events in a test, but every random number is keyed
by the event id, so it re-simulates sampled blocks of event ids one by one
and their hits must match the GPU's hits of the same ids (RNG-matched: equal
up to rare FP32-versus-FP64 branch flips).  The digitizer's adder and blur
act per (event, crystal), so the singles of the sampled events are checked
against the oracle's digitizer run on the GPU's own hits of those events;
the coincidences, which couple events through time, are checked through
properties that hold at any size.  The hot-rod workload (rod source in the
voxelized water cylinder, design C) gets the same sampled-event check at 1e7
events, so phantom tracking is covered at its full launch size too, and so
does the source with acollinearity and positron range on.
"""
import numpy as np
import pytest

import gpet_inputs as G

pytestmark = pytest.mark.gpu

N = 10_000_000
POS = G.SWEEP_POSITIONS[3]


@pytest.fixture(scope="module")
def run():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_07327_amd.gpet import Context
    c = Context(0)
    sc = G.small_animal_scene("C", POS, n_events=N)
    c.set_scene(sc)
    c.set_launch(0, 16, 0)
    hits, st = c.transport(N, seed=1001)
    singles, coinc = c.digitize(hits, seed=1001)
    out = {"scene": sc, "ctx": c, "stats": st, "hits_t": hits, "hits": hits.numpy(), "singles": singles.numpy(),
           "coinc": (coinc[0].cpu().numpy(), coinc[1].cpu().numpy()), "n_crystals": c.info.n_crystals,
           "cpp": c.info.crystals_per_panel}
    yield out
    c.close()


def _blocks(rng, n_blocks=20, size=100):
    starts = np.sort(rng.choice(N // size, n_blocks, replace=False)) * size
    return [(int(s), size) for s in starts] + [(0, size), (N - size, size)]


def _compare_sampled(scene, g, oracle_mod, seed, rng, n_blocks=20):
    """Re-simulate sampled blocks of event ids in the oracle and compare each
    event's hits (crystal ids exactly; energies and times to FP32 rounding)."""
    o = oracle_mod.OracleScene(scene)
    ev = g["event"].view(np.uint32)
    order = np.argsort(ev, kind="stable")
    evs = ev[order]
    n_ev = n_diff = n_hits = 0
    for first, size in _blocks(rng, n_blocks):
        rh, _ = o.transport(size, seed=seed, first=first)
        lo, hi = np.searchsorted(evs, [first, first + size])
        gh = {k: v[order[lo:hi]] for k, v in g.items()}
        for e in range(first, first + size):
            a = rh[rh["event"] == e]
            b_sel = gh["event"].view(np.uint32) == e
            gid_g = np.sort(gh["gid"][b_sel].view(np.uint32))
            gid_o = np.sort(a["gid"])
            n_ev += 1
            n_hits += len(a)
            if len(gid_g) != len(gid_o) or not np.array_equal(gid_g, gid_o):
                n_diff += 1
                continue
            if len(a):
                eg = np.sort(gh["edep_kev"][b_sel].astype(np.float64))
                np.testing.assert_allclose(eg, np.sort(a["edep"]), rtol=2e-4, atol=2e-3)
                tg = np.sort(gh["time_ps"][b_sel].view(np.uint64).astype(np.int64))
                assert np.all(np.abs(tg - np.sort(a["time_ps"].astype(np.int64))) <= 1)
    return n_ev, n_diff, n_hits


def test_sampled_events_match_oracle(run, oracle_mod):
    n_ev, n_diff, n_hits = _compare_sampled(run["scene"], run["hits"], oracle_mod, 1001, np.random.default_rng(5))
    print(f"{n_ev} sampled events, {n_hits} oracle hits, {n_diff} events differing")
    assert n_hits > 1000
    assert n_diff <= max(3, 0.01 * n_ev)


@pytest.fixture(scope="module")
def rods_run():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_07327_amd.gpet import Context
    c = Context(0)
    sc = G.hot_rod_scene(n_events=N)
    c.set_scene(sc)
    c.set_launch(0, 16, 0)
    hits, st = c.transport(N, seed=1002)
    out = {"scene": sc, "stats": st, "hits": hits.numpy(), "n_crystals": c.info.n_crystals}
    yield out
    c.close()


def test_hot_rods_sampled_events_match_oracle(rods_run, oracle_mod):
    st, g = rods_run["stats"], rods_run["hits"]
    assert st["events"] == N and st["capped"] == 0
    assert g["gid"].view(np.uint32).max() < rods_run["n_crystals"]
    n_ev, n_diff, n_hits = _compare_sampled(rods_run["scene"], g, oracle_mod, 1002, np.random.default_rng(7),
                                            n_blocks=10)
    print(f"hot rods: {len(g['event'])} hits; {n_ev} sampled events, {n_hits} oracle hits, {n_diff} differing")
    assert n_hits > 200
    assert n_diff <= max(3, 0.01 * n_ev)


def test_sampled_singles_match_oracle_digitizer(run, oracle_mod):
    o = oracle_mod.OracleScene(run["scene"])
    g, s = run["hits"], run["singles"]
    ev_h = g["event"].view(np.uint32)
    ev_s = s["event"].view(np.uint32)
    rng = np.random.default_rng(6)
    pick = np.sort(rng.choice(N, 3000, replace=False)).astype(np.uint32)
    hs = np.isin(ev_h, pick)
    h = np.zeros(int(hs.sum()), dtype=np.dtype(oracle_mod.Hit))
    h["event"] = ev_h[hs]
    h["gid"] = g["gid"][hs].view(np.uint32)
    h["edep"] = g["edep_kev"][hs]
    h["depth"] = g["depth_mm"][hs]
    h["time_ps"] = g["time_ps"][hs].view(np.uint64)
    h["photon"] = g["aux"][hs].view(np.uint32) & 1
    h["seq"] = g["aux"][hs].view(np.uint32) >> 8
    so, _ = o.digitize(h, seed=1001)
    ss = np.isin(ev_s, pick)
    assert np.array_equal(ev_s[ss], so["event"])
    assert np.array_equal(s["gid"][ss].view(np.uint32), so["gid"])
    assert np.array_equal(s["time_ps"][ss].view(np.uint64), so["time_ps"])
    np.testing.assert_allclose(s["edep_kev"][ss], so["edep"], rtol=1e-6, atol=1e-5)
    np.testing.assert_allclose(s["energy_kev"][ss], so["energy"], rtol=1e-5, atol=1e-3)
    edge = (np.abs(so["energy"] - 350) < 1e-2) | (np.abs(so["energy"] - 650) < 1e-2)
    assert np.array_equal((s["in_window"][ss] != 0)[~edge], (so["in_window"] != 0)[~edge])
    print(f"{len(so)} singles of {len(pick)} sampled events")
    assert len(so) > 1000


def test_full_size_properties(run):
    g, s = run["hits"], run["singles"]
    a, b = run["coinc"]
    st = run["stats"]
    assert st["events"] == N and st["capped"] == 0
    gid = g["gid"].view(np.uint32)
    assert gid.max() < run["n_crystals"]
    assert np.all((g["edep_kev"] > 0) & (g["edep_kev"] <= 511.001))
    # singles: (event, gid) strictly increasing, energies summed per crystal
    ev = s["event"].view(np.uint32).astype(np.int64)
    sg = s["gid"].view(np.uint32).astype(np.int64)
    key = ev * (1 << 20) + sg
    assert np.all(np.diff(key) > 0)
    assert abs(float(s["edep_kev"].astype(np.float64).sum()) - float(g["edep_kev"].astype(np.float64).sum())) \
        <= 1e-5 * float(g["edep_kev"].astype(np.float64).sum())
    # coincidences: both singles in the window, within 3 ns, in different panels, in time order
    win = s["in_window"].view(np.uint32)
    t = s["time_ps"].view(np.uint64).astype(np.int64)
    assert np.all(win[a] == 1) and np.all(win[b] == 1)
    dt = t[b] - t[a]
    assert np.all((dt >= 0) & (dt <= 3000))
    assert np.all(sg[a] // run["cpp"] != sg[b] // run["cpp"])
    assert np.all(np.diff(t[a]) >= 0)
    assert len(a) > 100_000
    print(f"{len(g['event'])} hits, {len(ev)} singles, {int(win.sum())} in window, {len(a)} coincidences")


def test_source_physics_sampled_events_match_oracle(oracle_mod):
    """The benchmark's optional-physics form at full size: design C, source at
    the centre with 0.5 deg acollinearity and a 0.102 mm positron range."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_07327_amd.gpet import Context
    sc = G.small_animal_scene("C", (0.0, 0.0, 0.0), n_events=N)
    src = G.point_source((0.0, 0.0, 0.0), N)
    src.update({"acolinearity_fwhm_deg": 0.5, "positron_range_fwhm_mm": 0.102})
    sc["source"] = src
    c = Context(0)
    try:
        c.set_scene(sc)
        c.set_launch(0, 16, 0)
        hits, st = c.transport(N, seed=1003)
        g = hits.numpy()
    finally:
        c.close()
    assert st["events"] == N and st["capped"] == 0
    n_ev, n_diff, n_hits = _compare_sampled(sc, g, oracle_mod, 1003, np.random.default_rng(8), n_blocks=10)
    print(f"source physics: {len(g['event'])} hits; {n_ev} sampled events, {n_hits} oracle hits, {n_diff} differing")
    assert n_hits > 200
    assert n_diff <= max(3, 0.01 * n_ev)


def test_sampled_singles_with_response_match_oracle(run, oracle_mod):
    """Time and DOI blur and light sharing (dead time off, as it couples events)
    on the full hit list; the singles of 3000 sampled events against the oracle
    digitizer run on the GPU's hits of those events with the same response."""
    resp = {"time_fwhm_ps": 300.0, "doi_fwhm_mm": 2.0, "light_sharing": 0.1}
    sg, _ = run["ctx"].digitize(run["hits_t"], seed=1004, response=resp)
    s = sg.numpy()
    g = run["hits"]
    ev_h = g["event"].view(np.uint32)
    pick = np.sort(np.random.default_rng(9).choice(N, 3000, replace=False)).astype(np.uint32)
    hs = np.isin(ev_h, pick)
    h = np.zeros(int(hs.sum()), dtype=np.dtype(oracle_mod.Hit))
    h["event"] = ev_h[hs]
    h["gid"] = g["gid"][hs].view(np.uint32)
    h["edep"] = g["edep_kev"][hs]
    h["depth"] = g["depth_mm"][hs]
    h["time_ps"] = g["time_ps"][hs].view(np.uint64)
    h["photon"] = g["aux"][hs].view(np.uint32) & 1
    h["seq"] = g["aux"][hs].view(np.uint32) >> 8
    o = oracle_mod.OracleScene(run["scene"])
    so, _ = o.digitize(h, seed=1004, time_fwhm_ps=300.0, doi_fwhm_mm=2.0, light_sharing=0.1)
    so0, _ = o.digitize(h, seed=1004)
    ss = np.isin(s["event"].view(np.uint32), pick)
    assert np.array_equal(s["event"][ss].view(np.uint32), so["event"])
    assert np.array_equal(s["gid"][ss].view(np.uint32), so["gid"])
    dt = s["time_ps"][ss].view(np.int64) - so["time_ps"].astype(np.int64)
    assert np.all(np.abs(dt) <= 1) and np.count_nonzero(dt) <= 1e-3 * len(so) + 5
    np.testing.assert_allclose(s["depth_mm"][ss], so["depth"], rtol=0, atol=1e-4)
    np.testing.assert_allclose(s["energy_kev"][ss], so["energy"], rtol=1e-5, atol=1e-3)
    edge = (np.abs(so["energy"] - 350) < 1e-2) | (np.abs(so["energy"] - 650) < 1e-2)
    assert np.array_equal((s["in_window"][ss].view(np.uint32) == 1)[~edge], (so["in_window"] != 0)[~edge])
    assert len(so0) == len(so)
    moved = int(np.count_nonzero(so0["gid"] != so["gid"]))
    print(f"{len(so)} singles of {len(pick)} sampled events with the response on, {moved} read by a neighbour")
    assert len(so) > 1000 and moved > 0.03 * len(so)
