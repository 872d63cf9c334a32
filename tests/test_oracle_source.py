"""Pins of the oracle's source (CPU only): the rod source and the event time.

Sec. 2.3 fixes a source of uniform activity density in its rods and a fixed
number of decays of a constant activity over the acquisition.  So:
 - a rod is chosen with probability proportional to its volume r^2 L, and the
   annihilation point is uniform in the rod: (rho/r)^2, the azimuth about the
   rod axis and the axial position (z - z0)/(z1 - z0) are each U[0, 1);
 - event times are uniform on [0, T): t_e = floor(X T / 2^64) for the 64-bit
   word X = w1 2^32 + w0 of event-stream block 2.
Each check is chosen so that a plausible slip fails it: rod weights by r or by
r^2 alone, rho = r u instead of r sqrt(u), a wrong block or word order of the
time, a truncated product.
"""
import math

import numpy as np
import pytest
from scipy import stats

import gpet_inputs as G

V_EMIT = 6

# rods (cx, cy, radius, z0, z1) of different radii and lengths, far apart:
# a weight by r^2 alone or by r L differs from r^2 L by factors of 2-6 here
RODS = np.array([(-6.0, -6.0, 0.5, -10.0, 10.0),
                 (6.0, -6.0, 1.0, -3.0, 2.0),
                 (-6.0, 6.0, 1.5, 0.0, 12.0),
                 (6.0, 6.0, 2.0, -8.0, -4.0),
                 (0.0, 0.0, 0.75, -15.0, 15.0)], np.float64)


def _emission_points(oracle_mod, n):
    sc = G.ring8_scene(n_events=n, source=G.rod_source(RODS, n))
    v = oracle_mod.OracleScene(sc).trace(n, seed=3)
    em = v[(v["kind"] == V_EMIT) & (v["photon"] == 0)]
    assert len(em) == n
    return np.stack([em["x"], em["y"], em["z"]], 1)


def _rod_of(p):
    rho = np.hypot(p[:, None, 0] - RODS[None, :, 0], p[:, None, 1] - RODS[None, :, 1])
    inside = (rho <= RODS[None, :, 2]) & (p[:, None, 2] >= RODS[None, :, 3]) & (p[:, None, 2] <= RODS[None, :, 4])
    assert np.all(inside.sum(1) == 1)  # every point lies in exactly one rod
    return inside.argmax(1), rho[np.arange(len(p)), inside.argmax(1)]


def test_rod_choice_proportional_to_volume(oracle_mod):
    n = 60_000
    p = _emission_points(oracle_mod, n)
    k, _ = _rod_of(p)
    counts = np.bincount(k, minlength=len(RODS))
    vol = RODS[:, 2] ** 2 * (RODS[:, 4] - RODS[:, 3])
    exp = n * vol / vol.sum()
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert stats.chi2.sf(chi2, len(RODS) - 1) > 0.01, (counts, exp)
    # the slips named above are far outside the noise at this n
    for wrong in (RODS[:, 2] ** 2, RODS[:, 2] * (RODS[:, 4] - RODS[:, 3])):
        ew = n * wrong / wrong.sum()
        assert stats.chi2.sf(float(((counts - ew) ** 2 / ew).sum()), len(RODS) - 1) < 1e-6


def test_point_uniform_in_rod(oracle_mod):
    n = 60_000
    p = _emission_points(oracle_mod, n)
    k, rho = _rod_of(p)
    rd = RODS[k]
    u_r = (rho / rd[:, 2]) ** 2
    psi = np.arctan2(p[:, 1] - rd[:, 1], p[:, 0] - rd[:, 0])
    u_z = (p[:, 2] - rd[:, 3]) / (rd[:, 4] - rd[:, 3])
    assert stats.kstest(u_r, "uniform").pvalue > 0.01
    assert stats.kstest((psi + math.pi) / (2 * math.pi), "uniform").pvalue > 0.01
    assert stats.kstest(u_z, "uniform").pvalue > 0.01
    # rho = r u would make (rho/r)^2 = u^2: far from uniform
    assert stats.kstest(rho / rd[:, 2], "uniform").pvalue < 1e-6
    # azimuth and radius independent: the quadrant counts of the offset vector
    # are equal within each radial half
    for half in (u_r < 0.5, u_r >= 0.5):
        q = np.bincount(((psi[half] > 0).astype(int) * 2 + (np.abs(psi[half]) > math.pi / 2)), minlength=4)
        assert stats.chisquare(q).pvalue > 0.001


@pytest.mark.parametrize("T", [1, 7, 786_000_000_000_000, 2**63 + 5, 2**64 - 1])
def test_event_time_crafted_words(oracle_mod, T):
    et = oracle_mod.event_time
    assert et(0, T) == 0
    assert et(2**64 - 1, T) == T - 1          # the largest word stays below T
    assert et(2**63, T) == T // 2             # one half of the acquisition
    assert et(2**62, T) == T // 4
    rng = np.random.default_rng(T % 1000)
    for x in rng.integers(0, 2**63, 50, dtype=np.uint64).tolist():
        x = 2 * x + 1
        assert et(x, T) == (x * T) >> 64      # exact: no truncation of the product
        assert 0 <= et(x, T) < T


def test_event_times_uniform_and_from_block_2(oracle_mod):
    """t_e recovered from the hits (time minus rounded flight time) is one
    value per event, equals floor(X T / 2^64) for the words of event-stream
    block 2 (counter (2, event, instance, 0)), and is uniform on [0, T)."""
    n, inst, seed = 120_000, 5, 11
    sc = G.ring8_scene(n_events=n)
    T = int(sc["source"]["duration_ps"])
    hits, _ = oracle_mod.OracleScene(sc).transport(n, seed=seed, instance=inst)
    te = hits["time_ps"].astype(np.int64) - np.floor(hits["tof_ps"] + 0.5).astype(np.int64)
    ev = hits["event"].astype(np.int64)
    order = np.argsort(ev, kind="stable")
    ev, te = ev[order], te[order]
    first = np.r_[True, ev[1:] != ev[:-1]]
    idx = np.cumsum(first) - 1
    assert np.array_equal(te, te[first][idx])  # one time per event
    evs, tes = ev[first], te[first]
    assert len(evs) > 4000
    ctr = np.stack([np.full(len(evs), 2), evs, np.full(len(evs), inst), np.zeros(len(evs))], 1)
    w = oracle_mod.philox(seed, ctr.astype(np.uint32))
    want = [((int(w1) << 32 | int(w0)) * T) >> 64 for w0, w1 in zip(w[:, 0], w[:, 1])]
    assert tes.tolist() == want
    assert np.all((tes >= 0) & (tes < T))
    assert stats.kstest(tes / T, "uniform").pvalue > 0.01
