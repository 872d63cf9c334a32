"""Woodcock tracking against analog tracking in the oracle (CPU only).

Woodcock tracking (Sec. 2.1: free paths on a majorant, real or virtual
collisions by acceptance) and analog tracking (flights from material
boundary to boundary, spending the sampled optical depth segment by
segment) sample the same collision law, so every tally of the two agrees in
distribution.  A wrong majorant, acceptance or material lookup in either
breaks that.  Compared at independent event streams: hits per (layer,
process), deposited energy per event, hits per event and the real-collision
rate, on a one-ring design, the 4-layer BGO/LYSO stack (a majorant over
several crystal materials) and the hot rods in a water phantom (phantom
tracking).
"""
import numpy as np
import pytest
from scipy import stats

import gpet_inputs as G
from tests.gpu_util import chi2_two_sample

N = 200_000


def _scene(kind):
    if kind == "C":
        return G.small_animal_scene("C", (5.0, 0.0, 0.0), n_events=N)
    if kind == "stack4":
        return G.stack_scene("stack4", (2.0, 1.0, 0.0), N)
    return G.hot_rod_scene(n_events=N)


def _tallies(hits, n_layers):
    ev = hits["event"].astype(np.int64)
    lp = np.bincount(hits["layer"].astype(np.int64) * 4 + hits["process"].astype(np.int64), minlength=4 * n_layers)
    edep = np.bincount(ev, weights=hits["edep"], minlength=N)
    e_hist = np.histogram(edep[edep > 0], bins=np.arange(0.0, 530.0, 10.0))[0]
    per_ev = np.bincount(np.minimum(np.bincount(ev, minlength=N), 5), minlength=6)
    return lp, e_hist, per_ev


@pytest.mark.parametrize("kind", ["C", "stack4", "rods_phantom"])
def test_woodcock_equals_analog_in_law(oracle_mod, kind):
    sc = _scene(kind)
    s = oracle_mod.OracleScene(sc)
    hw, cw = s.transport(N, seed=11)
    ha, ca = s.transport(N, seed=12, analog=True)
    n_layers = len(sc["scanner"]["layers"])
    tw, ta = _tallies(hw, n_layers), _tallies(ha, n_layers)
    for name, a, b in zip(("layer x process", "energy per event", "hits per event"), tw, ta):
        chi2, df, p = chi2_two_sample(a, b)
        print(f"{kind} {name}: chi2 {chi2:.1f} / {df}, p {p:.3f}")
        assert p > 1e-3, (kind, name)
    # real collisions per event: Woodcock counts accepted steps, analog every flight end
    rw, ra = cw["real"], ca["real"]
    z = (rw - ra) / np.sqrt(rw + ra)
    print(f"{kind} real collisions {rw} vs {ra} (z {z:.2f}); hits {len(hw)} vs {len(ha)}")
    assert abs(z) < 4
    assert cw["capped"] == 0 and ca["capped"] == 0
