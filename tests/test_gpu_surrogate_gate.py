"""The surrogate's acceptance gate on the hot-rod phantom workload (design C,
water cylinder, six-sector rods): a factored network (energy classes, then
the position in the 13 x 13 neighbourhood of both layers) trained on the
pairs that the full transport records from 1.64e9 events at seed 7 (about
1e8 pairs; those whose largest deposit lies outside the neighbourhood are
left out, so the network samples the outcome given that it lies inside),
then 1e8 events transported with it and digitized, against full transport.

Gates (the matched-tally bars of the surrogate form):
* matched seeds (seed 0 both; the photons that never reach the network
  follow identical histories): sensitivity within 0.5 % relative;
* independent seeds (full transport at seed 1): per-crystal in-window
  singles pass a two-sample chi-square at p > 0.01, and the two-proportion
  z-test of the sensitivity at p > 0.01."""
import math
import time

import numpy as np
import pytest
from scipy import stats

import gpet_inputs as G
from tests.gpu_util import chi2_two_sample

pytestmark = pytest.mark.gpu

# domain: entries whose 13 x 13 neighbourhood fits each layer's array; classes:
# the 25 x 25 neighbourhood (half width 12; positions past an array's edge are
# never drawn), so only deposits more than 12 crystals away or in another
# module or panel are truncated
SPEC = {"half_width": 6, "n_ebins": 18, "ebin_kev": 16.0, "class_half_width": 12}
W = 2 * SPEC["class_half_width"] + 1
N1, N2 = SPEC["n_ebins"] + 2, 2 * W * W
TRAIN_EVENTS = 1_640_000_000
SLICE = 20_000_000
SCHEDULE = ((8000, 1e-3), (3000, 3e-4), (1000, 1e-4))  # Adam steps of batch 8192 and their step size
N_EVAL = 100_000_000


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_07327_amd.gpet import Context
    c = Context(0)
    yield c
    c.close()


def _train(ctx):
    import torch

    from paper_2603_07327_amd.gpet import Mlp, pack_params
    hits = ctx.alloc_hits(int(1.3 * SLICE))
    pairs = ctx.alloc_pairs(2 * SLICE)
    xs, ys = [], []
    n_rec = n_trunc = 0
    for first in range(0, TRAIN_EVENTS, SLICE):
        rc, _ = ctx.surrogate_pairs_into(hits, pairs, SLICE, seed=7, first=first, spec=SPEC)
        assert rc == 0
        k = pairs["count"]
        fl = pairs["flags"][:k]
        keep = (fl & 1) == 0
        n_rec += k
        n_trunc += int(k - keep.sum())
        # pairs arrive in the order photons reach the queue: put them in
        # (event, photon) order so that the training batches are reproducible
        key = (pairs["event"][:k].to(torch.int64) * 2 + ((fl >> 2) & 1).to(torch.int64))[keep]
        order = torch.argsort(key)
        xs.append(pairs["x"][: 6 * k].view(k, 6)[keep][order].clone())
        ys.append(pairs["label"][:k][keep][order].clone())
    del pairs, hits
    x, y = torch.cat(xs), torch.cat(ys)
    del xs, ys
    sizes = [6, *G.SURROGATE_HIDDEN, N1 + N2]
    init = np.concatenate([pack_params(G.mlp_init(sizes, seed=1)), np.zeros((N1 - 1) * N2, np.float32)])
    net = Mlp(ctx, sizes, init, n_first=N1)
    t0 = time.perf_counter()
    for steps, lr in SCHEDULE:  # Adam continues across the calls; the step size decays
        losses = net.train(x, y, steps=steps, batch=8192, lr=lr, seed=3)
    torch.cuda.synchronize()
    print(f"pairs recorded {n_rec} (truncated {n_trunc / n_rec:.4f}), trained on {len(y)}, {SCHEDULE} in "
          f"{time.perf_counter() - t0:.1f} s, last loss {np.mean(losses[-200:]):.3f}", flush=True)
    del x, y
    torch.cuda.empty_cache()
    return net, n_trunc / n_rec


def test_surrogate_gate_against_full_transport(ctx):
    sc = G.hot_rod_scene(n_events=N_EVAL)
    ctx.set_scene(sc)
    net, p_trunc = _train(ctx)
    hits = ctx.alloc_hits(int(1.4 * N_EVAL))
    singles = ctx.alloc_singles(int(1.3 * N_EVAL))
    coinc = (ctx._empty(N_EVAL // 2, ctx.torch.int32), ctx._empty(N_EVAL // 2, ctx.torch.int32))
    nc = ctx.info.n_crystals

    def run(mode, seed):
        sst = None
        if mode == "plain":
            rc, _ = ctx.transport_into(hits, N_EVAL, seed=seed)
        else:
            rc, _, sst = ctx.surrogate_transport_into(net, hits, N_EVAL, seed=seed, spec=SPEC)
        assert rc == 0, mode
        rc, n_coinc = ctx.digitize_into(hits, singles, coinc, seed=seed)
        assert rc == 0, mode
        s = singles.numpy()
        return n_coinc, np.bincount(s["gid"][s["in_window"] != 0], minlength=nc), sst

    c_sur, h_sur, sst = run("surrogate", 0)
    c_plain, h_plain, _ = run("plain", 0)
    c_ind, h_ind, _ = run("plain", 1)
    rel = c_sur / c_plain - 1.0
    _, _, p_chi2 = chi2_two_sample(h_sur, h_ind)
    p1, p2 = c_sur / N_EVAL, c_ind / N_EVAL
    pp = (c_sur + c_ind) / (2 * N_EVAL)
    z = (p1 - p2) / math.sqrt(pp * (1 - pp) * 2 / N_EVAL)
    p_z = 2 * stats.norm.sf(abs(z))
    print(f"coincidences: surrogate {c_sur}, full transport {c_plain} (matched, {100 * rel:+.3f} %), "
          f"{c_ind} (independent, z {z:+.2f}, p {p_z:.3f}); per-crystal chi2 p {p_chi2:.3f}; "
          f"photons on the network {sst['entries'] / (2 * N_EVAL):.4f}, sampled none {sst['none'] / sst['entries']:.4f}, "
          f"truncated share of the recorded pairs {p_trunc:.4f}")
    net.close()
    assert abs(rel) <= 0.005
    assert p_chi2 > 0.01
    assert p_z > 0.01
