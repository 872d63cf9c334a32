"""Batched runs through the C ABI: one persistent launch over a table of
instances reproduces, instance by instance and bit for bit, the plain runs of
the same scanner, source, event range and instance id (which are themselves
parity-tested against the oracle), and a batch instance matches the oracle's
tallies for its own random-number instance id."""
import numpy as np
import pytest

import gpet_inputs as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctxs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_07327_amd.gpet import Context
    a, b = Context(0), Context(0)
    yield a, b
    a.close()
    b.close()


def _instances():
    """Uneven instances of three designs: a single event, an empty instance,
    ranges that do not start at 0 (one near 2^31), ragged counts."""
    spec = [("A", (0.0, 0.0, 0.0), 5000, 0, 0), ("B", (1.5, 0.0, 0.0), 1, 7, 3),
            ("C", (0.0, 2.0, 1.0), 12001, 100, 5), ("C", (0.0, 0.0, 0.0), 0, 0, 9),
            ("A", (3.0, 0.0, 0.0), 777, 2**31, 11), ("C", (10.0, 0.0, 0.0), 8191, 0, 12),
            ("B", (0.0, 0.0, 20.0), 3333, 40, 13)]
    out = []
    for d, pos, n, first, iid in spec:
        sc = G.small_animal_scene(d, pos, n_events=max(n, 1))
        out.append({"scanner": sc["scanner"], "source": sc["source"], "n_events": n, "first_event": first,
                    "instance": iid, "scene": sc})
    return out


def _canon(g):
    """Hits in (instance, event, gid, aux) order (instance ids repeat event ids)."""
    inst = g.get("instance", np.zeros(len(g["event"]), np.int32))
    key = np.lexsort((g["aux"], g["gid"], g["event"], inst))
    return {k: v[key] for k, v in g.items()}


def _plain(ctx, inst, seed):
    sc = inst["scene"]
    ctx.set_scene(sc)
    hits, st = ctx.transport(inst["n_events"], seed=seed, first=inst["first_event"], instance=inst["instance"])
    sg, (ca, cb) = ctx.digitize(hits, seed=seed + 1, instance=inst["instance"])
    return hits, sg, ca.cpu().numpy(), cb.cpu().numpy(), st


def test_batch_matches_plain_runs_bit_for_bit(ctxs):
    from paper_2603_07327_amd.gpet import Batch
    cb, cp = ctxs
    inst = _instances()
    sc0 = inst[0]["scene"]
    cb.set_materials(sc0["materials"], sc0["physics"])
    cb.set_phantom(None)
    b = Batch(cb, inst)
    seed = 77
    hits, st = b.transport(seed=seed)
    sg, (ca, cc), per = b.digitize(hits, seed=seed + 1)
    g = hits.numpy()
    s = sg.numpy()
    pa, pb = ca.cpu().numpy(), cc.cpu().numpy()
    assert st["events"] == sum(i["n_events"] for i in inst)
    assert np.all(np.diff(s["instance"]) >= 0)
    tot_steps = 0
    for i, d in enumerate(inst):
        ph, ps, qa, qb, pst = _plain(cp, d, seed)
        tot_steps += pst["steps"]
        mine = {k: v[g["instance"] == i] for k, v in g.items()}
        ref = ph.numpy()
        assert len(mine["event"]) == len(ref["event"]), i
        a, r = _canon(mine), _canon(ref)
        a.pop("instance")
        for k in r:
            assert np.array_equal(a[k], r[k]), (i, k)
        # singles: instance i's block of the batch list equals the plain list
        sel = np.nonzero(s["instance"] == i)[0]
        rs = ps.numpy()
        assert len(sel) == len(rs["event"]), i
        for k in rs:
            assert np.array_equal(s[k][sel], rs[k]), (i, k)
        # coincidences of instance i, as (event, gid) pairs, in the same order
        off = sel[0] if len(sel) else 0
        m = s["instance"][pa] == i if len(pa) else np.zeros(0, bool)
        got = np.stack([pa[m] - off, pb[m] - off], 1) if m.any() else np.zeros((0, 2), np.int64)
        want = np.stack([qa, qb], 1) if len(qa) else np.zeros((0, 2), np.int64)
        assert np.array_equal(got, want), i
        assert per[i] == len(qa), i
    assert st["steps"] == tot_steps
    b.close()


def test_batch_chunk_and_shape_invariance_and_autotune(ctxs):
    from paper_2603_07327_amd.gpet import Batch
    cb, _ = ctxs
    mats, phys, inst = G.batch_sweep(n_scale=2e-3, seed=1)
    inst = inst[:24]
    cb.set_materials(mats, phys)
    cb.set_phantom(None)
    b = Batch(cb, inst)
    ref = None
    for shape in [(0, 48, 1024), (0, 48, 64), (2, 32, 4096), (1, 64, 1)]:
        b.set_launch(*shape)
        h, st = b.transport(seed=5)
        cur = _canon(h.numpy()), h.numpy()["instance"], st["steps"]
        if ref is None:
            ref = cur
            continue
        for k in ref[0]:
            assert np.array_equal(ref[0][k], cur[0][k]), (shape, k)
        assert np.array_equal(np.bincount(ref[1], minlength=24), np.bincount(cur[1], minlength=24))
        assert ref[2] == cur[2]
    hits = b.alloc_hits(int(4 * sum(i["n_events"] for i in inst)))
    r = b.autotune(hits, seed=5)
    assert set(r) >= {"blocks_per_cu", "search_batch", "chunk", "ms", "trials"}
    assert len(r["trials"]) >= 10
    h, st = b.transport(seed=5)
    for k in ref[0]:
        assert np.array_equal(ref[0][k], _canon(h.numpy())[k]), k
    b.close()


def test_batch_instance_matches_oracle_tallies(ctxs, oracle_mod):
    """Batch instance with a nonzero instance id against the oracle run with
    that id (same seed and event ids): hit count within 0.2 %, coincidences
    within 0.5 %."""
    from paper_2603_07327_amd.gpet import Batch
    cb, _ = ctxs
    n = 300_000
    sc = G.small_animal_scene("C", (5.0, 0.0, 0.0), n_events=n)
    other = G.small_animal_scene("A", (0.0, 0.0, 0.0), n_events=20_000)
    cb.set_materials(sc["materials"], sc["physics"])
    cb.set_phantom(None)
    inst = [{"scanner": other["scanner"], "source": other["source"], "n_events": 20_000, "instance": 0},
            {"scanner": sc["scanner"], "source": sc["source"], "n_events": n, "instance": 42}]
    b = Batch(cb, inst)
    hits, _ = b.transport(seed=3)
    _, _, per = b.digitize(hits, seed=3)
    o = oracle_mod.OracleScene(sc)
    rh, _ = o.transport(n, seed=3, instance=42)
    _, rc = o.digitize(rh, seed=3, instance=42)
    nh = int((hits.numpy()["instance"] == 1).sum())
    print("hits", nh, len(rh), "coinc", per[1], len(rc))
    assert abs(nh - len(rh)) / len(rh) <= 0.002
    assert abs(per[1] - len(rc)) / len(rc) <= 0.005
    b.close()


def test_batch_errors(ctxs):
    from paper_2603_07327_amd.gpet import ERR_ARG, ERR_STATE, ERR_UNSUPPORTED, Batch, GpetError
    cb, _ = ctxs
    sc = G.small_animal_scene("C", n_events=1000)
    cb.set_materials(sc["materials"], sc["physics"])
    cb.set_phantom(None)
    inst = [{"scanner": sc["scanner"], "source": sc["source"], "n_events": 1000}]
    b = Batch(cb, inst)
    # hit buffers without instance ids are refused
    plain = cb.alloc_hits(10_000)
    with pytest.raises(GpetError) as e:
        b.transport_into(plain, seed=1)
    assert e.value.code == ERR_ARG
    # the batch points at the context's phantom: changing it invalidates the batch
    cb.set_phantom(None)
    with pytest.raises(GpetError) as e:
        b.transport(seed=1)
    assert e.value.code == ERR_STATE
    b.close()
    # more than four distinct detector materials over the batch
    mats = [G.material("lyso", density=7.4 - 0.1 * k) for k in range(5)] + [G.material("air")]
    cb.set_materials(mats, sc["physics"])
    inst = []
    for k in range(5):
        s = G.small_animal_scanner("A")
        s = dict(s, layers=[dict(s["layers"][0], mat_crystal=k, mat_interval=5)], mat_fill=5)
        inst.append({"scanner": s, "source": sc["source"], "n_events": 10})
    with pytest.raises(GpetError) as e:
        Batch(cb, inst)
    assert e.value.code == ERR_UNSUPPORTED
    # bad event range names the instance
    cb.set_materials(sc["materials"], sc["physics"])
    bad = [{"scanner": sc["scanner"], "source": sc["source"], "n_events": 10, "first_event": 2**32 - 5}]
    with pytest.raises(GpetError) as e:
        Batch(cb, bad)
    assert e.value.code == ERR_ARG and "instance 0" in str(e.value)


def test_batch_graph_replays_match_eager(ctxs):
    """The captured transport step, replayed three times with eager
    transports, digitizer work and synchronizations in between: every replay
    gives the eager hit set and counts."""
    import torch

    from paper_2603_07327_amd.gpet import Batch
    cb, _ = ctxs
    mats, phys, inst = G.batch_sweep(n_scale=1e-3, seed=2)
    inst = inst[:20]
    cb.set_materials(mats, phys)
    cb.set_phantom(None)
    b = Batch(cb, inst)
    ref_h, ref_st = b.transport(seed=9)
    ref = _canon(ref_h.numpy())
    g_hits = b.alloc_hits(ref_h.count + 4096)
    b.graph_capture(g_hits, seed=9)
    for rep in range(3):
        other, _ = b.transport(seed=100 + rep)        # eager work on the same counters
        b.digitize(other, seed=rep)
        torch.cuda.synchronize()
        b.graph_launch()
        rc, st = b.read_counts(g_hits)
        assert rc == 0 and g_hits.count == ref_h.count, rep
        # every work counter but the scheduling-dependent loop-trip count
        assert {k: v for k, v in st.items() if k != "wave_trips"} == \
            {k: v for k, v in ref_st.items() if k != "wave_trips"}, rep
        got = _canon(g_hits.numpy())
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (rep, k)
    b.close()


RESPONSE = {"time_fwhm_ps": 500.0, "doi_fwhm_mm": 2.0, "dead_time_ps": 100_000_000,
            "dead_time_mode": "nonparalyzable", "dead_time_level": "module", "light_sharing": 0.3}


@pytest.mark.parametrize("response", [None, RESPONSE], ids=["plain", "response"])
def test_batch_readout_and_sweep_match_plain(ctxs, response):
    """Module readout and a three-window sweep in one batched pass (and with
    time / DOI blur and a 100 us dead time per module): every instance's
    singles and counts equal its plain run's."""
    from paper_2603_07327_amd.gpet import Batch
    cb, cp = ctxs
    inst = _instances()
    sc0 = inst[0]["scene"]
    cb.set_materials(sc0["materials"], sc0["physics"])
    cb.set_phantom(None)
    b = Batch(cb, inst)
    seed = 31
    sweep = [(150.0, 700.0), (350.0, 700.0), (450.0, 700.0)]
    hits, _ = b.transport(seed=seed)
    sg, (ca, _), per, counts = b.digitize(hits, seed=seed + 1, readout="module", sweep=sweep, response=response)
    s = sg.numpy()
    assert counts.shape == (len(sweep), len(inst))
    if response:
        assert np.count_nonzero(s["in_window"].view(np.uint32) & 2) > 0
    for i, d in enumerate(inst):
        cp.set_scene(d["scene"])
        ph, _ = cp.transport(d["n_events"], seed=seed, first=d["first_event"], instance=d["instance"])
        ps, (qa, _), pc = cp.digitize(ph, seed=seed + 1, instance=d["instance"], readout="module", sweep=sweep,
                                      response=response)
        rs = ps.numpy()
        sel = s["instance"] == i
        for k in rs:
            assert np.array_equal(s[k][sel], rs[k]), (i, k)
        assert per[i] == len(qa), i
        assert np.array_equal(counts[:, i], pc), (i, counts[:, i], pc)
    b.close()


def test_batch_full_size_sampled_events(ctxs, oracle_mod):
    """The benchmark's batched sweep at full size (144 instances, 3.7e8
    events in one persistent launch): sampled blocks of event ids of sampled
    instances, selected on the device, match the oracle's re-simulation of
    the same ids with the instance's scanner, source and random-number id."""
    import torch
    from paper_2603_07327_amd.gpet import Batch
    cb, _ = ctxs
    mats, phys, inst = G.batch_sweep(n_scale=1.0, seed=0)
    total = sum(d["n_events"] for d in inst)
    cb.set_materials(mats, phys)
    cb.set_phantom(None)
    b = Batch(cb, inst)
    hits, st = b.transport(seed=0, capacity=int(1.2 * total))
    assert st["events"] == total and st["capped"] == 0
    v = hits.view()
    rng = np.random.default_rng(8)
    n_ev = n_diff = n_hits = 0
    for i in sorted(rng.choice(len(inst), 8, replace=False).tolist()):
        d = inst[i]
        o = oracle_mod.OracleScene(G.scene(mats, phys, d["scanner"], d["source"]))
        size = min(100, d["n_events"])
        for first in sorted({0, int(rng.integers(0, d["n_events"] - size + 1))}):
            sel = (v.instance == i) & (v.event >= first) & (v.event < first + size)
            idx = torch.nonzero(sel).flatten()
            g_ev = v.event[idx].cpu().numpy().view(np.uint32)
            g_gid = v.gid[idx].cpu().numpy().view(np.uint32)
            g_e = v.edep_kev[idx].cpu().numpy()
            rh, _ = o.transport(size, seed=0, first=first, instance=d["instance"])
            for e in range(first, first + size):
                a = rh[rh["event"] == e]
                m = g_ev == e
                n_ev += 1
                n_hits += len(a)
                if not np.array_equal(np.sort(g_gid[m]), np.sort(a["gid"])):
                    n_diff += 1
                    continue
                if len(a):
                    np.testing.assert_allclose(np.sort(g_e[m].astype(np.float64)), np.sort(a["edep"]),
                                               rtol=2e-4, atol=2e-3)
    print(f"{total} events in one launch; {n_ev} sampled events, {n_hits} oracle hits, {n_diff} differing")
    assert n_hits > 100
    assert n_diff <= max(3, 0.01 * n_ev)
    b.close()
