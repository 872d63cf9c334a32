"""gpet_digitize_noalloc (the digitizer on the library's static scratch)
against gpet_digitize: the same kernels, so every output must be equal bit
for bit.  Two calls in a row, the second on a smaller input with other
options, so that what the first call left in the shared scratch cannot leak
into the second; and a call too large for the scratch is refused."""
import numpy as np
import pytest

import gpet_inputs as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_07327_amd.gpet import Context
    c = Context(0)
    yield c
    c.close()


def _same_outputs(a, b):
    (sa, ca), (sb, cb) = a[:2], b[:2]
    assert sa.count == sb.count and sa.windowed == sb.windowed
    na, nb = sa.numpy(), sb.numpy()
    for k in na:
        assert np.array_equal(na[k], nb[k]), k
    assert np.array_equal(ca[0].cpu().numpy(), cb[0].cpu().numpy())
    assert np.array_equal(ca[1].cpu().numpy(), cb[1].cpu().numpy())
    if len(a) == 3:
        assert np.array_equal(a[2], b[2])


def test_noalloc_equals_digitize_on_two_calls(ctx, oracle_mod):
    cases = [
        # 300k events of design C: about 260k hits, crystal readout with tallies
        dict(n=300_000, seed=3, kw={}),
        # a smaller run: module readout, non-paralyzable module dead time, a window sweep
        dict(n=60_000, seed=4, kw={"readout": "module", "sweep": [(250.0, 700.0), (450.0, 700.0)],
                                   "response": {"dead_time_ps": 20_000, "dead_time_mode": "nonparalyzable",
                                                "dead_time_level": "module"}}),
    ]
    for c in cases:
        sc = G.small_animal_scene("C", pos=(5.0, 0.0, 0.0), n_events=c["n"])
        if c["kw"].get("response"):
            sc = dict(sc)
            sc["source"] = dict(sc["source"], duration_ps=50_000_000)
        ctx.set_scene(sc)
        hits, _ = ctx.transport(c["n"], seed=c["seed"])
        print(f"noalloc case: {c['n']} events, {hits.count} hits, options {sorted(c['kw'])}", flush=True)
        t_got, t_ref = ctx.alloc_tallies(), ctx.alloc_tallies()
        got = ctx.digitize_noalloc(hits, seed=c["seed"], tallies=t_got, **c["kw"])
        ref = ctx.digitize(hits, seed=c["seed"], tallies=t_ref, **c["kw"])
        _same_outputs(got, ref)
        for k in t_ref:
            assert np.array_equal(t_got[k].cpu().numpy(), t_ref[k].cpu().numpy()), k
        assert len(ref[1][0]) > 0


def test_noalloc_refuses_inputs_beyond_its_scratch(ctx, oracle_mod):
    import torch
    from paper_2603_07327_amd.gpet import GpetError, HitList
    sc = G.small_animal_scene("C", n_events=10)
    ctx.set_scene(sc)
    n = 4_000_000  # about 146 MB of sort buffers: beyond the 128 MiB scratch
    g = torch.Generator(device="cpu").manual_seed(0)
    ev = torch.sort(torch.randint(0, 4_000_000, (n,), generator=g, dtype=torch.int32)).values
    gid = torch.randint(0, ctx.info.n_crystals, (n,), generator=g, dtype=torch.int32)
    h = HitList(ev.to(ctx.dev), gid.to(ctx.dev), torch.full((n,), 511.0, device=ctx.dev),
                torch.full((n,), 1.0, device=ctx.dev), torch.zeros(n, dtype=torch.int64, device=ctx.dev),
                torch.zeros(n, dtype=torch.int32, device=ctx.dev), n, 0, 4_000_000)
    with pytest.raises(GpetError, match="fixed scratch"):
        ctx.digitize_noalloc(h, seed=1)
    # the no-allocation entry point still serves a small call afterwards
    m = 1000
    small = HitList(h.event[:m], h.gid[:m], h.edep_kev[:m], h.depth_mm[:m],
                    (h.event[:m].to(torch.int64) * 58_800_000), h.aux[:m], m, 0, 4_000_000)
    _same_outputs(ctx.digitize_noalloc(small, seed=2), ctx.digitize(small, seed=2))
