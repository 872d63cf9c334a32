"""Throughput benchmark: annihilation events/s on one MI355X.

Workload: the synthetic small-animal sensitivity sweep -- 12 panels at 65 mm,
4 modules of 24 x 24 LYSO crystals (1.0 mm pitch) per panel, designs A (one
20 mm layer), B (two aligned 10 mm layers, 0.2 mm gap) and C (two 10 mm
layers, inner 23 x 23 offset by half a pitch); point source stepped over the
sweep positions; 1e7 events per design and position; 350-650 keV window,
16 % resolution, 3 ns coincidence window.

One step = one source position run through all three designs (3e7 events):
transport (phantom-free) and the full digitizer (adder, blur, window,
coincidence sorting) for each design, with all buffers resident in HBM.

Prints one JSON line (see the keys below).  The CPU baseline times the FP64
oracle on a bounded sample of the same workload on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import gpet_inputs as G  # noqa: E402

# Algorithmic VALU work per primitive, in VALU lane-operations per lane, with
# quarter-rate instructions (32-bit integer multiplies, transcendentals) weighted
# 4: the weighted instruction counts of straight-line gfx950 builds of each
# primitive in its division-free form (hardware reciprocal, rsq, sin/cos in
# revolutions, 64-bit-multiply Philox), minus an empty load/store kernel.
UNIT_COST = {"philox": 156, "step": 142, "kahn": 38, "rotation": 54, "slab": 88, "source": 18,
             "ring_test": 65, "ring_axial": 26, "ring_prune": 131}
VALU_PEAK = 256 * 64 * 2.4e9  # lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz (no packed FP32)
# Philox blocks of the event stream per annihilation: direction and time for
# point and beam sources, plus the emission point for rod sources
EVENT_BLOCKS = {"point": 2, "beam": 2, "rods": 3}
TRANSPORT_SOURCES = ("paper_2603_07327_amd/csrc/transport.hip", "paper_2603_07327_amd/csrc/gpet_device.hpp",
                     "paper_2603_07327_amd/csrc/transport_common.hpp")


def algorithmic_work(stats: dict, ring: bool = True, source: str = "point") -> float:
    """VALU lane-ops the method needs for a transport launch with these counts:
    W = (N_blocks + b_event N_events) c_philox + N_steps c_step + N_trials c_kahn
        + N_scatter c_rot + W_search + N_events c_source, where N_blocks counts
    the photon streams' blocks and b_event the event stream's blocks per
    annihilation (EVENT_BLOCKS of the source kind), and for a ring of panels
    W_search = N_search c_axial + N_tests c_ring_test + N_pruned c_prune
    (N_tests: panel boxes tested, N_pruned: searches that first narrowed the
    candidates by azimuth) and otherwise N_tests c_slab."""
    if ring:
        w_search = (stats["searches"] * UNIT_COST["ring_axial"] + stats["panel_tests"] * UNIT_COST["ring_test"]
                    + stats["pruned_searches"] * UNIT_COST["ring_prune"])
    else:
        w_search = stats["panel_tests"] * UNIT_COST["slab"]
    return ((stats["blocks"] + EVENT_BLOCKS[source] * stats["events"]) * UNIT_COST["philox"]
            + stats["steps"] * UNIT_COST["step"] + stats["kahn_trials"] * UNIT_COST["kahn"]
            + stats["scatters"] * UNIT_COST["rotation"] + w_search + stats["events"] * UNIT_COST["source"])


# The same work in the survey's form, W = N_blk c_philox + N_step c_step +
# N_trial c_kahn + N_int c_rot + N_search n_panels c_slab + N_events c_src,
# with the survey's order-of-magnitude unit costs (c_src is not estimated
# there: the measured 18 is used) and the oracle's own counts; the full panel
# search is charged (every panel's slab test), not the pruned one the kernel
# runs.
SURVEY_UNIT_COST = {"philox": 140, "step": 65, "kahn": 25, "rotation": 35, "slab": 25, "source": 18}


def survey_form_work(counts: dict, n_panels: int, source: str = "point", cost=None) -> float:
    c = cost or SURVEY_UNIT_COST
    return ((counts["blocks"] + EVENT_BLOCKS[source] * counts["events"]) * c["philox"]
            + counts["steps"] * c["step"] + counts["kahn_trials"] * c["kahn"] + counts["scatters"] * c["rotation"]
            + counts["searches"] * n_panels * c["slab"] + counts["events"] * c["source"])


# Bytes each digitizer stage moves per item, as built: hit keys 24, hit sort
# 60 (count, scatter, wave sort), run heads and their scan 24, adder 32 per
# hit (key, index, segment, energy / depth / time) and 28 per single written;
# the blur (inside the adder at crystal readout) 12 written, window scan 12,
# time keys 20 per single; time keys written 12, time sort 96 (two radix
# passes, bucket starts, wave sort) and pairing 40 per windowed single; 8 per
# coincidence written.
DIGI_BYTES = {"hit": 24 + 60 + 24 + 32, "single": 28 + 12 + 12 + 20, "windowed": 12 + 96 + 40, "coinc": 8}


def digitizer_survey_bytes(hits: int, windowed: int) -> float:
    """The sort traffic in the survey's form: 2 (8 + 4) bytes per item and
    pass, 7 passes over the hits and 8 over the singles the sorter takes."""
    return 24.0 * (7 * hits + 8 * windowed)
HBM_PEAK = 8.0e12


def digitizer_bytes(hits: int, singles: int, windowed: int, coinc: int) -> float:
    return (hits * DIGI_BYTES["hit"] + singles * DIGI_BYTES["single"] + windowed * DIGI_BYTES["windowed"]
            + coinc * DIGI_BYTES["coinc"])


def transport_source_hash() -> str:
    """Hash of the transport kernel's sources without their // comments and
    blank lines, so that a change of comments keeps the counters valid."""
    import hashlib
    h = hashlib.sha256()
    for f in TRANSPORT_SOURCES:
        for line in open(os.path.join(ROOT, f), encoding="utf-8"):
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(events_per_launch: int):
    """HBM bytes per transport launch from the committed counter summary, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "k_transport_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != transport_source_hash():
        return None
    return d["bytes_per_event"] * events_per_launch


def survey_form_roofline(probe: dict, oracle_counts: dict, n: int) -> dict:
    """The transport fraction of the VALU peak three ways, for one launch of
    design C with the source at the centre (1e7 events): the headline work
    model (the kernel's own counts, pruned ring search), the survey's formula
    with its estimated unit costs and the oracle's counts (every panel's slab
    test charged per search), and the survey's formula with the measured unit
    costs and the oracle's counts."""
    sec = probe["kernel_ms"] * 1e-3
    oc = {k: v * n for k, v in oracle_counts.items()}
    w_head = algorithmic_work(probe["stats"], ring=True, source="point")
    w_survey = survey_form_work(oc, 12, "point")
    measured = dict(SURVEY_UNIT_COST, philox=UNIT_COST["philox"], step=UNIT_COST["step"], kahn=UNIT_COST["kahn"],
                    rotation=UNIT_COST["rotation"], slab=UNIT_COST["slab"], source=UNIT_COST["source"])
    w_survey_measured = survey_form_work(oc, 12, "point", measured)
    return {"workload": "design C, source at the centre, 1e7 events (one transport launch)", "kernel_ms": probe["kernel_ms"],
            "peak": VALU_PEAK / 1e12, "unit": "TVALU-op/s",
            "headline_model": {"work_per_launch": w_head, "frac": w_head / sec / VALU_PEAK,
                               "counts": "kernel counters", "search": "pruned ring tests"},
            "survey_form_survey_costs": {"work_per_launch": w_survey, "frac": w_survey / sec / VALU_PEAK,
                                         "unit_costs": SURVEY_UNIT_COST, "counts": "oracle (per event x 1e7)",
                                         "search": "12 slab tests per search"},
            "survey_form_measured_costs": {"work_per_launch": w_survey_measured,
                                           "frac": w_survey_measured / sec / VALU_PEAK, "unit_costs": measured,
                                           "counts": "oracle (per event x 1e7)", "search": "12 slab tests per search"},
            "oracle_counts_per_event": oracle_counts,
            "kernel_counts_per_event": {k: v / n for k, v in probe["stats"].items()}}


def cpu_baseline(target_s: float = 12.0):
    """Oracle events/s (transport + digitizer) on a bounded sample of design C:
    calls of up to 2e7 events (the oracle keeps every hit of a call in host
    memory) until at least target_s seconds have run; then one host thread
    on a smaller sample for at least 2 s.  Also returns the oracle's work
    counters per event."""
    from oracle import oracle as O
    O.build(force=False)
    threads = O.num_threads()
    sc = G.small_animal_scene("C", (0.0, 0.0, 0.0), n_events=200_000_000)
    s = O.OracleScene(sc)
    n0 = 100_000
    t0 = time.perf_counter()
    h, _ = s.transport(n0, seed=1)
    s.digitize(h, seed=1)
    dt0 = time.perf_counter() - t0
    per_call = int(min(20_000_000, max(n0, n0 * target_s / 3 / max(dt0, 1e-3))))
    done, dt, counts = 0, 0.0, {}
    while dt < target_s:
        t0 = time.perf_counter()
        h, c = s.transport(per_call, seed=1, first=done)
        s.digitize(h, seed=1)
        dt += time.perf_counter() - t0
        done += per_call
        for k, v in c.items():
            counts[k] = counts.get(k, 0) + v
        del h
    # one host thread (events are independent): a trial sizes a sample of
    # about 2.5 s
    O.set_threads(1)
    try:
        t0 = time.perf_counter()
        h, _ = s.transport(50_000, seed=1)
        s.digitize(h, seed=1)
        n1 = max(50_000, int(50_000 * 2.5 / max(time.perf_counter() - t0, 1e-3)))
        t0 = time.perf_counter()
        h, _ = s.transport(n1, seed=1)
        s.digitize(h, seed=1)
        dt1 = time.perf_counter() - t0
    finally:
        O.set_threads(threads)
    return {"value": done / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": f"design C, source at the centre, events [0, {done}) seed 1 in calls of {per_call}, "
                      f"transport + digitizer, {dt:.1f} s",
            "single_core": {"value": n1 / dt1, "events": n1, "seconds": dt1},
            "counts_per_event": {k: v / done for k, v in counts.items()}}


SWEEP_WINDOWS = [(150.0, 700.0), (250.0, 700.0), (350.0, 700.0), (450.0, 700.0)]


def window_sweep(ctxs, n, seed, pos):
    """The sensitivity study of the last step's hits (one source position):
    coincidences / events in the four energy windows at crystal, module and
    panel readout for each design, the symmetric difference
    200 (S_A - S_C) / (S_A + S_C) between the one-layer design A and the offset
    two-layer design C, and the digitizer time of a pass that lists the
    350-650 keV coincidences and counts the four windows."""
    import torch
    sens, ms = {}, {}
    for d, c, hits, singles, coinc in ctxs:
        sens[d] = {}
        for level in ("crystal", "module", "panel"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, _, cnt = c.digitize_into(hits, singles, coinc, seed=seed, readout=level, sweep=SWEEP_WINDOWS)
            torch.cuda.synchronize()
            ms.setdefault(level, []).append((time.perf_counter() - t0) * 1e3)
            if rc != 0:
                raise RuntimeError("window sweep: capacity")
            sens[d][level] = [int(x) / n for x in cnt]
    dsym = {level: [200.0 * (a - b) / (a + b) if a + b > 0 else 0.0
                    for a, b in zip(sens["A"][level], sens["C"][level])] for level in sens["A"]}
    return {"windows_kev": SWEEP_WINDOWS, "source_position_mm": list(pos), "events_per_design": n,
            "sensitivity": sens, "dsym_A_vs_C_percent": dsym,
            "ms_per_design": {k: float(np.mean(v)) for k, v in ms.items()}}


# the paper's Table 1 (Derenzo rods, 10 runs): hit and coincidence events
PAPER_TABLE1 = {"1CL": (2671908, 378152), "1CL-split": (2673328, 378866), "2CL": (2620170, 363893)}


def paper_scanners_form(n: int = 10_000_000):
    """The paper's three validation scanners (H2RSPET-1CL, -1CL-split, -2CL)
    with the Derenzo rods in a water cube: transport + digitizer events/s
    (median of 3 after one warm-up) and hits and coincidences of each, with
    their ratios to 1CL next to those of the paper's Table 1 (context only:
    the attenuation tables here are synthetic)."""
    import torch

    from paper_2603_07327_amd.gpet import Context
    out = {"workload": f"H2RSPET 1CL / 1CL-split / 2CL (10 panels at 85 mm, 6 modules of 51x51), Derenzo rods "
                       f"(116 rods, 0.3-1.0 mm) in a 40.25 mm water cube, {n:.0e} events"}
    res = {}
    for kind in ("1CL", "1CL-split", "2CL"):
        c = Context(0)
        c.set_scene(G.derenzo_scene(kind, n))
        c.enable_timing(True)
        hits = c.alloc_hits(int(3.0 * n))
        singles = c.alloc_singles(int(2.5 * n))
        coinc = (c._empty(n, torch.int32), c._empty(n, torch.int32))
        times, kms = [], []
        for r in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st = c.transport_into(hits, n, seed=0)
            rc2, nc = c.digitize_into(hits, singles, coinc, seed=0)
            torch.cuda.synchronize()
            if rc or rc2:
                raise RuntimeError("paper scanners: capacity")
            if r:
                times.append(time.perf_counter() - t0)
                kms.append(c.timings()[0])
        res[kind] = {"value": n / float(np.median(times)), "unit": "events/s", "ms": float(np.median(times)) * 1e3,
                     "transport_kernel_ms": float(np.median(kms)), "hits": hits.count, "singles": singles.count,
                     "coincidences": nc}
        c.close()
    for kind in res:
        res[kind]["hits_ratio_to_1CL"] = res[kind]["hits"] / res["1CL"]["hits"]
        res[kind]["coincidences_ratio_to_1CL"] = res[kind]["coincidences"] / res["1CL"]["coincidences"]
        ph, pc = PAPER_TABLE1[kind]
        res[kind]["paper_hits_ratio_to_1CL"] = ph / PAPER_TABLE1["1CL"][0]
        res[kind]["paper_coincidences_ratio_to_1CL"] = pc / PAPER_TABLE1["1CL"][1]
    out.update(res)
    return out


def config1_form():
    """The small ring (8 panels of 8 x 8 crystals, point source at the
    centre): transport + digitizer events/s at 1e5 events (launch-bound,
    median of 5) and 1e8 events, and the oracle's rate on a bounded sample."""
    import torch

    from oracle import oracle as O
    from paper_2603_07327_amd.gpet import Context
    out = {"workload": "8 panels at 40 mm, 8x8 LYSO 1.5 mm crystals, point source at the centre"}
    for n, reps in ((100_000, 5), (100_000_000, 1)):
        sc = G.ring8_scene(n_events=n)
        c = Context(0)
        c.set_scene(sc)
        hits = c.alloc_hits(max(4096, int(0.5 * n)))
        singles = c.alloc_singles(max(4096, int(0.5 * n)))
        coinc = (c._empty(max(4096, n // 10), torch.int32), c._empty(max(4096, n // 10), torch.int32))
        times = []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, _ = c.transport_into(hits, n, seed=r)
            rc2, nc = c.digitize_into(hits, singles, coinc, seed=r)
            torch.cuda.synchronize()
            if rc or rc2:
                raise RuntimeError("config 1: capacity")
            if r:
                times.append(time.perf_counter() - t0)
        out[f"events_{n}"] = {"value": n / float(np.median(times)), "unit": "events/s",
                              "ms": float(np.median(times)) * 1e3, "coincidences": nc}
        c.close()
    s = O.OracleScene(G.ring8_scene(n_events=1_000_000))
    t0 = time.perf_counter()
    h, _ = s.transport(1_000_000, seed=1)
    s.digitize(h, seed=1)
    dt = time.perf_counter() - t0
    out["oracle"] = {"value": 1_000_000 / dt, "unit": "events/s", "cores": O.num_threads(), "events": 1_000_000}
    return out


# the optional physics at published values: 0.5 deg acollinearity (photon
# pairs in water), the 0.102 mm positron range the paper quotes for 18F
# (Sec. 4), with a 300 ps timing and 2 mm DOI resolution, 10 % light sharing
# and a 1 us non-paralyzable dead time per crystal (the singles are crystal singles: at
# module level the second crystal single of a photon that scatters inside a
# module would fall in its dead time)
EXT_SOURCE = {"acolinearity_fwhm_deg": 0.5, "positron_range_fwhm_mm": 0.102}
EXT_RESPONSE = {"time_fwhm_ps": 300.0, "doi_fwhm_mm": 2.0, "dead_time_ps": 1_000_000,
                "dead_time_mode": "nonparalyzable", "dead_time_level": "crystal", "light_sharing": 0.1}


def extensions_form(n: int = 10_000_000):
    """Design C, source at the centre: transport + digitizer with every
    optional effect on against the paper's setting (all off), median of 3
    after one warm-up each; kernel times from the library's HIP events."""
    import torch

    from paper_2603_07327_amd.gpet import Context
    c = Context(0)
    c.enable_timing(True)
    hits = c.alloc_hits(int(3.2 * n))
    singles = c.alloc_singles(int(2.2 * n))
    coinc = (c._empty(n, torch.int32), c._empty(n, torch.int32))
    out = {"workload": f"design C, point source at the centre, {n:.0e} events",
           "source": EXT_SOURCE, "response": EXT_RESPONSE}
    for form in ("off", "on"):
        src = G.point_source((0.0, 0.0, 0.0), n)
        if form == "on":
            src.update(EXT_SOURCE)
        sc = G.small_animal_scene("C", (0.0, 0.0, 0.0), n_events=n)
        sc["source"] = src
        c.set_scene(sc)
        resp = EXT_RESPONSE if form == "on" else None
        wall, tk, dg = [], [], []
        for r in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, _ = c.transport_into(hits, n, seed=r)
            rc2, nc = c.digitize_into(hits, singles, coinc, seed=r, response=resp)
            torch.cuda.synchronize()
            if rc or rc2:
                raise RuntimeError("extensions: capacity")
            if r:
                wall.append(time.perf_counter() - t0)
                tm = c.timings()
                tk.append(tm[0])
                dg.append(tm[1])
        lost = 0
        if form == "on":
            lost = int(((singles.in_window[:singles.count] & 2) != 0).sum())
        out[form] = {"value": n / float(np.median(wall)), "unit": "events/s",
                     "transport_kernel_ms": float(np.median(tk)), "digitizer_ms": float(np.median(dg)),
                     "hits": hits.count, "singles": singles.count, "lost_to_dead_time": lost,
                     "coincidences": nc}
    out["slowdown"] = out["off"]["value"] / out["on"]["value"]
    c.close()
    return out


def batched_form(args):
    """The batched design sweep (36 designs x 4 source offsets, log-uniform event
    counts): one persistent transport launch over all instances plus one
    digitizer pass, against the same instances run one by one through the plain
    path (one context per design, source switched per instance).  Both forms
    give identical per-instance coincidence counts (the batch reproduces the
    plain runs bit for bit), so sensitivities match exactly."""
    import torch

    from paper_2603_07327_amd.gpet import ERR_CAPACITY, Batch, Context

    mats, phys, inst = G.batch_sweep(n_scale=args.batched_scale, seed=0)
    total = sum(d["n_events"] for d in inst)
    ctx = Context(0)
    ctx.set_materials(mats, phys)
    ctx.set_phantom(None)
    ctx.enable_timing(True)
    b = Batch(ctx, inst)
    hits = b.alloc_hits(int(3.0 * total))
    rc, _ = b.transport_into(hits, seed=0)
    if rc == ERR_CAPACITY:
        need = hits.count
        del hits
        hits = b.alloc_hits(int(1.02 * need) + 1024)
    tune = b.autotune(hits, seed=0, cache_path=args.autotune_cache,
                      key=f"sweep144 scale={args.batched_scale} {torch.cuda.get_device_name(0)}")
    singles = ctx.alloc_singles(hits.count + 1024, instance=True)
    coinc = (ctx._empty(total // 2 + 1024, torch.int32), ctx._empty(total // 2 + 1024, torch.int32))

    def batch_step(seed):
        rc, st = b.transport_into(hits, seed=seed)
        if rc != 0:
            raise RuntimeError("batched hit capacity too small")
        rc, nc, per = b.digitize_into(hits, singles, coinc, seed=seed)
        if rc != 0:
            raise RuntimeError("batched digitizer capacity too small")
        return per, st

    batch_step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms = []
    for k in range(args.steps):
        per_b, st_b = batch_step(2 + k)
        kms.append(ctx.timings()[0])
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t0) / args.steps
    last_seed = 1 + args.steps
    # the same step with the transport replayed from its captured HIP graph
    # (counter reset + persistent launch, seed fixed at capture), then the
    # digitizer pass (not capturable: it sizes its sort from counts it reads back)
    b.graph_capture(hits, seed=last_seed)

    def graph_step():
        b.graph_launch()
        rc, st = b.read_counts(hits)
        if rc != 0:
            raise RuntimeError("batched hit capacity too small")
        rc, nc, per = b.digitize_into(hits, singles, coinc, seed=last_seed)
        if rc != 0:
            raise RuntimeError("batched digitizer capacity too small")
        return per, st

    per_g, _ = graph_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        per_g, st_g = graph_step()
    torch.cuda.synchronize()
    dt_g = (time.perf_counter() - t0) / args.steps
    b.close()
    del hits, singles, coinc
    ctx.close()
    torch.cuda.empty_cache()

    # the same instances one by one through the plain path
    by_design = {}
    for d in inst:
        key = d["label"].rsplit("_x", 1)[0]
        by_design.setdefault(key, []).append(d)
    plain = []
    for key, group in by_design.items():
        c = Context(0)
        c.set_materials(mats, phys)
        c.set_scanner(group[0]["scanner"])
        c.set_phantom(None)
        nmax = max(d["n_events"] for d in group)
        h = c.alloc_hits(int(4.0 * nmax))
        sg = c.alloc_singles(int(4.0 * nmax))
        cc = (c._empty(nmax, torch.int32), c._empty(nmax, torch.int32))
        plain.append((c, group, h, sg, cc))
    per_p = {}

    def plain_pass(seed):
        for c, group, h, sg, cc in plain:
            for d in group:
                c.set_source(d["source"])
                rc, _ = c.transport_into(h, d["n_events"], seed=seed, first=d["first_event"], instance=d["instance"])
                if rc != 0:
                    raise RuntimeError("plain hit capacity too small")
                rc, nc = c.digitize_into(h, sg, cc, seed=seed, instance=d["instance"])
                if rc != 0:
                    raise RuntimeError("plain digitizer capacity too small")
                per_p[d["instance"]] = nc

    plain_pass(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_pass(last_seed)
    torch.cuda.synchronize()
    dt_p = time.perf_counter() - t0
    for c, *_ in plain:
        c.close()
    sens_b = np.array([per_b[i] for i in range(len(inst))], np.float64)
    sens_p = np.array([per_p[d["instance"]] for d in inst], np.float64)
    sens_g = np.array([per_g[i] for i in range(len(inst))], np.float64)
    rel = np.abs(sens_b - sens_p) / np.maximum(sens_p, 1.0)
    w_b = algorithmic_work(st_b, ring=True, source="point")
    k_ms = float(np.mean(kms))
    return {"workload": "batched design sweep: 36 designs (layer thickness 6/8/10/12 mm x offset 0/0.25/0.5 "
                        "pitch x gap 0/0.2/0.5 mm) x 4 radial source offsets = 144 instances, event counts "
                        "log-uniform in [1e5, 1e7], one persistent transport launch + one digitizer pass",
            "instances": len(inst), "events": total, "value": total / dt_b, "unit": "events/s",
            "ms_per_step": dt_b * 1e3, "transport_kernel_ms": k_ms,
            "roofline": {"bound": "alu", "kernel": "k_transport (batched)", "achieved": w_b / (k_ms * 1e-3) / 1e12,
                         "peak": VALU_PEAK / 1e12, "unit": "TVALU-op/s", "frac": w_b / (k_ms * 1e-3) / VALU_PEAK,
                         "work_per_launch": w_b},
            "graph_replay": {"value": total / dt_g, "ms_per_step": dt_g * 1e3,
                             "same_coincidences_as_plain": bool(np.array_equal(sens_g, sens_p)),
                             "note": "transport from the captured HIP graph (seed fixed at capture), digitizer eager"},
            "plain_one_by_one": {"value": total / dt_p, "ms": dt_p * 1e3},
            "speedup_vs_plain": dt_p / dt_b, "sensitivity_max_rel_diff": float(rel.max()),
            "coincidences": int(sens_b.sum()),
            "autotune": {k: tune[k] for k in ("blocks_per_cu", "search_batch", "chunk", "ms")},
            "stats_last": st_b}




def surrogate_form(args):
    """The hot-rod phantom workload (design C, water cylinder, six-sector rods)
    timed with full transport and with the detector-response surrogate, both
    followed by the full digitizer.  The network (6 -> 4 x 256 -> energy head
    of n_ebins + 2 classes and 2 (2 H + 1)^2 positions with the offset table,
    H = 12 crystals each way around the entry) is first trained on the pairs
    recorded from separate runs (seed 7), about 1e8 of them; those whose
    largest deposit lies outside that neighbourhood are left out, so the
    network samples the outcome given that it lies inside.  The timed runs use seed 0.  Reported: events/s of both forms,
    sensitivities at matched seeds (seed 0 both) and against an independent
    full-transport run (seed 1: two-proportion z-test, per-crystal in-window
    singles chi-square), the share of photons the network took over, the
    truncated share, training cost, and the network's matrix-core rate."""
    import torch
    from scipy import stats as sps

    from paper_2603_07327_amd.gpet import Context, Mlp, pack_params

    n = args.surrogate_events
    spec = {"half_width": args.surrogate_half_width, "n_ebins": args.surrogate_ebins,
            "ebin_kev": args.surrogate_ebin_kev, "class_half_width": args.surrogate_class_half_width}
    W = 2 * max(args.surrogate_half_width, args.surrogate_class_half_width) + 1
    n1, n2 = args.surrogate_ebins + 2, 2 * W * W
    flop_per_entry = 2 * (6 * 256 + 3 * 256 * 256 + 256 * (n1 + n2))  # forward pass
    sc = G.hot_rod_scene(n_events=n)
    ctx = Context(0)
    ctx.set_scene(sc)
    ctx.enable_timing(True)
    # ---- training pairs (seed 7), in slices; truncated pairs left out
    slice_ev = 20_000_000
    hits = ctx.alloc_hits(int(1.3 * slice_ev))
    pairs = ctx.alloc_pairs(2 * slice_ev)
    xs, ys = [], []
    n_rec = n_trunc = 0
    t0 = time.perf_counter()
    done = 0
    while done < args.surrogate_train_events:
        m = min(slice_ev, args.surrogate_train_events - done)
        rc, _ = ctx.surrogate_pairs_into(hits, pairs, m, seed=7, first=done, spec=spec)
        if rc != 0:
            raise RuntimeError("pair generation: capacity")
        k = pairs["count"]
        fl = pairs["flags"][:k]
        keep = (fl & 1) == 0
        n_rec += k
        n_trunc += int(k - int(keep.sum()))
        # (event, photon) order: reproducible batches whatever order the queue filled in
        key = (pairs["event"][:k].to(torch.int64) * 2 + ((fl >> 2) & 1).to(torch.int64))[keep]
        order = torch.argsort(key)
        xs.append(pairs["x"][: 6 * k].view(k, 6)[keep][order].clone())
        ys.append(pairs["label"][:k][keep][order].clone())
        done += m
    del pairs, hits
    x = torch.cat(xs)
    y = torch.cat(ys)
    del xs, ys
    label_none = float((y == 0).double().mean())
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    sizes = [6, *G.SURROGATE_HIDDEN, n1 + n2]
    init = np.concatenate([pack_params(G.mlp_init(sizes, seed=1)), np.zeros((n1 - 1) * n2, np.float32)])
    net = Mlp(ctx, sizes, init, n_first=n1)
    # two thirds of the steps at 1e-3, then a quarter at 3e-4 and the rest at
    # 1e-4 (Adam continues across the calls)
    s1 = args.surrogate_steps * 2 // 3
    s2 = args.surrogate_steps // 4
    schedule = [(s1, 1e-3), (s2, 3e-4), (args.surrogate_steps - s1 - s2, 1e-4)]
    t0 = time.perf_counter()
    losses = []
    for steps, lr in schedule:
        if steps > 0:
            losses.extend(net.train(x, y, steps=steps, batch=8192, lr=lr, seed=3).tolist())
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_pairs = int(y.numel())
    del x, y
    torch.cuda.empty_cache()
    train_flop = 3 * flop_per_entry * 8192 * args.surrogate_steps

    # ---- timed runs: plain and surrogate, each followed by the digitizer
    hits = ctx.alloc_hits(int(1.4 * n))
    singles = ctx.alloc_singles(int(1.3 * n))
    coinc = (ctx._empty(n // 2, torch.int32), ctx._empty(n // 2, torch.int32))

    def run(mode, seed):
        if mode == "plain":
            rc, st = ctx.transport_into(hits, n, seed=seed)
            sst = None
        else:
            rc, st, sst = ctx.surrogate_transport_into(net, hits, n, seed=seed, spec=spec)
        if rc != 0:
            raise RuntimeError(f"{mode}: hit capacity")
        rc, nc = ctx.digitize_into(hits, singles, coinc, seed=seed)
        if rc != 0:
            raise RuntimeError(f"{mode}: digitizer capacity")
        return nc, st, sst

    def in_window_per_crystal():
        s = singles.numpy()
        return np.bincount(s["gid"][s["in_window"] != 0], minlength=ctx.info.n_crystals)

    out = {}
    hist = {}
    for mode in ("plain", "surrogate"):
        run(mode, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nc, st, sst = run(mode, 0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        hist[mode] = in_window_per_crystal()
        out[mode] = {"value": n / dt, "ms": dt * 1e3, "coincidences": nc, "sensitivity": nc / n,
                     "transport_kernel_ms": ctx.timings()[0]}
        if mode == "plain":
            w3 = algorithmic_work(st, ring=True, source="rods")
            k3 = ctx.timings()[0] * 1e-3
            out[mode]["roofline"] = {"bound": "alu", "kernel": "k_transport (hot-rod phantom)",
                                     "achieved": w3 / k3 / 1e12, "peak": VALU_PEAK / 1e12, "unit": "TVALU-op/s",
                                     "frac": w3 / k3 / VALU_PEAK, "work_per_launch": w3,
                                     "note": "phantom Woodcock steps priced at c_step"}
        if sst is not None:
            out[mode].update({"entries": sst["entries"], "photons_on_network": sst["entries"] / (2.0 * n),
                              "none_fraction": sst["none"] / max(1, sst["entries"]),
                              "transport_ms": sst["ms_transport"], "network_ms": sst["ms_network"]})
            achieved = sst["entries"] * flop_per_entry / (sst["ms_network"] * 1e-3)
            out[mode]["network_roofline"] = {"bound": "mfma", "achieved": achieved / 1e12, "peak": 2500.0,
                                             "unit": "TFLOP/s", "frac": achieved / 2.5e15,
                                             "flop_per_entry": flop_per_entry}
            # the same time against HBM: FP32 logits written by the last
            # product and read by the draw (energy head, position head and
            # its offset row), the BF16 activations of the last hidden layer
            # written and read (the hidden layers before it stay on chip)
            c_pad = (n1 + n2 + 127) // 128 * 128
            bytes_per_entry = 4 * c_pad + 4 * (n1 + 2 * n2) + 2 * 2 * 256
            bw = sst["entries"] * bytes_per_entry / (sst["ms_network"] * 1e-3)
            out[mode]["network_hbm"] = {"bound": "hbm", "achieved": bw / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                        "frac": bw / HBM_PEAK, "bytes_per_entry": bytes_per_entry}
    # independent full-transport run (seed 1) for the statistical comparison
    nc_ind, _, _ = run("plain", 1)
    hist["independent"] = in_window_per_crystal()
    a, b = hist["independent"], hist["surrogate"]
    keep = (a + b) >= 10
    ka = np.r_[a[keep], a[~keep].sum()].astype(float)
    kb = np.r_[b[keep], b[~keep].sum()].astype(float)
    na, nb = ka.sum(), kb.sum()
    chi2 = float((((np.sqrt(nb / na) * ka - np.sqrt(na / nb) * kb) ** 2) / np.maximum(ka + kb, 1)).sum())
    dof = len(ka) - 1
    c_s = out["surrogate"]["coincidences"]
    pp = (c_s + nc_ind) / (2 * n)
    z = (c_s / n - nc_ind / n) / np.sqrt(pp * (1 - pp) * 2 / n)
    net.close()
    ctx.close()
    return {"workload": f"hot-rod phantom: design C, water cylinder 25 x 70 mm (0.5 mm voxels), six-sector rods, "
                        f"{n:.0e} events, transport + digitizer",
            "plain": out["plain"], "surrogate": out["surrogate"],
            "speedup_vs_plain": out["surrogate"]["value"] / out["plain"]["value"],
            "sensitivity_rel_diff": out["surrogate"]["sensitivity"] / out["plain"]["sensitivity"] - 1.0,
            "matched_seeds": {"sensitivity_rel_diff": out["surrogate"]["sensitivity"] / out["plain"]["sensitivity"]
                              - 1.0, "bar": 0.005},
            "independent_seeds": {"plain_seed1_coincidences": nc_ind,
                                  "sensitivity_rel_diff": c_s / nc_ind - 1.0, "z": float(z),
                                  "p_z": float(2 * sps.norm.sf(abs(z))),
                                  "singles_chi2": {"chi2": chi2, "dof": dof, "p": float(sps.chi2.sf(chi2, dof))}},
            "spec": dict(spec, energy_classes=n1, positions=n2),
            "training": {"pairs_recorded": n_rec, "truncated_fraction": n_trunc / max(1, n_rec),
                         "pairs_trained": n_pairs, "events": args.surrogate_train_events, "pair_gen_s": t_pairs,
                         "label_none_fraction": label_none, "steps": args.surrogate_steps, "batch": 8192,
                         "schedule": schedule,
                         "train_s": t_train, "train_tflop_s": train_flop / t_train / 1e12,
                         "loss_first": float(losses[0]), "loss_last200": float(np.mean(losses[-200:]))}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--events", type=int, default=10_000_000, help="events per design and position")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--search-batch", type=int, default=16)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this size (counter calibration)")
    ap.add_argument("--batched-scale", type=float, default=1.0,
                    help="event-count scale of the batched design sweep (0 skips it)")
    ap.add_argument("--autotune-cache", default=None, help="JSON cache of the batch autotuner")
    ap.add_argument("--no-extensions", dest="extensions", action="store_false",
                    help="skip the optional-physics form (acollinearity, positron range, resolutions, dead time)")
    ap.add_argument("--no-config1", dest="config1", action="store_false",
                    help="skip the small-ring rates at 1e5 and 1e8 events")
    ap.add_argument("--no-paper-scanners", dest="paper_scanners", action="store_false",
                    help="skip the H2RSPET / Derenzo workload")
    ap.add_argument("--surrogate-events", type=int, default=100_000_000,
                    help="events of the hot-rod phantom workload timed plain and with the surrogate (0 skips)")
    ap.add_argument("--surrogate-train-events", type=int, default=1_640_000_000,
                    help="events whose detector entries make the training pairs (1.64e9: about 1e8 pairs)")
    ap.add_argument("--surrogate-steps", type=int, default=12000, help="Adam steps of batch 8192 (about one epoch)")
    ap.add_argument("--surrogate-half-width", type=int, default=6,
                    help="half width (crystals) of the neighbourhood an entry's domain requires inside each layer")
    ap.add_argument("--surrogate-class-half-width", type=int, default=12,
                    help="half width of the neighbourhood the position classes cover")
    ap.add_argument("--surrogate-ebins", type=int, default=18, help="energy bins above 224 keV")
    ap.add_argument("--surrogate-ebin-kev", type=float, default=16.0, help="energy bin width")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the event-parallel sharding "
                                   "across GPUs (each GPU a disjoint event range, windowed singles "
                                   "exchanged by time bucket before the coincidence sort) is not built"}))
        sys.exit(2)

    import torch

    from paper_2603_07327_amd.gpet import Context

    n = args.events
    designs = ("A", "B", "C")
    ctxs = []
    for d in designs:
        c = Context(0)
        c.set_scene(G.small_animal_scene(d, (0.0, 0.0, 0.0), n_events=n))
        c.enable_timing(True)
        c.set_launch(args.blocks_per_cu, args.search_batch, args.schedule)
        hits = c.alloc_hits(int(3.2 * n))
        singles = c.alloc_singles(int(2.2 * n))
        coinc = (c._empty(n, torch.int32), c._empty(n, torch.int32))
        ctxs.append((d, c, hits, singles, coinc))

    kernel_ms, work, stats_last = [], [], None
    digi_ms, digi_bytes, digi_survey = [], [], []

    def step(i, record):
        nonlocal stats_last
        pos = G.SWEEP_POSITIONS[i % len(G.SWEEP_POSITIONS)]
        out = []
        for d, c, hits, singles, coinc in ctxs:
            c.set_source(G.point_source(pos, n))
            rc, st = c.transport_into(hits, n, seed=1000 + i)
            if rc != 0:
                raise RuntimeError(f"hit capacity too small ({hits.count})")
            rc, nc = c.digitize_into(hits, singles, coinc, seed=1000 + i)
            if rc != 0:
                raise RuntimeError("digitizer capacity too small")
            if record:
                tm = c.timings()
                kernel_ms.append(tm[0])
                work.append(algorithmic_work(st, ring=True, source="point"))
                stats_last = st
                digi_ms.append(tm[1])
                digi_bytes.append(digitizer_bytes(hits.count, singles.count, singles.windowed, nc))
                digi_survey.append(digitizer_survey_bytes(hits.count, singles.windowed))
            out.append((d, hits.count, singles.count, nc))
        return out

    if args.calib_copy_mib:
        a = torch.empty(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    for i in range(args.warmup):
        step(i, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = step(args.warmup + i, True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    events = args.steps * len(designs) * n
    value = events / dt
    avg_ms = float(np.mean(kernel_ms))
    achieved = float(np.mean(work)) / (avg_ms * 1e-3)
    line = {
        "metric": "annihilation events/s on 1 MI355X (plain vs batched vs surrogate) at matched tallies",
        "value": value, "unit": "events/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "small-animal sensitivity sweep, designs A/B/C, plain transport + digitizer",
                   "events_per_design": n, "designs": list(designs), "panels": 12,
                   "crystals": ctxs[2][1].info.n_crystals, "positions_per_step": 1, "form": "plain"},
        "roofline": {"bound": "alu", "kernel": "k_transport", "achieved": achieved / 1e12,
                     "peak": VALU_PEAK / 1e12, "unit": "TVALU-op/s", "frac": achieved / VALU_PEAK,
                     "traffic": measured_traffic(n), "kernel_ms": avg_ms,
                     "work_per_launch": float(np.mean(work)), "transport_source": transport_source_hash()},
        "last_step": res, "stats_last": stats_last,
        "digitizer_roofline": {"bound": "hbm", "achieved": float(np.mean(digi_bytes)) / (float(np.mean(digi_ms)) * 1e-3)
                               / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                               "frac": float(np.mean(digi_bytes)) / (float(np.mean(digi_ms)) * 1e-3) / HBM_PEAK,
                               "bytes_per_design": float(np.mean(digi_bytes)), "ms_per_design": float(np.mean(digi_ms)),
                               "bytes_per_item": DIGI_BYTES,
                               "survey_form": {"bytes_per_design": float(np.mean(digi_survey)),
                                               "frac": float(np.mean(digi_survey)) / (float(np.mean(digi_ms)) * 1e-3)
                                               / HBM_PEAK,
                                               "note": "24 B per item and pass, 7 passes over the hits, 8 over the "
                                                       "windowed singles"}},
    }
    line["window_sweep"] = window_sweep(ctxs, n, 1000 + args.warmup + args.steps - 1,
                                        G.SWEEP_POSITIONS[(args.warmup + args.steps - 1) % len(G.SWEEP_POSITIONS)])
    # design C with the source at the centre: one more timed launch whose work
    # is also priced in the survey's form with the oracle's counts (below)
    _, cC, hitsC, _, _ = ctxs[2]
    cC.set_source(G.point_source((0.0, 0.0, 0.0), n))
    cC.transport_into(hitsC, n, seed=1)
    rcC, stC = cC.transport_into(hitsC, n, seed=1)
    survey_probe = {"kernel_ms": cC.timings()[0], "stats": stC}
    for _, c, *_ in ctxs:
        c.close()
    del ctxs
    if args.extensions:
        line["extensions"] = extensions_form(n)
    if args.config1:
        line["config1"] = config1_form()
    if args.paper_scanners:
        line["paper_scanners"] = paper_scanners_form()
    if args.batched_scale > 0:
        line["batched"] = batched_form(args)
    if args.surrogate_events > 0:
        line["surrogate"] = surrogate_form(args)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
        oracle_counts = line["cpu_baseline"]["counts_per_event"]
    else:  # a small oracle sample of the same launch
        from oracle import oracle as O
        O.build(force=False)
        so = O.OracleScene(G.small_animal_scene("C", (0.0, 0.0, 0.0), n_events=200_000_000))
        _, oc = so.transport(200_000, seed=1)
        oracle_counts = {k: v / 200_000 for k, v in oc.items()}
    line["roofline_survey_form"] = survey_form_roofline(survey_probe, oracle_counts, n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
