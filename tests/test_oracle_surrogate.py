"""Pins of the FP64 surrogate reference (CPU): gradients against central finite
differences, softmax cross-entropy and Adam closed forms, inverse-CDF sampling
on hand-computed cumulative sums, bfloat16 rounding against torch's
conversion, and the entry domain, anchor, class and synthetic-hit layout on a
hand-worked design-C entry; deposits per photon from traced vertices against
the oracle's own hit list."""
import math

import numpy as np
import pytest

import gpet_inputs as G
from oracle import surrogate as S


def _params(sizes, seed=0, scale=0.5):
    rng = np.random.default_rng(seed)
    return [(rng.normal(0, scale, (j, i)), rng.normal(0, 0.1, j)) for i, j in zip(sizes[:-1], sizes[1:])]


def test_gradient_matches_central_differences():
    sizes = [6, 7, 5, 9]
    P = _params(sizes, 1)
    rng = np.random.default_rng(2)
    x = rng.normal(size=(11, 6))
    y = rng.integers(0, 9, 11)
    _, g = S.loss_and_grad(P, x, y)
    h = 1e-6
    worst = 0.0
    for k, (W, b) in enumerate(P):
        for arr, garr in ((W, g[k][0]), (b, g[k][1])):
            it = np.nditer(arr, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = arr[idx]
                arr[idx] = old + h
                lp, _ = S.loss_and_grad(P, x, y)
                arr[idx] = old - h
                lm, _ = S.loss_and_grad(P, x, y)
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                worst = max(worst, abs(fd - garr[idx]) / max(1e-3, abs(fd)))
    assert worst < 1e-6, worst


def test_storage_rounding_is_the_only_difference():
    """Rounding stored values with the identity reproduces the float64
    gradient exactly; BF16 storage changes it by a bounded amount that shrinks
    toward the output layer (fewer rounded stages behind it)."""
    sizes = [6, 32, 32, 32, 20]
    P = _params(sizes, 5, scale=0.4)
    rng = np.random.default_rng(6)
    x = S.bf16_round(rng.uniform(-1, 1, (300, 6)))
    y = rng.integers(0, 20, 300)
    l0, g0 = S.loss_and_grad(P, x, y)
    l1, g1 = S.loss_and_grad(P, x, y, store=lambda a: a)
    assert l0 == l1 and all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) for a, b in zip(g0, g1))
    l2, g2 = S.loss_and_grad(P, x, y, store=S.bf16_round)
    err = [np.linalg.norm(a[0] - b[0]) / np.linalg.norm(b[0]) for a, b in zip(g2, g0)]
    assert abs(l2 - l0) < 1e-2 * l0
    assert max(err) < 0.1 and err[-1] < err[0]


def test_cross_entropy_closed_forms():
    sizes = [6, 4, 5]
    P = [(np.zeros((j, i)), np.zeros(j)) for i, j in zip(sizes[:-1], sizes[1:])]
    x = np.random.default_rng(0).normal(size=(8, 6))
    y = np.array([0, 1, 2, 3, 4, 0, 0, 1])
    loss, g = S.loss_and_grad(P, x, y)
    assert abs(loss - math.log(5)) < 1e-15
    # last bias: mean over the batch of softmax - one-hot
    want = np.full(5, 0.2) - np.bincount(y, minlength=5) / 8.0
    np.testing.assert_allclose(g[-1][1], want, atol=1e-15)
    # zero hidden weights: hidden ReLU outputs are 0, so every weight gradient vanishes
    assert np.all(g[-1][0] == 0) and np.all(g[0][0] == 0)
    # a logit far above the rest: loss -> 0 for that class
    P[-1] = (np.zeros((5, 4)), np.array([50.0, 0, 0, 0, 0]))
    loss, _ = S.loss_and_grad(P, x[:1], np.array([0]))
    assert loss < 1e-20


def _factored_case(seed=11, groups=1):
    sizes = [6, 7, 5, 4 + 9 * groups]  # energy head of 4 classes (none + 3), blocks of 9 positions
    P = _params(sizes, seed)
    rng = np.random.default_rng(seed + 1)
    T = rng.normal(0, 0.7, (3, 9))
    x = rng.normal(size=(13, 6))
    y = S.factored_join(rng.integers(0, 4, 13), rng.integers(0, 9, 13), 4)
    y[:2] = 0
    return sizes, P, T, x, y


@pytest.mark.parametrize("groups", [1, 3])
def test_factored_gradient_matches_central_differences(groups):
    """The energy-then-position output (Sec. 4's learned stand-in, this
    build's factored head; with 3 groups each energy class has a position
    block of its own): gradients of every weight, bias and table entry
    against central differences of the loss."""
    sizes, P, T, x, y = _factored_case(groups=groups)
    _, g, gT = S.factored_loss_and_grad(P, T, x, y, 4, n_groups=groups)
    h = 1e-6
    worst = 0.0
    arrays = [(W, g[k][0]) for k, (W, _) in enumerate(P)] + [(b, g[k][1]) for k, (_, b) in enumerate(P)] + [(T, gT)]
    for arr, garr in arrays:
        it = np.nditer(arr, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            old = arr[idx]
            arr[idx] = old + h
            lp, _, _ = S.factored_loss_and_grad(P, T, x, y, 4, n_groups=groups)
            arr[idx] = old - h
            lm, _, _ = S.factored_loss_and_grad(P, T, x, y, 4, n_groups=groups)
            arr[idx] = old
            fd = (lp - lm) / (2 * h)
            worst = max(worst, abs(fd - garr[idx]) / max(1e-3, abs(fd)))
    assert worst < 1e-6, worst


def test_factored_closed_forms_and_normalization():
    """Zero weights: loss = log n_first + (share of labels with a single) log
    n_positions, the energy-head bias gradient is 1/n_first minus the label
    frequencies, the table gradient of energy e is the mean over its rows of
    1/n_positions minus the one-hot position.  For any weights the joint
    probabilities over all 1 + n_positions (n_first - 1) labels sum to 1."""
    sizes = [6, 5, 4 + 9]
    P = [(np.zeros((j, i)), np.zeros(j)) for i, j in zip(sizes[:-1], sizes[1:])]
    T = np.zeros((3, 9))
    x = np.random.default_rng(0).normal(size=(8, 6))
    e = np.array([0, 1, 2, 3, 0, 1, 1, 3])
    k = np.array([0, 4, 8, 0, 0, 4, 5, 2])
    y = S.factored_join(e, k, 4)
    assert np.array_equal(np.stack(S.factored_split(y, 4)), np.stack([e, np.where(e > 0, k, 0)]))
    loss, g, gT = S.factored_loss_and_grad(P, T, x, y, 4)
    assert abs(loss - (math.log(4) + 6 / 8 * math.log(9))) < 1e-14
    np.testing.assert_allclose(g[-1][1][:4], 0.25 - np.bincount(e, minlength=4) / 8.0, atol=1e-15)
    for ei in (1, 2, 3):
        rows = e == ei
        want = (rows.sum() / 9.0 - np.bincount(k[rows], minlength=9)) / 8.0
        np.testing.assert_allclose(gT[ei - 1], want, atol=1e-15)
    # joint label layout of outcome_class: 1 + position (n_ebins + 1) + bin, e = bin + 1
    assert S.factored_join(np.array([3]), np.array([5]), 4)[0] == 1 + 5 * 3 + 2
    for groups in (1, 3):
        sizes, P, T, x, _ = _factored_case(3, groups)
        z, _, _ = S.forward(P, x)
        labels = np.arange(1 + 9 * 3)
        tot = sum(np.exp(S.factored_log_prob(z, T, np.full(len(x), lab), 4, groups)) for lab in labels)
        np.testing.assert_allclose(tot, 1.0, rtol=1e-13)
    # with one block per energy class, the position law of class e reads block e - 1 only
    z = np.zeros((1, 4 + 27))
    z[0, 4 + 9 + 5] = 30.0  # block 1 (energy class 2) peaks at position 5
    T0 = np.zeros((3, 9))
    assert S.factored_sample(z, T0, 4, np.array([0.6]), np.array([0.5]), n_groups=3)[0] == 1 + 5 * 3 + 1
    assert S.factored_sample(z, T0, 4, np.array([0.3]), np.array([0.5]), n_groups=3)[0] == 1 + 4 * 3 + 0


@pytest.mark.parametrize("groups", [1, 3])
def test_factored_sampling_follows_its_probabilities(groups):
    """Stratified uniforms (u = (i + 1/2) / N on each axis, all pairs) give
    every joint label with its probability to within 2 / N."""
    sizes, P, T, x, _ = _factored_case(5, groups)
    z, _, _ = S.forward(P, x[:1])
    N = 400
    u = (np.arange(N) + 0.5) / N
    ue, up = np.meshgrid(u, u, indexing="ij")
    zz = np.repeat(z, N * N, axis=0)
    lab = S.factored_sample(zz, T, 4, ue.ravel(), up.ravel(), groups)
    freq = np.bincount(lab, minlength=28) / (N * N)
    prob = np.exp([S.factored_log_prob(z, T, np.array([c]), 4, groups)[0] for c in range(28)])
    assert np.max(np.abs(freq - prob)) < 2.0 / N
    # hand-computed: energy probabilities from the first head alone
    z1 = np.log(np.array([[0.5, 0.25, 0.125, 0.125]]))
    zfull = np.concatenate([z1, np.zeros((1, 9))], axis=1)
    assert S.factored_sample(zfull, np.zeros((3, 9)), 4, np.array([0.49]), np.array([0.5]))[0] == 0
    # e = 2 (u in (0.75, 0.875]), uniform positions: u_position = 0.35 -> position 3
    assert S.factored_sample(zfull, np.zeros((3, 9)), 4, np.array([0.8]), np.array([0.35]))[0] == 1 + 3 * 3 + 1


def test_wide_class_neighbourhood_hand_worked():
    """A class neighbourhood of half width 8 around anchors near the arrays'
    edges of design C (23 x 23 over 24 x 24): the positions that exist
    (inside each layer's array) counted by hand, the label layout with
    W = 17, and the sampler never drawing a position that does not exist."""
    spec = S.Spec(half_width=2, n_ebins=36, class_half_width=8)
    lat = _lat_c()
    ent = S.Entry(True, np.zeros(6), 0, [(6, 16), (6, 17)])
    ex = S.positions_exist(spec, lat, ent)
    W = 17
    assert len(ex) == 2 * W * W
    # layer 0: t offsets 2..16 (it = 0..14), a offsets 0..14 (ia = 8..22); layer 1 likewise up to 23
    assert ex[:W * W].sum() == 15 * 15 and ex[W * W:].sum() == 15 * 15
    assert not ex[(0 * W + 1) * W + 0] and ex[(0 * W + 2) * W + 0] and not ex[(0 * W + 2) * W + 15]
    # label of layer 1, crystal (it, ia) = (3, 20), bin 5: offsets (3 - 6 + 8, 20 - 17 + 8) = (5, 11)
    gid = lat.gid(0, 0, 1, 3, 20)
    c, trunc = S.outcome_class(spec, lat, ent, 0, 511.0, {gid: 224.0 + 8 * 5 + 1})
    assert not trunc and c == 1 + ((1 * W + 5) * W + 11) * 37 + 5
    assert S.class_hit(spec, lat, ent, 0, 511.0, c, 0.5)[0] == gid
    # a peaked position head on a position that does not exist: the sampler takes the best that does
    z = np.zeros((1, 38 + 2 * W * W))
    z[0, 37] = 50.0  # photopeak
    z[0, 38 + 0] = 40.0  # position 0 (layer 0, offsets (0, 0)): outside the array
    z[0, 38 + (0 * W + 2) * W + 3] = 30.0
    lab = S.factored_sample(z, np.zeros((37, 2 * W * W)), 38, np.array([0.5]), np.array([0.5]), exists=ex[None, :])
    assert lab[0] == 1 + ((0 * W + 2) * W + 3) * 37 + 36


def test_adam_first_step_is_signed_learning_rate():
    P = _params([3, 4], 3)
    g = [(np.array([[1e-3, -2.0, 0.5]] * 4), np.array([3.0, -1e-5, 0.25, -7.0]))]
    z = [(np.zeros((4, 3)), np.zeros(4))]
    lr, eps = 1e-2, 1e-8
    P1, m, v = S.adam_step(P, g, z, z, 1, lr, eps=eps)
    for (W0, b0), (W1, b1), (gW, gb) in zip(P, P1, g):
        np.testing.assert_allclose(W1 - W0, -lr * gW / (np.abs(gW) + eps), rtol=1e-12)
        np.testing.assert_allclose(b1 - b0, -lr * gb / (np.abs(gb) + eps), rtol=1e-12)
    np.testing.assert_allclose(m[0][1], 0.1 * g[0][1])
    np.testing.assert_allclose(v[0][1], 0.001 * g[0][1] ** 2)


def test_inverse_cdf_sampling():
    z = np.log(np.array([0.2, 0.3, 0.5]))
    cases = [(0.0, 0), (0.2 - 1e-12, 0), (0.2 + 1e-12, 1), (0.5 - 1e-12, 1), (0.5 + 1e-12, 2), (1.0, 2)]
    for u, c in cases:
        assert S.sample_class(z, np.array([u]))[0] == c, u


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.normal(0, 1, 100_000), rng.normal(0, 1e4, 1000),
                        [1.0, 1 + 2**-8, 1 + 3 * 2**-8, -1 - 2**-8, 0.0, 65504.0]]).astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16_round(a), ref)
    assert S.bf16_round(np.float32(1 + 2**-8)) == 1.0
    assert S.bf16_round(np.float32(1 + 3 * 2**-8)) == 1 + 2**-6


def _lat_c():
    return S.Lattice(G.small_animal_scanner("C"))


def test_entry_anchor_and_features_hand_worked():
    """Design C: modules 1 x 4 of 24 x 24 mm with 2 mm axial gaps; layer 0 is
    23 x 23 offset by half a pitch, layer 1 is 24 x 24.  A normal entry at
    module-local (10.3, 7.6) of module m_a = 1 anchors both layers at (10, 7)."""
    spec, lat = S.Spec(), _lat_c()
    t = -12.0 + 10.3
    a = -51.0 + 26.0 + 7.6
    ent = S.entry_state(spec, lat, np.array([0.0, t, a]), np.array([1.0, 0.0, 0.0]), 511.0)
    assert ent.in_domain and ent.module == 1
    assert ent.anchor == [(10, 7), (10, 7)]
    np.testing.assert_allclose(ent.x, [2 * 0.3 - 1, 2 * 0.6 - 1, 0, 0, 1, 1], atol=1e-12)
    # the mid-depth point decides: a slanted ray moves the anchor
    s = 0.2
    d = np.array([1.0, s, 0.0]) / math.sqrt(1 + s * s)
    ent2 = S.entry_state(spec, lat, np.array([0.0, t, a]), d, 511.0)
    # mid-depth (10 mm) shifts t by 2 mm: u_t = 12.3 -> anchor 12
    assert ent2.in_domain and ent2.anchor == [(12, 7), (12, 7)]
    np.testing.assert_allclose(ent2.x[2], s / spec.max_slope)


@pytest.mark.parametrize("case", ["slope", "depth", "energy", "edge_layer0", "edge_low", "gap", "backward"])
def test_entry_domain_limits(case):
    spec, lat = S.Spec(), _lat_c()
    t, a, d, e, x0 = -12.0 + 10.3, -51.0 + 26.0 + 7.6, np.array([1.0, 0.0, 0.0]), 400.0, 0.0
    if case == "slope":
        d = np.array([1.0, 0.0, 0.26]) / math.sqrt(1 + 0.26**2)
    elif case == "depth":
        x0 = 0.01
    elif case == "energy":
        e = 223.9
    elif case == "edge_layer0":
        t = -12.0 + 21.4   # layer 1 anchor 21 is allowed (24 wide), layer 0 anchor 21 is not (23 wide)
    elif case == "edge_low":
        a = -51.0 + 26.0 + 1.5
    elif case == "gap":
        a = -51.0 + 24.5   # the mid-depth point falls into the axial module gap
    elif case == "backward":
        d = np.array([-1.0, 0.0, 0.0])
    assert not S.entry_state(spec, lat, np.array([x0, t, a]), d, e).in_domain
    if case == "edge_layer0":
        assert S.entry_state(spec, lat, np.array([0.0, -12.0 + 20.4, a]), d, e).in_domain


def test_classes_and_synthetic_hits_hand_worked():
    spec, lat = S.Spec(), _lat_c()
    assert spec.n_classes(2) == 1851
    ent = S.entry_state(spec, lat, np.array([0.0, -1.7, -17.4]), np.array([1.0, 0.0, 0.0]), 511.0)
    # layer 1 crystal (11, 6) of panel 0, module 1: gid 1105 + 529 + 6 * 24 + 11
    g = 1105 + 529 + 6 * 24 + 11
    assert lat.decode(g) == (0, 1, 1, 11, 6)
    c, tr = S.outcome_class(spec, lat, ent, 0, 511.0, {g: 511.0})
    assert (c, tr) == (1 + ((1 * 5 + 3) * 5 + 1) * 37 + 36, False) == (1554, False)
    assert S.class_hit(spec, lat, ent, 0, 511.0, 1554, 0.3) == (g, 511.0, 15.0)
    # two deposits in one crystal sum to 350 keV: bin floor((350 - 224) / 8) = 15
    g0 = 1105 + 0 + 9 * 23 + 8   # layer 0 crystal (8, 9): offsets (-2, +2)
    c, tr = S.outcome_class(spec, lat, ent, 0, 511.0, {g0: 350.0, g: 100.0})
    assert c == 1 + ((0 * 5 + 0) * 5 + 4) * 37 + 15 and not tr
    gid, edep, depth = S.class_hit(spec, lat, ent, 0, 511.0, c, 0.5)
    assert gid == g0 and edep == 224.0 + 8.0 * 15.5 and depth == 5.0
    # the largest deposit outside the neighbourhood: class 0, truncated
    g_far = 1105 + 529 + 7 * 24 + 13
    assert S.outcome_class(spec, lat, ent, 0, 511.0, {g_far: 400.0, g: 300.0}) == (0, True)
    # another panel or module: truncated as well
    assert S.outcome_class(spec, lat, ent, 0, 511.0, {g + 4420: 400.0}) == (0, True)
    assert S.outcome_class(spec, lat, ent, 0, 511.0, {g + 1105: 400.0}) == (0, True)
    # below e_min, or nothing deposited
    assert S.outcome_class(spec, lat, ent, 0, 511.0, {g: 223.9}) == (0, False)
    assert S.outcome_class(spec, lat, ent, 0, 511.0, {}) == (0, False)
    # ties of equal sums go to the lower gid; the photopeak tolerance
    c, _ = S.outcome_class(spec, lat, ent, 0, 400.0, {g: 399.5, g0: 399.5})
    assert S.class_hit(spec, lat, ent, 0, 400.0, c, 0.0)[:2] == (g0, 400.0)
    c, _ = S.outcome_class(spec, lat, ent, 0, 400.0, {g: 398.9})
    assert (c - 1) % 37 == math.floor((398.9 - 224) / 8)


def test_trace_deposits_match_oracle_hits(oracle_mod):
    """Per photon that visits one panel once: deposits gathered from the traced
    vertices equal the oracle's hit list for that photon, and in-domain
    entries carry a label."""
    sc = G.small_animal_scene("C", n_events=3000)
    o = oracle_mod.OracleScene(sc)
    v = o.trace(3000, seed=4)
    hits, _ = o.transport(3000, seed=4)
    recs = S.photon_entries(S.Spec(), sc, o.poses(), v)
    key = v["event"].astype(np.int64) * 2 + v["photon"]
    n_enter = np.bincount(key[v["kind"] == S.K_ENTER_PANEL], minlength=6000)
    hk = hits["event"].astype(np.int64) * 2 + hits["photon"]
    checked = in_dom = 0
    for r in recs:
        k = r["event"] * 2 + r["photon"]
        if not r["entered"] or n_enter[k] != 1:
            continue
        sel = hk == k
        dep = {}
        for g, e in zip(hits["gid"][sel], hits["edep"][sel]):
            dep[int(g)] = dep.get(int(g), 0.0) + float(e)
        assert dep.keys() == r["dep"].keys()
        for g in dep:
            assert abs(dep[g] - r["dep"][g]) < 1e-9
        checked += 1
        if r["entry"].in_domain:
            in_dom += 1
            assert 0 <= r["label"] < 1851
    assert checked > 1000 and in_dom > 100
