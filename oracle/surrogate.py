"""FP64 reference of the learned detector-response surrogate.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the product path never imports it.

The surrogate replaces the in-panel transport of a photon that enters a panel
through its front face with one categorical draw from a small MLP (the paper's
Discussion points to learned stand-ins for detailed photon tracking as a route
to speed; the network and its outcome classes are this implementation's
design):

* entry state -> domain and features (decided from the entry state only);
* outcome class of a fully simulated photon: which crystal of the layer-wise
  neighbourhood around the entry receives the largest deposit, and that
  deposit's energy bin (or "no deposit that can reach the energy window");
* MLP forward pass, mean softmax cross-entropy, its analytic gradient and the
  Adam update, all in float64;
* inverse-CDF categorical sampling and the synthetic hit a class stands for.

Every function works on plain numpy arrays; the transport histories come from
the oracle's traced vertices.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

C_MM_PER_PS = 0.299792458
K_STEP, K_ENTER_PANEL, K_EXIT, K_ESCAPE, K_DEAD, K_ENTER_PHANTOM, K_EMIT = range(7)


@dataclass
class Spec:
    """Neighbourhood, energy classes and domain of the surrogate."""
    half_width: int = 2           # neighbourhood of (2 h + 1)^2 crystals per layer
    n_ebins: int = 36             # energy bins of ebin_kev above e_min_kev
    e_min_kev: float = 224.0      # smaller largest deposits: class 0
    ebin_kev: float = 8.0
    photopeak_tol_kev: float = 1.0  # largest deposit within this of the entry energy: photopeak
    max_slope: float = 0.25       # |d_t / d_depth| and |d_a / d_depth| inside the domain
    front_tol_mm: float = 1e-3    # entry depth coordinate of a front-face entry
    class_half_width: int = 0     # half width of the class neighbourhood (0: half_width)

    @property
    def chalf(self):
        """Half width of the neighbourhood the outcome classes cover (at least
        the domain's; wider, it may reach past a layer's array)."""
        return self.class_half_width or self.half_width

    @property
    def width(self):
        return 2 * self.chalf + 1

    def n_classes(self, n_layers: int) -> int:
        return 1 + n_layers * self.width ** 2 * (self.n_ebins + 1)


# ---------------------------------------------------------------------------
# geometry of the scanner description (panel-local frame: depth, t, a)
# ---------------------------------------------------------------------------
class Lattice:
    """Module grid and per-layer crystal lattices of a scanner description."""

    def __init__(self, g: dict):
        self.g = g
        self.w_mod = g["mod_n_t"] * g["mod_t"] + (g["mod_n_t"] - 1) * g["gap_t"]
        self.l_mod = g["mod_n_a"] * g["mod_a"] + (g["mod_n_a"] - 1) * g["gap_a"]
        self.t0, self.a0 = -0.5 * self.w_mod, -0.5 * self.l_mod
        self.step_t, self.step_a = g["mod_t"] + g["gap_t"], g["mod_a"] + g["gap_a"]
        self.layers = g["layers"]
        per_module = sum(y["n_t"] * y["n_a"] for y in self.layers)
        self.cpm = per_module
        self.cpp = per_module * g["mod_n_t"] * g["mod_n_a"]
        base, acc = [], 0
        for y in self.layers:
            base.append(acc)
            acc += y["n_t"] * y["n_a"]
        self.layer_base = base

    def module_of(self, t, a):
        """(m_t, m_a, u_t, u_a) module indices and module-local coordinates, or None."""
        mt = math.floor((t - self.t0) / self.step_t)
        ma = math.floor((a - self.a0) / self.step_a)
        if not (0 <= mt < self.g["mod_n_t"] and 0 <= ma < self.g["mod_n_a"]):
            return None
        ut = t - self.t0 - mt * self.step_t
        ua = a - self.a0 - ma * self.step_a
        if not (0.0 <= ut < self.g["mod_t"] and 0.0 <= ua < self.g["mod_a"]):
            return None
        return mt, ma, ut, ua

    def decode(self, gid: int):
        """gid -> (panel, module, layer, i_t, i_a)."""
        p, r = divmod(gid, self.cpp)
        m, r = divmod(r, self.cpm)
        for l in range(len(self.layers) - 1, -1, -1):
            if r >= self.layer_base[l]:
                ia, it = divmod(r - self.layer_base[l], self.layers[l]["n_t"])
                return p, m, l, it, ia
        raise ValueError(gid)

    def gid(self, panel, module, layer, it, ia):
        return panel * self.cpp + module * self.cpm + self.layer_base[layer] + ia * self.layers[layer]["n_t"] + it


@dataclass
class Entry:
    in_domain: bool
    x: np.ndarray | None = None   # 6 features
    module: int = -1
    anchor: list | None = None    # per layer (i_t, i_a) of the neighbourhood centre


def entry_state(spec: Spec, lat: Lattice, xl, dl, e) -> Entry:
    """Domain and features of a photon entering a panel at local position xl
    with local direction dl and energy e.

    Domain: e >= e_min; entry through the front face (depth ~ 0); lateral
    slopes within max_slope; the straight line's point at mid-depth lies in a
    module, and for every layer the neighbourhood around the anchor crystal
    lies inside that layer's crystal array.  The anchor: the crystal of the
    last layer whose pitch cell holds the mid-depth point; for another layer,
    its crystal whose cell holds the centre of that cell (a centre on a cell
    boundary goes to the upper cell).
    Features: the mid-depth point's position in the anchor cell (scaled to
    [-1, 1)), the two slopes over max_slope, the energy scaled to [-1, 1] over
    [e_min, 511], and the depth component of the direction."""
    g = lat.g
    if not (e >= spec.e_min_kev) or abs(xl[0]) > spec.front_tol_mm or not (dl[0] > 0.0):
        return Entry(False)
    st, sa = dl[1] / dl[0], dl[2] / dl[0]
    if abs(st) > spec.max_slope or abs(sa) > spec.max_slope:
        return Entry(False)
    s = (0.5 * g["depth"] - xl[0]) / dl[0]
    mod = lat.module_of(xl[1] + s * dl[1], xl[2] + s * dl[2])
    if mod is None:
        return Entry(False)
    mt, ma, ut, ua = mod
    ref = lat.layers[-1]
    qt = (ut - ref["off_t"]) / ref["pitch_t"]
    qa = (ua - ref["off_a"]) / ref["pitch_a"]
    it, ia = math.floor(qt), math.floor(qa)
    ft, fa = qt - it, qa - ia
    ct = ref["off_t"] + (it + 0.5) * ref["pitch_t"]
    ca = ref["off_a"] + (ia + 0.5) * ref["pitch_a"]
    h = spec.half_width
    anchor = []
    for y in lat.layers:
        # a cell centre on a crystal boundary of another layer (offset of half
        # a pitch) belongs to the upper crystal: nudge by 1e-3 pitch
        jt = math.floor((ct - y["off_t"]) / y["pitch_t"] + 1e-3)
        ja = math.floor((ca - y["off_a"]) / y["pitch_a"] + 1e-3)
        if not (h <= jt <= y["n_t"] - 1 - h and h <= ja <= y["n_a"] - 1 - h):
            return Entry(False)
        anchor.append((jt, ja))
    x = np.array([2.0 * ft - 1.0, 2.0 * fa - 1.0, st / spec.max_slope, sa / spec.max_slope,
                  2.0 * (e - spec.e_min_kev) / (511.0 - spec.e_min_kev) - 1.0, dl[0]])
    return Entry(True, x, ma * g["mod_n_t"] + mt, anchor)


def outcome_class(spec: Spec, lat: Lattice, ent: Entry, panel: int, e_in: float, dep: dict):
    """Class of a fully simulated photon from its per-crystal deposit sums in
    the panel it entered (dep: gid -> keV).  Returns (class, truncated): class 0
    when the largest deposit is below e_min or its crystal lies outside the
    neighbourhood (then truncated is True)."""
    if not dep:
        return 0, False
    best = min(dep, key=lambda k: (-dep[k], k))
    esum = dep[best]
    if esum < spec.e_min_kev:
        return 0, False
    p, m, l, it, ia = lat.decode(best)
    at, aa = ent.anchor[l]
    h, W = spec.chalf, spec.width
    if p != panel or m != ent.module or abs(it - at) > h or abs(ia - aa) > h:
        return 0, True
    if esum >= e_in - spec.photopeak_tol_kev:
        b = spec.n_ebins
    else:
        b = min(max(int(math.floor((esum - spec.e_min_kev) / spec.ebin_kev)), 0), spec.n_ebins - 1)
    return 1 + ((l * W + (it - at + h)) * W + (ia - aa + h)) * (spec.n_ebins + 1) + b, False


def class_hit(spec: Spec, lat: Lattice, ent: Entry, panel: int, e_in: float, c: int, u_energy: float):
    """The synthetic single a class stands for: (gid, deposit keV, depth mm),
    or None for class 0.  Deposit: the entry energy for the photopeak class,
    else uniform in the class's bin (u_energy)."""
    if c == 0:
        return None
    k, b = divmod(c - 1, spec.n_ebins + 1)
    W, h = spec.width, spec.chalf
    l, r = divmod(k, W * W)
    dt, da = divmod(r, W)
    at, aa = ent.anchor[l]
    y = lat.layers[l]
    gid = lat.gid(panel, ent.module, l, at + dt - h, aa + da - h)
    edep = e_in if b == spec.n_ebins else spec.e_min_kev + spec.ebin_kev * (b + u_energy)
    return gid, edep, y["depth0"] + 0.5 * y["thick"]


def positions_exist(spec: Spec, lat: Lattice, ent: Entry) -> np.ndarray:
    """Which positions of the class neighbourhood (layer, then offsets -H..H
    in t and a around the layer's anchor) lie inside their layer's crystal
    array: a largest deposit can only be there."""
    W, h = spec.width, spec.chalf
    out = np.zeros(len(lat.layers) * W * W, bool)
    for l, y in enumerate(lat.layers):
        at, aa = ent.anchor[l]
        for dt in range(W):
            for da in range(W):
                out[(l * W + dt) * W + da] = 0 <= at + dt - h < y["n_t"] and 0 <= aa + da - h < y["n_a"]
    return out


# ---------------------------------------------------------------------------
# pairs from traced histories
# ---------------------------------------------------------------------------
def photon_entries(spec: Spec, sc: dict, poses: np.ndarray, v: np.ndarray):
    """For every photon of a traced run: its first panel entry (if any), the
    entry's domain/features, the path length to the entry, and the outcome
    class of its stay in that panel.  Returns a list of dicts keyed by
    (event, photon)."""
    lat = Lattice(sc["scanner"])
    out = []
    key = v["event"].astype(np.int64) * 2 + v["photon"]
    order = np.argsort(key, kind="stable")
    v = v[order]
    key = key[order]
    starts = np.flatnonzero(np.r_[True, key[1:] != key[:-1]])
    ends = np.r_[starts[1:], len(v)]
    for s0, s1 in zip(starts, ends):
        w = v[s0:s1]
        kinds = w["kind"]
        ent_idx = np.flatnonzero(kinds == K_ENTER_PANEL)
        rec = {"event": int(w["event"][0]), "photon": int(w["photon"][0]), "entered": len(ent_idx) > 0}
        if not len(ent_idx):
            out.append(rec)
            continue
        j = int(ent_idx[0])
        p = int(w["panel"][j])
        P = poses[p]
        xg = np.array([w["x"][j], w["y"][j], w["z"][j]], np.float64)
        dg = np.array([w["dx"][j], w["dy"][j], w["dz"][j]], np.float64)
        r = xg - P[0:3]
        xl = np.array([r @ P[3:6], r @ P[6:9], r @ P[9:12]])
        dl = np.array([dg @ P[3:6], dg @ P[6:9], dg @ P[9:12]])
        e = float(w["e"][j])
        pts = np.stack([w["x"][: j + 1], w["y"][: j + 1], w["z"][: j + 1]], 1).astype(np.float64)
        L = float(np.sum(np.linalg.norm(np.diff(pts, axis=0), axis=1)))
        ent = entry_state(spec, lat, xl, dl, e)
        dep = {}
        for k in range(j + 1, len(w)):
            if kinds[k] in (K_EXIT, K_DEAD, K_ESCAPE):
                break
            if kinds[k] == K_STEP and w["accept"][k] == 1 and w["process"][k] in (1, 2) and w["gid"][k] >= 0:
                g = int(w["gid"][k])
                dep[g] = dep.get(g, 0.0) + float(w["edep"][k])
        rec.update(panel=p, xl=xl, dl=dl, e=e, L=L, entry=ent, dep=dep)
        if ent.in_domain:
            rec["label"], rec["truncated"] = outcome_class(spec, lat, ent, p, e, dep)
        out.append(rec)
    return out


# ---------------------------------------------------------------------------
# MLP in float64
# ---------------------------------------------------------------------------
def forward(params, x, store=None):
    """params: [(W [out, in], b [out]), ...]; ReLU after every layer but the
    last.  `store` (optional) rounds every hidden activation as it is stored
    (the method keeps activations in BF16; arithmetic stays float64).
    Returns (logits, list of layer inputs, list of pre-activations)."""
    keep = store or (lambda a: a)
    h = np.asarray(x, np.float64)
    ins, zs = [], []
    for k, (W, b) in enumerate(params):
        ins.append(h)
        z = h @ W.T + b
        zs.append(z)
        h = keep(np.maximum(z, 0.0)) if k < len(params) - 1 else z
    return h, ins, zs


def softmax(z):
    m = z.max(axis=1, keepdims=True)
    e = np.exp(z - m)
    return e / e.sum(axis=1, keepdims=True)


def loss_and_grad(params, x, y, store=None):
    """Mean softmax cross-entropy over the batch and its gradient with respect
    to every weight and bias (backpropagation written out).  `store`
    (optional) rounds the hidden activations as the forward pass stores them
    (the method's BF16 activations); the backward pass is exact float64."""
    z, ins, zs = forward(params, x, store)
    n = len(y)
    m = z.max(axis=1)
    lse = m + np.log(np.exp(z - m[:, None]).sum(axis=1))
    loss = float(np.mean(lse - z[np.arange(n), y]))
    dz = softmax(z)
    dz[np.arange(n), y] -= 1.0
    dz = dz / n
    grads = [None] * len(params)
    for k in range(len(params) - 1, -1, -1):
        W, _ = params[k]
        grads[k] = (dz.T @ ins[k], dz.sum(axis=0))
        if k:
            dz = (dz @ W) * (ins[k] > 0.0)
    return loss, grads


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) of every tensor; t counts from 1.
    Returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        new = []
        for w, g, mm, vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mm = beta1 * mm + (1.0 - beta1) * g
            vv = beta2 * vv + (1.0 - beta2) * g * g
            mh = mm / (1.0 - beta1 ** t)
            vh = vv / (1.0 - beta2 ** t)
            new.append((w - lr * mh / (np.sqrt(vh) + eps), mm, vv))
        out_p.append((new[0][0], new[1][0]))
        out_m.append((new[0][1], new[1][1]))
        out_v.append((new[0][2], new[1][2]))
    return out_p, out_m, out_v


def sample_class(logits, u):
    """First class whose cumulative softmax probability reaches u (per row)."""
    p = softmax(np.atleast_2d(logits))
    cdf = np.cumsum(p, axis=1)
    u = np.atleast_1d(u)
    return np.minimum((cdf < u[:, None]).sum(axis=1), p.shape[1] - 1)


# ---------------------------------------------------------------------------
# factored output: an energy head, then the position given the energy
# ---------------------------------------------------------------------------
# The outcome class (position k in the neighbourhood, energy index b, or
# none) is drawn in two steps: the energy class e (0 = none, 1 + b
# otherwise) from a softmax over the first n_first logits, then, for e > 0,
# the position from a softmax over one block of n2 position logits plus a
# learned row T[e - 1] of per-energy position offsets.  The logits after the
# energy head hold n_groups such blocks; energy class e uses block
# g(e) = (e - 1) n_groups // (n_first - 1), so contiguous groups of energy
# classes share one.  The joint label keeps the layout of outcome_class: 0,
# or 1 + k (n_first - 1) + (e - 1).
def factored_split(y, n_first):
    """Joint labels -> (energy class e, position k; k = 0 where e = 0)."""
    y = np.asarray(y, np.int64)
    c = np.maximum(y - 1, 0)
    e = np.where(y > 0, 1 + c % (n_first - 1), 0)
    k = np.where(y > 0, c // (n_first - 1), 0)
    return e, k


def factored_join(e, k, n_first):
    e = np.asarray(e, np.int64)
    return np.where(e > 0, 1 + np.asarray(k, np.int64) * (n_first - 1) + (e - 1), 0)


def _position_logits(z, T, e, n_first, n_groups):
    """Rows' position logits for energy classes e > 0: block g(e) plus T[e - 1]."""
    n2 = (z.shape[1] - n_first) // n_groups
    start = n_first + ((e - 1) * n_groups // (n_first - 1)) * n2
    cols = start[:, None] + np.arange(n2)[None, :]
    return np.take_along_axis(z, cols, axis=1) + T[e - 1], cols


def factored_log_prob(z, T, y, n_first, n_groups=1):
    """log P(y | x) per row from output logits z and the offset table T."""
    e, k = factored_split(y, n_first)
    z1 = z[:, :n_first]
    m1 = z1.max(axis=1)
    lp = z1[np.arange(len(e)), e] - (m1 + np.log(np.exp(z1 - m1[:, None]).sum(axis=1)))
    pos = e > 0
    if pos.any():
        z2p, _ = _position_logits(z[pos], T, e[pos], n_first, n_groups)
        m2 = z2p.max(axis=1)
        lp[pos] += z2p[np.arange(pos.sum()), k[pos]] - (m2 + np.log(np.exp(z2p - m2[:, None]).sum(axis=1)))
    return lp


def factored_loss_and_grad(params, T, x, y, n_first, store=None, n_groups=1):
    """Mean of -log P(y | x) under the factored output, and its gradient with
    respect to every weight and bias and to T (backpropagation written out;
    `store` rounds hidden activations as in loss_and_grad)."""
    z, ins, zs = forward(params, x, store)
    n = len(y)
    e, k = factored_split(y, n_first)
    loss = float(-np.mean(factored_log_prob(z, T, y, n_first, n_groups)))
    dz = np.zeros_like(z)
    dz[:, :n_first] = softmax(z[:, :n_first])
    dz[np.arange(n), e] -= 1.0
    pos = np.flatnonzero(e > 0)
    gT = np.zeros_like(T)
    if len(pos):
        z2p, cols = _position_logits(z[pos], T, e[pos], n_first, n_groups)
        p2 = softmax(z2p)
        p2[np.arange(len(pos)), k[pos]] -= 1.0
        block = dz[pos]
        np.put_along_axis(block, cols, p2, axis=1)
        dz[pos] = block
        np.add.at(gT, e[pos] - 1, p2 / n)
    dz = dz / n
    grads = [None] * len(params)
    for j in range(len(params) - 1, -1, -1):
        W, _ = params[j]
        grads[j] = (dz.T @ ins[j], dz.sum(axis=0))
        if j:
            dz = (dz @ W) * (ins[j] > 0.0)
    return loss, grads, gT


def factored_sample(z, T, n_first, u_energy_class, u_position, n_groups=1, exists=None):
    """Joint class per row: e = first energy class whose cumulative softmax
    mass reaches u_energy_class; for e > 0, the first position whose
    cumulative mass under softmax(block g(e) + T[e - 1]) reaches u_position.
    exists (optional, rows x positions): positions that cannot occur are
    left out of that softmax."""
    z = np.atleast_2d(z)
    e = sample_class(z[:, :n_first], u_energy_class)
    k = np.zeros_like(e)
    pos = np.flatnonzero(e > 0)
    if len(pos):
        z2p, _ = _position_logits(z[pos], T, e[pos], n_first, n_groups)
        if exists is not None:
            ex = np.atleast_2d(exists)[pos]
            z2p = np.where(ex, z2p, -np.inf)
            kk = sample_class(z2p, np.atleast_1d(u_position)[pos])
            # a target beyond the total by rounding: the last position that exists
            last = ex.shape[1] - 1 - np.argmax(ex[:, ::-1], axis=1)
            k[pos] = np.where(ex[np.arange(len(pos)), kk], kk, last)
        else:
            k[pos] = sample_class(z2p, np.atleast_1d(u_position)[pos])
    return factored_join(e, k, n_first)


def unpack(flat, sizes):
    """Packed float32 weights (per layer: W [out, in] row-major, then b [out])
    -> list of float64 (W, b)."""
    params, o = [], 0
    for i, j in zip(sizes[:-1], sizes[1:]):
        W = np.asarray(flat[o:o + i * j], np.float64).reshape(j, i)
        o += i * j
        b = np.asarray(flat[o:o + j], np.float64)
        o += j
        params.append((W, b))
    return params


def unpack_factored(flat, sizes, n_first, n_groups=1):
    """Packed weights of a factored network: the layers as in unpack, then the
    offset table T [n_first - 1][(sizes[-1] - n_first) / n_groups] row-major."""
    n_layers = sum(i * j + j for i, j in zip(sizes[:-1], sizes[1:]))
    n2 = (sizes[-1] - n_first) // n_groups
    T = np.asarray(flat[n_layers:n_layers + (n_first - 1) * n2], np.float64).reshape(n_first - 1, n2)
    return unpack(flat[:n_layers], sizes), T


def bf16_round(a):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float64."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
