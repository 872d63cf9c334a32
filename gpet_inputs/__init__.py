"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module only *describes* workloads: material compositions, scanner
parameters, phantom voxel grids and source descriptors, as plain Python
dicts and numpy arrays.  It holds none of the simulation's arithmetic (no
attenuation tables, no panel placement, no sampling); each side derives
those from these descriptions on its own.

Units: mm, keV, ps, g/cm^3.  Material ids index the scene's ``materials``
list.

The scanner description follows the four-level hierarchy of the paper
(panel -> module -> layer -> crystal, Sec. 2.1 and Fig. 1): panels placed
in repetition mode (count, front-face distance, first angle) or by explicit
poses; each panel carries a grid of modules; each module carries an ordered
list of layers, each with its own crystal count, size, pitch, offset and
crystal/interval materials.
"""
from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# Materials (composition only).  Atomic masses in g/mol.
# ---------------------------------------------------------------------------
_A = {1: 1.008, 7: 14.007, 8: 15.999, 14: 28.086, 18: 39.948, 32: 72.630, 39: 88.906, 71: 174.967,
      83: 208.980}

PROC_PE, PROC_COMPTON, PROC_RAYLEIGH = 1, 2, 4
PROC_ALL = PROC_PE | PROC_COMPTON | PROC_RAYLEIGH


def _by_atoms(counts: dict[int, float]) -> tuple[list[int], list[float], list[float]]:
    zs = sorted(counts)
    mass = [counts[z] * _A[z] for z in zs]
    tot = sum(mass)
    return zs, [_A[z] for z in zs], [m / tot for m in mass]


def material(name: str, density: float | None = None, mask: int = PROC_ALL) -> dict:
    """Composition of a named material.  ``density`` overrides the nominal one."""
    if name == "lyso":  # Lu1.8 Y0.2 Si O5
        zs, a, w = _by_atoms({71: 1.8, 39: 0.2, 14: 1.0, 8: 5.0})
        rho = 7.4
    elif name == "water":
        zs, a, w = _by_atoms({1: 2.0, 8: 1.0})
        rho = 1.0
    elif name == "bgo":  # Bi4 Ge3 O12
        zs, a, w = _by_atoms({83: 4.0, 32: 3.0, 8: 12.0})
        rho = 7.13
    elif name == "air":  # dry air by mass: N, O, Ar
        zs = [7, 8, 18]
        a = [_A[z] for z in zs]
        w = [0.7553, 0.2318, 0.0129]
        s = sum(w)
        w = [x / s for x in w]
        rho = 1.205e-3
    else:
        raise KeyError(name)
    return {"name": name, "density": float(rho if density is None else density),
            "Z": zs, "A": a, "w": w, "mask": int(mask)}


# Physics constants of the synthetic attenuation model: photoelectric
# K_pe Z^4/E^3 and Rayleigh K_R Z^2/E^2 per atom (E in MeV, cm^2).
K_PE = 7.9e-32
K_R = 6.67e-29
E_CUT_KEV = 10.0

POINT_ACTIVITY_BQ = 1.70e4          # 18F point source, about 1.7e-2 MBq
ROD_ACTIVITY_BQ_PER_MM3 = 92.1      # 9.21e-5 MBq/mm^3


def physics(rayleigh: bool = True) -> dict:
    return {"k_pe": K_PE, "k_r": K_R if rayleigh else 0.0, "e_cut": E_CUT_KEV}


def duration_ps(n_events: int, activity_bq: float) -> int:
    """Acquisition length that holds ``n_events`` decays at ``activity_bq``."""
    return int(round(n_events / activity_bq * 1e12))


# ---------------------------------------------------------------------------
# Scanners
# ---------------------------------------------------------------------------
def layer(depth0, thick, n_t, n_a, cryst_t, cryst_a, pitch_t, pitch_a,
          off_t=0.0, off_a=0.0, mat_crystal=0, mat_interval=1) -> dict:
    return {"depth0": float(depth0), "thick": float(thick), "n_t": int(n_t), "n_a": int(n_a),
            "cryst_t": float(cryst_t), "cryst_a": float(cryst_a),
            "pitch_t": float(pitch_t), "pitch_a": float(pitch_a),
            "off_t": float(off_t), "off_a": float(off_a),
            "mat_crystal": int(mat_crystal), "mat_interval": int(mat_interval)}


def scanner(n_panels, radius, depth, mod_n_t, mod_n_a, mod_t, mod_a, gap_t, gap_a,
            layers, mat_fill=1, phi0=0.0, z0=0.0, width=None, length=None,
            poses=None) -> dict:
    """Panel box = module array unless ``width``/``length`` are given."""
    w_mod = mod_n_t * mod_t + (mod_n_t - 1) * gap_t
    l_mod = mod_n_a * mod_a + (mod_n_a - 1) * gap_a
    return {"mode": "explicit" if poses is not None else "repeat",
            "n_panels": int(n_panels), "radius": float(radius), "phi0": float(phi0),
            "z0": float(z0), "poses": None if poses is None else np.asarray(poses, np.float64),
            "depth": float(depth), "width": float(w_mod if width is None else width),
            "length": float(l_mod if length is None else length),
            "mod_n_t": int(mod_n_t), "mod_n_a": int(mod_n_a),
            "mod_t": float(mod_t), "mod_a": float(mod_a),
            "gap_t": float(gap_t), "gap_a": float(gap_a),
            "mat_fill": int(mat_fill), "layers": list(layers)}


# ---------------------------------------------------------------------------
# Sources
# ---------------------------------------------------------------------------
SRC_POINT, SRC_CYLINDERS, SRC_BEAM = 0, 1, 2


def point_source(pos=(0.0, 0.0, 0.0), n_events=100_000, activity=POINT_ACTIVITY_BQ) -> dict:
    return {"kind": SRC_POINT, "pos": tuple(float(v) for v in pos), "dir": (0.0, 0.0, 1.0),
            "rods": None, "duration_ps": duration_ps(n_events, activity)}


def beam_source(pos, direction, n_events=100_000) -> dict:
    """Pencil beam: both photons of an event leave ``pos`` along +/-``direction``."""
    d = np.asarray(direction, np.float64)
    d = d / np.linalg.norm(d)
    return {"kind": SRC_BEAM, "pos": tuple(float(v) for v in pos), "dir": tuple(float(v) for v in d),
            "rods": None, "duration_ps": duration_ps(n_events, POINT_ACTIVITY_BQ)}


def hot_rod_layout(diameters=(0.8, 1.0, 1.25, 1.5, 1.75, 2.0), r_max=11.5, length=20.0) -> np.ndarray:
    """Six-sector hot-rod (Derenzo-style) source: rows of rods at 2d spacing.

    Sector k is centred on the bisector at 60k + 30 degrees.  Row j lies at
    distance h0 + j*2d*sqrt(3)/2 from the centre (h0 = d + 1 mm) and holds
    j + 1 rods spaced 2d apart, centred on the bisector.  Whole rows are kept
    while every rod edge stays within ``r_max``.  Returns rows of
    (cx, cy, radius, z0, z1).
    """
    rods = []
    for k, d in enumerate(diameters):
        ang = math.radians(60.0 * k + 30.0)
        ux, uy = math.cos(ang), math.sin(ang)          # along the bisector
        vx, vy = -uy, ux                                # across it
        j = 0
        while True:
            h = (d + 1.0) + j * 2.0 * d * math.sqrt(3.0) / 2.0
            row = []
            for i in range(j + 1):
                off = (i - j / 2.0) * 2.0 * d
                row.append((h * ux + off * vx, h * uy + off * vy))
            if any(math.hypot(x, y) + d / 2.0 > r_max for x, y in row):
                break
            for x, y in row:
                rods.append((x, y, d / 2.0, -length / 2.0, length / 2.0))
            j += 1
    return np.asarray(rods, np.float64)


def derenzo_layout(diameters=(0.3, 0.4, 0.5, 0.625, 0.75, 1.0), rows=(3, 4, 5, 6, 7, 8),
                   length=20.0) -> np.ndarray:
    """Derenzo rods of the paper's visibility study (Sec. 2.3): six sectors of
    rods of one diameter each, 2d centre-to-centre, 20 mm long; sector k holds
    rows[k] rows (1 + 2 + ... rods: 6, 10, 15, 21, 28, 36).  Placement follows
    hot_rod_layout (sector bisectors at 60k + 30 degrees, first row at d + 1 mm).
    Returns rows of (cx, cy, radius, z0, z1)."""
    rods = []
    for k, (d, n_rows) in enumerate(zip(diameters, rows)):
        ang = math.radians(60.0 * k + 30.0)
        ux, uy = math.cos(ang), math.sin(ang)
        vx, vy = -uy, ux
        for j in range(n_rows):
            h = (d + 1.0) + j * 2.0 * d * math.sqrt(3.0) / 2.0
            for i in range(j + 1):
                off = (i - j / 2.0) * 2.0 * d
                rods.append((h * ux + off * vx, h * uy + off * vy, d / 2.0, -length / 2.0, length / 2.0))
    return np.asarray(rods, np.float64)


def rod_source(rods: np.ndarray, n_events: int) -> dict:
    vol = float(np.sum(math.pi * rods[:, 2] ** 2 * (rods[:, 4] - rods[:, 3])))
    return {"kind": SRC_CYLINDERS, "pos": (0.0, 0.0, 0.0), "dir": (0.0, 0.0, 1.0),
            "rods": np.ascontiguousarray(rods, np.float64),
            "duration_ps": duration_ps(n_events, ROD_ACTIVITY_BQ_PER_MM3 * vol)}


# ---------------------------------------------------------------------------
# Phantoms
# ---------------------------------------------------------------------------
def water_cylinder_phantom(diameter=25.0, length=70.0, voxel=0.5, mat_water=2, mat_air=1,
                           water_density=1.0, air_density=1.205e-3) -> dict:
    """Voxelized water cylinder along z, air around it; voxel centres decide."""
    nx = ny = int(round(diameter / voxel))
    nz = int(round(length / voxel))
    ox, oy, oz = -diameter / 2.0, -diameter / 2.0, -length / 2.0
    xc = ox + (np.arange(nx) + 0.5) * voxel
    yc = oy + (np.arange(ny) + 0.5) * voxel
    inside = (xc[None, :] ** 2 + yc[:, None] ** 2) <= (diameter / 2.0) ** 2   # [iy, ix]
    mat2 = np.where(inside, mat_water, mat_air).astype(np.uint8)
    den2 = np.where(inside, water_density, air_density).astype(np.float32)
    mat = np.ascontiguousarray(np.broadcast_to(mat2, (nz, ny, nx)))
    den = np.ascontiguousarray(np.broadcast_to(den2, (nz, ny, nx)))
    return {"shape": (nx, ny, nz), "voxel": (voxel, voxel, voxel), "origin": (ox, oy, oz),
            "mat": mat, "dens": den}


def water_box_phantom(side=40.25, voxel=0.5, mat_water=2, water_density=1.0) -> dict:
    """Voxelized water cube centred at the origin (the Derenzo phantom's body)."""
    n = int(round(side / voxel))
    o = -n * voxel / 2.0
    return {"shape": (n, n, n), "voxel": (voxel, voxel, voxel), "origin": (o, o, o),
            "mat": np.full((n, n, n), mat_water, np.uint8), "dens": np.full((n, n, n), water_density, np.float32)}


def slab_phantom(mats, thicknesses, densities, cross=20.0, voxel=0.5) -> dict:
    """Stack of slabs along +x starting at x = 0 (for narrow-beam checks)."""
    n_per = [int(round(t / voxel)) for t in thicknesses]
    nx = sum(n_per)
    ny = nz = int(round(cross / voxel))
    mat = np.zeros((nz, ny, nx), np.uint8)
    den = np.zeros((nz, ny, nx), np.float32)
    x0 = 0
    for m, n, rho in zip(mats, n_per, densities):
        mat[:, :, x0:x0 + n] = m
        den[:, :, x0:x0 + n] = rho
        x0 += n
    return {"shape": (nx, ny, nz), "voxel": (voxel, voxel, voxel),
            "origin": (0.0, -cross / 2.0, -cross / 2.0), "mat": mat, "dens": den}


# ---------------------------------------------------------------------------
# Whole scenes for the standard workloads
# ---------------------------------------------------------------------------
def scene(materials, phys, scan, source, phantom=None) -> dict:
    return {"materials": materials, "physics": phys, "scanner": scan,
            "source": source, "phantom": phantom}


def ring8_scene(n_events=100_000, source=None, black=False) -> dict:
    """Ring of 8 flat panels at 40 mm, one module of 8x8 LYSO 1.5x1.5x10 mm
    crystals at 1.6 mm pitch, one layer, LYSO at 7.1 g/cm^3, no Rayleigh,
    no phantom, isotropic back-to-back point source at the centre.

    ``black``: crystals fill the module face (1x1 crystal of 12.8 mm) and are
    a photoelectric-only absorber, for the analytic solid-angle check.
    """
    if black:
        mats = [material("lyso", density=7.1e4, mask=PROC_PE), material("air")]
        lay = [layer(0.0, 10.0, 1, 1, 12.8, 12.8, 12.8, 12.8)]
    else:
        mats = [material("lyso", density=7.1), material("air")]
        lay = [layer(0.0, 10.0, 8, 8, 1.5, 1.5, 1.6, 1.6)]
    scan = scanner(8, 40.0, 10.0, 1, 1, 12.8, 12.8, 0.0, 0.0, lay)
    src = source if source is not None else point_source((0, 0, 0), n_events)
    return scene(mats, physics(rayleigh=False), scan, src)


DESIGNS = ("A", "B", "C", "B0")


def small_animal_layers(design: str, n=24, pitch=1.0, cryst=0.92, thick=10.0, gap=None,
                        offset=None):
    """Layer stacks of the synthetic small-animal designs.

    A: one 2*thick layer; B: two aligned layers with a 0.2 mm gap;
    C: inner (n-1)x(n-1) layer offset by half a pitch over an outer n x n layer;
    B0: two aligned layers with no gap (split of A).
    ``gap``/``offset`` (fraction of pitch) override for design sweeps.
    """
    if design == "A":
        return [layer(0.0, 2 * thick, n, n, cryst, cryst, pitch, pitch)]
    if design in ("B", "B0", "C", "X"):
        g = {"B": 0.2, "B0": 0.0, "C": 0.0, "X": 0.0}[design] if gap is None else gap
        o = {"B": 0.0, "B0": 0.0, "C": 0.5, "X": 0.0}[design] if offset is None else offset
        n0 = n - 1 if o > 0 else n
        l0 = layer(0.0, thick, n0, n0, cryst, cryst, pitch, pitch, o * pitch, o * pitch)
        l1 = layer(thick + g, thick, n, n, cryst, cryst, pitch, pitch)
        return [l0, l1]
    raise KeyError(design)


def small_animal_scanner(design: str, thick=10.0, gap=None, offset=None, black=False) -> dict:
    """12 panels at 65 mm; 1 x 4 modules of 24 x 24 crystals (0.92 + 0.08 air),
    2 mm axial module gap; LYSO 7.4 g/cm^3."""
    lays = small_animal_layers(design, thick=thick, gap=gap, offset=offset)
    if black:
        lays = [layer(0.0, 2 * thick, 1, 1, 24.0, 24.0, 24.0, 24.0)]
    depth = max(l["depth0"] + l["thick"] for l in lays)
    return scanner(12, 65.0, depth, 1, 4, 24.0, 24.0, 0.0, 2.0, lays)


STACKS = ("stack3", "stack4")


def stack_scanner(kind: str) -> dict:
    """Deeper stacks on the small-animal panel (12 panels at 65 mm, 1 x 4
    modules of 24 mm, 1 mm pitch, 0.92 mm crystals), for the 3- and 4-layer
    architectures the paper points to (Discussion).
    stack3: 22x22 (6 mm, centred), 0.2 mm gap, 23x23 (7 mm, half-pitch
    offset), 24x24 (7 mm);
    stack4: four 5 mm layers alternating BGO (material 2) and LYSO: 24x24,
    23x24 shifted half a pitch along t, 24x23 shifted along a, 23x23 shifted
    along both."""
    if kind == "stack3":
        lays = [layer(0.0, 6.0, 22, 22, 0.92, 0.92, 1.0, 1.0, 1.0, 1.0),
                layer(6.2, 7.0, 23, 23, 0.92, 0.92, 1.0, 1.0, 0.5, 0.5),
                layer(13.2, 7.0, 24, 24, 0.92, 0.92, 1.0, 1.0)]
    elif kind == "stack4":
        lays = [layer(0.0, 5.0, 24, 24, 0.92, 0.92, 1.0, 1.0, mat_crystal=2),
                layer(5.0, 5.0, 23, 24, 0.92, 0.92, 1.0, 1.0, 0.5, 0.0),
                layer(10.0, 5.0, 24, 23, 0.92, 0.92, 1.0, 1.0, 0.0, 0.5, mat_crystal=2),
                layer(15.0, 5.0, 23, 23, 0.92, 0.92, 1.0, 1.0, 0.5, 0.5)]
    else:
        raise KeyError(kind)
    depth = max(l["depth0"] + l["thick"] for l in lays)
    return scanner(12, 65.0, depth, 1, 4, 24.0, 24.0, 0.0, 2.0, lays)


def stack_scene(kind: str, pos=(0.0, 0.0, 0.0), n_events: int = 1_000_000) -> dict:
    mats = [material("lyso"), material("air"), material("bgo")]
    return scene(mats, physics(rayleigh=True), stack_scanner(kind), point_source(pos, n_events))


H2RSPET = ("1CL", "1CL-split", "2CL")


def h2rspet_scanner(kind: str) -> dict:
    """The paper's validation scanners (Sec. 2.2): 10 panels at 85 mm, each
    1.0 x 5.1 x 34.1 cm (radial x tangential x axial) holding 6 modules along
    the axis, 51 x 51 crystals of 0.92 mm at 1.0 mm pitch, 7 mm between
    modules; 1CL: one 10 mm layer; 1CL-split: two aligned 5 mm layers;
    2CL: an inner 50 x 50 layer offset by half a pitch (R-offset) over an outer
    51 x 51 layer, 5 mm each."""
    if kind == "1CL":
        lays = [layer(0.0, 10.0, 51, 51, 0.92, 0.92, 1.0, 1.0)]
    elif kind == "1CL-split":
        lays = [layer(0.0, 5.0, 51, 51, 0.92, 0.92, 1.0, 1.0), layer(5.0, 5.0, 51, 51, 0.92, 0.92, 1.0, 1.0)]
    elif kind == "2CL":
        lays = [layer(0.0, 5.0, 50, 50, 0.92, 0.92, 1.0, 1.0, 0.5, 0.5),
                layer(5.0, 5.0, 51, 51, 0.92, 0.92, 1.0, 1.0)]
    else:
        raise KeyError(kind)
    return scanner(10, 85.0, 10.0, 1, 6, 51.0, 51.0, 0.0, 7.0, lays)


def derenzo_scene(kind: str = "2CL", n_events: int = 1_000_000, with_phantom: bool = True) -> dict:
    """An H2RSPET scanner with the Derenzo rods in a water cube."""
    mats = [material("lyso", density=7.4), material("air"), material("water")]
    ph = water_box_phantom() if with_phantom else None
    return scene(mats, physics(rayleigh=True), h2rspet_scanner(kind), rod_source(derenzo_layout(), n_events), ph)


# Source positions of the sensitivity sweep: radial 0..50 mm (5 mm steps) along
# +x at z = 0, then axial 10..50 mm (10 mm steps) at r = 0.
SWEEP_POSITIONS = ([(float(r), 0.0, 0.0) for r in range(0, 55, 5)]
                   + [(0.0, 0.0, float(z)) for z in range(10, 60, 10)])


def small_animal_scene(design="C", pos=(0.0, 0.0, 0.0), n_events=10_000_000, black=False,
                       rayleigh=True) -> dict:
    if black:
        mats = [material("lyso", density=7.4e4, mask=PROC_PE), material("air")]
    else:
        mats = [material("lyso", density=7.4), material("air")]
    return scene(mats, physics(rayleigh=rayleigh), small_animal_scanner(design, black=black),
                 point_source(pos, n_events))


def hot_rod_scene(n_events=100_000_000, with_phantom=True) -> dict:
    """Design C with a voxelized water cylinder and the six-sector rod source."""
    mats = [material("lyso", density=7.4), material("air"), material("water")]
    ph = water_cylinder_phantom() if with_phantom else None
    return scene(mats, physics(rayleigh=True), small_animal_scanner("C"),
                 rod_source(hot_rod_layout(), n_events), ph)


def black_ring_scene(n_panels, radius, width, length, depth, n_events=1_000_000,
                     density=7.4e4) -> dict:
    """Ring of gap-free panels, each one crystal filling the panel face, made of a
    photoelectric-only LYSO at a very high density (an ideal absorber), for the
    analytic solid-angle efficiency of a centred point source."""
    mats = [material("lyso", density=density, mask=PROC_PE), material("air")]
    lay = [layer(0.0, depth, 1, 1, width, length, width, length)]
    scan = scanner(n_panels, radius, depth, 1, 1, width, length, 0.0, 0.0, lay)
    return scene(mats, physics(rayleigh=False), scan, point_source((0, 0, 0), n_events))


def tilted_ring_poses(n_panels=8, radius=40.0, tilt_deg=12.0) -> np.ndarray:
    """Explicit (non-repetition) panel poses: a ring whose panels are each tilted
    by ``tilt_deg`` about their own tangential axis, so no axis is global z.
    Rows: front-face centre, depth axis, t axis, a axis."""
    out = []
    tl = math.radians(tilt_deg)
    for k in range(n_panels):
        ph = 2 * math.pi * k / n_panels
        c, s = math.cos(ph), math.sin(ph)
        radial = np.array([c, s, 0.0])
        tang = np.array([-s, c, 0.0])
        z = np.array([0.0, 0.0, 1.0])
        depth = math.cos(tl) * radial + math.sin(tl) * z
        axial = -math.sin(tl) * radial + math.cos(tl) * z
        out.append(np.concatenate([radius * radial, depth, tang, axial]))
    return np.asarray(out)


def tilted_ring_scene(n_events=100_000) -> dict:
    sc = ring8_scene(n_events=n_events)
    g = sc["scanner"]
    sc["scanner"] = scanner(8, 40.0, g["depth"], 1, 1, 12.8, 12.8, 0.0, 0.0, g["layers"],
                            poses=tilted_ring_poses())
    return sc


# Batched design sweep: layer thickness (each of two layers) x inner-layer
# offset (fraction of the pitch) x inter-layer gap, each design at four radial
# point-source offsets.
SWEEP_THICK = (6.0, 8.0, 10.0, 12.0)
SWEEP_OFFSET = (0.0, 0.25, 0.5)
SWEEP_GAP = (0.0, 0.2, 0.5)
SWEEP_SOURCE_X = (0.0, 15.0, 30.0, 45.0)


def batch_sweep(n_scale=1.0, seed=0, n_lo=1e5, n_hi=1e7):
    """Instances of the batched sweep: 36 designs x 4 source offsets = 144.

    Event counts are log-uniform: n_i = round(n_scale * 10^(log10 n_lo + u_i
    log10(n_hi / n_lo))), u_i from numpy's PCG64 stream of `seed` (at least 1).
    Returns (materials, physics, instances); an instance is a dict with keys
    scanner, source, n_events, first_event (0), instance (its index) and label.
    """
    mats = [material("lyso", density=7.4), material("air")]
    u = np.random.default_rng(seed).random(len(SWEEP_THICK) * len(SWEEP_OFFSET) * len(SWEEP_GAP)
                                           * len(SWEEP_SOURCE_X))
    a, b = math.log10(n_lo), math.log10(n_hi)
    out = []
    i = 0
    for t in SWEEP_THICK:
        for o in SWEEP_OFFSET:
            for g in SWEEP_GAP:
                scan = small_animal_scanner("X", thick=t, gap=g, offset=o)
                for x in SWEEP_SOURCE_X:
                    n = max(1, int(round(n_scale * 10.0 ** (a + u[i] * (b - a)))))
                    out.append({"scanner": scan, "source": point_source((x, 0.0, 0.0), n), "n_events": n,
                                "first_event": 0, "instance": i,
                                "label": f"t{t:g}_o{o:g}_g{g:g}_x{x:g}"})
                    i += 1
    return mats, physics(rayleigh=True), out


SURROGATE_HIDDEN = (256, 256, 256, 256)


def mlp_init(sizes, seed=0):
    """Initial MLP parameters: He-normal weights (std sqrt(2 / fan_in)) on the
    hidden layers, std sqrt(1 / fan_in) / 4 on the output layer, zero biases;
    numpy PCG64 stream of `seed`.  Returns [(W [out, in], b [out]), ...] as
    float32."""
    rng = np.random.default_rng(seed)
    out = []
    n = len(sizes) - 1
    for k, (i, j) in enumerate(zip(sizes[:-1], sizes[1:])):
        std = math.sqrt(2.0 / i) if k < n - 1 else 0.25 * math.sqrt(1.0 / i)
        out.append((rng.normal(0.0, std, (j, i)).astype(np.float32), np.zeros(j, np.float32)))
    return out
