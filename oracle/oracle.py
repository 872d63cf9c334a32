"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module.  It builds ``liboracle.so`` from ``gpet_oracle.c`` with gcc and
marshals scene descriptions from :mod:`gpet_inputs` into the oracle's own
structs.  It shares no code with the HIP library or its binding.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gpet_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

MAX_EL, MAX_MAT, MAX_LAYERS, MAX_PANELS, NE = 8, 8, 4, 64, 511


def build(force: bool = True) -> str:
    """Compile the oracle (plain IEEE double: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Material(C.Structure):
    _fields_ = [("density", C.c_double), ("n_el", C.c_int32), ("mask", C.c_int32),
                ("Z", C.c_int32 * MAX_EL), ("A", C.c_double * MAX_EL), ("w", C.c_double * MAX_EL)]


class Physics(C.Structure):
    _fields_ = [("k_pe", C.c_double), ("k_r", C.c_double), ("e_cut", C.c_double)]


class Layer(C.Structure):
    _fields_ = [("depth0", C.c_double), ("thick", C.c_double), ("n_t", C.c_int32), ("n_a", C.c_int32),
                ("cryst_t", C.c_double), ("cryst_a", C.c_double), ("pitch_t", C.c_double),
                ("pitch_a", C.c_double), ("off_t", C.c_double), ("off_a", C.c_double),
                ("mat_crystal", C.c_int32), ("mat_interval", C.c_int32)]


class Scanner(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_panels", C.c_int32), ("radius", C.c_double),
                ("phi0", C.c_double), ("z0", C.c_double), ("pose", (C.c_double * 12) * MAX_PANELS),
                ("depth", C.c_double), ("width", C.c_double), ("length", C.c_double),
                ("mod_n_t", C.c_int32), ("mod_n_a", C.c_int32), ("mod_t", C.c_double),
                ("mod_a", C.c_double), ("gap_t", C.c_double), ("gap_a", C.c_double),
                ("mat_fill", C.c_int32), ("n_layers", C.c_int32), ("layer", Layer * MAX_LAYERS)]


class Phantom(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("ox", C.c_double), ("oy", C.c_double), ("oz", C.c_double),
                ("mat", C.POINTER(C.c_uint8)), ("dens", C.POINTER(C.c_float))]


class Source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pos", C.c_double * 3), ("dir", C.c_double * 3),
                ("n_rods", C.c_int32), ("rods", C.POINTER(C.c_double)), ("duration_ps", C.c_uint64),
                ("acol_fwhm_deg", C.c_double), ("prange_fwhm_mm", C.c_double)]


class Scene(C.Structure):
    _fields_ = [("n_mat", C.c_int32), ("mat", Material * MAX_MAT), ("phys", Physics),
                ("scan", Scanner), ("has_phantom", C.c_int32), ("ph", Phantom), ("src", Source),
                ("mu_mass", ((C.c_double * NE) * 3) * MAX_MAT), ("maj_det", C.c_double * NE),
                ("maj_ph", C.c_double * NE), ("crystals_per_module", C.c_int32),
                ("crystals_per_panel", C.c_int32), ("n_crystals", C.c_int32),
                ("layer_base", C.c_int32 * MAX_LAYERS), ("rod_cum", C.c_double * 1024),
                ("rod_total", C.c_double)]


class Hit(C.Structure):
    _fields_ = [("event", C.c_uint32), ("photon", C.c_uint32), ("gid", C.c_uint32),
                ("panel", C.c_uint32), ("module", C.c_uint32), ("layer", C.c_uint32),
                ("crystal", C.c_uint32), ("process", C.c_uint32), ("seq", C.c_uint32),
                ("edep", C.c_double), ("tof_ps", C.c_double), ("depth", C.c_double),
                ("t", C.c_double), ("a", C.c_double), ("time_ps", C.c_uint64)]


class Vertex(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("event", "photon", "kind", "region", "panel", "gid", "mat",
                                         "accept", "process", "trials", "block")] + \
               [(n, C.c_double) for n in ("x", "y", "z", "e", "edep", "dx", "dy", "dz")]


class Digitizer(C.Structure):
    _fields_ = [("fwhm_511", C.c_double), ("e_lo", C.c_double), ("e_hi", C.c_double),
                ("window_ps", C.c_uint64), ("seed", C.c_uint64), ("instance", C.c_uint32),
                ("doi_bins", C.c_int32), ("readout", C.c_int32), ("time_fwhm_ps", C.c_double),
                ("doi_fwhm_mm", C.c_double), ("dead_ps", C.c_uint64), ("dead_mode", C.c_int32),
                ("dead_level", C.c_int32), ("ls_prob", C.c_double)]


class Single(C.Structure):
    _fields_ = [("event", C.c_uint32), ("gid", C.c_uint32), ("edep", C.c_double),
                ("energy", C.c_double), ("depth", C.c_double), ("time_ps", C.c_uint64),
                ("in_window", C.c_int32), ("lost", C.c_int32)]


V_STEP, V_ENTER_PANEL, V_EXIT, V_ESCAPE, V_DEAD, V_ENTER_PHANTOM, V_EMIT = range(7)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        P = C.POINTER
        L.or_philox.argtypes = [C.c_uint32, C.c_uint32, P(C.c_uint32), P(C.c_uint32), C.c_int64]
        L.or_sigma_kn.restype = C.c_double
        L.or_sigma_kn.argtypes = [C.c_double]
        L.or_event_time.restype = C.c_uint64
        L.or_event_time.argtypes = [C.c_uint64, C.c_uint64]
        L.or_prepare.argtypes = [P(Scene)]
        L.or_mu.argtypes = [P(Scene), C.c_int, C.c_double, P(C.c_double)]
        L.or_sample_compton.restype = C.c_int64
        L.or_sample_compton.argtypes = [C.c_double, C.c_int64, C.c_uint64, P(C.c_double),
                                        P(C.c_double), P(C.c_int32)]
        L.or_sample_rayleigh.argtypes = [C.c_int64, C.c_uint64, P(C.c_double)]
        L.or_locate.argtypes = [P(Scene), C.c_int64, P(C.c_double), P(C.c_int32), P(C.c_double)]
        L.or_ray_locate.argtypes = [P(Scene), C.c_int64, P(C.c_double), P(C.c_double), C.c_int32,
                                    C.c_double, P(C.c_double), P(C.c_int32), P(C.c_double)]
        L.or_transport_analog.restype = C.c_int64
        L.or_transport_analog.argtypes = [P(Scene), C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32,
                                          P(Hit), C.c_int64, P(C.c_int64)]
        L.or_transport.restype = C.c_int64
        L.or_transport.argtypes = [P(Scene), C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32,
                                   P(Hit), C.c_int64, P(C.c_int64)]
        L.or_trace_analog.restype = C.c_int64
        L.or_trace_analog.argtypes = [P(Scene), C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32, P(Vertex),
                                      C.c_int64]
        L.or_trace.restype = C.c_int64
        L.or_trace.argtypes = [P(Scene), C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32, P(Vertex),
                               C.c_int64]
        L.or_digitize.restype = C.c_int64
        L.or_digitize.argtypes = [P(Scene), P(Hit), C.c_int64, P(Digitizer), P(Single), C.c_int64,
                                  P(C.c_uint32), C.c_int64, P(C.c_int64)]
        L.or_num_threads.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int]
        L.or_set_threads.restype = None
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


# ---------------------------------------------------------------------------
def philox(seed: int, ctr: np.ndarray) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    out = np.empty_like(ctr)
    lib().or_philox(seed & 0xFFFFFFFF, seed >> 32, _ptr(ctr, C.c_uint32), _ptr(out, C.c_uint32),
                    len(ctr))
    return out


def sigma_kn(e_kev: float) -> float:
    return lib().or_sigma_kn(e_kev)


def event_time(x: int, duration_ps: int) -> int:
    """Event time of the 64-bit event-stream word x on an acquisition of duration_ps."""
    return int(lib().or_event_time(x, duration_ps))


def sample_compton(e_kev, n, seed=0):
    c = np.empty(n)
    e = np.empty(n)
    t = np.empty(n, np.int32)
    lib().or_sample_compton(e_kev, n, seed, _ptr(c, C.c_double), _ptr(e, C.c_double),
                            _ptr(t, C.c_int32))
    return c, e, t


def sample_rayleigh(n, seed=0):
    c = np.empty(n)
    lib().or_sample_rayleigh(n, seed, _ptr(c, C.c_double))
    return c


class OracleScene:
    """An oracle scene built from a :mod:`gpet_inputs` scene dict."""

    def __init__(self, sc: dict):
        self.desc = sc
        s = Scene()
        mats = sc["materials"]
        s.n_mat = len(mats)
        for i, m in enumerate(mats):
            M = s.mat[i]
            M.density = m["density"]
            M.n_el = len(m["Z"])
            M.mask = m["mask"]
            for j, (z, a, w) in enumerate(zip(m["Z"], m["A"], m["w"])):
                M.Z[j], M.A[j], M.w[j] = z, a, w
        ph = sc["physics"]
        s.phys.k_pe, s.phys.k_r, s.phys.e_cut = ph["k_pe"], ph["k_r"], ph["e_cut"]
        g = sc["scanner"]
        S = s.scan
        S.mode = 1 if g["mode"] == "explicit" else 0
        S.n_panels = g["n_panels"]
        S.radius, S.phi0, S.z0 = g["radius"], g["phi0"], g["z0"]
        if g["poses"] is not None:
            for p in range(g["n_panels"]):
                for k in range(12):
                    S.pose[p][k] = float(g["poses"][p][k])
        S.depth, S.width, S.length = g["depth"], g["width"], g["length"]
        S.mod_n_t, S.mod_n_a = g["mod_n_t"], g["mod_n_a"]
        S.mod_t, S.mod_a, S.gap_t, S.gap_a = g["mod_t"], g["mod_a"], g["gap_t"], g["gap_a"]
        S.mat_fill = g["mat_fill"]
        S.n_layers = len(g["layers"])
        for i, ly in enumerate(g["layers"]):
            L = S.layer[i]
            for k in ("depth0", "thick", "n_t", "n_a", "cryst_t", "cryst_a", "pitch_t", "pitch_a",
                      "off_t", "off_a", "mat_crystal", "mat_interval"):
                setattr(L, k, ly[k])
        self._keep = []
        p = sc.get("phantom")
        if p is not None:
            s.has_phantom = 1
            s.ph.nx, s.ph.ny, s.ph.nz = p["shape"]
            s.ph.dx, s.ph.dy, s.ph.dz = p["voxel"]
            s.ph.ox, s.ph.oy, s.ph.oz = p["origin"]
            m8 = np.ascontiguousarray(p["mat"], np.uint8)
            d32 = np.ascontiguousarray(p["dens"], np.float32)
            self._keep += [m8, d32]
            s.ph.mat = _ptr(m8, C.c_uint8)
            s.ph.dens = _ptr(d32, C.c_float)
        src = sc["source"]
        s.src.kind = src["kind"]
        for k in range(3):
            s.src.pos[k] = src["pos"][k]
            s.src.dir[k] = src["dir"][k]
        if src["rods"] is not None:
            rods = np.ascontiguousarray(src["rods"], np.float64)
            self._keep.append(rods)
            s.src.n_rods = len(rods)
            s.src.rods = _ptr(rods, C.c_double)
        s.src.duration_ps = int(src["duration_ps"])
        s.src.acol_fwhm_deg = float(src.get("acolinearity_fwhm_deg", 0.0))
        s.src.prange_fwhm_mm = float(src.get("positron_range_fwhm_mm", 0.0))
        rc = lib().or_prepare(C.byref(s))
        if rc != 0:
            raise ValueError(f"oracle scene rejected ({rc})")
        self.s = s

    # -- derived quantities
    @property
    def n_crystals(self):
        return self.s.n_crystals

    @property
    def crystals_per_panel(self):
        return self.s.crystals_per_panel

    def mu(self, m: int, e_kev: float) -> np.ndarray:
        o = (C.c_double * 3)()
        lib().or_mu(C.byref(self.s), m, e_kev, o)
        return np.array(o[:])

    def mass_table(self) -> np.ndarray:
        return np.ctypeslib.as_array(self.s.mu_mass)[: self.s.n_mat].copy()

    def poses(self) -> np.ndarray:
        return np.ctypeslib.as_array(self.s.scan.pose)[: self.s.scan.n_panels].copy()

    def majorant_det(self) -> np.ndarray:
        return np.array(self.s.maj_det[:])

    def majorant_ph(self) -> np.ndarray:
        return np.array(self.s.maj_ph[:])

    # -- geometry
    def locate(self, xyz: np.ndarray):
        xyz = np.ascontiguousarray(xyz, np.float64).reshape(-1, 3)
        ids = np.empty((len(xyz), 6), np.int32)
        bd = np.empty(len(xyz))
        lib().or_locate(C.byref(self.s), len(xyz), _ptr(xyz, C.c_double), _ptr(ids, C.c_int32),
                        _ptr(bd, C.c_double))
        return ids, bd

    def ray_locate(self, o, d, n_samp, step):
        o = np.ascontiguousarray(o, np.float64).reshape(-1, 3)
        d = np.ascontiguousarray(d, np.float64).reshape(-1, 3)
        n = len(o)
        t_in = np.empty(n)
        ids = np.empty((n, n_samp, 6), np.int32)
        bd = np.empty((n, n_samp))
        lib().or_ray_locate(C.byref(self.s), n, _ptr(o, C.c_double), _ptr(d, C.c_double), n_samp,
                            step, _ptr(t_in, C.c_double), _ptr(ids, C.c_int32), _ptr(bd, C.c_double))
        return t_in, ids, bd

    # -- transport
    def transport(self, n_events, seed=0, first=0, instance=0, analog=False):
        """Returns (hits structured array, counters dict); analog=True tracks
        from material boundary to boundary instead of Woodcock tracking."""
        cnt = np.zeros(9, np.int64)
        cap = max(16, int(3 * n_events))
        fn = lib().or_transport_analog if analog else lib().or_transport
        while True:
            buf = (Hit * cap)()
            n = fn(C.byref(self.s), first, n_events, seed, instance, buf, cap, _ptr(cnt, C.c_int64))
            if n <= cap:
                break
            cap = int(n)
            cnt[:] = 0
        arr = np.frombuffer(buf, dtype=np.dtype(Hit), count=n).copy()
        names = ("events", "panel_entries", "steps", "real", "kahn_trials", "searches", "blocks",
                 "capped", "scatters")
        return arr, dict(zip(names, cnt.tolist()))

    def trace(self, n_events, seed=0, first=0, instance=0, cap=None, analog=False):
        cap = cap or max(64, 200 * n_events)
        buf = (Vertex * cap)()
        fn = lib().or_trace_analog if analog else lib().or_trace
        n = fn(C.byref(self.s), first, n_events, seed, instance, buf, cap)
        if n > cap:
            return self.trace(n_events, seed, first, instance, int(n), analog)
        return np.frombuffer(buf, dtype=np.dtype(Vertex), count=n).copy()

    def digitize(self, hits, seed=0, fwhm_511=0.16, e_lo=350.0, e_hi=650.0, window_ps=3000,
                 instance=0, readout=0, time_fwhm_ps=0.0, doi_fwhm_mm=0.0, dead_ps=0, dead_mode=0,
                 dead_level=1, light_sharing=0.0):
        """Adder, readout (0 crystal, 1 module, 2 panel), energy / time / depth
        blur, light sharing (probability of reading a neighbour crystal),
        dead time (mode 0 none, 1 paralyzable, 2 non-paralyzable; level as
        readout), window and coincidence sorter; returns (singles,
        coincidence index pairs)."""
        hits = np.ascontiguousarray(hits)
        dg = Digitizer(fwhm_511, e_lo, e_hi, window_ps, seed, instance, 200, readout, time_fwhm_ps,
                       doi_fwhm_mm, int(dead_ps), dead_mode, dead_level, light_sharing)
        n = len(hits)
        sg = (Single * max(1, n))()
        cc = np.empty((max(1, n), 2), np.uint32)
        nc = C.c_int64(0)
        hp = hits.ctypes.data_as(C.POINTER(Hit))
        ns = lib().or_digitize(C.byref(self.s), hp, n, C.byref(dg), sg, max(1, n),
                               _ptr(cc, C.c_uint32), max(1, n), C.byref(nc))
        singles = np.frombuffer(sg, dtype=np.dtype(Single), count=ns).copy()
        return singles, cc[: nc.value].copy()

    def tallies(self, hits, singles, doi_bins=200):
        """Scanner tallies of this scene's detector (see :func:`tallies`)."""
        return tallies(hits, singles, self.n_crystals, float(self.s.scan.depth), doi_bins)


def tallies(hits, singles, n_crystals, panel_depth, doi_bins=200):
    """The scanner tallies the paper reads its results from (Sec. 2.3
    sensitivity and energy windows; Sec. 3.1, Fig. 3: depth-of-interaction
    histograms of the hits), written out one item at a time:

    * ``hits_per_crystal[g]``: hits recorded in crystal g;
    * ``singles_per_crystal[g]``: singles of crystal g inside the energy
      window and not lost to dead time;
    * ``energy_spectrum[k]``: live singles whose blurred energy E lies in
      [k, k + 1) keV, k = 0..699 (energies outside [0, 700) are not counted);
    * ``doi[b]``: hits whose depth below the panel's front face lies in
      [b, b + 1) * panel_depth / doi_bins; depths outside the panel go to the
      first or last bin.
    """
    hpc = np.zeros(n_crystals, np.int64)
    spc = np.zeros(n_crystals, np.int64)
    spec = np.zeros(700, np.int64)
    doi = np.zeros(doi_bins, np.int64)
    for g, d in zip(hits["gid"].tolist(), hits["depth"].tolist()):
        hpc[g] += 1
        b = int(np.floor(d / panel_depth * doi_bins))
        doi[min(max(b, 0), doi_bins - 1)] += 1
    for g, e, w, lost in zip(singles["gid"].tolist(), singles["energy"].tolist(),
                             singles["in_window"].tolist(), singles["lost"].tolist()):
        if lost:
            continue
        if w:
            spc[g] += 1
        if 0.0 <= e < 700.0:
            spec[int(np.floor(e))] += 1
    return {"hits_per_crystal": hpc, "singles_per_crystal": spc, "energy_spectrum": spec, "doi": doi}


def num_threads() -> int:
    return lib().or_num_threads()


def set_threads(n: int) -> None:
    """Host threads of the following calls (results do not depend on it)."""
    lib().or_set_threads(int(n))
