"""Python binding of ``libgpet.so`` (C ABI in ``include/gpet.h``).

Argument marshalling only: scene descriptions are packed into the library's
structs, device buffers are torch tensors on the context's device, and every
step of the simulation runs in the library's HIP kernels.  There is no CPU
fallback: if the library is not built, or no GPU is present, construction of a
:class:`Context` raises.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpet.so")

MAX_EL, MAX_MAT, MAX_LAYERS, MAX_PANELS = 8, 8, 4, 64
NODES = 511

OK, ERR_ARG, ERR_GEOMETRY, ERR_STATE, ERR_CAPACITY, ERR_HIP, ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
PLACE_REPEAT, PLACE_EXPLICIT = 0, 1
SRC_POINT, SRC_CYLINDERS, SRC_BEAM = 0, 1, 2
V_STEP, V_ENTER_PANEL, V_EXIT, V_ESCAPE, V_DEAD, V_ENTER_PHANTOM, V_EMIT = range(7)

STAT_NAMES = ("events", "panel_entries", "steps", "real", "kahn_trials", "searches", "blocks", "capped",
              "scatters", "wave_trips", "panel_tests", "pruned_searches", "nonfinite")


class GpetError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gpet error {code}: {msg}")
        self.code = code


class Material(C.Structure):
    _fields_ = [("density_g_cm3", C.c_double), ("n_elements", C.c_int32), ("processes", C.c_uint32),
                ("Z", C.c_int32 * MAX_EL), ("A", C.c_double * MAX_EL), ("mass_fraction", C.c_double * MAX_EL)]


class Physics(C.Structure):
    _fields_ = [("k_pe", C.c_double), ("k_rayleigh", C.c_double), ("e_cut_kev", C.c_double)]


class Layer(C.Structure):
    _fields_ = [("depth0_mm", C.c_double), ("thickness_mm", C.c_double), ("n_t", C.c_int32), ("n_a", C.c_int32),
                ("cryst_t_mm", C.c_double), ("cryst_a_mm", C.c_double), ("pitch_t_mm", C.c_double),
                ("pitch_a_mm", C.c_double), ("offset_t_mm", C.c_double), ("offset_a_mm", C.c_double),
                ("crystal_material", C.c_int32), ("interval_material", C.c_int32)]


class Scanner(C.Structure):
    _fields_ = [("placement", C.c_int32), ("n_panels", C.c_int32), ("radius_mm", C.c_double),
                ("phi0_rad", C.c_double), ("z0_mm", C.c_double), ("poses", C.POINTER(C.c_double)),
                ("depth_mm", C.c_double), ("width_mm", C.c_double), ("length_mm", C.c_double),
                ("mod_n_t", C.c_int32), ("mod_n_a", C.c_int32), ("mod_t_mm", C.c_double),
                ("mod_a_mm", C.c_double), ("gap_t_mm", C.c_double), ("gap_a_mm", C.c_double),
                ("fill_material", C.c_int32), ("n_layers", C.c_int32), ("layers", Layer * MAX_LAYERS)]


class GeometryInfo(C.Structure):
    _fields_ = [("n_crystals", C.c_int32), ("crystals_per_panel", C.c_int32),
                ("crystals_per_module", C.c_int32), ("layer_base", C.c_int32 * MAX_LAYERS)]


class Phantom(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("voxel_mm", C.c_double * 3),
                ("origin_mm", C.c_double * 3), ("material", C.POINTER(C.c_uint8)),
                ("density", C.POINTER(C.c_float))]


class Source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pos_mm", C.c_double * 3), ("dir", C.c_double * 3),
                ("n_rods", C.c_int32), ("rods", C.POINTER(C.c_double)), ("duration_ps", C.c_uint64),
                ("acolinearity_fwhm_deg", C.c_double), ("positron_range_fwhm_mm", C.c_double)]


class Hits(C.Structure):
    _fields_ = [("event", C.c_void_p), ("gid", C.c_void_p), ("edep_kev", C.c_void_p), ("depth_mm", C.c_void_p),
                ("time_ps", C.c_void_p), ("aux", C.c_void_p), ("instance", C.c_void_p), ("capacity", C.c_uint64),
                ("count", C.c_uint64)]


class Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in STAT_NAMES]


class Digitizer(C.Structure):
    _fields_ = [("fwhm_511", C.c_double), ("e_lo_kev", C.c_double), ("e_hi_kev", C.c_double),
                ("window_ps", C.c_uint64), ("seed", C.c_uint64), ("instance", C.c_uint32),
                ("first_event", C.c_uint64), ("n_events", C.c_uint64), ("readout", C.c_uint32),
                ("n_sweep", C.c_uint32), ("sweep_lo_kev", C.c_void_p), ("sweep_hi_kev", C.c_void_p),
                ("sweep_coincidences", C.c_void_p), ("time_fwhm_ps", C.c_double), ("doi_fwhm_mm", C.c_double),
                ("dead_time_ps", C.c_uint64), ("dead_time_mode", C.c_uint32), ("dead_time_level", C.c_uint32),
                ("light_sharing", C.c_double)]


READOUT = {"crystal": 0, "module": 1, "panel": 2}
DEAD_TIME = {"none": 0, "paralyzable": 1, "nonparalyzable": 2}


def _readout_code(readout) -> int:
    return READOUT[readout] if isinstance(readout, str) else int(readout)


def _digitizer(fwhm_511, e_lo, e_hi, window_ps, seed, instance, first, n_events, readout, sweep, response=None):
    """The parameter struct plus the host arrays its sweep pointers refer to
    (kept alive by the caller for the duration of the call).  response: dict of
    the optional detector response -- time_fwhm_ps, doi_fwhm_mm, dead_time_ps,
    dead_time_mode ("paralyzable" / "nonparalyzable"), dead_time_level
    ("crystal" / "module" / "panel"), light_sharing (probability of reading
    a neighbour crystal)."""
    dg = Digitizer(fwhm_511, e_lo, e_hi, window_ps, seed, instance, first, n_events, _readout_code(readout))
    r = response or {}
    dg.time_fwhm_ps = float(r.get("time_fwhm_ps", 0.0))
    dg.doi_fwhm_mm = float(r.get("doi_fwhm_mm", 0.0))
    dg.dead_time_ps = int(r.get("dead_time_ps", 0))
    mode = r.get("dead_time_mode", "none")
    dg.dead_time_mode = DEAD_TIME[mode] if isinstance(mode, str) else int(mode)
    dg.dead_time_level = _readout_code(r.get("dead_time_level", "module"))
    dg.light_sharing = float(r.get("light_sharing", 0.0))
    keep = None
    if sweep:
        lo = np.ascontiguousarray([w[0] for w in sweep], np.float64)
        hi = np.ascontiguousarray([w[1] for w in sweep], np.float64)
        keep = (lo, hi)
        dg.n_sweep = len(sweep)
        dg.sweep_lo_kev = lo.ctypes.data
        dg.sweep_hi_kev = hi.ctypes.data
    return dg, keep


class Singles(C.Structure):
    _fields_ = [("event", C.c_void_p), ("gid", C.c_void_p), ("edep_kev", C.c_void_p), ("energy_kev", C.c_void_p),
                ("depth_mm", C.c_void_p), ("time_ps", C.c_void_p), ("in_window", C.c_void_p),
                ("instance", C.c_void_p), ("capacity", C.c_uint64), ("count", C.c_uint64),
                ("windowed", C.c_uint64)]


class Coincidences(C.Structure):
    _fields_ = [("first", C.c_void_p), ("second", C.c_void_p), ("capacity", C.c_uint64), ("count", C.c_uint64)]


class Tallies(C.Structure):
    _fields_ = [("hits_per_crystal", C.c_void_p), ("singles_per_crystal", C.c_void_p),
                ("energy_spectrum", C.c_void_p), ("doi", C.c_void_p), ("doi_bins", C.c_int32)]


class TrainParams(C.Structure):
    _fields_ = [("batch", C.c_uint32), ("steps", C.c_uint32), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("seed", C.c_uint64)]


class SurrogateSpec(C.Structure):
    _fields_ = [("half_width", C.c_int32), ("n_ebins", C.c_int32), ("e_min_kev", C.c_double),
                ("ebin_kev", C.c_double), ("photopeak_tol_kev", C.c_double), ("max_slope", C.c_double),
                ("front_tol_mm", C.c_double), ("class_half_width", C.c_int32)]


class Pairs(C.Structure):
    _fields_ = [("x", C.c_void_p), ("label", C.c_void_p), ("event", C.c_void_p), ("flags", C.c_void_p),
                ("capacity", C.c_uint64), ("count", C.c_uint64)]


class SurrogateStats(C.Structure):
    _fields_ = [("entries", C.c_uint64), ("none", C.c_uint64), ("ms_transport", C.c_float),
                ("ms_network", C.c_float)]


class Instance(C.Structure):
    _fields_ = [("scanner", C.POINTER(Scanner)), ("source", C.POINTER(Source)), ("first_event", C.c_uint64),
                ("n_events", C.c_uint64), ("instance", C.c_uint32)]


EXPORTS = ("gpet_ctx_create", "gpet_ctx_destroy", "gpet_last_error", "gpet_ctx_set_stream", "gpet_materials_set",
           "gpet_geometry_create", "gpet_phantom_set", "gpet_source_set", "gpet_transport", "gpet_digitize",
           "gpet_philox", "gpet_tables_get", "gpet_locate", "gpet_ray_locate", "gpet_sample_compton",
           "gpet_sample_rayleigh", "gpet_trace", "gpet_ctx_enable_timing", "gpet_timings",
           "gpet_ctx_set_launch", "gpet_batch_create", "gpet_batch_destroy", "gpet_batch_info",
           "gpet_batch_set_launch", "gpet_batch_transport", "gpet_batch_digitize", "gpet_batch_autotune",
           "gpet_mlp_create", "gpet_mlp_destroy", "gpet_mlp_set_weights", "gpet_mlp_get_weights",
           "gpet_mlp_forward", "gpet_mlp_loss_grad", "gpet_mlp_train", "gpet_surrogate_pairs",
           "gpet_surrogate_transport", "gpet_batch_graph_capture", "gpet_batch_graph_launch",
           "gpet_batch_read_counts", "gpet_digitize_noalloc", "gpet_mlp_create_factored", "gpet_mlp_get_state",
           "gpet_mlp_set_state")

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgpet.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2603_07327_amd.build`")
    L = C.CDLL(path)
    P, vp = C.POINTER, C.c_void_p
    L.gpet_ctx_create.argtypes = [C.c_int, vp, P(vp)]
    L.gpet_ctx_destroy.argtypes = [vp]
    L.gpet_ctx_destroy.restype = None
    L.gpet_last_error.argtypes = [vp]
    L.gpet_last_error.restype = C.c_char_p
    L.gpet_ctx_set_stream.argtypes = [vp, vp]
    L.gpet_materials_set.argtypes = [vp, C.c_int32, P(Material), P(Physics)]
    L.gpet_geometry_create.argtypes = [vp, P(Scanner), P(GeometryInfo)]
    L.gpet_phantom_set.argtypes = [vp, P(Phantom)]
    L.gpet_source_set.argtypes = [vp, P(Source)]
    L.gpet_transport.argtypes = [vp, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32, P(Hits), P(Stats)]
    L.gpet_digitize.argtypes = [vp, P(Hits), P(Digitizer), P(Singles), P(Coincidences), P(Tallies)]
    L.gpet_digitize_noalloc.argtypes = [vp, P(Hits), P(Digitizer), P(Singles), P(Coincidences), P(Tallies)]
    L.gpet_philox.argtypes = [vp, C.c_uint64, vp, C.c_uint32, vp]
    L.gpet_tables_get.argtypes = [vp, vp, vp]
    L.gpet_locate.argtypes = [vp, C.c_uint32, vp, vp]
    L.gpet_ray_locate.argtypes = [vp, C.c_uint32, vp, vp, C.c_int32, C.c_float, vp, vp]
    L.gpet_sample_compton.argtypes = [vp, C.c_float, C.c_uint32, C.c_uint64, vp, vp, vp]
    L.gpet_sample_rayleigh.argtypes = [vp, C.c_uint32, C.c_uint64, vp]
    L.gpet_trace.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, C.c_int32, vp, vp, vp]
    L.gpet_ctx_enable_timing.argtypes = [vp, C.c_int]
    L.gpet_timings.argtypes = [vp, P(C.c_float)]
    L.gpet_ctx_set_launch.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
    L.gpet_batch_create.argtypes = [vp, C.c_int32, P(Instance), P(vp)]
    L.gpet_batch_destroy.argtypes = [vp]
    L.gpet_batch_destroy.restype = None
    L.gpet_batch_info.argtypes = [vp, C.c_int32, P(GeometryInfo)]
    L.gpet_batch_set_launch.argtypes = [vp, C.c_int32, C.c_int32, C.c_uint32]
    L.gpet_batch_transport.argtypes = [vp, C.c_uint64, P(Hits), P(Stats)]
    L.gpet_batch_digitize.argtypes = [vp, P(Hits), P(Digitizer), P(Singles), P(Coincidences), vp]
    L.gpet_batch_autotune.argtypes = [vp, C.c_uint64, P(Hits), C.c_char_p, C.c_size_t]
    L.gpet_mlp_create.argtypes = [vp, C.c_int32, vp, vp, P(vp)]
    L.gpet_mlp_create_factored.argtypes = [vp, C.c_int32, vp, C.c_int32, C.c_int32, vp, P(vp)]
    L.gpet_mlp_destroy.argtypes = [vp]
    L.gpet_mlp_destroy.restype = None
    L.gpet_mlp_set_weights.argtypes = [vp, vp]
    L.gpet_mlp_get_weights.argtypes = [vp, vp]
    L.gpet_mlp_get_state.argtypes = [vp, vp, vp, vp, P(C.c_uint64)]
    L.gpet_mlp_set_state.argtypes = [vp, vp, vp, vp, C.c_uint64]
    L.gpet_mlp_forward.argtypes = [vp, C.c_uint32, vp, vp]
    L.gpet_mlp_loss_grad.argtypes = [vp, C.c_uint32, vp, vp, P(C.c_double), vp]
    L.gpet_mlp_train.argtypes = [vp, C.c_uint64, vp, vp, P(TrainParams), vp]
    L.gpet_batch_graph_capture.argtypes = [vp, C.c_uint64, P(Hits)]
    L.gpet_batch_graph_launch.argtypes = [vp]
    L.gpet_batch_read_counts.argtypes = [vp, P(Hits), P(Stats)]
    L.gpet_surrogate_pairs.argtypes = [vp, P(SurrogateSpec), C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32,
                                       P(Hits), P(Pairs), P(Stats)]
    L.gpet_surrogate_transport.argtypes = [vp, vp, P(SurrogateSpec), C.c_uint64, C.c_uint64, C.c_uint64,
                                           C.c_uint32, P(Hits), P(Stats), P(SurrogateStats)]
    for name in EXPORTS:
        if name not in ("gpet_ctx_destroy", "gpet_last_error", "gpet_batch_destroy", "gpet_mlp_destroy"):
            getattr(L, name).restype = C.c_int32
    _lib = L
    return L


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


@dataclass
class HitList:
    event: "torch.Tensor"
    gid: "torch.Tensor"
    edep_kev: "torch.Tensor"
    depth_mm: "torch.Tensor"
    time_ps: "torch.Tensor"
    aux: "torch.Tensor"
    count: int
    first_event: int
    n_events: int
    instance: "torch.Tensor | None" = None

    def view(self):
        n = self.count
        return HitList(self.event[:n], self.gid[:n], self.edep_kev[:n], self.depth_mm[:n], self.time_ps[:n],
                       self.aux[:n], n, self.first_event, self.n_events,
                       None if self.instance is None else self.instance[:n])

    def numpy(self):
        v = self.view()
        keys = ("event", "gid", "edep_kev", "depth_mm", "time_ps", "aux") + (("instance",) if v.instance is not None
                                                                            else ())
        return {k: getattr(v, k).cpu().numpy() for k in keys}

    def struct(self):
        return Hits(self.event.data_ptr(), self.gid.data_ptr(), self.edep_kev.data_ptr(), self.depth_mm.data_ptr(),
                    self.time_ps.data_ptr(), self.aux.data_ptr(),
                    self.instance.data_ptr() if self.instance is not None else None, self.event.numel(), self.count)


@dataclass
class SingleList:
    event: "torch.Tensor"
    gid: "torch.Tensor"
    edep_kev: "torch.Tensor"
    energy_kev: "torch.Tensor"
    depth_mm: "torch.Tensor"
    time_ps: "torch.Tensor"
    in_window: "torch.Tensor"
    count: int
    instance: "torch.Tensor | None" = None
    windowed: int = 0  # singles inside the main energy window

    def numpy(self):
        n = self.count
        keys = ("event", "gid", "edep_kev", "energy_kev", "depth_mm", "time_ps", "in_window")
        keys += ("instance",) if self.instance is not None else ()
        return {k: getattr(self, k)[:n].cpu().numpy() for k in keys}

    def struct(self):
        return Singles(*(getattr(self, k).data_ptr() for k in
                         ("event", "gid", "edep_kev", "energy_kev", "depth_mm", "time_ps", "in_window")),
                       self.instance.data_ptr() if self.instance is not None else None, self.event.numel(), 0)


def pack_materials(mats, ph):
    arr = (Material * len(mats))()
    for i, m in enumerate(mats):
        q = arr[i]
        q.density_g_cm3 = m["density"]
        q.n_elements = len(m["Z"])
        q.processes = m["mask"]
        for j, (z, a, w) in enumerate(zip(m["Z"], m["A"], m["w"])):
            q.Z[j], q.A[j], q.mass_fraction[j] = z, a, w
    return arr, Physics(ph["k_pe"], ph["k_r"], ph["e_cut"])


def pack_scanner(g: dict):
    """Scanner struct of a scanner description, and the array its poses point into."""
    s = Scanner()
    s.placement = PLACE_EXPLICIT if g["mode"] == "explicit" else PLACE_REPEAT
    s.n_panels = g["n_panels"]
    s.radius_mm, s.phi0_rad, s.z0_mm = g["radius"], g["phi0"], g["z0"]
    keep = None
    if g["poses"] is not None:
        keep = np.ascontiguousarray(g["poses"], np.float64)
        s.poses = keep.ctypes.data_as(C.POINTER(C.c_double))
    s.depth_mm, s.width_mm, s.length_mm = g["depth"], g["width"], g["length"]
    s.mod_n_t, s.mod_n_a = g["mod_n_t"], g["mod_n_a"]
    s.mod_t_mm, s.mod_a_mm, s.gap_t_mm, s.gap_a_mm = g["mod_t"], g["mod_a"], g["gap_t"], g["gap_a"]
    s.fill_material = g["mat_fill"]
    s.n_layers = len(g["layers"])
    for i, y in enumerate(g["layers"]):
        L = s.layers[i]
        L.depth0_mm, L.thickness_mm = y["depth0"], y["thick"]
        L.n_t, L.n_a = y["n_t"], y["n_a"]
        L.cryst_t_mm, L.cryst_a_mm = y["cryst_t"], y["cryst_a"]
        L.pitch_t_mm, L.pitch_a_mm = y["pitch_t"], y["pitch_a"]
        L.offset_t_mm, L.offset_a_mm = y["off_t"], y["off_a"]
        L.crystal_material, L.interval_material = y["mat_crystal"], y["mat_interval"]
    return s, keep


def pack_source(src: dict):
    """Source struct of a source description, and the array its rods point into."""
    s = Source()
    s.kind = src["kind"]
    for k in range(3):
        s.pos_mm[k] = src["pos"][k]
        s.dir[k] = src["dir"][k]
    keep = None
    if src["rods"] is not None:
        keep = np.ascontiguousarray(src["rods"], np.float64)
        s.n_rods = len(keep)
        s.rods = keep.ctypes.data_as(C.POINTER(C.c_double))
    s.duration_ps = int(src["duration_ps"])
    s.acolinearity_fwhm_deg = float(src.get("acolinearity_fwhm_deg", 0.0))
    s.positron_range_fwhm_mm = float(src.get("positron_range_fwhm_mm", 0.0))
    return s, keep


class Context:
    """One library context on a GPU, ordering work on torch's current stream."""

    def __init__(self, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the gpet library runs only on the device")
        self.torch = torch
        self.L = load_library()
        self.dev = torch.device("cuda", device)
        self.stream = torch.cuda.current_stream(self.dev)
        h = C.c_void_p()
        self._check(self.L.gpet_ctx_create(device, C.c_void_p(self.stream.cuda_stream), C.byref(h)), "create")
        self.h = h
        self.info = None
        self.scene = None
        self._batches = weakref.WeakSet()  # batches and networks made from this context

    def close(self):
        """Destroys the context (and first every batch and network made from it)."""
        for b in list(getattr(self, "_batches", ())):
            b.close()
        if getattr(self, "h", None):
            self.L.gpet_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what=""):
        if rc != OK:
            msg = self.L.gpet_last_error(self.h).decode() if getattr(self, "h", None) else what
            raise GpetError(rc, msg or what)

    def _empty(self, n, dtype):
        return self.torch.empty(max(int(n), 1), dtype=dtype, device=self.dev)

    def set_launch(self, blocks_per_cu=0, search_batch=16, schedule=0):
        self._check(self.L.gpet_ctx_set_launch(self.h, blocks_per_cu, search_batch, schedule))

    def enable_timing(self, on=True):
        self._check(self.L.gpet_ctx_enable_timing(self.h, 1 if on else 0))

    def timings(self):
        """(transport kernel ms, digitizer ms) of the last calls."""
        out = (C.c_float * 2)()
        self._check(self.L.gpet_timings(self.h, out))
        return float(out[0]), float(out[1])

    # ------------------------------------------------------------------ scene
    def set_scene(self, sc: dict):
        """Materials, scanner, phantom and source from a scene description."""
        self.set_materials(sc["materials"], sc["physics"])
        self.set_scanner(sc["scanner"])
        self.set_phantom(sc.get("phantom"))
        self.set_source(sc["source"])
        self.scene = sc
        return self.info

    def set_materials(self, mats, physics):
        arr, phys = pack_materials(mats, physics)
        self._check(self.L.gpet_materials_set(self.h, len(mats), arr, C.byref(phys)))
        self.n_mat = len(mats)

    def set_scanner(self, g: dict):
        s, keep = pack_scanner(g)
        info = GeometryInfo()
        self._check(self.L.gpet_geometry_create(self.h, C.byref(s), C.byref(info)))
        del keep
        self.info = info
        return info

    def set_phantom(self, p):
        if p is None:
            self._check(self.L.gpet_phantom_set(self.h, None))
            return
        ph = Phantom()
        ph.nx, ph.ny, ph.nz = p["shape"]
        for k in range(3):
            ph.voxel_mm[k] = p["voxel"][k]
            ph.origin_mm[k] = p["origin"][k]
        m8 = np.ascontiguousarray(p["mat"], np.uint8)
        d32 = np.ascontiguousarray(p["dens"], np.float32)
        ph.material = m8.ctypes.data_as(C.POINTER(C.c_uint8))
        ph.density = d32.ctypes.data_as(C.POINTER(C.c_float))
        self._check(self.L.gpet_phantom_set(self.h, C.byref(ph)))

    def set_source(self, src: dict):
        s, keep = pack_source(src)
        self._check(self.L.gpet_source_set(self.h, C.byref(s)))
        del keep

    # -------------------------------------------------------------- transport
    def alloc_hits(self, capacity: int, first_event=0, n_events=0, instance=False) -> HitList:
        t = self.torch
        return HitList(self._empty(capacity, t.int32), self._empty(capacity, t.int32),
                       self._empty(capacity, t.float32), self._empty(capacity, t.float32),
                       self._empty(capacity, t.int64), self._empty(capacity, t.int32), 0, first_event, n_events,
                       self._empty(capacity, t.int32) if instance else None)

    def transport_into(self, hits: HitList, n_events, seed=0, first=0, instance=0):
        """Transport into preallocated hits; returns (status, stats dict)."""
        h = hits.struct()
        h.count = 0
        st = Stats()
        rc = self.L.gpet_transport(self.h, first, n_events, seed, instance, C.byref(h), C.byref(st))
        hits.count = int(h.count)
        hits.first_event, hits.n_events = first, n_events
        if rc not in (OK, ERR_CAPACITY):
            self._check(rc)
        return rc, {n: int(getattr(st, n)) for n in STAT_NAMES}

    def transport(self, n_events, seed=0, first=0, instance=0, capacity=None):
        cap = capacity or max(1024, int(3.5 * n_events))
        hits = self.alloc_hits(cap)
        rc, stats = self.transport_into(hits, n_events, seed, first, instance)
        if rc == ERR_CAPACITY:
            hits = self.alloc_hits(hits.count)
            rc, stats = self.transport_into(hits, n_events, seed, first, instance)
            self._check(rc)
        return hits, stats

    # -------------------------------------------------------------- digitizer
    def alloc_singles(self, capacity, instance=False) -> SingleList:
        t = self.torch
        return SingleList(self._empty(capacity, t.int32), self._empty(capacity, t.int32),
                          self._empty(capacity, t.float32), self._empty(capacity, t.float32),
                          self._empty(capacity, t.float32), self._empty(capacity, t.int64),
                          self._empty(capacity, t.int32), 0,
                          self._empty(capacity, t.int32) if instance else None)

    def digitize_into(self, hits: HitList, singles: SingleList, coinc, seed=0, fwhm_511=0.16, e_lo=350.0,
                      e_hi=650.0, window_ps=3000, instance=0, tallies=None, readout="crystal", sweep=None,
                      response=None, noalloc=False):
        """Digitize into preallocated outputs; returns (status, coincidences) or,
        with sweep = [(e_lo, e_hi), ...], (status, coincidences, counts of the
        sweep windows).  readout: "crystal", "module" or "panel"; response: the
        optional time / DOI blur and dead time (see _digitizer); noalloc: call
        gpet_digitize_noalloc (the library's static scratch) instead of
        gpet_digitize."""
        h = hits.struct()
        dg, keep = _digitizer(fwhm_511, e_lo, e_hi, window_ps, seed, instance, hits.first_event,
                              max(1, hits.n_events), readout, sweep, response)
        counts = np.zeros(len(sweep) if sweep else 0, np.uint64)
        if sweep:
            dg.sweep_coincidences = counts.ctypes.data
        s = singles.struct()
        cc = Coincidences(coinc[0].data_ptr(), coinc[1].data_ptr(), coinc[0].numel(), 0)
        tl = None
        if tallies is not None:
            tl = Tallies(*(tallies[k].data_ptr() if tallies.get(k) is not None else None for k in
                           ("hits_per_crystal", "singles_per_crystal", "energy_spectrum", "doi")),
                         int(tallies["doi"].numel()) if tallies.get("doi") is not None else 0)
        fn = self.L.gpet_digitize_noalloc if noalloc else self.L.gpet_digitize
        rc = fn(self.h, C.byref(h), C.byref(dg), C.byref(s), C.byref(cc), C.byref(tl) if tl is not None else None)
        del keep
        singles.count = int(s.count)
        singles.windowed = int(s.windowed)
        if rc not in (OK, ERR_CAPACITY):
            self._check(rc)
        if sweep is not None:
            return rc, int(cc.count), counts.astype(np.int64)
        return rc, int(cc.count)

    def alloc_tallies(self, doi_bins=200):
        t = self.torch
        n = self.info.n_crystals
        z = lambda k: t.zeros(k, dtype=t.int32, device=self.dev)  # noqa: E731
        return {"hits_per_crystal": z(n), "singles_per_crystal": z(n), "energy_spectrum": z(700),
                "doi": z(doi_bins)}

    def digitize_noalloc(self, hits: HitList, seed=0, tallies=None, **kw):
        """digitize() through gpet_digitize_noalloc (the outputs are still
        allocated here, by torch; the library allocates nothing)."""
        return self.digitize(hits, seed=seed, tallies=tallies, noalloc=True, **kw)

    def digitize(self, hits: HitList, seed=0, tallies=None, **kw):
        """(singles, (first, second)) and, with sweep=..., the sweep counts."""
        t = self.torch
        cap = max(1024, hits.count)
        singles = self.alloc_singles(cap)
        coinc = (self._empty(cap // 2 + 16, t.int32), self._empty(cap // 2 + 16, t.int32))
        out = self.digitize_into(hits, singles, coinc, seed=seed, tallies=tallies, **kw)
        self._check(out[0])
        nc = out[1]
        if len(out) == 3:
            return singles, (coinc[0][:nc], coinc[1][:nc]), out[2]
        return singles, (coinc[0][:nc], coinc[1][:nc])

    # ------------------------------------------------------------ check surface
    def philox(self, seed: int, ctr: np.ndarray) -> np.ndarray:
        t = self.torch
        c = t.from_numpy(np.ascontiguousarray(ctr, np.uint32).view(np.int32).reshape(-1)).to(self.dev)
        out = t.empty_like(c)
        self._check(self.L.gpet_philox(self.h, seed, _ptr(c), c.numel() // 4, _ptr(out)))
        return out.cpu().numpy().view(np.uint32).reshape(-1, 4)

    def tables(self):
        n = len(self.scene["materials"]) if self.scene else MAX_MAT
        mu = np.zeros((n, 4, NODES), np.float32)
        maj = np.zeros(NODES, np.float32)
        self._check(self.L.gpet_tables_get(self.h, mu.ctypes.data_as(C.c_void_p), maj.ctypes.data_as(C.c_void_p)))
        return mu, maj

    def locate(self, xyz: np.ndarray) -> np.ndarray:
        t = self.torch
        x = t.from_numpy(np.ascontiguousarray(xyz, np.float32).reshape(-1)).to(self.dev)
        n = x.numel() // 3
        ids = self._empty(6 * n, t.int32)
        self._check(self.L.gpet_locate(self.h, n, _ptr(x), _ptr(ids)))
        return ids[: 6 * n].cpu().numpy().reshape(n, 6)

    def ray_locate(self, o, d, n_samp, step):
        t = self.torch
        ot = t.from_numpy(np.ascontiguousarray(o, np.float32).reshape(-1)).to(self.dev)
        dt = t.from_numpy(np.ascontiguousarray(d, np.float32).reshape(-1)).to(self.dev)
        n = ot.numel() // 3
        tin = self._empty(n, t.float32)
        ids = self._empty(6 * n * n_samp, t.int32)
        self._check(self.L.gpet_ray_locate(self.h, n, _ptr(ot), _ptr(dt), n_samp, step, _ptr(tin), _ptr(ids)))
        return tin[:n].cpu().numpy(), ids[: 6 * n * n_samp].cpu().numpy().reshape(n, n_samp, 6)

    def sample_compton(self, e_kev, n, seed=0):
        t = self.torch
        c, e, tr = self._empty(n, t.float32), self._empty(n, t.float32), self._empty(n, t.int32)
        self._check(self.L.gpet_sample_compton(self.h, e_kev, n, seed, _ptr(c), _ptr(e), _ptr(tr)))
        return c[:n].cpu().numpy(), e[:n].cpu().numpy(), tr[:n].cpu().numpy()

    def sample_rayleigh(self, n, seed=0):
        c = self._empty(n, self.torch.float32)
        self._check(self.L.gpet_sample_rayleigh(self.h, n, seed, _ptr(c)))
        return c[:n].cpu().numpy()

    def trace(self, n_events, seed=0, first=0, instance=0, max_vertices=256):
        """Traced histories as a numpy structured array in photon order."""
        t = self.torch
        np_ = 2 * n_events
        vi = self._empty(np_ * max_vertices * 11, t.int32)
        vf = self._empty(np_ * max_vertices * 8, t.float32)
        cnt = self._empty(np_, t.int32)
        self._check(self.L.gpet_trace(self.h, first, n_events, seed, instance, max_vertices, _ptr(vi), _ptr(vf),
                                      _ptr(cnt)))
        cnt = cnt[:np_].cpu().numpy()
        if cnt.max(initial=0) > max_vertices:
            return self.trace(n_events, seed, first, instance, int(cnt.max()))
        vi = vi[: np_ * max_vertices * 11].cpu().numpy().reshape(np_, max_vertices, 11)
        vf = vf[: np_ * max_vertices * 8].cpu().numpy().reshape(np_, max_vertices, 8)
        keep = np.arange(max_vertices)[None, :] < cnt[:, None]
        ints, flts = vi[keep], vf[keep]
        names_i = ("event", "photon", "kind", "region", "panel", "gid", "mat", "accept", "process", "trials",
                   "block")
        names_f = ("x", "y", "z", "e", "edep", "dx", "dy", "dz")
        out = np.zeros(len(ints), dtype=[(n, np.int32) for n in names_i] + [(n, np.float32) for n in names_f])
        for k, n in enumerate(names_i):
            out[n] = ints[:, k]
        for k, n in enumerate(names_f):
            out[n] = flts[:, k]
        return out

    # ------------------------------------------------------------- surrogate
    @staticmethod
    def spec_struct(spec=None):
        """SurrogateSpec from a dict or object with the oracle's Spec fields."""
        d = {"half_width": 2, "n_ebins": 36, "e_min_kev": 224.0, "ebin_kev": 8.0, "photopeak_tol_kev": 1.0,
             "max_slope": 0.25, "front_tol_mm": 1e-3, "class_half_width": 0}
        if spec is not None:
            d.update(spec if isinstance(spec, dict) else {k: getattr(spec, k) for k in d})
        return SurrogateSpec(**d)

    def alloc_pairs(self, capacity):
        t = self.torch
        return {"x": self._empty(6 * capacity, t.float32), "label": self._empty(capacity, t.int32),
                "event": self._empty(capacity, t.int32), "flags": self._empty(capacity, t.int32),
                "capacity": int(capacity), "count": 0}

    def surrogate_pairs_into(self, hits: HitList, pairs: dict, n_events, seed=0, first=0, instance=0, spec=None):
        h = hits.struct()
        h.count = 0
        pr = Pairs(pairs["x"].data_ptr(), pairs["label"].data_ptr(), pairs["event"].data_ptr(),
                   pairs["flags"].data_ptr(), pairs["capacity"], 0)
        st = Stats()
        rc = self.L.gpet_surrogate_pairs(self.h, C.byref(self.spec_struct(spec)), first, n_events, seed, instance,
                                         C.byref(h), C.byref(pr), C.byref(st))
        hits.count = int(h.count)
        hits.first_event, hits.n_events = first, n_events
        pairs["count"] = int(pr.count)
        if rc not in (OK, ERR_CAPACITY):
            self._check(rc)
        return rc, {n: int(getattr(st, n)) for n in STAT_NAMES}

    def surrogate_pairs(self, n_events, seed=0, first=0, instance=0, spec=None):
        """(hits, pairs as numpy dict x/label/event/flags, stats)."""
        hits = self.alloc_hits(max(1024, int(3.5 * n_events)))
        pairs = self.alloc_pairs(max(1024, 2 * n_events))
        rc, st = self.surrogate_pairs_into(hits, pairs, n_events, seed, first, instance, spec)
        self._check(rc)
        n = pairs["count"]
        out = {"x": pairs["x"][: 6 * n].cpu().numpy().reshape(n, 6), "label": pairs["label"][:n].cpu().numpy(),
               "event": pairs["event"][:n].cpu().numpy().view(np.uint32),
               "flags": pairs["flags"][:n].cpu().numpy().view(np.uint32)}
        return hits, out, st

    def surrogate_transport_into(self, mlp, hits: HitList, n_events, seed=0, first=0, instance=0, spec=None):
        h = hits.struct()
        h.count = 0
        st, ss = Stats(), SurrogateStats()
        rc = self.L.gpet_surrogate_transport(self.h, mlp.h, C.byref(self.spec_struct(spec)), first, n_events, seed,
                                             instance, C.byref(h), C.byref(st), C.byref(ss))
        hits.count = int(h.count)
        hits.first_event, hits.n_events = first, n_events
        if rc not in (OK, ERR_CAPACITY):
            self._check(rc)
        sst = {"entries": int(ss.entries), "none": int(ss.none), "ms_transport": float(ss.ms_transport),
               "ms_network": float(ss.ms_network)}
        return rc, {n: int(getattr(st, n)) for n in STAT_NAMES}, sst

    def surrogate_transport(self, mlp, n_events, seed=0, first=0, instance=0, spec=None):
        hits = self.alloc_hits(max(1024, int(3.5 * n_events)))
        rc, st, sst = self.surrogate_transport_into(mlp, hits, n_events, seed, first, instance, spec)
        self._check(rc)
        return hits, st, sst


class Batch:
    """A table of instances (scanner, source, event range, RNG instance id)
    transported by one persistent launch and digitized in one pass.  The
    instances share the context's materials and phantom."""

    def __init__(self, ctx: Context, instances):
        """instances: dicts with keys scanner, source, n_events and optionally
        first_event (0) and instance (the RNG id; default: the list index)."""
        self.ctx, self.L = ctx, ctx.L
        self.n = len(instances)
        arr = (Instance * self.n)()
        keep = []
        for i, d in enumerate(instances):
            sc, k1 = pack_scanner(d["scanner"])
            so, k2 = pack_source(d["source"])
            keep += [sc, so, k1, k2]
            arr[i].scanner = C.pointer(sc)
            arr[i].source = C.pointer(so)
            arr[i].first_event = int(d.get("first_event", 0))
            arr[i].n_events = int(d["n_events"])
            arr[i].instance = int(d.get("instance", i))
        h = C.c_void_p()
        ctx._check(self.L.gpet_batch_create(ctx.h, self.n, arr, C.byref(h)), "batch")
        del keep
        self.h = h
        ctx._batches.add(self)
        self.first = np.array([int(d.get("first_event", 0)) for d in instances], np.int64)
        self.n_events = np.array([int(d["n_events"]) for d in instances], np.int64)
        self.ids = np.array([int(d.get("instance", i)) for i, d in enumerate(instances)], np.int64)
        self.infos = []
        for i in range(self.n):
            info = GeometryInfo()
            ctx._check(self.L.gpet_batch_info(self.h, i, C.byref(info)))
            self.infos.append(info)

    def close(self):
        if getattr(self, "h", None):
            self.L.gpet_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch(self, blocks_per_cu=0, search_batch=16, chunk=1024):
        self.ctx._check(self.L.gpet_batch_set_launch(self.h, blocks_per_cu, search_batch, chunk))

    def alloc_hits(self, capacity):
        return self.ctx.alloc_hits(capacity, 0, int(self.n_events.sum()), instance=True)

    def transport_into(self, hits: HitList, seed=0):
        h = hits.struct()
        h.count = 0
        st = Stats()
        rc = self.L.gpet_batch_transport(self.h, seed, C.byref(h), C.byref(st))
        hits.count = int(h.count)
        if rc not in (OK, ERR_CAPACITY):
            self.ctx._check(rc)
        return rc, {n: int(getattr(st, n)) for n in STAT_NAMES}

    def transport(self, seed=0, capacity=None):
        cap = capacity or max(1024, int(3.5 * self.n_events.sum()))
        hits = self.alloc_hits(cap)
        rc, stats = self.transport_into(hits, seed)
        if rc == ERR_CAPACITY:
            hits = self.alloc_hits(hits.count)
            rc, stats = self.transport_into(hits, seed)
            self.ctx._check(rc)
        return hits, stats

    def graph_capture(self, hits: HitList, seed=0):
        """Capture the transport step (counter reset + persistent launch) into a HIP graph."""
        h = hits.struct()
        h.count = 0
        self.ctx._check(self.L.gpet_batch_graph_capture(self.h, seed, C.byref(h)))

    def graph_launch(self):
        """Enqueue the captured step on the context's stream (no synchronization)."""
        self.ctx._check(self.L.gpet_batch_graph_launch(self.h))

    def read_counts(self, hits: HitList):
        """Synchronize; (status, stats) of the last transport, hit count into hits."""
        h = hits.struct()
        st = Stats()
        rc = self.L.gpet_batch_read_counts(self.h, C.byref(h), C.byref(st))
        hits.count = int(h.count)
        if rc not in (OK, ERR_CAPACITY):
            self.ctx._check(rc)
        return rc, {n: int(getattr(st, n)) for n in STAT_NAMES}

    def digitize_into(self, hits: HitList, singles: SingleList, coinc, seed=0, fwhm_511=0.16, e_lo=350.0,
                      e_hi=650.0, window_ps=3000, readout="crystal", sweep=None, response=None):
        """Returns (status, coincidence count, coincidences per instance) and,
        with sweep = [(e_lo, e_hi), ...], the sweep counts [window][instance]."""
        h = hits.struct()
        dg, keep = _digitizer(fwhm_511, e_lo, e_hi, window_ps, seed, 0, 0, 1, readout, sweep, response)
        counts = np.zeros((len(sweep) if sweep else 0, self.n), np.uint64)
        if sweep:
            dg.sweep_coincidences = counts.ctypes.data
        s = singles.struct()
        cc = Coincidences(coinc[0].data_ptr(), coinc[1].data_ptr(), coinc[0].numel(), 0)
        per = np.zeros(self.n, np.uint64)
        rc = self.L.gpet_batch_digitize(self.h, C.byref(h), C.byref(dg), C.byref(s), C.byref(cc),
                                        per.ctypes.data_as(C.c_void_p))
        del keep
        singles.count = int(s.count)
        singles.windowed = int(s.windowed)
        if rc not in (OK, ERR_CAPACITY):
            self.ctx._check(rc)
        if sweep is not None:
            return rc, int(cc.count), per.astype(np.int64), counts.astype(np.int64)
        return rc, int(cc.count), per.astype(np.int64)

    def digitize(self, hits: HitList, seed=0, **kw):
        t = self.ctx.torch
        cap = max(1024, hits.count)
        singles = self.ctx.alloc_singles(cap, instance=True)
        coinc = (self.ctx._empty(cap // 2 + 16, t.int32), self.ctx._empty(cap // 2 + 16, t.int32))
        out = self.digitize_into(hits, singles, coinc, seed=seed, **kw)
        self.ctx._check(out[0])
        nc = out[1]
        if len(out) == 4:
            return singles, (coinc[0][:nc], coinc[1][:nc]), out[2], out[3]
        return singles, (coinc[0][:nc], coinc[1][:nc]), out[2]

    def autotune(self, hits: HitList, seed=0, cache_path=None, key=None):
        """Launch shape and chunk size for this batch: read from the JSON cache
        under `key` if present, else measured by the library's autotuner (and
        stored).  Returns the chosen settings as a dict."""
        import json
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        if key is not None and key in cache:
            r = cache[key]
            self.set_launch(r["blocks_per_cu"], r["search_batch"], r["chunk"])
            return r
        buf = C.create_string_buffer(1 << 14)
        h = hits.struct()
        self.ctx._check(self.L.gpet_batch_autotune(self.h, seed, C.byref(h), buf, len(buf)))
        r = json.loads(buf.value.decode())
        if cache_path and key is not None:
            cache[key] = r
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1)
        return r


def pack_params(params) -> np.ndarray:
    """[(W [out, in], b [out]), ...] -> packed float32 vector (the C ABI layout)."""
    return np.concatenate([np.concatenate([np.asarray(W, np.float32).reshape(-1), np.asarray(b, np.float32)])
                           for W, b in params]).astype(np.float32)


def unpack_params(flat, sizes):
    out, o = [], 0
    for i, j in zip(sizes[:-1], sizes[1:]):
        W = np.asarray(flat[o:o + i * j]).reshape(j, i)
        o += i * j
        out.append((W, np.asarray(flat[o:o + j])))
        o += j
    return out


class Mlp:
    """The surrogate network on the GPU (BF16 matrix cores, FP32 master weights).
    n_first > 0: factored output (energy head of n_first classes, n_groups
    blocks of positions, an offset table; gpet_mlp_create_factored)."""

    def __init__(self, ctx: Context, sizes, weights=None, n_first=0, n_groups=1):
        self.ctx, self.L = ctx, ctx.L
        self.sizes = [int(v) for v in sizes]
        self.n_first, self.n_groups = int(n_first), int(n_groups)
        self.n_params = sum(i * j + j for i, j in zip(self.sizes[:-1], self.sizes[1:]))
        if self.n_first:
            self.n_params += (self.n_first - 1) * ((self.sizes[-1] - self.n_first) // self.n_groups)
        sz = np.array(self.sizes, np.int32)
        w = None if weights is None else np.ascontiguousarray(weights, np.float32)
        if w is not None and w.size != self.n_params:
            raise ValueError("packed weights of the wrong size")
        h = C.c_void_p()
        wp = None if w is None else w.ctypes.data_as(C.c_void_p)
        if self.n_first:
            rc = self.L.gpet_mlp_create_factored(ctx.h, len(sz), sz.ctypes.data_as(C.c_void_p), self.n_first,
                                                 self.n_groups, wp, C.byref(h))
        else:
            rc = self.L.gpet_mlp_create(ctx.h, len(sz), sz.ctypes.data_as(C.c_void_p), wp, C.byref(h))
        ctx._check(rc, "mlp")
        self.h = h
        ctx._batches.add(self)

    def close(self):
        if getattr(self, "h", None):
            self.L.gpet_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, flat):
        w = np.ascontiguousarray(flat, np.float32)
        assert w.size == self.n_params
        self.ctx._check(self.L.gpet_mlp_set_weights(self.h, w.ctypes.data_as(C.c_void_p)))

    def get_weights(self) -> np.ndarray:
        w = np.empty(self.n_params, np.float32)
        self.ctx._check(self.L.gpet_mlp_get_weights(self.h, w.ctypes.data_as(C.c_void_p)))
        return w

    def get_state(self) -> dict:
        """Training checkpoint: weights, Adam moments m and v, step count."""
        w, m, v = (np.empty(self.n_params, np.float32) for _ in range(3))
        step = C.c_uint64()
        self.ctx._check(self.L.gpet_mlp_get_state(self.h, w.ctypes.data_as(C.c_void_p), m.ctypes.data_as(C.c_void_p),
                                                  v.ctypes.data_as(C.c_void_p), C.byref(step)))
        return {"weights": w, "m": m, "v": v, "step": int(step.value)}

    def set_state(self, state: dict):
        w, m, v = (np.ascontiguousarray(state[k], np.float32) for k in ("weights", "m", "v"))
        assert w.size == m.size == v.size == self.n_params
        self.ctx._check(self.L.gpet_mlp_set_state(self.h, w.ctypes.data_as(C.c_void_p), m.ctypes.data_as(C.c_void_p),
                                                  v.ctypes.data_as(C.c_void_p), int(state["step"])))

    def _dev(self, a, dtype):
        t = self.ctx.torch
        if isinstance(a, t.Tensor):
            return a.contiguous()
        return t.from_numpy(np.ascontiguousarray(a, dtype)).to(self.ctx.dev)

    def forward(self, x) -> np.ndarray:
        xd = self._dev(x, np.float32)
        n = xd.shape[0]
        out = self.ctx._empty(n * self.sizes[-1], self.ctx.torch.float32)
        self.ctx._check(self.L.gpet_mlp_forward(self.h, n, _ptr(xd), _ptr(out)))
        return out[: n * self.sizes[-1]].cpu().numpy().reshape(n, self.sizes[-1])

    def loss_grad(self, x, y):
        xd, yd = self._dev(x, np.float32), self._dev(y, np.int32)
        loss = C.c_double()
        g = np.empty(self.n_params, np.float32)
        self.ctx._check(self.L.gpet_mlp_loss_grad(self.h, xd.shape[0], _ptr(xd), _ptr(yd), C.byref(loss),
                                                  g.ctypes.data_as(C.c_void_p)))
        return loss.value, g

    def train(self, x, y, steps, batch=8192, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0):
        """Adam steps on device (or host) pairs; returns the per-step batch losses."""
        xd, yd = self._dev(x, np.float32), self._dev(y, np.int32)
        hp = TrainParams(batch, steps, lr, beta1, beta2, eps, seed)
        losses = np.empty(max(steps, 1), np.float32)
        self.ctx._check(self.L.gpet_mlp_train(self.h, yd.shape[0], _ptr(xd), _ptr(yd), C.byref(hp),
                                              losses.ctypes.data_as(C.c_void_p)))
        return losses[:steps]
