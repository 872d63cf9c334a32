// gpet_api.cpp -- the C ABI: context, validation, host-side tables and
// geometry preparation, and the launches of the transport and digitizer
// kernels.  Declarations and contracts are in include/gpet.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gpet_internal.hpp"

using namespace gpet;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kMec2Kev = 510.99895;
constexpr double kReCm = 2.8179403262e-13;
constexpr double kAvogadro = 6.02214076e23;
constexpr uint32_t kPlainChunk = 256; // events a wave claims at a time in a plain run
constexpr size_t kSceneBytes = (sizeof(DevScene) + 255) / 256 * 256;

gpet_status fail(gpet_ctx *c, gpet_status code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

gpet_status hip_check(gpet_ctx *c, hipError_t e, const char *what) {
  if (e == hipSuccess) return GPET_OK;
  return fail(c, GPET_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T> gpet_status upload(gpet_ctx *c, T *&dst, const T *src, size_t n, const char *what) {
  if (dst) (void)hipFree(dst);
  dst = nullptr;
  if (n == 0) return GPET_OK;
  gpet_status s = hip_check(c, hipMalloc((void **)&dst, n * sizeof(T)), what);
  if (s) return s;
  return hip_check(c, hipMemcpy(dst, src, n * sizeof(T), hipMemcpyHostToDevice), what);
}

// Klein-Nishina total cross-section per electron (barn)
double klein_nishina_barn(double e_kev) {
  const double k = e_kev / kMec2Kev;
  const double lg = std::log1p(2.0 * k);
  const double b = 1.0 + 2.0 * k;
  const double part1 = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / b - lg / k);
  const double part2 = lg / (2.0 * k) - (1.0 + 3.0 * k) / (b * b);
  return 2.0 * kPi * kReCm * kReCm * (part1 + part2) * 1e24;
}

// per-process attenuation per unit density (1/mm per g/cm^3) at e_kev
void attenuation_per_density(const gpet_material &m, const gpet_physics &ph, double e_kev, double out[3]) {
  const double e_mev = e_kev * 1e-3;
  const double sig_e = klein_nishina_barn(e_kev) * 1e-24;
  double pe = 0.0, co = 0.0, ra = 0.0;
  for (int j = 0; j < m.n_elements; ++j) {
    const double atoms_per_g = kAvogadro * m.mass_fraction[j] / m.A[j];
    const double z = (double)m.Z[j];
    const double z2 = z * z;
    co += atoms_per_g * z * sig_e;
    pe += atoms_per_g * ph.k_pe * z2 * z2 / (e_mev * e_mev * e_mev);
    ra += atoms_per_g * ph.k_rayleigh * z2 / (e_mev * e_mev);
  }
  // cm^2/g -> (1/mm) / (g/cm^3)
  out[0] = (m.processes & GPET_PROC_PHOTOELECTRIC) ? pe * 0.1 : 0.0;
  out[1] = (m.processes & GPET_PROC_COMPTON) ? co * 0.1 : 0.0;
  out[2] = (m.processes & GPET_PROC_RAYLEIGH) ? ra * 0.1 : 0.0;
}

int bits_for(uint64_t max_value) {
  int b = 0;
  while (b < 64 && (max_value >> b) != 0) ++b;
  return b;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// A scanner prepared on the host: validated, the DevScene's geometry fields
// filled (table and pose pointers left unset), poses in device layout and the
// materials present in the panel.
struct GeomBuild {
  DevScene S{};
  gpet_geometry_info info{};
  std::vector<float> pose;
  std::vector<bool> used;
};

// Validates g and fills B.  Detector table slots: materials already in
// slot_mat keep their slot, new ones are appended (at most 4 slots).
gpet_status build_geometry(gpet_ctx *c, const gpet_scanner *g, std::vector<int> &slot_mat, GeomBuild &B,
                           const std::string &who) {
  if (!g) return fail(c, GPET_ERR_ARG, who + "null scanner");
  auto bad = [&](const char *w) { return fail(c, GPET_ERR_GEOMETRY, who + w); };
  const double eps = 1e-9;
  if (g->n_panels < 1 || g->n_panels > GPET_MAX_PANELS) return bad("panel count out of range");
  if (!finite_pos(g->depth_mm) || !finite_pos(g->width_mm) || !finite_pos(g->length_mm)) return bad("panel size");
  if (g->mod_n_t < 1 || g->mod_n_a < 1 || !finite_pos(g->mod_t_mm) || !finite_pos(g->mod_a_mm) ||
      !(g->gap_t_mm >= 0) || !(g->gap_a_mm >= 0))
    return bad("module grid");
  const double w_mod = g->mod_n_t * g->mod_t_mm + (g->mod_n_t - 1) * g->gap_t_mm;
  const double l_mod = g->mod_n_a * g->mod_a_mm + (g->mod_n_a - 1) * g->gap_a_mm;
  if (w_mod > g->width_mm + eps || l_mod > g->length_mm + eps) return bad("modules do not fit the panel");
  if (g->fill_material < 0 || g->fill_material >= c->n_mat) return bad("fill material");
  if (g->n_layers < 1 || g->n_layers > GPET_MAX_LAYERS) return bad("layer count");
  double prev_end = 0.0;
  int64_t per_module = 0;
  for (int l = 0; l < g->n_layers; ++l) {
    const gpet_layer &y = g->layers[l];
    if (!(y.depth0_mm >= prev_end - eps) || !finite_pos(y.thickness_mm) ||
        y.depth0_mm + y.thickness_mm > g->depth_mm + eps)
      return bad("layers must lie in the panel depth, in order, without overlap");
    if (y.n_t < 1 || y.n_a < 1 || !finite_pos(y.cryst_t_mm) || !finite_pos(y.cryst_a_mm) ||
        y.pitch_t_mm < y.cryst_t_mm || y.pitch_a_mm < y.cryst_a_mm || !(y.offset_t_mm >= 0) ||
        !(y.offset_a_mm >= 0))
      return bad("crystal size, pitch or offset");
    if (y.offset_t_mm + y.n_t * y.pitch_t_mm > g->mod_t_mm + 1e-6 ||
        y.offset_a_mm + y.n_a * y.pitch_a_mm > g->mod_a_mm + 1e-6)
      return bad("crystal array exceeds the module");
    if (y.crystal_material < 0 || y.crystal_material >= c->n_mat || y.interval_material < 0 ||
        y.interval_material >= c->n_mat)
      return bad("layer material");
    prev_end = y.depth0_mm + y.thickness_mm;
    per_module += (int64_t)y.n_t * y.n_a;
  }
  const int64_t per_panel = per_module * g->mod_n_t * g->mod_n_a;
  const int64_t total = per_panel * g->n_panels;
  if (total >= (1 << 20)) return bad("more than 2^20 crystals");

  // panel poses: repetition mode places panel k at angle phi0 + 2 pi k / n.
  // Device layout per panel: rows of the local axes (depth, t, a) in global
  // coordinates, then the front-face centre projected on each axis.
  std::vector<float> &pose = B.pose;
  pose.assign((size_t)g->n_panels * 12, 0.f);
  for (int k = 0; k < g->n_panels; ++k) {
    double o[3], ax[9];
    if (g->placement == GPET_PLACE_REPEAT) {
      const double a = g->phi0_rad + 2.0 * kPi * k / g->n_panels;
      const double ca = std::cos(a), sa = std::sin(a);
      const double oo[3] = {g->radius_mm * ca, g->radius_mm * sa, g->z0_mm};
      const double aa[9] = {ca, sa, 0.0, -sa, ca, 0.0, 0.0, 0.0, 1.0};
      std::memcpy(o, oo, sizeof(o));
      std::memcpy(ax, aa, sizeof(ax));
    } else if (g->placement == GPET_PLACE_EXPLICIT) {
      if (!g->poses) return bad("explicit placement needs poses");
      std::memcpy(o, g->poses + 12 * k, sizeof(o));
      std::memcpy(ax, g->poses + 12 * k + 3, sizeof(ax));
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          const double dot = ax[3 * i] * ax[3 * j] + ax[3 * i + 1] * ax[3 * j + 1] + ax[3 * i + 2] * ax[3 * j + 2];
          if (std::fabs(dot - (i == j ? 1.0 : 0.0)) > 1e-6) return bad("pose axes are not orthonormal");
        }
    } else {
      return bad("unknown placement mode");
    }
    float *P = &pose[(size_t)k * 12];
    for (int i = 0; i < 9; ++i) P[i] = (float)ax[i];
    for (int i = 0; i < 3; ++i) P[9 + i] = (float)(ax[3 * i] * o[0] + ax[3 * i + 1] * o[1] + ax[3 * i + 2] * o[2]);
  }

  // materials present in the panel and their detector table slots
  B.used.assign(c->n_mat, false);
  B.used[g->fill_material] = true;
  for (int l = 0; l < g->n_layers; ++l)
    B.used[g->layers[l].crystal_material] = B.used[g->layers[l].interval_material] = true;
  auto slot = [&](int m) {
    for (size_t q = 0; q < slot_mat.size(); ++q)
      if (slot_mat[q] == m) return (int)q;
    slot_mat.push_back(m);
    return (int)slot_mat.size() - 1;
  };
  const int fill_slot = slot(g->fill_material);
  int slot_c[GPET_MAX_LAYERS], slot_i[GPET_MAX_LAYERS];
  for (int l = 0; l < g->n_layers; ++l) {
    slot_c[l] = slot(g->layers[l].crystal_material);
    slot_i[l] = slot(g->layers[l].interval_material);
  }
  if (slot_mat.size() > 4) return fail(c, GPET_ERR_UNSUPPORTED, who + "more than 4 distinct detector materials");

  DevScene &S = B.S;
  S.n_panels = g->n_panels;
  S.ring = 1;
  for (int k = 0; k < g->n_panels; ++k) {
    const float *P = &pose[(size_t)k * 12];
    if (P[2] != 0.0f || P[5] != 0.0f || P[6] != 0.0f || P[7] != 0.0f || P[8] != 1.0f || P[11] != pose[11]) S.ring = 0;
  }
  S.depth = (float)g->depth_mm;
  S.half_w = (float)(0.5 * g->width_mm);
  S.half_l = (float)(0.5 * g->length_mm);
  S.ring_reg = (S.ring && g->placement == GPET_PLACE_REPEAT && g->radius_mm > 0.0) ? 1 : 0;
  if (S.ring_reg) {
    const double R = g->radius_mm, hw = 0.5 * g->width_mm, D = g->depth_mm;
    S.ring_R2 = (float)(R * R * (1.0 - 2e-6));
    S.ring_rmax2 = (float)(((R + D) * (R + D) + hw * hw) * (1.0 + 2e-6));
    S.ring_n = (float)g->n_panels;
    S.ring_u0 = (float)(g->phi0_rad * g->n_panels / (2.0 * kPi));
    // half span, plus twice the azimuth approximation's bound (6.0e-4 turn) and rounding slack
    S.ring_a = (float)(std::atan(hw / R) * g->n_panels / (2.0 * kPi) + 2.0 * 6.0e-4 * g->n_panels + 1e-3);
  }
  S.mod_n_t = g->mod_n_t;
  S.mod_n_a = g->mod_n_a;
  S.mod_t0 = (float)(-0.5 * w_mod);
  S.mod_a0 = (float)(-0.5 * l_mod);
  S.mod_step_t = (float)(g->mod_t_mm + g->gap_t_mm);
  S.mod_step_a = (float)(g->mod_a_mm + g->gap_a_mm);
  S.inv_step_t = (float)(1.0 / (g->mod_t_mm + g->gap_t_mm));
  S.inv_step_a = (float)(1.0 / (g->mod_a_mm + g->gap_a_mm));
  S.mod_t = (float)g->mod_t_mm;
  S.mod_a = (float)g->mod_a_mm;
  S.fill = g->fill_material;
  S.fill_slot = fill_slot;
  S.n_layers = g->n_layers;
  int base = 0;
  for (int l = 0; l < g->n_layers; ++l) {
    const gpet_layer &y = g->layers[l];
    LayerD &d = S.layer[l];
    d.d0 = (float)y.depth0_mm;
    d.d1 = (float)(y.depth0_mm + y.thickness_mm);
    d.off_t = (float)y.offset_t_mm;
    d.off_a = (float)y.offset_a_mm;
    d.pitch_t = (float)y.pitch_t_mm;
    d.pitch_a = (float)y.pitch_a_mm;
    d.inv_pitch_t = (float)(1.0 / y.pitch_t_mm);
    d.inv_pitch_a = (float)(1.0 / y.pitch_a_mm);
    d.slot_crystal = slot_c[l];
    d.slot_interval = slot_i[l];
    d.lo_t = (float)(0.5 * (y.pitch_t_mm - y.cryst_t_mm));
    d.hi_t = (float)(0.5 * (y.pitch_t_mm + y.cryst_t_mm));
    d.lo_a = (float)(0.5 * (y.pitch_a_mm - y.cryst_a_mm));
    d.hi_a = (float)(0.5 * (y.pitch_a_mm + y.cryst_a_mm));
    d.n_t = y.n_t;
    d.n_a = y.n_a;
    d.mat_crystal = y.crystal_material;
    d.mat_interval = y.interval_material;
    d.base = base;
    B.info.layer_base[l] = base;
    base += y.n_t * y.n_a;
  }
  S.crystals_per_module = (int)per_module;
  S.crystals_per_panel = (int)per_panel;
  S.e_cut = (float)c->phys.e_cut_kev;
  B.info.n_crystals = (int32_t)total;
  B.info.crystals_per_panel = (int32_t)per_panel;
  B.info.crystals_per_module = (int32_t)per_module;
  for (int l = g->n_layers; l < GPET_MAX_LAYERS; ++l) B.info.layer_base[l] = -1;
  return GPET_OK;
}

// Detector tables: one attenuation row per slot (read by the transport
// kernels) and the node-wise maximum of the attenuation over the
// materials marked in `used` (the detector majorant).
void detector_tables(const gpet_ctx *c, const std::vector<int> &slot_mat, const std::vector<bool> &used,
                     std::vector<float4> &rows, std::vector<float> &maj) {
  rows.assign(slot_mat.size() * kTabStride, make_float4(0.f, 0.f, 0.f, 0.f));
  for (size_t q = 0; q < slot_mat.size(); ++q)
    for (int k = 0; k < kTabStride; ++k) {
      const int node = std::min(k, kNodes - 1);
      const float *src = &c->mu_host[((size_t)slot_mat[q] * 4) * kNodes + node];
      rows[q * kTabStride + k] = make_float4(src[0], src[kNodes], src[2 * kNodes], src[3 * kNodes]);
    }
  maj.assign(kTabStride, 0.f);
  for (int k = 0; k < kTabStride; ++k) {
    const int node = std::min(k, kNodes - 1);
    double mx = 0.0;
    for (int i = 0; i < c->n_mat; ++i)
      if (used[i]) {
        double a[3];
        attenuation_per_density(c->mats[i], c->phys, (double)(node + 1), a);
        mx = std::max(mx, c->mats[i].density_g_cm3 * (a[0] + a[1] + a[2]));
      }
    maj[k] = (float)mx;
  }
}

// Validates a source and fills the source fields of S (rod pointers left
// unset); rods (5 floats each) and their cumulative volume weights go to the
// vectors.
gpet_status build_source(gpet_ctx *c, const gpet_source *src, DevScene &S, std::vector<float> &rods,
                         std::vector<float> &cum, const std::string &who) {
  if (!src) return fail(c, GPET_ERR_ARG, who + "null");
  if (src->duration_ps == 0) return fail(c, GPET_ERR_ARG, who + "duration must be positive");
  rods.clear();
  cum.clear();
  S.n_rods = 0;
  S.rod_total = 0.f;
  if (src->kind == GPET_SRC_CYLINDERS) {
    if (src->n_rods < 1 || src->n_rods > GPET_MAX_RODS || !src->rods) return fail(c, GPET_ERR_ARG, who + "rods");
    rods.resize((size_t)src->n_rods * 5);
    cum.resize(src->n_rods);
    double acc = 0.0;
    for (int i = 0; i < src->n_rods; ++i) {
      const double *r = src->rods + 5 * i;
      if (!finite_pos(r[2]) || !(r[4] > r[3])) return fail(c, GPET_ERR_ARG, who + "bad rod");
      acc += r[2] * r[2] * (r[4] - r[3]); // weight by rod volume
      cum[i] = (float)acc;
      for (int k = 0; k < 5; ++k) rods[(size_t)i * 5 + k] = (float)r[k];
    }
    S.n_rods = src->n_rods;
    S.rod_total = (float)acc;
  } else if (src->kind == GPET_SRC_BEAM) {
    const double n = std::sqrt(src->dir[0] * src->dir[0] + src->dir[1] * src->dir[1] + src->dir[2] * src->dir[2]);
    if (!(std::fabs(n - 1.0) < 1e-6)) return fail(c, GPET_ERR_ARG, who + "beam direction must be a unit vector");
  } else if (src->kind != GPET_SRC_POINT) {
    return fail(c, GPET_ERR_ARG, who + "unknown kind");
  }
  S.src_kind = src->kind;
  S.sx = (float)src->pos_mm[0];
  S.sy = (float)src->pos_mm[1];
  S.sz = (float)src->pos_mm[2];
  S.bdx = (float)src->dir[0];
  S.bdy = (float)src->dir[1];
  S.bdz = (float)src->dir[2];
  S.duration_ps = src->duration_ps;
  if (!(src->acolinearity_fwhm_deg >= 0.0 && src->acolinearity_fwhm_deg <= 10.0))
    return fail(c, GPET_ERR_ARG, who + "acollinearity FWHM must lie in [0, 10] degrees");
  if (!(src->positron_range_fwhm_mm >= 0.0 && src->positron_range_fwhm_mm <= 10.0))
    return fail(c, GPET_ERR_ARG, who + "positron range FWHM must lie in [0, 10] mm");
  const double fwhm_per_sigma = 2.354820045030949; // 2 sqrt(2 ln 2)
  S.acol_sigma = (float)(src->acolinearity_fwhm_deg * (3.14159265358979323846 / 180.0) / fwhm_per_sigma);
  S.prange_sigma = (float)(src->positron_range_fwhm_mm / fwhm_per_sigma);
  return GPET_OK;
}

// copies the geometry fields of G into S (everything from n_panels through
// crystals_per_panel plus the detector slot count)
void set_geometry_fields(DevScene &S, const DevScene &G) {
  S.n_panels = G.n_panels;
  S.ring = G.ring;
  S.ring_reg = G.ring_reg;
  S.ring_R2 = G.ring_R2;
  S.ring_rmax2 = G.ring_rmax2;
  S.ring_n = G.ring_n;
  S.ring_u0 = G.ring_u0;
  S.ring_a = G.ring_a;
  S.depth = G.depth;
  S.half_w = G.half_w;
  S.half_l = G.half_l;
  S.mod_n_t = G.mod_n_t;
  S.mod_n_a = G.mod_n_a;
  S.mod_t0 = G.mod_t0;
  S.mod_a0 = G.mod_a0;
  S.mod_step_t = G.mod_step_t;
  S.mod_step_a = G.mod_step_a;
  S.inv_step_t = G.inv_step_t;
  S.inv_step_a = G.inv_step_a;
  S.mod_t = G.mod_t;
  S.mod_a = G.mod_a;
  S.fill = G.fill;
  S.fill_slot = G.fill_slot;
  S.n_layers = G.n_layers;
  for (int l = 0; l < kMaxLayers; ++l) S.layer[l] = G.layer[l];
  S.crystals_per_module = G.crystals_per_module;
  S.crystals_per_panel = G.crystals_per_panel;
}

} // namespace

extern "C" {

gpet_status gpet_ctx_create(int device, void *hip_stream, gpet_ctx **out) {
  if (!out) return GPET_ERR_ARG;
  *out = nullptr;
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev) return GPET_ERR_HIP;
  gpet_ctx *c = new (std::nothrow) gpet_ctx();
  if (!c) return GPET_ERR_ARG;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return GPET_ERR_HIP;
  }
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cu > 0)
    c->n_cu = cu;
  static_assert(kCtrlWords <= 16 && kCtrlWorkWord >= 16 && kCtrlPairWord >= kCtrlWorkWord + 16 &&
                    kCtrlPairWord < kCtrlAlloc, "control words");
  if (hipMalloc((void **)&c->d_ctrl, kCtrlAlloc * sizeof(unsigned long long)) != hipSuccess) {
    delete c;
    return GPET_ERR_HIP;
  }
  if (hipHostMalloc((void **)&c->h_ctrl, kCtrlAlloc * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess ||
      hipMalloc((void **)&c->d_plain, kSceneBytes + 256) != hipSuccess ||
      hipHostMalloc((void **)&c->h_plain, kSceneBytes + 256, hipHostMallocDefault) != hipSuccess) {
    gpet_ctx_destroy(c);
    return GPET_ERR_HIP;
  }
  // the static digitizer scratch of this device (with the device current)
  c->fixed_scratch = fixed_scratch(device, c->err);
  if (!c->fixed_scratch) {
    gpet_ctx_destroy(c);
    return GPET_ERR_HIP;
  }
  *out = c;
  return GPET_OK;
}

void gpet_ctx_destroy(gpet_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->squeue.blob) (void)hipFree(c->squeue.blob);
  for (void *p : {(void *)c->d_mu, (void *)c->d_mu_mass, (void *)c->d_mu_det, (void *)c->d_maj_det, (void *)c->d_maj_ph,
                  (void *)c->d_pose, (void *)c->d_vmat, (void *)c->d_vden, (void *)c->d_rods,
                  (void *)c->d_rod_cum, (void *)c->d_ctrl, (void *)c->d_plain})
    if (p) (void)hipFree(p);
  if (c->h_ctrl) (void)hipHostFree(c->h_ctrl);
  if (c->h_plain) (void)hipHostFree(c->h_plain);
  for (hipEvent_t &e : c->ev)
    if (e) (void)hipEventDestroy(e);
  free_scratch(c->scratch);
  delete c;
}

const char *gpet_last_error(const gpet_ctx *c) { return c ? c->err.c_str() : "null context"; }

gpet_status gpet_ctx_set_stream(gpet_ctx *c, void *hip_stream) {
  if (!c) return GPET_ERR_ARG;
  c->stream = (hipStream_t)hip_stream;
  return GPET_OK;
}

gpet_status gpet_materials_set(gpet_ctx *c, int32_t n, const gpet_material *m, const gpet_physics *ph) {
  if (!c) return GPET_ERR_ARG;
  if (n < 1 || n > GPET_MAX_MATERIALS || !m || !ph) return fail(c, GPET_ERR_ARG, "materials: bad count or null");
  if (!(ph->k_pe >= 0) || !(ph->k_rayleigh >= 0) || !(ph->e_cut_kev >= 1.0 && ph->e_cut_kev < 511.0))
    return fail(c, GPET_ERR_ARG, "materials: physics constants out of range");
  for (int i = 0; i < n; ++i) {
    const gpet_material &q = m[i];
    if (!finite_pos(q.density_g_cm3) || q.n_elements < 1 || q.n_elements > GPET_MAX_ELEMENTS)
      return fail(c, GPET_ERR_ARG, "materials: bad density or element count");
    double wsum = 0;
    for (int j = 0; j < q.n_elements; ++j) {
      if (q.Z[j] < 1 || q.Z[j] > 118 || !finite_pos(q.A[j]) || !(q.mass_fraction[j] >= 0))
        return fail(c, GPET_ERR_ARG, "materials: bad element");
      wsum += q.mass_fraction[j];
    }
    if (std::fabs(wsum - 1.0) > 1e-6) return fail(c, GPET_ERR_ARG, "materials: mass fractions must sum to 1");
  }
  (void)hipSetDevice(c->device);
  c->n_mat = n;
  c->mats.assign(m, m + n);
  c->phys = *ph;
  std::vector<float4> mass((size_t)n * kTabStride), nom((size_t)n * kTabStride);
  c->mu_host.assign((size_t)n * 4 * kNodes, 0.f);
  c->mu_mass_host.assign((size_t)n * 4 * kNodes, 0.f);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < kTabStride; ++k) {
      const int node = std::min(k, kNodes - 1);
      double a[3];
      attenuation_per_density(m[i], *ph, (double)(node + 1), a);
      const double rho = m[i].density_g_cm3;
      mass[(size_t)i * kTabStride + k] = make_float4((float)a[0], (float)a[1], (float)a[2], (float)(a[0] + a[1] + a[2]));
      nom[(size_t)i * kTabStride + k] =
          make_float4((float)(rho * a[0]), (float)(rho * a[1]), (float)(rho * a[2]), (float)(rho * (a[0] + a[1] + a[2])));
      if (k < kNodes) {
        const float4 f = nom[(size_t)i * kTabStride + k], g = mass[(size_t)i * kTabStride + k];
        float *dn = &c->mu_host[((size_t)i * 4) * kNodes + k];
        float *dm = &c->mu_mass_host[((size_t)i * 4) * kNodes + k];
        dn[0] = f.x; dn[kNodes] = f.y; dn[2 * kNodes] = f.z; dn[3 * kNodes] = f.w;
        dm[0] = g.x; dm[kNodes] = g.y; dm[2 * kNodes] = g.z; dm[3 * kNodes] = g.w;
      }
    }
  gpet_status s = upload(c, c->d_mu, nom.data(), nom.size(), "materials: upload");
  if (!s) s = upload(c, c->d_mu_mass, mass.data(), mass.size(), "materials: upload");
  if (s) return s;
  // geometry and phantom majorants depend on the material list
  c->have_geometry = false;
  if (c->d_vmat) (void)hipFree(c->d_vmat);
  if (c->d_vden) (void)hipFree(c->d_vden);
  c->d_vmat = nullptr;
  c->d_vden = nullptr;
  c->scene.has_phantom = 0;
  ++c->mat_gen;
  ++c->phantom_gen;
  c->scene.e_cut = (float)ph->e_cut_kev;
  c->scene.mu = c->d_mu;
  c->scene.mu_mass = c->d_mu_mass;
  return GPET_OK;
}

gpet_status gpet_geometry_create(gpet_ctx *c, const gpet_scanner *g, gpet_geometry_info *info) {
  if (!c) return GPET_ERR_ARG;
  if (c->n_mat == 0) return fail(c, GPET_ERR_STATE, "geometry: set materials first");
  GeomBuild B;
  std::vector<int> slot_mat;
  gpet_status s = build_geometry(c, g, slot_mat, B, "geometry: ");
  if (s) return s;
  std::vector<float4> rows;
  std::vector<float> maj;
  detector_tables(c, slot_mat, B.used, rows, maj);
  (void)hipSetDevice(c->device);
  s = upload(c, c->d_pose, B.pose.data(), B.pose.size(), "geometry: upload");
  if (!s) s = upload(c, c->d_maj_det, maj.data(), maj.size(), "geometry: upload");
  if (!s) s = upload(c, c->d_mu_det, rows.data(), rows.size(), "geometry: upload");
  if (s) return s;
  c->maj_det_host.assign(maj.begin(), maj.begin() + kNodes);
  DevScene &S = c->scene;
  set_geometry_fields(S, B.S);
  S.pose = c->d_pose;
  S.maj_det = c->d_maj_det;
  S.mu_det = c->d_mu_det;
  S.n_det_slots = (int)slot_mat.size();
  S.mu = c->d_mu;
  S.mu_mass = c->d_mu_mass;
  S.e_cut = (float)c->phys.e_cut_kev;
  c->info = B.info;
  c->have_geometry = true;
  if (info) *info = c->info;
  return GPET_OK;
}

gpet_status gpet_phantom_set(gpet_ctx *c, const gpet_phantom *ph) {
  if (!c) return GPET_ERR_ARG;
  if (c->n_mat == 0) return fail(c, GPET_ERR_STATE, "phantom: set materials first");
  (void)hipSetDevice(c->device);
  DevScene &S = c->scene;
  ++c->phantom_gen;
  if (!ph) {
    S.has_phantom = 0;
    return GPET_OK;
  }
  if (ph->nx < 1 || ph->ny < 1 || ph->nz < 1 || !ph->material || !ph->density)
    return fail(c, GPET_ERR_ARG, "phantom: bad dimensions or null arrays");
  for (int k = 0; k < 3; ++k)
    if (!finite_pos(ph->voxel_mm[k]) || !std::isfinite(ph->origin_mm[k]))
      return fail(c, GPET_ERR_ARG, "phantom: bad voxel size or origin");
  const size_t nv = (size_t)ph->nx * ph->ny * ph->nz;
  if (nv >= ((size_t)1 << 31)) return fail(c, GPET_ERR_ARG, "phantom: too many voxels");
  std::vector<double> rmax(c->n_mat, 0.0);
  for (size_t v = 0; v < nv; ++v) {
    const int m = ph->material[v];
    const float r = ph->density[v];
    if (m >= c->n_mat) return fail(c, GPET_ERR_ARG, "phantom: material id out of range");
    if (!(r >= 0.0f) || !std::isfinite(r)) return fail(c, GPET_ERR_ARG, "phantom: bad density");
    rmax[m] = std::max(rmax[m], (double)r);
  }
  std::vector<float> maj(kTabStride, 0.f);
  for (int k = 0; k < kTabStride; ++k) {
    const int node = std::min(k, kNodes - 1);
    double mx = 0.0;
    for (int i = 0; i < c->n_mat; ++i)
      if (rmax[i] > 0) {
        double a[3];
        attenuation_per_density(c->mats[i], c->phys, (double)(node + 1), a);
        mx = std::max(mx, rmax[i] * (a[0] + a[1] + a[2]));
      }
    maj[k] = (float)mx;
  }
  if (maj[510] <= 0.f) return fail(c, GPET_ERR_ARG, "phantom: all voxels are void");
  S.has_phantom = 0;
  gpet_status s = upload(c, c->d_vmat, ph->material, nv, "phantom: upload");
  if (!s) s = upload(c, c->d_vden, ph->density, nv, "phantom: upload");
  if (!s) s = upload(c, c->d_maj_ph, maj.data(), maj.size(), "phantom: upload");
  if (s) return s;
  S.has_phantom = 1;
  S.nx = ph->nx;
  S.ny = ph->ny;
  S.nz = ph->nz;
  S.ox = (float)ph->origin_mm[0];
  S.oy = (float)ph->origin_mm[1];
  S.oz = (float)ph->origin_mm[2];
  S.ivx = (float)(1.0 / ph->voxel_mm[0]);
  S.ivy = (float)(1.0 / ph->voxel_mm[1]);
  S.ivz = (float)(1.0 / ph->voxel_mm[2]);
  S.bx = (float)(ph->origin_mm[0] + ph->nx * ph->voxel_mm[0]);
  S.by = (float)(ph->origin_mm[1] + ph->ny * ph->voxel_mm[1]);
  S.bz = (float)(ph->origin_mm[2] + ph->nz * ph->voxel_mm[2]);
  S.vmat = c->d_vmat;
  S.vden = c->d_vden;
  S.maj_ph = c->d_maj_ph;
  return GPET_OK;
}

gpet_status gpet_source_set(gpet_ctx *c, const gpet_source *src) {
  if (!c) return GPET_ERR_ARG;
  DevScene &S = c->scene;
  std::vector<float> rods, cum;
  DevScene T = S;
  gpet_status s = build_source(c, src, T, rods, cum, "source: ");
  if (s) return s;
  (void)hipSetDevice(c->device);
  if (!rods.empty()) {
    s = upload(c, c->d_rods, rods.data(), rods.size(), "source: upload");
    if (!s) s = upload(c, c->d_rod_cum, cum.data(), cum.size(), "source: upload");
    if (s) return s;
  }
  S = T;
  S.rods = rods.empty() ? nullptr : c->d_rods;
  S.rod_cum = rods.empty() ? nullptr : c->d_rod_cum;
  c->have_source = true;
  return GPET_OK;
}

static gpet_status ready(gpet_ctx *c) {
  if (!c) return GPET_ERR_ARG;
  if (!c->have_geometry) return fail(c, GPET_ERR_STATE, "no geometry (gpet_geometry_create)");
  if (!c->have_source) return fail(c, GPET_ERR_STATE, "no source (gpet_source_set)");
  return GPET_OK;
}


// Launch arguments of a plain run: a one-instance table (the context's scene,
// chunk prefix {0, chunks}, first event, count, instance id) staged through
// pinned memory; the call synchronizes before the staging area is reused.
static gpet_status run_args(gpet_ctx *c, uint64_t first, uint64_t n, uint64_t seed, uint32_t instance,
                            RunArgs &A) {
  A = RunArgs{};
  const uint32_t chunks = (uint32_t)((n + kPlainChunk - 1) / kPlainChunk);
  std::memcpy(c->h_plain, &c->scene, sizeof(DevScene));
  uint32_t *w = (uint32_t *)(c->h_plain + kSceneBytes);
  w[0] = 0;
  w[1] = chunks;
  w[2] = (uint32_t)first;
  w[3] = (uint32_t)n;
  w[4] = instance;
  gpet_status s = hip_check(c, hipMemcpyAsync(c->d_plain, c->h_plain, kSceneBytes + 32, hipMemcpyHostToDevice,
                                              c->stream), "transport: table upload");
  if (s) return s;
  const uint32_t *dw = (const uint32_t *)(c->d_plain + kSceneBytes);
  A.scenes = (const DevScene *)c->d_plain;
  A.chunk_prefix = dw;
  A.inst_first = dw + 2;
  A.inst_count = dw + 3;
  A.inst_id = dw + 4;
  A.n_inst = 1;
  A.chunk = kPlainChunk;
  A.total_chunks = chunks;
  A.first = (uint32_t)first;
  A.n = (uint32_t)n;
  A.k0 = (uint32_t)seed;
  A.k1 = (uint32_t)(seed >> 32);
  A.work = (uint32_t *)(c->d_ctrl + kCtrlWorkWord);
  A.hit_count = c->d_ctrl + 1;
  A.stats = c->d_ctrl + 2;
  A.search_batch = c->shape.search_batch;
  A.schedule = c->shape.schedule;
  return GPET_OK;
}

static void set_hits(RunArgs &A, gpet_hits *h) {
  A.h_event = h->event;
  A.h_gid = h->gid;
  A.h_edep = h->edep_kev;
  A.h_depth = h->depth_mm;
  A.h_time = (unsigned long long *)h->time_ps;
  A.h_aux = h->aux;
  A.h_inst = h->instance;
  A.capacity = h->capacity;
}

// zeroes the control words (counts, work counters), the event-claim counter
// and the pair / entry counter
static void reset_ctrl(gpet_ctx *c, hipStream_t st) {
  launch_fill_u32((uint32_t *)c->d_ctrl, 0u, 2 * kCtrlWords, st);
  launch_fill_u32((uint32_t *)(c->d_ctrl + kCtrlWorkWord), 0u, 2, st);
  launch_fill_u32((uint32_t *)(c->d_ctrl + kCtrlPairWord), 0u, 2, st);
}

// runs a prepared transport launch and reads back the counts
static gpet_status run_transport(gpet_ctx *c, const RunArgs &A, const LaunchShape &shape,
                                 gpet_hits *h, gpet_stats *stats, int mode = kModePlain) {
  reset_ctrl(c, c->stream);
  if (c->timing) (void)hipEventRecord(c->ev[0], c->stream);
  if (A.total_chunks) launch_transport(A, shape, c->n_cu, c->stream, mode);
  if (c->timing) (void)hipEventRecord(c->ev[1], c->stream);
  gpet_status s = hip_check(c, hipGetLastError(), "transport: launch");
  if (s) return s;
  s = hip_check(c, hipMemcpyAsync(c->h_ctrl, c->d_ctrl, kCtrlWords * 8, hipMemcpyDeviceToHost, c->stream), "transport: readback");
  if (!s && mode == kModeRecord)
    s = hip_check(c, hipMemcpyAsync(c->h_ctrl + kCtrlPairWord, c->d_ctrl + kCtrlPairWord, 8, hipMemcpyDeviceToHost,
                                    c->stream), "transport: readback");
  if (!s) s = hip_check(c, wait_stream(c->stream), "transport: kernel");
  if (s) return s;
  h->count = c->h_ctrl[1];
  if (c->timing) (void)hipEventElapsedTime(&c->last_ms[0], c->ev[0], c->ev[1]);
  if (stats) {
    uint64_t *o = (uint64_t *)stats;
    for (int k = 0; k < kStatCount; ++k) o[k] = c->h_ctrl[2 + k];
  }
  if (h->count > h->capacity) return fail(c, GPET_ERR_CAPACITY, "transport: hit capacity too small");
  return GPET_OK;
}

static bool hits_ok(const gpet_hits *h) {
  return !h->capacity || (h->event && h->gid && h->edep_kev && h->depth_mm && h->time_ps && h->aux);
}

gpet_status gpet_transport(gpet_ctx *c, uint64_t first, uint64_t n, uint64_t seed, uint32_t instance,
                           gpet_hits *h, gpet_stats *stats) {
  gpet_status s = ready(c);
  if (s) return s;
  if (!h) return fail(c, GPET_ERR_ARG, "transport: null hits");
  if (n > 0x7fffffffull || first + n > 0x100000000ull) return fail(c, GPET_ERR_ARG, "transport: event range");
  if (!hits_ok(h)) return fail(c, GPET_ERR_ARG, "transport: null hit array");
  (void)hipSetDevice(c->device);
  RunArgs A;
  s = run_args(c, first, n, seed, instance, A);
  if (s) return s;
  set_hits(A, h);
  return run_transport(c, A, c->shape, h, stats);
}

// shared validation of digitizer parameters
static gpet_status digitizer_params(gpet_ctx *c, const gpet_hits *h, const gpet_digitizer *p, gpet_singles *sg,
                                    gpet_coincidences *cc, DigitizeArgs &D) {
  if (!h || !p || !sg || !cc) return fail(c, GPET_ERR_ARG, "digitize: null argument");
  if (h->count > h->capacity) return fail(c, GPET_ERR_ARG, "digitize: hit count exceeds capacity");
  if (h->count >= 0xffffffffull) return fail(c, GPET_ERR_UNSUPPORTED, "digitize: more than 2^32 hits");
  if (h->count && (!h->event || !h->gid || !h->edep_kev || !h->depth_mm || !h->time_ps || !h->aux))
    return fail(c, GPET_ERR_ARG, "digitize: null hit array");
  if (!(p->fwhm_511 >= 0) || !(p->e_lo_kev <= p->e_hi_kev)) return fail(c, GPET_ERR_ARG, "digitize: parameters");
  D.n_hits = h->count;
  D.h_event = h->event;
  D.h_gid = h->gid;
  D.h_aux = h->aux;
  D.h_edep = h->edep_kev;
  D.h_depth = h->depth_mm;
  D.h_time = (const unsigned long long *)h->time_ps;
  D.fwhm_511 = (float)p->fwhm_511;
  D.e_lo = (float)p->e_lo_kev;
  D.e_hi = (float)p->e_hi_kev;
  D.window_ps = p->window_ps;
  D.k0 = (uint32_t)p->seed;
  D.k1 = (uint32_t)(p->seed >> 32);
  if (p->readout > GPET_READOUT_PANEL) return fail(c, GPET_ERR_ARG, "digitize: unknown readout level");
  D.readout = p->readout;
  if (p->n_sweep) {
    if (!p->sweep_lo_kev || !p->sweep_hi_kev || !p->sweep_coincidences)
      return fail(c, GPET_ERR_ARG, "digitize: null sweep array");
    for (uint32_t w = 0; w < p->n_sweep; ++w) {
      if (!(p->sweep_lo_kev[w] <= p->sweep_hi_kev[w])) return fail(c, GPET_ERR_ARG, "digitize: sweep window");
      D.sweep_lo.push_back((float)p->sweep_lo_kev[w]);
      D.sweep_hi.push_back((float)p->sweep_hi_kev[w]);
    }
    D.sweep_out = p->sweep_coincidences;
  }
  if (!(p->time_fwhm_ps >= 0.0 && p->time_fwhm_ps <= 1e6))
    return fail(c, GPET_ERR_ARG, "digitize: timing resolution must lie in [0, 1e6] ps");
  if (!(p->doi_fwhm_mm >= 0.0 && p->doi_fwhm_mm <= 100.0))
    return fail(c, GPET_ERR_ARG, "digitize: DOI resolution must lie in [0, 100] mm");
  if (p->dead_time_mode > GPET_DEAD_NONPARALYZABLE) return fail(c, GPET_ERR_ARG, "digitize: unknown dead-time mode");
  if (p->dead_time_level > GPET_READOUT_PANEL) return fail(c, GPET_ERR_ARG, "digitize: unknown dead-time level");
  const double fwhm_per_sigma = 2.354820045030949; // 2 sqrt(2 ln 2)
  D.time_sigma = (float)(p->time_fwhm_ps / fwhm_per_sigma);
  D.doi_sigma = (float)(p->doi_fwhm_mm / fwhm_per_sigma);
  D.dead_mode = p->dead_time_ps ? p->dead_time_mode : (uint32_t)GPET_DEAD_NONE;
  D.dead_level = p->dead_time_level;
  D.dead_ps = p->dead_time_ps;
  if (!(p->light_sharing >= 0.0 && p->light_sharing <= 1.0))
    return fail(c, GPET_ERR_ARG, "digitize: light-sharing probability must lie in [0, 1]");
  D.ls_thresh = p->light_sharing >= 1.0 ? (1ull << 32) : (unsigned long long)std::floor(p->light_sharing * 4294967296.0);
  D.singles = sg;
  D.coinc = cc;
  return GPET_OK;
}

static gpet_status timed_digitize(gpet_ctx *c, DigitizeArgs &D, DigitizeScratch *scr = nullptr) {
  if (c->timing) (void)hipEventRecord(c->ev[2], c->stream);
  const int r = run_digitize(D, scr ? *scr : c->scratch, c->stream, c->err);
  if (r != GPET_OK) return r;
  if (c->timing) {
    (void)hipEventRecord(c->ev[3], c->stream);
    (void)hipEventSynchronize(c->ev[3]);
    (void)hipEventElapsedTime(&c->last_ms[1], c->ev[2], c->ev[3]);
  }
  return hip_check(c, hipGetLastError(), "digitize: launch");
}

// arguments of a plain (one-scanner) digitizer call
static gpet_status plain_digitizer_args(gpet_ctx *c, const gpet_hits *h, const gpet_digitizer *p, gpet_singles *sg,
                                        gpet_coincidences *cc, gpet_tallies *t, DigitizeArgs &D) {
  if (!c) return GPET_ERR_ARG;
  if (!c->have_geometry) return fail(c, GPET_ERR_STATE, "digitize: no geometry");
  gpet_status s = digitizer_params(c, h, p, sg, cc, D);
  if (s) return s;
  if (p->n_events == 0 || p->n_events > 0xffffffffull || p->first_event + p->n_events > 0x100000000ull)
    return fail(c, GPET_ERR_ARG, "digitize: event range");
  if (t && t->doi && t->doi_bins < 1) return fail(c, GPET_ERR_ARG, "digitize: doi_bins");
  D.first = {(uint32_t)p->first_event};
  D.n_events = {(uint32_t)p->n_events};
  D.cpp = {(uint32_t)c->info.crystals_per_panel};
  D.cpm = {(uint32_t)c->info.crystals_per_module};
  D.ncr = {(uint32_t)c->info.n_crystals};
  layer_words(c->scene, D.layers);
  D.rng = {p->instance};
  D.duration = {c->have_source ? (unsigned long long)c->scene.duration_ps : 0ull};
  D.gid_bits = bits_for((uint64_t)c->info.n_crystals - 1);
  D.panel_depth = c->scene.depth;
  D.tallies = t;
  return GPET_OK;
}

gpet_status gpet_digitize(gpet_ctx *c, const gpet_hits *h, const gpet_digitizer *p, gpet_singles *sg,
                          gpet_coincidences *cc, gpet_tallies *t) {
  DigitizeArgs D;
  const gpet_status s = plain_digitizer_args(c, h, p, sg, cc, t, D);
  if (s) return s;
  (void)hipSetDevice(c->device);
  return timed_digitize(c, D);
}

gpet_status gpet_digitize_noalloc(gpet_ctx *c, const gpet_hits *h, const gpet_digitizer *p, gpet_singles *sg,
                                  gpet_coincidences *cc, gpet_tallies *t) {
  DigitizeArgs D;
  const gpet_status s = plain_digitizer_args(c, h, p, sg, cc, t, D);
  if (s) return s;
  if (!c->fixed_scratch) return fail(c, GPET_ERR_STATE, "digitize_noalloc: no fixed scratch on this device");
  (void)hipSetDevice(c->device);
  DigitizeScratch fixed;
  fixed.buf = c->fixed_scratch;
  fixed.bytes = kFixedScratchBytes;
  fixed.fixed = true;
  return timed_digitize(c, D, &fixed);
}

gpet_status gpet_ctx_set_launch(gpet_ctx *c, int32_t blocks_per_cu, int32_t search_batch, int32_t schedule) {
  if (!c) return GPET_ERR_ARG;
  if (blocks_per_cu < 0 || blocks_per_cu > 64 || search_batch < 1 || search_batch > 64 || schedule < 0 ||
      schedule > 2)
    return fail(c, GPET_ERR_ARG, "launch: blocks_per_cu in 0..64, search_batch in 1..64, schedule 0, 1 or 2");
  c->shape.blocks_per_cu = blocks_per_cu;
  c->shape.search_batch = (uint32_t)search_batch;
  c->shape.schedule = (uint32_t)schedule;
  return GPET_OK;
}

gpet_status gpet_ctx_enable_timing(gpet_ctx *c, int enable) {
  if (!c) return GPET_ERR_ARG;
  (void)hipSetDevice(c->device);
  if (enable && !c->ev[0])
    for (hipEvent_t &e : c->ev)
      if (hipEventCreate(&e) != hipSuccess) return fail(c, GPET_ERR_HIP, "timing: event creation failed");
  c->timing = enable != 0;
  return GPET_OK;
}

gpet_status gpet_timings(gpet_ctx *c, float *ms2) {
  if (!c || !ms2) return GPET_ERR_ARG;
  ms2[0] = c->last_ms[0];
  ms2[1] = c->last_ms[1];
  return GPET_OK;
}

gpet_status gpet_philox(gpet_ctx *c, uint64_t seed, const uint32_t *ctr4, uint32_t n, uint32_t *out4) {
  if (!c || (n && (!ctr4 || !out4))) return GPET_ERR_ARG;
  (void)hipSetDevice(c->device);
  launch_philox(seed, ctr4, n, out4, c->stream);
  gpet_status s = hip_check(c, hipGetLastError(), "philox: launch");
  return s ? s : hip_check(c, hipStreamSynchronize(c->stream), "philox");
}

gpet_status gpet_tables_get(gpet_ctx *c, float *mu, float *maj) {
  if (!c) return GPET_ERR_ARG;
  if (c->n_mat == 0) return fail(c, GPET_ERR_STATE, "tables: no materials");
  if (mu) std::memcpy(mu, c->mu_host.data(), c->mu_host.size() * sizeof(float));
  if (maj) {
    if (!c->have_geometry) return fail(c, GPET_ERR_STATE, "tables: no geometry for the majorant");
    std::memcpy(maj, c->maj_det_host.data(), kNodes * sizeof(float));
  }
  return GPET_OK;
}

gpet_status gpet_locate(gpet_ctx *c, uint32_t n, const float *xyz, int32_t *ids6) {
  if (!c) return GPET_ERR_ARG;
  if (!c->have_geometry) return fail(c, GPET_ERR_STATE, "locate: no geometry");
  if (n && (!xyz || !ids6)) return fail(c, GPET_ERR_ARG, "locate: null");
  (void)hipSetDevice(c->device);
  launch_locate(c->scene, n, xyz, ids6, c->stream);
  gpet_status s = hip_check(c, hipGetLastError(), "locate: launch");
  return s ? s : hip_check(c, hipStreamSynchronize(c->stream), "locate");
}

gpet_status gpet_ray_locate(gpet_ctx *c, uint32_t n, const float *o, const float *d, int32_t ns, float step,
                            float *t_in, int32_t *ids6) {
  if (!c) return GPET_ERR_ARG;
  if (!c->have_geometry) return fail(c, GPET_ERR_STATE, "ray_locate: no geometry");
  if (ns < 0 || (n && (!o || !d || !t_in || (ns && !ids6)))) return fail(c, GPET_ERR_ARG, "ray_locate: args");
  (void)hipSetDevice(c->device);
  launch_ray_locate(c->scene, n, o, d, ns, step, t_in, ids6, c->stream);
  gpet_status s = hip_check(c, hipGetLastError(), "ray_locate: launch");
  return s ? s : hip_check(c, hipStreamSynchronize(c->stream), "ray_locate");
}

gpet_status gpet_sample_compton(gpet_ctx *c, float e, uint32_t n, uint64_t seed, float *cos_t, float *e_out,
                                int32_t *trials) {
  if (!c || !(e > 0.0f) || (n && (!cos_t || !e_out))) return c ? fail(c, GPET_ERR_ARG, "compton: args") : GPET_ERR_ARG;
  (void)hipSetDevice(c->device);
  launch_compton(e, n, seed, cos_t, e_out, trials, c->stream);
  gpet_status s = hip_check(c, hipGetLastError(), "compton: launch");
  return s ? s : hip_check(c, hipStreamSynchronize(c->stream), "compton");
}

gpet_status gpet_sample_rayleigh(gpet_ctx *c, uint32_t n, uint64_t seed, float *cos_t) {
  if (!c || (n && !cos_t)) return GPET_ERR_ARG;
  (void)hipSetDevice(c->device);
  launch_rayleigh(n, seed, cos_t, c->stream);
  gpet_status s = hip_check(c, hipGetLastError(), "rayleigh: launch");
  return s ? s : hip_check(c, hipStreamSynchronize(c->stream), "rayleigh");
}

gpet_status gpet_trace(gpet_ctx *c, uint64_t first, uint32_t n, uint64_t seed, uint32_t instance, int32_t maxv,
                       int32_t *vint, float *vflt, int32_t *counts) {
  gpet_status s = ready(c);
  if (s) return s;
  if (maxv < 1 || !vint || !vflt || !counts) return fail(c, GPET_ERR_ARG, "trace: buffers");
  if (first + n > 0x100000000ull || n > (1u << 24)) return fail(c, GPET_ERR_ARG, "trace: event range");
  (void)hipSetDevice(c->device);
  RunArgs A;
  s = run_args(c, first, n, seed, instance, A);
  if (s) return s;
  A.capacity = 0;
  A.vint = vint;
  A.vflt = vflt;
  A.vcount = counts;
  A.max_vertices = maxv;
  reset_ctrl(c, c->stream);
  launch_fill_u32((uint32_t *)counts, 0u, 2 * (size_t)n, c->stream);
  if (n) launch_trace(A, c->stream);
  s = hip_check(c, hipGetLastError(), "trace: launch");
  return s ? s : hip_check(c, hipStreamSynchronize(c->stream), "trace");
}

// ---------------------------------------------------------------------------
// surrogate
// ---------------------------------------------------------------------------
static gpet_status surrogate_spec(gpet_ctx *c, const gpet_surrogate_spec *p, SurSpecD &P, int &n_classes) {
  if (!p) return fail(c, GPET_ERR_ARG, "surrogate: null spec");
  if (p->half_width < 0 || p->half_width > 7 || p->n_ebins < 1 || p->n_ebins > 1024 ||
      !(p->e_min_kev > 0 && p->e_min_kev < 511.0) || !(p->ebin_kev > 0) || !(p->photopeak_tol_kev >= 0) ||
      !(p->max_slope > 0) || !(p->front_tol_mm > 0) ||
      (p->class_half_width != 0 && (p->class_half_width < p->half_width || p->class_half_width > 15)))
    return fail(c, GPET_ERR_ARG, "surrogate: spec out of range");
  const DevScene &S = c->scene;
  const int W = 2 * p->half_width + 1;
  const int H = p->class_half_width ? p->class_half_width : p->half_width, Wc = 2 * H + 1;
  for (int l = 0; l < S.n_layers; ++l)
    if (S.layer[l].n_t < W || S.layer[l].n_a < W || S.layer[l].n_t > 65535 || S.layer[l].n_a > 65535)
      return fail(c, GPET_ERR_UNSUPPORTED, "surrogate: a layer is narrower than the neighbourhood (or wider than 65535)");
  if (S.n_panels > 127 || S.mod_n_t * S.mod_n_a > (1 << 24))
    return fail(c, GPET_ERR_UNSUPPORTED, "surrogate: more than 127 panels or 2^24 modules");
  P.half = p->half_width;
  P.chalf = H;
  P.n_ebins = p->n_ebins;
  P.e_min = (float)p->e_min_kev;
  P.ebin = (float)p->ebin_kev;
  P.tol = (float)p->photopeak_tol_kev;
  P.max_slope = (float)p->max_slope;
  P.front_tol = (float)p->front_tol_mm;
  n_classes = 1 + S.n_layers * Wc * Wc * (p->n_ebins + 1);
  return GPET_OK;
}

gpet_status gpet_surrogate_pairs(gpet_ctx *c, const gpet_surrogate_spec *spec, uint64_t first, uint64_t n,
                                 uint64_t seed, uint32_t instance, gpet_hits *h, gpet_pairs *pairs,
                                 gpet_stats *stats) {
  gpet_status s = ready(c);
  if (s) return s;
  SurSpecD P;
  int n_classes = 0;
  s = surrogate_spec(c, spec, P, n_classes);
  if (s) return s;
  if (!h || !pairs) return fail(c, GPET_ERR_ARG, "surrogate pairs: null output");
  if (n > 0x7fffffffull || first + n > 0x100000000ull) return fail(c, GPET_ERR_ARG, "surrogate pairs: event range");
  if (!hits_ok(h)) return fail(c, GPET_ERR_ARG, "surrogate pairs: null hit array");
  if (pairs->capacity && (!pairs->x || !pairs->label || !pairs->flags || !pairs->event))
    return fail(c, GPET_ERR_ARG, "surrogate pairs: null pair array");
  (void)hipSetDevice(c->device);
  RunArgs A;
  s = run_args(c, first, n, seed, instance, A);
  if (s) return s;
  set_hits(A, h);
  A.sur = P;
  A.px = pairs->x;
  A.plabel = pairs->label;
  A.pflags = pairs->flags;
  A.pevent = pairs->event;
  A.pcount = c->d_ctrl + kCtrlPairWord;
  A.pcap = pairs->capacity;
  s = run_transport(c, A, c->shape, h, stats, kModeRecord);
  pairs->count = c->h_ctrl[kCtrlPairWord];
  if (s) return s;
  if (pairs->count > pairs->capacity) return fail(c, GPET_ERR_CAPACITY, "surrogate pairs: pair capacity too small");
  return GPET_OK;
}

// the entry queue for `cap` entries
static gpet_status ensure_queue(gpet_ctx *c, size_t cap) {
  SurQueue &Q = c->squeue;
  if (Q.cap >= cap) return GPET_OK;
  if (Q.blob) (void)hipFree(Q.blob);
  Q = SurQueue{};
  const size_t tmp = scan_tmp_words(cap);
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t bytes = al(cap * 24) + al(cap * 4) * 6 + al(cap * 4 * kMaxLayers) + al(cap * 8) + al(tmp * 4);
  if (hipMalloc(&Q.blob, bytes) != hipSuccess) {
    Q.blob = nullptr;
    return fail(c, GPET_ERR_HIP, "surrogate: queue allocation failed");
  }
  char *p = (char *)Q.blob;
  auto take = [&](size_t b) {
    char *r = p;
    p += al(b);
    return (void *)r;
  };
  Q.x = (float *)take(cap * 24);
  Q.e = (float *)take(cap * 4);
  Q.ev = (uint32_t *)take(cap * 4);
  Q.meta = (uint32_t *)take(cap * 4);
  Q.cls = (uint32_t *)take(cap * 4);
  Q.pos = (uint32_t *)take(cap * 4);
  Q.anchor = (uint32_t *)take(cap * 4 * kMaxLayers);
  Q.time = (unsigned long long *)take(cap * 8);
  Q.scan_tmp = (uint32_t *)take(tmp * 4);
  Q.cap = cap;
  return GPET_OK;
}

gpet_status gpet_surrogate_transport(gpet_ctx *c, gpet_mlp *q, const gpet_surrogate_spec *spec, uint64_t first,
                                     uint64_t n, uint64_t seed, uint32_t instance, gpet_hits *h, gpet_stats *stats,
                                     gpet_surrogate_stats *ss) {
  gpet_status s = ready(c);
  if (s) return s;
  SurSpecD P;
  int n_classes = 0;
  s = surrogate_spec(c, spec, P, n_classes);
  if (s) return s;
  if (!q || q->ctx != c) return fail(c, GPET_ERR_ARG, "surrogate: network missing or made on another context");
  if (q->n_first) {
    const int W = 2 * P.chalf + 1;
    if (c->scene.n_layers * ((W * W + 63) / 64) > 32)
      return fail(c, GPET_ERR_UNSUPPORTED,
                  "surrogate: at most 32 chunks of 64 positions per block (layers x ceil((2 H + 1)^2 / 64))");
    if (q->size[0] != 6 || q->n_first != spec->n_ebins + 2 || q->n_second != c->scene.n_layers * W * W)
      return fail(c, GPET_ERR_ARG, "surrogate: a factored network must map 6 features to " +
                                       std::to_string(spec->n_ebins + 2) + " energy classes and " +
                                       std::to_string(c->scene.n_layers * W * W) + " positions per block");
  } else if (q->size[0] != 6 || q->size[q->n_layers] != n_classes) {
    return fail(c, GPET_ERR_ARG, "surrogate: the network must map 6 features to " + std::to_string(n_classes) +
                                     " classes for this scanner and spec");
  } else if (P.chalf != P.half) {
    return fail(c, GPET_ERR_ARG, "surrogate: a class neighbourhood wider than the domain's needs a factored network");
  }
  if (!h) return fail(c, GPET_ERR_ARG, "surrogate: null hits");
  if (n > 0x7fffffffull || first + n > 0x100000000ull) return fail(c, GPET_ERR_ARG, "surrogate: event range");
  if (!hits_ok(h)) return fail(c, GPET_ERR_ARG, "surrogate: null hit array");
  (void)hipSetDevice(c->device);
  constexpr uint64_t kSlice = 32u << 20; // most events per transport launch (queue of 2 per event, 72 B each)
  // equal slices (no short last launch whose tail would leave the chip idle)
  const uint64_t n_slices = std::max<uint64_t>(1, (n + kSlice - 1) / kSlice);
  const uint64_t slice = (n + n_slices - 1) / n_slices;
  s = ensure_queue(c, (size_t)2 * std::min<uint64_t>(std::max<uint64_t>(n, 1), kSlice));
  if (s) return s;
  const SurQueue &Q = c->squeue;
  hipEvent_t ev[4];
  for (hipEvent_t &e : ev)
    if (hipEventCreate(&e) != hipSuccess) return fail(c, GPET_ERR_HIP, "surrogate: event creation failed");
  float ms_t = 0.f, ms_n = 0.f;
  uint64_t entries = 0, none = 0;
  reset_ctrl(c, c->stream);
  for (uint64_t off = 0; off < n && !s; off += slice) {
    const uint64_t len = std::min(slice, n - off);
    RunArgs A;
    s = run_args(c, first + off, len, seed, instance, A);
    if (s) break;
    set_hits(A, h);
    A.sur = P;
    A.px = Q.x;
    A.qev = Q.ev;
    A.qmeta = Q.meta;
    A.qanchor = Q.anchor;
    A.qe = Q.e;
    A.qtime = Q.time;
    A.pcount = c->d_ctrl + kCtrlPairWord;
    A.pholes = c->d_ctrl + kCtrlPairWord + 1;
    A.pcap = Q.cap;
    launch_fill_u32((uint32_t *)(c->d_ctrl + kCtrlWorkWord), 0u, 2, c->stream); // event-chunk counter
    launch_fill_u32((uint32_t *)(c->d_ctrl + kCtrlPairWord), 0u, 4, c->stream); // queue slots, empty slots
    (void)hipEventRecord(ev[0], c->stream);
    launch_transport(A, c->shape, c->n_cu, c->stream, kModeSurrogate);
    (void)hipEventRecord(ev[1], c->stream);
    s = hip_check(c, hipGetLastError(), "surrogate: transport launch");
    if (!s) s = hip_check(c, hipMemcpyAsync(c->h_ctrl + kCtrlPairWord, c->d_ctrl + kCtrlPairWord, 16, hipMemcpyDeviceToHost, c->stream),
                          "surrogate: readback");
    if (!s) s = hip_check(c, wait_stream(c->stream), "surrogate: transport");
    if (s) break;
    const uint64_t nq = c->h_ctrl[kCtrlPairWord];
    if (nq > Q.cap) {
      s = fail(c, GPET_ERR_HIP, "surrogate: entry queue overflow");
      break;
    }
    const uint64_t holes = c->h_ctrl[kCtrlPairWord + 1];
    entries += nq - holes;
    (void)hipEventRecord(ev[2], c->stream);
    const int r = surrogate_hits(q, (const DevScene *)c->d_plain, P, Q, (uint32_t)nq, A.k0, A.k1, instance, A,
                                 c->stream, c->err, &none);
    none -= holes; // empty slots draw no class
    (void)hipEventRecord(ev[3], c->stream);
    if (r != GPET_OK) {
      s = r;
      break;
    }
    s = hip_check(c, wait_stream(c->stream), "surrogate: network");
    float a = 0.f, b = 0.f;
    (void)hipEventElapsedTime(&a, ev[0], ev[1]);
    (void)hipEventElapsedTime(&b, ev[2], ev[3]);
    ms_t += a;
    ms_n += b;
  }
  for (hipEvent_t &e : ev) (void)hipEventDestroy(e);
  if (s) return s;
  s = hip_check(c, hipMemcpy(c->h_ctrl, c->d_ctrl, kCtrlWords * 8, hipMemcpyDeviceToHost), "surrogate: readback");
  if (s) return s;
  h->count = c->h_ctrl[1];
  if (stats) {
    uint64_t *o = (uint64_t *)stats;
    for (int k = 0; k < kStatCount; ++k) o[k] = c->h_ctrl[2 + k];
  }
  if (ss) {
    ss->entries = entries;
    ss->none = none;
    ss->ms_transport = ms_t;
    ss->ms_network = ms_n;
  }
  c->last_ms[0] = ms_t;
  if (h->count > h->capacity) return fail(c, GPET_ERR_CAPACITY, "surrogate: hit capacity too small");
  return GPET_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// chunk table of the batch for its current chunk size, uploaded to the device
static gpet_status batch_prefix(gpet_batch *b) {
  gpet_ctx *c = b->ctx;
  std::vector<uint32_t> prefix(b->n + 1, 0);
  uint64_t acc = 0;
  for (uint32_t i = 0; i < b->n; ++i) {
    prefix[i] = (uint32_t)acc;
    acc += (b->count[i] + b->chunk - 1) / b->chunk;
  }
  if (acc > 0x7fffffffull) return fail(c, GPET_ERR_ARG, "batch: too many chunks (raise the chunk size)");
  prefix[b->n] = (uint32_t)acc;
  b->base.total_chunks = (uint32_t)acc;
  b->base.chunk = b->chunk;
  gpet_status s = hip_check(c, hipMemcpyAsync(b->d_prefix, prefix.data(), prefix.size() * 4, hipMemcpyHostToDevice,
                                              c->stream), "batch: table upload");
  return s ? s : hip_check(c, hipStreamSynchronize(c->stream), "batch: table upload");
}

gpet_status gpet_batch_create(gpet_ctx *c, int32_t n, const gpet_instance *inst, gpet_batch **out) {
  if (!c || !out) return GPET_ERR_ARG;
  *out = nullptr;
  if (n < 1 || n > 65536 || !inst) return fail(c, GPET_ERR_ARG, "batch: instance count in 1..65536");
  if (c->n_mat == 0) return fail(c, GPET_ERR_STATE, "batch: set materials first");
  std::vector<GeomBuild> G(n);
  std::vector<DevScene> S(n);
  std::vector<std::vector<float>> rods(n), cum(n);
  std::vector<int> slot_mat;
  std::vector<bool> used(c->n_mat, false);
  gpet_batch *b = new (std::nothrow) gpet_batch();
  if (!b) return fail(c, GPET_ERR_ARG, "batch: out of host memory");
  b->ctx = c;
  b->device = c->device;
  b->n = (uint32_t)n;
  b->shape = c->shape;
  for (int i = 0; i < n; ++i) {
    const std::string who = "batch instance " + std::to_string(i) + ": ";
    gpet_status s = GPET_OK;
    if (inst[i].n_events > 0x7fffffffull || inst[i].first_event + inst[i].n_events > 0x100000000ull)
      s = fail(c, GPET_ERR_ARG, who + "event range");
    if (!s) s = build_geometry(c, inst[i].scanner, slot_mat, G[i], who + "geometry: ");
    S[i] = c->scene; // materials, phantom
    if (!s) s = build_source(c, inst[i].source, S[i], rods[i], cum[i], who + "source: ");
    if (s) {
      delete b;
      return s;
    }
    set_geometry_fields(S[i], G[i].S);
    for (int m = 0; m < c->n_mat; ++m)
      if (G[i].used[m]) used[m] = true;
    b->info.push_back(G[i].info);
    b->first.push_back((uint32_t)inst[i].first_event);
    b->count.push_back((uint32_t)inst[i].n_events);
    b->id.push_back(inst[i].instance);
    b->cpp.push_back((uint32_t)G[i].info.crystals_per_panel);
    b->cpm.push_back((uint32_t)G[i].info.crystals_per_module);
    b->ncr.push_back((uint32_t)G[i].info.n_crystals);
    layer_words(S[i], b->layers);
    b->duration.push_back(inst[i].source->duration_ps);
    b->gid_bits = std::max(b->gid_bits, bits_for((uint64_t)G[i].info.n_crystals - 1));
    b->total_events += inst[i].n_events;
  }
  std::vector<float4> rows;
  std::vector<float> maj;
  detector_tables(c, slot_mat, used, rows, maj);
  b->det_slots = (int)slot_mat.size();
  // blob layout
  size_t off = align256(n * sizeof(DevScene));
  const size_t off_tab = off;
  off = align256(off + (size_t)(4 * n + 1) * 4);
  const size_t off_rows = off;
  off = align256(off + rows.size() * sizeof(float4));
  const size_t off_maj = off;
  off = align256(off + maj.size() * sizeof(float));
  std::vector<size_t> off_pose(n), off_rods(n), off_cum(n);
  for (int i = 0; i < n; ++i) {
    off_pose[i] = off;
    off = align256(off + G[i].pose.size() * sizeof(float));
    off_rods[i] = off;
    off = align256(off + rods[i].size() * sizeof(float));
    off_cum[i] = off;
    off = align256(off + cum[i].size() * sizeof(float));
  }
  (void)hipSetDevice(c->device);
  if (hipMalloc((void **)&b->d_blob, off) != hipSuccess) {
    delete b;
    return fail(c, GPET_ERR_HIP, "batch: device allocation failed");
  }
  std::vector<char> blob(off, 0);
  char *d = b->d_blob;
  for (int i = 0; i < n; ++i) {
    DevScene &T = S[i];
    T.pose = (const float *)(d + off_pose[i]);
    T.mu_det = (const float4 *)(d + off_rows);
    T.maj_det = (const float *)(d + off_maj);
    T.n_det_slots = b->det_slots;
    T.rods = rods[i].empty() ? nullptr : (const float *)(d + off_rods[i]);
    T.rod_cum = rods[i].empty() ? nullptr : (const float *)(d + off_cum[i]);
    std::memcpy(blob.data() + (size_t)i * sizeof(DevScene), &T, sizeof(DevScene));
    std::memcpy(blob.data() + off_pose[i], G[i].pose.data(), G[i].pose.size() * sizeof(float));
    if (!rods[i].empty()) {
      std::memcpy(blob.data() + off_rods[i], rods[i].data(), rods[i].size() * sizeof(float));
      std::memcpy(blob.data() + off_cum[i], cum[i].data(), cum[i].size() * sizeof(float));
    }
  }
  uint32_t *tab = (uint32_t *)(blob.data() + off_tab);
  for (int i = 0; i < n; ++i) {
    tab[n + 1 + i] = b->first[i];
    tab[2 * n + 1 + i] = b->count[i];
    tab[3 * n + 1 + i] = b->id[i];
  }
  std::memcpy(blob.data() + off_rows, rows.data(), rows.size() * sizeof(float4));
  std::memcpy(blob.data() + off_maj, maj.data(), maj.size() * sizeof(float));
  if (hipMemcpy(b->d_blob, blob.data(), off, hipMemcpyHostToDevice) != hipSuccess) {
    gpet_batch_destroy(b);
    return fail(c, GPET_ERR_HIP, "batch: upload failed");
  }
  RunArgs &A = b->base;
  const uint32_t *dtab = (const uint32_t *)(d + off_tab);
  b->d_prefix = (uint32_t *)(d + off_tab);
  A.scenes = (const DevScene *)d;
  A.chunk_prefix = dtab;
  A.inst_first = dtab + n + 1;
  A.inst_count = dtab + 2 * n + 1;
  A.inst_id = dtab + 3 * n + 1;
  A.n_inst = (uint32_t)n;
  A.work = (uint32_t *)(c->d_ctrl + kCtrlWorkWord);
  A.hit_count = c->d_ctrl + 1;
  A.stats = c->d_ctrl + 2;
  b->mat_gen = c->mat_gen;
  b->phantom_gen = c->phantom_gen;
  gpet_status s = batch_prefix(b);
  if (s) {
    gpet_batch_destroy(b);
    return s;
  }
  *out = b;
  return GPET_OK;
}

void gpet_batch_destroy(gpet_batch *b) {
  if (!b) return;
  if (b->d_blob || b->graph) { // the context may be gone already: touch only the device
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->d_blob) (void)hipFree(b->d_blob);
  }
  delete b;
}

static gpet_status batch_ready(gpet_batch *b) {
  if (!b) return GPET_ERR_ARG;
  if (b->mat_gen != b->ctx->mat_gen || b->phantom_gen != b->ctx->phantom_gen)
    return fail(b->ctx, GPET_ERR_STATE, "batch: the context's materials or phantom changed since the batch was made");
  (void)hipSetDevice(b->ctx->device);
  return GPET_OK;
}

gpet_status gpet_batch_info(gpet_batch *b, int32_t i, gpet_geometry_info *info) {
  if (!b || !info) return GPET_ERR_ARG;
  if (i < 0 || (uint32_t)i >= b->n) return fail(b->ctx, GPET_ERR_ARG, "batch: instance index");
  *info = b->info[i];
  return GPET_OK;
}

gpet_status gpet_batch_set_launch(gpet_batch *b, int32_t blocks_per_cu, int32_t search_batch, uint32_t chunk) {
  if (!b) return GPET_ERR_ARG;
  if (blocks_per_cu < 0 || blocks_per_cu > 64 || search_batch < 1 || search_batch > 64 || chunk < 1 ||
      chunk > (1u << 20))
    return fail(b->ctx, GPET_ERR_ARG, "batch launch: blocks_per_cu in 0..64, search_batch in 1..64, chunk in 1..2^20");
  (void)hipSetDevice(b->ctx->device);
  const uint32_t old = b->chunk;
  b->shape.blocks_per_cu = blocks_per_cu;
  b->shape.search_batch = (uint32_t)search_batch;
  b->chunk = chunk;
  gpet_status s = batch_prefix(b);
  if (s) {
    b->chunk = old;
    (void)batch_prefix(b);
  }
  return s;
}

gpet_status gpet_batch_transport(gpet_batch *b, uint64_t seed, gpet_hits *h, gpet_stats *stats) {
  gpet_status s = batch_ready(b);
  if (s) return s;
  gpet_ctx *c = b->ctx;
  if (!h) return fail(c, GPET_ERR_ARG, "batch transport: null hits");
  if (!hits_ok(h) || (h->capacity && !h->instance)) return fail(c, GPET_ERR_ARG, "batch transport: null hit array");
  RunArgs A = b->base;
  A.k0 = (uint32_t)seed;
  A.k1 = (uint32_t)(seed >> 32);
  A.search_batch = b->shape.search_batch;
  A.schedule = b->shape.schedule;
  set_hits(A, h);
  return run_transport(c, A, b->shape, h, stats);
}

gpet_status gpet_batch_graph_capture(gpet_batch *b, uint64_t seed, gpet_hits *h) {
  gpet_status s = batch_ready(b);
  if (s) return s;
  gpet_ctx *c = b->ctx;
  if (!h) return fail(c, GPET_ERR_ARG, "batch graph: null hits");
  if (!hits_ok(h) || (h->capacity && !h->instance)) return fail(c, GPET_ERR_ARG, "batch graph: null hit array");
  RunArgs A = b->base;
  A.k0 = (uint32_t)seed;
  A.k1 = (uint32_t)(seed >> 32);
  A.search_batch = b->shape.search_batch;
  A.schedule = b->shape.schedule;
  set_hits(A, h);
  hipStream_t cs = nullptr;
  if (hipStreamCreate(&cs) != hipSuccess) return fail(c, GPET_ERR_HIP, "batch graph: stream creation failed");
  hipGraph_t g = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    reset_ctrl(c, cs); // kernels, not memset nodes
    if (A.total_chunks) launch_transport(A, b->shape, c->n_cu, cs);
    ok = hipStreamEndCapture(cs, &g) == hipSuccess && g;
  }
  ok = ok && hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  if (!ok) {
    if (exec) (void)hipGraphExecDestroy(exec);
    return fail(c, GPET_ERR_HIP, "batch graph: capture failed");
  }
  if (b->graph) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipGraphExecDestroy(b->graph);
  }
  b->graph = exec;
  return GPET_OK;
}

gpet_status gpet_batch_graph_launch(gpet_batch *b) {
  gpet_status s = batch_ready(b);
  if (s) return s;
  if (!b->graph) return fail(b->ctx, GPET_ERR_STATE, "batch graph: nothing captured");
  return hip_check(b->ctx, hipGraphLaunch(b->graph, b->ctx->stream), "batch graph: launch");
}

gpet_status gpet_batch_read_counts(gpet_batch *b, gpet_hits *h, gpet_stats *stats) {
  gpet_status s = batch_ready(b);
  if (s) return s;
  gpet_ctx *c = b->ctx;
  if (!h) return fail(c, GPET_ERR_ARG, "batch counts: null hits");
  s = hip_check(c, hipMemcpyAsync(c->h_ctrl, c->d_ctrl, kCtrlWords * 8, hipMemcpyDeviceToHost, c->stream), "batch counts");
  if (!s) s = hip_check(c, wait_stream(c->stream), "batch counts");
  if (s) return s;
  h->count = c->h_ctrl[1];
  if (stats) {
    uint64_t *o = (uint64_t *)stats;
    for (int k = 0; k < kStatCount; ++k) o[k] = c->h_ctrl[2 + k];
  }
  if (h->count > h->capacity) return fail(c, GPET_ERR_CAPACITY, "batch counts: hit capacity too small");
  return GPET_OK;
}

gpet_status gpet_batch_digitize(gpet_batch *b, const gpet_hits *h, const gpet_digitizer *p, gpet_singles *sg,
                                gpet_coincidences *cc, uint64_t *coinc_per_instance) {
  gpet_status s = batch_ready(b);
  if (s) return s;
  gpet_ctx *c = b->ctx;
  DigitizeArgs D;
  s = digitizer_params(c, h, p, sg, cc, D);
  if (s) return s;
  if (b->n > 1 && h->count && !h->instance) return fail(c, GPET_ERR_ARG, "batch digitize: hits need instance ids");
  D.h_inst = b->n > 1 ? h->instance : nullptr;
  D.first = b->first;
  D.n_events = b->count;
  for (uint32_t i = 0; i < b->n; ++i)
    if (D.n_events[i] == 0) D.n_events[i] = 1; // empty instance: no hit can name it
  D.cpp = b->cpp;
  D.cpm = b->cpm;
  D.ncr = b->ncr;
  D.layers = b->layers;
  D.rng = b->id;
  D.duration = b->duration;
  D.gid_bits = b->gid_bits;
  D.coinc_per_inst = (unsigned long long *)coinc_per_instance;
  return timed_digitize(c, D);
}

gpet_status gpet_batch_autotune(gpet_batch *b, uint64_t seed, gpet_hits *h, char *json, size_t cap) {
  gpet_status s = batch_ready(b);
  if (s) return s;
  gpet_ctx *c = b->ctx;
  const bool timing = c->timing;
  s = gpet_ctx_enable_timing(c, 1);
  if (s) return s;
  struct Trial {
    int bpc, sb;
    uint32_t chunk;
    float ms;
  };
  std::vector<Trial> trials;
  Trial best{b->shape.blocks_per_cu, (int)b->shape.search_batch, b->chunk, 1e30f};
  auto run = [&](int bpc, int sb, uint32_t chunk) -> gpet_status {
    gpet_status r = gpet_batch_set_launch(b, bpc, sb, chunk);
    if (!r) r = gpet_batch_transport(b, seed, h, nullptr);
    if (r) return r;
    const float ms = c->last_ms[0];
    trials.push_back({bpc, sb, chunk, ms});
    if (ms < best.ms) best = {bpc, sb, chunk, ms};
    return GPET_OK;
  };
  s = gpet_batch_transport(b, seed, h, nullptr); // warm-up
  const int bpcs[] = {0, 2, 4};
  const int sbs[] = {8, 16, 24, 32, 48};
  const uint32_t chunks[] = {64, 256, 1024, 4096};
  for (uint32_t ch : chunks)
    if (!s) s = run(best.bpc, best.sb, ch);
  const uint32_t ch_best = best.chunk;
  for (int sb : sbs)
    if (!s) s = run(best.bpc, sb, ch_best);
  const int sb_best = best.sb;
  for (int bpc : bpcs)
    if (!s) s = run(bpc, sb_best, ch_best);
  c->timing = timing;
  if (s) return s;
  s = gpet_batch_set_launch(b, best.bpc, best.sb, best.chunk);
  if (s) return s;
  if (json && cap) {
    std::string j = "{\"blocks_per_cu\": " + std::to_string(best.bpc) + ", \"search_batch\": " +
                    std::to_string(best.sb) + ", \"chunk\": " + std::to_string(best.chunk) +
                    ", \"ms\": " + std::to_string(best.ms) + ", \"trials\": [";
    for (size_t k = 0; k < trials.size(); ++k) {
      if (k) j += ", ";
      j += "[" + std::to_string(trials[k].bpc) + ", " + std::to_string(trials[k].sb) + ", " +
           std::to_string(trials[k].chunk) + ", " + std::to_string(trials[k].ms) + "]";
    }
    j += "]}";
    const size_t m = std::min(cap - 1, j.size());
    std::memcpy(json, j.data(), m);
    json[m] = '\0';
  }
  return GPET_OK;
}

} // extern "C"
