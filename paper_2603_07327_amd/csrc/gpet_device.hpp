// gpet_device.hpp -- device-side scene layout and FP32 primitives of the
// multi-layer PET transport (gfx950).
//
// Everything here runs per lane in FP32: counter-based Philox streams,
// attenuation-table interpolation, panel search, the hierarchical locate with
// layer selection by depth (paper Sec. 2.1), Compton (Kahn) and Rayleigh
// (Thomson) sampling and the direction update.  The hot path is free of IEEE
// division sequences: reciprocals of geometric constants are precomputed on
// the host, and the remaining ones use the hardware reciprocal (1 ulp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpet {

constexpr int kNodes = 511;     // energy nodes 1..511 keV
constexpr int kTabStride = 512; // padded row length of a table
constexpr float kMec2 = 510.99895f;
constexpr float kInvMec2 = 1.0f / 510.99895f;
constexpr float kInvCmmPerPs = 1.0f / 0.299792458f; // ps per mm
constexpr float kLn2 = 0.69314718055994531f;
constexpr int kMaxSteps = 1 << 20;
constexpr int kMaxLayers = 4;

// single-instruction hardware approximations (about 1 ulp)
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Value of lane (lane ^ lx) for lx in {1, 2, 4, 8, 16, 32} without the LDS
// crossbar: DPP quad permutes (1, 2), row shifts (4), a row rotation (8) and
// the gfx950 half-row / half-wave swaps (16, 32).  lx must fold to a constant.
__device__ __forceinline__ uint32_t lane_xor(uint32_t x, int lx) {
  const uint32_t lane = __lane_id();
  switch (lx) {
  case 1:
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false); // quad_perm [1,0,3,2]
  case 2:
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false); // quad_perm [2,3,0,1]
  case 4: {
    const uint32_t up = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x104, 0xF, 0xF, false); // lane + 4
    const uint32_t dn = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false); // lane - 4
    return (lane & 4u) ? dn : up;
  }
  case 8:
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xF, 0xF, false); // row_ror:8
  case 16: {
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return (lane & 16u) ? r[0] : r[1];
  }
  case 32: {
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (lane & 32u) ? r[0] : r[1];
  }
  default:
    return (uint32_t)__shfl_xor((int)x, lx);
  }
}

__device__ __forceinline__ float lane_xor_f(float x, int lx) {
  return __uint_as_float(lane_xor(__float_as_uint(x), lx));
}
__device__ __forceinline__ float neg_ln(float u) { return -kLn2 * __builtin_amdgcn_logf(u); } // -ln u
// sine and cosine of 2*pi*u for u in revolutions
__device__ __forceinline__ float sin_rev(float u) { return __builtin_amdgcn_sinf(u); }
__device__ __forceinline__ float cos_rev(float u) { return __builtin_amdgcn_cosf(u); }

struct LayerD {
  float d0, d1;                 // depth range [d0, d1)
  float off_t, off_a;           // crystal array start from the module edge
  float pitch_t, pitch_a;
  float inv_pitch_t, inv_pitch_a;
  float lo_t, hi_t, lo_a, hi_a; // crystal extent inside its pitch cell
  int n_t, n_a;
  int mat_crystal, mat_interval;
  int slot_crystal, slot_interval; // rows of the detector attenuation table
  int base;                        // first crystal id of the layer inside a module
  int pad_;
};

// Everything a kernel needs about one scene (one instance of a batch).  The
// transport kernel reads it through a wave-uniform pointer in the constant
// address space, so its fields are scalar loads; large arrays stay in device
// memory.
struct DevScene {
  // panels
  int n_panels;
  int ring; // all panels have axial axis +z and one common axial offset
  // repeated ring (evenly spaced panels, front faces at one radius): searches
  // from inside the front-face radius test only the panels whose azimuth
  // range the ray sweeps while between that radius and the outer one
  int ring_reg;
  float ring_R2, ring_rmax2; // squared front-face radius (shrunk by 2e-6) and outer corner radius
  float ring_n, ring_u0;     // panels per turn; panel 0's azimuth in panel units
  float ring_a;              // half azimuth span of a panel in panel units, plus the azimuth error bound
  float depth, half_w, half_l;
  // n_panels x 12: rows of the local axes (depth, t, a) in global coordinates,
  // then the front-face centre projected on them; local = R x - R o
  const float *pose;
  // modules
  int mod_n_t, mod_n_a;
  float mod_t0, mod_a0;         // start of the module array (local t, a)
  float mod_step_t, mod_step_a; // module size + gap
  float inv_step_t, inv_step_a;
  float mod_t, mod_a; // module size
  int fill, fill_slot;
  int n_layers;
  LayerD layer[kMaxLayers];
  int crystals_per_module, crystals_per_panel;
  // attenuation (1/mm): per material rows of kTabStride float4 (PE, Compton, Rayleigh, total)
  const float4 *mu;      // at the nominal density
  const float4 *mu_det;  // the detector's materials, one row per slot
  int n_det_slots;
  const float4 *mu_mass; // per g/cm^3
  const float *maj_det;  // detector majorant
  const float *maj_ph;   // phantom majorant
  float e_cut;
  // phantom
  int has_phantom;
  int nx, ny, nz;
  float ox, oy, oz;    // origin
  float ivx, ivy, ivz; // inverse voxel size
  float bx, by, bz;    // upper corner of the box
  const uint8_t *vmat;
  const float *vden;
  // source
  int src_kind;
  float sx, sy, sz, bdx, bdy, bdz;
  int n_rods;
  const float *rods;    // n_rods x 5: cx, cy, radius, z0, z1
  const float *rod_cum; // cumulative rod weights
  float rod_total;
  unsigned long long duration_ps;
  float acol_sigma;   // acollinearity: sigma of each transverse angle component (rad), 0 = off
  float prange_sigma; // positron range: sigma of each offset component (mm), 0 = off
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): counter (block, event, instance,
// stream), key = seed.  Each round's two 32x32 products are single 64-bit
// multiplies (v_mad_u64_u32).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t k0, uint32_t k1, uint4 c) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const unsigned long long p0 = (unsigned long long)0xD2511F53u * c.x;
    const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
                   (uint32_t)p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// odd multiple of 2^-24: exact in FP32, strictly inside (0, 1)
__device__ __forceinline__ float to_unit(uint32_t w) {
  return (float)(((w >> 9) << 1) | 1u) * 5.9604644775390625e-8f;
}
__device__ __forceinline__ float4 to_unit4(uint4 w) {
  return make_float4(to_unit(w.x), to_unit(w.y), to_unit(w.z), to_unit(w.w));
}

struct Stream {
  uint32_t k0, k1, event, instance, id, n;
  __device__ __forceinline__ float4 next() {
    const uint4 o = philox(k0, k1, make_uint4(n, event, instance, id));
    ++n;
    return to_unit4(o);
  }
};

// ---------------------------------------------------------------------------
// Tables: linear interpolation on 1 keV nodes, j = clamp(floor(E), 1, 510).
// ---------------------------------------------------------------------------
struct Lerp {
  int j;   // index of the upper node (node energy j+1)
  float f; // weight of the upper node
};
__device__ __forceinline__ Lerp lerp_at(float e) {
  float jf = floorf(e);
  jf = fminf(fmaxf(jf, 1.0f), 510.0f);
  return Lerp{(int)jf, e - jf};
}
__device__ __forceinline__ float lerp1(const float *t, Lerp l) {
  return (1.0f - l.f) * t[l.j - 1] + l.f * t[l.j];
}
__device__ __forceinline__ float4 lerp4(const float4 *t, int m, Lerp l) {
  const float4 a = t[m * kTabStride + l.j - 1], b = t[m * kTabStride + l.j];
  const float g = 1.0f - l.f;
  return make_float4(g * a.x + l.f * b.x, g * a.y + l.f * b.y, g * a.z + l.f * b.z,
                     g * a.w + l.f * b.w);
}

// ---------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------
struct Vec {
  float x, y, z;
};
typedef __attribute__((address_space(4))) const float CFloat; // read-only view (scalar loads when uniform)
template <class PT> __device__ __forceinline__ Vec to_local(PT P, Vec g) {
  return Vec{g.x * P[0] + g.y * P[1] + g.z * P[2] - P[9], g.x * P[3] + g.y * P[4] + g.z * P[5] - P[10],
             g.x * P[6] + g.y * P[7] + g.z * P[8] - P[11]};
}
template <class PT> __device__ __forceinline__ Vec dir_to_local(PT P, Vec d) {
  return Vec{d.x * P[0] + d.y * P[1] + d.z * P[2], d.x * P[3] + d.y * P[4] + d.z * P[5],
             d.x * P[6] + d.y * P[7] + d.z * P[8]};
}
template <class PT> __device__ __forceinline__ Vec to_global(PT P, Vec l) {
  const float a = l.x + P[9], b = l.y + P[10], c = l.z + P[11];
  return Vec{a * P[0] + b * P[3] + c * P[6], a * P[1] + b * P[4] + c * P[7], a * P[2] + b * P[5] + c * P[8]};
}
template <class PT> __device__ __forceinline__ Vec dir_to_global(PT P, Vec l) {
  return Vec{l.x * P[0] + l.y * P[3] + l.z * P[6], l.x * P[1] + l.y * P[4] + l.z * P[7],
             l.x * P[2] + l.y * P[5] + l.z * P[8]};
}

template <class SC> __device__ __forceinline__ bool inside_panel(SC &S, Vec l) {
  return l.x >= 0.0f && l.x < S.depth && l.y >= -S.half_w && l.y < S.half_w && l.z >= -S.half_l &&
         l.z < S.half_l;
}

// One axis of a slab test: entry/exit parameters of the ray o + t d against
// [lo, hi]; a ray parallel to the slab is kept (whole line) when its origin
// lies inside and rejected otherwise.
__device__ __forceinline__ void slab_axis(float o, float d, float lo, float hi, float &tn, float &tf) {
  float t1, t2;
  if (d == 0.0f) {
    t1 = -INFINITY;
    t2 = (o >= lo && o <= hi) ? INFINITY : -INFINITY;
  } else {
    const float inv = rcp(d);
    t1 = (lo - o) * inv;
    t2 = (hi - o) * inv;
  }
  tn = fmaxf(tn, fminf(t1, t2));
  tf = fminf(tf, fmaxf(t1, t2));
}

// Slab test against [lo, hi] per axis; entry distance clamped at 0 (a start
// inside counts as entering at once).
__device__ __forceinline__ bool ray_box(Vec o, Vec d, Vec lo, Vec hi, float &t_enter) {
  float tn = -INFINITY, tf = INFINITY;
  slab_axis(o.x, d.x, lo.x, hi.x, tn, tf);
  slab_axis(o.y, d.y, lo.y, hi.y, tn, tf);
  slab_axis(o.z, d.z, lo.z, hi.z, tn, tf);
  if (tn > tf || tf <= 0.0f) return false;
  t_enter = fmaxf(tn, 0.0f);
  return true;
}

// Line-plane projection to the panels (Sec. 2.1): nearest panel box along
// the ray, excluding the panel just left; ties to the lower index.
template <class SC> __device__ __forceinline__ int panel_search(SC &S, Vec x, Vec d, int exclude, float &t_in) {
  int best = -1;
  float bt = INFINITY;
  const Vec lo{0.0f, -S.half_w, -S.half_l}, hi{S.depth, S.half_w, S.half_l};
  for (int p = 0; p < S.n_panels; ++p) {
    CFloat *P = (CFloat *)(S.pose + 12 * p);
    float te;
    if (ray_box(to_local(P, x), dir_to_local(P, d), lo, hi, te) && p != exclude && te < bt) {
      bt = te;
      best = p;
    }
  }
  t_in = bt;
  return best;
}

// Panel search for rings: every panel's axial axis is +z and all panels share
// one axial range, so the axial slab is computed once for the ray and the
// depth/tangential axes need only 2-D dot products (pose rows have zero z).
template <class SC>
__device__ __forceinline__ int panel_search_ring(SC &S, Vec x, Vec d, int exclude, float &t_in) {
  float tn_a = -INFINITY, tf_a = INFINITY;
  slab_axis(x.z - ((CFloat *)S.pose)[11], d.z, -S.half_l, S.half_l, tn_a, tf_a);
  int best = -1;
  float bt = INFINITY;
  for (int p = 0; p < S.n_panels; ++p) {
    CFloat *P = (CFloat *)(S.pose + 12 * p);
    float tn = tn_a, tf = tf_a;
    slab_axis(x.x * P[0] + x.y * P[1] - P[9], d.x * P[0] + d.y * P[1], 0.0f, S.depth, tn, tf);
    slab_axis(x.x * P[3] + x.y * P[4] - P[10], d.x * P[3] + d.y * P[4], -S.half_w, S.half_w, tn, tf);
    const float te = fmaxf(tn, 0.0f);
    if (tn <= tf && tf > 0.0f && p != exclude && te < bt) {
      bt = te;
      best = p;
    }
  }
  t_in = bt;
  return best;
}

// Azimuth of (x, y) in turns, (-1/2, 1/2]: octant reduction and the
// arctangent approximation atan(z) ~ z (pi/4 + 0.273 (1 - z)) on [0, 1]
// (Rajan et al., IEEE Signal Processing Magazine 2006), whose error stays
// below 0.0038 rad = 6.0e-4 turn.
__device__ __forceinline__ float azimuth_turns(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float z = fminf(ax, ay) * rcp(fmaxf(fmaxf(ax, ay), 1e-30f));
  float t = z * (0.125f + 0.0434494f * (1.0f - z));
  if (ay > ax) t = 0.25f - t;
  if (x < 0.0f) t = 0.5f - t;
  return y < 0.0f ? -t : t;
}

// The ring search restricted to candidate panels (same tests, same result)
// for a repeated ring.  Every point of panel k lies within atan(w / 2R) of
// k's axis in azimuth and at a radius in [R, r_max].  Along the ray the
// azimuth changes monotonically (the line does not wrap around the axis), so
// only panels whose azimuth range meets the sweep of the part of the ray that
// can still lie in that radius band are candidates: from the ray's start (or
// its first crossing of R when it starts inside R, or of r_max when it starts
// beyond) to its last exit through r_max.  u is the azimuth in panel units;
// ring_a includes the azimuth approximation's error.  A sweep of nearly half
// a turn (a ray passing by the axis) takes the full search.  Ties keep the
// lower index as in the full search.
template <class SC>
__device__ __forceinline__ int panel_search_ring_pruned(SC &S, Vec x, Vec d, int exclude, float &t_in, int &tested) {
  tested = 0;
  t_in = INFINITY;
  const float a = d.x * d.x + d.y * d.y, b = x.x * d.x + x.y * d.y, c0 = x.x * x.x + x.y * x.y;
  float ta = 0.0f, tb = 0.0f;
  if (!(a > 1e-20f)) {
    // parallel to the axis: the radius stays put
    if (c0 < S.ring_R2 || c0 > S.ring_rmax2) return -1;
  } else {
    const float inv_a = rcp(a);
    const float disc = b * b - a * (c0 - S.ring_rmax2);
    if (!(disc >= 0.0f)) return -1; // never within r_max
    const float sq = hw_sqrt(disc);
    tb = (-b + sq) * inv_a;
    if (tb < 0.0f) return -1; // only moves away beyond r_max
    if (c0 < S.ring_R2) ta = (-b + hw_sqrt(fmaxf(b * b - a * (c0 - S.ring_R2), 0.0f))) * inv_a;
    else ta = fmaxf((-b - sq) * inv_a, 0.0f);
  }
  const float z1 = azimuth_turns(x.y + ta * d.y, x.x + ta * d.x);
  float dz = azimuth_turns(x.y + tb * d.y, x.x + tb * d.x) - z1;
  dz = dz > 0.5f ? dz - 1.0f : (dz < -0.5f ? dz + 1.0f : dz);
  if (fabsf(dz) > 0.45f) {
    tested = S.n_panels;
    return panel_search_ring(S, x, d, exclude, t_in);
  }
  const float u1 = z1 * S.ring_n - S.ring_u0, u2 = u1 + dz * S.ring_n;
  const int k0 = (int)ceilf(fminf(u1, u2) - S.ring_a), k1 = (int)floorf(fmaxf(u1, u2) + S.ring_a);
  float tn_a = -INFINITY, tf_a = INFINITY;
  slab_axis(x.z - ((CFloat *)S.pose)[11], d.z, -S.half_l, S.half_l, tn_a, tf_a);
  int best = -1;
  float bt = INFINITY;
  const int n = S.n_panels;
  for (int k = k0; k <= k1 && k < k0 + n; ++k) {
    int p = k % n;
    if (p < 0) p += n;
    CFloat *P = (CFloat *)(S.pose + 12 * p);
    float tn = tn_a, tf = tf_a;
    slab_axis(x.x * P[0] + x.y * P[1] - P[9], d.x * P[0] + d.y * P[1], 0.0f, S.depth, tn, tf);
    slab_axis(x.x * P[3] + x.y * P[4] - P[10], d.x * P[3] + d.y * P[4], -S.half_w, S.half_w, tn, tf);
    const float te = fmaxf(tn, 0.0f);
    if (tn <= tf && tf > 0.0f && p != exclude && (te < bt || (te == bt && p < best))) {
      bt = te;
      best = p;
    }
    ++tested;
  }
  t_in = bt;
  return best;
}

// The transport's panel search: the pruned ring search for a repeated ring,
// the full ring or general search otherwise; `tested` counts panel boxes.
template <class SC> __device__ __forceinline__ int search_panels(SC &S, Vec x, Vec d, int exclude, float &t_in,
                                                                 int &tested) {
  if (S.ring_reg) return panel_search_ring_pruned(S, x, d, exclude, t_in, tested);
  tested = S.n_panels;
  return S.ring ? panel_search_ring(S, x, d, exclude, t_in) : panel_search(S, x, d, exclude, t_in);
}

template <class SC> __device__ __forceinline__ int find_panel(SC &S, Vec x, Vec d, int exclude, float &t_in) {
  return S.ring ? panel_search_ring(S, x, d, exclude, t_in) : panel_search(S, x, d, exclude, t_in);
}

struct Loc {
  int mat, slot, module, layer, crystal, gid;
};

typedef __attribute__((address_space(4))) const DevScene CScene; // constant-address-space view

// Hierarchical locate in panel p at local (depth, t, a): module grid, then
// the layer selected by depth, then that layer's crystal array.
template <class SC> __device__ __forceinline__ Loc locate(SC &S, int p, Vec l) {
  const float mt = floorf((l.y - S.mod_t0) * S.inv_step_t);
  const float ma = floorf((l.z - S.mod_a0) * S.inv_step_a);
  const float ut = l.y - S.mod_t0 - mt * S.mod_step_t;
  const float ua = l.z - S.mod_a0 - ma * S.mod_step_a;
  const bool in_mod = !(mt < 0.0f || mt >= (float)S.mod_n_t || ma < 0.0f || ma >= (float)S.mod_n_a ||
                        ut >= S.mod_t || ua >= S.mod_a);
  // the layer holding the depth (the lowest matching layer wins), then its
  // fields, loaded lane by lane from the scene's layer table (those of layer 0
  // where no layer matches: they are not used then)
  int L = -1;
#pragma unroll
  for (int k = kMaxLayers - 1; k >= 0; --k)
    if (k < S.n_layers) L = (l.x >= S.layer[k].d0 && l.x < S.layer[k].d1) ? k : L;
  const auto &y = S.layer[L < 0 ? 0 : L];
  const int nt = y.n_t, na = y.n_a, mat_c = y.mat_crystal, slot_c = y.slot_crystal, mat_i = y.mat_interval,
            slot_i = y.slot_interval, base = y.base;
  const float off_t = y.off_t, off_a = y.off_a, ipt = y.inv_pitch_t, ipa = y.inv_pitch_a, pt = y.pitch_t,
              pa = y.pitch_a, lo_t = y.lo_t, hi_t = y.hi_t, lo_a = y.lo_a, hi_a = y.hi_a;
  const float it = floorf((ut - off_t) * ipt);
  const float ia = floorf((ua - off_a) * ipa);
  const float ct = ut - off_t - it * pt;
  const float ca = ua - off_a - ia * pa;
  const bool has_layer = in_mod && L >= 0;
  const bool crystal = has_layer && !(it < 0.0f || it >= (float)nt || ia < 0.0f || ia >= (float)na) &&
                       !(ct < lo_t || ct >= hi_t || ca < lo_a || ca >= hi_a);
  Loc r;
  r.module = in_mod ? (int)ma * S.mod_n_t + (int)mt : -1;
  r.layer = has_layer ? L : -1;
  r.mat = crystal ? mat_c : has_layer ? mat_i : S.fill;
  r.slot = crystal ? slot_c : has_layer ? slot_i : S.fill_slot;
  r.crystal = crystal ? (int)ia * nt + (int)it : -1;
  r.gid = crystal ? p * S.crystals_per_panel + r.module * S.crystals_per_module + base + r.crystal : -1;
  return r;
}

// voxel index of a global point, -1 outside the phantom box
template <class SC> __device__ __forceinline__ int voxel_of(SC &S, Vec x) {
  const float ix = floorf((x.x - S.ox) * S.ivx);
  const float iy = floorf((x.y - S.oy) * S.ivy);
  const float iz = floorf((x.z - S.oz) * S.ivz);
  if (ix < 0.0f || ix >= (float)S.nx || iy < 0.0f || iy >= (float)S.ny || iz < 0.0f ||
      iz >= (float)S.nz)
    return -1;
  return ((int)iz * S.ny + (int)iy) * S.nx + (int)ix;
}

// ---------------------------------------------------------------------------
// Interactions
// ---------------------------------------------------------------------------
// One trial of Kahn's rejection method for Compton scattering with uniforms
// (r1, r2, r3).  On acceptance returns true with cos(theta) and E' = E / rho.
__device__ __forceinline__ bool kahn_trial(float e, float4 r, float &cos_t, float &e_out) {
  const float a = e * kInvMec2;
  const float b = 1.0f + 2.0f * a;
  float rho, acc;
  if (r.x * (9.0f + 2.0f * a) <= b) {
    rho = 1.0f + 2.0f * a * r.y;
    const float ir = rcp(rho);
    acc = 4.0f * (ir - ir * ir);
  } else {
    rho = b * rcp(1.0f + 2.0f * a * r.y);
    const float c = 1.0f - (rho - 1.0f) * rcp(a);
    acc = 0.5f * (c * c + rcp(rho));
  }
  if (!(r.z <= acc)) return false;
  e_out = e * rcp(rho);
  cos_t = 1.0f - (rho - 1.0f) * rcp(a);
  return true;
}

// Compton scattering: Kahn trials until one is accepted (one block each).
__device__ __forceinline__ float kahn(Stream &rng, float e, float &e_out, int &trials) {
  int n = 0;
  float c = 1.0f;
  for (;;) {
    ++n;
    if (kahn_trial(e, rng.next(), c, e_out)) break;
  }
  trials = n;
  return c;
}

// Thomson angular law: mu^3 + 3 mu = 8u - 4 solved with Cardano's formula.
__device__ __forceinline__ float thomson(float u) {
  const float q = 4.0f * u - 2.0f;
  const float s = sqrtf(q * q + 1.0f);
  return cbrtf(q + s) + cbrtf(q - s);
}

// Direction update for polar cosine c (sine st) and azimuth 2*pi*u_phi about
// the old direction (the reference axis for phi is fixed by the old direction).
__device__ __forceinline__ void rotate_cs(Vec &d, float c, float st, float u_phi) {
  const float sp = sin_rev(u_phi), cp = cos_rev(u_phi);
  const float s2 = d.x * d.x + d.y * d.y;
  Vec n;
  if (s2 < 1e-12f) {
    n = Vec{st * cp, st * sp, (d.z >= 0.0f ? 1.0f : -1.0f) * c};
  } else {
    const float is = rsq(s2), s = s2 * is;
    const float k = st * is;
    n = Vec{d.x * c + k * (d.x * d.z * cp - d.y * sp), d.y * c + k * (d.y * d.z * cp + d.x * sp),
            d.z * c - s * st * cp};
  }
  const float inn = rsq(n.x * n.x + n.y * n.y + n.z * n.z);
  d = Vec{n.x * inn, n.y * inn, n.z * inn};
}
__device__ __forceinline__ void rotate(Vec &d, float c, float u_phi) {
  rotate_cs(d, c, hw_sqrt(fmaxf(0.0f, 1.0f - c * c)), u_phi);
}

// process of a real collision: 1 photoelectric, 2 Compton, 3 Rayleigh
__device__ __forceinline__ int pick_process(float4 mu, float mut, float u) {
  if (u * mut < mu.x) return 1;
  if (u * mut < mu.x + mu.y) return 2;
  return 3;
}

} // namespace gpet
