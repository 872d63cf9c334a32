// gpet_device.hpp -- device-side scene layout and FP32 primitives of the
// multi-layer PET transport (gfx950).
//
// Everything here runs per lane in FP32: counter-based Philox streams,
// attenuation-table interpolation, panel search, the hierarchical locate with
// layer selection by depth (paper Sec. 2.1), Compton (Kahn) and Rayleigh
// (Thomson) sampling and the direction update.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpet {

constexpr int kNodes = 511;     // energy nodes 1..511 keV
constexpr int kTabStride = 512; // padded row length of a table
constexpr float kMec2 = 510.99895f;
constexpr float kCmmPerPs = 0.299792458f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr int kMaxSteps = 1 << 20;
constexpr int kMaxLayers = 4;

struct LayerD {
  float d0, d1;               // depth range [d0, d1)
  float off_t, off_a;         // crystal array start from the module edge
  float pitch_t, pitch_a;
  float lo_t, hi_t, lo_a, hi_a; // crystal extent inside its pitch cell
  int n_t, n_a;
  int mat_crystal, mat_interval;
  int base;                   // first crystal id of the layer inside a module
  int pad_;
};

// Everything a kernel needs about the scene, passed by value as a kernel
// argument (scalar-loaded); large arrays stay in device memory.
struct DevScene {
  // panels
  int n_panels;
  float depth, half_w, half_l;
  const float *pose; // n_panels x 12: origin, e_depth, e_t, e_a
  // modules
  int mod_n_t, mod_n_a;
  float mod_t0, mod_a0;         // start of the module array (local t, a)
  float mod_step_t, mod_step_a; // module size + gap
  float mod_t, mod_a;           // module size
  int fill;
  int n_layers;
  LayerD layer[kMaxLayers];
  int crystals_per_module, crystals_per_panel;
  // attenuation (1/mm): per material rows of kTabStride float4 (PE, Compton, Rayleigh, total)
  const float4 *mu;      // at the nominal density
  const float4 *mu_mass; // per g/cm^3
  const float *maj_det;  // detector majorant
  const float *maj_ph;   // phantom majorant
  float e_cut;
  // phantom
  int has_phantom;
  int nx, ny, nz;
  float ox, oy, oz, vx, vy, vz; // origin and voxel size
  float bx, by, bz;             // upper corner of the box
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
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): counter (block, event, instance,
// stream), key = seed.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t k0, uint32_t k1, uint4 c) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// odd multiple of 2^-24: exact in FP32, strictly inside (0, 1)
__device__ __forceinline__ float to_unit(uint32_t w) {
  return (float)(((w >> 9) << 1) | 1u) * 5.9604644775390625e-8f;
}

struct Stream {
  uint32_t k0, k1, event, instance, id, n;
  __device__ __forceinline__ float4 next() {
    const uint4 o = philox(k0, k1, make_uint4(n, event, instance, id));
    ++n;
    return make_float4(to_unit(o.x), to_unit(o.y), to_unit(o.z), to_unit(o.w));
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
__device__ __forceinline__ Vec to_local(const float *P, Vec g) {
  const float rx = g.x - P[0], ry = g.y - P[1], rz = g.z - P[2];
  return Vec{rx * P[3] + ry * P[4] + rz * P[5], rx * P[6] + ry * P[7] + rz * P[8],
             rx * P[9] + ry * P[10] + rz * P[11]};
}
__device__ __forceinline__ Vec dir_to_local(const float *P, Vec d) {
  return Vec{d.x * P[3] + d.y * P[4] + d.z * P[5], d.x * P[6] + d.y * P[7] + d.z * P[8],
             d.x * P[9] + d.y * P[10] + d.z * P[11]};
}
__device__ __forceinline__ Vec to_global(const float *P, Vec l) {
  return Vec{P[0] + l.x * P[3] + l.y * P[6] + l.z * P[9], P[1] + l.x * P[4] + l.y * P[7] + l.z * P[10],
             P[2] + l.x * P[5] + l.y * P[8] + l.z * P[11]};
}
__device__ __forceinline__ Vec dir_to_global(const float *P, Vec l) {
  return Vec{l.x * P[3] + l.y * P[6] + l.z * P[9], l.x * P[4] + l.y * P[7] + l.z * P[10],
             l.x * P[5] + l.y * P[8] + l.z * P[11]};
}

__device__ __forceinline__ bool inside_panel(const DevScene &S, Vec l) {
  return l.x >= 0.0f && l.x < S.depth && l.y >= -S.half_w && l.y < S.half_w && l.z >= -S.half_l &&
         l.z < S.half_l;
}

// Slab test of a ray against a box [lo, hi] per axis; entry distance
// clamped at 0 (a start inside counts as entering at once).
__device__ __forceinline__ bool ray_box(Vec o, Vec d, Vec lo, Vec hi, float &t_enter) {
  float tn = -INFINITY, tf = INFINITY;
  const float oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
  const float ll[3] = {lo.x, lo.y, lo.z}, hh[3] = {hi.x, hi.y, hi.z};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (dd[k] == 0.0f) {
      if (oo[k] < ll[k] || oo[k] > hh[k]) return false;
      continue;
    }
    const float t1 = (ll[k] - oo[k]) / dd[k], t2 = (hh[k] - oo[k]) / dd[k];
    tn = fmaxf(tn, fminf(t1, t2));
    tf = fminf(tf, fmaxf(t1, t2));
  }
  if (tn > tf || tf <= 0.0f) return false;
  t_enter = fmaxf(tn, 0.0f);
  return true;
}

// Line-plane projection to the panels (Sec. 2.1): nearest panel box along
// the ray, excluding the panel just left; ties to the lower index.
__device__ __forceinline__ int panel_search(const DevScene &S, Vec x, Vec d, int exclude, float &t_in) {
  int best = -1;
  float bt = INFINITY;
  const Vec lo{0.0f, -S.half_w, -S.half_l}, hi{S.depth, S.half_w, S.half_l};
  for (int p = 0; p < S.n_panels; ++p) {
    if (p == exclude) continue;
    const float *P = S.pose + 12 * p;
    float te;
    if (ray_box(to_local(P, x), dir_to_local(P, d), lo, hi, te) && te < bt) {
      bt = te;
      best = p;
    }
  }
  t_in = bt;
  return best;
}

struct Loc {
  int mat, module, layer, crystal, gid;
};

// Hierarchical locate in panel p at local (depth, t, a): module grid, then
// the layer selected by depth, then that layer's crystal array.
__device__ __forceinline__ Loc locate(const DevScene &S, int p, Vec l) {
  Loc r{S.fill, -1, -1, -1, -1};
  const float mt = floorf((l.y - S.mod_t0) / S.mod_step_t);
  const float ma = floorf((l.z - S.mod_a0) / S.mod_step_a);
  const float ut = l.y - S.mod_t0 - mt * S.mod_step_t;
  const float ua = l.z - S.mod_a0 - ma * S.mod_step_a;
  if (mt < 0.0f || mt >= (float)S.mod_n_t || ma < 0.0f || ma >= (float)S.mod_n_a || ut >= S.mod_t ||
      ua >= S.mod_a)
    return r;
  r.module = (int)ma * S.mod_n_t + (int)mt;
  int L = -1;
  for (int k = 0; k < S.n_layers; ++k)
    if (L < 0 && l.x >= S.layer[k].d0 && l.x < S.layer[k].d1) L = k;
  if (L < 0) return r;
  const LayerD &y = S.layer[L];
  r.layer = L;
  r.mat = y.mat_interval;
  const float it = floorf((ut - y.off_t) / y.pitch_t);
  const float ia = floorf((ua - y.off_a) / y.pitch_a);
  const float ct = ut - y.off_t - it * y.pitch_t;
  const float ca = ua - y.off_a - ia * y.pitch_a;
  if (it < 0.0f || it >= (float)y.n_t || ia < 0.0f || ia >= (float)y.n_a) return r;
  if (ct < y.lo_t || ct >= y.hi_t || ca < y.lo_a || ca >= y.hi_a) return r;
  r.mat = y.mat_crystal;
  r.crystal = (int)ia * y.n_t + (int)it;
  r.gid = p * S.crystals_per_panel + r.module * S.crystals_per_module + y.base + r.crystal;
  return r;
}

// voxel index of a global point, -1 outside the phantom box
__device__ __forceinline__ int voxel_of(const DevScene &S, Vec x) {
  const float ix = floorf((x.x - S.ox) / S.vx);
  const float iy = floorf((x.y - S.oy) / S.vy);
  const float iz = floorf((x.z - S.oz) / S.vz);
  if (ix < 0.0f || ix >= (float)S.nx || iy < 0.0f || iy >= (float)S.ny || iz < 0.0f ||
      iz >= (float)S.nz)
    return -1;
  return ((int)iz * S.ny + (int)iy) * S.nx + (int)ix;
}

// ---------------------------------------------------------------------------
// Interactions
// ---------------------------------------------------------------------------
// Compton scattering by Kahn's rejection method, one Philox block per trial;
// returns cos(theta) and sets e_out = E / rho.
__device__ __forceinline__ float kahn(Stream &rng, float e, float &e_out, int &trials) {
  const float a = e / kMec2;
  const float b = 1.0f + 2.0f * a;
  const float p_first = b / (9.0f + 2.0f * a);
  int n = 0;
  for (;;) {
    const float4 r = rng.next();
    ++n;
    float rho, acc;
    if (r.x <= p_first) {
      rho = 1.0f + 2.0f * a * r.y;
      acc = 4.0f * (1.0f / rho - 1.0f / (rho * rho));
    } else {
      rho = b / (1.0f + 2.0f * a * r.y);
      const float c = 1.0f - (rho - 1.0f) / a;
      acc = 0.5f * (c * c + 1.0f / rho);
    }
    if (r.z <= acc) {
      e_out = e / rho;
      trials = n;
      return 1.0f - (rho - 1.0f) / a;
    }
  }
}

// Thomson angular law: mu^3 + 3 mu = 8u - 4 solved with Cardano's formula.
__device__ __forceinline__ float thomson(float u) {
  const float q = 4.0f * u - 2.0f;
  const float s = sqrtf(q * q + 1.0f);
  return cbrtf(q + s) + cbrtf(q - s);
}

// Direction update for polar cosine c and azimuth phi about the old direction.
__device__ __forceinline__ void rotate(Vec &d, float c, float phi) {
  const float st = sqrtf(fmaxf(0.0f, 1.0f - c * c));
  float sp, cp;
  sincosf(phi, &sp, &cp);
  const float s = sqrtf(d.x * d.x + d.y * d.y);
  Vec n;
  if (s < 1e-6f) {
    n = Vec{st * cp, st * sp, (d.z >= 0.0f ? 1.0f : -1.0f) * c};
  } else {
    n = Vec{d.x * c + st * (d.x * d.z * cp - d.y * sp) / s,
            d.y * c + st * (d.y * d.z * cp + d.x * sp) / s, d.z * c - s * st * cp};
  }
  const float nn = sqrtf(n.x * n.x + n.y * n.y + n.z * n.z);
  d = Vec{n.x / nn, n.y / nn, n.z / nn};
}

// process of a real collision: 1 photoelectric, 2 Compton, 3 Rayleigh
__device__ __forceinline__ int pick_process(float4 mu, float mut, float u) {
  if (u * mut < mu.x) return 1;
  if (u * mut < mu.x + mu.y) return 2;
  return 3;
}

// Real collision; returns false when the photon stops.  edep gets the local
// deposit (a below-cutoff remainder included).
__device__ __forceinline__ bool interact(Stream &rng, int proc, float &e, Vec &d, float phi, float e_cut,
                                         float &edep, int &trials) {
  trials = 0;
  if (proc == 1) {
    edep = e;
    e = 0.0f;
    return false;
  }
  if (proc == 2) {
    float e1;
    const float c = kahn(rng, e, e1, trials);
    rotate(d, c, phi);
    edep = e - e1;
    e = e1;
    if (e < e_cut) {
      edep += e;
      e = 0.0f;
      return false;
    }
    return true;
  }
  const float4 r = rng.next();
  rotate(d, thomson(r.x), phi);
  edep = 0.0f;
  return true;
}

} // namespace gpet
