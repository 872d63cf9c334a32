// transport.hip -- photon-pair transport kernel for gfx950.
//
// One lane owns one annihilation event at a time and runs it as a small state
// machine, one action per loop trip: a Woodcock step in the phantom, a panel
// search, or a Woodcock step inside a panel (paper Sec. 2.1: line-plane
// projection to the panel, transform to the panel frame, step-by-step
// transport with the layer chosen from the depth coordinate).  A lane whose
// event is finished fetches the next event id with one wave-aggregated atomic,
// so lanes stay busy however long their histories are.  Hits are appended
// with one wave-aggregated atomic per loop trip into structure-of-arrays
// outputs.
#include "gpet_internal.hpp"

namespace gpet {

enum : int { P_FETCH = 0, P_PHANTOM = 1, P_SEARCH = 2, P_PANEL = 3, P_DONE = 4 };
enum : int { V_STEP = 0, V_ENTER_PANEL = 1, V_EXIT = 2, V_ESCAPE = 3, V_DEAD = 4, V_ENTER_PHANTOM = 5,
             V_EMIT = 6 };

template <bool TRACE>
__device__ __forceinline__ void vertex(const RunArgs &A, uint32_t ev, int ph, int kind, int region,
                                       int panel, int gid, int mat, int acc, int proc, int trials,
                                       uint32_t block, Vec x, float e, float edep, Vec d) {
  if constexpr (TRACE) {
    const size_t p = 2 * (size_t)(ev - A.first) + ph;
    const int c = A.vcount[p];
    if (c < A.max_vertices) {
      int32_t *vi = A.vint + (p * A.max_vertices + c) * 11;
      float *vf = A.vflt + (p * A.max_vertices + c) * 8;
      vi[0] = (int32_t)ev; vi[1] = ph; vi[2] = kind; vi[3] = region; vi[4] = panel; vi[5] = gid;
      vi[6] = mat; vi[7] = acc; vi[8] = proc; vi[9] = trials; vi[10] = (int32_t)block;
      vf[0] = x.x; vf[1] = x.y; vf[2] = x.z; vf[3] = e; vf[4] = edep; vf[5] = d.x; vf[6] = d.y;
      vf[7] = d.z;
    }
    A.vcount[p] = c + 1;
  }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <bool TRACE>
__global__ void __launch_bounds__(256) k_transport(DevScene S, RunArgs A) {
  const int lane = (int)__lane_id();
  const uint64_t below = __lanemask_lt();

  int phase = P_FETCH;
  uint32_t ev = 0;
  int ph = 0;
  Vec x{0.f, 0.f, 0.f}, d{0.f, 0.f, 1.f};
  float e = 0.f, L = 0.f;
  Stream rng{A.k0, A.k1, 0u, A.instance, 0u, 0u};
  int panel = -1, last = -1, steps = 0;
  uint32_t seq = 0;
  Vec src{0.f, 0.f, 0.f}, sdir{0.f, 0.f, 1.f};
  unsigned long long t_event = 0;
  uint32_t c_events = 0, c_entries = 0, c_steps = 0, c_real = 0, c_trials = 0, c_search = 0,
           c_blocks = 0, c_capped = 0;

  // start photon `which` of the current event (A: +d, B: -d)
  auto start_photon = [&](int which) {
    ph = which;
    x = src;
    d = which ? Vec{-sdir.x, -sdir.y, -sdir.z} : sdir;
    e = 511.0f;
    L = 0.0f;
    seq = 0;
    steps = 0;
    last = -1;
    rng.event = ev;
    rng.id = 1u + (uint32_t)which;
    rng.n = 0;
    vertex<TRACE>(A, ev, ph, V_EMIT, -1, -1, -1, -1, 0, 0, 0, 0, x, e, 0.f, d);
    phase = P_SEARCH;
    if (S.has_phantom) {
      if (voxel_of(S, x) >= 0) {
        phase = P_PHANTOM;
      } else {
        float t0;
        if (ray_box(x, d, Vec{S.ox, S.oy, S.oz}, Vec{S.bx, S.by, S.bz}, t0)) {
          x = Vec{x.x + t0 * d.x, x.y + t0 * d.y, x.z + t0 * d.z};
          L += t0;
          phase = P_PHANTOM;
          vertex<TRACE>(A, ev, ph, V_ENTER_PHANTOM, 0, -1, -1, -1, 0, 0, 0, rng.n, x, e, 0.f, d);
        }
      }
    }
  };

  // annihilation point, isotropic direction and event time (event stream 0)
  auto emit = [&]() {
    Stream r0{A.k0, A.k1, ev, A.instance, 0u, 0u};
    const float4 a = r0.next();
    const float4 b = r0.next();
    const uint4 w = philox(A.k0, A.k1, make_uint4(2u, ev, A.instance, 0u));
    t_event = __umul64hi(((unsigned long long)w.y << 32) | w.x, S.duration_ps);
    const float ct = 2.0f * a.x - 1.0f, st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
    float sp, cp;
    sincosf(kTwoPi * a.y, &sp, &cp);
    sdir = Vec{st * cp, st * sp, ct};
    src = Vec{S.sx, S.sy, S.sz};
    if (S.src_kind == 2) {
      sdir = Vec{S.bdx, S.bdy, S.bdz};
    } else if (S.src_kind == 1) {
      const float tgt = a.z * S.rod_total;
      int i = 0;
      while (i < S.n_rods - 1 && S.rod_cum[i] < tgt) ++i;
      const float *rd = S.rods + 5 * i;
      const float rr = rd[2] * sqrtf(a.w);
      float ps, pc;
      sincosf(kTwoPi * b.x, &ps, &pc);
      src = Vec{rd[0] + rr * pc, rd[1] + rr * ps, rd[3] + b.y * (rd[4] - rd[3])};
    }
    ++c_events;
    start_photon(0);
  };

  for (;;) {
    // lanes without an event take the next ids, one atomic per wave
    const bool need = phase == P_FETCH;
    const uint64_t m = __ballot(need);
    if (m) {
      const int leader = __ffsll((unsigned long long)m) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(A.work, (uint32_t)__popcll(m));
      base = __shfl(base, leader);
      if (need) {
        const uint32_t idx = base + (uint32_t)__popcll(m & below);
        if (idx < A.n) {
          ev = A.first + idx;
          emit();
        } else {
          phase = P_DONE;
        }
      }
    }
    if (__ballot(phase != P_DONE) == 0) break;

    bool hit = false, ended = false;
    uint32_t h_gid = 0, h_aux = 0;
    float h_edep = 0.f, h_depth = 0.f;
    unsigned long long h_time = 0;

    if (phase == P_PHANTOM) {
      const float4 r = rng.next();
      ++c_blocks;
      const Lerp lp = lerp_at(e);
      const float mb = lerp1(S.maj_ph, lp);
      const float s = -logf(r.x) / mb;
      const Vec xn{x.x + s * d.x, x.y + s * d.y, x.z + s * d.z};
      const int vox = voxel_of(S, xn);
      if (vox < 0) {
        vertex<TRACE>(A, ev, ph, V_EXIT, 0, -1, -1, -1, 0, 0, 0, rng.n, x, e, 0.f, d);
        phase = P_SEARCH;
      } else {
        x = xn;
        L += s;
        ++c_steps;
        if (++steps > kMaxSteps) {
          ++c_capped;
          ended = true;
        } else {
          const int mat = S.vmat[vox];
          const float rho = S.vden[vox];
          const float4 mm = lerp4(S.mu_mass, mat, lp);
          const float4 mu = make_float4(rho * mm.x, rho * mm.y, rho * mm.z, 0.f);
          const float mut = mu.x + mu.y + mu.z;
          if (r.y * mb < mut) {
            ++c_real;
            const int proc = pick_process(mu, mut, r.z);
            float edep;
            int tr;
            const bool alive = interact(rng, proc, e, d, kTwoPi * r.w, S.e_cut, edep, tr);
            c_trials += tr;
            c_blocks += tr + (proc == 3);
            vertex<TRACE>(A, ev, ph, V_STEP, 0, -1, -1, mat, 1, proc, tr, rng.n, x, e, edep, d);
            if (!alive) {
              vertex<TRACE>(A, ev, ph, V_DEAD, 0, -1, -1, mat, 0, proc, 0, rng.n, x, 0.f, 0.f, d);
              ended = true;
            }
          } else {
            vertex<TRACE>(A, ev, ph, V_STEP, 0, -1, -1, mat, 0, 0, 0, rng.n, x, e, 0.f, d);
          }
        }
      }
    } else if (phase == P_SEARCH) {
      ++c_search;
      float ti;
      const int p = panel_search(S, x, d, last, ti);
      if (p < 0) {
        vertex<TRACE>(A, ev, ph, V_ESCAPE, -1, -1, -1, -1, 0, 0, 0, rng.n, x, e, 0.f, d);
        ended = true;
      } else {
        x = Vec{x.x + ti * d.x, x.y + ti * d.y, x.z + ti * d.z};
        L += ti;
        ++c_entries;
        if (++steps > kMaxSteps) { // bounds panel-to-panel hops as well
          ++c_capped;
          ended = true;
        }
        vertex<TRACE>(A, ev, ph, V_ENTER_PANEL, 1, p, -1, -1, 0, 0, 0, rng.n, x, e, 0.f, d);
        panel = p;
        const float *P = S.pose + 12 * p;
        x = to_local(P, x);
        d = dir_to_local(P, d);
        phase = P_PANEL;
      }
    } else if (phase == P_PANEL) {
      const float4 r = rng.next();
      ++c_blocks;
      const Lerp lp = lerp_at(e);
      const float mb = lerp1(S.maj_det, lp);
      const float s = -logf(r.x) / mb;
      const Vec xn{x.x + s * d.x, x.y + s * d.y, x.z + s * d.z};
      if (!inside_panel(S, xn)) {
        vertex<TRACE>(A, ev, ph, V_EXIT, 1, panel, -1, -1, 0, 0, 0, rng.n, x, e, 0.f, d);
        const float *P = S.pose + 12 * panel;
        x = to_global(P, x);
        d = dir_to_global(P, d);
        last = panel;
        phase = P_SEARCH;
      } else {
        x = xn;
        L += s;
        ++c_steps;
        if (++steps > kMaxSteps) {
          ++c_capped;
          ended = true;
        } else {
          const Loc lc = locate(S, panel, x);
          const float4 mu = lerp4(S.mu, lc.mat, lp);
          const float mut = mu.x + mu.y + mu.z;
          if (r.y * mb < mut) {
            ++c_real;
            const int proc = pick_process(mu, mut, r.z);
            float edep;
            int tr;
            const bool alive = interact(rng, proc, e, d, kTwoPi * r.w, S.e_cut, edep, tr);
            c_trials += tr;
            c_blocks += tr + (proc == 3);
            vertex<TRACE>(A, ev, ph, V_STEP, 1, panel, lc.gid, lc.mat, 1, proc, tr, rng.n, x, e, edep, d);
            if (lc.gid >= 0 && proc != 3) {
              hit = true;
              h_gid = (uint32_t)lc.gid;
              h_edep = edep;
              h_depth = x.x;
              h_time = t_event + (unsigned long long)floorf(L / kCmmPerPs + 0.5f);
              h_aux = (uint32_t)ph | ((uint32_t)proc << 1) | (seq << 8);
              ++seq;
            }
            if (!alive) {
              vertex<TRACE>(A, ev, ph, V_DEAD, 1, panel, lc.gid, lc.mat, 0, proc, 0, rng.n, x, 0.f, 0.f, d);
              ended = true;
            }
          } else {
            vertex<TRACE>(A, ev, ph, V_STEP, 1, panel, lc.gid, lc.mat, 0, 0, 0, rng.n, x, e, 0.f, d);
          }
        }
      }
    }

    // hit append: one atomic per wave and loop trip
    const uint64_t hm = __ballot(hit);
    if (hm) {
      const int leader = __ffsll((unsigned long long)hm) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(A.hit_count, (unsigned long long)__popcll(hm));
      base = __shfl(base, leader);
      if (hit) {
        const unsigned long long i = base + (unsigned long long)__popcll(hm & below);
        if (i < A.capacity) {
          A.h_event[i] = ev;
          A.h_gid[i] = h_gid;
          A.h_edep[i] = h_edep;
          A.h_depth[i] = h_depth;
          A.h_time[i] = h_time;
          A.h_aux[i] = h_aux;
        }
      }
    }
    if (ended) {
      if (ph == 0) start_photon(1);
      else phase = P_FETCH;
    }
  }

  const uint32_t cnt[8] = {c_events, c_entries, c_steps, c_real, c_trials, c_search, c_blocks, c_capped};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t t = wave_sum(cnt[k]);
    if (lane == 0 && t) atomicAdd(A.stats + k, (unsigned long long)t);
  }
}

void launch_transport(const DevScene &S, const RunArgs &A, const LaunchShape &L, int n_cu, hipStream_t st) {
  const uint64_t need = (A.n + L.block - 1) / L.block;
  uint64_t grid = (uint64_t)n_cu * L.blocks_per_cu;
  if (need < grid) grid = need;
  if (grid == 0) grid = 1;
  hipLaunchKernelGGL(k_transport<false>, dim3((unsigned)grid), dim3(L.block), 0, st, S, A);
}

void launch_trace(const DevScene &S, const RunArgs &A, hipStream_t st) {
  const unsigned grid = (A.n + 255) / 256;
  hipLaunchKernelGGL(k_transport<true>, dim3(grid ? grid : 1), dim3(256), 0, st, S, A);
}

// ---------------------------------------------------------------------------
// small utility and check kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}
void launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t st) {
  if (!n) return;
  size_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, st, p, v, n);
}

__global__ void k_philox(uint32_t k0, uint32_t k1, const uint32_t *ctr, uint32_t n, uint32_t *out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint4 c = make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
  const uint4 o = philox(k0, k1, c);
  out[4 * i] = o.x; out[4 * i + 1] = o.y; out[4 * i + 2] = o.z; out[4 * i + 3] = o.w;
}
void launch_philox(uint64_t seed, const uint32_t *ctr, uint32_t n, uint32_t *out, hipStream_t st) {
  if (!n) return;
  hipLaunchKernelGGL(k_philox, dim3((n + 255) / 256), dim3(256), 0, st, (uint32_t)seed,
                     (uint32_t)(seed >> 32), ctr, n, out);
}

__device__ __forceinline__ void write_ids(int32_t *o, int p, const Loc &l) {
  o[0] = p; o[1] = l.module; o[2] = l.layer; o[3] = l.crystal; o[4] = l.gid; o[5] = l.mat;
}

__global__ void k_locate(DevScene S, uint32_t n, const float *xyz, int32_t *ids6) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Vec g{xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
  int32_t *o = ids6 + 6 * (size_t)i;
  o[0] = o[1] = o[2] = o[3] = o[4] = o[5] = -1;
  for (int p = 0; p < S.n_panels; ++p) {
    const Vec l = to_local(S.pose + 12 * p, g);
    if (!inside_panel(S, l)) continue;
    write_ids(o, p, locate(S, p, l));
    break;
  }
}
void launch_locate(const DevScene &S, uint32_t n, const float *xyz, int32_t *ids6, hipStream_t st) {
  if (!n) return;
  hipLaunchKernelGGL(k_locate, dim3((n + 255) / 256), dim3(256), 0, st, S, n, xyz, ids6);
}

__global__ void k_ray_locate(DevScene S, uint32_t n, const float *o, const float *d, int ns, float step,
                             float *t_in, int32_t *ids6) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const Vec ro{o[3 * r], o[3 * r + 1], o[3 * r + 2]}, rd{d[3 * r], d[3 * r + 1], d[3 * r + 2]};
  float ti;
  const int p = panel_search(S, ro, rd, -1, ti);
  t_in[r] = p >= 0 ? ti : -1.0f;
  for (int k = 0; k < ns; ++k) {
    int32_t *q = ids6 + 6 * ((size_t)r * ns + k);
    q[0] = p; q[1] = q[2] = q[3] = q[4] = q[5] = -1;
    if (p < 0) continue;
    const float tt = ti + ((float)k + 0.5f) * step;
    const Vec l = to_local(S.pose + 12 * p, Vec{ro.x + tt * rd.x, ro.y + tt * rd.y, ro.z + tt * rd.z});
    if (!inside_panel(S, l)) {
      q[0] = -2;
      continue;
    }
    write_ids(q, p, locate(S, p, l));
  }
}
void launch_ray_locate(const DevScene &S, uint32_t n, const float *o, const float *d, int ns, float step,
                       float *t_in, int32_t *ids6, hipStream_t st) {
  if (!n) return;
  hipLaunchKernelGGL(k_ray_locate, dim3((n + 255) / 256), dim3(256), 0, st, S, n, o, d, ns, step, t_in, ids6);
}

__global__ void k_compton(float e, uint32_t n, uint32_t k0, uint32_t k1, float *c, float *eo, int32_t *tr) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Stream r{k0, k1, i, 0u, 7u, 0u};
  float e1;
  int t;
  c[i] = kahn(r, e, e1, t);
  eo[i] = e1;
  if (tr) tr[i] = t;
}
void launch_compton(float e, uint32_t n, uint64_t seed, float *c, float *eo, int32_t *tr, hipStream_t st) {
  if (!n) return;
  hipLaunchKernelGGL(k_compton, dim3((n + 255) / 256), dim3(256), 0, st, e, n, (uint32_t)seed,
                     (uint32_t)(seed >> 32), c, eo, tr);
}

__global__ void k_rayleigh(uint32_t n, uint32_t k0, uint32_t k1, float *c) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Stream r{k0, k1, i, 0u, 8u, 0u};
  c[i] = thomson(r.next().x);
}
void launch_rayleigh(uint32_t n, uint64_t seed, float *c, hipStream_t st) {
  if (!n) return;
  hipLaunchKernelGGL(k_rayleigh, dim3((n + 255) / 256), dim3(256), 0, st, n, (uint32_t)seed,
                     (uint32_t)(seed >> 32), c);
}

} // namespace gpet
