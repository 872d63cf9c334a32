// transport.hip -- photon-pair transport kernel for gfx950.
//
// One lane owns one annihilation event at a time and runs it as a small state
// machine.  A loop trip holds one action that draws random numbers -- an
// emission step, a Woodcock step in the phantom, a Woodcock step inside a
// panel (paper Sec. 2.1: step-by-step transport in the panel frame with the
// layer chosen from the depth coordinate), a Kahn trial or a Rayleigh angle --
// and then, at the end of the trip, the panel search (line-plane projection
// to the panels, transform to the panel frame) of every photon that needs
// one, including those that the trip's first action just emitted or sent out
// of a panel or the phantom.  A search draws nothing, so folding it into the
// trip that made it necessary saves a trip per search without changing any
// photon's random numbers.
//
// Every action that needs random numbers takes one Philox block, drawn at a
// single call site at the top of the trip, so the costliest primitive runs
// once per trip with all its lanes together instead of once per divergent
// branch.  The one exception: the emission draws its positron-range and time
// blocks inside its last step (the direction step of point and beam sources,
// the rod-point step of rod sources), so photon A starts one or two trips
// earlier (a trip of every event saved costs less than the extra call sites).
// The launch covers a table of instances (scanner + source; one for a
// plain run, many for a batched sweep): waves claim chunks of consecutive events
// of one instance with one atomic and switch instance only once drained, so the
// scene stays wave-uniform (scalar loads).
// Hits are staged per wave in LDS and written out kFlushAt or more at a time
// (one atomic and coalesced stores per flush).  The detector attenuation rows
// and majorant (a few KB) are read through the vector caches.
#include "transport_common.hpp"

namespace gpet {

// LDS bytes of one block: the per-wave hit staging areas
size_t transport_lds_bytes() { return (size_t)kWaves * kStage * kStageBytes; }

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

// Surrogate domain of a photon entering a panel at local position xl with
// local direction dl and energy e: front-face entry, lateral slopes within
// the limit, the mid-depth point of its straight line inside a module, and
// every layer's neighbourhood around its anchor crystal inside the layer's
// array.  Anchors: the last layer's crystal whose pitch cell holds the
// mid-depth point; in another layer, the crystal whose cell holds that cell's
// centre.  Outputs the 6 features, the module and the anchors (one word per
// layer: i_t | i_a << 16).
template <class SC>
__device__ __forceinline__ bool entry_domain(SC &S, const SurSpecD &P, const Vec &xl, const Vec &dl, float e,
                                             float f[6], int &module, uint32_t anchor[kMaxLayers]) {
  if (!(e >= P.e_min) || fabsf(xl.x) > P.front_tol || !(dl.x > 0.0f)) return false;
  const float st = dl.y / dl.x, sa = dl.z / dl.x;
  if (fabsf(st) > P.max_slope || fabsf(sa) > P.max_slope) return false;
  const float s = (0.5f * S.depth - xl.x) / dl.x;
  const float t = xl.y + s * dl.y, a = xl.z + s * dl.z;
  const float mtf = floorf((t - S.mod_t0) * S.inv_step_t), maf = floorf((a - S.mod_a0) * S.inv_step_a);
  if (!(mtf >= 0.0f && mtf < (float)S.mod_n_t && maf >= 0.0f && maf < (float)S.mod_n_a)) return false;
  const int mt = (int)mtf, ma = (int)maf;
  const float ut = t - S.mod_t0 - (float)mt * S.mod_step_t, ua = a - S.mod_a0 - (float)ma * S.mod_step_a;
  if (!(ut >= 0.0f && ut < S.mod_t && ua >= 0.0f && ua < S.mod_a)) return false;
  const int nl = S.n_layers;
  const float rt = S.layer[nl - 1].off_t, ra = S.layer[nl - 1].off_a;
  const float pt = S.layer[nl - 1].pitch_t, pa = S.layer[nl - 1].pitch_a;
  const float qt = (ut - rt) / pt, qa = (ua - ra) / pa;
  const float it = floorf(qt), ia = floorf(qa);
  const float ct = rt + (it + 0.5f) * pt, ca = ra + (ia + 0.5f) * pa;
  for (int l = 0; l < nl; ++l) {
    const int jt = (int)floorf((ct - S.layer[l].off_t) / S.layer[l].pitch_t + 1e-3f);
    const int ja = (int)floorf((ca - S.layer[l].off_a) / S.layer[l].pitch_a + 1e-3f);
    if (jt < P.half || jt > S.layer[l].n_t - 1 - P.half || ja < P.half || ja > S.layer[l].n_a - 1 - P.half)
      return false;
    anchor[l] = (uint32_t)jt | ((uint32_t)ja << 16);
  }
  f[0] = 2.0f * (qt - it) - 1.0f;
  f[1] = 2.0f * (qa - ia) - 1.0f;
  f[2] = st / P.max_slope;
  f[3] = sa / P.max_slope;
  f[4] = 2.0f * (e - P.e_min) / (511.0f - P.e_min) - 1.0f;
  f[5] = dl.x;
  module = ma * S.mod_n_t + mt;
  return true;
}

// The surrogate mode is held to 5 waves per SIMD (96 registers, one spilled),
// as the plain mode reaches by itself; the trace and record modes are test and
// training-data paths and keep the compiler's allocation.
template <int MODE>
__global__ void __launch_bounds__(kBlock, MODE == kModeSurrogate ? 5 : 1) k_transport(RunArgs A) {
  constexpr bool TRACE = MODE == kModeTrace, REC = MODE == kModeRecord, SUR = MODE == kModeSurrogate;
  extern __shared__ float4 lds4[];
  const int lane = (int)__lane_id();
  const int wave = (int)(threadIdx.x >> 6);
  const uint64_t below = __lanemask_lt();

  // ---- the instances share their materials: instance 0's detector
  //      attenuation rows and majorant (a few KB per material, read through
  //      the vector caches, which leaves LDS to the hit staging)
  CScene *sp = (CScene *)A.scenes;
  const float4 *s_mu = sp->mu_det;
  const float *s_maj = sp->maj_det;
  char *stage_base = (char *)lds4 + (size_t)wave * kStage * kStageBytes;
  Stage st;
  st.time = (unsigned long long *)stage_base;
  st.ev = (uint32_t *)(st.time + kStage);
  st.gid = st.ev + kStage;
  st.aux = st.gid + kStage;
  st.edep = (float *)(st.aux + kStage);
  st.depth = st.edep + kStage;
  __syncthreads();

  int phase = P_FETCH;
  uint32_t ev = 0, n = 0, sid = 0, seq = 0;
  int ph = 0, panel = -1, last = -1, steps = 0;
  Vec x{0.f, 0.f, 0.f}, d{0.f, 0.f, 1.f};
  float e = 0.f, L = 0.f;
  Vec src{0.f, 0.f, 0.f}, sdir{0.f, 0.f, 1.f};
  unsigned long long t_event = 0;
  // pending interaction (or emission) state
  float q_u0 = 0.f, q_u1 = 0.f; // azimuth uniform of the pending scatter / rod uniforms
  int q_gid = -1, q_mat = -1, q_trials = 0, q_back = P_PANEL;
  // wave-uniform bookkeeping: the instance the wave works on, its current
  // range of event indices, a claimed next range, and the hit staging count
  // record mode: the pair being labelled and its per-crystal deposit sums
  constexpr int kSlots = 8;
  uint32_t rec_idx = ~0u, rec_anchor[kMaxLayers] = {0u, 0u, 0u, 0u}, rec_gid[kSlots];
  float rec_sum[kSlots], rec_e = 0.f;
  int rec_module = 0, rec_panel = 0, rec_n = 0;
  bool rec_ovf = false;
  uint32_t inst = 0, inst_rng = A.inst_id[0];
  uint32_t cur_next = 0, cur_end = 0, pend_inst = 0, pend_next = 0, pend_end = 0, staged = 0;
  bool have_pend = false, exhausted = false;
  // work counters: per-lane counts (summed over the wave at the end), trips per wave
  uint32_t c_events = 0, c_entries = 0, c_steps = 0, c_real = 0, c_trials = 0, c_search = 0, c_blocks = 0,
           c_capped = 0, c_scatter = 0, c_tests = 0, c_pruned = 0, c_nonfinite = 0;
  unsigned long long c_trips = 0;
  // surrogate mode: the wave's current queue reservation [q_base, q_base + q_left)
  unsigned long long q_base = 0;
  uint32_t q_left = 0;

  // start photon `which` of the current event (A: +d, B: -d)
  auto start_photon = [&](CScene &S, int which) {
    ph = which;
    x = src;
    if (which) d = Vec{-sdir.x, -sdir.y, -sdir.z}; // photon A's direction is already in d
    e = 511.0f;
    L = 0.0f;
    seq = 0;
    steps = 0;
    last = -1;
    n = 0;
    sid = 1u + (uint32_t)which;
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
          vertex<TRACE>(A, ev, ph, V_ENTER_PHANTOM, 0, -1, -1, -1, 0, 0, 0, n, x, e, 0.f, d);
        }
      }
    }
  };

  // the end of an emission: the positron-range block (3) when asked for, then
  // the time block (2) with the acollinearity, drawn here rather than in trips
  // of their own; photon A starts at the trip's start site
  bool start_a = false;
  auto emit_finish = [&](CScene &S) {
    if (S.prange_sigma > 0.0f)
      src = positron_offset(S, src, to_unit4(philox(A.k0, A.k1, make_uint4(3u, ev, inst_rng, 0u))));
    const uint4 w2 = philox(A.k0, A.k1, make_uint4(2u, ev, inst_rng, 0u));
    const float4 r2 = to_unit4(w2);
    t_event = __umul64hi(((unsigned long long)w2.y << 32) | w2.x, S.duration_ps);
    const Vec bdir = photon_b_dir(S, sdir, r2.z, r2.w);
    d = sdir;
    sdir = Vec{-bdir.x, -bdir.y, -bdir.z};
    start_a = true;
  };

  for (;;) {
    // ---- lanes without an event take the next ids: first from the current
    //      range, then from a claimed range of the same instance; a range of
    //      another instance is opened only once the wave has drained
    const bool need = phase == P_FETCH;
    const uint64_t m = __ballot(need);
    if (m) {
      const uint32_t k = (uint32_t)__popcll(m);
      uint32_t avail = cur_end - cur_next;
      if (k > avail && !have_pend && !exhausted) {
        uint32_t c = 0;
        if (lane == 0) c = atomicAdd(A.work, 1u);
        c = __builtin_amdgcn_readfirstlane(__shfl(c, 0));
        if (c >= A.total_chunks) {
          exhausted = true;
        } else {
          uint32_t lo = 0, hi = A.n_inst; // owner: largest i with chunk_prefix[i] <= c
          while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (A.chunk_prefix[mid] <= c) lo = mid;
            else hi = mid;
          }
          const uint32_t b0 = (c - A.chunk_prefix[lo]) * A.chunk;
          pend_inst = lo;
          pend_next = b0;
          pend_end = min(b0 + A.chunk, A.inst_count[lo]);
          have_pend = true;
        }
      }
      if (have_pend && pend_inst != inst && __ballot(phase != P_FETCH && phase != P_DONE) == 0 && avail == 0) {
        flush_stage(A, st, staged, lane, inst); // staged hits carry the wave's instance
        staged = 0;
        inst = pend_inst; // drained: switch the wave to the claimed instance
        inst_rng = A.inst_id[inst];
        sp = (CScene *)(A.scenes + inst);
        cur_next = cur_end = pend_next;
      }
      const bool use_pend = have_pend && pend_inst == inst;
      const uint32_t extra = use_pend ? pend_end - pend_next : 0u;
      const uint32_t rank = (uint32_t)__popcll(m & below);
      if (need) {
        if (rank < avail) {
          ev = A.inst_first[inst] + cur_next + rank;
          phase = P_EMIT_DIR;
        } else if (rank - avail < extra) {
          ev = A.inst_first[inst] + pend_next + (rank - avail);
          phase = P_EMIT_DIR;
        } else if (exhausted && !have_pend) {
          phase = P_DONE;
        }
        n = 0;
        sid = 0;
      }
      const uint32_t take_cur = min(k, avail);
      cur_next += take_cur;
      if (use_pend) {
        const uint32_t take_pend = min(k - take_cur, extra);
        cur_next = pend_next + take_pend;
        cur_end = pend_end;
        have_pend = false;
      }
    }
    if (__ballot(phase != P_DONE) == 0) break;
    ++c_trips;
    CScene &S = *sp;

    // ---- which lanes act this trip (panel searches come at its end)
    bool run, search_pick = true;
    if (A.schedule == 0 || A.schedule == 2) { // (2: the pool schedule, here in the modes it does not cover)
      run = phase != P_DONE && phase != P_FETCH && phase != P_SEARCH;
    } else {
      // only the phase held by the most lanes runs (ties to the later phase),
      // so each phase body executes with as many lanes as possible
      int best = P_EMIT_DIR;
      uint32_t best_n = 0;
#pragma unroll
      for (int q = P_EMIT_DIR; q <= P_RAYLEIGH; ++q) {
        const uint32_t nq = (uint32_t)__popcll(__ballot(phase == q));
        if (nq >= best_n) {
          best_n = nq;
          best = q;
        }
      }
      run = phase == best && best != P_SEARCH;
      search_pick = best == P_SEARCH;
    }

    // ---- the one Philox block of this trip
    const bool draw = run;
    uint4 w = make_uint4(0u, 0u, 0u, 0u);
    if (draw) {
      w = philox(A.k0, A.k1, make_uint4(n, ev, inst_rng, sid));
      ++n;
    }
    const float4 r = to_unit4(w);
    c_blocks += (draw && sid != 0u) ? 1u : 0u;

    bool hit = false, ended = false;
    start_a = false;
    float h_edep = 0.f;
    int h_proc = 0;
    bool stepped = false, real = false, trial = false, scattered = false, capped = false, emitted = false;

    if (!run) {
      // waits for its phase to be scheduled (or for events)
    } else if (phase == P_EMIT_DIR) {
      // block 0 of the event stream: isotropic direction, two source uniforms
      const float ct = 2.0f * r.x - 1.0f, stt = hw_sqrt(fmaxf(0.0f, 1.0f - ct * ct));
      sdir = Vec{stt * cos_rev(r.y), stt * sin_rev(r.y), ct};
      q_u0 = r.z;
      q_u1 = r.w;
      src = Vec{S.sx, S.sy, S.sz};
      if (S.src_kind == 2) sdir = Vec{S.bdx, S.bdy, S.bdz};
      if (S.src_kind == 1) {
        phase = P_EMIT_POS;
      } else { // block 1 is not needed
        emit_finish(S);
        emitted = true;
      }
    } else if (phase == P_EMIT_POS) {
      // block 1: point in the chosen rod (rod ~ volume, uniform in its disk and length)
      const float tgt = q_u0 * S.rod_total;
      // the first rod whose cumulative weight reaches tgt, the last rod if no
      // other does: a binary search over rod_cum[0 .. n_rods - 2] (rod_cum
      // never decreases), the same rod as a scan from the first
      int i = 0, hi = S.n_rods - 1;
      while (i < hi) {
        const int mid = (i + hi) >> 1;
        if (S.rod_cum[mid] < tgt) i = mid + 1;
        else hi = mid;
      }
      const float *rd = S.rods + 5 * i;
      const float rr = rd[2] * hw_sqrt(q_u1);
      src = Vec{rd[0] + rr * cos_rev(r.x), rd[1] + rr * sin_rev(r.x), rd[3] + r.y * (rd[4] - rd[3])};
      emit_finish(S);
      emitted = true;
    } else if (phase == P_PHANTOM) {
      const Lerp lp = lerp_at(e);
      const float mb = lerp1(S.maj_ph, lp);
      const float s = neg_ln(r.x) * rcp(mb);
      const Vec xn{x.x + s * d.x, x.y + s * d.y, x.z + s * d.z};
      const int vox = voxel_of(S, xn);
      if (vox < 0) {
        vertex<TRACE>(A, ev, ph, V_EXIT, 0, -1, -1, -1, 0, 0, 0, n, x, e, 0.f, d);
        phase = P_SEARCH;
      } else {
        x = xn;
        L += s;
        stepped = true;
        if (++steps > kMaxSteps) {
          capped = ended = true;
        } else {
          const int mat = S.vmat[vox];
          const float rho = S.vden[vox];
          const float4 mm = lerp4(S.mu_mass, mat, lp);
          const float4 mu = make_float4(rho * mm.x, rho * mm.y, rho * mm.z, 0.f);
          const float mut = mu.x + mu.y + mu.z;
          if (r.y * mb < mut) {
            real = true;
            const int proc = pick_process(mu, mut, r.z);
            if (proc == 1) {
              vertex<TRACE>(A, ev, ph, V_STEP, 0, -1, -1, mat, 1, 1, 0, n, x, 0.f, e, d);
              vertex<TRACE>(A, ev, ph, V_DEAD, 0, -1, -1, mat, 0, 1, 0, n, x, 0.f, 0.f, d);
              ended = true;
            } else {
              q_u0 = r.w;
              q_gid = -1;
              q_mat = mat;
              q_trials = 0;
              q_back = P_PHANTOM;
              phase = proc == 2 ? P_KAHN : P_RAYLEIGH;
            }
          } else {
            vertex<TRACE>(A, ev, ph, V_STEP, 0, -1, -1, mat, 0, 0, 0, n, x, e, 0.f, d);
          }
        }
      }
    } else if (phase == P_PANEL) {
      const Lerp lp = lerp_at(e);
      const float mb = lerp1(s_maj, lp);
      const float s = neg_ln(r.x) * rcp(mb);
      const Vec xn{x.x + s * d.x, x.y + s * d.y, x.z + s * d.z};
      if (!inside_panel(S, xn)) {
        vertex<TRACE>(A, ev, ph, V_EXIT, 1, panel, -1, -1, 0, 0, 0, n, x, e, 0.f, d);
        CFloat *P = (CFloat *)(S.pose + 12 * panel);
        x = to_global(P, x);
        d = dir_to_global(P, d);
        last = panel;
        phase = P_SEARCH;
      } else {
        x = xn;
        L += s;
        stepped = true;
        if (++steps > kMaxSteps) {
          capped = ended = true;
        } else {
          const Loc lc = locate(S, panel, x);
          const float4 mu = lerp4(s_mu, lc.slot, lp);
          const float mut = mu.x + mu.y + mu.z;
          if (r.y * mb < mut) {
            real = true;
            const int proc = pick_process(mu, mut, r.z);
            q_gid = lc.gid;
            if (proc == 1) {
              vertex<TRACE>(A, ev, ph, V_STEP, 1, panel, lc.gid, lc.mat, 1, 1, 0, n, x, 0.f, e, d);
              vertex<TRACE>(A, ev, ph, V_DEAD, 1, panel, lc.gid, lc.mat, 0, 1, 0, n, x, 0.f, 0.f, d);
              if (lc.gid >= 0) {
                hit = true;
                h_edep = e;
                h_proc = 1;
              }
              ended = true;
            } else {
              q_u0 = r.w;
              q_mat = lc.mat;
              q_trials = 0;
              q_back = P_PANEL;
              phase = proc == 2 ? P_KAHN : P_RAYLEIGH;
            }
          } else {
            vertex<TRACE>(A, ev, ph, V_STEP, 1, panel, lc.gid, lc.mat, 0, 0, 0, n, x, e, 0.f, d);
          }
        }
      }
    } else if (phase == P_KAHN) {
      trial = true;
      ++q_trials;
      float c, e1;
      if (kahn_trial(e, r, c, e1)) {
        scattered = true;
        rotate(d, c, q_u0);
        float edep = e - e1;
        e = e1;
        const bool alive = e >= S.e_cut;
        if (!alive) { // below the cutoff: the rest is deposited here
          edep += e;
          e = 0.0f;
        }
        const int region = q_back == P_PANEL ? 1 : 0;
        vertex<TRACE>(A, ev, ph, V_STEP, region, region ? panel : -1, q_gid, q_mat, 1, 2, q_trials, n, x, e,
                      edep, d);
        if (region && q_gid >= 0) {
          hit = true;
          h_edep = edep;
          h_proc = 2;
        }
        if (!alive) {
          vertex<TRACE>(A, ev, ph, V_DEAD, region, region ? panel : -1, q_gid, q_mat, 0, 2, 0, n, x, 0.f, 0.f,
                        d);
          ended = true;
        } else {
          phase = q_back;
        }
      }
    } else if (phase == P_RAYLEIGH) {
      scattered = true;
      rotate(d, thomson(r.x), q_u0);
      const int region = q_back == P_PANEL ? 1 : 0;
      vertex<TRACE>(A, ev, ph, V_STEP, region, region ? panel : -1, q_gid, q_mat, 1, 3, 0, n, x, e, 0.f, d);
      phase = q_back;
    }

    // ---- guard: a photon whose state stopped being finite ends here
    bool bad = false;
    if (scattered && nonfinite_state(x, d, e)) {
      bad = ended = true;
      hit = false;
    }
    c_nonfinite += bad ? 1u : 0u;

    // ---- work counters (scalar)
    c_events += emitted ? 1u : 0u;
    c_steps += stepped ? 1u : 0u;
    c_real += real ? 1u : 0u;
    c_trials += trial ? 1u : 0u;
    c_scatter += scattered ? 1u : 0u;
    c_capped += capped ? 1u : 0u;

    if constexpr (REC) {
      if (rec_idx != ~0u) {
        if (hit) { // per-crystal deposit sums of the photon's stay in its first panel
          int k = 0;
          while (k < rec_n && rec_gid[k] != (uint32_t)q_gid) ++k;
          if (k < rec_n) {
            rec_sum[k] += h_edep;
          } else if (rec_n < kSlots) {
            rec_gid[rec_n] = (uint32_t)q_gid;
            rec_sum[rec_n] = h_edep;
            ++rec_n;
          } else {
            rec_ovf = true;
          }
        }
        if (ended || phase == P_SEARCH) { // left the panel or stopped: label the pair
          int best = -1;
          for (int k = 0; k < rec_n; ++k)
            if (best < 0 || rec_sum[k] > rec_sum[best] || (rec_sum[k] == rec_sum[best] && rec_gid[k] < rec_gid[best]))
              best = k;
          int cls = 0;
          uint32_t flags = (rec_ovf ? 2u : 0u) | ((uint32_t)ph << 2);
          if (best >= 0 && rec_sum[best] >= A.sur.e_min) {
            const int g = (int)rec_gid[best];
            const int r = g - rec_panel * S.crystals_per_panel;
            const int m = r >= 0 ? r / S.crystals_per_module : -1;
            const int r2 = r - m * S.crystals_per_module;
            int l = S.n_layers - 1;
            while (l > 0 && r2 < S.layer[l].base) --l;
            const int idx = r2 - S.layer[l].base;
            const int ia = idx / S.layer[l].n_t, it = idx - ia * S.layer[l].n_t;
            const uint32_t aw = rec_anchor[l];
            const int at = (int)(aw & 0xFFFFu), aa = (int)(aw >> 16);
            const int h = A.sur.chalf, W = 2 * h + 1; // the class neighbourhood
            if (r < 0 || r >= S.crystals_per_panel || m != rec_module || abs(it - at) > h || abs(ia - aa) > h) {
              flags |= 1u; // the largest deposit lies outside the neighbourhood
            } else {
              int b;
              if (rec_sum[best] >= rec_e - A.sur.tol) b = A.sur.n_ebins;
              else b = min(max((int)floorf((rec_sum[best] - A.sur.e_min) / A.sur.ebin), 0), A.sur.n_ebins - 1);
              cls = 1 + ((l * W + (it - at + h)) * W + (ia - aa + h)) * (A.sur.n_ebins + 1) + b;
            }
          }
          A.plabel[rec_idx] = cls;
          A.pflags[rec_idx] = flags;
          rec_idx = ~0u;
        }
      }
    }

    // ---- stage hits in LDS; write out kFlushAt or more at a time
    const uint64_t hm = __ballot(hit);
    if (hm) {
      if (hit) {
        const uint32_t k = staged + (uint32_t)__popcll(hm & below);
        st.ev[k] = ev;
        st.gid[k] = (uint32_t)q_gid;
        st.edep[k] = h_edep;
        st.depth[k] = x.x;
        st.time[k] = t_event + (unsigned long long)floorf(L * kInvCmmPerPs + 0.5f);
        st.aux[k] = (uint32_t)ph | ((uint32_t)h_proc << 1) | (seq << 8);
        ++seq;
      }
      staged += (uint32_t)__popcll(hm);
      if (staged >= kFlushAt) {
        flush_stage(A, st, staged, lane, inst);
        staged = 0;
      }
    }
    // ---- photon starts: A after the emission, B once A has ended
    if (start_a || (ended && ph == 0)) start_photon(S, start_a ? 0 : 1);
    else if (ended) phase = P_FETCH;

    // ---- panel searches, at the end of the trip, so that a photon just
    //      emitted or just out of a panel or the phantom searches in the trip
    //      that put it there; they run in batches: lanes that need one wait
    //      until at least `search_batch` lanes of the wave do, or nothing else
    //      can run.  A search draws no random numbers.
    bool s_run;
    if (A.schedule == 1) {
      s_run = search_pick && phase == P_SEARCH;
    } else {
      const uint64_t sm = __ballot(phase == P_SEARCH);
      const uint64_t om = __ballot(phase != P_SEARCH && phase != P_DONE && phase != P_FETCH);
      s_run = phase == P_SEARCH && ((uint32_t)__popcll(sm) >= A.search_batch || om == 0);
    }
    ended = capped = false;
    bool push = false, entered = false;
    int n_tested = 0;
    float sf[6];
    int s_module = 0;
    uint32_t s_anchor[kMaxLayers] = {0u, 0u, 0u, 0u};
    if (s_run) {
      float ti;
      const int p = search_panels(S, x, d, last, ti, n_tested);
      if (p < 0) {
        vertex<TRACE>(A, ev, ph, V_ESCAPE, -1, -1, -1, -1, 0, 0, 0, n, x, e, 0.f, d);
        ended = true;
      } else {
        x = Vec{x.x + ti * d.x, x.y + ti * d.y, x.z + ti * d.z};
        L += ti;
        entered = true;
        vertex<TRACE>(A, ev, ph, V_ENTER_PANEL, 1, p, -1, -1, 0, 0, 0, n, x, e, 0.f, d);
        panel = p;
        CFloat *P = (CFloat *)(S.pose + 12 * p);
        x = to_local(P, x);
        d = dir_to_local(P, d);
        phase = P_PANEL;
        if (++steps > kMaxSteps) capped = ended = true; // bounds panel-to-panel hops as well
        if constexpr (REC || SUR) {
          if (last < 0 && !capped && entry_domain(S, A.sur, x, d, e, sf, s_module, s_anchor)) {
            push = true;
            if constexpr (SUR) ended = true; // the network takes over from here
          }
        }
      }
    }
    bad = false;
    if (entered && nonfinite_state(x, d, e)) {
      bad = ended = true;
      push = false;
    }
    c_nonfinite += bad ? 1u : 0u;
    c_search += s_run ? 1u : 0u;
    c_tests += (uint32_t)n_tested;
    c_pruned += (s_run && S.ring_reg) ? 1u : 0u;
    c_entries += entered ? 1u : 0u;
    c_capped += capped ? 1u : 0u;

    // ---- record / surrogate: one atomic per wave reserves the new entries
    if constexpr (REC || SUR) {
      const uint64_t pm = __ballot(push);
      if (pm) {
        const uint32_t kp = (uint32_t)__popcll(pm), rank = (uint32_t)__popcll(pm & below);
        unsigned long long i;
        if constexpr (SUR) {
          // entries fill the wave's reservation; a new one of kQueueResv slots
          // (or as many as the rest needs) is claimed when it runs out
          if (kp > q_left) {
            const uint32_t rest = kp - q_left, need = rest > kQueueResv ? rest : kQueueResv;
            unsigned long long nb = 0;
            if (lane == 0) nb = atomicAdd(A.pcount, (unsigned long long)need);
            nb = __shfl(nb, 0);
            i = rank < q_left ? q_base + rank : nb + (rank - q_left);
            q_base = nb + rest;
            q_left = need - rest;
          } else {
            i = q_base + rank;
            q_base += kp;
            q_left -= kp;
          }
        } else {
          unsigned long long base = 0;
          if (lane == 0) base = atomicAdd(A.pcount, (unsigned long long)kp);
          base = __shfl(base, 0);
          i = base + rank;
        }
        if (push) {
          const bool fits = i < A.pcap;
          if (fits) {
#pragma unroll
            for (int k = 0; k < 6; ++k) A.px[6 * i + k] = sf[k];
          }
          if constexpr (REC) {
            if (fits) A.pevent[i] = ev;
            rec_idx = fits ? (uint32_t)i : ~0u;
#pragma unroll
            for (int l = 0; l < kMaxLayers; ++l) rec_anchor[l] = s_anchor[l];
            rec_module = s_module;
            rec_panel = panel;
            rec_e = e;
            rec_n = 0;
            rec_ovf = false;
          } else if (fits) {
            A.qev[i] = ev;
            A.qmeta[i] = (uint32_t)ph | ((uint32_t)panel << 1) | ((uint32_t)s_module << 8);
#pragma unroll
            for (int l = 0; l < kMaxLayers; ++l) A.qanchor[kMaxLayers * i + l] = s_anchor[l];
            A.qe[i] = e;
            A.qtime[i] = t_event + (unsigned long long)floorf(L * kInvCmmPerPs + 0.5f);
          }
        }
      }
    }
    if (ended) {
      if (ph == 0) start_photon(S, 1);
      else phase = P_FETCH;
    }
  }
  flush_stage(A, st, staged, lane, inst);
  if constexpr (SUR) {
    // the unused rest of the last reservation: empty slots (q_left < 64)
    if ((uint32_t)lane < q_left) {
      const unsigned long long i = q_base + (unsigned long long)lane;
      if (i < A.pcap) {
        A.qmeta[i] = kQueueHole;
#pragma unroll
        for (int k = 0; k < 6; ++k) A.px[6 * i + k] = 0.0f;
      }
    }
    if (lane == 0 && q_left) atomicAdd(A.pholes, (unsigned long long)q_left);
  }

  uint32_t lc[kStatCount] = {c_events, c_entries, c_steps,   c_real, c_trials, c_search,
                             c_blocks, c_capped,  c_scatter, 0u,     c_tests,  c_pruned, c_nonfinite};
  unsigned long long cnt[kStatCount];
#pragma unroll
  for (int k = 0; k < kStatCount; ++k) {
    unsigned long long t = lc[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    cnt[k] = t;
  }
  cnt[9] = c_trips;
  // the block's four waves add up their counters in LDS: one atomic per
  // counter and block instead of per wave (they share the hit counter's line)
  __shared__ unsigned long long s_cnt[kWaves][kStatCount];
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kStatCount; ++k) s_cnt[wave][k] = cnt[k];
  }
  __syncthreads();
  if (threadIdx.x < kStatCount) {
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += s_cnt[w][threadIdx.x];
    if (t) atomicAdd(A.stats + threadIdx.x, t);
  }
}

template <int MODE>
static void launch_mode(const RunArgs &A, const LaunchShape &L, int n_cu, hipStream_t st) {
  // one resident wave set: as many blocks per CU as the kernel's registers and
  // LDS allow (unless the shape asks for a given number)
  const size_t lds = transport_lds_bytes();
  int per_cu = L.blocks_per_cu;
  if (per_cu <= 0) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_transport<MODE>, kBlock, lds) != hipSuccess || occ < 1)
      occ = 4;
    per_cu = occ;
  }
  const uint64_t need = ((uint64_t)A.total_chunks * A.chunk + kBlock - 1) / kBlock;
  uint64_t grid = (uint64_t)n_cu * per_cu;
  if (need < grid) grid = need;
  if (grid == 0) grid = 1;
  hipLaunchKernelGGL(k_transport<MODE>, dim3((unsigned)grid), dim3(kBlock), lds, st, A);
}

void launch_transport(const RunArgs &A, const LaunchShape &L, int n_cu, hipStream_t st, int mode) {
  if (mode == kModePlain && L.schedule == 2) {
    launch_transport_pool(A, L, n_cu, st);
    return;
  }
  if (mode == kModeRecord) launch_mode<kModeRecord>(A, L, n_cu, st);
  else if (mode == kModeSurrogate) launch_mode<kModeSurrogate>(A, L, n_cu, st);
  else launch_mode<kModePlain>(A, L, n_cu, st);
}

void launch_trace(const RunArgs &A, hipStream_t st) {
  const unsigned grid = (A.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_transport<kModeTrace>, dim3(grid ? grid : 1), dim3(kBlock), transport_lds_bytes(), st,
                     A);
}

// ---------------------------------------------------------------------------
// small utility and check kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}
// zeroes up to three word ranges in one launch (null or empty ranges skipped)
__global__ void k_zero3(uint32_t *a, size_t na, uint32_t *b, size_t nb, uint32_t *c, size_t nc) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb + nc; i += stride) {
    if (i < na) a[i] = 0u;
    else if (i < na + nb) b[i - na] = 0u;
    else c[i - na - nb] = 0u;
  }
}

void launch_zero3(uint32_t *a, size_t na, uint32_t *b, size_t nb, uint32_t *c, size_t nc, hipStream_t st) {
  if (!a) na = 0;
  if (!b) nb = 0;
  if (!c) nc = 0;
  const size_t n = na + nb + nc;
  if (!n) return;
  size_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_zero3, dim3((unsigned)g), dim3(256), 0, st, a, na, b, nb, c, nc);
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
  int tested;
  const int p = search_panels(S, ro, rd, -1, ti, tested); // the transport's search
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
