// transport_pool.hip -- plain-mode photon transport with per-wave photon pools.
//
// The lane-per-event kernel runs, on every loop trip, the union of the phase
// bodies its lanes hold, so most lanes idle through most of each trip.  Here a
// wave keeps a pool of photon states in LDS; a new event takes two free slots
// (photon A, and photon B's slot reserved until the emission is complete), and
// a finished photon frees its slot at once.  Every trip
// the wave runs the one phase held by the most slots: it gathers up to 64 of
// those slots onto its lanes, loads their states, draws one Philox block per
// lane, runs that phase's body and stores the states back.  A photon draws the
// same blocks at the same counters and does the same arithmetic as in the
// lane kernel, so both kernels produce the same hits, in another order.
//
// The paper's method per photon (Sec. 2.1): Woodcock tracking in the phantom,
// line-plane search of the next panel, transform to the panel frame, Woodcock
// steps inside the panel with the layer chosen from the depth coordinate.
#include "transport_common.hpp"

namespace gpet {

constexpr int kPool = 128;      // photon slots per wave; lane l counts slots l and l + 64
constexpr int kPoolWords = 16;  // state words per slot (SoA)
constexpr int kSlotDead = 0;    // slot phases besides P_EMIT_DIR .. P_RAYLEIGH
constexpr int kSlotReserved = 15;

// state words of a slot
enum : int {
  W_X = 0, W_Y, W_Z, W_DX, W_DY, W_DZ, W_E, W_L, W_EV, W_N, W_TLO, W_THI, W_U0, W_GID, W_FLAGS, W_STEPS
};
// W_FLAGS: phase (4 bits) | photon (1) | panel + 1 (7) | last + 1 (7) | back to panel (1) | seq (12)
__device__ __forceinline__ uint32_t pack_flags(int phase, int ph, int panel, int last, bool back_panel,
                                               uint32_t seq) {
  return (uint32_t)phase | ((uint32_t)ph << 4) | ((uint32_t)(panel + 1) << 5) | ((uint32_t)(last + 1) << 12) |
         ((back_panel ? 1u : 0u) << 19) | (min(seq, 4095u) << 20);
}

size_t transport_pool_lds_bytes() {
  return (size_t)kWaves * ((size_t)kStage * kStageBytes + (size_t)kPool * kPoolWords * 4 + kPool * 4);
}

__global__ void __launch_bounds__(kBlock) k_transport_pool(RunArgs A) {
  extern __shared__ float4 lds4[];
  const int lane = (int)__lane_id();
  const int wave = (int)(threadIdx.x >> 6);
  const uint64_t below = __lanemask_lt();

  // ---- detector attenuation rows and majorant of the instances (shared
  //      materials, read through the vector caches)
  CScene *sp = (CScene *)A.scenes;
  const float4 *s_mu = sp->mu_det;
  const float *s_maj = sp->maj_det;
  char *wave_base = (char *)lds4 +
                    (size_t)wave * ((size_t)kStage * kStageBytes + (size_t)kPool * kPoolWords * 4 + kPool * 4);
  Stage st;
  st.time = (unsigned long long *)wave_base;
  st.ev = (uint32_t *)(st.time + kStage);
  st.gid = st.ev + kStage;
  st.aux = st.gid + kStage;
  st.edep = (float *)(st.aux + kStage);
  st.depth = st.edep + kStage;
  uint32_t *pool = (uint32_t *)(st.depth + kStage); // pool[w * kPool + slot]
  uint32_t *list = pool + kPoolWords * kPool;
  for (int k = lane; k < kPool; k += 64) pool[W_FLAGS * kPool + k] = kSlotDead;
  __syncthreads();

  auto P = [&](int w, uint32_t s) -> uint32_t & { return pool[w * kPool + s]; };
  auto PF = [&](int w, uint32_t s) -> float & { return *(float *)&pool[w * kPool + s]; };

  uint32_t inst = 0, inst_rng = A.inst_id[0];
  uint32_t cur_next = 0, cur_end = 0, pend_inst = 0, pend_next = 0, pend_end = 0, staged = 0;
  bool have_pend = false, exhausted = false;
  uint32_t c_events = 0, c_entries = 0, c_steps = 0, c_real = 0, c_trials = 0, c_search = 0, c_blocks = 0,
           c_capped = 0, c_scatter = 0, c_tests = 0, c_pruned = 0, c_nonfinite = 0;
  unsigned long long c_trips = 0;

  for (;;) {
    // ---- the two slots this lane counts
    int pa = (int)(P(W_FLAGS, lane) & 15u), pb = (int)(P(W_FLAGS, lane + 64) & 15u);

    // ---- new events take free slots two by two: the next event ids come first
    //      from the current range, then from a claimed range of the same
    //      instance; a range of another instance is opened only once the pool
    //      has drained
    const uint64_t fm0 = __ballot(pa == kSlotDead), fm1 = __ballot(pb == kSlotDead);
    const uint32_t n_free = (uint32_t)__popcll(fm0) + (uint32_t)__popcll(fm1);
    const uint32_t want = n_free / 2u; // events that fit (at most 64)
    if (want) {
      // free slots in order: the requester of rank j takes list[2j] (A) and list[2j + 1] (B)
      if (pa == kSlotDead) list[__popcll(fm0 & below)] = (uint32_t)lane;
      if (pb == kSlotDead) list[__popcll(fm0) + __popcll(fm1 & below)] = (uint32_t)lane + 64u;
      wave_sync_lds();
      const bool need = (uint32_t)lane < want;
      const uint32_t k = want;
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
      if (have_pend && pend_inst != inst && n_free == (uint32_t)kPool && avail == 0) {
        flush_stage(A, st, staged, lane, inst); // staged hits carry the wave's instance
        staged = 0;
        inst = pend_inst; // drained: switch the wave to the claimed instance
        inst_rng = A.inst_id[inst];
        sp = (CScene *)(A.scenes + inst);
        cur_next = cur_end = pend_next;
      }
      const bool use_pend = have_pend && pend_inst == inst;
      const uint32_t extra = use_pend ? pend_end - pend_next : 0u;
      const uint32_t rank = (uint32_t)lane;
      if (need) {
        uint32_t ev = 0;
        bool got = false;
        if (rank < avail) {
          ev = A.inst_first[inst] + cur_next + rank;
          got = true;
        } else if (rank - avail < extra) {
          ev = A.inst_first[inst] + pend_next + (rank - avail);
          got = true;
        }
        if (got) {
          const uint32_t sa = list[2 * rank], sb = list[2 * rank + 1];
          P(W_EV, sa) = ev;
          P(W_N, sa) = 0u;
          P(W_GID, sa) = sb; // photon B's slot, until the emission completes
          P(W_FLAGS, sa) = pack_flags(P_EMIT_DIR, 0, -1, -1, false, 0u);
          P(W_FLAGS, sb) = kSlotReserved;
        }
      }
      const uint32_t take_cur = min(k, avail);
      cur_next += take_cur;
      if (use_pend) {
        const uint32_t take_pend = min(k - take_cur, extra);
        cur_next = pend_next + take_pend;
        cur_end = pend_end;
        have_pend = false;
      }
      wave_sync_lds();
      pa = (int)(P(W_FLAGS, lane) & 15u);
      pb = (int)(P(W_FLAGS, lane + 64) & 15u);
    }
    const bool live = pa != kSlotDead || pb != kSlotDead;
    if (__ballot(live) == 0) {
      if (exhausted && !have_pend) break;
      continue; // the claimed range opens on the next trip
    }
    ++c_trips;
    CScene &S = *sp;

    // ---- the phase held by the most slots runs (ties to the later phase)
    int best = P_EMIT_DIR;
    uint32_t best_n = 0;
#pragma unroll
    for (int q = P_EMIT_DIR; q <= P_RAYLEIGH; ++q) {
      const uint32_t nq = (uint32_t)__popcll(__ballot(pa == q)) + (uint32_t)__popcll(__ballot(pb == q));
      if (nq >= best_n) {
        best_n = nq;
        best = q;
      }
    }
    // ---- gather up to 64 of its slots onto the lanes
    const uint64_t m0 = __ballot(pa == best), m1 = __ballot(pb == best);
    const uint32_t n0 = (uint32_t)__popcll(m0);
    if (pa == best) list[__popcll(m0 & below)] = (uint32_t)lane;
    if (pb == best) {
      const uint32_t r = n0 + (uint32_t)__popcll(m1 & below);
      if (r < 64u) list[r] = (uint32_t)lane + 64u;
    }
    wave_sync_lds();
    const uint32_t total = min(64u, best_n);
    const bool run = (uint32_t)lane < total;
    const uint32_t slot = run ? list[lane] : 0u;
    wave_sync_lds();

    // ---- state of the gathered photon
    Vec x{0.f, 0.f, 0.f}, d{0.f, 0.f, 1.f};
    float e = 0.f, L = 0.f, q_u0 = 0.f;
    uint32_t ev = 0, n = 0, seq = 0;
    unsigned long long t_event = 0;
    int ph = 0, panel = -1, last = -1, q_gid = -1, steps = 0;
    bool back_panel = false;
    if (run) {
      x = Vec{PF(W_X, slot), PF(W_Y, slot), PF(W_Z, slot)};
      d = Vec{PF(W_DX, slot), PF(W_DY, slot), PF(W_DZ, slot)};
      e = PF(W_E, slot);
      L = PF(W_L, slot);
      ev = P(W_EV, slot);
      n = P(W_N, slot);
      t_event = (unsigned long long)P(W_TLO, slot) | ((unsigned long long)P(W_THI, slot) << 32);
      q_u0 = PF(W_U0, slot);
      q_gid = (int)P(W_GID, slot);
      const uint32_t f = P(W_FLAGS, slot);
      ph = (int)((f >> 4) & 1u);
      panel = (int)((f >> 5) & 127u) - 1;
      last = (int)((f >> 12) & 127u) - 1;
      back_panel = ((f >> 19) & 1u) != 0;
      seq = f >> 20;
      steps = (int)P(W_STEPS, slot);
    }
    int phase = best;

    // ---- the one Philox block of this trip
    const bool emission = best <= P_EMIT_TIME;
    const uint32_t sid = emission ? 0u : 1u + (uint32_t)ph;
    const bool draw = run && best != P_SEARCH;
    uint4 w = make_uint4(0u, 0u, 0u, 0u);
    if (draw) {
      w = philox(A.k0, A.k1, make_uint4(n, ev, inst_rng, sid));
      ++n;
    }
    const float4 r = to_unit4(w);
    c_blocks += (draw && !emission) ? 1u : 0u;

    bool hit = false, ended = false;
    int n_tested = 0;
    float h_edep = 0.f;
    int h_proc = 0;
    bool stepped = false, real = false, searched = false, entered = false, trial = false, scattered = false,
         capped = false, emitted = false;

    if (!run) {
      // idle this trip
    } else if (best == P_EMIT_DIR) {
      // block 0 of the event stream: isotropic direction, two source uniforms;
      // the direction waits in d, the rod uniforms in q_u0 and L, the point in x
      const float ct = 2.0f * r.x - 1.0f, stt = hw_sqrt(fmaxf(0.0f, 1.0f - ct * ct));
      d = Vec{stt * cos_rev(r.y), stt * sin_rev(r.y), ct};
      q_u0 = r.z;
      L = r.w;
      x = Vec{S.sx, S.sy, S.sz};
      if (S.src_kind == 2) d = Vec{S.bdx, S.bdy, S.bdz};
      if (S.src_kind == 1) {
        phase = P_EMIT_POS;
      } else if (S.prange_sigma > 0.0f) {
        phase = P_EMIT_RANGE; // block 1 is not needed
        n = 3;
      } else {
        phase = P_EMIT_TIME; // blocks 1 and 3 are not needed
        n = 2;
      }
    } else if (best == P_EMIT_POS) {
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
      const float rr = rd[2] * hw_sqrt(L);
      x = Vec{rd[0] + rr * cos_rev(r.x), rd[1] + rr * sin_rev(r.x), rd[3] + r.y * (rd[4] - rd[3])};
      if (S.prange_sigma > 0.0f) {
        phase = P_EMIT_RANGE;
        n = 3;
      } else {
        phase = P_EMIT_TIME;
      }
    } else if (best == P_EMIT_RANGE) {
      // block 3: the annihilation point
      x = positron_offset(S, x, r);
      phase = P_EMIT_TIME;
      n = 2;
    } else if (best == P_EMIT_TIME) {
      // block 2: event time uniform on [0, T) from the raw 64-bit word; both
      // photons start (A here along +d, B in the pair's other slot along -d)
      t_event = __umul64hi(((unsigned long long)w.y << 32) | w.x, S.duration_ps);
      emitted = true;
      const Vec src = x, sdir = d, bdir = photon_b_dir(S, d, r.z, r.w);
#pragma unroll
      for (int which = 0; which < 2; ++which) {
        Vec xs = src, ds = which ? bdir : sdir;
        float Ls = 0.0f;
        int p0 = P_SEARCH;
        if (S.has_phantom) {
          if (voxel_of(S, xs) >= 0) {
            p0 = P_PHANTOM;
          } else {
            float t0;
            if (ray_box(xs, ds, Vec{S.ox, S.oy, S.oz}, Vec{S.bx, S.by, S.bz}, t0)) {
              xs = Vec{xs.x + t0 * ds.x, xs.y + t0 * ds.y, xs.z + t0 * ds.z};
              Ls += t0;
              p0 = P_PHANTOM;
            }
          }
        }
        if (which == 0) {
          x = xs;
          d = ds;
          e = 511.0f;
          L = Ls;
          n = 0;
          ph = 0;
          seq = 0;
          steps = 0;
          last = -1;
          panel = -1;
          q_gid = -1;
          q_u0 = 0.0f;
          back_panel = false;
          phase = p0;
        } else {
          const uint32_t b = P(W_GID, slot); // the slot reserved for photon B
          PF(W_X, b) = xs.x;
          PF(W_Y, b) = xs.y;
          PF(W_Z, b) = xs.z;
          PF(W_DX, b) = ds.x;
          PF(W_DY, b) = ds.y;
          PF(W_DZ, b) = ds.z;
          PF(W_E, b) = 511.0f;
          PF(W_L, b) = Ls;
          P(W_EV, b) = ev;
          P(W_N, b) = 0u;
          P(W_TLO, b) = (uint32_t)t_event;
          P(W_THI, b) = (uint32_t)(t_event >> 32);
          P(W_STEPS, b) = 0u;
          P(W_GID, b) = (uint32_t)-1;
          PF(W_U0, b) = 0.0f;
          P(W_FLAGS, b) = pack_flags(p0, 1, -1, -1, false, 0u);
        }
      }
    } else if (best == P_PHANTOM) {
      const Lerp lp = lerp_at(e);
      const float mb = lerp1(S.maj_ph, lp);
      const float s = neg_ln(r.x) * rcp(mb);
      const Vec xn{x.x + s * d.x, x.y + s * d.y, x.z + s * d.z};
      const int vox = voxel_of(S, xn);
      if (vox < 0) {
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
              ended = true;
            } else {
              q_u0 = r.w;
              q_gid = -1;
              back_panel = false;
              phase = proc == 2 ? P_KAHN : P_RAYLEIGH;
            }
          }
        }
      }
    } else if (best == P_SEARCH) {
      searched = true;
      float ti;
      const int p = search_panels(S, x, d, last, ti, n_tested);
      if (p < 0) {
        ended = true;
      } else {
        x = Vec{x.x + ti * d.x, x.y + ti * d.y, x.z + ti * d.z};
        L += ti;
        entered = true;
        panel = p;
        CFloat *Pz = (CFloat *)(S.pose + 12 * p);
        x = to_local(Pz, x);
        d = dir_to_local(Pz, d);
        phase = P_PANEL;
        if (++steps > kMaxSteps) capped = ended = true; // bounds panel-to-panel hops as well
      }
    } else if (best == P_PANEL) {
      const Lerp lp = lerp_at(e);
      const float mb = lerp1(s_maj, lp);
      const float s = neg_ln(r.x) * rcp(mb);
      const Vec xn{x.x + s * d.x, x.y + s * d.y, x.z + s * d.z};
      if (!inside_panel(S, xn)) {
        CFloat *Pz = (CFloat *)(S.pose + 12 * panel);
        x = to_global(Pz, x);
        d = dir_to_global(Pz, d);
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
              if (lc.gid >= 0) {
                hit = true;
                h_edep = e;
                h_proc = 1;
              }
              ended = true;
            } else {
              q_u0 = r.w;
              back_panel = true;
              phase = proc == 2 ? P_KAHN : P_RAYLEIGH;
            }
          }
        }
      }
    } else if (best == P_KAHN) {
      trial = true;
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
        if (back_panel && q_gid >= 0) {
          hit = true;
          h_edep = edep;
          h_proc = 2;
        }
        if (!alive) ended = true;
        else phase = back_panel ? P_PANEL : P_PHANTOM;
      }
    } else if (best == P_RAYLEIGH) {
      scattered = true;
      rotate(d, thomson(r.x), q_u0);
      phase = back_panel ? P_PANEL : P_PHANTOM;
    }

    // ---- guard: a photon whose state stopped being finite ends here
    bool bad = false;
    if ((scattered || entered) && nonfinite_state(x, d, e)) {
      bad = ended = true;
      hit = false;
    }
    c_nonfinite += bad ? 1u : 0u;

    // ---- work counters (per lane, summed over the wave at the end)
    c_events += emitted ? 1u : 0u;
    c_steps += stepped ? 1u : 0u;
    c_real += real ? 1u : 0u;
    c_search += searched ? 1u : 0u;
    c_tests += (uint32_t)n_tested;
    c_pruned += (searched && S.ring_reg) ? 1u : 0u;
    c_entries += entered ? 1u : 0u;
    c_trials += trial ? 1u : 0u;
    c_scatter += scattered ? 1u : 0u;
    c_capped += capped ? 1u : 0u;

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

    // ---- store the state back (a finished photon frees its slot)
    if (run) {
      PF(W_X, slot) = x.x;
      PF(W_Y, slot) = x.y;
      PF(W_Z, slot) = x.z;
      PF(W_DX, slot) = d.x;
      PF(W_DY, slot) = d.y;
      PF(W_DZ, slot) = d.z;
      PF(W_E, slot) = e;
      PF(W_L, slot) = L;
      P(W_N, slot) = n;
      P(W_TLO, slot) = (uint32_t)t_event;
      P(W_THI, slot) = (uint32_t)(t_event >> 32);
      PF(W_U0, slot) = q_u0;
      P(W_GID, slot) = (uint32_t)q_gid;
      P(W_STEPS, slot) = (uint32_t)steps;
      P(W_FLAGS, slot) = ended ? (uint32_t)kSlotDead : pack_flags(phase, ph, panel, last, back_panel, seq);
    }
    wave_sync_lds();
  }
  flush_stage(A, st, staged, lane, inst);

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

void launch_transport_pool(const RunArgs &A, const LaunchShape &L, int n_cu, hipStream_t st) {
  const size_t lds = transport_pool_lds_bytes();
  int per_cu = L.blocks_per_cu;
  if (per_cu <= 0) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_transport_pool, kBlock, lds) != hipSuccess || occ < 1)
      occ = 1;
    per_cu = occ;
  }
  // each wave holds 64 events at once
  const uint64_t need = ((uint64_t)A.total_chunks * A.chunk + kBlock - 1) / kBlock;
  uint64_t grid = (uint64_t)n_cu * per_cu;
  if (need < grid) grid = need;
  if (grid == 0) grid = 1;
  hipLaunchKernelGGL(k_transport_pool, dim3((unsigned)grid), dim3(kBlock), lds, st, A);
}

} // namespace gpet
