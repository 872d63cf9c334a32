// transport_common.hpp -- pieces shared by the transport kernels: the photon
// state machine's phases, the per-wave hit staging in LDS and its flush.
#pragma once
#include "gpet_internal.hpp"

namespace gpet {

// emission runs event-stream blocks 0 (direction), 1 (rod point), 3 (positron
// range) and 2 (time, acollinearity), each phase drawing one block in the
// photon-pool kernel; the lane kernel draws blocks 3 and 2 inside P_EMIT_DIR
// (point and beam sources) or P_EMIT_POS (rod sources) and never enters
// P_EMIT_RANGE or P_EMIT_TIME
enum : int {
  P_FETCH = 0, P_EMIT_DIR = 1, P_EMIT_POS = 2, P_EMIT_RANGE = 3, P_EMIT_TIME = 4, P_PHANTOM = 5,
  P_SEARCH = 6, P_PANEL = 7, P_KAHN = 8, P_RAYLEIGH = 9, P_DONE = 10
};

// photon B's direction: -d, turned by the acollinearity angle when it is on
// (theta from words 2, 3 of event block 2 as the length of a 2-D normal
// vector, azimuth uniform)
template <class SC> __device__ __forceinline__ Vec photon_b_dir(SC &S, Vec d, float u_len, float u_phi) {
  Vec b{-d.x, -d.y, -d.z};
  if (S.acol_sigma > 0.0f) {
    // theta stays below 6 sigma (sigma <= 10 deg / 2.355): the Taylor series
    // of sin and cos to theta^9 and theta^10 are exact to float rounding there
    const float th = S.acol_sigma * hw_sqrt(2.0f * neg_ln(u_len)), t2 = th * th;
    const float sn =
        th * (1.0f + t2 * (-1.0f / 6.0f + t2 * (1.0f / 120.0f + t2 * (-1.0f / 5040.0f + t2 * (1.0f / 362880.0f)))));
    const float cs =
        1.0f + t2 * (-0.5f + t2 * (1.0f / 24.0f + t2 * (-1.0f / 720.0f + t2 * (1.0f / 40320.0f +
                                                                                  t2 * (-1.0f / 3628800.0f)))));
    rotate_cs(b, cs, sn, u_phi);
  }
  return b;
}

// positron range: the emission point plus a normal offset per axis (event
// block 3, two Box-Muller pairs)
template <class SC> __device__ __forceinline__ Vec positron_offset(SC &S, Vec x, float4 r) {
  const float a = S.prange_sigma * hw_sqrt(2.0f * neg_ln(r.x));
  const float b = S.prange_sigma * hw_sqrt(2.0f * neg_ln(r.z));
  return Vec{x.x + a * cos_rev(r.y), x.y + a * sin_rev(r.y), x.z + b * cos_rev(r.w)};
}
enum : int { V_STEP = 0, V_ENTER_PANEL = 1, V_EXIT = 2, V_ESCAPE = 3, V_DEAD = 4, V_ENTER_PHANTOM = 5,
             V_EMIT = 6 };

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
// staged hits per wave: flushed once kFlushAt or more are pending, so a trip
// (at most one hit per lane) always fits.  The one output counter is shared
// by every wave of the chip: halving the flush size from 128 costs a quarter
// of the transport rate, 192 gains a few per cent over 128 and larger gains
// nothing more.  28 KB per block leaves room for 5 blocks per CU
constexpr int kFlushAt = 192;
constexpr int kStage = kFlushAt + 64;
constexpr int kStageBytes = 4 * 5 + 8; // event, gid, aux, edep, depth, time

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// per-wave staging area of hits in LDS (structure of arrays)
struct Stage {
  uint32_t *ev, *gid, *aux;
  float *edep, *depth;
  unsigned long long *time;
};

// write `cnt` staged hits of this wave (all of instance `inst`) to the global SoA arrays
__device__ __forceinline__ void flush_stage(const RunArgs &A, const Stage &st, uint32_t cnt, int lane,
                                            uint32_t inst) {
  if (cnt == 0) return;
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(A.hit_count, (unsigned long long)cnt);
  base = __shfl(base, 0);
  wave_sync_lds();
  for (uint32_t k = (uint32_t)lane; k < cnt; k += 64) {
    const unsigned long long i = base + k;
    if (i < A.capacity) {
      A.h_event[i] = st.ev[k];
      A.h_gid[i] = st.gid[k];
      A.h_edep[i] = st.edep[k];
      A.h_depth[i] = st.depth[k];
      A.h_time[i] = st.time[k];
      A.h_aux[i] = st.aux[k];
      if (A.h_inst) A.h_inst[i] = inst;
    }
  }
  wave_sync_lds();
}


// The photon's state is no longer finite (a NaN or an infinity out of the
// arithmetic): checked after each direction change and panel entry, where such
// values would first appear; the photon is then ended and counted.
__device__ __forceinline__ bool nonfinite_state(const Vec &x, const Vec &d, float e) {
  return !isfinite(x.x + x.y + x.z + d.x + d.y + d.z + e);
}

} // namespace gpet
