// transport_common.hpp -- pieces shared by the transport kernels: the photon
// state machine's phases, the per-wave hit staging in LDS and its flush.
#pragma once
#include "gpet_internal.hpp"

namespace gpet {

enum : int {
  P_FETCH = 0, P_EMIT_DIR = 1, P_EMIT_POS = 2, P_EMIT_TIME = 3, P_PHANTOM = 4, P_SEARCH = 5,
  P_PANEL = 6, P_KAHN = 7, P_RAYLEIGH = 8, P_DONE = 9
};
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


} // namespace gpet
