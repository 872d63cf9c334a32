// gpet_internal.hpp -- host-side context and the launch interface between the
// C-ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/gpet.h"
#include "gpet_device.hpp"

namespace gpet {

// Device outputs and controls of one transport launch over a table of
// instances (one instance for a plain run).  Work is handed out in chunks of
// `chunk` consecutive events of one instance; chunk c of the launch belongs to
// the instance i with chunk_prefix[i] <= c < chunk_prefix[i + 1].
struct RunArgs {
  const DevScene *scenes;       // n_inst scenes (device)
  const uint32_t *chunk_prefix; // n_inst + 1 (device)
  const uint32_t *inst_first;   // first event id of each instance's range (device)
  const uint32_t *inst_count;   // events of each instance (device)
  const uint32_t *inst_id;      // instance id used in random-number counters (device)
  uint32_t n_inst, chunk, total_chunks;
  uint32_t first, n; // plain runs: event range [first, first + n) (trace indexing)
  uint32_t k0, k1;
  uint32_t *h_event, *h_gid, *h_aux, *h_inst;
  float *h_edep, *h_depth;
  unsigned long long *h_time;
  unsigned long long capacity;
  unsigned long long *hit_count; // device
  uint32_t *work;                // device event-fetch counter
  unsigned long long *stats;     // device, 10 counters (gpet_stats order)
  // trace mode
  int32_t *vint;
  float *vflt;
  int32_t *vcount;
  int max_vertices;
  uint32_t search_batch; // lanes of a wave that must wait for a panel search before it runs
  uint32_t schedule;     // 0: all phases each trip; 1: the most-populated phase only
};

struct LaunchShape {
  int blocks_per_cu = 0;      // blocks of 256 lanes per CU; 0 = the occupancy limit
  uint32_t search_batch = 48; // see RunArgs::search_batch
  uint32_t schedule = 0;      // see RunArgs::schedule
};
size_t transport_lds_bytes(int det_slots);

// kernels (transport.hip)
void launch_transport(const DevScene &S, const RunArgs &A, const LaunchShape &L, int n_cu,
                      hipStream_t st);
void launch_trace(const DevScene &S, const RunArgs &A, hipStream_t st);
void launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t st);
void launch_philox(uint64_t seed, const uint32_t *ctr, uint32_t n, uint32_t *out, hipStream_t st);
void launch_locate(const DevScene &S, uint32_t n, const float *xyz, int32_t *ids6, hipStream_t st);
void launch_ray_locate(const DevScene &S, uint32_t n, const float *o, const float *d, int ns,
                       float step, float *t_in, int32_t *ids6, hipStream_t st);
void launch_compton(float e, uint32_t n, uint64_t seed, float *c, float *eo, int32_t *tr,
                    hipStream_t st);
void launch_rayleigh(uint32_t n, uint64_t seed, float *c, hipStream_t st);

// digitizer (digitize.hip)
struct DigitizeScratch {
  void *buf = nullptr;
  size_t bytes = 0;
  void *pinned = nullptr; // small pinned host buffer for count readbacks
};
struct DigitizeArgs {
  uint64_t n_hits;
  const uint32_t *h_event, *h_gid, *h_aux;
  const float *h_edep, *h_depth;
  const unsigned long long *h_time;
  uint32_t first_event;
  uint64_t n_events;
  int gid_bits, event_bits;
  int crystals_per_panel, n_crystals;
  float fwhm_511, e_lo, e_hi;
  unsigned long long window_ps;
  uint32_t k0, k1, instance;
  float panel_depth;
  // outputs
  gpet_singles *singles;
  gpet_coincidences *coinc;
  const gpet_tallies *tallies;
};
// returns GPET_OK or an error code; fills counts
int run_digitize(DigitizeArgs &D, DigitizeScratch &scr, hipStream_t st, std::string &err);
void free_scratch(DigitizeScratch &scr);

} // namespace gpet

struct gpet_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 256;
  std::string err;
  // materials
  int n_mat = 0;
  std::vector<gpet_material> mats;
  gpet_physics phys{};
  std::vector<float> mu_host;      // [n_mat][4][kNodes] nominal density
  std::vector<float> mu_mass_host; // [n_mat][4][kNodes] per g/cm^3
  float4 *d_mu = nullptr, *d_mu_mass = nullptr, *d_mu_det = nullptr;
  float *d_maj_det = nullptr, *d_maj_ph = nullptr;
  std::vector<float> maj_det_host;
  // geometry
  bool have_geometry = false;
  gpet_geometry_info info{};
  float *d_pose = nullptr;
  // phantom
  uint8_t *d_vmat = nullptr;
  float *d_vden = nullptr;
  // source
  bool have_source = false;
  float *d_rods = nullptr, *d_rod_cum = nullptr;
  // device controls: [0] work (u32 x2), [1] hit count, [2..11] stats
  unsigned long long *d_ctrl = nullptr;
  unsigned long long *h_ctrl = nullptr; // pinned mirror of d_ctrl
  gpet::DevScene scene{};
  gpet::LaunchShape shape{};
  gpet::DigitizeScratch scratch{};
  // optional kernel timing
  bool timing = false;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  float last_ms[2] = {0.f, 0.f};
};
