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

// kernels (transport.hip); det_slots is the largest detector material slot
// count of the launch's scenes (it sizes the LDS tables)
void launch_transport(const RunArgs &A, int det_slots, const LaunchShape &L, int n_cu, hipStream_t st);
void launch_trace(const RunArgs &A, int det_slots, hipStream_t st);
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
  void *pinned = nullptr; // pinned host words for count readbacks and table uploads
  size_t pinned_bytes = 0;
};
// One digitizer pass over the hits of one or more instances.  Instance i owns
// the event ids [first[i], first[i] + n_events[i]); its hits carry i in h_inst
// (h_inst may be null when there is one instance).
struct DigitizeArgs {
  uint64_t n_hits = 0;
  const uint32_t *h_event = nullptr, *h_gid = nullptr, *h_aux = nullptr, *h_inst = nullptr;
  const float *h_edep = nullptr, *h_depth = nullptr;
  const unsigned long long *h_time = nullptr;
  std::vector<uint32_t> first, n_events, cpp, rng; // per instance: range, crystals per panel, RNG id
  std::vector<unsigned long long> duration;        // per instance acquisition length in ps (0: unknown)
  int gid_bits = 1;
  float fwhm_511 = 0.f, e_lo = 0.f, e_hi = 0.f;
  unsigned long long window_ps = 0;
  uint32_t k0 = 0, k1 = 0;
  float panel_depth = 0.f;
  // outputs
  gpet_singles *singles = nullptr;
  gpet_coincidences *coinc = nullptr;
  const gpet_tallies *tallies = nullptr;
  unsigned long long *coinc_per_inst = nullptr; // host, one count per instance (optional)
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
  // one-instance launch table of plain runs (scene + chunk table) and its
  // pinned staging area
  char *d_plain = nullptr, *h_plain = nullptr;
  gpet::DevScene scene{};
  gpet::LaunchShape shape{};
  gpet::DigitizeScratch scratch{};
  // generations of the material list and phantom; a batch made from this
  // context refuses to run once either changed (its scenes point at them)
  uint64_t mat_gen = 0, phantom_gen = 0;
  // optional kernel timing
  bool timing = false;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  float last_ms[2] = {0.f, 0.f};
};

// A batch of instances (scanner + source + event range + RNG id) transported
// by one launch.  Device blob: DevScene[n], then the u32 tables chunk_prefix
// (n + 1), first, count, id (n each), then the shared detector rows and
// majorant, then per-instance poses and rods.
struct gpet_batch {
  gpet_ctx *ctx = nullptr;
  int device = 0;
  uint32_t n = 0;
  std::vector<gpet_geometry_info> info;
  std::vector<uint32_t> first, count, id, cpp;
  std::vector<unsigned long long> duration;
  uint64_t mat_gen = 0, phantom_gen = 0;
  int det_slots = 0;
  int gid_bits = 1;
  uint64_t total_events = 0;
  uint32_t chunk = 1024;
  gpet::LaunchShape shape{};
  char *d_blob = nullptr;
  uint32_t *d_prefix = nullptr;
  gpet::RunArgs base{}; // table pointers and controls; hits and seed set per call
};
