// gpet_internal.hpp -- host-side context and the launch interface between the
// C-ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/gpet.h"
#include "gpet_device.hpp"

namespace gpet {

// Surrogate entry domain and outcome classes on the device (see
// gpet_surrogate_spec in the C header).
struct SurSpecD {
  int half, n_ebins;
  int chalf; // half width of the class neighbourhood (>= half)
  float e_min, ebin, tol, max_slope, front_tol;
};

// Device control words of a context (u64): [0] spare, [1] hit count, [2, 2 + kStatCount) work counters in gpet_stats order,
// [kCtrlPairs] spare (pairs and surrogate entries are counted at kCtrlPairWord).
constexpr int kStatCount = 13;
constexpr int kCtrlPairs = 2 + kStatCount;
constexpr int kCtrlWords = kCtrlPairs + 1;
// the event-claim counter of the transport sits on a cache line of its own,
// apart from the hit counter: both take one atomic per wave now and then from
// every CU, and sharing a line serialises them (about 5 % of a launch)
constexpr int kCtrlWorkWord = 32;
// the pair / surrogate-entry counter likewise (one atomic per wave and trip
// that records or queues an entry)
constexpr int kCtrlPairWord = 48;
constexpr int kCtrlAlloc = 64; // u64 words of the control buffer

// Transport kernel modes
enum : int { kModePlain = 0, kModeTrace = 1, kModeRecord = 2, kModeSurrogate = 3 };

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
  unsigned long long *stats;     // device, kStatCount counters (gpet_stats order)
  // trace mode
  int32_t *vint;
  float *vflt;
  int32_t *vcount;
  int max_vertices;
  uint32_t search_batch; // lanes of a wave that must wait for a panel search before it runs
  uint32_t schedule;     // 0: all phases each trip (searches at its end); 1: the most-populated phase only;
                         // 2: plain runs use the per-wave photon pools (k_transport_pool)
  // record and surrogate modes: photons entering their first panel inside the
  // surrogate domain get an entry with features px (6 per entry).  Record:
  // label and flags once the photon leaves the panel.  Surrogate: an entry
  // queue (event, meta = photon | panel << 1 | module << 8, one anchor word
  // per layer i_t | i_a << 16, entry energy, entry time) and the photon ends.
  SurSpecD sur;
  float *px;
  int32_t *plabel;
  uint32_t *pflags, *pevent;
  uint32_t *qev, *qmeta, *qanchor;
  float *qe;
  unsigned long long *qtime;
  unsigned long long *pcount; // device: pairs / queue entries produced
  unsigned long long *pholes = nullptr; // device (surrogate): queue slots reserved but left empty
  unsigned long long pcap;
};

struct LaunchShape {
  int blocks_per_cu = 0;      // blocks of 256 lanes per CU; 0 = the occupancy limit
  uint32_t search_batch = 16; // see RunArgs::search_batch
  uint32_t schedule = 0;      // see RunArgs::schedule
};
size_t transport_lds_bytes();

// kernels (transport.hip)
void launch_transport(const RunArgs &A, const LaunchShape &L, int n_cu, hipStream_t st,
                      int mode = kModePlain);
// plain runs with per-wave photon pools (LaunchShape::schedule 2)
void launch_transport_pool(const RunArgs &A, const LaunchShape &L, int n_cu, hipStream_t st);
void launch_trace(const RunArgs &A, hipStream_t st);
void launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t st);
void launch_zero3(uint32_t *a, size_t na, uint32_t *b, size_t nb, uint32_t *c, size_t nc, hipStream_t st);
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
  // a fixed buffer (the library's static device scratch): never grown or
  // freed, no pinned words; calls that need more than `bytes` are refused
  bool fixed = false;
  // the instance table last uploaded into buf, and where (not kept for the
  // fixed buffer, which other contexts share)
  const void *tab_at = nullptr;
  std::vector<uint32_t> tab_last;
};
// host words a call on the fixed scratch stages its readbacks and uploads in
constexpr size_t kFixedHostWords = 64;
// size of the static device scratch of gpet_digitize_noalloc
constexpr size_t kFixedScratchBytes = GPET_DIGITIZE_NOALLOC_SCRATCH_BYTES;
// Device address of the static digitizer scratch on `device` (which must be
// the current device); looked up once per device and kept.  Null on failure.
void *fixed_scratch(int device, std::string &err);
// One digitizer pass over the hits of one or more instances.  Instance i owns
// the event ids [first[i], first[i] + n_events[i]); its hits carry i in h_inst
// (h_inst may be null when there is one instance).
constexpr int kLayerWords = 1 + 3 * kMaxLayers;
// layer words of a scene: count, first ids, n_t, n_a
inline void layer_words(const DevScene &S, std::vector<uint32_t> &out) {
  out.push_back((uint32_t)S.n_layers);
  for (int k = 0; k < kMaxLayers; ++k) out.push_back(k < S.n_layers ? (uint32_t)S.layer[k].base : 0u);
  for (int k = 0; k < kMaxLayers; ++k) out.push_back(k < S.n_layers ? (uint32_t)S.layer[k].n_t : 1u);
  for (int k = 0; k < kMaxLayers; ++k) out.push_back(k < S.n_layers ? (uint32_t)S.layer[k].n_a : 1u);
}

struct DigitizeArgs {
  uint64_t n_hits = 0;
  const uint32_t *h_event = nullptr, *h_gid = nullptr, *h_aux = nullptr, *h_inst = nullptr;
  const float *h_edep = nullptr, *h_depth = nullptr;
  const unsigned long long *h_time = nullptr;
  std::vector<uint32_t> first, n_events, cpp, rng; // per instance: range, crystals per panel, RNG id
  std::vector<uint32_t> cpm;                        // per instance: crystals per module
  std::vector<uint32_t> ncr;                        // per instance: crystals of the scanner
  uint32_t readout = 0;                             // GPET_READOUT_*
  // energy-window sweep: windows and host counts (window-major, one per instance)
  std::vector<float> sweep_lo, sweep_hi;
  uint64_t *sweep_out = nullptr;
  std::vector<unsigned long long> duration;        // per instance acquisition length in ps (0: unknown)
  int gid_bits = 1;
  float fwhm_511 = 0.f, e_lo = 0.f, e_hi = 0.f;
  unsigned long long window_ps = 0;
  uint32_t k0 = 0, k1 = 0;
  float panel_depth = 0.f;
  // detector response options: time and depth blur sigmas (ps, mm; 0 = off),
  // dead time (GPET_DEAD_*, unit level GPET_READOUT_*, length in ps)
  float time_sigma = 0.f, doi_sigma = 0.f;
  uint32_t dead_mode = 0, dead_level = 0;
  unsigned long long dead_ps = 0;
  // light sharing: Philox word 0 below this moves the crystal (0 = off, 2^32 = always)
  unsigned long long ls_thresh = 0;
  // per instance kLayerWords words: layer count, then first crystal id, n_t and
  // n_a of up to kMaxLayers layers (the crystal id layout inside a module)
  std::vector<uint32_t> layers;
  // outputs
  gpet_singles *singles = nullptr;
  gpet_coincidences *coinc = nullptr;
  const gpet_tallies *tallies = nullptr;
  unsigned long long *coinc_per_inst = nullptr; // host, one count per instance (optional)
};
// Waits for the stream by polling it: the host thread stays awake, so the
// work it queues after a long kernel starts without a blocking wait's
// wake-up delay.  Returns what the stream reports (hipSuccess when idle).
hipError_t wait_stream(hipStream_t st);

// exclusive prefix sum of n u32 in place; tmp holds scan_tmp_words(n) words;
// `total` (may be null, may be pinned host memory) receives the sum
size_t scan_tmp_words(size_t n);
void scan_exclusive_u32(uint32_t *a, size_t n, uint32_t *tmp, hipStream_t st, uint32_t *total = nullptr);

// Surrogate entry queue (library scratch): SoA of `cap` entries
// Surrogate queue: a wave reserves kQueueResv slots at a time (one atomic per
// reservation); the slots its last reservation leaves unused are marked by
// meta = kQueueHole (features zero) and carry no entry.
constexpr uint32_t kQueueResv = 32;
constexpr uint32_t kQueueHole = 0xFFFFFFFFu;

struct SurQueue {
  size_t cap = 0;
  void *blob = nullptr;
  float *x = nullptr, *e = nullptr;
  uint32_t *ev = nullptr, *meta = nullptr, *anchor = nullptr, *cls = nullptr, *pos = nullptr, *scan_tmp = nullptr;
  unsigned long long *time = nullptr;
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
  // device control words (see kCtrlWords)
  unsigned long long *d_ctrl = nullptr;
  unsigned long long *h_ctrl = nullptr; // pinned mirror of d_ctrl
  // one-instance launch table of plain runs (scene + chunk table) and its
  // pinned staging area
  char *d_plain = nullptr, *h_plain = nullptr;
  gpet::DevScene scene{};
  gpet::LaunchShape shape{};
  gpet::DigitizeScratch scratch{};
  void *fixed_scratch = nullptr; // this device's static digitizer scratch (not owned)
  gpet::SurQueue squeue{};
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
  std::vector<uint32_t> first, count, id, cpp, cpm, ncr;
  std::vector<uint32_t> layers; // kLayerWords per instance (see DigitizeArgs)
  std::vector<unsigned long long> duration;
  uint64_t mat_gen = 0, phantom_gen = 0;
  int det_slots = 0;
  int gid_bits = 1;
  uint64_t total_events = 0;
  uint32_t chunk = 1024;
  gpet::LaunchShape shape{};
  char *d_blob = nullptr;
  uint32_t *d_prefix = nullptr;
  hipGraphExec_t graph = nullptr; // captured transport step (gpet_batch_graph_capture)
  gpet::RunArgs base{}; // table pointers and controls; hits and seed set per call
};

// The surrogate network: a ReLU MLP with FP32 master weights and Adam moments,
// padded BF16 weight copies for the matrix cores, and a workspace of `cap`
// rows (activations, logits, gradient buffers).
struct gpet_mlp {
  gpet_ctx *ctx = nullptr;
  int device = 0;
  std::vector<int> size;  // layer widths, input first
  std::vector<int> psize; // padded widths: input to a multiple of 64, the others of 128
  int n_layers = 0;       // weight matrices
  size_t n_params = 0;
  std::vector<size_t> w_off, b_off;                  // offsets in the packed parameter vector
  // factored output: the first n_first outputs are the energy head, then
  // n_groups blocks of n_second positions (energy class e > 0 uses block
  // (e - 1) n_groups / (n_first - 1)), with an fp32 offset table
  // [n_first - 1][n_second] at tab_off in the packed parameters (n_first = 0:
  // one joint softmax)
  int n_first = 0, n_second = 0, n_groups = 0;
  size_t tab_off = 0;
  float *master = nullptr, *m = nullptr, *v = nullptr; // packed fp32 (per layer W [out][in], then b)
  std::vector<uint16_t *> wb;                        // padded bf16 weights per layer [out_pad][in_pad]
  std::vector<float *> gw;                           // padded fp32 weight gradients per layer
  float *gb = nullptr;                               // packed gradients (biases at b_off)
  float *bp = nullptr;                               // padded fp32 biases, bp_stride per layer
  int bp_stride = 0;
  uint64_t adam_t = 0;
  uint32_t cap = 0;
  std::vector<uint16_t *> act; // bf16 input of every layer (act[0]: packed network input)
  float *logits = nullptr;
  uint16_t *dz[2] = {nullptr, nullptr};
  int32_t *yb = nullptr;
  uint32_t *idx = nullptr;
  double *row_loss = nullptr, *loss_sum = nullptr;
  int32_t *erow = nullptr;  // energy class of each row (factored output)
  uint32_t *flag = nullptr; // bit 0: a label outside the classes
  float *part = nullptr, *part_b = nullptr; // split-K partial weight gradients, partial bias sums
  void *tstats = nullptr; // float2 (max, sum of exponentials) per row and 128-class tile of the logits
};

namespace gpet {
// Network inference on the first nq entries of a surrogate queue: classes
// sampled from the softmax (Philox key (k0, k1), counter (0, event, inst_rng,
// 4 + photon)), then one synthetic hit per entry whose class is not 0,
// appended after *hit_count (device) in queue order.  d_scene: the scene the
// entries were made in (device).  Adds the class-0 count to *n_none.
int surrogate_hits(gpet_mlp *q, const DevScene *d_scene, const SurSpecD &P, const SurQueue &Q, uint32_t nq,
                   uint32_t k0, uint32_t k1, uint32_t inst_rng, const RunArgs &hits, hipStream_t st, std::string &err,
                   uint64_t *n_none);
} // namespace gpet
