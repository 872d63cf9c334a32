/*
 * gpet.h -- C ABI of the MI355X (gfx950) multi-layer PET Monte Carlo library.
 *
 * Monte Carlo transport of back-to-back 511 keV annihilation photon pairs
 * through an optional voxelized phantom and a parameterized detector
 * hierarchy panel -> module -> layer -> crystal, followed by a crystal-level
 * digitizer (per-crystal energy summing, Gaussian energy blurring, energy
 * window, coincidence sorting).  Method: "Extending gPET for Multi-Layer PET
 * Simulation", Sec. 2.1 (hierarchy, inputs, layer selection by depth during
 * in-panel Woodcock transport) and Sec. 2.3 (source, 3 ns coincidence
 * window, 16 % energy resolution).
 *
 * Conventions
 *  - Units: mm, keV, ps, g/cm^3.  Arithmetic on the GPU is FP32 (event times
 *    are integer ps).
 *  - Every call returns gpet_status; GPET_OK is 0, errors are negative and
 *    gpet_last_error() returns a message for the context.  No C++ exception
 *    crosses this boundary.
 *  - Input descriptors (materials, scanner, phantom, source) are HOST memory
 *    and are copied during the call; the caller keeps ownership.
 *  - Output buffers (hits, singles, coincidences, tallies) are caller-owned
 *    DEVICE memory on the context's device, passed as raw pointers plus a
 *    capacity.  When an output needs more room than its capacity the call
 *    writes nothing past the capacity, stores the required size in `count`
 *    and returns GPET_ERR_CAPACITY; a rerun with a larger buffer gives the
 *    same results (all random numbers come from counter-based Philox streams
 *    keyed by the seed and the event id).
 *  - All work is ordered on the context's HIP stream.  gpet_transport and
 *    gpet_digitize synchronize that stream before returning counts.
 *  - A context is used by one host thread at a time.
 *  - The library owns internal device scratch (tables, sort buffers); it is
 *    freed by gpet_ctx_destroy.
 */
#ifndef GPET_H
#define GPET_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gpet_status;
#define GPET_OK 0
#define GPET_ERR_ARG (-1)
#define GPET_ERR_GEOMETRY (-2)
#define GPET_ERR_STATE (-3)
#define GPET_ERR_CAPACITY (-4)
#define GPET_ERR_HIP (-5)
#define GPET_ERR_UNSUPPORTED (-6)

#define GPET_MAX_ELEMENTS 8
#define GPET_MAX_MATERIALS 8
#define GPET_MAX_LAYERS 4
#define GPET_MAX_PANELS 64
#define GPET_MAX_RODS 1024

/* interaction processes a material takes part in (bit mask) */
#define GPET_PROC_PHOTOELECTRIC 1u
#define GPET_PROC_COMPTON 2u
#define GPET_PROC_RAYLEIGH 4u

typedef struct gpet_ctx gpet_ctx;

/* Create a context on HIP device `device`, ordering its work on `hip_stream`
 * (a hipStream_t; NULL = the null stream). */
gpet_status gpet_ctx_create(int device, void *hip_stream, gpet_ctx **out);
void gpet_ctx_destroy(gpet_ctx *ctx);
const char *gpet_last_error(const gpet_ctx *ctx);
/* Change the stream later work is ordered on. */
gpet_status gpet_ctx_set_stream(gpet_ctx *ctx, void *hip_stream);

/* ---------------------------------------------------------------------- */
/* Materials and physics.  Crystal and inter-crystal interval materials and  */
/* their densities are detector inputs (Sec. 2.1).  Attenuation per process: */
/*   Compton       Klein-Nishina per electron,                             */
/*   photoelectric k_pe * Z^4 / E^3 per atom (E in MeV),                    */
/*   Rayleigh      k_rayleigh * Z^2 / E^2 per atom,                         */
/* tabulated on 1 keV nodes 1..511 keV with linear interpolation.           */
/* ---------------------------------------------------------------------- */
typedef struct {
  double density_g_cm3;  /* nominal density (detector); phantom voxels carry their own */
  int32_t n_elements;    /* 1..GPET_MAX_ELEMENTS */
  uint32_t processes;    /* GPET_PROC_* mask */
  int32_t Z[GPET_MAX_ELEMENTS];
  double A[GPET_MAX_ELEMENTS];             /* g/mol */
  double mass_fraction[GPET_MAX_ELEMENTS]; /* sums to 1 */
} gpet_material;

typedef struct {
  double k_pe;        /* cm^2 MeV^3 per atom per Z^4 */
  double k_rayleigh;  /* cm^2 MeV^2 per atom per Z^2 (0 disables Rayleigh) */
  double e_cut_kev;   /* photons below this energy deposit it locally and stop */
} gpet_physics;

/* Replaces the material list (ids 0..n-1).  Invalidates geometry and phantom. */
gpet_status gpet_materials_set(gpet_ctx *ctx, int32_t n, const gpet_material *materials,
                               const gpet_physics *physics);

/* ---------------------------------------------------------------------- */
/* Detector geometry (Sec. 2.1, Fig. 1): panels placed in repetition mode    */
/* (count and rotation step) or non-repetition mode (explicit pose per      */
/* panel); each panel holds a grid of modules; each module an ordered list  */
/* of layers along the panel depth; each layer its own crystal array.       */
/*                                                                          */
/* Panel-local frame: depth along the panel normal pointing away from the   */
/* axis (0 at the front face), t tangential, a axial.  The panel box is     */
/* depth [0, depth_mm) x t [-width/2, width/2) x a [-length/2, length/2).   */
/* Modules tile the (t, a) face, centred, with gaps between them.  Layer l  */
/* covers depth [depth0, depth0 + thickness); its crystal (i_t, i_a) lies   */
/* in the pitch cell starting at offset + i * pitch from the module edge,   */
/* centred in the cell.  Space in a layer outside its crystals is the       */
/* layer's interval material; module gaps, inter-layer gaps and the rest of */
/* the panel are the fill material.  Outside panels and phantom: vacuum.    */
/* ---------------------------------------------------------------------- */
typedef struct {
  double depth0_mm, thickness_mm;
  int32_t n_t, n_a;
  double cryst_t_mm, cryst_a_mm;
  double pitch_t_mm, pitch_a_mm;
  double offset_t_mm, offset_a_mm;
  int32_t crystal_material, interval_material;
} gpet_layer;

#define GPET_PLACE_REPEAT 0   /* panel k at angle phi0 + 2 pi k / n_panels */
#define GPET_PLACE_EXPLICIT 1 /* poses[] given per panel */

typedef struct {
  int32_t placement;
  int32_t n_panels;                  /* 1..GPET_MAX_PANELS */
  double radius_mm, phi0_rad, z0_mm; /* repeat mode: front-face distance from the z axis */
  const double *poses;               /* explicit mode: n_panels x 12 doubles:
                                        front-face centre xyz, depth axis, t axis, a axis */
  double depth_mm, width_mm, length_mm;
  int32_t mod_n_t, mod_n_a;
  double mod_t_mm, mod_a_mm, gap_t_mm, gap_a_mm;
  int32_t fill_material;
  int32_t n_layers; /* 1..GPET_MAX_LAYERS */
  gpet_layer layers[GPET_MAX_LAYERS];
} gpet_scanner;

/* Global crystal id (gid) layout:
 *   gid = panel * crystals_per_panel + module * crystals_per_module
 *         + layer_base[layer] + i_a * n_t(layer) + i_t,
 * module = m_a * mod_n_t + m_t. */
typedef struct {
  int32_t n_crystals, crystals_per_panel, crystals_per_module;
  int32_t layer_base[GPET_MAX_LAYERS];
} gpet_geometry_info;

/* Validates and uploads the scanner.  Errors: GPET_ERR_GEOMETRY for
 * non-positive sizes, crystals wider than their pitch, layers outside the
 * panel depth or overlapping, crystal arrays outside the module, or more
 * than 2^20 crystals; GPET_ERR_STATE if no materials are set. */
gpet_status gpet_geometry_create(gpet_ctx *ctx, const gpet_scanner *scanner, gpet_geometry_info *info);

/* ---------------------------------------------------------------------- */
/* Voxelized phantom, transported with Woodcock tracking against the        */
/* node-wise maximum attenuation over its voxels.  Voxel (ix, iy, iz) is     */
/* material[(iz*ny + iy)*nx + ix] with density density[...] (g/cm^3); the    */
/* box is [origin, origin + n*voxel) per axis.  A photon that leaves the box */
/* does not re-enter it.  Passing NULL removes the phantom (vacuum).         */
/* ---------------------------------------------------------------------- */
typedef struct {
  int32_t nx, ny, nz;
  double voxel_mm[3];
  double origin_mm[3];
  const uint8_t *material; /* host */
  const float *density;    /* host */
} gpet_phantom;

gpet_status gpet_phantom_set(gpet_ctx *ctx, const gpet_phantom *phantom);

/* ---------------------------------------------------------------------- */
/* Source (Sec. 2.3): each event is one annihilation at the emission site     */
/* (no positron range) sending photon A along +d and photon B along -d at     */
/* 511 keV, d isotropic (BEAM: d fixed).  Event times are uniform on          */
/* [0, duration_ps) (a fixed number of decays of a constant activity).       */
/* Optional physics the paper leaves out (0 = off, the paper's setting):     */
/*  acolinearity_fwhm_deg  photon B leaves at polar angle theta from -d,      */
/*                         theta the length of a 2-D normal vector of this   */
/*                         FWHM per component (0.5 deg in water), azimuth     */
/*                         uniform;                                           */
/*  positron_range_fwhm_mm the annihilation point is the emission point plus */
/*                         a 3-D normal offset of this FWHM per axis (Sec. 4 */
/*                         quotes 0.102 mm for 18F).                          */
/* ---------------------------------------------------------------------- */
#define GPET_SRC_POINT 0
#define GPET_SRC_CYLINDERS 1 /* rods (cx, cy, radius, z0, z1), uniform activity density */
#define GPET_SRC_BEAM 2

typedef struct {
  int32_t kind;
  double pos_mm[3];   /* POINT, BEAM */
  double dir[3];      /* BEAM */
  int32_t n_rods;     /* CYLINDERS: 1..GPET_MAX_RODS */
  const double *rods; /* host, n_rods x 5 */
  uint64_t duration_ps;
  double acolinearity_fwhm_deg;  /* 0 .. 10 */
  double positron_range_fwhm_mm; /* 0 .. 10 */
} gpet_source;

gpet_status gpet_source_set(gpet_ctx *ctx, const gpet_source *source);

/* ---------------------------------------------------------------------- */
/* Transport                                                                 */
/* ---------------------------------------------------------------------- */
/* Hit list, one entry per photoelectric or Compton interaction inside a
 * crystal (Sec. 2.1: each interaction labelled with crystal, layer, module
 * and panel; all four follow from gid).  SoA device arrays of `capacity`
 * entries.  Order of entries is unspecified. */
typedef struct {
  uint32_t *event;   /* event id */
  uint32_t *gid;     /* global crystal id */
  float *edep_kev;   /* deposited energy (includes a below-cutoff remainder) */
  float *depth_mm;   /* panel-local depth of the interaction */
  uint64_t *time_ps; /* event time + time of flight, rounded to ps */
  uint32_t *aux;     /* bit 0 photon (0 = A, 1 = B); bits 1-2 process (1 PE, 2 Compton);
                        bits 8-31 index of the hit within its photon */
  uint32_t *instance; /* index of the hit's instance in its batch (0 for a plain run);
                         may be NULL for plain runs, required by gpet_batch_transport */
  uint64_t capacity;
  uint64_t count;    /* out: hits produced */
} gpet_hits;

/* Work counters of a transport call (for roofline accounting). */
typedef struct {
  uint64_t events, panel_entries, steps, real_interactions, kahn_trials, panel_searches,
      rng_blocks, capped, scatters;
  uint64_t wave_trips;      /* loop trips summed over wavefronts (64 lanes each) */
  uint64_t panel_tests;     /* panel boxes tested by the searches */
  uint64_t pruned_searches; /* searches from inside a repeated ring that tested only the panels
                               whose azimuth range the ray sweeps */
  uint64_t nonfinite;       /* photons ended because their position, direction or energy stopped
                               being finite (checked after each scatter and panel entry; 0 expected) */
} gpet_stats;

/* Transport events [first_event, first_event + n_events) with key `seed`.
 * `instance` enters every random-number counter so that independent runs can
 * share event ids.  stats may be NULL.  first_event + n_events <= 2^32. */
gpet_status gpet_transport(gpet_ctx *ctx, uint64_t first_event, uint64_t n_events, uint64_t seed,
                           uint32_t instance, gpet_hits *hits, gpet_stats *stats);

/* ---------------------------------------------------------------------- */
/* Digitizer                                                                 */
/*  adder:  hits of one event in one crystal form a single: energy = sum of  */
/*          deposits, time = earliest hit time, depth = energy-weighted mean;*/
/*  readout (Sec. 2.1 readout levels): at module (panel) level the crystal   */
/*          singles of one event in one module (panel) merge into one single:*/
/*          energies summed, earliest time, crystal id and depth of the      */
/*          largest deposit (the lower id on a tie);                         */
/*  blur:   E + N(0,1) * fwhm_511 * sqrt(511 E) / 2.3548 (16 % at 511 keV);   */
/*          optional time blur (timing resolution): t + rint(N(0,1) *        */
/*          time_fwhm_ps / 2.3548), not below 0; optional depth blur (DOI    */
/*          resolution): depth + N(0,1) * doi_fwhm_mm / 2.3548;              */
/*  light:  optional light sharing: the crystal read as a neighbour        */
/*          (light_sharing, below);                                          */
/*  dead:   optional dead time per crystal, module or panel (dead_time_level)*/
/*          over the blurred singles in (time, list position) order: one is  */
/*          lost when the previous single of its unit (paralyzable) or the   */
/*          last one kept (non-paralyzable) came less than dead_time_ps      */
/*          earlier; lost singles stay listed and enter no window;           */
/*  window: e_lo <= blurred E <= e_hi;                                       */
/*  sorter: windowed singles in (time, list position) order; a window of    */
/*          window_ps (inclusive) opens at the earliest unused single and    */
/*          does not retrigger; exactly two singles in different panels make */
/*          a coincidence, any other content is discarded.                   */
/* ---------------------------------------------------------------------- */
typedef struct {
  double fwhm_511;    /* relative FWHM at 511 keV (0.16) */
  double e_lo_kev, e_hi_kev;
  uint64_t window_ps; /* 3000 */
  uint64_t seed;      /* key of the blur stream */
  uint32_t instance;
  uint64_t first_event, n_events; /* event range the hits came from */
  uint32_t readout;   /* GPET_READOUT_CRYSTAL, _MODULE or _PANEL */
  /* Energy-window sweep (Sec. 2.3 evaluates 150/250/350/450-700 keV): for
   * each of n_sweep extra windows [sweep_lo_kev[w], sweep_hi_kev[w]] the
   * coincidences of the same blurred singles are counted (not listed) into
   * sweep_coincidences[w * n_instances + i] (host memory; n_instances is 1
   * for gpet_digitize).  The arrays are read and written during the call and
   * may be NULL when n_sweep is 0.  The listed outputs keep the main window. */
  uint32_t n_sweep;
  const double *sweep_lo_kev, *sweep_hi_kev;
  uint64_t *sweep_coincidences;
  /* Detector response the paper leaves to analytic models (Sec. 4); 0 = off.
   * Time deviate: words 2, 3 of the energy-blur Philox block; depth deviate:
   * Philox counter (gid, event, instance, 6). */
  double time_fwhm_ps;       /* 0 .. 1e6 */
  double doi_fwhm_mm;        /* 0 .. 100 */
  uint64_t dead_time_ps;
  uint32_t dead_time_mode;   /* GPET_DEAD_NONE, _PARALYZABLE, _NONPARALYZABLE */
  uint32_t dead_time_level;  /* GPET_READOUT_CRYSTAL, _MODULE or _PANEL */
  /* Light sharing (Sec. 4, analytic): probability 0..1 that a single's crystal
   * is read as one of its existing edge neighbours in the same layer and
   * module (order t-1, t+1, a-1, a+1), chosen uniformly; Philox counter (gid,
   * event, instance, 8): word 0 < floor(p 2^32) moves it, neighbour
   * (word 1 * count) >> 32.  Applied after the blur; the list keeps its order. */
  double light_sharing;
} gpet_digitizer;

enum { GPET_READOUT_CRYSTAL = 0, GPET_READOUT_MODULE = 1, GPET_READOUT_PANEL = 2 };
enum { GPET_DEAD_NONE = 0, GPET_DEAD_PARALYZABLE = 1, GPET_DEAD_NONPARALYZABLE = 2 };

/* Singles in (instance, event, gid) order; at module or panel readout gid is
 * the crystal of the largest deposit and edep the readout unit's sum. */
typedef struct {
  uint32_t *event, *gid;
  float *edep_kev;    /* summed deposit */
  float *energy_kev;  /* blurred */
  float *depth_mm;
  uint64_t *time_ps;
  uint32_t *in_window; /* bit 0: blurred energy inside the main window; bit 1:
                          lost to dead time.  A single enters the coincidence
                          sorter when in_window == 1 */
  uint32_t *instance; /* optional (may be NULL): instance index of the single */
  uint64_t capacity;
  uint64_t count;     /* out */
  uint64_t windowed;  /* out: singles inside the (main) energy window and not lost */
} gpet_singles;

/* Coincidences as index pairs into the singles arrays, earlier single first,
 * ordered by (instance, time of their first single). */
typedef struct {
  uint32_t *first, *second;
  uint64_t capacity;
  uint64_t count; /* out */
} gpet_coincidences;

/* Optional histograms (device arrays, accumulated, not cleared). */
typedef struct {
  uint32_t *hits_per_crystal;    /* n_crystals */
  uint32_t *singles_per_crystal; /* n_crystals, in-window singles */
  uint32_t *energy_spectrum;     /* 700 bins of 1 keV over [0, 700) keV, blurred singles */
  uint32_t *doi;                 /* doi_bins over the panel depth, hits */
  int32_t doi_bins;
} gpet_tallies;

gpet_status gpet_digitize(gpet_ctx *ctx, const gpet_hits *hits, const gpet_digitizer *params,
                          gpet_singles *singles, gpet_coincidences *coincidences,
                          gpet_tallies *tallies /* NULL: none */);

/* gpet_digitize for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels, arguments, outputs and errors, but the call allocates no device or
 * pinned host memory.  Its sort buffers, counters and readback words live in
 * a static device array of GPET_DIGITIZE_NOALLOC_SCRATCH_BYTES (128 MiB) per
 * GPU, which the library looks up when a context is created on that GPU and
 * which stays held until the process ends.  A call whose hits need more than
 * that (about 36.5 bytes per hit plus small tables: some 3.6 million hits)
 * returns GPET_ERR_ARG with the sizes in gpet_last_error and changes no
 * output.  Every call on one GPU shares that GPU's array, so calls that
 * overlap on one GPU (two contexts or streams at once) race and must be
 * serialized by the caller; each call initializes what it reads, so no state
 * carries over from the previous call.  Counts come back through pageable
 * copies at the call's synchronization points. */
#define GPET_DIGITIZE_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
gpet_status gpet_digitize_noalloc(gpet_ctx *ctx, const gpet_hits *hits, const gpet_digitizer *params,
                                  gpet_singles *singles, gpet_coincidences *coincidences,
                                  gpet_tallies *tallies /* NULL: none */);

/* ---------------------------------------------------------------------- */
/* Batched runs: one persistent transport launch over a table of instances  */
/* (a design sweep: each instance has its own scanner and source and its    */
/* own event range), then one digitizer pass over all of their hits.  Waves */
/* of the launch claim chunks of `chunk` consecutive events of one instance */
/* from a device counter, so the tail of one instance overlaps the next and */
/* small instances cost no launch of their own.  Every random number is     */
/* keyed by (event, instance id), so instance i of a batch reproduces a     */
/* plain gpet_transport / gpet_digitize run of the same scanner, source,    */
/* event range and instance id bit for bit.                                 */
/*                                                                          */
/* The instances share the context's materials, physics and phantom.  The   */
/* detector attenuation rows are staged once per launch, so the union of    */
/* the instances' detector materials may hold at most 4 materials; the      */
/* detector majorant is the maximum over that union (when it differs from   */
/* an instance's own majorant, that instance matches a plain run in          */
/* distribution only).                                                      */
/* ---------------------------------------------------------------------- */
typedef struct {
  const gpet_scanner *scanner; /* host */
  const gpet_source *source;   /* host */
  uint64_t first_event, n_events; /* first_event + n_events <= 2^32 */
  uint32_t instance;           /* id entering the random-number counters */
} gpet_instance;

typedef struct gpet_batch gpet_batch;

/* Validates and uploads n instances (1..65536); descriptors are copied.  The
 * batch keeps a pointer to ctx: every call but gpet_batch_destroy needs ctx
 * alive.  Errors as gpet_geometry_create and gpet_source_set, naming the
 * instance. */
gpet_status gpet_batch_create(gpet_ctx *ctx, int32_t n, const gpet_instance *instances, gpet_batch **out);
void gpet_batch_destroy(gpet_batch *batch);
/* crystal id layout of instance i */
gpet_status gpet_batch_info(gpet_batch *batch, int32_t i, gpet_geometry_info *info);
/* Launch shape of the batch (see gpet_ctx_set_launch) and the chunk of events
 * a wave claims at a time (1..2^20). */
gpet_status gpet_batch_set_launch(gpet_batch *batch, int32_t blocks_per_cu, int32_t search_batch, uint32_t chunk);
/* Transports every instance; hits->instance receives the instance index.
 * Same capacity contract and stats as gpet_transport (summed over instances). */
gpet_status gpet_batch_transport(gpet_batch *batch, uint64_t seed, gpet_hits *hits, gpet_stats *stats);
/* Digitizes the hits of a batch; params->first_event, n_events and instance
 * are ignored (each instance uses its own).  Singles come out in (instance,
 * event, gid) order and coincidences in (instance, time) order; a window never
 * spans two instances.  coinc_per_instance (host, n entries, may be NULL)
 * receives each instance's coincidence count. */
gpet_status gpet_batch_digitize(gpet_batch *batch, const gpet_hits *hits, const gpet_digitizer *params,
                                gpet_singles *singles, gpet_coincidences *coincidences,
                                uint64_t *coinc_per_instance);
/* Autotuner: times the batch's transport launch (kernel time, HIP events) over
 * launch shapes and chunk sizes, by coordinate search from the current shape,
 * and keeps the fastest.  `hits` is scratch output of sufficient capacity.
 * Writes a JSON summary {"blocks_per_cu", "search_batch", "chunk", "ms",
 * "trials": [[blocks_per_cu, search_batch, chunk, ms], ...]} into json
 * (NUL-terminated, truncated to cap bytes; may be NULL). */
gpet_status gpet_batch_autotune(gpet_batch *batch, uint64_t seed, gpet_hits *hits, char *json, size_t cap);

/* ---------------------------------------------------------------------- */
/* Surrogate network: a ReLU MLP (widths sizes[0] -> ... -> sizes[n-1]) with  */
/* BF16 weights and activations on the matrix cores, FP32 accumulation,     */
/* softmax cross-entropy over sizes[n-1] classes and Adam on FP32 master     */
/* weights.  Packed parameter layout (host float32): per layer l, W_l        */
/* [sizes[l+1]][sizes[l]] row-major, then b_l [sizes[l+1]].                  */
/* ---------------------------------------------------------------------- */
typedef struct gpet_mlp gpet_mlp;

typedef struct {
  uint32_t batch;       /* rows per step, drawn uniformly with replacement */
  uint32_t steps;
  double lr, beta1, beta2, eps; /* Adam (Kingma and Ba) */
  uint64_t seed;        /* key of the batch-index stream */
} gpet_train_params;

/* sizes: n_sizes (2..16) widths, input 1..256, others 1..8192; weights: packed
 * host initial values (NULL: zeros).  The network keeps a pointer to ctx and
 * uses its stream. */
gpet_status gpet_mlp_create(gpet_ctx *ctx, int32_t n_sizes, const int32_t *sizes, const float *weights,
                            gpet_mlp **out);
/* The same network with a factored output (the surrogate's form): of the
 * last layer's sizes[n_sizes - 1] outputs, the first n_first (2..64) are an
 * energy head (class 0 = no single) and the rest n_groups (1..n_first - 1)
 * equal blocks of n2 position logits; the position given energy class e > 0
 * follows softmax(block g + T[e - 1]) with g = (e - 1) n_groups / (n_first -
 * 1) (contiguous groups of energy classes share a block) and a learned FP32
 * offset table T of (n_first - 1) x n2, packed after the layers (row-major).  Labels are
 * joint: 0 for e = 0, else 1 + k (n_first - 1) + (e - 1) for position k
 * (the layout of the surrogate's classes with n_first = n_ebins + 2).  The
 * loss is -log P(e) - [e > 0] log P(k | e); gpet_mlp_forward returns the raw
 * last-layer outputs (T not added).  A design choice of this library; the
 * paper names learned surrogates only as a route to speed (Sec. 4). */
gpet_status gpet_mlp_create_factored(gpet_ctx *ctx, int32_t n_sizes, const int32_t *sizes, int32_t n_first,
                                     int32_t n_groups, const float *weights, gpet_mlp **out);
void gpet_mlp_destroy(gpet_mlp *mlp);
/* Replaces the master weights (host, packed) and clears the Adam state. */
gpet_status gpet_mlp_set_weights(gpet_mlp *mlp, const float *weights);
gpet_status gpet_mlp_get_weights(gpet_mlp *mlp, float *weights);
/* Training checkpoint: the packed master weights, Adam's first and second
 * moments (host, n_params floats each, the weights' packing) and the number
 * of Adam steps taken, which is also the training's data cursor (the batch of
 * step t is drawn from (seed, t)).  gpet_mlp_set_state restores all four, so
 * training resumed from a checkpoint continues exactly as an uninterrupted
 * run; GPET_ERR_ARG for non-finite values or a negative second moment. */
gpet_status gpet_mlp_get_state(gpet_mlp *mlp, float *weights, float *m, float *v, uint64_t *step);
gpet_status gpet_mlp_set_state(gpet_mlp *mlp, const float *weights, const float *m, const float *v,
                               uint64_t step);
/* Logits (device, n x classes, FP32) of device inputs x (n x sizes[0], FP32;
 * rounded to BF16 on entry). */
gpet_status gpet_mlp_forward(gpet_mlp *mlp, uint32_t n, const float *x, float *logits);
/* Mean cross-entropy of (x, y) (device; labels in [0, classes)) and its
 * gradient with respect to the packed parameters (host, float32). */
gpet_status gpet_mlp_loss_grad(gpet_mlp *mlp, uint32_t n, const float *x, const int32_t *y, double *loss,
                               float *grad);
/* `steps` Adam steps on mini-batches of (x, y) (device, n_pairs rows); the
 * mean loss of every step's batch (before its update) goes to loss_per_step
 * (host, steps entries; may be NULL).  Batch row r of step t is pair
 * floor(w n_pairs / 2^32), w = word r % 4 of Philox(seed; t, r / 4, 0, 9),
 * t counting the network's Adam steps from 1. */
gpet_status gpet_mlp_train(gpet_mlp *mlp, uint64_t n_pairs, const float *x, const int32_t *y,
                           const gpet_train_params *params, float *loss_per_step);

/* ---------------------------------------------------------------------- */
/* Detector-response surrogate.  A photon entering its first panel through  */
/* the front face, inside the domain below, can be handed to the network   */
/* instead of being transported through the panel.                          */
/*                                                                          */
/* Domain (decided from the entry state only): energy >= e_min_kev; entry   */
/* depth coordinate within front_tol_mm of the front face; |d_t / d_depth|  */
/* and |d_a / d_depth| <= max_slope; the straight line's point at mid-depth */
/* inside a module; every layer's neighbourhood of (2 half_width + 1)^2     */
/* crystals around its anchor inside that layer's crystal array.  Anchor:   */
/* the last layer's crystal whose pitch cell holds the mid-depth point; in   */
/* another layer, the crystal whose cell holds that cell's centre (a centre */
/* on a cell boundary goes to the upper cell).                               */
/* Features x[6]: 2 f_t - 1, 2 f_a - 1 (f: position of the mid-depth point  */
/* in the anchor cell), the two slopes over max_slope, 2 (E - e_min) /      */
/* (511 - e_min) - 1, and the depth component of the direction.             */
/* Classes: 0 = no crystal of the panel stay collects e_min_kev or more, or  */
/* the largest sum lies outside the class neighbourhood (half width H =     */
/* class_half_width, or half_width when 0); else 1 + ((layer W + i) W + j)  */
/* (n_ebins + 1) + bin for the crystal with the largest deposit sum (ties:  */
/* lower gid), (i, j) its offset + H from the anchor, W = 2 H + 1, bin =    */
/* n_ebins when the sum is within photopeak_tol_kev of the entry energy,    */
/* else floor((sum - e_min) / ebin) clipped to [0, n_ebins - 1].  With H >  */
/* half_width, class positions may fall outside a layer's array: they never */
/* occur as labels, and the sampler of a factored network leaves them out.  */
/* A class stands for one single: the entry energy (photopeak) or e_min +   */
/* ebin (bin + u) deposited at the layer's mid-depth in that crystal, at    */
/* the entry time.                                                          */
/* ---------------------------------------------------------------------- */
typedef struct {
  int32_t half_width;  /* 0..7: the domain's neighbourhood */
  int32_t n_ebins;     /* 1..1024 */
  double e_min_kev, ebin_kev, photopeak_tol_kev, max_slope, front_tol_mm;
  int32_t class_half_width; /* 0 (= half_width) or half_width..15: the classes' neighbourhood
                               (above half_width: factored networks only) */
} gpet_surrogate_spec;

/* Training pairs (device SoA): features x[6 per pair], class label, event
 * id, flags (bit 0: the largest deposit lay outside the neighbourhood; bit 1:
 * the photon touched more than 8 crystals, only the first 8 were summed;
 * bit 2: photon B). */
typedef struct {
  float *x;
  int32_t *label;
  uint32_t *event;
  uint32_t *flags;
  uint64_t capacity;
  uint64_t count; /* out */
} gpet_pairs;

typedef struct {
  uint64_t entries;          /* photons handed to the network */
  uint64_t none;             /* of them, sampled class 0 (no single) */
  float ms_transport, ms_network;
} gpet_surrogate_stats;

/* Full transport of events [first_event, first_event + n_events) (hits as
 * gpet_transport) that also records one pair per photon entering its first
 * panel inside the domain, labelled from that photon's deposits in the
 * panel.  Pair order is unspecified; GPET_ERR_CAPACITY if pairs overflow. */
gpet_status gpet_surrogate_pairs(gpet_ctx *ctx, const gpet_surrogate_spec *spec, uint64_t first_event,
                                 uint64_t n_events, uint64_t seed, uint32_t instance, gpet_hits *hits,
                                 gpet_pairs *pairs, gpet_stats *stats);
/* Transport with the surrogate: in-domain photons end at their first panel
 * entry and the network samples their single (Philox counter (0, event,
 * instance, 4 + photon): word 0 the class -- for a factored network the
 * energy class --, word 1 the energy in its bin, word 2 the position of a
 * factored network); every other photon is transported in full.  The
 * network must map 6 features to the spec's class count for this scanner
 * (factored: n_ebins + 2 energy classes and n_layers (2 H + 1)^2 positions
 * per block, with n_layers ceil((2 H + 1)^2 / 64) at most 32:
 * GPET_ERR_UNSUPPORTED beyond).  Hits as gpet_transport (surrogate singles
 * carry process 3 in aux). */
gpet_status gpet_surrogate_transport(gpet_ctx *ctx, gpet_mlp *mlp, const gpet_surrogate_spec *spec,
                                     uint64_t first_event, uint64_t n_events, uint64_t seed, uint32_t instance,
                                     gpet_hits *hits, gpet_stats *stats, gpet_surrogate_stats *sstats);

/* HIP graph of the batched transport step, for callers that replay one batch
 * step many times from a tight loop: gpet_batch_graph_capture records the
 * reset of the context's counters and the persistent transport launch for
 * this seed and these hit buffers (hits->instance required) into a graph
 * owned by the batch, replacing an earlier one; the launch shape and chunk
 * size in force are baked in.  gpet_batch_graph_launch enqueues it on the
 * context's stream and returns without synchronizing; every replay
 * reproduces gpet_batch_transport's hits.  gpet_batch_read_counts
 * synchronizes the stream and returns the hit count (GPET_ERR_CAPACITY if it
 * exceeds the capacity) and stats (may be NULL) of the last transport on
 * the context, eager or replayed. */
gpet_status gpet_batch_graph_capture(gpet_batch *batch, uint64_t seed, gpet_hits *hits);
gpet_status gpet_batch_graph_launch(gpet_batch *batch);
gpet_status gpet_batch_read_counts(gpet_batch *batch, gpet_hits *hits, gpet_stats *stats);

/* Launch shape of the transport kernel: blocks of 256 lanes per compute unit
 * (0 = as many as fit); the scheduling of lane actions within a wavefront
 * (0: every pending action runs each loop trip, and the panel searches at the
 * end of the trip, held until `search_batch` lanes (1..64) need one; 1: only
 * the action held by the most lanes runs (a search, or one of the others
 * followed by the searches it leads to); 2: plain transport only -- each
 * wavefront keeps a pool of 128
 * photons in LDS and every loop trip gathers up to 64 photons waiting for the
 * same action onto its lanes; other calls run as schedule 0).  Results do not
 * depend on the shape (every random number is keyed by event id). */
gpet_status gpet_ctx_set_launch(gpet_ctx *ctx, int32_t blocks_per_cu, int32_t search_batch, int32_t schedule);

/* Kernel timing: when enabled, HIP events bracket the transport kernel and
 * the digitizer on the context's stream; gpet_timings returns the last
 * durations in ms: [0] transport kernel, [1] whole digitizer. */
gpet_status gpet_ctx_enable_timing(gpet_ctx *ctx, int enable);
gpet_status gpet_timings(gpet_ctx *ctx, float *ms2);

/* ---------------------------------------------------------------------- */
/* Deterministic check surface (no hidden state; device output buffers).    */
/* ---------------------------------------------------------------------- */
/* Philox4x32-10 blocks for key `seed` and n counters (device, 4 u32 each). */
gpet_status gpet_philox(gpet_ctx *ctx, uint64_t seed, const uint32_t *ctr4, uint32_t n, uint32_t *out4);
/* Attenuation tables: mu (n_mat x 4 x 511 floats, 1/mm at nominal density,
 * processes PE, Compton, Rayleigh, total) and detector majorant (511). */
gpet_status gpet_tables_get(gpet_ctx *ctx, float *mu_host, float *majorant_host);
/* Locate n global points (device xyz[3n]); ids6 per point: panel, module,
 * layer, crystal-in-layer, gid, material (-1 where not applicable). */
gpet_status gpet_locate(gpet_ctx *ctx, uint32_t n, const float *xyz, int32_t *ids6);
/* Fixed rays: panel search from o along d (device, 3 floats each), then
 * locate at t_in + (k + 1/2) step, k < n_samples.  t_in < 0: no panel.
 * ids6 [n][n_samples][6]; panel -2 marks a sample already outside. */
gpet_status gpet_ray_locate(gpet_ctx *ctx, uint32_t n, const float *o, const float *d,
                            int32_t n_samples, float step_mm, float *t_in, int32_t *ids6);
/* Compton (Kahn) and Rayleigh (Thomson) samplers, sample i on stream 7 / 8. */
gpet_status gpet_sample_compton(gpet_ctx *ctx, float e_kev, uint32_t n, uint64_t seed,
                                float *cos_t, float *e_out, int32_t *trials);
gpet_status gpet_sample_rayleigh(gpet_ctx *ctx, uint32_t n, uint64_t seed, float *cos_t);

/* Traced histories: every vertex of events [first, first + n) with the same
 * kernel code as gpet_transport.  Per photon (index 2*(e-first) + photon) at
 * most max_vertices records of 11 int32 (event, photon, kind, region, panel,
 * gid, material, accept, process, kahn trials, rng block) and 8 floats
 * (x, y, z, energy, deposit, dx, dy, dz); counts[photon] may exceed
 * max_vertices (then the rest were dropped).  Kinds: 0 step, 1 enter panel,
 * 2 exit region, 3 escape, 4 absorbed, 5 enter phantom, 6 emission.  Panel
 * steps are in the panel-local frame, everything else global. */
gpet_status gpet_trace(gpet_ctx *ctx, uint64_t first_event, uint32_t n_events, uint64_t seed,
                       uint32_t instance, int32_t max_vertices, int32_t *vint, float *vflt,
                       int32_t *counts);

#ifdef __cplusplus
}
#endif
#endif /* GPET_H */
