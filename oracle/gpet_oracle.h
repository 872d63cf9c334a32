/*
 * gpet_oracle.h -- FP64 CPU oracle for multi-layer PET Monte Carlo.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, step-by-step reference of
 * what the GPU path computes; only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code with the
 * HIP library.
 *
 * Units: mm, keV, ps, g/cm^3.  All arithmetic is IEEE double.
 *
 * Parity status per function (what pins it, see tests/test_oracle_*.py):
 *   or_philox            Philox4x32-10 known-answer vectors
 *   or_sigma_kn          quadrature of the Klein-Nishina differential cross-section
 *   or_tables            composition sums checked against hand-derived values
 *   or_sample_compton    KS against the quadrature CDF of Klein-Nishina
 *   or_sample_rayleigh   KS against the Thomson CDF
 *   or_locate            brute-force enumeration of crystal boxes
 *   or_transport         narrow-beam exp(-mu L), black-ring solid angle,
 *                        collinearity, energy conservation, split-layer invariance,
 *                        tallies equal in law to analog tracking
 *   or_digitize          brute-force adder / O(n^2) coincidence reference;
 *                        time and depth blur against the normal law, light
 *                        sharing against the neighbour set and its law, dead
 *                        time against brute force and the Poisson throughput
 *                        of both dead-time models
 *   source extensions    acollinearity and positron range against the normal
 *                        law of each transverse / spatial component
 */
#ifndef GPET_ORACLE_H
#define GPET_ORACLE_H
#include <stdint.h>

#define OR_MAX_EL 8
#define OR_MAX_MAT 8
#define OR_MAX_LAYERS 4
#define OR_MAX_PANELS 64
#define OR_NE 511 /* energy nodes 1..511 keV */

typedef struct {
  double density; /* g/cm^3 (nominal; phantom voxels carry their own) */
  int32_t n_el;
  int32_t mask; /* 1 photoelectric | 2 Compton | 4 Rayleigh */
  int32_t Z[OR_MAX_EL];
  double A[OR_MAX_EL]; /* g/mol */
  double w[OR_MAX_EL]; /* mass fractions */
} or_material;

typedef struct {
  double k_pe;  /* cm^2 MeV^3 per atom per Z^4 */
  double k_r;   /* cm^2 MeV^2 per atom per Z^2 */
  double e_cut; /* keV */
} or_physics;

typedef struct {
  double depth0, thick;     /* depth range of the layer inside the module */
  int32_t n_t, n_a;         /* crystals along t and a */
  double cryst_t, cryst_a;  /* crystal size */
  double pitch_t, pitch_a;  /* crystal pitch */
  double off_t, off_a;      /* start of the crystal array from the module edge */
  int32_t mat_crystal, mat_interval;
} or_layer;

typedef struct {
  int32_t mode;     /* 0 repetition, 1 explicit poses */
  int32_t n_panels;
  double radius, phi0, z0;               /* repetition mode */
  double pose[OR_MAX_PANELS][12];        /* origin, e_depth, e_t, e_a */
  double depth, width, length;           /* panel box */
  int32_t mod_n_t, mod_n_a;
  double mod_t, mod_a, gap_t, gap_a;
  int32_t mat_fill;
  int32_t n_layers;
  or_layer layer[OR_MAX_LAYERS];
} or_scanner;

typedef struct {
  int32_t nx, ny, nz;
  double dx, dy, dz, ox, oy, oz;
  const uint8_t *mat; /* [nz][ny][nx] */
  const float *dens;  /* g/cm^3 */
} or_phantom;

typedef struct {
  int32_t kind; /* 0 point, 1 cylinders, 2 beam */
  double pos[3];
  double dir[3];
  int32_t n_rods;
  const double *rods; /* n_rods x (cx, cy, radius, z0, z1) */
  uint64_t duration_ps;
  double acol_fwhm_deg;  /* photon-pair acollinearity (0: back to back) */
  double prange_fwhm_mm; /* positron range, FWHM of each axis (0: annihilation at the emission site) */
} or_source;

typedef struct {
  int32_t n_mat;
  or_material mat[OR_MAX_MAT];
  or_physics phys;
  or_scanner scan;
  int32_t has_phantom;
  or_phantom ph;
  or_source src;
  /* derived by or_prepare */
  double mu_mass[OR_MAX_MAT][3][OR_NE]; /* cm^2/g: photoelectric, Compton, Rayleigh */
  double maj_det[OR_NE];                /* 1/mm */
  double maj_ph[OR_NE];                 /* 1/mm */
  int32_t crystals_per_module, crystals_per_panel, n_crystals;
  int32_t layer_base[OR_MAX_LAYERS];
  double rod_cum[1024];
  double rod_total;
} or_scene;

/* one hit: a photoelectric or Compton interaction inside a crystal */
typedef struct {
  uint32_t event, photon, gid, panel, module, layer, crystal, process, seq;
  double edep, tof_ps, depth, t, a;
  uint64_t time_ps;
} or_hit;

/* one vertex of a traced history */
typedef struct {
  int32_t event, photon, kind, region, panel, gid, mat, accept, process, trials, block;
  double x, y, z, e, edep, dx, dy, dz;
} or_vertex;

enum { OR_V_STEP = 0, OR_V_ENTER_PANEL = 1, OR_V_EXIT = 2, OR_V_ESCAPE = 3, OR_V_DEAD = 4,
       OR_V_ENTER_PHANTOM = 5, OR_V_EMIT = 6 };

typedef struct {
  double fwhm_511;     /* relative FWHM at 511 keV */
  double e_lo, e_hi;   /* energy window, inclusive */
  uint64_t window_ps;  /* coincidence window */
  uint64_t seed;
  uint32_t instance;
  int32_t doi_bins;
  int32_t readout;     /* single readout level: 0 crystal, 1 module, 2 panel */
  double time_fwhm_ps; /* timing resolution (0: none) */
  double doi_fwhm_mm;  /* depth-of-interaction resolution (0: none) */
  uint64_t dead_ps;    /* dead time of a unit */
  int32_t dead_mode;   /* 0 none, 1 paralyzable, 2 non-paralyzable */
  int32_t dead_level;  /* dead-time unit: 0 crystal, 1 module, 2 panel */
  double ls_prob;      /* light sharing: probability of reading a neighbour crystal */
} or_digitizer;

typedef struct {
  uint32_t event, gid;
  double edep, energy, depth;
  uint64_t time_ps;
  int32_t in_window; /* blurred energy inside [e_lo, e_hi] */
  int32_t lost;      /* dropped by the dead time of its unit */
} or_single;

void or_philox(uint32_t k0, uint32_t k1, const uint32_t *ctr, uint32_t *out, int64_t n);
double or_sigma_kn(double e_kev); /* barn per electron */
uint64_t or_event_time(uint64_t X, uint64_t T); /* floor(X T / 2^64) */
int or_prepare(or_scene *s);
void or_mu(const or_scene *s, int m, double e, double mu3[3]); /* 1/mm at nominal density */
int64_t or_sample_compton(double e_kev, int64_t n, uint64_t seed, double *cos_t, double *e_out,
                          int32_t *trials);
void or_sample_rayleigh(int64_t n, uint64_t seed, double *cos_t);
void or_locate(const or_scene *s, int64_t n, const double *xyz, int32_t *ids6, double *bdist);
void or_ray_locate(const or_scene *s, int64_t n_rays, const double *o, const double *d,
                   int32_t n_samp, double step, double *t_in, int32_t *ids6, double *bdist);
/* counters (9, added to): events, panel entries, Woodcock steps, real
 * interactions, Kahn trials, panel searches, photon-stream Philox blocks,
 * capped photons, scatters (Compton or Rayleigh) */
int64_t or_transport(const or_scene *s, uint64_t first, uint64_t n, uint64_t seed,
                     uint32_t instance, or_hit *hits, int64_t cap, int64_t *counters);
/* the same with analog tracking (flights from material boundary to boundary)
 * instead of Woodcock tracking: a check of the latter, equal in law */
int64_t or_transport_analog(const or_scene *s, uint64_t first, uint64_t n, uint64_t seed,
                            uint32_t instance, or_hit *hits, int64_t cap, int64_t *counters);
int64_t or_trace(const or_scene *s, uint64_t first, uint64_t n, uint64_t seed, uint32_t instance,
                 or_vertex *v, int64_t cap);
int64_t or_trace_analog(const or_scene *s, uint64_t first, uint64_t n, uint64_t seed, uint32_t instance,
                        or_vertex *v, int64_t cap);
int64_t or_digitize(const or_scene *s, const or_hit *hits, int64_t n_hits,
                    const or_digitizer *dg, or_single *singles, int64_t cap_s,
                    uint32_t *coinc, int64_t cap_c, int64_t *n_coinc);
int or_num_threads(void);
void or_set_threads(int n);
#endif
