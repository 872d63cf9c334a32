/*
 * gpet_oracle.c -- FP64 CPU oracle: the simulation written out step by step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.  Shares no code with
 * the HIP library.  Plain double arithmetic, no blocking or fusion, OpenMP over
 * independent events only.
 *
 * Method (paper Sec. 2.1): a photon that leaves the phantom is carried to the
 * panel it meets (line-plane / ray-box intersection), moved into that panel's
 * local frame and transported step by step with Woodcock free paths; at each
 * real interaction the depth coordinate selects the layer, whose crystal
 * parameters then decide crystal or interval material and the crystal index.
 * Interactions are labelled with panel, module, layer and crystal (Sec. 2.1,
 * Fig. 1).  The parts the paper inherits from gPET without spelling out
 * (interaction physics, tables, digitizer) follow the readings listed with
 * each function below.
 */
#include "gpet_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846
#define MEC2 510.99895         /* electron rest energy, keV */
#define R_E 2.8179403262e-13   /* classical electron radius, cm */
#define N_AV 6.02214076e23     /* Avogadro, 1/mol */
#define C_MM_PER_PS 0.299792458
#define FWHM_PER_SIGMA 2.354820045030949 /* 2 sqrt(2 ln 2) */
#define MAX_STEPS (1 << 20)

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two      */
/* 32x32->64 multiplies with the counter words, key added between rounds     */
/* by the Weyl constants.                                                     */
/* ------------------------------------------------------------------------ */
static void philox_block(uint32_t k0, uint32_t k1, const uint32_t in[4], uint32_t out[4]) {
  uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
  for (int r = 0; r < 10; r++) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void or_philox(uint32_t k0, uint32_t k1, const uint32_t *ctr, uint32_t *out, int64_t n) {
  for (int64_t i = 0; i < n; i++) philox_block(k0, k1, ctr + 4 * i, out + 4 * i);
}

/* u32 -> uniform on the open interval (0,1): odd multiples of 2^-24 */
static double u01(uint32_t w) { return (2.0 * (double)(w >> 9) + 1.0) * (1.0 / 16777216.0); }

typedef struct {
  uint32_t k0, k1, event, instance, stream, n;
} rng_t;

static void rng_init(rng_t *r, uint64_t seed, uint32_t event, uint32_t instance, uint32_t stream) {
  r->k0 = (uint32_t)seed;
  r->k1 = (uint32_t)(seed >> 32);
  r->event = event;
  r->instance = instance;
  r->stream = stream;
  r->n = 0;
}

/* next block of the stream as four uniforms */
static void rng_next(rng_t *r, double u[4]) {
  uint32_t c[4] = {r->n, r->event, r->instance, r->stream}, o[4];
  philox_block(r->k0, r->k1, c, o);
  r->n++;
  for (int i = 0; i < 4; i++) u[i] = u01(o[i]);
}

static void rng_raw(const rng_t *r, uint32_t n, uint32_t o[4]) {
  uint32_t c[4] = {n, r->event, r->instance, r->stream};
  philox_block(r->k0, r->k1, c, o);
}

/* ------------------------------------------------------------------------ */
/* Cross-sections and tables                                                 */
/* ------------------------------------------------------------------------ */
/* Klein-Nishina total cross-section per free electron, in barn. */
double or_sigma_kn(double e_kev) {
  double a = e_kev / MEC2;
  double l = log(1.0 + 2.0 * a);
  double t1 = (1.0 + a) / (a * a) * (2.0 * (1.0 + a) / (1.0 + 2.0 * a) - l / a);
  double t2 = l / (2.0 * a);
  double t3 = (1.0 + 3.0 * a) / ((1.0 + 2.0 * a) * (1.0 + 2.0 * a));
  return 2.0 * PI * R_E * R_E * (t1 + t2 - t3) * 1e24;
}

/* Mass attenuation (cm^2/g) of material m at node energy e (keV):
 *   Compton      N_A sum_j w_j Z_j / A_j * sigma_KN(E)
 *   photoelectric N_A sum_j w_j / A_j * K_pe Z_j^4 / E_MeV^3
 *   Rayleigh     N_A sum_j w_j / A_j * K_R Z_j^2 / E_MeV^2
 */
static void mass_atten(const or_material *m, const or_physics *p, double e, double out[3]) {
  double em = e / 1000.0;
  double pe = 0, co = 0, ra = 0;
  for (int j = 0; j < m->n_el; j++) {
    double z = m->Z[j], na = N_AV * m->w[j] / m->A[j];
    pe += na * p->k_pe * z * z * z * z / (em * em * em);
    co += na * z * or_sigma_kn(e) * 1e-24;
    ra += na * p->k_r * z * z / (em * em);
  }
  out[0] = (m->mask & 1) ? pe : 0.0;
  out[1] = (m->mask & 2) ? co : 0.0;
  out[2] = (m->mask & 4) ? ra : 0.0;
}

/* linear interpolation on 1 keV nodes: j = clamp(floor(E),1,510), f = E - j */
static double interp(const double *tab, double e) {
  double jf = floor(e);
  if (jf < 1.0) jf = 1.0;
  if (jf > 510.0) jf = 510.0;
  int j = (int)jf;
  double f = e - jf;
  return (1.0 - f) * tab[j - 1] + f * tab[j];
}

/* per-process linear attenuation (1/mm) of material m at density rho */
static void mu_at(const or_scene *s, int m, double rho, double e, double mu3[3]) {
  for (int k = 0; k < 3; k++) mu3[k] = rho * interp(s->mu_mass[m][k], e) / 10.0;
}

void or_mu(const or_scene *s, int m, double e, double mu3[3]) { mu_at(s, m, s->mat[m].density, e, mu3); }

/* ------------------------------------------------------------------------ */
/* Scene preparation: tables, majorants, panel poses, crystal id layout      */
/* ------------------------------------------------------------------------ */
int or_prepare(or_scene *s) {
  if (s->n_mat < 1 || s->n_mat > OR_MAX_MAT) return -1;
  for (int m = 0; m < s->n_mat; m++)
    for (int i = 0; i < OR_NE; i++) {
      double o[3];
      mass_atten(&s->mat[m], &s->phys, (double)(i + 1), o);
      for (int k = 0; k < 3; k++) s->mu_mass[m][k][i] = o[k];
    }
  /* detector majorant: node-wise max over the materials the panel contains */
  or_scanner *sc = &s->scan;
  int used[OR_MAX_MAT] = {0};
  used[sc->mat_fill] = 1;
  for (int l = 0; l < sc->n_layers; l++) {
    used[sc->layer[l].mat_crystal] = 1;
    used[sc->layer[l].mat_interval] = 1;
  }
  for (int i = 0; i < OR_NE; i++) {
    double mx = 0;
    for (int m = 0; m < s->n_mat; m++)
      if (used[m]) {
        double t = s->mat[m].density * (s->mu_mass[m][0][i] + s->mu_mass[m][1][i] + s->mu_mass[m][2][i]) / 10.0;
        if (t > mx) mx = t;
      }
    s->maj_det[i] = mx;
  }
  /* phantom majorant: per material the largest voxel density present */
  if (s->has_phantom) {
    double rmax[OR_MAX_MAT] = {0};
    int64_t nv = (int64_t)s->ph.nx * s->ph.ny * s->ph.nz;
    for (int64_t v = 0; v < nv; v++) {
      int m = s->ph.mat[v];
      if (m >= s->n_mat) return -2;
      if (s->ph.dens[v] > rmax[m]) rmax[m] = s->ph.dens[v];
    }
    for (int i = 0; i < OR_NE; i++) {
      double mx = 0;
      for (int m = 0; m < s->n_mat; m++) {
        double t = rmax[m] * (s->mu_mass[m][0][i] + s->mu_mass[m][1][i] + s->mu_mass[m][2][i]) / 10.0;
        if (t > mx) mx = t;
      }
      s->maj_ph[i] = mx;
    }
  }
  /* repetition mode: panel k faces the axis at angle phi0 + 2 pi k / n, its
   * front face at distance `radius`; depth points outward, t tangential, a = z */
  if (sc->mode == 0) {
    for (int k = 0; k < sc->n_panels; k++) {
      double ph = sc->phi0 + 2.0 * PI * k / sc->n_panels;
      double c = cos(ph), sn = sin(ph);
      double *P = sc->pose[k];
      P[0] = sc->radius * c; P[1] = sc->radius * sn; P[2] = sc->z0;
      P[3] = c; P[4] = sn; P[5] = 0;
      P[6] = -sn; P[7] = c; P[8] = 0;
      P[9] = 0; P[10] = 0; P[11] = 1;
    }
  }
  /* crystal id layout: gid = panel*C_panel + module*C_module + layer base + i_a*n_t + i_t */
  int cm = 0;
  for (int l = 0; l < sc->n_layers; l++) {
    s->layer_base[l] = cm;
    cm += sc->layer[l].n_t * sc->layer[l].n_a;
  }
  s->crystals_per_module = cm;
  s->crystals_per_panel = cm * sc->mod_n_t * sc->mod_n_a;
  s->n_crystals = s->crystals_per_panel * sc->n_panels;
  /* rod selection weights proportional to rod volume */
  if (s->src.kind == 1) {
    if (s->src.n_rods > 1024) return -3;
    double c = 0;
    for (int i = 0; i < s->src.n_rods; i++) {
      const double *r = s->src.rods + 5 * i;
      c += r[2] * r[2] * (r[4] - r[3]);
      s->rod_cum[i] = c;
    }
    s->rod_total = c;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */
static void to_local(const double *P, const double x[3], double l[3]) {
  double r[3] = {x[0] - P[0], x[1] - P[1], x[2] - P[2]};
  l[0] = r[0] * P[3] + r[1] * P[4] + r[2] * P[5];
  l[1] = r[0] * P[6] + r[1] * P[7] + r[2] * P[8];
  l[2] = r[0] * P[9] + r[1] * P[10] + r[2] * P[11];
}
static void dir_to_local(const double *P, const double d[3], double l[3]) {
  l[0] = d[0] * P[3] + d[1] * P[4] + d[2] * P[5];
  l[1] = d[0] * P[6] + d[1] * P[7] + d[2] * P[8];
  l[2] = d[0] * P[9] + d[1] * P[10] + d[2] * P[11];
}
static void to_global(const double *P, const double l[3], double x[3]) {
  for (int i = 0; i < 3; i++) x[i] = P[i] + l[0] * P[3 + i] + l[1] * P[6 + i] + l[2] * P[9 + i];
}
static void dir_to_global(const double *P, const double l[3], double d[3]) {
  for (int i = 0; i < 3; i++) d[i] = l[0] * P[3 + i] + l[1] * P[6 + i] + l[2] * P[9 + i];
}

static int inside_panel(const or_scanner *sc, const double l[3]) {
  return l[0] >= 0.0 && l[0] < sc->depth && l[1] >= -0.5 * sc->width && l[1] < 0.5 * sc->width &&
         l[2] >= -0.5 * sc->length && l[2] < 0.5 * sc->length;
}

/* slab test of a ray against [lo,hi) per axis; returns 1 and the entry distance */
static int ray_box(const double o[3], const double d[3], const double lo[3], const double hi[3],
                   double *t_enter, double *t_exit) {
  double tn = -INFINITY, tf = INFINITY;
  for (int k = 0; k < 3; k++) {
    if (d[k] == 0.0) {
      if (o[k] < lo[k] || o[k] > hi[k]) return 0;
      continue;
    }
    double t1 = (lo[k] - o[k]) / d[k], t2 = (hi[k] - o[k]) / d[k];
    double a = t1 < t2 ? t1 : t2, b = t1 < t2 ? t2 : t1;
    if (a > tn) tn = a;
    if (b < tf) tf = b;
  }
  if (tn > tf || tf <= 0.0) return 0;
  *t_enter = tn > 0.0 ? tn : 0.0;
  *t_exit = tf;
  return 1;
}

/* Panel search (Sec. 2.1: a photon that leaves the phantom is carried to its
 * panel by line-plane intersection): nearest panel box along the ray, the
 * panel just left excluded; ties go to the lower index. */
static int panel_search(const or_scene *s, const double x[3], const double d[3], int exclude,
                        double *t_in) {
  const or_scanner *sc = &s->scan;
  double lo[3] = {0.0, -0.5 * sc->width, -0.5 * sc->length};
  double hi[3] = {sc->depth, 0.5 * sc->width, 0.5 * sc->length};
  int best = -1;
  double bt = INFINITY;
  for (int p = 0; p < sc->n_panels; p++) {
    if (p == exclude) continue;
    double lo_[3], ld[3], te, tx;
    to_local(sc->pose[p], x, lo_);
    dir_to_local(sc->pose[p], d, ld);
    if (ray_box(lo_, ld, lo, hi, &te, &tx) && te < bt) {
      bt = te;
      best = p;
    }
  }
  *t_in = bt;
  return best;
}

typedef struct {
  int mat, module, layer, crystal, gid; /* -1 where not applicable */
} loc_t;

static double dmin(double a, double b) { return a < b ? a : b; }

/* Hierarchical locate inside panel p at local (depth, t, a): module from the
 * (t, a) grid, then the layer from the depth coordinate (the paper's
 * layer-selection step, Sec. 2.1), then the crystal from that layer's pitch,
 * offset and size.  bd (optional) receives the distance to the nearest
 * boundary plane met on the way. */
static loc_t locate_local(const or_scene *s, int p, const double l[3], double *bd) {
  const or_scanner *sc = &s->scan;
  loc_t r = {sc->mat_fill, -1, -1, -1, -1};
  double b = INFINITY;
  b = dmin(b, fabs(l[0]));
  b = dmin(b, fabs(sc->depth - l[0]));
  b = dmin(b, fabs(l[1] + 0.5 * sc->width));
  b = dmin(b, fabs(0.5 * sc->width - l[1]));
  b = dmin(b, fabs(l[2] + 0.5 * sc->length));
  b = dmin(b, fabs(0.5 * sc->length - l[2]));
  double t0 = -0.5 * (sc->mod_n_t * sc->mod_t + (sc->mod_n_t - 1) * sc->gap_t);
  double a0 = -0.5 * (sc->mod_n_a * sc->mod_a + (sc->mod_n_a - 1) * sc->gap_a);
  double mt = floor((l[1] - t0) / (sc->mod_t + sc->gap_t));
  double ma = floor((l[2] - a0) / (sc->mod_a + sc->gap_a));
  double ut = l[1] - t0 - mt * (sc->mod_t + sc->gap_t);
  double ua = l[2] - a0 - ma * (sc->mod_a + sc->gap_a);
  b = dmin(b, dmin(fabs(ut), fabs(ut - sc->mod_t)));
  b = dmin(b, dmin(fabs(ua), fabs(ua - sc->mod_a)));
  b = dmin(b, fabs(ut - (sc->mod_t + sc->gap_t)));
  b = dmin(b, fabs(ua - (sc->mod_a + sc->gap_a)));
  if (bd) *bd = b;
  if (mt < 0 || mt >= sc->mod_n_t || ma < 0 || ma >= sc->mod_n_a || ut >= sc->mod_t || ua >= sc->mod_a)
    return r;
  r.module = (int)ma * sc->mod_n_t + (int)mt;
  int L = -1;
  for (int k = 0; k < sc->n_layers; k++) {
    const or_layer *ly = &sc->layer[k];
    b = dmin(b, dmin(fabs(l[0] - ly->depth0), fabs(l[0] - ly->depth0 - ly->thick)));
    if (L < 0 && l[0] >= ly->depth0 && l[0] < ly->depth0 + ly->thick) L = k;
  }
  if (bd) *bd = b;
  if (L < 0) return r;
  const or_layer *ly = &sc->layer[L];
  r.layer = L;
  r.mat = ly->mat_interval;
  double it = floor((ut - ly->off_t) / ly->pitch_t);
  double ia = floor((ua - ly->off_a) / ly->pitch_a);
  double ct = ut - ly->off_t - it * ly->pitch_t;
  double ca = ua - ly->off_a - ia * ly->pitch_a;
  double lo_t = 0.5 * (ly->pitch_t - ly->cryst_t), hi_t = 0.5 * (ly->pitch_t + ly->cryst_t);
  double lo_a = 0.5 * (ly->pitch_a - ly->cryst_a), hi_a = 0.5 * (ly->pitch_a + ly->cryst_a);
  b = dmin(b, dmin(dmin(fabs(ct), fabs(ct - ly->pitch_t)), dmin(fabs(ct - lo_t), fabs(ct - hi_t))));
  b = dmin(b, dmin(dmin(fabs(ca), fabs(ca - ly->pitch_a)), dmin(fabs(ca - lo_a), fabs(ca - hi_a))));
  if (bd) *bd = b;
  if (it < 0 || it >= ly->n_t || ia < 0 || ia >= ly->n_a) return r;
  if (ct < lo_t || ct >= hi_t || ca < lo_a || ca >= hi_a) return r;
  r.mat = ly->mat_crystal;
  r.crystal = (int)ia * ly->n_t + (int)it;
  r.gid = p * s->crystals_per_panel + r.module * s->crystals_per_module + s->layer_base[L] + r.crystal;
  return r;
}

/* distance from a local point outside the panel box to the box */
static double outside_distance(const or_scanner *sc, const double l[3]) {
  double lo[3] = {0.0, -0.5 * sc->width, -0.5 * sc->length};
  double hi[3] = {sc->depth, 0.5 * sc->width, 0.5 * sc->length};
  double q = 0;
  for (int k = 0; k < 3; k++) {
    double e = l[k] < lo[k] ? lo[k] - l[k] : (l[k] > hi[k] ? l[k] - hi[k] : 0.0);
    q += e * e;
  }
  return sqrt(q);
}

/* locate global points: ids6 = (panel, module, layer, crystal, gid, material);
 * bdist: distance to the nearest boundary (panel faces included) */
void or_locate(const or_scene *s, int64_t n, const double *xyz, int32_t *ids6, double *bdist) {
  const or_scanner *sc = &s->scan;
  for (int64_t i = 0; i < n; i++) {
    int32_t *o = ids6 + 6 * i;
    o[0] = o[1] = o[2] = o[3] = o[4] = o[5] = -1;
    if (bdist) bdist[i] = INFINITY;
    for (int p = 0; p < sc->n_panels; p++) {
      double l[3];
      to_local(sc->pose[p], xyz + 3 * i, l);
      if (!inside_panel(sc, l)) {
        double od = outside_distance(sc, l);
        if (bdist && od < bdist[i]) bdist[i] = od;
        continue;
      }
      double b;
      loc_t r = locate_local(s, p, l, &b);
      o[0] = p; o[1] = r.module; o[2] = r.layer; o[3] = r.crystal; o[4] = r.gid; o[5] = r.mat;
      if (bdist && b < bdist[i]) bdist[i] = b;
      break;
    }
  }
}

/* Fixed rays: panel search from o along d, then locate at n_samp points
 * t_in + (k + 1/2) * step in that panel's local frame. */
void or_ray_locate(const or_scene *s, int64_t n_rays, const double *o, const double *d,
                   int32_t n_samp, double step, double *t_in, int32_t *ids6, double *bdist) {
  const or_scanner *sc = &s->scan;
  for (int64_t r = 0; r < n_rays; r++) {
    double ti;
    int p = panel_search(s, o + 3 * r, d + 3 * r, -1, &ti);
    t_in[r] = p >= 0 ? ti : -1.0;
    for (int k = 0; k < n_samp; k++) {
      int32_t *q = ids6 + 6 * (r * n_samp + k);
      double *bq = bdist + r * n_samp + k;
      q[0] = p; q[1] = q[2] = q[3] = q[4] = q[5] = -1;
      *bq = INFINITY;
      if (p < 0) continue;
      double x[3], l[3];
      double tt = ti + (k + 0.5) * step;
      for (int i = 0; i < 3; i++) x[i] = o[3 * r + i] + tt * d[3 * r + i];
      to_local(sc->pose[p], x, l);
      if (!inside_panel(sc, l)) { q[0] = -2; continue; }
      loc_t lc = locate_local(s, p, l, bq);
      q[1] = lc.module; q[2] = lc.layer; q[3] = lc.crystal; q[4] = lc.gid; q[5] = lc.mat;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Interaction sampling                                                      */
/* ------------------------------------------------------------------------ */
/* Compton scattering by Kahn's rejection method (Kahn 1954), one block per
 * trial: rho = E/E' sampled from one of two branches, accepted against the
 * remaining Klein-Nishina factor.  Returns cos(theta); *e_out = E/rho. */
static double kahn(rng_t *r, double e, double *e_out, int *trials) {
  double a = e / MEC2;
  int n = 0;
  for (;;) {
    double u[4];
    rng_next(r, u);
    n++;
    double rho, acc;
    if (u[0] <= (1.0 + 2.0 * a) / (9.0 + 2.0 * a)) {
      rho = 1.0 + 2.0 * a * u[1];
      acc = 4.0 * (1.0 / rho - 1.0 / (rho * rho));
    } else {
      rho = (1.0 + 2.0 * a) / (1.0 + 2.0 * a * u[1]);
      double c = 1.0 - (rho - 1.0) / a;
      acc = 0.5 * (c * c + 1.0 / rho);
    }
    if (u[2] <= acc) {
      *e_out = e / rho;
      *trials = n;
      return 1.0 - (rho - 1.0) / a;
    }
  }
}

/* Thomson angular law p(mu) ~ 1 + mu^2: invert F(mu) = (mu^3 + 3 mu + 4)/8
 * with Cardano's formula for mu^3 + 3 mu - (8u - 4) = 0. */
static double thomson(double u) {
  double q = 4.0 * u - 2.0;
  double s = sqrt(q * q + 1.0);
  return cbrt(q + s) + cbrt(q - s);
}

/* Direction update for polar cosine c and azimuth phi about the old direction. */
static void rotate(double d[3], double c, double phi) {
  double st = sqrt(fmax(0.0, 1.0 - c * c));
  double cp = cos(phi), sp = sin(phi);
  double u = d[0], v = d[1], w = d[2];
  double s = sqrt(u * u + v * v);
  double nu, nv, nw;
  if (s < 1e-6) {
    nu = st * cp;
    nv = st * sp;
    nw = (w >= 0 ? 1.0 : -1.0) * c;
  } else {
    nu = u * c + st * (u * w * cp - v * sp) / s;
    nv = v * c + st * (v * w * cp + u * sp) / s;
    nw = w * c - s * st * cp;
  }
  double nn = sqrt(nu * nu + nv * nv + nw * nw);
  d[0] = nu / nn; d[1] = nv / nn; d[2] = nw / nn;
}

int64_t or_sample_compton(double e_kev, int64_t n, uint64_t seed, double *cos_t, double *e_out,
                          int32_t *trials) {
  int64_t tot = 0;
  for (int64_t i = 0; i < n; i++) {
    rng_t r;
    rng_init(&r, seed, (uint32_t)i, 0, 7);
    int t;
    cos_t[i] = kahn(&r, e_kev, &e_out[i], &t);
    if (trials) trials[i] = t;
    tot += t;
  }
  return tot;
}

void or_sample_rayleigh(int64_t n, uint64_t seed, double *cos_t) {
  for (int64_t i = 0; i < n; i++) {
    rng_t r;
    rng_init(&r, seed, (uint32_t)i, 0, 8);
    double u[4];
    rng_next(&r, u);
    cos_t[i] = thomson(u[0]);
  }
}

/* ------------------------------------------------------------------------ */
/* One event                                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
  or_hit *hits;
  int64_t n, cap;
  or_vertex *v; /* trace mode */
  int64_t nv, vcap;
  int64_t cnt[9]; /* events, panel entries, steps, real, trials, searches, blocks, capped, scatters */
  int analog;     /* analog tracking instead of Woodcock (a check of the latter) */
} sink_t;

static void push_hit(sink_t *k, const or_hit *h) {
  if (k->n >= k->cap) {
    int64_t nc = k->cap ? 2 * k->cap : 1024;
    k->hits = (or_hit *)realloc(k->hits, (size_t)nc * sizeof(or_hit));
    k->cap = nc;
  }
  k->hits[k->n++] = *h;
}

static void vtx(sink_t *k, uint32_t ev, int ph, int kind, int region, int panel, int gid, int mat,
                int acc, int proc, int trials, int block, const double x[3], double e, double edep,
                const double *d) {
  if (!k->v) return;
  if (k->nv < k->vcap) {
    or_vertex *q = &k->v[k->nv];
    q->event = (int32_t)ev; q->photon = ph; q->kind = kind; q->region = region; q->panel = panel;
    q->gid = gid; q->mat = mat; q->accept = acc; q->process = proc; q->trials = trials;
    q->block = block; q->x = x[0]; q->y = x[1]; q->z = x[2]; q->e = e; q->edep = edep;
    q->dx = d ? d[0] : 0.0; q->dy = d ? d[1] : 0.0; q->dz = d ? d[2] : 0.0;
  }
  k->nv++;
}

/* Interaction at a real collision; returns 0 if the photon dies.  *edep gets
 * the locally deposited energy. */
static int interact(const or_scene *s, rng_t *r, int proc, double *e, double d[3], double phi,
                    double *edep, int *trials) {
  *trials = 0;
  if (proc == 1) { /* photoelectric: absorbed */
    *edep = *e;
    *e = 0;
    return 0;
  }
  if (proc == 2) { /* Compton */
    double e1, c = kahn(r, *e, &e1, trials);
    rotate(d, c, phi);
    *edep = *e - e1;
    *e = e1;
    if (*e < s->phys.e_cut) { /* below cutoff: deposit the rest locally */
      *edep += *e;
      *e = 0;
      return 0;
    }
    return 1;
  }
  { /* Rayleigh */
    double u[4];
    rng_next(r, u);
    rotate(d, thomson(u[0]), phi);
    *edep = 0;
    return 1;
  }
}

static int pick_process(const double mu3[3], double mu, double u) {
  if (u * mu < mu3[0]) return 1;
  if (u * mu < mu3[0] + mu3[1]) return 2;
  return 3;
}

static void phantom_voxel(const or_phantom *ph, const double x[3], int64_t *vox) {
  double ix = floor((x[0] - ph->ox) / ph->dx);
  double iy = floor((x[1] - ph->oy) / ph->dy);
  double iz = floor((x[2] - ph->oz) / ph->dz);
  if (ix < 0 || ix >= ph->nx || iy < 0 || iy >= ph->ny || iz < 0 || iz >= ph->nz) {
    *vox = -1;
    return;
  }
  *vox = ((int64_t)iz * ph->ny + (int64_t)iy) * ph->nx + (int64_t)ix;
}

/* ---- analog tracking: the photon flies to the next plane where the
 * material may change, spending the sampled optical depth segment by segment
 * (the textbook method that Woodcock tracking must agree with in law) ---- */
#define ANALOG_NUDGE 1e-9 /* mm past a plane, so the next lookup sees the next cell */

static double ahead(double c, double dc, double pos) {
  if (dc > 0.0 && pos > c) return (pos - c) / dc;
  if (dc < 0.0 && pos < c) return (pos - c) / dc;
  return INFINITY;
}

/* distance from a phantom point to the next voxel face along d */
static double next_voxel_plane(const or_phantom *P, const double x[3], const double d[3]) {
  const double o[3] = {P->ox, P->oy, P->oz}, h[3] = {P->dx, P->dy, P->dz};
  double b = INFINITY;
  for (int i = 0; i < 3; i++) {
    if (d[i] == 0.0) continue;
    double idx = floor((x[i] - o[i]) / h[i]);
    double lo = o[i] + idx * h[i], hi = lo + h[i];
    b = dmin(b, d[i] > 0.0 ? ahead(x[i], d[i], hi) : ahead(x[i], d[i], lo > x[i] - 1e-12 ? lo - h[i] : lo));
  }
  return b;
}

/* distance from a panel-local point to the next plane where the material
 * may change: panel faces, layer faces, module edges and the crystal edges of
 * every layer (a superset of the material boundaries) */
static double next_material_plane(const or_scanner *sc, const double l[3], const double d[3]) {
  double b = dmin(ahead(l[0], d[0], 0.0), ahead(l[0], d[0], sc->depth));
  for (int k = 0; k < sc->n_layers; k++) {
    b = dmin(b, ahead(l[0], d[0], sc->layer[k].depth0));
    b = dmin(b, ahead(l[0], d[0], sc->layer[k].depth0 + sc->layer[k].thick));
  }
  for (int ax = 1; ax <= 2; ax++) {
    const double c = l[ax], dc = d[ax];
    if (dc == 0.0) continue;
    const double half = ax == 1 ? 0.5 * sc->width : 0.5 * sc->length;
    b = dmin(b, dmin(ahead(c, dc, -half), ahead(c, dc, half)));
    const int n_mod = ax == 1 ? sc->mod_n_t : sc->mod_n_a;
    const double msz = ax == 1 ? sc->mod_t : sc->mod_a, gap = ax == 1 ? sc->gap_t : sc->gap_a;
    const double step = msz + gap, m0 = -0.5 * (n_mod * msz + (n_mod - 1) * gap);
    const int km = (int)floor((c - m0) / step);
    for (int kk = km - 1; kk <= km + 1; kk++) {
      if (kk < 0 || kk >= n_mod) continue;
      const double ms = m0 + kk * step;
      b = dmin(b, dmin(ahead(c, dc, ms), ahead(c, dc, ms + msz)));
      for (int L = 0; L < sc->n_layers; L++) {
        const or_layer *ly = &sc->layer[L];
        const double off = ax == 1 ? ly->off_t : ly->off_a, pitch = ax == 1 ? ly->pitch_t : ly->pitch_a;
        const double cr = ax == 1 ? ly->cryst_t : ly->cryst_a;
        const int n = ax == 1 ? ly->n_t : ly->n_a;
        const double lo = 0.5 * (pitch - cr), hi = 0.5 * (pitch + cr);
        const int j = (int)floor((c - ms - off) / pitch);
        for (int jj = j - 1; jj <= j + 1; jj++) {
          if (jj < 0 || jj >= n) continue;
          const double base = ms + off + jj * pitch;
          b = dmin(b, dmin(ahead(c, dc, base + lo), ahead(c, dc, base + hi)));
        }
      }
    }
  }
  return b;
}

/* Transport one photon: phantom phase, then panel search / in-panel phase. */
static void photon(const or_scene *s, sink_t *k, uint64_t seed, uint32_t ev, uint32_t inst, int ph,
                   const double x0[3], const double d0[3], uint64_t t_e) {
  rng_t r;
  rng_init(&r, seed, ev, inst, 1 + ph);
  double x[3] = {x0[0], x0[1], x0[2]}, d[3] = {d0[0], d0[1], d0[2]};
  double e = 511.0, L = 0.0;
  uint32_t seq = 0;
  int steps = 0;
  const or_scanner *sc = &s->scan;
  vtx(k, ev, ph, OR_V_EMIT, -1, -1, -1, -1, 0, 0, 0, 0, x, e, 0, d);

  /* ---- phantom phase (Woodcock with the phantom majorant) ---- */
  if (s->has_phantom) {
    const or_phantom *P = &s->ph;
    int64_t vox;
    phantom_voxel(P, x, &vox);
    int in = vox >= 0;
    if (!in) {
      double lo[3] = {P->ox, P->oy, P->oz};
      double hi[3] = {P->ox + P->nx * P->dx, P->oy + P->ny * P->dy, P->oz + P->nz * P->dz};
      double te, tx;
      if (ray_box(x, d, lo, hi, &te, &tx)) {
        for (int i = 0; i < 3; i++) x[i] += te * d[i];
        L += te;
        in = 1;
        vtx(k, ev, ph, OR_V_ENTER_PHANTOM, 0, -1, -1, -1, 0, 0, 0, (int)r.n, x, e, 0, d);
      }
    }
    if (in && k->analog) { /* inside the box from its surface */
      for (int i = 0; i < 3; i++) x[i] += ANALOG_NUDGE * d[i];
      L += ANALOG_NUDGE;
    }
    while (in && k->analog) {
      double u[4];
      rng_next(&r, u);
      k->cnt[6]++;
      double tau = -log(u[0]), mu3[3], mu = 0;
      int m = -1, real = 0;
      for (;;) {
        phantom_voxel(P, x, &vox);
        if (vox < 0) break;
        m = P->mat[vox];
        mu_at(s, m, (double)P->dens[vox], e, mu3);
        mu = mu3[0] + mu3[1] + mu3[2];
        double sb = next_voxel_plane(P, x, d);
        if (tau < mu * sb) {
          double sdist = tau / mu;
          for (int i = 0; i < 3; i++) x[i] += sdist * d[i];
          L += sdist;
          real = 1;
          break;
        }
        tau -= mu * sb;
        for (int i = 0; i < 3; i++) x[i] += (sb + ANALOG_NUDGE) * d[i];
        L += sb + ANALOG_NUDGE;
      }
      if (!real) {
        vtx(k, ev, ph, OR_V_EXIT, 0, -1, -1, -1, 0, 0, 0, (int)r.n, x, e, 0, d);
        break;
      }
      k->cnt[2]++;
      k->cnt[3]++;
      if (++steps > MAX_STEPS) { k->cnt[7]++; return; }
      int proc = pick_process(mu3, mu, u[2]);
      double edep;
      int tr;
      int alive = interact(s, &r, proc, &e, d, 2.0 * PI * u[3], &edep, &tr);
      k->cnt[8] += proc != 1; /* Compton or Rayleigh: a direction change */
      k->cnt[4] += tr;
      k->cnt[6] += tr + (proc == 3);
      vtx(k, ev, ph, OR_V_STEP, 0, -1, -1, m, 1, proc, tr, (int)r.n, x, e, edep, d);
      if (!alive) {
        vtx(k, ev, ph, OR_V_DEAD, 0, -1, -1, m, 0, proc, 0, (int)r.n, x, 0, 0, d);
        return;
      }
    }
    while (in && !k->analog) {
      double u[4];
      rng_next(&r, u);
      k->cnt[6]++;
      double sd = -log(u[0]) / interp(s->maj_ph, e);
      double xn[3] = {x[0] + sd * d[0], x[1] + sd * d[1], x[2] + sd * d[2]};
      phantom_voxel(P, xn, &vox);
      if (vox < 0) { /* left the phantom: continue from the last point inside */
        vtx(k, ev, ph, OR_V_EXIT, 0, -1, -1, -1, 0, 0, 0, (int)r.n, x, e, 0, d);
        break;
      }
      x[0] = xn[0]; x[1] = xn[1]; x[2] = xn[2];
      L += sd;
      k->cnt[2]++;
      if (++steps > MAX_STEPS) { k->cnt[7]++; return; }
      int m = P->mat[vox];
      double mu3[3];
      mu_at(s, m, (double)P->dens[vox], e, mu3);
      double mu = mu3[0] + mu3[1] + mu3[2];
      double mub = interp(s->maj_ph, e);
      int acc = u[1] * mub < mu;
      if (!acc) {
        vtx(k, ev, ph, OR_V_STEP, 0, -1, -1, m, 0, 0, 0, (int)r.n, x, e, 0, d);
        continue;
      }
      k->cnt[3]++;
      int proc = pick_process(mu3, mu, u[2]);
      double edep;
      int tr;
      int alive = interact(s, &r, proc, &e, d, 2.0 * PI * u[3], &edep, &tr);
      k->cnt[8] += proc != 1; /* Compton or Rayleigh: a direction change */
      k->cnt[4] += tr;
      k->cnt[6] += tr + (proc == 3);
      vtx(k, ev, ph, OR_V_STEP, 0, -1, -1, m, 1, proc, tr, (int)r.n, x, e, edep, d);
      if (!alive) {
        vtx(k, ev, ph, OR_V_DEAD, 0, -1, -1, m, 0, proc, 0, (int)r.n, x, 0, 0, d);
        return;
      }
    }
  }

  /* ---- detector phase ---- */
  int last = -1;
  for (;;) {
    double ti;
    k->cnt[5]++;
    int p = panel_search(s, x, d, last, &ti);
    if (p < 0) {
      vtx(k, ev, ph, OR_V_ESCAPE, -1, -1, -1, -1, 0, 0, 0, (int)r.n, x, e, 0, d);
      return;
    }
    for (int i = 0; i < 3; i++) x[i] += ti * d[i];
    L += ti;
    k->cnt[1]++;
    vtx(k, ev, ph, OR_V_ENTER_PANEL, 1, p, -1, -1, 0, 0, 0, (int)r.n, x, e, 0, d);
    const double *P = sc->pose[p];
    double xl[3], dl[3];
    to_local(P, x, xl);
    dir_to_local(P, d, dl);
    if (k->analog) {
      for (int i = 0; i < 3; i++) xl[i] += ANALOG_NUDGE * dl[i];
      L += ANALOG_NUDGE;
    }
    for (; k->analog;) {
      double u[4];
      rng_next(&r, u);
      k->cnt[6]++;
      double tau = -log(u[0]), mu3[3], mu = 0;
      int real = 0;
      loc_t lc = {0, -1, -1, -1, -1};
      for (;;) {
        if (!inside_panel(sc, xl)) break;
        lc = locate_local(s, p, xl, NULL);
        mu_at(s, lc.mat, s->mat[lc.mat].density, e, mu3);
        mu = mu3[0] + mu3[1] + mu3[2];
        double sb = next_material_plane(sc, xl, dl);
        if (tau < mu * sb) {
          double sdist = tau / mu;
          for (int i = 0; i < 3; i++) xl[i] += sdist * dl[i];
          L += sdist;
          real = 1;
          break;
        }
        tau -= mu * sb;
        for (int i = 0; i < 3; i++) xl[i] += (sb + ANALOG_NUDGE) * dl[i];
        L += sb + ANALOG_NUDGE;
      }
      if (!real) { /* left the panel */
        to_global(P, xl, x);
        dir_to_global(P, dl, d);
        vtx(k, ev, ph, OR_V_EXIT, 1, p, -1, -1, 0, 0, 0, (int)r.n, xl, e, 0, dl);
        last = p;
        break;
      }
      k->cnt[2]++;
      k->cnt[3]++;
      if (++steps > MAX_STEPS) { k->cnt[7]++; return; }
      lc = locate_local(s, p, xl, NULL);
      int proc = pick_process(mu3, mu, u[2]);
      double edep;
      int tr;
      int alive = interact(s, &r, proc, &e, dl, 2.0 * PI * u[3], &edep, &tr);
      k->cnt[8] += proc != 1; /* Compton or Rayleigh: a direction change */
      k->cnt[4] += tr;
      k->cnt[6] += tr + (proc == 3);
      vtx(k, ev, ph, OR_V_STEP, 1, p, lc.gid, lc.mat, 1, proc, tr, (int)r.n, xl, e, edep, dl);
      if (lc.gid >= 0 && proc != 3) {
        or_hit h;
        h.event = ev; h.photon = (uint32_t)ph; h.gid = (uint32_t)lc.gid; h.panel = (uint32_t)p;
        h.module = (uint32_t)lc.module; h.layer = (uint32_t)lc.layer; h.crystal = (uint32_t)lc.crystal;
        h.process = (uint32_t)proc; h.seq = seq++;
        h.edep = edep; h.tof_ps = L / C_MM_PER_PS;
        h.depth = xl[0]; h.t = xl[1]; h.a = xl[2];
        h.time_ps = t_e + (uint64_t)floor(h.tof_ps + 0.5);
        push_hit(k, &h);
      }
      if (!alive) {
        vtx(k, ev, ph, OR_V_DEAD, 1, p, lc.gid, lc.mat, 0, proc, 0, (int)r.n, xl, 0, 0, dl);
        return;
      }
    }
    if (k->analog) continue;
    for (;;) {
      double u[4];
      rng_next(&r, u);
      k->cnt[6]++;
      double sd = -log(u[0]) / interp(s->maj_det, e);
      double xn[3] = {xl[0] + sd * dl[0], xl[1] + sd * dl[1], xl[2] + sd * dl[2]};
      if (!inside_panel(sc, xn)) { /* exit: back to the global frame */
        to_global(P, xl, x);
        dir_to_global(P, dl, d);
        vtx(k, ev, ph, OR_V_EXIT, 1, p, -1, -1, 0, 0, 0, (int)r.n, xl, e, 0, dl);
        last = p;
        break;
      }
      xl[0] = xn[0]; xl[1] = xn[1]; xl[2] = xn[2];
      L += sd;
      k->cnt[2]++;
      if (++steps > MAX_STEPS) { k->cnt[7]++; return; }
      loc_t lc = locate_local(s, p, xl, NULL);
      double mu3[3];
      mu_at(s, lc.mat, s->mat[lc.mat].density, e, mu3);
      double mu = mu3[0] + mu3[1] + mu3[2];
      double mub = interp(s->maj_det, e);
      if (!(u[1] * mub < mu)) {
        vtx(k, ev, ph, OR_V_STEP, 1, p, lc.gid, lc.mat, 0, 0, 0, (int)r.n, xl, e, 0, dl);
        continue;
      }
      k->cnt[3]++;
      int proc = pick_process(mu3, mu, u[2]);
      double edep;
      int tr;
      int alive = interact(s, &r, proc, &e, dl, 2.0 * PI * u[3], &edep, &tr);
      k->cnt[8] += proc != 1; /* Compton or Rayleigh: a direction change */
      k->cnt[4] += tr;
      k->cnt[6] += tr + (proc == 3);
      vtx(k, ev, ph, OR_V_STEP, 1, p, lc.gid, lc.mat, 1, proc, tr, (int)r.n, xl, e, edep, dl);
      if (lc.gid >= 0 && proc != 3) {
        or_hit h;
        h.event = ev; h.photon = (uint32_t)ph; h.gid = (uint32_t)lc.gid; h.panel = (uint32_t)p;
        h.module = (uint32_t)lc.module; h.layer = (uint32_t)lc.layer; h.crystal = (uint32_t)lc.crystal;
        h.process = (uint32_t)proc; h.seq = seq++;
        h.edep = edep; h.tof_ps = L / C_MM_PER_PS;
        h.depth = xl[0]; h.t = xl[1]; h.a = xl[2];
        h.time_ps = t_e + (uint64_t)floor(h.tof_ps + 0.5);
        push_hit(k, &h);
      }
      if (!alive) {
        vtx(k, ev, ph, OR_V_DEAD, 1, p, lc.gid, lc.mat, 0, proc, 0, (int)r.n, xl, 0, 0, dl);
        return;
      }
    }
  }
}

/* Event time (Sec. 2.3: a fixed number of decays of a constant activity, so
 * the times are uniform over the acquisition [0, T)): the 64-bit word X of
 * the event stream read as a fraction X / 2^64 of T, floor(X T / 2^64),
 * taken exactly as the high half of the 128-bit product. */
uint64_t or_event_time(uint64_t X, uint64_t T) { return (uint64_t)(((unsigned __int128)X * T) >> 64); }

/* Event: the annihilation point and an isotropic direction from the event
 * stream; photon A leaves along +d, photon B along -d, both at 511 keV
 * (Sec. 2.3: no positron range, annihilation at the emission site).
 * Optional physics the paper leaves out (Sec. 2.3, Sec. 4):
 *  acollinearity   - photon B leaves at polar angle theta from -d, theta the
 *                    length of a 2-D normal vector with the given FWHM per
 *                    component, azimuth uniform (words 2, 3 of block 2);
 *  positron range  - the annihilation point is the emission point plus a 3-D
 *                    normal offset with the given FWHM per axis (block 3). */
static void event(const or_scene *s, sink_t *k, uint64_t seed, uint32_t ev, uint32_t inst) {
  rng_t r;
  rng_init(&r, seed, ev, inst, 0);
  double u0[4], u1[4];
  rng_next(&r, u0);
  rng_next(&r, u1);
  uint32_t w[4];
  rng_raw(&r, 2, w);
  uint64_t t_e = or_event_time(((uint64_t)w[1] << 32) | w[0], s->src.duration_ps);
  double ct = 2.0 * u0[0] - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct)), ph = 2.0 * PI * u0[1];
  double d[3] = {st * cos(ph), st * sin(ph), ct};
  double x[3] = {s->src.pos[0], s->src.pos[1], s->src.pos[2]};
  if (s->src.kind == 2) {
    d[0] = s->src.dir[0]; d[1] = s->src.dir[1]; d[2] = s->src.dir[2];
  } else if (s->src.kind == 1) {
    double tgt = u0[2] * s->rod_total;
    int i = 0;
    while (i < s->src.n_rods - 1 && s->rod_cum[i] < tgt) i++;
    const double *rd = s->src.rods + 5 * i;
    double rr = rd[2] * sqrt(u0[3]), psi = 2.0 * PI * u1[0];
    x[0] = rd[0] + rr * cos(psi);
    x[1] = rd[1] + rr * sin(psi);
    x[2] = rd[3] + u1[1] * (rd[4] - rd[3]);
  }
  double dm[3] = {-d[0], -d[1], -d[2]};
  if (s->src.acol_fwhm_deg > 0) {
    double sig = s->src.acol_fwhm_deg * (PI / 180.0) / FWHM_PER_SIGMA;
    double th = sig * sqrt(-2.0 * log(u01(w[2])));
    rotate(dm, cos(th), 2.0 * PI * u01(w[3]));
  }
  if (s->src.prange_fwhm_mm > 0) {
    uint32_t b[4];
    rng_raw(&r, 3, b);
    double sig = s->src.prange_fwhm_mm / FWHM_PER_SIGMA;
    double a = sqrt(-2.0 * log(u01(b[0]))), c = sqrt(-2.0 * log(u01(b[2])));
    x[0] += sig * a * cos(2.0 * PI * u01(b[1]));
    x[1] += sig * a * sin(2.0 * PI * u01(b[1]));
    x[2] += sig * c * cos(2.0 * PI * u01(b[3]));
  }
  k->cnt[0]++;
  photon(s, k, seed, ev, inst, 0, x, d, t_e);
  photon(s, k, seed, ev, inst, 1, x, dm, t_e);
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Host threads the next calls use (n >= 1); results do not depend on it. */
void or_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* Transport events [first, first+n).  Writes at most cap hits in event order;
 * returns the number of hits produced (which may exceed cap). */
static int64_t transport_mode(const or_scene *s, uint64_t first, uint64_t n, uint64_t seed, uint32_t instance,
                              or_hit *hits, int64_t cap, int64_t *counters, int analog) {
  int nt = or_num_threads();
  sink_t *sk = (sink_t *)calloc((size_t)nt, sizeof(sink_t));
  for (int t = 0; t < nt; t++) sk[t].analog = analog;
#pragma omp parallel num_threads(nt)
  {
#ifdef _OPENMP
    int t = omp_get_thread_num();
#else
    int t = 0;
#endif
    uint64_t lo = first + n * (uint64_t)t / nt, hi = first + n * (uint64_t)(t + 1) / nt;
    for (uint64_t e = lo; e < hi; e++) event(s, &sk[t], seed, (uint32_t)e, instance);
  }
  int64_t tot = 0;
  for (int t = 0; t < nt; t++) {
    for (int64_t i = 0; i < sk[t].n; i++) {
      if (tot + i < cap) hits[tot + i] = sk[t].hits[i];
    }
    tot += sk[t].n;
    if (counters)
      for (int c = 0; c < 9; c++) counters[c] += sk[t].cnt[c];
    free(sk[t].hits);
  }
  free(sk);
  return tot;
}

int64_t or_transport(const or_scene *s, uint64_t first, uint64_t n, uint64_t seed, uint32_t instance,
                     or_hit *hits, int64_t cap, int64_t *counters) {
  return transport_mode(s, first, n, seed, instance, hits, cap, counters, 0);
}

int64_t or_transport_analog(const or_scene *s, uint64_t first, uint64_t n, uint64_t seed, uint32_t instance,
                            or_hit *hits, int64_t cap, int64_t *counters) {
  return transport_mode(s, first, n, seed, instance, hits, cap, counters, 1);
}

static int64_t trace_mode(const or_scene *s, uint64_t first, uint64_t n, uint64_t seed, uint32_t instance,
                          or_vertex *v, int64_t cap, int analog) {
  sink_t k;
  memset(&k, 0, sizeof(k));
  k.v = v;
  k.vcap = cap;
  k.analog = analog;
  for (uint64_t e = first; e < first + n; e++) event(s, &k, seed, (uint32_t)e, instance);
  free(k.hits);
  return k.nv;
}

int64_t or_trace(const or_scene *s, uint64_t first, uint64_t n, uint64_t seed, uint32_t instance,
                 or_vertex *v, int64_t cap) {
  return trace_mode(s, first, n, seed, instance, v, cap, 0);
}

int64_t or_trace_analog(const or_scene *s, uint64_t first, uint64_t n, uint64_t seed, uint32_t instance,
                        or_vertex *v, int64_t cap) {
  return trace_mode(s, first, n, seed, instance, v, cap, 1);
}

/* ------------------------------------------------------------------------ */
/* Digitizer                                                                 */
/* ------------------------------------------------------------------------ */
static int cmp_hit(const void *a, const void *b) {
  const or_hit *x = *(const or_hit *const *)a, *y = *(const or_hit *const *)b;
  if (x->event != y->event) return x->event < y->event ? -1 : 1;
  if (x->gid != y->gid) return x->gid < y->gid ? -1 : 1;
  if (x->photon != y->photon) return x->photon < y->photon ? -1 : 1;
  if (x->seq != y->seq) return x->seq < y->seq ? -1 : 1;
  return 0;
}

static const or_single *g_sorted_base;
/* time order; equal times keep the list order, which is (event, crystal)
 * order as the adder left it */
static int cmp_single_time(const void *a, const void *b) {
  const int64_t ia = *(const int64_t *)a, ib = *(const int64_t *)b;
  const or_single *x = &g_sorted_base[ia], *y = &g_sorted_base[ib];
  if (x->time_ps != y->time_ps) return x->time_ps < y->time_ps ? -1 : 1;
  return ia < ib ? -1 : ia > ib;
}

/* dead-time order: unit, then (time, list position) */
static uint32_t g_dead_unit = 1;
static int cmp_single_unit_time(const void *a, const void *b) {
  const or_single *x = &g_sorted_base[*(const int64_t *)a], *y = &g_sorted_base[*(const int64_t *)b];
  const uint32_t ux = x->gid / g_dead_unit, uy = y->gid / g_dead_unit;
  if (ux != uy) return ux < uy ? -1 : 1;
  return cmp_single_time(a, b);
}

/* Digitizer:
 *  adder   - hits of one event in one crystal sum into a single; its time is the
 *            earliest hit time, its depth the energy-weighted mean;
 *  readout - at module (panel) level the crystal singles of one event in one
 *            module (panel) merge into one single: energies summed, the
 *            earliest time, the crystal and depth of the largest deposit (the
 *            lower crystal id on a tie) -- the readout levels of Sec. 2.1;
 *  blur    - Gaussian with FWHM(E) = fwhm_511 * sqrt(511 E) (16 % at 511 keV,
 *            Sec. 2.3), normal deviate by Box-Muller from the digitizer stream;
 *  time    - (timing resolution, optional) the time moves by a normal
 *            deviate of the given FWHM rounded to the nearest ps (ties to
 *            even), not below 0: words 2, 3 of the blur block;
 *  depth   - (DOI resolution, optional) the depth moves by a normal deviate
 *            of the given FWHM: block 0 of digitizer stream 6;
 *  light   - (light sharing, optional) with probability ls_prob the
 *            crystal is read as one of its edge neighbours in the same layer
 *            and module (those that exist, in the order t-1, t+1, a-1, a+1),
 *            chosen uniformly; block 0 of digitizer stream 8, decided in
 *            integers: word 0 < floor(ls_prob 2^32), neighbour (word 1 * n) >> 32.
 *            The list keeps its order;
 *  dead    - (optional) each unit of the dead-time level sees its blurred
 *            singles in (time, list position) order; paralyzable: a single
 *            is lost when the previous one of its unit came less than dead_ps
 *            earlier; non-paralyzable: when the last single kept came less
 *            than dead_ps earlier.  Lost singles stay in the list (lost = 1)
 *            but pass no window;
 *  window  - e_lo <= E <= e_hi on the blurred energy;
 *  sorter  - windowed singles in time order; a non-retriggering window of
 *            width window_ps (3 ns, Sec. 2.3) opens at the earliest unused
 *            single; exactly two singles in different panels make a
 *            coincidence, two in one panel or more than two are discarded.
 * Singles are returned in (event, crystal) order; coincidences as index pairs
 * into that array, earlier single first.  Returns the number of singles. */
int64_t or_digitize(const or_scene *s, const or_hit *hits, int64_t n_hits, const or_digitizer *dg,
                    or_single *singles, int64_t cap_s, uint32_t *coinc, int64_t cap_c,
                    int64_t *n_coinc) {
  const or_hit **ord = (const or_hit **)malloc((size_t)(n_hits ? n_hits : 1) * sizeof(*ord));
  for (int64_t i = 0; i < n_hits; i++) ord[i] = &hits[i];
  qsort(ord, (size_t)n_hits, sizeof(*ord), cmp_hit);
  or_single *sg = (or_single *)malloc((size_t)(n_hits ? n_hits : 1) * sizeof(or_single));
  int64_t ns = 0;
  for (int64_t i = 0; i < n_hits;) {
    int64_t j = i;
    double e = 0, ed = 0;
    uint64_t tm = UINT64_MAX;
    while (j < n_hits && ord[j]->event == ord[i]->event && ord[j]->gid == ord[i]->gid) {
      e += ord[j]->edep;
      ed += ord[j]->edep * ord[j]->depth;
      if (ord[j]->time_ps < tm) tm = ord[j]->time_ps;
      j++;
    }
    or_single *q = &sg[ns++];
    q->event = ord[i]->event;
    q->gid = ord[i]->gid;
    q->edep = e;
    q->depth = e > 0 ? ed / e : 0.0;
    q->time_ps = tm;
    i = j;
  }
  free(ord);
  if (dg->readout == 1 || dg->readout == 2) {
    const uint32_t G = (uint32_t)(dg->readout == 1 ? s->crystals_per_module : s->crystals_per_panel);
    int64_t m = 0;
    for (int64_t i = 0; i < ns;) {
      int64_t j = i, best = i;
      double e = 0;
      uint64_t tm = UINT64_MAX;
      while (j < ns && sg[j].event == sg[i].event && sg[j].gid / G == sg[i].gid / G) {
        e += sg[j].edep;
        if (sg[j].time_ps < tm) tm = sg[j].time_ps;
        /* the crystal with the largest deposit (the first, i.e. lowest id, on a tie) */
        if (sg[j].edep > sg[best].edep) best = j;
        j++;
      }
      or_single q = sg[best]; /* best >= i >= m: read before the slot is reused */
      q.edep = e;
      q.time_ps = tm;
      sg[m++] = q;
      i = j;
    }
    ns = m;
  }
  for (int64_t i = 0; i < ns; i++) {
    or_single *q = &sg[i];
    rng_t r;
    rng_init(&r, dg->seed, q->event, dg->instance, 3);
    uint32_t w[4];
    rng_raw(&r, q->gid, w);
    double u0 = u01(w[0]), u1 = u01(w[1]);
    double nrm = sqrt(-2.0 * log(u0)) * cos(2.0 * PI * u1);
    double sig = dg->fwhm_511 * sqrt(511.0 * q->edep) / FWHM_PER_SIGMA;
    q->energy = q->edep + sig * nrm;
    q->in_window = q->energy >= dg->e_lo && q->energy <= dg->e_hi;
    q->lost = 0;
    if (dg->time_fwhm_ps > 0) {
      double z = sqrt(-2.0 * log(u01(w[2]))) * cos(2.0 * PI * u01(w[3]));
      double tb = (double)q->time_ps + nearbyint(dg->time_fwhm_ps / FWHM_PER_SIGMA * z);
      q->time_ps = tb > 0 ? (uint64_t)tb : 0;
    }
    if (dg->doi_fwhm_mm > 0) {
      rng_t r6;
      rng_init(&r6, dg->seed, q->event, dg->instance, 6);
      uint32_t v[4];
      rng_raw(&r6, q->gid, v);
      double z = sqrt(-2.0 * log(u01(v[0]))) * cos(2.0 * PI * u01(v[1]));
      q->depth += dg->doi_fwhm_mm / FWHM_PER_SIGMA * z;
    }
  }
  if (dg->ls_prob > 0) {
    const uint64_t thr = dg->ls_prob >= 1.0 ? (1ull << 32) : (uint64_t)floor(dg->ls_prob * 4294967296.0);
    const uint32_t cpm = (uint32_t)s->crystals_per_module;
    for (int64_t i = 0; i < ns; i++) {
      or_single *q = &sg[i];
      rng_t r8;
      rng_init(&r8, dg->seed, q->event, dg->instance, 8);
      uint32_t v[4];
      rng_raw(&r8, q->gid, v);
      if ((uint64_t)v[0] >= thr) continue;
      /* the crystal's place in its module: layer by its first id, then (t, a) */
      const uint32_t local = q->gid % cpm;
      int l = 0;
      for (int k = 1; k < s->scan.n_layers; k++)
        if (local >= (uint32_t)s->layer_base[k]) l = k;
      const uint32_t nt = (uint32_t)s->scan.layer[l].n_t, na = (uint32_t)s->scan.layer[l].n_a;
      const uint32_t it = (local - (uint32_t)s->layer_base[l]) % nt;
      const uint32_t ia = (local - (uint32_t)s->layer_base[l]) / nt;
      uint32_t nb[4];
      int n = 0;
      if (it > 0) nb[n++] = q->gid - 1;
      if (it + 1 < nt) nb[n++] = q->gid + 1;
      if (ia > 0) nb[n++] = q->gid - nt;
      if (ia + 1 < na) nb[n++] = q->gid + nt;
      if (n) q->gid = nb[((uint64_t)v[1] * (uint64_t)n) >> 32];
    }
  }
  if (dg->dead_mode == 1 || dg->dead_mode == 2) {
    const uint32_t G = (uint32_t)(dg->dead_level == 1 ? s->crystals_per_module
                                  : dg->dead_level == 2 ? s->crystals_per_panel : 1);
    int64_t *ord = (int64_t *)malloc((size_t)(ns ? ns : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < ns; i++) ord[i] = i;
    g_sorted_base = sg;
    g_dead_unit = G;
    qsort(ord, (size_t)ns, sizeof(int64_t), cmp_single_unit_time);
    uint64_t ref = 0; /* previous single (paralyzable) or last kept one */
    for (int64_t k = 0; k < ns; k++) {
      or_single *q = &sg[ord[k]];
      const int first = k == 0 || sg[ord[k - 1]].gid / G != q->gid / G;
      if (!first && q->time_ps - ref < dg->dead_ps) q->lost = 1;
      if (dg->dead_mode == 1 || !q->lost) ref = q->time_ps;
    }
    free(ord);
  }
  int64_t nw = 0;
  int64_t *idx = (int64_t *)malloc((size_t)(ns ? ns : 1) * sizeof(int64_t));
  for (int64_t i = 0; i < ns; i++)
    if (sg[i].in_window && !sg[i].lost) idx[nw++] = i;
  g_sorted_base = sg;
  qsort(idx, (size_t)nw, sizeof(int64_t), cmp_single_time);
  int64_t nc = 0;
  for (int64_t i = 0; i < nw;) {
    int64_t j = i + 1;
    while (j < nw && sg[idx[j]].time_ps - sg[idx[i]].time_ps <= dg->window_ps) j++;
    if (j - i == 2) {
      uint32_t pa = sg[idx[i]].gid / (uint32_t)s->crystals_per_panel;
      uint32_t pb = sg[idx[i + 1]].gid / (uint32_t)s->crystals_per_panel;
      if (pa != pb) {
        if (nc < cap_c) {
          coinc[2 * nc] = (uint32_t)idx[i];
          coinc[2 * nc + 1] = (uint32_t)idx[i + 1];
        }
        nc++;
      }
    }
    i = j;
  }
  free(idx);
  for (int64_t i = 0; i < ns && i < cap_s; i++) singles[i] = sg[i];
  free(sg);
  *n_coinc = nc;
  return ns;
}
