/*
 * FP64 CPU oracle for the 3-D Yee leapfrog with a moving shower current.
 * TEST INFRASTRUCTURE ONLY -- see yee_oracle.h for what it computes and for
 * the lattice conventions.  Plain loops, no blocking or fusion: each function
 * follows one equation of the paper (or one textbook boundary scheme where
 * the paper is silent) so that it can be read against it.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC yee_oracle.c -o liborc.so -lm
 */
#include "yee_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static const double C0 = 299792458.0;
static const double MU0 = 1.25663706212e-6; /* CODATA 2018 */
static double eps0(void) { return 1.0 / (MU0 * C0 * C0); }

double orc_c0(void) { return C0; }
double orc_mu0(void) { return MU0; }
double orc_eps0(void) { return eps0(); }
int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

static __thread char g_err[256];
const char *orc_last_error(void) { return g_err; }
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }

/* 1-D CPML grading along one axis. */
typedef struct {
  int n;
  int *pe, *ph;          /* slab slot of integer / half positions, -1 outside PML */
  double *ae, *be, *ke;  /* grading at integer positions (E-update derivatives) */
  double *ah, *bh, *kh;  /* grading at half positions (H-update derivatives) */
} pml_axis;

struct orc_state {
  orc_cfg c;
  double *q, *obs;
  size_t ncell;
  double *f[6];
  double *eold[3];
  pml_axis ax[3];
  int np2;
  double *psi_e[3][3], *psi_h[3][3]; /* [field component][derivative axis] */
  double *wr;                        /* radial weights on the Ez (i,j) lattice */
  double ca, cb, db, v_med, v_src;
  double *ca_map[3], *cb_map[3];     /* per-E-node coefficients of a permittivity map, or NULL */
  int32_t n;
};

#define IDX(s, i, j, k) ((((size_t)(k)) * (size_t)(s)->c.ny + (size_t)(j)) * (size_t)(s)->c.nx + (size_t)(i))

static size_t psi_len(const orc_state *s, int u) {
  size_t nx = s->c.nx, ny = s->c.ny, nz = s->c.nz, p = s->np2;
  return u == 0 ? p * ny * nz : (u == 1 ? nx * p * nz : nx * ny * p);
}

static size_t psi_idx(const orc_state *s, int u, int i, int j, int k, int p) {
  size_t nx = s->c.nx, ny = s->c.ny, np2 = s->np2;
  if (u == 0) return ((size_t)k * ny + j) * np2 + p;
  if (u == 1) return ((size_t)k * np2 + p) * nx + i;
  return ((size_t)p * ny + j) * nx + i;
}

/* ------------------------------------------------------------------ CPML */
/* Convolutional PML with complex-frequency-shifted stretching
   s_u = kappa + sigma/(alpha + j omega eps0) (Roden & Gedney, 2000):
   psi^{new} = b psi + a dF/du, and dF/du -> dF/du / kappa + psi^{new}. */
static void pml_grade(const orc_state *s, double depth_cells, double delta, double *a, double *b,
                      double *k) {
  const orc_cfg *c = &s->c;
  const double eta0 = MU0 * C0;
  double rho = depth_cells / c->npml; /* 0 at the inner edge, 1 at the wall */
  double sig_opt = 0.8 * (c->pml_m + 1.0) / (eta0 * delta * sqrt(c->eps_r * c->mu_r));
  double sigma = c->pml_sigma_scale * sig_opt * pow(rho, c->pml_m);
  double kappa = 1.0 + (c->pml_kappa_max - 1.0) * pow(rho, c->pml_m);
  double alpha = c->pml_alpha_max * (1.0 - rho);
  double bb = exp(-(sigma / kappa + alpha) * c->dt / eps0());
  *b = bb;
  *k = kappa;
  *a = sigma * (bb - 1.0) / (sigma * kappa + kappa * kappa * alpha);
}

static int pml_axis_init(orc_state *s, pml_axis *a, int n, double delta) {
  int npml = s->c.bc == ORC_BC_CPML ? s->c.npml : 0;
  a->n = n;
  a->pe = malloc(sizeof(int) * n);
  a->ph = malloc(sizeof(int) * n);
  a->ae = calloc(n, sizeof(double));
  a->be = calloc(n, sizeof(double));
  a->ke = calloc(n, sizeof(double));
  a->ah = calloc(n, sizeof(double));
  a->bh = calloc(n, sizeof(double));
  a->kh = calloc(n, sizeof(double));
  if (!a->pe || !a->ph || !a->ae || !a->be || !a->ke || !a->ah || !a->bh || !a->kh) return -1;
  for (int i = 0; i < n; i++) {
    a->pe[i] = a->ph[i] = -1;
    a->ke[i] = a->kh[i] = 1.0;
    if (npml <= 0) continue;
    /* integer position i: depth measured from the inner PML planes npml and n-1-npml */
    double de = fmax(fmax((double)npml - i, (double)i - (n - 1 - npml)), 0.0);
    if (de > 0.0) {
      a->pe[i] = i < npml ? i : npml + (i - (n - npml));
      pml_grade(s, de, delta, &a->ae[i], &a->be[i], &a->ke[i]);
    }
    /* half position i+1/2 (exists for i <= n-2) */
    if (i <= n - 2) {
      double dh = fmax(fmax((double)npml - (i + 0.5), (i + 0.5) - (n - 1 - npml)), 0.0);
      if (dh > 0.0) {
        a->ph[i] = i < npml ? i : npml + (i - (n - 1 - npml));
        pml_grade(s, dh, delta, &a->ah[i], &a->bh[i], &a->kh[i]);
      }
    }
  }
  return 0;
}

static void pml_axis_free(pml_axis *a) {
  free(a->pe); free(a->ph); free(a->ae); free(a->be); free(a->ke);
  free(a->ah); free(a->bh); free(a->kh);
}

/* Stretched derivative: returns d/kappa + psi (updating psi) inside the PML, d outside. */
static double pml_term(orc_state *s, double *psi, int u, int pos, int half, int i, int j, int k,
                       double d) {
  const pml_axis *a = &s->ax[u];
  int p = half ? a->ph[pos] : a->pe[pos];
  if (p < 0) return d;
  size_t id = psi_idx(s, u, i, j, k, p);
  double aa = half ? a->ah[pos] : a->ae[pos];
  double bb = half ? a->bh[pos] : a->be[pos];
  double kk = half ? a->kh[pos] : a->ke[pos];
  psi[id] = bb * psi[id] + aa * d;
  return d / kk + psi[id];
}

/* ------------------------------------------------------------- source */
/* Total charge excess Q(z) from the profile bins with hat-function interpolation. */
static double profile_q(const orc_state *s, double z) {
  double u = (z - s->c.z_bin0) / s->c.dz_bin;
  double fl = floor(u);
  int b0 = (int)fl;
  double t = u - fl;
  double q = 0.0;
  if (b0 >= 0 && b0 < s->c.n_bins) q += (1.0 - t) * s->q[b0];
  if (b0 + 1 >= 0 && b0 + 1 < s->c.n_bins) q += t * s->q[b0 + 1];
  return q;
}

/* Hat weight of bin b at position z (the derivative of Q(z) with respect to q_b). */
static double profile_hat(const orc_state *s, int b, double z) {
  double u = (z - s->c.z_bin0) / s->c.dz_bin - b;
  double w = 1.0 - fabs(u);
  return w > 0.0 ? w : 0.0;
}

static double source_zs(const orc_state *s, int32_t n) {
  double t = (n + 0.5) * s->c.dt;
  return s->c.z_entry + s->v_src * (t - s->c.t_entry);
}

static int source_active(const orc_state *s, int32_t n) {
  return s->c.src_on && (n + 0.5) * s->c.dt >= s->c.t_entry;
}

/* Longitudinal weights W_z(k) for the Ez nodes at z=(k+1/2)dz around z_s, truncated at
   cut*sigma_z and normalised on the lattice (sum W_z dz = 1).  Returns the first k and
   fills wz[0..count-1]; count <= cap. */
static int source_wz(const orc_state *s, double zs, double *wz, int cap, int *count) {
  const orc_cfg *c = &s->c;
  double half = c->cut_sigmas * c->sigma_z;
  int klo = (int)ceil((zs - half) / c->dz - 0.5);
  int khi = (int)floor((zs + half) / c->dz - 0.5);
  int m = khi - klo + 1;
  if (m > cap) m = cap;
  double norm = 0.0;
  for (int t = 0; t < m; t++) {
    double d = (klo + t + 0.5) * c->dz - zs;
    wz[t] = exp(-0.5 * d * d / (c->sigma_z * c->sigma_z));
    norm += wz[t] * c->dz;
  }
  for (int t = 0; t < m; t++) wz[t] /= norm;
  *count = m;
  return klo;
}

/* Charge-density snapshot of the Simulation Setup section, times v: J_z on the Ez lattice. */
void orc_source_current(const orc_state *s, int32_t n, double *jz) {
  memset(jz, 0, sizeof(double) * s->ncell);
  if (!source_active(s, n)) return;
  double zs = source_zs(s, n);
  double qz = profile_q(s, zs);
  double wz[64];
  int m;
  int klo = source_wz(s, zs, wz, 64, &m);
  for (int t = 0; t < m; t++) {
    int k = klo + t;
    if (k < 0 || k > s->c.nz - 2) continue;
    for (int j = 1; j <= s->c.ny - 2; j++)
      for (int i = 1; i <= s->c.nx - 2; i++) {
        double w = s->wr[(size_t)j * s->c.nx + i];
        if (w != 0.0) jz[IDX(s, i, j, k)] = s->v_src * qz * w * wz[t];
      }
  }
}

/* ---------------------------------------------------------- create/free */
orc_state *orc_create(const orc_cfg *cfg) {
  const orc_cfg *c = cfg;
  if (c->nx < 3 || c->ny < 3 || c->nz < 3 || c->n_steps < 0) { set_err("bad grid"); return NULL; }
  if (!(c->dx > 0 && c->dy > 0 && c->dz > 0 && c->dt > 0)) { set_err("bad spacing"); return NULL; }
  if (!(c->eps_r > 0 && c->mu_r > 0 && c->sigma >= 0)) { set_err("bad medium"); return NULL; }
  if (c->bc < 0 || c->bc > 2) { set_err("bad boundary kind"); return NULL; }
  if (c->bc == ORC_BC_CPML && (c->npml < 1 || 2 * c->npml + 3 > c->nx || 2 * c->npml + 3 > c->ny ||
                               2 * c->npml + 3 > c->nz)) {
    set_err("bad npml");
    return NULL;
  }
  orc_state *s = calloc(1, sizeof *s);
  if (!s) return NULL;
  s->c = *cfg;
  s->ncell = (size_t)c->nx * c->ny * c->nz;
  s->v_med = C0 / sqrt(c->eps_r * c->mu_r);
  s->v_src = c->beta * C0;
  double eps = eps0() * c->eps_r, mu = MU0 * c->mu_r;
  double loss = c->sigma * c->dt / (2.0 * eps);
  s->ca = (1.0 - loss) / (1.0 + loss);
  s->cb = (c->dt / eps) / (1.0 + loss);
  s->db = c->dt / mu;
  for (int f = 0; f < 6; f++) {
    s->f[f] = calloc(s->ncell, sizeof(double));
    if (!s->f[f]) { set_err("out of memory"); orc_destroy(s); return NULL; }
  }
  if (c->bc == ORC_BC_MUR1)
    for (int f = 0; f < 3; f++) {
      s->eold[f] = calloc(s->ncell, sizeof(double));
      if (!s->eold[f]) { set_err("out of memory"); orc_destroy(s); return NULL; }
    }
  s->np2 = c->bc == ORC_BC_CPML ? 2 * c->npml : 0;
  int dims[3] = {c->nx, c->ny, c->nz};
  double del[3] = {c->dx, c->dy, c->dz};
  for (int u = 0; u < 3; u++)
    if (pml_axis_init(s, &s->ax[u], dims[u], del[u])) { set_err("out of memory"); orc_destroy(s); return NULL; }
  if (c->bc == ORC_BC_CPML) {
    for (int f = 0; f < 3; f++)
      for (int u = 0; u < 3; u++) {
        if (u == f) continue;
        s->psi_e[f][u] = calloc(psi_len(s, u), sizeof(double));
        s->psi_h[f][u] = calloc(psi_len(s, u), sizeof(double));
        if (!s->psi_e[f][u] || !s->psi_h[f][u]) { set_err("out of memory"); orc_destroy(s); return NULL; }
      }
  }
  s->q = calloc(c->n_bins > 0 ? c->n_bins : 1, sizeof(double));
  s->obs = calloc(c->n_obs > 0 ? 3 * c->n_obs : 1, sizeof(double));
  s->wr = calloc((size_t)c->nx * c->ny, sizeof(double));
  if (!s->q || !s->obs || !s->wr) { set_err("out of memory"); orc_destroy(s); return NULL; }
  if (c->n_bins > 0 && c->q_bins) memcpy(s->q, c->q_bins, sizeof(double) * c->n_bins);
  if (c->n_obs > 0 && c->obs_xyz) memcpy(s->obs, c->obs_xyz, sizeof(double) * 3 * c->n_obs);
  s->c.q_bins = s->q;
  s->c.obs_xyz = s->obs;
  if (c->src_on) {
    if (!(c->sigma_r > 0 && c->sigma_z > 0 && c->cut_sigmas > 0 && c->n_bins >= 1 && c->dz_bin > 0)) {
      set_err("bad source");
      orc_destroy(s);
      return NULL;
    }
    if (c->sigma_z * c->cut_sigmas / c->dz > 30.0) { set_err("sigma_z too wide"); orc_destroy(s); return NULL; }
    /* radial weights at the Ez nodes (x_i, y_j), truncated at cut*sigma_r, sum W dx dy = 1 */
    double cut2 = c->cut_sigmas * c->sigma_r * c->cut_sigmas * c->sigma_r, norm = 0.0;
    for (int j = 1; j <= c->ny - 2; j++)
      for (int i = 1; i <= c->nx - 2; i++) {
        double ddx = i * c->dx - c->x_axis, ddy = j * c->dy - c->y_axis;
        double r2 = ddx * ddx + ddy * ddy;
        if (r2 <= cut2) {
          double w = exp(-0.5 * r2 / (c->sigma_r * c->sigma_r));
          s->wr[(size_t)j * c->nx + i] = w;
          norm += w * c->dx * c->dy;
        }
      }
    if (norm <= 0.0) { set_err("source misses the grid"); orc_destroy(s); return NULL; }
    for (size_t t = 0; t < (size_t)c->nx * c->ny; t++) s->wr[t] /= norm;
  }
  /* every trilinear stencil must lie inside, clear of walls and PML */
  int margin = c->bc == ORC_BC_CPML ? c->npml : 1;
  for (int o = 0; o < c->n_obs; o++)
    for (int comp = 0; comp < 3; comp++)
      for (int u = 0; u < 3; u++) {
        double off = (u == comp) ? 0.5 : 0.0;
        double fpos = s->obs[3 * o + u] / del[u] - off;
        double i0 = floor(fpos);
        if (i0 < margin || i0 + 1 > dims[u] - 1 - margin) {
          set_err("observer stencil outside the interior");
          orc_destroy(s);
          return NULL;
        }
      }
  return s;
}

void orc_destroy(orc_state *s) {
  if (!s) return;
  for (int f = 0; f < 6; f++) free(s->f[f]);
  for (int f = 0; f < 3; f++) { free(s->eold[f]); free(s->ca_map[f]); free(s->cb_map[f]); }
  for (int f = 0; f < 3; f++)
    for (int u = 0; u < 3; u++) { free(s->psi_e[f][u]); free(s->psi_h[f][u]); }
  for (int u = 0; u < 3; u++) pml_axis_free(&s->ax[u]);
  free(s->q); free(s->obs); free(s->wr);
  free(s);
}

double *orc_field(orc_state *s, int comp) { return (comp >= 0 && comp < 6) ? s->f[comp] : NULL; }
int32_t orc_step_index(const orc_state *s) { return s->n; }

/* A heterogeneous medium: Ampere's law with conductivity keeps its form node by node, so each E
   node takes Ca and Cb from the relative permittivity of its own position.  The CPML grading and
   the Mur coefficients keep the configuration's uniform eps_r (they belong to the absorber). */
int orc_set_eps_map(orc_state *s, const double *eps_r_map) {
  for (int f = 0; f < 3; f++) {
    free(s->ca_map[f]);
    free(s->cb_map[f]);
    s->ca_map[f] = s->cb_map[f] = NULL;
  }
  if (!eps_r_map) return 0;
  for (size_t t = 0; t < 3 * s->ncell; t++)
    if (!(eps_r_map[t] > 0)) { set_err("bad permittivity map"); return -1; }
  for (int f = 0; f < 3; f++) {
    s->ca_map[f] = malloc(sizeof(double) * s->ncell);
    s->cb_map[f] = malloc(sizeof(double) * s->ncell);
    if (!s->ca_map[f] || !s->cb_map[f]) { set_err("out of memory"); orc_set_eps_map(s, NULL); return -1; }
    for (size_t t = 0; t < s->ncell; t++) {
      double eps = eps0() * eps_r_map[f * s->ncell + t];
      double loss = s->c.sigma * s->c.dt / (2.0 * eps);
      s->ca_map[f][t] = (1.0 - loss) / (1.0 + loss);
      s->cb_map[f][t] = (s->c.dt / eps) / (1.0 + loss);
    }
  }
  return 0;
}

/* ------------------------------------------------------------ updates */
#define EX(i, j, k) s->f[0][IDX(s, i, j, k)]
#define EY(i, j, k) s->f[1][IDX(s, i, j, k)]
#define EZ(i, j, k) s->f[2][IDX(s, i, j, k)]
#define HX(i, j, k) s->f[3][IDX(s, i, j, k)]
#define HY(i, j, k) s->f[4][IDX(s, i, j, k)]
#define HZ(i, j, k) s->f[5][IDX(s, i, j, k)]

/* Faraday's law, -mu dH/dt = curl E, with forward differences of E. */
void orc_update_h(orc_state *s) {
  const int nx = s->c.nx, ny = s->c.ny, nz = s->c.nz;
  const double dx = s->c.dx, dy = s->c.dy, dz = s->c.dz, db = s->db;
  /* Hx(i, j+1/2, k+1/2) */
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz - 1; k++)
    for (int j = 0; j < ny - 1; j++)
      for (int i = 0; i < nx; i++) {
        double dez_dy = (EZ(i, j + 1, k) - EZ(i, j, k)) / dy;
        double dey_dz = (EY(i, j, k + 1) - EY(i, j, k)) / dz;
        double ty = pml_term(s, s->psi_h[0][1], 1, j, 1, i, j, k, dez_dy);
        double tz = pml_term(s, s->psi_h[0][2], 2, k, 1, i, j, k, dey_dz);
        HX(i, j, k) -= db * (ty - tz);
      }
  /* Hy(i+1/2, j, k+1/2) */
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz - 1; k++)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i < nx - 1; i++) {
        double dex_dz = (EX(i, j, k + 1) - EX(i, j, k)) / dz;
        double dez_dx = (EZ(i + 1, j, k) - EZ(i, j, k)) / dx;
        double tz = pml_term(s, s->psi_h[1][2], 2, k, 1, i, j, k, dex_dz);
        double tx = pml_term(s, s->psi_h[1][0], 0, i, 1, i, j, k, dez_dx);
        HY(i, j, k) -= db * (tz - tx);
      }
  /* Hz(i+1/2, j+1/2, k) */
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; k++)
    for (int j = 0; j < ny - 1; j++)
      for (int i = 0; i < nx - 1; i++) {
        double dey_dx = (EY(i + 1, j, k) - EY(i, j, k)) / dx;
        double dex_dy = (EX(i, j + 1, k) - EX(i, j, k)) / dy;
        double tx = pml_term(s, s->psi_h[2][0], 0, i, 1, i, j, k, dey_dx);
        double ty = pml_term(s, s->psi_h[2][1], 1, j, 1, i, j, k, dex_dy);
        HZ(i, j, k) -= db * (tx - ty);
      }
}

/* First-order Mur on the face-interior tangential E of all six faces (edges stay 0). */
static void mur_faces(orc_state *s) {
  const int nx = s->c.nx, ny = s->c.ny, nz = s->c.nz;
  const double vdt = s->v_med * s->c.dt;
  const double kx = (vdt - s->c.dx) / (vdt + s->c.dx);
  const double ky = (vdt - s->c.dy) / (vdt + s->c.dy);
  const double kz = (vdt - s->c.dz) / (vdt + s->c.dz);
  double *ox = s->eold[0], *oy = s->eold[1], *oz = s->eold[2];
#define OLD(a, i, j, k) a[IDX(s, i, j, k)]
  /* x faces: Ey, Ez */
  for (int k = 1; k <= nz - 2; k++)
    for (int j = 0; j <= ny - 2; j++) {
      EY(0, j, k) = OLD(oy, 1, j, k) + kx * (EY(1, j, k) - OLD(oy, 0, j, k));
      EY(nx - 1, j, k) = OLD(oy, nx - 2, j, k) + kx * (EY(nx - 2, j, k) - OLD(oy, nx - 1, j, k));
    }
  for (int k = 0; k <= nz - 2; k++)
    for (int j = 1; j <= ny - 2; j++) {
      EZ(0, j, k) = OLD(oz, 1, j, k) + kx * (EZ(1, j, k) - OLD(oz, 0, j, k));
      EZ(nx - 1, j, k) = OLD(oz, nx - 2, j, k) + kx * (EZ(nx - 2, j, k) - OLD(oz, nx - 1, j, k));
    }
  /* y faces: Ex, Ez */
  for (int k = 1; k <= nz - 2; k++)
    for (int i = 0; i <= nx - 2; i++) {
      EX(i, 0, k) = OLD(ox, i, 1, k) + ky * (EX(i, 1, k) - OLD(ox, i, 0, k));
      EX(i, ny - 1, k) = OLD(ox, i, ny - 2, k) + ky * (EX(i, ny - 2, k) - OLD(ox, i, ny - 1, k));
    }
  for (int k = 0; k <= nz - 2; k++)
    for (int i = 1; i <= nx - 2; i++) {
      EZ(i, 0, k) = OLD(oz, i, 1, k) + ky * (EZ(i, 1, k) - OLD(oz, i, 0, k));
      EZ(i, ny - 1, k) = OLD(oz, i, ny - 2, k) + ky * (EZ(i, ny - 2, k) - OLD(oz, i, ny - 1, k));
    }
  /* z faces: Ex, Ey */
  for (int j = 1; j <= ny - 2; j++)
    for (int i = 0; i <= nx - 2; i++) {
      EX(i, j, 0) = OLD(ox, i, j, 1) + kz * (EX(i, j, 1) - OLD(ox, i, j, 0));
      EX(i, j, nz - 1) = OLD(ox, i, j, nz - 2) + kz * (EX(i, j, nz - 2) - OLD(ox, i, j, nz - 1));
    }
  for (int j = 0; j <= ny - 2; j++)
    for (int i = 1; i <= nx - 2; i++) {
      EY(i, j, 0) = OLD(oy, i, j, 1) + kz * (EY(i, j, 1) - OLD(oy, i, j, 0));
      EY(i, j, nz - 1) = OLD(oy, i, j, nz - 2) + kz * (EY(i, j, nz - 2) - OLD(oy, i, j, nz - 1));
    }
#undef OLD
}

/* Ampere's law with conductivity, eps dE/dt + sigma E = curl H - J, with backward
   differences of H; the tangential E on the walls is left to the boundary scheme. */
void orc_update_e(orc_state *s) {
  const int nx = s->c.nx, ny = s->c.ny, nz = s->c.nz;
  const double dx = s->c.dx, dy = s->c.dy, dz = s->c.dz, ca = s->ca, cb = s->cb;
  if (s->c.bc == ORC_BC_MUR1)
    for (int f = 0; f < 3; f++) memcpy(s->eold[f], s->f[f], sizeof(double) * s->ncell);
  /* Ex(i+1/2, j, k) */
#pragma omp parallel for schedule(static)
  for (int k = 1; k <= nz - 2; k++)
    for (int j = 1; j <= ny - 2; j++)
      for (int i = 0; i <= nx - 2; i++) {
        double dhz_dy = (HZ(i, j, k) - HZ(i, j - 1, k)) / dy;
        double dhy_dz = (HY(i, j, k) - HY(i, j, k - 1)) / dz;
        double ty = pml_term(s, s->psi_e[0][1], 1, j, 0, i, j, k, dhz_dy);
        double tz = pml_term(s, s->psi_e[0][2], 2, k, 0, i, j, k, dhy_dz);
        size_t id = IDX(s, i, j, k);
        double a = s->ca_map[0] ? s->ca_map[0][id] : ca, b = s->cb_map[0] ? s->cb_map[0][id] : cb;
        EX(i, j, k) = a * EX(i, j, k) + b * (ty - tz);
      }
  /* Ey(i, j+1/2, k) */
#pragma omp parallel for schedule(static)
  for (int k = 1; k <= nz - 2; k++)
    for (int j = 0; j <= ny - 2; j++)
      for (int i = 1; i <= nx - 2; i++) {
        double dhx_dz = (HX(i, j, k) - HX(i, j, k - 1)) / dz;
        double dhz_dx = (HZ(i, j, k) - HZ(i - 1, j, k)) / dx;
        double tz = pml_term(s, s->psi_e[1][2], 2, k, 0, i, j, k, dhx_dz);
        double tx = pml_term(s, s->psi_e[1][0], 0, i, 0, i, j, k, dhz_dx);
        size_t id = IDX(s, i, j, k);
        double a = s->ca_map[1] ? s->ca_map[1][id] : ca, b = s->cb_map[1] ? s->cb_map[1][id] : cb;
        EY(i, j, k) = a * EY(i, j, k) + b * (tz - tx);
      }
  /* Ez(i, j, k+1/2), with the shower current J_z = v Q(z_s) W_r(i,j) W_z(k) */
  double wz[64], vq = 0.0;
  int m = 0, klo = 0;
  if (source_active(s, s->n)) {
    double zs = source_zs(s, s->n);
    vq = s->v_src * profile_q(s, zs);
    klo = source_wz(s, zs, wz, 64, &m);
  }
#pragma omp parallel for schedule(static)
  for (int k = 0; k <= nz - 2; k++)
    for (int j = 1; j <= ny - 2; j++)
      for (int i = 1; i <= nx - 2; i++) {
        double dhy_dx = (HY(i, j, k) - HY(i - 1, j, k)) / dx;
        double dhx_dy = (HX(i, j, k) - HX(i, j - 1, k)) / dy;
        double tx = pml_term(s, s->psi_e[2][0], 0, i, 0, i, j, k, dhy_dx);
        double ty = pml_term(s, s->psi_e[2][1], 1, j, 0, i, j, k, dhx_dy);
        double j_src = 0.0;
        if (k >= klo && k < klo + m) j_src = vq * s->wr[(size_t)j * nx + i] * wz[k - klo];
        size_t id = IDX(s, i, j, k);
        double a = s->ca_map[2] ? s->ca_map[2][id] : ca, b = s->cb_map[2] ? s->cb_map[2][id] : cb;
        EZ(i, j, k) = a * EZ(i, j, k) + b * (tx - ty - j_src);
      }
  if (s->c.bc == ORC_BC_MUR1) mur_faces(s);
  s->n += 1;
}

/* Trilinear interpolation of each E component on its own staggered sub-lattice. */
static void obs_stencil(const orc_state *s, int o, int comp, int *i0, double *t) {
  const double del[3] = {s->c.dx, s->c.dy, s->c.dz};
  for (int u = 0; u < 3; u++) {
    double off = (u == comp) ? 0.5 : 0.0;
    double fpos = s->obs[3 * o + u] / del[u] - off;
    double fl = floor(fpos);
    i0[u] = (int)fl;
    t[u] = fpos - fl;
  }
}

void orc_sample(const orc_state *s, double *w) {
  for (int o = 0; o < s->c.n_obs; o++)
    for (int comp = 0; comp < 3; comp++) {
      int i0[3];
      double t[3], acc = 0.0;
      obs_stencil(s, o, comp, i0, t);
      for (int c = 0; c < 2; c++)
        for (int b = 0; b < 2; b++)
          for (int a = 0; a < 2; a++) {
            double wgt = (a ? t[0] : 1.0 - t[0]) * (b ? t[1] : 1.0 - t[1]) * (c ? t[2] : 1.0 - t[2]);
            acc += wgt * s->f[comp][IDX(s, i0[0] + a, i0[1] + b, i0[2] + c)];
          }
      w[3 * o + comp] = acc;
    }
}

void orc_step(orc_state *s, double *w) {
  orc_update_h(s);
  orc_update_e(s);
  if (w) orc_sample(s, w);
}

int orc_run(const orc_cfg *cfg, double *waveforms) { return orc_run_eps(cfg, NULL, waveforms); }

int orc_run_eps(const orc_cfg *cfg, const double *eps_r_map, double *waveforms) {
  orc_state *s = orc_create(cfg);
  if (!s) return -1;
  if (orc_set_eps_map(s, eps_r_map)) { orc_destroy(s); return -1; }
  int no = cfg->n_obs, T = cfg->n_steps;
  double *w = malloc(sizeof(double) * (no > 0 ? 3 * no : 1));
  if (!w) { orc_destroy(s); return -1; }
  for (int n = 0; n < T; n++) {
    orc_step(s, w);
    for (int o = 0; o < no; o++)
      for (int c = 0; c < 3; c++) waveforms[((size_t)o * 3 + c) * T + n] = w[3 * o + c];
  }
  free(w);
  orc_destroy(s);
  return 0;
}

/* ------------------------------------------------------------ adjoint */
/* Reverse-mode transpose of the stretched derivative t = d/kappa + psi', psi' = b psi + a d,
   given the cotangent tb of t.  psib holds the cotangent of psi' carried from later steps;
   on return it holds the cotangent of the old psi.  Returns the cotangent of d. */
static double pml_term_t(const orc_state *s, double *psib, int u, int pos, int half, int i, int j,
                         int k, double tb) {
  const pml_axis *a = &s->ax[u];
  int p = half ? a->ph[pos] : a->pe[pos];
  if (p < 0) return tb;
  size_t id = psi_idx(s, u, i, j, k, p);
  double aa = half ? a->ah[pos] : a->ae[pos];
  double bb = half ? a->bh[pos] : a->be[pos];
  double kk = half ? a->kh[pos] : a->ke[pos];
  double pnew = psib[id] + tb; /* psi' feeds t and the next step */
  psib[id] = bb * pnew;
  return tb / kk + aa * pnew;
}

int orc_adjoint(const orc_cfg *cfg, const double *dl_dw, double *dl_dq) {
  if (cfg->bc == ORC_BC_MUR1) { set_err("adjoint: Mur boundary not supported"); return -2; }
  orc_state *s = orc_create(cfg);
  if (!s) return -1;
  const int nx = s->c.nx, ny = s->c.ny, nz = s->c.nz, T = s->c.n_steps, no = s->c.n_obs;
  const double dx = s->c.dx, dy = s->c.dy, dz = s->c.dz, ca = s->ca, cb = s->cb, db = s->db;
  /* s->f[] now serve as the cotangents Eb (0..2) and Hb (3..5); psi arrays as psi cotangents */
  for (int b = 0; b < s->c.n_bins; b++) dl_dq[b] = 0.0;
#define EB(c, i, j, k) s->f[c][IDX(s, i, j, k)]
#define HB(c, i, j, k) s->f[3 + c][IDX(s, i, j, k)]
  for (int n = T - 1; n >= 0; n--) {
    /* sampling transpose: Eb += G^T g^n */
    for (int o = 0; o < no; o++)
      for (int comp = 0; comp < 3; comp++) {
        int i0[3];
        double t[3];
        obs_stencil(s, o, comp, i0, t);
        double g = dl_dw[((size_t)o * 3 + comp) * T + n];
        for (int c = 0; c < 2; c++)
          for (int b = 0; b < 2; b++)
            for (int a = 0; a < 2; a++) {
              double wgt = (a ? t[0] : 1.0 - t[0]) * (b ? t[1] : 1.0 - t[1]) * (c ? t[2] : 1.0 - t[2]);
              EB(comp, i0[0] + a, i0[1] + b, i0[2] + c) += wgt * g;
            }
      }
    /* source transpose: dL/dq_b += -cb * sum Eb_z * v * hat_b(z_s) * W_r * W_z */
    if (source_active(s, n)) {
      double zs = source_zs(s, n), wz[64];
      int m, klo = source_wz(s, zs, wz, 64, &m);
      double acc = 0.0;
      for (int t = 0; t < m; t++) {
        int k = klo + t;
        if (k < 0 || k > nz - 2) continue;
        for (int j = 1; j <= ny - 2; j++)
          for (int i = 1; i <= nx - 2; i++) {
            double w = s->wr[(size_t)j * nx + i];
            if (w != 0.0) acc += EB(2, i, j, k) * w * wz[t];
          }
      }
      for (int b = 0; b < s->c.n_bins; b++) dl_dq[b] += -cb * s->v_src * profile_hat(s, b, zs) * acc;
    }
    /* E-update transpose (scatter), then Eb <- ca Eb on updated nodes */
    for (int k = 1; k <= nz - 2; k++)
      for (int j = 1; j <= ny - 2; j++)
        for (int i = 0; i <= nx - 2; i++) {
          double tb = cb * EB(0, i, j, k);
          double d1 = pml_term_t(s, s->psi_e[0][1], 1, j, 0, i, j, k, tb);
          double d2 = pml_term_t(s, s->psi_e[0][2], 2, k, 0, i, j, k, -tb);
          HB(2, i, j, k) += d1 / dy; HB(2, i, j - 1, k) -= d1 / dy;
          HB(1, i, j, k) += d2 / dz; HB(1, i, j, k - 1) -= d2 / dz;
          EB(0, i, j, k) *= ca;
        }
    for (int k = 1; k <= nz - 2; k++)
      for (int j = 0; j <= ny - 2; j++)
        for (int i = 1; i <= nx - 2; i++) {
          double tb = cb * EB(1, i, j, k);
          double d1 = pml_term_t(s, s->psi_e[1][2], 2, k, 0, i, j, k, tb);
          double d2 = pml_term_t(s, s->psi_e[1][0], 0, i, 0, i, j, k, -tb);
          HB(0, i, j, k) += d1 / dz; HB(0, i, j, k - 1) -= d1 / dz;
          HB(2, i, j, k) += d2 / dx; HB(2, i - 1, j, k) -= d2 / dx;
          EB(1, i, j, k) *= ca;
        }
    for (int k = 0; k <= nz - 2; k++)
      for (int j = 1; j <= ny - 2; j++)
        for (int i = 1; i <= nx - 2; i++) {
          double tb = cb * EB(2, i, j, k);
          double d1 = pml_term_t(s, s->psi_e[2][0], 0, i, 0, i, j, k, tb);
          double d2 = pml_term_t(s, s->psi_e[2][1], 1, j, 0, i, j, k, -tb);
          HB(1, i, j, k) += d1 / dx; HB(1, i - 1, j, k) -= d1 / dx;
          HB(0, i, j, k) += d2 / dy; HB(0, i, j - 1, k) -= d2 / dy;
          EB(2, i, j, k) *= ca;
        }
    /* H-update transpose (scatter); Hb keeps its own value (coefficient 1) */
    for (int k = 0; k < nz - 1; k++)
      for (int j = 0; j < ny - 1; j++)
        for (int i = 0; i < nx; i++) {
          double tb = -db * HB(0, i, j, k);
          double d1 = pml_term_t(s, s->psi_h[0][1], 1, j, 1, i, j, k, tb);
          double d2 = pml_term_t(s, s->psi_h[0][2], 2, k, 1, i, j, k, -tb);
          EB(2, i, j + 1, k) += d1 / dy; EB(2, i, j, k) -= d1 / dy;
          EB(1, i, j, k + 1) += d2 / dz; EB(1, i, j, k) -= d2 / dz;
        }
    for (int k = 0; k < nz - 1; k++)
      for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx - 1; i++) {
          double tb = -db * HB(1, i, j, k);
          double d1 = pml_term_t(s, s->psi_h[1][2], 2, k, 1, i, j, k, tb);
          double d2 = pml_term_t(s, s->psi_h[1][0], 0, i, 1, i, j, k, -tb);
          EB(0, i, j, k + 1) += d1 / dz; EB(0, i, j, k) -= d1 / dz;
          EB(2, i + 1, j, k) += d2 / dx; EB(2, i, j, k) -= d2 / dx;
        }
    for (int k = 0; k < nz; k++)
      for (int j = 0; j < ny - 1; j++)
        for (int i = 0; i < nx - 1; i++) {
          double tb = -db * HB(2, i, j, k);
          double d1 = pml_term_t(s, s->psi_h[2][0], 0, i, 1, i, j, k, tb);
          double d2 = pml_term_t(s, s->psi_h[2][1], 1, j, 1, i, j, k, -tb);
          EB(1, i + 1, j, k) += d1 / dx; EB(1, i, j, k) -= d1 / dx;
          EB(0, i, j + 1, k) += d2 / dy; EB(0, i, j, k) -= d2 / dy;
        }
  }
#undef EB
#undef HB
  orc_destroy(s);
  return 0;
}
