/*
 * FP64 CPU oracle for the 3-D Yee leapfrog driven by a moving shower current.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the HIP path.
 *
 * What it computes (the paper's Numerical Method section):
 *   - Maxwell's curl equations with conductivity (Faraday and Ampere with
 *     sigma*E), discretised on the staggered Yee lattice with second-order
 *     central differences in space and leapfrog in time.
 *   - The source is the charge-excess current of the shower: a Gaussian
 *     charge snapshot in r and z (the snapshot density of the Simulation
 *     Setup section) whose centre moves along +z; its total charge Q(z_s)
 *     follows the longitudinal profile, interpolated from bins with hat
 *     functions.  Only J_z is injected.
 *   - The electric field is recorded at detector positions every step.
 * Boundaries (the paper names none): PEC walls, first-order Mur on the
 * tangential E of each face, or a CFS convolutional PML backed by PEC.
 *
 * Conventions: N nodes per axis, walls on node planes 0 and N-1; Ex(i+1/2,j,k),
 * Ey(i,j+1/2,k), Ez(i,j,k+1/2), Hx(i,j+1/2,k+1/2), Hy(i+1/2,j,k+1/2),
 * Hz(i+1/2,j+1/2,k); every component array is nx*ny*nz doubles, x fastest.
 * E lives at t = n dt, H at (n+1/2) dt.  One step: H update, E update (with
 * -J at (n+1/2) dt), boundary, then sampling of E^{n+1}; waveform index n
 * therefore belongs to time (n+1) dt.
 */
#ifndef YEE_ORACLE_H
#define YEE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_PEC = 0, ORC_BC_MUR1 = 1, ORC_BC_CPML = 2 };

typedef struct {
  int32_t nx, ny, nz, n_steps;
  double dx, dy, dz, dt;
  double eps_r, mu_r, sigma;
  int32_t bc, npml;
  /* CPML grading: sigma = sigma_scale*sigma_opt*(d/L)^m, kappa = 1+(kappa_max-1)(d/L)^m,
     alpha = alpha_max*(1-d/L); sigma_opt = 0.8(m+1)/(eta0*delta*sqrt(eps_r*mu_r)). */
  double pml_m, pml_sigma_scale, pml_kappa_max, pml_alpha_max;
  /* moving source */
  int32_t src_on, n_bins;
  double x_axis, y_axis, z_entry, t_entry, beta, sigma_r, sigma_z, cut_sigmas;
  double z_bin0, dz_bin;
  const double *q_bins; /* [n_bins] coulomb, copied at create */
  int32_t n_obs, pad0;
  const double *obs_xyz; /* [n_obs][3] metre, copied at create */
} orc_cfg;

typedef struct orc_state orc_state;

/* Returns NULL on invalid configuration (message via orc_last_error). */
orc_state *orc_create(const orc_cfg *cfg);
void orc_destroy(orc_state *s);
const char *orc_last_error(void);

/* Direct access to a field array: comp 0..5 = Ex,Ey,Ez,Hx,Hy,Hz. */
double *orc_field(orc_state *s, int comp);
int32_t orc_step_index(const orc_state *s);

/* Half steps, exposed so tests can pin each operator on its own. */
void orc_update_h(orc_state *s);
void orc_update_e(orc_state *s); /* includes -J at (n+1/2)dt, boundary, n += 1 */
/* Sample E at the observers into w[n_obs*3] (component fastest). */
void orc_sample(const orc_state *s, double *w);
/* One full step; writes the step's samples into w (may be NULL). */
void orc_step(orc_state *s, double *w);
/* J_z at half step n+1/2 on the whole Ez lattice (nx*ny*nz, zero elsewhere). */
void orc_source_current(const orc_state *s, int32_t n, double *jz);

/* Relative permittivity per E node, eps_r_map [3][nz][ny][nx] (component-major, each
   component on its own staggered lattice), replacing the uniform eps_r in the E update only;
   NULL restores the uniform medium.  0 on success, -1 on a non-positive entry. */
int orc_set_eps_map(orc_state *s, const double *eps_r_map);

/* Full forward run from zero fields: waveforms [n_obs][3][n_steps]. */
int orc_run(const orc_cfg *cfg, double *waveforms);
/* The same with a permittivity map (NULL = uniform). */
int orc_run_eps(const orc_cfg *cfg, const double *eps_r_map, double *waveforms);
/* Discrete-adjoint gradient of L with respect to the profile bins, given
   dL/dw [n_obs][3][n_steps]; PEC and CPML boundaries only. */
int orc_adjoint(const orc_cfg *cfg, const double *dl_dw, double *dl_dq);

/* Physical constants used throughout (CODATA 2018 mu0). */
double orc_c0(void);
double orc_mu0(void);
double orc_eps0(void);
/* OpenMP threads the loops above run on (1 without OpenMP). */
int orc_threads(void);
/* Threads for the following calls (n > 0). */
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
