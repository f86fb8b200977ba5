/*
 * chfdtd -- spectral post-processing of recorded pulses (libchfdtd.so).
 *
 * What is computed (the paper's Results section: E_omega spectra at fixed distance R and angle
 * theta, their change with R and their angular distribution; Comparison section: the 1-D
 * far-field formula, eq. 1d_appro):
 *   - the spectrum of sampled waveforms, E(omega) = int E(t) exp(+i omega t) dt, evaluated as
 *     sum_n E(t0 + n dt) exp(i omega (t0 + n dt)) dt in FP64 (the sign convention of the paper's
 *     Green's-function integral, eq. GreenMethod);
 *   - its component along theta-hat, the polarisation direction n_perp of eq. 1d_appro, for
 *     observers seen from the axis point z_origin (the shower maximum in the paper's detector
 *     coordinates), and its modulus;
 *   - the far-field (Fraunhofer, eq. fraun_appr) spectrum of the moving charge profile
 *     Q(z) = sum_b q_b hat((z - z_bin0)/dz_bin - b) whose bunch passes z at
 *     t = t_entry + (z - z_entry)/v:
 *       E_theta = -i omega sin(theta) mu0/(4 pi R) e^{ikR} e^{i omega t_off} e^{ik cos(theta) z_origin} F(p),
 *       F(p) = int Q e^{ipz} dz = dz_bin sinc^2(p dz_bin/2) sum_b q_b e^{i p z_b},
 *       p = omega/v - k cos(theta), k = n omega/c0, t_off = t_entry - z_entry/v
 *     (eq. 1d_appro for v = c0, with e N_e(z) = Q(z)).
 * Status codes and chf_last_error are those of chfdtd.h.  Device arrays are the caller's; the
 * calls are stream-ordered and allocate nothing.
 */
#ifndef CHFDTD_SPECTRAL_H
#define CHFDTD_SPECTRAL_H

#include "chfdtd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Spectra of n_series real waveforms.  w_dev: DEVICE FP64 [n_series][ld] (sample n of series s
   at w_dev[s*ld + n], time t0 + n dt; n < n_t <= ld).  omega_dev: DEVICE FP64 [n_freq] angular
   frequencies (rad/s).  spec_dev: DEVICE FP64 [n_series][n_freq][2] (re, im), V s/m for fields
   in V/m.  n_series <= 65535; CHF_EINVAL on bad sizes or NULL pointers. */
chf_status chf_spectrum(void *stream, const double *w_dev, int32_t n_series, int32_t n_t, int32_t ld,
                        double dt, double t0, const double *omega_dev, int32_t n_freq, double *spec_dev);

/* Per-observer projection of component spectra: out[o][f] = sum_c weights[o][c] spec[o][c][f]
   (complex), with spec_dev DEVICE [n_obs][n_comp][n_freq][2] as written by chf_spectrum for the
   series (o, c) and weights_dev DEVICE [n_obs][n_comp].  out_dev: DEVICE [n_obs][n_freq][2] and
   mag_dev: DEVICE [n_obs][n_freq] (modulus); either may be NULL. */
chf_status chf_spectrum_project(void *stream, const double *spec_dev, int32_t n_obs, int32_t n_comp,
                                int32_t n_freq, const double *weights_dev, double *out_dev, double *mag_dev);

/* Observer geometry on the HOST (no device call): R, theta of each observer seen from the axis
   point, and the theta-hat weights.  (r, z) observers: rz[n][2] -> r_theta[n][2], weights[n][2]
   on (E_r, E_z) = (cos theta, -sin theta).  3-D observers: xyz[n][3] with the axis at
   (x_axis, y_axis) -> r_theta[n][2], weights[n][3] on (E_x, E_y, E_z) =
   (cos theta cos phi, cos theta sin phi, -sin theta).  Observers on the origin: CHF_EDOMAIN. */
chf_status chf_geometry_rz(int32_t n_obs, const double *rz, double z_origin, double *r_theta, double *weights);
chf_status chf_geometry_xyz(int32_t n_obs, const double *xyz, double x_axis, double y_axis, double z_origin,
                            double *r_theta, double *weights);

/* Far-field formula parameters: refractive index, bunch speed beta (v = beta c0), the source
   clock (z_entry, t_entry) and the observation origin on the axis. */
typedef struct {
  double n_index, beta, z_entry, t_entry, z_origin;
} chf_far_field_params;

/* E_theta(omega) of the far-field formula for n_obs (R, theta) pairs.  q_dev: DEVICE FP64
   [n_bins] profile bins (coulomb); r_theta_dev: DEVICE [n_obs][2]; omega_dev: DEVICE [n_freq];
   out_dev: DEVICE [n_obs][n_freq][2]. */
chf_status chf_far_field_1d(void *stream, const double *q_dev, int32_t n_bins, double z_bin0, double dz_bin,
                            const double *r_theta_dev, int32_t n_obs, const chf_far_field_params *prm,
                            const double *omega_dev, int32_t n_freq, double *out_dev);

#ifdef __cplusplus
}
#endif
#endif /* CHFDTD_SPECTRAL_H */
