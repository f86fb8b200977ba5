/*
 * chfdtd -- axisymmetric (r, z) solver of libchfdtd.so: the paper's own scheme.
 *
 * What is computed (the paper's Numerical Method section, eqs. fdtd_Er, fdtd_Ez and
 * fdtd_Hphi): with cylindrical symmetry about the shower axis and the Cherenkov polarisation,
 * only E_r, E_z and H_phi survive, and Maxwell's curl equations with conductivity become
 *   eps dE_r/dt + sigma E_r = -dH_phi/dz,
 *   eps dE_z/dt + sigma E_z = (1/r) d(r H_phi)/dr - J_z,
 *   mu dH_phi/dt            = dE_z/dr - dE_r/dz,
 * discretised with second-order central differences and the leapfrog in time.  The source
 * is the moving charge-excess bunch of the Simulation Setup section, centred on the axis.
 * Status codes, chf_medium and the error functions are those of chfdtd.h.
 *
 * Lattice conventions:
 *   nr x nz nodes; node (i, k) at r = i dr, z = k dz; the axis is i = 0, the outer wall
 *   i = nr-1, the z walls k = 0 and k = nz-1.  E_r at (i+1/2, k), E_z at (i, k+1/2), H_phi at
 *   (i+1/2, k+1/2).  E lives at t = n dt, H at (n+1/2) dt.  One step: H update, E update with
 *   -J_z at (n+1/2) dt, boundary, then sampling of E^{n+1}: waveform column n is time (n+1) dt.
 *   The radial term of the E_z update divides the net flux r H_phi by the ring area of the
 *   E_z cell: r_i dr for i >= 1, and on the axis the disc of radius dr/2 (Stokes' theorem,
 *   giving E_z(0) += 4 Cb H_phi(1/2)/dr).
 *   Walls: PEC (tangential E = 0), or first-order Mur on E_z at r = r_max and on E_r at the
 *   two z walls.  The axis needs no boundary condition.
 *
 * Memory and ownership: as for the 3-D plans in chfdtd.h.  Descriptors are copied during
 * chf_rz_plan_create; all device memory (workspace, waveforms, profiles) is the caller's;
 * calls taking a stream are stream-ordered; a plan must not be used from two threads at once.
 */
#ifndef CHFDTD_RZ_H
#define CHFDTD_RZ_H

#include "chfdtd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Lattice: node counts (nr >= 4, nz >= 4), spacings in metres, time step in seconds. */
typedef struct {
  int32_t nr, nz, n_steps, pad0;
  double dr, dz, dt;
} chf_rz_grid;

/* Moving shower source on the axis.  The bunch centre is at z_s = z_entry + beta c0 (t - t_entry)
   for t >= t_entry; Gaussian charge snapshot of width sigma_r across and sigma_z along the
   axis, truncated at cut_sigmas, the radial weights normalised with the E_z ring areas
   (sum 2 pi a_i dr W_i = 1 over the nodes i <= nr-2) and the longitudinal weights over the
   E_z rows of the window; total charge Q(z_s) from the hat-function bins q_bins (HOST array of
   n_bins doubles, coulomb, copied).  J_z = beta c0 Q W_r W_z.  n_bins = 0 disables it. */
typedef struct {
  double z_entry, t_entry, beta, sigma_r, sigma_z, cut_sigmas;
  int32_t n_bins, pad0;
  double z_bin0, dz_bin;
  const double *q_bins;
} chf_rz_source;

/* Detector positions: HOST array rz[n_obs][2] (r, z) in metres, copied.  E_r and E_z are
   interpolated bilinearly on their own sub-lattices; both 4-node stencils must lie inside
   the lattice with r >= dr/2 (else CHF_EDOMAIN). */
typedef struct {
  int32_t n_obs, pad0;
  const double *rz;
} chf_rz_observers;

/* Execution: bc is CHF_BC_PEC or CHF_BC_MUR1 (CHF_BC_CPML: CHF_EUNSUPPORTED).  The sweep tiles
   the lattice into workgroups of waves_per_block waves (1, 2, 4 or 8), each wave owning 64*vx
   consecutive radial nodes (vx = 1, 2, 4 or 8) of z_chunk rows (>= 1); 0 picks the defaults
   (vx 4, 4 waves, 32 rows).  steps_per_launch: 1, or 2 to advance two Yee steps per pass over
   the fields (temporal blocking; needs vx 4 or 8; an odd remainder takes a one-step pass);
   0 = 2 when vx >= 4, else 1.  None of these changes a result bit (with fixed scales).
   storage: CHF_FP32, CHF_BF16 or CHF_FP16 field storage (arithmetic FP32, round to nearest
   even on store; 16-bit types hold scale * value).  scale_e, scale_h: power-of-two storage
   scales of E and H (0 = automatic: H at the power of two nearest the wave impedance times the
   E scale; FP16 puts the Coulomb field of the largest bin charge at one radial width near 2^14).
   dynamic_scaling (FP16 only): every launch instead picks the largest power-of-two scales that
   keep a bound on the magnitudes it writes (twice the previous level's maxima, plus the growth
   one step can add through the curl terms and the source) below 2^14, so fields that grow or
   decay by orders of magnitude keep FP16 precision; the scales then depend on steps_per_launch.
   nan_watch: check waveforms for non-finite values every step (reported by chf_rz_sync). */
typedef struct {
  int32_t bc, vx, waves_per_block, z_chunk, nan_watch, steps_per_launch;
  int32_t storage, dynamic_scaling;
  double scale_e, scale_h;
} chf_rz_exec;

typedef struct chf_rz_plan chf_rz_plan;

/* Validate descriptors and build the FP64 coefficient tables.  Checks: sizes (CHF_EINVAL or
   CHF_ENOMEM), dt below the stability limit of the axisymmetric lattice
   dt <= 2 / (v sqrt(4.85/dr^2 + 4/dz^2)), v = c0/sqrt(eps_r mu_r) (the radial operator's largest
   eigenvalue, which the axis cell raises from 4/dr^2 to about 4.842/dr^2; else CHF_ECFL),
   observer stencils (CHF_EDOMAIN), the tile shape (CHF_EINVAL).  No device call is made. */
chf_status chf_rz_plan_create(const chf_rz_grid *grid, const chf_medium *medium, const chf_rz_source *src,
                              const chf_rz_observers *obs, const chf_rz_exec *ex, chf_rz_plan **out);

void chf_rz_plan_destroy(chf_rz_plan *plan);

/* Bytes of device workspace: E_r, E_z, H_phi in two time levels ([nz][pitch] of the storage
   type each) and the small tables. */
chf_status chf_rz_workspace_bytes(const chf_rz_plan *plan, uint64_t *bytes);

/* Bind caller-owned DEVICE memory (>= the reported size, 256-byte aligned), upload the tables
   with hipMemcpyAsync on `stream` and zero the fields. */
chf_status chf_rz_bind_workspace(chf_rz_plan *plan, void *device_ptr, uint64_t bytes, void *stream);

/* Zero the fields (E^0 = 0, H^{-1/2} = 0) and the step counter. */
chf_status chf_rz_reset(chf_rz_plan *plan, void *stream);

/* Advance n_steps steps.  q_bins_dev: DEVICE array of n_bins doubles overriding the plan's
   profile (NULL = plan's).  waveforms_dev: DEVICE FP64 [n_obs][2][ld_steps] (component 0 = E_r,
   1 = E_z); step s of this call writes column first_column + s. */
chf_status chf_rz_forward(chf_rz_plan *plan, void *stream, const double *q_bins_dev, double *waveforms_dev,
                          int32_t n_steps, int32_t first_column, int32_t ld_steps);

/* chf_rz_forward plus a hipEvent pair on `stream` around every launch of the field sweep;
   waits for `stream` and returns the summed sweep time in *sweep_ms. */
chf_status chf_rz_forward_timed(chf_rz_plan *plan, void *stream, const double *q_bins_dev,
                                double *waveforms_dev, int32_t n_steps, int32_t first_column,
                                int32_t ld_steps, double *sweep_ms);

/* The plan's full run (reset plus n_steps steps, waveforms [n_obs][2][n_steps]) captured once
   into a hipGraph per (waveform pointer, profile pointer) and replayed on later calls. */
chf_status chf_rz_forward_graph(chf_rz_plan *plan, void *stream, const double *q_bins_dev,
                                double *waveforms_dev);

/* Wait for `stream`; CHF_EHIP on a kernel fault, CHF_ENAN if the watchdog fired. */
chf_status chf_rz_sync(chf_rz_plan *plan, void *stream);

/* Copy one component (0 = E_r, 1 = E_z, 2 = H_phi) of the current time level to / from a
   DEVICE FP32 array [nz][nr]. */
chf_status chf_rz_get_field(chf_rz_plan *plan, void *stream, int32_t comp, float *out_dev);
chf_status chf_rz_set_field(chf_rz_plan *plan, void *stream, int32_t comp, const float *in_dev);

typedef struct {
  int32_t vx, waves_per_block, z_chunk, pitch, n_blocks, n_src, steps_per_launch, storage;
  int32_t dynamic_scaling, pad0;
  uint64_t field_bytes, workspace_bytes;
  double bytes_per_cell_update; /* algorithmic HBM bytes per node of one pass (one launch) */
  double scale_e, scale_h;      /* fixed storage scales (the initial ones with dynamic scaling) */
} chf_rz_info;
chf_status chf_rz_get_info(const chf_rz_plan *plan, chf_rz_info *info);

#ifdef __cplusplus
}
#endif
#endif /* CHFDTD_RZ_H */
