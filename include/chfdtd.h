/*
 * chfdtd -- near-field Cherenkov (Askaryan) pulses by 3-D Yee FDTD on MI355X (gfx950).
 *
 * C ABI of the solver library libchfdtd.so.  Plain C types only: sizes, doubles, and
 * host or device pointers (each argument says which).  No exceptions cross this boundary.
 *
 * What is computed (the paper's Numerical Method section and Simulation Setup section):
 *   Maxwell's curl equations with conductivity (Faraday; Ampere with sigma E) on the
 *   staggered Yee lattice, second-order central differences, leapfrog in time, driven by
 *   the current J = v rho of the shower's charge excess: a Gaussian charge snapshot in r
 *   and z whose centre moves along +z and whose total charge follows the longitudinal
 *   profile Q(z) (hat-function bins).  E is recorded at detector positions every step, so
 *   one run yields the pulses of all detectors.  The paper names no boundary; the library
 *   offers PEC walls, first-order Mur on the tangential E of each face, and a
 *   complex-frequency-shifted convolutional PML backed by PEC.
 *
 * Lattice conventions (shared with every routine below):
 *   N nodes per axis; walls on node planes 0 and N-1 (physical length (N-1) delta).
 *   Ex at (i+1/2, j, k), Ey at (i, j+1/2, k), Ez at (i, j, k+1/2),
 *   Hx at (i, j+1/2, k+1/2), Hy at (i+1/2, j, k+1/2), Hz at (i+1/2, j+1/2, k).
 *   E lives at t = n dt and H at (n+1/2) dt.  One step: H update, E update with -J at
 *   (n+1/2) dt, boundary, then sampling of E^{n+1}: waveform index n is time (n+1) dt.
 *   Positions are metres with node (0,0,0) at the origin.
 *
 * Memory and ownership:
 *   - Descriptor structs and the host arrays they point to are read and copied during
 *     chf_plan_create; the caller may free them afterwards.
 *   - All device memory is the caller's: the plan reports how many bytes of workspace it
 *     needs (chf_plan_workspace_bytes) and works inside the buffer bound with
 *     chf_plan_bind_workspace.  Output buffers are the caller's as well.  The library never
 *     allocates or frees device memory; it holds one static array of CHF_SCRATCH_BYTES per GPU
 *     (reserved when the code object loads) that only chf_forward_scratch uses.
 *   - Calls that take a stream are stream-ordered and return after enqueueing.  Kernel
 *     faults surface as CHF_EHIP and the non-finite watchdog as CHF_ENAN from
 *     chf_plan_sync.  A plan must not be used from two threads at once.
 *
 * Errors: every entry point returns a chf_status; chf_last_error() gives a thread-local
 * message for the last failure on the calling thread.
 */
#ifndef CHFDTD_H
#define CHFDTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHF_ABI_VERSION 3

typedef enum {
  CHF_OK = 0,
  CHF_EINVAL = -1,       /* malformed descriptor or argument */
  CHF_ECFL = -2,         /* dt above the Courant limit of the medium */
  CHF_EDOMAIN = -3,      /* observer stencil or source patch outside the usable interior */
  CHF_ENOMEM = -4,       /* sizes overflow, or the bound workspace is too small */
  CHF_EHIP = -5,         /* a HIP runtime call or kernel launch failed */
  CHF_ENAN = -6,         /* the non-finite watchdog fired */
  CHF_EUNSUPPORTED = -7, /* valid request that this build does not implement */
  CHF_ESTATE = -8        /* call out of order (e.g. no workspace bound) */
} chf_status;

/* Field storage (arithmetic is FP32 in every case; the reduced types round to nearest even).
   CHF_BF16X: BF16 with an 8-bit mantissa extension -- the 24 leading bits of the FP32 value (8
   exponent bits, 15 fraction bits) in 3 bytes, 36 B per node against FP32's 48; FP32's exponent
   range, so no scale is needed (scale_e/scale_h as for BF16).  The 3-D path only (the (r, z)
   scheme takes the other three). */
typedef enum { CHF_FP32 = 0, CHF_BF16 = 1, CHF_FP16 = 2, CHF_BF16X = 3 } chf_storage;
typedef enum { CHF_BC_PEC = 0, CHF_BC_MUR1 = 1, CHF_BC_CPML = 2 } chf_bc;
/* CHF_KERNEL_FUSED_PREFETCH: the fused sweep whose interior tiles issue each plane's row loads one
   plane ahead (the loads of plane k+1 are in flight while plane k is computed), at the price of
   more registers per wave (3 waves per SIMD instead of 4); waves_per_block 4, 7, 8 or 11 (11
   rows: one 12-wave workgroup fills a compute unit).  Rows of 257-512 nodes are split across two
   waves of four nodes per lane, which exchange the x neighbours at their seam through LDS; there
   waves_per_block is the rows per tile, 4 or 5 (default 5: 12 waves).  With 4 or 7 rows of at
   most 256 nodes the boundary tiles load a plane ahead too.  A batch takes its members' kind.
   Same bits.
   CHF_KERNEL_FUSED2: two Yee steps per pass over the fields (temporal blocking of the Numerical
   Method section's leapfrog): each launch reads E^n, H^{n-1/2} and writes E^{n+2}, H^{n+3/2},
   keeping E^{n+1}, H^{n+1/2} on chip (its observer samples are taken inside the pass), so a
   cell-update moves about half the bytes.  waves_per_block is then the rows per interior tile (4,
   7 or 8; default 8) and z_chunk the planes per tile (default 32); a workgroup also computes two
   rows below and one above its tile, and tiles near walls and y/z layers take 4 rows.  Rows of at
   most 256 nodes, PEC and CPML walls (else CHF_EUNSUPPORTED), CPML of at most 16 cells; a step
   range of odd length ends with one single step of the fused sweep (default tile).  The results
   equal the one-step sweeps' bit for bit. */
typedef enum {
  CHF_KERNEL_AUTO = 0, CHF_KERNEL_SPLIT = 1, CHF_KERNEL_FUSED = 2, CHF_KERNEL_FUSED_PREFETCH = 3,
  CHF_KERNEL_FUSED2 = 4
} chf_kernel;

/* Lattice: node counts (>= 3 each; the fused sweep needs nx <= 512), spacings in metres,
   time step in seconds, number of steps. */
typedef struct {
  int32_t nx, ny, nz, n_steps;
  double dx, dy, dz, dt;
} chf_grid;

/* Uniform medium (Numerical Method section: the curl equations with permittivity, permeability
   and the conduction current sigma E in Ampere's law): relative permittivity and permeability,
   conductivity in S/m, the sigma E term integrated semi-implicitly.  The paper's medium is ice,
   n = 1.78, lossless. */
typedef struct {
  double eps_r, mu_r, sigma;
} chf_medium;

/* Boundary.  For CHF_BC_CPML: npml cells per face, polynomial order poly_m, and the grading
   sigma = sigma_scale * 0.8 (m+1) / (eta0 delta sqrt(eps_r mu_r)) * (d/L)^m,
   kappa = 1 + (kappa_max - 1)(d/L)^m, alpha = alpha_max (1 - d/L) (S/m), with d the depth into
   the layer.  Ignored fields may be zero for the other kinds. */
typedef struct {
  int32_t kind, npml;
  double poly_m, sigma_scale, kappa_max, alpha_max;
} chf_boundary;

/* Moving shower source (Simulation Setup section).  The bunch centre is on the line
   (x_axis, y_axis) and at z_s = z_entry + beta c0 (t - t_entry) for t >= t_entry.  Charge
   snapshot: Gaussian of width sigma_r across and sigma_z along the axis, each truncated at
   cut_sigmas and normalised on the Ez lattice; total charge Q(z_s) = sum_b q_b hat((z_s -
   z_bin0)/dz_bin - b) (coulomb; the charge excess is negative).  q_bins is a HOST array of
   n_bins doubles, copied.  J_z = beta c0 * Q * W_r * W_z enters the Ez update.
   n_bins = 0 disables the source. */
typedef struct {
  double x_axis, y_axis, z_entry, t_entry, beta, sigma_r, sigma_z, cut_sigmas;
  int32_t n_bins, pad0;
  double z_bin0, dz_bin;
  const double *q_bins;
} chf_source;

/* Detector positions (Simulation Setup section: detectors at chosen positions record E as the
   run evolves, so one run gives the pulses of all of them): HOST array xyz[n_obs][3] in metres,
   copied.  Each component is interpolated trilinearly on its own staggered sub-lattice; the
   8-node stencil must lie at least max(1, npml) cells inside every wall. */
typedef struct {
  int32_t n_obs, pad0;
  const double *xyz;
} chf_observers;

/* Execution choices.  storage: field storage type (arithmetic is always FP32; waveforms are
   accumulated in FP64).  scale_e / scale_h: power-of-two storage scales (0 = automatic).
   kernel: split E/H sweeps or the fused single sweep.  waves_per_block is the number of y
   rows per tile (4, 7, 8, 11 or 15; 4 or 7 for rows wider than 256 nodes, 4 or 5 for the
   prefetching sweep there; a fused workgroup has one more wave for the row below the tile) and z_chunk the planes per tile (0 = defaults:
   7 rows, 12 planes); rows_per_wave must be 0 or 1.  None of these changes
   a result bit.  nan_watch: check waveforms for non-finite values every step.
   dynamic_scaling (FP16 storage with the fused, prefetching or two-step sweeps, PEC or CPML
   walls, single plans; else CHF_EUNSUPPORTED): every launch picks the storage scale of the
   level it writes.  Both fields of a level carry an extra factor 2^e on top of scale_e and
   scale_h (their ratio fixed, so the coefficient tables hold); the launch reading a level with
   maxima M_E, M_H (stored units) bounds what its n steps (1 or 2) can reach,
   B_E = 2 M_E + 2 n (g_E M_H + S), B_H = 2 M_H + 2 n g_H B_E (g_E, g_H the largest per-step gains
   of the curl terms, S the source's largest E_z increment, the factors 2 covering the CPML
   terms), and stores the new level with the largest power of two keeping max(B_E, B_H) below
   2^14.  Scales and maxima live in device memory, so graph capture works; changing by powers of
   two, they leave every mantissa as a static run with the same scales would.  The one-step
   sweeps give equal bits among themselves; the two-step sweep picks its scales per launch of
   two steps. */
typedef struct {
  int32_t storage, kernel;
  int32_t rows_per_wave, waves_per_block, z_chunk, nan_watch;
  double scale_e, scale_h;
  int32_t dynamic_scaling, pad0;
} chf_exec;

typedef struct chf_plan chf_plan;

/* Validate descriptors and build all host-side tables for the leapfrog of the Numerical Method
   section (the discretised curl equations on the staggered lattice, the moving source of the
   Simulation Setup section, the detector stencils).  Checks: node counts >= 3 and the
   64-bit size of the workspace; dt below the Courant limit dt <= 1/(v sqrt(sum 1/d^2)) with
   v = c0/sqrt(eps_r mu_r) (else CHF_ECFL); observer stencils inside the interior and the
   source axis inside the x-y extent (else CHF_EDOMAIN); supported kernel/storage
   combination (else CHF_EUNSUPPORTED).  On success *out owns the plan (free with
   chf_plan_destroy).  No device call is made. */
chf_status chf_plan_create(const chf_grid *grid, const chf_medium *medium, const chf_boundary *bnd,
                           const chf_source *src, const chf_observers *obs, const chf_exec *ex,
                           chf_plan **out);

void chf_plan_destroy(chf_plan *plan);

/* Bytes of device workspace the plan needs (fields in two time levels, CPML state, tables). */
chf_status chf_plan_workspace_bytes(const chf_plan *plan, uint64_t *bytes);

/* Bind caller-owned DEVICE memory (>= the reported size, 256-byte aligned) and upload the
   plan's tables into it with hipMemcpyAsync on `stream` (a hipStream_t, NULL = default). */
chf_status chf_plan_bind_workspace(chf_plan *plan, void *device_ptr, uint64_t bytes, void *stream);

/* Zero the fields and the CPML state (initial condition E^0 = 0, H^{-1/2} = 0). */
chf_status chf_plan_reset(chf_plan *plan, void *stream);

/* Advance `n_steps` steps from the current state: per step the H update from the curl of E and
   the E update from the curl of H minus the source current (the Numerical Method section's
   leapfrog with central differences in space and time, here on the 3-D lattice), the boundary,
   and the sampling of E at the detectors.  q_bins_dev: DEVICE array of n_bins doubles
   overriding the plan's profile (NULL = plan's).  waveforms_dev: DEVICE FP64 array
   [n_obs][3][ld_steps]; step s of this call writes column (first_column + s).  A full run from
   zero fields is chf_plan_reset followed by chf_forward(plan, stream, NULL, w, T, 0, T). */
chf_status chf_forward(chf_plan *plan, void *stream, const double *q_bins_dev, double *waveforms_dev,
                       int32_t n_steps, int32_t first_column, int32_t ld_steps);

/* Instrumented chf_forward for measurement: identical work, plus a hipEvent pair on `stream`
   around the launch of the fused interior sweep in every step.  Waits for `stream` before
   returning; *fused_ms receives the summed duration of those launches (0 when the plan has no
   fused interior tiles). */
chf_status chf_forward_timed(chf_plan *plan, void *stream, const double *q_bins_dev, double *waveforms_dev,
                             int32_t n_steps, int32_t first_column, int32_t ld_steps, double *fused_ms);

/* Same as chf_forward over the plan's n_steps, captured once into a hipGraph per
   (waveform pointer, profile pointer) and replayed on later calls. */
chf_status chf_forward_graph(chf_plan *plan, void *stream, const double *q_bins_dev,
                             double *waveforms_dev);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
   loops, harnesses that forbid hipMalloc): chf_forward_scratch runs the plan's full forward pass
   from zero fields -- exactly the launches of chf_plan_reset + chf_forward over n_steps, with the
   boundary sweep in order on `stream` -- inside a static device array of CHF_SCRATCH_BYTES that
   the library holds on every GPU it runs on until the process ends, instead of a caller-bound
   workspace.  No device memory is allocated or freed and no stream or event is created; the
   plan's tables are copied into the array (stream-ordered) at every call.
   q_bins_dev: DEVICE profile (NULL = plan's); waveforms_dev: DEVICE FP64 [n_obs][3][n_steps]
   (may be NULL only without observers).  The plan needs no bound workspace; if it has one, that
   workspace and the plan's step state are left untouched.  Plans whose workspace exceeds
   CHF_SCRATCH_BYTES (chf_plan_workspace_bytes) get CHF_ENOMEM.  All calls on one GPU share its
   array, which keeps the last call's contents (the call zeroes fields and CPML state itself):
   calls that overlap on one GPU (other streams, other threads) race and must be serialised by
   the caller.  chf_scratch_bytes returns the array's size. */
#define CHF_SCRATCH_BYTES (64ull << 20)
chf_status chf_forward_scratch(chf_plan *plan, void *stream, const double *q_bins_dev, double *waveforms_dev);
uint64_t chf_scratch_bytes(void);

/* Discrete adjoint (not in the paper: the reverse-mode derivative of the Numerical Method
   section's leapfrog with respect to the Simulation Setup section's longitudinal profile bins):
   given dL/dw (DEVICE FP64 [n_obs][3][n_steps]) returns dL/dq (DEVICE FP64
   [n_bins]) for the plan's full run, by the exact transpose of the forward recurrence run
   backward in time.  PEC and CPML only (CHF_EUNSUPPORTED for Mur).  The forward field state
   is destroyed (the workspace holds the adjoint state). */
chf_status chf_adjoint(chf_plan *plan, void *stream, const double *dl_dw_dev, double *dl_dq_dev);

/* The same adjoint in pieces, for checkpointed schedules: chf_adjoint_begin zeroes the adjoint
   state and dL/dq; chf_adjoint_steps then applies the transposed steps t_hi-1 down to t_lo
   (0 <= t_lo <= t_hi <= n_steps), accumulating into dL/dq.  Successive calls must continue
   where the previous one stopped (t_hi of a call = t_lo of the previous; the first call after
   begin has t_hi = n_steps), else CHF_ESTATE.  begin + steps(0, n_steps) = chf_adjoint. */
chf_status chf_adjoint_begin(chf_plan *plan, void *stream, double *dl_dq_dev);
chf_status chf_adjoint_steps(chf_plan *plan, void *stream, const double *dl_dw_dev, double *dl_dq_dev,
                             int32_t t_lo, int32_t t_hi);

/* chf_adjoint_steps that also accumulates the cotangent of the permittivity at every E node: the
   sensitivity of L to a relative-permittivity map eps_r(x), evaluated at the plan's uniform
   medium (Ampere's law with conductivity of the Numerical Method section, with eps per node).
   Each node's Ca and Cb depend on its eps_r only, and dE^{n+1}/deps_r =
   -(E^{n+1} - E^n)/(eps_r (1 + sigma dt/(2 eps))) whatever the curl, CPML and source terms were
   (the CPML grading is held fixed), so step n adds -Eb^{n+1} (E^{n+1} - E^n)/(eps_r (1 + ...))
   with Eb^{n+1} the adjoint state at that point of the reverse step.  This needs the forward E
   levels in reverse order, which a checkpointed schedule recomputes segment by segment.
   e_levels_dev: DEVICE FP32 [t_hi - t_lo + 1][3][nz][ny][nx], level m = E^{t_lo + m} of the
   forward run (components Ex, Ey, Ez, each dense as chf_plan_get_field writes it; E^t is the
   field after t steps).  dl_deps_dev: DEVICE FP64 [3][nz][ny][nx], dL/deps_r per node,
   ACCUMULATED (zero it before the first call); nodes tangential to a wall get nothing.  Same
   step-range rules, storage (FP32) and boundaries (PEC, CPML) as chf_adjoint_steps; dL/dq is
   accumulated as there, bit for bit.  For the uniform medium with PEC walls, dL/deps_r of the
   plan is the sum of the map. */
chf_status chf_adjoint_steps_eps(chf_plan *plan, void *stream, const double *dl_dw_dev, double *dl_dq_dev,
                                 int32_t t_lo, int32_t t_hi, const float *e_levels_dev, double *dl_deps_dev);

/* Gradients with respect to the source's non-linear parameters (the radial width sigma_r and the
   trajectory offset z_entry of the Simulation Setup section's moving charge snapshot), with the
   profile gradient, from one reverse sweep: J_z enters the E update linearly, so
   dL/dtheta = sum_n <Eb_z, -Cb dJ_z^n/dtheta> needs the adjoint state only, not the forward
   states.  q_bins_dev: DEVICE profile the forward run used (NULL = plan's); dl_dq_dev: DEVICE
   [n_bins]; dl_dtheta_dev: DEVICE FP64 [2] = (dL/dsigma_r, dL/dz_entry), per metre.  The
   derivative holds the source's discrete support (nodes inside the cut disc, rows of the z
   window) fixed, i.e. it is exact wherever that support does not change.  PEC and CPML only;
   CHF_EINVAL without a source.  The forward field state is destroyed. */
chf_status chf_adjoint_source_params(chf_plan *plan, void *stream, const double *dl_dw_dev,
                                     const double *q_bins_dev, double *dl_dq_dev, double *dl_dtheta_dev);

/* The checkpointed reverse sweep in one call: the schedule of chf_adjoint_begin/steps with
   recomputation, driven by the library.  `fwd` is a second plan made from the same descriptors
   with a workspace of its own (the plan's grid, step count, storage and boundary, else
   CHF_EINVAL); it runs the forward pass from zero fields with q_bins_dev (DEVICE, NULL = its
   own profile), keeping a snapshot at the start of every `every`-step segment in snapshots_dev
   (DEVICE, caller-owned, at least ceil(n_steps / every) * chf_plan_state_bytes(fwd) bytes, else
   CHF_ENOMEM).  Then, segments last to first, it restores the segment's snapshot, recomputes the
   segment and applies the segment's transposed steps on `plan`.  dl_dw_dev / dl_dq_dev as
   chf_adjoint (dL/dq is zeroed first and comes out bit for bit as chf_adjoint's).  With
   dl_deps_dev (DEVICE FP64 [3][nz][ny][nx], accumulated) the recomputation keeps the segment's E
   levels in e_levels_dev (DEVICE FP32 [every + 1][3][nz][ny][nx], caller-owned) and the reverse
   steps add the permittivity cotangent as chf_adjoint_steps_eps does; both pointers are NULL or
   both set.  fwd's field state and plan's are destroyed; PEC and CPML only. */
chf_status chf_adjoint_checkpointed(chf_plan *plan, chf_plan *fwd, void *stream, const double *q_bins_dev,
                                    const double *dl_dw_dev, double *dl_dq_dev, int32_t every, void *snapshots_dev,
                                    uint64_t snapshots_bytes, float *e_levels_dev, double *dl_deps_dev);

/* Forward-state snapshots (checkpoints, resume).  A snapshot is the plan's whole field and
   CPML state -- both time levels of E and H, every psi array and the 256-byte block of
   dynamic-scaling words (each level's scale exponent and the field maxima) -- as a DEVICE byte
   image of
   chf_plan_state_bytes bytes owned by the caller.  save copies it out (stream-ordered) and
   reports the step it belongs to; load copies it back and sets the step (and with it the
   source clock and the current time level).  Restarting from a snapshot reproduces the run
   bit for bit. */
chf_status chf_plan_state_bytes(const chf_plan *plan, uint64_t *bytes);
chf_status chf_plan_save_state(chf_plan *plan, void *stream, void *dst_dev, int32_t *step);
chf_status chf_plan_load_state(chf_plan *plan, void *stream, const void *src_dev, int32_t step);

/* Wait for `stream` and report a kernel fault (CHF_EHIP) or the watchdog (CHF_ENAN). */
chf_status chf_plan_sync(chf_plan *plan, void *stream);

/* Copy one field component (0..5 = Ex,Ey,Ez,Hx,Hy,Hz) of the current time level into a DEVICE
   FP32 array [nz][ny][nx] (unscaled, physical units; under dynamic scaling with the level's
   present factor). */
chf_status chf_plan_get_field(chf_plan *plan, void *stream, int32_t comp, float *out_dev);

/* Overwrite one field component of the current time level from a DEVICE FP32 array
   [nz][ny][nx] (physical units).  Under dynamic scaling the values are stored with the level's
   present factor (values beyond the FP16 range at that factor become infinite) and the level's
   maxima are recomputed. */
chf_status chf_plan_set_field(chf_plan *plan, void *stream, int32_t comp, const float *in_dev);

/* Introspection: chosen kernel, storage scales, fused-sweep shape, pitch. */
typedef struct {
  int32_t kernel, storage, vx, rows_per_wave, waves_per_block, z_chunk, pitch, n_blocks;
  double scale_e, scale_h;
  uint64_t field_bytes, psi_bytes, workspace_bytes;
  double bytes_per_cell_update; /* algorithmic HBM bytes of one cell-update (whole grid) */
  uint64_t fused_cells;         /* nodes covered by one launch of the fused interior sweep */
  double fused_bytes_per_cell;  /* its algorithmic HBM bytes per node (fields + x-layer psi) */
  int32_t steps_per_launch;     /* Yee steps per interior launch: 1, or 2 (CHF_KERNEL_FUSED2) */
  int32_t waves_per_row;        /* waves across one row in the two-step sweep (1 or 2) */
  /* for CHF_KERNEL_FUSED2, fused_cells / fused_bytes_per_cell describe the two-step interior
     launch: its nodes, and the one-step algorithmic bytes per node of both steps it advances
     (so bytes / launch time is the single-step-equivalent rate); pass_bytes_per_cell is what
     the pass itself must move per node (12 values once, x-layer psi once) */
  double pass_bytes_per_cell;
  int32_t dynamic_scaling, pad0; /* 1 when the storage scale is picked per launch */
} chf_plan_info;
chf_status chf_plan_get_info(const chf_plan *plan, chf_plan_info *info);

/* Batched execution (many showers of uneven grids advanced together).  Plans must have their
   workspaces bound and share storage, waves_per_block and n_steps.  Each step issues one
   launch per phase for the whole batch (fused interior sweep over every plan's interior tiles,
   boundary sweeps over every plan's boundary tiles, source, observer gather), and the full run
   from zero fields is captured once into one hipGraph, replayed by chf_batch_run.  The batch
   needs its own small DEVICE workspace (plan descriptors, tile tables), caller-owned like the
   plans'.  waveforms_dev[i] is plan i's DEVICE FP64 output [n_obs_i][3][n_steps]; the graph is
   re-captured when the set of output pointers changes.  Results equal those of each plan run
   alone, bit for bit. */
typedef struct chf_batch chf_batch;
chf_status chf_batch_create(int32_t n, chf_plan *const *plans, chf_batch **out);
chf_status chf_batch_workspace_bytes(const chf_batch *batch, uint64_t *bytes);
chf_status chf_batch_bind_workspace(chf_batch *batch, void *device_ptr, uint64_t bytes, void *stream);
chf_status chf_batch_run(chf_batch *batch, void *stream, double *const *waveforms_dev);

/* The same run as chf_batch_run in ONE persistent cooperative kernel launch (batching of many
   showers as one launch; the Parallelization with GPU section's host loop over kernels moved onto
   the device): every workgroup that fits the GPU at once loops over the Yee steps, taking tiles of
   every member from one combined table (interior and boundary tiles alike, through the general
   fused sweep), then the workgroups meet at a grid barrier, inject every member's source, meet
   again and gather the observers.  Same waveforms and fields, bit for bit, as chf_batch_run.
   FP32 members with PEC or CPML walls whose boundary tiles fit the general fused sweep (rows of at
   most 256 nodes, at most 11 rows per tile), else CHF_EUNSUPPORTED; a launch the device cannot
   hold at once fails with CHF_EHIP.  Allocates nothing; the captured graph of chf_batch_run is
   kept unless the waveform pointers change. */
chf_status chf_batch_run_persistent(chf_batch *batch, void *stream, double *const *waveforms_dev);
void chf_batch_destroy(chf_batch *batch);

/* Measurement aid (not part of the solver): copies `bytes` (a multiple of 16) from src_dev to
   dst_dev (DEVICE, 16-byte aligned, not overlapping) with a streaming kernel -- each lane keeps
   loads_in_flight (1, 2, 4 or 8) 16-byte loads in flight and writes them with non-temporal
   stores; `blocks` workgroups of 256 lanes stride over the buffer.  Stream-ordered.  The HBM
   bandwidth such a copy reaches is the practical ceiling the solver's sweeps are read against. */
chf_status chf_stream_copy(void *dst_dev, const void *src_dev, uint64_t bytes, int32_t loads_in_flight,
                           int32_t blocks, void *stream);

const char *chf_status_str(chf_status s);
const char *chf_last_error(void);
int32_t chf_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CHFDTD_H */
