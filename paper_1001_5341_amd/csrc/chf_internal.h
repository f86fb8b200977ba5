// Internal types shared by the host plan code and the kernel launchers of libchfdtd.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/chfdtd.h"

namespace chf {

constexpr int kMaxVX = 8;        // cells per lane along x in the fused sweep (nx <= 64*8)
constexpr int kMaxFusedLayer = 64;  // 2*npml the fused sweep handles (x-slab psi, one per lane)
constexpr int kMaxGeneralVX = 4;    // widest rows (64*VX nodes) of the general fused sweep
constexpr int kMaxGeneralW = 11;     // and most rows per workgroup
constexpr int kMaxObsPerPlan = 4096;
constexpr int kMaxWz = 64;       // longitudinal source support in cells
constexpr int kMaxStep2Layer = 32;  // 2*npml the two-step sweep handles (x-slab psi in LDS)
constexpr int kStep2BoundaryRows = 4;  // rows per boundary tile of the two-step sweep

// Per-axis coefficient tables, one entry per node index along the axis.  "e" entries belong
// to the E-update derivative (backward difference, integer position), "h" entries to the
// H-update derivative (forward difference, half position).
struct AxisTab {
  const float *ce, *ch;      // main-term coefficient  Cb/(delta kappa) resp. Db/(delta kappa), scaled
  const float *ae, *be;      // CPML psi recursion at integer positions (a prescaled)
  const float *ah, *bh;      // CPML psi recursion at half positions
  const int *se, *sh;        // slab slot (0..2*npml-1) or -1 outside the layer
  // adjoint (physical units): 1/(delta kappa) and a/delta at integer and half positions
  const float *ike, *ade, *ikh, *adh;
};

// Everything a kernel needs, passed by value.
struct Dev {
  int nx, ny, nz, pitch, npml, np2;
  // origin of the one-step tile grid: tile ty holds rows from ty*W - ysh, chunk zc planes from
  // zc*Z - zsh (clipped to the grid), so that the interior rectangle starts at the first row and
  // plane clear of walls and layers
  int ysh, zsh;
  long long plane;           // pitch*ny
  float ca;
  // field arrays, [time level][component]; element type depends on the storage
  void *e[2][3];
  void *h[2][3];
  // CPML psi slabs.  Axis u: 0 (x) -> (Ey,Ez) / (Hy,Hz); 1 (y) -> (Ex,Ez) / (Hx,Hz);
  // 2 (z) -> (Ex,Ey) / (Hx,Hy).  psi_h is kept in two time levels (halo recompute).
  float *psi_e[3][2];
  float *psi_h[2][3][2];
  float *psi_e2[3][2];       // second level of psi_E, written by the two-step sweeps
  float *psi_eb[3][2];       // second set of the E-term psi cotangents (adjoint only)
  AxisTab ax[3];
  // storage scales: stored = scale * physical
  float se, sh;
  // source
  int src_on, n_bins, src_i0, src_j0, src_ni, src_nj;
  double x_axis, y_axis, z_entry, t_entry, v_src, sigma_z, cut_sigmas, z_bin0, dz_bin, dz, dt;
  double cb_src;             // scale_e * Cb: E increment per unit current density
  const double *q_bins;      // device, the plan's profile
  const double *wr;          // device [src_nj][src_ni] radial weights
  const double *dwr;         // device [src_nj][src_ni] their derivative with respect to sigma_r
  // observers
  int n_obs;
  const int *obs_idx;        // [n_obs][3 comps][3] base node of the trilinear stencil
  const double *obs_t;       // [n_obs][3 comps][3] fractional offsets
  // transposed sampling: one key per distinct (component, stencil node), its contributions
  // (observer, FP64 weight) in observer order
  int n_skeys;
  const long long *sk_node;
  const int *sk_comp, *sk_ptr, *se_obs;
  const double *se_w;
  double inv_se;             // 1/scale_e for the gather
  int *nan_flag;
  // samples of the intermediate level of a two-step pass: entries (j, i, comp, slot) of the
  // observers' distinct stencil nodes sorted by plane (smp_ptr[k] .. smp_ptr[k+1]), the FP32
  // values (smp[slot]) and the slot of each (observer, comp, corner)
  const int *smp_ptr;
  const int4 *smp_ent;
  float *smp;
  const int *smp_slot;
  const int *slow_tiles;     // [n_slow][2] (ty, zc) of the tiles taking the general path
  const int *layer_tiles;    // [n_layer][2] (ty, zc) of the wall-free tiles touching a layer
  // Mur
  float mur_kx, mur_ky, mur_kz;
  int bc;
  // adjoint coefficients (physical units)
  float a_cb, a_db, a_ca;
  double a_cb_src;           // Cb (unscaled)
  // dynamic FP16 scaling (dyn != 0): per time level the exponent e of its extra storage factor
  // (stored = 2^e * scale * physical) and the index of the slot holding the level's maxima;
  // three slots of (max |E|, max |H|) in stored units, as float bits; the per-step gains of the
  // curl terms and the source's largest Ez increment, in stored units at e = 0
  int dyn;
  int *dexp[2];
  int *dslot[2];
  unsigned *dmax;
  float dyn_ge, dyn_gh, dyn_src;
};

struct FusedShape {
  int vx, rows, waves, zchunk, nty, nzc, n_tiles, n_blocks;
  // tiles clear of walls and y/z layers form the rectangle [ty_lo,ty_hi) x [zc_lo,zc_hi); the
  // other tiles are listed in two tables: clear of walls (layer) and touching a wall (slow)
  int ty_lo, ty_hi, zc_lo, zc_hi, n_fast, fast_blocks, n_layer, layer_blocks, n_slow, slow_blocks;
  int n_slow_y;  // leading entries of the tile table whose planes lie in [zc_lo, zc_hi) chunks
  int prefetch;  // interior tiles issue each plane's loads one plane ahead
  int ysh, zsh;  // tile grid origin (rows from ty*waves - ysh, planes from zc*zchunk - zsh)
  int xs;        // waves per row: 2 splits rows of 257-512 nodes (prefetching sweep, VX 4)
};

// Two-step sweep shape: W rows per tile (XS waves of 64 VX nodes per row), Z planes per chunk;
// tiles whose computed rows and planes (two below, one above) lie clear of walls and y/z
// layers form the rectangle [ty_lo, ty_hi) x [zc_lo, zc_hi); the remaining rows are covered by
// tiles of kStep2BoundaryRows rows listed in the table as (first row, end of owned rows, chunk),
// first those in the rectangle's z range (y walls and layers only), then the rest.
struct Shape2 {
  int on, vx, xs, waves, zchunk, nty, nzc;
  int ty_lo, ty_hi, zc_lo, zc_hi, n_fast, fast_blocks, n_slow, n_slow_y;
  int ysh, zsh;  // grid origin: rectangle tile ty owns rows from ty*waves - ysh, chunk zc planes from zc*zchunk - zsh
};

}  // namespace chf

struct chf_plan {
  chf_grid grid;
  chf_medium med;
  chf_boundary bnd;
  chf_source src;
  chf_exec ex;
  std::vector<double> q_bins;
  std::vector<double> obs_xyz;
  int kernel;       // resolved CHF_KERNEL_SPLIT / CHF_KERNEL_FUSED
  int storage;
  int elem_bytes;
  chf::FusedShape fs;
  chf::Shape2 fs2;             // two Yee steps per pass (CHF_KERNEL_FUSED2)
  // host-side tables (uploaded at bind time)
  std::vector<float> tabf;     // all float axis tables
  std::vector<int> tabi;       // all int slot tables
  std::vector<double> wr;      // radial weights
  std::vector<int> obs_idx;
  std::vector<double> obs_t;
  std::vector<long long> sk_node;
  std::vector<int> sk_comp, sk_ptr, se_obs;
  std::vector<double> se_w;
  size_t off_tabf[3][10], off_tabi[3][2];
  // workspace layout (byte offsets)
  uint64_t off_e[2][3], off_h[2][3], off_psi_e[3][2], off_psi_h[2][3][2];
  uint64_t off_tf, off_ti, off_wr, off_q, off_oidx, off_ot, off_nan, off_tiles, off_ltiles, ws_bytes;
  uint64_t off_psi_eb[3][2];   // after the snapshot region: not part of the forward state
  uint64_t off_sknode, off_skcomp, off_skptr, off_seobs, off_sew;
  std::vector<int> slow_tiles, layer_tiles;
  std::vector<int> tiles2;               // boundary tiles of the two-step sweep
  std::vector<int> smp_ptr, smp_ent, smp_slot;
  uint64_t off_psi_e2[3][2], off_tiles2, off_smp_ptr, off_smp_ent, off_smp, off_smp_slot;
  // dynamic scaling words (inside the state region, after psi): per level (exponent, maxima slot)
  // at off_dyn + 16 l, the three maxima slots at off_dyn + 32
  uint64_t off_dyn = 0;
  size_t n_smp = 0;
  // the two field levels (with psi_H) and the two psi_E levels are exchanged relative to their
  // workspace offsets after every two-step launch, so that level `parity` always holds the
  // state after n_done steps; snapshots are stored in the unexchanged order
  int lev_swap = 0, pe_swap = 0;
  uint64_t field_bytes, psi_bytes, psi_len[3];
  char *ws = nullptr;
  chf::Dev dev;
  int parity = 0;   // time level holding the current state
  int n_done = 0;   // steps advanced since the last reset (source clock)
  int adj_next = -1;  // next adjoint step range ends here (-1: no adjoint in progress)
  double scale_e = 1.0, scale_h = 1.0;
  double ca, cb, db;
  // side stream for the boundary H sweep, which runs beside the fused interior sweep
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // a second side stream: the z-boundary sweep beside the y-boundary one
  hipStream_t aux2 = nullptr;
  hipEvent_t ev_join2 = nullptr;
  // graph cache
  hipGraphExec_t graph = nullptr;
  const void *graph_w = nullptr, *graph_q = nullptr;
  int graph_parity = -1;
  int graph_swap = 0;  // level exchange state at the end of the captured run
};

struct chf_batch {
  std::vector<chf_plan *> plans;
  int storage = 0, vx = 1, waves = 4, n_steps = 0, max_patch = 0, total_obs = 0;
  int prefetch = 0;  // the members' sweep kind (all equal): tiles load a plane ahead
  bool any_mur = false;
  std::vector<int> zchunks;   // per plan
  std::vector<int> fast_tab;  // (plan, ty, zc) over the interior rectangles
  std::vector<int> slow_tab;  // (plan, ty, zc, x block) over the boundary tiles (split sweeps)
  // (plan, ty, zc) over the boundary tiles in the general fused sweep: interior z range, rest
  bool gen = false;
  std::vector<int> gen_tab[2];
  std::vector<int> obs_tab;   // (plan, observer)
  uint64_t off_devs = 0, off_z = 0, off_fast = 0, off_slow = 0, off_obs = 0, off_wptr = 0, ws_bytes = 0;
  uint64_t off_gen[2] = {0, 0};
  std::vector<int> all_tab;  // (plan, ty, zc) over every tile: the persistent launch's work list
  uint64_t off_all = 0;
  char *ws = nullptr;
  std::vector<chf::Dev> devs;
  std::vector<double *> wptr;
  hipGraphExec_t graph = nullptr;
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // a second side stream: the z-boundary sweep beside the y-boundary one
  hipStream_t aux2 = nullptr;
  hipEvent_t ev_join2 = nullptr;
};

namespace chf {
// kernel launchers (chf_kernels.hip)
hipError_t launch_step(const chf_plan &p, const Dev &d, int parity, int step, const double *q_dev,
                       double *w_dev, int column, int ld, hipStream_t s, hipEvent_t ev_a = nullptr,
                       hipEvent_t ev_b = nullptr);
hipError_t launch_zero(const chf_plan &p, hipStream_t s);
// two Yee steps (step, step+1) from level `parity` into level parity^1 (chf_step2.hip): the
// waveform columns `column` (intermediate level) and `column + 1`
hipError_t launch_step2(const chf_plan &p, const Dev &d, int parity, int step, const double *q_dev,
                        double *w_dev, int column, int ld, hipStream_t s, hipEvent_t ev_a = nullptr,
                        hipEvent_t ev_b = nullptr);
// exchange the level pointers after a two-step launch; canonical pointers from the offsets
void swap_levels(chf_plan &p, Dev &d);
void canonical_pointers(chf_plan &p);
// n steps from the plan's state (chf_api.hip): two-step launches while two or more steps remain
// on a two-step plan, single steps otherwise; with `ev`, an event pair around every interior
// launch of the dominant kind, their number in *n_ev
hipError_t advance(chf_plan &p, hipStream_t s, const double *q, double *w, int col0, int ld, int n,
                   hipEvent_t *ev = nullptr, int *n_ev = nullptr);
// dynamic scaling: after the sweeps of a launch of n steps from level `parity`, publish the
// written level's exponent and maxima slot and clear the slot the next launch raises; and the
// maxima of level `parity` recomputed from its fields (after a direct write)
hipError_t launch_dyn_publish(const Dev &d, int parity, int n, hipStream_t s);
hipError_t launch_dyn_levelmax(const chf_plan &p, int parity, hipStream_t s);
hipError_t launch_get_field(const chf_plan &p, int parity, int comp, float *out, hipStream_t s);
hipError_t launch_set_field(const chf_plan &p, int parity, int comp, const float *in, hipStream_t s);
// forward E levels of one step and the permittivity cotangent they feed (adjoint of eps_r)
struct EpsTerm {
  const float *e0, *e1;  // E^n, E^{n+1}: dense [3][nz][ny][nx] FP32
  double *g;             // dL/deps_r per E node, same layout, FP64, accumulated
  double coef;           // 1/(eps_r (1 + sigma dt / (2 eps)))
};
hipError_t launch_adjoint_step(const chf_plan &p, const Dev &d, int parity, int step,
                               const double *dl_dw, double *dl_dq, hipStream_t s,
                               const double *q_dev = nullptr, double *dl_dtheta = nullptr,
                               const EpsTerm *eps = nullptr);
hipError_t launch_adjoint_init(const chf_plan &p, double *dl_dq, hipStream_t s, int n = -1);
hipError_t launch_adjoint_clear(const chf_plan &p, hipStream_t s);
hipError_t launch_batch_step(const chf_batch &b, int parity, int step, hipStream_t s);
// the whole batch run in one cooperative launch over the combined tile table `tab` (device,
// n_tab entries of (plan, ty, zc)); FP32 members with boundary tiles in the general fused sweep
hipError_t launch_batch_persistent(const chf_batch &b, const int *tab, int n_tab, hipStream_t s);
void set_error(const std::string &msg);
// plan tables into a workspace (chf_api.hip)
hipError_t bind_tables(chf_plan *p, char *ws, hipStream_t s);
}  // namespace chf
