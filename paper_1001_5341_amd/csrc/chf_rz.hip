// Axisymmetric (r, z) solver of libchfdtd for gfx950: E_r, E_z, H_phi on the (r, z) restriction
// of the Yee lattice (eqs. fdtd_Er, fdtd_Ez, fdtd_Hphi of the Numerical Method section), the
// entry points declared in include/chfdtd_rz.h.
//
// Data layout: each component is a row-major [nz][pitch] FP32 array (r fastest, pitch a
// multiple of 64 nodes, padding columns zero), in two time levels.  Step n reads level `par`
// (E^n, H^{n-1/2}) and writes level par^1, so one sweep can recompute the H values its tile
// borrows from neighbouring tiles without racing them.
//
// The sweep: a wave owns 64*VX consecutive radial nodes (VX per lane, 16-byte loads) and
// marches up a chunk of z rows.  Per row it loads E_r(k+1), E_z(k) and H(k) once, forms
// H^{n+1/2}(k) (the E_z(i+1) of the last node of a lane comes from the next lane by a
// shuffle, or for lane 63 from the next wave's first node), then E_r^{n+1}(k) from H(k) and
// the H(k-1) kept in registers, and E_z^{n+1}(k) from H(i) and H(i-1) (H(i-1) of the first
// node of a lane by shuffle; lane 0 recomputes it from the input level).  A chunk starts by
// recomputing H of the row below it.  Every variant and tile shape evaluates each node with
// the same expression in the same order, so results do not depend on the tiling.
//
//   H   += db/dr (E_z(i+1) - E_z(i)) - db/dz (E_r(k+1) - E_r(k))
//   E_r  = ca E_r - cb/dz (H(k) - H(k-1))
//   E_z  = ca E_z + cp_i H(i) - cm_i H(i-1),  cp_i = cb r_{i+1/2}/(a_i dr), cm_i = cb r_{i-1/2}/(a_i dr)
// with a_i = r_i (a_0 = dr/8, the disc of radius dr/2 on the axis).  The same launch subtracts
// cb J_z of the moving source on the nodes it covers, writes the Mur (or PEC) wall values, and
// samples the previous step's E at the observers in FP64 (that level is this launch's input, so
// the sampling races nothing); a small gather kernel samples the last step of each call.  A step
// is thus one kernel launch.
#include <hip/hip_runtime.h>

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/chfdtd_rz.h"
#include "chf_internal.h"

namespace {

constexpr double kC0 = 299792458.0;
constexpr double kMu0 = 1.25663706212e-6;  // CODATA 2018
constexpr double kPi = 3.14159265358979323846;
const double kEps0 = 1.0 / (kMu0 * kC0 * kC0);
constexpr int kRzMaxWz = 64;          // longitudinal source support in rows
constexpr int kRzMaxObs = 1 << 16;
// Largest eigenvalue of the radial operator times dr^2 (4 on a Cartesian line; the axis cell
// raises it to 4.8419...), rounded up.
constexpr double kRadialEig = 4.85;

struct RDev {
  int nr, nz, pitch, zchunk, nrb, n_blocks, n_gblocks, wv;
  int nrb2, n_waves2, n_blocks2;  // two-step launches: overlapped waves of 62*VX stored nodes
  float ca, db_dr, db_dz, cb_dz;
  void *f[2][3];           // [level][E_r, E_z, H_phi], element type = the storage type
  // 16-bit storage keeps scale * physical value (FP32 stores physical values): fixed scales, or
  // (dyn) scales chosen by every launch from the maxima of the level it reads
  float s_e, s_h;
  int dyn;
  float *lvl_scale;        // [2 levels][2] (s_e, s_h) of the values a level slot holds
  unsigned *maxes;         // [3][2] max |E|, max |H| (FP32 bits) of a level, by launch index mod 3
  float ge, gh, target;    // per-step growth bounds (E from H, H from E); largest stored value aimed at
  double src_bound;        // Cb v max W_r e^{dz^2/8 sigma_z^2} / dz (source increment per unit charge)
  const float *cp, *cm;    // [pitch]
  // source
  int src_on, n_bins, n_src;
  double z_entry, t_entry, v_src, sigma_z, cut_sigmas, z_bin0, dz_bin, dz, dt, cb;
  const double *q_bins, *wr;
  // Mur
  int mur;
  float mur_kr, mur_kz;
  // observers
  int n_obs;
  const int *obs_idx;      // [n_obs][2][2] (i0, k0) per component
  const double *obs_t;     // [n_obs][2][2] (tr, tz)
  int *nan_flag;
  // observer stencil nodes by row, for the intermediate level of two-step launches
  const int *row_ptr;      // [nz+1]
  const int2 *ent;         // (node i, slot | component << 30), slot = (obs*2 + comp)*4 + corner
  const double *ent_w;     // bilinear weights
  double *samp;            // [2][8 n_obs] weight * E^{n+1}
};

chf_status fail(chf_status s, const std::string &m) {
  chf::set_error(m);
  return s;
}

chf_status hip_fail(hipError_t e, const char *what) {
  chf::set_error(std::string(what) + ": " + hipGetErrorString(e));
  return CHF_EHIP;
}

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

}  // namespace

struct chf_rz_plan {
  chf_rz_grid g;
  chf_medium med;
  chf_rz_source src;
  chf_rz_exec ex;
  std::vector<double> q_bins;
  int vx = 4, wv = 4, zchunk = 32, pitch = 0, nrb = 0, nzc = 0, n_blocks = 0, n_src = 0;
  int spl = 1;                // Yee steps per launch (2: temporally blocked)
  int nrb2 = 0, n_waves2 = 0, n_blocks2 = 0;
  int samp_par = 0;           // sample buffer the last two-step launch wrote
  bool mur_r_kernel = false;  // the r-wall node starts a wave: its Mur value takes a kernel of its own
  double ca = 1, cb = 0, db = 0;
  std::vector<float> cp, cm;
  std::vector<double> wr;
  std::vector<int> oidx;
  std::vector<double> ot;
  std::vector<int> row_ptr, ent;  // observer stencil nodes by row: (node, slot | comp << 30)
  std::vector<double> ent_w;
  uint64_t off_f[2][3] = {}, off_cp = 0, off_cm = 0, off_wr = 0, off_q = 0, off_oidx = 0, off_ot = 0,
           off_nan = 0, off_rowptr = 0, off_ent = 0, off_entw = 0, off_samp = 0, field_bytes = 0, ws_bytes = 0;
  char *ws = nullptr;
  RDev dev{};
  int parity = 0, n_done = 0;
  int li = 0;                 // launches since the reset (dynamic-scale slots)
  int storage = CHF_FP32, elem = 4;
  double scale_e = 1.0, scale_h = 1.0;
  uint64_t off_scale = 0;
  hipGraphExec_t graph = nullptr;
  const void *graph_w = nullptr, *graph_q = nullptr;
};

namespace {

// ------------------------------------------------------------------ kernels
template <int N>
struct alignas(4 * N) F {
  float v[N];
};

template <int N>
__device__ __forceinline__ void ld(const float *p, float (&o)[N], bool on) {
  if (on) {
    const F<N> x = *reinterpret_cast<const F<N> *>(p);
#pragma unroll
    for (int v = 0; v < N; v++) o[v] = x.v[v];
  } else {
#pragma unroll
    for (int v = 0; v < N; v++) o[v] = 0.f;
  }
}

// Row stores are non-temporal: a launch writes the other time level (and the other Mur
// memory), which nothing in the same launch reads, so it streams past L2.
template <int B>
__device__ __forceinline__ void st_nt(void *p, const void *x) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  if constexpr (B == 16) {
    u4 b;
    __builtin_memcpy(&b, x, 16);
    __builtin_nontemporal_store(b, reinterpret_cast<u4 *>(p));
  } else if constexpr (B == 8) {
    u2 b;
    __builtin_memcpy(&b, x, 8);
    __builtin_nontemporal_store(b, reinterpret_cast<u2 *>(p));
  } else if constexpr (B == 4) {
    unsigned b;
    __builtin_memcpy(&b, x, 4);
    __builtin_nontemporal_store(b, reinterpret_cast<unsigned *>(p));
  } else {
    __builtin_memcpy(p, x, B);
  }
}

template <int N>
__device__ __forceinline__ void st(float *p, const float (&o)[N], bool on) {
  if (!on) return;
  F<N> x;
#pragma unroll
  for (int v = 0; v < N; v++) x.v[v] = o[v];
  st_nt<sizeof(x)>(p, &x);
}

// Field storage: FP32 holds physical values; 16-bit types hold scale * value, rounded to
// nearest even on the store.
template <typename T>
__device__ __forceinline__ float to_f(T x) { return static_cast<float>(x); }
template <typename T>
__device__ __forceinline__ T from_f(float x) { return static_cast<T>(x); }

template <typename T, int N>
struct alignas(sizeof(T) * N) V {
  T v[N];
};

template <typename T>
constexpr bool kF32 = std::is_same<T, float>::value;

template <typename T, int N>
__device__ __forceinline__ void ldf(const T *p, float (&o)[N], bool on, float inv) {
  if (on) {
    const V<T, N> x = *reinterpret_cast<const V<T, N> *>(p);
#pragma unroll
    for (int v = 0; v < N; v++) o[v] = kF32<T> ? to_f<T>(x.v[v]) : to_f<T>(x.v[v]) * inv;
  } else {
#pragma unroll
    for (int v = 0; v < N; v++) o[v] = 0.f;
  }
}

template <typename T>
__device__ __forceinline__ float lds(const T *p, float inv) {
  return kF32<T> ? to_f<T>(*p) : to_f<T>(*p) * inv;
}

template <typename T, int N>
__device__ __forceinline__ void stf(T *p, const float (&o)[N], bool on, float s) {
  if (!on) return;
  V<T, N> x;
#pragma unroll
  for (int v = 0; v < N; v++) x.v[v] = from_f<T>(kF32<T> ? o[v] : o[v] * s);
  st_nt<sizeof(x)>(p, &x);
}

// the value a store with scale s followed by a load returns
template <typename T, int N>
__device__ __forceinline__ void as_stored(float (&o)[N], float s, float inv) {
  if constexpr (!kF32<T>) {
#pragma unroll
    for (int v = 0; v < N; v++) o[v] = to_f<T>(from_f<T>(o[v] * s)) * inv;
  }
}

// Scales of one launch: inverse scales of the level read, scales of the level written.
struct Sc {
  float ei, hi, eo, ho;
};

__device__ __forceinline__ float pow2_floor(float x) { return exp2f(floorf(log2f(x))); }

// Bound on the source's E_z increment over `n` steps from `step`, for the dynamic scale bound:
// Cb v |Q(z_s)| max W_r max W_z, where max W_z <= e^{dz^2 / 8 sigma_z^2} / dz because the
// normalising window always holds a row within dz/2 of z_s (src_bound = Cb v max W_r times that).
__device__ float source_peak(const RDev &d, int step, int n, const double *q) {
  if (!d.src_on || d.n_src <= 0) return 0.f;
  double peak = 0.0;
  const double *qb = q ? q : d.q_bins;
  for (int t = 0; t < n; t++) {
    const double tt = (step + t + 0.5) * d.dt;
    if (tt < d.t_entry) continue;
    const double u = (d.z_entry + d.v_src * (tt - d.t_entry) - d.z_bin0) / d.dz_bin;
    const double fl = floor(u);
    const int b0 = (int)fl;
    const double fr = u - fl;
    double qz = 0.0;
    if (b0 >= 0 && b0 < d.n_bins) qz += (1.0 - fr) * qb[b0];
    if (b0 + 1 >= 0 && b0 + 1 < d.n_bins) qz += fr * qb[b0 + 1];
    peak = fmax(peak, fabs(qz));
  }
  return (float)(peak * d.src_bound);
}

// Launch li (reading level par, advancing n steps): static scales, or (dyn) the scales of the
// level read from lvl_scale and, for the level written, the largest power of two keeping the
// bound B on its magnitudes below `target`: B_E = 2 max|E| + n ge max|H| + 2 n (source peak),
// B_H = 2 max|H| + n gh B_E (maxima of the level read, slot li mod 3).  Every wave computes the
// same values.
__device__ __forceinline__ Sc launch_scales(const RDev &d, int par, int li, int step, int n, const double *q,
                                           int lane) {
  if (!d.dyn) return Sc{1.f / d.s_e, 1.f / d.s_h, d.s_e, d.s_h};
  const float se_in = d.lvl_scale[2 * par], sh_in = d.lvl_scale[2 * par + 1];
  const unsigned *mx = d.maxes + 2 * (li % 3);
  const float me = __uint_as_float(mx[0]), mh = __uint_as_float(mx[1]);
  const float pk = source_peak(d, step, n, q);
  const float be = 2.f * me + n * d.ge * mh + 2.f * n * pk;
  const float bh = 2.f * mh + n * d.gh * be;
  const float cap = 1.0e30f;
  const float se = be > 0.f ? fminf(pow2_floor(d.target / be), cap) : 1.f;
  const float sh = bh > 0.f ? fminf(pow2_floor(d.target / bh), cap) : 1.f;
  return Sc{1.f / se_in, 1.f / sh_in, se, sh};
}

// dyn bookkeeping at the start of launch li (one thread of the grid): publish the written level's
// scales and clear the maxima slot the next launch but one will fill.
__device__ __forceinline__ void publish_scales(const RDev &d, int par, int li, const Sc &sc) {
  d.lvl_scale[2 * (par ^ 1)] = sc.eo;
  d.lvl_scale[2 * (par ^ 1) + 1] = sc.ho;
  d.maxes[2 * ((li + 2) % 3)] = 0u;
  d.maxes[2 * ((li + 2) % 3) + 1] = 0u;
}

// wave maximum of two values, then at most one atomic per value and wave into the slot of the
// level written
__device__ __forceinline__ void record_max(const RDev &d, int li, float me, float mh, int lane) {
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) {
    me = fmaxf(me, __shfl_xor(me, k));
    mh = fmaxf(mh, __shfl_xor(mh, k));
  }
  if (lane == 0) {  // the atomic only where it raises the maximum: thousands of waves share the words
    unsigned *mx = d.maxes + 2 * ((li + 1) % 3);
    const unsigned ue = __float_as_uint(me), uh = __float_as_uint(mh);
    if (ue > *(volatile unsigned *)mx) atomicMax(mx, ue);
    if (uh > *(volatile unsigned *)(mx + 1)) atomicMax(mx + 1, uh);
  }
}

template <int N>
__device__ __forceinline__ float amax(const float (&a)[N], float m) {
#pragma unroll
  for (int v = 0; v < N; v++) m = fmaxf(m, fabsf(a[v]));
  return m;
}

// H' = H - db/dz dEr + db/dr dEz (the order every kernel and tile shape uses)
__device__ __forceinline__ float h_node(float h, float d_er, float d_ez, const RDev &d) {
  return fmaf(d.db_dr, d_ez, fmaf(-d.db_dz, d_er, h));
}

// Observer sampling of level `par` into waveform column `column`: eight observers per wave,
// lane = 8*observer + 4*component + corner; each lane forms weight * E in FP64 and two
// butterflies sum the corners.
template <typename T>
__device__ __forceinline__ void gather_wave(const RDev &d, int par, double *w, int column, int ld, int o0,
                                            int lane, float inv_e) {
  const int o = o0 + (lane >> 3);
  const int comp = (lane >> 2) & 1, a = lane & 1, b = (lane >> 1) & 1;
  double val = 0.0;
  if (o < d.n_obs) {
    const int *ix = d.obs_idx + (o * 2 + comp) * 2;
    const double *tf = d.obs_t + (o * 2 + comp) * 2;
    const double wgt = (a ? tf[0] : 1.0 - tf[0]) * (b ? tf[1] : 1.0 - tf[1]);
    const long long node = (long long)(ix[1] + b) * d.pitch + ix[0] + a;
    val = wgt * (double)lds<T>((const T *)d.f[par][comp] + node, inv_e);
  }
  val += __shfl_xor(val, 1);
  val += __shfl_xor(val, 2);
  if (o < d.n_obs && (lane & 3) == 0) {
    w[((long long)o * 2 + comp) * ld + column] = val;
    if (d.nan_flag && !isfinite(val)) *d.nan_flag = 1;
  }
}

// The work a launch does for its predecessor: sample the level it starts from into column gcol,
// and sum the stencil samples a two-step launch took of its intermediate level (buffer sb) into
// column scol, corners added in the order the gather uses.
template <typename T>
__device__ __forceinline__ void pending_wave(const RDev &d, int par, double *w, int ld, int gcol, int scol, int sb,
                                             int o0, int lane, float inv_e) {
  if (gcol >= 0) gather_wave<T>(d, par, w, gcol, ld, o0, lane, inv_e);
  if (scol >= 0) {
    const int o = o0 + (lane >> 1), comp = lane & 1;
    if (lane < 16 && o < d.n_obs) {
      const double *s = d.samp + (long long)sb * 8 * d.n_obs + (o * 2 + comp) * 4;
      const double val = (s[0] + s[1]) + (s[2] + s[3]);
      w[((long long)o * 2 + comp) * ld + scol] = val;
      if (d.nan_flag && !isfinite(val)) *d.nan_flag = 1;
    }
  }
}

// Source rows of one step for a wave (FP64 bookkeeping: bunch position, Q(z_s) from the hat
// bins, longitudinal weights normalised over the window; lane j holds the weight of row lo + j).
struct SrcRows {
  int lo, m;
  double amp, w;
};

__device__ __forceinline__ SrcRows source_rows(const RDev &d, int step, const double *q, int w0, int lane) {
  SrcRows s{0, 0, 0.0, 0.0};
  if (!d.src_on || w0 >= d.n_src) return s;
  const double tt = (step + 0.5) * d.dt;
  if (tt < d.t_entry) return s;
  const double zs = d.z_entry + d.v_src * (tt - d.t_entry);
  const double u = (zs - d.z_bin0) / d.dz_bin;
  const double fl = floor(u);
  const int b0 = (int)fl;
  const double t = u - fl;
  const double *qb = q ? q : d.q_bins;
  double qz = 0.0;
  if (b0 >= 0 && b0 < d.n_bins) qz += (1.0 - t) * qb[b0];
  if (b0 + 1 >= 0 && b0 + 1 < d.n_bins) qz += t * qb[b0 + 1];
  const double half = d.cut_sigmas * d.sigma_z;
  s.lo = (int)ceil((zs - half) / d.dz - 0.5);
  const int hi = (int)floor((zs + half) / d.dz - 0.5);
  s.m = max(0, min(hi - s.lo + 1, 64));
  const double dd = (s.lo + lane + 0.5) * d.dz - zs;
  double e = lane < s.m ? exp(-0.5 * dd * dd / (d.sigma_z * d.sigma_z)) : 0.0;
  double norm = e;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) norm += __shfl_xor(norm, m);
  s.w = e / (norm * d.dz);
  s.amp = d.cb * d.v_src * qz;
  return s;
}

// E_z -= Cb J_z on row k for the nodes of this lane (wave-uniform branch and shuffle)
template <int VX>
__device__ __forceinline__ void sub_source(const RDev &d, const SrcRows &s, int k, int c0, float (&ez)[VX]) {
  if (s.m > 0 && k - s.lo >= 0 && k - s.lo < s.m) {
    const double wz = __shfl(s.w, k - s.lo);
#pragma unroll
    for (int v = 0; v < VX; v++)
      if (c0 + v >= 0 && c0 + v < d.n_src) ez[v] = ez[v] - (float)(s.amp * d.wr[c0 + v] * wz);
  }
}

// E_z on r = r_max: inner^n + K (inner^{n+1} - wall^n), by the lane that owns the wall node
// (a wall node in lane 0 takes the value shuffled from no lane: callers never keep it)
template <int VX>
__device__ __forceinline__ void mur_r(const RDev &d, int vw, bool wall_here, float (&ezo)[VX], const float (&ez)[VX]) {
  const float en = __shfl_up(ezo[VX - 1], 1), ei = __shfl_up(ez[VX - 1], 1);
  if (wall_here) {
#pragma unroll
    for (int v = 0; v < VX; v++)
      if (v == vw) {
        const float inner_new = v > 0 ? ezo[v > 0 ? v - 1 : 0] : en;
        const float inner_old = v > 0 ? ez[v > 0 ? v - 1 : 0] : ei;
        ezo[v] = fmaf(d.mur_kr, inner_new - ez[v], inner_old);
      }
  }
}

template <int VX>
__device__ __forceinline__ void right_of(const float (&a)[VX], float (&r)[VX]) {
  const float t = __shfl_down(a[0], 1);
#pragma unroll
  for (int v = 0; v < VX; v++) r[v] = v + 1 < VX ? a[v + 1 < VX ? v + 1 : 0] : t;
}

// One whole step in one launch.  Workgroups [0, n_blocks) sweep tiles (a tile = wv waves side by
// side in r, each 64*VX nodes wide, times a chunk of z rows); the n_gblocks workgroups after
// them do the pending work of the previous launch (pending_wave).  Rows 0..nz-2 are marched;
// the E_r rows on the z walls are written from rows 1 and nz-2 (copied, or the Mur value).  The
// moving source is subtracted from E_z by the lanes that own its nodes, and the Mur value of E_z
// on the r wall by the lane that owns the wall (the host adds k_rz_mur_r when the wall is the
// first node of a wave).
template <typename T, int VX>
__global__ void __launch_bounds__(512) k_rz_step(RDev d, int par, int step, const double *q, double *w,
                                                 int gcol, int scol, int sb, int ldw, int li) {
  const int n_all = d.n_blocks + d.n_gblocks;
  const int per = (n_all + 7) >> 3;  // hardware block b runs on XCD b % 8
  const int logical = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (logical >= n_all) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const Sc sc = launch_scales(d, par, li, step, 1, q, lane);
  if (d.dyn && blockIdx.x == 0 && threadIdx.x == 0) publish_scales(d, par, li, sc);
  if (logical >= d.n_blocks) {
    pending_wave<T>(d, par, w, ldw, gcol, scol, sb, ((logical - d.n_blocks) * d.wv + wv) * 8, lane, sc.ei);
    return;
  }
  const int rb = logical % d.nrb, zc = logical / d.nrb;
  const int w0 = (rb * d.wv + wv) * 64 * VX;  // first node of the wave
  if (w0 >= d.nr) return;                     // whole wave beyond the last node
  const int c0 = w0 + lane * VX;
  const bool on = c0 < d.nr;
  const int nr = d.nr, nz = d.nz;
  const int k0 = zc * d.zchunk, k1 = min(k0 + d.zchunk, nz - 1);
  const long long P = d.pitch;
  const T *Er = (const T *)d.f[par][0], *Ez = (const T *)d.f[par][1], *Hp = (const T *)d.f[par][2];
  T *Ero = (T *)d.f[par ^ 1][0], *Ezo = (T *)d.f[par ^ 1][1], *Hpo = (T *)d.f[par ^ 1][2];
  float mx_e = 0.f, mx_h = 0.f;  // magnitudes written (dyn)
  const bool halo_l = lane == 0 && c0 > 0;          // lane 0 recomputes H(c0-1)
  const bool halo_r = lane == 63 && c0 + VX < nr;   // lane 63 reads E_z(c0+VX)

  float cp[VX], cm[VX];
  ld<VX>(d.cp + c0, cp, on);
  ld<VX>(d.cm + c0, cm, on);
  bool live[VX];
#pragma unroll
  for (int v = 0; v < VX; v++) live[v] = c0 + v <= nr - 2;
  const SrcRows S = source_rows(d, step, q, w0, lane);
  const int vw = nr - 1 - c0;
  const bool wall_here = d.mur && vw >= 0 && vw < VX && !(vw == 0 && lane == 0);
  const bool wall_wave = d.mur && nr - 1 > w0 && nr - 1 < w0 + 64 * VX;  // some lane > 0 or v > 0

  float er_k[VX], hn_b[VX];  // E_r(k) of the input level, H^{n+1/2}(k-1)
  float erl_k = 0.f;         // lane 0: E_r(c0-1, k)
  if (k0 > 0) {
    const int kb = k0 - 1;
    float erb[VX], ezb[VX], hb[VX];
    ldf<T, VX>(Er + kb * P + c0, erb, on, sc.ei);
    ldf<T, VX>(Er + k0 * P + c0, er_k, on, sc.ei);
    ldf<T, VX>(Ez + kb * P + c0, ezb, on, sc.ei);
    ldf<T, VX>(Hp + kb * P + c0, hb, on, sc.hi);
    float ezr = __shfl_down(ezb[0], 1);
    if (lane == 63) ezr = halo_r ? lds<T>(Ez + kb * P + c0 + VX, sc.ei) : 0.f;
#pragma unroll
    for (int v = 0; v < VX; v++) {
      const float e1 = v + 1 < VX ? ezb[v + 1] : ezr;
      hn_b[v] = live[v] ? h_node(hb[v], er_k[v] - erb[v], e1 - ezb[v], d) : hb[v];
    }
  } else {
    ldf<T, VX>(Er + c0, er_k, on, sc.ei);
#pragma unroll
    for (int v = 0; v < VX; v++) hn_b[v] = 0.f;
  }
  if (halo_l) erl_k = lds<T>(Er + k0 * P + c0 - 1, sc.ei);

  for (int k = k0; k < k1; k++) {  // k <= nz-2
    float er1[VX], ez[VX], h[VX];
    ldf<T, VX>(Er + (k + 1) * P + c0, er1, on, sc.ei);
    ldf<T, VX>(Ez + k * P + c0, ez, on, sc.ei);
    ldf<T, VX>(Hp + k * P + c0, h, on, sc.hi);
    float ezr = __shfl_down(ez[0], 1);
    if (lane == 63) ezr = halo_r ? lds<T>(Ez + k * P + c0 + VX, sc.ei) : 0.f;
    float hn[VX];
#pragma unroll
    for (int v = 0; v < VX; v++) {
      const float e1 = v + 1 < VX ? ez[v + 1] : ezr;
      hn[v] = live[v] ? h_node(h[v], er1[v] - er_k[v], e1 - ez[v], d) : h[v];
    }
    // H(c0-1, k): from the lane below, or recomputed by lane 0 from the input level
    float hl = __shfl_up(hn[VX - 1], 1);
    if (lane == 0) {
      hl = 0.f;
      if (halo_l) {
        const long long c = k * P + c0 - 1;
        const float h_l = lds<T>(Hp + c, sc.hi), ez_l = lds<T>(Ez + c, sc.ei), er1_l = lds<T>(Er + c + P, sc.ei);
        hl = h_node(h_l, er1_l - erl_k, ez[0] - ez_l, d);
        erl_k = er1_l;
      }
    }
    const bool erow = k >= 1;
    float ero[VX], ezo[VX];
#pragma unroll
    for (int v = 0; v < VX; v++) {
      ero[v] = live[v] && erow ? fmaf(-d.cb_dz, hn[v] - hn_b[v], d.ca * er_k[v]) : er_k[v];
      const float hm = v > 0 ? hn[v - 1] : hl;
      ezo[v] = live[v] ? fmaf(-cm[v], hm, fmaf(cp[v], hn[v], d.ca * ez[v])) : ez[v];
    }
    sub_source<VX>(d, S, k, c0, ezo);
    if (wall_wave) mur_r<VX>(d, vw, wall_here, ezo, ez);
    stf<T, VX>(Hpo + k * P + c0, hn, on, sc.ho);
    if (k >= 1) stf<T, VX>(Ero + k * P + c0, ero, on, sc.eo);
    stf<T, VX>(Ezo + k * P + c0, ezo, on, sc.eo);
    if (d.dyn) {
      mx_h = amax<VX>(hn, mx_h);
      mx_e = amax<VX>(ezo, amax<VX>(ero, mx_e));
    }
    if (k == 1) {  // z = 0 wall from row 1
      float w0v[VX];
      ldf<T, VX>(Er + c0, w0v, on, sc.ei);
#pragma unroll
      for (int v = 0; v < VX; v++)
        if (d.mur && live[v]) w0v[v] = fmaf(d.mur_kz, ero[v] - w0v[v], er_k[v]);
      stf<T, VX>(Ero + c0, w0v, on, sc.eo);
      if (d.dyn) mx_e = amax<VX>(w0v, mx_e);
    }
    if (k == nz - 2) {  // z = z_max wall from row nz-2
      float w1v[VX];
#pragma unroll
      for (int v = 0; v < VX; v++)
        w1v[v] = d.mur && live[v] ? fmaf(d.mur_kz, ero[v] - er1[v], er_k[v]) : er1[v];
      stf<T, VX>(Ero + (k + 1) * P + c0, w1v, on, sc.eo);
      if (d.dyn) mx_e = amax<VX>(w1v, mx_e);
    }
#pragma unroll
    for (int v = 0; v < VX; v++) {
      er_k[v] = er1[v];
      hn_b[v] = hn[v];
    }
  }
  if (d.dyn) record_max(d, li, mx_e, mx_h, lane);
}

// Two steps in one launch (temporal blocking).  Waves overlap: wave g covers the 64*VX nodes from
// g*62*VX - VX, and only lanes 1..62 store, so every H and E a stored node needs is formed inside
// the wave from the input level (VX >= 4 keeps the lanes' own halo cells exact): step n+1 (stage
// 1) for row m, then step n+2 (stage 2) for row m-1 from stage-1 values held in registers.  The
// intermediate level never reaches HBM: its observer-stencil values are written, weighted, to
// the sample buffer sb (summed by the next launch).  Per node and step the arithmetic is that of
// k_rz_step, so the two kernels give the same bits.
template <typename T, int VX>
__global__ void __launch_bounds__(512) k_rz_step2(RDev d, int par, int step, const double *q, double *w,
                                                  int gcol, int scol, int sb_in, int sb_out, int ldw, int li) {
  const int n_all = d.n_blocks2 + d.n_gblocks;
  const int per = (n_all + 7) >> 3;
  const int logical = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (logical >= n_all) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // both steps store with the written level's scales; the intermediate level is rounded as a
  // store and load with them would round it
  const Sc sc = launch_scales(d, par, li, step, 2, q, lane);
  if (d.dyn && blockIdx.x == 0 && threadIdx.x == 0) publish_scales(d, par, li, sc);
  if (logical >= d.n_blocks2) {
    pending_wave<T>(d, par, w, ldw, gcol, scol, sb_in, ((logical - d.n_blocks2) * d.wv + wv) * 8, lane, sc.ei);
    return;
  }
  const int rb = logical % d.nrb2, zc = logical / d.nrb2;
  const int g = rb * d.wv + wv;
  if (g >= d.n_waves2) return;
  const int nr = d.nr, nz = d.nz;
  const int w0 = g * 62 * VX - VX;  // node of lane 0, cell 0
  const int c0 = w0 + lane * VX;
  const bool on = c0 >= 0 && c0 < nr;
  const bool outl = on && lane >= 1 && lane <= 62;
  const int k0 = zc * d.zchunk, k1 = min(k0 + d.zchunk, nz - 1);  // stage-2 rows [k0, k1)
  const int m0 = max(0, k0 - 2);
  const long long P = d.pitch;
  const T *Er = (const T *)d.f[par][0], *Ez = (const T *)d.f[par][1], *Hp = (const T *)d.f[par][2];
  T *Ero = (T *)d.f[par ^ 1][0], *Ezo = (T *)d.f[par ^ 1][1], *Hpo = (T *)d.f[par ^ 1][2];
  const float mi_e = 1.f / sc.eo, mi_h = 1.f / sc.ho;  // intermediate level: stored with the out scales
  float mx_e = 0.f, mx_h = 0.f;

  float cp[VX], cm[VX];
  ld<VX>(d.cp + c0, cp, on);
  ld<VX>(d.cm + c0, cm, on);
  bool live[VX];
#pragma unroll
  for (int v = 0; v < VX; v++) live[v] = on && c0 + v <= nr - 2;
  const SrcRows S1 = source_rows(d, step, q, w0, lane);
  const SrcRows S2 = source_rows(d, step + 1, q, w0, lane);
  const int vw = nr - 1 - c0;
  const bool wall_here = d.mur && on && vw >= 0 && vw < VX;
  const bool wall_wave = d.mur && nr - 1 >= w0 && nr - 1 < w0 + 64 * VX;
  double *samp = d.samp + (long long)sb_out * 8 * d.n_obs;

  float er_in[VX];                     // E_r^n(m)
  float er1_b[VX], ez1_b[VX], h1_b[VX];  // stage 1 of row m-1 (as stored)
  float h1u_b[VX];                     // stage-1 H of row m-1 before rounding (stage 1's own E_r)
  float h2_b[VX];                      // stage 2 H of row j-1
  float er1w0[VX];                     // stage-1 E_r of the z = 0 wall row (chunks from row 0 or 1)
  ldf<T, VX>(Er + m0 * P + c0, er_in, on, sc.ei);
#pragma unroll
  for (int v = 0; v < VX; v++) {
    er1_b[v] = 0.f;
    ez1_b[v] = 0.f;
    h1_b[v] = 0.f;
    h1u_b[v] = 0.f;
    h2_b[v] = 0.f;
    er1w0[v] = 0.f;
  }

  for (int m = m0; m <= k1; m++) {
    // ---- stage 1 (step n -> n+1), row m
    float er1[VX], ez1[VX], h1[VX], er1n[VX];
    if (m <= nz - 2) {
      float ez[VX], h[VX], e1[VX];
      ldf<T, VX>(Er + (m + 1) * P + c0, er1n, on, sc.ei);
      ldf<T, VX>(Ez + m * P + c0, ez, on, sc.ei);
      ldf<T, VX>(Hp + m * P + c0, h, on, sc.hi);
      right_of<VX>(ez, e1);
#pragma unroll
      for (int v = 0; v < VX; v++) h1[v] = live[v] ? h_node(h[v], er1n[v] - er_in[v], e1[v] - ez[v], d) : h[v];
      const float hl = __shfl_up(h1[VX - 1], 1);
#pragma unroll
      for (int v = 0; v < VX; v++) {
        er1[v] = live[v] && m >= 1 ? fmaf(-d.cb_dz, h1[v] - h1u_b[v], d.ca * er_in[v]) : er_in[v];
        const float hm = v > 0 ? h1[v - 1] : hl;
        ez1[v] = live[v] ? fmaf(-cm[v], hm, fmaf(cp[v], h1[v], d.ca * ez[v])) : ez[v];
      }
      sub_source<VX>(d, S1, m, c0, ez1);
      if (wall_wave) mur_r<VX>(d, vw, wall_here, ez1, ez);
      if (m == nz - 2) {  // stage-1 z = z_max wall row from the new row nz-2, kept in er1n
#pragma unroll
        for (int v = 0; v < VX; v++)
          er1n[v] = d.mur && live[v] ? fmaf(d.mur_kz, er1[v] - er1n[v], er_in[v]) : er1n[v];
      }
    } else {  // m == nz-1: only the E_r wall row, formed with row nz-2
#pragma unroll
      for (int v = 0; v < VX; v++) {
        er1[v] = er_in[v];
        ez1[v] = 0.f;
        h1[v] = 0.f;
        er1n[v] = 0.f;
      }
    }
    if (m == 1 && m0 == 0) {  // stage-1 z = 0 wall from the new row 1 (er1_b holds E_r^n(0))
#pragma unroll
      for (int v = 0; v < VX; v++)
        if (d.mur && live[v]) er1_b[v] = fmaf(d.mur_kz, er1[v] - er1_b[v], er_in[v]);
      as_stored<T, VX>(er1_b, sc.eo, mi_e);
#pragma unroll
      for (int v = 0; v < VX; v++) er1w0[v] = er1_b[v];
    }
    // stage-1 row m as the next step would read it from a stored level (its own E_r update above
    // used H unrounded, as a one-step launch does within its step)
    float h1u[VX];
#pragma unroll
    for (int v = 0; v < VX; v++) h1u[v] = h1[v];
    as_stored<T, VX>(er1, sc.eo, mi_e);
    as_stored<T, VX>(ez1, sc.eo, mi_e);
    as_stored<T, VX>(h1, sc.ho, mi_h);
    // ---- stage 2 (step n+1 -> n+2), row j = m-1
    const int j = m - 1;
    if (j >= max(0, k0 - 1)) {
      float e1[VX], h2[VX];
      right_of<VX>(ez1_b, e1);
#pragma unroll
      for (int v = 0; v < VX; v++) h2[v] = live[v] ? h_node(h1_b[v], er1[v] - er1_b[v], e1[v] - ez1_b[v], d) : h1_b[v];
      if (j >= k0) {
        const float hl = __shfl_up(h2[VX - 1], 1);
        float er2[VX], ez2[VX];
#pragma unroll
        for (int v = 0; v < VX; v++) {
          er2[v] = live[v] && j >= 1 ? fmaf(-d.cb_dz, h2[v] - h2_b[v], d.ca * er1_b[v]) : er1_b[v];
          const float hm = v > 0 ? h2[v - 1] : hl;
          ez2[v] = live[v] ? fmaf(-cm[v], hm, fmaf(cp[v], h2[v], d.ca * ez1_b[v])) : ez1_b[v];
        }
        sub_source<VX>(d, S2, j, c0, ez2);
        if (wall_wave) mur_r<VX>(d, vw, wall_here, ez2, ez1_b);
        stf<T, VX>(Hpo + j * P + c0, h2, outl, sc.ho);
        if (j >= 1) stf<T, VX>(Ero + j * P + c0, er2, outl, sc.eo);
        stf<T, VX>(Ezo + j * P + c0, ez2, outl, sc.eo);
        if (d.dyn && outl) {
          mx_h = amax<VX>(h2, mx_h);
          mx_e = amax<VX>(ez2, amax<VX>(er2, mx_e));
        }
        if (j == 1) {  // stage-2 z = 0 wall, with the stage-1 wall row kept since row 1
          float wv0[VX];
#pragma unroll
          for (int v = 0; v < VX; v++)
            wv0[v] = d.mur && live[v] ? fmaf(d.mur_kz, er2[v] - er1w0[v], er1_b[v]) : er1w0[v];
          stf<T, VX>(Ero + c0, wv0, outl, sc.eo);
          if (d.dyn && outl) mx_e = amax<VX>(wv0, mx_e);
        }
        if (j == nz - 2) {  // stage-2 z = z_max wall
          float wv1[VX];
#pragma unroll
          for (int v = 0; v < VX; v++) wv1[v] = d.mur && live[v] ? fmaf(d.mur_kz, er2[v] - er1[v], er1_b[v]) : er1[v];
          stf<T, VX>(Ero + (j + 1) * P + c0, wv1, outl, sc.eo);
          if (d.dyn && outl) mx_e = amax<VX>(wv1, mx_e);
        }
        // observer stencil nodes of the intermediate level on row j (and on row nz-1 with it)
        for (int pass = 0; pass < (j == nz - 2 ? 2 : 1); pass++) {
          const int row = pass ? nz - 1 : j;
          const int e_lo = d.row_ptr[row], e_hi = d.row_ptr[row + 1];
          for (int e = e_lo; e < e_hi; e++) {
            const int2 en = d.ent[e];  // (node, slot | comp << 30)
            const int rel = en.x - w0;
            const int L = rel / VX, cell = rel - L * VX;
            if (rel >= 0 && L == lane && outl) {
              const int comp = (unsigned)en.y >> 30;
              float val = 0.f;
#pragma unroll
              for (int v = 0; v < VX; v++)
                if (v == cell) val = comp ? ez1_b[v] : (pass ? er1[v] : er1_b[v]);
              samp[en.y & 0x3fffffff] = d.ent_w[e] * (double)val;
            }
          }
        }
      }
#pragma unroll
      for (int v = 0; v < VX; v++) h2_b[v] = h2[v];
    }
    // ---- shift
#pragma unroll
    for (int v = 0; v < VX; v++) {
      if (m <= nz - 2) er_in[v] = er1n[v];
      er1_b[v] = er1[v];
      ez1_b[v] = ez1[v];
      h1_b[v] = h1[v];
      h1u_b[v] = h1u[v];
    }
  }
  if (d.dyn) record_max(d, li, mx_e, mx_h, lane);
}

// Mur value of E_z on the r wall (rows 0..nz-2) for single-step tilings whose wall node starts a
// wave.
template <typename T>
__global__ void k_rz_mur_r(RDev d, int par, int li) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.nz - 1) return;
  const long long c0 = k * (long long)d.pitch + d.nr - 1, c1 = c0 - 1;
  const T *Ein = (const T *)d.f[par][1];
  T *Eout = (T *)d.f[par ^ 1][1];
  const float si = d.dyn ? 1.f / d.lvl_scale[2 * par] : 1.f / d.s_e;
  const float so = d.dyn ? d.lvl_scale[2 * (par ^ 1)] : d.s_e;
  const float e = fmaf(d.mur_kr, lds<T>(Eout + c1, 1.f / so) - lds<T>(Ein + c0, si), lds<T>(Ein + c1, si));
  Eout[c0] = from_f<T>(kF32<T> ? e : e * so);
  if (d.dyn) atomicMax(d.maxes + 2 * ((li + 1) % 3), __float_as_uint(fabsf(e)));
}

// The last launch's pending work, after the last step of a call.
template <typename T>
__global__ void __launch_bounds__(64) k_rz_finish(RDev d, int par, double *w, int gcol, int scol, int sb, int ld) {
  const float inv_e = d.dyn ? 1.f / d.lvl_scale[2 * par] : 1.f / d.s_e;
  pending_wave<T>(d, par, w, ld, gcol, scol, sb, blockIdx.x * 8, threadIdx.x, inv_e);
}

// Largest |E| and |H| of a level into maxes slot `slot` (dyn, after fields were set directly).
template <typename T>
__global__ void k_rz_levelmax(RDev d, int par, int slot) {
  const long long n = (long long)d.nz * d.pitch;
  const float ie = d.dyn ? 1.f / d.lvl_scale[2 * par] : 1.f, ih = d.dyn ? 1.f / d.lvl_scale[2 * par + 1] : 1.f;
  float me = 0.f, mh = 0.f;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x) {
    me = fmaxf(me, fmaxf(fabsf(lds<T>((const T *)d.f[par][0] + t, ie)), fabsf(lds<T>((const T *)d.f[par][1] + t, ie))));
    mh = fmaxf(mh, fabsf(lds<T>((const T *)d.f[par][2] + t, ih)));
  }
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) {
    me = fmaxf(me, __shfl_xor(me, k));
    mh = fmaxf(mh, __shfl_xor(mh, k));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(d.maxes + 2 * slot, __float_as_uint(me));
    atomicMax(d.maxes + 2 * slot + 1, __float_as_uint(mh));
  }
}

// Initial scales and maxima (reset): level slots scaled by 1 until a launch sets them.
__global__ void k_rz_init_scales(RDev d) {
  const int t = threadIdx.x;
  if (t < 4) d.lvl_scale[t] = 1.f;
  if (t < 6) d.maxes[t] = 0u;
}

__global__ void k_rz_clear_slot(RDev d, int slot) {
  if (threadIdx.x < 2) d.maxes[2 * slot + threadIdx.x] = 0u;
}

__global__ void k_rz_zero(uint4 *p, long long n) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
    p[t] = make_uint4(0u, 0u, 0u, 0u);
}

// Dense FP32 [nz][nr] physical values <-> a stored component of level `par`.
template <typename T>
__global__ void k_rz_copy(RDev d, int par, int comp, const float *src, float *dst, int to_dense) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int nr = d.nr;
  if (t >= (long long)nr * d.nz) return;
  const int i = (int)(t % nr);
  const long long k = t / nr;
  T *f = (T *)d.f[par][comp];
  const float s = d.dyn ? d.lvl_scale[2 * par + (comp == 2)] : (comp == 2 ? d.s_h : d.s_e);
  if (to_dense) dst[t] = lds<T>(f + k * d.pitch + i, 1.f / s);
  else f[k * d.pitch + i] = from_f<T>(kF32<T> ? src[t] : src[t] * s);
}

// ------------------------------------------------------------------ launchers
// Pending work a launch leaves for the next one: the level it wrote sampled into gcol, and the
// stencil samples of its intermediate level (buffer sb) summed into scol.
struct Pending {
  int gcol = -1, scol = -1, sb = 0;
};

// One launch: `two` steps (k_rz_step2) or one (k_rz_step, plus the r-wall Mur kernel in the
// wave-start tiling), launch index li since the reset.  Updates `pend` to what this launch leaves.
template <typename T>
hipError_t launch_rz_t(const chf_rz_plan &p, const RDev &d, int par, int step, bool two, const double *q,
                       double *w, int col, int ld, Pending &pend, int &samp_par, int li, hipStream_t s,
                       hipEvent_t ev_a, hipEvent_t ev_b) {
  hipError_t e = hipSuccess;
  if (ev_a) e = hipEventRecord(ev_a, s);
  if (e != hipSuccess) return e;
  const int gcol = w ? pend.gcol : -1, scol = w ? pend.scol : -1;
  const dim3 block(64 * p.wv);
  if (two) {
    const int sb_out = samp_par ^ 1;
    const dim3 grid(8 * ((p.n_blocks2 + d.n_gblocks + 7) / 8));
    if (p.vx == 4) k_rz_step2<T, 4><<<grid, block, 0, s>>>(d, par, step, q, w, gcol, scol, pend.sb, sb_out, ld, li);
    else k_rz_step2<T, 8><<<grid, block, 0, s>>>(d, par, step, q, w, gcol, scol, pend.sb, sb_out, ld, li);
    samp_par = sb_out;
    pend.scol = col;
    pend.sb = sb_out;
    pend.gcol = col + 1;
  } else {
    const dim3 grid(8 * ((p.n_blocks + d.n_gblocks + 7) / 8));
    switch (p.vx) {
      case 1: k_rz_step<T, 1><<<grid, block, 0, s>>>(d, par, step, q, w, gcol, scol, pend.sb, ld, li); break;
      case 2: k_rz_step<T, 2><<<grid, block, 0, s>>>(d, par, step, q, w, gcol, scol, pend.sb, ld, li); break;
      case 4: k_rz_step<T, 4><<<grid, block, 0, s>>>(d, par, step, q, w, gcol, scol, pend.sb, ld, li); break;
      default: k_rz_step<T, 8><<<grid, block, 0, s>>>(d, par, step, q, w, gcol, scol, pend.sb, ld, li); break;
    }
    pend.scol = -1;
    pend.gcol = col;
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ev_b) e = hipEventRecord(ev_b, s);
  if (e != hipSuccess) return e;
  if (!two && d.mur && p.mur_r_kernel) {
    k_rz_mur_r<T><<<(d.nz - 1 + 255) / 256, 256, 0, s>>>(d, par, li);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_rz(const chf_rz_plan &p, const RDev &d, int par, int step, bool two, const double *q, double *w,
                     int col, int ld, Pending &pend, int &samp_par, int li, hipStream_t s, hipEvent_t ev_a = nullptr,
                     hipEvent_t ev_b = nullptr) {
  switch (p.storage) {
    case CHF_BF16: return launch_rz_t<__hip_bfloat16>(p, d, par, step, two, q, w, col, ld, pend, samp_par, li, s, ev_a, ev_b);
    case CHF_FP16: return launch_rz_t<__half>(p, d, par, step, two, q, w, col, ld, pend, samp_par, li, s, ev_a, ev_b);
    default: return launch_rz_t<float>(p, d, par, step, two, q, w, col, ld, pend, samp_par, li, s, ev_a, ev_b);
  }
}

hipError_t launch_rz_finish(const chf_rz_plan &p, const RDev &d, int par, double *w, const Pending &pend, int ld,
                            hipStream_t s) {
  if (d.n_obs <= 0 || !w || (pend.gcol < 0 && pend.scol < 0)) return hipSuccess;
  const dim3 grid((d.n_obs + 7) / 8);
  switch (p.storage) {
    case CHF_BF16: k_rz_finish<__hip_bfloat16><<<grid, 64, 0, s>>>(d, par, w, pend.gcol, pend.scol, pend.sb, ld); break;
    case CHF_FP16: k_rz_finish<__half><<<grid, 64, 0, s>>>(d, par, w, pend.gcol, pend.scol, pend.sb, ld); break;
    default: k_rz_finish<float><<<grid, 64, 0, s>>>(d, par, w, pend.gcol, pend.scol, pend.sb, ld); break;
  }
  return hipGetLastError();
}

hipError_t launch_rz_zero(const chf_rz_plan &p, hipStream_t s) {
  // both levels of all three fields are contiguous from offset 0, plus the watchdog flag
  const long long n16 = (long long)(p.off_cp / 16);
  k_rz_zero<<<2048, 256, 0, s>>>((uint4 *)p.ws, n16);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_rz_zero<<<1, 64, 0, s>>>((uint4 *)(p.ws + p.off_nan), 16);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_rz_init_scales<<<1, 64, 0, s>>>(p.dev);
  return hipGetLastError();
}

// Maxima of the current level into the slot the next launch reads (dynamic scaling, after the
// fields were set directly).
hipError_t launch_rz_levelmax(const chf_rz_plan &p, hipStream_t s) {
  const int slot = p.li % 3;
  k_rz_clear_slot<<<1, 64, 0, s>>>(p.dev, slot);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (p.storage) {
    case CHF_BF16: k_rz_levelmax<__hip_bfloat16><<<1024, 256, 0, s>>>(p.dev, p.parity, slot); break;
    case CHF_FP16: k_rz_levelmax<__half><<<1024, 256, 0, s>>>(p.dev, p.parity, slot); break;
    default: k_rz_levelmax<float><<<1024, 256, 0, s>>>(p.dev, p.parity, slot); break;
  }
  return hipGetLastError();
}

}  // namespace

extern "C" {

chf_status chf_rz_plan_create(const chf_rz_grid *grid, const chf_medium *medium, const chf_rz_source *src,
                              const chf_rz_observers *obs, const chf_rz_exec *ex, chf_rz_plan **out) {
  if (!grid || !medium || !src || !obs || !ex || !out) return fail(CHF_EINVAL, "NULL descriptor");
  *out = nullptr;
  const chf_rz_grid &g = *grid;
  if (g.nr < 4 || g.nz < 4 || g.n_steps < 0) return fail(CHF_EINVAL, "need nr, nz >= 4 and n_steps >= 0");
  if (!(g.dr > 0) || !(g.dz > 0) || !(g.dt > 0) || !std::isfinite(g.dr) || !std::isfinite(g.dz) ||
      !std::isfinite(g.dt))
    return fail(CHF_EINVAL, "spacings and time step must be positive and finite");
  if (!(medium->eps_r > 0) || !(medium->mu_r > 0) || !(medium->sigma >= 0))
    return fail(CHF_EINVAL, "medium needs eps_r > 0, mu_r > 0, sigma >= 0");
  const double v = kC0 / std::sqrt(medium->eps_r * medium->mu_r);
  const double dt_max = 2.0 / (v * std::sqrt(kRadialEig / (g.dr * g.dr) + 4.0 / (g.dz * g.dz)));
  if (g.dt > dt_max) return fail(CHF_ECFL, "dt above the stability limit of the (r, z) lattice");
  if (ex->bc == CHF_BC_CPML) return fail(CHF_EUNSUPPORTED, "the (r, z) solver offers PEC and Mur walls");
  if (ex->bc != CHF_BC_PEC && ex->bc != CHF_BC_MUR1) return fail(CHF_EINVAL, "unknown boundary kind");
  const int vx = ex->vx ? ex->vx : 4, wv = ex->waves_per_block ? ex->waves_per_block : 4;
  const int zchunk = ex->z_chunk ? ex->z_chunk : 32;
  if (vx != 1 && vx != 2 && vx != 4 && vx != 8) return fail(CHF_EINVAL, "vx must be 1, 2, 4 or 8");
  if (wv != 1 && wv != 2 && wv != 4 && wv != 8) return fail(CHF_EINVAL, "waves_per_block must be 1, 2, 4 or 8");
  if (zchunk < 1) return fail(CHF_EINVAL, "z_chunk must be >= 1");
  const int spl = ex->steps_per_launch ? ex->steps_per_launch : (vx >= 4 ? 2 : 1);
  if (ex->storage != CHF_FP32 && ex->storage != CHF_BF16 && ex->storage != CHF_FP16)
    return fail(CHF_EINVAL, "unknown storage type");
  if (ex->dynamic_scaling && ex->storage != CHF_FP16)
    return fail(CHF_EINVAL, "dynamic scaling is for FP16 storage");
  if (!(ex->scale_e >= 0) || !(ex->scale_h >= 0)) return fail(CHF_EINVAL, "negative storage scale");
  if (spl != 1 && spl != 2) return fail(CHF_EINVAL, "steps_per_launch must be 1 or 2");
  if (spl == 2 && vx < 4) return fail(CHF_EINVAL, "two steps per launch need vx 4 or 8");
  const bool src_on = src->n_bins > 0;
  if (src->n_bins < 0) return fail(CHF_EINVAL, "n_bins < 0");
  if (src_on) {
    if (!src->q_bins) return fail(CHF_EINVAL, "q_bins is NULL");
    if (!(src->sigma_r > 0) || !(src->sigma_z > 0) || !(src->cut_sigmas > 0) || !(src->dz_bin > 0) ||
        !(src->beta > 0))
      return fail(CHF_EINVAL, "source widths, cut, bin width and beta must be positive");
    if (2.0 * src->cut_sigmas * src->sigma_z / g.dz + 2.0 > kRzMaxWz)
      return fail(CHF_EUNSUPPORTED, "longitudinal source support above 64 rows");
  }
  if (obs->n_obs < 0 || obs->n_obs > kRzMaxObs || (obs->n_obs > 0 && !obs->rz))
    return fail(CHF_EINVAL, "bad observer list");

  chf_rz_plan *p = new (std::nothrow) chf_rz_plan();
  if (!p) return fail(CHF_ENOMEM, "host allocation");
  p->g = g;
  p->med = *medium;
  p->src = *src;
  p->ex = *ex;
  p->vx = vx;
  p->wv = wv;
  p->zchunk = std::min(zchunk, g.nz - 1);
  p->pitch = (g.nr + 63) / 64 * 64;
  const uint64_t elems = (uint64_t)p->pitch * (uint64_t)g.nz;
  if (elems > (uint64_t(1) << 40)) {
    delete p;
    return fail(CHF_ENOMEM, "grid too large");
  }
  p->nrb = (g.nr + 64 * vx * wv - 1) / (64 * vx * wv);
  p->nzc = (g.nz - 1 + p->zchunk - 1) / p->zchunk;  // rows 0..nz-2 are marched
  if ((uint64_t)p->nrb * p->nzc > (uint64_t)0x7fffffff / 8) {
    delete p;
    return fail(CHF_EINVAL, "too many workgroups for this tile shape");
  }
  p->n_blocks = p->nrb * p->nzc;
  p->spl = spl;
  p->n_waves2 = (g.nr + 62 * vx - 1) / (62 * vx);
  p->nrb2 = (p->n_waves2 + wv - 1) / wv;
  p->n_blocks2 = p->nrb2 * p->nzc;
  if ((uint64_t)p->n_blocks2 > (uint64_t)0x7fffffff / 8) {
    delete p;
    return fail(CHF_EINVAL, "too many workgroups for this tile shape");
  }
  if (src_on) p->q_bins.assign(src->q_bins, src->q_bins + src->n_bins);
  else p->q_bins.assign(1, 0.0);

  // coefficients (FP64, rounded once)
  const double eps = kEps0 * medium->eps_r, mu = kMu0 * medium->mu_r;
  const double loss = medium->sigma * g.dt / (2.0 * eps);
  p->ca = (1.0 - loss) / (1.0 + loss);
  p->cb = (g.dt / eps) / (1.0 + loss);
  p->db = g.dt / mu;
  p->cp.assign(p->pitch, 0.f);
  p->cm.assign(p->pitch, 0.f);
  for (int i = 0; i <= g.nr - 2; i++) {
    const double a = i == 0 ? g.dr / 8.0 : i * g.dr;
    p->cp[i] = (float)(p->cb * (i + 0.5) * g.dr / (a * g.dr));
    p->cm[i] = i == 0 ? 0.f : (float)(p->cb * (i - 0.5) * g.dr / (a * g.dr));
  }
  // radial source weights on the E_z nodes 0..nr-2, normalised with the ring areas
  if (src_on) {
    std::vector<double> gr;
    double norm = 0.0;
    for (int i = 0; i <= g.nr - 2; i++) {
      const double r = i * g.dr;
      if (r > src->cut_sigmas * src->sigma_r) break;
      const double x = std::exp(-0.5 * (r / src->sigma_r) * (r / src->sigma_r));
      const double a = i == 0 ? g.dr / 8.0 : r;
      gr.push_back(x);
      norm += x * 2.0 * kPi * a * g.dr;
    }
    for (double &x : gr) x /= norm;
    p->wr = gr;
    p->n_src = (int)gr.size();
  }
  if (p->wr.empty()) p->wr.assign(1, 0.0);

  // observers: base node and fractions of the bilinear stencils
  p->oidx.assign(std::max(1, obs->n_obs) * 4, 0);
  p->ot.assign(std::max(1, obs->n_obs) * 4, 0.0);
  for (int o = 0; o < obs->n_obs; o++) {
    const double r = obs->rz[2 * o], z = obs->rz[2 * o + 1];
    if (!std::isfinite(r) || !std::isfinite(z)) {
      delete p;
      return fail(CHF_EINVAL, "non-finite observer position");
    }
    for (int c = 0; c < 2; c++) {
      const double fr = r / g.dr - (c == 0 ? 0.5 : 0.0);
      const double fz = z / g.dz - (c == 1 ? 0.5 : 0.0);
      const double i0 = std::floor(fr), k0 = std::floor(fz);
      // E_r lives on nodes i <= nr-2, rows 0..nz-1; E_z on nodes 0..nr-1, rows 0..nz-2
      const double imax = c == 0 ? g.nr - 3 : g.nr - 2, kmax = c == 0 ? g.nz - 2 : g.nz - 3;
      if (!(i0 >= 0 && i0 <= imax && k0 >= 0 && k0 <= kmax)) {
        delete p;
        return fail(CHF_EDOMAIN, "observer stencil outside the (r, z) lattice");
      }
      p->oidx[(o * 2 + c) * 2] = (int)i0;
      p->oidx[(o * 2 + c) * 2 + 1] = (int)k0;
      p->ot[(o * 2 + c) * 2] = fr - i0;
      p->ot[(o * 2 + c) * 2 + 1] = fz - k0;
    }
  }

  // observer stencil nodes by row (slot = (o*2 + comp)*4 + corner, corner = a + 2b, the order in
  // which the gather adds them), for the intermediate level of two-step launches
  {
    std::vector<std::vector<int>> rows_i(g.nz), rows_s(g.nz);
    std::vector<std::vector<double>> rows_w(g.nz);
    for (int o = 0; o < obs->n_obs; o++)
      for (int c = 0; c < 2; c++)
        for (int corner = 0; corner < 4; corner++) {
          const int a = corner & 1, b = corner >> 1;
          const double tr = p->ot[(o * 2 + c) * 2], tz = p->ot[(o * 2 + c) * 2 + 1];
          const int k = p->oidx[(o * 2 + c) * 2 + 1] + b;
          rows_i[k].push_back(p->oidx[(o * 2 + c) * 2] + a);
          rows_s[k].push_back(((o * 2 + c) * 4 + corner) | (c << 30));
          rows_w[k].push_back((a ? tr : 1.0 - tr) * (b ? tz : 1.0 - tz));
        }
    p->row_ptr.assign(g.nz + 1, 0);
    for (int k = 0; k < g.nz; k++) {
      p->row_ptr[k + 1] = p->row_ptr[k] + (int)rows_i[k].size();
      for (size_t e = 0; e < rows_i[k].size(); e++) {
        p->ent.push_back(rows_i[k][e]);
        p->ent.push_back(rows_s[k][e]);
        p->ent_w.push_back(rows_w[k][e]);
      }
    }
    if (p->ent.empty()) {
      p->ent.assign(2, 0);
      p->ent_w.assign(1, 0.0);
    }
  }

  // workspace layout: 6 field arrays first (zeroed together), then the tables
  p->storage = ex->storage;
  p->elem = ex->storage == CHF_FP32 ? 4 : 2;
  const uint64_t fbytes = align256(elems * (uint64_t)p->elem);
  uint64_t off = 0;
  for (int l = 0; l < 2; l++)
    for (int c = 0; c < 3; c++) {
      p->off_f[l][c] = off;
      off += fbytes;
    }
  p->field_bytes = off;
  p->off_cp = off;
  off = align256(off + p->cp.size() * sizeof(float));
  p->off_cm = off;
  off = align256(off + p->cm.size() * sizeof(float));
  p->off_wr = off;
  off = align256(off + p->wr.size() * sizeof(double));
  p->off_q = off;
  off = align256(off + p->q_bins.size() * sizeof(double));
  p->off_oidx = off;
  off = align256(off + p->oidx.size() * sizeof(int));
  p->off_ot = off;
  off = align256(off + p->ot.size() * sizeof(double));
  p->off_nan = off;
  off = align256(off + 256);
  p->off_scale = off;  // level scales [2][2] floats, then maxima [3][2] uints
  off = align256(off + 64);
  p->off_rowptr = off;
  off = align256(off + p->row_ptr.size() * sizeof(int));
  p->off_ent = off;
  off = align256(off + p->ent.size() * sizeof(int));
  p->off_entw = off;
  off = align256(off + p->ent_w.size() * sizeof(double));
  p->off_samp = off;
  off = align256(off + 2 * 8 * (size_t)std::max(1, obs->n_obs) * sizeof(double));
  p->ws_bytes = off;

  RDev &D = p->dev;
  D.nr = g.nr;
  D.nz = g.nz;
  D.pitch = p->pitch;
  D.zchunk = p->zchunk;
  D.nrb = p->nrb;
  D.n_blocks = p->n_blocks;
  D.wv = wv;
  D.n_gblocks = (obs->n_obs + 8 * wv - 1) / (8 * wv);
  D.nrb2 = p->nrb2;
  D.n_waves2 = p->n_waves2;
  D.n_blocks2 = p->n_blocks2;
  p->mur_r_kernel = ex->bc == CHF_BC_MUR1 && (g.nr - 1) % (64 * vx) == 0;
  D.ca = (float)p->ca;
  D.db_dr = (float)(p->db / g.dr);
  D.db_dz = (float)(p->db / g.dz);
  D.cb_dz = (float)(p->cb / g.dz);
  D.src_on = src_on ? 1 : 0;
  D.n_bins = src_on ? src->n_bins : 0;
  D.n_src = p->n_src;
  D.z_entry = src->z_entry;
  D.t_entry = src->t_entry;
  D.v_src = src->beta * kC0;
  D.sigma_z = src->sigma_z;
  D.cut_sigmas = src->cut_sigmas;
  D.z_bin0 = src->z_bin0;
  D.dz_bin = src->dz_bin;
  D.dz = g.dz;
  D.dt = g.dt;
  D.cb = p->cb;
  D.mur = ex->bc == CHF_BC_MUR1;
  // storage scales: stored = scale * physical.  H is kept at the power of two nearest the wave
  // impedance times the E scale; FP16 puts the Coulomb field of the largest bin charge at one
  // radial width near 2^14 (static), or rescales every launch (dynamic).
  {
    const double eta = std::sqrt(mu / eps);
    const double pow2_eta = std::ldexp(1.0, (int)std::lround(std::log2(eta)));
    double se = 1.0;
    if (ex->storage == CHF_FP16 && src_on) {
      double qmax = 0.0;
      for (double qv : p->q_bins) qmax = std::max(qmax, std::fabs(qv));
      const double e_est = qmax / (4.0 * kPi * eps * src->sigma_r * src->sigma_r);
      if (e_est > 0) se = std::ldexp(1.0, (int)std::floor(std::log2(16384.0 / e_est)));
    }
    if (ex->scale_e > 0) se = ex->scale_e;
    const double sh = ex->scale_h > 0 ? ex->scale_h : se * pow2_eta;
    p->scale_e = ex->storage == CHF_FP32 ? 1.0 : se;
    p->scale_h = ex->storage == CHF_FP32 ? 1.0 : sh;
    D.s_e = (float)p->scale_e;
    D.s_h = (float)p->scale_h;
    D.dyn = ex->dynamic_scaling ? 1 : 0;
    double gmax = 2.0 * p->cb / g.dz;
    for (int i = 0; i <= g.nr - 2; i++) gmax = std::max(gmax, (double)p->cp[i] + (double)p->cm[i]);
    D.ge = (float)gmax;
    D.gh = (float)(2.0 * (p->db / g.dr + p->db / g.dz));
    D.target = 16384.f;
    D.src_bound = src_on ? p->cb * src->beta * kC0 * p->wr[0] *
                               std::exp(g.dz * g.dz / (8.0 * src->sigma_z * src->sigma_z)) / g.dz
                         : 0.0;
  }
  D.mur_kr = (float)((v * g.dt - g.dr) / (v * g.dt + g.dr));
  D.mur_kz = (float)((v * g.dt - g.dz) / (v * g.dt + g.dz));
  D.n_obs = obs->n_obs;
  *out = p;
  return CHF_OK;
}

void chf_rz_plan_destroy(chf_rz_plan *p) {
  if (!p) return;
  if (p->graph) (void)hipGraphExecDestroy(p->graph);
  delete p;
}

chf_status chf_rz_workspace_bytes(const chf_rz_plan *p, uint64_t *bytes) {
  if (!p || !bytes) return fail(CHF_EINVAL, "NULL argument");
  *bytes = p->ws_bytes;
  return CHF_OK;
}

chf_status chf_rz_reset(chf_rz_plan *p, void *stream) {
  if (!p) return fail(CHF_EINVAL, "NULL plan");
  if (!p->ws) return fail(CHF_ESTATE, "no workspace bound");
  hipError_t e = launch_rz_zero(*p, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "reset");
  p->parity = 0;
  p->n_done = 0;
  p->li = 0;
  return CHF_OK;
}

chf_status chf_rz_bind_workspace(chf_rz_plan *p, void *dev_ptr, uint64_t bytes, void *stream) {
  if (!p || !dev_ptr) return fail(CHF_EINVAL, "NULL argument");
  if (bytes < p->ws_bytes) return fail(CHF_ENOMEM, "workspace smaller than chf_rz_workspace_bytes");
  if ((uintptr_t)dev_ptr % 256) return fail(CHF_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)dev_ptr;
  p->ws = ws;
  RDev &D = p->dev;
  D.cp = (const float *)(ws + p->off_cp);
  D.cm = (const float *)(ws + p->off_cm);
  D.wr = (const double *)(ws + p->off_wr);
  D.q_bins = (const double *)(ws + p->off_q);
  D.obs_idx = (const int *)(ws + p->off_oidx);
  D.obs_t = (const double *)(ws + p->off_ot);
  D.nan_flag = (int *)(ws + p->off_nan);
  D.row_ptr = (const int *)(ws + p->off_rowptr);
  D.ent = (const int2 *)(ws + p->off_ent);
  D.ent_w = (const double *)(ws + p->off_entw);
  D.samp = (double *)(ws + p->off_samp);
  D.lvl_scale = (float *)(ws + p->off_scale);
  D.maxes = (unsigned *)(ws + p->off_scale + 16);
  for (int l = 0; l < 2; l++)
    for (int c = 0; c < 3; c++) D.f[l][c] = ws + p->off_f[l][c];
  struct Up {
    uint64_t off;
    const void *src;
    size_t n;
  } ups[] = {
      {p->off_cp, p->cp.data(), p->cp.size() * sizeof(float)},
      {p->off_cm, p->cm.data(), p->cm.size() * sizeof(float)},
      {p->off_wr, p->wr.data(), p->wr.size() * sizeof(double)},
      {p->off_q, p->q_bins.data(), p->q_bins.size() * sizeof(double)},
      {p->off_oidx, p->oidx.data(), p->oidx.size() * sizeof(int)},
      {p->off_ot, p->ot.data(), p->ot.size() * sizeof(double)},
      {p->off_rowptr, p->row_ptr.data(), p->row_ptr.size() * sizeof(int)},
      {p->off_ent, p->ent.data(), p->ent.size() * sizeof(int)},
      {p->off_entw, p->ent_w.data(), p->ent_w.size() * sizeof(double)},
  };
  for (const Up &u : ups) {
    hipError_t e = hipMemcpyAsync(ws + u.off, u.src, u.n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "upload of plan tables");
  }
  if (p->graph) {
    (void)hipGraphExecDestroy(p->graph);
    p->graph = nullptr;
  }
  return chf_rz_reset(p, stream);
}

static chf_status rz_forward(chf_rz_plan *p, void *stream, const double *q, double *w, int32_t n_steps,
                             int32_t first_column, int32_t ld, std::vector<hipEvent_t> *ev, int *n_launches = nullptr) {
  if (!p) return fail(CHF_EINVAL, "NULL plan");
  if (!p->ws) return fail(CHF_ESTATE, "no workspace bound");
  if (n_steps < 0 || first_column < 0) return fail(CHF_EINVAL, "negative step count or column");
  if (p->dev.n_obs > 0 && w && ld < first_column + n_steps)
    return fail(CHF_EINVAL, "ld_steps too small for first_column + n_steps");
  RDev d = p->dev;
  if (!p->ex.nan_watch) d.nan_flag = nullptr;
  hipStream_t s = (hipStream_t)stream;
  Pending pend;  // each launch samples its predecessor's results
  for (int t = 0, li = 0; t < n_steps; li++) {
    const bool two = p->spl == 2 && t + 1 < n_steps;
    hipError_t e = launch_rz(*p, d, p->parity, p->n_done, two, q, w, first_column + t, ld, pend, p->samp_par,
                             p->li, s, ev ? (*ev)[2 * li] : nullptr, ev ? (*ev)[2 * li + 1] : nullptr);
    if (e != hipSuccess) return hip_fail(e, "step launch");
    p->li++;
    p->parity ^= 1;
    p->n_done += two ? 2 : 1;
    t += two ? 2 : 1;
    if (n_launches) *n_launches = li + 1;
  }
  hipError_t e = launch_rz_finish(*p, d, p->parity, w, pend, ld, s);
  if (e != hipSuccess) return hip_fail(e, "gather launch");
  return CHF_OK;
}

chf_status chf_rz_forward(chf_rz_plan *p, void *stream, const double *q, double *w, int32_t n_steps,
                          int32_t first_column, int32_t ld) {
  return rz_forward(p, stream, q, w, n_steps, first_column, ld, nullptr);
}

chf_status chf_rz_forward_timed(chf_rz_plan *p, void *stream, const double *q, double *w, int32_t n_steps,
                                int32_t first_column, int32_t ld, double *sweep_ms) {
  if (!p || !sweep_ms) return fail(CHF_EINVAL, "NULL argument");
  if (n_steps < 0) return fail(CHF_EINVAL, "negative step count");
  *sweep_ms = 0.0;
  std::vector<hipEvent_t> ev(2 * (size_t)n_steps, nullptr);
  hipError_t e = hipSuccess;
  for (size_t t = 0; t < ev.size() && e == hipSuccess; t++) e = hipEventCreate(&ev[t]);
  chf_status st = CHF_OK;
  int launches = 0;
  if (e == hipSuccess) st = rz_forward(p, stream, q, w, n_steps, first_column, ld, &ev, &launches);
  if (e == hipSuccess && st == CHF_OK) e = hipStreamSynchronize((hipStream_t)stream);
  double total = 0.0;
  for (int t = 0; t < launches && e == hipSuccess && st == CHF_OK; t++) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, ev[2 * t], ev[2 * t + 1]);
    total += ms;
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (st != CHF_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "timed forward");
  *sweep_ms = total;
  return CHF_OK;
}

chf_status chf_rz_forward_graph(chf_rz_plan *p, void *stream, const double *q, double *w) {
  if (!p) return fail(CHF_EINVAL, "NULL plan");
  if (!p->ws) return fail(CHF_ESTATE, "no workspace bound");
  hipStream_t s = (hipStream_t)stream;
  const int T = p->g.n_steps;
  if (!p->graph || p->graph_w != w || p->graph_q != q) {
    if (p->graph) {
      (void)hipGraphExecDestroy(p->graph);
      p->graph = nullptr;
    }
    hipStream_t cs;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return hip_fail(e, "begin capture");
    }
    RDev d = p->dev;
    if (!p->ex.nan_watch) d.nan_flag = nullptr;
    hipError_t le = launch_rz_zero(*p, cs);
    int par = 0, sp = p->samp_par, li = 0;
    Pending pend;
    for (int t = 0; t < T && le == hipSuccess;) {
      const bool two = p->spl == 2 && t + 1 < T;
      le = launch_rz(*p, d, par, t, two, q, w, t, T, pend, sp, li, cs);
      par ^= 1;
      li++;
      t += two ? 2 : 1;
    }
    if (le == hipSuccess) le = launch_rz_finish(*p, d, par, w, pend, T, cs);
    hipGraph_t gr = nullptr;
    e = hipStreamEndCapture(cs, &gr);
    (void)hipStreamDestroy(cs);
    if (le != hipSuccess) {
      if (gr) (void)hipGraphDestroy(gr);
      return hip_fail(le, "captured launch");
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    e = hipGraphInstantiate(&p->graph, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) {
      p->graph = nullptr;
      return hip_fail(e, "graph instantiate");
    }
    p->graph_w = w;
    p->graph_q = q;
  }
  hipError_t e = hipGraphLaunch(p->graph, s);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  const int launches = p->spl == 2 ? T / 2 + (T & 1) : T;
  p->parity = launches & 1;
  p->n_done = T;
  p->li = launches;
  return CHF_OK;
}

chf_status chf_rz_sync(chf_rz_plan *p, void *stream) {
  if (!p) return fail(CHF_EINVAL, "NULL plan");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "pending error");
  if (p->ws && p->ex.nan_watch) {
    int flag = 0;
    e = hipMemcpy(&flag, p->dev.nan_flag, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read watchdog flag");
    if (flag) return fail(CHF_ENAN, "non-finite waveform value");
  }
  return CHF_OK;
}

static chf_status rz_copy(chf_rz_plan *p, void *stream, int comp, const float *src, float *dst, int to_dense) {
  if (!p || comp < 0 || comp > 2 || !(to_dense ? (const void *)dst : (const void *)src))
    return fail(CHF_EINVAL, "bad argument");
  if (!p->ws) return fail(CHF_ESTATE, "no workspace bound");
  const long long n = (long long)p->g.nr * p->g.nz;
  if ((n + 255) / 256 > 0x7fffffffLL) return fail(CHF_EUNSUPPORTED, "field too large to copy in one launch");
  hipStream_t s = (hipStream_t)stream;
  const unsigned g = (unsigned)((n + 255) / 256);
  switch (p->storage) {
    case CHF_BF16: k_rz_copy<__hip_bfloat16><<<g, 256, 0, s>>>(p->dev, p->parity, comp, src, dst, to_dense); break;
    case CHF_FP16: k_rz_copy<__half><<<g, 256, 0, s>>>(p->dev, p->parity, comp, src, dst, to_dense); break;
    default: k_rz_copy<float><<<g, 256, 0, s>>>(p->dev, p->parity, comp, src, dst, to_dense); break;
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && !to_dense && p->dev.dyn) e = launch_rz_levelmax(*p, s);
  return e == hipSuccess ? CHF_OK : hip_fail(e, "field copy");
}

chf_status chf_rz_get_field(chf_rz_plan *p, void *stream, int32_t comp, float *out_dev) {
  return rz_copy(p, stream, comp, nullptr, out_dev, 1);
}

chf_status chf_rz_set_field(chf_rz_plan *p, void *stream, int32_t comp, const float *in_dev) {
  return rz_copy(p, stream, comp, in_dev, nullptr, 0);
}

chf_status chf_rz_get_info(const chf_rz_plan *p, chf_rz_info *info) {
  if (!p || !info) return fail(CHF_EINVAL, "NULL argument");
  info->vx = p->vx;
  info->waves_per_block = p->wv;
  info->z_chunk = p->zchunk;
  info->pitch = p->pitch;
  info->n_blocks = p->n_blocks;
  info->n_src = p->n_src;
  info->steps_per_launch = p->spl;
  info->storage = p->storage;
  info->dynamic_scaling = p->dev.dyn;
  info->pad0 = 0;
  info->scale_e = p->scale_e;
  info->scale_h = p->scale_h;
  info->field_bytes = p->field_bytes;
  info->workspace_bytes = p->ws_bytes;
  info->bytes_per_cell_update = 6.0 * p->elem;  // read E_r, E_z, H; write all three
  return CHF_OK;
}

}  // extern "C"
