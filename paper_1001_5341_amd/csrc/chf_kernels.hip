// HIP kernels of libchfdtd for gfx950 (CDNA4, wave64).
//
// Step n reads time level `par` (E^n, H^{n-1/2}) and writes level par^1 (H^{n+1/2},
// E^{n+1}); both levels live in HBM, so a single sweep can recompute tile halos from the
// untouched input level without racing neighbouring workgroups.
//
// Per-node arithmetic (FP32, explicit fmaf, built with -ffp-contract=off) lives in h_plain /
// e_plain / add_layers / pml_psi and is applied in one fixed order by every sweep variant, so
// the fused single sweep and the split E/H sweeps produce identical bits.
//
//   H (Faraday, forward differences of E):
//     Hx += -chy*(Ez[j+1]-Ez[j]) + chz*(Ey[k+1]-Ey[k])   (- psi_y + psi_z in the CPML)
//     Hy += -chz*(Ex[k+1]-Ex[k]) + chx*(Ez[i+1]-Ez[i])
//     Hz += -chx*(Ey[i+1]-Ey[i]) + chy*(Ex[j+1]-Ex[j])
//   E (Ampere with sigma, backward differences of H):
//     Ex = ca*Ex + cey*(Hz[j]-Hz[j-1]) - cez*(Hy[k]-Hy[k-1])   (+ psi_y - psi_z)
//     Ey = ca*Ey + cez*(Hx[k]-Hx[k-1]) - cex*(Hz[i]-Hz[i-1])
//     Ez = ca*Ez + cex*(Hy[i]-Hy[i-1]) - cey*(Hx[j]-Hx[j-1])
//   with chu = Db/(du kappa_u) and ceu = Cb/(du kappa_u) folded with the storage scales, and
//   the CFS-CPML recursion psi <- b psi + a d  (a prescaled the same way).
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "chf_cell.h"
#include "chf_internal.h"

namespace chf {

__device__ __forceinline__ long long psi_index(const Dev &d, int u, int i, int j, int k, int s) {
  if (u == 0) return ((long long)k * d.ny + j) * d.np2 + s;
  if (u == 1) return ((long long)k * d.np2 + s) * d.pitch + i;
  return ((long long)s * d.ny + j) * d.pitch + i;
}

// One stretched-derivative psi update.  Reads `in`, writes `out` when `wr`.
__device__ __forceinline__ float psi_step(const Dev &d, const float *in, float *out, bool wr, int u,
                                          int i, int j, int k, int s, float a, float b, float dd) {
  long long id = psi_index(d, u, i, j, k, s);
  float p = pml_psi(in[id], a, b, dd);
  if (wr) out[id] = p;
  return p;
}

// psi of an H node term along axis u at position pos (H-update tables, half positions)
__device__ __forceinline__ float psi_h(const Dev &d, const float *in, float *out, bool wr, int u, int pos,
                                       int i, int j, int k, int s, float dd) {
  return psi_step(d, in, out, wr, u, i, j, k, s, d.ax[u].ah[pos], d.ax[u].bh[pos], dd);
}

// psi of an E node term along axis u (E-update tables, integer positions), updated in place
__device__ __forceinline__ float psi_e(const Dev &d, float *p, int u, int pos, int i, int j, int k, int s,
                                       float dd) {
  return psi_step(d, p, p, true, u, i, j, k, s, d.ax[u].ae[pos], d.ax[u].be[pos], dd);
}

// --------------------------------------------------------------- fused sweep
// One Yee step in a single pass over the fields: a workgroup owns W consecutive y rows of the
// full x extent (64 lanes x VX nodes per row, nx <= 64 VX) and marches a z chunk, updating H
// then E plane by plane.  Each wave loads only its own row (E at k+1, H at k: 6 vector loads
// per plane); the y neighbours it needs -- Ex, Ez of the row above for H, Hx, Hz of the row
// below for E -- come from the neighbouring waves through LDS, with two barriers per plane.
// One extra wave per workgroup computes the H row below the tile (read by the tile's first
// row) and stores nothing.  x neighbours move between lanes with shuffles.  Plane base
// pointers are wave-uniform and in-plane offsets 32-bit.  Workgroups are ordered so that
// consecutive logical tiles (neighbours in y, then in z) land on the same XCD and share its L2.
//
// k_fused covers the rectangle of tiles whose rows and planes (and the row and plane below
// them) lie clear of the walls and of the y/z layers: every node takes the unmasked update,
// lanes holding x-layer nodes add the x CPML term, x-wall / padding nodes keep their old
// values.  k_fused_gen covers the remaining tiles from a table, with the wall masks of every
// component and the y/z CPML terms (uniform per row and per plane).  Both apply the canonical
// per-node sequence, as the split sweeps do.
// G = 0: the interior rectangle (no wall and no y/z layer in reach; x walls and the x layer are
// per-lane fix-ups).  G = 1: boundary tiles whose planes lie in the interior z range (y walls
// and y layers: masks and terms uniform per row).  G = 2: any tile, adding the z walls and the
// z layers (uniform per plane).
// XS = 2: rows of up to 512 nodes split across two waves of 64 VX nodes each (the x neighbour
// across the split comes through LDS words published with the row exchange).
// DYN: dynamically scaled FP16 levels -- the step is computed in the units of the level read and
// every value stored (fields and psi) is multiplied by the launch's power of two r on the way
// out; the wave's largest stored magnitudes raise the written level's maxima.
template <typename T, int VX, int W, int G, bool PREFETCH = false, int XS = 1, bool DYN = false>
__device__ __forceinline__ void fused_body(const Dev &d, int ty, int zc, int zchunk, int par) {
  // Wave r of the workgroup owns row j = j0 - 1 + r: r = 1..W are the tile's rows, r = 0 is
  // the row below the tile, whose H the E update of row j0 needs (it computes H only and
  // stores nothing; the tile below owns that row).  Rows exchange through LDS:
  //   sEx/sEz slot s: Ex, Ez(k) of row j0 - 1 + s (s = 1..W+1; the top wave also loads row
  //   j0 + W), read by the row below for its H update;
  //   sHx/sHz slot s: Hx, Hz^{n+1/2}(k) of row j0 - 1 + s (s = 0..W-1), read by the row above
  //   for its E update.
  // Two barriers per plane.  Per plane a wave loads only its own row (6 vector loads), so the
  // registers that wait on HBM hold no duplicated data.
  constexpr int NL = 64 * VX * XS;
  __shared__ float sEx[W + 2][NL], sEz[W + 2][NL], sHx[W][NL], sHz[W][NL];
  // split rows: (Ey, Ez) of the first node of each wave's segment (E(k) of the own row), and
  // (Hy, Hz) of its last node (H^{n+1/2}(k)), per row
  __shared__ float sBE[W + 1][XS][2], sBH[W + 1][XS][2];
  __shared__ float sTab[8][NL];  // per x node: ch, ce, ah, bh, ae, be, x-slab index (H, E)
  // x-slab psi of the own row (H: Hy, Hz terms; E: Ey, Ez terms), staged so that both the
  // loads and the stores of a row's slab are one contiguous value per lane; the node that owns
  // slab index s replaces its value in place
  __shared__ float sPsi[(W + 1) * XS][4][kMaxFusedLayer];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int r = wv / XS, xs = wv - r * XS;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const int j0 = ty * W - d.ysh;
  const int j = j0 - 1 + r;
  constexpr bool GY = G >= 1, GZ = G >= 2;
  const bool act = !GY || (j >= 0 && j < ny);  // row exists (always, in the interior rectangle)
  const int jc = G ? min(max(j, 0), ny - 1) : j;
  const bool own = r > 0 && act, top = r == W;
  const bool top_ld = top && (!GY || j + 1 < ny);
  const int k0 = max(zc * zchunk - d.zsh, 0), k1 = min(zc * zchunk - d.zsh + zchunk, nz);
  const int ib = xs * 64 * VX + lane * VX;
  const bool on = ib < nx && act;
  // x-slab psi slots this wave writes back: those whose node lies in its segment
  bool own_sh = true, own_se = true;
  if constexpr (XS > 1) {
    if (lane < d.np2) {
      const int npml = d.npml;
      const int nh = lane < npml ? lane : lane - npml + (nx - 1 - npml);
      const int ne = lane < npml ? lane : lane - npml + (nx - npml);
      own_sh = nh / (64 * VX) == xs;
      own_se = ne / (64 * VX) == xs;
    }
  }
  const unsigned esz = (unsigned)sizeof(T);
  const unsigned o0 = ((unsigned)jc * (unsigned)d.pitch + (unsigned)ib) * esz;  // own row
  const unsigned op = ((unsigned)min(jc + 1, ny - 1) * (unsigned)d.pitch + (unsigned)ib) * esz;  // row above
  const long long plane = d.plane;
  const int np2 = d.np2;
  const T *Ei0 = (const T *)d.e[par][0], *Ei1 = (const T *)d.e[par][1], *Ei2 = (const T *)d.e[par][2];
  const T *Hi0 = (const T *)d.h[par][0], *Hi1 = (const T *)d.h[par][1], *Hi2 = (const T *)d.h[par][2];
  T *Eo0 = (T *)d.e[par ^ 1][0], *Eo1 = (T *)d.e[par ^ 1][1], *Eo2 = (T *)d.e[par ^ 1][2];
  T *Ho0 = (T *)d.h[par ^ 1][0], *Ho1 = (T *)d.h[par ^ 1][1], *Ho2 = (T *)d.h[par ^ 1][2];
  const float *phi0 = d.psi_h[par][0][0], *phi1 = d.psi_h[par][0][1];
  float *pho0 = d.psi_h[par ^ 1][0][0], *pho1 = d.psi_h[par ^ 1][0][1];
  float *pe0 = d.psi_e[0][0], *pe1 = d.psi_e[0][1];
  float dyn_r = 1.f, dyn_me = 0.f, dyn_mh = 0.f;
  if constexpr (DYN) dyn_r = ldexpf(1.f, dyn_shift(d, par, 1));

  for (int i = threadIdx.x; i < NL; i += 64 * (W + 1) * XS) {
    const int ic = min(i, nx - 1);
    const bool lay = np2 > 0 && i < nx;
    sTab[0][i] = d.ax[0].ch[ic];
    sTab[1][i] = d.ax[0].ce[ic];
    sTab[2][i] = lay ? d.ax[0].ah[i] : 0.f;
    sTab[3][i] = lay ? d.ax[0].bh[i] : 0.f;
    sTab[4][i] = lay ? d.ax[0].ae[i] : 0.f;
    sTab[5][i] = lay ? d.ax[0].be[i] : 0.f;
    sTab[6][i] = __int_as_float(lay ? d.ax[0].sh[i] : -1);
    sTab[7][i] = __int_as_float(lay ? d.ax[0].se[i] : -1);
  }
  // lanes holding x walls, padding or x-layer nodes take the fix-up paths below
  bool xfix = ib == 0 || ib + VX - 1 >= nx - 1;
  if (np2 > 0) {
#pragma unroll
    for (int v = 0; v < VX; v++) {
      const int i = ib + v;
      xfix = xfix || (i < nx && (d.ax[0].sh[i] >= 0 || d.ax[0].se[i] >= 0));
    }
  }
  const float chy = d.ax[1].ch[jc], cey = d.ax[1].ce[jc];
  // y layer and wall masks of the own row (uniform per wave)
  const int shy = GY && np2 > 0 ? d.ax[1].sh[jc] : -1, sey = GY && np2 > 0 ? d.ax[1].se[jc] : -1;
  const float ahy = shy >= 0 ? d.ax[1].ah[jc] : 0.f, bhy = shy >= 0 ? d.ax[1].bh[jc] : 0.f;
  const float aey = sey >= 0 ? d.ax[1].ae[jc] : 0.f, bey = sey >= 0 ? d.ax[1].be[jc] : 0.f;
  const bool jh = !GY || j <= ny - 2;               // Hx, Hz have their y difference
  const bool je = !GY || (j >= 1 && j <= ny - 2);   // Ex, Ez are not tangential to a y wall
  __syncthreads();  // sTab

  // E(k0) of the own row (and, for the top wave, Ex, Ez of the row above the tile)
  float exc[VX], eyc[VX], ezc[VX], etx[VX], etz[VX];
  ld_at<T, VX>(Ei0 + k0 * plane, o0, exc, on);
  ld_at<T, VX>(Ei1 + k0 * plane, o0, eyc, on);
  ld_at<T, VX>(Ei2 + k0 * plane, o0, ezc, on);
  ld_at<T, VX>(Ei0 + k0 * plane, op, etx, on && top_ld);
  ld_at<T, VX>(Ei2 + k0 * plane, op, etz, on && top_ld);

  // Hx, Hy^{n+1/2}(k0-1) of the own row, for the backward z differences of the first plane
  float hxp[VX], hyp[VX];
  if (k0 > 0 && own) {
    const int km = k0 - 1;
    float ex_[VX], ey_[VX], ez_[VX], ezu[VX], hxo[VX], hyo[VX];
    ld_at<T, VX>(Ei0 + km * plane, o0, ex_, on);
    ld_at<T, VX>(Ei1 + km * plane, o0, ey_, on);
    ld_at<T, VX>(Ei2 + km * plane, o0, ez_, on);
    ld_at<T, VX>(Ei2 + km * plane, op, ezu, on);
    ld_at<T, VX>(Hi0 + km * plane, o0, hxo, on);
    ld_at<T, VX>(Hi1 + km * plane, o0, hyo, on);
    const float chz = d.ax[2].ch[km];
    const int shz = np2 > 0 ? d.ax[2].sh[km] : -1;
    float ezn = __shfl_down(ez_[0], 1);
    if constexpr (XS > 1) {  // the next segment's first node, read directly
      if (lane == 63 && xs + 1 < XS && ib + VX < nx)
        ezn = to_f(*reinterpret_cast<const T *>(reinterpret_cast<const char *>(Ei2 + km * plane) + o0 + VX * esz));
    }
#pragma unroll
    for (int v = 0; v < VX; v++) {
      const int i = ib + v;
      const int shx = __float_as_int(sTab[6][i]);
      const float ezx = (v + 1 < VX) ? ez_[v + 1] : ezn;
      {
        const float d1 = ezu[v] - ez_[v], d2 = eyc[v] - ey_[v];
        const bool u = i < nx && j <= ny - 2 && km <= nz - 2;
        float sy = 0.f, sz = 0.f;
        if (shy >= 0 && u) sy = -psi_h(d, d.psi_h[par][1][0], nullptr, false, 1, j, i, j, km, shy, d1);
        if (shz >= 0 && u) sz = psi_h(d, d.psi_h[par][2][0], nullptr, false, 2, km, i, j, km, shz, d2);
        hxp[v] = u ? add_layers(h_plain(hxo[v], d1, chy, d2, chz), false, 0.f, shy >= 0, sy, shz >= 0, sz) : hxo[v];
      }
      {
        const float d1 = exc[v] - ex_[v], d2 = ezx - ez_[v];
        const bool u = i <= nx - 2 && km <= nz - 2;
        float sx = 0.f, sz = 0.f;
        if (shx >= 0 && u) sx = psi_h(d, d.psi_h[par][0][0], nullptr, false, 0, i, i, j, km, shx, d2);
        if (shz >= 0 && u) sz = -psi_h(d, d.psi_h[par][2][1], nullptr, false, 2, km, i, j, km, shz, d1);
        hyp[v] = u ? add_layers(h_plain(hyo[v], d1, chz, d2, sTab[0][i]), shx >= 0, sx, false, 0.f, shz >= 0, sz) : hyo[v];
      }
    }
    as_stored<T, VX>(hxp);
    as_stored<T, VX>(hyp);
  } else {
#pragma unroll
    for (int v = 0; v < VX; v++) hxp[v] = hyp[v] = 0.f;
  }

  // The sweep can issue each plane's row loads one plane ahead: the raw values of
  // E(k+2), H(k+1) and the x-slab psi of plane k+1 are in flight while plane k is computed.
  constexpr bool PF = PREFETCH;
  Vec<T, VX> rE0, rE1, rE2, rH0, rH1, rH2, rT0, rT2;
  float rq0 = 0.f, rq1 = 0.f, rq2 = 0.f, rq3 = 0.f;
  if constexpr (PF) {
    const long long pn = (long long)min(k0 + 1, nz - 1) * plane, pk = (long long)k0 * plane;
    ld_raw<T, VX>(Ei0 + pn, o0, rE0, on);
    ld_raw<T, VX>(Ei1 + pn, o0, rE1, on);
    ld_raw<T, VX>(Ei2 + pn, o0, rE2, on);
    ld_raw<T, VX>(Hi0 + pk, o0, rH0, on);
    ld_raw<T, VX>(Hi1 + pk, o0, rH1, on);
    ld_raw<T, VX>(Hi2 + pk, o0, rH2, on);
    ld_raw<T, VX>(Ei0 + pn, op, rT0, on && top_ld);
    ld_raw<T, VX>(Ei2 + pn, op, rT2, on && top_ld);
    if (lane < np2 && act) {
      const long long prow0 = ((long long)k0 * ny + jc) * np2;
      rq0 = phi0[prow0 + lane];
      rq1 = phi1[prow0 + lane];
      if (own) {
        rq2 = pe0[prow0 + lane];
        rq3 = pe1[prow0 + lane];
      }
    }
  }

  for (int k = k0; k < k1; k++) {
    const int kp = min(k + 1, nz - 1);
    const long long pk = k * plane, pn = kp * plane;
    // publish E(k) of the own row (slot r) and of the row above the tile (slot W+1)
    if (own) {
#pragma unroll
      for (int v = 0; v < VX; v++) {
        sEx[r][ib + v] = exc[v];
        sEz[r][ib + v] = ezc[v];
      }
    }
    if constexpr (XS > 1) {
      if (lane == 0) {
        sBE[r][xs][0] = eyc[0];
        sBE[r][xs][1] = ezc[0];
      }
    }
    if (top) {
#pragma unroll
      for (int v = 0; v < VX; v++) {
        sEx[W + 1][ib + v] = etx[v];
        sEz[W + 1][ib + v] = etz[v];
      }
    }
    // loads: E(k+1) and H^{n-1/2}(k) of the own row, Ex, Ez(k+1) of the row above the tile
    // (top wave), the own row's x-slab psi (one value per lane) and y/z-slab psi rows
    const float chz = d.ax[2].ch[k], cez = d.ax[2].ce[k];
    // z layer and wall masks of this plane (uniform)
    const int shz = GZ && np2 > 0 ? d.ax[2].sh[k] : -1, sez = GZ && np2 > 0 ? d.ax[2].se[k] : -1;
    const bool kh = !GZ || k <= nz - 2;              // Hx, Hy have their z difference
    const bool ke = !GZ || (k >= 1 && k <= nz - 2);  // Ex, Ey are not tangential to a z wall
    // y/z slab rows: H terms Hx(y), Hz(y), Hx(z), Hy(z); E terms Ex(y), Ez(y), Ex(z), Ey(z)
    // (issued before the row loads of the next plane, which the prefetching sweep issues below:
    // waiting for these then never waits for those)
    float qhxy[VX], qhzy[VX], qhxz[VX], qhyz[VX], qexy[VX], qezy[VX], qexz[VX], qeyz[VX];
    long long iyh = 0, iye = 0, izh = 0, ize = 0;
    if constexpr (GY) {
      iyh = ((long long)k * np2 + max(shy, 0)) * d.pitch + ib;
      iye = ((long long)k * np2 + max(sey, 0)) * d.pitch + ib;
      izh = ((long long)max(shz, 0) * ny + jc) * d.pitch + ib;
      ize = ((long long)max(sez, 0) * ny + jc) * d.pitch + ib;
      ld_row<float, VX>(d.psi_h[par][1][0] + iyh, qhxy, on && shy >= 0);
      ld_row<float, VX>(d.psi_h[par][1][1] + iyh, qhzy, on && shy >= 0);
      ld_row<float, VX>(d.psi_h[par][2][0] + izh, qhxz, on && shz >= 0);
      ld_row<float, VX>(d.psi_h[par][2][1] + izh, qhyz, on && shz >= 0);
      ld_row<float, VX>(d.psi_e[1][0] + iye, qexy, own && on && sey >= 0);
      ld_row<float, VX>(d.psi_e[1][1] + iye, qezy, own && on && sey >= 0);
      ld_row<float, VX>(d.psi_e[2][0] + ize, qexz, own && on && sez >= 0);
      ld_row<float, VX>(d.psi_e[2][1] + ize, qeyz, own && on && sez >= 0);
    }
    float nxc[VX], nyc[VX], nzc[VX], hx0[VX], hy0[VX], hz0[VX];
    const long long prow = ((long long)k * ny + jc) * np2;
    float q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
    if constexpr (PF) {
      unpack<T, VX>(rE0, nxc);
      unpack<T, VX>(rE1, nyc);
      unpack<T, VX>(rE2, nzc);
      unpack<T, VX>(rH0, hx0);
      unpack<T, VX>(rH1, hy0);
      unpack<T, VX>(rH2, hz0);
      unpack<T, VX>(rT0, etx);
      unpack<T, VX>(rT2, etz);
      q0 = rq0;
      q1 = rq1;
      q2 = rq2;
      q3 = rq3;
      // the next plane's loads (clamped to the last plane; values past k1 - 1 are not used)
      const long long pa = (long long)min(k + 2, nz - 1) * plane;
      ld_raw<T, VX>(Ei0 + pa, o0, rE0, on);
      ld_raw<T, VX>(Ei1 + pa, o0, rE1, on);
      ld_raw<T, VX>(Ei2 + pa, o0, rE2, on);
      ld_raw<T, VX>(Hi0 + pn, o0, rH0, on);
      ld_raw<T, VX>(Hi1 + pn, o0, rH1, on);
      ld_raw<T, VX>(Hi2 + pn, o0, rH2, on);
      ld_raw<T, VX>(Ei0 + pa, op, rT0, on && top_ld);
      ld_raw<T, VX>(Ei2 + pa, op, rT2, on && top_ld);
      if (lane < np2 && act) {
        const long long prn = ((long long)kp * ny + jc) * np2;
        rq0 = phi0[prn + lane];
        rq1 = phi1[prn + lane];
        if (own) {
          rq2 = pe0[prn + lane];
          rq3 = pe1[prn + lane];
        }
      }
    } else {
      ld_at<T, VX>(Ei0 + pn, o0, nxc, on);
      ld_at<T, VX>(Ei1 + pn, o0, nyc, on);
      ld_at<T, VX>(Ei2 + pn, o0, nzc, on);
      ld_at<T, VX>(Hi0 + pk, o0, hx0, on);
      ld_at<T, VX>(Hi1 + pk, o0, hy0, on);
      ld_at<T, VX>(Hi2 + pk, o0, hz0, on);
      ld_at<T, VX>(Ei0 + pn, op, etx, on && top_ld);
      ld_at<T, VX>(Ei2 + pn, op, etz, on && top_ld);
      if (lane < np2 && act) {
        q0 = phi0[prow + lane];
        q1 = phi1[prow + lane];
        if (own) {
          q2 = pe0[prow + lane];
          q3 = pe1[prow + lane];
        }
      }
    }
    __syncthreads();

    // ---- H^{n+1/2}(k) of the own row
    if (lane < np2) {
      sPsi[wv][0][lane] = q0;
      sPsi[wv][1][lane] = q1;
      sPsi[wv][2][lane] = q2;
      sPsi[wv][3][lane] = q3;
    }
    float eux[VX], euz[VX], chx[VX];
#pragma unroll
    for (int v = 0; v < VX; v++) {
      eux[v] = sEx[r + 1][ib + v];
      euz[v] = sEz[r + 1][ib + v];
      chx[v] = sTab[0][ib + v];
    }
    float eyn = __shfl_down(eyc[0], 1), ezn = __shfl_down(ezc[0], 1);
    if constexpr (XS > 1) {
      if (lane == 63 && xs + 1 < XS) {
        eyn = sBE[r][xs + 1][0];
        ezn = sBE[r][xs + 1][1];
      }
    }
    float hx[VX], hy[VX], hz[VX];
#pragma unroll
    for (int v = 0; v < VX; v++) {
      const float eyx = (v + 1 < VX) ? eyc[v + 1] : eyn;
      const float ezx = (v + 1 < VX) ? ezc[v + 1] : ezn;
      hx[v] = h_plain(hx0[v], euz[v] - ezc[v], chy, nyc[v] - eyc[v], chz);
      hy[v] = h_plain(hy0[v], nxc[v] - exc[v], chz, ezx - ezc[v], chx[v]);
      hz[v] = h_plain(hz0[v], eyx - eyc[v], chx[v], eux[v] - exc[v], chy);
    }
    if (xfix) {  // x walls and padding keep old values; x-layer terms
#pragma unroll
      for (int v = 0; v < VX; v++) {
        const int i = ib + v;
        const int sh = __float_as_int(sTab[6][i]);
        if (i >= nx - 1) {
          hy[v] = hy0[v];
          hz[v] = hz0[v];
          if (i >= nx) hx[v] = hx0[v];
        } else if (sh >= 0) {
          const float eyx = (v + 1 < VX) ? eyc[v + 1] : eyn;
          const float ezx = (v + 1 < VX) ? ezc[v + 1] : ezn;
          const float ah = sTab[2][i], bh = sTab[3][i];
          if (kh) {
            const float py = pml_psi(sPsi[wv][0][sh], ah, bh, ezx - ezc[v]);
            hy[v] = hy[v] + py;
            sPsi[wv][0][sh] = py;
          }
          if (jh) {
            const float pz = pml_psi(sPsi[wv][1][sh], ah, bh, eyx - eyc[v]);
            hz[v] = hz[v] + -pz;
            sPsi[wv][1][sh] = pz;
          }
        }
      }
    }
    if constexpr (GY) {  // y and z layer terms (after the x term), then the wall masks
      const float ahz = shz >= 0 ? d.ax[2].ah[k] : 0.f, bhz = shz >= 0 ? d.ax[2].bh[k] : 0.f;
#pragma unroll
      for (int v = 0; v < VX; v++) {
        const int i = ib + v;
        const bool ux = i < nx && jh && kh, uy = i <= nx - 2 && kh, uz = i <= nx - 2 && jh;
        if (shy >= 0) {
          if (ux) {
            const float p = pml_psi(qhxy[v], ahy, bhy, euz[v] - ezc[v]);
            qhxy[v] = p;
            hx[v] = hx[v] + -p;
          }
          if (uz) {
            const float p = pml_psi(qhzy[v], ahy, bhy, eux[v] - exc[v]);
            qhzy[v] = p;
            hz[v] = hz[v] + p;
          }
        }
        if (shz >= 0) {
          if (ux) {
            const float p = pml_psi(qhxz[v], ahz, bhz, nyc[v] - eyc[v]);
            qhxz[v] = p;
            hx[v] = hx[v] + p;
          }
          if (uy) {
            const float p = pml_psi(qhyz[v], ahz, bhz, nxc[v] - exc[v]);
            qhyz[v] = p;
            hy[v] = hy[v] + -p;
          }
        }
        if (!ux) hx[v] = hx0[v];
        if (!uy) hy[v] = hy0[v];
        if (!uz) hz[v] = hz0[v];
      }
    }
    as_stored<T, VX>(hx);
    as_stored<T, VX>(hy);
    as_stored<T, VX>(hz);

    // publish Hx, Hz(k) of the own row for the row above
    if (r < W) {
#pragma unroll
      for (int v = 0; v < VX; v++) {
        sHx[r][ib + v] = hx[v];
        sHz[r][ib + v] = hz[v];
      }
    }
    if constexpr (XS > 1) {
      if (lane == 63) {
        sBH[r][xs][0] = hy[VX - 1];
        sBH[r][xs][1] = hz[VX - 1];
      }
    }
    __syncthreads();

    if (own) {
      // ---- E^{n+1}(k) of the own row
      float hxm[VX], hzm[VX], cex[VX];
#pragma unroll
      for (int v = 0; v < VX; v++) {
        hxm[v] = sHx[r - 1][ib + v];
        hzm[v] = sHz[r - 1][ib + v];
        cex[v] = sTab[1][ib + v];
      }
      float hzw0 = __shfl_up(hz[VX - 1], 1), hyw0 = __shfl_up(hy[VX - 1], 1);
      if constexpr (XS > 1) {
        if (lane == 0 && xs > 0) {
          hyw0 = sBH[r][xs - 1][0];
          hzw0 = sBH[r][xs - 1][1];
        }
      }
      float oex[VX], oey[VX], oez[VX];
#pragma unroll
      for (int v = 0; v < VX; v++) {
        const float hzw = (v > 0) ? hz[v - 1] : hzw0;
        const float hyw = (v > 0) ? hy[v - 1] : hyw0;
        oex[v] = e_plain(d.ca, exc[v], hz[v] - hzm[v], cey, hy[v] - hyp[v], cez);
        oey[v] = e_plain(d.ca, eyc[v], hx[v] - hxp[v], cez, hz[v] - hzw, cex[v]);
        oez[v] = e_plain(d.ca, ezc[v], hy[v] - hyw, cex[v], hx[v] - hxm[v], cey);
      }
      if (xfix) {
#pragma unroll
        for (int v = 0; v < VX; v++) {
          const int i = ib + v;
          const int se = __float_as_int(sTab[7][i]);
          if (i >= nx - 1) {
            oex[v] = exc[v];
            oey[v] = eyc[v];
            oez[v] = ezc[v];
          } else if (i == 0) {
            oey[v] = eyc[v];
            oez[v] = ezc[v];
          } else if (se >= 0) {
            const float hzw = (v > 0) ? hz[v - 1] : hzw0;
            const float hyw = (v > 0) ? hy[v - 1] : hyw0;
            const float ae = sTab[4][i], be = sTab[5][i];
            if (jh && ke) {
              const float py = pml_psi(sPsi[wv][2][se], ae, be, hz[v] - hzw);
              oey[v] = oey[v] + -py;
              sPsi[wv][2][se] = py;
            }
            if (je && kh) {
              const float pz = pml_psi(sPsi[wv][3][se], ae, be, hy[v] - hyw);
              oez[v] = oez[v] + pz;
              sPsi[wv][3][se] = pz;
            }
          }
        }
      }
      if constexpr (GY) {
        const float aez = sez >= 0 ? d.ax[2].ae[k] : 0.f, bez = sez >= 0 ? d.ax[2].be[k] : 0.f;
#pragma unroll
        for (int v = 0; v < VX; v++) {
          const int i = ib + v;
          const bool ux = i <= nx - 2 && je && ke;
          const bool uy = i >= 1 && i <= nx - 2 && jh && ke;
          const bool uz = i >= 1 && i <= nx - 2 && je && kh;
          if (sey >= 0) {
            if (ux) {
              const float p = pml_psi(qexy[v], aey, bey, hz[v] - hzm[v]);
              qexy[v] = p;
              oex[v] = oex[v] + p;
            }
            if (uz) {
              const float p = pml_psi(qezy[v], aey, bey, hx[v] - hxm[v]);
              qezy[v] = p;
              oez[v] = oez[v] + -p;
            }
          }
          if (sez >= 0) {
            if (ux) {
              const float p = pml_psi(qexz[v], aez, bez, hy[v] - hyp[v]);
              qexz[v] = p;
              oex[v] = oex[v] + -p;
            }
            if (uy) {
              const float p = pml_psi(qeyz[v], aez, bez, hx[v] - hxp[v]);
              qeyz[v] = p;
              oey[v] = oey[v] + p;
            }
          }
          if (!ux) oex[v] = exc[v];
          if (!uy) oey[v] = eyc[v];
          if (!uz) oez[v] = ezc[v];
        }
      }
      if constexpr (DYN) {
        dyn_mh = absmax<VX>(absmax<VX>(absmax<VX>(dyn_mh, hx, on), hy, on), hz, on);
        dyn_me = absmax<VX>(absmax<VX>(absmax<VX>(dyn_me, oex, on), oey, on), oez, on);
        st_at_s<T, VX>(Ho0 + pk, o0, hx, on, dyn_r);
        st_at_s<T, VX>(Ho1 + pk, o0, hy, on, dyn_r);
        st_at_s<T, VX>(Ho2 + pk, o0, hz, on, dyn_r);
        st_at_s<T, VX>(Eo0 + pk, o0, oex, on, dyn_r);
        st_at_s<T, VX>(Eo1 + pk, o0, oey, on, dyn_r);
        st_at_s<T, VX>(Eo2 + pk, o0, oez, on, dyn_r);
      } else {
        st_at<T, VX>(Ho0 + pk, o0, hx, on);
        st_at<T, VX>(Ho1 + pk, o0, hy, on);
        st_at<T, VX>(Ho2 + pk, o0, hz, on);
        st_at<T, VX>(Eo0 + pk, o0, oex, on);
        st_at<T, VX>(Eo1 + pk, o0, oey, on);
        st_at<T, VX>(Eo2 + pk, o0, oez, on);
      }
      // the row's x-slab psi back to memory (slab indices of wall nodes keep their values)
      if (lane < np2) {
        if (own_sh) {
          pho0[prow + lane] = DYN ? sPsi[wv][0][lane] * dyn_r : sPsi[wv][0][lane];
          pho1[prow + lane] = DYN ? sPsi[wv][1][lane] * dyn_r : sPsi[wv][1][lane];
        }
        if (own_se) {
          pe0[prow + lane] = DYN ? sPsi[wv][2][lane] * dyn_r : sPsi[wv][2][lane];
          pe1[prow + lane] = DYN ? sPsi[wv][3][lane] * dyn_r : sPsi[wv][3][lane];
        }
      }
      if constexpr (GY) {
        if (shy >= 0) {
          st_row_s<float, VX>(d.psi_h[par ^ 1][1][0] + iyh, qhxy, on, dyn_r);
          st_row_s<float, VX>(d.psi_h[par ^ 1][1][1] + iyh, qhzy, on, dyn_r);
        }
        if (shz >= 0) {
          st_row_s<float, VX>(d.psi_h[par ^ 1][2][0] + izh, qhxz, on, dyn_r);
          st_row_s<float, VX>(d.psi_h[par ^ 1][2][1] + izh, qhyz, on, dyn_r);
        }
        if (sey >= 0) {
          st_row_s<float, VX>(d.psi_e[1][0] + iye, qexy, on, dyn_r);
          st_row_s<float, VX>(d.psi_e[1][1] + iye, qezy, on, dyn_r);
        }
        if (sez >= 0) {
          st_row_s<float, VX>(d.psi_e[2][0] + ize, qexz, on, dyn_r);
          st_row_s<float, VX>(d.psi_e[2][1] + ize, qeyz, on, dyn_r);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < VX; v++) {
      hxp[v] = hx[v];
      hyp[v] = hy[v];
      exc[v] = nxc[v];
      eyc[v] = nyc[v];
      ezc[v] = nzc[v];
    }
  }
  if constexpr (DYN) {
    unsigned *slot = d.dmax + 2 * ((*d.dslot[par] + 1) % 3);
    dyn_raise(slot, dyn_me);
    dyn_raise(slot + 1, dyn_mh);
  }
}
template <typename T, int VX, int W, bool PF, int XS = 1, bool DYN = false>
__global__ void __launch_bounds__(64 * (W + 1) * XS) k_fused(Dev d, FusedShape fs, int par) {
  const int logical = xcd_logical();
  if (logical >= fs.n_fast) return;
  const int fw = fs.ty_hi - fs.ty_lo;
  fused_body<T, VX, W, 0, PF, XS, DYN>(d, fs.ty_lo + logical % fw, fs.zc_lo + logical / fw, fs.zchunk, par);
}
// Boundary tiles (walls, y/z layers) from the tile table, in the general fused sweep: G = 1
// over the table's first n_slow_y entries (interior z range), G = 2 over the rest.
template <typename T, int VX, int W, int G, bool PF, int XS = 1, bool DYN = false>
__global__ void __launch_bounds__(64 * (W + 1) * XS) k_fused_gen(Dev d, FusedShape fs, const int *tiles, int n,
                                                                  int par) {
  const int logical = xcd_logical();
  if (logical >= n) return;
  fused_body<T, VX, W, G, PF, XS, DYN>(d, tiles[2 * logical], tiles[2 * logical + 1], fs.zchunk, par);
}

// Batched: entries (plan, ty, zc) over the interior rectangles of every plan of a batch.
template <typename T, int VX, int W, bool PF>
__global__ void __launch_bounds__(64 * (W + 1)) k_fused_batch(const Dev *devs, const int *zchunks, const int *tab,
                                                       int n, int par) {
  const int logical = xcd_logical();
  if (logical >= n) return;
  const int pl = tab[3 * logical];
  fused_body<T, VX, W, 0, PF>(devs[pl], tab[3 * logical + 1], tab[3 * logical + 2], zchunks[pl], par);
}
// Batched boundary tiles in the general fused sweep: entries (plan, ty, zc) of one class.
template <typename T, int VX, int W, int G, bool PF>
__global__ void __launch_bounds__(64 * (W + 1)) k_fused_gen_batch(const Dev *devs, const int *zchunks, const int *tab,
                                                                 int n, int par) {
  const int logical = xcd_logical();
  if (logical >= n) return;
  const int pl = tab[3 * logical];
  fused_body<T, VX, W, G, PF>(devs[pl], tab[3 * logical + 1], tab[3 * logical + 2], zchunks[pl], par);
}

// --------------------------------------------------------------- split sweeps
// Every tile when the split sweeps are selected (and the boundary tiles of fused plans whose
// rows are wider than 256 nodes): a workgroup of 64 x W threads covers 64 nodes of the W rows
// of one tile and marches its z chunk, one thread per (i, j) column; H then E in two launches.
// Same canonical per-node arithmetic as the fused sweeps.
template <typename T>
__device__ __forceinline__ void split_h_body(const Dev &d, int i, int j, int k0, int k1, int par);
template <typename T>
__device__ __forceinline__ void split_e_body(const Dev &d, int i, int j, int k0, int k1, int par);

template <typename T>
__device__ __forceinline__ void split_h_body(const Dev &d, int i, int j, int k0, int k1, int par) {
  if (i >= d.nx || j < 0 || j >= d.ny) return;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const T *E0 = (const T *)d.e[par][0], *E1 = (const T *)d.e[par][1], *E2 = (const T *)d.e[par][2];
  const T *Hi0 = (const T *)d.h[par][0], *Hi1 = (const T *)d.h[par][1], *Hi2 = (const T *)d.h[par][2];
  T *Ho0 = (T *)d.h[par ^ 1][0], *Ho1 = (T *)d.h[par ^ 1][1], *Ho2 = (T *)d.h[par ^ 1][2];
  float *pi_[3][2], *po_[3][2];
  for (int u = 0; u < 3; u++)
    for (int t = 0; t < 2; t++) {
      pi_[u][t] = d.psi_h[par][u][t];
      po_[u][t] = d.psi_h[par ^ 1][u][t];
    }
  const bool pml = d.np2 > 0;
  const int ip = min(i + 1, nx - 1), jp = min(j + 1, ny - 1);
  const float chx = d.ax[0].ch[i], chy = d.ax[1].ch[j];
  const int shx = pml ? d.ax[0].sh[i] : -1, shy = pml ? d.ax[1].sh[j] : -1;
  const bool xl = shx >= 0, yl = shy >= 0;
  for (int k = k0; k < k1; k++) {
    const int kp = min(k + 1, nz - 1);
    const long long c = (long long)k * d.plane + (long long)j * d.pitch + i;
    const long long cxp = (long long)k * d.plane + (long long)j * d.pitch + ip;
    const long long cyp = (long long)k * d.plane + (long long)jp * d.pitch + i;
    const long long czp = (long long)kp * d.plane + (long long)j * d.pitch + i;
    const float chz = d.ax[2].ch[k];
    const int shz = pml ? d.ax[2].sh[k] : -1;
    const bool zl = shz >= 0;
    const float ex = to_f(E0[c]), ey = to_f(E1[c]), ez = to_f(E2[c]);
    {  // Hx: y, z
      const float d1 = to_f(E2[cyp]) - ez, d2 = to_f(E1[czp]) - ey;
      const bool u = j <= ny - 2 && k <= nz - 2;
      float sy = 0.f, sz = 0.f;
      if (yl && u) sy = -psi_h(d, pi_[1][0], po_[1][0], true, 1, j, i, j, k, shy, d1);
      if (zl && u) sz = psi_h(d, pi_[2][0], po_[2][0], true, 2, k, i, j, k, shz, d2);
      const float h = to_f(Hi0[c]);
      Ho0[c] = from_f<T>(u ? add_layers(h_plain(h, d1, chy, d2, chz), false, 0.f, yl, sy, zl, sz) : h);
    }
    {  // Hy: z, x
      const float d1 = to_f(E0[czp]) - ex, d2 = to_f(E2[cxp]) - ez;
      const bool u = i <= nx - 2 && k <= nz - 2;
      float sx = 0.f, sz = 0.f;
      if (xl && u) sx = psi_h(d, pi_[0][0], po_[0][0], true, 0, i, i, j, k, shx, d2);
      if (zl && u) sz = -psi_h(d, pi_[2][1], po_[2][1], true, 2, k, i, j, k, shz, d1);
      const float h = to_f(Hi1[c]);
      Ho1[c] = from_f<T>(u ? add_layers(h_plain(h, d1, chz, d2, chx), xl, sx, false, 0.f, zl, sz) : h);
    }
    {  // Hz: x, y
      const float d1 = to_f(E1[cxp]) - ey, d2 = to_f(E0[cyp]) - ex;
      const bool u = i <= nx - 2 && j <= ny - 2;
      float sx = 0.f, sy = 0.f;
      if (xl && u) sx = -psi_h(d, pi_[0][1], po_[0][1], true, 0, i, i, j, k, shx, d1);
      if (yl && u) sy = psi_h(d, pi_[1][1], po_[1][1], true, 1, j, i, j, k, shy, d2);
      const float h = to_f(Hi2[c]);
      Ho2[c] = from_f<T>(u ? add_layers(h_plain(h, d1, chx, d2, chy), xl, sx, yl, sy, false, 0.f) : h);
    }
  }
}

template <typename T>
__device__ __forceinline__ void split_e_body(const Dev &d, int i, int j, int k0, int k1, int par) {
  if (i >= d.nx || j < 0 || j >= d.ny) return;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const T *Ei0 = (const T *)d.e[par][0], *Ei1 = (const T *)d.e[par][1], *Ei2 = (const T *)d.e[par][2];
  const T *H0 = (const T *)d.h[par ^ 1][0], *H1 = (const T *)d.h[par ^ 1][1], *H2 = (const T *)d.h[par ^ 1][2];
  T *Eo0 = (T *)d.e[par ^ 1][0], *Eo1 = (T *)d.e[par ^ 1][1], *Eo2 = (T *)d.e[par ^ 1][2];
  const bool pml = d.np2 > 0;
  const int im = max(i - 1, 0), jm = max(j - 1, 0);
  const float cex = d.ax[0].ce[i], cey = d.ax[1].ce[j];
  const int sex = pml ? d.ax[0].se[i] : -1, sey = pml ? d.ax[1].se[j] : -1;
  const bool xl = sex >= 0, yl = sey >= 0;
  for (int k = k0; k < k1; k++) {
    const int km = max(k - 1, 0);
    const long long c = (long long)k * d.plane + (long long)j * d.pitch + i;
    const long long cxm = (long long)k * d.plane + (long long)j * d.pitch + im;
    const long long cym = (long long)k * d.plane + (long long)jm * d.pitch + i;
    const long long czm = (long long)km * d.plane + (long long)j * d.pitch + i;
    const float cez = d.ax[2].ce[k];
    const int sez = pml ? d.ax[2].se[k] : -1;
    const bool zl = sez >= 0;
    const float hx = to_f(H0[c]), hy = to_f(H1[c]), hz = to_f(H2[c]);
    {  // Ex: y, z
      const float d1 = hz - to_f(H2[cym]), d2 = hy - to_f(H1[czm]);
      const bool u = i <= nx - 2 && j >= 1 && j <= ny - 2 && k >= 1 && k <= nz - 2;
      float sy = 0.f, sz = 0.f;
      if (yl && u) sy = psi_e(d, d.psi_e[1][0], 1, j, i, j, k, sey, d1);
      if (zl && u) sz = -psi_e(d, d.psi_e[2][0], 2, k, i, j, k, sez, d2);
      const float e = to_f(Ei0[c]);
      Eo0[c] = from_f<T>(u ? add_layers(e_plain(d.ca, e, d1, cey, d2, cez), false, 0.f, yl, sy, zl, sz) : e);
    }
    {  // Ey: z, x
      const float d1 = hx - to_f(H0[czm]), d2 = hz - to_f(H2[cxm]);
      const bool u = i >= 1 && i <= nx - 2 && j <= ny - 2 && k >= 1 && k <= nz - 2;
      float sx = 0.f, sz = 0.f;
      if (xl && u) sx = -psi_e(d, d.psi_e[0][0], 0, i, i, j, k, sex, d2);
      if (zl && u) sz = psi_e(d, d.psi_e[2][1], 2, k, i, j, k, sez, d1);
      const float e = to_f(Ei1[c]);
      Eo1[c] = from_f<T>(u ? add_layers(e_plain(d.ca, e, d1, cez, d2, cex), xl, sx, false, 0.f, zl, sz) : e);
    }
    {  // Ez: x, y
      const float d1 = hy - to_f(H1[cxm]), d2 = hx - to_f(H0[cym]);
      const bool u = i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2 && k <= nz - 2;
      float sx = 0.f, sy = 0.f;
      if (xl && u) sx = psi_e(d, d.psi_e[0][1], 0, i, i, j, k, sex, d1);
      if (yl && u) sy = -psi_e(d, d.psi_e[1][1], 1, j, i, j, k, sey, d2);
      const float e = to_f(Ei2[c]);
      Eo2[c] = from_f<T>(u ? add_layers(e_plain(d.ca, e, d1, cex, d2, cey), xl, sx, yl, sy, false, 0.f) : e);
    }
  }
}

// Single plan: workgroup -> (tile from the table, 64-node x block).
template <typename T, bool H>
__global__ void __launch_bounds__(1024) k_split(Dev d, FusedShape fs, const int *tiles, int n_tiles, int par) {
  const int nxb = (d.nx + 63) / 64;
  const int tile = blockIdx.x / nxb;
  if (tile >= n_tiles) return;
  const int ty = tiles[2 * tile], zc = tiles[2 * tile + 1];
  const int i = (blockIdx.x % nxb) * 64 + (threadIdx.x & 63);
  const int j = ty * fs.waves - d.ysh + (threadIdx.x >> 6);
  const int k0 = max(zc * fs.zchunk - d.zsh, 0), k1 = min(zc * fs.zchunk - d.zsh + fs.zchunk, d.nz);
  if constexpr (H) split_h_body<T>(d, i, j, k0, k1, par);
  else split_e_body<T>(d, i, j, k0, k1, par);
}

// Batched: entries (plan, ty, zc, x block) over the boundary tiles of every plan.
template <typename T, bool H>
__global__ void __launch_bounds__(1024) k_split_batch(const Dev *devs, const int *zchunks, const int *tab, int n,
                                                     int rows, int par) {
  if ((int)blockIdx.x >= n) return;
  const int *e = tab + 4 * blockIdx.x;
  const Dev &d = devs[e[0]];
  const int zchunk = zchunks[e[0]];
  const int i = e[3] * 64 + (threadIdx.x & 63);
  const int j = e[1] * rows - d.ysh + (threadIdx.x >> 6);
  const int k0 = max(e[2] * zchunk - d.zsh, 0), k1 = min(e[2] * zchunk - d.zsh + zchunk, d.nz);
  if constexpr (H) split_h_body<T>(d, i, j, k0, k1, par);
  else split_e_body<T>(d, i, j, k0, k1, par);
}

// ------------------------------------------------------------------- source
// J_z of the moving Gaussian charge snapshot at (n+1/2) dt, subtracted (times scale*Cb)
// from Ez^{n+1}.  Bookkeeping in FP64: bunch position, Q(z_s) from the hat bins, and the
// lattice-normalised longitudinal weights.  One thread per (i, j) of the radial patch.
// Returns the largest |Ez| this thread stored (dynamic scaling raises the level's maxima by it).
template <typename T>
__device__ __forceinline__ float source_body(const Dev &d, int out_par, int step, const double *q, int t) {
  if (!d.src_on || t >= d.src_ni * d.src_nj) return 0.f;
  const double tt = (step + 0.5) * d.dt;
  if (tt < d.t_entry) return 0.f;
  const double wr = d.wr[t];
  if (wr == 0.0) return 0.f;
  const int i = d.src_i0 + t % d.src_ni, j = d.src_j0 + t / d.src_ni;
  const double zs = d.z_entry + d.v_src * (tt - d.t_entry);
  const double qz = source_q(d, q, zs);
  int klo;
  const int m = source_window(d, zs, &klo);
  double norm = 0.0;
  for (int s = 0; s < m; s++) {
    const double dd = (klo + s + 0.5) * d.dz - zs;
    norm += exp(-0.5 * dd * dd / (d.sigma_z * d.sigma_z)) * d.dz;
  }
  T *Ez = (T *)d.e[out_par][2];
  // a dynamically scaled level holds 2^e times the static scale: the increment scales exactly
  const double cb = d.dyn ? ldexp(d.cb_src, *d.dexp[out_par]) : d.cb_src;
  float mx = 0.f;
  for (int s = 0; s < m; s++) {
    const int k = klo + s;
    if (k < 0 || k > d.nz - 2) continue;
    const double dd = (klo + s + 0.5) * d.dz - zs;
    const double wz = exp(-0.5 * dd * dd / (d.sigma_z * d.sigma_z)) / norm;
    const double inc = cb * d.v_src * qz * wr * wz;
    const long long c = (long long)k * d.plane + (long long)j * d.pitch + i;
    const float nv = to_f(Ez[c]) - (float)inc;
    Ez[c] = from_f<T>(nv);
    mx = fmaxf(mx, fabsf(nv));
  }
  return mx;
}

template <typename T>
__global__ void k_source(Dev d, int out_par, int step, const double *q) {
  const float m = source_body<T>(d, out_par, step, q, blockIdx.x * blockDim.x + threadIdx.x);
  if (d.dyn) dyn_raise(d.dmax + 2 * *d.dslot[out_par], m);
}

// Batched: blockIdx.y is the plan; each plan uses its own profile.
template <typename T>
__global__ void k_source_batch(const Dev *devs, int out_par, int step) {
  const Dev &d = devs[blockIdx.y];
  (void)source_body<T>(d, out_par, step, d.q_bins, blockIdx.x * blockDim.x + threadIdx.x);
}

// --------------------------------------------------------------------- Mur-1
// E0^{n+1} = E1^n + K (E1^{n+1} - E0^n) on the face-interior tangential E of each face;
// level `par` holds E^n and par^1 holds E^{n+1} (edges keep their zero).
template <typename T>
__global__ void k_mur(Dev d, int par) {
  const int fc = blockIdx.z;  // 0..11: face (x-,x+,y-,y+,z-,z+) x tangential component
  const int face = fc >> 1, which = fc & 1;
  const int axis = face >> 1, hi = face & 1;
  const int comp = axis == 0 ? (which ? 2 : 1) : axis == 1 ? (which ? 2 : 0) : (which ? 1 : 0);
  const int n[3] = {d.nx, d.ny, d.nz};
  const int ua = axis == 0 ? 1 : 0, ub = axis == 2 ? 1 : 2;  // in-face axes
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y * blockDim.y + threadIdx.y;
  // face-interior range of `comp` along each in-face axis: a staggered (half) axis spans
  // 0..n-2, an integer axis spans 1..n-2
  auto lo_of = [&](int ax) { return ax == comp ? 0 : 1; };
  const int alo = lo_of(ua), ahi = n[ua] - 2, blo = lo_of(ub), bhi = n[ub] - 2;
  const int ia = alo + a, jb = blo + b;
  if (ia > ahi || jb > bhi) return;
  int idx[3];
  idx[ua] = ia;
  idx[ub] = jb;
  const int w0 = hi ? n[axis] - 1 : 0, w1 = hi ? n[axis] - 2 : 1;
  const float K = axis == 0 ? d.mur_kx : axis == 1 ? d.mur_ky : d.mur_kz;
  idx[axis] = w0;
  const long long c0 = (long long)idx[2] * d.plane + (long long)idx[1] * d.pitch + idx[0];
  idx[axis] = w1;
  const long long c1 = (long long)idx[2] * d.plane + (long long)idx[1] * d.pitch + idx[0];
  const T *Ein = (const T *)d.e[par][comp];
  T *Eout = (T *)d.e[par ^ 1][comp];
  const float e1n = to_f(Ein[c1]), e0n = to_f(Ein[c0]), e1new = to_f(Eout[c1]);
  Eout[c0] = from_f<T>(fmaf(K, e1new - e0n, e1n));
}

// ------------------------------------------------------------------- gather
template <typename T>
__global__ void __launch_bounds__(64) k_gather(Dev d, int par, double *w, int column, int ld) {
  gather_body<T>(d, par, w, column, ld, blockIdx.x);
}

// Batched: entries (plan, observer) over every observer of the batch; plan p writes waves[p].
template <typename T>
__global__ void __launch_bounds__(64) k_gather_batch(const Dev *devs, double *const *waves, const int *tab,
                                                    int par, int column, int ld) {
  const int pl = tab[2 * blockIdx.x];
  gather_body<T>(devs[pl], par, waves[pl], column, ld, tab[2 * blockIdx.x + 1]);
}

// ------------------------------------------------------------ fill / copies
__global__ void k_fill_zero(uint4 *p, long long n16) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n16;
       t += (long long)gridDim.x * blockDim.x)
    p[t] = make_uint4(0u, 0u, 0u, 0u);
}

// Dense [nz][ny][nx] copies of one component: one wave per (j, k) row at a time (rows dealt
// round-robin over the waves of the grid), lanes along x, so one division per row.
template <typename T>
__global__ void k_get_field(Dev d, const T *src, float *out, float inv_scale, const int *dexp) {
  if (dexp) inv_scale = ldexpf(inv_scale, -*dexp);
  const long long rows = (long long)d.ny * d.nz;
  const int lane = threadIdx.x & 63;
  const long long nw = (long long)gridDim.x * (blockDim.x >> 6);
  for (long long r = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < rows; r += nw) {
    const int j = (int)(r % d.ny), k = (int)(r / d.ny);
    const T *sr = src + (long long)k * d.plane + (long long)j * d.pitch;
    float *o = out + r * d.nx;
    for (int i = lane; i < d.nx; i += 64) o[i] = to_f(sr[i]) * inv_scale;
  }
}

template <typename T>
__global__ void k_set_field(Dev d, T *dst, const float *in, float scale, const int *dexp) {
  if (dexp) scale = ldexpf(scale, *dexp);
  const long long rows = (long long)d.ny * d.nz;
  const int lane = threadIdx.x & 63;
  const long long nw = (long long)gridDim.x * (blockDim.x >> 6);
  for (long long r = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < rows; r += nw) {
    const int j = (int)(r % d.ny), k = (int)(r / d.ny);
    T *dr = dst + (long long)k * d.plane + (long long)j * d.pitch;
    const float *ir = in + r * d.nx;
    for (int i = lane; i < d.nx; i += 64) dr[i] = from_f<T>(ir[i] * scale);
  }
}

// ------------------------------------------------------------------ launch
// general sweeps: part bit 0 launches the y-boundary tiles (G = 1), bit 1 the z-boundary ones (G = 2)
template <typename T, int VX, int W, bool DYN>
static hipError_t fused_launch(const chf_plan &p, const Dev &d, int par, bool general, hipStream_t s, int part) {
  if (general) {
    if constexpr (VX <= kMaxGeneralVX && W <= kMaxGeneralW) {
      const int ny_ = p.fs.n_slow_y, nr = p.fs.n_slow - p.fs.n_slow_y;
      // boundary tiles load a plane ahead as well, with workgroups of at most 8 waves (2 waves per
      // SIMD hold their registers; 9- and 12-wave workgroups would need 3 and spill); the plain
      // boundary sweeps of 11-row tiles fit 3 waves per SIMD (the z-wall one with a small spill)
      if (p.fs.prefetch && W <= 7) {
        if (ny_ > 0 && (part & 1))
          hipLaunchKernelGGL((k_fused_gen<T, VX, W, 1, true, 1, DYN>), dim3((ny_ + 7) / 8 * 8), dim3(64 * (W + 1)), 0, s, d,
                             p.fs, d.slow_tiles, ny_, par);
        if (nr > 0 && (part & 2))
          hipLaunchKernelGGL((k_fused_gen<T, VX, W, 2, true, 1, DYN>), dim3((nr + 7) / 8 * 8), dim3(64 * (W + 1)), 0, s, d,
                             p.fs, d.slow_tiles + 2 * ny_, nr, par);
      } else {
        if (ny_ > 0 && (part & 1))
          hipLaunchKernelGGL((k_fused_gen<T, VX, W, 1, false, 1, DYN>), dim3((ny_ + 7) / 8 * 8), dim3(64 * (W + 1)), 0, s, d,
                             p.fs, d.slow_tiles, ny_, par);
        if (nr > 0 && (part & 2))
          hipLaunchKernelGGL((k_fused_gen<T, VX, W, 2, false, 1, DYN>), dim3((nr + 7) / 8 * 8), dim3(64 * (W + 1)), 0, s, d,
                             p.fs, d.slow_tiles + 2 * ny_, nr, par);
      }
    } else
      return hipErrorInvalidValue;
  } else if (p.fs.prefetch) {
    if constexpr (VX <= 4 && W <= 11)
      hipLaunchKernelGGL((k_fused<T, VX, W, true, 1, DYN>), dim3(p.fs.fast_blocks), dim3(64 * (W + 1)), 0, s, d, p.fs, par);
    else
      return hipErrorInvalidValue;
  } else
    hipLaunchKernelGGL((k_fused<T, VX, W, false, 1, DYN>), dim3(p.fs.fast_blocks), dim3(64 * (W + 1)), 0, s, d, p.fs, par);
  return hipGetLastError();
}

template <typename T, int VX, bool DYN>
static hipError_t fused_dispatch_w(const chf_plan &p, const Dev &d, int par, bool general, hipStream_t s,
                                   int part) {
  switch (p.fs.waves) {
    case 4: return fused_launch<T, VX, 4, DYN>(p, d, par, general, s, part);
    case 7: return fused_launch<T, VX, 7, DYN>(p, d, par, general, s, part);
    case 8:
      if constexpr (VX <= 4) return fused_launch<T, VX, 8, DYN>(p, d, par, general, s, part);
      return hipErrorInvalidValue;
    case 11:
      if constexpr (VX <= 4) return fused_launch<T, VX, 11, DYN>(p, d, par, general, s, part);
      return hipErrorInvalidValue;
    case 15:
      if constexpr (VX <= 4) return fused_launch<T, VX, 15, DYN>(p, d, par, general, s, part);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

// Rows of up to 512 nodes split across two waves (VX 4): the prefetching interior sweep with 4 or 5
// rows per tile (10 or 12 waves) and the plain general sweep for the boundary tiles.
template <typename T, int W, bool DYN>
static hipError_t split_rows_launch(const chf_plan &p, const Dev &d, int par, bool general, hipStream_t s, int part) {
  const dim3 block(64 * (W + 1) * 2);
  if (general) {
    const int ny_ = p.fs.n_slow_y, nr = p.fs.n_slow - p.fs.n_slow_y;
    if (ny_ > 0 && (part & 1))
      hipLaunchKernelGGL((k_fused_gen<T, 4, W, 1, false, 2, DYN>), dim3((ny_ + 7) / 8 * 8), block, 0, s, d, p.fs,
                         d.slow_tiles, ny_, par);
    if (nr > 0 && (part & 2))
      hipLaunchKernelGGL((k_fused_gen<T, 4, W, 2, false, 2, DYN>), dim3((nr + 7) / 8 * 8), block, 0, s, d, p.fs,
                         d.slow_tiles + 2 * ny_, nr, par);
  } else {
    hipLaunchKernelGGL((k_fused<T, 4, W, true, 2, DYN>), dim3(p.fs.fast_blocks), block, 0, s, d, p.fs, par);
  }
  return hipGetLastError();
}

// general = false: the interior rectangle; true: the boundary tiles of the tile table
template <typename T, bool DYN>
static hipError_t fused_dispatch_t(const chf_plan &p, const Dev &d, int par, bool general, hipStream_t s,
                                   int part = 3) {
  if (p.fs.xs == 2) {
    if (p.fs.waves == 4) return split_rows_launch<T, 4, DYN>(p, d, par, general, s, part);
    if (p.fs.waves == 5) return split_rows_launch<T, 5, DYN>(p, d, par, general, s, part);
    return hipErrorInvalidValue;
  }
  switch (p.fs.vx) {
    case 1: return fused_dispatch_w<T, 1, DYN>(p, d, par, general, s, part);
    case 2: return fused_dispatch_w<T, 2, DYN>(p, d, par, general, s, part);
    case 4: return fused_dispatch_w<T, 4, DYN>(p, d, par, general, s, part);
    case 8: return fused_dispatch_w<T, 8, DYN>(p, d, par, general, s, part);
    default: return hipErrorInvalidValue;
  }
}

// Dynamically scaled levels exist for FP16 storage only (plan validation), so only the FP16
// sweeps are built in that form.
template <typename T>
static hipError_t fused_dispatch(const chf_plan &p, const Dev &d, int par, bool general, hipStream_t s,
                                 int part = 3) {
  if constexpr (std::is_same<T, _Float16>::value) {
    if (d.dyn) return fused_dispatch_t<T, true>(p, d, par, general, s, part);
  } else {
    if (d.dyn) return hipErrorInvalidValue;
  }
  return fused_dispatch_t<T, false>(p, d, par, general, s, part);
}

template <typename T>
static hipError_t step_t(const chf_plan &p, const Dev &d_in, int par, int step, const double *q,
                         double *w, int column, int ld, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b) {
  hipError_t e = hipSuccess;
  const Dev &d = d_in;
  const int nxb = (d.nx + 63) / 64;
  const dim3 sgrid(p.fs.n_slow * nxb), sblock(64 * p.fs.waves);
  if (p.kernel == CHF_KERNEL_FUSED) {
    // The interior rectangle in one fused sweep; the boundary tiles in the general fused sweep
    // (or, for rows wider than 256 nodes and for 15-row tiles, whose general sweep would not
    // fit its registers, in split H and E sweeps).  Both read only the input
    // level and write disjoint nodes, so the boundary sweep (its H half, when split) runs on
    // the side stream beside the interior one; the general sweep's z-boundary tiles on a second
    // side stream beside its y-boundary ones.
    const bool gen = (p.fs.vx <= kMaxGeneralVX && p.fs.waves <= kMaxGeneralW) || p.fs.xs == 2;
    const bool fork = p.fs.n_fast > 0 && p.fs.n_slow > 0 && p.aux;
    const bool fork2 = fork && gen && p.aux2 && p.fs.n_slow_y > 0 && p.fs.n_slow > p.fs.n_slow_y;
    if (fork) {
      e = hipEventRecord(p.ev_fork, s);
      if (e == hipSuccess) e = hipStreamWaitEvent(p.aux, p.ev_fork, 0);
      if (e == hipSuccess && fork2) e = hipStreamWaitEvent(p.aux2, p.ev_fork, 0);
      if (e == hipSuccess) {
        if (fork2) {
          e = fused_dispatch<T>(p, d, par, true, p.aux, 1);
          if (e == hipSuccess) e = fused_dispatch<T>(p, d, par, true, p.aux2, 2);
          if (e == hipSuccess) e = hipEventRecord(p.ev_join2, p.aux2);
        } else if (gen) {
          e = fused_dispatch<T>(p, d, par, true, p.aux);
        } else {
          hipLaunchKernelGGL((k_split<T, true>), sgrid, sblock, 0, p.aux, d, p.fs, d.slow_tiles, p.fs.n_slow, par);
          e = hipGetLastError();
        }
      }
      if (e == hipSuccess) e = hipEventRecord(p.ev_join, p.aux);
      if (e != hipSuccess) return e;
    }
    if (p.fs.n_fast > 0) {
      if (ev_a) e = hipEventRecord(ev_a, s);
      if (e == hipSuccess) e = fused_dispatch<T>(p, d, par, false, s);
      if (e == hipSuccess && ev_b) e = hipEventRecord(ev_b, s);
      if (e != hipSuccess) return e;
    }
    if (p.fs.n_slow > 0) {
      if (fork) {
        e = hipStreamWaitEvent(s, p.ev_join, 0);
        if (e == hipSuccess && fork2) e = hipStreamWaitEvent(s, p.ev_join2, 0);
      } else if (gen) {
        e = fused_dispatch<T>(p, d, par, true, s);
      } else {
        hipLaunchKernelGGL((k_split<T, true>), sgrid, sblock, 0, s, d, p.fs, d.slow_tiles, p.fs.n_slow, par);
      }
      if (e == hipSuccess && !gen)
        hipLaunchKernelGGL((k_split<T, false>), sgrid, sblock, 0, s, d, p.fs, d.slow_tiles, p.fs.n_slow, par);
      if (e == hipSuccess) e = hipGetLastError();
    }
  } else if (p.fs.n_slow > 0) {
    // split sweeps over every tile: H, then E reading the fresh H
    hipLaunchKernelGGL((k_split<T, true>), sgrid, sblock, 0, s, d, p.fs, d.slow_tiles, p.fs.n_slow, par);
    hipLaunchKernelGGL((k_split<T, false>), sgrid, sblock, 0, s, d, p.fs, d.slow_tiles, p.fs.n_slow, par);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  if (d.dyn) {
    e = launch_dyn_publish(d, par, 1, s);
    if (e != hipSuccess) return e;
  }
  if (d.src_on) {
    const int n = d.src_ni * d.src_nj;
    hipLaunchKernelGGL(k_source<T>, dim3((n + 255) / 256), dim3(256), 0, s, d, par ^ 1, step,
                       q ? q : d.q_bins);
  }
  if (d.bc == CHF_BC_MUR1) {
    const int m = max(d.nx, max(d.ny, d.nz));
    dim3 grid((m + 15) / 16, (m + 15) / 16, 12);
    hipLaunchKernelGGL(k_mur<T>, grid, dim3(16, 16), 0, s, d, par);
  }
  if (d.n_obs > 0 && w) hipLaunchKernelGGL(k_gather<T>, dim3(d.n_obs), dim3(64), 0, s, d, par ^ 1, w, column, ld);
  return hipGetLastError();
}

hipError_t launch_step(const chf_plan &p, const Dev &d, int par, int step, const double *q, double *w,
                       int column, int ld, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b) {
  switch (p.storage) {
    case CHF_FP32: return step_t<float>(p, d, par, step, q, w, column, ld, s, ev_a, ev_b);
    case CHF_BF16: return step_t<__bf16>(p, d, par, step, q, w, column, ld, s, ev_a, ev_b);
    case CHF_BF16X: return step_t<bf16x>(p, d, par, step, q, w, column, ld, s, ev_a, ev_b);
    case CHF_FP16: return step_t<_Float16>(p, d, par, step, q, w, column, ld, s, ev_a, ev_b);
  }
  return hipErrorInvalidValue;
}

// general = false: the interior tiles of every member; true: their boundary tiles
template <typename T, int VX, int W>
static hipError_t batch_fused(const chf_batch &b, const Dev *devs, const int *z, int par, bool general,
                              hipStream_t s, int part) {
  if (general) {
    if constexpr (VX <= kMaxGeneralVX && W <= kMaxGeneralW) {
      const int n1 = (int)(b.gen_tab[0].size() / 3), n2 = (int)(b.gen_tab[1].size() / 3);
      const int *t1 = (const int *)(b.ws + b.off_gen[0]), *t2 = (const int *)(b.ws + b.off_gen[1]);
      if (b.prefetch && W <= 7) {  // as for single plans: only 8-wave workgroups hold the registers
        if (n1 > 0 && (part & 1))
          hipLaunchKernelGGL((k_fused_gen_batch<T, VX, W, 1, true>), dim3((n1 + 7) / 8 * 8), dim3(64 * (W + 1)), 0,
                             s, devs, z, t1, n1, par);
        if (n2 > 0 && (part & 2))
          hipLaunchKernelGGL((k_fused_gen_batch<T, VX, W, 2, true>), dim3((n2 + 7) / 8 * 8), dim3(64 * (W + 1)), 0,
                             s, devs, z, t2, n2, par);
      } else {
        if (n1 > 0 && (part & 1))
          hipLaunchKernelGGL((k_fused_gen_batch<T, VX, W, 1, false>), dim3((n1 + 7) / 8 * 8), dim3(64 * (W + 1)), 0,
                             s, devs, z, t1, n1, par);
        if (n2 > 0 && (part & 2))
          hipLaunchKernelGGL((k_fused_gen_batch<T, VX, W, 2, false>), dim3((n2 + 7) / 8 * 8), dim3(64 * (W + 1)), 0,
                             s, devs, z, t2, n2, par);
      }
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  const int n = (int)(b.fast_tab.size() / 3);
  if (n == 0) return hipSuccess;
  const int blocks = (n + 7) / 8 * 8;
  if (b.prefetch) {
    if constexpr (VX <= 4 && W <= 11)
      hipLaunchKernelGGL((k_fused_batch<T, VX, W, true>), dim3(blocks), dim3(64 * (W + 1)), 0, s, devs, z,
                         (const int *)(b.ws + b.off_fast), n, par);
    else
      return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((k_fused_batch<T, VX, W, false>), dim3(blocks), dim3(64 * (W + 1)), 0, s, devs, z,
                       (const int *)(b.ws + b.off_fast), n, par);
  }
  return hipGetLastError();
}

template <typename T, int VX>
static hipError_t batch_fused_w(const chf_batch &b, const Dev *devs, const int *z, int par, bool general,
                                hipStream_t s, int part) {
  switch (b.waves) {
    case 4: return batch_fused<T, VX, 4>(b, devs, z, par, general, s, part);
    case 7: return batch_fused<T, VX, 7>(b, devs, z, par, general, s, part);
    case 8:
      if constexpr (VX <= 4) return batch_fused<T, VX, 8>(b, devs, z, par, general, s, part);
      return hipErrorInvalidValue;
    case 11:
      if constexpr (VX <= 4) return batch_fused<T, VX, 11>(b, devs, z, par, general, s, part);
      return hipErrorInvalidValue;
    case 15:
      if constexpr (VX <= 4) return batch_fused<T, VX, 15>(b, devs, z, par, general, s, part);
      return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t batch_fused_v(const chf_batch &b, const Dev *devs, const int *z, int par, bool general,
                                hipStream_t s, int part = 3) {
  switch (b.vx) {
    case 1: return batch_fused_w<T, 1>(b, devs, z, par, general, s, part);
    case 2: return batch_fused_w<T, 2>(b, devs, z, par, general, s, part);
    case 4: return batch_fused_w<T, 4>(b, devs, z, par, general, s, part);
    default: return batch_fused_w<T, 8>(b, devs, z, par, general, s, part);
  }
}

template <typename T>
static hipError_t batch_step_t(const chf_batch &b, int par, int step, hipStream_t s) {
  const Dev *devs = (const Dev *)(b.ws + b.off_devs);
  const int *z = (const int *)(b.ws + b.off_z);
  hipError_t e = hipSuccess;
  const int ns = (int)(b.slow_tab.size() / 4);
  const int *stab = (const int *)(b.ws + b.off_slow);
  // boundary tiles (general fused sweep, or split H then E) on the side stream beside the
  // interior tiles; the source injection joins them
  const bool fork = ns > 0 && !b.fast_tab.empty() && b.aux;
  // the z-boundary tiles of the general sweep on a second side stream beside the y-boundary ones
  const bool fork2 = fork && b.gen && b.aux2 && !b.gen_tab[0].empty() && !b.gen_tab[1].empty();
  hipStream_t sb = fork ? b.aux : s;
  if (fork) {
    e = hipEventRecord(b.ev_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(b.aux, b.ev_fork, 0);
    if (e == hipSuccess && fork2) e = hipStreamWaitEvent(b.aux2, b.ev_fork, 0);
    if (e != hipSuccess) return e;
  }
  if (ns > 0) {
    if (fork2) {
      e = batch_fused_v<T>(b, devs, z, par, true, b.aux, 1);
      if (e == hipSuccess) e = batch_fused_v<T>(b, devs, z, par, true, b.aux2, 2);
      if (e == hipSuccess) e = hipEventRecord(b.ev_join2, b.aux2);
    } else if (b.gen) {
      e = batch_fused_v<T>(b, devs, z, par, true, sb);
    } else {
      hipLaunchKernelGGL((k_split_batch<T, true>), dim3(ns), dim3(64 * b.waves), 0, sb, devs, z, stab, ns,
                         b.waves, par);
      e = hipGetLastError();
    }
    if (e == hipSuccess && fork) e = hipEventRecord(b.ev_join, b.aux);
    if (e != hipSuccess) return e;
  }
  e = batch_fused_v<T>(b, devs, z, par, false, s);
  if (e != hipSuccess) return e;
  if (fork) e = hipStreamWaitEvent(s, b.ev_join, 0);
  if (e == hipSuccess && fork2) e = hipStreamWaitEvent(s, b.ev_join2, 0);
  if (e != hipSuccess) return e;
  // the split E sweep reads the fresh H of the interior tiles next to the boundary ones
  if (ns > 0 && !b.gen)
    hipLaunchKernelGGL((k_split_batch<T, false>), dim3(ns), dim3(64 * b.waves), 0, s, devs, z, stab, ns,
                       b.waves, par);
  if (b.max_patch > 0)
    hipLaunchKernelGGL(k_source_batch<T>, dim3((b.max_patch + 255) / 256, (int)b.plans.size()), dim3(256), 0, s,
                       devs, par ^ 1, step);
  if (b.any_mur)
    for (const chf_plan *p : b.plans)
      if (p->dev.bc == CHF_BC_MUR1) {
        const int m = max(p->dev.nx, max(p->dev.ny, p->dev.nz));
        hipLaunchKernelGGL(k_mur<T>, dim3((m + 15) / 16, (m + 15) / 16, 12), dim3(16, 16), 0, s, p->dev, par);
      }
  if (b.total_obs > 0)
    hipLaunchKernelGGL(k_gather_batch<T>, dim3(b.total_obs), dim3(64), 0, s, devs,
                       (double *const *)(b.ws + b.off_wptr), (const int *)(b.ws + b.off_obs), par ^ 1, step,
                       b.n_steps);
  return hipGetLastError();
}

// ------------------------------------------------------ persistent batch launch
// The whole batch run in one cooperative launch: every resident workgroup loops over the Yee
// steps; per step it takes tiles of every member from the combined table (interior and boundary
// alike, through the general fused sweep, whose per-node arithmetic is the canonical one, so the
// results equal the per-phase launches bit for bit), then all workgroups meet at a grid barrier,
// inject the sources of every member, meet again, and gather the observers (one wave each; the
// gathers read the level the next step only reads, so no barrier follows them).  Every loop is
// bounded and every workgroup passes every barrier.
template <int VX, int W>
__global__ void __launch_bounds__(64 * (W + 1)) k_batch_persistent(const Dev *devs, const int *zchunks, const int *tab,
                                                                   int n_tab, const int *obs, int n_obs,
                                                                   double *const *waves, int n_plans, int max_patch,
                                                                   int n_steps) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  const int gt = blockIdx.x * blockDim.x + threadIdx.x, gs = gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63, wave = gt >> 6, n_waves = gs >> 6;
  for (int step = 0; step < n_steps; step++) {
    const int par = step & 1;
    for (int t = blockIdx.x; t < n_tab; t += gridDim.x) {
      const int *e = tab + 3 * t;
      fused_body<float, VX, W, 2, false>(devs[e[0]], e[1], e[2], zchunks[e[0]], par);
      __syncthreads();  // the tile's LDS rows and tables before the next tile overwrites them
    }
    grid.sync();
    for (int u = gt; u < n_plans * max_patch; u += gs) {
      const Dev &d = devs[u / max_patch];
      (void)source_body<float>(d, par ^ 1, step, d.q_bins, u % max_patch);
    }
    grid.sync();
    for (int o = wave; o < n_obs; o += n_waves) {
      const int pl = obs[2 * o];
      gather_body<float>(devs[pl], par ^ 1, waves[pl], step, n_steps, obs[2 * o + 1], lane);
    }
  }
}

template <int VX, int W>
static hipError_t persistent_launch(const chf_batch &b, const int *tab, int n_tab, hipStream_t s) {
  const void *fn = reinterpret_cast<const void *>(&k_batch_persistent<VX, W>);
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * (W + 1), 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  // every workgroup resident at once (the cooperative launch checks it), no more than there are tiles
  const int grid = std::max(1, std::min(cus * per_cu, n_tab));
  const Dev *devs = (const Dev *)(b.ws + b.off_devs);
  const int *z = (const int *)(b.ws + b.off_z);
  const int *obs = (const int *)(b.ws + b.off_obs);
  double *const *waves = (double *const *)(b.ws + b.off_wptr);
  int n_obs = b.total_obs, n_plans = (int)b.plans.size(), max_patch = b.max_patch, n_steps = b.n_steps;
  void *args[] = {(void *)&devs, (void *)&z, (void *)&tab, (void *)&n_tab, (void *)&obs, (void *)&n_obs,
                  (void *)&waves, (void *)&n_plans, (void *)&max_patch, (void *)&n_steps};
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(64 * (W + 1)), args, 0, s);
}

hipError_t launch_batch_persistent(const chf_batch &b, const int *tab, int n_tab, hipStream_t s) {
  if (b.storage != CHF_FP32) return hipErrorInvalidValue;
  switch (b.vx * 100 + b.waves) {
    case 104: return persistent_launch<1, 4>(b, tab, n_tab, s);
    case 107: return persistent_launch<1, 7>(b, tab, n_tab, s);
    case 108: return persistent_launch<1, 8>(b, tab, n_tab, s);
    case 111: return persistent_launch<1, 11>(b, tab, n_tab, s);
    case 204: return persistent_launch<2, 4>(b, tab, n_tab, s);
    case 207: return persistent_launch<2, 7>(b, tab, n_tab, s);
    case 208: return persistent_launch<2, 8>(b, tab, n_tab, s);
    case 211: return persistent_launch<2, 11>(b, tab, n_tab, s);
    case 404: return persistent_launch<4, 4>(b, tab, n_tab, s);
    case 407: return persistent_launch<4, 7>(b, tab, n_tab, s);
    case 408: return persistent_launch<4, 8>(b, tab, n_tab, s);
    case 411: return persistent_launch<4, 11>(b, tab, n_tab, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_step(const chf_batch &b, int par, int step, hipStream_t s) {
  switch (b.storage) {
    case CHF_FP32: return batch_step_t<float>(b, par, step, s);
    case CHF_BF16: return batch_step_t<__bf16>(b, par, step, s);
    case CHF_BF16X: return batch_step_t<bf16x>(b, par, step, s);
    case CHF_FP16: return batch_step_t<_Float16>(b, par, step, s);
  }
  return hipErrorInvalidValue;
}

// --------------------------------------------------------- dynamic scaling
// After the sweeps of a launch of n steps from level par: the written level's exponent (the
// sweeps' own choice, recomputed from the same words), its maxima slot, and the slot the next
// launch raises cleared.  One lane.
__global__ void k_dyn_publish(Dev d, int par, int n) {
  if (threadIdx.x != 0) return;
  const int sh = dyn_shift(d, par, n);
  const int sl = *d.dslot[par];
  *d.dexp[par ^ 1] = *d.dexp[par] + sh;
  *d.dslot[par ^ 1] = (sl + 1) % 3;
  const int nx = (sl + 2) % 3;
  d.dmax[2 * nx] = 0u;
  d.dmax[2 * nx + 1] = 0u;
}

hipError_t launch_dyn_publish(const Dev &d, int par, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_dyn_publish, dim3(1), dim3(64), 0, s, d, par, n);
  return hipGetLastError();
}

// The maxima of level par from its stored values: the slot cleared (one lane), then raised by
// every wave (rows dealt round-robin as in the field copies).
__global__ void k_dyn_clear(Dev d, int par) {
  if (threadIdx.x == 0) {
    const int sl = *d.dslot[par];
    d.dmax[2 * sl] = 0u;
    d.dmax[2 * sl + 1] = 0u;
  }
}

template <typename T>
__global__ void k_dyn_levelmax(Dev d, int par) {
  const long long rows = (long long)d.ny * d.nz;
  const int lane = threadIdx.x & 63;
  const long long nw = (long long)gridDim.x * (blockDim.x >> 6);
  float me = 0.f, mh = 0.f;
  for (long long r = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < rows; r += nw) {
    const int j = (int)(r % d.ny), k = (int)(r / d.ny);
    const long long o = (long long)k * d.plane + (long long)j * d.pitch;
    for (int c = 0; c < 3; c++) {
      const T *e = (const T *)d.e[par][c] + o, *h = (const T *)d.h[par][c] + o;
      for (int i = lane; i < d.nx; i += 64) {
        me = fmaxf(me, fabsf(to_f(e[i])));
        mh = fmaxf(mh, fabsf(to_f(h[i])));
      }
    }
  }
  unsigned *slot = d.dmax + 2 * *d.dslot[par];
  dyn_raise(slot, me);
  dyn_raise(slot + 1, mh);
}

hipError_t launch_dyn_levelmax(const chf_plan &p, int par, hipStream_t s) {
  hipLaunchKernelGGL(k_dyn_clear, dim3(1), dim3(64), 0, s, p.dev, par);
  if (p.storage == CHF_FP16)
    hipLaunchKernelGGL(k_dyn_levelmax<_Float16>, dim3(1024), dim3(256), 0, s, p.dev, par);
  return hipGetLastError();
}

hipError_t launch_zero(const chf_plan &p, hipStream_t s) {
  // fields and psi occupy [0, off_tf) of the workspace (16-byte multiples)
  const long long n16 = (long long)(p.off_tf / 16);
  hipLaunchKernelGGL(k_fill_zero, dim3(2048), dim3(256), 0, s, (uint4 *)p.ws, n16);
  // and the watchdog flag (a kernel, not a memset/copy, so that graphs may capture it)
  hipLaunchKernelGGL(k_fill_zero, dim3(1), dim3(64), 0, s, (uint4 *)(p.ws + p.off_nan), 16LL);
  return hipGetLastError();
}

template <typename T>
static hipError_t get_t(const chf_plan &p, int par, int comp, float *out, hipStream_t s) {
  const T *src = (const T *)(comp < 3 ? p.dev.e[par][comp] : p.dev.h[par][comp - 3]);
  const float inv = (float)(1.0 / (comp < 3 ? p.scale_e : p.scale_h));
  hipLaunchKernelGGL(k_get_field<T>, dim3(2048), dim3(256), 0, s, p.dev, src, out, inv,
                     (const int *)(p.dev.dyn ? p.dev.dexp[par] : nullptr));
  return hipGetLastError();
}

template <typename T>
static hipError_t set_t(const chf_plan &p, int par, int comp, const float *in, hipStream_t s) {
  T *dst = (T *)(comp < 3 ? p.dev.e[par][comp] : p.dev.h[par][comp - 3]);
  const float sc = (float)(comp < 3 ? p.scale_e : p.scale_h);
  hipLaunchKernelGGL(k_set_field<T>, dim3(2048), dim3(256), 0, s, p.dev, dst, in, sc,
                     (const int *)(p.dev.dyn ? p.dev.dexp[par] : nullptr));
  if (p.dev.dyn) return launch_dyn_levelmax(p, par, s);
  return hipGetLastError();
}

hipError_t launch_get_field(const chf_plan &p, int par, int comp, float *out, hipStream_t s) {
  switch (p.storage) {
    case CHF_FP32: return get_t<float>(p, par, comp, out, s);
    case CHF_BF16: return get_t<__bf16>(p, par, comp, out, s);
    case CHF_BF16X: return get_t<bf16x>(p, par, comp, out, s);
    case CHF_FP16: return get_t<_Float16>(p, par, comp, out, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_set_field(const chf_plan &p, int par, int comp, const float *in, hipStream_t s) {
  switch (p.storage) {
    case CHF_FP32: return set_t<float>(p, par, comp, in, s);
    case CHF_BF16: return set_t<__bf16>(p, par, comp, in, s);
    case CHF_BF16X: return set_t<bf16x>(p, par, comp, in, s);
    case CHF_FP16: return set_t<_Float16>(p, par, comp, in, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace chf
