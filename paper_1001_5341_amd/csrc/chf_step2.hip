// Two Yee steps per pass over the fields: temporal blocking of the 3-D leapfrog.
//
// A workgroup owns W consecutive y rows of the full x extent (XS waves per row, 64 VX nodes per
// wave) and marches a z chunk.  Per plane it advances the fields from level n to n+1 (stage 1)
// and, one plane behind, from n+1 to n+2 (stage 2), so level n+1 never leaves the chip: a pass
// reads E^n, H^{n-1/2} and writes E^{n+2}, H^{n+3/2} once -- 12 values per node for two steps
// instead of 24.
//
// Dependencies.  Stage 2 of the tile's rows needs stage 1 one row below (E's backward y
// difference) and one row above (H's forward difference), and stage 1 of that lower row needs
// stage-1 H one row further down: the workgroup computes rows j0-2 .. j0+W (row r = 0 .. W+2):
// row j0-2 stage-1 H only, row j0-1 up to stage-2 H, the tile's rows everything, row j0+W
// stage 1; the row above that is only loaded (its E).  Along z, plane by plane, the same: chunk
// [k0, k1) runs stage 1 over planes k0-2 .. k1 and stage 2 over k0-1 .. k1-1.  Halo rows and
// planes are recomputed from the untouched input level, so tiles never wait for each other.
// Rows exchange through LDS, x neighbours through shuffles (and LDS words across the waves of
// a split row).
//
// Iteration k (stage 1 at plane k, stage 2 at plane k-1), two barriers:
//   A  stage-1 H(k) (the row above's E^n(k) was published in the previous iteration); publish.
//   -- barrier --
//   B  stage-1 E(k) from the row below's H(k), with the moving source of step n and the samples
//      of E^{n+1} at the observers; stage-2 H(k-1) from the row above's E^{n+1}(k-1) (previous
//      iteration); publish E^{n+1}(k), H^{n+3/2}(k-1) and E^n(k+1).
//   -- barrier --
//   C  stage-2 E(k-1) from the row below's H^{n+3/2}(k-1), with the source of step n+1; store.
//
// Every node of every step takes the one-step sweeps' operations in their order (chf_cell.h),
// values carried from stage 1 to stage 2 are rounded through the storage type exactly as a
// store and a reload would round them, and the source and the sampling repeat the one-step
// kernels' expressions: a two-step pass gives the bits of two one-step passes.
//
// CPML: the x-slab psi of a row sits in LDS, one copy per plane parity (stage 1 of plane k
// updates the copy that stage 2 of plane k updates again one iteration later); y- and z-slab
// psi rows stay in registers between the stages.  psi_E is read from one level and written to
// the other (as psi_H is), since halo rows read psi a neighbouring tile is replacing.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "chf_cell.h"
#include "chf_internal.h"

namespace chf {

// Source constants of the pass's two steps, computed once per workgroup into LDS with the
// one-step source kernel's FP64 expressions: the longitudinal window [klo, klo + m) of each
// step, its normalised weights wz (per window row) and the product cb_src v Q(z_s).
struct SrcLds {
  int klo[2], m[2];
  double a[2];
  double wz[2][kMaxWz];
};

__device__ __forceinline__ void src_prepare(const Dev &d, int step, const double *q, SrcLds &S, int dyn_e) {
  const int t = threadIdx.x;
  if (t < 2) {
    S.m[t] = 0;
    S.klo[t] = 0;
    S.a[t] = 0.0;
    const double tt = (step + t + 0.5) * d.dt;
    if (d.src_on && tt >= d.t_entry) {
      const double zs = d.z_entry + d.v_src * (tt - d.t_entry);
      const double qz = source_q(d, q, zs);
      int klo;
      const int m = source_window(d, zs, &klo);
      double norm = 0.0;
      for (int u = 0; u < m; u++) {
        const double dd = (klo + u + 0.5) * d.dz - zs;
        norm += exp(-0.5 * dd * dd / (d.sigma_z * d.sigma_z)) * d.dz;
      }
      for (int u = 0; u < m; u++) {
        const double dd = (klo + u + 0.5) * d.dz - zs;
        S.wz[t][u] = exp(-0.5 * dd * dd / (d.sigma_z * d.sigma_z)) / norm;
      }
      S.klo[t] = klo;
      S.m[t] = m;
      // dynamic scaling: the pass computes in the units of the level it writes, 2^dyn_e times
      // the static scale, which scales the increment exactly
      S.a[t] = (d.dyn ? ldexp(d.cb_src, dyn_e) : d.cb_src) * d.v_src * qz;
    }
  }
}

// Ez -= Cb J of the pass's step `st` (0 or 1) on the lane's nodes of row j at plane k; ez holds
// values as stored.  inc = cb_src v Q W_r W_z, multiplied in the one-step kernel's order.
template <typename T, int VX>
__device__ __forceinline__ void src_apply(const Dev &d, const SrcLds &S, int st, int ib, int j, int k,
                                          float (&ez)[VX]) {
  const int klo = S.klo[st], m = S.m[st];
  if (k < klo || k >= klo + m || k < 0 || k > d.nz - 2) return;
  if (j < d.src_j0 || j >= d.src_j0 + d.src_nj || ib + VX <= d.src_i0 || ib >= d.src_i0 + d.src_ni) return;
  const double a = S.a[st], wz = S.wz[st][k - klo];
#pragma unroll
  for (int v = 0; v < VX; v++) {
    const int i = ib + v;
    if (i < d.src_i0 || i >= d.src_i0 + d.src_ni) continue;
    const double wr = d.wr[(j - d.src_j0) * d.src_ni + (i - d.src_i0)];
    if (wr == 0.0) continue;
    const double inc = a * wr * wz;
    ez[v] = to_f(from_f<T>(ez[v] - (float)inc));
  }
}

// DYN: dynamically scaled FP16 levels -- every value the pass loads (fields and psi) is multiplied
// by the launch's power of two r, so both stages, the source, the intermediate level's rounding
// and its samples work in the units of the level written (chosen for both steps); the wave's
// largest stored magnitudes raise that level's maxima.
template <typename T, int VX, int W, int XS, int G, bool DYN = false>
__device__ __forceinline__ void step2_body(const Dev &d, int j0, int jend, int k0, int k1, int par, int step,
                                           const double *q) {
  constexpr int NR = W + 3;  // computed rows: j0-2 .. j0+W; row NR (j0+W+1) is only loaded
  constexpr int SEG = 64 * VX, NL = SEG * XS;
  constexpr bool GY = G >= 1, GZ = G >= 2;
  constexpr int NP = kMaxStep2Layer;
  // Row exchange.  sE0: E^n(k) of row j0-2+s for s <= W+2 (read by the row itself and by the row
  // below), s = NR the row above the top halo.  sH1: H^{n+1/2}(k) of rows s = 0 .. W+1.  sE1[k & 1]: E^{n+1}(k) of rows s+1, s = 0 .. W+1
  // (read by the row itself one iteration later and by the row below).
  // sH2: H^{n+3/2}(k-1) of rows s+1, s = 0 .. W-1.
  __shared__ float sE0x[NR + 1][NL], sE0y[NR + 1][NL], sE0z[NR + 1][NL];
  __shared__ float sH1x[NR - 1][NL], sH1z[NR - 1][NL];
  __shared__ float sE1x[2][NR - 1][NL], sE1y[2][NR - 1][NL], sE1z[2][NR - 1][NL];
  __shared__ float sH2x[NR - 3][NL], sH2z[NR - 3][NL];
  // x tables: ch, ce, ah, bh, ae, be, x-slab slot (H), x-slab slot (E)
  __shared__ float sTab[8][NL];
  // x-slab psi of each wave's row, per plane parity: Hy, Hz terms (slots 0, 1), Ey, Ez terms (2, 3)
  __shared__ float sPsi[(NR + 1) * XS][2][4][NP];
  // split rows: the x neighbours across a wave boundary -- the last node's (Hy, Hz) of H levels,
  // per row and wave (E levels are whole rows in LDS)
  __shared__ float sBH1[NR + 1][XS][2], sBH2[NR + 1][XS][2];

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = wv / XS, xs = wv - r * XS;
  const int nx = d.nx, ny = d.ny, nz = d.nz, np2 = d.np2;
  const int j = j0 - 2 + r;
  const bool loader = r == NR;  // loads the E^n rows of j0+W+1 for the top halo row's H
  const bool act = !GY || (j >= 0 && j < ny);
  const int jc = GY ? min(max(j, 0), ny - 1) : j;
  const bool doH1 = act && !loader;
  const bool doE1 = r >= 1 && act && !loader, doH2 = r >= 1 && r <= W + 1 && act, own = r >= 2 && r <= W + 1 && act && j < jend;
  const int ib = xs * SEG + lane * VX;
  float dyn_r = 1.f, dyn_me = 0.f, dyn_mh = 0.f;
  int dyn_e = 0;  // exponent of the written level
  if constexpr (DYN) {
    const int sh = dyn_shift(d, par, 2);
    dyn_r = ldexpf(1.f, sh);
    dyn_e = *d.dexp[par] + sh;
  }
  const bool on = ib < nx && act;
  const unsigned esz = (unsigned)sizeof(T);
  const unsigned o0 = ((unsigned)jc * (unsigned)d.pitch + (unsigned)ib) * esz;
  const long long plane = d.plane;
  const T *Ei0 = (const T *)d.e[par][0], *Ei1 = (const T *)d.e[par][1], *Ei2 = (const T *)d.e[par][2];
  const T *Hi0 = (const T *)d.h[par][0], *Hi1 = (const T *)d.h[par][1], *Hi2 = (const T *)d.h[par][2];
  T *Eo0 = (T *)d.e[par ^ 1][0], *Eo1 = (T *)d.e[par ^ 1][1], *Eo2 = (T *)d.e[par ^ 1][2];
  T *Ho0 = (T *)d.h[par ^ 1][0], *Ho1 = (T *)d.h[par ^ 1][1], *Ho2 = (T *)d.h[par ^ 1][2];

  for (int i = threadIdx.x; i < NL; i += 64 * (NR + 1) * XS) {
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
  bool xfix = ib == 0 || ib + VX - 1 >= nx - 1;
  if (np2 > 0) {
#pragma unroll
    for (int v = 0; v < VX; v++) {
      const int i = ib + v;
      xfix = xfix || (i < nx && (d.ax[0].sh[i] >= 0 || d.ax[0].se[i] >= 0));
    }
  }
  // x-slab slots this wave stores (the slot's node lies in its x segment)
  bool ownH = false, ownE = false;
  if (lane < np2) {
    const int npml = d.npml;
    const int nh = lane < npml ? lane : lane - npml + (nx - 1 - npml);
    const int ne = lane < npml ? lane : lane - npml + (nx - npml);
    ownH = nh / SEG == xs;
    ownE = ne / SEG == xs;
  }
  const float chy = d.ax[1].ch[jc], cey = d.ax[1].ce[jc];
  const int shy = GY && np2 > 0 ? d.ax[1].sh[jc] : -1, sey = GY && np2 > 0 ? d.ax[1].se[jc] : -1;
  const float ahy = shy >= 0 ? d.ax[1].ah[jc] : 0.f, bhy = shy >= 0 ? d.ax[1].bh[jc] : 0.f;
  const float aey = sey >= 0 ? d.ax[1].ae[jc] : 0.f, bey = sey >= 0 ? d.ax[1].be[jc] : 0.f;
  const bool jh = !GY || j <= ny - 2;
  const bool je = !GY || (j >= 1 && j <= ny - 2);
  // source constants of the two steps (LDS; visible after the prologue's barrier)
  __shared__ SrcLds sSrc;
  src_prepare(d, step, q, sSrc, dyn_e);
  float *psA = &sPsi[wv][0][0][0];  // this wave's x-slab psi, [parity][term][slot]
  auto PS = [&](int par_k, int t) -> float * { return psA + (par_k * 4 + t) * NP; };

  // ---------------------------------------------------------------- the two node updates
  // H at plane k of this row (one-step sweep's sequence): old H (h0), E^(k) of the row (e), the
  // x and y components at k+1 (nn), the row above's Ex, Ez at k (ua), the next node's Ey, Ez
  // (eyn, ezn); x-slab psi in LDS (pbuf), y/z-slab psi rows (qy*, qz*) updated in place.
  auto h_upd = [&](int k, const float (&h0x)[VX], const float (&h0y)[VX], const float (&h0z)[VX],
                   const float (&ex)[VX], const float (&ey)[VX], const float (&ez)[VX], const float (&nxv)[VX],
                   const float (&nyv)[VX], const float (&uax)[VX], const float (&uaz)[VX], float eyn, float ezn,
                   int pbuf, float (&qhxy)[VX], float (&qhzy)[VX], float (&qhxz)[VX], float (&qhyz)[VX],
                   float (&hx)[VX], float (&hy)[VX], float (&hz)[VX]) {
    const float chz = d.ax[2].ch[k];
    const int shz = GZ && np2 > 0 ? d.ax[2].sh[k] : -1;
    const bool kh = !GZ || k <= nz - 2;
#pragma unroll
    for (int v = 0; v < VX; v++) {
      const float eyx = (v + 1 < VX) ? ey[v + 1] : eyn;
      const float ezx = (v + 1 < VX) ? ez[v + 1] : ezn;
      const float chx = sTab[0][ib + v];
      hx[v] = h_plain(h0x[v], uaz[v] - ez[v], chy, nyv[v] - ey[v], chz);
      hy[v] = h_plain(h0y[v], nxv[v] - ex[v], chz, ezx - ez[v], chx);
      hz[v] = h_plain(h0z[v], eyx - ey[v], chx, uax[v] - ex[v], chy);
    }
    if (xfix) {
      float *p0 = PS(pbuf, 0), *p1 = PS(pbuf, 1);
#pragma unroll
      for (int v = 0; v < VX; v++) {
        const int i = ib + v;
        const int sh = __float_as_int(sTab[6][i]);
        if (i >= nx - 1) {
          hy[v] = h0y[v];
          hz[v] = h0z[v];
          if (i >= nx) hx[v] = h0x[v];
        } else if (sh >= 0) {
          const float eyx = (v + 1 < VX) ? ey[v + 1] : eyn;
          const float ezx = (v + 1 < VX) ? ez[v + 1] : ezn;
          const float ah = sTab[2][i], bh = sTab[3][i];
          if (kh) {
            const float py = pml_psi(p0[sh], ah, bh, ezx - ez[v]);
            hy[v] = hy[v] + py;
            p0[sh] = py;
          }
          if (jh) {
            const float pz = pml_psi(p1[sh], ah, bh, eyx - ey[v]);
            hz[v] = hz[v] + -pz;
            p1[sh] = pz;
          }
        }
      }
    }
    if constexpr (GY) {
      const float ahz = shz >= 0 ? d.ax[2].ah[k] : 0.f, bhz = shz >= 0 ? d.ax[2].bh[k] : 0.f;
#pragma unroll
      for (int v = 0; v < VX; v++) {
        const int i = ib + v;
        const bool ux = i < nx && jh && kh, uy = i <= nx - 2 && kh, uz = i <= nx - 2 && jh;
        if (shy >= 0) {
          if (ux) {
            const float p = pml_psi(qhxy[v], ahy, bhy, uaz[v] - ez[v]);
            qhxy[v] = p;
            hx[v] = hx[v] + -p;
          }
          if (uz) {
            const float p = pml_psi(qhzy[v], ahy, bhy, uax[v] - ex[v]);
            qhzy[v] = p;
            hz[v] = hz[v] + p;
          }
        }
        if (shz >= 0) {
          if (ux) {
            const float p = pml_psi(qhxz[v], ahz, bhz, nyv[v] - ey[v]);
            qhxz[v] = p;
            hx[v] = hx[v] + p;
          }
          if (uy) {
            const float p = pml_psi(qhyz[v], ahz, bhz, nxv[v] - ex[v]);
            qhyz[v] = p;
            hy[v] = hy[v] + -p;
          }
        }
        if (!ux) hx[v] = h0x[v];
        if (!uy) hy[v] = h0y[v];
        if (!uz) hz[v] = h0z[v];
      }
    }
    as_stored<T, VX>(hx);
    as_stored<T, VX>(hy);
    as_stored<T, VX>(hz);
  };

  // E at plane k of this row: old E (e0), the new H of the row at k (h) and the x, y components
  // at k-1 (hxp, hyp), the row below's Hx, Hz at k (bx, bz), the previous node's Hz, Hy
  // (hzw0, hyw0); x-slab psi in LDS (pbuf), y/z-slab psi rows updated in place.
  auto e_upd = [&](int k, const float (&e0x)[VX], const float (&e0y)[VX], const float (&e0z)[VX],
                   const float (&hx)[VX], const float (&hy)[VX], const float (&hz)[VX], const float (&hxp)[VX],
                   const float (&hyp)[VX], const float (&bx)[VX], const float (&bz)[VX], float hzw0, float hyw0,
                   int pbuf, float (&qexy)[VX], float (&qezy)[VX], float (&qexz)[VX], float (&qeyz)[VX],
                   float (&oex)[VX], float (&oey)[VX], float (&oez)[VX]) {
    const float cez = d.ax[2].ce[k];
    const int sez = GZ && np2 > 0 ? d.ax[2].se[k] : -1;
    const bool kh = !GZ || k <= nz - 2;
    const bool ke = !GZ || (k >= 1 && k <= nz - 2);
#pragma unroll
    for (int v = 0; v < VX; v++) {
      const float hzw = (v > 0) ? hz[v - 1] : hzw0;
      const float hyw = (v > 0) ? hy[v - 1] : hyw0;
      const float cex = sTab[1][ib + v];
      oex[v] = e_plain(d.ca, e0x[v], hz[v] - bz[v], cey, hy[v] - hyp[v], cez);
      oey[v] = e_plain(d.ca, e0y[v], hx[v] - hxp[v], cez, hz[v] - hzw, cex);
      oez[v] = e_plain(d.ca, e0z[v], hy[v] - hyw, cex, hx[v] - bx[v], cey);
    }
    if (xfix) {
      float *p2 = PS(pbuf, 2), *p3 = PS(pbuf, 3);
#pragma unroll
      for (int v = 0; v < VX; v++) {
        const int i = ib + v;
        const int se = __float_as_int(sTab[7][i]);
        if (i >= nx - 1) {
          oex[v] = e0x[v];
          oey[v] = e0y[v];
          oez[v] = e0z[v];
        } else if (i == 0) {
          oey[v] = e0y[v];
          oez[v] = e0z[v];
        } else if (se >= 0) {
          const float hzw = (v > 0) ? hz[v - 1] : hzw0;
          const float hyw = (v > 0) ? hy[v - 1] : hyw0;
          const float ae = sTab[4][i], be = sTab[5][i];
          if (jh && ke) {
            const float py = pml_psi(p2[se], ae, be, hz[v] - hzw);
            oey[v] = oey[v] + -py;
            p2[se] = py;
          }
          if (je && kh) {
            const float pz = pml_psi(p3[se], ae, be, hy[v] - hyw);
            oez[v] = oez[v] + pz;
            p3[se] = pz;
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
            const float p = pml_psi(qexy[v], aey, bey, hz[v] - bz[v]);
            qexy[v] = p;
            oex[v] = oex[v] + p;
          }
          if (uz) {
            const float p = pml_psi(qezy[v], aey, bey, hx[v] - bx[v]);
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
        if (!ux) oex[v] = e0x[v];
        if (!uy) oey[v] = e0y[v];
        if (!uz) oez[v] = e0z[v];
      }
    }
    as_stored<T, VX>(oex);
    as_stored<T, VX>(oey);
    as_stored<T, VX>(oez);
  };

  // x neighbour of H levels: the previous node's value (lane - 1, or the previous wave of a
  // split row); E levels sit in LDS as whole rows
  auto prev_of = [&](float last, const float *bword) -> float {
    float p = __shfl_up(last, 1);
    if constexpr (XS > 1) {
      if (lane == 0 && xs > 0) p = bword[2 * (xs - 1)];
    }
    return p;
  };

  // ---------------------------------------------------------------- prologue
  // E^n(k0-2) of the row (and the row above the top halo), published for stage-1 H(k0-2)
  {
    float e0x[VX], e0y[VX], e0z[VX];
    const int kb = max(k0 - 2, 0);
    const bool pk = k0 - 2 >= 0;
    ld_at<T, VX>(Ei0 + kb * plane, o0, e0x, on && pk);
    ld_at<T, VX>(Ei1 + kb * plane, o0, e0y, on && pk && !loader);
    ld_at<T, VX>(Ei2 + kb * plane, o0, e0z, on && pk);
    if constexpr (DYN) {
      scale_in<VX>(e0x, dyn_r);
      scale_in<VX>(e0y, dyn_r);
      scale_in<VX>(e0z, dyn_r);
    }
#pragma unroll
    for (int v = 0; v < VX; v++) {
      sE0x[r][ib + v] = e0x[v];
      sE0y[r][ib + v] = e0y[v];
      sE0z[r][ib + v] = e0z[v];
    }
  }
  // raw loads of the first iteration: E^n(k+1), H^{n-1/2}(k), x-slab psi(k) (the loader wave:
  // Ex, Ez of its row at k+1 only)
  Vec<T, VX> rE0, rE1, rE2, rH0, rH1, rH2;
  float rq0 = 0.f, rq1 = 0.f, rq2 = 0.f, rq3 = 0.f;
  auto issue = [&](int k) {
    const bool pk = k >= 0 && k <= nz - 1, pn = k + 1 >= 0 && k + 1 <= nz - 1;
    const long long ok = (long long)min(max(k, 0), nz - 1) * plane;
    const long long on_ = (long long)min(max(k + 1, 0), nz - 1) * plane;
    ld_raw<T, VX>(Ei0 + on_, o0, rE0, on && pn);
    ld_raw<T, VX>(Ei1 + on_, o0, rE1, on && pn && !loader);
    ld_raw<T, VX>(Ei2 + on_, o0, rE2, on && pn);
    ld_raw<T, VX>(Hi0 + ok, o0, rH0, on && pk && !loader);
    ld_raw<T, VX>(Hi1 + ok, o0, rH1, on && pk && !loader);
    ld_raw<T, VX>(Hi2 + ok, o0, rH2, on && pk && !loader);
    rq0 = rq1 = rq2 = rq3 = 0.f;
    if (lane < np2 && act && pk && !loader) {
      const long long prow = ((long long)k * ny + jc) * np2;
      rq0 = d.psi_h[par][0][0][prow + lane];
      rq1 = d.psi_h[par][0][1][prow + lane];
      rq2 = d.psi_e[0][0][prow + lane];
      rq3 = d.psi_e[0][1][prow + lane];
    }
  };
  issue(k0 - 2);
  __syncthreads();

  // carried between iterations: stage-1 H and E of the previous plane, stage-2 H two planes back,
  // y/z-slab psi of the previous plane's stage 1
  float h1x[VX], h1y[VX], h1z[VX], h2x[VX], h2y[VX];
  float c_hxy[VX], c_hzy[VX], c_hxz[VX], c_hyz[VX], c_exy[VX], c_ezy[VX], c_exz[VX], c_eyz[VX];
#pragma unroll
  for (int v = 0; v < VX; v++) {
    h1x[v] = h1y[v] = h1z[v] = h2x[v] = h2y[v] = 0.f;
    c_hxy[v] = c_hzy[v] = c_hxz[v] = c_hyz[v] = c_exy[v] = c_ezy[v] = c_exz[v] = c_eyz[v] = 0.f;
  }

  for (int k = k0 - 2; k <= k1; k++) {
    const int m = k - 1;
    const bool pk = k >= 0 && k <= nz - 1;           // stage-1 plane exists
    const bool st1E = pk && k >= k0 - 1;             // stage-1 E(k) is needed
    const bool st2H = m >= k0 - 1 && m >= 0;         // stage-2 H(m) is needed (m <= k1 - 1 < nz)
    const bool st2E = m >= k0;                       // stage-2 E(m) is stored
    // this iteration's operands
    float nxc[VX], nyc[VX], h0x[VX], h0y[VX], h0z[VX];
    unpack<T, VX>(rE0, nxc);
    unpack<T, VX>(rE1, nyc);
    unpack<T, VX>(rH0, h0x);
    unpack<T, VX>(rH1, h0y);
    unpack<T, VX>(rH2, h0z);
    float q0 = rq0, q1 = rq1, q2 = rq2, q3 = rq3;
    if constexpr (DYN) {
      scale_in<VX>(nxc, dyn_r);
      scale_in<VX>(nyc, dyn_r);
      scale_in<VX>(h0x, dyn_r);
      scale_in<VX>(h0y, dyn_r);
      scale_in<VX>(h0z, dyn_r);
      q0 *= dyn_r;
      q1 *= dyn_r;
      q2 *= dyn_r;
      q3 *= dyn_r;
    }
    // y/z-slab psi rows of stage 1 at plane k (boundary tiles only)
    float qhxy[VX], qhzy[VX], qhxz[VX], qhyz[VX], qexy[VX], qezy[VX], qexz[VX], qeyz[VX];
    int shz1 = -1, sez1 = -1;
    if constexpr (GY) {
      const int kk = min(max(k, 0), nz - 1);
      shz1 = GZ && np2 > 0 && pk ? d.ax[2].sh[kk] : -1;
      sez1 = GZ && np2 > 0 && pk ? d.ax[2].se[kk] : -1;
      const long long iyh = ((long long)kk * np2 + max(shy, 0)) * d.pitch + ib;
      const long long iye = ((long long)kk * np2 + max(sey, 0)) * d.pitch + ib;
      const long long izh = ((long long)max(shz1, 0) * ny + jc) * d.pitch + ib;
      const long long ize = ((long long)max(sez1, 0) * ny + jc) * d.pitch + ib;
      ld_row<float, VX>(d.psi_h[par][1][0] + iyh, qhxy, on && pk && shy >= 0);
      ld_row<float, VX>(d.psi_h[par][1][1] + iyh, qhzy, on && pk && shy >= 0);
      ld_row<float, VX>(d.psi_h[par][2][0] + izh, qhxz, on && pk && shz1 >= 0);
      ld_row<float, VX>(d.psi_h[par][2][1] + izh, qhyz, on && pk && shz1 >= 0);
      ld_row<float, VX>(d.psi_e[1][0] + iye, qexy, on && pk && sey >= 0);
      ld_row<float, VX>(d.psi_e[1][1] + iye, qezy, on && pk && sey >= 0);
      ld_row<float, VX>(d.psi_e[2][0] + ize, qexz, on && pk && sez1 >= 0);
      ld_row<float, VX>(d.psi_e[2][1] + ize, qeyz, on && pk && sez1 >= 0);
      if constexpr (DYN) {
        scale_in<VX>(qhxy, dyn_r);
        scale_in<VX>(qhzy, dyn_r);
        scale_in<VX>(qhxz, dyn_r);
        scale_in<VX>(qhyz, dyn_r);
        scale_in<VX>(qexy, dyn_r);
        scale_in<VX>(qezy, dyn_r);
        scale_in<VX>(qexz, dyn_r);
        scale_in<VX>(qeyz, dyn_r);
      }
    } else {
#pragma unroll
      for (int v = 0; v < VX; v++) qhxy[v] = qhzy[v] = qhxz[v] = qhyz[v] = qexy[v] = qezy[v] = qexz[v] = qeyz[v] = 0.f;
    }
    const int pb = k & 1, pm = m & 1;
    if (lane < np2 && !loader) {
      float *p0 = PS(pb, 0), *p1 = PS(pb, 1), *p2 = PS(pb, 2), *p3 = PS(pb, 3);
      p0[lane] = q0;
      p1[lane] = q1;
      p2[lane] = q2;
      p3[lane] = q3;
    }

    // ---- A: stage-1 H(k)
    float hx[VX], hy[VX], hz[VX];
    if (pk && doH1) {
      float uax[VX], uaz[VX], e0x[VX], e0y[VX], e0z[VX];
#pragma unroll
      for (int v = 0; v < VX; v++) {
        uax[v] = sE0x[r + 1][ib + v];
        uaz[v] = sE0z[r + 1][ib + v];
        e0x[v] = sE0x[r][ib + v];
        e0y[v] = sE0y[r][ib + v];
        e0z[v] = sE0z[r][ib + v];
      }
      // the next node's Ey, Ez: the row is contiguous in LDS across the waves of a split row (the
      // last node of the row reads a clamped slot; its update does not use it)
      const int inx = min(ib + VX, NL - 1);
      const float eyn = sE0y[r][inx], ezn = sE0z[r][inx];
      h_upd(k, h0x, h0y, h0z, e0x, e0y, e0z, nxc, nyc, uax, uaz, eyn, ezn, pb, qhxy, qhzy, qhxz, qhyz, hx, hy, hz);
    } else {
#pragma unroll
      for (int v = 0; v < VX; v++) hx[v] = hy[v] = hz[v] = 0.f;
    }
    if (r <= W + 1) {
#pragma unroll
      for (int v = 0; v < VX; v++) {
        sH1x[r][ib + v] = hx[v];
        sH1z[r][ib + v] = hz[v];
      }
      if constexpr (XS > 1) {
        if (lane == 63) {
          sBH1[r][xs][0] = hy[VX - 1];
          sBH1[r][xs][1] = hz[VX - 1];
        }
      }
    }
    __syncthreads();

    // ---- B: stage-1 E(k), stage-2 H(m)
    float ox[VX], oy[VX], oz[VX];
    if (doE1 && st1E) {
      float bx[VX], bz[VX], e0x[VX], e0y[VX], e0z[VX];
#pragma unroll
      for (int v = 0; v < VX; v++) {
        bx[v] = sH1x[r - 1][ib + v];
        bz[v] = sH1z[r - 1][ib + v];
        e0x[v] = sE0x[r][ib + v];
        e0y[v] = sE0y[r][ib + v];
        e0z[v] = sE0z[r][ib + v];
      }
      const float hzw0 = prev_of(hz[VX - 1], &sBH1[r][0][1]), hyw0 = prev_of(hy[VX - 1], &sBH1[r][0][0]);
      e_upd(k, e0x, e0y, e0z, hx, hy, hz, h1x, h1y, bx, bz, hzw0, hyw0, pb, qexy, qezy, qexz, qeyz, ox, oy, oz);
      src_apply<T, VX>(d, sSrc, 0, ib, j, k, oz);
      // samples of E^{n+1} at the observers' stencil nodes (rows and planes this tile owns)
      if (own && k >= k0 && k < k1 && d.smp_ptr) {
        const int e_lo = d.smp_ptr[k], e_hi = d.smp_ptr[k + 1];
        for (int e = e_lo; e < e_hi; e++) {
          const int4 en = d.smp_ent[e];
          if (en.x != j) continue;
          // static indices only (a selected register array would go to scratch memory)
#pragma unroll
          for (int v = 0; v < VX; v++) {
            if (en.y != ib + v) continue;
            float val = oz[v];
            if (en.z == 0) val = ox[v];
            if (en.z == 1) val = oy[v];
            d.smp[en.w] = val;
          }
        }
      }
    } else {
#pragma unroll
      for (int v = 0; v < VX; v++) ox[v] = oy[v] = oz[v] = 0.f;
    }
    if (r >= 1 && r <= NR - 1) {
#pragma unroll
      for (int v = 0; v < VX; v++) {
        sE1x[pb][r - 1][ib + v] = ox[v];
        sE1y[pb][r - 1][ib + v] = oy[v];
        sE1z[pb][r - 1][ib + v] = oz[v];
      }
    }
    float gx[VX], gy[VX], gz[VX];
    if (doH2 && st2H) {
      float uax[VX], uaz[VX], e1x[VX], e1y[VX], e1z[VX];
#pragma unroll
      for (int v = 0; v < VX; v++) {
        uax[v] = sE1x[pm][r][ib + v];
        uaz[v] = sE1z[pm][r][ib + v];
        e1x[v] = sE1x[pm][r - 1][ib + v];
        e1y[v] = sE1y[pm][r - 1][ib + v];
        e1z[v] = sE1z[pm][r - 1][ib + v];
      }
      const int inx = min(ib + VX, NL - 1);
      const float eyn = sE1y[pm][r - 1][inx], ezn = sE1z[pm][r - 1][inx];
      h_upd(m, h1x, h1y, h1z, e1x, e1y, e1z, ox, oy, uax, uaz, eyn, ezn, pm, c_hxy, c_hzy, c_hxz, c_hyz, gx, gy, gz);
    } else {
#pragma unroll
      for (int v = 0; v < VX; v++) gx[v] = gy[v] = gz[v] = 0.f;
    }
    if (r >= 1 && r <= W) {
#pragma unroll
      for (int v = 0; v < VX; v++) {
        sH2x[r - 1][ib + v] = gx[v];
        sH2z[r - 1][ib + v] = gz[v];
      }
    }
    if constexpr (XS > 1) {
      if (lane == 63) {
        sBH2[r][xs][0] = gy[VX - 1];
        sBH2[r][xs][1] = gz[VX - 1];
      }
    }
    // E^n(k+1) of the row for the next iteration (its own stages and the row below's H); then the
    // next iteration's row loads, in flight through stage-2 E and the barriers
    {
      float t0[VX], t1[VX], t2[VX];
      unpack<T, VX>(rE0, t0);
      unpack<T, VX>(rE1, t1);
      unpack<T, VX>(rE2, t2);
      if constexpr (DYN) {
        scale_in<VX>(t0, dyn_r);
        scale_in<VX>(t1, dyn_r);
        scale_in<VX>(t2, dyn_r);
      }
#pragma unroll
      for (int v = 0; v < VX; v++) {
        sE0x[r][ib + v] = t0[v];
        sE0y[r][ib + v] = t1[v];
        sE0z[r][ib + v] = t2[v];
      }
    }
    issue(k + 1);
    __syncthreads();

    // ---- C: stage-2 E(m), stores
    if (own && st2E) {
      float bx[VX], bz[VX], fx[VX], fy[VX], fz[VX], e1x[VX], e1y[VX], e1z[VX];
#pragma unroll
      for (int v = 0; v < VX; v++) {
        bx[v] = sH2x[r - 2][ib + v];
        bz[v] = sH2z[r - 2][ib + v];
        e1x[v] = sE1x[pm][r - 1][ib + v];
        e1y[v] = sE1y[pm][r - 1][ib + v];
        e1z[v] = sE1z[pm][r - 1][ib + v];
      }
      const float hzw0 = prev_of(gz[VX - 1], &sBH2[r][0][1]), hyw0 = prev_of(gy[VX - 1], &sBH2[r][0][0]);
      e_upd(m, e1x, e1y, e1z, gx, gy, gz, h2x, h2y, bx, bz, hzw0, hyw0, pm, c_exy, c_ezy, c_exz, c_eyz, fx, fy, fz);
      src_apply<T, VX>(d, sSrc, 1, ib, j, m, fz);
      const long long pmo = (long long)m * plane;
      if constexpr (DYN) {
        dyn_mh = absmax<VX>(absmax<VX>(absmax<VX>(dyn_mh, gx, on), gy, on), gz, on);
        dyn_me = absmax<VX>(absmax<VX>(absmax<VX>(dyn_me, fx, on), fy, on), fz, on);
      }
      st_at<T, VX>(Ho0 + pmo, o0, gx, on);
      st_at<T, VX>(Ho1 + pmo, o0, gy, on);
      st_at<T, VX>(Ho2 + pmo, o0, gz, on);
      st_at<T, VX>(Eo0 + pmo, o0, fx, on);
      st_at<T, VX>(Eo1 + pmo, o0, fy, on);
      st_at<T, VX>(Eo2 + pmo, o0, fz, on);
      if (lane < np2) {
        const long long prow = ((long long)m * ny + jc) * np2;
        if (ownH) {
          d.psi_h[par ^ 1][0][0][prow + lane] = PS(pm, 0)[lane];
          d.psi_h[par ^ 1][0][1][prow + lane] = PS(pm, 1)[lane];
        }
        if (ownE) {
          d.psi_e2[0][0][prow + lane] = PS(pm, 2)[lane];
          d.psi_e2[0][1][prow + lane] = PS(pm, 3)[lane];
        }
      }
      if constexpr (GY) {
        const int shz2 = GZ && np2 > 0 ? d.ax[2].sh[m] : -1, sez2 = GZ && np2 > 0 ? d.ax[2].se[m] : -1;
        if (shy >= 0) {
          const long long iyh = ((long long)m * np2 + shy) * d.pitch + ib;
          st_row<float, VX>(d.psi_h[par ^ 1][1][0] + iyh, c_hxy, on);
          st_row<float, VX>(d.psi_h[par ^ 1][1][1] + iyh, c_hzy, on);
        }
        if (shz2 >= 0) {
          const long long izh = ((long long)shz2 * ny + jc) * d.pitch + ib;
          st_row<float, VX>(d.psi_h[par ^ 1][2][0] + izh, c_hxz, on);
          st_row<float, VX>(d.psi_h[par ^ 1][2][1] + izh, c_hyz, on);
        }
        if (sey >= 0) {
          const long long iye = ((long long)m * np2 + sey) * d.pitch + ib;
          st_row<float, VX>(d.psi_e2[1][0] + iye, c_exy, on);
          st_row<float, VX>(d.psi_e2[1][1] + iye, c_ezy, on);
        }
        if (sez2 >= 0) {
          const long long ize = ((long long)sez2 * ny + jc) * d.pitch + ib;
          st_row<float, VX>(d.psi_e2[2][0] + ize, c_exz, on);
          st_row<float, VX>(d.psi_e2[2][1] + ize, c_eyz, on);
        }
      }
    }
    // rotate: this plane's stage-1 values become the previous plane's
#pragma unroll
    for (int v = 0; v < VX; v++) {
      h2x[v] = gx[v];
      h2y[v] = gy[v];
      h1x[v] = hx[v];
      h1y[v] = hy[v];
      h1z[v] = hz[v];
      if constexpr (GY) {
        c_hxy[v] = qhxy[v];
        c_hzy[v] = qhzy[v];
        c_hxz[v] = qhxz[v];
        c_hyz[v] = qhyz[v];
        c_exy[v] = qexy[v];
        c_ezy[v] = qezy[v];
        c_exz[v] = qexz[v];
        c_eyz[v] = qeyz[v];
      }
    }
  }
  if constexpr (DYN) {
    unsigned *slot = d.dmax + 2 * ((*d.dslot[par] + 1) % 3);
    dyn_raise(slot, dyn_me);
    dyn_raise(slot + 1, dyn_mh);
  }
}

// The interior rectangle (no wall and no y/z layer within any computed row or plane).
template <typename T, int VX, int W, int XS, bool DYN = false>
__global__ void __launch_bounds__(64 * (W + 4) * XS) k_step2(Dev d, Shape2 f2, int par, int step, const double *q) {
  const int logical = xcd_logical();
  if (logical >= f2.n_fast) return;
  const int fw = f2.ty_hi - f2.ty_lo;
  const int j0 = (f2.ty_lo + logical % fw) * W - f2.ysh;
  const int k0 = (f2.zc_lo + logical / fw) * f2.zchunk - f2.zsh;
  step2_body<T, VX, W, XS, 0, DYN>(d, j0, j0 + W, k0, k0 + f2.zchunk, par, step, q);
}

// Boundary tiles of kStep2BoundaryRows rows from the table (first row, end of the rows the tile
// owns, chunk): G = 1 over the first n_slow_y entries (y walls and layers), G = 2 over the rest
// (z walls and layers as well).
template <typename T, int VX, int XS, int G, bool DYN = false>
__global__ void __launch_bounds__(64 * (kStep2BoundaryRows + 4) * XS)
    k_step2_gen(Dev d, Shape2 f2, const int *tiles, int n, int par, int step, const double *q) {
  const int logical = xcd_logical();
  if (logical >= n) return;
  const int *t = tiles + 3 * logical;
  const int k0 = t[2] * f2.zchunk - f2.zsh;
  step2_body<T, VX, kStep2BoundaryRows, XS, G, DYN>(d, t[0], t[1], max(k0, 0), min(k0 + f2.zchunk, d.nz), par, step, q);
}

template <typename T>
__global__ void __launch_bounds__(64) k_gather_level(Dev d, int par, double *w, int column, int ld) {
  gather_body<T>(d, par, w, column, ld, blockIdx.x);
}

// Waveform column of the intermediate level from the samples a two-step pass took: the
// one-step gather's arithmetic (FP64 weight times the stored value, butterfly over the corners).
__global__ void __launch_bounds__(64) k_gather_smp(Dev d, int par, double *w, int column, int ld) {
  const int o = blockIdx.x, lane = threadIdx.x;
  const int comp = lane >> 3, corner = lane & 7;
  double val = 0.0;
  if (comp < 3) {
    const double *tf = d.obs_t + (o * 3 + comp) * 3;
    const int a = corner & 1, b = (corner >> 1) & 1, c = corner >> 2;
    const double wgt = (a ? tf[0] : 1.0 - tf[0]) * (b ? tf[1] : 1.0 - tf[1]) * (c ? tf[2] : 1.0 - tf[2]);
    val = wgt * (double)d.smp[d.smp_slot[(o * 3 + comp) * 8 + corner]];
  }
  val += __shfl_xor(val, 1);
  val += __shfl_xor(val, 2);
  val += __shfl_xor(val, 4);
  if (comp < 3 && corner == 0) {
    // samples are in the units of level `par` (dynamic scaling: the level the pass wrote)
    const double out = val * (d.dyn ? ldexp(d.inv_se, -*d.dexp[par]) : d.inv_se);
    w[((long long)o * 3 + comp) * ld + column] = out;
    if (d.nan_flag && !isfinite(out)) *d.nan_flag = 1;
  }
}

template <typename T, int VX, int W, bool DYN>
static hipError_t step2_launch(const chf_plan &p, const Dev &d, int par, int step, const double *q, bool general,
                               hipStream_t s, int part) {
  const Shape2 &f2 = p.fs2;
  if (general) {
    const dim3 block(64 * (kStep2BoundaryRows + 4));
    const int *tiles = (const int *)(p.ws + p.off_tiles2);
    const int n1 = f2.n_slow_y, n2 = f2.n_slow - f2.n_slow_y;
    if (n1 > 0 && (part & 1))
      hipLaunchKernelGGL((k_step2_gen<T, VX, 1, 1, DYN>), dim3((n1 + 7) / 8 * 8), block, 0, s, d, f2, tiles, n1, par, step,
                         q);
    if (n2 > 0 && (part & 2))
      hipLaunchKernelGGL((k_step2_gen<T, VX, 1, 2, DYN>), dim3((n2 + 7) / 8 * 8), block, 0, s, d, f2, tiles + 3 * n1, n2,
                         par, step, q);
  } else if (f2.n_fast > 0) {
    hipLaunchKernelGGL((k_step2<T, VX, W, 1, DYN>), dim3(f2.fast_blocks), dim3(64 * (W + 4)), 0, s, d, f2, par, step, q);
  }
  return hipGetLastError();
}

template <typename T, bool DYN>
static hipError_t step2_dispatch_t(const chf_plan &p, const Dev &d, int par, int step, const double *q, bool general,
                                   hipStream_t s, int part) {
  const Shape2 &f2 = p.fs2;
  switch (f2.vx * 100 + f2.waves) {
    case 104: return step2_launch<T, 1, 4, DYN>(p, d, par, step, q, general, s, part);
    case 107: return step2_launch<T, 1, 7, DYN>(p, d, par, step, q, general, s, part);
    case 108: return step2_launch<T, 1, 8, DYN>(p, d, par, step, q, general, s, part);
    case 204: return step2_launch<T, 2, 4, DYN>(p, d, par, step, q, general, s, part);
    case 207: return step2_launch<T, 2, 7, DYN>(p, d, par, step, q, general, s, part);
    case 208: return step2_launch<T, 2, 8, DYN>(p, d, par, step, q, general, s, part);
    case 404: return step2_launch<T, 4, 4, DYN>(p, d, par, step, q, general, s, part);
    case 407: return step2_launch<T, 4, 7, DYN>(p, d, par, step, q, general, s, part);
    case 408: return step2_launch<T, 4, 8, DYN>(p, d, par, step, q, general, s, part);
  }
  return hipErrorInvalidValue;
}

// dynamically scaled levels exist for FP16 storage only
template <typename T>
static hipError_t step2_dispatch(const chf_plan &p, const Dev &d, int par, int step, const double *q, bool general,
                                 hipStream_t s, int part = 3) {
  if constexpr (std::is_same<T, _Float16>::value) {
    if (d.dyn) return step2_dispatch_t<T, true>(p, d, par, step, q, general, s, part);
  } else {
    if (d.dyn) return hipErrorInvalidValue;
  }
  return step2_dispatch_t<T, false>(p, d, par, step, q, general, s, part);
}

template <typename T>
static hipError_t step2_t(const chf_plan &p, const Dev &d, int par, int step, const double *q, double *w, int column,
                          int ld, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b) {
  const Shape2 &f2 = p.fs2;
  const double *qq = q ? q : d.q_bins;
  hipError_t e = hipSuccess;
  // boundary tiles on the side stream beside the interior ones (both read only level par and
  // write disjoint nodes of level par^1), the z-boundary tiles on a second side stream beside
  // the y-boundary ones
  const bool fork = f2.n_fast > 0 && f2.n_slow > 0 && p.aux;
  const bool fork2 = fork && p.aux2 && f2.n_slow_y > 0 && f2.n_slow > f2.n_slow_y;
  if (fork) {
    e = hipEventRecord(p.ev_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(p.aux, p.ev_fork, 0);
    if (fork2) {
      if (e == hipSuccess) e = hipStreamWaitEvent(p.aux2, p.ev_fork, 0);
      if (e == hipSuccess) e = step2_dispatch<T>(p, d, par, step, qq, true, p.aux, 1);
      if (e == hipSuccess) e = step2_dispatch<T>(p, d, par, step, qq, true, p.aux2, 2);
      if (e == hipSuccess) e = hipEventRecord(p.ev_join2, p.aux2);
    } else if (e == hipSuccess) {
      e = step2_dispatch<T>(p, d, par, step, qq, true, p.aux);
    }
    if (e == hipSuccess) e = hipEventRecord(p.ev_join, p.aux);
    if (e != hipSuccess) return e;
  }
  if (f2.n_fast > 0) {
    if (ev_a) e = hipEventRecord(ev_a, s);
    if (e == hipSuccess) e = step2_dispatch<T>(p, d, par, step, qq, false, s);
    if (e == hipSuccess && ev_b) e = hipEventRecord(ev_b, s);
    if (e != hipSuccess) return e;
  }
  if (f2.n_slow > 0) {
    e = fork ? hipStreamWaitEvent(s, p.ev_join, 0) : step2_dispatch<T>(p, d, par, step, qq, true, s);
    if (e == hipSuccess && fork2) e = hipStreamWaitEvent(s, p.ev_join2, 0);
    if (e != hipSuccess) return e;
  }
  if (d.dyn) {
    e = launch_dyn_publish(d, par, 2, s);
    if (e != hipSuccess) return e;
  }
  if (d.n_obs > 0 && w) {
    hipLaunchKernelGGL(k_gather_smp, dim3(d.n_obs), dim3(64), 0, s, d, par ^ 1, w, column, ld);
    hipLaunchKernelGGL(k_gather_level<T>, dim3(d.n_obs), dim3(64), 0, s, d, par ^ 1, w, column + 1, ld);
  }
  return hipGetLastError();
}

hipError_t launch_step2(const chf_plan &p, const Dev &d, int par, int step, const double *q, double *w, int column,
                        int ld, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b) {
  switch (p.storage) {
    case CHF_FP32: return step2_t<float>(p, d, par, step, q, w, column, ld, s, ev_a, ev_b);
    case CHF_BF16: return step2_t<__bf16>(p, d, par, step, q, w, column, ld, s, ev_a, ev_b);
    case CHF_BF16X: return step2_t<bf16x>(p, d, par, step, q, w, column, ld, s, ev_a, ev_b);
    case CHF_FP16: return step2_t<_Float16>(p, d, par, step, q, w, column, ld, s, ev_a, ev_b);
  }
  return hipErrorInvalidValue;
}

}  // namespace chf
