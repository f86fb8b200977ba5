// HIP kernels of libchfdtd for gfx950 (CDNA4, wave64).
//
// Step n reads time level `par` (E^n, H^{n-1/2}) and writes level par^1 (H^{n+1/2},
// E^{n+1}); both levels live in HBM, so a single sweep can recompute tile halos from the
// untouched input level without racing neighbouring workgroups.
//
// Per-cell arithmetic (FP32, explicit fmaf, built with -ffp-contract=off) lives in h_cell /
// e_cell / pml_psi and is shared by every sweep variant, so the fused single sweep and the
// split E/H sweeps produce identical bits.
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
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "chf_internal.h"

namespace chf {

// ------------------------------------------------------------------ storage
template <typename T>
__device__ __forceinline__ float to_f(T x) { return static_cast<float>(x); }
template <typename T>
__device__ __forceinline__ T from_f(float x) { return static_cast<T>(x); }  // RNE

template <typename T, int N>
struct alignas(sizeof(T) * N) Vec {
  T v[N];
};

// Lanes whose cells start beyond the last node (`on` false) neither load nor store.
template <typename T, int N>
__device__ __forceinline__ void ld_row(const T *p, float (&o)[N], bool on) {
  if (on) {
    Vec<T, N> x = *reinterpret_cast<const Vec<T, N> *>(p);
#pragma unroll
    for (int v = 0; v < N; v++) o[v] = to_f<T>(x.v[v]);
  } else {
#pragma unroll
    for (int v = 0; v < N; v++) o[v] = 0.f;
  }
}

template <typename T, int N>
__device__ __forceinline__ void st_row(T *p, const float (&o)[N], bool on) {
  if (!on) return;
  Vec<T, N> x;
#pragma unroll
  for (int v = 0; v < N; v++) x.v[v] = from_f<T>(o[v]);
  *reinterpret_cast<Vec<T, N> *>(p) = x;
}

// ------------------------------------------------------------- cell updates
__device__ __forceinline__ float pml_psi(float psi, float a, float b, float d) {
  return fmaf(b, psi, a * d);
}

// h' = h - c1 d1 + c2 d2 (- p1 + p2)
__device__ __forceinline__ float h_cell(float h, float d1, float c1, float d2, float c2, bool q1,
                                        float p1, bool q2, float p2) {
  float t = fmaf(-c1, d1, h);
  t = fmaf(c2, d2, t);
  if (q1) t = t - p1;
  if (q2) t = t + p2;
  return t;
}

// e' = ca e + c1 d1 - c2 d2 (+ p1 - p2)
__device__ __forceinline__ float e_cell(float ca, float e, float d1, float c1, float d2, float c2,
                                        bool q1, float p1, bool q2, float p2) {
  float t = ca * e;
  t = fmaf(c1, d1, t);
  t = fmaf(-c2, d2, t);
  if (q1) t = t + p1;
  if (q2) t = t - p2;
  return t;
}

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

// --------------------------------------------------------------- fused sweep
// One wave owns R consecutive y rows of the full x extent (64 lanes x VX cells, nx <= 64 VX)
// and marches a z chunk.  Per plane it recomputes the H row just below its first row (the
// E update needs H^{n+1/2}(j0-1)) and, at the chunk start, the H plane below.  x neighbours
// move between lanes with shuffles.  Workgroups are laid out so that consecutive logical
// tiles (neighbours in y, then in z) land on the same XCD and share its L2.
template <typename T, int VX, int R>
__global__ void __launch_bounds__(256) k_fused(Dev d, FusedShape fs, int par) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int b = blockIdx.x;
  const int logical = (b & 7) * (gridDim.x >> 3) + (b >> 3);
  if (logical >= fs.n_tiles) return;
  const int ty = logical % fs.nty;
  const int zc = logical / fs.nty;
  const int j0 = (ty * fs.waves + wave) * R;
  if (j0 >= d.ny) return;
  const int k0 = zc * fs.zchunk;
  const int k1 = min(k0 + fs.zchunk, d.nz);
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const int ib = lane * VX;
  const bool on = ib < nx;

  const T *Ei0 = (const T *)d.e[par][0], *Ei1 = (const T *)d.e[par][1], *Ei2 = (const T *)d.e[par][2];
  const T *Hi0 = (const T *)d.h[par][0], *Hi1 = (const T *)d.h[par][1], *Hi2 = (const T *)d.h[par][2];
  T *Eo0 = (T *)d.e[par ^ 1][0], *Eo1 = (T *)d.e[par ^ 1][1], *Eo2 = (T *)d.e[par ^ 1][2];
  T *Ho0 = (T *)d.h[par ^ 1][0], *Ho1 = (T *)d.h[par ^ 1][1], *Ho2 = (T *)d.h[par ^ 1][2];
  const bool pml = d.np2 > 0;

  // per-lane x tables
  float cex[VX], chx[VX];
  int sex[VX], shx[VX];
#pragma unroll
  for (int v = 0; v < VX; v++) {
    int i = ib + v, ic = min(i, nx - 1);
    cex[v] = d.ax[0].ce[ic];
    chx[v] = d.ax[0].ch[ic];
    sex[v] = (pml && i < nx) ? d.ax[0].se[i] : -1;
    shx[v] = (pml && i < nx) ? d.ax[0].sh[i] : -1;
  }
  // rows r = -1..R (array index r+1), clamped into the grid
  int jr[R + 2];
  float cey[R + 2], chy[R + 2];
  int sey[R + 2], shy[R + 2];
#pragma unroll
  for (int r = 0; r < R + 2; r++) {
    int j = j0 + r - 1;
    int jc = min(max(j, 0), ny - 1);
    jr[r] = jc;
    cey[r] = d.ax[1].ce[jc];
    chy[r] = d.ax[1].ch[jc];
    sey[r] = pml ? d.ax[1].se[jc] : -1;
    shy[r] = pml ? d.ax[1].sh[jc] : -1;
  }
  auto at = [&](int r, int k) -> long long {
    return (long long)k * d.plane + (long long)jr[r] * d.pitch + ib;
  };

  float ex[R + 2][VX], ey[R + 2][VX], ez[R + 2][VX];
  float hxp[R][VX], hyp[R][VX];

  // ---- prologue: H^{n+1/2}(k0-1) for Hx, Hy of the owned rows (not stored)
  if (k0 > 0) {
    const int km = k0 - 1;
    const float chz = d.ax[2].ch[km];
    const int shz = pml ? d.ax[2].sh[km] : -1;
    float ezR[VX];
    ld_row<T, VX>(Ei2 + at(R + 1, km), ezR, on);
#pragma unroll
    for (int r = 0; r < R; r++) {
      float exm[VX], eym[VX], ezm[VX], ex0[VX], ey0[VX], hxo[VX], hyo[VX], ez1[VX];
      ld_row<T, VX>(Ei0 + at(r + 1, km), exm, on);
      ld_row<T, VX>(Ei1 + at(r + 1, km), eym, on);
      ld_row<T, VX>(Ei2 + at(r + 1, km), ezm, on);
      ld_row<T, VX>(Ei0 + at(r + 1, k0), ex0, on);
      ld_row<T, VX>(Ei1 + at(r + 1, k0), ey0, on);
      ld_row<T, VX>(Hi0 + at(r + 1, km), hxo, on);
      ld_row<T, VX>(Hi1 + at(r + 1, km), hyo, on);
      if (r + 1 < R) ld_row<T, VX>(Ei2 + at(r + 2, km), ez1, on);
      const int j = j0 + r;
#pragma unroll
      for (int v = 0; v < VX; v++) {
        if (r + 1 >= R) ez1[v] = ezR[v];
      }
      float ezn = __shfl_down(ezm[0], 1);
#pragma unroll
      for (int v = 0; v < VX; v++) {
        const int i = ib + v;
        float ezip = (v + 1 < VX) ? ezm[v + 1] : ezn;
        // Hx(j+1/2, k0-1/2)
        float d1 = ez1[v] - ezm[v], d2 = ey0[v] - eym[v];
        bool q1 = shy[r + 1] >= 0, q2 = shz >= 0;
        float p1 = 0.f, p2 = 0.f;
        bool ux = i < nx && j <= ny - 2 && km <= nz - 2;
        if (q1 && ux) p1 = psi_step(d, d.psi_h[par][1][0], nullptr, false, 1, i, j, km, shy[r + 1],
                              d.ax[1].ah[j], d.ax[1].bh[j], d1);
        if (q2 && ux) p2 = psi_step(d, d.psi_h[par][2][0], nullptr, false, 2, i, j, km, shz,
                              d.ax[2].ah[km], d.ax[2].bh[km], d2);
        hxp[r][v] = ux ? h_cell(hxo[v], d1, chy[r + 1], d2, chz, q1, p1, q2, p2) : hxo[v];
        // Hy(i+1/2, k0-1/2)
        d1 = ex0[v] - exm[v];
        d2 = ezip - ezm[v];
        q1 = shz >= 0;
        q2 = shx[v] >= 0;
        p1 = p2 = 0.f;
        bool uy = i <= nx - 2 && j < ny && km <= nz - 2;
        if (q1 && uy) p1 = psi_step(d, d.psi_h[par][2][1], nullptr, false, 2, i, j, km, shz,
                              d.ax[2].ah[km], d.ax[2].bh[km], d1);
        if (q2 && uy) p2 = psi_step(d, d.psi_h[par][0][0], nullptr, false, 0, i, j, km, shx[v],
                              d.ax[0].ah[i], d.ax[0].bh[i], d2);
        hyp[r][v] = uy ? h_cell(hyo[v], d1, chz, d2, chx[v], q1, p1, q2, p2) : hyo[v];
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
      for (int v = 0; v < VX; v++) hxp[r][v] = hyp[r][v] = 0.f;
  }

  // ---- current plane E(k0), rows -1..R
#pragma unroll
  for (int r = 0; r < R + 2; r++) {
    ld_row<T, VX>(Ei0 + at(r, k0), ex[r], on);
    ld_row<T, VX>(Ei2 + at(r, k0), ez[r], on);
    if (r < R + 1) ld_row<T, VX>(Ei1 + at(r, k0), ey[r], on);
  }

  for (int k = k0; k < k1; k++) {
    const int kn = min(k + 1, nz - 1);
    const float chz = d.ax[2].ch[k], cez = d.ax[2].ce[k];
    const int shz = pml ? d.ax[2].sh[k] : -1, sez = pml ? d.ax[2].se[k] : -1;
    // next plane E(k+1) for rows -1..R, old H(k) for rows -1..R-1
    float nex[R + 2][VX], ney[R + 1][VX], nez[R + 2][VX];
    float hxo[R + 1][VX], hyo[R + 1][VX], hzo[R + 1][VX];
#pragma unroll
    for (int r = 0; r < R + 2; r++) {
      ld_row<T, VX>(Ei0 + at(r, kn), nex[r], on);
      ld_row<T, VX>(Ei2 + at(r, kn), nez[r], on);
      if (r < R + 1) ld_row<T, VX>(Ei1 + at(r, kn), ney[r], on);
    }
#pragma unroll
    for (int r = 0; r < R + 1; r++) {
      ld_row<T, VX>(Hi0 + at(r, k), hxo[r], on);
      ld_row<T, VX>(Hi2 + at(r, k), hzo[r], on);
      if (r > 0) ld_row<T, VX>(Hi1 + at(r, k), hyo[r], on);
    }

    // ---- H^{n+1/2}(k): rows -1..R-1 (row -1 only Hx, Hz; it is not stored)
    float hx[R + 1][VX], hy[R + 1][VX], hz[R + 1][VX];
#pragma unroll
    for (int r = 0; r < R + 1; r++) {
      const int j = j0 + r - 1;
      const bool own = r > 0;
      const bool halo_ok = own || j >= 0;
      float eyn = __shfl_down(ey[r][0], 1);
      float ezn = __shfl_down(ez[r][0], 1);
#pragma unroll
      for (int v = 0; v < VX; v++) {
        const int i = ib + v;
        float eyip = (v + 1 < VX) ? ey[r][v + 1] : eyn;
        float ezip = (v + 1 < VX) ? ez[r][v + 1] : ezn;
        const bool wr = own && j < ny;
        // Hx
        {
          float d1 = ez[r + 1][v] - ez[r][v], d2 = ney[r][v] - ey[r][v];
          bool q1 = shy[r] >= 0, q2 = shz >= 0;
          bool u = halo_ok && i < nx && j <= ny - 2 && k <= nz - 2;
          float p1 = 0.f, p2 = 0.f;
          if (q1 && u) p1 = psi_step(d, d.psi_h[par][1][0], d.psi_h[par ^ 1][1][0], wr, 1, i, j, k,
                                     shy[r], d.ax[1].ah[j], d.ax[1].bh[j], d1);
          if (q2 && u) p2 = psi_step(d, d.psi_h[par][2][0], d.psi_h[par ^ 1][2][0], wr, 2, i, j, k,
                                     shz, d.ax[2].ah[k], d.ax[2].bh[k], d2);
          hx[r][v] = u ? h_cell(hxo[r][v], d1, chy[r], d2, chz, q1, p1, q2, p2) : hxo[r][v];
        }
        // Hz
        {
          float d1 = eyip - ey[r][v], d2 = ex[r + 1][v] - ex[r][v];
          bool q1 = shx[v] >= 0, q2 = shy[r] >= 0;
          bool u = halo_ok && i <= nx - 2 && j <= ny - 2;
          float p1 = 0.f, p2 = 0.f;
          if (q1 && u) p1 = psi_step(d, d.psi_h[par][0][1], d.psi_h[par ^ 1][0][1], wr, 0, i, j, k,
                                     shx[v], d.ax[0].ah[i], d.ax[0].bh[i], d1);
          if (q2 && u) p2 = psi_step(d, d.psi_h[par][1][1], d.psi_h[par ^ 1][1][1], wr, 1, i, j, k,
                                     shy[r], d.ax[1].ah[j], d.ax[1].bh[j], d2);
          hz[r][v] = u ? h_cell(hzo[r][v], d1, chx[v], d2, chy[r], q1, p1, q2, p2) : hzo[r][v];
        }
        // Hy (owned rows only)
        if (own) {
          float d1 = nex[r][v] - ex[r][v], d2 = ezip - ez[r][v];
          bool q1 = shz >= 0, q2 = shx[v] >= 0;
          bool u = i <= nx - 2 && j < ny && k <= nz - 2;
          float p1 = 0.f, p2 = 0.f;
          if (q1 && u) p1 = psi_step(d, d.psi_h[par][2][1], d.psi_h[par ^ 1][2][1], wr, 2, i, j, k,
                                     shz, d.ax[2].ah[k], d.ax[2].bh[k], d1);
          if (q2 && u) p2 = psi_step(d, d.psi_h[par][0][0], d.psi_h[par ^ 1][0][0], wr, 0, i, j, k,
                                     shx[v], d.ax[0].ah[i], d.ax[0].bh[i], d2);
          hy[r][v] = u ? h_cell(hyo[r][v], d1, chz, d2, chx[v], q1, p1, q2, p2) : hyo[r][v];
        } else {
          hy[r][v] = 0.f;
        }
      }
    }
    // store H rows 0..R-1
#pragma unroll
    for (int r = 1; r < R + 1; r++) {
      if (j0 + r - 1 < ny) {
        st_row<T, VX>(Ho0 + at(r, k), hx[r], on);
        st_row<T, VX>(Ho1 + at(r, k), hy[r], on);
        st_row<T, VX>(Ho2 + at(r, k), hz[r], on);
      }
    }

    // ---- E^{n+1}(k): rows 0..R-1
#pragma unroll
    for (int r = 1; r < R + 1; r++) {
      const int j = j0 + r - 1;
      if (j >= ny) continue;
      float hzm = __shfl_up(hz[r][VX - 1], 1);
      float hym = __shfl_up(hy[r][VX - 1], 1);
      float oex[VX], oey[VX], oez[VX];
#pragma unroll
      for (int v = 0; v < VX; v++) {
        const int i = ib + v;
        float hzim = (v > 0) ? hz[r][v - 1] : hzm;
        float hyim = (v > 0) ? hy[r][v - 1] : hym;
        // Ex
        {
          float d1 = hz[r][v] - hz[r - 1][v], d2 = hy[r][v] - hyp[r - 1][v];
          bool u = i <= nx - 2 && j >= 1 && j <= ny - 2 && k >= 1 && k <= nz - 2;
          bool q1 = sey[r] >= 0, q2 = sez >= 0;
          float p1 = 0.f, p2 = 0.f;
          if (q1 && u) p1 = psi_step(d, d.psi_e[1][0], d.psi_e[1][0], true, 1, i, j, k, sey[r],
                                     d.ax[1].ae[j], d.ax[1].be[j], d1);
          if (q2 && u) p2 = psi_step(d, d.psi_e[2][0], d.psi_e[2][0], true, 2, i, j, k, sez,
                                     d.ax[2].ae[k], d.ax[2].be[k], d2);
          oex[v] = u ? e_cell(d.ca, ex[r][v], d1, cey[r], d2, cez, q1, p1, q2, p2) : ex[r][v];
        }
        // Ey
        {
          float d1 = hx[r][v] - hxp[r - 1][v], d2 = hz[r][v] - hzim;
          bool u = i >= 1 && i <= nx - 2 && j <= ny - 2 && k >= 1 && k <= nz - 2;
          bool q1 = sez >= 0, q2 = sex[v] >= 0;
          float p1 = 0.f, p2 = 0.f;
          if (q1 && u) p1 = psi_step(d, d.psi_e[2][1], d.psi_e[2][1], true, 2, i, j, k, sez,
                                     d.ax[2].ae[k], d.ax[2].be[k], d1);
          if (q2 && u) p2 = psi_step(d, d.psi_e[0][0], d.psi_e[0][0], true, 0, i, j, k, sex[v],
                                     d.ax[0].ae[i], d.ax[0].be[i], d2);
          oey[v] = u ? e_cell(d.ca, ey[r][v], d1, cez, d2, cex[v], q1, p1, q2, p2) : ey[r][v];
        }
        // Ez
        {
          float d1 = hy[r][v] - hyim, d2 = hx[r][v] - hx[r - 1][v];
          bool u = i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2 && k <= nz - 2;
          bool q1 = sex[v] >= 0, q2 = sey[r] >= 0;
          float p1 = 0.f, p2 = 0.f;
          if (q1 && u) p1 = psi_step(d, d.psi_e[0][1], d.psi_e[0][1], true, 0, i, j, k, sex[v],
                                     d.ax[0].ae[i], d.ax[0].be[i], d1);
          if (q2 && u) p2 = psi_step(d, d.psi_e[1][1], d.psi_e[1][1], true, 1, i, j, k, sey[r],
                                     d.ax[1].ae[j], d.ax[1].be[j], d2);
          oez[v] = u ? e_cell(d.ca, ez[r][v], d1, cex[v], d2, cey[r], q1, p1, q2, p2) : ez[r][v];
        }
      }
      st_row<T, VX>(Eo0 + at(r, k), oex, on);
      st_row<T, VX>(Eo1 + at(r, k), oey, on);
      st_row<T, VX>(Eo2 + at(r, k), oez, on);
    }

    // ---- march: E(k) <- E(k+1); H(k-1) <- H(k)
#pragma unroll
    for (int r = 0; r < R + 2; r++)
#pragma unroll
      for (int v = 0; v < VX; v++) {
        ex[r][v] = nex[r][v];
        ez[r][v] = nez[r][v];
        if (r < R + 1) ey[r][v] = ney[r][v];
      }
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
      for (int v = 0; v < VX; v++) {
        hxp[r][v] = hx[r + 1][v];
        hyp[r][v] = hy[r + 1][v];
      }
  }
}

// --------------------------------------------------------------- split sweeps
// General-size fallback: one thread per (i, j) column over a z chunk, H then E in two
// launches.  Same per-cell arithmetic as the fused sweep.
constexpr int kSplitZ = 16;

template <typename T>
__global__ void __launch_bounds__(256) k_split_h(Dev d, int par) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= d.nx || j >= d.ny) return;
  const int k0 = blockIdx.z * kSplitZ, k1 = min(k0 + kSplitZ, d.nz);
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const T *E0 = (const T *)d.e[par][0], *E1 = (const T *)d.e[par][1], *E2 = (const T *)d.e[par][2];
  const T *Hi0 = (const T *)d.h[par][0], *Hi1 = (const T *)d.h[par][1], *Hi2 = (const T *)d.h[par][2];
  T *Ho0 = (T *)d.h[par ^ 1][0], *Ho1 = (T *)d.h[par ^ 1][1], *Ho2 = (T *)d.h[par ^ 1][2];
  const bool pml = d.np2 > 0;
  const int ip = min(i + 1, nx - 1), jp = min(j + 1, ny - 1);
  const float chx = d.ax[0].ch[i], chy = d.ax[1].ch[j];
  const int shx = pml ? d.ax[0].sh[i] : -1, shy = pml ? d.ax[1].sh[j] : -1;
  for (int k = k0; k < k1; k++) {
    const int kp = min(k + 1, nz - 1);
    const long long c = (long long)k * d.plane + (long long)j * d.pitch + i;
    const long long cxp = (long long)k * d.plane + (long long)j * d.pitch + ip;
    const long long cyp = (long long)k * d.plane + (long long)jp * d.pitch + i;
    const long long czp = (long long)kp * d.plane + (long long)j * d.pitch + i;
    const float chz = d.ax[2].ch[k];
    const int shz = pml ? d.ax[2].sh[k] : -1;
    float ex = to_f(E0[c]), ey = to_f(E1[c]), ez = to_f(E2[c]);
    {
      float d1 = to_f(E2[cyp]) - ez, d2 = to_f(E1[czp]) - ey;
      bool u = j <= ny - 2 && k <= nz - 2;
      bool q1 = shy >= 0, q2 = shz >= 0;
      float p1 = 0.f, p2 = 0.f;
      if (q1 && u) p1 = psi_step(d, d.psi_h[par][1][0], d.psi_h[par ^ 1][1][0], true, 1, i, j, k, shy,
                                 d.ax[1].ah[j], d.ax[1].bh[j], d1);
      if (q2 && u) p2 = psi_step(d, d.psi_h[par][2][0], d.psi_h[par ^ 1][2][0], true, 2, i, j, k, shz,
                                 d.ax[2].ah[k], d.ax[2].bh[k], d2);
      float h = to_f(Hi0[c]);
      Ho0[c] = from_f<T>(u ? h_cell(h, d1, chy, d2, chz, q1, p1, q2, p2) : h);
    }
    {
      float d1 = to_f(E0[czp]) - ex, d2 = to_f(E2[cxp]) - ez;
      bool u = i <= nx - 2 && k <= nz - 2;
      bool q1 = shz >= 0, q2 = shx >= 0;
      float p1 = 0.f, p2 = 0.f;
      if (q1 && u) p1 = psi_step(d, d.psi_h[par][2][1], d.psi_h[par ^ 1][2][1], true, 2, i, j, k, shz,
                                 d.ax[2].ah[k], d.ax[2].bh[k], d1);
      if (q2 && u) p2 = psi_step(d, d.psi_h[par][0][0], d.psi_h[par ^ 1][0][0], true, 0, i, j, k, shx,
                                 d.ax[0].ah[i], d.ax[0].bh[i], d2);
      float h = to_f(Hi1[c]);
      Ho1[c] = from_f<T>(u ? h_cell(h, d1, chz, d2, chx, q1, p1, q2, p2) : h);
    }
    {
      float d1 = to_f(E1[cxp]) - ey, d2 = to_f(E0[cyp]) - ex;
      bool u = i <= nx - 2 && j <= ny - 2;
      bool q1 = shx >= 0, q2 = shy >= 0;
      float p1 = 0.f, p2 = 0.f;
      if (q1 && u) p1 = psi_step(d, d.psi_h[par][0][1], d.psi_h[par ^ 1][0][1], true, 0, i, j, k, shx,
                                 d.ax[0].ah[i], d.ax[0].bh[i], d1);
      if (q2 && u) p2 = psi_step(d, d.psi_h[par][1][1], d.psi_h[par ^ 1][1][1], true, 1, i, j, k, shy,
                                 d.ax[1].ah[j], d.ax[1].bh[j], d2);
      float h = to_f(Hi2[c]);
      Ho2[c] = from_f<T>(u ? h_cell(h, d1, chx, d2, chy, q1, p1, q2, p2) : h);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_split_e(Dev d, int par) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= d.nx || j >= d.ny) return;
  const int k0 = blockIdx.z * kSplitZ, k1 = min(k0 + kSplitZ, d.nz);
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const T *Ei0 = (const T *)d.e[par][0], *Ei1 = (const T *)d.e[par][1], *Ei2 = (const T *)d.e[par][2];
  const T *H0 = (const T *)d.h[par ^ 1][0], *H1 = (const T *)d.h[par ^ 1][1], *H2 = (const T *)d.h[par ^ 1][2];
  T *Eo0 = (T *)d.e[par ^ 1][0], *Eo1 = (T *)d.e[par ^ 1][1], *Eo2 = (T *)d.e[par ^ 1][2];
  const bool pml = d.np2 > 0;
  const int im = max(i - 1, 0), jm = max(j - 1, 0);
  const float cex = d.ax[0].ce[i], cey = d.ax[1].ce[j];
  const int sex = pml ? d.ax[0].se[i] : -1, sey = pml ? d.ax[1].se[j] : -1;
  for (int k = k0; k < k1; k++) {
    const int km = max(k - 1, 0);
    const long long c = (long long)k * d.plane + (long long)j * d.pitch + i;
    const long long cxm = (long long)k * d.plane + (long long)j * d.pitch + im;
    const long long cym = (long long)k * d.plane + (long long)jm * d.pitch + i;
    const long long czm = (long long)km * d.plane + (long long)j * d.pitch + i;
    const float cez = d.ax[2].ce[k];
    const int sez = pml ? d.ax[2].se[k] : -1;
    float hx = to_f(H0[c]), hy = to_f(H1[c]), hz = to_f(H2[c]);
    {
      float d1 = hz - to_f(H2[cym]), d2 = hy - to_f(H1[czm]);
      bool u = i <= nx - 2 && j >= 1 && j <= ny - 2 && k >= 1 && k <= nz - 2;
      bool q1 = sey >= 0, q2 = sez >= 0;
      float p1 = 0.f, p2 = 0.f;
      if (q1 && u) p1 = psi_step(d, d.psi_e[1][0], d.psi_e[1][0], true, 1, i, j, k, sey,
                                 d.ax[1].ae[j], d.ax[1].be[j], d1);
      if (q2 && u) p2 = psi_step(d, d.psi_e[2][0], d.psi_e[2][0], true, 2, i, j, k, sez,
                                 d.ax[2].ae[k], d.ax[2].be[k], d2);
      float e = to_f(Ei0[c]);
      Eo0[c] = from_f<T>(u ? e_cell(d.ca, e, d1, cey, d2, cez, q1, p1, q2, p2) : e);
    }
    {
      float d1 = hx - to_f(H0[czm]), d2 = hz - to_f(H2[cxm]);
      bool u = i >= 1 && i <= nx - 2 && j <= ny - 2 && k >= 1 && k <= nz - 2;
      bool q1 = sez >= 0, q2 = sex >= 0;
      float p1 = 0.f, p2 = 0.f;
      if (q1 && u) p1 = psi_step(d, d.psi_e[2][1], d.psi_e[2][1], true, 2, i, j, k, sez,
                                 d.ax[2].ae[k], d.ax[2].be[k], d1);
      if (q2 && u) p2 = psi_step(d, d.psi_e[0][0], d.psi_e[0][0], true, 0, i, j, k, sex,
                                 d.ax[0].ae[i], d.ax[0].be[i], d2);
      float e = to_f(Ei1[c]);
      Eo1[c] = from_f<T>(u ? e_cell(d.ca, e, d1, cez, d2, cex, q1, p1, q2, p2) : e);
    }
    {
      float d1 = hy - to_f(H1[cxm]), d2 = hx - to_f(H0[cym]);
      bool u = i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2 && k <= nz - 2;
      bool q1 = sex >= 0, q2 = sey >= 0;
      float p1 = 0.f, p2 = 0.f;
      if (q1 && u) p1 = psi_step(d, d.psi_e[0][1], d.psi_e[0][1], true, 0, i, j, k, sex,
                                 d.ax[0].ae[i], d.ax[0].be[i], d1);
      if (q2 && u) p2 = psi_step(d, d.psi_e[1][1], d.psi_e[1][1], true, 1, i, j, k, sey,
                                 d.ax[1].ae[j], d.ax[1].be[j], d2);
      float e = to_f(Ei2[c]);
      Eo2[c] = from_f<T>(u ? e_cell(d.ca, e, d1, cex, d2, cey, q1, p1, q2, p2) : e);
    }
  }
}

// ------------------------------------------------------------------- source
// J_z of the moving Gaussian charge snapshot at (n+1/2) dt, subtracted (times scale*Cb)
// from Ez^{n+1}.  Bookkeeping in FP64: bunch position, Q(z_s) from the hat bins, and the
// lattice-normalised longitudinal weights.  One thread per (i, j) of the radial patch.
__device__ __forceinline__ int source_window(const Dev &d, double zs, int *klo) {
  const double half = d.cut_sigmas * d.sigma_z;
  const int lo = (int)ceil((zs - half) / d.dz - 0.5);
  const int hi = (int)floor((zs + half) / d.dz - 0.5);
  *klo = lo;
  return min(hi - lo + 1, kMaxWz);
}

__device__ __forceinline__ double source_q(const Dev &d, const double *q, double zs) {
  const double u = (zs - d.z_bin0) / d.dz_bin;
  const double fl = floor(u);
  const int b0 = (int)fl;
  const double t = u - fl;
  double acc = 0.0;
  if (b0 >= 0 && b0 < d.n_bins) acc += (1.0 - t) * q[b0];
  if (b0 + 1 >= 0 && b0 + 1 < d.n_bins) acc += t * q[b0 + 1];
  return acc;
}

template <typename T>
__global__ void k_source(Dev d, int out_par, int step, const double *q) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.src_ni * d.src_nj) return;
  const double tt = (step + 0.5) * d.dt;
  if (tt < d.t_entry) return;
  const double wr = d.wr[t];
  if (wr == 0.0) return;
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
  for (int s = 0; s < m; s++) {
    const int k = klo + s;
    if (k < 0 || k > d.nz - 2) continue;
    const double dd = (klo + s + 0.5) * d.dz - zs;
    const double wz = exp(-0.5 * dd * dd / (d.sigma_z * d.sigma_z)) / norm;
    const double inc = d.cb_src * d.v_src * qz * wr * wz;
    const long long c = (long long)k * d.plane + (long long)j * d.pitch + i;
    Ez[c] = from_f<T>(to_f(Ez[c]) - (float)inc);
  }
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
// One wave per observer: lane = 8*component + corner.  Each lane forms weight * E in FP64,
// then a butterfly over the 8 corners sums each component; lanes 0, 8, 16 write.
template <typename T>
__global__ void __launch_bounds__(64) k_gather(Dev d, int par, double *w, int column, int ld) {
  const int o = blockIdx.x;
  const int lane = threadIdx.x;
  const int comp = lane >> 3, corner = lane & 7;
  double val = 0.0;
  if (comp < 3) {
    const int *ix = d.obs_idx + (o * 3 + comp) * 3;
    const double *tf = d.obs_t + (o * 3 + comp) * 3;
    const int a = corner & 1, b = (corner >> 1) & 1, c = corner >> 2;
    const double wgt = (a ? tf[0] : 1.0 - tf[0]) * (b ? tf[1] : 1.0 - tf[1]) * (c ? tf[2] : 1.0 - tf[2]);
    const long long node = (long long)(ix[2] + c) * d.plane + (long long)(ix[1] + b) * d.pitch + ix[0] + a;
    const T *E = (const T *)d.e[par][comp];
    val = wgt * (double)to_f(E[node]);
  }
  val += __shfl_xor(val, 1);
  val += __shfl_xor(val, 2);
  val += __shfl_xor(val, 4);
  if (comp < 3 && corner == 0) {
    const double out = val * d.inv_se;
    w[((long long)o * 3 + comp) * ld + column] = out;
    if (d.nan_flag && !isfinite(out)) *d.nan_flag = 1;
  }
}

// ------------------------------------------------------------ fill / copies
__global__ void k_fill_zero(uint4 *p, long long n16) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n16;
       t += (long long)gridDim.x * blockDim.x)
    p[t] = make_uint4(0u, 0u, 0u, 0u);
}

template <typename T>
__global__ void k_get_field(Dev d, const T *src, float *out, float inv_scale) {
  const long long n = (long long)d.nx * d.ny * d.nz;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t % d.nx);
    const long long r = t / d.nx;
    const int j = (int)(r % d.ny), k = (int)(r / d.ny);
    out[t] = to_f(src[(long long)k * d.plane + (long long)j * d.pitch + i]) * inv_scale;
  }
}

template <typename T>
__global__ void k_set_field(Dev d, T *dst, const float *in, float scale) {
  const long long n = (long long)d.nx * d.ny * d.nz;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t % d.nx);
    const long long r = t / d.nx;
    const int j = (int)(r % d.ny), k = (int)(r / d.ny);
    dst[(long long)k * d.plane + (long long)j * d.pitch + i] = from_f<T>(in[t] * scale);
  }
}

// ------------------------------------------------------------------ launch
template <typename T, int VX, int R>
static hipError_t fused_launch(const chf_plan &p, const Dev &d, int par, hipStream_t s) {
  hipLaunchKernelGGL((k_fused<T, VX, R>), dim3(p.fs.n_blocks), dim3(64 * p.fs.waves), 0, s, d, p.fs, par);
  return hipGetLastError();
}

template <typename T, int VX>
static hipError_t fused_dispatch_r(const chf_plan &p, const Dev &d, int par, hipStream_t s) {
  switch (p.fs.rows) {
    case 1: return fused_launch<T, VX, 1>(p, d, par, s);
    case 2: return fused_launch<T, VX, 2>(p, d, par, s);
    case 4: return fused_launch<T, VX, 4>(p, d, par, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t fused_dispatch(const chf_plan &p, const Dev &d, int par, hipStream_t s) {
  switch (p.fs.vx) {
    case 1: return fused_dispatch_r<T, 1>(p, d, par, s);
    case 2: return fused_dispatch_r<T, 2>(p, d, par, s);
    case 4: return fused_dispatch_r<T, 4>(p, d, par, s);
    case 8: return fused_dispatch_r<T, 8>(p, d, par, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t step_t(const chf_plan &p, const Dev &d, int par, int step, const double *q,
                         double *w, int column, int ld, hipStream_t s) {
  hipError_t e;
  if (p.kernel == CHF_KERNEL_FUSED) {
    e = fused_dispatch<T>(p, d, par, s);
  } else {
    dim3 grid((d.nx + 63) / 64, (d.ny + 3) / 4, (d.nz + kSplitZ - 1) / kSplitZ);
    hipLaunchKernelGGL(k_split_h<T>, grid, dim3(256), 0, s, d, par);
    hipLaunchKernelGGL(k_split_e<T>, grid, dim3(256), 0, s, d, par);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
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
                       int column, int ld, hipStream_t s) {
  switch (p.storage) {
    case CHF_FP32: return step_t<float>(p, d, par, step, q, w, column, ld, s);
    case CHF_BF16: return step_t<__bf16>(p, d, par, step, q, w, column, ld, s);
    case CHF_FP16: return step_t<_Float16>(p, d, par, step, q, w, column, ld, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_zero(const chf_plan &p, hipStream_t s) {
  // fields and psi occupy [0, off_tf) of the workspace (16-byte multiples)
  const long long n16 = (long long)(p.off_tf / 16);
  hipLaunchKernelGGL(k_fill_zero, dim3(2048), dim3(256), 0, s, (uint4 *)p.ws, n16);
  return hipGetLastError();
}

template <typename T>
static hipError_t get_t(const chf_plan &p, int par, int comp, float *out, hipStream_t s) {
  const T *src = (const T *)(comp < 3 ? p.dev.e[par][comp] : p.dev.h[par][comp - 3]);
  const float inv = (float)(1.0 / (comp < 3 ? p.scale_e : p.scale_h));
  hipLaunchKernelGGL(k_get_field<T>, dim3(1024), dim3(256), 0, s, p.dev, src, out, inv);
  return hipGetLastError();
}

template <typename T>
static hipError_t set_t(const chf_plan &p, int par, int comp, const float *in, hipStream_t s) {
  T *dst = (T *)(comp < 3 ? p.dev.e[par][comp] : p.dev.h[par][comp - 3]);
  const float sc = (float)(comp < 3 ? p.scale_e : p.scale_h);
  hipLaunchKernelGGL(k_set_field<T>, dim3(1024), dim3(256), 0, s, p.dev, dst, in, sc);
  return hipGetLastError();
}

hipError_t launch_get_field(const chf_plan &p, int par, int comp, float *out, hipStream_t s) {
  switch (p.storage) {
    case CHF_FP32: return get_t<float>(p, par, comp, out, s);
    case CHF_BF16: return get_t<__bf16>(p, par, comp, out, s);
    case CHF_FP16: return get_t<_Float16>(p, par, comp, out, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_set_field(const chf_plan &p, int par, int comp, const float *in, hipStream_t s) {
  switch (p.storage) {
    case CHF_FP32: return set_t<float>(p, par, comp, in, s);
    case CHF_BF16: return set_t<__bf16>(p, par, comp, in, s);
    case CHF_FP16: return set_t<_Float16>(p, par, comp, in, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace chf
