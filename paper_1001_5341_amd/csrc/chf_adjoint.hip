// Discrete adjoint of the forward recurrence (FP32 fields, FP64 gradient accumulation).
//
// The forward map q -> w is linear (zero initial fields), so dL/dq = A^T dL/dw.  One reverse
// step n applies, in reverse order, the exact transposes of the forward operations of step n:
//   sampling^T       Eb += G^T g^n                         (one wave, observers in sequence)
//   source^T         dL/dq_b += -Cb v hat_b(z_s) sum W_r W_z Eb_z   (FP64 block reduction)
//   E update^T       per E node and derivative term: tb = +-Cb Eb; in a layer
//                    psib_tot = psib + tb, s = (tb/kappa + a psib_tot)/delta, psib <- b psib_tot,
//                    else s = tb/delta; then Eb <- ca Eb.  Hb gathers s(p) - s(p + e_u).
//   H update^T       same with tb = -+Db Hb; Eb gathers s(p - e_u) - s(p).
// Gathers replace the scatter of the textbook transpose, so every value is written by one
// thread and the result is deterministic.  The forward workspace is reused: level-0 E/H hold
// Eb/Hb, level-1 E/H hold the six per-term cotangents s, the psi slabs hold psib.
#include <hip/hip_runtime.h>

#include "chf_internal.h"

namespace chf {

namespace {

constexpr int kAdjZ = 16;

__device__ __forceinline__ long long cidx(const Dev &d, int i, int j, int k) {
  return (long long)k * d.plane + (long long)j * d.pitch + i;
}

__device__ __forceinline__ long long pidx(const Dev &d, int u, int i, int j, int k, int s) {
  if (u == 0) return ((long long)k * d.ny + j) * d.np2 + s;
  if (u == 1) return ((long long)k * d.np2 + s) * d.pitch + i;
  return ((long long)s * d.ny + j) * d.pitch + i;
}

// cotangent of one stretched derivative divided by delta, updating psib in place
__device__ __forceinline__ float adj_term(const Dev &d, float *psib, int u, int pos, int slot, bool half,
                                          int i, int j, int k, float tb) {
  const AxisTab &A = d.ax[u];
  const float ik = half ? A.ikh[pos] : A.ike[pos];
  if (slot < 0) return tb * ik;
  const float a = half ? A.adh[pos] : A.ade[pos];
  const float b = half ? A.bh[pos] : A.be[pos];
  const long long id = pidx(d, u, i, j, k, slot);
  const float tot = psib[id] + tb;
  psib[id] = b * tot;
  return fmaf(a, tot, tb * ik);
}

__global__ void k_adj_zero_q(double *q, int n) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) q[t] = 0.0;
}

__global__ void __launch_bounds__(64) k_adj_sample(Dev d, const double *g, int n, int T) {
  const int lane = threadIdx.x;
  const int comp = lane >> 3, corner = lane & 7;
  if (comp >= 3) return;
  float *Eb = (float *)d.e[0][comp];
  for (int o = 0; o < d.n_obs; o++) {
    const int *ix = d.obs_idx + (o * 3 + comp) * 3;
    const double *tf = d.obs_t + (o * 3 + comp) * 3;
    const int a = corner & 1, b = (corner >> 1) & 1, c = corner >> 2;
    const double wgt = (a ? tf[0] : 1.0 - tf[0]) * (b ? tf[1] : 1.0 - tf[1]) * (c ? tf[2] : 1.0 - tf[2]);
    const double gv = g[((long long)o * 3 + comp) * T + n];
    const long long node = cidx(d, ix[0] + a, ix[1] + b, ix[2] + c);
    Eb[node] = (float)((double)Eb[node] + wgt * gv);
    __threadfence();  // observers one after the other: a later stencil may share a node
  }
}

// With dth: also the cotangents of the source's non-linear parameters,
//   dL/dsigma_r  += -Cb v Q(z_s) sum dW_r/dsigma_r W_z Eb_z,
//   dL/dz_entry  += -Cb v [Q'(z_s) sum W_r W_z Eb_z + Q(z_s) sum W_r dW_z/dz_s Eb_z]
// (z_s moves one for one with z_entry; Q' is the slope of the hat interpolation, W_z' that of the
// window-normalised Gaussian with the window held fixed), Q from the profile q.
__global__ void __launch_bounds__(256) k_adj_source(Dev d, int n, double *dq, const double *q, double *dth) {
  __shared__ double part[256], part_r[256], part_z[256];
  const double tt = (n + 0.5) * d.dt;
  if (!d.src_on || tt < d.t_entry) return;
  const double zs = d.z_entry + d.v_src * (tt - d.t_entry);
  const double half = d.cut_sigmas * d.sigma_z;
  const int klo = (int)ceil((zs - half) / d.dz - 0.5);
  const int khi = (int)floor((zs + half) / d.dz - 0.5);
  const int m = min(khi - klo + 1, kMaxWz);
  const double sz2 = d.sigma_z * d.sigma_z;
  double norm = 0.0, dnorm = 0.0;
  for (int s = 0; s < m; s++) {
    const double dd = (klo + s + 0.5) * d.dz - zs;
    const double e = exp(-0.5 * dd * dd / sz2);
    norm += e * d.dz;
    dnorm += e * dd / sz2 * d.dz;
  }
  const float *Ebz = (const float *)d.e[0][2];
  const int npatch = d.src_ni * d.src_nj;
  double acc = 0.0, acc_r = 0.0, acc_z = 0.0;
  for (int t = threadIdx.x; t < npatch * m; t += blockDim.x) {
    const int s = t / npatch, c = t % npatch;
    const int k = klo + s;
    if (k < 0 || k > d.nz - 2) continue;
    const double wr = d.wr[c];
    if (wr == 0.0) continue;
    const int i = d.src_i0 + c % d.src_ni, j = d.src_j0 + c / d.src_ni;
    const double dd = (k + 0.5) * d.dz - zs;
    const double e = exp(-0.5 * dd * dd / sz2);
    const double wz = e / norm;
    const double eb = (double)Ebz[cidx(d, i, j, k)];
    acc += wr * wz * eb;
    if (dth) {
      acc_r += d.dwr[c] * wz * eb;
      acc_z += wr * (e * dd / sz2 / norm - wz * dnorm / norm) * eb;
    }
  }
  part[threadIdx.x] = acc;
  part_r[threadIdx.x] = acc_r;
  part_z[threadIdx.x] = acc_z;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      part[threadIdx.x] += part[threadIdx.x + w];
      part_r[threadIdx.x] += part_r[threadIdx.x + w];
      part_z[threadIdx.x] += part_z[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double u = (zs - d.z_bin0) / d.dz_bin;
    const double fl = floor(u);
    const int b0 = (int)fl;
    const double tfr = u - fl;
    const double base = -d.a_cb_src * d.v_src * part[0];
    if (b0 >= 0 && b0 < d.n_bins) dq[b0] += base * (1.0 - tfr);
    if (b0 + 1 >= 0 && b0 + 1 < d.n_bins) dq[b0 + 1] += base * tfr;
    if (dth) {
      const double *qb = q ? q : d.q_bins;
      const double q0 = b0 >= 0 && b0 < d.n_bins ? qb[b0] : 0.0;
      const double q1 = b0 + 1 >= 0 && b0 + 1 < d.n_bins ? qb[b0 + 1] : 0.0;
      const double Q = (1.0 - tfr) * q0 + tfr * q1, dQ = (q1 - q0) / d.dz_bin;
      const double g = -d.a_cb_src * d.v_src;
      dth[0] += g * Q * part_r[0];
      dth[1] += g * (dQ * part[0] + Q * part_z[0]);
    }
  }
}

// Permittivity cotangent of step n at every E node.  With eps = eps0 eps_r(node) in Ampere's law
// with conductivity, Ca and Cb of the node move with eps_r so that
//   dE^{n+1}/deps_r = -(E^{n+1} - E^n) / (eps_r (1 + l)),   l = sigma dt / (2 eps),
// whatever the curl, psi and source terms were (they do not depend on eps_r; the absorber's
// grading is held fixed).  Eb, at this point of the reverse step, is the full cotangent of
// E^{n+1}, so g += -coef Eb (E^{n+1} - E^n) with coef = 1/(eps_r (1 + l)).  e0/e1 hold E^n and
// E^{n+1} as dense [3][nz][ny][nx] FP32; g is FP64 in the same layout.  Only nodes the Yee
// update advances (not tangential to a wall) collect a value.
__global__ void __launch_bounds__(256) k_adj_eps(Dev d, const float *e0, const float *e1, double *g, double coef) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= d.nx || j >= d.ny) return;
  const int k0 = blockIdx.z * kAdjZ, k1 = min(k0 + kAdjZ, d.nz);
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const long long N = (long long)nx * ny * nz;
  for (int k = k0; k < k1; k++) {
    const long long c = cidx(d, i, j, k);
    const long long dn = ((long long)k * ny + j) * nx + i;
    const bool up[3] = {i <= nx - 2 && j >= 1 && j <= ny - 2 && k >= 1 && k <= nz - 2,
                        i >= 1 && i <= nx - 2 && j <= ny - 2 && k >= 1 && k <= nz - 2,
                        i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2 && k <= nz - 2};
#pragma unroll
    for (int u = 0; u < 3; u++) {
      if (!up[u]) continue;
      const long long t = u * N + dn;
      const double eb = (double)((const float *)d.e[0][u])[c];
      g[t] -= coef * eb * ((double)e1[t] - (double)e0[t]);
    }
  }
}

// E update transpose: per-term cotangents into S[0..5] = (Ex-y, Ex-z, Ey-z, Ey-x, Ez-x, Ez-y)
__global__ void __launch_bounds__(256) k_adj_e(Dev d) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= d.nx || j >= d.ny) return;
  const int k0 = blockIdx.z * kAdjZ, k1 = min(k0 + kAdjZ, d.nz);
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  float *Eb[3] = {(float *)d.e[0][0], (float *)d.e[0][1], (float *)d.e[0][2]};
  float *S[6] = {(float *)d.e[1][0], (float *)d.e[1][1], (float *)d.e[1][2],
                 (float *)d.h[1][0], (float *)d.h[1][1], (float *)d.h[1][2]};
  const bool pml = d.np2 > 0;
  const int sx = pml ? d.ax[0].se[i] : -1, sy = pml ? d.ax[1].se[j] : -1;
  for (int k = k0; k < k1; k++) {
    const int sz = pml ? d.ax[2].se[k] : -1;
    const long long c = cidx(d, i, j, k);
    const bool ux = i <= nx - 2 && j >= 1 && j <= ny - 2 && k >= 1 && k <= nz - 2;
    const bool uy = i >= 1 && i <= nx - 2 && j <= ny - 2 && k >= 1 && k <= nz - 2;
    const bool uz = i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2 && k <= nz - 2;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f, s5 = 0.f;
    if (ux) {
      const float tb = d.a_cb * Eb[0][c];
      s0 = adj_term(d, d.psi_e[1][0], 1, j, sy, false, i, j, k, tb);
      s1 = adj_term(d, d.psi_e[2][0], 2, k, sz, false, i, j, k, -tb);
      Eb[0][c] = d.a_ca * Eb[0][c];
    }
    if (uy) {
      const float tb = d.a_cb * Eb[1][c];
      s2 = adj_term(d, d.psi_e[2][1], 2, k, sz, false, i, j, k, tb);
      s3 = adj_term(d, d.psi_e[0][0], 0, i, sx, false, i, j, k, -tb);
      Eb[1][c] = d.a_ca * Eb[1][c];
    }
    if (uz) {
      const float tb = d.a_cb * Eb[2][c];
      s4 = adj_term(d, d.psi_e[0][1], 0, i, sx, false, i, j, k, tb);
      s5 = adj_term(d, d.psi_e[1][1], 1, j, sy, false, i, j, k, -tb);
      Eb[2][c] = d.a_ca * Eb[2][c];
    }
    S[0][c] = s0; S[1][c] = s1; S[2][c] = s2; S[3][c] = s3; S[4][c] = s4; S[5][c] = s5;
  }
}

// Hb(p) += s(p) - s(p + e_u) over the E terms that read H(p)
__global__ void __launch_bounds__(256) k_adj_hgather(Dev d) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= d.nx || j >= d.ny) return;
  const int k0 = blockIdx.z * kAdjZ, k1 = min(k0 + kAdjZ, d.nz);
  const float *S[6] = {(const float *)d.e[1][0], (const float *)d.e[1][1], (const float *)d.e[1][2],
                       (const float *)d.h[1][0], (const float *)d.h[1][1], (const float *)d.h[1][2]};
  float *Hb[3] = {(float *)d.h[0][0], (float *)d.h[0][1], (float *)d.h[0][2]};
  for (int k = k0; k < k1; k++) {
    const long long c = cidx(d, i, j, k);
    const bool xp = i + 1 < d.nx, yp = j + 1 < d.ny, zp = k + 1 < d.nz;
    const long long cx = c + 1, cy = c + d.pitch, cz = c + d.plane;
    const float hx = (S[2][c] - (zp ? S[2][cz] : 0.f)) + (S[5][c] - (yp ? S[5][cy] : 0.f));
    const float hy = (S[1][c] - (zp ? S[1][cz] : 0.f)) + (S[4][c] - (xp ? S[4][cx] : 0.f));
    const float hz = (S[0][c] - (yp ? S[0][cy] : 0.f)) + (S[3][c] - (xp ? S[3][cx] : 0.f));
    Hb[0][c] += hx;
    Hb[1][c] += hy;
    Hb[2][c] += hz;
  }
}

// H update transpose: per-term cotangents into S[0..5] = (Hx-y, Hx-z, Hy-z, Hy-x, Hz-x, Hz-y)
__global__ void __launch_bounds__(256) k_adj_h(Dev d) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= d.nx || j >= d.ny) return;
  const int k0 = blockIdx.z * kAdjZ, k1 = min(k0 + kAdjZ, d.nz);
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const float *Hb[3] = {(const float *)d.h[0][0], (const float *)d.h[0][1], (const float *)d.h[0][2]};
  float *S[6] = {(float *)d.e[1][0], (float *)d.e[1][1], (float *)d.e[1][2],
                 (float *)d.h[1][0], (float *)d.h[1][1], (float *)d.h[1][2]};
  const bool pml = d.np2 > 0;
  const int sx = pml ? d.ax[0].sh[i] : -1, sy = pml ? d.ax[1].sh[j] : -1;
  for (int k = k0; k < k1; k++) {
    const int sz = pml ? d.ax[2].sh[k] : -1;
    const long long c = cidx(d, i, j, k);
    const bool ux = j <= ny - 2 && k <= nz - 2;
    const bool uy = i <= nx - 2 && k <= nz - 2;
    const bool uz = i <= nx - 2 && j <= ny - 2;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f, s5 = 0.f;
    if (ux) {
      const float tb = -d.a_db * Hb[0][c];
      s0 = adj_term(d, d.psi_h[0][1][0], 1, j, sy, true, i, j, k, tb);
      s1 = adj_term(d, d.psi_h[0][2][0], 2, k, sz, true, i, j, k, -tb);
    }
    if (uy) {
      const float tb = -d.a_db * Hb[1][c];
      s2 = adj_term(d, d.psi_h[0][2][1], 2, k, sz, true, i, j, k, tb);
      s3 = adj_term(d, d.psi_h[0][0][0], 0, i, sx, true, i, j, k, -tb);
    }
    if (uz) {
      const float tb = -d.a_db * Hb[2][c];
      s4 = adj_term(d, d.psi_h[0][0][1], 0, i, sx, true, i, j, k, tb);
      s5 = adj_term(d, d.psi_h[0][1][1], 1, j, sy, true, i, j, k, -tb);
    }
    S[0][c] = s0; S[1][c] = s1; S[2][c] = s2; S[3][c] = s3; S[4][c] = s4; S[5][c] = s5;
  }
}

// Eb(p) += s(p - e_u) - s(p) over the H terms that read E(p)
__global__ void __launch_bounds__(256) k_adj_egather(Dev d) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= d.nx || j >= d.ny) return;
  const int k0 = blockIdx.z * kAdjZ, k1 = min(k0 + kAdjZ, d.nz);
  const float *S[6] = {(const float *)d.e[1][0], (const float *)d.e[1][1], (const float *)d.e[1][2],
                       (const float *)d.h[1][0], (const float *)d.h[1][1], (const float *)d.h[1][2]};
  float *Eb[3] = {(float *)d.e[0][0], (float *)d.e[0][1], (float *)d.e[0][2]};
  for (int k = k0; k < k1; k++) {
    const long long c = cidx(d, i, j, k);
    const bool xm = i >= 1, ym = j >= 1, zm = k >= 1;
    const long long cx = c - 1, cy = c - d.pitch, cz = c - d.plane;
    const float ex = ((zm ? S[2][cz] : 0.f) - S[2][c]) + ((ym ? S[5][cy] : 0.f) - S[5][c]);
    const float ey = ((zm ? S[1][cz] : 0.f) - S[1][c]) + ((xm ? S[4][cx] : 0.f) - S[4][c]);
    const float ez = ((ym ? S[0][cy] : 0.f) - S[0][c]) + ((xm ? S[3][cx] : 0.f) - S[3][c]);
    Eb[0][c] += ex;
    Eb[1][c] += ey;
    Eb[2][c] += ez;
  }
}

}  // namespace

hipError_t launch_adjoint_init(const chf_plan &p, double *dl_dq, hipStream_t s, int n_out) {
  const int n = n_out >= 0 ? n_out : p.dev.n_bins;
  hipLaunchKernelGGL(k_adj_zero_q, dim3((std::max(n, 1) + 255) / 256), dim3(256), 0, s, dl_dq, n);
  return hipGetLastError();
}

hipError_t launch_adjoint_step(const chf_plan &p, const Dev &d, int parity, int step, const double *dl_dw,
                               double *dl_dq, hipStream_t s, const double *q_dev, double *dl_dtheta,
                               const EpsTerm *eps) {
  (void)parity;
  const int T = p.grid.n_steps;
  if (d.n_obs > 0) hipLaunchKernelGGL(k_adj_sample, dim3(1), dim3(64), 0, s, d, dl_dw, step, T);
  if (d.src_on) hipLaunchKernelGGL(k_adj_source, dim3(1), dim3(256), 0, s, d, step, dl_dq, q_dev, dl_dtheta);
  dim3 grid((d.nx + 63) / 64, (d.ny + 3) / 4, (d.nz + kAdjZ - 1) / kAdjZ);
  if (eps) hipLaunchKernelGGL(k_adj_eps, grid, dim3(256), 0, s, d, eps->e0, eps->e1, eps->g, eps->coef);
  hipLaunchKernelGGL(k_adj_e, grid, dim3(256), 0, s, d);
  hipLaunchKernelGGL(k_adj_hgather, grid, dim3(256), 0, s, d);
  hipLaunchKernelGGL(k_adj_h, grid, dim3(256), 0, s, d);
  hipLaunchKernelGGL(k_adj_egather, grid, dim3(256), 0, s, d);
  return hipGetLastError();
}

}  // namespace chf
