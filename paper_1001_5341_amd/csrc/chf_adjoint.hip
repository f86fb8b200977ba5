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
// Each per-term cotangent s is a pure function of the old adjoint state and the old psib, so
// the step runs as two stencil sweeps that read one level and write the other, recomputing the
// few neighbour terms they need instead of storing them: sweep A writes Hb' = Hb + (gather of
// the E terms); sweep B writes Eb' = (ca) Eb + (gather of the H terms of Hb').  The psib of the
// E terms and of the H terms are double-buffered the same way (the node that owns a term
// writes its new psib).  Every value is written by one thread: deterministic, and the same
// arithmetic, in the same order, as a scatter-free gather of stored terms.
#include <hip/hip_runtime.h>

#include "chf_internal.h"

namespace chf {

namespace {

// planes per workgroup of the reverse sweeps: each chunk reads one plane beyond it (the carried
// z term), so longer chunks read less (measured on 128 x 128 x 1024: 8 planes 1.19 s per 3000
// reverse steps, 16 planes 1.16 s, 32 planes 1.14 s); the result does not depend on it
constexpr int kAdjZ = 32;

__device__ __forceinline__ long long cidx(const Dev &d, int i, int j, int k) {
  return (long long)k * d.plane + (long long)j * d.pitch + i;
}

__device__ __forceinline__ long long pidx(const Dev &d, int u, int i, int j, int k, int s) {
  if (u == 0) return ((long long)k * d.ny + j) * d.np2 + s;
  if (u == 1) return ((long long)k * d.np2 + s) * d.pitch + i;
  return ((long long)s * d.ny + j) * d.pitch + i;
}

__global__ void k_adj_zero_q(double *q, int n) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) q[t] = 0.0;
}

// Transposed sampling: Eb += w g^n at every stencil node, one thread per distinct (component,
// node) of the plan's table, its contributions added in observer order (each rounded to FP32 as
// a stored field is), so that stencils sharing a node give the same bits as observers applied
// one after the other.
__global__ void __launch_bounds__(256) k_adj_sample(Dev d, const double *g, int n, int T, int cur) {
  const int key = blockIdx.x * 256 + threadIdx.x;
  if (key >= d.n_skeys) return;
  const int comp = d.sk_comp[key];
  float *Eb = (float *)d.e[cur][comp];
  const long long node = d.sk_node[key];
  float v = Eb[node];
  for (int e = d.sk_ptr[key]; e < d.sk_ptr[key + 1]; e++)
    v = (float)((double)v + d.se_w[e] * g[((long long)d.se_obs[e] * 3 + comp) * T + n]);
  Eb[node] = v;
}

// Transposed source of step n, dL/dq_b += -Cb v hat_b(z_s) sum W_r W_z Eb_z, as one FP64 workgroup
// reduction (fixed order, deterministic).  With dth: also the cotangents of the source's
// non-linear parameters,
//   dL/dsigma_r  += -Cb v Q(z_s) sum dW_r/dsigma_r W_z Eb_z,
//   dL/dz_entry  += -Cb v [Q'(z_s) sum W_r W_z Eb_z + Q(z_s) sum W_r dW_z/dz_s Eb_z]
// (z_s moves one for one with z_entry; Q' is the slope of the hat interpolation, W_z' that of the
// window-normalised Gaussian with the window held fixed), Q from the profile q.
constexpr int kSrcThreads = 1024;

__global__ void __launch_bounds__(kSrcThreads) k_adj_source(Dev d, int n, double *dq, const double *q, double *dth,
                                                           int cur) {
  __shared__ double part[kSrcThreads], part_r[kSrcThreads], part_z[kSrcThreads];
  __shared__ double row_e[kMaxWz], row_d[kMaxWz], sums[2];
  const double tt = (n + 0.5) * d.dt;
  if (!d.src_on || tt < d.t_entry) return;
  const double zs = d.z_entry + d.v_src * (tt - d.t_entry);
  const double half = d.cut_sigmas * d.sigma_z;
  const int klo = (int)ceil((zs - half) / d.dz - 0.5);
  const int khi = (int)floor((zs + half) / d.dz - 0.5);
  const int m = min(khi - klo + 1, kMaxWz);
  const double sz2 = d.sigma_z * d.sigma_z;
  // the window's Gaussian per row, then its normalisation summed in row order
  if ((int)threadIdx.x < m) {
    const double dd = (klo + (int)threadIdx.x + 0.5) * d.dz - zs;
    row_e[threadIdx.x] = exp(-0.5 * dd * dd / sz2);
    row_d[threadIdx.x] = dd;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double norm = 0.0, dnorm = 0.0;
    for (int s = 0; s < m; s++) {
      norm += row_e[s] * d.dz;
      dnorm += row_e[s] * row_d[s] / sz2 * d.dz;
    }
    sums[0] = norm;
    sums[1] = dnorm;
  }
  __syncthreads();
  const double norm = sums[0], dnorm = sums[1];
  const float *Ebz = (const float *)d.e[cur][2];
  const int npatch = d.src_ni * d.src_nj;
  double acc = 0.0, acc_r = 0.0, acc_z = 0.0;
#pragma unroll 4
  for (int t = threadIdx.x; t < npatch * m; t += kSrcThreads) {
    const int s = t / npatch, c = t % npatch;
    const int k = klo + s;
    const int kc = min(max(k, 0), d.nz - 2);
    const int i = d.src_i0 + c % d.src_ni, j = d.src_j0 + c / d.src_ni;
    // every operand loaded before the tests, so the loads of several items are in flight
    const double wr = d.wr[c];
    const double eb = (double)Ebz[cidx(d, i, j, kc)];
    const double dwr = dth ? d.dwr[c] : 0.0;
    if (k < 0 || k > d.nz - 2 || wr == 0.0) continue;
    const double e = row_e[s], dd = row_d[s];
    const double wz = e / norm;
    acc += wr * wz * eb;
    if (dth) {
      acc_r += dwr * wz * eb;
      acc_z += wr * (e * dd / sz2 / norm - wz * dnorm / norm) * eb;
    }
  }
  part[threadIdx.x] = acc;
  part_r[threadIdx.x] = acc_r;
  part_z[threadIdx.x] = acc_z;
  __syncthreads();
  for (int w = kSrcThreads / 2; w > 0; w >>= 1) {
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
__global__ void __launch_bounds__(256) k_adj_eps(Dev d, const float *e0, const float *e1, double *g, double coef,
                                                 int cur) {
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
      const double eb = (double)((const float *)d.e[cur][u])[c];
      g[t] -= coef * eb * ((double)e1[t] - (double)e0[t]);
    }
  }
}

// Coefficients of one stretched derivative at one axis position: 1/(delta kappa), and inside a
// layer the psi slot with a/delta and b.
struct TP {
  float ik, a, b;
  int slot;
};

__device__ __forceinline__ TP tparam(const AxisTab &A, bool pml, int pos, bool half) {
  TP t;
  t.ik = half ? A.ikh[pos] : A.ike[pos];
  t.slot = pml ? (half ? A.sh[pos] : A.se[pos]) : -1;
  t.a = t.slot >= 0 ? (half ? A.adh[pos] : A.ade[pos]) : 0.f;
  t.b = t.slot >= 0 ? (half ? A.bh[pos] : A.be[pos]) : 0.f;
  return t;
}

// psi arrays of one set as [u * 2 + t]: (Ey-x, Ez-x, Ex-y, Ez-y, Ex-z, Ey-z) for the E terms and
// (Hy-x, Hz-x, Hx-y, Hz-y, Hx-z, Hy-z) for the H terms
struct PsiSet {
  float *p[6];
};

// One cotangent term of a stretched derivative divided by delta, given tb and the old psib
// loaded beforehand: zero where the node is not updated.  Inside a layer psib_tot = psib + tb,
// s = tb/(delta kappa) + (a/delta) psib_tot, and the owner (pw non-null) stores the new psib
// b psib_tot: the transposed CPML recursion.
__device__ __forceinline__ float term(bool upd, float tb, const TP &q, float psib, float *pw, long long id) {
  if (!upd) return 0.f;
  if (q.slot < 0) return tb * q.ik;
  const float tot = psib + tb;
  if (pw) __builtin_nontemporal_store(q.b * tot, pw + id);  // the other psib set
  return fmaf(q.a, tot, tb * q.ik);
}

// psib slot index of a term (slot clamped to 0 outside a layer, so that the address is valid
// and the load can be issued with the others; its value is then not used)
__device__ __forceinline__ long long pslot(const Dev &d, int u, int i, int j, int k, const TP &q) {
  return pidx(d, u, i, j, k, q.slot > 0 ? q.slot : 0);
}

// Sweep A: Hb' (level cur ^ 1) = Hb (level cur) + sum of s(p) - s(p + e_u) over the E terms
// that read H(p); the E-term psib move from set `er` to set `ew`.  A workgroup is 64 x nodes by
// 4 y rows marching a z chunk downwards; s(p + e_z) is the previous plane's own term, and each
// node evaluates the terms of its x and y neighbours itself (without storing their psib).
// Every load of a plane (own values, the neighbours' values and all psib) is issued before any
// of them is used, so a plane costs one memory round trip.
__global__ void __launch_bounds__(256) k_adj_ha(Dev d, int cur, PsiSet er, PsiSet ew) {
  const int lane = threadIdx.x & 63, r = threadIdx.x >> 6;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const int i = blockIdx.x * 64 + lane, j = blockIdx.y * 4 + r;
  const bool on = i < nx && j < ny;
  if (!on) return;
  const int k0 = blockIdx.z * kAdjZ, k1 = min(k0 + kAdjZ, nz);
  const bool pml = d.np2 > 0;
  const bool xp = i + 1 < nx, yp = j + 1 < ny;
  const int ip = min(i + 1, nx - 1), jp = min(j + 1, ny - 1);
  const TP x0 = tparam(d.ax[0], pml, i, false), x1 = tparam(d.ax[0], pml, ip, false);
  const TP y0 = tparam(d.ax[1], pml, j, false), y1 = tparam(d.ax[1], pml, jp, false);
  // update masks split by axis: Ex (i <= nx-2, 1 <= j <= ny-2, 1 <= k <= nz-2),
  // Ey (1 <= i <= nx-2, j <= ny-2, 1 <= k <= nz-2), Ez (1 <= i <= nx-2, 1 <= j <= ny-2, k <= nz-2)
  const bool ix = i <= nx - 2, iyz = i >= 1 && i <= nx - 2;
  const bool iyz1 = xp && ip >= 1 && ip <= nx - 2;
  const bool jxz = j >= 1 && j <= ny - 2, jy = j <= ny - 2;
  const bool jxz1 = yp && jp >= 1 && jp <= ny - 2;
  const float *E0 = (const float *)d.e[cur][0], *E1 = (const float *)d.e[cur][1], *E2 = (const float *)d.e[cur][2];
  const float *H0 = (const float *)d.h[cur][0], *H1 = (const float *)d.h[cur][1], *H2 = (const float *)d.h[cur][2];
  float *O0 = (float *)d.h[cur ^ 1][0], *O1 = (float *)d.h[cur ^ 1][1], *O2 = (float *)d.h[cur ^ 1][2];
  const float cb = d.a_cb;
  float s1n = 0.f, s2n = 0.f;  // terms Ex-z, Ey-z of the node above (p + e_z)
  if (k1 < nz) {
    const int ku = k1;
    const bool kxyu = ku >= 1 && ku <= nz - 2;
    const TP zu = tparam(d.ax[2], pml, ku, false);
    const long long cu = cidx(d, i, j, ku);
    const long long iz = pslot(d, 2, i, j, ku, zu);
    const float pa = pml ? er.p[4][iz] : 0.f, pb = pml ? er.p[5][iz] : 0.f;
    s1n = term(ix && jxz && kxyu, -cb * E0[cu], zu, pa, nullptr, 0);
    s2n = term(iyz && jy && kxyu, cb * E1[cu], zu, pb, nullptr, 0);
  }
  for (int k = k1 - 1; k >= k0; k--) {
    const bool kxy = k >= 1 && k <= nz - 2, kz = k <= nz - 2;
    const TP zk = tparam(d.ax[2], pml, k, false);
    const long long c = cidx(d, i, j, k), cx = cidx(d, ip, j, k), cy = cidx(d, i, jp, k);
    // loads
    const float e0 = E0[c], e1 = E1[c], e2 = E2[c];
    const float h0 = H0[c], h1 = H1[c], h2 = H2[c];
    const float e1x = E1[cx], e2x = E2[cx], e0y = E0[cy], e2y = E2[cy];
    const long long iy0 = pslot(d, 1, i, j, k, y0), iz0 = pslot(d, 2, i, j, k, zk), ix0 = pslot(d, 0, i, j, k, x0);
    const long long ix1 = pslot(d, 0, ip, j, k, x1), iy1 = pslot(d, 1, i, jp, k, y1);
    float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f, p4 = 0.f, p5 = 0.f, q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
    if (pml) {
      p0 = er.p[2][iy0];  // Ex-y
      p1 = er.p[4][iz0];  // Ex-z
      p2 = er.p[5][iz0];  // Ey-z
      p3 = er.p[0][ix0];  // Ey-x
      p4 = er.p[1][ix0];  // Ez-x
      p5 = er.p[3][iy0];  // Ez-y
      q0 = er.p[0][ix1];  // Ey-x of p + e_x
      q1 = er.p[1][ix1];  // Ez-x of p + e_x
      q2 = er.p[2][iy1];  // Ex-y of p + e_y
      q3 = er.p[3][iy1];  // Ez-y of p + e_y
    }
    // terms
    const float bx = cb * e0, by = cb * e1, bz = cb * e2;
    const bool ux = ix && jxz && kxy, uy = iyz && jy && kxy, uz = iyz && jxz && kz;
    const float s0 = term(ux, bx, y0, p0, ew.p[2], iy0);
    const float s1 = term(ux, -bx, zk, p1, ew.p[4], iz0);
    const float s2 = term(uy, by, zk, p2, ew.p[5], iz0);
    const float s3 = term(uy, -by, x0, p3, ew.p[0], ix0);
    const float s4 = term(uz, bz, x0, p4, ew.p[1], ix0);
    const float s5 = term(uz, -bz, y0, p5, ew.p[3], iy0);
    const float s3x = xp ? term(iyz1 && jy && kxy, -cb * e1x, x1, q0, nullptr, 0) : 0.f;
    const float s4x = xp ? term(iyz1 && jxz && kz, cb * e2x, x1, q1, nullptr, 0) : 0.f;
    const float s0y = yp ? term(ix && jxz1 && kxy, cb * e0y, y1, q2, nullptr, 0) : 0.f;
    const float s5y = yp ? term(iyz && jxz1 && kz, -cb * e2y, y1, q3, nullptr, 0) : 0.f;
    // the new level is not read within this sweep: non-temporal stores
    __builtin_nontemporal_store(h0 + ((s2 - s2n) + (s5 - s5y)), O0 + c);
    __builtin_nontemporal_store(h1 + ((s1 - s1n) + (s4 - s4x)), O1 + c);
    __builtin_nontemporal_store(h2 + ((s0 - s0y) + (s3 - s3x)), O2 + c);
    s1n = s1;
    s2n = s2;
  }
}

// Sweep B: Eb' (level cur ^ 1) = (ca) Eb (level cur) + sum of s(p - e_u) - s(p) over the H terms
// of Hb' (level cur ^ 1) that read E(p); the H-term psib move from set `hr` to set `hw`.  Same
// workgroup shape, marching upwards: s(p - e_z) is the previous plane's own term; the x and y
// neighbours' terms are evaluated in place; all loads of a plane are issued first.
__global__ void __launch_bounds__(256) k_adj_eb(Dev d, int cur, PsiSet hr, PsiSet hw) {
  const int lane = threadIdx.x & 63, r = threadIdx.x >> 6;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const int i = blockIdx.x * 64 + lane, j = blockIdx.y * 4 + r;
  const bool on = i < nx && j < ny;
  if (!on) return;
  const int k0 = blockIdx.z * kAdjZ, k1 = min(k0 + kAdjZ, nz);
  const bool pml = d.np2 > 0;
  const bool xm = i >= 1, ym = j >= 1;
  const int im = max(i - 1, 0), jm = max(j - 1, 0);
  const TP x0 = tparam(d.ax[0], pml, i, true), x1 = tparam(d.ax[0], pml, im, true);
  const TP y0 = tparam(d.ax[1], pml, j, true), y1 = tparam(d.ax[1], pml, jm, true);
  // H masks: Hx (j <= ny-2, k <= nz-2), Hy (i <= nx-2, k <= nz-2), Hz (i <= nx-2, j <= ny-2)
  const bool ih = i <= nx - 2, jh = j <= ny - 2;
  const bool ih1 = xm && im <= nx - 2, jh1 = ym && jm <= ny - 2;
  // E masks of the own node
  const bool ex_i = i <= nx - 2, eyz_i = i >= 1 && i <= nx - 2;
  const bool exz_j = j >= 1 && j <= ny - 2, ey_j = j <= ny - 2;
  const float *E0 = (const float *)d.e[cur][0], *E1 = (const float *)d.e[cur][1], *E2 = (const float *)d.e[cur][2];
  const float *H0 = (const float *)d.h[cur ^ 1][0], *H1 = (const float *)d.h[cur ^ 1][1],
              *H2 = (const float *)d.h[cur ^ 1][2];
  float *O0 = (float *)d.e[cur ^ 1][0], *O1 = (float *)d.e[cur ^ 1][1], *O2 = (float *)d.e[cur ^ 1][2];
  const float db = d.a_db, ca = d.a_ca;
  float t1p = 0.f, t2p = 0.f;  // terms Hx-z, Hy-z of the node below (p - e_z)
  if (k0 >= 1) {
    const int kd = k0 - 1;
    const TP zd = tparam(d.ax[2], pml, kd, true);
    const long long cd = cidx(d, i, j, kd);
    const long long iz = pslot(d, 2, i, j, kd, zd);
    const float pa = pml ? hr.p[4][iz] : 0.f, pb = pml ? hr.p[5][iz] : 0.f;
    t1p = term(jh, db * H0[cd], zd, pa, nullptr, 0);
    t2p = term(ih, -db * H1[cd], zd, pb, nullptr, 0);
  }
  for (int k = k0; k < k1; k++) {
    const bool kh = k <= nz - 2;
    const TP zk = tparam(d.ax[2], pml, k, true);
    const long long c = cidx(d, i, j, k), cx = cidx(d, im, j, k), cy = cidx(d, i, jm, k);
    const float hx = H0[c], hy = H1[c], hz = H2[c];
    const float e0 = E0[c], e1 = E1[c], e2 = E2[c];
    const float hyx = H1[cx], hzx = H2[cx], hxy = H0[cy], hzy = H2[cy];
    const long long iy0 = pslot(d, 1, i, j, k, y0), iz0 = pslot(d, 2, i, j, k, zk), ix0 = pslot(d, 0, i, j, k, x0);
    const long long ix1 = pslot(d, 0, im, j, k, x1), iy1 = pslot(d, 1, i, jm, k, y1);
    float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f, p4 = 0.f, p5 = 0.f, q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
    if (pml) {
      p0 = hr.p[2][iy0];  // Hx-y
      p1 = hr.p[4][iz0];  // Hx-z
      p2 = hr.p[5][iz0];  // Hy-z
      p3 = hr.p[0][ix0];  // Hy-x
      p4 = hr.p[1][ix0];  // Hz-x
      p5 = hr.p[3][iy0];  // Hz-y
      q0 = hr.p[0][ix1];  // Hy-x of p - e_x
      q1 = hr.p[1][ix1];  // Hz-x of p - e_x
      q2 = hr.p[2][iy1];  // Hx-y of p - e_y
      q3 = hr.p[3][iy1];  // Hz-y of p - e_y
    }
    const float ax = -db * hx, ay = -db * hy, az = -db * hz;
    const bool ux = jh && kh, uy = ih && kh, uz = ih && jh;
    const float t0 = term(ux, ax, y0, p0, hw.p[2], iy0);
    const float t1 = term(ux, -ax, zk, p1, hw.p[4], iz0);
    const float t2 = term(uy, ay, zk, p2, hw.p[5], iz0);
    const float t3 = term(uy, -ay, x0, p3, hw.p[0], ix0);
    const float t4 = term(uz, az, x0, p4, hw.p[1], ix0);
    const float t5 = term(uz, -az, y0, p5, hw.p[3], iy0);
    const float t3x = xm ? term(ih1 && kh, db * hyx, x1, q0, nullptr, 0) : 0.f;
    const float t4x = xm ? term(ih1 && jh, -db * hzx, x1, q1, nullptr, 0) : 0.f;
    const float t0y = ym ? term(jh1 && kh, -db * hxy, y1, q2, nullptr, 0) : 0.f;
    const float t5y = ym ? term(ih && jh1, db * hzy, y1, q3, nullptr, 0) : 0.f;
    const bool kxy = k >= 1 && k <= nz - 2;
    const float ex = (t2p - t2) + (t5y - t5);
    const float ey = (t1p - t1) + (t4x - t4);
    const float ez = (t0y - t0) + (t3x - t3);
    __builtin_nontemporal_store(((ex_i && exz_j && kxy) ? ca * e0 : e0) + ex, O0 + c);
    __builtin_nontemporal_store(((eyz_i && ey_j && kxy) ? ca * e1 : e1) + ey, O1 + c);
    __builtin_nontemporal_store(((eyz_i && exz_j && kh) ? ca * e2 : e2) + ez, O2 + c);
    t1p = t1;
    t2p = t2;
  }
}

__global__ void k_adj_zero_f(float *p, long long n) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
    p[t] = 0.f;
}

}  // namespace

hipError_t launch_adjoint_init(const chf_plan &p, double *dl_dq, hipStream_t s, int n_out) {
  const int n = n_out >= 0 ? n_out : p.dev.n_bins;
  hipLaunchKernelGGL(k_adj_zero_q, dim3((std::max(n, 1) + 255) / 256), dim3(256), 0, s, dl_dq, n);
  return hipGetLastError();
}

hipError_t launch_adjoint_clear(const chf_plan &p, hipStream_t s) {
  for (int u = 0; u < 3; u++)
    for (int t = 0; t < 2; t++)
      if (p.psi_len[u] > 0 && p.dev.np2 > 0)
        hipLaunchKernelGGL(k_adj_zero_f, dim3(1024), dim3(256), 0, s, p.dev.psi_eb[u][t], (long long)p.psi_len[u]);
  return hipGetLastError();
}

hipError_t launch_adjoint_step(const chf_plan &p, const Dev &d, int parity, int step, const double *dl_dw,
                               double *dl_dq, hipStream_t s, const double *q_dev, double *dl_dtheta,
                               const EpsTerm *eps) {
  const int T = p.grid.n_steps;
  const int cur = parity & 1;
  if (d.n_skeys > 0)
    hipLaunchKernelGGL(k_adj_sample, dim3((d.n_skeys + 255) / 256), dim3(256), 0, s, d, dl_dw, step, T, cur);
  if (d.src_on)
    hipLaunchKernelGGL(k_adj_source, dim3(1), dim3(kSrcThreads), 0, s, d, step, dl_dq, q_dev, dl_dtheta, cur);
  dim3 grid((d.nx + 63) / 64, (d.ny + 3) / 4, (d.nz + kAdjZ - 1) / kAdjZ);
  if (eps) hipLaunchKernelGGL(k_adj_eps, grid, dim3(256), 0, s, d, eps->e0, eps->e1, eps->g, eps->coef, cur);
  // psib of the E terms alternate between the forward's psi_e slabs and the adjoint's second
  // set; those of the H terms between the two psi_h levels
  PsiSet e0, e1, h0, h1;
  for (int u = 0; u < 3; u++)
    for (int t = 0; t < 2; t++) {
      e0.p[u * 2 + t] = d.psi_e[u][t];
      e1.p[u * 2 + t] = d.psi_eb[u][t];
      h0.p[u * 2 + t] = d.psi_h[0][u][t];
      h1.p[u * 2 + t] = d.psi_h[1][u][t];
    }
  hipLaunchKernelGGL(k_adj_ha, grid, dim3(256), 0, s, d, cur, cur ? e1 : e0, cur ? e0 : e1);
  hipLaunchKernelGGL(k_adj_eb, grid, dim3(256), 0, s, d, cur, cur ? h1 : h0, cur ? h0 : h1);
  return hipGetLastError();
}

}  // namespace chf
