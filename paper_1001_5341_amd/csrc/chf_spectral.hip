// Spectral post-processing for gfx950 (entry points of include/chfdtd_spectral.h): FP64 DFT of
// recorded waveforms, theta-hat projection, and the far-field formula of the hat-binned profile.
//
// Both transforms are sums S(w) = sum_b x_b exp(i w (x0 + b h)) over uniformly spaced samples
// with one "frequency" w per thread.  A workgroup stages the samples through LDS in chunks
// (coalesced loads, then broadcast reads), and each thread advances four interleaved phase
// factors by the rotation exp(4 i w h), re-anchored with an exact sincos every kAnchor samples
// so the rounding of the recurrence stays near 1e-14 relative.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/chfdtd_spectral.h"
#include "chf_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 2048;  // samples per LDS stage (16 KiB)
constexpr int kAnchor = 128;  // exact phase every kAnchor samples
constexpr double kC0 = 299792458.0;
constexpr double kMu0 = 1.25663706212e-6;
constexpr double kPi = 3.14159265358979323846;

chf_status fail(chf_status s, const std::string &m) {
  chf::set_error(m);
  return s;
}

// Block-wide: every thread of the block must call it (it synchronises); `active` threads
// accumulate sum_b x[b] exp(i w (x0 + b h)) for b < n into (re, im).  Each thread runs four
// independent phase chains over the samples b = 4c + r (r = 0..3), rotated by exp(4 i w h), so the
// recurrence's latency overlaps; every kAnchor samples chain 0 is re-anchored with an exact
// sincos and chains 1-3 follow from it by fixed rotations.
__device__ void accumulate(const double *x, int n, double x0, double h, double w, bool active, double &re,
                           double &im) {
  __shared__ double sx[kChunk];
  // rotations by w h, 2 w h, 3 w h (chain offsets) and 4 w h (chain step)
  double rs[4] = {0.0, 0.0, 0.0, 0.0}, rc[4] = {1.0, 1.0, 1.0, 1.0};
  if (active) {
#pragma unroll
    for (int r = 1; r < 4; r++) sincos(r * w * h, &rs[r], &rc[r]);
    sincos(4.0 * w * h, &rs[0], &rc[0]);
  }
  const double s4 = rs[0], c4 = rc[0];
  double ar[4] = {0.0, 0.0, 0.0, 0.0}, ai[4] = {0.0, 0.0, 0.0, 0.0};
  for (int base = 0; base < n; base += kChunk) {
    const int m = min(kChunk, n - base);
    __syncthreads();
    for (int t = threadIdx.x; t < kChunk; t += blockDim.x) sx[t] = t < m ? x[base + t] : 0.0;
    __syncthreads();
    if (active) {
      for (int a = 0; a < m; a += kAnchor) {
        double c[4], s[4];
        sincos(w * (x0 + (base + a) * h), &s[0], &c[0]);
#pragma unroll
        for (int r = 1; r < 4; r++) {
          c[r] = c[0] * rc[r] - s[0] * rs[r];
          s[r] = fma(s[0], rc[r], c[0] * rs[r]);
        }
        const int e = min(a + kAnchor, m);
#pragma unroll 4
        for (int b = a; b < e; b += 4) {  // samples past m are zero in LDS
#pragma unroll
          for (int r = 0; r < 4; r++) {
            const double v = sx[b + r];
            ar[r] = fma(v, c[r], ar[r]);
            ai[r] = fma(v, s[r], ai[r]);
            const double c2 = c[r] * c4 - s[r] * s4;
            s[r] = fma(s[r], c4, c[r] * s4);
            c[r] = c2;
          }
        }
      }
    }
  }
  re += (ar[0] + ar[1]) + (ar[2] + ar[3]);
  im += (ai[0] + ai[1]) + (ai[2] + ai[3]);
}

__global__ void __launch_bounds__(kThreads) k_spectrum(const double *w, int n_t, int ld, double dt, double t0,
                                                       const double *omega, int n_freq, double *spec) {
  const int s = blockIdx.y;
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = f < n_freq;
  const double om = active ? omega[f] : 0.0;
  double re = 0.0, im = 0.0;
  accumulate(w + (long long)s * ld, n_t, t0, dt, om, active, re, im);
  if (active) {
    double *o = spec + ((long long)s * n_freq + f) * 2;
    o[0] = re * dt;
    o[1] = im * dt;
  }
}

__global__ void k_project(const double *spec, int n_obs, int n_comp, int n_freq, const double *wts, double *out,
                          double *mag) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)n_obs * n_freq) return;
  const int o = (int)(t / n_freq), f = (int)(t % n_freq);
  double re = 0.0, im = 0.0;
  for (int c = 0; c < n_comp; c++) {
    const double wc = wts[o * n_comp + c];
    const double *x = spec + (((long long)o * n_comp + c) * n_freq + f) * 2;
    re = fma(wc, x[0], re);
    im = fma(wc, x[1], im);
  }
  if (out) {
    out[t * 2] = re;
    out[t * 2 + 1] = im;
  }
  if (mag) mag[t] = sqrt(re * re + im * im);
}

__global__ void __launch_bounds__(kThreads) k_far_field(const double *q, int n_bins, double z0, double h,
                                                        const double *r_theta, chf_far_field_params prm,
                                                        const double *omega, int n_freq, double *out) {
  const int o = blockIdx.y;
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = f < n_freq;
  const double om = active ? omega[f] : 0.0;
  const double R = r_theta[2 * o], th = r_theta[2 * o + 1];
  const double v = prm.beta * kC0;
  const double k = prm.n_index * om / kC0;
  const double ct = cos(th);
  const double p = om / v - k * ct;
  double re = 0.0, im = 0.0;
  accumulate(q, n_bins, z0, h, p, active, re, im);
  if (!active) return;
  // F = h sinc^2(p h / 2) S
  const double x = 0.5 * p * h;
  const double sinc = x == 0.0 ? 1.0 : sin(x) / x;
  const double fh = h * sinc * sinc;
  re *= fh;
  im *= fh;
  // A = mu0/(4 pi R) exp(i (k R + w t_off + k cos(theta) z_origin)) F; E_theta = -i w sin(theta) A
  const double t_off = prm.t_entry - prm.z_entry / v;
  double sp, cp;
  sincos(k * R + om * t_off + k * ct * prm.z_origin, &sp, &cp);
  const double amp = kMu0 / (4.0 * kPi * R);
  const double ar = amp * (re * cp - im * sp), ai = amp * (re * sp + im * cp);
  const double g = om * sin(th);
  double *y = out + ((long long)o * n_freq + f) * 2;
  y[0] = g * ai;   // -i g (ar + i ai) = g ai - i g ar
  y[1] = -g * ar;
}

}  // namespace

extern "C" {

chf_status chf_spectrum(void *stream, const double *w_dev, int32_t n_series, int32_t n_t, int32_t ld, double dt,
                        double t0, const double *omega_dev, int32_t n_freq, double *spec_dev) {
  if (!w_dev || !omega_dev || !spec_dev) return fail(CHF_EINVAL, "NULL device array");
  if (n_series < 0 || n_series > 65535 || n_t < 0 || ld < n_t || n_freq < 0)
    return fail(CHF_EINVAL, "bad sizes (need 0 <= n_series <= 65535, 0 <= n_t <= ld, n_freq >= 0)");
  if (!std::isfinite(dt) || !std::isfinite(t0)) return fail(CHF_EINVAL, "non-finite dt or t0");
  if (n_series == 0 || n_freq == 0) return CHF_OK;
  const dim3 grid((n_freq + kThreads - 1) / kThreads, n_series);
  k_spectrum<<<grid, kThreads, 0, (hipStream_t)stream>>>(w_dev, n_t, ld, dt, t0, omega_dev, n_freq, spec_dev);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CHF_OK : fail(CHF_EHIP, std::string("spectrum launch: ") + hipGetErrorString(e));
}

chf_status chf_spectrum_project(void *stream, const double *spec_dev, int32_t n_obs, int32_t n_comp, int32_t n_freq,
                                const double *weights_dev, double *out_dev, double *mag_dev) {
  if (!spec_dev || !weights_dev) return fail(CHF_EINVAL, "NULL device array");
  if (n_obs < 0 || n_comp < 1 || n_freq < 0) return fail(CHF_EINVAL, "bad sizes");
  const long long n = (long long)n_obs * n_freq;
  if (n == 0 || (!out_dev && !mag_dev)) return CHF_OK;
  if ((n + 255) / 256 > 0x7fffffffLL) return fail(CHF_EINVAL, "too many outputs");
  k_project<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(spec_dev, n_obs, n_comp, n_freq, weights_dev,
                                                                         out_dev, mag_dev);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CHF_OK : fail(CHF_EHIP, std::string("projection launch: ") + hipGetErrorString(e));
}

chf_status chf_geometry_rz(int32_t n_obs, const double *rz, double z_origin, double *r_theta, double *weights) {
  if (n_obs < 0 || (n_obs > 0 && (!rz || !r_theta || !weights))) return fail(CHF_EINVAL, "bad arguments");
  for (int o = 0; o < n_obs; o++) {
    const double r = rz[2 * o], dz = rz[2 * o + 1] - z_origin;
    const double R = std::hypot(r, dz);
    if (!(R > 0)) return fail(CHF_EDOMAIN, "observer at the origin");
    const double th = std::atan2(r, dz);
    r_theta[2 * o] = R;
    r_theta[2 * o + 1] = th;
    weights[2 * o] = std::cos(th);
    weights[2 * o + 1] = -std::sin(th);
  }
  return CHF_OK;
}

chf_status chf_geometry_xyz(int32_t n_obs, const double *xyz, double x_axis, double y_axis, double z_origin,
                            double *r_theta, double *weights) {
  if (n_obs < 0 || (n_obs > 0 && (!xyz || !r_theta || !weights))) return fail(CHF_EINVAL, "bad arguments");
  for (int o = 0; o < n_obs; o++) {
    const double dx = xyz[3 * o] - x_axis, dy = xyz[3 * o + 1] - y_axis, dz = xyz[3 * o + 2] - z_origin;
    const double rho = std::hypot(dx, dy);
    const double R = std::hypot(rho, dz);
    if (!(R > 0)) return fail(CHF_EDOMAIN, "observer at the origin");
    const double th = std::atan2(rho, dz), ph = std::atan2(dy, dx);
    r_theta[2 * o] = R;
    r_theta[2 * o + 1] = th;
    weights[3 * o] = std::cos(th) * std::cos(ph);
    weights[3 * o + 1] = std::cos(th) * std::sin(ph);
    weights[3 * o + 2] = -std::sin(th);
  }
  return CHF_OK;
}

chf_status chf_far_field_1d(void *stream, const double *q_dev, int32_t n_bins, double z_bin0, double dz_bin,
                            const double *r_theta_dev, int32_t n_obs, const chf_far_field_params *prm,
                            const double *omega_dev, int32_t n_freq, double *out_dev) {
  if (!q_dev || !r_theta_dev || !prm || !omega_dev || !out_dev) return fail(CHF_EINVAL, "NULL argument");
  if (n_bins < 0 || n_obs < 0 || n_obs > 65535 || n_freq < 0) return fail(CHF_EINVAL, "bad sizes");
  if (!(dz_bin > 0) || !(prm->beta > 0) || !(prm->n_index > 0)) return fail(CHF_EINVAL, "need dz_bin, beta, n > 0");
  if (n_obs == 0 || n_freq == 0) return CHF_OK;
  const dim3 grid((n_freq + kThreads - 1) / kThreads, n_obs);
  k_far_field<<<grid, kThreads, 0, (hipStream_t)stream>>>(q_dev, n_bins, z_bin0, dz_bin, r_theta_dev, *prm, omega_dev,
                                                          n_freq, out_dev);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CHF_OK : fail(CHF_EHIP, std::string("far-field launch: ") + hipGetErrorString(e));
}

}  // extern "C"
