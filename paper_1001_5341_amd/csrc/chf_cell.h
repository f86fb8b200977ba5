// Per-node arithmetic and row access shared by every sweep of the 3-D path (the one-step
// sweeps of chf_kernels.hip and the two-step sweeps of chf_step2.hip), so that all of them
// apply the same operations in the same order and agree bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <type_traits>

#include "chf_internal.h"

namespace chf {

// ------------------------------------------------------------------ storage
// BF16X: BF16 with an 8-bit mantissa extension -- the 24 leading bits of the FP32 value (sign,
// 8 exponent bits, 15 fraction bits), rounded to nearest even, in 3 bytes (little endian: the
// extension byte, then the BF16 half).  FP32's exponent range, so no storage scale.
struct bf16x {
  unsigned char b[3];
};

template <typename T>
__device__ __forceinline__ float to_f(T x) { return static_cast<float>(x); }
template <typename T>
__device__ __forceinline__ T from_f(float x) { return static_cast<T>(x); }  // RNE

template <>
__device__ __forceinline__ float to_f<bf16x>(bf16x x) {
  const unsigned u = (unsigned)x.b[0] | ((unsigned)x.b[1] << 8) | ((unsigned)x.b[2] << 16);
  return __uint_as_float(u << 8);
}
__device__ __forceinline__ unsigned bf16x_round(float x);
template <>
__device__ __forceinline__ bf16x from_f<bf16x>(float x) {
  const unsigned r = bf16x_round(x);
  bf16x o;
  o.b[0] = (unsigned char)(r >> 8);
  o.b[1] = (unsigned char)(r >> 16);
  o.b[2] = (unsigned char)(r >> 24);
  return o;
}

// Row vectors: aligned to their size when it is a power of two, else to the largest power of
// two dividing it.  BF16X rows of a multiple of four values are held as whole dwords (three per
// four values), so that they live in registers and move with dword loads and stores.
constexpr unsigned vec_align(unsigned b) { return (b & (b - 1)) == 0 ? b : (b & (~b + 1)); }

template <typename T, int N>
constexpr bool kDwordRow = std::is_same<T, bf16x>::value && N % 4 == 0;

template <typename T, int N, bool D = kDwordRow<T, N>>
struct alignas(vec_align(sizeof(T) * N)) Vec {
  T v[N];
};
template <typename T, int N>
struct alignas(vec_align(sizeof(T) * N)) Vec<T, N, true> {
  unsigned w[3 * N / 4];
};

// 24-bit rounding of BF16X on a register: the FP32 bits rounded to nearest even at bit 8 (the low
// byte is left as it falls).  Integer rounding of the bit pattern carries into the exponent
// exactly as IEEE rounding does: the largest finite values round to infinity, infinity stays,
// and a NaN with a fraction bit at or above bit 8 (every NaN that arithmetic produces) stays NaN.
__device__ __forceinline__ unsigned bf16x_round(float x) {
  const unsigned u = __float_as_uint(x);
  return u + 0x7fu + ((u >> 8) & 1u);
}

// BF16X rows of a multiple of four values are whole dwords: value k of a group of four is the
// dword starting one byte before it with its low byte cleared (the 24 bits shifted into place).
template <int N>
__device__ __forceinline__ void bf16x_decode(const unsigned (&d)[3 * N / 4], float (&o)[N]) {
#pragma unroll
  for (int g = 0; g < N / 4; g++) {
    const unsigned d0 = d[3 * g], d1 = d[3 * g + 1], d2 = d[3 * g + 2];
    o[4 * g + 0] = __uint_as_float(d0 << 8);
    o[4 * g + 1] = __uint_as_float(__builtin_amdgcn_alignbyte(d1, d0, 2) & 0xffffff00u);
    o[4 * g + 2] = __uint_as_float(__builtin_amdgcn_alignbyte(d2, d1, 1) & 0xffffff00u);
    o[4 * g + 3] = __uint_as_float(d2 & 0xffffff00u);
  }
}

// Lanes whose cells start beyond the last node (`on` false) neither load nor store.
template <typename T, int N>
__device__ __forceinline__ void ld_row(const T *p, float (&o)[N], bool on) {
  if constexpr (kDwordRow<T, N>) {
    if (on) {
      unsigned d[3 * N / 4];
      const unsigned *q = reinterpret_cast<const unsigned *>(p);
#pragma unroll
      for (int t = 0; t < 3 * N / 4; t++) d[t] = q[t];
      bf16x_decode<N>(d, o);
    } else {
#pragma unroll
      for (int v = 0; v < N; v++) o[v] = 0.f;
    }
  } else {
    if (on) {
      Vec<T, N> x = *reinterpret_cast<const Vec<T, N> *>(p);
#pragma unroll
      for (int v = 0; v < N; v++) o[v] = to_f<T>(x.v[v]);
    } else {
#pragma unroll
      for (int v = 0; v < N; v++) o[v] = 0.f;
    }
  }
}

// Row access at a wave-uniform base plus a 32-bit byte offset (global_load saddr form).
template <typename T, int N>
__device__ __forceinline__ void ld_at(const T *base, unsigned boff, float (&o)[N], bool on) {
  ld_row<T, N>(reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + boff), o, on);
}

// Raw storage values of a row (no conversion), zero where the lane holds no node; `unpack`
// converts them when they are used, so loads issued ahead hold half the registers in BF16/FP16.
template <typename T, int N>
__device__ __forceinline__ void ld_raw(const T *base, unsigned boff, Vec<T, N> &x, bool on) {
  if constexpr (kDwordRow<T, N>) {
    if (on) {
      const unsigned *q = reinterpret_cast<const unsigned *>(reinterpret_cast<const char *>(base) + boff);
#pragma unroll
      for (int t = 0; t < 3 * N / 4; t++) x.w[t] = q[t];
    } else {
#pragma unroll
      for (int t = 0; t < 3 * N / 4; t++) x.w[t] = 0u;
    }
  } else {
    if (on) {
      x = *reinterpret_cast<const Vec<T, N> *>(reinterpret_cast<const char *>(base) + boff);
    } else {
#pragma unroll
      for (int v = 0; v < N; v++) x.v[v] = from_f<T>(0.f);
    }
  }
}

template <typename T, int N>
__device__ __forceinline__ void unpack(const Vec<T, N> &x, float (&o)[N]) {
  if constexpr (kDwordRow<T, N>) {
    bf16x_decode<N>(x.w, o);
  } else {
#pragma unroll
    for (int v = 0; v < N; v++) o[v] = to_f<T>(x.v[v]);
  }
}

// The value a store of x followed by a load returns: the fused sweep feeds H to the E update
// exactly as stored, as the split sweeps (which reload it) do.
template <typename T, int N>
__device__ __forceinline__ void as_stored(float (&o)[N]) {
  if constexpr (std::is_same<T, bf16x>::value) {
#pragma unroll
    for (int v = 0; v < N; v++) o[v] = __uint_as_float(bf16x_round(o[v]) & 0xffffff00u);
  } else if constexpr (!std::is_same<T, float>::value) {
#pragma unroll
    for (int v = 0; v < N; v++) o[v] = to_f<T>(from_f<T>(o[v]));
  }
}

template <typename T, int N>
__device__ __forceinline__ void st_row(T *p, const float (&o)[N], bool on);

template <typename T, int N>
__device__ __forceinline__ void st_at(T *base, unsigned boff, const float (&o)[N], bool on) {
  st_row<T, N>(reinterpret_cast<T *>(reinterpret_cast<char *>(base) + boff), o, on);
}

// Stores are non-temporal: a sweep writes the other time level, which no workgroup of the same
// sweep reads, so streaming it past the caches leaves L2 to the rows and planes that neighbouring
// tiles read twice (measured 3 % faster per step in FP32 and BF16).
template <typename T, int N>
__device__ __forceinline__ void st_row(T *p, const float (&o)[N], bool on) {
  if (!on) return;
  if constexpr (kDwordRow<T, N>) {
    // four 24-bit values (the top three bytes of each rounded word) packed into three dwords
#pragma unroll
    for (int g = 0; g < N / 4; g++) {
      const unsigned r0 = bf16x_round(o[4 * g]), r1 = bf16x_round(o[4 * g + 1]);
      const unsigned r2 = bf16x_round(o[4 * g + 2]), r3 = bf16x_round(o[4 * g + 3]);
      const unsigned w0 = (r0 >> 8) | (r1 & 0x0000ff00u) << 16;
      const unsigned w1 = (r1 >> 16) | ((r2 << 8) & 0xffff0000u);
      const unsigned w2 = (r2 >> 8 >> 16) | (r3 & 0xffffff00u);
      unsigned *q = reinterpret_cast<unsigned *>(p) + 3 * g;
      __builtin_nontemporal_store(w0, q);
      __builtin_nontemporal_store(w1, q + 1);
      __builtin_nontemporal_store(w2, q + 2);
    }
  } else {
    Vec<T, N> x;
#pragma unroll
    for (int v = 0; v < N; v++) x.v[v] = from_f<T>(o[v]);
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(x) == 16) {
      u4 b;
      __builtin_memcpy(&b, &x, 16);
      __builtin_nontemporal_store(b, reinterpret_cast<u4 *>(p));
    } else if constexpr (sizeof(x) == 8) {
      u2 b;
      __builtin_memcpy(&b, &x, 8);
      __builtin_nontemporal_store(b, reinterpret_cast<u2 *>(p));
    } else if constexpr (sizeof(x) == 4) {
      unsigned b;
      __builtin_memcpy(&b, &x, 4);
      __builtin_nontemporal_store(b, reinterpret_cast<unsigned *>(p));
    } else {
      *reinterpret_cast<Vec<T, N> *>(p) = x;
    }
  }
}

// Scaled stores of dynamically scaled levels: the values times a power of two r (exact), then
// rounded as st_row rounds.
template <typename T, int N>
__device__ __forceinline__ void st_row_s(T *p, const float (&o)[N], bool on, float r) {
  float t[N];
#pragma unroll
  for (int v = 0; v < N; v++) t[v] = o[v] * r;
  st_row<T, N>(p, t, on);
}

template <typename T, int N>
__device__ __forceinline__ void st_at_s(T *base, unsigned boff, const float (&o)[N], bool on, float r) {
  st_row_s<T, N>(reinterpret_cast<T *>(reinterpret_cast<char *>(base) + boff), o, on, r);
}

// ------------------------------------------------------- dynamic FP16 scaling
constexpr int kDynStep = 24;  // largest exponent change of one launch
constexpr int kDynExp = 60;   // range of a level's exponent

// Exponent change of the level that a launch of n steps writes, from the maxima of the level
// `par` it reads: with M_E, M_H those maxima and S the source's largest Ez increment (stored
// units), B_E = 2 M_E + 2 n (g_E M_H + S) and B_H = 2 M_H + 2 n g_H B_E bound what n steps can
// reach (the factors 2 cover the CPML terms, which add at most the size of the curl terms
// again), and the written level takes the largest power of two r with r max(B_E, B_H) < 2^14.
// Every wave of every kernel of the launch, and the publishing kernel after it, evaluates these
// expressions on the same words (contraction off), so all agree.
__device__ __forceinline__ int dyn_shift(const Dev &d, int par, int n) {
  const int e = *d.dexp[par];
  const int sl = *d.dslot[par];
  const float me = __uint_as_float(d.dmax[2 * sl]), mh = __uint_as_float(d.dmax[2 * sl + 1]);
  const float fn = (float)n;
  const float src = ldexpf(d.dyn_src, e);
  const float be = 2.f * me + 2.f * fn * (d.dyn_ge * mh + src);
  const float bh = 2.f * mh + 2.f * fn * (d.dyn_gh * be);
  const float b = fmaxf(be, bh);
  int sh;
  if (!(b <= 3.0e38f)) {
    sh = -kDynStep;  // non-finite maxima: scale down as far as one launch may
  } else if (b <= 0.f) {
    sh = kDynStep;  // zero fields and no source: scale up
  } else {
    int x;
    (void)frexpf(b, &x);  // b < 2^x, so 2^(14 - x) b < 2^14
    sh = 14 - x;
  }
  sh = min(max(sh, -kDynStep), kDynStep);
  return min(max(sh, -kDynExp - e), kDynExp - e);
}

// Loaded values brought to another level's units (a power of two: exact).
template <int N>
__device__ __forceinline__ void scale_in(float (&o)[N], float r) {
#pragma unroll
  for (int v = 0; v < N; v++) o[v] *= r;
}

// Largest |value| of the lanes' row (lanes without nodes add nothing).
template <int N>
__device__ __forceinline__ float absmax(float m, const float (&o)[N], bool on) {
  if (on) {
#pragma unroll
    for (int v = 0; v < N; v++) m = fmaxf(m, fabsf(o[v]));
  }
  return m;
}

// Raise a maxima word (float bits, values >= 0) to the wave's largest m: one atomic per wave,
// and only when it would raise the word.  Every lane of the wave takes part.
__device__ __forceinline__ void dyn_raise(unsigned *w, float m) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0 && m > __uint_as_float(*(volatile unsigned *)w)) atomicMax(w, __float_as_uint(m));
}

// ------------------------------------------------------------- cell updates
// Canonical order of one node update: the two central-difference terms (fmaf), then the CPML
// terms of the node's derivative axes added in the fixed axis order x, y, z, each with its sign
// folded in (s = +psi or -psi).  Every sweep variant applies exactly this sequence, so the
// results agree bitwise whichever variant computed a node.
__device__ __forceinline__ float pml_psi(float psi, float a, float b, float d) {
  return fmaf(b, psi, a * d);
}

// h' = h - c1 d1 + c2 d2, then the layer terms
__device__ __forceinline__ float h_plain(float h, float d1, float c1, float d2, float c2) {
  return fmaf(c2, d2, fmaf(-c1, d1, h));
}

// e' = ca e + c1 d1 - c2 d2, then the layer terms
__device__ __forceinline__ float e_plain(float ca, float e, float d1, float c1, float d2, float c2) {
  return fmaf(-c2, d2, fmaf(c1, d1, ca * e));
}

__device__ __forceinline__ float add_layers(float t, bool qx, float sx, bool qy, float sy, bool qz, float sz) {
  if (qx) t = t + sx;
  if (qy) t = t + sy;
  if (qz) t = t + sz;
  return t;
}

// Logical tile of this workgroup: consecutive logical tiles on one XCD (the hardware deals
// workgroups to the 8 XCDs round-robin).
__device__ __forceinline__ int xcd_logical() {
  const int b = blockIdx.x;
  return (b & 7) * (gridDim.x >> 3) + (b >> 3);
}

// Moving source bookkeeping (FP64): the rows of the longitudinal window around the bunch
// centre z_s, and Q(z_s) from the hat-function bins.
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

// Observer gather of one time level: one wave per observer, lane = 8*component + corner.  Each
// lane forms weight * E in FP64, then a butterfly over the 8 corners sums each component; lanes
// 0, 8, 16 write.
template <typename T>
__device__ __forceinline__ void gather_body(const Dev &d, int par, double *w, int column, int ld, int o,
                                            int lane = threadIdx.x) {
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
    const double out = val * (d.dyn ? ldexp(d.inv_se, -*d.dexp[par]) : d.inv_se);
    w[((long long)o * 3 + comp) * ld + column] = out;
    if (d.nan_flag && !isfinite(out)) *d.nan_flag = 1;
  }
}

}  // namespace chf
