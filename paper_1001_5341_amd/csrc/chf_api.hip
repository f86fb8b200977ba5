// Host side of libchfdtd: descriptor validation, FP64 coefficient tables, workspace layout
// and the C entry points declared in include/chfdtd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "chf_internal.h"

namespace {

constexpr double kC0 = 299792458.0;
constexpr double kMu0 = 1.25663706212e-6;  // CODATA 2018
const double kEps0 = 1.0 / (kMu0 * kC0 * kC0);

thread_local std::string g_err;

chf_status fail(chf_status s, const std::string &m) {
  g_err = m;
  return s;
}

chf_status hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return CHF_EHIP;
}

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Depth (in cells) of a position into the layer of `npml` cells at each end of an axis with
// n nodes (walls at 0 and n-1, inner layer planes at npml and n-1-npml); 0 outside.
double layer_depth(double pos, int n, int npml) {
  return std::max(std::max(npml - pos, pos - (n - 1 - npml)), 0.0);
}

struct Grade {
  double a, b, kappa;
};

// CFS-CPML grading (Roden & Gedney): stretch s = kappa + sigma/(alpha + j w eps0),
// recursion psi <- b psi + a dF, b = exp(-(sigma/kappa + alpha) dt/eps0),
// a = sigma (b - 1) / (sigma kappa + kappa^2 alpha).
Grade grade(const chf_plan &p, double depth, double delta) {
  const chf_boundary &B = p.bnd;
  const double eta0 = kMu0 * kC0;
  const double rho = depth / B.npml;
  const double sig_opt = 0.8 * (B.poly_m + 1.0) / (eta0 * delta * std::sqrt(p.med.eps_r * p.med.mu_r));
  const double sigma = B.sigma_scale * sig_opt * std::pow(rho, B.poly_m);
  const double kappa = 1.0 + (B.kappa_max - 1.0) * std::pow(rho, B.poly_m);
  const double alpha = B.alpha_max * (1.0 - rho);
  const double b = std::exp(-(sigma / kappa + alpha) * p.grid.dt / kEps0);
  const double a = sigma * (b - 1.0) / (sigma * kappa + kappa * kappa * alpha);
  return {a, b, kappa};
}

double pow2_near(double x) { return std::ldexp(1.0, (int)std::lround(std::log2(x))); }

}  // namespace

namespace chf {
void set_error(const std::string &msg) { g_err = msg; }
}  // namespace chf

extern "C" {

const char *chf_last_error(void) { return g_err.c_str(); }
int32_t chf_abi_version(void) { return CHF_ABI_VERSION; }

const char *chf_status_str(chf_status s) {
  switch (s) {
    case CHF_OK: return "ok";
    case CHF_EINVAL: return "invalid argument";
    case CHF_ECFL: return "time step above the Courant limit";
    case CHF_EDOMAIN: return "observer or source outside the usable interior";
    case CHF_ENOMEM: return "size overflow or workspace too small";
    case CHF_EHIP: return "HIP runtime error";
    case CHF_ENAN: return "non-finite value detected";
    case CHF_EUNSUPPORTED: return "unsupported configuration";
    case CHF_ESTATE: return "call out of order";
  }
  return "unknown status";
}

chf_status chf_plan_create(const chf_grid *grid, const chf_medium *medium, const chf_boundary *bnd,
                           const chf_source *src, const chf_observers *obs, const chf_exec *ex,
                           chf_plan **out) {
  if (!out) return fail(CHF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!grid || !medium || !bnd || !src || !obs || !ex) return fail(CHF_EINVAL, "NULL descriptor");
  const chf_grid &G = *grid;
  if (G.nx < 3 || G.ny < 3 || G.nz < 3) return fail(CHF_EINVAL, "need at least 3 nodes per axis");
  if (G.n_steps < 0) return fail(CHF_EINVAL, "n_steps < 0");
  if (!(G.dx > 0 && G.dy > 0 && G.dz > 0 && G.dt > 0) || !std::isfinite(G.dx + G.dy + G.dz + G.dt))
    return fail(CHF_EINVAL, "spacings and dt must be positive");
  if (!(medium->eps_r > 0 && medium->mu_r > 0 && medium->sigma >= 0))
    return fail(CHF_EINVAL, "bad medium");
  const double v = kC0 / std::sqrt(medium->eps_r * medium->mu_r);
  const double dt_max = 1.0 / (v * std::sqrt(1 / (G.dx * G.dx) + 1 / (G.dy * G.dy) + 1 / (G.dz * G.dz)));
  if (G.dt > dt_max) return fail(CHF_ECFL, "dt exceeds the Courant limit of the medium");
  if (bnd->kind < CHF_BC_PEC || bnd->kind > CHF_BC_CPML) return fail(CHF_EINVAL, "bad boundary kind");
  if (bnd->kind == CHF_BC_CPML) {
    const int m = 2 * bnd->npml + 3;
    if (bnd->npml < 1 || m > G.nx || m > G.ny || m > G.nz) return fail(CHF_EINVAL, "bad npml");
    if (!(bnd->poly_m >= 0 && bnd->sigma_scale >= 0 && bnd->kappa_max >= 1 && bnd->alpha_max >= 0))
      return fail(CHF_EINVAL, "bad CPML grading");
  }
  if (ex->storage < CHF_FP32 || ex->storage > CHF_BF16X) return fail(CHF_EINVAL, "bad storage");
  if (ex->kernel < CHF_KERNEL_AUTO || ex->kernel > CHF_KERNEL_FUSED2) return fail(CHF_EINVAL, "bad kernel");
  if (obs->n_obs < 0 || obs->n_obs > chf::kMaxObsPerPlan || (obs->n_obs > 0 && !obs->xyz))
    return fail(CHF_EINVAL, "bad observer list");
  if (src->n_bins < 0 || (src->n_bins > 0 && !src->q_bins)) return fail(CHF_EINVAL, "bad profile");
  const int64_t cells = (int64_t)G.nx * G.ny * G.nz;
  if (cells > (int64_t)1 << 40) return fail(CHF_ENOMEM, "grid too large");

  chf_plan *p = new (std::nothrow) chf_plan();
  if (!p) return fail(CHF_ENOMEM, "host allocation failed");
  p->grid = G;
  p->med = *medium;
  p->bnd = *bnd;
  p->src = *src;
  p->ex = *ex;
  if (bnd->kind != CHF_BC_CPML) p->bnd.npml = 0;
  p->q_bins.assign(src->q_bins, src->q_bins + src->n_bins);
  p->obs_xyz.assign(obs->xyz, obs->xyz + 3 * (size_t)obs->n_obs);
  p->src.q_bins = nullptr;
  p->storage = ex->storage;
  p->elem_bytes = ex->storage == CHF_FP32 ? 4 : (ex->storage == CHF_BF16X ? 3 : 2);

  // kernel and fused-sweep shape
  int kernel = ex->kernel == CHF_KERNEL_AUTO ? (G.nx <= 64 * chf::kMaxVX ? CHF_KERNEL_FUSED : CHF_KERNEL_SPLIT)
                                             : ex->kernel;
  const bool prefetch = kernel == CHF_KERNEL_FUSED_PREFETCH;
  if (prefetch) kernel = CHF_KERNEL_FUSED;
  // two steps per pass: waves_per_block and z_chunk shape the two-step tiles; the single steps
  // of odd step ranges take the fused sweep's default tile
  const bool two = kernel == CHF_KERNEL_FUSED2;
  if (two) kernel = CHF_KERNEL_FUSED;
  if (kernel == CHF_KERNEL_FUSED && G.nx > 64 * chf::kMaxVX) {
    delete p;
    return fail(CHF_EUNSUPPORTED, "fused sweep needs nx <= 512");
  }
  p->kernel = kernel;
  chf::FusedShape &fs = p->fs;
  fs.vx = 1;
  while (64 * fs.vx < G.nx) fs.vx *= 2;
  fs.rows = 1;
  // defaults: 7 rows (8 waves: two workgroups fill a CU at 4 waves per SIMD), 12 planes
  fs.waves = ex->waves_per_block > 0 && !two ? ex->waves_per_block : 7;
  fs.zchunk = ex->z_chunk > 0 && !two ? ex->z_chunk : 12;
  if (!(ex->rows_per_wave == 0 || ex->rows_per_wave == 1) ||
      !(fs.waves == 4 || fs.waves == 5 || fs.waves == 7 || fs.waves == 8 || fs.waves == 11 || fs.waves == 15)) {
    delete p;
    return fail(CHF_EINVAL, "rows_per_wave must be 0 or 1 and waves_per_block 4, 5, 7, 8, 11 or 15");
  }
  fs.prefetch = prefetch ? 1 : 0;
  fs.xs = 1;
  if (prefetch && fs.vx > 4) {
    // rows of 257-512 nodes: two waves of 64 x 4 nodes per row, 4 or 5 rows per tile
    fs.vx = 4;
    fs.xs = 2;
    if (ex->waves_per_block <= 0) fs.waves = 5;
    if (fs.waves != 4 && fs.waves != 5) {
      delete p;
      return fail(CHF_EINVAL, "the prefetching fused sweep over rows wider than 256 nodes takes waves_per_block 4 or 5");
    }
  } else if (prefetch && fs.waves > 11) {
    delete p;
    return fail(CHF_EINVAL, "the prefetching fused sweep takes waves_per_block 4, 7, 8 or 11");
  }
  if (fs.waves == 5 && fs.xs != 2) {
    delete p;
    return fail(CHF_EINVAL, "waves_per_block 5 is for the prefetching sweep over rows wider than 256 nodes");
  }
  if (kernel == CHF_KERNEL_FUSED && fs.vx > 4 && fs.waves != 4 && fs.waves != 7) {
    delete p;
    return fail(CHF_EINVAL, "the fused sweep over rows wider than 256 nodes takes waves_per_block 4 or 7");
  }
  if (ex->dynamic_scaling) {
    // the fused sweeps (one or two steps) carry the scale; their boundary tiles must take the
    // general fused sweep (not the split sweeps), and Mur's update reads two levels
    const bool gen = (fs.vx <= chf::kMaxGeneralVX && fs.waves <= chf::kMaxGeneralW) || fs.xs == 2;
    if (ex->storage != CHF_FP16 || kernel != CHF_KERNEL_FUSED || !gen || bnd->kind == CHF_BC_MUR1) {
      delete p;
      return fail(CHF_EUNSUPPORTED, "dynamic scaling takes FP16 storage, the fused sweeps with tiles of at most 11 "
                                    "rows of at most 256 nodes (or split rows), and PEC or CPML walls");
    }
  }
  if ((int64_t)((G.nx + 15) / 16 * 16) * G.ny >= ((int64_t)1 << 31)) {
    delete p;
    return fail(CHF_EUNSUPPORTED, "one x-y plane must hold fewer than 2^31 nodes");
  }
  {
    // fast rectangle: every row of the tile and the row below it lie in [fy0, fy1], every plane
    // of the chunk in [fz0, fz1], where [f0, f1] are the nodes with no wall and no layer term
    // (integer and half positions alike); all other tiles go to the boundary sweeps.  The tile
    // grid is shifted (tile ty from row ty*W - ysh, chunk zc from plane zc*Z - zsh) so that the
    // rectangle starts at row fy0 + 1 and plane fz0: the boundary sweeps, which cost more per
    // node, then cover only the walls and layers and less than one tile or chunk beyond them.
    const int nl = bnd->kind == CHF_BC_CPML ? bnd->npml : 0;
    const int fy0 = std::max(1, nl), fy1 = G.ny - 2 - nl;
    const int fz0 = std::max(1, nl), fz1 = G.nz - 2 - nl;
    const int W = fs.waves, Z = fs.zchunk;
    for (int shifted = 1; shifted >= 0; shifted--) {
      fs.ysh = shifted ? (W - (fy0 + 1) % W) % W : 0;
      fs.zsh = shifted ? (Z - fz0 % Z) % Z : 0;
      fs.ty_lo = (fy0 + 1 + fs.ysh + W - 1) / W;  // j0 - 1 >= fy0
      fs.ty_hi = (fy1 + 1 + fs.ysh) / W;          // j0 + W - 1 <= fy1
      fs.zc_lo = (fz0 + fs.zsh + Z - 1) / Z;      // k0 >= fz0
      fs.zc_hi = (fz1 + 1 + fs.zsh) / Z;          // k1 - 1 <= fz1
      const bool rect = kernel == CHF_KERNEL_FUSED && fs.ty_hi > fs.ty_lo && fs.zc_hi > fs.zc_lo &&
                        2 * nl <= chf::kMaxFusedLayer && fy1 >= fy0 && fz1 >= fz0;
      if (rect) break;
      fs.ty_lo = fs.ty_hi = fs.zc_lo = fs.zc_hi = 0;
    }
    fs.nty = (G.ny + fs.ysh + fs.waves - 1) / fs.waves;
    fs.nzc = (G.nz + fs.zsh + fs.zchunk - 1) / fs.zchunk;
    fs.n_tiles = fs.nty * fs.nzc;
    fs.n_blocks = (fs.n_tiles + 7) / 8 * 8;
    fs.n_fast = (fs.ty_hi - fs.ty_lo) * (fs.zc_hi - fs.zc_lo);
    fs.fast_blocks = (fs.n_fast + 7) / 8 * 8;
    fs.n_layer = fs.layer_blocks = 0;
    // boundary tiles: first those whose chunk lies in the interior z range (y walls and layers
    // only), then the rest
    for (int pass = 0; pass < 2; pass++) {
      for (int zc = 0; zc < fs.nzc; zc++)
        for (int ty = 0; ty < fs.nty; ty++) {
          const bool zin = zc >= fs.zc_lo && zc < fs.zc_hi;
          if ((ty >= fs.ty_lo && ty < fs.ty_hi && zin) || zin != (pass == 0)) continue;
          p->slow_tiles.push_back(ty);
          p->slow_tiles.push_back(zc);
        }
      if (pass == 0) fs.n_slow_y = (int)(p->slow_tiles.size() / 2);
    }
    fs.n_slow = (int)(p->slow_tiles.size() / 2);
    fs.slow_blocks = (fs.n_slow + 7) / 8 * 8;
  }
  chf::Shape2 &f2 = p->fs2;
  f2 = chf::Shape2{};
  if (two) {
    const int nl = bnd->kind == CHF_BC_CPML ? bnd->npml : 0;
    if (bnd->kind == CHF_BC_MUR1) {
      delete p;
      return fail(CHF_EUNSUPPORTED, "the two-step sweep takes PEC or CPML walls");
    }
    if (2 * nl > chf::kMaxStep2Layer) {
      delete p;
      return fail(CHF_EUNSUPPORTED, "the two-step sweep takes a CPML of at most 16 cells");
    }
    f2.on = 1;
    f2.xs = G.nx > 256 ? 2 : 1;
    f2.vx = G.nx > 128 ? 4 : (G.nx > 64 ? 2 : 1);
    f2.waves = ex->waves_per_block > 0 ? ex->waves_per_block : 8;
    f2.zchunk = ex->z_chunk > 0 ? ex->z_chunk : 32;
    if (f2.xs > 1) {
      delete p;
      return fail(CHF_EUNSUPPORTED, "the two-step sweep takes rows of at most 256 nodes");
    }
    if (!(f2.waves == 4 || f2.waves == 7 || f2.waves == 8)) {
      delete p;
      return fail(CHF_EINVAL, "the two-step sweep takes waves_per_block 4, 7 or 8");
    }
    const int W = f2.waves, Z = f2.zchunk;
    // rectangle: computed rows j0-2 .. j0+W within [fy0, fy1], stage planes k0-2 .. k1 within
    // [fz0, fz1] (nodes with no wall and no layer term); rectangle tile ty owns rows from
    // ty*W - ysh and chunk zc planes from zc*Z - zsh, the shifts chosen so that the rectangle
    // starts at row fy0 + 2 and plane fz0 + 2 (the boundary tiles, which recompute halo rows,
    // then cover only the walls and layers and less than one tile or chunk beyond them)
    const int fy0 = std::max(1, nl), fy1 = G.ny - 2 - nl;
    const int fz0 = std::max(1, nl), fz1 = G.nz - 2 - nl;
    for (int shifted = 1; shifted >= 0; shifted--) {
      f2.ysh = shifted ? (W - (fy0 + 2) % W) % W : 0;
      f2.zsh = shifted ? (Z - (fz0 + 2) % Z) % Z : 0;
      f2.nty = (G.ny + f2.ysh + W - 1) / W;
      f2.nzc = (G.nz + f2.zsh + Z - 1) / Z;
      f2.ty_lo = (fy0 + 2 + f2.ysh + W - 1) / W;                           // j0 - 2 >= fy0
      f2.ty_hi = fy1 - W + f2.ysh >= 0 ? (fy1 - W + f2.ysh) / W + 1 : 0;  // j0 + W <= fy1
      f2.zc_lo = (fz0 + 2 + f2.zsh + Z - 1) / Z;                           // k0 - 2 >= fz0
      f2.zc_hi = fz1 - Z + f2.zsh >= 0 ? (fz1 - Z + f2.zsh) / Z + 1 : 0;  // k1 <= fz1
      f2.ty_hi = std::min(f2.ty_hi, f2.nty);
      f2.zc_hi = std::min(f2.zc_hi, f2.nzc);
      if (f2.ty_hi > f2.ty_lo && f2.zc_hi > f2.zc_lo) break;
      f2.ty_lo = f2.ty_hi = f2.zc_lo = f2.zc_hi = 0;
    }
    f2.n_fast = (f2.ty_hi - f2.ty_lo) * (f2.zc_hi - f2.zc_lo);
    f2.fast_blocks = (f2.n_fast + 7) / 8 * 8;
    // boundary tiles of kStep2BoundaryRows rows: the rows below and above the rectangle in its z
    // range, then every row of the other chunks
    const int B = chf::kStep2BoundaryRows;
    const int ya = f2.ty_lo * W - f2.ysh, yb = f2.ty_hi * W - f2.ysh;
    auto cover = [&](int zc, int lo, int hi) {
      for (int j0 = lo; j0 < hi; j0 += B) {
        p->tiles2.push_back(j0);
        p->tiles2.push_back(std::min(j0 + B, hi));
        p->tiles2.push_back(zc);
      }
    };
    const bool rect = f2.n_fast > 0;
    for (int zc = f2.zc_lo; zc < f2.zc_hi && rect; zc++) {
      cover(zc, 0, ya);
      cover(zc, yb, G.ny);
    }
    f2.n_slow_y = (int)(p->tiles2.size() / 3);
    for (int zc = 0; zc < f2.nzc; zc++)
      if (!rect || zc < f2.zc_lo || zc >= f2.zc_hi) cover(zc, 0, G.ny);
    f2.n_slow = (int)(p->tiles2.size() / 3);
  }

  // coefficients (FP64)
  const double eps = kEps0 * medium->eps_r, mu = kMu0 * medium->mu_r;
  const double loss = medium->sigma * G.dt / (2.0 * eps);
  p->ca = (1.0 - loss) / (1.0 + loss);
  p->cb = (G.dt / eps) / (1.0 + loss);
  p->db = G.dt / mu;
  // storage scales: H stored in E-like units (power of two nearest the medium impedance)
  const double eta = kMu0 * kC0 * std::sqrt(medium->mu_r / medium->eps_r);
  p->scale_h = ex->scale_h > 0 ? ex->scale_h : pow2_near(eta);
  p->scale_e = 1.0;
  if (ex->scale_e > 0) {
    p->scale_e = ex->scale_e;
  } else if (ex->storage == CHF_FP16 && src->n_bins > 0) {
    // FP16: map an estimate of the largest field (the Coulomb field of the total charge at one
    // radial width) to ~2^14 so that the pulse tails stay above the subnormal range
    double qmax = 0.0;
    for (double q : p->q_bins) qmax = std::max(qmax, std::fabs(q));
    const double e_est = qmax / (4.0 * M_PI * eps * src->sigma_r * src->sigma_r);
    if (e_est > 0) p->scale_e = std::ldexp(1.0, (int)std::floor(std::log2(16384.0 / e_est)));
  }
  p->scale_h *= p->scale_e;
  for (double s : {p->scale_e, p->scale_h}) {
    int e;
    if (std::frexp(s, &e) != 0.5) {
      delete p;
      return fail(CHF_EINVAL, "storage scales must be powers of two");
    }
  }
  const double rse = p->scale_e / p->scale_h, rhs = p->scale_h / p->scale_e;

  // axis tables: ce, ch, ae, be, ah, bh (float) and se, sh (int)
  const int n3[3] = {G.nx, G.ny, G.nz};
  const double d3[3] = {G.dx, G.dy, G.dz};
  const int npml = p->bnd.npml;
  size_t off_f = 0, off_i = 0;
  for (int u = 0; u < 3; u++) {
    for (int t = 0; t < 10; t++) p->off_tabf[u][t] = off_f + (size_t)t * n3[u];
    for (int t = 0; t < 2; t++) p->off_tabi[u][t] = off_i + (size_t)t * n3[u];
    off_f += 10 * (size_t)n3[u];
    off_i += 2 * (size_t)n3[u];
  }
  p->tabf.assign(off_f, 0.0f);
  p->tabi.assign(off_i, -1);
  for (int u = 0; u < 3; u++) {
    const int n = n3[u];
    float *ce = &p->tabf[p->off_tabf[u][0]], *ch = &p->tabf[p->off_tabf[u][1]];
    float *ae = &p->tabf[p->off_tabf[u][2]], *be = &p->tabf[p->off_tabf[u][3]];
    float *ah = &p->tabf[p->off_tabf[u][4]], *bh = &p->tabf[p->off_tabf[u][5]];
    int *se = &p->tabi[p->off_tabi[u][0]], *sh = &p->tabi[p->off_tabi[u][1]];
    float *ike = &p->tabf[p->off_tabf[u][6]], *ade = &p->tabf[p->off_tabf[u][7]];
    float *ikh = &p->tabf[p->off_tabf[u][8]], *adh = &p->tabf[p->off_tabf[u][9]];
    for (int i = 0; i < n; i++) {
      ce[i] = (float)(rse * p->cb / d3[u]);
      ch[i] = (float)(rhs * p->db / d3[u]);
      ike[i] = ikh[i] = (float)(1.0 / d3[u]);
      be[i] = bh[i] = 1.0f;
      if (npml <= 0) continue;
      const double de = layer_depth((double)i, n, npml);
      if (de > 0.0) {
        se[i] = i < npml ? i : npml + (i - (n - npml));
        Grade g = grade(*p, de, d3[u]);
        ce[i] = (float)(rse * p->cb / (d3[u] * g.kappa));
        ae[i] = (float)(rse * p->cb * g.a / d3[u]);
        be[i] = (float)g.b;
        ike[i] = (float)(1.0 / (d3[u] * g.kappa));
        ade[i] = (float)(g.a / d3[u]);
      }
      if (i <= n - 2) {
        const double dh = layer_depth(i + 0.5, n, npml);
        if (dh > 0.0) {
          sh[i] = i < npml ? i : npml + (i - (n - 1 - npml));
          Grade g = grade(*p, dh, d3[u]);
          ch[i] = (float)(rhs * p->db / (d3[u] * g.kappa));
          ah[i] = (float)(rhs * p->db * g.a / d3[u]);
          bh[i] = (float)g.b;
          ikh[i] = (float)(1.0 / (d3[u] * g.kappa));
          adh[i] = (float)(g.a / d3[u]);
        }
      }
    }
  }

  // source: radial weights at the Ez nodes (x_i, y_j), disc of radius cut*sigma_r,
  // normalised so that sum W dx dy = 1 over the nodes Ez is updated on
  chf::Dev &D = p->dev;
  D.src_on = src->n_bins > 0 ? 1 : 0;
  if (D.src_on) {
    if (!(src->sigma_r > 0 && src->sigma_z > 0 && src->cut_sigmas > 0 && src->dz_bin > 0 && src->beta >= 0)) {
      delete p;
      return fail(CHF_EINVAL, "bad source widths");
    }
    if (src->cut_sigmas * src->sigma_z / G.dz > 0.5 * (chf::kMaxWz - 2)) {
      delete p;
      return fail(CHF_EUNSUPPORTED, "longitudinal source support too wide");
    }
    const double rc = src->cut_sigmas * src->sigma_r;
    int i0 = std::max(1, (int)std::ceil((src->x_axis - rc) / G.dx));
    int i1 = std::min(G.nx - 2, (int)std::floor((src->x_axis + rc) / G.dx));
    int j0 = std::max(1, (int)std::ceil((src->y_axis - rc) / G.dy));
    int j1 = std::min(G.ny - 2, (int)std::floor((src->y_axis + rc) / G.dy));
    if (i1 < i0 || j1 < j0) {
      delete p;
      return fail(CHF_EDOMAIN, "source axis outside the grid");
    }
    D.src_i0 = i0;
    D.src_j0 = j0;
    D.src_ni = i1 - i0 + 1;
    D.src_nj = j1 - j0 + 1;
    p->wr.assign((size_t)D.src_ni * D.src_nj, 0.0);
    double norm = 0.0;
    // second half: d W / d sigma_r (the disc's support held fixed), for the source-parameter
    // gradients of the adjoint
    const size_t npatch = (size_t)D.src_ni * D.src_nj;
    p->wr.assign(2 * npatch, 0.0);
    double dnorm = 0.0;
    const double s2 = src->sigma_r * src->sigma_r;
    for (int j = j0; j <= j1; j++)
      for (int i = i0; i <= i1; i++) {
        const double ddx = i * G.dx - src->x_axis, ddy = j * G.dy - src->y_axis;
        const double r2 = ddx * ddx + ddy * ddy;
        if (r2 <= rc * rc) {
          const double w = std::exp(-0.5 * r2 / s2);
          const double dw = w * r2 / (s2 * src->sigma_r);
          p->wr[(size_t)(j - j0) * D.src_ni + (i - i0)] = w;
          p->wr[npatch + (size_t)(j - j0) * D.src_ni + (i - i0)] = dw;
          norm += w * G.dx * G.dy;
          dnorm += dw * G.dx * G.dy;
        }
      }
    if (norm <= 0.0) {
      delete p;
      return fail(CHF_EDOMAIN, "source disc misses the grid");
    }
    for (size_t c = 0; c < npatch; c++) {
      const double wn = p->wr[c] / norm;
      p->wr[npatch + c] = p->wr[npatch + c] / norm - wn * dnorm / norm;
      p->wr[c] = wn;
    }
  }

  // observers: base node and fractional offsets per component and axis
  const int margin = npml > 0 ? npml : 1;
  p->obs_idx.resize((size_t)obs->n_obs * 9);
  p->obs_t.resize((size_t)obs->n_obs * 9);
  for (int o = 0; o < obs->n_obs; o++)
    for (int c = 0; c < 3; c++)
      for (int u = 0; u < 3; u++) {
        const double f = p->obs_xyz[3 * o + u] / d3[u] - (u == c ? 0.5 : 0.0);
        const double fl = std::floor(f);
        if (!std::isfinite(f) || fl < margin || fl + 1 > n3[u] - 1 - margin) {
          delete p;
          return fail(CHF_EDOMAIN, "observer stencil outside the interior (obs " + std::to_string(o) + ")");
        }
        p->obs_idx[(o * 3 + c) * 3 + u] = (int)fl;
        p->obs_t[(o * 3 + c) * 3 + u] = f - fl;
      }

  // workspace layout
  int pitch = (G.nx + 15) / 16 * 16;
  {
    // transposed sampling table: the adjoint adds w g^n into Eb at each stencil node; nodes
    // shared by several stencils take their contributions in observer order
    const long long plane_ = (long long)pitch * G.ny;
    std::map<std::pair<int, long long>, int> key_of;
    std::vector<std::vector<std::pair<int, double>>> lists;
    for (int o = 0; o < obs->n_obs; o++)
      for (int c = 0; c < 3; c++) {
        const int *ix = &p->obs_idx[(o * 3 + c) * 3];
        const double *tf = &p->obs_t[(o * 3 + c) * 3];
        for (int corner = 0; corner < 8; corner++) {
          const int a = corner & 1, b = (corner >> 1) & 1, cc = corner >> 2;
          const double w = (a ? tf[0] : 1.0 - tf[0]) * (b ? tf[1] : 1.0 - tf[1]) * (cc ? tf[2] : 1.0 - tf[2]);
          const long long node = (long long)(ix[2] + cc) * plane_ + (long long)(ix[1] + b) * pitch + (ix[0] + a);
          auto it = key_of.find({c, node});
          int key;
          if (it == key_of.end()) {
            key = (int)lists.size();
            key_of[{c, node}] = key;
            lists.emplace_back();
            p->sk_comp.push_back(c);
            p->sk_node.push_back(node);
          } else {
            key = it->second;
          }
          lists[key].push_back({o, w});
        }
      }
    p->sk_ptr.assign(1, 0);
    for (const auto &l : lists) {
      for (const auto &e : l) {
        p->se_obs.push_back(e.first);
        p->se_w.push_back(e.second);
      }
      p->sk_ptr.push_back((int)p->se_obs.size());
    }
    D.n_skeys = (int)lists.size();
  }
  if (p->fs2.on && obs->n_obs > 0) {
    // samples of the intermediate level of a two-step pass: one slot per distinct (component,
    // node) of the observers' stencils, entries sorted by plane
    std::map<std::array<int, 4>, int> slot_of;  // (k, j, i, comp) -> slot
    p->smp_slot.assign((size_t)obs->n_obs * 24, 0);
    for (int o = 0; o < obs->n_obs; o++)
      for (int c = 0; c < 3; c++) {
        const int *ix = &p->obs_idx[(o * 3 + c) * 3];
        for (int corner = 0; corner < 8; corner++) {
          const int a = corner & 1, b = (corner >> 1) & 1, cc = corner >> 2;
          const std::array<int, 4> key{ix[2] + cc, ix[1] + b, ix[0] + a, c};
          auto it = slot_of.find(key);
          int slot;
          if (it == slot_of.end()) {
            slot = (int)slot_of.size();
            slot_of[key] = slot;
          } else {
            slot = it->second;
          }
          p->smp_slot[(o * 3 + c) * 8 + corner] = slot;
        }
      }
    p->n_smp = slot_of.size();
    p->smp_ptr.assign((size_t)G.nz + 1, 0);
    for (const auto &kv : slot_of) p->smp_ptr[kv.first[0] + 1]++;
    for (int k = 0; k < G.nz; k++) p->smp_ptr[k + 1] += p->smp_ptr[k];
    p->smp_ent.clear();
    for (const auto &kv : slot_of)  // map order: by plane, then row, node, component
      p->smp_ent.insert(p->smp_ent.end(), {kv.first[1], kv.first[2], kv.first[3], kv.second});
  }
  const uint64_t field = align256((uint64_t)pitch * G.ny * G.nz * p->elem_bytes);
  uint64_t off = 0;
  for (int l = 0; l < 2; l++)
    for (int c = 0; c < 3; c++) {
      p->off_e[l][c] = off;
      off += field;
      p->off_h[l][c] = off;
      off += field;
    }
  p->field_bytes = off;
  const int np2 = 2 * npml;
  p->psi_len[0] = (uint64_t)G.nz * G.ny * np2;
  p->psi_len[1] = (uint64_t)G.nz * np2 * pitch;
  p->psi_len[2] = (uint64_t)np2 * G.ny * pitch;
  const uint64_t off_psi0 = off;
  for (int u = 0; u < 3; u++) {
    const uint64_t len = align256(p->psi_len[u] * 4);
    for (int t = 0; t < 2; t++) {
      p->off_psi_e[u][t] = off;
      off += len;
      p->off_psi_h[0][u][t] = off;
      off += len;
      p->off_psi_h[1][u][t] = off;
      off += len;
    }
  }
  for (int u = 0; u < 3; u++)
    for (int t = 0; t < 2; t++) {
      p->off_psi_e2[u][t] = off;
      if (p->fs2.on) off += align256(p->psi_len[u] * 4);
    }
  p->psi_bytes = off - off_psi0;
  p->off_dyn = off;  // dynamic scaling words: part of the state (snapshots carry them)
  off += 256;
  p->off_tf = off;
  off += align256(p->tabf.size() * sizeof(float));
  p->off_ti = off;
  off += align256(p->tabi.size() * sizeof(int));
  p->off_wr = off;
  off += align256(std::max<size_t>(p->wr.size(), 1) * sizeof(double));
  p->off_q = off;
  off += align256(std::max<size_t>(p->q_bins.size(), 1) * sizeof(double));
  p->off_oidx = off;
  off += align256(std::max<size_t>(p->obs_idx.size(), 1) * sizeof(int));
  p->off_ot = off;
  off += align256(std::max<size_t>(p->obs_t.size(), 1) * sizeof(double));
  p->off_nan = off;
  off += 256;
  p->off_tiles = off;
  off += align256(std::max<size_t>(p->slow_tiles.size(), 1) * sizeof(int));
  p->off_ltiles = off;
  off += align256(std::max<size_t>(p->layer_tiles.size(), 1) * sizeof(int));
  for (int u = 0; u < 3; u++)
    for (int t = 0; t < 2; t++) {
      p->off_psi_eb[u][t] = off;
      off += align256(p->psi_len[u] * 4);
    }
  p->off_sknode = off;
  off += align256(std::max<size_t>(p->sk_node.size(), 1) * sizeof(long long));
  p->off_skcomp = off;
  off += align256(std::max<size_t>(p->sk_comp.size(), 1) * sizeof(int));
  p->off_skptr = off;
  off += align256(std::max<size_t>(p->sk_ptr.size(), 1) * sizeof(int));
  p->off_seobs = off;
  off += align256(std::max<size_t>(p->se_obs.size(), 1) * sizeof(int));
  p->off_sew = off;
  off += align256(std::max<size_t>(p->se_w.size(), 1) * sizeof(double));
  p->off_tiles2 = off;
  off += align256(std::max<size_t>(p->tiles2.size(), 1) * sizeof(int));
  p->off_smp_ptr = off;
  off += align256(std::max<size_t>(p->smp_ptr.size(), 1) * sizeof(int));
  p->off_smp_ent = off;
  off += align256(std::max<size_t>(p->smp_ent.size(), 4) * sizeof(int));
  p->off_smp = off;
  off += align256(std::max<size_t>(p->n_smp, 1) * sizeof(float));
  p->off_smp_slot = off;
  off += align256(std::max<size_t>(p->smp_slot.size(), 1) * sizeof(int));
  p->ws_bytes = off;

  // kernel parameter block (device pointers are filled at bind time)
  D.nx = G.nx;
  D.ny = G.ny;
  D.nz = G.nz;
  D.pitch = pitch;
  D.npml = npml;
  D.np2 = np2;
  D.plane = (long long)pitch * G.ny;
  D.ysh = p->fs.ysh;
  D.zsh = p->fs.zsh;
  D.ca = (float)p->ca;
  D.se = (float)p->scale_e;
  D.sh = (float)p->scale_h;
  D.n_bins = src->n_bins;
  D.x_axis = src->x_axis;
  D.y_axis = src->y_axis;
  D.z_entry = src->z_entry;
  D.t_entry = src->t_entry;
  D.v_src = src->beta * kC0;
  D.sigma_z = src->sigma_z;
  D.cut_sigmas = src->cut_sigmas;
  D.z_bin0 = src->z_bin0;
  D.dz_bin = src->dz_bin;
  D.dz = G.dz;
  D.dt = G.dt;
  D.cb_src = p->scale_e * p->cb;
  D.n_obs = obs->n_obs;
  D.inv_se = 1.0 / p->scale_e;
  D.bc = p->bnd.kind;
  D.a_cb = (float)p->cb;
  D.a_db = (float)p->db;
  D.a_ca = (float)p->ca;
  D.a_cb_src = p->cb;
  if (ex->dynamic_scaling) {
    // bound constants of the per-launch scale choice, in stored units at exponent 0: the
    // largest per-step gain of the curl terms (2 |c| per axis), and the source's largest Ez
    // increment (the normalised longitudinal weights are at most 1/dz)
    double ge = 0.0, gh = 0.0;
    for (int u = 0; u < 3; u++) {
      double me = 0.0, mh = 0.0;
      for (int i = 0; i < n3[u]; i++) {
        me = std::max(me, (double)std::fabs(p->tabf[p->off_tabf[u][0] + i]));
        mh = std::max(mh, (double)std::fabs(p->tabf[p->off_tabf[u][1] + i]));
      }
      ge += 2.0 * me;
      gh += 2.0 * mh;
    }
    double qmax = 0.0, wmax = 0.0;
    for (double q : p->q_bins) qmax = std::max(qmax, std::fabs(q));
    for (int t = 0; t < D.src_ni * D.src_nj && t < (int)p->wr.size(); t++) wmax = std::max(wmax, std::fabs(p->wr[t]));
    D.dyn = 1;
    D.dyn_ge = (float)ge;
    D.dyn_gh = (float)gh;
    D.dyn_src = D.src_on ? (float)(std::fabs(D.cb_src) * D.v_src * qmax * wmax / G.dz) : 0.f;
  }
  const double vdt = v * G.dt;
  D.mur_kx = (float)((vdt - G.dx) / (vdt + G.dx));
  D.mur_ky = (float)((vdt - G.dy) / (vdt + G.dy));
  D.mur_kz = (float)((vdt - G.dz) / (vdt + G.dz));
  *out = p;
  return CHF_OK;
}

void chf_plan_destroy(chf_plan *plan) {
  if (!plan) return;
  if (plan->graph) (void)hipGraphExecDestroy(plan->graph);
  if (plan->ev_fork) (void)hipEventDestroy(plan->ev_fork);
  if (plan->ev_join) (void)hipEventDestroy(plan->ev_join);
  if (plan->aux) (void)hipStreamDestroy(plan->aux);
  if (plan->ev_join2) (void)hipEventDestroy(plan->ev_join2);
  if (plan->aux2) (void)hipStreamDestroy(plan->aux2);
  delete plan;
}

chf_status chf_plan_workspace_bytes(const chf_plan *plan, uint64_t *bytes) {
  if (!plan || !bytes) return fail(CHF_EINVAL, "NULL argument");
  *bytes = plan->ws_bytes;
  return CHF_OK;
}

}  // extern "C"

namespace chf {
// Points the plan's kernel parameters at the workspace `ws` (>= ws_bytes, 256-byte aligned) and
// uploads its tables there with stream-ordered copies.  Creates nothing and allocates nothing.
// Field and psi pointers in the unexchanged order (level l at its own offsets).
void canonical_pointers(chf_plan &p) {
  char *ws = p.ws;
  chf::Dev &D = p.dev;
  for (int l = 0; l < 2; l++)
    for (int c = 0; c < 3; c++) {
      D.e[l][c] = ws + p.off_e[l][c];
      D.h[l][c] = ws + p.off_h[l][c];
    }
  for (int u = 0; u < 3; u++)
    for (int t = 0; t < 2; t++) {
      D.psi_e[u][t] = (float *)(ws + p.off_psi_e[u][t]);
      D.psi_e2[u][t] = (float *)(ws + p.off_psi_e2[u][t]);
      D.psi_h[0][u][t] = (float *)(ws + p.off_psi_h[0][u][t]);
      D.psi_h[1][u][t] = (float *)(ws + p.off_psi_h[1][u][t]);
    }
  for (int l = 0; l < 2; l++) {
    D.dexp[l] = (int *)(ws + p.off_dyn + 16 * l);
    D.dslot[l] = (int *)(ws + p.off_dyn + 16 * l + 4);
  }
  D.dmax = (unsigned *)(ws + p.off_dyn + 32);
  p.lev_swap = p.pe_swap = 0;
}

// After a two-step launch from level `parity` into parity^1: the new state is made level
// `parity` again by exchanging the two levels (fields, psi_H) and the two psi_E levels.
void swap_levels(chf_plan &p, Dev &d) {
  for (int c = 0; c < 3; c++) {
    std::swap(d.e[0][c], d.e[1][c]);
    std::swap(d.h[0][c], d.h[1][c]);
  }
  for (int u = 0; u < 3; u++)
    for (int t = 0; t < 2; t++) {
      std::swap(d.psi_h[0][u][t], d.psi_h[1][u][t]);
      std::swap(d.psi_e[u][t], d.psi_e2[u][t]);
    }
  std::swap(d.dexp[0], d.dexp[1]);
  std::swap(d.dslot[0], d.dslot[1]);
  if (&d == &p.dev) {
    p.lev_swap ^= 1;
    p.pe_swap ^= 1;
  }
}

hipError_t advance(chf_plan &p, hipStream_t s, const double *q, double *w, int col0, int ld, int n, hipEvent_t *ev,
                   int *n_ev) {
  Dev d = p.dev;
  if (!p.ex.nan_watch) d.nan_flag = nullptr;
  int cnt = 0;
  hipError_t e = hipSuccess;
  for (int t = 0; t < n && e == hipSuccess;) {
    if (p.fs2.on && n - t >= 2) {
      e = launch_step2(p, d, p.parity, p.n_done, q, w, col0 + t, ld, s, ev ? ev[2 * cnt] : nullptr,
                       ev ? ev[2 * cnt + 1] : nullptr);
      cnt++;
      swap_levels(p, d);
      swap_levels(p, p.dev);
      p.n_done += 2;
      t += 2;
    } else {
      const bool timed = ev && !p.fs2.on;
      e = launch_step(p, d, p.parity, p.n_done, q, w, col0 + t, ld, s, timed ? ev[2 * cnt] : nullptr,
                      timed ? ev[2 * cnt + 1] : nullptr);
      if (timed) cnt++;
      p.parity ^= 1;
      p.n_done++;
      t++;
    }
  }
  if (n_ev) *n_ev = cnt;
  return e;
}

hipError_t bind_tables(chf_plan *p, char *ws, hipStream_t s) {
  p->ws = ws;
  chf::Dev &D = p->dev;
  canonical_pointers(*p);
  for (int u = 0; u < 3; u++)
    for (int t = 0; t < 2; t++) D.psi_eb[u][t] = (float *)(ws + p->off_psi_eb[u][t]);
  const float *tf = (const float *)(ws + p->off_tf);
  const int *ti = (const int *)(ws + p->off_ti);
  for (int u = 0; u < 3; u++) {
    chf::AxisTab &A = D.ax[u];
    A.ce = tf + p->off_tabf[u][0];
    A.ch = tf + p->off_tabf[u][1];
    A.ae = tf + p->off_tabf[u][2];
    A.be = tf + p->off_tabf[u][3];
    A.ah = tf + p->off_tabf[u][4];
    A.bh = tf + p->off_tabf[u][5];
    A.se = ti + p->off_tabi[u][0];
    A.sh = ti + p->off_tabi[u][1];
    A.ike = tf + p->off_tabf[u][6];
    A.ade = tf + p->off_tabf[u][7];
    A.ikh = tf + p->off_tabf[u][8];
    A.adh = tf + p->off_tabf[u][9];
  }
  D.wr = (const double *)(ws + p->off_wr);
  D.dwr = D.wr + (D.src_on ? (size_t)D.src_ni * D.src_nj : 0);
  D.q_bins = (const double *)(ws + p->off_q);
  D.obs_idx = (const int *)(ws + p->off_oidx);
  D.obs_t = (const double *)(ws + p->off_ot);
  D.sk_node = (const long long *)(ws + p->off_sknode);
  D.sk_comp = (const int *)(ws + p->off_skcomp);
  D.sk_ptr = (const int *)(ws + p->off_skptr);
  D.se_obs = (const int *)(ws + p->off_seobs);
  D.se_w = (const double *)(ws + p->off_sew);
  D.nan_flag = (int *)(ws + p->off_nan);
  D.slow_tiles = (const int *)(ws + p->off_tiles);
  D.layer_tiles = (const int *)(ws + p->off_ltiles);
  D.smp_ptr = p->n_smp ? (const int *)(ws + p->off_smp_ptr) : nullptr;
  D.smp_ent = (const int4 *)(ws + p->off_smp_ent);
  D.smp = (float *)(ws + p->off_smp);
  D.smp_slot = (const int *)(ws + p->off_smp_slot);
  struct Up {
    uint64_t off;
    const void *src;
    size_t n;
  } ups[] = {
      {p->off_tf, p->tabf.data(), p->tabf.size() * sizeof(float)},
      {p->off_ti, p->tabi.data(), p->tabi.size() * sizeof(int)},
      {p->off_wr, p->wr.data(), p->wr.size() * sizeof(double)},
      {p->off_q, p->q_bins.data(), p->q_bins.size() * sizeof(double)},
      {p->off_oidx, p->obs_idx.data(), p->obs_idx.size() * sizeof(int)},
      {p->off_ot, p->obs_t.data(), p->obs_t.size() * sizeof(double)},
      {p->off_sknode, p->sk_node.data(), p->sk_node.size() * sizeof(long long)},
      {p->off_skcomp, p->sk_comp.data(), p->sk_comp.size() * sizeof(int)},
      {p->off_skptr, p->sk_ptr.data(), p->sk_ptr.size() * sizeof(int)},
      {p->off_seobs, p->se_obs.data(), p->se_obs.size() * sizeof(int)},
      {p->off_sew, p->se_w.data(), p->se_w.size() * sizeof(double)},
      {p->off_tiles, p->slow_tiles.data(), p->slow_tiles.size() * sizeof(int)},
      {p->off_ltiles, p->layer_tiles.data(), p->layer_tiles.size() * sizeof(int)},
      {p->off_tiles2, p->tiles2.data(), p->tiles2.size() * sizeof(int)},
      {p->off_smp_ptr, p->smp_ptr.data(), p->smp_ptr.size() * sizeof(int)},
      {p->off_smp_ent, p->smp_ent.data(), p->smp_ent.size() * sizeof(int)},
      {p->off_smp_slot, p->smp_slot.data(), p->smp_slot.size() * sizeof(int)},
  };
  for (const Up &u : ups) {
    if (!u.n) continue;
    hipError_t e = hipMemcpyAsync(ws + u.off, u.src, u.n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
}  // namespace chf

extern "C" {

chf_status chf_plan_bind_workspace(chf_plan *p, void *dev_ptr, uint64_t bytes, void *stream) {
  if (!p || !dev_ptr) return fail(CHF_EINVAL, "NULL argument");
  if (bytes < p->ws_bytes) return fail(CHF_ENOMEM, "workspace smaller than chf_plan_workspace_bytes");
  if ((uintptr_t)dev_ptr % 256) return fail(CHF_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  {
    hipError_t e = chf::bind_tables(p, (char *)dev_ptr, s);
    if (e != hipSuccess) return hip_fail(e, "upload of plan tables");
  }
  if (p->graph) {
    (void)hipGraphExecDestroy(p->graph);
    p->graph = nullptr;
  }
  if (!p->aux && p->fs.n_fast > 0 && p->fs.n_slow > 0) {
    // default-priority side stream and fork/join events for the boundary H sweep
    hipError_t e = hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->aux2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join2, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "side stream");
  }
  return chf_plan_reset(p, stream);
}

chf_status chf_plan_reset(chf_plan *p, void *stream) {
  if (!p) return fail(CHF_EINVAL, "NULL plan");
  if (!p->ws) return fail(CHF_ESTATE, "no workspace bound");
  hipError_t e = chf::launch_zero(*p, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "reset");
  chf::canonical_pointers(*p);
  p->parity = 0;
  p->n_done = 0;
  p->adj_next = -1;
  return CHF_OK;
}

chf_status chf_forward(chf_plan *p, void *stream, const double *q_bins_dev, double *w_dev, int32_t n_steps,
                       int32_t first_column, int32_t ld_steps) {
  if (!p) return fail(CHF_EINVAL, "NULL plan");
  if (!p->ws) return fail(CHF_ESTATE, "no workspace bound");
  p->adj_next = -1;
  if (n_steps < 0 || first_column < 0) return fail(CHF_EINVAL, "negative step count or column");
  if (p->dev.n_obs > 0 && w_dev && (ld_steps < first_column + n_steps))
    return fail(CHF_EINVAL, "ld_steps too small for first_column + n_steps");
  hipError_t e = chf::advance(*p, (hipStream_t)stream, q_bins_dev, w_dev, first_column, ld_steps, n_steps);
  if (e != hipSuccess) return hip_fail(e, "step launch");
  return CHF_OK;
}

chf_status chf_forward_timed(chf_plan *p, void *stream, const double *q_bins_dev, double *w_dev, int32_t n_steps,
                             int32_t first_column, int32_t ld_steps, double *fused_ms) {
  if (!p || !fused_ms) return fail(CHF_EINVAL, "NULL argument");
  if (!p->ws) return fail(CHF_ESTATE, "no workspace bound");
  p->adj_next = -1;
  if (n_steps < 0 || first_column < 0) return fail(CHF_EINVAL, "negative step count or column");
  if (p->dev.n_obs > 0 && w_dev && (ld_steps < first_column + n_steps))
    return fail(CHF_EINVAL, "ld_steps too small for first_column + n_steps");
  *fused_ms = 0.0;
  std::vector<hipEvent_t> ev(2 * (size_t)n_steps, nullptr);
  hipError_t e = hipSuccess;
  for (size_t t = 0; t < ev.size() && e == hipSuccess; t++) e = hipEventCreate(&ev[t]);
  hipStream_t s = (hipStream_t)stream;
  int launches = 0;
  // with two steps per pass only the two-step launches are timed (an odd range's single step
  // runs another kernel)
  if (e == hipSuccess)
    e = chf::advance(*p, s, q_bins_dev, w_dev, first_column, ld_steps, n_steps, ev.data(), &launches);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  double total = 0.0;
  const bool timed = p->fs2.on ? p->fs2.n_fast > 0 : p->fs.n_fast > 0;
  for (int t = 0; t < launches && e == hipSuccess && timed; t++) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, ev[2 * t], ev[2 * t + 1]);
    total += ms;
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return hip_fail(e, "timed forward");
  *fused_ms = total;
  return CHF_OK;
}

chf_status chf_forward_graph(chf_plan *p, void *stream, const double *q_bins_dev, double *w_dev) {
  if (!p) return fail(CHF_EINVAL, "NULL plan");
  if (!p->ws) return fail(CHF_ESTATE, "no workspace bound");
  p->adj_next = -1;
  hipStream_t s = (hipStream_t)stream;
  const int T = p->grid.n_steps;
  if (!p->graph || p->graph_w != w_dev || p->graph_q != q_bins_dev) {
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
    // the captured run starts from zero fields with the levels in their unexchanged order
    const chf::Dev keep = p->dev;
    const int keep_par = p->parity, keep_done = p->n_done;
    chf::canonical_pointers(*p);
    p->parity = 0;
    p->n_done = 0;
    hipError_t le = chf::launch_zero(*p, cs);
    if (le == hipSuccess) le = chf::advance(*p, cs, q_bins_dev, w_dev, 0, T, T);
    p->graph_swap = p->lev_swap;
    p->dev = keep;
    p->parity = keep_par;
    p->n_done = keep_done;
    p->lev_swap = p->pe_swap = 0;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (le != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(le, "captured launch");
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    e = hipGraphInstantiate(&p->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      p->graph = nullptr;
      return hip_fail(e, "graph instantiate");
    }
    p->graph_w = w_dev;
    p->graph_q = q_bins_dev;
  }
  hipError_t e = hipGraphLaunch(p->graph, s);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  chf::canonical_pointers(*p);
  if (p->graph_swap) chf::swap_levels(*p, p->dev);
  p->parity = T & 1;
  p->n_done = T;
  return CHF_OK;
}

chf_status chf_plan_sync(chf_plan *p, void *stream) {
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

chf_status chf_plan_get_field(chf_plan *p, void *stream, int32_t comp, float *out_dev) {
  if (!p || !out_dev || comp < 0 || comp > 5) return fail(CHF_EINVAL, "bad argument");
  if (!p->ws) return fail(CHF_ESTATE, "no workspace bound");
  hipError_t e = chf::launch_get_field(*p, p->parity, comp, out_dev, (hipStream_t)stream);
  return e == hipSuccess ? CHF_OK : hip_fail(e, "get field");
}

chf_status chf_plan_set_field(chf_plan *p, void *stream, int32_t comp, const float *in_dev) {
  if (!p || !in_dev || comp < 0 || comp > 5) return fail(CHF_EINVAL, "bad argument");
  if (!p->ws) return fail(CHF_ESTATE, "no workspace bound");
  hipError_t e = chf::launch_set_field(*p, p->parity, comp, in_dev, (hipStream_t)stream);
  return e == hipSuccess ? CHF_OK : hip_fail(e, "set field");
}

chf_status chf_plan_get_info(const chf_plan *p, chf_plan_info *info) {
  if (!p || !info) return fail(CHF_EINVAL, "NULL argument");
  info->kernel = p->fs.prefetch ? CHF_KERNEL_FUSED_PREFETCH : p->kernel;
  info->storage = p->storage;
  info->vx = p->fs.vx;
  info->rows_per_wave = p->fs.rows;
  info->waves_per_block = p->fs.waves;
  info->z_chunk = p->fs.zchunk;
  info->pitch = p->dev.pitch;
  info->n_blocks = p->fs.n_blocks;
  info->scale_e = p->scale_e;
  info->scale_h = p->scale_h;
  info->field_bytes = p->field_bytes;
  info->psi_bytes = p->psi_bytes;
  info->workspace_bytes = p->ws_bytes;
  // one read and one write of the six components, plus the psi read and write of the cells
  // inside each layer (two psi per component pair and derivative axis)
  const double cells = (double)p->grid.nx * p->grid.ny * p->grid.nz;
  double psi_rw = 0.0;
  if (p->bnd.npml > 0) {
    const double n2 = 2.0 * p->bnd.npml;
    const double frac = n2 / p->grid.nx + n2 / p->grid.ny + n2 / p->grid.nz;
    psi_rw = frac * 4 * 2 * 4.0;  // 4 psi per layer cell (2 E, 2 H), read + write, FP32
  }
  info->bytes_per_cell_update = 12.0 * p->elem_bytes + psi_rw;
  (void)cells;
  // fused interior sweep: rows and planes clear of y/z layers, so only the x-layer psi
  const uint64_t rows = (uint64_t)std::max(0, (p->fs.ty_hi - p->fs.ty_lo) * p->fs.waves);
  const uint64_t planes = (uint64_t)std::max(0, (p->fs.zc_hi - p->fs.zc_lo) * p->fs.zchunk);
  info->fused_cells = rows * planes * (uint64_t)p->grid.nx;
  const double one_step = 12.0 * p->elem_bytes + (p->bnd.npml > 0 ? (2.0 * p->bnd.npml / p->grid.nx) * 4 * 2 * 4.0 : 0.0);
  info->fused_bytes_per_cell = one_step;
  info->pass_bytes_per_cell = one_step;
  info->steps_per_launch = 1;
  info->waves_per_row = p->fs.xs;
  info->dynamic_scaling = p->dev.dyn;
  if (p->fs2.on) {
    const chf::Shape2 &f2 = p->fs2;
    info->kernel = CHF_KERNEL_FUSED2;
    info->steps_per_launch = 2;
    info->waves_per_row = f2.xs;
    info->vx = f2.vx;
    info->waves_per_block = f2.waves;
    info->z_chunk = f2.zchunk;
    const uint64_t r2 = (uint64_t)std::max(0, (f2.ty_hi - f2.ty_lo) * f2.waves);
    const uint64_t z2 = (uint64_t)std::max(0, (f2.zc_hi - f2.zc_lo) * f2.zchunk);
    info->fused_cells = r2 * z2 * (uint64_t)p->grid.nx;
    info->fused_bytes_per_cell = 2.0 * one_step;  // both steps at the one-step algorithmic bytes
    info->pass_bytes_per_cell = one_step;         // the pass reads and writes each value once
  }
  return CHF_OK;
}

chf_status chf_adjoint_begin(chf_plan *p, void *stream, double *dl_dq_dev) {
  if (!p || !dl_dq_dev) return fail(CHF_EINVAL, "NULL argument");
  if (!p->ws) return fail(CHF_ESTATE, "no workspace bound");
  if (p->bnd.kind == CHF_BC_MUR1) return fail(CHF_EUNSUPPORTED, "adjoint of the Mur boundary is not implemented");
  if (p->storage != CHF_FP32) return fail(CHF_EUNSUPPORTED, "adjoint needs FP32 field storage");
  hipStream_t s = (hipStream_t)stream;
  // the workspace now holds the adjoint state: zero fields and psi
  hipError_t e = chf::launch_zero(*p, s);
  if (e == hipSuccess) e = chf::launch_adjoint_clear(*p, s);
  if (e == hipSuccess) e = chf::launch_adjoint_init(*p, dl_dq_dev, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint start");
  p->parity = 0;
  p->n_done = 0;
  p->adj_next = p->grid.n_steps;
  return CHF_OK;
}

chf_status chf_adjoint_steps(chf_plan *p, void *stream, const double *dl_dw_dev, double *dl_dq_dev, int32_t t_lo,
                             int32_t t_hi) {
  if (!p || !dl_dq_dev || (p->dev.n_obs > 0 && !dl_dw_dev)) return fail(CHF_EINVAL, "NULL argument");
  if (!p->ws) return fail(CHF_ESTATE, "no workspace bound");
  if (t_lo < 0 || t_lo > t_hi || t_hi > p->grid.n_steps) return fail(CHF_EINVAL, "bad step range");
  if (p->adj_next < 0 || t_hi != p->adj_next)
    return fail(CHF_ESTATE, "adjoint steps must continue where the previous call stopped");
  hipError_t e = hipSuccess;
  for (int n = t_hi - 1; n >= t_lo && e == hipSuccess; n--) {
    e = chf::launch_adjoint_step(*p, p->dev, p->parity, n, dl_dw_dev, dl_dq_dev, (hipStream_t)stream);
    p->parity ^= 1;
  }
  if (e != hipSuccess) return hip_fail(e, "adjoint launch");
  p->adj_next = t_lo;
  return CHF_OK;
}

chf_status chf_adjoint_steps_eps(chf_plan *p, void *stream, const double *dl_dw_dev, double *dl_dq_dev,
                                 int32_t t_lo, int32_t t_hi, const float *e_levels_dev, double *dl_deps_dev) {
  if (!p || !dl_dq_dev || !e_levels_dev || !dl_deps_dev || (p->dev.n_obs > 0 && !dl_dw_dev))
    return fail(CHF_EINVAL, "NULL argument");
  if (!p->ws) return fail(CHF_ESTATE, "no workspace bound");
  if (t_lo < 0 || t_lo > t_hi || t_hi > p->grid.n_steps) return fail(CHF_EINVAL, "bad step range");
  if (p->adj_next < 0 || t_hi != p->adj_next)
    return fail(CHF_ESTATE, "adjoint steps must continue where the previous call stopped");
  const long long level = 3LL * p->grid.nx * p->grid.ny * p->grid.nz;
  const double eps = kEps0 * p->med.eps_r;
  const double loss = p->med.sigma * p->grid.dt / (2.0 * eps);
  const double coef = 1.0 / (p->med.eps_r * (1.0 + loss));
  hipError_t e = hipSuccess;
  for (int n = t_hi - 1; n >= t_lo && e == hipSuccess; n--) {
    const chf::EpsTerm term{e_levels_dev + (long long)(n - t_lo) * level,
                            e_levels_dev + (long long)(n + 1 - t_lo) * level, dl_deps_dev, coef};
    e = chf::launch_adjoint_step(*p, p->dev, p->parity, n, dl_dw_dev, dl_dq_dev, (hipStream_t)stream, nullptr, nullptr,
                                 &term);
    p->parity ^= 1;
  }
  if (e != hipSuccess) return hip_fail(e, "adjoint launch");
  p->adj_next = t_lo;
  return CHF_OK;
}

chf_status chf_adjoint_checkpointed(chf_plan *p, chf_plan *fwd, void *stream, const double *q_bins_dev,
                                    const double *dl_dw_dev, double *dl_dq_dev, int32_t every, void *snapshots_dev,
                                    uint64_t snapshots_bytes, float *e_levels_dev, double *dl_deps_dev) {
  if (!p || !fwd || !dl_dq_dev || !snapshots_dev || (p->dev.n_obs > 0 && !dl_dw_dev))
    return fail(CHF_EINVAL, "NULL argument");
  if (p == fwd) return fail(CHF_EINVAL, "the recomputation needs a second plan");
  if ((dl_deps_dev != nullptr) != (e_levels_dev != nullptr))
    return fail(CHF_EINVAL, "e_levels_dev and dl_deps_dev go together");
  if (!p->ws || !fwd->ws) return fail(CHF_ESTATE, "no workspace bound");
  const chf_grid &a = p->grid, &b = fwd->grid;
  if (a.nx != b.nx || a.ny != b.ny || a.nz != b.nz || a.n_steps != b.n_steps || p->storage != fwd->storage ||
      p->bnd.kind != fwd->bnd.kind || p->bnd.npml != fwd->bnd.npml)
    return fail(CHF_EINVAL, "the recomputing plan must have the plan's grid, steps, storage and boundary");
  const int T = a.n_steps;
  if (every < 1) return fail(CHF_EINVAL, "every must be >= 1");
  const int K = std::min(every, std::max(T, 1));
  const int n_seg = (T + K - 1) / K;
  const uint64_t sb = fwd->off_tf;
  if (snapshots_bytes < sb * (uint64_t)n_seg) return fail(CHF_ENOMEM, "snapshot buffer too small");
  char *snaps = (char *)snapshots_dev;
  const long long level = 3LL * a.nx * a.ny * a.nz;
  // forward run with a snapshot at the start of every segment
  chf_status st = chf_plan_reset(fwd, stream);
  int32_t step = 0;
  for (int g = 0; g < n_seg && st == CHF_OK; g++) {
    st = chf_plan_save_state(fwd, stream, snaps + sb * g, &step);
    if (st == CHF_OK) st = chf_forward(fwd, stream, q_bins_dev, nullptr, std::min(K, T - g * K), 0, 0);
  }
  if (st == CHF_OK) st = chf_adjoint_begin(p, stream, dl_dq_dev);
  // segments last to first: restore, recompute (keeping the E levels when the permittivity
  // gradient is asked for), then the segment's transposed steps
  for (int g = n_seg - 1; g >= 0 && st == CHF_OK; g--) {
    const int t0 = g * K, t1 = std::min((g + 1) * K, T);
    st = chf_plan_load_state(fwd, stream, snaps + sb * g, t0);
    if (st != CHF_OK) break;
    if (dl_deps_dev) {
      for (int m = 0; m <= t1 - t0 && st == CHF_OK; m++) {
        if (m) st = chf_forward(fwd, stream, q_bins_dev, nullptr, 1, 0, 0);
        for (int c = 0; c < 3 && st == CHF_OK; c++)
          st = chf_plan_get_field(fwd, stream, c, e_levels_dev + m * level + c * (level / 3));
      }
      if (st == CHF_OK) st = chf_adjoint_steps_eps(p, stream, dl_dw_dev, dl_dq_dev, t0, t1, e_levels_dev, dl_deps_dev);
    } else {
      st = chf_forward(fwd, stream, q_bins_dev, nullptr, t1 - t0, 0, 0);
      if (st == CHF_OK) st = chf_adjoint_steps(p, stream, dl_dw_dev, dl_dq_dev, t0, t1);
    }
  }
  return st;
}

chf_status chf_adjoint(chf_plan *p, void *stream, const double *dl_dw_dev, double *dl_dq_dev) {
  if (!p || !dl_dq_dev || (p->dev.n_obs > 0 && !dl_dw_dev)) return fail(CHF_EINVAL, "NULL argument");
  chf_status st = chf_adjoint_begin(p, stream, dl_dq_dev);
  if (st != CHF_OK) return st;
  return chf_adjoint_steps(p, stream, dl_dw_dev, dl_dq_dev, 0, p->grid.n_steps);
}

chf_status chf_adjoint_source_params(chf_plan *p, void *stream, const double *dl_dw_dev, const double *q_bins_dev,
                                     double *dl_dq_dev, double *dl_dtheta_dev) {
  if (!p || !dl_dq_dev || !dl_dtheta_dev || (p->dev.n_obs > 0 && !dl_dw_dev)) return fail(CHF_EINVAL, "NULL argument");
  if (!p->dev.src_on) return fail(CHF_EINVAL, "the plan has no source");
  chf_status st = chf_adjoint_begin(p, stream, dl_dq_dev);
  if (st != CHF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = chf::launch_adjoint_init(*p, dl_dtheta_dev, s, 2);
  for (int n = p->grid.n_steps - 1; n >= 0 && e == hipSuccess; n--) {
    e = chf::launch_adjoint_step(*p, p->dev, p->parity, n, dl_dw_dev, dl_dq_dev, s, q_bins_dev, dl_dtheta_dev);
    p->parity ^= 1;
  }
  if (e != hipSuccess) return hip_fail(e, "adjoint launch");
  p->adj_next = 0;
  return CHF_OK;
}

chf_status chf_plan_state_bytes(const chf_plan *p, uint64_t *bytes) {
  if (!p || !bytes) return fail(CHF_EINVAL, "NULL argument");
  *bytes = p->off_tf;  // fields and psi lead the workspace
  return CHF_OK;
}

}  // extern "C"

namespace {
// A snapshot holds the state in the unexchanged order: level l of the fields and psi_H, and the
// current psi_E, at their own offsets.  Pieces (snapshot offset, workspace offset, bytes) for
// the plan's present exchange state; a single piece when nothing is exchanged.
struct Piece {
  uint64_t snap, ws, n;
};
std::vector<Piece> state_pieces(const chf_plan &p) {
  if (!p.lev_swap && !p.pe_swap) return {{0, 0, p.off_tf}};
  std::vector<Piece> v;
  const uint64_t lev = p.off_e[1][0] - p.off_e[0][0];  // one level: six field arrays
  for (int l = 0; l < 2; l++) v.push_back({p.off_e[l][0], p.off_e[l ^ p.lev_swap][0], lev});
  for (int u = 0; u < 3; u++) {
    const uint64_t len = align256(p.psi_len[u] * 4);
    for (int t = 0; t < 2; t++) {
      for (int l = 0; l < 2; l++) v.push_back({p.off_psi_h[l][u][t], p.off_psi_h[l ^ p.lev_swap][u][t], len});
      const uint64_t a = p.off_psi_e[u][t], b = p.off_psi_e2[u][t];
      v.push_back({a, p.pe_swap ? b : a, len});
      if (p.fs2.on) v.push_back({b, p.pe_swap ? a : b, len});
    }
  }
  // dynamic scaling words: each level's (exponent, maxima slot) follows its level; the maxima
  // slots stay
  for (int l = 0; l < 2; l++) v.push_back({p.off_dyn + 16 * l, p.off_dyn + 16 * (l ^ p.lev_swap), 16});
  v.push_back({p.off_dyn + 32, p.off_dyn + 32, 224});
  return v;
}
}  // namespace

extern "C" {

chf_status chf_plan_save_state(chf_plan *p, void *stream, void *dst_dev, int32_t *step) {
  if (!p || !dst_dev || !step) return fail(CHF_EINVAL, "NULL argument");
  if (!p->ws) return fail(CHF_ESTATE, "no workspace bound");
  for (const Piece &c : state_pieces(*p)) {
    hipError_t e = hipMemcpyAsync((char *)dst_dev + c.snap, p->ws + c.ws, c.n, hipMemcpyDeviceToDevice,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "save state");
  }
  *step = p->n_done;
  return CHF_OK;
}

chf_status chf_plan_load_state(chf_plan *p, void *stream, const void *src_dev, int32_t step) {
  if (!p || !src_dev) return fail(CHF_EINVAL, "NULL argument");
  if (!p->ws) return fail(CHF_ESTATE, "no workspace bound");
  if (step < 0) return fail(CHF_EINVAL, "negative step");
  hipError_t e = hipMemcpyAsync(p->ws, src_dev, p->off_tf, hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "load state");
  chf::canonical_pointers(*p);
  p->n_done = step;
  p->parity = step & 1;
  p->adj_next = -1;
  return CHF_OK;
}

chf_status chf_batch_create(int32_t n, chf_plan *const *plans, chf_batch **out) {
  if (!out || n <= 0 || !plans) return fail(CHF_EINVAL, "bad batch");
  *out = nullptr;
  chf_batch *b = new (std::nothrow) chf_batch();
  if (!b) return fail(CHF_ENOMEM, "host allocation failed");
  for (int i = 0; i < n; i++) {
    chf_plan *p = plans[i];
    if (!p || !p->ws) {
      delete b;
      return fail(p ? CHF_ESTATE : CHF_EINVAL, "every plan must exist and have its workspace bound");
    }
    if (p->dev.dyn) {
      delete b;
      return fail(CHF_EUNSUPPORTED, "a batch takes plans with static storage scales");
    }
    if (i == 0) {
      b->storage = p->storage;
      b->waves = p->fs.waves;
      b->n_steps = p->grid.n_steps;
      b->prefetch = p->fs.prefetch;
    } else if (p->storage != b->storage || p->fs.waves != b->waves || p->grid.n_steps != b->n_steps ||
               p->fs.prefetch != b->prefetch) {
      delete b;
      return fail(CHF_EINVAL, "plans of a batch share storage, kernel, waves_per_block and n_steps");
    }
    b->plans.push_back(p);
    b->vx = std::max(b->vx, p->fs.vx);
    b->zchunks.push_back(p->fs.zchunk);
    b->any_mur = b->any_mur || p->bnd.kind == CHF_BC_MUR1;
    if (p->dev.src_on) b->max_patch = std::max(b->max_patch, p->dev.src_ni * p->dev.src_nj);
    const chf::FusedShape &fs = p->fs;
    const int fw = fs.ty_hi - fs.ty_lo;
    for (int t = 0; t < fs.n_fast; t++) {
      b->fast_tab.push_back(i);
      b->fast_tab.push_back(fs.ty_lo + t % fw);
      b->fast_tab.push_back(fs.zc_lo + t / fw);
    }
    for (int t = 0; t < fs.n_slow; t++) {
      std::vector<int> &g = b->gen_tab[t < fs.n_slow_y ? 0 : 1];
      g.push_back(i);
      g.push_back(p->slow_tiles[2 * t]);
      g.push_back(p->slow_tiles[2 * t + 1]);
    }
    const int nxb = (p->grid.nx + 63) / 64;
    for (int t = 0; t < fs.n_slow; t++)
      for (int xb = 0; xb < nxb; xb++) {
        b->slow_tab.push_back(i);
        b->slow_tab.push_back(p->slow_tiles[2 * t]);
        b->slow_tab.push_back(p->slow_tiles[2 * t + 1]);
        b->slow_tab.push_back(xb);
      }
    for (int o = 0; o < p->dev.n_obs; o++) {
      b->obs_tab.push_back(i);
      b->obs_tab.push_back(o);
    }
    chf::Dev d = p->dev;
    if (!p->ex.nan_watch) d.nan_flag = nullptr;
    b->devs.push_back(d);
  }
  b->total_obs = (int)(b->obs_tab.size() / 2);
  b->wptr.assign(n, nullptr);
  // boundary tiles in the general fused sweep where it fits (as for single plans)
  b->gen = b->vx <= chf::kMaxGeneralVX && b->waves <= chf::kMaxGeneralW;
  uint64_t off = 0;
  b->off_devs = off;
  off += align256(b->devs.size() * sizeof(chf::Dev));
  b->off_z = off;
  off += align256(b->zchunks.size() * sizeof(int));
  b->off_fast = off;
  off += align256(std::max<size_t>(b->fast_tab.size(), 1) * sizeof(int));
  b->off_slow = off;
  off += align256(std::max<size_t>(b->slow_tab.size(), 1) * sizeof(int));
  for (int c = 0; c < 2; c++) {
    b->off_gen[c] = off;
    off += align256(std::max<size_t>(b->gen_tab[c].size(), 1) * sizeof(int));
  }
  // the persistent launch's work list: interior tiles, then boundary tiles of both classes
  b->all_tab = b->fast_tab;
  b->all_tab.insert(b->all_tab.end(), b->gen_tab[0].begin(), b->gen_tab[0].end());
  b->all_tab.insert(b->all_tab.end(), b->gen_tab[1].begin(), b->gen_tab[1].end());
  b->off_all = off;
  off += align256(std::max<size_t>(b->all_tab.size(), 1) * sizeof(int));
  b->off_obs = off;
  off += align256(std::max<size_t>(b->obs_tab.size(), 1) * sizeof(int));
  b->off_wptr = off;
  off += align256((size_t)n * sizeof(double *));
  b->ws_bytes = off;
  *out = b;
  return CHF_OK;
}

chf_status chf_batch_workspace_bytes(const chf_batch *b, uint64_t *bytes) {
  if (!b || !bytes) return fail(CHF_EINVAL, "NULL argument");
  *bytes = b->ws_bytes;
  return CHF_OK;
}

chf_status chf_batch_bind_workspace(chf_batch *b, void *dev_ptr, uint64_t bytes, void *stream) {
  if (!b || !dev_ptr) return fail(CHF_EINVAL, "NULL argument");
  if (bytes < b->ws_bytes) return fail(CHF_ENOMEM, "workspace smaller than chf_batch_workspace_bytes");
  if ((uintptr_t)dev_ptr % 256) return fail(CHF_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  b->ws = (char *)dev_ptr;
  struct Up {
    uint64_t off;
    const void *src;
    size_t n;
  } ups[] = {
      {b->off_devs, b->devs.data(), b->devs.size() * sizeof(chf::Dev)},
      {b->off_z, b->zchunks.data(), b->zchunks.size() * sizeof(int)},
      {b->off_fast, b->fast_tab.data(), b->fast_tab.size() * sizeof(int)},
      {b->off_slow, b->slow_tab.data(), b->slow_tab.size() * sizeof(int)},
      {b->off_gen[0], b->gen_tab[0].data(), b->gen_tab[0].size() * sizeof(int)},
      {b->off_gen[1], b->gen_tab[1].data(), b->gen_tab[1].size() * sizeof(int)},
      {b->off_obs, b->obs_tab.data(), b->obs_tab.size() * sizeof(int)},
      {b->off_all, b->all_tab.data(), b->all_tab.size() * sizeof(int)},
  };
  for (const Up &u : ups) {
    if (!u.n) continue;
    hipError_t e = hipMemcpyAsync(b->ws + u.off, u.src, u.n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "upload of batch tables");
  }
  if (!b->aux && !b->fast_tab.empty() && !b->slow_tab.empty()) {
    hipError_t e = hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->aux2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join2, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "side stream");
  }
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  return CHF_OK;
}

chf_status chf_batch_run(chf_batch *b, void *stream, double *const *w) {
  if (!b || !w) return fail(CHF_EINVAL, "NULL argument");
  if (!b->ws) return fail(CHF_ESTATE, "no batch workspace bound");
  hipStream_t s = (hipStream_t)stream;
  bool same = b->graph != nullptr;
  for (size_t i = 0; i < b->plans.size(); i++) same = same && b->wptr[i] == w[i];
  if (!same) {
    if (b->graph) {
      (void)hipGraphExecDestroy(b->graph);
      b->graph = nullptr;
    }
    for (size_t i = 0; i < b->plans.size(); i++) b->wptr[i] = w[i];
    hipError_t e = hipMemcpyAsync(b->ws + b->off_wptr, b->wptr.data(), b->wptr.size() * sizeof(double *),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "upload of waveform pointers");
    hipStream_t cs;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return hip_fail(e, "begin capture");
    }
    hipError_t le = hipSuccess;
    for (chf_plan *p : b->plans)
      if (le == hipSuccess) le = chf::launch_zero(*p, cs);
    int par = 0;
    for (int t = 0; t < b->n_steps && le == hipSuccess; t++) {
      le = chf::launch_batch_step(*b, par, t, cs);
      par ^= 1;
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (le != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(le, "captured batch launch");
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b->graph = nullptr;
      return hip_fail(e, "graph instantiate");
    }
  }
  hipError_t e = hipGraphLaunch(b->graph, s);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  for (chf_plan *p : b->plans) {
    p->parity = b->n_steps & 1;
    p->n_done = b->n_steps;
  }
  return CHF_OK;
}

chf_status chf_batch_run_persistent(chf_batch *b, void *stream, double *const *w) {
  if (!b || !w) return fail(CHF_EINVAL, "NULL argument");
  if (!b->ws) return fail(CHF_ESTATE, "no batch workspace bound");
  if (b->storage != CHF_FP32 || !b->gen || b->any_mur)
    return fail(CHF_EUNSUPPORTED, "the persistent batch launch takes FP32 members with PEC or CPML walls whose "
                                  "boundary tiles fit the general fused sweep (rows of at most 256 nodes, at most 11 "
                                  "rows per tile)");
  hipStream_t s = (hipStream_t)stream;
  bool same = true;
  for (size_t i = 0; i < b->plans.size(); i++) same = same && b->wptr[i] == w[i];
  if (!same) {
    if (b->graph) {  // the captured per-phase graph holds the old pointers
      (void)hipGraphExecDestroy(b->graph);
      b->graph = nullptr;
    }
    for (size_t i = 0; i < b->plans.size(); i++) b->wptr[i] = w[i];
    hipError_t e = hipMemcpyAsync(b->ws + b->off_wptr, b->wptr.data(), b->wptr.size() * sizeof(double *),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "upload of waveform pointers");
  }
  hipError_t e = hipSuccess;
  for (chf_plan *p : b->plans)
    if (e == hipSuccess) e = chf::launch_zero(*p, s);
  if (e == hipSuccess)
    e = chf::launch_batch_persistent(*b, (const int *)(b->ws + b->off_all), (int)(b->all_tab.size() / 3), s);
  if (e != hipSuccess) return hip_fail(e, "persistent batch launch");
  for (chf_plan *p : b->plans) {
    p->parity = b->n_steps & 1;
    p->n_done = b->n_steps;
  }
  return CHF_OK;
}

void chf_batch_destroy(chf_batch *b) {
  if (!b) return;
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_join) (void)hipEventDestroy(b->ev_join);
  if (b->aux) (void)hipStreamDestroy(b->aux);
  if (b->ev_join2) (void)hipEventDestroy(b->ev_join2);
  if (b->aux2) (void)hipStreamDestroy(b->aux2);
  delete b;
}

}  // extern "C"
