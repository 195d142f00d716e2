// md_fm.hip -- force matching: loss L = sum_c sum_i |F_i - Fref_i|^2 over static
// configurations and its adjoint with respect to the per-segment spline
// coefficients of phi, rho and F.
//
// Forces follow Eq. (EAMforce) of the paper (arXiv 2405.07898, Sec. II-A),
// with rho, F and phi polynomial splines of any coefficients, as the paper allows.  The
// gradient is reverse-mode differentiation of the density and force passes:
//   g_i = 2 (F_i - Fref_i),  u_ij = (x_j - x_i)/r,  w_ij = g_i . u_ij
//   lambda_i = sum_j (g_i - g_j) . u_ij rho'(r_ij),  mu_i = lambda_i F''(rho_i)
//   dL/dphi_k,m = sum_(i,j) w_ij d phi'(r_ij)/dc_m
//   dL/drho_k,m = sum_(i,j) w_ij (F'_i + F'_j) d rho'(r_ij)/dc_m + mu_i d rho(r_ij)/dc_m
//   dL/dF_k,m   = sum_i lambda_i d F'(rho_i)/dc_m
// with d f/dc_m = t^m and d f'/dc_m = m t^(m-1) / dx on the segment holding
// the argument.  Coefficient sums are accumulated as 64-bit fixed-point
// integers: integer addition is associative, so the gradient is bitwise
// reproducible without ordering the float adds.  The fixed-point scale is a
// power of two chosen on the device from a per-atom bound on the terms, so
// that (number of pair terms) x (largest term) stays below 2^61.
//
// Binning and the (static) neighbour lists come from an internal MD context
// with zero skin, so every listed pair has r^2 < r_cut^2.
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "md.h"
#include "md_internal.h"
#include "md_device.h"

#pragma clang fp contract(off)

using namespace mdk;

namespace {

constexpr int kFmBlocks = 2048;  // blocks of the coefficient pass (8 waves per CU)
constexpr int kFmSplit = 16;    // first-stage groups of block histograms in the reduction
constexpr size_t kFmLds = 65536;  // LDS of the coefficient pass's histogram

struct FmSpline {
  const double* coef;  // device [(n-1)][4]
  double x0, inv_dx;
  int32_t n;
  int32_t pad;
};

struct FmArgs {
  Geometry g;
  State s;
  FmSpline phi, rho, emb;
  double rc2;
  double* rho_i;     // [N]
  double* fp;        // [N]
  double* fpp;       // [N]
  double4* frc;      // [N]
  double4* gvec;     // [N] 2 (F - Fref)
  double4* fref;     // [N] internal order
  double* lam;       // [N]
  double* mu;        // [N]
  double* partial;   // [tiles]
  double* loss;      // [1]
  unsigned long long* hist;  // [kFmBlocks][nbins]
  unsigned long long* part;  // [kFmSplit][nbins] first-stage sums of hist
  double* bound;     // [tiles] largest gradient term per tile
  double* scale;     // [2]: fixed-point scale and its inverse
  int32_t* flag;     // overflow / non-finite
  int32_t nb_phi, nb_rho, nb_emb;  // bins per function = 4 (n - 1)
};

__device__ __forceinline__ void seg(const FmSpline& sp, double v, int& k, double& t) {
  const double x = (v - sp.x0) * sp.inv_dx;
  const int last = sp.n - 2;
  k = (x >= (double)last) ? last : ((x > 0.0) ? (int)x : 0);
  t = x - (double)k;
}

// Past the last knot (t > 1) a table continues along its end tangent.
__device__ __forceinline__ double sp_f(const FmSpline& sp, double v) {
  int k;
  double t;
  seg(sp, v, k, t);
  const double* c = sp.coef + 4 * k;
  if (t > 1.0) return (c[0] + c[1] + c[2] + c[3]) + (c[1] + 2.0 * c[2] + 3.0 * c[3]) * (t - 1.0);
  return c[0] + t * (c[1] + t * (c[2] + t * c[3]));
}

__device__ __forceinline__ double sp_df(const FmSpline& sp, double v) {
  int k;
  double t;
  seg(sp, v, k, t);
  t = fmin(t, 1.0);
  const double* c = sp.coef + 4 * k;
  return (c[1] + t * (2.0 * c[2] + t * (3.0 * c[3]))) * sp.inv_dx;
}

__device__ __forceinline__ double sp_ddf(const FmSpline& sp, double v) {
  int k;
  double t;
  seg(sp, v, k, t);
  if (t > 1.0) return 0.0;
  const double* c = sp.coef + 4 * k;
  return (2.0 * c[2] + 6.0 * c[3] * t) * sp.inv_dx * sp.inv_dx;
}

__device__ __forceinline__ void sep(const RepDev& rp, uint32_t e, const double4& pi,
                                    const double4& pj, double& dx, double& dy, double& dz) {
  dx = pj.x - pi.x;
  dy = pj.y - pi.y;
  dz = pj.z - pi.z;
  const uint32_t code = e >> kIndexBits;
  dx += (double)((int)(code & 3u) - 1) * rp.box[0];
  dy += (double)((int)((code >> 2) & 3u) - 1) * rp.box[1];
  dz += (double)((int)(code >> 4) - 1) * rp.box[2];
}

// The pair loops below take kFmBatch list entries at a time: all their list
// loads, then all their neighbour loads, then the arithmetic in list order (so
// every sum keeps its order).  Entries past the list end read the atom itself
// and are skipped.
constexpr int kFmBatch = 4;

// rho_i, F'(rho_i), F''(rho_i)
__global__ __launch_bounds__(64) void k_fm_density(FmArgs a) {
  const AtomTile tl = a.g.atiles[blockIdx.x];
  if ((int)threadIdx.x >= tl.count) return;
  const RepDev& rp = a.g.reps[tl.rep];
  const int64_t i = tl.begin + threadIdx.x;
  const double4 pi = a.s.pos[i];
  const int m = min(a.s.cnt[i], a.g.nbr_cap);
  double acc = 0.0;
  for (int k0 = 0; k0 < m; k0 += kFmBatch) {
    uint32_t e[kFmBatch];
    double4 pj[kFmBatch];
#pragma unroll
    for (int u = 0; u < kFmBatch; ++u)
      e[u] = (k0 + u < m) ? a.s.nbr[(int64_t)(k0 + u) * a.g.n + i] : (uint32_t)i;
#pragma unroll
    for (int u = 0; u < kFmBatch; ++u) pj[u] = a.s.pos[e[u] & kIndexMask];
#pragma unroll
    for (int u = 0; u < kFmBatch; ++u) {
      if (k0 + u >= m) continue;
      double dx, dy, dz;
      sep(rp, e[u], pi, pj[u], dx, dy, dz);
      const double r2 = (dx * dx + dy * dy) + dz * dz;
      if (r2 < a.rc2) acc += sp_f(a.rho, r2 * rsq64(r2));
    }
  }
  a.rho_i[i] = acc;
  a.fp[i] = sp_df(a.emb, acc);
  a.fpp[i] = sp_ddf(a.emb, acc);
}

// F_i, g_i = 2 (F_i - Fref_i) and the tile's share of the loss (fixed tree).
__global__ __launch_bounds__(64) void k_fm_force(FmArgs a) {
  __shared__ double s_l[64];
  const AtomTile tl = a.g.atiles[blockIdx.x];
  double l = 0.0;
  if ((int)threadIdx.x < tl.count) {
    const RepDev& rp = a.g.reps[tl.rep];
    const int64_t i = tl.begin + threadIdx.x;
    const double4 pi = a.s.pos[i];
    const int m = min(a.s.cnt[i], a.g.nbr_cap);
    double fx = 0.0, fy = 0.0, fz = 0.0;
    const double fpi = a.fp[i];
    for (int k0 = 0; k0 < m; k0 += kFmBatch) {
      uint32_t e[kFmBatch];
      double4 pj[kFmBatch];
      double fpj[kFmBatch];
#pragma unroll
      for (int u = 0; u < kFmBatch; ++u)
        e[u] = (k0 + u < m) ? a.s.nbr[(int64_t)(k0 + u) * a.g.n + i] : (uint32_t)i;
#pragma unroll
      for (int u = 0; u < kFmBatch; ++u) {
        pj[u] = a.s.pos[e[u] & kIndexMask];
        fpj[u] = a.fp[e[u] & kIndexMask];
      }
#pragma unroll
      for (int u = 0; u < kFmBatch; ++u) {
        if (k0 + u >= m) continue;
        double dx, dy, dz;
        sep(rp, e[u], pi, pj[u], dx, dy, dz);
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        if (r2 < a.rc2) {
          // r^-1 as in the MD passes: no division, no square root
          const double rinv = rsq64(r2);
          const double r = r2 * rinv;
          const double sc = (fpi + fpj[u]) * sp_df(a.rho, r) + sp_df(a.phi, r);
          fx += sc * dx * rinv;
          fy += sc * dy * rinv;
          fz += sc * dz * rinv;
        }
      }
    }
    const double4 fr = a.fref[i];
    const double ex = fx - fr.x, ey = fy - fr.y, ez = fz - fr.z;
    l = (ex * ex + ey * ey) + ez * ez;
    a.frc[i] = make_double4(fx, fy, fz, 0.0);
    a.gvec[i] = make_double4(2.0 * ex, 2.0 * ey, 2.0 * ez, 0.0);
    if (!isfinite(l)) atomicOr(a.flag, 1);
  }
  s_l[threadIdx.x] = l;
  __syncthreads();
  for (int o = 32; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s_l[threadIdx.x] += s_l[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partial[blockIdx.x] = s_l[0];
}

__global__ __launch_bounds__(256) void k_fm_loss_reduce(FmArgs a, double* __restrict__ out) {
  __shared__ double s_l[256];
  double l = 0.0;
  for (int b = threadIdx.x; b < a.g.n_atiles; b += 256) l += a.partial[b];
  s_l[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s_l[threadIdx.x] += s_l[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *a.loss = s_l[0];
    if (out) *out = s_l[0];
  }
}

// lambda_i = sum_j (g_i - g_j) . u_ij rho'(r_ij),  mu_i = lambda_i F''(rho_i),
// plus a bound on the magnitude of every coefficient-gradient term of atom i
// (max per tile, fixed tree).
__global__ __launch_bounds__(64) void k_fm_lambda(FmArgs a) {
  __shared__ double s_b[64];
  const AtomTile tl = a.g.atiles[blockIdx.x];
  double bnd = 0.0;
  if ((int)threadIdx.x < tl.count) {
    const RepDev& rp = a.g.reps[tl.rep];
    const int64_t i = tl.begin + threadIdx.x;
    const double4 pi = a.s.pos[i];
    const double4 gi = a.gvec[i];
    const int m = min(a.s.cnt[i], a.g.nbr_cap);
    double acc = 0.0, fpmax = 0.0;
    for (int k0 = 0; k0 < m; k0 += kFmBatch) {
      uint32_t e[kFmBatch];
      double4 pj[kFmBatch], gj[kFmBatch];
      double fpj[kFmBatch];
#pragma unroll
      for (int u = 0; u < kFmBatch; ++u)
        e[u] = (k0 + u < m) ? a.s.nbr[(int64_t)(k0 + u) * a.g.n + i] : (uint32_t)i;
#pragma unroll
      for (int u = 0; u < kFmBatch; ++u) {
        const uint32_t j = e[u] & kIndexMask;
        pj[u] = a.s.pos[j];
        gj[u] = a.gvec[j];
        fpj[u] = a.fp[j];
      }
#pragma unroll
      for (int u = 0; u < kFmBatch; ++u) {
        if (k0 + u >= m) continue;
        double dx, dy, dz;
        sep(rp, e[u], pi, pj[u], dx, dy, dz);
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        if (r2 < a.rc2) {
          const double rinv = rsq64(r2);
          const double r = r2 * rinv;
          const double sij =
              ((gi.x - gj[u].x) * dx + (gi.y - gj[u].y) * dy + (gi.z - gj[u].z) * dz) * rinv;
          acc += sij * sp_df(a.rho, r);
          fpmax = fmax(fpmax, fabs(fpj[u]));
        }
      }
    }
    const double mu = acc * a.fpp[i];
    a.lam[i] = acc;
    a.mu[i] = mu;
    // |w| <= |g_i|; factors m t^(m-1) <= 3 (t <= 1, also past the F table,
    // where F continues along its end tangent)
    const double gn = sqrt((gi.x * gi.x + gi.y * gi.y) + gi.z * gi.z);
    const double a_pr = 3.0 * fmax(a.phi.inv_dx, a.rho.inv_dx);
    bnd = fmax(gn * a_pr * (1.0 + fabs(a.fp[i]) + fpmax) + fabs(mu),
               fabs(acc) * 3.0 * a.emb.inv_dx);
    if (!isfinite(bnd)) bnd = HUGE_VAL;
  }
  s_b[threadIdx.x] = bnd;
  __syncthreads();
  for (int o = 32; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s_b[threadIdx.x] = fmax(s_b[threadIdx.x], s_b[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) a.bound[blockIdx.x] = s_b[0];
}

// Fixed-point scale 2^e with (total list entries) x (largest term) x 2^e < 2^61.
__global__ __launch_bounds__(256) void k_fm_scale(FmArgs a, double n_terms) {
  __shared__ double s_b[256];
  double b = 0.0;
  for (int k = threadIdx.x; k < a.g.n_atiles; k += 256) b = fmax(b, a.bound[k]);
  s_b[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s_b[threadIdx.x] = fmax(s_b[threadIdx.x], s_b[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double tot = fmax(s_b[0], 1e-300) * fmax(n_terms, 1.0);
    if (!isfinite(tot)) {
      atomicOr(a.flag, 2);
      a.scale[0] = 0.0;
      a.scale[1] = 0.0;
      return;
    }
    int e = 61 - (int)ceil(log2(tot));
    e = max(-60, min(e, 60));
    a.scale[0] = ldexp(1.0, e);
    a.scale[1] = ldexp(1.0, -e);
  }
}

__device__ __forceinline__ void fix_add(unsigned long long* h, int bin, double v, double scale,
                                        int32_t* flag) {
  const double q = v * scale;
  if (!(fabs(q) < 4611686018427387904.0)) {  // 2^62: outside the bound, or not finite
    atomicOr(flag, 2);
    return;
  }
  atomicAdd(h + bin, (unsigned long long)(long long)llrint(q));
}

// Coefficient gradients into a per-block fixed-point histogram in LDS, then
// stored per block (phi bins, then rho bins, then F bins).
__global__ __launch_bounds__(64) void k_fm_coef(FmArgs a) {
  extern __shared__ unsigned long long h[];
  const int nb = a.nb_phi + a.nb_rho + a.nb_emb;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) h[b] = 0ull;
  __syncthreads();
  unsigned long long* hp = h;
  unsigned long long* hr = h + a.nb_phi;
  unsigned long long* he = h + a.nb_phi + a.nb_rho;
  const double S = a.scale[0];
  for (int tb = blockIdx.x; tb < a.g.n_atiles; tb += gridDim.x) {
    const AtomTile tl = a.g.atiles[tb];
    if ((int)threadIdx.x >= tl.count) continue;
    const RepDev& rp = a.g.reps[tl.rep];
    const int64_t i = tl.begin + threadIdx.x;
    const double4 pi = a.s.pos[i];
    const double4 gi = a.gvec[i];
    const double fpi = a.fp[i], mui = a.mu[i];
    const int m = min(a.s.cnt[i], a.g.nbr_cap);
    for (int k0 = 0; k0 < m; k0 += kFmBatch) {
      uint32_t e[kFmBatch];
      double4 pj[kFmBatch];
      double fpj[kFmBatch];
#pragma unroll
      for (int u = 0; u < kFmBatch; ++u)
        e[u] = (k0 + u < m) ? a.s.nbr[(int64_t)(k0 + u) * a.g.n + i] : (uint32_t)i;
#pragma unroll
      for (int u = 0; u < kFmBatch; ++u) {
        pj[u] = a.s.pos[e[u] & kIndexMask];
        fpj[u] = a.fp[e[u] & kIndexMask];
      }
#pragma unroll
      for (int u = 0; u < kFmBatch; ++u) {
        if (k0 + u >= m) break;
        double dx, dy, dz;
        sep(rp, e[u], pi, pj[u], dx, dy, dz);
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        if (!(r2 < a.rc2)) continue;
        const double rinv = rsq64(r2);
        const double r = r2 * rinv;
        const double w = (gi.x * dx + gi.y * dy + gi.z * dz) * rinv;
        int kp;
        double tp;
        seg(a.phi, r, kp, tp);
        const double ap = a.phi.inv_dx;
        fix_add(hp, 4 * kp + 1, w * ap, S, a.flag);
        fix_add(hp, 4 * kp + 2, w * 2.0 * tp * ap, S, a.flag);
        fix_add(hp, 4 * kp + 3, w * 3.0 * tp * tp * ap, S, a.flag);
        int kr;
        double tr;
        seg(a.rho, r, kr, tr);
        const double ar = a.rho.inv_dx;
        const double wf = w * (fpi + fpj[u]);
        fix_add(hr, 4 * kr + 0, mui, S, a.flag);
        fix_add(hr, 4 * kr + 1, wf * ar + mui * tr, S, a.flag);
        fix_add(hr, 4 * kr + 2, wf * 2.0 * tr * ar + mui * tr * tr, S, a.flag);
        fix_add(hr, 4 * kr + 3, wf * 3.0 * tr * tr * ar + mui * tr * tr * tr, S, a.flag);
      }
    }
    int ke;
    double te;
    seg(a.emb, a.rho_i[i], ke, te);
    te = fmin(te, 1.0);  // end tangent past the last knot
    const double li = a.lam[i], ae = a.emb.inv_dx;
    fix_add(he, 4 * ke + 1, li * ae, S, a.flag);
    fix_add(he, 4 * ke + 2, li * 2.0 * te * ae, S, a.flag);
    fix_add(he, 4 * ke + 3, li * 3.0 * te * te * ae, S, a.flag);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += blockDim.x) a.hist[(int64_t)blockIdx.x * nb + b] = h[b];
}

// Sum of the kFmBlocks block histograms in two stages (integer sums: any
// order gives the same bits).  Stage 1: workgroup (x, y) sums, for 64
// consecutive bins, the histograms of blocks y, y + kFmSplit, ... with its
// four rows of 64 lanes taking every fourth of them (coalesced over the bins);
// stage 2 adds the kFmSplit partial sums of each bin.
__global__ __launch_bounds__(256) void k_fm_coef_reduce1(FmArgs a, int nblocks) {
  __shared__ unsigned long long s_acc[4][64];
  const int nb = a.nb_phi + a.nb_rho + a.nb_emb;
  const int lane = (int)threadIdx.x & 63, row = (int)threadIdx.x >> 6;
  const int b = blockIdx.x * 64 + lane;
  unsigned long long acc = 0ull;
  if (b < nb)
    for (int k = (int)blockIdx.y + kFmSplit * row; k < nblocks; k += 4 * kFmSplit)
      acc += a.hist[(int64_t)k * nb + b];
  s_acc[row][lane] = acc;
  __syncthreads();
  if (row == 0 && b < nb)
    a.part[(int64_t)blockIdx.y * nb + b] = ((s_acc[0][lane] + s_acc[1][lane]) + s_acc[2][lane]) +
                                           s_acc[3][lane];
}

__global__ __launch_bounds__(256) void k_fm_coef_reduce(FmArgs a, double seed,
                                                        const double* __restrict__ seed_dev,
                                                        double* gp, double* gr, double* ge) {
  const int nb = a.nb_phi + a.nb_rho + a.nb_emb;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  if (seed_dev) seed = *seed_dev;
  unsigned long long acc = 0ull;
  for (int k = 0; k < kFmSplit; ++k) acc += a.part[(int64_t)k * nb + b];
  const double v = seed * ((double)(long long)acc * a.scale[1]);
  if (b < a.nb_phi) gp[b] = v;
  else if (b < a.nb_phi + a.nb_rho) gr[b - a.nb_phi] = v;
  else ge[b - a.nb_phi - a.nb_rho] = v;
}

__global__ __launch_bounds__(64) void k_fm_import_ref(FmArgs a, const double* __restrict__ fref) {
  const AtomTile tl = a.g.atiles[blockIdx.x];
  if ((int)threadIdx.x >= tl.count) return;
  const int64_t i = tl.begin + threadIdx.x;
  const int64_t o = a.s.id[i];
  a.fref[i] = make_double4(fref[3 * o], fref[3 * o + 1], fref[3 * o + 2], 0.0);
}

__global__ __launch_bounds__(64) void k_fm_export_f(FmArgs a, double* __restrict__ f) {
  const AtomTile tl = a.g.atiles[blockIdx.x];
  if ((int)threadIdx.x >= tl.count) return;
  const int64_t i = tl.begin + threadIdx.x;
  const int64_t o = a.s.id[i];
  const double4 v = a.frc[i];
  f[3 * o] = v.x;
  f[3 * o + 1] = v.y;
  f[3 * o + 2] = v.z;
}

struct Carve2 {
  size_t off = 0;
  char* base = nullptr;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

md_params internal_params(double r_cut, int32_t cap) {
  md_params p;
  memset(&p, 0, sizeof(p));
  p.mass = 1.0;
  p.dt = 0.0;
  p.r_cut = r_cut;
  p.skin = 0.0;
  p.ftm2v = 1.0;
  p.kboltz = 1.0;
  p.precision = MD_FP64;
  p.nbr_capacity = cap;
  p.cell_capacity = 64;
  p.chunk_steps = 2;
  p.lanes_per_atom = 1;
  p.sort_every = 0;
  p.list_mode = MD_LIST_FULL;
  p.n_types = 0;
  p.launch_mode = MD_LAUNCH_GRAPH;
  p.reserved = 0;
  return p;
}

size_t fm_part_bytes(char* base, int64_t n, int64_t tiles, int nbins, FmArgs* a) {
  Carve2 c;
  c.base = base;
  const size_t N = (size_t)(n > 0 ? n : 1);
  FmArgs tmp;
  FmArgs& o = a ? *a : tmp;
  o.rho_i = c.take<double>(N);
  o.fp = c.take<double>(N);
  o.fpp = c.take<double>(N);
  o.frc = c.take<double4>(N);
  o.gvec = c.take<double4>(N);
  o.fref = c.take<double4>(N);
  o.lam = c.take<double>(N);
  o.mu = c.take<double>(N);
  o.partial = c.take<double>((size_t)tiles);
  o.bound = c.take<double>((size_t)tiles);
  o.scale = c.take<double>(2);
  // the loss and the flag word side by side: the forward returns both with one copy
  o.loss = c.take<double>(2);
  o.flag = o.loss ? reinterpret_cast<int32_t*>(o.loss + 1) : nullptr;
  o.hist = c.take<unsigned long long>((size_t)kFmBlocks * nbins);
  o.part = c.take<unsigned long long>((size_t)kFmSplit * nbins);
  return (c.off + 255) & ~size_t(255);
}

}  // namespace

struct md_fm_ctx {
  md_ctx* md = nullptr;
  size_t md_bytes = 0;
  CtxView v{};
  FmArgs a{};
  hipStream_t stream = nullptr;
  int64_t n = 0;
  bool have_forward = false;
  double* host = nullptr;  // pinned: the loss and the flag word copied back
  std::string err;
};

static md_status fm_fail(md_fm_ctx* c, hipError_t e, const char* what) {
  if (c) c->err = std::string(what) + ": " + hipGetErrorString(e);
  return MD_E_HIP;
}

#define FMC(ctx, expr)                                     \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return fm_fail(ctx, e_, #expr);  \
  } while (0)

extern "C" {

md_status md_fm_workspace_size(int32_t n_cfg, const int64_t* cfg_atoms, const double* cfg_box,
                               double r_cut, int32_t nbr_capacity, const int32_t n_knots[3],
                               size_t* bytes) {
  if (!bytes || !n_knots || n_cfg < 1) return MD_E_ARG;
  md_params p = internal_params(r_cut, nbr_capacity);
  size_t mb = 0;
  md_status s = md_workspace_size(&p, n_cfg, cfg_atoms, cfg_box, &mb);
  if (s != MD_OK) return s;
  int64_t n = 0, tiles = 0;
  for (int c = 0; c < n_cfg; ++c) {
    n += cfg_atoms[c];
    tiles += (cfg_atoms[c] + 63) / 64;
  }
  tiles = ((tiles + kXcd - 1) / kXcd) * kXcd;
  const int nbins = 4 * ((n_knots[0] - 1) + (n_knots[1] - 1) + (n_knots[2] - 1));
  // one histogram of all coefficient bins must fit the coefficient pass's LDS
  if ((size_t)nbins * sizeof(unsigned long long) > kFmLds) return MD_E_TABLE;
  *bytes = ((mb + 255) & ~size_t(255)) + fm_part_bytes(nullptr, n, tiles, nbins, nullptr);
  return MD_OK;
}

md_status md_fm_create(md_fm_ctx** out, int32_t n_cfg, const int64_t* cfg_atoms,
                       const double* cfg_box, double r_cut, int32_t nbr_capacity,
                       const md_spline* grid_phi, const md_spline* grid_rho,
                       const md_spline* grid_emb, const double* x, const double* fref,
                       void* workspace, size_t workspace_bytes, void* stream) {
  if (!out || !x || !fref || !grid_phi || !grid_rho || !grid_emb) return MD_E_ARG;
  *out = nullptr;
  const int32_t nk[3] = {grid_phi->n_knots, grid_rho->n_knots, grid_emb->n_knots};
  size_t need = 0;
  md_status s = md_fm_workspace_size(n_cfg, cfg_atoms, cfg_box, r_cut, nbr_capacity, nk, &need);
  if (s != MD_OK) return s;
  if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return MD_E_WORKSPACE;
  md_params p = internal_params(r_cut, nbr_capacity);
  size_t mb = 0;
  md_workspace_size(&p, n_cfg, cfg_atoms, cfg_box, &mb);
  mb = (mb + 255) & ~size_t(255);
  md_fm_ctx* c = new (std::nothrow) md_fm_ctx();
  if (!c) return MD_E_ARG;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  s = md_create(&c->md, &p, n_cfg, cfg_atoms, cfg_box, grid_phi, grid_rho, grid_emb, workspace,
                mb, stream);
  if (s != MD_OK) {
    delete c;
    return s;
  }
  // zero velocities: the internal context only bins and builds lists
  int64_t n = 0;
  for (int k = 0; k < n_cfg; ++k) n += cfg_atoms[k];
  c->n = n;
  char* fm_base = reinterpret_cast<char*>(workspace) + mb;
  const int nbins = 4 * ((nk[0] - 1) + (nk[1] - 1) + (nk[2] - 1));
  // the velocity import reads 3n doubles; use the force-reference scratch as zeros
  double* zeros = reinterpret_cast<double*>(fm_base);
  hipError_t e = hipMemsetAsync(zeros, 0, (size_t)n * 3 * sizeof(double), c->stream);
  if (e != hipSuccess) {
    md_destroy(c->md);
    delete c;
    return fm_fail(nullptr, e, "hipMemsetAsync");
  }
  s = md_set_state(c->md, x, zeros);
  if (s >= 0) s = md_build_neighbors(c->md);
  // warnings (a density past the embedding table) do not stop set-up
  if (s < 0) {
    md_destroy(c->md);
    delete c;
    return s;
  }
  if (md_internal_view(c->md, &c->v) != MD_OK) {
    md_destroy(c->md);
    delete c;
    return MD_E_ORDER;
  }
  FmArgs& a = c->a;
  fm_part_bytes(fm_base, n, c->v.g.n_atiles, nbins, &a);
  a.g = c->v.g;
  a.s = c->v.s;
  a.rc2 = r_cut * r_cut;
  a.nb_phi = 4 * (nk[0] - 1);
  a.nb_rho = 4 * (nk[1] - 1);
  a.nb_emb = 4 * (nk[2] - 1);
  a.phi = FmSpline{nullptr, grid_phi->x0, grid_phi->inv_dx, nk[0], 0};
  a.rho = FmSpline{nullptr, grid_rho->x0, grid_rho->inv_dx, nk[1], 0};
  a.emb = FmSpline{nullptr, grid_emb->x0, grid_emb->inv_dx, nk[2], 0};
  hipLaunchKernelGGL(k_fm_import_ref, dim3(c->v.L.atile_blocks), dim3(64), 0, c->stream, a, fref);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  const char* what = "import fref";
  if (e == hipSuccess) {
    what = "hipHostMalloc";
    e = hipHostMalloc(reinterpret_cast<void**>(&c->host), 2 * sizeof(double));
  }
  if (e != hipSuccess) {
    md_destroy(c->md);
    delete c;
    return fm_fail(nullptr, e, what);
  }
  *out = c;
  return MD_OK;
}

// The passes of one forward evaluation (no host synchronisation).
static md_status fm_forward_launch(md_fm_ctx* c, const double* coef_phi, const double* coef_rho,
                                   const double* coef_emb, double* loss_dev, double* f_out) {
  FmArgs& a = c->a;
  a.phi.coef = coef_phi;
  a.rho.coef = coef_rho;
  a.emb.coef = coef_emb;
  const int tb = c->v.L.atile_blocks;
  hipLaunchKernelGGL(k_fm_density, dim3(tb), dim3(64), 0, c->stream, a);
  FMC(c, hipGetLastError());
  hipLaunchKernelGGL(k_fm_force, dim3(tb), dim3(64), 0, c->stream, a);
  FMC(c, hipGetLastError());
  hipLaunchKernelGGL(k_fm_loss_reduce, dim3(1), dim3(256), 0, c->stream, a, loss_dev);
  FMC(c, hipGetLastError());
  if (f_out) {
    hipLaunchKernelGGL(k_fm_export_f, dim3(tb), dim3(64), 0, c->stream, a, f_out);
    FMC(c, hipGetLastError());
  }
  c->have_forward = true;
  return MD_OK;
}

// The passes of one backward evaluation (no host synchronisation).
static md_status fm_backward_launch(md_fm_ctx* c, double seed, const double* seed_dev,
                                    double* g_phi, double* g_rho, double* g_emb) {
  FmArgs& a = c->a;
  const int tb = c->v.L.atile_blocks;
  const int nb = a.nb_phi + a.nb_rho + a.nb_emb;
  hipLaunchKernelGGL(k_fm_lambda, dim3(tb), dim3(64), 0, c->stream, a);
  FMC(c, hipGetLastError());
  hipLaunchKernelGGL(k_fm_scale, dim3(1), dim3(256), 0, c->stream, a,
                     (double)c->n * (double)a.g.nbr_cap);
  FMC(c, hipGetLastError());
  hipLaunchKernelGGL(k_fm_coef, dim3(kFmBlocks), dim3(64), nb * sizeof(unsigned long long),
                     c->stream, a);
  FMC(c, hipGetLastError());
  hipLaunchKernelGGL(k_fm_coef_reduce1, dim3((nb + 63) / 64, kFmSplit), dim3(256), 0, c->stream,
                     a, kFmBlocks);
  FMC(c, hipGetLastError());
  hipLaunchKernelGGL(k_fm_coef_reduce, dim3((nb + 255) / 256), dim3(256), 0, c->stream, a, seed,
                     seed_dev, g_phi, g_rho, g_emb);
  FMC(c, hipGetLastError());
  return MD_OK;
}

// The flag word (non-finite values or fixed-point overflow latched by the
// kernels) to the host, then cleared.
static md_status fm_take_flag(md_fm_ctx* c, bool with_loss) {
  FmArgs& a = c->a;
  if (with_loss)
    FMC(c, hipMemcpyAsync(c->host, a.loss, sizeof(double) + sizeof(int32_t),
                          hipMemcpyDeviceToHost, c->stream));
  else
    FMC(c, hipMemcpyAsync(c->host + 1, a.flag, sizeof(int32_t), hipMemcpyDeviceToHost,
                          c->stream));
  FMC(c, hipMemsetAsync(a.flag, 0, sizeof(int32_t), c->stream));
  FMC(c, hipStreamSynchronize(c->stream));
  int32_t flag = 0;
  memcpy(&flag, c->host + 1, sizeof(int32_t));
  return flag ? MD_E_NONFINITE : MD_OK;
}

md_status md_fm_forward(md_fm_ctx* c, const double* coef_phi, const double* coef_rho,
                        const double* coef_emb, double* loss, double* f_out) {
  if (!c || !coef_phi || !coef_rho || !coef_emb) return MD_E_ARG;
  FMC(c, hipMemsetAsync(c->a.flag, 0, sizeof(int32_t), c->stream));
  md_status rc = fm_forward_launch(c, coef_phi, coef_rho, coef_emb, nullptr, f_out);
  if (rc != MD_OK) return rc;
  rc = fm_take_flag(c, true);
  if (loss) *loss = c->host[0];
  return rc;
}

md_status md_fm_backward(md_fm_ctx* c, double seed, double* g_phi, double* g_rho, double* g_emb) {
  if (!c || !g_phi || !g_rho || !g_emb) return MD_E_ARG;
  if (!c->have_forward) return MD_E_ORDER;
  const md_status rc = fm_backward_launch(c, seed, nullptr, g_phi, g_rho, g_emb);
  if (rc != MD_OK) return rc;
  return fm_take_flag(c, false);
}

md_status md_fm_forward_async(md_fm_ctx* c, const double* coef_phi, const double* coef_rho,
                              const double* coef_emb, double* loss_dev, double* f_out) {
  if (!c || !coef_phi || !coef_rho || !coef_emb || !loss_dev) return MD_E_ARG;
  return fm_forward_launch(c, coef_phi, coef_rho, coef_emb, loss_dev, f_out);
}

md_status md_fm_backward_async(md_fm_ctx* c, const double* seed_dev, double* g_phi,
                               double* g_rho, double* g_emb) {
  if (!c || !seed_dev || !g_phi || !g_rho || !g_emb) return MD_E_ARG;
  if (!c->have_forward) return MD_E_ORDER;
  return fm_backward_launch(c, 0.0, seed_dev, g_phi, g_rho, g_emb);
}

md_status md_fm_check(md_fm_ctx* c) {
  if (!c) return MD_E_ARG;
  return fm_take_flag(c, false);
}

void md_fm_destroy(md_fm_ctx* c) {
  if (!c) return;
  if (c->md) md_destroy(c->md);
  if (c->host) (void)hipHostFree(c->host);
  delete c;
}

}  // extern "C"
