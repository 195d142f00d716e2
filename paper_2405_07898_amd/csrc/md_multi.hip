// md_multi.hip -- the pair passes and energy of the multi-species form, float64.
//
// Sec. II-A lets the density, embedding and pair functions depend on the atom
// types (after Eq. potential; tables per type, as the paper's per-core
// interpolation tables are):
//   rho_i = sum_j rho_{t_j}(r_ij)                                Eq. (density)
//   F_i   = sum_j [F'_i rho'_{t_j}(r) + F'_j rho'_{t_i}(r) + phi'_{t_i t_j}(r)]
//           (x_j - x_i)/r                                        Eq. (EAMforce)
//   U     = 1/2 sum phi_{t_i t_j} + sum_i F_{t_i}(rho_i)         Eq. (potential)
// The list walk, batching, lanes per atom and the fused leap-frog update are
// those of the one-species passes.  The density rows of all types go to the
// LDS when they fit (T = 2 with 2000 knots: 128 KB).  The force rows (T rho'
// and T(T+1)/2 phi' quadratics per segment, 240 KB for T = 2) do not: the LDS
// holds the segments from the far end of the table down to where 150 KB runs
// out (r >= 1.8 A for T = 2 with 2000 knots on [0, 5]), and closer pairs, rare
// in a solid or a melt, read the rows from global memory, interleaved by
// segment so that the three rows one pair needs share a 128-byte line.  Each
// neighbour's type comes from a one-byte array indexed like the positions.
#include "md_device.h"

#include <algorithm>

#pragma clang fp contract(off)

namespace mdk {

namespace {

constexpr int kMultiThreads = 768;  // density: 12 waves
constexpr int kMultiForceThreads = 512;  // force: 8 waves (more registers per lane)

__device__ __forceinline__ double cubic(const double4 c, double t) {
  return fma(fma(fma(c.w, t, c.z), t, c.y), t, c.x);
}

// F'(rho) of type ti; past the last knot the table continues along its end tangent.
__device__ __forceinline__ double emb_slope(const MultiTables& t, int ti, double rho, bool& range) {
  const double xe = (rho - t.e_x0) * t.e_inv_dx;
  const int le = t.ne - 2;
  const int ke = (xe >= (double)le) ? le : ((xe > 0.0) ? (int)xe : 0);
  const double te = fmin(xe - (double)ke, 1.0);
  const double4 ce = t.emb_val[(size_t)ti * (t.ne - 1) + ke];
  range = xe > (double)(t.ne - 1);
  return fma(fma(3.0 * ce.w, te, 2.0 * ce.z), te, ce.y) * t.e_inv_dx;
}

template <int LPA, bool kLds>
__global__ __launch_bounds__(kMultiThreads) void k_density_multi(
    Geometry g, State s, MultiTables t, double4* __restrict__ pos, const int32_t* cond_zero,
    int32_t* clear_flag, int32_t* rclear, int64_t ncells, int want_rho) {
  extern __shared__ double4 lds_d4[];
  const int32_t zero_bins = cond_zero ? *cond_zero : 0;
  const bool err = has_error(s.status);
  if (clear_flag && blockIdx.x == 0) {
    if (threadIdx.x == 0) *clear_flag = 0;
    for (int r = threadIdx.x; r < g.n_rep; r += blockDim.x) rclear[r] = 0;
  }
  const int nrow = (t.nr - 1) * t.n_types;
  if (kLds) lds_fill<4>(lds_d4, t.rho_seg, nrow, lds_d4 + nrow);
  if (zero_bins) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ncells;
         k += (int64_t)gridDim.x * blockDim.x)
      s.bin_cnt[k] = 0;
  }
  if (kLds) __syncthreads();
  if (err) return;
  const double4* __restrict__ tab = kLds ? lds_d4 : t.rho_seg;
  const uint32_t N = (uint32_t)g.n;
  const int T = t.n_types;
  const int last = t.nr - 2;
  const TileWalk w = tile_walk<LPA>();
  for (int64_t it = w.q;; it += w.tpi) {
    const int64_t b = walk_tile(it, g.n_atiles);
    if (b < 0) break;
    const AtomTile tl = g.atiles[b];
    const bool active = w.a < tl.count;
    const RepDev& rp = g.reps[tl.rep];
    const int64_t i = tl.begin + (active ? w.a : 0);
    const uint32_t self_e = (uint32_t)i | (kNoShift << kIndexBits);
    const int m = active ? min(s.cnt[i], g.nbr_cap) : 0;
    const double4 pi = pos[i];
    double acc = 0.0;
    const int kstep = LPA * kBatch;
    uint32_t e[kBatch];
    load_entries<LPA>(s.nbr, N, (uint32_t)i, w.sub, m, self_e, e);
    for (int k0 = w.sub; k0 < m; k0 += kstep) {
      double4 q[kBatch];
      int tj[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const uint32_t j = e[u] & kIndexMask;
        q[u] = pos[j];
        tj[u] = s.type[j];
      }
      uint32_t en[kBatch];
      load_entries<LPA>(s.nbr, N, (uint32_t)i, k0 + kstep, m, self_e, en);
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        double dx, dy, dz;
        separation(e[u], rp, q[u].x, q[u].y, q[u].z, pi.x, pi.y, pi.z, dx, dy, dz);
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const bool in = (k0 + u * LPA < m) && r2 < g.rc2;
        const double rr = in ? r2 : 1.0;
        const double x = (rr * rsq64(rr)) * t.r_inv_dx;
        const int kk = min(max((int)x, 0), last);
        const double tt = x - (double)kk;
        const double4 c = tab[kk * T + tj[u]];
        if (in) acc += cubic(c, tt);
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) e[u] = en[u];
    }
    const double rho_i = lane_sum_sym<LPA>(acc);
    if (!active || w.sub != 0) continue;
    bool range;
    pos[i].w = emb_slope(t, s.type[i], rho_i, range);
    if (want_rho) s.rho[i] = rho_i;
    if (range) set_bits(s.status, ST_RHO_RANGE);
  }
}

// Rows per segment of the force table and the LDS the force pass may use.
constexpr size_t kForceLdsMax = 150 * 1024;

__device__ __forceinline__ int force_rows(int T) { return T + T * (T + 1) / 2; }

// Force segments [lds_seg0, nr-1) into the LDS, 3 * rows doubles each, packed.
// As in the one-species fill, each thread requests kU values before storing
// any; indexes past the end load the last value again and store into a junk
// slot of the lane (64 doubles after the rows).
__device__ __forceinline__ void fill_force_rows(double* lds, const MultiTables& t) {
  constexpr int kU = 8;
  const int w = 3 * force_rows(t.n_types);
  const int n = (t.nr - 1 - t.lds_seg0) * w;
  const int nt = (int)blockDim.x;
  double* const junk = lds + n + (threadIdx.x & 63);
  for (int b = (int)threadIdx.x; b < n; b += kU * nt) {
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int idx = min(b + u * nt, n - 1);
      const int seg = idx / w;
      v[u] = t.frow[(size_t)(t.lds_seg0 + seg) * t.seg_stride + (idx - seg * w)];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) *(b + u * nt < n ? lds + b + u * nt : junk) = v[u];
  }
}

// A read of the force rows in the LDS through an LDS-typed pointer: the
// compiler then cannot fold it with the global-memory fallback below into one
// generic (flat) load, which would wait on global memory as well.
__device__ __forceinline__ double lds_ld(const double* p) {
  return *(const __attribute__((address_space(3))) double*)p;
}

template <int LPA>
__device__ __forceinline__ void pair_forces_multi(const Geometry& g, const State& s,
                                                  const MultiTables& t, const double* lds_rows,
                                                  const RepDev& rp,
                                                  const double4* __restrict__ pos, int64_t i,
                                                  bool active, int sub, double4 pi, double& fx,
                                                  double& fy, double& fz) {
  const int lw = 3 * force_rows(t.n_types);
  const uint32_t N = (uint32_t)g.n;
  const uint32_t self_e = (uint32_t)i | (kNoShift << kIndexBits);
  const int m = active ? min(s.cnt[i], g.nbr_cap) : 0;
  const int last = t.nr - 2;
  const int T = t.n_types;
  const int ti = s.type[i];
  double ax = 0.0, ay = 0.0, az = 0.0;
  const int kstep = LPA * kBatch;
  uint32_t e[kBatch];
  load_entries<LPA>(s.nbr, N, (uint32_t)i, sub, m, self_e, e);
  for (int k0 = sub; k0 < m; k0 += kstep) {
    double4 q[kBatch];
    int tj[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const uint32_t j = e[u] & kIndexMask;
      q[u] = pos[j];
      tj[u] = s.type[j];
    }
    uint32_t en[kBatch];
    load_entries<LPA>(s.nbr, N, (uint32_t)i, k0 + kstep, m, self_e, en);
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      double dx, dy, dz;
      separation(e[u], rp, q[u].x, q[u].y, q[u].z, pi.x, pi.y, pi.z, dx, dy, dz);
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      const bool in = (k0 + u * LPA < m) && r2 < g.rc2;
      const double rr = in ? r2 : 1.0;
      const double rinv = rsq64(rr);
      const double x = (rr * rinv) * t.r_inv_dx;
      // pairs that do not interact read the last segment (held in the LDS)
      const int kk = in ? min(max((int)x, 0), last) : last;
      const double tt = x - (double)kk;
      // the segment's rows rho'_{t_j}, rho'_{t_i}, phi'_{t_i t_j}: from the LDS,
      // or (a pair closer than the LDS segments, rare) from global memory
      const int oj = 3 * tj[u], oi = 3 * ti, op = 3 * t.pair_row[ti * T + tj[u]];
      const double* seg = lds_rows + max(kk - t.lds_seg0, 0) * lw;
      double c[9] = {lds_ld(seg + oj), lds_ld(seg + oj + 1), lds_ld(seg + oj + 2),
                     lds_ld(seg + oi), lds_ld(seg + oi + 1), lds_ld(seg + oi + 2),
                     lds_ld(seg + op), lds_ld(seg + op + 1), lds_ld(seg + op + 2)};
      if (kk < t.lds_seg0) {
        const double* gs = t.frow + (size_t)kk * t.seg_stride;
        c[0] = gs[oj]; c[1] = gs[oj + 1]; c[2] = gs[oj + 2];
        c[3] = gs[oi]; c[4] = gs[oi + 1]; c[5] = gs[oi + 2];
        c[6] = gs[op]; c[7] = gs[op + 1]; c[8] = gs[op + 2];
      }
      const double drho_j = fma(fma(c[2], tt, c[1]), tt, c[0]);
      const double drho_i = fma(fma(c[5], tt, c[4]), tt, c[3]);
      const double dphi = fma(fma(c[8], tt, c[7]), tt, c[6]);
      const double sc = fma(pi.w, drho_j, fma(q[u].w, drho_i, dphi)) * rinv;
      if (in) {
        ax = fma(sc, dx, ax);
        ay = fma(sc, dy, ay);
        az = fma(sc, dz, az);
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) e[u] = en[u];
  }
  fx = lane_sum_sym<LPA>(ax);
  fy = lane_sum_sym<LPA>(ay);
  fz = lane_sum_sym<LPA>(az);
}

template <int LPA>
__global__ __launch_bounds__(kMultiForceThreads) void k_force_integrate_multi(
    Geometry g, State s, MultiTables t, const double4* __restrict__ pos_in,
    double4* __restrict__ pos_out, int32_t* flag_next, int32_t* rflag_next) {
  extern __shared__ double lds_rows[];
  const bool err = has_error(s.status);
  fill_force_rows(lds_rows, t);
  __syncthreads();
  if (err) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter64(s.status, SW_STEPS) += 1ull;
  const TileWalk w = tile_walk<LPA>();
  for (int64_t it = w.q;; it += w.tpi) {
    const int64_t b = walk_tile(it, g.n_atiles);
    if (b < 0) break;
    const AtomTile tl = g.atiles[b];
    const bool active = w.a < tl.count;
    const RepDev& rp = g.reps[tl.rep];
    const int64_t i = tl.begin + (active ? w.a : 0);
    const double4 pi = pos_in[i];
    double4 v = make_double4(0.0, 0.0, 0.0, 0.0), xr = v;
    double a_i = 0.0;
    if (active && w.sub == 0) {
      v = s.vel[i];
      xr = s.xref[i];
      a_i = g.acc_t[s.type[i]];
    }
    double fx, fy, fz;
    pair_forces_multi<LPA>(g, s, t, lds_rows, rp, pos_in, i, active, w.sub, pi, fx, fy, fz);
    bool far = false;
    if (active && w.sub == 0) {
      const double k = g.dt * a_i;
      v.x = fma(k, fx, v.x);
      v.y = fma(k, fy, v.y);
      v.z = fma(k, fz, v.z);
      double4 xn;
      xn.x = fma(g.dt, v.x, pi.x);
      xn.y = fma(g.dt, v.y, pi.y);
      xn.z = fma(g.dt, v.z, pi.z);
      xn.w = 0.0;
      pos_out[i] = xn;
      s.vel[i] = v;
      const double ex = xn.x - xr.x, ey = xn.y - xr.y, ez = xn.z - xr.z;
      const double d2 = fma(ex, ex, fma(ey, ey, ez * ez));
      far = !(d2 <= g.lim2);
      if (!isfinite(fx + fy + fz) || !isfinite(xn.x + xn.y + xn.z))
        set_bits(s.status, ST_NONFINITE);
    }
    if (__ballot(far) != 0ull && lane_id() == 0) {
      *flag_next = 1;
      rflag_next[tl.rep] = 1;
    }
  }
}

template <int LPA>
__global__ __launch_bounds__(kMultiForceThreads) void k_force_only_multi(Geometry g, State s,
                                                                    MultiTables t,
                                                                    const double4* __restrict__ pos) {
  extern __shared__ double lds_rows[];
  const bool err = has_error(s.status);
  fill_force_rows(lds_rows, t);
  __syncthreads();
  if (err) return;
  const TileWalk w = tile_walk<LPA>();
  for (int64_t it = w.q;; it += w.tpi) {
    const int64_t b = walk_tile(it, g.n_atiles);
    if (b < 0) break;
    const AtomTile tl = g.atiles[b];
    const bool active = w.a < tl.count;
    const RepDev& rp = g.reps[tl.rep];
    const int64_t i = tl.begin + (active ? w.a : 0);
    const double4 pi = pos[i];
    double fx, fy, fz;
    pair_forces_multi<LPA>(g, s, t, lds_rows, rp, pos, i, active, w.sub, pi, fx, fy, fz);
    if (active && w.sub == 0) {
      s.frc[i] = make_double4(fx, fy, fz, 0.0);
      if (!isfinite(fx + fy + fz)) set_bits(s.status, ST_NONFINITE);
    }
  }
}

// Per-atom energies e_i = 1/2 sum_j phi_{t_i t_j} + F_{t_i}(rho_i) and the
// kinetic energy with the type's mass; block sums into the per-tile partials.
__global__ __launch_bounds__(64) void k_energy_multi_atoms(Geometry g, State s, MultiTables t,
                                                           double coef) {
  __shared__ double s_e[64], s_k[64];
  const AtomTile tl = g.atiles[blockIdx.x];
  const bool active = (int)threadIdx.x < tl.count;
  double ep = 0.0, ek = 0.0;
  if (active) {
    const RepDev& rp = g.reps[tl.rep];
    const int64_t i = tl.begin + threadIdx.x;
    const double4 pi = s.pos[i];
    const int ti = s.type[i];
    const size_t rows = (size_t)(t.nr - 1);
    const int m = min(s.cnt[i], g.nbr_cap);
    double rho = 0.0, ph = 0.0;
    const int last = t.nr - 2;
    for (int k = 0; k < m; ++k) {
      const uint32_t e = s.nbr[(int64_t)k * g.n + i];
      const uint32_t j = e & kIndexMask;
      const double4 q = s.pos[j];
      double dx, dy, dz;
      separation(e, rp, q.x, q.y, q.z, pi.x, pi.y, pi.z, dx, dy, dz);
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      if (r2 < g.rc2) {
        const int tj = s.type[j];
        const double x = sqrt(r2) * t.r_inv_dx;
        const int kk = min(max((int)x, 0), last);
        const double tt = x - (double)kk;
        rho += cubic(t.rho_val[(size_t)tj * rows + kk], tt);
        ph += cubic(t.phi_val[(size_t)(ti * t.n_types + tj) * rows + kk], tt);
      }
    }
    const double xe = (rho - t.e_x0) * t.e_inv_dx;
    const int le = t.ne - 2;
    const int ke = (xe >= (double)le) ? le : ((xe > 0.0) ? (int)xe : 0);
    const double te = xe - (double)ke;
    const double4 c = t.emb_val[(size_t)ti * (t.ne - 1) + ke];
    const double fe = (te > 1.0) ? ((c.x + c.y + c.z + c.w) +
                                    (c.y + 2.0 * c.z + 3.0 * c.w) * (te - 1.0))
                                 : cubic(c, te);
    ep = 0.5 * ph + fe;
    const double a_i = g.acc_t[ti];
    const double vscale = coef * a_i;
    const double4 v = s.vel[i];
    const double4 f = s.frc[i];
    const double ux = fma(vscale, f.x, v.x), uy = fma(vscale, f.y, v.y), uz = fma(vscale, f.z, v.z);
    ek = 0.5 * (1.0 / a_i) * ((ux * ux + uy * uy) + uz * uz);
  }
  s_e[threadIdx.x] = ep;
  s_k[threadIdx.x] = ek;
  __syncthreads();
  for (int o = 32; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s_e[threadIdx.x] += s_e[threadIdx.x + o];
      s_k[threadIdx.x] += s_k[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && tl.count > 0) {
    const RepDev& rp = g.reps[tl.rep];
    const int64_t slot = rp.tile0 + (tl.begin - rp.atom0) / 64;
    s.partial[2 * slot] = s_e[0];
    s.partial[2 * slot + 1] = s_k[0];
  }
}

// Types of the atoms in original order, checked against the type count.
__global__ __launch_bounds__(256) void k_types_in(State s, int64_t n, const int32_t* __restrict__ in,
                                                  int32_t n_types) {
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int32_t t = in[o];
    if (t < 0 || t >= n_types) {
      s.status[SW_TYPE_CHECK] = 1;
      s.type_orig[o] = 0;
    } else {
      s.type_orig[o] = (uint8_t)t;
    }
  }
}

// Slot types from the original-order types through the slot -> atom map.
__global__ __launch_bounds__(256) void k_types_to_slots(State s, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s.type[i] = s.type_orig[s.id[i]];
}

}  // namespace

static int force_rows_host(int T) { return T + T * (T + 1) / 2; }

// First segment of the force rows held in the LDS: as many segments from the
// far end of the table as fit in kForceLdsMax bytes.
int multi_force_lds_seg0(int nr, int n_types) {
  const size_t per = (size_t)3 * force_rows_host(n_types) * sizeof(double);
  const int fit = (int)(kForceLdsMax / per);
  return std::max(0, (nr - 1) - fit);
}

size_t multi_force_lds_bytes(const MultiTables& t) {
  return ((size_t)(t.nr - 1 - t.lds_seg0) * 3 * force_rows_host(t.n_types) + 64) * sizeof(double);
}

// Density rows of all types in the LDS, plus the junk rows of the fill; 0 when
// they do not fit.
size_t multi_density_lds_bytes(const MultiTables& t) {
  const size_t b = (size_t)(t.nr - 1) * t.n_types * sizeof(double4) + kLdsJunkBytes;
  return b <= 150 * 1024 ? b : 0;
}

namespace {

int multi_threads(int lpa, int waves = 12) {
  int tpi = waves / lpa;
  if (tpi < 1) tpi = 1;
  return 64 * lpa * tpi;
}

int grid_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return (int)b;
}

}  // namespace

#define MDK_MULTI_LPA(lpa, CALL) \
  switch (lpa) {                 \
    case 1: CALL(1); break;      \
    case 2: CALL(2); break;      \
    case 4: CALL(4); break;      \
    default: CALL(8); break;     \
  }

hipError_t launch_multi_density(const Launch& L, const Geometry& g, const State& s,
                                const MultiTables& t, int lpa, const double4* pos,
                                const int32_t* cond_zero, int32_t* clear_flag, int32_t* rclear,
                                int64_t n_cells_total, bool want_rho) {
  double4* p = const_cast<double4*>(pos);
  const int w = want_rho ? 1 : 0;
  const size_t lds = multi_density_lds_bytes(t);
  // LDS rows: as many workgroups per CU as the LDS holds (one for T = 2)
  const int grid = lds > 80 * 1024 ? L.persist_blocks : 2 * L.persist_blocks;
#define MDK_GO(Lp)                                                                           \
  if (lds)                                                                                   \
    hipLaunchKernelGGL((k_density_multi<Lp, true>), dim3(grid), dim3(multi_threads(Lp)), lds, \
                       L.stream, g, s, t, p, cond_zero, clear_flag, rclear, n_cells_total, w); \
  else                                                                                       \
    hipLaunchKernelGGL((k_density_multi<Lp, false>), dim3(2 * L.persist_blocks),             \
                       dim3(multi_threads(Lp)), 0, L.stream, g, s, t, p, cond_zero,          \
                       clear_flag, rclear, n_cells_total, w)
  MDK_MULTI_LPA(lpa, MDK_GO)
#undef MDK_GO
  return hipGetLastError();
}

hipError_t allow_multi_lds(const MultiTables& t) {
  const size_t fl = multi_force_lds_bytes(t);
  const void* fk[8] = {reinterpret_cast<const void*>(&k_force_integrate_multi<1>),
                       reinterpret_cast<const void*>(&k_force_integrate_multi<2>),
                       reinterpret_cast<const void*>(&k_force_integrate_multi<4>),
                       reinterpret_cast<const void*>(&k_force_integrate_multi<8>),
                       reinterpret_cast<const void*>(&k_force_only_multi<1>),
                       reinterpret_cast<const void*>(&k_force_only_multi<2>),
                       reinterpret_cast<const void*>(&k_force_only_multi<4>),
                       reinterpret_cast<const void*>(&k_force_only_multi<8>)};
  for (const void* f : fk) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fl);
    if (e != hipSuccess) return e;
  }
  const size_t lds = multi_density_lds_bytes(t);
  if (!lds) return hipSuccess;
  const void* k[4] = {reinterpret_cast<const void*>(&k_density_multi<1, true>),
                      reinterpret_cast<const void*>(&k_density_multi<2, true>),
                      reinterpret_cast<const void*>(&k_density_multi<4, true>),
                      reinterpret_cast<const void*>(&k_density_multi<8, true>)};
  for (const void* f : k) {
    const hipError_t e =
        hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_multi_force_integrate(const Launch& L, const Geometry& g, const State& s,
                                        const MultiTables& t, int lpa, const double4* pos_in,
                                        double4* pos_out, int32_t* flag_next, int32_t* rflag_next) {
  const size_t lds = multi_force_lds_bytes(t);
#define MDK_GO(Lp)                                                                             \
  hipLaunchKernelGGL((k_force_integrate_multi<Lp>), dim3(L.persist_blocks),                    \
                     dim3(multi_threads(Lp, 8)), lds, L.stream, g, s, t, pos_in, pos_out, flag_next, \
                     rflag_next)
  MDK_MULTI_LPA(lpa, MDK_GO)
#undef MDK_GO
  return hipGetLastError();
}

hipError_t launch_multi_force_only(const Launch& L, const Geometry& g, const State& s,
                                   const MultiTables& t, int lpa, const double4* pos) {
  const size_t lds = multi_force_lds_bytes(t);
#define MDK_GO(Lp)                                                                             \
  hipLaunchKernelGGL((k_force_only_multi<Lp>), dim3(L.persist_blocks), dim3(multi_threads(Lp, 8)), \
                     lds, L.stream, g, s, t, pos)
  MDK_MULTI_LPA(lpa, MDK_GO)
#undef MDK_GO
  return hipGetLastError();
}

hipError_t launch_multi_energy(const Launch& L, const Geometry& g, const State& s,
                               const MultiTables& t, double* out_pe_ke, int32_t n_rep) {
  hipLaunchKernelGGL(k_energy_multi_atoms, dim3(L.atile_blocks), dim3(64), 0, L.stream, g, s, t,
                     0.5 * g.dt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_energy_reduce(L, g, s, out_pe_ke, n_rep);
}

hipError_t launch_set_types(const Launch& L, const Geometry& g, const State& s,
                            const int32_t* type_in, int32_t n_types, bool has_slots) {
  hipLaunchKernelGGL(k_types_in, dim3(grid_blocks(g.n)), dim3(256), 0, L.stream, s, g.n, type_in,
                     n_types);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !has_slots) return e;
  hipLaunchKernelGGL(k_types_to_slots, dim3(grid_blocks(g.n)), dim3(256), 0, L.stream, s, g.n);
  return hipGetLastError();
}

}  // namespace mdk
