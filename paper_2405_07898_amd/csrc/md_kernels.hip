// md_kernels.hip -- HIP kernels of the EAM timestep loop for gfx950 (MI355X).
//
// Every per-atom pass walks a full (both directions) Verlet list in a fixed
// order and writes only its own atom, so no float atomics are used and every
// result is bitwise reproducible.  Paper: arXiv 2405.07898, Sec. II-A
// (Eqs. density, potential, EAMforce, leapfrog), Sec. III-A (per-atom
// timestep), Sec. III-C (neighbour list), Sec. V-F (periodic offsets instead
// of modular arithmetic) and Table "flopmodel" (segment arithmetic, r^-1 by
// Newton-Raphson).
//
// Compiled with -ffp-contract=off: every fused multiply-add below is written
// as fma(); the list build and binning reproduce the reference expression
// order exactly (bit-identical cells and neighbour sets).
#include "md_internal.h"

#include <math.h>

#pragma clang fp contract(off)

namespace mdk {

// ============================================================ device helpers

__device__ __forceinline__ double wrap1(double x, double L) {
  if (x >= L) x -= L;
  else if (x < 0.0) {
    x += L;
    if (x >= L) x = 0.0;
  }
  return x;
}

// 1/sqrt(x) in float64: hardware estimate, then two Newton-Raphson steps
// y <- y + y/2 (1 - x y^2) (the paper evaluates r^-1 = (r^2)^-1/2 by
// Newton-Raphson, Table "flopmodel").
__device__ __forceinline__ double rsq64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, h, y);
  h = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, h, y);
  return y;
}

// Knuth TwoSum accumulation of v into (s, c): s + c carries the exact sum of
// the rounded terms up to O(n eps^2).
__device__ __forceinline__ void two_sum_acc(float& s, float& c, float v) {
  float t = s + v;
  float bp = t - s;
  float e = (s - (t - bp)) + (v - bp);
  s = t;
  c += e;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ long long wave_sum_i64(long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ bool has_error(const int32_t* status) {
  return (__hip_atomic_load(status + SW_BITS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
          ST_ERR_MASK) != 0;
}

__device__ __forceinline__ void set_bits(int32_t* status, int32_t bits) {
  __hip_atomic_fetch_or(status + SW_BITS, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long* counter64(int32_t* status, int word) {
  return reinterpret_cast<unsigned long long*>(status + word);
}

// Image shift encoded in a list entry: 2 bits per dimension, value s+1 for a
// shift of s box lengths (s in -1, 0, +1) added to x_j - x_i.
__device__ __forceinline__ void apply_shift(uint32_t code, const RepDev& rp, double& dx, double& dy,
                                            double& dz) {
  dx += (double)((int)(code & 3u) - 1) * rp.box[0];
  dy += (double)((int)((code >> 2) & 3u) - 1) * rp.box[1];
  dz += (double)((int)(code >> 4) - 1) * rp.box[2];
}

// ============================================================ import / export

__global__ __launch_bounds__(64) void k_import(Geometry g, State s, const double* __restrict__ x,
                                               const double* __restrict__ v) {
  const AtomTile tl = g.atiles[blockIdx.x];
  if ((int)threadIdx.x >= tl.count) return;
  const RepDev& rp = g.reps[tl.rep];
  const int64_t i = tl.begin + threadIdx.x;
  double4 p;
  p.x = wrap1(x[3 * i + 0], rp.box[0]);
  p.y = wrap1(x[3 * i + 1], rp.box[1]);
  p.z = wrap1(x[3 * i + 2], rp.box[2]);
  p.w = 0.0;
  if (!(p.x >= 0.0 && p.x < rp.box[0] && p.y >= 0.0 && p.y < rp.box[1] && p.z >= 0.0 &&
        p.z < rp.box[2]))
    set_bits(s.status, ST_LOST);
  s.pos[i] = p;
  s.vel[i] = make_double4(v[3 * i + 0], v[3 * i + 1], v[3 * i + 2], 0.0);
  s.id[i] = (int32_t)i;
}

__global__ __launch_bounds__(64) void k_export(Geometry g, State s, double* __restrict__ x,
                                               double* __restrict__ v, double* __restrict__ f,
                                               double* __restrict__ rho, double* __restrict__ fp,
                                               double vscale) {
  const AtomTile tl = g.atiles[blockIdx.x];
  if ((int)threadIdx.x >= tl.count) return;
  const RepDev& rp = g.reps[tl.rep];
  const int64_t i = tl.begin + threadIdx.x;
  const int64_t o = s.id[i];
  const double4 p = s.pos[i];
  if (x) {
    x[3 * o + 0] = wrap1(p.x, rp.box[0]);
    x[3 * o + 1] = wrap1(p.y, rp.box[1]);
    x[3 * o + 2] = wrap1(p.z, rp.box[2]);
  }
  const double4 fr = s.frc[i];
  if (v) {
    const double4 u = s.vel[i];
    v[3 * o + 0] = fma(vscale, fr.x, u.x);
    v[3 * o + 1] = fma(vscale, fr.y, u.y);
    v[3 * o + 2] = fma(vscale, fr.z, u.z);
  }
  if (f) {
    f[3 * o + 0] = fr.x;
    f[3 * o + 1] = fr.y;
    f[3 * o + 2] = fr.z;
  }
  if (rho) rho[o] = s.rho[i];
  if (fp) fp[o] = p.w;
}

__global__ __launch_bounds__(64) void k_export_cells(Geometry g, State s, int32_t* __restrict__ cell) {
  const AtomTile tl = g.atiles[blockIdx.x];
  if ((int)threadIdx.x >= tl.count) return;
  const int64_t i = tl.begin + threadIdx.x;
  cell[s.id[i]] = s.cell_of[i];
}

__global__ __launch_bounds__(64) void k_export_nbrs(Geometry g, State s, int32_t* __restrict__ cnt,
                                                    int32_t* __restrict__ nbr, int32_t cap_out) {
  const AtomTile tl = g.atiles[blockIdx.x];
  if ((int)threadIdx.x >= tl.count) return;
  const int64_t i = tl.begin + threadIdx.x;
  const int64_t o = s.id[i];
  const int32_t c = s.cnt[i];
  cnt[o] = c;
  const int32_t m = min(min(c, g.nbr_cap), cap_out);
  for (int32_t k = 0; k < cap_out; ++k) {
    int32_t val = -1;
    if (k < m) val = s.id[s.nbr[(size_t)k * g.n + i] & kIndexMask];
    nbr[o * cap_out + k] = val;
  }
}

// ============================================================ binning

__global__ __launch_bounds__(256) void k_zero_i32(int32_t* __restrict__ p, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    p[k] = 0;
}

// Wrap each atom into its box (rule: one shift by L, a result equal to L
// becomes 0), assign it to cell (cz*ny + cy)*nx + cx with
// c_d = min(int(x_d * n_d/L_d), n_d - 1), append it to that cell's bin, and
// snapshot the reference positions for the skin check.
__global__ __launch_bounds__(64) void k_bin(Geometry g, State s, const int32_t* cond) {
  if (cond && *cond == 0) return;
  if (has_error(s.status)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (cond) *counter64(s.status, SW_REBUILDS) += 1ull;
    s.status[SW_MAX_LIST] = 0;
    s.status[SW_MAX_CELL] = 0;
    *counter64(s.status, SW_LIST_TOTAL) = 0ull;
  }
  const AtomTile tl = g.atiles[blockIdx.x];
  if ((int)threadIdx.x >= tl.count) return;
  const RepDev& rp = g.reps[tl.rep];
  const int64_t i = tl.begin + threadIdx.x;
  double4 p = s.pos[i];
  p.x = wrap1(p.x, rp.box[0]);
  p.y = wrap1(p.y, rp.box[1]);
  p.z = wrap1(p.z, rp.box[2]);
  if (!(p.x >= 0.0 && p.x < rp.box[0] && p.y >= 0.0 && p.y < rp.box[1] && p.z >= 0.0 &&
        p.z < rp.box[2])) {
    set_bits(s.status, ST_LOST);
    return;
  }
  s.pos[i] = p;
  s.xref[i] = p;
  int32_t c[3];
  const double q[3] = {p.x, p.y, p.z};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double sc = q[d] * rp.inv_cell[d];
    int32_t k = (sc > 0.0) ? (int32_t)sc : 0;
    c[d] = min(k, rp.nc[d] - 1);
  }
  const int32_t cl = (c[2] * rp.nc[1] + c[1]) * rp.nc[0] + c[0];
  s.cell_of[i] = cl;
  const int64_t cg = (int64_t)rp.cell0 + cl;
  const int32_t slot = atomicAdd(&s.bin_cnt[cg], 1);
  if (slot < g.cell_cap) s.bin_idx[cg * g.cell_cap + slot] = (int32_t)i;
  else set_bits(s.status, ST_CELL_OVERFLOW);
}

// ============================================================ list build

// One wave per cell.  The atoms of the 27 surrounding cells are staged in LDS
// (each cell ordered by atom index, so the candidate order is deterministic,
// Sec. III-C), then every atom of the centre cell scans them 64 at a time;
// admitted candidates (r^2 < (r_cut+skin)^2 under the minimum image, same
// expression order as the reference) are compacted with a ballot and written
// to the ELL list together with their image shift.
__global__ __launch_bounds__(64) void k_build(Geometry g, State s, const int32_t* cond) {
  if (cond && *cond == 0) return;
  if (has_error(s.status)) return;
  const CellTile ct = g.ctiles[blockIdx.x];
  if (ct.cell < 0) return;
  const RepDev& rp = g.reps[ct.rep];
  __shared__ int32_t s_q[27], s_n[27], s_off[28];
  __shared__ int32_t s_raw[kMaxStage];
  __shared__ int32_t s_idx[kMaxStage];
  __shared__ double s_x[kMaxStage], s_y[kMaxStage], s_z[kMaxStage];
  __shared__ int32_t s_center[kMaxCellCap], s_base[kMaxCellCap];
  const int lane = threadIdx.x;
  const int32_t nx = rp.nc[0], ny = rp.nc[1], nz = rp.nc[2];
  const int32_t c = ct.cell;
  const int32_t cx = c % nx, cy = (c / nx) % ny, cz = c / (nx * ny);
  const int32_t ccap = g.cell_cap;
  if (lane < 27) {
    const int dz = lane / 9 - 1, dy = (lane / 3) % 3 - 1, dx = lane % 3 - 1;
    const int32_t qx = (cx + dx + nx) % nx, qy = (cy + dy + ny) % ny, qz = (cz + dz + nz) % nz;
    const int32_t q = rp.cell0 + (qz * ny + qy) * nx + qx;
    int32_t n = s.bin_cnt[q];
    if (n > ccap) n = ccap;
    s_q[lane] = q;
    s_n[lane] = n;
  }
  __syncthreads();
  if (lane == 0) {
    s_off[0] = 0;
    for (int k = 0; k < 27; ++k) s_off[k + 1] = s_off[k] + s_n[k];
  }
  __syncthreads();
  // centre atoms in increasing index
  const int32_t qc = s_q[13], n_c = s_n[13];
  for (int u = lane; u < n_c; u += 64) s_raw[u] = s.bin_idx[(int64_t)qc * ccap + u];
  __syncthreads();
  for (int u = lane; u < n_c; u += 64) {
    const int32_t e = s_raw[u];
    int r = 0;
    for (int w = 0; w < n_c; ++w) r += (s_raw[w] < e);
    s_center[r] = e;
    s_base[r] = 0;
  }
  __syncthreads();
  const double Lx = rp.box[0], Ly = rp.box[1], Lz = rp.box[2];
  const double hx = rp.half[0], hy = rp.half[1], hz = rp.half[2];
  const double rl2 = g.rl2;
  const int64_t N = g.n;
  const int32_t cap = g.nbr_cap;
  int s0 = 0;
  while (s0 < 27) {
    int s1 = s0 + 1;
    while (s1 < 27 && s_off[s1 + 1] - s_off[s0] <= kMaxStage) ++s1;
    const int base_off = s_off[s0];
    const int T = s_off[s1] - base_off;
    for (int p = lane; p < T; p += 64) {
      const int gs = base_off + p;
      int sc = s0;
      while (s_off[sc + 1] <= gs) ++sc;
      s_raw[p] = s.bin_idx[(int64_t)s_q[sc] * ccap + (gs - s_off[sc])];
    }
    __syncthreads();
    for (int p = lane; p < T; p += 64) {
      const int gs = base_off + p;
      int sc = s0;
      while (s_off[sc + 1] <= gs) ++sc;
      const int lo = s_off[sc] - base_off, n = s_n[sc];
      const int32_t e = s_raw[p];
      int r = 0;
      for (int w = lo; w < lo + n; ++w) r += (s_raw[w] < e);
      const int dst = lo + r;
      const double4 q = s.pos[e];
      s_idx[dst] = e;
      s_x[dst] = q.x;
      s_y[dst] = q.y;
      s_z[dst] = q.z;
    }
    __syncthreads();
    for (int u = 0; u < n_c; ++u) {
      const int32_t i = s_center[u];
      const double4 pi = s.pos[i];
      int base = s_base[u];
      for (int p0 = 0; p0 < T; p0 += 64) {
        const int p = p0 + lane;
        bool ok = false;
        uint32_t entry = 0;
        if (p < T) {
          const int32_t j = s_idx[p];
          if (j != i) {
            double dx = s_x[p] - pi.x, dy = s_y[p] - pi.y, dz = s_z[p] - pi.z;
            uint32_t kx = 1, ky = 1, kz = 1;
            if (dx > hx) { dx -= Lx; kx = 0; } else if (dx < -hx) { dx += Lx; kx = 2; }
            if (dy > hy) { dy -= Ly; ky = 0; } else if (dy < -hy) { dy += Ly; ky = 2; }
            if (dz > hz) { dz -= Lz; kz = 0; } else if (dz < -hz) { dz += Lz; kz = 2; }
            const double r2 = (dx * dx + dy * dy) + dz * dz;
            ok = r2 < rl2;
            entry = (uint32_t)j | ((kx | (ky << 2) | (kz << 4)) << kIndexBits);
          }
        }
        const unsigned long long m = __ballot(ok);
        if (ok) {
          const int k = base + (int)__builtin_amdgcn_mbcnt_hi(
                                   (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
          if (k < cap) s.nbr[(int64_t)k * N + i] = entry;
        }
        base += __popcll(m);
      }
      if (lane == 0) s_base[u] = base;
    }
    __syncthreads();
    s0 = s1;
  }
  int32_t mx = 0;
  long long tot = 0;
  for (int u = lane; u < n_c; u += 64) {
    const int32_t b = s_base[u];
    s.cnt[s_center[u]] = b;
    mx = max(mx, b);
    tot += b;
  }
  mx = wave_max_i32(mx);
  tot = wave_sum_i64(tot);
  if (lane == 0) {
    if (mx > cap) set_bits(s.status, ST_NBR_OVERFLOW);
    if (s.bin_cnt[qc] > ccap) set_bits(s.status, ST_CELL_OVERFLOW);
    atomicMax(&s.status[SW_MAX_LIST], mx);
    atomicMax(&s.status[SW_MAX_CELL], s.bin_cnt[qc]);
    atomicAdd(counter64(s.status, SW_LIST_TOTAL), (unsigned long long)tot);
  }
}

// ============================================================ sort by cell

// Exclusive scan of the (capped) bin counts over all cells, one block.
__global__ __launch_bounds__(1024) void k_scan_cells(const int32_t* __restrict__ cnt,
                                                     int32_t* __restrict__ start, int64_t m,
                                                     int32_t cap) {
  __shared__ long long s_sum[1024];
  const int t = threadIdx.x;
  const int64_t per = (m + 1023) / 1024;
  const int64_t b = t * per, e = min(m, b + per);
  long long acc = 0;
  for (int64_t k = b; k < e; ++k) acc += min(cnt[k], cap);
  s_sum[t] = acc;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    long long v = (t >= o) ? s_sum[t - o] : 0;
    __syncthreads();
    s_sum[t] += v;
    __syncthreads();
  }
  long long run = s_sum[t] - acc;
  for (int64_t k = b; k < e; ++k) {
    start[k] = (int32_t)run;
    run += min(cnt[k], cap);
  }
  if (t == 1023) start[m] = (int32_t)s_sum[1023];
}

// One thread per cell: order the cell's atoms by original id and gather
// positions, velocities and ids into the sorted scratch arrays.
__global__ __launch_bounds__(256) void k_sort_scatter(State s, int64_t m, int32_t cap) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= m) return;
  const int32_t n = min(s.bin_cnt[c], cap);
  const int32_t* b = s.bin_idx + c * cap;
  const int32_t base = s.cell_start[c];
  for (int32_t u = 0; u < n; ++u) {
    const int32_t e = b[u];
    const int32_t key = s.id[e];
    int32_t r = 0;
    for (int32_t w = 0; w < n; ++w) r += (s.id[b[w]] < key);
    s.sort_pos[base + r] = s.pos[e];
    s.sort_vel[base + r] = s.vel[e];
    s.sort_id[base + r] = key;
  }
}

__global__ __launch_bounds__(256) void k_sort_copyback(State s, int64_t n, int64_t m) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    s.pos[k] = s.sort_pos[k];
    s.vel[k] = s.sort_vel[k];
    s.id[k] = s.sort_id[k];
  }
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m;
       k += (int64_t)gridDim.x * blockDim.x)
    s.bin_cnt[k] = 0;
}

// ============================================================ density pass

template <int LPA>
__device__ __forceinline__ double lane_sum(double v) {
#pragma unroll
  for (int o = 1; o < LPA; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int LPA>
__device__ __forceinline__ void lane_sum2(float& s, float& c) {
#pragma unroll
  for (int o = 1; o < LPA; o <<= 1) {
    const float so = __shfl_xor(s, o, 64), co = __shfl_xor(c, o, 64);
    // combine in a lane-symmetric order so all lanes agree bitwise
    const float lo_s = ((threadIdx.x & o) == 0) ? s : so, hi_s = ((threadIdx.x & o) == 0) ? so : s;
    const float lo_c = ((threadIdx.x & o) == 0) ? c : co, hi_c = ((threadIdx.x & o) == 0) ? co : c;
    s = lo_s;
    c = lo_c + hi_c;
    two_sum_acc(s, c, hi_s);
  }
}

template <int LPA>
__device__ __forceinline__ double lane_sum_sym(double v) {
#pragma unroll
  for (int o = 1; o < LPA; o <<= 1) {
    const double w = __shfl_xor(v, o, 64);
    v = ((threadIdx.x & o) == 0) ? v + w : w + v;
  }
  return v;
}

// rho_i = sum_{j in list, r^2 < rc^2} rho(r_ij); F'_i stored in pos[i].w.
// Side jobs used inside the step graph: clear the next step's rebuild flag,
// and zero the bins after a rebuild (cond_zero set).
template <int PREC, int LPA>
__global__ __launch_bounds__(64 * LPA) void k_density(Geometry g, State s, Tables t,
                                                      double4* __restrict__ pos,
                                                      const int32_t* cond_zero, int32_t* clear_flag,
                                                      int64_t ncells, int want_rho) {
  if (clear_flag && blockIdx.x == 0 && threadIdx.x == 0) *clear_flag = 0;
  if (cond_zero && *cond_zero) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ncells;
         k += (int64_t)gridDim.x * blockDim.x)
      s.bin_cnt[k] = 0;
  }
  if (has_error(s.status)) return;
  const AtomTile tl = g.atiles[blockIdx.x];
  const int a = threadIdx.x / LPA, sub = threadIdx.x % LPA;
  const bool active = a < tl.count;
  const RepDev& rp = g.reps[tl.rep];
  const int64_t i = tl.begin + (active ? a : 0);
  const int64_t N = g.n;
  const double2 pxy = *reinterpret_cast<const double2*>(&pos[i]);
  const double pz = pos[i].z;
  const int m = active ? min(s.cnt[i], g.nbr_cap) : 0;
  const uint32_t* __restrict__ lst = s.nbr + i;
  const int last = t.nr - 2;
  double rho_i;
  if (PREC == 0) {
    double acc = 0.0;
    for (int k = sub; k < m; k += LPA) {
      const uint32_t e = lst[(int64_t)k * N];
      const uint32_t j = e & kIndexMask;
      const double2 qxy = *reinterpret_cast<const double2*>(&pos[j]);
      double dx = qxy.x - pxy.x, dy = qxy.y - pxy.y, dz = pos[j].z - pz;
      const uint32_t code = e >> kIndexBits;
      if (code != kNoShift) apply_shift(code, rp, dx, dy, dz);
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      if (r2 < g.rc2) {
        const double r = r2 * rsq64(r2);
        const double x = r * t.r_inv_dx;
        const int kk = min(max((int)x, 0), last);
        const double tt = x - (double)kk;
        const double4 c = t.rho_val[kk];
        acc += fma(fma(fma(c.w, tt, c.z), tt, c.y), tt, c.x);
      }
    }
    rho_i = lane_sum_sym<LPA>(acc);
  } else {
    float sum = 0.0f, comp = 0.0f;
    const float a32 = t.r_inv_dx32;
    for (int k = sub; k < m; k += LPA) {
      const uint32_t e = lst[(int64_t)k * N];
      const uint32_t j = e & kIndexMask;
      const double2 qxy = *reinterpret_cast<const double2*>(&pos[j]);
      double dx = qxy.x - pxy.x, dy = qxy.y - pxy.y, dz = pos[j].z - pz;
      const uint32_t code = e >> kIndexBits;
      if (code != kNoShift) apply_shift(code, rp, dx, dy, dz);
      const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
      const float r2 = fmaf(fx, fx, fmaf(fy, fy, fz * fz));
      if (r2 < g.rc2f) {
        const float r = r2 * __builtin_amdgcn_rsqf(r2);
        const float x = r * a32;
        const int kk = min(max((int)x, 0), last);
        const float tt = x - (float)kk;
        const float4 c = t.rho_val32[kk];
        two_sum_acc(sum, comp, fmaf(fmaf(fmaf(c.w, tt, c.z), tt, c.y), tt, c.x));
      }
    }
    lane_sum2<LPA>(sum, comp);
    rho_i = (double)sum + (double)comp;
  }
  if (!active || sub != 0) return;
  // F'(rho_i) from the embedding table (float64 for both forms)
  const double xe = (rho_i - t.e_x0) * t.e_inv_dx;
  const int le = t.ne - 2;
  const int ke = (xe >= (double)le) ? le : ((xe > 0.0) ? (int)xe : 0);
  const double te = xe - (double)ke;
  const double4 ce = t.emb_val[ke];
  double fp = fma(fma(3.0 * ce.w, te, 2.0 * ce.z), te, ce.y) * t.e_inv_dx;
  if (PREC != 0) fp = (double)(float)fp;
  pos[i].w = fp;
  if (want_rho) s.rho[i] = rho_i;
  if (xe > (double)(t.ne - 1)) set_bits(s.status, ST_RHO_RANGE);
}

// ============================================================ force pass

// F_i = sum_j [(F'_i + F'_j) rho'(r) + phi'(r)] (x_j - x_i)/r   (Eq. EAMforce)
template <int PREC, int LPA>
__device__ __forceinline__ void pair_forces(const Geometry& g, const State& s, const Tables& t,
                                            const RepDev& rp, const double4* __restrict__ pos,
                                            int64_t i, int m, int sub, double4 pi, double& fx,
                                            double& fy, double& fz) {
  const uint32_t* __restrict__ lst = s.nbr + i;
  const int64_t N = g.n;
  const int last = t.nr - 2;
  if (PREC == 0) {
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int k = sub; k < m; k += LPA) {
      const uint32_t e = lst[(int64_t)k * N];
      const uint32_t j = e & kIndexMask;
      const double4 q = pos[j];
      double dx = q.x - pi.x, dy = q.y - pi.y, dz = q.z - pi.z;
      const uint32_t code = e >> kIndexBits;
      if (code != kNoShift) apply_shift(code, rp, dx, dy, dz);
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      if (r2 < g.rc2) {
        const double rinv = rsq64(r2);
        const double r = r2 * rinv;
        const double x = r * t.r_inv_dx;
        const int kk = min(max((int)x, 0), last);
        const double tt = x - (double)kk;
        const double4 A = t.dpair_a[kk];
        const double2 B = t.dpair_b[kk];
        const double drho = fma(fma(A.z, tt, A.y), tt, A.x);
        const double dphi = fma(fma(B.y, tt, B.x), tt, A.w);
        const double sc = fma(pi.w + q.w, drho, dphi) * rinv;
        ax = fma(sc, dx, ax);
        ay = fma(sc, dy, ay);
        az = fma(sc, dz, az);
      }
    }
    fx = lane_sum_sym<LPA>(ax);
    fy = lane_sum_sym<LPA>(ay);
    fz = lane_sum_sym<LPA>(az);
  } else {
    float sx = 0.f, cx = 0.f, sy = 0.f, cy = 0.f, sz = 0.f, cz = 0.f;
    const float a32 = t.r_inv_dx32;
    const float fpi = (float)pi.w;
    for (int k = sub; k < m; k += LPA) {
      const uint32_t e = lst[(int64_t)k * N];
      const uint32_t j = e & kIndexMask;
      const double4 q = pos[j];
      double dx = q.x - pi.x, dy = q.y - pi.y, dz = q.z - pi.z;
      const uint32_t code = e >> kIndexBits;
      if (code != kNoShift) apply_shift(code, rp, dx, dy, dz);
      const float ex = (float)dx, ey = (float)dy, ez = (float)dz;
      const float r2 = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
      if (r2 < g.rc2f) {
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float r = r2 * rinv;
        const float x = r * a32;
        const int kk = min(max((int)x, 0), last);
        const float tt = x - (float)kk;
        const float4 A = t.dpair_a32[kk];
        const float2 B = t.dpair_b32[kk];
        const float drho = fmaf(fmaf(A.z, tt, A.y), tt, A.x);
        const float dphi = fmaf(fmaf(B.y, tt, B.x), tt, A.w);
        const float sc = fmaf(fpi + (float)q.w, drho, dphi) * rinv;
        two_sum_acc(sx, cx, sc * ex);
        two_sum_acc(sy, cy, sc * ey);
        two_sum_acc(sz, cz, sc * ez);
      }
    }
    lane_sum2<LPA>(sx, cx);
    lane_sum2<LPA>(sy, cy);
    lane_sum2<LPA>(sz, cz);
    fx = (double)sx + (double)cx;
    fy = (double)sy + (double)cy;
    fz = (double)sz + (double)cz;
  }
}

// Force pass fused with the leap-frog update (Eq. leapfrog):
//   v <- v + dt F ftm2v/m ; x' <- x + dt v ; flag a rebuild if |x' - x_ref| > skin/2.
// Positions ping-pong between two buffers (neighbours read pos_in while the
// new positions go to pos_out).
template <int PREC, int LPA>
__global__ __launch_bounds__(64 * LPA) void k_force_integrate(Geometry g, State s, Tables t,
                                                              const double4* __restrict__ pos_in,
                                                              double4* __restrict__ pos_out,
                                                              int32_t* flag_next) {
  if (has_error(s.status)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter64(s.status, SW_STEPS) += 1ull;
  const AtomTile tl = g.atiles[blockIdx.x];
  const int a = threadIdx.x / LPA, sub = threadIdx.x % LPA;
  const bool active = a < tl.count;
  const RepDev& rp = g.reps[tl.rep];
  const int64_t i = tl.begin + (active ? a : 0);
  const double4 pi = pos_in[i];
  const int m = active ? min(s.cnt[i], g.nbr_cap) : 0;
  double fx, fy, fz;
  pair_forces<PREC, LPA>(g, s, t, rp, pos_in, i, m, sub, pi, fx, fy, fz);
  bool far = false;
  if (active && sub == 0) {
    double4 v = s.vel[i];
    const double k = g.dt * g.acc;
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
    const double4 xr = s.xref[i];
    const double ex = xn.x - xr.x, ey = xn.y - xr.y, ez = xn.z - xr.z;
    const double d2 = fma(ex, ex, fma(ey, ey, ez * ez));
    far = !(d2 <= g.lim2);  // also true for NaN
    if (!isfinite(fx + fy + fz) || !isfinite(xn.x + xn.y + xn.z)) set_bits(s.status, ST_NONFINITE);
  }
  if (__ballot(far) != 0ull && lane_id() == 0) *flag_next = 1;
}

// Forces only (no integration), into s.frc.
template <int PREC, int LPA>
__global__ __launch_bounds__(64 * LPA) void k_force_only(Geometry g, State s, Tables t,
                                                         const double4* __restrict__ pos) {
  if (has_error(s.status)) return;
  const AtomTile tl = g.atiles[blockIdx.x];
  const int a = threadIdx.x / LPA, sub = threadIdx.x % LPA;
  const bool active = a < tl.count;
  const RepDev& rp = g.reps[tl.rep];
  const int64_t i = tl.begin + (active ? a : 0);
  const double4 pi = pos[i];
  const int m = active ? min(s.cnt[i], g.nbr_cap) : 0;
  double fx, fy, fz;
  pair_forces<PREC, LPA>(g, s, t, rp, pos, i, m, sub, pi, fx, fy, fz);
  if (active && sub == 0) {
    s.frc[i] = make_double4(fx, fy, fz, 0.0);
    if (!isfinite(fx + fy + fz)) set_bits(s.status, ST_NONFINITE);
  }
}

__global__ __launch_bounds__(64) void k_halfkick(Geometry g, State s, double scale) {
  const AtomTile tl = g.atiles[blockIdx.x];
  if ((int)threadIdx.x >= tl.count) return;
  const int64_t i = tl.begin + threadIdx.x;
  double4 v = s.vel[i];
  const double4 f = s.frc[i];
  v.x = fma(scale, f.x, v.x);
  v.y = fma(scale, f.y, v.y);
  v.z = fma(scale, f.z, v.z);
  s.vel[i] = v;
}

// ============================================================ energy

// Per atom: e_pot = 1/2 sum_j phi(r_ij) + F(rho_i) (Eq. potential, float64),
// e_kin = 1/2 m |v|^2 / ftm2v with on-step v = v_half + vscale F.  Each block
// reduces its tile in a fixed tree order into partial[blockIdx].
__global__ __launch_bounds__(64) void k_energy_atoms(Geometry g, State s, Tables t, double mass_over,
                                                     double vscale) {
  __shared__ double s_e[64], s_k[64];
  const AtomTile tl = g.atiles[blockIdx.x];
  const bool active = (int)threadIdx.x < tl.count;
  double ep = 0.0, ek = 0.0;
  if (active) {
    const RepDev& rp = g.reps[tl.rep];
    const int64_t i = tl.begin + threadIdx.x;
    const double4 pi = s.pos[i];
    const int m = min(s.cnt[i], g.nbr_cap);
    double rho = 0.0, ph = 0.0;
    const int last = t.nr - 2;
    for (int k = 0; k < m; ++k) {
      const uint32_t e = s.nbr[(int64_t)k * g.n + i];
      const double4 q = s.pos[e & kIndexMask];
      double dx = q.x - pi.x, dy = q.y - pi.y, dz = q.z - pi.z;
      const uint32_t code = e >> kIndexBits;
      if (code != kNoShift) apply_shift(code, rp, dx, dy, dz);
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      if (r2 < g.rc2) {
        const double r = sqrt(r2);
        const double x = r * t.r_inv_dx;
        const int kk = min(max((int)x, 0), last);
        const double tt = x - (double)kk;
        const double4 c = t.rho_val[kk];
        const double4 f = t.phi_val[kk];
        rho += fma(fma(fma(c.w, tt, c.z), tt, c.y), tt, c.x);
        ph += fma(fma(fma(f.w, tt, f.z), tt, f.y), tt, f.x);
      }
    }
    const double xe = (rho - t.e_x0) * t.e_inv_dx;
    const int le = t.ne - 2;
    const int ke = (xe >= (double)le) ? le : ((xe > 0.0) ? (int)xe : 0);
    const double te = xe - (double)ke;
    const double4 c = t.emb_val[ke];
    ep = 0.5 * ph + fma(fma(fma(c.w, te, c.z), te, c.y), te, c.x);
    const double4 v = s.vel[i];
    const double4 f = s.frc[i];
    const double ux = fma(vscale, f.x, v.x), uy = fma(vscale, f.y, v.y), uz = fma(vscale, f.z, v.z);
    ek = 0.5 * mass_over * ((ux * ux + uy * uy) + uz * uz);
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
  if (threadIdx.x == 0) {
    s.partial[2 * blockIdx.x] = s_e[0];
    s.partial[2 * blockIdx.x + 1] = s_k[0];
  }
}

// One block per replica: add the tile partials of replica r in tile order.
__global__ __launch_bounds__(256) void k_energy_reduce(Geometry g, State s, double* out) {
  __shared__ double s_e[256], s_k[256];
  const int r = blockIdx.x;
  double e = 0.0, k = 0.0;
  for (int b = threadIdx.x; b < g.n_atiles; b += 256) {
    const AtomTile tl = g.atiles[b];
    if (tl.rep == r && tl.count > 0) {
      e += s.partial[2 * b];
      k += s.partial[2 * b + 1];
    }
  }
  s_e[threadIdx.x] = e;
  s_k[threadIdx.x] = k;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s_e[threadIdx.x] += s_e[threadIdx.x + o];
      s_k[threadIdx.x] += s_k[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * r] = s_e[0];
    out[2 * r + 1] = s_k[0];
  }
}

// ============================================================ snapshots

// Save (restore = 0) or restore the current positions and velocities.  A
// save is skipped once an error is latched, so the snapshot stays the last
// clean state; the device step counter travels with it.
__global__ __launch_bounds__(256) void k_snapshot(State s, int64_t n, double4* __restrict__ sp,
                                                  double4* __restrict__ sv, int restore) {
  if (!restore && has_error(s.status)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (restore) *counter64(s.status, SW_STEPS) = *counter64(s.status, SW_SNAP_STEPS);
    else *counter64(s.status, SW_SNAP_STEPS) = *counter64(s.status, SW_STEPS);
  }
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (restore) {
      s.pos[k] = sp[k];
      s.vel[k] = sv[k];
    } else {
      sp[k] = s.pos[k];
      sv[k] = s.vel[k];
    }
  }
}

// ============================================================ launchers

static int grid_stride_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return (int)b;
}

hipError_t launch_import(const Launch& L, const Geometry& g, const State& s, const double* x,
                         const double* v) {
  hipLaunchKernelGGL(k_import, dim3(L.atile_blocks), dim3(64), 0, L.stream, g, s, x, v);
  return hipGetLastError();
}

hipError_t launch_zero_bins(const Launch& L, const State& s, int64_t n_cells_total) {
  hipLaunchKernelGGL(k_zero_i32, dim3(grid_stride_blocks(n_cells_total)), dim3(256), 0, L.stream,
                     s.bin_cnt, n_cells_total);
  return hipGetLastError();
}

hipError_t launch_bin(const Launch& L, const Geometry& g, const State& s, const int32_t* cond) {
  hipLaunchKernelGGL(k_bin, dim3(L.atile_blocks), dim3(64), 0, L.stream, g, s, cond);
  return hipGetLastError();
}

hipError_t launch_build(const Launch& L, const Geometry& g, const State& s, const int32_t* cond) {
  hipLaunchKernelGGL(k_build, dim3(L.ctile_blocks), dim3(kBuildBlock), 0, L.stream, g, s, cond);
  return hipGetLastError();
}

hipError_t launch_sort(const Launch& L, const Geometry& g, const State& s, int64_t m) {
  hipError_t e;
  if ((e = launch_zero_bins(L, s, m)) != hipSuccess) return e;
  if ((e = launch_bin(L, g, s, nullptr)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_cells, dim3(1), dim3(1024), 0, L.stream, s.bin_cnt, s.cell_start, m,
                     g.cell_cap);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, L.stream, s,
                     m, g.cell_cap);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_sort_copyback, dim3(grid_stride_blocks(g.n)), dim3(256), 0, L.stream, s,
                     g.n, m);
  return hipGetLastError();
}

template <int PREC>
static hipError_t density_lpa(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                              int lpa, double4* pos, const int32_t* cz, int32_t* cf, int64_t m,
                              int want) {
  switch (lpa) {
    case 1:
      hipLaunchKernelGGL((k_density<PREC, 1>), dim3(L.atile_blocks), dim3(64), 0, L.stream, g, s, t,
                         pos, cz, cf, m, want);
      break;
    case 2:
      hipLaunchKernelGGL((k_density<PREC, 2>), dim3(L.atile_blocks), dim3(128), 0, L.stream, g, s,
                         t, pos, cz, cf, m, want);
      break;
    case 4:
      hipLaunchKernelGGL((k_density<PREC, 4>), dim3(L.atile_blocks), dim3(256), 0, L.stream, g, s,
                         t, pos, cz, cf, m, want);
      break;
    default:
      hipLaunchKernelGGL((k_density<PREC, 8>), dim3(L.atile_blocks), dim3(512), 0, L.stream, g, s,
                         t, pos, cz, cf, m, want);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_density(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                          int precision, int lpa, const double4* pos, const int32_t* cond_zero,
                          int32_t* clear_flag, int64_t n_cells_total, bool want_rho) {
  double4* p = const_cast<double4*>(pos);
  if (precision == 0)
    return density_lpa<0>(L, g, s, t, lpa, p, cond_zero, clear_flag, n_cells_total, want_rho);
  return density_lpa<1>(L, g, s, t, lpa, p, cond_zero, clear_flag, n_cells_total, want_rho);
}

template <int PREC>
static hipError_t force_int_lpa(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                                int lpa, const double4* pi, double4* po, int32_t* fl) {
  switch (lpa) {
    case 1:
      hipLaunchKernelGGL((k_force_integrate<PREC, 1>), dim3(L.atile_blocks), dim3(64), 0, L.stream,
                         g, s, t, pi, po, fl);
      break;
    case 2:
      hipLaunchKernelGGL((k_force_integrate<PREC, 2>), dim3(L.atile_blocks), dim3(128), 0,
                         L.stream, g, s, t, pi, po, fl);
      break;
    case 4:
      hipLaunchKernelGGL((k_force_integrate<PREC, 4>), dim3(L.atile_blocks), dim3(256), 0,
                         L.stream, g, s, t, pi, po, fl);
      break;
    default:
      hipLaunchKernelGGL((k_force_integrate<PREC, 8>), dim3(L.atile_blocks), dim3(512), 0,
                         L.stream, g, s, t, pi, po, fl);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_force_integrate(const Launch& L, const Geometry& g, const State& s,
                                  const Tables& t, int precision, int lpa, const double4* pos_in,
                                  double4* pos_out, int32_t* flag_next) {
  if (precision == 0) return force_int_lpa<0>(L, g, s, t, lpa, pos_in, pos_out, flag_next);
  return force_int_lpa<1>(L, g, s, t, lpa, pos_in, pos_out, flag_next);
}

template <int PREC>
static hipError_t force_only_lpa(const Launch& L, const Geometry& g, const State& s,
                                 const Tables& t, int lpa, const double4* pos) {
  switch (lpa) {
    case 1:
      hipLaunchKernelGGL((k_force_only<PREC, 1>), dim3(L.atile_blocks), dim3(64), 0, L.stream, g,
                         s, t, pos);
      break;
    case 2:
      hipLaunchKernelGGL((k_force_only<PREC, 2>), dim3(L.atile_blocks), dim3(128), 0, L.stream, g,
                         s, t, pos);
      break;
    case 4:
      hipLaunchKernelGGL((k_force_only<PREC, 4>), dim3(L.atile_blocks), dim3(256), 0, L.stream, g,
                         s, t, pos);
      break;
    default:
      hipLaunchKernelGGL((k_force_only<PREC, 8>), dim3(L.atile_blocks), dim3(512), 0, L.stream, g,
                         s, t, pos);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_force_only(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                             int precision, int lpa, const double4* pos) {
  if (precision == 0) return force_only_lpa<0>(L, g, s, t, lpa, pos);
  return force_only_lpa<1>(L, g, s, t, lpa, pos);
}

hipError_t launch_halfkick(const Launch& L, const Geometry& g, const State& s, double scale) {
  hipLaunchKernelGGL(k_halfkick, dim3(L.atile_blocks), dim3(64), 0, L.stream, g, s, scale);
  return hipGetLastError();
}

hipError_t launch_energy(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                         double* out_pe_ke, int32_t n_rep) {
  // out_pe_ke: device [n_rep][2]; mass/ftm2v and the half-kick scale are in g
  const double mass_over = 1.0 / g.acc;  // m / ftm2v
  hipLaunchKernelGGL(k_energy_atoms, dim3(L.atile_blocks), dim3(64), 0, L.stream, g, s, t,
                     mass_over, 0.5 * g.dt * g.acc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_reduce, dim3(n_rep), dim3(256), 0, L.stream, g, s, out_pe_ke);
  return hipGetLastError();
}

hipError_t launch_export(const Launch& L, const Geometry& g, const State& s, double* x, double* v,
                         double* f, double* rho, double* fp, double vscale) {
  hipLaunchKernelGGL(k_export, dim3(L.atile_blocks), dim3(64), 0, L.stream, g, s, x, v, f, rho, fp,
                     vscale);
  return hipGetLastError();
}

hipError_t launch_export_cells(const Launch& L, const Geometry& g, const State& s, int32_t* cell) {
  hipLaunchKernelGGL(k_export_cells, dim3(L.atile_blocks), dim3(64), 0, L.stream, g, s, cell);
  return hipGetLastError();
}

hipError_t launch_export_nbrs(const Launch& L, const Geometry& g, const State& s, int32_t* cnt,
                              int32_t* nbr, int32_t cap_out) {
  hipLaunchKernelGGL(k_export_nbrs, dim3(L.atile_blocks), dim3(64), 0, L.stream, g, s, cnt, nbr,
                     cap_out);
  return hipGetLastError();
}

hipError_t launch_snapshot(const Launch& L, const Geometry& g, const State& s, double4* snap_pos,
                           double4* snap_vel, bool restore) {
  hipLaunchKernelGGL(k_snapshot, dim3(grid_stride_blocks(g.n)), dim3(256), 0, L.stream, s, g.n,
                     snap_pos, snap_vel, restore ? 1 : 0);
  return hipGetLastError();
}

}  // namespace mdk
