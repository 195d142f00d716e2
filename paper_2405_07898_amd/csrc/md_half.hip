// md_half.hip -- the pair passes with force symmetry (half list), float64.
//
// The paper evaluates every pair term on both atoms and projects a saving from
// using the symmetry of the pair interactions (Sec. VI-A).  Here each pair
// (i, j) with slot j > slot i is evaluated once, by atom i, and its value goes
// to a pair slot (k, i) (k = its position in i's half list).  A second pass
// gives every atom the values of the slots where it is the j side, read in
// ascending slot order; no float atomics are used, so every sum has a fixed
// order and results are bitwise repeatable.
//
//   density:  rho(r) of slot (k, i) -> pval;   rho_i = sum over own slots
//             + sum over reverse slots (Eq. density)
//   force:    f_ij = [(F'_i + F'_j) rho'(r) + phi'(r)] (x_j - x_i)/r -> qval;
//             F_i = sum over own slots f - sum over reverse slots f
//             (Eq. EAMforce; the pair force on j is exactly -f_ij)
//
// The half list and the reverse slots are derived from the full list after
// each rebuild, inside the density passes: the first pass splits each atom's
// list and scatters its pair slots to the partners (an integer counter per
// atom; the order of arrival varies), the second sorts each atom's reverse
// slots, which makes the order fixed.
#include "md_device.h"

#pragma clang fp contract(off)

namespace mdk {

namespace {

constexpr int kHalfThreads = 768;  // 12 waves, one atom per lane
constexpr int kHB = 4;             // list entries in flight per lane

// rho_i side jobs as in the full-list density pass: clear the next step's
// rebuild flags, zero the bins after a rebuild.  Then per atom i: split the
// full list (after a rebuild) and evaluate rho(r) of each own pair slot.
__global__ __launch_bounds__(kHalfThreads) void k_half_density(
    Geometry g, State s, Tables t, const double4* __restrict__ pos, const int32_t* cond,
    int force_reindex, int32_t* clear_flag, int32_t* rclear, int64_t ncells) {
  extern __shared__ double4 lds_d4[];
  const int32_t rebuilt = cond ? *cond : 0;
  const bool err = has_error(s.status);
  if (clear_flag && blockIdx.x == 0) {
    if (threadIdx.x == 0) *clear_flag = 0;
    for (int r = threadIdx.x; r < g.n_rep; r += blockDim.x) rclear[r] = 0;
  }
  lds_fill<4>(lds_d4, t.rho_val, t.nr - 1, lds_d4 + (t.nr - 1));
  if (rebuilt) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ncells;
         k += (int64_t)gridDim.x * blockDim.x)
      s.bin_cnt[k] = 0;
  }
  __syncthreads();
  if (err) return;
  const bool reindex = force_reindex || rebuilt;
  const size_t N = (size_t)g.n;
  const int cap = g.nbr_cap;
  const int last = t.nr - 2;
  const TileWalk w = tile_walk<1>();
  for (int64_t it = w.q;; it += w.tpi) {
    const int64_t b = walk_tile(it, g.n_atiles);
    if (b < 0) break;
    const AtomTile tl = g.atiles[b];
    if (w.a >= tl.count) continue;
    const RepDev& rp = g.reps[tl.rep];
    const int64_t i = tl.begin + w.a;
    if (reindex) {
      const int m = min(s.cnt[i], cap);
      int hc = 0;
      for (int k = 0; k < m; ++k) {
        const uint32_t e = s.nbr[(size_t)k * N + i];
        if ((e & kIndexMask) > (uint32_t)i) {
          s.hnbr[(size_t)hc * N + i] = e;
          ++hc;
        }
      }
      s.hcnt[i] = hc;
      // scatter the pair slots to the partners, kHB counters in flight
      for (int k0 = 0; k0 < hc; k0 += kHB) {
        uint32_t j[kHB];
        int32_t r[kHB];
#pragma unroll
        for (int u = 0; u < kHB; ++u)
          j[u] = (k0 + u < hc) ? (s.hnbr[(size_t)(k0 + u) * N + i] & kIndexMask) : 0u;
#pragma unroll
        for (int u = 0; u < kHB; ++u) r[u] = (k0 + u < hc) ? atomicAdd(&s.rfill[j[u]], 1) : cap;
        // at most cnt[j] <= cap arrivals unless the list overflowed (then the
        // step is rolled back); the guard keeps the store in bounds
#pragma unroll
        for (int u = 0; u < kHB; ++u)
          if (r[u] < cap)
            s.rslot_u[(size_t)r[u] * N + j[u]] = (uint32_t)((size_t)(k0 + u) * N + (size_t)i);
      }
    }
    const int hc = s.hcnt[i];
    const double4 pi = pos[i];
    double acc = 0.0;
    for (int k0 = 0; k0 < hc; k0 += kHB) {
      uint32_t e[kHB];
      double4 q[kHB];
#pragma unroll
      for (int u = 0; u < kHB; ++u)
        e[u] = (k0 + u < hc) ? s.hnbr[(size_t)(k0 + u) * N + i] : (uint32_t)i | (kNoShift << kIndexBits);
#pragma unroll
      for (int u = 0; u < kHB; ++u) q[u] = pos[e[u] & kIndexMask];
#pragma unroll
      for (int u = 0; u < kHB; ++u) {
        double dx, dy, dz;
        separation(e[u], rp, q[u].x, q[u].y, q[u].z, pi.x, pi.y, pi.z, dx, dy, dz);
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const bool in = (k0 + u < hc) && r2 < g.rc2;
        const double rr = in ? r2 : 1.0;
        const double x = (rr * rsq64(rr)) * t.r_inv_dx;
        const int kk = min(max((int)x, 0), last);
        const double tt = x - (double)kk;
        const double4 c = lds_d4[kk];
        const double v = in ? fma(fma(fma(c.w, tt, c.z), tt, c.y), tt, c.x) : 0.0;
        if (k0 + u < hc) s.pval[(size_t)(k0 + u) * N + i] = v;
        acc += v;
      }
    }
    s.own_rho[i] = acc;
  }
}

// Ascending sort of one atom's reverse slots (column stride N) with a bitonic
// network in registers; M is a power of two >= m, pads sort to the end.
template <int M>
__device__ __forceinline__ void sort_slots(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                           size_t N, int m) {
  uint32_t v[M];
#pragma unroll
  for (int p = 0; p < M; ++p) v[p] = (p < m) ? in[(size_t)p * N] : 0xffffffffu;
#pragma unroll
  for (int k = 2; k <= M; k <<= 1) {
#pragma unroll
    for (int h = k >> 1; h > 0; h >>= 1) {
#pragma unroll
      for (int p = 0; p < M; ++p) {
        const int l = p ^ h;
        if (l > p) {
          const uint32_t lo = min(v[p], v[l]), hi = max(v[p], v[l]);
          const bool up = (p & k) == 0;
          v[p] = up ? lo : hi;
          v[l] = up ? hi : lo;
        }
      }
    }
  }
#pragma unroll
  for (int p = 0; p < M; ++p)
    if (p < m) out[(size_t)p * N] = v[p];
}

// Per atom j: after a rebuild, sort its reverse slots and reset its counter;
// then rho_j = own sum + reverse slots in ascending order, and F'(rho_j) into
// pos[j].w.
__global__ __launch_bounds__(64) void k_half_rho_gather(Geometry g, State s, Tables t,
                                                        double4* __restrict__ pos,
                                                        const int32_t* cond, int force_reindex,
                                                        int want_rho) {
  const int32_t rebuilt = cond ? *cond : 0;
  if (has_error(s.status)) return;
  const AtomTile tl = g.atiles[blockIdx.x];
  if ((int)threadIdx.x >= tl.count) return;
  const int64_t j = tl.begin + threadIdx.x;
  const size_t N = (size_t)g.n;
  if (force_reindex || rebuilt) {
    const int m = min(s.rfill[j], g.nbr_cap);
    const uint32_t* in = s.rslot_u + j;
    uint32_t* out = s.rslot + j;
    if (m <= 16) {
      sort_slots<16>(in, out, N, m);
    } else if (m <= 32) {
      sort_slots<32>(in, out, N, m);
    } else if (m <= 64) {
      sort_slots<64>(in, out, N, m);
    } else {
      // longer columns: rank of each slot among them (slots are distinct, so
      // the ranks are a permutation)
      for (int p = 0; p < m; ++p) {
        const uint32_t a = in[(size_t)p * N];
        int r = 0;
        for (int q = 0; q < m; ++q) r += (in[(size_t)q * N] < a) ? 1 : 0;
        out[(size_t)r * N] = a;
      }
    }
    s.rcnt[j] = m;
    s.rfill[j] = 0;
  }
  const int m = s.rcnt[j];
  double rho = s.own_rho[j];
  int p = 0;
  for (; p + kHB <= m; p += kHB) {
    uint32_t sl[kHB];
#pragma unroll
    for (int u = 0; u < kHB; ++u) sl[u] = s.rslot[(size_t)(p + u) * N + j];
    double v[kHB];
#pragma unroll
    for (int u = 0; u < kHB; ++u) v[u] = s.pval[sl[u]];
#pragma unroll
    for (int u = 0; u < kHB; ++u) rho += v[u];
  }
  for (; p < m; ++p) rho += s.pval[s.rslot[(size_t)p * N + j]];
  // F'(rho_j): float64 embedding table, end-tangent continuation past its end
  const double xe = (rho - t.e_x0) * t.e_inv_dx;
  const int le = t.ne - 2;
  const int ke = (xe >= (double)le) ? le : ((xe > 0.0) ? (int)xe : 0);
  const double te = fmin(xe - (double)ke, 1.0);
  const double4 ce = t.emb_val[ke];
  pos[j].w = fma(fma(3.0 * ce.w, te, 2.0 * ce.z), te, ce.y) * t.e_inv_dx;
  if (want_rho) s.rho[j] = rho;
  if (xe > (double)(t.ne - 1)) set_bits(s.status, ST_RHO_RANGE);
}

// Per atom i: the pair force of each own slot (on i, towards j's side
// convention x_j - x_i) into qval, and their sum.
__global__ __launch_bounds__(kHalfThreads) void k_half_force(Geometry g, State s, Tables t,
                                                             const double4* __restrict__ pos) {
  extern __shared__ double4 lds_d4[];
  const bool err = has_error(s.status);
  double2* tab = reinterpret_cast<double2*>(lds_d4);
  lds_fill<8>(tab, t.dpair3, 3 * (t.nr - 1), tab + 3 * (t.nr - 1));
  __syncthreads();
  if (err) return;
  const size_t N = (size_t)g.n;
  const int last = t.nr - 2;
  const TileWalk w = tile_walk<1>();
  for (int64_t it = w.q;; it += w.tpi) {
    const int64_t b = walk_tile(it, g.n_atiles);
    if (b < 0) break;
    const AtomTile tl = g.atiles[b];
    if (w.a >= tl.count) continue;
    const RepDev& rp = g.reps[tl.rep];
    const int64_t i = tl.begin + w.a;
    const int hc = s.hcnt[i];
    const double4 pi = pos[i];
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int k0 = 0; k0 < hc; k0 += kHB) {
      uint32_t e[kHB];
      double4 q[kHB];
#pragma unroll
      for (int u = 0; u < kHB; ++u)
        e[u] = (k0 + u < hc) ? s.hnbr[(size_t)(k0 + u) * N + i] : (uint32_t)i | (kNoShift << kIndexBits);
#pragma unroll
      for (int u = 0; u < kHB; ++u) q[u] = pos[e[u] & kIndexMask];
#pragma unroll
      for (int u = 0; u < kHB; ++u) {
        double dx, dy, dz;
        separation(e[u], rp, q[u].x, q[u].y, q[u].z, pi.x, pi.y, pi.z, dx, dy, dz);
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const bool in = (k0 + u < hc) && r2 < g.rc2;
        const double rr = in ? r2 : 1.0;
        const double rinv = rsq64(rr);
        const double x = (rr * rinv) * t.r_inv_dx;
        const int kk = min(max((int)x, 0), last);
        const double tt = x - (double)kk;
        const double2 r0 = tab[3 * kk], r1 = tab[3 * kk + 1], r2v = tab[3 * kk + 2];
        // r0 = (rho'0, rho'1), r1 = (rho'2, phi'0), r2v = (phi'1, phi'2)
        const double drho = fma(fma(r1.x, tt, r0.y), tt, r0.x);
        const double dphi = fma(fma(r2v.y, tt, r2v.x), tt, r1.y);
        const double sc = in ? fma(pi.w + q[u].w, drho, dphi) * rinv : 0.0;
        const double fx = sc * dx, fy = sc * dy, fz = sc * dz;
        // one 32-byte record per slot: the gather reads one line per slot
        if (k0 + u < hc) s.qval[(size_t)(k0 + u) * N + i] = make_double4(fx, fy, fz, 0.0);
        ax += fx;
        ay += fy;
        az += fz;
      }
    }
    s.own_f[i] = make_double4(ax, ay, az, 0.0);
  }
}

// F_j = own sum - reverse slots in ascending order (a pair's force on its j
// side is minus the force on its i side).
__device__ __forceinline__ double3 gather_force(const Geometry& g, const State& s, int64_t j) {
  const size_t N = (size_t)g.n;
  const double4 o = s.own_f[j];
  double fx = o.x, fy = o.y, fz = o.z;
  const int m = s.rcnt[j];
  int p = 0;
  for (; p + kHB <= m; p += kHB) {
    uint32_t sl[kHB];
#pragma unroll
    for (int u = 0; u < kHB; ++u) sl[u] = s.rslot[(size_t)(p + u) * N + j];
    double4 q[kHB];
#pragma unroll
    for (int u = 0; u < kHB; ++u) q[u] = s.qval[sl[u]];
#pragma unroll
    for (int u = 0; u < kHB; ++u) {
      fx -= q[u].x;
      fy -= q[u].y;
      fz -= q[u].z;
    }
  }
  for (; p < m; ++p) {
    const double4 q = s.qval[s.rslot[(size_t)p * N + j]];
    fx -= q.x;
    fy -= q.y;
    fz -= q.z;
  }
  return make_double3(fx, fy, fz);
}

// Gather fused with the leap-frog update, as in the full-list force pass.
__global__ __launch_bounds__(64) void k_half_force_gather_integrate(
    Geometry g, State s, const double4* __restrict__ pos_in, double4* __restrict__ pos_out,
    int32_t* flag_next, int32_t* rflag_next) {
  if (has_error(s.status)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter64(s.status, SW_STEPS) += 1ull;
  const AtomTile tl = g.atiles[blockIdx.x];
  const bool active = (int)threadIdx.x < tl.count;
  bool far = false;
  if (active) {
    const int64_t j = tl.begin + threadIdx.x;
    const double4 pj = pos_in[j];
    double4 v = s.vel[j];
    const double4 xr = s.xref[j];
    const double3 f = gather_force(g, s, j);
    const double k = g.dt * g.acc;
    v.x = fma(k, f.x, v.x);
    v.y = fma(k, f.y, v.y);
    v.z = fma(k, f.z, v.z);
    double4 xn;
    xn.x = fma(g.dt, v.x, pj.x);
    xn.y = fma(g.dt, v.y, pj.y);
    xn.z = fma(g.dt, v.z, pj.z);
    xn.w = 0.0;
    pos_out[j] = xn;
    s.vel[j] = v;
    const double ex = xn.x - xr.x, ey = xn.y - xr.y, ez = xn.z - xr.z;
    const double d2 = fma(ex, ex, fma(ey, ey, ez * ez));
    far = !(d2 <= g.lim2);
    if (!isfinite(f.x + f.y + f.z) || !isfinite(xn.x + xn.y + xn.z))
      set_bits(s.status, ST_NONFINITE);
  }
  // a block is one atom tile, hence one replica
  if (__ballot(far) != 0ull && threadIdx.x == 0) {
    *flag_next = 1;
    rflag_next[tl.rep] = 1;
  }
}

__global__ __launch_bounds__(64) void k_half_force_gather_only(Geometry g, State s) {
  if (has_error(s.status)) return;
  const AtomTile tl = g.atiles[blockIdx.x];
  if ((int)threadIdx.x >= tl.count) return;
  const int64_t j = tl.begin + threadIdx.x;
  const double3 f = gather_force(g, s, j);
  s.frc[j] = make_double4(f.x, f.y, f.z, 0.0);
  if (!isfinite(f.x + f.y + f.z)) set_bits(s.status, ST_NONFINITE);
}

}  // namespace

hipError_t launch_half_density(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                               const double4* pos, const int32_t* cond, bool force_reindex,
                               int32_t* clear_flag, int32_t* rclear, int64_t n_cells_total,
                               bool want_rho) {
  const int fr = force_reindex ? 1 : 0;
  hipLaunchKernelGGL(k_half_density, dim3(2 * L.persist_blocks), dim3(kHalfThreads),
                     density_lds_bytes(t, 0), L.stream, g, s, t, pos, cond, fr, clear_flag,
                     rclear, n_cells_total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_half_rho_gather, dim3(L.atile_blocks), dim3(64), 0, L.stream, g, s, t,
                     const_cast<double4*>(pos), cond, fr, want_rho ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_half_force_integrate(const Launch& L, const Geometry& g, const State& s,
                                       const Tables& t, const double4* pos_in, double4* pos_out,
                                       int32_t* flag_next, int32_t* rflag_next) {
  hipLaunchKernelGGL(k_half_force, dim3(L.persist_blocks), dim3(kHalfThreads),
                     force_lds_bytes(t, 0), L.stream, g, s, t, pos_in);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_half_force_gather_integrate, dim3(L.atile_blocks), dim3(64), 0, L.stream,
                     g, s, pos_in, pos_out, flag_next, rflag_next);
  return hipGetLastError();
}

hipError_t launch_half_force_only(const Launch& L, const Geometry& g, const State& s,
                                  const Tables& t, const double4* pos) {
  hipLaunchKernelGGL(k_half_force, dim3(L.persist_blocks), dim3(kHalfThreads),
                     force_lds_bytes(t, 0), L.stream, g, s, t, pos);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_half_force_gather_only, dim3(L.atile_blocks), dim3(64), 0, L.stream, g, s);
  return hipGetLastError();
}

hipError_t allow_half_lds(const Tables& t) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_half_density),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)density_lds_bytes(t, 0));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_half_force),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)force_lds_bytes(t, 0));
}

}  // namespace mdk
