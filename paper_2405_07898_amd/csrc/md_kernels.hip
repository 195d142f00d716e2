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
// as fma(); the list build and binning evaluate each expression in the plain
// order of its definition (bit-identical cells and neighbour sets).
#include "md_device.h"

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

// Wrap into the replica's box in its periodic dimensions; open dimensions keep
// the coordinate.  `bad` becomes true for a non-finite coordinate or one still
// outside [0, L) in a periodic dimension (moved more than one box length).
__device__ __forceinline__ double4 wrap_pos(double4 p, const RepDev& rp, bool& bad) {
  double q[3] = {p.x, p.y, p.z};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const bool open = (rp.open >> d) & 1;
    if (!open) q[d] = wrap1(q[d], rp.box[d]);
    bad = bad || !isfinite(q[d]) || (!open && !(q[d] >= 0.0 && q[d] < rp.box[d]));
  }
  return make_double4(q[0], q[1], q[2], p.w);
}

// Fixed-point coordinate of the mixed form (RepDev::qinv): round to nearest,
// then the low 32 bits (the periodic wrap in a periodic dimension).
__device__ __forceinline__ uint32_t quantize(double x, double qinv) {
  return (uint32_t)(unsigned long long)__double2ll_rn(x * qinv);
}

// The mixed form's record of a position (F' slot cleared).
__device__ __forceinline__ uint4 pos_record(const RepDev& rp, double x, double y, double z) {
  return make_uint4(quantize(x, rp.qinv[0]), quantize(y, rp.qinv[1]), quantize(z, rp.qinv[2]),
                    0u);
}

// ============================================================ import / export

__global__ __launch_bounds__(64) void k_import(Geometry g, State s, const double* __restrict__ x,
                                               const double* __restrict__ v) {
  const AtomTile tl = g.atiles[blockIdx.x];
  if ((int)threadIdx.x >= tl.count) return;
  const RepDev& rp = g.reps[tl.rep];
  const int64_t i = tl.begin + threadIdx.x;
  bool bad = false;
  const double4 p =
      wrap_pos(make_double4(x[3 * i + 0], x[3 * i + 1], x[3 * i + 2], 0.0), rp, bad);
  if (bad) set_bits(s.status, ST_LOST);
  s.pos[i] = p;
  if (s.rec) s.rec[i] = pos_record(rp, p.x, p.y, p.z);
  s.vel[i] = v ? make_double4(v[3 * i + 0], v[3 * i + 1], v[3 * i + 2], 0.0)
               : make_double4(0.0, 0.0, 0.0, 0.0);
  s.id[i] = (int32_t)i;
  if (s.type) s.type[i] = s.type_orig[i];
}

__global__ __launch_bounds__(64) void k_export(Geometry g, State s, double* __restrict__ x,
                                               double* __restrict__ v, double* __restrict__ f,
                                               double* __restrict__ rho, double* __restrict__ fp,
                                               double coef) {
  const AtomTile tl = g.atiles[blockIdx.x];
  if ((int)threadIdx.x >= tl.count) return;
  const RepDev& rp = g.reps[tl.rep];
  const int64_t i = tl.begin + threadIdx.x;
  const int64_t o = s.id[i];
  const double4 p = s.pos[i];
  if (x) {
    bool bad = false;
    const double4 q = wrap_pos(p, rp, bad);
    x[3 * o + 0] = q.x;
    x[3 * o + 1] = q.y;
    x[3 * o + 2] = q.z;
  }
  const double4 fr = s.frc[i];
  if (v) {
    const double4 u = s.vel[i];
    const double vscale = coef * acc_of(g, s, i);
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
// Launched with a grid smaller than the tile count (workgroup b takes tiles
// b, b + G, ...), so that the launch that finds no rebuild due ends quickly.
__device__ __forceinline__ void bin_tile(const Geometry& g, const State& s, const AtomTile& tl,
                                         const int32_t* rcond, int a) {
  if (a >= tl.count) return;
  if (rcond && rcond[tl.rep] == 0) return;  // this replica keeps its list
  const RepDev& rp = g.reps[tl.rep];
  const int64_t i = tl.begin + a;
  bool bad = false;
  const double4 p = wrap_pos(s.pos[i], rp, bad);
  if (bad) {
    set_bits(s.status, ST_LOST);
    return;
  }
  s.pos[i] = p;
  s.xref[i] = p;
  if (s.rec) s.rec[i] = pos_record(rp, p.x, p.y, p.z);
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
  const int32_t cg = rp.cell0 + cl;
  // Atoms of a wave are mostly in a few cells (cell-sorted order): group the
  // lanes by cell, let one leader per cell reserve all their slots with one
  // atomic, and rank the others behind it.
  const int lane = lane_id();
  unsigned long long todo = __ballot(1);
  int leader = lane, rank = 0, count = 0;
  while (todo) {
    const int l = __builtin_ctzll(todo);
    const int32_t c0 = __shfl(cg, l, 64);
    const unsigned long long peers = __ballot(cg == c0) & todo;
    if (cg == c0) {
      leader = l;
      rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
    }
    if (lane == l) count = __popcll(peers);
    todo &= ~peers;
  }
  int base = 0;
  if (lane == leader) base = atomicAdd(&s.bin_cnt[cg], count);
  const int32_t slot = __shfl(base, leader, 64) + rank;
  if (slot < g.cell_cap) s.bin_idx[(int64_t)cg * g.cell_cap + slot] = (int32_t)i;
  else set_bits(s.status, ST_CELL_OVERFLOW);
}

__global__ __launch_bounds__(64) void k_bin(Geometry g, State s, const int32_t* cond,
                                            const int32_t* rcond) {
  // both words are read before either is tested: one memory latency, not two
  const int32_t due = cond ? *cond : 1;
  const bool err = has_error(s.status);
  if (due == 0 || err) return;
  if (cond && blockIdx.x == 0 && threadIdx.x == 0) *counter64(s.status, SW_REBUILDS) += 1ull;
  for (int b = blockIdx.x; b < g.n_atiles; b += gridDim.x)
    bin_tile(g, s, g.atiles[b], rcond, (int)threadIdx.x);
}

// ============================================================ list build

// One wave per cell.  The atoms of the 27 surrounding cells are gathered,
// each cell ordered by atom index (a deterministic candidate order,
// Sec. III-C), into registers: lane l holds candidates l, l+64, ... .  Every
// atom of the centre cell then tests all candidates against
// r^2 < (r_cut+skin)^2 and compacts the admitted ones with a ballot into its
// ELL row, each entry carrying its image shift.
//
// The shift of a candidate is that of its stencil cell (a wrapped cell index
// means one box length).  For every pair within the list radius this is the
// minimum image, and d = fma(s, L, x_j - x_i) rounds exactly like x_j - x_i
// followed by adding -L or +L, so the admitted set is bit-identical to that of
// the plain minimum-image rule; pairs at other images are farther than the
// list radius under either rule.
// Candidates staged per batch in the small-system node, whose 512-thread
// workgroups have registers to spare: at about 9 atoms per cell a stencil
// often holds more than kMaxStage, and a second batch doubles the cell's chain.
constexpr int kSmallStage = 384;

// LDS of one build workgroup; the centre-cell arrays are sized by the cell
// capacity at launch (dynamic shared memory).
struct BuildLds {
  int32_t* q;       // [27] global cell index of each stencil cell
  int32_t* n;       // [27] atoms in it (clamped to the capacity)
  int32_t* off;     // [28] exclusive prefix of n
  int32_t* code;    // [27] image code of the stencil cell
  int32_t* raw;     // [kMaxStage] staged candidate ids, bin order
  int32_t* idx;     // [kMaxStage] staged candidate ids, ordered per stencil cell
  int32_t* center;  // [cap] centre atoms in increasing id
  int32_t* base;    // [cap] list length so far of each centre atom
  double* cx;       // [cap] centre positions
  double* cy;
  double* cz;
  int8_t* cell;     // [kMaxStage] stencil cell of each staged slot
};

__host__ __device__ inline size_t build_lds_bytes(int ccap, int stage = kMaxStage) {
  return sizeof(int32_t) * (27 * 3 + 28 + 2 * (size_t)stage + 2 * (size_t)ccap) +
         sizeof(double) * 3 * (size_t)ccap + (size_t)stage;
}

__device__ __forceinline__ BuildLds carve_build_lds(char* p, int ccap, int stage = kMaxStage) {
  BuildLds L;
  // doubles first (8-byte aligned at the start of dynamic LDS)
  L.cx = reinterpret_cast<double*>(p);
  L.cy = L.cx + ccap;
  L.cz = L.cy + ccap;
  int32_t* w = reinterpret_cast<int32_t*>(L.cz + ccap);
  L.q = w;
  L.n = w + 27;
  L.code = w + 54;
  L.off = w + 81;
  L.raw = w + 109;
  L.idx = L.raw + stage;
  L.center = L.idx + stage;
  L.base = L.center + ccap;
  L.cell = reinterpret_cast<int8_t*>(L.base + ccap);
  return L;
}

// Synchronisation of the lanes that build one cell: the whole (one-wave)
// workgroup, or only the wave when several waves of a workgroup build
// different cells (LDS accesses of one wave are ordered by the fences).
template <bool kWave>
__device__ __forceinline__ void build_sync() {
  if (kWave) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Stencil cell `lane` (< 27) of cell c: its global index, image code and
// whether it lies past an open dimension's grid edge (then it is empty).
__device__ __forceinline__ void stencil_cell(const RepDev& rp, int32_t c, int lane, int32_t& q,
                                             int32_t& code, bool& outside) {
  const int32_t nx = rp.nc[0], ny = rp.nc[1], nz = rp.nc[2];
  const int32_t cx = c % nx, cy = (c / nx) % ny, cz = c / (nx * ny);
  const int dz = lane / 9 - 1, dy = (lane / 3) % 3 - 1, dx = lane % 3 - 1;
  const int32_t ux = cx + dx, uy = cy + dy, uz = cz + dz;
  // wrapped index below 0: candidate near L, shift -L (code 0); above: +L (code 2)
  uint32_t kx = ux < 0 ? 0u : (ux >= nx ? 2u : 1u);
  uint32_t ky = uy < 0 ? 0u : (uy >= ny ? 2u : 1u);
  uint32_t kz = uz < 0 ? 0u : (uz >= nz ? 2u : 1u);
  // an open dimension has no image: a stencil cell past its grid edge is empty
  outside = (((rp.open & 1) && kx != 1u) || ((rp.open & 2) && ky != 1u) ||
             ((rp.open & 4) && kz != 1u));
  if (rp.open & 1) kx = 1u;
  if (rp.open & 2) ky = 1u;
  if (rp.open & 4) kz = 1u;
  q = rp.cell0 + (((uz + nz) % nz) * ny + (uy + ny) % ny) * nx + (ux + nx) % nx;
  code = (int32_t)(kx | (ky << 2) | (kz << 4));
}

// Exclusive prefix of the 27 stencil counts (lane k holds n_k) into L.off.
template <bool kWave>
__device__ __forceinline__ void stencil_offsets(const BuildLds& L, int lane, int32_t n) {
  int32_t incl = n;
#pragma unroll
  for (int o = 1; o < 32; o <<= 1) {
    const int32_t t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane < 27) L.off[lane] = incl - n;
  if (lane == 26) L.off[27] = incl;
  build_sync<kWave>();
}

// Staged candidates p < T (ids in L.raw, stencil cell in L.cell) ordered by id
// within their stencil cell into L.idx.
template <bool kWave>
__device__ __forceinline__ void rank_stage(const BuildLds& L, int lane, int T, int base_off) {
  for (int p = lane; p < T; p += 64) {
    const int sc = L.cell[p];
    const int lo = L.off[sc] - base_off, nn = L.n[sc];
    const int32_t e = L.raw[p];
    int r = 0;
    for (int w = lo; w < lo + nn; ++w) r += (L.raw[w] < e);
    L.idx[lo + r] = e;
  }
  build_sync<kWave>();
}

// The distance tests of every centre atom against the staged candidates
// (positions px.., image shifts sx.., entries ent.. in registers, T of them),
// appending the admitted ones to the centre atoms' rows in candidate order.
template <int kC>
__device__ __forceinline__ void test_stage(const Geometry& g, const State& s, const RepDev& rp,
                                           const BuildLds& L, int lane, int T, int n_c,
                                           const double (&px)[kC], const double (&py)[kC],
                                           const double (&pz)[kC], const double (&sx)[kC],
                                           const double (&sy)[kC], const double (&sz)[kC],
                                           const uint32_t (&ent)[kC]) {
  const double Lx = rp.box[0], Ly = rp.box[1], Lz = rp.box[2];
  const double rl2 = g.rl2;
  const int64_t N = g.n;
  const int32_t cap = g.nbr_cap;
  for (int u = 0; u < n_c; ++u) {
    const int32_t i = L.center[u];
    const uint32_t self_e = (uint32_t)i | (kNoShift << kIndexBits);
    const double qx = L.cx[u], qy = L.cy[u], qz = L.cz[u];
    int base = L.base[u];
#pragma unroll
    for (int k = 0; k < kC; ++k) {
      if (k * 64 >= T) break;
      const double dx = fma(sx[k], Lx, px[k] - qx);
      const double dy = fma(sy[k], Ly, py[k] - qy);
      const double dz = fma(sz[k], Lz, pz[k] - qz);
      const double r2 = (dx * dx + dy * dy) + dz * dz;
      // the centre atom itself is the only candidate with its own id in the
      // centre cell (code kNoShift)
      const bool ok = ent[k] != self_e && r2 < rl2;
      const unsigned long long m = __ballot(ok);
      if (ok) {
        const uint32_t kk = (uint32_t)base + __builtin_amdgcn_mbcnt_hi(
                                 (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (kk < (uint32_t)cap) st32(s.nbr, (kk * (uint32_t)N + (uint32_t)i) * 4u, ent[k]);
      }
      base += __popcll(m);
    }
    if (lane == 0) L.base[u] = base;
  }
}

// List lengths of the centre atoms, and the cell's statistics and overflow checks.
__device__ __forceinline__ void finish_cell(const Geometry& g, const State& s, const BuildLds& L,
                                            int lane, int n_c, int32_t qc) {
  int32_t mx = 0;
  long long tot = 0;
  for (int u = lane; u < n_c; u += 64) {
    const int32_t b = L.base[u];
    s.cnt[L.center[u]] = b;
    mx = max(mx, b);
    tot += b;
  }
  mx = wave_max_i32(mx);
  tot = wave_sum_i64(tot);
  if (lane == 0) {
    // per-cell statistics (reduced on demand); the status word is only
    // touched in the rare overflow cases
    const int32_t full = s.bin_cnt[qc];
    s.cell_stat[3 * (int64_t)qc + 0] = mx;
    s.cell_stat[3 * (int64_t)qc + 1] = (int32_t)tot;
    s.cell_stat[3 * (int64_t)qc + 2] = full;
    if (mx > g.nbr_cap) set_bits(s.status, ST_NBR_OVERFLOW);
    if (full > g.cell_cap) set_bits(s.status, ST_CELL_OVERFLOW);
  }
}

// Candidate registers of stage slots p = k * 64 + lane (< T): position, image
// shift and list entry; empty slots sit infinitely far away (r^2 = inf fails).
template <int kC>
__device__ __forceinline__ void load_candidates(const State& s, const BuildLds& L, int lane, int T,
                                                double (&px)[kC], double (&py)[kC],
                                                double (&pz)[kC], double (&sx)[kC],
                                                double (&sy)[kC], double (&sz)[kC],
                                                uint32_t (&ent)[kC]) {
#pragma unroll
  for (int k = 0; k < kC; ++k) {
    const int p = k * 64 + lane;
    px[k] = py[k] = pz[k] = HUGE_VAL;
    sx[k] = sy[k] = sz[k] = 0.0;
    ent[k] = 0xffffffffu;
    if (p < T) {
      const int32_t j = L.idx[p];
      const uint32_t code = (uint32_t)L.code[L.cell[p]];
      const double4 q = s.pos[j];
      px[k] = q.x;
      py[k] = q.y;
      pz[k] = q.z;
      sx[k] = (double)((int)(code & 3u) - 1);
      sy[k] = (double)((int)((code >> 2) & 3u) - 1);
      sz[k] = (double)((int)(code >> 4) - 1);
      ent[k] = (uint32_t)j | (code << kIndexBits);
    }
  }
}

// The list rows of one cell's atoms: every atom of the 27 stencil cells is a
// candidate (Sec. III-C: the candidate filter), admitted when r^2 < (r_c +
// skin)^2 under the stencil cell's image shift; rows in stencil-cell order,
// by id within a cell.  The stencil's candidates are staged in batches of at
// most kStage (the batches do not change the rows).
template <bool kWave, int kStage = kMaxStage>
__device__ __forceinline__ void build_cell(const Geometry& g, const State& s, const CellTile& ct,
                                           const BuildLds& L, int lane) {
  const RepDev& rp = g.reps[ct.rep];
  const int32_t ccap = g.cell_cap;
  // stencil cells: lane k < 27 owns cell k (z-major, then y, then x)
  int32_t n = 0;
  if (lane < 27) {
    int32_t q, code;
    bool outside;
    stencil_cell(rp, ct.cell, lane, q, code, outside);
    n = outside ? 0 : min(s.bin_cnt[q], ccap);
    L.q[lane] = q;
    L.n[lane] = n;
    L.code[lane] = code;
  }
  stencil_offsets<kWave>(L, lane, n);
  // centre atoms in increasing index, with their positions
  const int32_t qc = L.q[13], n_c = L.n[13];
  for (int u = lane; u < n_c; u += 64) L.raw[u] = s.bin_idx[(int64_t)qc * ccap + u];
  build_sync<kWave>();
  for (int u = lane; u < n_c; u += 64) {
    const int32_t e = L.raw[u];
    int r = 0;
    for (int w = 0; w < n_c; ++w) r += (L.raw[w] < e);
    const double4 q = s.pos[e];
    L.center[r] = e;
    L.base[r] = 0;
    L.cx[r] = q.x;
    L.cy[r] = q.y;
    L.cz[r] = q.z;
  }
  build_sync<kWave>();
  int s0 = 0;
  while (s0 < 27) {
    // the largest run of stencil cells whose candidates fit the stage (one
    // cell always fits: the capacity is at most kMaxStage)
    int s1 = s0 + 1;
    while (s1 < 27 && L.off[s1 + 1] - L.off[s0] <= kStage) ++s1;
    const int base_off = L.off[s0];
    const int T = L.off[s1] - base_off;
    // each stencil cell's lane marks its slots, then every lane loads its slots
    if (lane >= s0 && lane < s1) {
      const int lo = L.off[lane] - base_off;
      for (int w = 0; w < n; ++w) L.cell[lo + w] = (int8_t)lane;
    }
    build_sync<kWave>();
    for (int p = lane; p < T; p += 64) {
      const int sc = L.cell[p];
      L.raw[p] = s.bin_idx[(int64_t)L.q[sc] * ccap + (p + base_off - L.off[sc])];
    }
    build_sync<kWave>();
    rank_stage<kWave>(L, lane, T, base_off);
    // candidates into registers (L.cell is per stencil cell, unchanged by the sort)
    constexpr int kC = kStage / 64;
    double px[kC], py[kC], pz[kC];
    double sx[kC], sy[kC], sz[kC];
    uint32_t ent[kC];
    load_candidates<kC>(s, L, lane, T, px, py, pz, sx, sy, sz, ent);
    test_stage<kC>(g, s, rp, L, lane, T, n_c, px, py, pz, sx, sy, sz, ent);
    build_sync<kWave>();
    s0 = s1;
  }
  finish_cell(g, s, L, lane, n_c, qc);
}

// Launched with a grid smaller than the cell count (workgroup b takes cell
// tiles b, b + G, ...; G is a multiple of the XCD count, so every tile stays on
// the XCD the tile table placed it on).  The register budget asks for six
// waves per SIMD: the build is latency-bound, and the few spilled registers
// cost less than the lost occupancy (measured: 330 us against 435 us at
// 802k atoms).
__global__ __launch_bounds__(64, 6) void k_build(Geometry g, State s, const int32_t* cond,
                                              const int32_t* rcond) {
  const int32_t due = cond ? *cond : 1;
  const bool err = has_error(s.status);
  if (due == 0 || err) return;
  extern __shared__ double build_lds_raw[];
  const BuildLds lds = carve_build_lds(reinterpret_cast<char*>(build_lds_raw), g.cell_cap);
  for (int b = blockIdx.x; b < g.n_ctiles; b += gridDim.x) {
    const CellTile ct = g.ctiles[b];
    if (ct.cell < 0) continue;
    if (rcond && rcond[ct.rep] == 0) continue;  // this replica keeps its list
    build_cell<false>(g, s, ct, lds, (int)threadIdx.x);
    __syncthreads();  // the next cell reuses the staging arrays
  }
}

// Fixed-order reduction of the per-cell build statistics into the status
// block (longest list, fullest cell, total list entries).
__global__ __launch_bounds__(1024) void k_cell_stats(State s, int64_t m) {
  __shared__ int32_t s_mx[1024], s_mc[1024];
  __shared__ long long s_tot[1024];
  int32_t mx = 0, mc = 0;
  long long tot = 0;
  for (int64_t c = threadIdx.x; c < m; c += 1024) {
    mx = max(mx, s.cell_stat[3 * c + 0]);
    tot += s.cell_stat[3 * c + 1];
    mc = max(mc, s.cell_stat[3 * c + 2]);
  }
  s_mx[threadIdx.x] = mx;
  s_mc[threadIdx.x] = mc;
  s_tot[threadIdx.x] = tot;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s_mx[threadIdx.x] = max(s_mx[threadIdx.x], s_mx[threadIdx.x + o]);
      s_mc[threadIdx.x] = max(s_mc[threadIdx.x], s_mc[threadIdx.x + o]);
      s_tot[threadIdx.x] += s_tot[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    s.status[SW_MAX_LIST] = s_mx[0];
    s.status[SW_MAX_CELL] = s_mc[0];
    *counter64(s.status, SW_LIST_TOTAL) = (unsigned long long)s_tot[0];
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
// positions, velocities and ids into the sorted scratch arrays.  A binning
// that overflowed a cell or lost an atom (error latched) places fewer than n
// atoms: then neither this kernel nor the copy-back moves anything, and the
// slot order stays as it was.
__global__ __launch_bounds__(256) void k_sort_scatter(State s, int64_t m, int32_t cap) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= m || has_error(s.status)) return;
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
    if (s.type) s.sort_type[base + r] = s.type[e];
    if (s.rec) s.sort_rec[base + r] = s.rec[e];
  }
}

__global__ __launch_bounds__(256) void k_sort_copyback(State s, int64_t n, int64_t m) {
  // a failed binning (error latched, or fewer than n atoms placed) moves nothing
  const bool moved = !has_error(s.status) && s.cell_start[m] == (int32_t)n;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; moved && k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    s.pos[k] = s.sort_pos[k];
    s.vel[k] = s.sort_vel[k];
    s.id[k] = s.sort_id[k];
    if (s.type) s.type[k] = s.sort_type[k];
    if (s.rec) s.rec[k] = s.sort_rec[k];
  }
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m;
       k += (int64_t)gridDim.x * blockDim.x)
    s.bin_cnt[k] = 0;
}

// ============================================================ density pass


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


// Neighbours are processed in batches of kBatch per lane: the list entries of
// a batch are loaded together, then all their positions, then all their table
// rows, so each batch pays the position -> table latency chain once; the list
// entries of the next batch are requested while a batch is in flight.

// rho_i of one atom (its lane's share), table rows from LDS.  Each batch
// loads kBatch list entries, then their positions, then table rows.

// One list entry's density term: float64 from the gathered position (x, y
// in qxy, z in qz), mixed from the fixed-point records.
__device__ __forceinline__ void dens_term64(const Geometry& g, const Tables& t, const RepDev& rp,
                                            const void* lds_tab, uint32_t e, bool v, double2 qxy,
                                            double qz, double2 pxy, double pz, double& acc) {
  double dx, dy, dz;
  separation(e, rp, qxy.x, qxy.y, qz, pxy.x, pxy.y, pz, dx, dy, dz);
  const double4* tab = reinterpret_cast<const double4*>(lds_tab);
  const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
  const bool in = v && r2 < g.rc2;
  const double rr = in ? r2 : 1.0;
  const double x = (rr * rsq64(rr)) * t.r_inv_dx;
  const int kk = min(max((int)x, 0), t.nr - 2);
  const double tt = x - (double)kk;
  const double4 c = tab[kk];
  if (in) acc += fma(fma(fma(c.w, tt, c.z), tt, c.y), tt, c.x);
}

__device__ __forceinline__ void dens_term32(const Geometry& g, const Tables& t, const RepDev& rp,
                                            const void* lds_tab, bool v, uint4 qr, uint4 qi,
                                            float& sum, float& comp) {
  const float4* tab = reinterpret_cast<const float4*>(lds_tab);
  // separation from the fixed-point records (int32 wrap-around gives the
  // minimum image, the listed one for every list pair)
  const float fx = (float)(int32_t)(qr.x - qi.x) * rp.qs[0];
  const float fy = (float)(int32_t)(qr.y - qi.y) * rp.qs[1];
  const float fz = (float)(int32_t)(qr.z - qi.z) * rp.qs[2];
  const float r2 = fmaf(fx, fx, fmaf(fy, fy, fz * fz));
  const bool in = v && r2 < g.rc2f;
  const float rr = in ? r2 : 1.0f;
  const float x = (rr * __builtin_amdgcn_rsqf(rr)) * t.r_inv_dx32;
  const int kk = min(max((int)x, 0), t.nr - 2);
  const float tt = x - (float)kk;
  const float4 c = tab[kk];
  if (in) two_sum_acc(sum, comp, fmaf(fmaf(fmaf(c.w, tt, c.z), tt, c.y), tt, c.x));
}

// The list entries k0, k0 + LPA, ... (below m) of atom i's density sum, in
// batches of kBatch entries, added to this lane's sum in list order.
template <int PREC, int LPA>
__device__ __forceinline__ void density_from(const Geometry& g, const State& s, const Tables& t,
                                             const RepDev& rp, const double4* __restrict__ pos,
                                             const void* lds_tab, int64_t i, int k_first, int m,
                                             double2 pxy, double pz, uint4 qi, double& acc,
                                             float& sum, float& comp) {
  const uint32_t N = (uint32_t)g.n;
  const uint32_t self_e = (uint32_t)i | (kNoShift << kIndexBits);
  const double2* __restrict__ pos2 = reinterpret_cast<const double2*>(pos);
  const double* __restrict__ posd = reinterpret_cast<const double*>(pos);
  // the next batch's list entries are requested before this batch's
  // positions are used, so the list latency hides behind the gather
  const int kstep = LPA * kBatch;
  uint32_t e[kBatch];
  load_entries<LPA>(s.nbr, N, (uint32_t)i, k_first, m, self_e, e);
  for (int k0 = k_first; k0 < m; k0 += kstep) {
    double2 qxy[kBatch];
    double qz[kBatch];
    uint4 qr[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      if (PREC == 0) {
        const uint32_t off = (e[u] & kIndexMask) * 32u;
        qxy[u] = ld32(pos2, off);
        qz[u] = ld32(posd, off + 16u);
      } else {
        qr[u] = ld32(s.rec, (e[u] & kIndexMask) * 16u);
      }
    }
    uint32_t en[kBatch];
    load_entries<LPA>(s.nbr, N, (uint32_t)i, k0 + kstep, m, self_e, en);
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const bool v = k0 + u * LPA < m;
      if (PREC == 0) dens_term64(g, t, rp, lds_tab, e[u], v, qxy[u], qz[u], pxy, pz, acc);
      else dens_term32(g, t, rp, lds_tab, v, qr[u], qi, sum, comp);
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) e[u] = en[u];
  }
}

template <int PREC, int LPA>
__device__ __forceinline__ double density_end(double acc, float sum, float comp) {
  if (PREC == 0) return lane_sum_sym<LPA>(acc);
  lane_sum2<LPA>(sum, comp);
  return (double)sum + (double)comp;
}

// rho_i of one atom (its lane's share), table rows from LDS.
template <int PREC, int LPA>
__device__ __forceinline__ double density_of(const Geometry& g, const State& s, const Tables& t,
                                             const RepDev& rp, const double4* __restrict__ pos,
                                             const void* lds_tab, int64_t i, bool active,
                                             int sub) {
  const int m = active ? min(s.cnt[i], g.nbr_cap) : 0;
  double2 pxy = make_double2(0.0, 0.0);
  double pz = 0.0;
  uint4 qi = make_uint4(0u, 0u, 0u, 0u);
  if (PREC == 0) {
    pxy = *reinterpret_cast<const double2*>(&pos[i]);
    pz = pos[i].z;
  } else {
    qi = s.rec[i];
  }
  double acc = 0.0;
  float sum = 0.0f, comp = 0.0f;
  density_from<PREC, LPA>(g, s, t, rp, pos, lds_tab, i, sub, m, pxy, pz, qi, acc, sum, comp);
  return density_end<PREC, LPA>(acc, sum, comp);
}

// F'(rho_i) from the embedding table (float64 for both forms; the mixed form
// rounds it to float32, the precision its force pass gathers).  Past the last
// knot F continues along its end tangent: F' = F'(end); beyond_range is set
// when rho_i passes the table's end.
template <int PREC>
__device__ __forceinline__ double fprime_of(const Tables& t, double rho_i, bool& beyond_range) {
  const double xe = (rho_i - t.e_x0) * t.e_inv_dx;
  const int le = t.ne - 2;
  const int ke = (xe >= (double)le) ? le : ((xe > 0.0) ? (int)xe : 0);
  const double te = fmin(xe - (double)ke, 1.0);
  const double4 ce = t.emb_val[ke];
  double fp = fma(fma(3.0 * ce.w, te, 2.0 * ce.z), te, ce.y) * t.e_inv_dx;
  if (PREC != 0) fp = (double)(float)fp;
  beyond_range = xe > (double)(t.ne - 1);
  return fp;
}

// F'(rho_i) into pos[i].w; the mixed form also into its record's fourth word
// (float32), which the force pass gathers with the fixed-point position.
template <int PREC>
__device__ __forceinline__ void store_fprime(const State& s, const Tables& t, double4* pos,
                                             int64_t i, double rho_i, int want_rho) {
  bool beyond = false;
  const double fp = fprime_of<PREC>(t, rho_i, beyond);
  if (PREC != 0) s.rec[i].w = __float_as_uint((float)fp);
  pos[i].w = fp;
  if (want_rho) s.rho[i] = rho_i;
  if (beyond) set_bits(s.status, ST_RHO_RANGE);
}

// rho_i = sum_{j in list, r^2 < rc^2} rho(r_ij); F'_i stored in pos[i].w.
// Side jobs used inside the step graph: clear the next step's rebuild flag,
// and zero the bins after a rebuild (cond_zero set).
template <int PREC, int LPA>
__global__ __launch_bounds__(768) void k_density(Geometry g, State s, Tables t,
                                                  double4* __restrict__ pos,
                                                  const int32_t* cond_zero, int32_t* clear_flag,
                                                  int32_t* rclear, int64_t ncells, int want_rho) {
  extern __shared__ double4 lds_d4[];
  // both control words are read before either is used (one memory latency),
  // and the table is loaded while they arrive; the error test is uniform
  const int32_t zero_bins = cond_zero ? *cond_zero : 0;
  const bool err = has_error(s.status);
  if (clear_flag && blockIdx.x == 0) {
    if (threadIdx.x == 0) *clear_flag = 0;
    for (int r = threadIdx.x; r < g.n_rep; r += blockDim.x) rclear[r] = 0;
  }
  if (PREC == 0) lds_fill<4>(lds_d4, t.rho_val, t.nr - 1, lds_d4 + (t.nr - 1));
  else
    lds_fill<4>(reinterpret_cast<float4*>(lds_d4), t.rho_val32, t.nr - 1,
                reinterpret_cast<float4*>(lds_d4) + (t.nr - 1));
  if (zero_bins) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ncells;
         k += (int64_t)gridDim.x * blockDim.x)
      s.bin_cnt[k] = 0;
  }
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
    const double rho_i = density_of<PREC, LPA>(g, s, t, rp, pos, lds_d4, i, active, w.sub);
    if (!active || w.sub != 0) continue;
    store_fprime<PREC>(s, t, pos, i, rho_i, want_rho);
  }
}

// ============================================================ force pass

// F_i = sum_j [(F'_i + F'_j) rho'(r) + phi'(r)] (x_j - x_i)/r   (Eq. EAMforce),
// derivative rows from LDS (float64: 3 double2 per segment; mixed: float4 +
// float2 arrays).  Same batching as the density pass.

// One list entry's force term: float64 from the gathered record q (position
// and F'_j) and the atom's own pi (position and F'_i); mixed from the
// fixed-point records, F'_i = fpi.
__device__ __forceinline__ void force_term64(const Geometry& g, const Tables& t, const RepDev& rp,
                                             const void* lds_tab, uint32_t e, bool v, double4 q,
                                             double4 pi, double& ax, double& ay, double& az) {
  double dx, dy, dz;
  separation(e, rp, q.x, q.y, q.z, pi.x, pi.y, pi.z, dx, dy, dz);
  const double2* tab = reinterpret_cast<const double2*>(lds_tab);
  const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
  const bool in = v && r2 < g.rc2;
  const double rr = in ? r2 : 1.0;
  const double rinv = rsq64(rr);
  const double x = (rr * rinv) * t.r_inv_dx;
  const int kk = min(max((int)x, 0), t.nr - 2);
  const double tt = x - (double)kk;
  const double2 r0 = tab[3 * kk], r1 = tab[3 * kk + 1], r2v = tab[3 * kk + 2];
  // r0 = (rho'0, rho'1), r1 = (rho'2, phi'0), r2v = (phi'1, phi'2)
  const double drho = fma(fma(r1.x, tt, r0.y), tt, r0.x);
  const double dphi = fma(fma(r2v.y, tt, r2v.x), tt, r1.y);
  const double sc = fma(pi.w + q.w, drho, dphi) * rinv;
  if (in) {
    ax = fma(sc, dx, ax);
    ay = fma(sc, dy, ay);
    az = fma(sc, dz, az);
  }
}

struct MixedForce {
  float sx = 0.f, cx = 0.f, sy = 0.f, cy = 0.f, sz = 0.f, cz = 0.f;
};

__device__ __forceinline__ void force_term32(const Geometry& g, const Tables& t, const RepDev& rp,
                                             const void* lds_tab, bool v, uint4 qr, uint4 qi,
                                             float fpi, MixedForce& a) {
  const float4* ta = reinterpret_cast<const float4*>(lds_tab);
  const float2* tb = reinterpret_cast<const float2*>(ta + (t.nr - 1));
  // separation from the fixed-point difference: int32 wrap-around gives
  // the minimum image, which is the listed image for every list pair
  const float ex = (float)(int32_t)(qr.x - qi.x) * rp.qs[0];
  const float ey = (float)(int32_t)(qr.y - qi.y) * rp.qs[1];
  const float ez = (float)(int32_t)(qr.z - qi.z) * rp.qs[2];
  const float r2 = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
  const bool in = v && r2 < g.rc2f;
  const float rr = in ? r2 : 1.0f;
  const float rinv = __builtin_amdgcn_rsqf(rr);
  const float x = (rr * rinv) * t.r_inv_dx32;
  const int kk = min(max((int)x, 0), t.nr - 2);
  const float tt = x - (float)kk;
  const float4 A = ta[kk];
  const float2 B = tb[kk];
  const float drho = fmaf(fmaf(A.z, tt, A.y), tt, A.x);
  const float dphi = fmaf(fmaf(B.y, tt, B.x), tt, A.w);
  const float sc = fmaf(fpi + __uint_as_float(qr.w), drho, dphi) * rinv;
  if (in) {
    two_sum_acc(a.sx, a.cx, sc * ex);
    two_sum_acc(a.sy, a.cy, sc * ey);
    two_sum_acc(a.sz, a.cz, sc * ez);
  }
}

// The list entries k0, k0 + LPA, ... (below m) of atom i's force sum, in
// batches, added to this lane's sums in list order.
template <int PREC, int LPA>
__device__ __forceinline__ void forces_from(const Geometry& g, const State& s, const Tables& t,
                                            const RepDev& rp, const double4* __restrict__ pos,
                                            const void* lds_tab, int64_t i, int k_first, int m,
                                            double4 pi, uint4 qi, double& ax, double& ay,
                                            double& az, MixedForce& mf) {
  const uint32_t N = (uint32_t)g.n;
  const uint32_t self_e = (uint32_t)i | (kNoShift << kIndexBits);
  const float fpi = PREC == 0 ? 0.0f : __uint_as_float(qi.w);
  constexpr int kB = PREC == 0 ? kBatch : kBatchMixed;
  const int kstep = LPA * kB;
  uint32_t e[kB];
  load_entries<LPA>(s.nbr, N, (uint32_t)i, k_first, m, self_e, e);
  for (int k0 = k_first; k0 < m; k0 += kstep) {
    double4 q[kB];
    uint4 qr[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      if (PREC == 0) q[u] = ld32(pos, (e[u] & kIndexMask) * 32u);
      else qr[u] = ld32(s.rec, (e[u] & kIndexMask) * 16u);
    }
    uint32_t en[kB];
    load_entries<LPA>(s.nbr, N, (uint32_t)i, k0 + kstep, m, self_e, en);
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const bool v = k0 + u * LPA < m;
      if (PREC == 0) force_term64(g, t, rp, lds_tab, e[u], v, q[u], pi, ax, ay, az);
      else force_term32(g, t, rp, lds_tab, v, qr[u], qi, fpi, mf);
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) e[u] = en[u];
  }
}

template <int PREC, int LPA>
__device__ __forceinline__ void forces_end(double ax, double ay, double az, MixedForce& mf,
                                           double& fx, double& fy, double& fz) {
  if (PREC == 0) {
    fx = lane_sum_sym<LPA>(ax);
    fy = lane_sum_sym<LPA>(ay);
    fz = lane_sum_sym<LPA>(az);
  } else {
    lane_sum2<LPA>(mf.sx, mf.cx);
    lane_sum2<LPA>(mf.sy, mf.cy);
    lane_sum2<LPA>(mf.sz, mf.cz);
    fx = (double)mf.sx + (double)mf.cx;
    fy = (double)mf.sy + (double)mf.cy;
    fz = (double)mf.sz + (double)mf.cz;
  }
}

template <int PREC, int LPA>
__device__ __forceinline__ void pair_forces(const Geometry& g, const State& s, const Tables& t,
                                            const RepDev& rp, const double4* __restrict__ pos,
                                            const void* lds_tab, int64_t i, bool active, int sub,
                                            double4 pi, double& fx, double& fy, double& fz) {
  const int m = active ? min(s.cnt[i], g.nbr_cap) : 0;
  double ax = 0.0, ay = 0.0, az = 0.0;
  MixedForce mf;
  // mixed form: the atom's own record (fixed-point position, F' in float32)
  const uint4 qi = PREC == 0 ? make_uint4(0u, 0u, 0u, 0u) : s.rec[i];
  forces_from<PREC, LPA>(g, s, t, rp, pos, lds_tab, i, sub, m, pi, qi, ax, ay, az, mf);
  forces_end<PREC, LPA>(ax, ay, az, mf, fx, fy, fz);
}

template <int PREC>
__device__ __forceinline__ void fill_force_table(void* lds, const Tables& t) {
  if (PREC == 0) {
    double2* d = reinterpret_cast<double2*>(lds);
    lds_fill<8>(d, t.dpair3, 3 * (t.nr - 1), d + 3 * (t.nr - 1));
  } else {
    float4* ta = reinterpret_cast<float4*>(lds);
    float2* tb = reinterpret_cast<float2*>(ta + (t.nr - 1));
    lds_fill<2>(ta, t.dpair_a32, t.nr - 1, tb + (t.nr - 1));
    lds_fill<2>(tb, t.dpair_b32, t.nr - 1, tb + (t.nr - 1));
  }
}

// Leap-frog kick and drift (Eq. leapfrog): v <- v + dt F ftm2v/m, returns
// x' = x + dt v (w = 0).
__device__ __forceinline__ double4 kick_drift(const Geometry& g, double4 pi, double4& v, double fx,
                                              double fy, double fz) {
  const double k = g.dt * g.acc;
  v.x = fma(k, fx, v.x);
  v.y = fma(k, fy, v.y);
  v.z = fma(k, fz, v.z);
  double4 xn;
  xn.x = fma(g.dt, v.x, pi.x);
  xn.y = fma(g.dt, v.y, pi.y);
  xn.z = fma(g.dt, v.z, pi.z);
  xn.w = 0.0;
  return xn;
}

// Whether x' moved more than skin/2 from the last list build (also true for
// NaN); raises ST_NONFINITE on a non-finite force or position.
__device__ __forceinline__ bool moved_far(const Geometry& g, const State& s, double4 xn, double4 xr,
                                          double fx, double fy, double fz) {
  const double ex = xn.x - xr.x, ey = xn.y - xr.y, ez = xn.z - xr.z;
  const double d2 = fma(ex, ex, fma(ey, ey, ez * ez));
  if (!isfinite(fx + fy + fz) || !isfinite(xn.x + xn.y + xn.z)) set_bits(s.status, ST_NONFINITE);
  return !(d2 <= g.lim2);
}

// Leap-frog update of atom i from its force into pos_out and vel; returns
// whether it moved more than skin/2 since the last list build.
__device__ __forceinline__ bool leapfrog(const Geometry& g, const State& s, const RepDev& rp,
                                         int64_t i, double4 pi, double4 v, double4 xr, double fx,
                                         double fy, double fz, double4* __restrict__ pos_out) {
  const double4 xn = kick_drift(g, pi, v, fx, fy, fz);
  pos_out[i] = xn;
  // the mixed form's record goes with the position (pos_out is always the
  // other buffer of s)
  if (s.rec) s.rec_alt[i] = pos_record(rp, xn.x, xn.y, xn.z);
  s.vel[i] = v;
  return moved_far(g, s, xn, xr, fx, fy, fz);
}

// Force pass fused with the leap-frog update (Eq. leapfrog):
//   v <- v + dt F ftm2v/m ; x' <- x + dt v ; flag a rebuild if |x' - x_ref| > skin/2.
// Positions ping-pong between two buffers (neighbours read pos_in while the
// new positions go to pos_out).
template <int PREC, int LPA>
__global__ __launch_bounds__(PREC == 0 ? 768 : 1024) void k_force_integrate(
    Geometry g, State s, Tables t, const double4* __restrict__ pos_in,
    double4* __restrict__ pos_out, int32_t* flag_next, int32_t* rflag_next) {
  extern __shared__ double4 lds_d4[];
  // the status word arrives while the table loads (the test is uniform)
  const bool err = has_error(s.status);
  fill_force_table<PREC>(lds_d4, t);
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
    // own-atom state needed after the pair loop, fetched up front
    double4 v = make_double4(0.0, 0.0, 0.0, 0.0), xr = v;
    if (active && w.sub == 0) {
      v = s.vel[i];
      xr = s.xref[i];
    }
    double fx, fy, fz;
    pair_forces<PREC, LPA>(g, s, t, rp, pos_in, lds_d4, i, active, w.sub, pi, fx, fy, fz);
    bool far = false;
    if (active && w.sub == 0) far = leapfrog(g, s, rp, i, pi, v, xr, fx, fy, fz, pos_out);
    // one wave covers atoms of one tile, hence of one replica
    if (__ballot(far) != 0ull && lane_id() == 0) {
      *flag_next = 1;
      rflag_next[tl.rep] = 1;
    }
  }
}

// Forces only (no integration), into s.frc.
template <int PREC, int LPA>
__global__ __launch_bounds__(PREC == 0 ? 768 : 1024) void k_force_only(Geometry g, State s,
                                                                        Tables t,
                                                                        const double4* __restrict__ pos) {
  extern __shared__ double4 lds_d4[];
  const bool err = has_error(s.status);
  fill_force_table<PREC>(lds_d4, t);
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
    pair_forces<PREC, LPA>(g, s, t, rp, pos, lds_d4, i, active, w.sub, pi, fx, fy, fz);
    if (active && w.sub == 0) {
      s.frc[i] = make_double4(fx, fy, fz, 0.0);
      if (!isfinite(fx + fy + fz)) set_bits(s.status, ST_NONFINITE);
    }
  }
}

// ============================================================ per-replica schedules

// Batched replicas of very different sizes may each want their own lanes per
// atom.  These kernels walk pair tiles instead of atom tiles: wave w of a
// workgroup takes the workgroup's pair tiles w, w + W, w + 2W, ... (W waves),
// and works on each with the tile's own lanes per atom (a wave-uniform
// branch into the same device code as the uniform kernels, so a replica's
// results depend only on its own lanes-per-atom value).

template <int PREC, int LPA>
__device__ __forceinline__ void density_tile(const Geometry& g, const State& s, const Tables& t,
                                             double4* pos, const void* lds, const PairTile& tl,
                                             int lane, int want_rho) {
  const int a = lane / LPA, sub = lane % LPA;
  const bool active = a < tl.count;
  const int64_t i = tl.begin + (active ? a : 0);
  const double rho_i = density_of<PREC, LPA>(g, s, t, g.reps[tl.rep], pos, lds, i, active, sub);
  if (active && sub == 0) store_fprime<PREC>(s, t, pos, i, rho_i, want_rho);
}

template <int PREC>
__global__ __launch_bounds__(768) void k_density_dyn(Geometry g, State s, Tables t,
                                                      double4* __restrict__ pos,
                                                      const int32_t* cond_zero, int32_t* clear_flag,
                                                      int32_t* rclear, int64_t ncells, int want_rho) {
  extern __shared__ double4 lds_d4[];
  const int32_t zero_bins = cond_zero ? *cond_zero : 0;
  const bool err = has_error(s.status);
  if (clear_flag && blockIdx.x == 0) {
    if (threadIdx.x == 0) *clear_flag = 0;
    for (int r = threadIdx.x; r < g.n_rep; r += blockDim.x) rclear[r] = 0;
  }
  if (PREC == 0) lds_fill<4>(lds_d4, t.rho_val, t.nr - 1, lds_d4 + (t.nr - 1));
  else
    lds_fill<4>(reinterpret_cast<float4*>(lds_d4), t.rho_val32, t.nr - 1,
                reinterpret_cast<float4*>(lds_d4) + (t.nr - 1));
  if (zero_bins) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ncells;
         k += (int64_t)gridDim.x * blockDim.x)
      s.bin_cnt[k] = 0;
  }
  __syncthreads();
  if (err) return;
  const int nw = (int)blockDim.x >> 6, wave = (int)threadIdx.x >> 6, lane = lane_id();
  for (int64_t it = wave;; it += nw) {
    const int64_t b = walk_tile(it, g.n_ptiles);
    if (b < 0) break;
    const PairTile tl = g.ptiles[b];
    switch (tl.lpa) {
      case 1: density_tile<PREC, 1>(g, s, t, pos, lds_d4, tl, lane, want_rho); break;
      case 2: density_tile<PREC, 2>(g, s, t, pos, lds_d4, tl, lane, want_rho); break;
      case 4: density_tile<PREC, 4>(g, s, t, pos, lds_d4, tl, lane, want_rho); break;
      default: density_tile<PREC, 8>(g, s, t, pos, lds_d4, tl, lane, want_rho); break;
    }
  }
}

// Forces of one pair tile; with pos_out, the leap-frog update as in
// k_force_integrate (returns whether this wave saw an atom move past skin/2),
// else the forces into s.frc as in k_force_only.
template <int PREC, int LPA>
__device__ __forceinline__ bool force_tile(const Geometry& g, const State& s, const Tables& t,
                                           const double4* __restrict__ pos_in,
                                           double4* __restrict__ pos_out, const void* lds,
                                           const PairTile& tl, int lane) {
  const int a = lane / LPA, sub = lane % LPA;
  const bool active = a < tl.count;
  const int64_t i = tl.begin + (active ? a : 0);
  const double4 pi = pos_in[i];
  double4 v = make_double4(0.0, 0.0, 0.0, 0.0), xr = v;
  if (pos_out && active && sub == 0) {
    v = s.vel[i];
    xr = s.xref[i];
  }
  double fx, fy, fz;
  pair_forces<PREC, LPA>(g, s, t, g.reps[tl.rep], pos_in, lds, i, active, sub, pi, fx, fy, fz);
  bool far = false;
  if (active && sub == 0) {
    if (pos_out) {
      far = leapfrog(g, s, g.reps[tl.rep], i, pi, v, xr, fx, fy, fz, pos_out);
    } else {
      s.frc[i] = make_double4(fx, fy, fz, 0.0);
      if (!isfinite(fx + fy + fz)) set_bits(s.status, ST_NONFINITE);
    }
  }
  return __ballot(far) != 0ull;
}

// pos_out null: forces only (into s.frc); else force pass fused with the
// leap-frog update, as k_force_integrate.
template <int PREC>
__global__ __launch_bounds__(PREC == 0 ? 768 : 1024) void k_force_dyn(
    Geometry g, State s, Tables t, const double4* __restrict__ pos_in,
    double4* __restrict__ pos_out, int32_t* flag_next, int32_t* rflag_next) {
  extern __shared__ double4 lds_d4[];
  const bool err = has_error(s.status);
  fill_force_table<PREC>(lds_d4, t);
  __syncthreads();
  if (err) return;
  if (pos_out && blockIdx.x == 0 && threadIdx.x == 0) *counter64(s.status, SW_STEPS) += 1ull;
  const int nw = (int)blockDim.x >> 6, wave = (int)threadIdx.x >> 6, lane = lane_id();
  for (int64_t it = wave;; it += nw) {
    const int64_t b = walk_tile(it, g.n_ptiles);
    if (b < 0) break;
    const PairTile tl = g.ptiles[b];
    bool far;
    switch (tl.lpa) {
      case 1: far = force_tile<PREC, 1>(g, s, t, pos_in, pos_out, lds_d4, tl, lane); break;
      case 2: far = force_tile<PREC, 2>(g, s, t, pos_in, pos_out, lds_d4, tl, lane); break;
      case 4: far = force_tile<PREC, 4>(g, s, t, pos_in, pos_out, lds_d4, tl, lane); break;
      default: far = force_tile<PREC, 8>(g, s, t, pos_in, pos_out, lds_d4, tl, lane); break;
    }
    // one wave covers atoms of one pair tile, hence of one replica
    if (far && lane == 0) {
      *flag_next = 1;
      rflag_next[tl.rep] = 1;
    }
  }
}

// ============================================================ persistent steps

// Grid barrier of a cooperative launch (every workgroup is resident): one
// arrival counter and a generation word.  The last workgroup to arrive reads
// the status word and publishes whether to stop (an error was latched during
// the phase), so all workgroups leave the step loop at the same barrier.  The
// wait is bounded: past kBarrierSpins polls the workgroup raises ST_STALL and
// stops, and so, in turn, do the others.  Release/acquire at agent scope make
// the phase's global writes of every XCD visible after the barrier.
constexpr long long kBarrierSpins = 4000000;

// LDS of the density table (rows plus the fill's junk rows), 16-byte aligned.
__host__ __device__ inline size_t density_table_bytes(int nr, int prec) {
  const size_t b = (size_t)(nr - 1) * (prec == 0 ? sizeof(double4) : sizeof(float4)) + kLdsJunkBytes;
  return (b + 15) & ~size_t(15);
}

// LDS of the force table (rows plus the fill's junk rows), 16-byte aligned.
__host__ __device__ inline size_t persist_table_bytes(int nr, int prec) {
  const size_t b = (size_t)(nr - 1) * (prec == 0 ? 3 * sizeof(double2)
                                                 : sizeof(float4) + sizeof(float2)) +
                   kLdsJunkBytes;
  return (b + 15) & ~size_t(15);
}

// Barrier of all workgroups of a persistent launch (an arrival counter, a
// generation word and the last arrival's stop decision, all accessed only by
// atomics; the wait is bounded).  Each thread's stores have completed before
// its workgroup arrives, and the spin polls with relaxed loads: one fence on
// each side per workgroup, not one per poll.  The workgroups may sit on
// different XCDs, whose L2 caches are not coherent with each other, so the
// arrival writes this XCD's L2 back and the departure invalidates it
// (agent-scope release / acquire).
__device__ bool grid_sync(int32_t* status) {
  const int32_t np = (int32_t)gridDim.x;
  __shared__ int32_t s_go;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    int32_t* count = status + SW_BAR_COUNT;
    int32_t* gen = status + SW_BAR_GEN;
    int32_t* stop = status + SW_BAR_STOP;
    const int32_t g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);  // the generation is read before the arrival counts
    const int32_t arrived =
        __hip_atomic_fetch_add(count, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int32_t go = 1;
    if (arrived == np - 1) {
      const int32_t bits = __hip_atomic_load(status + SW_BITS, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
      go = (bits & ST_ERR_MASK) ? 0 : 1;
      __hip_atomic_store(count, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(stop, go ? 0 : 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_s_waitcnt(0);  // counter and decision are in place before the release
      __hip_atomic_store(gen, g0 + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long long spins = 0;
      while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
        if (++spins > kBarrierSpins) {
          set_bits(status, ST_STALL);
          go = -1;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (go > 0) go = __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 0 : 1;
    }
    // invalidates this CU's L1 and the clean lines of the L2 (an invalidation
    // at workgroup scope leaves the L1 alone in a dispatch whose workgroups
    // are not split over CUs)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __builtin_amdgcn_s_waitcnt(0);  // the invalidation is done before any wave reads on
    s_go = go > 0;
  }
  __syncthreads();
  return s_go != 0;
}

// The XCD this wave runs on (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ int xcd_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15;
}

// Table position of the it-th atom tile that participant pid of np takes
// (positions pid, pid + np, ...), or -1 when it has none left.
__device__ __forceinline__ int64_t walk_tile_of(int64_t it, int64_t n_tiles, int32_t pid,
                                                int32_t np) {
  const int64_t b = pid + (int64_t)np * it;
  return b < n_tiles ? b : -1;
}

// nsteps whole steps in one cooperative launch (small systems, where graph
// node launches dominate): per step, when the previous step flagged it,
// binning, barrier, list build, barrier; then density, barrier, force pass
// fused with the leap-frog update, barrier.  The phases are the device code of
// the per-phase kernels (same arithmetic, same order: results are bitwise
// those of the graph path).  The force table stays in the LDS for the whole
// launch; the density rows are read from global memory; each wave builds its
// own cells with its own staging area.  s0 / s1: the state with buffer 0 / 1
// current; nsteps is even, so buffer 0 is current again at the end.
template <int PREC, int LPA>
__global__ __launch_bounds__(kPersistThreads) void k_persist(Geometry g, State s0, State s1,
                                                             Tables t, int32_t nsteps,
                                                             int64_t ncells) {
  extern __shared__ double4 lds_d4[];
  fill_force_table<PREC>(lds_d4, t);
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int nwaves = (int)blockDim.x >> 6;
  const size_t bl = (build_lds_bytes(g.cell_cap) + 15) & ~size_t(15);
  char* build_base = reinterpret_cast<char*>(lds_d4) + persist_table_bytes(t.nr, PREC);
  const BuildLds L = carve_build_lds(build_base + (size_t)wave * bl, g.cell_cap);
  const void* dens_tab = PREC == 0 ? static_cast<const void*>(t.rho_val)
                                   : static_cast<const void*>(t.rho_val32);
  int32_t* status = s0.status;
  // the first barrier also publishes one decision on errors latched before the launch
  if (!grid_sync(status)) return;
  const int32_t pid = (int32_t)blockIdx.x, np = (int32_t)gridDim.x;
  const int64_t gstride = (int64_t)np * nwaves;
  const int64_t gwave = (int64_t)pid * nwaves + wave;
  const int tpi = (int)blockDim.x / (64 * LPA);
  for (int32_t step = 0; step < nsteps; ++step) {
    const int k = step & 1;
    const State& s = k ? s1 : s0;
    int32_t* fl_cur = status + (k == 0 ? SW_FLAG0 : SW_FLAG1);
    int32_t* fl_nxt = status + (k == 0 ? SW_FLAG1 : SW_FLAG0);
    const int32_t* rf_cur = s.rflag + (k == 0 ? 0 : g.n_rep);
    int32_t* rf_nxt = s.rflag + (k == 0 ? g.n_rep : 0);
    // written with plain stores before the last barrier: read past the L1
    const bool rebuild =
        __hip_atomic_load(fl_cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0;
    if (rebuild) {
      if (pid == 0 && threadIdx.x == 0) *counter64(status, SW_REBUILDS) += 1ull;
      for (int64_t b = gwave; b < g.n_atiles; b += gstride) bin_tile(g, s, g.atiles[b], rf_cur, lane);
      if (!grid_sync(status)) return;
      for (int64_t b = gwave; b < g.n_ctiles; b += gstride) {
        const CellTile ct = g.ctiles[b];
        if (ct.cell < 0 || rf_cur[ct.rep] == 0) continue;
        build_cell<true>(g, s, ct, L, lane);
        build_sync<true>();  // the wave's next cell reuses its staging arrays
      }
      if (!grid_sync(status)) return;
    }
    // density pass; side jobs: zero the bins after a rebuild, clear the next
    // step's rebuild flags
    if (rebuild) {
      for (int64_t c = pid * (int64_t)blockDim.x + threadIdx.x; c < ncells;
           c += (int64_t)np * blockDim.x)
        s.bin_cnt[c] = 0;
    }
    if (pid == 0) {
      if (threadIdx.x == 0) *fl_nxt = 0;
      for (int r = threadIdx.x; r < g.n_rep; r += blockDim.x) rf_nxt[r] = 0;
    }
    {
      const TileWalk w = tile_walk<LPA>();
      for (int64_t it = w.q;; it += tpi) {
        const int64_t b = walk_tile_of(it, g.n_atiles, pid, np);
        if (b < 0) break;
        const AtomTile tl = g.atiles[b];
        const bool active = w.a < tl.count;
        const RepDev& rp = g.reps[tl.rep];
        const int64_t i = tl.begin + (active ? w.a : 0);
        const double rho_i =
            density_of<PREC, LPA>(g, s, t, rp, s.pos, dens_tab, i, active, w.sub);
        if (!active || w.sub != 0) continue;
        store_fprime<PREC>(s, t, s.pos, i, rho_i, 0);
      }
    }
    if (!grid_sync(status)) return;
    // force pass fused with the leap-frog update, into the other buffer
    if (pid == 0 && threadIdx.x == 0) *counter64(status, SW_STEPS) += 1ull;
    {
      const TileWalk w = tile_walk<LPA>();
      for (int64_t it = w.q;; it += tpi) {
        const int64_t b = walk_tile_of(it, g.n_atiles, pid, np);
        if (b < 0) break;
        const AtomTile tl = g.atiles[b];
        const bool active = w.a < tl.count;
        const RepDev& rp = g.reps[tl.rep];
        const int64_t i = tl.begin + (active ? w.a : 0);
        const double4 pi = s.pos[i];
        double4 v = make_double4(0.0, 0.0, 0.0, 0.0), xr = v;
        if (active && w.sub == 0) {
          v = s.vel[i];
          xr = s.xref[i];
        }
        double fx, fy, fz;
        pair_forces<PREC, LPA>(g, s, t, rp, s.pos, lds_d4, i, active, w.sub, pi, fx, fy, fz);
        bool far = false;
        if (active && w.sub == 0) far = leapfrog(g, s, rp, i, pi, v, xr, fx, fy, fz, s.pos_alt);
        if (__ballot(far) != 0ull && lane_id() == 0) {
          *fl_nxt = 1;
          rf_nxt[tl.rep] = 1;
        }
      }
    }
    if (!grid_sync(status)) return;
  }
}

// Barrier of the np participants of a persistent launch (np <= kMaxSlots):
// participant p publishes the barrier's sequence number e in its slot of
// parity e & 1, and wave 0 of each workgroup polls all np slots at once until
// every one holds e.  No participant gets more than one barrier ahead of the
// slowest, so a parity's slots are not rewritten while anyone still reads
// them.  Each arrival carries whether the participant saw an error latched (its
// own set_bits completed before it reads the status word), so every
// participant reads the same slots and takes the same decision.  kWriteBack:
// the L2 is written back before the arrival (needed when the participants'
// next phase communicates through atomics, which this barrier does not assume
// to meet the plain stores in the L2).  The departure invalidates the CU's L1
// and the clean L2 lines; all participants run on one XCD, whose L2 keeps the
// dirty lines of the phase just ended.  The slots start at zero (cleared by
// the host before the launch).
template <bool kWriteBack>
__device__ bool slot_sync(int32_t* status, int32_t pid, int32_t np, int32_t& epoch) {
  __shared__ int32_t s_go;
  ++epoch;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x < 64) {
    int32_t* slot = status + SW_SLOTS + kMaxSlots * (epoch & 1);
    if (threadIdx.x == 0) {
      if (kWriteBack) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const int32_t bits =
          __hip_atomic_load(status + SW_BITS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(slot + pid, 2 * epoch + ((bits & ST_ERR_MASK) ? 1 : 0), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    const int l = (int)threadIdx.x;
    long long spins = 0;
    bool stall = false;
    int32_t v = 2 * epoch;
    while (true) {
      v = l < np ? __hip_atomic_load(slot + l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                 : 2 * epoch;
      if (__all((v >> 1) >= epoch)) break;
      if (++spins > kBarrierSpins) {
        stall = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    const bool err = __any((v & 1) != 0);
    if (threadIdx.x == 0) {
      if (stall) set_bits(status, ST_STALL);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __builtin_amdgcn_s_waitcnt(0);
      s_go = !(stall || err);
    }
  }
  __syncthreads();
  return s_go != 0;
}

// List entries per lane that the small-system step kernel keeps in registers.
constexpr int kRegEntries = 8;

// Whole steps of a small system in one launch on one XCD, every thread owning
// one (atom, lane) slot for the whole launch (the host checks that the atom
// tiles fit the participants at once).  Each lane keeps its atom's position
// and F', velocity, list length and first kRegEntries list entries in
// registers across steps (reloaded after a rebuild), so a pass is the
// neighbour gathers, the table rows and one store; the density and force
// passes share the entries.  Phases, their device code and the order of every
// sum are those of k_persist and of the per-phase kernels: results are bitwise
// those of the graph path.  Every lane of an atom computes the same update
// (the lane sums are symmetric), and lane 0 of the atom stores it.
template <int PREC, int LPA>
__global__ __launch_bounds__(kPersistThreads) void k_persist_small(Geometry g, State s0,
                                                                   State s1, Tables t,
                                                                   int32_t nsteps,
                                                                   int64_t ncells) {
  extern __shared__ double4 lds_d4[];
  __shared__ int32_t s_ticket;
  fill_force_table<PREC>(lds_d4, t);
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int nwaves = (int)blockDim.x >> 6;
  const size_t bl = (build_lds_bytes(g.cell_cap) + 15) & ~size_t(15);
  char* build_base = reinterpret_cast<char*>(lds_d4) + persist_table_bytes(t.nr, PREC);
  const BuildLds L = carve_build_lds(build_base + (size_t)wave * bl, g.cell_cap);
  const void* dens_tab = PREC == 0 ? static_cast<const void*>(t.rho_val)
                                   : static_cast<const void*>(t.rho_val32);
  int32_t* status = s0.status;
  if (threadIdx.x == 0)
    s_ticket = xcd_id() == 0
                   ? __hip_atomic_fetch_add(status + SW_XCD_TICKET, 1, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT)
                   : -1;
  // every workgroup meets once (full fences), then those not on XCD 0 leave
  if (!grid_sync(status)) return;
  if (s_ticket < 0) return;
  const int32_t pid = s_ticket;
  const int32_t np =
      __hip_atomic_load(status + SW_XCD_TICKET, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int32_t epoch = 0;
  // every atom tile needs a thread of XCD 0 (the host sized the grid for the
  // round-robin placement of workgroups over the XCDs); the test is uniform
  const int tpi = (int)blockDim.x / (64 * LPA);
  if (np > kMaxSlots || g.n_atiles > (int64_t)np * tpi) {
    if (pid == 0 && threadIdx.x == 0) set_bits(status, ST_PLACEMENT);
    return;
  }
  const int64_t gstride = (int64_t)np * nwaves;
  const int64_t gwave = (int64_t)pid * nwaves + wave;
  // this thread's atom slot
  const TileWalk w = tile_walk<LPA>();
  const int64_t tb = walk_tile_of(w.q, g.n_atiles, pid, np);
  const bool has = tb >= 0;
  const AtomTile tl = g.atiles[has ? tb : 0];
  const bool active = has && w.a < tl.count;
  const RepDev& rp = g.reps[tl.rep];
  const int64_t i = tl.begin + (active ? w.a : 0);
  const uint32_t N = (uint32_t)g.n;
  const uint32_t self_e = (uint32_t)i | (kNoShift << kIndexBits);
  // registers carried across steps
  int m = 0;
  uint32_t e[kRegEntries];
  double4 pi, v = make_double4(0.0, 0.0, 0.0, 0.0), xr = v;
  uint4 qi = make_uint4(0u, 0u, 0u, 0u);
  auto load_own = [&](const State& s) {
    pi = s.pos[i];
    if (PREC != 0) qi = s.rec[i];
  };
  auto load_list = [&](const State& s) {
    m = active ? min(s.cnt[i], g.nbr_cap) : 0;
    load_entries<LPA>(s.nbr, N, (uint32_t)i, w.sub, m, self_e, e);
    xr = s.xref[i];
  };
  load_own(s0);
  load_list(s0);
  v = s0.vel[i];
  for (int32_t step = 0; step < nsteps; ++step) {
    const int k = step & 1;
    const State& s = k ? s1 : s0;
    int32_t* fl_cur = status + (k == 0 ? SW_FLAG0 : SW_FLAG1);
    int32_t* fl_nxt = status + (k == 0 ? SW_FLAG1 : SW_FLAG0);
    const int32_t* rf_cur = s.rflag + (k == 0 ? 0 : g.n_rep);
    int32_t* rf_nxt = s.rflag + (k == 0 ? g.n_rep : 0);
    const bool rebuild =
        __hip_atomic_load(fl_cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0;
    if (rebuild) {
      // the bins' zeroing reaches memory before the binning's atomics, and
      // their counts before the build reads them
      if (!slot_sync<true>(status, pid, np, epoch)) return;
      if (pid == 0 && threadIdx.x == 0) *counter64(status, SW_REBUILDS) += 1ull;
      for (int64_t b = gwave; b < g.n_atiles; b += gstride) bin_tile(g, s, g.atiles[b], rf_cur, lane);
      if (!slot_sync<true>(status, pid, np, epoch)) return;
      for (int64_t b = gwave; b < g.n_ctiles; b += gstride) {
        const CellTile ct = g.ctiles[b];
        if (ct.cell < 0 || rf_cur[ct.rep] == 0) continue;
        build_cell<true>(g, s, ct, L, lane);
        build_sync<true>();  // the wave's next cell reuses its staging arrays
      }
      if (!slot_sync<false>(status, pid, np, epoch)) return;
      // the binning wrapped the positions; the build moved the reference ones
      load_own(s);
      load_list(s);
    }
    // density pass; side jobs: zero the bins after a rebuild, clear the next
    // step's rebuild flags
    if (rebuild) {
      for (int64_t c = pid * (int64_t)blockDim.x + threadIdx.x; c < ncells;
           c += (int64_t)np * blockDim.x)
        s.bin_cnt[c] = 0;
    }
    if (pid == 0) {
      if (threadIdx.x == 0) *fl_nxt = 0;
      for (int r = threadIdx.x; r < g.n_rep; r += blockDim.x) rf_nxt[r] = 0;
    }
    if (has) {
      double acc = 0.0;
      float sum = 0.0f, comp = 0.0f;
      {
        double2 qxy[kRegEntries];
        double qz[kRegEntries];
        uint4 qr[kRegEntries];
        const double2* pos2 = reinterpret_cast<const double2*>(s.pos);
        const double* posd = reinterpret_cast<const double*>(s.pos);
#pragma unroll
        for (int u = 0; u < kRegEntries; ++u) {
          if (PREC == 0) {
            const uint32_t off = (e[u] & kIndexMask) * 32u;
            qxy[u] = ld32(pos2, off);
            qz[u] = ld32(posd, off + 16u);
          } else {
            qr[u] = ld32(s.rec, (e[u] & kIndexMask) * 16u);
          }
        }
#pragma unroll
        for (int u = 0; u < kRegEntries; ++u) {
          const bool ok = w.sub + u * LPA < m;
          if (PREC == 0)
            dens_term64(g, t, rp, dens_tab, e[u], ok, qxy[u], qz[u],
                        make_double2(pi.x, pi.y), pi.z, acc);
          else dens_term32(g, t, rp, dens_tab, ok, qr[u], qi, sum, comp);
        }
      }
      if (w.sub + kRegEntries * LPA < m)
        density_from<PREC, LPA>(g, s, t, rp, s.pos, dens_tab, i, w.sub + kRegEntries * LPA, m,
                                make_double2(pi.x, pi.y), pi.z, qi, acc, sum, comp);
      const double rho_i = density_end<PREC, LPA>(acc, sum, comp);
      bool beyond = false;
      const double fp = fprime_of<PREC>(t, rho_i, beyond);
      pi.w = fp;
      if (PREC != 0) qi.w = __float_as_uint((float)fp);
      if (active && w.sub == 0) {
        if (PREC != 0) s.rec[i].w = qi.w;
        s.pos[i].w = fp;
        if (beyond) set_bits(s.status, ST_RHO_RANGE);
      }
    }
    if (!slot_sync<false>(status, pid, np, epoch)) return;
    // force pass fused with the leap-frog update, into the other buffer
    if (pid == 0 && threadIdx.x == 0) *counter64(status, SW_STEPS) += 1ull;
    if (has) {
      double ax = 0.0, ay = 0.0, az = 0.0;
      MixedForce mf;
      {
        double4 q[kRegEntries];
        uint4 qr[kRegEntries];
#pragma unroll
        for (int u = 0; u < kRegEntries; ++u) {
          if (PREC == 0) q[u] = ld32(s.pos, (e[u] & kIndexMask) * 32u);
          else qr[u] = ld32(s.rec, (e[u] & kIndexMask) * 16u);
        }
        const float fpi = PREC == 0 ? 0.0f : __uint_as_float(qi.w);
#pragma unroll
        for (int u = 0; u < kRegEntries; ++u) {
          const bool ok = w.sub + u * LPA < m;
          if (PREC == 0) force_term64(g, t, rp, lds_d4, e[u], ok, q[u], pi, ax, ay, az);
          else force_term32(g, t, rp, lds_d4, ok, qr[u], qi, fpi, mf);
        }
      }
      if (w.sub + kRegEntries * LPA < m)
        forces_from<PREC, LPA>(g, s, t, rp, s.pos, lds_d4, i, w.sub + kRegEntries * LPA, m, pi,
                               qi, ax, ay, az, mf);
      double fx, fy, fz;
      forces_end<PREC, LPA>(ax, ay, az, mf, fx, fy, fz);
      bool far = false;
      if (active) {
        const double4 xn = kick_drift(g, pi, v, fx, fy, fz);
        if (w.sub == 0) {
          s.pos_alt[i] = xn;
          if (PREC != 0) s.rec_alt[i] = pos_record(rp, xn.x, xn.y, xn.z);
          s.vel[i] = v;
          far = moved_far(g, s, xn, xr, fx, fy, fz);
        }
        pi = xn;
        if (PREC != 0) qi = pos_record(rp, xn.x, xn.y, xn.z);
      }
      if (__ballot(far) != 0ull && lane_id() == 0) {
        *fl_nxt = 1;
        rf_nxt[tl.rep] = 1;
      }
    }
    if (!slot_sync<false>(status, pid, np, epoch)) return;
  }
}

// Binning, list build and density pass of a step in one launch, for systems
// small enough that grid barriers between the phases are cheaper than graph
// nodes (a node costs a few microseconds even when it only finds no rebuild
// due, and in most steps none is).  When the step's rebuild flag is set:
// binning, barrier, list build, barrier (then the bins are cleared); in every
// step: the density pass and F'.  The phases are the device code of k_bin,
// k_build and k_density (results are bitwise theirs) and the barrier is the
// persistent kernel's bounded one.  The density rows sit in the LDS beside
// the build's per-wave staging.  The grid never exceeds the workgroups that fit
// on the chip at once (checked when the context is created).  Side jobs as in
// k_density: clear the next step's rebuild flags.
template <int PREC, int LPA>
__global__ __launch_bounds__(kPersistThreads) void k_bin_build_density(
    Geometry g, State s, Tables t, const int32_t* cond, const int32_t* rcond,
    int32_t* clear_flag, int32_t* rclear, int64_t ncells) {
  extern __shared__ double4 lds_d4[];
  // the rebuild flag is written only by earlier kernels, so every workgroup
  // reads the same value; the status word is not (an error raised by the
  // binning of one workgroup may or may not be seen by another at its start),
  // so the barriers' last arrivals decide for all whether to go on
  const int32_t due = cond ? *cond : 1;
  const bool err = has_error(s.status);
  if (clear_flag && blockIdx.x == 0) {
    if (threadIdx.x == 0) *clear_flag = 0;
    for (int r = threadIdx.x; r < g.n_rep; r += blockDim.x) rclear[r] = 0;
  }
  if (PREC == 0) lds_fill<4>(lds_d4, t.rho_val, t.nr - 1, lds_d4 + (t.nr - 1));
  else
    lds_fill<4>(reinterpret_cast<float4*>(lds_d4), t.rho_val32, t.nr - 1,
                reinterpret_cast<float4*>(lds_d4) + (t.nr - 1));
  if (due) {
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int nwaves = (int)blockDim.x >> 6;
    const size_t bl = (build_lds_bytes(g.cell_cap, kSmallStage) + 15) & ~size_t(15);
    char* base = reinterpret_cast<char*>(lds_d4) + density_table_bytes(t.nr, PREC);
    const BuildLds L = carve_build_lds(base + (size_t)wave * bl, g.cell_cap, kSmallStage);
    if (cond && !err && blockIdx.x == 0 && threadIdx.x == 0)
      *counter64(s.status, SW_REBUILDS) += 1ull;
    const int64_t gstride = (int64_t)gridDim.x * nwaves;
    const int64_t gwave = (int64_t)blockIdx.x * nwaves + wave;
    if (!err)
      for (int64_t b = gwave; b < g.n_atiles; b += gstride) bin_tile(g, s, g.atiles[b], rcond, lane);
    if (!grid_sync(s.status)) return;
    for (int64_t b = gwave; b < g.n_ctiles; b += gstride) {
      const CellTile ct = g.ctiles[b];
      if (ct.cell < 0 || (rcond && rcond[ct.rep] == 0)) continue;
      build_cell<true, kSmallStage>(g, s, ct, L, lane);
      build_sync<true>();  // the wave's next cell reuses its staging arrays
    }
    if (!grid_sync(s.status)) return;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncells;
         c += (int64_t)gridDim.x * blockDim.x)
      s.bin_cnt[c] = 0;
  } else {
    __syncthreads();  // the table is in place
    if (err) return;
  }
  const TileWalk w = tile_walk<LPA>();
  for (int64_t it = w.q;; it += w.tpi) {
    const int64_t b = walk_tile(it, g.n_atiles);
    if (b < 0) break;
    const AtomTile tl = g.atiles[b];
    const bool active = w.a < tl.count;
    const RepDev& rp = g.reps[tl.rep];
    const int64_t i = tl.begin + (active ? w.a : 0);
    const double rho_i = density_of<PREC, LPA>(g, s, t, rp, s.pos, lds_d4, i, active, w.sub);
    if (!active || w.sub != 0) continue;
    store_fprime<PREC>(s, t, s.pos, i, rho_i, 0);
  }
}

size_t bbd_lds_bytes(const Tables& t, int prec, int cell_cap) {
  return density_table_bytes(t.nr, prec) +
         (size_t)(kPersistThreads / 64) * ((build_lds_bytes(cell_cap, kSmallStage) + 15) & ~size_t(15));
}

template <int PREC, int LPA>
static int bbd_fit_one(size_t bytes) {
  const void* fn = reinterpret_cast<const void*>(&k_bin_build_density<PREC, LPA>);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) !=
      hipSuccess)
    return 0;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kPersistThreads, bytes) != hipSuccess)
    return 0;
  return n;
}

int bbd_blocks_per_cu(const Tables& t, int precision, int cell_cap) {
  const size_t b = bbd_lds_bytes(t, precision, cell_cap);
  int n;
  if (precision == 0)
    n = std::min(std::min(bbd_fit_one<0, 1>(b), bbd_fit_one<0, 2>(b)),
                 std::min(bbd_fit_one<0, 4>(b), bbd_fit_one<0, 8>(b)));
  else
    n = std::min(std::min(bbd_fit_one<1, 1>(b), bbd_fit_one<1, 2>(b)),
                 std::min(bbd_fit_one<1, 4>(b), bbd_fit_one<1, 8>(b)));
  return n;
}


__global__ __launch_bounds__(64) void k_halfkick(Geometry g, State s, double coef) {
  const AtomTile tl = g.atiles[blockIdx.x];
  if ((int)threadIdx.x >= tl.count) return;
  const int64_t i = tl.begin + threadIdx.x;
  const double scale = coef * acc_of(g, s, i);
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
// reduces its tile in a fixed tree order into partial[replica tile number],
// so a replica's sums do not depend on the other replicas of the batch.
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
    // past the last knot F continues along its end tangent
    const double fe = (te > 1.0) ? ((c.x + c.y + c.z + c.w) +
                                    (c.y + 2.0 * c.z + 3.0 * c.w) * (te - 1.0))
                                 : fma(fma(fma(c.w, te, c.z), te, c.y), te, c.x);
    ep = 0.5 * ph + fe;
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
  if (threadIdx.x == 0 && tl.count > 0) {
    const RepDev& rp = g.reps[tl.rep];
    const int64_t slot = rp.tile0 + (tl.begin - rp.atom0) / 64;
    s.partial[2 * slot] = s_e[0];
    s.partial[2 * slot + 1] = s_k[0];
  }
}

// One block per replica: add the tile partials of replica r in its tile order.
__global__ __launch_bounds__(256) void k_energy_reduce(Geometry g, State s, double* out) {
  __shared__ double s_e[256], s_k[256];
  const int r = blockIdx.x;
  const RepDev& rp = g.reps[r];
  double e = 0.0, k = 0.0;
  for (int b = threadIdx.x; b < rp.ntiles; b += 256) {
    e += s.partial[2 * (rp.tile0 + b)];
    k += s.partial[2 * (rp.tile0 + b) + 1];
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
      if (s.rec) s.rec[k] = s.snap_rec[k];
    } else {
      sp[k] = s.pos[k];
      sv[k] = s.vel[k];
      if (s.rec) s.snap_rec[k] = s.rec[k];
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

hipError_t launch_cell_stats(const Launch& L, const State& s, int64_t n_cells_total) {
  hipLaunchKernelGGL(k_cell_stats, dim3(1), dim3(1024), 0, L.stream, s, n_cells_total);
  return hipGetLastError();
}

hipError_t launch_zero_bins(const Launch& L, const State& s, int64_t n_cells_total) {
  hipLaunchKernelGGL(k_zero_i32, dim3(grid_stride_blocks(n_cells_total)), dim3(256), 0, L.stream,
                     s.bin_cnt, n_cells_total);
  return hipGetLastError();
}

hipError_t launch_bin(const Launch& L, const Geometry& g, const State& s, const int32_t* cond,
                      const int32_t* rcond) {
  const int grid = std::min(L.atile_blocks, 16 * L.persist_blocks);
  hipLaunchKernelGGL(k_bin, dim3(grid), dim3(64), 0, L.stream, g, s, cond, rcond);
  return hipGetLastError();
}

hipError_t launch_build(const Launch& L, const Geometry& g, const State& s, const int32_t* cond,
                        const int32_t* rcond) {
  const int grid = std::min(L.ctile_blocks, 24 * L.persist_blocks);
  hipLaunchKernelGGL(k_build, dim3(grid), dim3(kBuildBlock), build_lds_bytes(g.cell_cap),
                     L.stream, g, s, cond, rcond);
  return hipGetLastError();
}

hipError_t launch_sort(const Launch& L, const Geometry& g, const State& s, int64_t m) {
  hipError_t e;
  if ((e = launch_zero_bins(L, s, m)) != hipSuccess) return e;
  if ((e = launch_bin(L, g, s, nullptr, nullptr)) != hipSuccess) return e;
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

// Persistent launches: one workgroup per CU slot (grid = L.persist_blocks).
static int pair_threads(int prec, bool force, int lpa) {
  const int waves = (force && prec != 0) ? 16 : 12;
  int tpi = waves / lpa;
  if (tpi < 1) tpi = 1;
  return 64 * lpa * tpi;
}

// table rows plus the junk rows of the fill
size_t density_lds_bytes(const Tables& t, int prec) {
  return (size_t)(t.nr - 1) * (prec == 0 ? sizeof(double4) : sizeof(float4)) + kLdsJunkBytes;
}

size_t force_lds_bytes(const Tables& t, int prec) {
  return (size_t)(t.nr - 1) * (prec == 0 ? 3 * sizeof(double2) : sizeof(float4) + sizeof(float2)) +
         kLdsJunkBytes;
}

template <int PREC, int LPA>
static hipError_t density_go(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                             double4* pos, const int32_t* cz, int32_t* cf, int32_t* rc, int64_t m,
                             int want) {
  hipLaunchKernelGGL((k_density<PREC, LPA>), dim3(2 * L.persist_blocks),
                     dim3(pair_threads(PREC, false, LPA)), density_lds_bytes(t, PREC), L.stream, g,
                     s, t, pos, cz, cf, rc, m, want);
  return hipGetLastError();
}

template <int PREC, int LPA>
static hipError_t force_int_go(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                               const double4* pi, double4* po, int32_t* fl, int32_t* rfl) {
  hipLaunchKernelGGL((k_force_integrate<PREC, LPA>), dim3(L.persist_blocks),
                     dim3(pair_threads(PREC, true, LPA)), force_lds_bytes(t, PREC), L.stream, g, s,
                     t, pi, po, fl, rfl);
  return hipGetLastError();
}

template <int PREC, int LPA>
static hipError_t force_only_go(const Launch& L, const Geometry& g, const State& s,
                                const Tables& t, const double4* pos) {
  hipLaunchKernelGGL((k_force_only<PREC, LPA>), dim3(L.persist_blocks),
                     dim3(pair_threads(PREC, true, LPA)), force_lds_bytes(t, PREC), L.stream, g, s,
                     t, pos);
  return hipGetLastError();
}

#define MDK_LPA_SWITCH(P, lpa, CALL) \
  switch (lpa) {                     \
    case 1: return CALL(P, 1);       \
    case 2: return CALL(P, 2);       \
    case 4: return CALL(P, 4);       \
    default: return CALL(P, 8);      \
  }

hipError_t launch_density(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                          int precision, int lpa, const double4* pos, const int32_t* cond_zero,
                          int32_t* clear_flag, int32_t* rclear, int64_t n_cells_total,
                          bool want_rho) {
  double4* p = const_cast<double4*>(pos);
  const int w = want_rho ? 1 : 0;
#define MDK_D(P, Lp) \
  density_go<P, Lp>(L, g, s, t, p, cond_zero, clear_flag, rclear, n_cells_total, w)
  if (precision == 0) { MDK_LPA_SWITCH(0, lpa, MDK_D) }
  MDK_LPA_SWITCH(1, lpa, MDK_D)
#undef MDK_D
}

hipError_t launch_force_integrate(const Launch& L, const Geometry& g, const State& s,
                                  const Tables& t, int precision, int lpa, const double4* pos_in,
                                  double4* pos_out, int32_t* flag_next, int32_t* rflag_next) {
#define MDK_F(P, Lp) force_int_go<P, Lp>(L, g, s, t, pos_in, pos_out, flag_next, rflag_next)
  if (precision == 0) { MDK_LPA_SWITCH(0, lpa, MDK_F) }
  MDK_LPA_SWITCH(1, lpa, MDK_F)
#undef MDK_F
}

hipError_t launch_force_only(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                             int precision, int lpa, const double4* pos) {
#define MDK_O(P, Lp) force_only_go<P, Lp>(L, g, s, t, pos)
  if (precision == 0) { MDK_LPA_SWITCH(0, lpa, MDK_O) }
  MDK_LPA_SWITCH(1, lpa, MDK_O)
#undef MDK_O
}

template <int PREC, int LPA>
static hipError_t bbd_go(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                         const int32_t* cond, const int32_t* rcond, int32_t* clear_flag,
                         int32_t* rclear, int64_t ncells, int grid) {
  hipLaunchKernelGGL((k_bin_build_density<PREC, LPA>), dim3(grid), dim3(kPersistThreads),
                     bbd_lds_bytes(t, PREC, g.cell_cap), L.stream, g, s, t, cond, rcond,
                     clear_flag, rclear, ncells);
  return hipGetLastError();
}

hipError_t launch_bin_build_density(const Launch& L, const Geometry& g, const State& s,
                                    const Tables& t, int precision, int lpa,
                                    const int32_t* cond, const int32_t* rcond,
                                    int32_t* clear_flag, int32_t* rclear, int64_t ncells,
                                    int grid) {
#define MDK_B(P, Lp) bbd_go<P, Lp>(L, g, s, t, cond, rcond, clear_flag, rclear, ncells, grid)
  if (precision == 0) { MDK_LPA_SWITCH(0, lpa, MDK_B) }
  MDK_LPA_SWITCH(1, lpa, MDK_B)
#undef MDK_B
}

hipError_t launch_density_dyn(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                              int precision, const double4* pos, const int32_t* cond_zero,
                              int32_t* clear_flag, int32_t* rclear, int64_t n_cells_total,
                              bool want_rho) {
  double4* p = const_cast<double4*>(pos);
  const int w = want_rho ? 1 : 0;
  if (precision == 0)
    hipLaunchKernelGGL(k_density_dyn<0>, dim3(2 * L.persist_blocks), dim3(768),
                       density_lds_bytes(t, 0), L.stream, g, s, t, p, cond_zero, clear_flag,
                       rclear, n_cells_total, w);
  else
    hipLaunchKernelGGL(k_density_dyn<1>, dim3(2 * L.persist_blocks), dim3(768),
                       density_lds_bytes(t, 1), L.stream, g, s, t, p, cond_zero, clear_flag,
                       rclear, n_cells_total, w);
  return hipGetLastError();
}

hipError_t launch_force_integrate_dyn(const Launch& L, const Geometry& g, const State& s,
                                      const Tables& t, int precision, const double4* pos_in,
                                      double4* pos_out, int32_t* flag_next, int32_t* rflag_next) {
  if (precision == 0)
    hipLaunchKernelGGL(k_force_dyn<0>, dim3(L.persist_blocks), dim3(768), force_lds_bytes(t, 0),
                       L.stream, g, s, t, pos_in, pos_out, flag_next, rflag_next);
  else
    hipLaunchKernelGGL(k_force_dyn<1>, dim3(L.persist_blocks), dim3(1024), force_lds_bytes(t, 1),
                       L.stream, g, s, t, pos_in, pos_out, flag_next, rflag_next);
  return hipGetLastError();
}

hipError_t launch_force_only_dyn(const Launch& L, const Geometry& g, const State& s,
                                 const Tables& t, int precision, const double4* pos) {
  return launch_force_integrate_dyn(L, g, s, t, precision, pos, nullptr, nullptr, nullptr);
}

// The persistent step kernel: the force table (as in the force pass) and one
// build staging area per wave.
size_t persist_lds_bytes(const Tables& t, int prec, int cell_cap) {
  const size_t bl = (build_lds_bytes(cell_cap) + 15) & ~size_t(15);
  return persist_table_bytes(t.nr, prec) + (size_t)(kPersistThreads / 64) * bl;
}

template <int PREC, int LPA>
static hipError_t persist_go(const Launch& L, const Geometry& g, const State& s0, const State& s1,
                             const Tables& t, int32_t nsteps, int64_t ncells, int grid,
                             int small) {
  Geometry ga = g;
  State a0 = s0, a1 = s1;
  Tables ta = t;
  int32_t n = nsteps;
  int64_t m = ncells;
  void* args[] = {&ga, &a0, &a1, &ta, &n, &m};
  const void* fn = small ? reinterpret_cast<const void*>(&k_persist_small<PREC, LPA>)
                         : reinterpret_cast<const void*>(&k_persist<PREC, LPA>);
  return hipLaunchCooperativeKernel(fn,
                                    dim3(grid), dim3(kPersistThreads), args,
                                    (unsigned int)persist_lds_bytes(t, PREC, g.cell_cap), L.stream);
}

hipError_t launch_persist(const Launch& L, const Geometry& g, const State& s0, const State& s1,
                          const Tables& t, int precision, int lpa, int32_t nsteps, int64_t ncells,
                          int grid, int small) {
#define MDK_P(P, Lp) persist_go<P, Lp>(L, g, s0, s1, t, nsteps, ncells, grid, small)
  if (precision == 0) { MDK_LPA_SWITCH(0, lpa, MDK_P) }
  MDK_LPA_SWITCH(1, lpa, MDK_P)
#undef MDK_P
}

template <int PREC, int LPA>
static hipError_t allow_persist_one(size_t bytes) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_persist<PREC, LPA>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_persist_small<PREC, LPA>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t allow_persist_lds(const Tables& t, int precision, int cell_cap) {
  const size_t b = persist_lds_bytes(t, precision, cell_cap);
  hipError_t e;
  if (precision == 0) {
    if ((e = allow_persist_one<0, 1>(b)) != hipSuccess) return e;
    if ((e = allow_persist_one<0, 2>(b)) != hipSuccess) return e;
    if ((e = allow_persist_one<0, 4>(b)) != hipSuccess) return e;
    return allow_persist_one<0, 8>(b);
  }
  if ((e = allow_persist_one<1, 1>(b)) != hipSuccess) return e;
  if ((e = allow_persist_one<1, 2>(b)) != hipSuccess) return e;
  if ((e = allow_persist_one<1, 4>(b)) != hipSuccess) return e;
  return allow_persist_one<1, 8>(b);
}

// Dynamic LDS above the default limit must be allowed per kernel.
template <int PREC, int LPA>
static hipError_t allow_lds_one(size_t dens, size_t force) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_density<PREC, LPA>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)dens);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_force_integrate<PREC, LPA>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)force);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_force_only<PREC, LPA>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)force);
}

hipError_t allow_pair_lds(const Tables& t, int precision) {
  const size_t d = density_lds_bytes(t, precision), f = force_lds_bytes(t, precision);
  hipError_t e;
  const void* dk = precision == 0 ? reinterpret_cast<const void*>(&k_density_dyn<0>)
                                  : reinterpret_cast<const void*>(&k_density_dyn<1>);
  const void* fk = precision == 0 ? reinterpret_cast<const void*>(&k_force_dyn<0>)
                                  : reinterpret_cast<const void*>(&k_force_dyn<1>);
  if ((e = hipFuncSetAttribute(dk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)d)) !=
      hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute(fk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)f)) !=
      hipSuccess)
    return e;
  if (precision == 0) {
    if ((e = allow_lds_one<0, 1>(d, f)) != hipSuccess) return e;
    if ((e = allow_lds_one<0, 2>(d, f)) != hipSuccess) return e;
    if ((e = allow_lds_one<0, 4>(d, f)) != hipSuccess) return e;
    return allow_lds_one<0, 8>(d, f);
  }
  if ((e = allow_lds_one<1, 1>(d, f)) != hipSuccess) return e;
  if ((e = allow_lds_one<1, 2>(d, f)) != hipSuccess) return e;
  if ((e = allow_lds_one<1, 4>(d, f)) != hipSuccess) return e;
  return allow_lds_one<1, 8>(d, f);
}

hipError_t launch_halfkick(const Launch& L, const Geometry& g, const State& s, double coef) {
  hipLaunchKernelGGL(k_halfkick, dim3(L.atile_blocks), dim3(64), 0, L.stream, g, s, coef);
  return hipGetLastError();
}

hipError_t launch_energy_reduce(const Launch& L, const Geometry& g, const State& s,
                                double* out_pe_ke, int32_t n_rep) {
  hipLaunchKernelGGL(k_energy_reduce, dim3(n_rep), dim3(256), 0, L.stream, g, s, out_pe_ke);
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
                         double* f, double* rho, double* fp, double coef) {
  hipLaunchKernelGGL(k_export, dim3(L.atile_blocks), dim3(64), 0, L.stream, g, s, x, v, f, rho, fp,
                     coef);
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
