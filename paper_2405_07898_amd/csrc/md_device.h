// md_device.h -- device helpers shared by the kernel sources of the MI355X
// EAM library (md_kernels.hip, md_half.hip, md_multi.hip, md_fm.hip).
#pragma once

#include <math.h>

#include "md_internal.h"

namespace mdk {

// 1/sqrt(x) in float64: hardware estimate (relative error below 2^-24 on
// gfx950, measured), then one Newton-Raphson step y <- y + y/2 (1 - x y^2),
// which leaves a relative error of a few 1e-15 (the paper evaluates
// r^-1 = (r^2)^-1/2 by Newton-Raphson, Table "flopmodel").
__device__ __forceinline__ double rsq64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double h = fma(-x * y, y, 1.0);
  return fma(0.5 * y, h, y);
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

// Errors latched by earlier kernels (plain load: kernel boundaries make
// them visible; errors raised inside the running kernel are not waited for).
__device__ __forceinline__ bool has_error(const int32_t* status) {
  return (status[SW_BITS] & ST_ERR_MASK) != 0;
}

__device__ __forceinline__ void set_bits(int32_t* status, int32_t bits) {
  __hip_atomic_fetch_or(status + SW_BITS, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long* counter64(int32_t* status, int word) {
  return reinterpret_cast<unsigned long long*>(status + word);
}

// ftm2v / mass of the atom in slot i (per type in the multi-species form).
__device__ __forceinline__ double acc_of(const Geometry& g, const State& s, int64_t i) {
  return s.type ? g.acc_t[s.type[i]] : g.acc;
}

// Image shift encoded in a list entry: 2 bits per dimension, value s+1 for a
// shift of s box lengths (s in -1, 0, +1) added to x_j - x_i.
__device__ __forceinline__ void apply_shift(uint32_t code, const RepDev& rp, double& dx, double& dy,
                                            double& dz) {
  dx += (double)((int)(code & 3u) - 1) * rp.box[0];
  dy += (double)((int)((code >> 2) & 3u) - 1) * rp.box[1];
  dz += (double)((int)(code >> 4) - 1) * rp.box[2];
}

// Loads through a uniform base pointer and a 32-bit byte offset (the
// compiler's scalar-base + 32-bit vector-offset addressing; every buffer that
// is indexed this way is below 4 GiB, checked when the context is created).
template <class T>
__device__ __forceinline__ T ld32(const T* __restrict__ base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

template <class T>
__device__ __forceinline__ void st32(T* __restrict__ base, uint32_t byte_off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// The spline rows of a pass live in LDS for the whole kernel: one persistent
// workgroup per CU loads them once, then walks its atom tiles.  Workgroup w
// takes tile-table entries w, w + G, w + 2G, ... (G = grid size, a multiple of
// the XCD count), i.e. only tiles the tile table placed on its own XCD.
struct TileWalk {
  int tpi;  // tiles per iteration
  int q;    // this thread's tile slot
  int a;    // atom within the tile
  int sub;  // lane within the atom
};

// Table position of the it-th atom tile (it = 0, 1, ...) a workgroup of a
// pair pass takes, or -1 when it has none left: workgroup w takes positions
// w, w + G, w + 2G, ... (G = grid size, a multiple of the XCD count), so every
// tile it takes is one the tile table placed on its own XCD.  (Giving each
// workgroup a contiguous run of its XCD's tiles instead, so that the tiles in
// flight on a CU are neighbours in space, was measured slower.)
__device__ __forceinline__ int64_t walk_tile(int64_t it, int64_t n_tiles) {
  const int64_t b = blockIdx.x + (int64_t)gridDim.x * it;
  return b < n_tiles ? b : -1;
}

template <int LPA>
__device__ __forceinline__ TileWalk tile_walk() {
  TileWalk w;
  w.tpi = (int)blockDim.x / (64 * LPA);
  w.q = (int)threadIdx.x / (64 * LPA);
  const int r = (int)threadIdx.x - w.q * 64 * LPA;
  w.a = r / LPA;
  w.sub = r % LPA;
  return w;
}

// Table rows into LDS: each thread requests all its rows of a round (kU of
// them) before storing any, so a round costs one memory latency, not one per
// row.  Nothing branches: indexes past the end load the last row again and
// store into a junk row of the lane (a branch around each load or store makes
// the compiler wait for every load before the next).
constexpr size_t kLdsJunkBytes = 64 * sizeof(double4);

template <int kU, class T>
__device__ __forceinline__ void lds_fill(T* dst, const T* __restrict__ src, int n, void* junk) {
  const int nt = (int)blockDim.x;
  T* const jr = reinterpret_cast<T*>(junk) + (threadIdx.x & 63);
  for (int b = (int)threadIdx.x; b < n; b += kU * nt) {
    T v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = src[min(b + u * nt, n - 1)];
#pragma unroll
    for (int u = 0; u < kU; ++u) *(b + u * nt < n ? dst + b + u * nt : jr) = v[u];
  }
}

__device__ __forceinline__ void separation(uint32_t e, const RepDev& rp, double qx, double qy,
                                           double qz, double px, double py, double pz, double& dx,
                                           double& dy, double& dz) {
  dx = qx - px;
  dy = qy - py;
  dz = qz - pz;
  const uint32_t code = e >> kIndexBits;
  if (code != kNoShift) apply_shift(code, rp, dx, dy, dz);
}

// Sum over the LPA lanes of one atom, combined in a lane-symmetric order so
// every lane ends with the same bits.
template <int LPA>
__device__ __forceinline__ double lane_sum_sym(double v) {
#pragma unroll
  for (int o = 1; o < LPA; o <<= 1) {
    const double w = __shfl_xor(v, o, 64);
    v = ((threadIdx.x & o) == 0) ? v + w : w + v;
  }
  return v;
}

// List entries in flight per lane in the pair passes.
constexpr int kBatch = 4;
// The same in the mixed form's force pass (16-byte neighbour records).
constexpr int kBatchMixed = 4;

// The next kBatch list entries of atom i for this lane (entries past the list
// end read as the atom itself with no image shift).
template <int LPA, int B>
__device__ __forceinline__ void load_entries(const uint32_t* __restrict__ nbr, uint32_t N,
                                             uint32_t i, int k0, int m, uint32_t self_e,
                                             uint32_t (&e)[B]) {
  uint32_t off = ((uint32_t)k0 * N + i) * 4u;
  const uint32_t step = (uint32_t)LPA * N * 4u;
#pragma unroll
  for (int u = 0; u < B; ++u) {
    e[u] = (k0 + u * LPA < m) ? ld32(nbr, off) : self_e;
    off += step;
  }
}

}  // namespace mdk
