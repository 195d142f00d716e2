// md_internal.h -- device data structures, helpers and kernel launchers of
// the MI355X EAM library.  Host API in md_api.hip, kernels in md_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mdk {

// ---------------------------------------------------------------- constants

constexpr int kBuildBlock = 64;      // one wave per cell in the list build
constexpr int kMaxStage = 256;       // candidates staged per build batch (>= kMaxCellCap)
constexpr int kMaxCellCap = 256;     // hard limit of cell_capacity
constexpr int kMaxNbrCap = 1024;     // hard limit of nbr_capacity
constexpr int kIndexBits = 26;       // list entry: j | image code << 26
constexpr uint32_t kIndexMask = (1u << kIndexBits) - 1u;
constexpr uint32_t kNoShift = 21u;   // code of the zero image shift: 1 | 1<<2 | 1<<4
constexpr int kXcd = 8;              // MI355X dispatches workgroups round-robin over 8 XCDs
constexpr int kMaxTypes = 4;         // atom types of the multi-species form
constexpr int kPersistThreads = 512; // threads per workgroup of the persistent step kernel
constexpr int kMaxSlots = 64;        // participants of a one-XCD persistent launch (at most)
constexpr int kMaxBinbuildGrid = 64;  // largest grid of the fused bin + build + density launch (its barrier's cost grows with it)

// status word bits (device, sticky)
constexpr int32_t ST_NBR_OVERFLOW = 1;
constexpr int32_t ST_CELL_OVERFLOW = 2;
constexpr int32_t ST_NONFINITE = 4;
constexpr int32_t ST_LOST = 8;
constexpr int32_t ST_STALL = 32;      // a grid barrier of the persistent launch timed out
constexpr int32_t ST_PLACEMENT = 64;  // a one-XCD persistent launch found too few workgroups on XCD 0
constexpr int32_t ST_ERR_MASK = 0xff;
constexpr int32_t ST_RHO_RANGE = 256;

// status block layout (int32 words; 64-bit counters at even word offsets)
enum StatusWord : int {
  SW_BITS = 0,
  SW_FLAG0 = 1,  // rebuild request, step parity 0
  SW_FLAG1 = 2,  // rebuild request, step parity 1
  SW_MAX_LIST = 3,
  SW_MAX_CELL = 4,
  SW_SCRATCH = 5,      // throw-away flag for timing launches
  SW_TYPE_CHECK = 6,   // set when md_set_types finds a type out of range
  SW_ZERO = 7,         // no kernel writes it: the never-due rebuild flag of timing launches
  SW_STEPS = 8,        // int64
  SW_REBUILDS = 10,    // int64
  SW_LIST_TOTAL = 12,  // int64
  SW_SNAP_STEPS = 14,  // int64, SW_STEPS at the last snapshot
  SW_BAR_COUNT = 20,   // grid barrier of the persistent launch: arrivals
  SW_BAR_GEN = 21,     //   generation
  SW_BAR_STOP = 22,    //   stop decision of the last arrival
  SW_XCD_TICKET = 23,  //   workgroups of a one-XCD persistent launch that found themselves on XCD 0
  SW_SLOTS = 128,      //   arrival slots of its participants, two parities of kMaxSlots
  SW_WORDS = 256
};

// ---------------------------------------------------------------- structs

struct RepDev {
  double box[3];      // lengths (periodic) or cell-grid extents (open)
  double inv_cell[3];
  int64_t atom0;
  int32_t n_atoms;
  int32_t cell0;
  int32_t nc[3];
  int32_t ncell;
  int32_t tile0;   // first atom tile of the replica, in replica order
  int32_t ntiles;  // atom tiles of the replica
  int32_t open;    // bit d set: dimension d is open (not periodic)
  int32_t pad;
  // fixed-point positions of the mixed form: q = round(x * qinv) modulo 2^32,
  // x = q * qs.  A periodic dimension maps L to 2^32, so integer wrap-around is
  // the periodic wrap and q_j - q_i (int32) is the minimum image; an open one
  // uses 2^26 quanta per A (differences up to 32 A).
  double qinv[3];
  float qs[3];
  int32_t pad2;
};

struct AtomTile {
  int32_t rep;
  int32_t begin;  // global atom index of the first atom
  int32_t count;  // atoms in this tile (0 = idle block)
  int32_t pad;
};

// Work unit of the pair passes under a per-replica schedule: one wave takes
// `count` (<= 64 / lpa) atoms from `begin`, with lpa lanes on each atom.
struct PairTile {
  int32_t rep;
  int32_t begin;
  int32_t count;
  int32_t lpa;
};

struct CellTile {
  int32_t rep;
  int32_t cell;  // cell index within the replica (-1 = idle block)
};

// Per-segment tables in the library's own layout (built on the host).
struct Tables {
  const double4* rho_val;  // [nr-1] c0..c3 of rho(r)
  const double4* phi_val;  // [nr-1] c0..c3 of phi(r)
  const double2* dpair3;   // [nr-1][3]: (rho'0, rho'1), (rho'2, phi'0), (phi'1, phi'2):
                           // derivative quadratics in t, pre-scaled by 1/dx
  const double4* emb_val;  // [ne-1] c0..c3 of F(rho)
  const float4* rho_val32;  // float copies for the mixed form
  const float4* dpair_a32;
  const float2* dpair_b32;
  double r_inv_dx;          // knots of phi and rho share the same grid starting at 0
  double e_x0, e_inv_dx;
  int32_t nr, ne;           // knot counts
  float r_inv_dx32;
  float pad;
};

struct Geometry {
  const RepDev* reps;
  const AtomTile* atiles;
  const CellTile* ctiles;
  const PairTile* ptiles;  // per-replica schedule (null: one lanes-per-atom value)
  int64_t n_ptiles;        // a multiple of the XCD count
  int64_t n;        // total atoms (ELL stride)
  int32_t n_atiles;
  int32_t n_ctiles;
  int32_t n_rep;
  int32_t nbr_cap;
  int32_t cell_cap;
  double rc2;       // r_cut^2
  double rl2;       // (r_cut + skin)^2
  double lim2;      // (skin/2)^2
  double dt;
  double acc;       // ftm2v / mass (one species)
  double acc_t[kMaxTypes];  // ftm2v / mass of each type (multi-species form)
  float rc2f;
  float pad;
};

struct State {
  double4* pos;      // current positions, w = F'(rho_i)
  double4* pos_alt;  // other position buffer (leap-frog ping-pong)
  double4* vel;      // velocity (half step inside md_step)
  double4* xref;     // positions at the last list build
  // mixed form only (null otherwise): per slot {x, y, z in fixed point, F'(rho_i)
  // float bits}, the 16-byte record both pair passes gather; kept beside pos
  // (same buffer parity) by every kernel that writes positions
  uint4* rec;
  uint4* rec_alt;
  uint4* sort_rec;
  uint4* snap_rec;
  double4* frc;      // forces when requested
  double* rho;       // rho_i when requested
  double* epair;     // 1/2 sum phi when requested
  int32_t* id;       // original atom index of each slot
  int32_t* cell_of;  // cell (within replica) of each slot at the last binning
  uint32_t* nbr;     // ELL [cap][n]
  int32_t* cnt;      // list length (true count, may exceed cap)
  int32_t* bin_cnt;  // [total cells]
  int32_t* bin_idx;  // [total cells][cell_cap]
  int32_t* cell_start;  // [total cells + 1]
  int32_t* cell_stat;   // [total cells][3]: longest list, list entries, atoms (last build)
  int32_t* status;   // SW_WORDS
  int32_t* rflag;    // [3][n_rep]: per-replica rebuild requests (parity 0, 1, scratch)
  double4* sort_pos;
  double4* sort_vel;
  int32_t* sort_id;
  double* partial;   // per-atom-tile energy partials [n_atiles][2]
  // half-list form (null for the full list): pair slot (k, i) = k N + i
  uint32_t* hnbr;    // [cap][n] entries of i's list with j > i, in list order
  int32_t* hcnt;     // entries of hnbr per atom
  uint32_t* rslot_u; // [cap][n] pair slots where the atom is the j side, unsorted
  uint32_t* rslot;   // the same, ascending
  int32_t* rcnt;     // entries of rslot per atom
  int32_t* rfill;    // scatter counters (zero between rebuilds)
  double* pval;      // [cap][n] rho(r) of each pair slot
  double4* qval;     // [cap][n] force on the i side of each pair slot (w unused)
  double* own_rho;   // [n] sum over the atom's own pair slots
  double4* own_f;    // [n] force sum over the atom's own pair slots
  // multi-species form (null for one species)
  uint8_t* type;       // type of each slot
  uint8_t* type_orig;  // type of each atom, original order
  uint8_t* sort_type;
};

// Tables of the multi-species form.  rho, phi share one knot grid (x0 = 0),
// the embedding tables another.  The pair passes' rows are interleaved by
// segment, so the rows one pair needs share a cache line (T = 2).
struct MultiTables {
  const double4* rho_seg;  // [nr-1][T] c0..c3 of rho_t(r), segment-major
  const double* frow;      // [nr-1][seg_stride]: per segment the derivative quadratics
                           // (3 doubles, in t, pre-scaled by 1/dx) of rho'_t for t < T,
                           // then of phi'_ab for the pairs a <= b
  const double4* phi_val;  // [T*T][nr-1] c0..c3 of phi_ab(r) (energy)
  const double4* rho_val;  // [T][nr-1] c0..c3 of rho_t(r) (energy)
  const double4* emb_val;  // [T][ne-1] c0..c3 of F_t(rho)
  double r_inv_dx;
  double e_x0, e_inv_dx;
  int32_t nr, ne;
  int32_t n_types;
  int32_t seg_stride;      // doubles per segment of frow (a multiple of 16)
  int32_t pair_row[kMaxTypes * kMaxTypes];  // row of phi'_ab within a segment of frow
  int32_t lds_seg0;        // first segment of frow held in the force pass's LDS
  int32_t lds_pad;
};

// ---------------------------------------------------------------- launchers

struct Launch {
  hipStream_t stream;
  int32_t atile_blocks;  // blocks of the per-atom passes
  int32_t ctile_blocks;  // blocks of the per-cell passes
  int32_t persist_blocks;  // workgroups of the persistent pair passes (CU count, multiple of 8)
};

hipError_t launch_import(const Launch& L, const Geometry& g, const State& s, const double* x,
                         const double* v);
hipError_t launch_zero_bins(const Launch& L, const State& s, int64_t n_cells_total);
hipError_t launch_cell_stats(const Launch& L, const State& s, int64_t n_cells_total);
hipError_t launch_bin(const Launch& L, const Geometry& g, const State& s, const int32_t* cond,
                      const int32_t* rcond);
// Binning and list build in one launch with a grid barrier (small systems);
// grid at most binbuild_blocks_per_cu() x compute units.
hipError_t launch_bin_build_density(const Launch& L, const Geometry& g, const State& s,
                                    const Tables& t, int precision, int lpa,
                                    const int32_t* cond, const int32_t* rcond,
                                    int32_t* clear_flag, int32_t* rclear, int64_t ncells,
                                    int grid);
size_t bbd_lds_bytes(const Tables& t, int prec, int cell_cap);
int bbd_blocks_per_cu(const Tables& t, int precision, int cell_cap);
hipError_t launch_build(const Launch& L, const Geometry& g, const State& s, const int32_t* cond,
                        const int32_t* rcond);
hipError_t launch_sort(const Launch& L, const Geometry& g, const State& s, int64_t n_cells_total);
hipError_t launch_density(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                          int precision, int lpa, const double4* pos, const int32_t* cond_zero,
                          int32_t* clear_flag, int32_t* rclear, int64_t n_cells_total,
                          bool want_rho);
hipError_t launch_force_integrate(const Launch& L, const Geometry& g, const State& s,
                                  const Tables& t, int precision, int lpa, const double4* pos_in,
                                  double4* pos_out, int32_t* flag_next, int32_t* rflag_next);
hipError_t launch_force_only(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                             int precision, int lpa, const double4* pos);
// The same three passes under a per-replica schedule (g.ptiles): each wave
// takes one pair tile and works on it with that tile's lanes per atom.
hipError_t launch_density_dyn(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                              int precision, const double4* pos, const int32_t* cond_zero,
                              int32_t* clear_flag, int32_t* rclear, int64_t n_cells_total,
                              bool want_rho);
hipError_t launch_force_integrate_dyn(const Launch& L, const Geometry& g, const State& s,
                                      const Tables& t, int precision, const double4* pos_in,
                                      double4* pos_out, int32_t* flag_next, int32_t* rflag_next);
hipError_t launch_force_only_dyn(const Launch& L, const Geometry& g, const State& s,
                                 const Tables& t, int precision, const double4* pos);
size_t density_lds_bytes(const Tables& t, int precision);
size_t force_lds_bytes(const Tables& t, int precision);
hipError_t allow_pair_lds(const Tables& t, int precision);
// Half-list form of the pair passes (md_half.hip).  `reindex` rebuilds the
// half list and the sorted reverse slots from the full list first (cond: the
// device flag of a rebuild in this step; force: do it regardless).
hipError_t launch_half_density(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                               const double4* pos, const int32_t* cond, bool force_reindex,
                               int32_t* clear_flag, int32_t* rclear, int64_t n_cells_total,
                               bool want_rho);
hipError_t launch_half_force_integrate(const Launch& L, const Geometry& g, const State& s,
                                       const Tables& t, const double4* pos_in, double4* pos_out,
                                       int32_t* flag_next, int32_t* rflag_next);
hipError_t launch_half_force_only(const Launch& L, const Geometry& g, const State& s,
                                  const Tables& t, const double4* pos);
hipError_t allow_half_lds(const Tables& t);
// Multi-species pair passes, energy and type upload (md_multi.hip).
size_t multi_density_lds_bytes(const MultiTables& t);  // 0 when the rows do not fit the LDS
int multi_force_lds_seg0(int nr, int n_types);  // first force segment that fits the LDS
size_t multi_force_lds_bytes(const MultiTables& t);
hipError_t allow_multi_lds(const MultiTables& t);
hipError_t launch_multi_density(const Launch& L, const Geometry& g, const State& s,
                                const MultiTables& t, int lpa, const double4* pos,
                                const int32_t* cond_zero, int32_t* clear_flag, int32_t* rclear,
                                int64_t n_cells_total, bool want_rho);
hipError_t launch_multi_force_integrate(const Launch& L, const Geometry& g, const State& s,
                                        const MultiTables& t, int lpa, const double4* pos_in,
                                        double4* pos_out, int32_t* flag_next, int32_t* rflag_next);
hipError_t launch_multi_force_only(const Launch& L, const Geometry& g, const State& s,
                                   const MultiTables& t, int lpa, const double4* pos);
hipError_t launch_multi_energy(const Launch& L, const Geometry& g, const State& s,
                               const MultiTables& t, double* out_pe_ke, int32_t n_rep);
hipError_t launch_set_types(const Launch& L, const Geometry& g, const State& s,
                            const int32_t* type_in, int32_t n_types, bool has_slots);
hipError_t launch_energy_reduce(const Launch& L, const Geometry& g, const State& s,
                                double* out_pe_ke, int32_t n_rep);
// scale of the kick = coef * ftm2v / mass of the atom's type
hipError_t launch_halfkick(const Launch& L, const Geometry& g, const State& s, double coef);
// nsteps (even) steps in one cooperative launch of `grid` workgroups; s0 / s1 =
// the state with position buffer 0 / 1 current (buffer 0 current at entry).
hipError_t launch_persist(const Launch& L, const Geometry& g, const State& s0, const State& s1,
                          const Tables& t, int precision, int lpa, int32_t nsteps, int64_t ncells,
                          int grid, int small);
hipError_t allow_persist_lds(const Tables& t, int precision, int cell_cap);
size_t persist_lds_bytes(const Tables& t, int precision, int cell_cap);
hipError_t launch_energy(const Launch& L, const Geometry& g, const State& s, const Tables& t,
                         double* out_pe_ke, int32_t n_rep);
// on-step velocity = v + coef * ftm2v / mass * f (coef = dt/2 after a step, else 0)
hipError_t launch_export(const Launch& L, const Geometry& g, const State& s, double* x, double* v,
                         double* f, double* rho, double* fp, double coef);
hipError_t launch_export_cells(const Launch& L, const Geometry& g, const State& s, int32_t* cell);
hipError_t launch_export_nbrs(const Launch& L, const Geometry& g, const State& s, int32_t* cnt,
                              int32_t* nbr, int32_t cap_out);
hipError_t launch_snapshot(const Launch& L, const Geometry& g, const State& s, double4* snap_pos,
                           double4* snap_vel, bool restore);

// Read-only view of a context's device state for companion modules (force
// matching): geometry, the current-buffer state and launch configuration.
struct CtxView {
  Geometry g;
  State s;
  Launch L;
  int64_t n_cells;
  int32_t n_rep;
};

}  // namespace mdk

struct md_ctx;
// Defined in md_api.hip; valid after md_build_neighbors.
int md_internal_view(const md_ctx* ctx, mdk::CtxView* out);
