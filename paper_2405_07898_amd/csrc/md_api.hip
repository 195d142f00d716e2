// md_api.hip -- host side of the EAM library: contexts, workspace carving,
// tile tables, spline-table layouts, step graphs and the C ABI of md.h.
#include "md.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "md_internal.h"

using namespace mdk;

namespace {

thread_local std::string g_last_error;

struct Carve {
  size_t off = 0;
  char* base = nullptr;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct RepHost {
  int64_t n;
  double box[3];   // lengths (periodic) or cell-grid extents (open)
  int32_t nc[3];
  int32_t open;    // bit d: dimension d is open
};

bool valid_spline(const md_spline* s) {
  return s && s->coef && s->n_knots >= 3 && std::isfinite(s->x0) && std::isfinite(s->inv_dx) &&
         s->inv_dx > 0.0;
}

md_status check_params(const md_params* p) {
  if (!p) return MD_E_ARG;
  if (!(p->mass > 0) || !(p->dt >= 0) || !(p->r_cut > 0) || !(p->skin >= 0) || !(p->ftm2v > 0))
    return MD_E_ARG;
  if (p->precision != MD_FP64 && p->precision != MD_MIXED) return MD_E_ARG;
  if (p->nbr_capacity < 1 || p->nbr_capacity > kMaxNbrCap) return MD_E_ARG;
  if (p->cell_capacity < 1 || p->cell_capacity > kMaxCellCap) return MD_E_ARG;
  if (p->chunk_steps < 2 || (p->chunk_steps & 1)) return MD_E_ARG;
  const int l = p->lanes_per_atom;
  if (!(l == 0 || l == 1 || l == 2 || l == 4 || l == 8)) return MD_E_ARG;
  if (p->sort_every < 0) return MD_E_ARG;
  if (p->list_mode != MD_LIST_FULL && p->list_mode != MD_LIST_HALF) return MD_E_ARG;
  // the half-list passes exist in float64 only
  if (p->list_mode == MD_LIST_HALF && p->precision != MD_FP64) return MD_E_ARG;
  // several atom types: float64, full list
  if (p->n_types < 0 || p->n_types > kMaxTypes) return MD_E_ARG;
  if (p->n_types > 1 && (p->precision != MD_FP64 || p->list_mode != MD_LIST_FULL)) return MD_E_ARG;
  if (p->launch_mode != MD_LAUNCH_GRAPH && p->launch_mode != MD_LAUNCH_PERSISTENT) return MD_E_ARG;
  // the persistent step kernel runs the one-species full-list passes
  if (p->launch_mode == MD_LAUNCH_PERSISTENT && (p->n_types > 1 || p->list_mode != MD_LIST_FULL))
    return MD_E_ARG;
  return MD_OK;
}

// Cells per edge: floor(L / (r_cut + skin)).  A periodic dimension needs at
// least 3 (and L >= 2 (r_cut + skin), which keeps the minimum image unique
// inside the list radius); an open one at least 1.
md_status rep_cells(const md_params* p, const double* box, int32_t open, int32_t nc[3]) {
  const double rl = p->r_cut + p->skin;
  for (int d = 0; d < 3; ++d) {
    if (!(box[d] > 0.0) || !std::isfinite(box[d])) return MD_E_BOX;
    double q = std::floor(box[d] / rl);
    if ((open >> d) & 1) {
      q = std::max(q, 1.0);
    } else if (!(box[d] >= 2.0 * rl) || q < 3.0) {
      return MD_E_BOX;
    }
    if (q > 4096.0) return MD_E_BOX;
    nc[d] = (int32_t)q;
  }
  return MD_OK;
}

// XCD-aware order: block b runs on XCD b % 8; give each XCD a contiguous run
// of tiles so neighbouring tiles share that XCD's L2.
template <class T>
std::vector<T> xcd_order(const std::vector<T>& tiles, const T& idle) {
  const size_t n = tiles.size();
  const size_t per = (n + kXcd - 1) / kXcd;
  std::vector<T> out(per * kXcd, idle);
  for (size_t b = 0; b < out.size(); ++b) {
    const size_t t = (b % kXcd) * per + b / kXcd;
    if (t < n) out[b] = tiles[t];
  }
  return out;
}

struct LayoutSizes {
  int64_t n = 0;
  int64_t cells = 0;
  size_t atile_blocks = 0, ctile_blocks = 0;
};

}  // namespace

struct md_ctx {
  md_params p{};
  int32_t n_rep = 0;
  std::vector<RepHost> reps;
  LayoutSizes sz;
  Geometry g{};
  State st[2]{};  // st[c].pos = current buffer when cur == c
  Tables t{};
  Launch L{};
  double4* pos_buf[2]{};
  double4* snap_pos = nullptr;
  double4* snap_vel = nullptr;
  double* energy_dev = nullptr;
  int32_t* status = nullptr;
  int cur = 0;
  int lpa = 1;
  // per-replica lanes per atom (empty: every replica takes `lpa`); the pair
  // passes then walk the pair-tile table
  std::vector<int32_t> rep_lpa;
  PairTile* ptile_buf = nullptr;
  bool half = false;    // half-list pair passes
  bool multi = false;   // several atom types
  MultiTables mt{};
  bool has_state = false;
  bool built = false;
  bool v_half = false;  // velocities are half-step (after build)
  int64_t chunks_since_sort = 0;
  hipGraphExec_t graph = nullptr;  // chunk_steps steps from position buffer 0
  // shorter graphs (len steps from position buffer `parity`) for the steps of
  // an md_step call that do not fill a chunk; a few are kept
  struct Tail {
    int32_t len;
    int32_t parity;
    hipGraphExec_t exec;
  };
  std::vector<Tail> tails;
  int persist_cap = 0;  // most co-resident workgroups of the persistent kernel
  int binbuild_grid = 0;  // workgroups of the fused bin + build + density launch (0: three launches)
  std::string err;
};

struct md_fm_ctx;

namespace {

md_status hip_fail(md_ctx* c, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (c) c->err = m;
  g_last_error = m;
  return MD_E_HIP;
}

#define HIPC(ctx, expr)                                  \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
  } while (0)

LayoutSizes layout(const md_params* p, int32_t n_rep, const std::vector<RepHost>& reps) {
  LayoutSizes s;
  size_t at = 0, ct = 0;
  for (int r = 0; r < n_rep; ++r) {
    s.n += reps[r].n;
    const int64_t nc = (int64_t)reps[r].nc[0] * reps[r].nc[1] * reps[r].nc[2];
    s.cells += nc;
    at += (size_t)((reps[r].n + 63) / 64);
    ct += (size_t)nc;
  }
  s.atile_blocks = ((at + kXcd - 1) / kXcd) * kXcd;
  s.ctile_blocks = ((ct + kXcd - 1) / kXcd) * kXcd;
  (void)p;
  return s;
}

struct Buffers {
  RepDev* reps;
  AtomTile* atiles;
  CellTile* ctiles;
  double4 *rho_val, *phi_val, *emb_val;
  double2* dpair3;
  float4 *rho_val32, *dpair_a32;
  float2* dpair_b32;
  double4 *pos0, *pos1, *vel, *xref, *frc;
  uint4 *rec0, *rec1, *sort_rec, *snap_rec;
  double *rho, *epair;
  int32_t *id, *cell_of, *cnt;
  uint32_t* nbr;
  int32_t *bin_cnt, *bin_idx, *cell_start, *cell_stat, *status, *rflag;
  double4 *sort_pos, *sort_vel;
  int32_t* sort_id;
  double4 *snap_pos, *snap_vel;
  double *partial, *energy;
  PairTile* ptiles;
  // multi-species form only
  double4 *m_rho_seg, *m_phi_val, *m_rho_val, *m_emb_val;
  double* m_frow;
  uint8_t *type, *type_orig, *sort_type;
  // half-list form only
  uint32_t *hnbr, *rslot_u, *rslot;
  int32_t *hcnt, *rcnt, *rfill;
  double *pval, *own_rho;
  double4 *qval, *own_f;
};

// Doubles per segment of the interleaved force rows: 3 per rho'_t and per
// unordered pair phi'_ab, rounded up to a 128-byte line.
int multi_seg_stride(int nt) {
  const int rows = nt + nt * (nt + 1) / 2;
  return (3 * rows + 15) / 16 * 16;
}

// Row of phi'_ab (a, b in any order) within a segment of the force rows.
int multi_pair_row(int nt, int a, int b) {
  if (a > b) std::swap(a, b);
  return nt + a * nt - a * (a - 1) / 2 + (b - a);
}

// Fixed-point scales of the mixed form's positions (see RepDev).
void set_quanta(RepDev& d) {
  for (int k = 0; k < 3; ++k) {
    const bool open = (d.open >> k) & 1;
    d.qinv[k] = open ? 67108864.0 : 4294967296.0 / d.box[k];
    d.qs[k] = open ? (float)(1.0 / 67108864.0) : (float)(d.box[k] / 4294967296.0);
  }
}

size_t carve(char* base, const md_params* p, int32_t n_rep, const LayoutSizes& s, int nr, int ne,
             Buffers* b) {
  Carve c;
  c.base = base;
  const size_t N = (size_t)std::max<int64_t>(s.n, 1);
  Buffers tmp;
  Buffers& o = b ? *b : tmp;
  o.reps = c.take<RepDev>(n_rep);
  o.atiles = c.take<AtomTile>(s.atile_blocks);
  o.ctiles = c.take<CellTile>(s.ctile_blocks);
  o.rho_val = c.take<double4>(nr - 1);
  o.phi_val = c.take<double4>(nr - 1);
  o.dpair3 = c.take<double2>(3 * (size_t)(nr - 1));
  o.emb_val = c.take<double4>(ne - 1);
  o.rho_val32 = c.take<float4>(nr - 1);
  o.dpair_a32 = c.take<float4>(nr - 1);
  o.dpair_b32 = c.take<float2>(nr - 1);
  o.pos0 = c.take<double4>(N);
  o.pos1 = c.take<double4>(N);
  o.vel = c.take<double4>(N);
  o.xref = c.take<double4>(N);
  o.frc = c.take<double4>(N);
  o.rec0 = o.rec1 = o.sort_rec = o.snap_rec = nullptr;
  if (p->precision == MD_MIXED) {
    o.rec0 = c.take<uint4>(N);
    o.rec1 = c.take<uint4>(N);
    o.sort_rec = c.take<uint4>(N);
    o.snap_rec = c.take<uint4>(N);
  }
  o.rho = c.take<double>(N);
  o.epair = c.take<double>(N);
  o.id = c.take<int32_t>(N);
  o.cell_of = c.take<int32_t>(N);
  o.cnt = c.take<int32_t>(N);
  o.nbr = c.take<uint32_t>(N * (size_t)p->nbr_capacity);
  o.bin_cnt = c.take<int32_t>((size_t)s.cells);
  o.bin_idx = c.take<int32_t>((size_t)s.cells * p->cell_capacity);
  o.cell_start = c.take<int32_t>((size_t)s.cells + 1);
  o.cell_stat = c.take<int32_t>(3 * (size_t)s.cells);
  o.status = c.take<int32_t>(SW_WORDS);
  o.rflag = c.take<int32_t>(3 * (size_t)n_rep);
  o.sort_pos = c.take<double4>(N);
  o.sort_vel = c.take<double4>(N);
  o.sort_id = c.take<int32_t>(N);
  o.snap_pos = c.take<double4>(N);
  o.snap_vel = c.take<double4>(N);
  o.partial = c.take<double>(2 * s.atile_blocks);
  o.energy = c.take<double>(2 * (size_t)n_rep);
  // pair tiles of a per-replica schedule: at most 8 per atom tile, and padding
  o.ptiles = c.take<PairTile>(8 * s.atile_blocks + 8 * (size_t)n_rep + kXcd);
  o.m_rho_seg = o.m_phi_val = o.m_rho_val = o.m_emb_val = nullptr;
  o.m_frow = nullptr;
  o.type = o.type_orig = o.sort_type = nullptr;
  if (p->n_types > 1) {
    const size_t T = (size_t)p->n_types;
    o.m_rho_seg = c.take<double4>(T * (nr - 1));
    o.m_frow = c.take<double>((size_t)multi_seg_stride((int)T) * (nr - 1));
    o.m_phi_val = c.take<double4>(T * T * (nr - 1));
    o.m_rho_val = c.take<double4>(T * (nr - 1));
    o.m_emb_val = c.take<double4>(T * (ne - 1));
    o.type = c.take<uint8_t>(N);
    o.type_orig = c.take<uint8_t>(N);
    o.sort_type = c.take<uint8_t>(N);
  }
  o.hnbr = o.rslot_u = o.rslot = nullptr;
  o.hcnt = o.rcnt = o.rfill = nullptr;
  o.pval = o.own_rho = nullptr;
  o.qval = o.own_f = nullptr;
  if (p->list_mode == MD_LIST_HALF) {
    const size_t slots = N * (size_t)p->nbr_capacity;
    o.hnbr = c.take<uint32_t>(slots);
    o.rslot_u = c.take<uint32_t>(slots);
    o.rslot = c.take<uint32_t>(slots);
    o.hcnt = c.take<int32_t>(N);
    o.rcnt = c.take<int32_t>(N);
    o.rfill = c.take<int32_t>(N);
    o.pval = c.take<double>(slots);
    o.qval = c.take<double4>(slots);
    o.own_rho = c.take<double>(N);
    o.own_f = c.take<double4>(N);
  }
  return (c.off + 255) & ~size_t(255);
}

md_status gather_reps(const md_params* p, int32_t n_rep, const int64_t* rep_atoms,
                      const double* rep_box, std::vector<RepHost>* out) {
  if (n_rep < 1 || !rep_atoms || !rep_box) return MD_E_ARG;
  out->resize(n_rep);
  int64_t tot = 0;
  for (int r = 0; r < n_rep; ++r) {
    RepHost& h = (*out)[r];
    h.n = rep_atoms[r];
    if (h.n < 1) return MD_E_ARG;
    tot += h.n;
    // a negative length marks an open dimension; its magnitude is the extent
    // of the cell grid
    h.open = 0;
    for (int d = 0; d < 3; ++d) {
      const double b = rep_box[3 * r + d];
      h.box[d] = std::fabs(b);
      if (b < 0.0) h.open |= 1 << d;
    }
    md_status s = rep_cells(p, h.box, h.open, h.nc);
    if (s != MD_OK) return s;
  }
  if (tot >= (int64_t(1) << kIndexBits)) return MD_E_ARG;
  // the list is addressed with 32-bit byte offsets
  if ((uint64_t)tot * (uint64_t)p->nbr_capacity * 4ull >= (1ull << 32)) return MD_E_ARG;
  return MD_OK;
}

int auto_lpa(int64_t n) {
  if (n <= 32768) return 8;
  if (n <= 262144) return 4;
  return 2;
}

md_status read_status(md_ctx* c, int32_t* words) {
  HIPC(c, hipMemcpyAsync(words, c->status, SW_WORDS * sizeof(int32_t), hipMemcpyDeviceToHost,
                         c->L.stream));
  HIPC(c, hipStreamSynchronize(c->L.stream));
  return MD_OK;
}

md_status status_code(int32_t bits) {
  if (bits & (ST_STALL | ST_PLACEMENT)) return MD_E_STALL;
  if (bits & ST_NBR_OVERFLOW) return MD_E_NBR_OVERFLOW;
  if (bits & ST_CELL_OVERFLOW) return MD_E_CELL_OVERFLOW;
  if (bits & ST_LOST) return MD_E_LOST_ATOM;
  if (bits & ST_NONFINITE) return MD_E_NONFINITE;
  if (bits & ST_RHO_RANGE) return MD_W_RHO_RANGE;
  return MD_OK;
}

// The pair passes in the context's list form.  cond: device flag of a
// rebuild in this step (the half form re-derives its half list then).
hipError_t density_pass(md_ctx* c, const State& s, int lpa, const double4* pos,
                        const int32_t* cond, int32_t* clear_flag, int32_t* rclear, bool want_rho) {
  if (c->multi)
    return launch_multi_density(c->L, c->g, s, c->mt, lpa, pos, cond, clear_flag, rclear,
                                c->sz.cells, want_rho);
  if (c->half)
    return launch_half_density(c->L, c->g, s, c->t, pos, cond, false, clear_flag, rclear,
                               c->sz.cells, want_rho);
  if (lpa == 0)
    return launch_density_dyn(c->L, c->g, s, c->t, c->p.precision, pos, cond, clear_flag, rclear,
                              c->sz.cells, want_rho);
  return launch_density(c->L, c->g, s, c->t, c->p.precision, lpa, pos, cond, clear_flag, rclear,
                        c->sz.cells, want_rho);
}

hipError_t force_integrate_pass(md_ctx* c, const State& s, int lpa, const double4* pos_in,
                                double4* pos_out, int32_t* flag_next, int32_t* rflag_next) {
  if (c->multi)
    return launch_multi_force_integrate(c->L, c->g, s, c->mt, lpa, pos_in, pos_out, flag_next,
                                        rflag_next);
  if (c->half)
    return launch_half_force_integrate(c->L, c->g, s, c->t, pos_in, pos_out, flag_next,
                                       rflag_next);
  if (lpa == 0)
    return launch_force_integrate_dyn(c->L, c->g, s, c->t, c->p.precision, pos_in, pos_out,
                                      flag_next, rflag_next);
  return launch_force_integrate(c->L, c->g, s, c->t, c->p.precision, lpa, pos_in, pos_out,
                                flag_next, rflag_next);
}

hipError_t force_only_pass(md_ctx* c, const State& s, const double4* pos) {
  if (c->multi) return launch_multi_force_only(c->L, c->g, s, c->mt, c->lpa, pos);
  if (c->half) return launch_half_force_only(c->L, c->g, s, c->t, pos);
  if (c->lpa == 0) return launch_force_only_dyn(c->L, c->g, s, c->t, c->p.precision, pos);
  return launch_force_only(c->L, c->g, s, c->t, c->p.precision, c->lpa, pos);
}

// After an eager list build: the half form's half list and reverse slots
// (the density passes derive them; their rho and F' are recomputed later).
hipError_t half_reindex(md_ctx* c, const State& s) {
  if (!c->half) return hipSuccess;
  return launch_half_density(c->L, c->g, s, c->t, s.pos, nullptr, true, nullptr, nullptr,
                             c->sz.cells, false);
}

// Sort by cell (new slot order), then bin and build the list, leaving the
// bins zeroed.  Positions are wrapped; x_ref is reset.
md_status rebuild_sorted(md_ctx* c, bool sort) {
  State& s = c->st[c->cur];
  HIPC(c, hipMemsetAsync(c->status + SW_FLAG0, 0, 2 * sizeof(int32_t), c->L.stream));
  HIPC(c, hipMemsetAsync(s.rflag, 0, 2 * (size_t)c->n_rep * sizeof(int32_t), c->L.stream));
  if (sort) HIPC(c, launch_sort(c->L, c->g, s, c->sz.cells));
  HIPC(c, launch_zero_bins(c->L, s, c->sz.cells));
  HIPC(c, launch_bin(c->L, c->g, s, nullptr, nullptr));
  HIPC(c, launch_build(c->L, c->g, s, nullptr, nullptr));
  HIPC(c, launch_zero_bins(c->L, s, c->sz.cells));
  HIPC(c, half_reindex(c, s));
  return MD_OK;
}

md_status forces_now(md_ctx* c, bool want_rho) {
  State& s = c->st[c->cur];
  HIPC(c, density_pass(c, s, c->lpa, s.pos, nullptr, nullptr, nullptr, want_rho));
  HIPC(c, force_only_pass(c, s, s.pos));
  return MD_OK;
}

// Whether the persistent launch runs the small-system kernel: its atom tiles
// fit one thread slot each on the workgroups of one XCD (a workgroup takes
// 8 / lanes_per_atom tiles of 64 atoms at once), at most one XCD's share of
// the resident workgroups.
int64_t persist_small_blocks(const md_ctx* c) {
  if (c->lpa <= 0) return 0;  // per-replica schedules never run persistent
  const int per = std::max(1, (kPersistThreads / 64) / c->lpa);
  const int64_t need = (c->g.n_atiles + per - 1) / per;
  const int64_t fit = std::min<int64_t>(std::max(c->persist_cap, kXcd) / kXcd, kMaxSlots);
  return need <= fit ? need : 0;
}

// Workgroups of the persistent launch.  The small-system kernel asks for eight
// times the workgroups it wants working, since only those that run on XCD 0
// take part (workgroups go round-robin over the eight XCDs).  Otherwise:
// enough that each takes about one tile per pass, at least 8 and at most 64 (a
// barrier's cost grows with the count) and never more than can be resident; a
// multiple of the XCD count.
int persist_grid(const md_ctx* c) {
  if (const int64_t w = persist_small_blocks(c)) return (int)(w * kXcd);
  const int64_t tiles = (c->sz.n + 63) / 64 + c->n_rep;
  const int per = std::max(1, (kPersistThreads / 64) / c->lpa);
  int64_t g = (tiles + per - 1) / per;
  g = std::min<int64_t>(std::max<int64_t>(g, kXcd), 64);
  g = (g + kXcd - 1) / kXcd * kXcd;
  return (int)std::min<int64_t>(g, std::max(c->persist_cap, kXcd));
}

// One step with eager launches (parity cur -> 1 - cur).
md_status step_eager(md_ctx* c) {
  const int k = c->cur;
  State& s = c->st[k];
  int32_t* fl_cur = c->status + (k == 0 ? SW_FLAG0 : SW_FLAG1);
  int32_t* fl_nxt = c->status + (k == 0 ? SW_FLAG1 : SW_FLAG0);
  int32_t* rf_cur = s.rflag + (k == 0 ? 0 : c->n_rep);
  int32_t* rf_nxt = s.rflag + (k == 0 ? c->n_rep : 0);
  if (c->binbuild_grid && c->lpa > 0 && !c->multi && !c->half) {
    HIPC(c, launch_bin_build_density(c->L, c->g, s, c->t, c->p.precision, c->lpa, fl_cur, rf_cur,
                                     fl_nxt, rf_nxt, c->sz.cells, c->binbuild_grid));
  } else {
    HIPC(c, launch_bin(c->L, c->g, s, fl_cur, rf_cur));
    HIPC(c, launch_build(c->L, c->g, s, fl_cur, rf_cur));
    HIPC(c, density_pass(c, s, c->lpa, s.pos, fl_cur, fl_nxt, rf_nxt, false));
  }
  HIPC(c, force_integrate_pass(c, s, c->lpa, s.pos, c->st[1 - k].pos, fl_nxt, rf_nxt));
  c->cur = 1 - k;
  return MD_OK;
}

// Capture `len` steps starting from the current position buffer into one
// executable graph (the context's buffer parity is left unchanged).
md_status capture_steps(md_ctx* c, int len, hipGraphExec_t* out) {
  *out = nullptr;
  hipGraph_t gr = nullptr;
  HIPC(c, hipStreamBeginCapture(c->L.stream, hipStreamCaptureModeRelaxed));
  const int saved = c->cur;
  md_status rc = MD_OK;
  for (int k = 0; k < len && rc == MD_OK; ++k) rc = step_eager(c);
  c->cur = saved;
  hipError_t e = hipStreamEndCapture(c->L.stream, &gr);
  if (rc != MD_OK) {
    if (gr) (void)hipGraphDestroy(gr);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
  e = hipGraphInstantiate(out, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (e != hipSuccess) {
    *out = nullptr;
    return hip_fail(c, e, "hipGraphInstantiate");
  }
  // move the graph to the device now, so that its first launch costs no more than later ones
  e = hipGraphUpload(*out, c->L.stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipGraphUpload");
  return MD_OK;
}

md_status capture_chunk(md_ctx* c) {
  if (c->graph) return MD_OK;
  return capture_steps(c, c->p.chunk_steps, &c->graph);
}

constexpr size_t kMaxTailGraphs = 4;

// The graph of `len` steps from the current buffer parity (captured on first use).
md_status tail_graph(md_ctx* c, int len, hipGraphExec_t* out) {
  for (const md_ctx::Tail& t : c->tails)
    if (t.len == len && t.parity == c->cur) {
      *out = t.exec;
      return MD_OK;
    }
  if (c->tails.size() >= kMaxTailGraphs) {
    // the oldest may still run on the stream
    HIPC(c, hipStreamSynchronize(c->L.stream));
    (void)hipGraphExecDestroy(c->tails.front().exec);
    c->tails.erase(c->tails.begin());
  }
  md_status s = capture_steps(c, len, out);
  if (s != MD_OK) return s;
  c->tails.push_back(md_ctx::Tail{len, c->cur, *out});
  return MD_OK;
}

// Drop every captured graph (the schedule they were captured with changed).
md_status drop_graphs(md_ctx* c) {
  if (!c->graph && c->tails.empty()) return MD_OK;
  HIPC(c, hipStreamSynchronize(c->L.stream));
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  c->graph = nullptr;
  for (const md_ctx::Tail& t : c->tails) (void)hipGraphExecDestroy(t.exec);
  c->tails.clear();
  return MD_OK;
}

// Library tables from the caller's per-segment coefficients.
void build_tables(const md_spline* phi, const md_spline* rho, const md_spline* emb,
                  std::vector<double4>* rv, std::vector<double4>* pv, std::vector<double2>* d3,
                  std::vector<double4>* ev, std::vector<float4>* rv32, std::vector<float4>* da32,
                  std::vector<float2>* db32) {
  const int ns = rho->n_knots - 1;
  const double a = rho->inv_dx;
  rv->resize(ns);
  pv->resize(ns);
  d3->resize(3 * (size_t)ns);
  rv32->resize(ns);
  da32->resize(ns);
  db32->resize(ns);
  for (int k = 0; k < ns; ++k) {
    const double* r = rho->coef + 4 * k;
    const double* f = phi->coef + 4 * k;
    (*rv)[k] = make_double4(r[0], r[1], r[2], r[3]);
    (*pv)[k] = make_double4(f[0], f[1], f[2], f[3]);
    // derivative quadratics in t, pre-scaled by alpha: f'(t) = (c1 + 2 c2 t + 3 c3 t^2) alpha
    const double r0 = r[1] * a, r1 = 2.0 * r[2] * a, r2 = 3.0 * r[3] * a;
    const double p0 = f[1] * a, p1 = 2.0 * f[2] * a, p2 = 3.0 * f[3] * a;
    (*d3)[3 * k + 0] = make_double2(r0, r1);
    (*d3)[3 * k + 1] = make_double2(r2, p0);
    (*d3)[3 * k + 2] = make_double2(p1, p2);
    (*rv32)[k] = make_float4((float)r[0], (float)r[1], (float)r[2], (float)r[3]);
    (*da32)[k] = make_float4((float)r0, (float)r1, (float)r2, (float)p0);
    (*db32)[k] = make_float2((float)p1, (float)p2);
  }
  const int ne = emb->n_knots - 1;
  ev->resize(ne);
  for (int k = 0; k < ne; ++k) {
    const double* e = emb->coef + 4 * k;
    (*ev)[k] = make_double4(e[0], e[1], e[2], e[3]);
  }
}

}  // namespace

int md_internal_view(const md_ctx* c, mdk::CtxView* out) {
  if (!c || !out || !c->built) return MD_E_ORDER;
  out->g = c->g;
  out->s = c->st[c->cur];
  out->L = c->L;
  out->n_cells = c->sz.cells;
  out->n_rep = c->n_rep;
  return MD_OK;
}

extern "C" {

const char* md_status_string(md_status s) {
  switch (s) {
    case MD_OK: return "ok";
    case MD_E_ARG: return "invalid argument";
    case MD_E_BOX:
      return "periodic edge smaller than 2 (r_cut + skin) or fewer than 3 cells, or zero edge";
    case MD_E_TABLE: return "malformed spline table";
    case MD_E_NBR_OVERFLOW: return "neighbour list capacity exceeded";
    case MD_E_CELL_OVERFLOW: return "cell capacity exceeded";
    case MD_E_NONFINITE: return "non-finite position or force";
    case MD_E_HIP: return "HIP runtime error";
    case MD_E_ORDER: return "call out of order";
    case MD_E_LOST_ATOM: return "atom moved more than one box length";
    case MD_E_STALL:
      return "a grid barrier of a persistent launch timed out, or too few of its workgroups ran on "
             "the XCD that a one-XCD launch works on";
    case MD_E_WORKSPACE: return "workspace too small or misaligned";
    case MD_W_RHO_RANGE: return "warning: density beyond the embedding table";
    default: return "unknown status";
  }
}

const char* md_last_error(const md_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_last_error.c_str();
}

md_status md_workspace_size(const md_params* p, int32_t n_rep, const int64_t* rep_atoms,
                            const double* rep_box, size_t* bytes) {
  md_status s = check_params(p);
  if (s != MD_OK) return s;
  if (!bytes) return MD_E_ARG;
  std::vector<RepHost> reps;
  if ((s = gather_reps(p, n_rep, rep_atoms, rep_box, &reps)) != MD_OK) return s;
  LayoutSizes ls = layout(p, n_rep, reps);
  // the table sizes are not known here: reserve for up to 8192 knots each
  *bytes = carve(nullptr, p, n_rep, ls, 8192, 8192, nullptr);
  return MD_OK;
}

}  // extern "C"

namespace {

// Tables and masses of the multi-species form (validated by md_create_multi).
struct MultiIn {
  int32_t nt;
  const md_spline* phi;  // [nt * nt]
  const md_spline* rho;  // [nt]
  const md_spline* emb;  // [nt]
  const double* masses;  // [nt]
};

void multi_tables(const MultiIn& mi, std::vector<double4>* rseg, std::vector<double>* frow,
                  std::vector<double4>* pv, std::vector<double4>* rv, std::vector<double4>* ev) {
  const int nt = mi.nt;
  const int ns = mi.rho[0].n_knots - 1;
  const double a = mi.rho[0].inv_dx;
  const int S = multi_seg_stride(nt);
  auto value_rows = [&](const md_spline& sp, std::vector<double4>* out) {
    for (int k = 0; k < sp.n_knots - 1; ++k) {
      const double* c = sp.coef + 4 * (size_t)k;
      out->push_back(make_double4(c[0], c[1], c[2], c[3]));
    }
  };
  // derivative quadratic in t, pre-scaled by alpha: f'(t) = (c1 + 2 c2 t + 3 c3 t^2) alpha
  auto slope_row = [&](const md_spline& sp, int k, double* dst) {
    const double* c = sp.coef + 4 * (size_t)k;
    dst[0] = c[1] * a;
    dst[1] = 2.0 * c[2] * a;
    dst[2] = 3.0 * c[3] * a;
  };
  rseg->resize((size_t)ns * nt);
  frow->assign((size_t)ns * S, 0.0);
  for (int k = 0; k < ns; ++k) {
    double* seg = frow->data() + (size_t)k * S;
    for (int t = 0; t < nt; ++t) {
      const double* c = mi.rho[t].coef + 4 * (size_t)k;
      (*rseg)[(size_t)k * nt + t] = make_double4(c[0], c[1], c[2], c[3]);
      slope_row(mi.rho[t], k, seg + 3 * t);
    }
    for (int p = 0; p < nt; ++p)
      for (int q = p; q < nt; ++q) slope_row(mi.phi[p * nt + q], k, seg + 3 * multi_pair_row(nt, p, q));
  }
  for (int t = 0; t < nt; ++t) {
    value_rows(mi.rho[t], rv);
    value_rows(mi.emb[t], ev);
  }
  for (int q = 0; q < nt * nt; ++q) value_rows(mi.phi[q], pv);
}

md_status create_impl(md_ctx** out, const md_params* p, int32_t n_rep, const int64_t* rep_atoms,
                      const double* rep_box, const md_spline* phi, const md_spline* rho,
                      const md_spline* emb, const MultiIn* mi, void* workspace,
                      size_t workspace_bytes, void* stream) {
  if (!out) return MD_E_ARG;
  *out = nullptr;
  md_status s = check_params(p);
  if (s != MD_OK) return s;
  if (!valid_spline(phi) || !valid_spline(rho) || !valid_spline(emb)) return MD_E_TABLE;
  if (phi->n_knots != rho->n_knots || phi->inv_dx != rho->inv_dx || phi->x0 != 0.0 ||
      rho->x0 != 0.0 || phi->n_knots > 8192 || emb->n_knots > 8192)
    return MD_E_TABLE;
  // the r tables must reach r_cut
  if ((double)(rho->n_knots - 1) / rho->inv_dx < p->r_cut * (1.0 - 1e-12)) return MD_E_TABLE;
  std::vector<RepHost> reps;
  if ((s = gather_reps(p, n_rep, rep_atoms, rep_box, &reps)) != MD_OK) return s;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) return MD_E_WORKSPACE;
  LayoutSizes ls = layout(p, n_rep, reps);
  const size_t need = carve(nullptr, p, n_rep, ls, 8192, 8192, nullptr);
  if (workspace_bytes < need) return MD_E_WORKSPACE;

  md_ctx* c = new (std::nothrow) md_ctx();
  if (!c) return MD_E_ARG;
  c->p = *p;
  c->n_rep = n_rep;
  c->reps = reps;
  c->sz = ls;
  c->L.stream = reinterpret_cast<hipStream_t>(stream);
  c->L.atile_blocks = (int32_t)ls.atile_blocks;
  c->L.ctile_blocks = (int32_t)ls.ctile_blocks;
  c->lpa = p->lanes_per_atom ? p->lanes_per_atom : auto_lpa(ls.n / n_rep);

  Buffers b;
  carve(reinterpret_cast<char*>(workspace), p, n_rep, ls, rho->n_knots, emb->n_knots, &b);

  // replica table, atom tiles (64 atoms, aligned to replicas), cell tiles
  std::vector<RepDev> rd(n_rep);
  std::vector<AtomTile> at;
  std::vector<CellTile> ct;
  int64_t a0 = 0, c0 = 0;
  for (int r = 0; r < n_rep; ++r) {
    RepDev& d = rd[r];
    memset(&d, 0, sizeof(d));
    for (int k = 0; k < 3; ++k) {
      d.box[k] = reps[r].box[k];
      d.nc[k] = reps[r].nc[k];
      d.inv_cell[k] = (double)reps[r].nc[k] / reps[r].box[k];
    }
    d.atom0 = a0;
    d.n_atoms = (int32_t)reps[r].n;
    d.cell0 = (int32_t)c0;
    d.ncell = d.nc[0] * d.nc[1] * d.nc[2];
    d.open = reps[r].open;
    set_quanta(d);
    d.tile0 = (int32_t)at.size();
    d.ntiles = (int32_t)((reps[r].n + 63) / 64);
    for (int64_t t0 = 0; t0 < reps[r].n; t0 += 64)
      at.push_back(AtomTile{r, (int32_t)(a0 + t0), (int32_t)std::min<int64_t>(64, reps[r].n - t0), 0});
    for (int32_t q = 0; q < d.ncell; ++q) ct.push_back(CellTile{r, q});
    a0 += reps[r].n;
    c0 += d.ncell;
  }
  std::vector<AtomTile> atx = xcd_order(at, AtomTile{0, 0, 0, 0});
  std::vector<CellTile> ctx = xcd_order(ct, CellTile{0, -1});

  std::vector<double4> rv, pv, ev;
  std::vector<double2> d3;
  std::vector<float4> rv32, da32;
  std::vector<float2> db32;
  build_tables(phi, rho, emb, &rv, &pv, &d3, &ev, &rv32, &da32, &db32);

#define UP(dst, vec)                                                                          \
  do {                                                                                        \
    hipError_t e_ = hipMemcpy(dst, vec.data(), vec.size() * sizeof(vec[0]), hipMemcpyHostToDevice); \
    if (e_ != hipSuccess) {                                                                   \
      md_status r_ = hip_fail(c, e_, "upload " #vec);                                         \
      delete c;                                                                               \
      return r_;                                                                              \
    }                                                                                         \
  } while (0)
  UP(b.reps, rd);
  UP(b.atiles, atx);
  UP(b.ctiles, ctx);
  UP(b.rho_val, rv);
  UP(b.phi_val, pv);
  UP(b.dpair3, d3);
  UP(b.emb_val, ev);
  UP(b.rho_val32, rv32);
  UP(b.dpair_a32, da32);
  UP(b.dpair_b32, db32);
  if (mi) {
    std::vector<double4> mrs, mpv, mrv, mev;
    std::vector<double> mfr;
    multi_tables(*mi, &mrs, &mfr, &mpv, &mrv, &mev);
    UP(b.m_rho_seg, mrs);
    UP(b.m_frow, mfr);
    UP(b.m_phi_val, mpv);
    UP(b.m_rho_val, mrv);
    UP(b.m_emb_val, mev);
  }
#undef UP
  hipError_t e = hipMemset(b.status, 0, SW_WORDS * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemset(b.bin_cnt, 0, (size_t)ls.cells * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemset(b.cnt, 0, (size_t)ls.n * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemset(b.rflag, 0, 3 * (size_t)n_rep * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemset(b.cell_stat, 0, 3 * (size_t)ls.cells * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemset(b.frc, 0, (size_t)ls.n * sizeof(double4));
  if (e == hipSuccess && b.rfill) e = hipMemset(b.rfill, 0, (size_t)ls.n * sizeof(int32_t));
  if (e == hipSuccess && b.type) e = hipMemset(b.type, 0, (size_t)ls.n);
  if (e == hipSuccess && b.type_orig) e = hipMemset(b.type_orig, 0, (size_t)ls.n);
  if (e == hipSuccess && b.hcnt) e = hipMemset(b.hcnt, 0, (size_t)ls.n * sizeof(int32_t));
  if (e == hipSuccess && b.rcnt) e = hipMemset(b.rcnt, 0, (size_t)ls.n * sizeof(int32_t));
  if (e != hipSuccess) {
    md_status r_ = hip_fail(c, e, "hipMemset");
    delete c;
    return r_;
  }

  Geometry& g = c->g;
  g.reps = b.reps;
  g.atiles = b.atiles;
  g.ctiles = b.ctiles;
  g.n = ls.n;
  g.n_atiles = (int32_t)ls.atile_blocks;
  g.n_ctiles = (int32_t)ls.ctile_blocks;
  g.n_rep = n_rep;
  g.nbr_cap = p->nbr_capacity;
  g.cell_cap = p->cell_capacity;
  g.rc2 = p->r_cut * p->r_cut;
  g.rl2 = (p->r_cut + p->skin) * (p->r_cut + p->skin);
  g.lim2 = 0.25 * p->skin * p->skin;
  g.dt = p->dt;
  g.acc = p->ftm2v / p->mass;
  for (int q = 0; q < kMaxTypes; ++q) g.acc_t[q] = g.acc;
  if (mi)
    for (int q = 0; q < mi->nt; ++q) g.acc_t[q] = p->ftm2v / mi->masses[q];
  g.rc2f = (float)g.rc2;

  Tables& t = c->t;
  t.rho_val = b.rho_val;
  t.phi_val = b.phi_val;
  t.dpair3 = b.dpair3;
  t.emb_val = b.emb_val;
  t.rho_val32 = b.rho_val32;
  t.dpair_a32 = b.dpair_a32;
  t.dpair_b32 = b.dpair_b32;
  t.r_inv_dx = rho->inv_dx;
  t.r_inv_dx32 = (float)rho->inv_dx;
  t.e_x0 = emb->x0;
  t.e_inv_dx = emb->inv_dx;
  t.nr = rho->n_knots;
  t.ne = emb->n_knots;

  // persistent pair passes: one workgroup per CU, a multiple of the XCD count
  {
    int dev = 0, cus = 0, lds_max = 0;
    hipError_t e2 = hipGetDevice(&dev);
    if (e2 == hipSuccess) e2 = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e2 == hipSuccess)
      e2 = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e2 != hipSuccess) {
      md_status r_ = hip_fail(c, e2, "device attributes");
      delete c;
      return r_;
    }
    c->L.persist_blocks = std::max(kXcd, (cus / kXcd) * kXcd);
    if (force_lds_bytes(t, p->precision) > (size_t)lds_max ||
        density_lds_bytes(t, p->precision) > (size_t)lds_max) {
      delete c;
      return MD_E_TABLE;
    }
    e2 = allow_pair_lds(t, p->precision);
    if (e2 == hipSuccess && p->launch_mode == MD_LAUNCH_PERSISTENT) {
      if (persist_lds_bytes(t, p->precision, p->cell_capacity) > (size_t)lds_max) {
        delete c;
        return MD_E_ARG;
      }
      e2 = allow_persist_lds(t, p->precision, p->cell_capacity);
      // one workgroup per CU fits the LDS the kernel takes
      c->persist_cap = (c->L.persist_blocks / kXcd) * kXcd;
    }
    if (e2 == hipSuccess && p->list_mode == MD_LIST_HALF) e2 = allow_half_lds(t);
    // small systems: binning, list build and density pass of each step in one
    // launch (grid barriers between them), if every workgroup it needs fits at
    // once; one species, full list
    if (e2 == hipSuccess && p->list_mode == MD_LIST_FULL && !mi &&
        bbd_lds_bytes(t, p->precision, p->cell_capacity) <= (size_t)lds_max) {
      const int64_t waves = std::max<int64_t>(ls.ctile_blocks, ls.atile_blocks);
      int64_t grid = (waves + kPersistThreads / 64 - 1) / (kPersistThreads / 64);
      grid = (std::max<int64_t>(grid, kXcd) + kXcd - 1) / kXcd * kXcd;
      if (grid <= kMaxBinbuildGrid) {
        const int per_cu = bbd_blocks_per_cu(t, p->precision, p->cell_capacity);
        if (grid <= (int64_t)per_cu * cus) c->binbuild_grid = (int)grid;
      }
    }
    if (e2 != hipSuccess) {
      md_status r_ = hip_fail(c, e2, "hipFuncSetAttribute");
      delete c;
      return r_;
    }
  }

  State base{};
  base.vel = b.vel;
  base.xref = b.xref;
  base.sort_rec = b.sort_rec;
  base.snap_rec = b.snap_rec;
  base.frc = b.frc;
  base.rho = b.rho;
  base.epair = b.epair;
  base.id = b.id;
  base.cell_of = b.cell_of;
  base.nbr = b.nbr;
  base.cnt = b.cnt;
  base.bin_cnt = b.bin_cnt;
  base.bin_idx = b.bin_idx;
  base.cell_start = b.cell_start;
  base.cell_stat = b.cell_stat;
  base.status = b.status;
  base.rflag = b.rflag;
  base.sort_pos = b.sort_pos;
  base.sort_vel = b.sort_vel;
  base.sort_id = b.sort_id;
  base.partial = b.partial;
  base.hnbr = b.hnbr;
  base.hcnt = b.hcnt;
  base.rslot_u = b.rslot_u;
  base.rslot = b.rslot;
  base.rcnt = b.rcnt;
  base.rfill = b.rfill;
  base.pval = b.pval;
  base.qval = b.qval;
  base.own_rho = b.own_rho;
  base.own_f = b.own_f;
  c->half = (p->list_mode == MD_LIST_HALF);
  base.type = b.type;
  base.type_orig = b.type_orig;
  base.sort_type = b.sort_type;
  if (mi) {
    c->multi = true;
    MultiTables& m = c->mt;
    m.rho_seg = b.m_rho_seg;
    m.frow = b.m_frow;
    m.phi_val = b.m_phi_val;
    m.rho_val = b.m_rho_val;
    m.emb_val = b.m_emb_val;
    m.seg_stride = multi_seg_stride(mi->nt);
    m.lds_seg0 = multi_force_lds_seg0(mi->rho[0].n_knots, mi->nt);
    for (int q = 0; q < kMaxTypes * kMaxTypes; ++q) m.pair_row[q] = 0;
    for (int p = 0; p < mi->nt; ++p)
      for (int q = 0; q < mi->nt; ++q) m.pair_row[p * mi->nt + q] = multi_pair_row(mi->nt, p, q);
    m.r_inv_dx = mi->rho[0].inv_dx;
    m.e_x0 = mi->emb[0].x0;
    m.e_inv_dx = mi->emb[0].inv_dx;
    m.nr = mi->rho[0].n_knots;
    m.ne = mi->emb[0].n_knots;
    m.n_types = mi->nt;
    hipError_t e3 = allow_multi_lds(m);
    if (e3 != hipSuccess) {
      md_status r_ = hip_fail(c, e3, "hipFuncSetAttribute");
      delete c;
      return r_;
    }
  }
  c->st[0] = base;
  c->st[1] = base;
  c->st[0].pos = b.pos0;
  c->st[0].pos_alt = b.pos1;
  c->st[1].pos = b.pos1;
  c->st[1].pos_alt = b.pos0;
  c->st[0].rec = b.rec0;
  c->st[0].rec_alt = b.rec1;
  c->st[1].rec = b.rec1;
  c->st[1].rec_alt = b.rec0;
  c->pos_buf[0] = b.pos0;
  c->pos_buf[1] = b.pos1;
  c->snap_pos = b.snap_pos;
  c->snap_vel = b.snap_vel;
  c->ptile_buf = b.ptiles;
  c->g.ptiles = b.ptiles;
  c->g.n_ptiles = 0;
  c->energy_dev = b.energy;
  c->status = b.status;
  *out = c;
  return MD_OK;
}

bool same_coef(const md_spline& a, const md_spline& b) {
  return a.n_knots == b.n_knots && a.x0 == b.x0 && a.inv_dx == b.inv_dx &&
         std::memcmp(a.coef, b.coef, 4 * sizeof(double) * (size_t)(a.n_knots - 1)) == 0;
}

}  // namespace

extern "C" {

md_status md_create(md_ctx** out, const md_params* p, int32_t n_rep, const int64_t* rep_atoms,
                    const double* rep_box, const md_spline* phi, const md_spline* rho,
                    const md_spline* emb, void* workspace, size_t workspace_bytes, void* stream) {
  if (p && p->n_types > 1) return MD_E_ARG;  // several types: md_create_multi
  return create_impl(out, p, n_rep, rep_atoms, rep_box, phi, rho, emb, nullptr, workspace,
                     workspace_bytes, stream);
}

md_status md_create_multi(md_ctx** out, const md_params* p, int32_t n_rep,
                          const int64_t* rep_atoms, const double* rep_box, const md_spline* phi,
                          const md_spline* rho, const md_spline* emb, const double* masses,
                          void* workspace, size_t workspace_bytes, void* stream) {
  if (!out) return MD_E_ARG;
  *out = nullptr;
  if (!p || p->n_types < 2 || p->n_types > kMaxTypes || !phi || !rho || !emb || !masses)
    return MD_E_ARG;
  const int nt = p->n_types;
  for (int t = 0; t < nt; ++t)
    if (!(masses[t] > 0.0) || !std::isfinite(masses[t])) return MD_E_ARG;
  // every rho and phi table on the grid of rho[0], every F table on the grid of emb[0]
  for (int q = 0; q < nt * nt; ++q) {
    if (!valid_spline(&phi[q])) return MD_E_TABLE;
    if (phi[q].n_knots != rho[0].n_knots || phi[q].inv_dx != rho[0].inv_dx || phi[q].x0 != 0.0)
      return MD_E_TABLE;
  }
  for (int t = 0; t < nt; ++t) {
    if (!valid_spline(&rho[t]) || !valid_spline(&emb[t])) return MD_E_TABLE;
    if (rho[t].n_knots != rho[0].n_knots || rho[t].inv_dx != rho[0].inv_dx || rho[t].x0 != 0.0)
      return MD_E_TABLE;
    if (emb[t].n_knots != emb[0].n_knots || emb[t].inv_dx != emb[0].inv_dx ||
        emb[t].x0 != emb[0].x0)
      return MD_E_TABLE;
  }
  // phi_ab and phi_ba must be one function (else no energy is conserved)
  for (int a = 0; a < nt; ++a)
    for (int b = a + 1; b < nt; ++b)
      if (!same_coef(phi[a * nt + b], phi[b * nt + a])) return MD_E_TABLE;
  const MultiIn mi{nt, phi, rho, emb, masses};
  return create_impl(out, p, n_rep, rep_atoms, rep_box, &phi[0], &rho[0], &emb[0], &mi, workspace,
                     workspace_bytes, stream);
}

size_t md_workspace_bytes(const md_params* p, int32_t n_rep, const int64_t* rep_atoms,
                          const double* rep_box) {
  size_t b = 0;
  return md_workspace_size(p, n_rep, rep_atoms, rep_box, &b) == MD_OK ? b : 0;
}

md_status md_init_batch(md_ctx** out, const md_params* p, int32_t n_rep,
                        const int64_t* rep_atoms, const double* rep_box, const md_spline* phi,
                        const md_spline* rho, const md_spline* emb, const double* x,
                        const double* v, void* workspace, size_t workspace_bytes,
                        void* stream) {
  if (!out) return MD_E_ARG;
  *out = nullptr;
  if (!x || !v) return MD_E_ARG;
  md_ctx* c = nullptr;
  md_status s = md_create(&c, p, n_rep, rep_atoms, rep_box, phi, rho, emb, workspace,
                          workspace_bytes, stream);
  if (s != MD_OK) return s;
  s = md_set_state(c, x, v);
  if (s < 0) {
    g_last_error = c->err;
    md_destroy(c);
    return s;
  }
  *out = c;
  return s;
}

md_status md_init(md_ctx** out, const md_params* p, int64_t n_atoms, const double* box,
                  const md_spline* phi, const md_spline* rho, const md_spline* emb,
                  const double* x, const double* v, void* workspace, size_t workspace_bytes,
                  void* stream) {
  return md_init_batch(out, p, 1, &n_atoms, box, phi, rho, emb, x, v, workspace,
                       workspace_bytes, stream);
}

md_status md_set_types(md_ctx* c, const int32_t* type) {
  if (!c || !type) return MD_E_ARG;
  if (!c->multi) return MD_E_ARG;
  HIPC(c, hipMemsetAsync(c->status + SW_TYPE_CHECK, 0, sizeof(int32_t), c->L.stream));
  HIPC(c, launch_set_types(c->L, c->g, c->st[c->cur], type, c->mt.n_types, c->has_state));
  int32_t w[SW_WORDS];
  md_status s = read_status(c, w);
  if (s != MD_OK) return s;
  // forces and the half-step velocities belong to the old types
  c->built = false;
  return w[SW_TYPE_CHECK] ? MD_E_ARG : MD_OK;
}

md_status md_set_state(md_ctx* c, const double* x, const double* v) {
  if (!c || !x || !v) return MD_E_ARG;
  c->cur = 0;
  HIPC(c, hipMemsetAsync(c->status, 0, SW_WORDS * sizeof(int32_t), c->L.stream));
  HIPC(c, launch_import(c->L, c->g, c->st[0], x, v));
  c->has_state = true;
  c->built = false;
  c->v_half = false;
  int32_t w[SW_WORDS];
  md_status s = read_status(c, w);
  if (s != MD_OK) return s;
  return status_code(w[SW_BITS] & ST_ERR_MASK);
}

md_status md_build_neighbors(md_ctx* c) {
  if (!c) return MD_E_ARG;
  if (!c->has_state) return MD_E_ORDER;
  md_status s = rebuild_sorted(c, true);
  if (s != MD_OK) return s;
  if ((s = forces_now(c, false)) != MD_OK) return s;
  if (!c->v_half) {
    HIPC(c, launch_halfkick(c->L, c->g, c->st[c->cur], -0.5 * c->p.dt));
    c->v_half = true;
  }
  c->chunks_since_sort = 0;
  HIPC(c, hipMemsetAsync(c->status + SW_STEPS, 0, 2 * sizeof(int32_t), c->L.stream));
  // a clean rollback point exists from here on
  HIPC(c, launch_snapshot(c->L, c->g, c->st[c->cur], c->snap_pos, c->snap_vel, false));
  int32_t w[SW_WORDS];
  if ((s = read_status(c, w)) != MD_OK) return s;
  s = status_code(w[SW_BITS]);
  c->built = (s >= 0);
  return s;
}

md_status md_step(md_ctx* c, int64_t n) {
  if (!c || n < 0) return MD_E_ARG;
  if (!c->built) return MD_E_ORDER;
  md_status s;
  int64_t done = 0;
  const int chunk = c->p.chunk_steps;
  // every graph and persistent launch below snapshots first; the persistent
  // form's kernel-by-kernel steps need one from here
  if (c->p.launch_mode == MD_LAUNCH_PERSISTENT)
    HIPC(c, launch_snapshot(c->L, c->g, c->st[c->cur], c->snap_pos, c->snap_vel, false));
  while (done < n) {
    if (c->cur == 0 && n - done >= chunk) {
      if (c->p.sort_every > 0 && c->chunks_since_sort >= c->p.sort_every) {
        if ((s = rebuild_sorted(c, true)) != MD_OK) return s;
        c->chunks_since_sort = 0;
      }
      if (c->p.launch_mode == MD_LAUNCH_PERSISTENT) {
        HIPC(c, launch_snapshot(c->L, c->g, c->st[0], c->snap_pos, c->snap_vel, false));
        HIPC(c, hipMemsetAsync(c->status + SW_BAR_COUNT, 0, (SW_WORDS - SW_BAR_COUNT) * sizeof(int32_t), c->L.stream));
        HIPC(c, launch_persist(c->L, c->g, c->st[0], c->st[1], c->t, c->p.precision, c->lpa,
                               chunk, c->sz.cells, persist_grid(c),
                               persist_small_blocks(c) > 0 ? 1 : 0));
      } else {
        if ((s = capture_chunk(c)) != MD_OK) return s;
        HIPC(c, launch_snapshot(c->L, c->g, c->st[0], c->snap_pos, c->snap_vel, false));
        HIPC(c, hipGraphLaunch(c->graph, c->L.stream));
      }
      ++c->chunks_since_sort;
      done += chunk;
    } else if (c->p.launch_mode == MD_LAUNCH_PERSISTENT) {
      if ((s = step_eager(c)) != MD_OK) return s;
      ++done;
    } else {
      // fewer steps than a chunk, or an odd buffer parity: one shorter graph
      // (chunk_steps - 1 is odd, so a parity-1 start ends on buffer 0)
      const int len = (int)std::min<int64_t>(n - done, chunk - 1);
      hipGraphExec_t ge = nullptr;
      if ((s = tail_graph(c, len, &ge)) != MD_OK) return s;
      HIPC(c, launch_snapshot(c->L, c->g, c->st[c->cur], c->snap_pos, c->snap_vel, false));
      HIPC(c, hipGraphLaunch(ge, c->L.stream));
      if (len & 1) c->cur = 1 - c->cur;
      done += len;
    }
  }
  int32_t w[SW_WORDS];
  if ((s = read_status(c, w)) != MD_OK) return s;
  s = status_code(w[SW_BITS]);
  if (s < 0) {
    // roll back to the last clean snapshot (its step count comes with it)
    // and rebuild the list there
    c->cur = 0;
    HIPC(c, hipMemsetAsync(c->status + SW_BITS, 0, sizeof(int32_t), c->L.stream));
    // a barrier left by a stalled launch starts again from no arrivals
    HIPC(c, hipMemsetAsync(c->status + SW_BAR_COUNT, 0, (SW_WORDS - SW_BAR_COUNT) * sizeof(int32_t), c->L.stream));
    HIPC(c, launch_snapshot(c->L, c->g, c->st[0], c->snap_pos, c->snap_vel, true));
    md_status r = rebuild_sorted(c, true);
    if (r == MD_OK) r = forces_now(c, false);
    if (r == MD_OK) r = read_status(c, w);
    // the list built at the restored positions can overflow in turn (it was
    // last built at other positions): then no list is valid and md_step
    // refuses to run until md_set_state starts over
    if (r != MD_OK || status_code(w[SW_BITS]) < 0) c->built = false;
    return s;
  }
  return s;
}

md_status md_prepare(md_ctx* c, int64_t n) {
  if (!c || n < 0) return MD_E_ARG;
  if (!c->built) return MD_E_ORDER;
  if (c->p.launch_mode == MD_LAUNCH_PERSISTENT) return MD_OK;
  // walk md_step's launch plan from the current buffer parity
  const int chunk = c->p.chunk_steps;
  const int saved = c->cur;
  md_status s = MD_OK;
  for (int64_t done = 0; done < n && s == MD_OK;) {
    if (c->cur == 0 && n - done >= chunk) {
      s = capture_chunk(c);
      done += (n - done) / chunk * chunk;
    } else {
      const int len = (int)std::min<int64_t>(n - done, chunk - 1);
      hipGraphExec_t ge = nullptr;
      s = tail_graph(c, len, &ge);
      if (len & 1) c->cur = 1 - c->cur;
      done += len;
    }
  }
  c->cur = saved;
  return s;
}

md_status md_energy(md_ctx* c, double* pe, double* ke) {
  if (!c) return MD_E_ARG;
  if (!c->has_state) return MD_E_ORDER;
  md_status s;
  if (!c->built) {
    if ((s = rebuild_sorted(c, false)) != MD_OK) return s;
  }
  if ((s = forces_now(c, false)) != MD_OK) return s;
  State& st = c->st[c->cur];
  Geometry g = c->g;
  if (!c->v_half) {
    // velocities are on-step: no half-kick correction
    g.dt = 0.0;
  }
  if (c->multi)
    HIPC(c, launch_multi_energy(c->L, g, st, c->mt, c->energy_dev, c->n_rep));
  else
    HIPC(c, launch_energy(c->L, g, st, c->t, c->energy_dev, c->n_rep));
  std::vector<double> h(2 * (size_t)c->n_rep);
  HIPC(c, hipMemcpyAsync(h.data(), c->energy_dev, h.size() * sizeof(double),
                         hipMemcpyDeviceToHost, c->L.stream));
  HIPC(c, hipStreamSynchronize(c->L.stream));
  for (int r = 0; r < c->n_rep; ++r) {
    if (pe) pe[r] = h[2 * r];
    if (ke) ke[r] = h[2 * r + 1];
  }
  int32_t w[SW_WORDS];
  if ((s = read_status(c, w)) != MD_OK) return s;
  return status_code(w[SW_BITS]);
}

md_status md_get_state(md_ctx* c, double* x, double* v, double* f) {
  if (!c) return MD_E_ARG;
  if (!c->has_state) return MD_E_ORDER;
  md_status s;
  if (c->built) {
    if ((s = forces_now(c, true)) != MD_OK) return s;
  } else if (f) {
    return MD_E_ORDER;
  }
  const double coef = c->v_half ? 0.5 * c->p.dt : 0.0;
  HIPC(c, launch_export(c->L, c->g, c->st[c->cur], x, v, f, nullptr, nullptr, coef));
  HIPC(c, hipStreamSynchronize(c->L.stream));
  return MD_OK;
}

md_status md_compute_forces(md_ctx* c, double* f, double* rho, double* fp) {
  if (!c) return MD_E_ARG;
  if (!c->built) return MD_E_ORDER;
  md_status s;
  if ((s = forces_now(c, true)) != MD_OK) return s;
  HIPC(c, launch_export(c->L, c->g, c->st[c->cur], nullptr, nullptr, f, rho, fp, 0.0));
  int32_t w[SW_WORDS];
  if ((s = read_status(c, w)) != MD_OK) return s;
  return status_code(w[SW_BITS]);
}

md_status md_stats(md_ctx* c, md_stats_t* o) {
  if (!c || !o) return MD_E_ARG;
  HIPC(c, launch_cell_stats(c->L, c->st[c->cur], c->sz.cells));
  int32_t w[SW_WORDS];
  md_status s = read_status(c, w);
  if (s != MD_OK) return s;
  int64_t v64[3];
  memcpy(&v64[0], &w[SW_STEPS], 8);
  memcpy(&v64[1], &w[SW_REBUILDS], 8);
  memcpy(&v64[2], &w[SW_LIST_TOTAL], 8);
  o->steps = v64[0];
  o->rebuilds = v64[1];
  o->list_entries = v64[2];
  o->max_list = w[SW_MAX_LIST];
  o->max_cell = w[SW_MAX_CELL];
  o->status_bits = w[SW_BITS];
  o->reserved = 0;
  return MD_OK;
}

md_status md_get_cells(md_ctx* c, int32_t* cell) {
  if (!c || !cell) return MD_E_ARG;
  if (!c->built) return MD_E_ORDER;
  HIPC(c, launch_export_cells(c->L, c->g, c->st[c->cur], cell));
  HIPC(c, hipStreamSynchronize(c->L.stream));
  return MD_OK;
}

md_status md_get_neighbors(md_ctx* c, int32_t* cnt, int32_t* nbr, int32_t cap_out) {
  if (!c || !cnt || !nbr || cap_out < 1) return MD_E_ARG;
  if (!c->built) return MD_E_ORDER;
  HIPC(c, launch_export_nbrs(c->L, c->g, c->st[c->cur], cnt, nbr, cap_out));
  HIPC(c, hipStreamSynchronize(c->L.stream));
  return MD_OK;
}

md_status md_launch_pass(md_ctx* c, int32_t pass, int32_t reps) {
  if (!c || reps < 0 || pass < 0 || pass > 4) return MD_E_ARG;
  if (!c->built) return MD_E_ORDER;
  State& s = c->st[c->cur];
  if (reps == 0) return MD_OK;
  switch (pass) {
    case 0:
      for (int r = 0; r < reps; ++r)
        HIPC(c, density_pass(c, s, c->lpa, s.pos, nullptr, nullptr, nullptr, false));
      break;
    case 1:
      // the kernel md_step runs, writing the other position buffer; positions,
      // velocities and the step counter come back from a snapshot afterwards
      HIPC(c, launch_snapshot(c->L, c->g, s, c->snap_pos, c->snap_vel, false));
      for (int r = 0; r < reps; ++r)
        HIPC(c, force_integrate_pass(c, s, c->lpa, s.pos, c->st[1 - c->cur].pos,
                                     c->status + SW_SCRATCH, s.rflag + 2 * c->n_rep));
      HIPC(c, launch_snapshot(c->L, c->g, s, c->snap_pos, c->snap_vel, true));
      break;
    case 4:
      // the same kernel with no snapshot around it: velocities advance on every
      // launch while positions are read from the unchanged current buffer
      for (int r = 0; r < reps; ++r)
        HIPC(c, force_integrate_pass(c, s, c->lpa, s.pos, c->st[1 - c->cur].pos,
                                     c->status + SW_SCRATCH, s.rflag + 2 * c->n_rep));
      break;
    case 2:
      // list build from freshly filled bins (one binning first, bins zeroed after)
      HIPC(c, launch_zero_bins(c->L, s, c->sz.cells));
      HIPC(c, launch_bin(c->L, c->g, s, nullptr, nullptr));
      for (int r = 0; r < reps; ++r) HIPC(c, launch_build(c->L, c->g, s, nullptr, nullptr));
      HIPC(c, launch_zero_bins(c->L, s, c->sz.cells));
      HIPC(c, half_reindex(c, s));
      break;
    default:
      // binning (wraps positions and resets x_ref), then one build keeps the list consistent
      for (int r = 0; r < reps; ++r) {
        HIPC(c, launch_zero_bins(c->L, s, c->sz.cells));
        HIPC(c, launch_bin(c->L, c->g, s, nullptr, nullptr));
      }
      HIPC(c, launch_build(c->L, c->g, s, nullptr, nullptr));
      HIPC(c, launch_zero_bins(c->L, s, c->sz.cells));
      HIPC(c, half_reindex(c, s));
      break;
  }
  return MD_OK;
}

md_status md_set_schedule(md_ctx* c, int32_t lanes_per_atom) {
  if (!c) return MD_E_ARG;
  const int l = lanes_per_atom;
  if (!(l == 1 || l == 2 || l == 4 || l == 8)) return MD_E_ARG;
  if (l != c->lpa) {
    md_status s = drop_graphs(c);
    if (s != MD_OK) return s;
  }
  c->lpa = l;
  c->rep_lpa.clear();
  return MD_OK;
}

md_status md_set_replica_schedule(md_ctx* c, const int32_t* lanes) {
  if (!c || !lanes) return MD_E_ARG;
  for (int r = 0; r < c->n_rep; ++r)
    if (!(lanes[r] == 1 || lanes[r] == 2 || lanes[r] == 4 || lanes[r] == 8)) return MD_E_ARG;
  bool same = true;
  for (int r = 1; r < c->n_rep; ++r) same = same && lanes[r] == lanes[0];
  // one value for all, or a form whose passes walk atom tiles only: the uniform kernels
  if (same) return md_set_schedule(c, lanes[0]);
  if (c->half || c->multi || c->p.launch_mode == MD_LAUNCH_PERSISTENT) return MD_E_ARG;
  // pair tiles: replica r in tiles of 64 / lanes[r] atoms, in replica order, then
  // each XCD's contiguous share at positions xcd, xcd + 8, ...
  std::vector<PairTile> pt;
  int64_t a0 = 0;
  for (int r = 0; r < c->n_rep; ++r) {
    const int64_t per = 64 / lanes[r];
    for (int64_t t0 = 0; t0 < c->reps[r].n; t0 += per)
      pt.push_back(PairTile{r, (int32_t)(a0 + t0), (int32_t)std::min<int64_t>(per, c->reps[r].n - t0),
                            lanes[r]});
    a0 += c->reps[r].n;
  }
  std::vector<PairTile> ptx = xcd_order(pt, PairTile{0, 0, 0, 1});
  md_status s = drop_graphs(c);
  if (s != MD_OK) return s;
  HIPC(c, hipStreamSynchronize(c->L.stream));
  HIPC(c, hipMemcpy(c->ptile_buf, ptx.data(), ptx.size() * sizeof(PairTile),
                    hipMemcpyHostToDevice));
  c->g.n_ptiles = (int64_t)ptx.size();
  c->rep_lpa.assign(lanes, lanes + c->n_rep);
  c->lpa = 0;
  return MD_OK;
}

md_status md_get_replica_schedule(md_ctx* c, int32_t* lanes) {
  if (!c || !lanes) return MD_E_ARG;
  for (int r = 0; r < c->n_rep; ++r) lanes[r] = c->rep_lpa.empty() ? c->lpa : c->rep_lpa[r];
  return MD_OK;
}

}  // extern "C"

namespace {

// Microseconds per round of the step's density and force+integrate kernels
// under the schedule `lpa` (a uniform value, or 0 for the pair-tile table):
// one untimed round, then reps timed rounds (events on the context stream).
// The rebuild flags written go to scratch words; the caller restores the state.
md_status time_rounds(md_ctx* c, int lpa, int reps, hipEvent_t e0, hipEvent_t e1, float* us) {
  State& s = c->st[c->cur];
  // the kernels a step launches: a small system's density pass runs inside
  // its fused binning + build + density node (here with a flag that is never
  // set, as in the steps without a rebuild)
  const bool fused = c->binbuild_grid && lpa > 0 && !c->multi && !c->half;
  for (int r = 0; r <= reps; ++r) {
    if (r == 1) HIPC(c, hipEventRecord(e0, c->L.stream));
    if (fused)
      HIPC(c, launch_bin_build_density(c->L, c->g, s, c->t, c->p.precision, lpa,
                                       c->status + SW_ZERO, nullptr, nullptr, nullptr, c->sz.cells,
                                       c->binbuild_grid));
    else
      HIPC(c, density_pass(c, s, lpa, s.pos, nullptr, nullptr, nullptr, false));
    HIPC(c, force_integrate_pass(c, s, lpa, s.pos, c->st[1 - c->cur].pos, c->status + SW_SCRATCH,
                                 s.rflag + 2 * c->n_rep));
  }
  float ms = 0.f;
  HIPC(c, hipEventRecord(e1, c->L.stream));
  HIPC(c, hipEventSynchronize(e1));
  HIPC(c, hipEventElapsedTime(&ms, e0, e1));
  *us = 1000.f * ms / (float)reps;
  return MD_OK;
}

// Replica size class of the per-replica search: up to 2,048 atoms, up to
// 8,192, larger.
int size_class(int64_t n) { return n <= 2048 ? 0 : (n <= 8192 ? 1 : 2); }

md_status autotune_impl(md_ctx* c, int32_t reps, hipEvent_t e0, hipEvent_t e1, int* best_lpa,
                        float* best_us) {
  const int cand[4] = {1, 2, 4, 8};
  // the half-list passes run one lane per atom: time that one schedule
  const int n_cand = c->half ? 1 : 4;
  float per[4] = {3.4e38f, 3.4e38f, 3.4e38f, 3.4e38f};
  md_status rc;
  // two sweeps over the uniform candidates, keeping each one's faster sweep
  for (int sweep = 0; sweep < 2; ++sweep)
    for (int q = 0; q < n_cand; ++q) {
      float us = 0.f;
      if ((rc = time_rounds(c, cand[q], reps, e0, e1, &us)) != MD_OK) return rc;
      per[q] = std::min(per[q], us);
    }
  float best = 3.4e38f;
  int pick = c->lpa > 0 ? c->lpa : 1;
  for (int q = 0; q < n_cand; ++q)
    if (per[q] < best) {
      best = per[q];
      pick = cand[q];
    }
  *best_lpa = pick;
  *best_us = best;
  if ((rc = md_set_schedule(c, pick)) != MD_OK) return rc;
  if (c->n_rep < 2 || c->half || c->multi || c->p.launch_mode == MD_LAUNCH_PERSISTENT)
    return MD_OK;
  // batched replicas: one lanes-per-atom value per size class, found class by
  // class from the uniform choice (two passes), kept if it beats that choice
  std::vector<int32_t> lanes(c->n_rep, pick);
  bool present[3] = {false, false, false};
  for (int r = 0; r < c->n_rep; ++r) present[size_class(c->reps[r].n)] = true;
  float cur_best = best;
  for (int pass = 0; pass < 2; ++pass)
    for (int k = 0; k < 3; ++k) {
      if (!present[k]) continue;
      int keep = -1;
      for (int q = 0; q < 4; ++q) {
        std::vector<int32_t> trial = lanes;
        for (int r = 0; r < c->n_rep; ++r)
          if (size_class(c->reps[r].n) == k) trial[r] = cand[q];
        if ((rc = md_set_replica_schedule(c, trial.data())) != MD_OK) return rc;
        float us = 0.f;
        if ((rc = time_rounds(c, c->lpa, reps, e0, e1, &us)) != MD_OK) return rc;
        if (us < cur_best) {
          cur_best = us;
          keep = cand[q];
        }
      }
      if (keep > 0)
        for (int r = 0; r < c->n_rep; ++r)
          if (size_class(c->reps[r].n) == k) lanes[r] = keep;
    }
  if (cur_best < best) {
    *best_us = cur_best;
    return md_set_replica_schedule(c, lanes.data());
  }
  return md_set_schedule(c, pick);
}

}  // namespace

extern "C" {

md_status md_autotune(md_ctx* c, int32_t reps, int32_t* best_lpa, float* best_us) {
  if (!c || reps < 1) return MD_E_ARG;
  if (!c->built) return MD_E_ORDER;
  hipEvent_t e0, e1;
  HIPC(c, hipEventCreate(&e0));
  HIPC(c, hipEventCreate(&e1));
  // velocities and positions come back from a snapshot after the sweeps
  md_status rc = MD_OK;
  hipError_t e = launch_snapshot(c->L, c->g, c->st[c->cur], c->snap_pos, c->snap_vel, false);
  if (e != hipSuccess) rc = hip_fail(c, e, "autotune snapshot");
  int pick = 0;
  float best = 0.f;
  if (rc == MD_OK) rc = autotune_impl(c, reps, e0, e1, &pick, &best);
  e = launch_snapshot(c->L, c->g, c->st[c->cur], c->snap_pos, c->snap_vel, true);
  if (rc == MD_OK && e != hipSuccess) rc = hip_fail(c, e, "autotune restore");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != MD_OK) return rc;
  if (best_lpa) *best_lpa = pick;
  if (best_us) *best_us = best;
  return MD_OK;
}

void md_destroy(md_ctx* c) {
  if (!c) return;
  (void)drop_graphs(c);
  delete c;
}

}  // extern "C"

// ================================================== allocation-free force evaluation
//
// md_forces_static: the force evaluation of md_create + md_set_state +
// md_build_neighbors + md_compute_forces for one box, with every intermediate
// (replica and tile tables, spline rows, sorted state, bins, neighbour list,
// status words) in `scratch`, a fixed device array that each GPU holds until
// the process ends.  Nothing is allocated: the tables come from the caller's
// device coefficient arrays through a set-up kernel, and the status returns by
// one small copy.  Calls that overlap on one GPU share the array and race.

#include <mutex>

static constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

struct StaticDevice {
  char* ptr = nullptr;  // device address of `scratch` on this GPU
  int persist_blocks = 0;
  int lds_max = 0;
};
constexpr int kStaticDevices = 64;
std::mutex g_static_mu;
StaticDevice g_static[kStaticDevices];

// Address of `scratch` and launch sizes on the current device, looked up once
// per device (the array's name is a host-side stand-in, not a device address).
md_status static_device(StaticDevice* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
  if (dev < 0 || dev >= kStaticDevices) return MD_E_ARG;
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticDevice& d = g_static[dev];
  if (!d.ptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
    int cus = 0, lds = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "device attributes");
    d.persist_blocks = std::max(kXcd, (cus / kXcd) * kXcd);
    d.lds_max = lds;
    d.ptr = static_cast<char*>(p);
  }
  *out = d;
  return MD_OK;
}

// Set-up of one box in the scratch array: replica table, XCD-ordered atom and
// cell tiles (as md_create lays them out), spline rows from the caller's
// device coefficients (the host layout of md_create's build_tables, same
// arithmetic), and zeroed counters.
__global__ __launch_bounds__(256) void k_static_setup(RepDev rep, Geometry g, State s, Tables t,
                                                      const double* __restrict__ phi_c,
                                                      const double* __restrict__ rho_c,
                                                      const double* __restrict__ emb_c,
                                                      int64_t ncells) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t0 == 0) *const_cast<RepDev*>(g.reps) = rep;
  const int64_t ntiles = rep.ntiles;
  const int64_t aper = (ntiles + kXcd - 1) / kXcd;
  for (int64_t b = t0; b < g.n_atiles; b += stride) {
    const int64_t q = (b % kXcd) * aper + b / kXcd;
    AtomTile a{0, 0, 0, 0};
    if (q < ntiles) a = AtomTile{0, (int32_t)(64 * q), (int32_t)min<int64_t>(64, g.n - 64 * q), 0};
    const_cast<AtomTile*>(g.atiles)[b] = a;
  }
  const int64_t cper = (ncells + kXcd - 1) / kXcd;
  for (int64_t b = t0; b < g.n_ctiles; b += stride) {
    const int64_t q = (b % kXcd) * cper + b / kXcd;
    const_cast<CellTile*>(g.ctiles)[b] = CellTile{0, q < ncells ? (int32_t)q : -1};
  }
  const double a = t.r_inv_dx;
  for (int64_t k = t0; k < t.nr - 1; k += stride) {
    const double* r = rho_c + 4 * k;
    const double* f = phi_c + 4 * k;
    const_cast<double4*>(t.rho_val)[k] = make_double4(r[0], r[1], r[2], r[3]);
    const_cast<double4*>(t.phi_val)[k] = make_double4(f[0], f[1], f[2], f[3]);
    const double r0 = r[1] * a, r1 = 2.0 * r[2] * a, r2 = 3.0 * r[3] * a;
    const double p0 = f[1] * a, p1 = 2.0 * f[2] * a, p2 = 3.0 * f[3] * a;
    double2* d3 = const_cast<double2*>(t.dpair3) + 3 * k;
    d3[0] = make_double2(r0, r1);
    d3[1] = make_double2(r2, p0);
    d3[2] = make_double2(p1, p2);
    const_cast<float4*>(t.rho_val32)[k] =
        make_float4((float)r[0], (float)r[1], (float)r[2], (float)r[3]);
    const_cast<float4*>(t.dpair_a32)[k] = make_float4((float)r0, (float)r1, (float)r2, (float)p0);
    const_cast<float2*>(t.dpair_b32)[k] = make_float2((float)p1, (float)p2);
  }
  for (int64_t k = t0; k < t.ne - 1; k += stride) {
    const double* e = emb_c + 4 * k;
    const_cast<double4*>(t.emb_val)[k] = make_double4(e[0], e[1], e[2], e[3]);
  }
  for (int64_t k = t0; k < SW_WORDS; k += stride) s.status[k] = 0;
  for (int64_t k = t0; k < 3; k += stride) s.rflag[k] = 0;
  for (int64_t k = t0; k < ncells; k += stride) {
    s.bin_cnt[k] = 0;
    s.cell_stat[3 * k + 0] = s.cell_stat[3 * k + 1] = s.cell_stat[3 * k + 2] = 0;
  }
  for (int64_t k = t0; k < g.n; k += stride) {
    s.cnt[k] = 0;
    s.frc[k] = make_double4(0.0, 0.0, 0.0, 0.0);
  }
}

bool valid_device_spline(const md_spline* s) {
  return s && s->coef && s->n_knots >= 3 && s->n_knots <= MD_STATIC_MAX_KNOTS &&
         std::isfinite(s->x0) && std::isfinite(s->inv_dx) && s->inv_dx > 0.0;
}

}  // namespace

extern "C" md_status md_forces_static(const md_params* p, int64_t n_atoms, const double* box,
                                      const md_spline* phi, const md_spline* rho,
                                      const md_spline* emb, const double* x, double* f,
                                      double* rho_out, double* fp_out, void* stream) {
  // host-side checks first: nothing touches the device before they pass
  md_status s = check_params(p);
  if (s != MD_OK) return s;
  if (p->list_mode != MD_LIST_FULL || p->n_types > 1 || p->nbr_capacity > 128 ||
      p->cell_capacity > 64 || !x || !box)
    return MD_E_ARG;
  if (n_atoms < 1 || n_atoms > MD_STATIC_MAX_ATOMS) return MD_E_ARG;
  if (!valid_device_spline(phi) || !valid_device_spline(rho) || !valid_device_spline(emb))
    return MD_E_TABLE;
  if (phi->n_knots != rho->n_knots || phi->inv_dx != rho->inv_dx || phi->x0 != 0.0 ||
      rho->x0 != 0.0)
    return MD_E_TABLE;
  if ((double)(rho->n_knots - 1) / rho->inv_dx < p->r_cut * (1.0 - 1e-12)) return MD_E_TABLE;
  std::vector<RepHost> reps;
  if ((s = gather_reps(p, 1, &n_atoms, box, &reps)) != MD_OK) return s;
  const LayoutSizes ls = layout(p, 1, reps);
  if (ls.cells > MD_STATIC_MAX_CELLS) return MD_E_ARG;
  if (carve(nullptr, p, 1, ls, rho->n_knots, emb->n_knots, nullptr) > kScratchBytes)
    return MD_E_ARG;

  StaticDevice dev;
  if ((s = static_device(&dev)) != MD_OK) return s;
  Buffers b;
  carve(dev.ptr, p, 1, ls, rho->n_knots, emb->n_knots, &b);

  RepDev rd;
  memset(&rd, 0, sizeof(rd));
  for (int k = 0; k < 3; ++k) {
    rd.box[k] = reps[0].box[k];
    rd.nc[k] = reps[0].nc[k];
    rd.inv_cell[k] = (double)reps[0].nc[k] / reps[0].box[k];
  }
  rd.n_atoms = (int32_t)n_atoms;
  rd.ncell = rd.nc[0] * rd.nc[1] * rd.nc[2];
  rd.open = reps[0].open;
  set_quanta(rd);
  rd.ntiles = (int32_t)((n_atoms + 63) / 64);

  Geometry g{};
  g.reps = b.reps;
  g.atiles = b.atiles;
  g.ctiles = b.ctiles;
  g.n = ls.n;
  g.n_atiles = (int32_t)ls.atile_blocks;
  g.n_ctiles = (int32_t)ls.ctile_blocks;
  g.n_rep = 1;
  g.nbr_cap = p->nbr_capacity;
  g.cell_cap = p->cell_capacity;
  g.rc2 = p->r_cut * p->r_cut;
  g.rl2 = (p->r_cut + p->skin) * (p->r_cut + p->skin);
  g.lim2 = 0.25 * p->skin * p->skin;
  g.dt = p->dt;
  g.acc = p->ftm2v / p->mass;
  for (int q = 0; q < kMaxTypes; ++q) g.acc_t[q] = g.acc;
  g.rc2f = (float)g.rc2;

  Tables t{};
  t.rho_val = b.rho_val;
  t.phi_val = b.phi_val;
  t.dpair3 = b.dpair3;
  t.emb_val = b.emb_val;
  t.rho_val32 = b.rho_val32;
  t.dpair_a32 = b.dpair_a32;
  t.dpair_b32 = b.dpair_b32;
  t.r_inv_dx = rho->inv_dx;
  t.r_inv_dx32 = (float)rho->inv_dx;
  t.e_x0 = emb->x0;
  t.e_inv_dx = emb->inv_dx;
  t.nr = rho->n_knots;
  t.ne = emb->n_knots;
  if (force_lds_bytes(t, p->precision) > (size_t)dev.lds_max ||
      density_lds_bytes(t, p->precision) > (size_t)dev.lds_max)
    return MD_E_TABLE;

  State st{};
  st.pos = b.pos0;
  st.pos_alt = b.pos1;
  st.vel = b.vel;
  st.xref = b.xref;
  st.rec = b.rec0;
  st.rec_alt = b.rec1;
  st.sort_rec = b.sort_rec;
  st.snap_rec = b.snap_rec;
  st.frc = b.frc;
  st.rho = b.rho;
  st.epair = b.epair;
  st.id = b.id;
  st.cell_of = b.cell_of;
  st.nbr = b.nbr;
  st.cnt = b.cnt;
  st.bin_cnt = b.bin_cnt;
  st.bin_idx = b.bin_idx;
  st.cell_start = b.cell_start;
  st.cell_stat = b.cell_stat;
  st.status = b.status;
  st.rflag = b.rflag;
  st.sort_pos = b.sort_pos;
  st.sort_vel = b.sort_vel;
  st.sort_id = b.sort_id;
  st.partial = b.partial;

  Launch L{};
  L.stream = reinterpret_cast<hipStream_t>(stream);
  L.atile_blocks = (int32_t)ls.atile_blocks;
  L.ctile_blocks = (int32_t)ls.ctile_blocks;
  L.persist_blocks = dev.persist_blocks;
  const int lpa = p->lanes_per_atom ? p->lanes_per_atom : auto_lpa(ls.n);

  // the kernels' dynamic LDS limits follow this call's table sizes
  hipError_t e = allow_pair_lds(t, p->precision);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipFuncSetAttribute");
  const int64_t setup_items = std::max<int64_t>({ls.n, ls.cells, (int64_t)ls.atile_blocks,
                                                 (int64_t)ls.ctile_blocks, (int64_t)t.nr,
                                                 (int64_t)t.ne, (int64_t)SW_WORDS});
  hipLaunchKernelGGL(k_static_setup, dim3((unsigned)std::min<int64_t>((setup_items + 255) / 256, 1024)),
                     dim3(256), 0, L.stream, rd, g, st, t, phi->coef, rho->coef, emb->coef,
                     (int64_t)ls.cells);
  e = hipGetLastError();
  // the sequence of md_set_state, md_build_neighbors and md_compute_forces
  if (e == hipSuccess) e = launch_import(L, g, st, x, nullptr);
  if (e == hipSuccess) e = launch_sort(L, g, st, ls.cells);
  if (e == hipSuccess) e = launch_zero_bins(L, st, ls.cells);
  if (e == hipSuccess) e = launch_bin(L, g, st, nullptr, nullptr);
  if (e == hipSuccess) e = launch_build(L, g, st, nullptr, nullptr);
  if (e == hipSuccess) e = launch_zero_bins(L, st, ls.cells);
  if (e == hipSuccess)
    e = launch_density(L, g, st, t, p->precision, lpa, st.pos, nullptr, nullptr, nullptr,
                       ls.cells, true);
  if (e == hipSuccess) e = launch_force_only(L, g, st, t, p->precision, lpa, st.pos);
  if (e == hipSuccess) e = launch_export(L, g, st, nullptr, nullptr, f, rho_out, fp_out, 0.0);
  if (e != hipSuccess) return hip_fail(nullptr, e, "md_forces_static launch");
  int32_t bits = 0;
  e = hipMemcpyAsync(&bits, st.status + SW_BITS, sizeof(int32_t), hipMemcpyDeviceToHost, L.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L.stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "md_forces_static status");
  return status_code(bits);
}
