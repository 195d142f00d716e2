/*
 * eam_oracle.c -- plain, slow, FP64 CPU oracle of the EAM timestep loop.
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
 * benchmark's CPU-baseline leg are its only users.  It shares no code, header
 * or table generator with the GPU library, and the library never calls it.
 *
 * What it computes (paper: "Breaking the Molecular Dynamics Timescale Barrier
 * Using a Wafer-Scale System", arXiv 2405.07898):
 *   - electron density rho_i = sum_j rho(r_ij)                Sec. II-A, Eq. (density)
 *   - potential U = 1/2 sum_{i!=j} phi(r_ij) + sum_i F(rho_i)  Sec. II-A, Eq. (potential)
 *   - pairs beyond the cutoff contribute nothing; squared distances are
 *     compared against the squared cutoff                        Sec. II-A; Sec. III-C
 *   - force -dU/dx_i = sum_j [(F'_i + F'_j) rho'(r) + phi'(r)] (x_j - x_i)/r
 *                                                              Sec. II-A, Eq. (EAMforce)
 *   - time integration, second order and symplectic            Sec. II-A, Eq. (leapfrog),
 *     written in its velocity-Verlet form (same positions, velocities on
 *     whole steps)
 *   - spline segment arithmetic x = alpha*s, k = int(x), t = x - k
 *                                                              Table "flopmodel", segment row
 *   - several atom types: rho_{t_j}, F_{t_i}, phi_{t_i t_j}   Sec. II-A, after Eq. (potential)
 * Readings where the paper is silent: self term excluded from rho_i; strict
 * "<" for both cutoffs; natural-cubic per-segment tables; wrap-then-minimum-
 * image periodic boxes; cells of edge >= r_cut + skin with index
 * min(int(x * n/L), n-1); Verlet list rebuilt when any atom has moved more
 * than skin/2 since the last build.
 *
 * Layout: positions, velocities and forces are AoS [n][3] float64 in original
 * atom order.  Neighbour lists are row-major nbr[i*cap + k] of original ids.
 * All per-atom sums run sequentially in list order, so results are bitwise
 * independent of the OpenMP thread count.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int32_t n_knots;
  int32_t reserved;
  double x0;
  double inv_dx;
  const double *coef; /* [(n_knots-1)][4]: c0..c3 in t */
} or_spline;

typedef struct {
  double box[3];
  double mass;  /* amu */
  double dt;    /* fs */
  double r_cut; /* A */
  double skin;  /* A */
  double ftm2v; /* (eV/A)/amu -> A/fs^2 */
  int32_t cap;  /* neighbour-list capacity per atom */
  int32_t reserved;
} or_md_params;

typedef struct {
  int64_t steps;
  int64_t rebuilds;
  int64_t list_entries; /* sum of list lengths at the last build */
  int32_t max_count;
  int32_t flags; /* bit0: rho beyond the F table */
} or_md_stats;

enum { OR_OK = 0, OR_E_BOX = -2, OR_E_OVERFLOW = -4, OR_E_NONFINITE = -6, OR_E_LOST = -9 };

/* ------------------------------------------------------------------ threads */

void or_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int32_t or_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ splines */

/* Segment of a per-segment cubic table: x = alpha (s - x0), k = int(x) clamped
 * to [0, n-2], t = x - k.  Past the last knot (t > 1 on the last segment) the
 * function continues as the straight line tangent at that knot: value
 * f(1) + f_t(1) (t - 1), slope f_t(1), curvature 0.  (Reading: the paper does
 * not say what a table does outside its range; the last cubic itself, taken
 * far outside its interval, grows like t^3, and for F it turns a dense
 * cluster at rho > rho_max into a runaway.) */
static void seg_of(const or_spline *sp, double s, int *k, double *t) {
  double x = (s - sp->x0) * sp->inv_dx;
  int last = sp->n_knots - 2;
  int kk;
  if (x >= (double)last) kk = last;
  else if (x > 0.0) kk = (int)x;
  else kk = 0;
  *k = kk;
  *t = x - (double)kk;
}

static double spl_f(const or_spline *sp, double s) {
  int k;
  double t;
  seg_of(sp, s, &k, &t);
  const double *c = sp->coef + 4 * (size_t)k;
  if (t > 1.0) return (c[0] + c[1] + c[2] + c[3]) + (c[1] + 2.0 * c[2] + 3.0 * c[3]) * (t - 1.0);
  return c[0] + t * (c[1] + t * (c[2] + t * c[3]));
}

static double spl_df(const or_spline *sp, double s) {
  int k;
  double t;
  seg_of(sp, s, &k, &t);
  if (t > 1.0) t = 1.0;
  const double *c = sp->coef + 4 * (size_t)k;
  return (c[1] + t * (2.0 * c[2] + t * (3.0 * c[3]))) * sp->inv_dx;
}

static double spl_ddf(const or_spline *sp, double s) {
  int k;
  double t;
  seg_of(sp, s, &k, &t);
  if (t > 1.0) return 0.0;
  const double *c = sp->coef + 4 * (size_t)k;
  return (2.0 * c[2] + 6.0 * c[3] * t) * sp->inv_dx * sp->inv_dx;
}

static double spl_end(const or_spline *sp) {
  return sp->x0 + (double)(sp->n_knots - 1) / sp->inv_dx;
}

void or_spline_eval(const or_spline *sp, int64_t n, const double *s, double *f, double *df,
                    double *ddf) {
  for (int64_t i = 0; i < n; ++i) {
    if (f) f[i] = spl_f(sp, s[i]);
    if (df) df[i] = spl_df(sp, s[i]);
    if (ddf) ddf[i] = spl_ddf(sp, s[i]);
  }
}

/* ------------------------------------------------------- periodic geometry */

/* Boundaries.  A box length L > 0 is a periodic dimension of period L.  A
 * negative box length marks an open (non-periodic) dimension: no wrap, no
 * minimum image; cells cover [0, |L|) and atoms outside it belong to the edge
 * cells. */

/* One shift into [0, L); a value that lands on L (tiny negative x) becomes 0.
 * Open dimensions are left as they are. */
static double wrap1(double x, double L) {
  if (L < 0.0) return x;
  if (x >= L) x -= L;
  else if (x < 0.0) {
    x += L;
    if (x >= L) x = 0.0;
  }
  return x;
}

/* Minimum image of a separation, valid for |d| < 1.5 L (open: unchanged). */
static double min_image(double d, double L, double half) {
  if (L < 0.0) return d;
  if (d > half) d -= L;
  else if (d < -half) d += L;
  return d;
}

/* Wrap every coordinate; returns the number of coordinates non-finite or, in
 * a periodic dimension, still outside [0, L) afterwards (moved more than one
 * box length in one step). */
int64_t or_wrap(int64_t n, double *x, const double box[3]) {
  int64_t bad = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int d = 0; d < 3; ++d) {
      double w = wrap1(x[3 * i + d], box[d]);
      x[3 * i + d] = w;
      if (!isfinite(w) || (box[d] > 0.0 && !(w >= 0.0 && w < box[d]))) ++bad;
    }
  }
  return bad;
}

/* Squared minimum-image distance from i to j, (dx dx + dy dy) + dz dz, no FMA. */
static double dist2(const double *xi, const double *xj, const double box[3], const double half[3],
                    double d[3]) {
  for (int a = 0; a < 3; ++a) d[a] = min_image(xj[a] - xi[a], box[a], half[a]);
  return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

/* Cell grid: n_d = floor(|L_d| / r_list) cells per dimension (at least 3 when
 * periodic, at least 1 when open), inv_cell_d = n_d / |L_d|. */
int32_t or_cell_grid(const double box[3], double rlist, int32_t ncell[3], double inv_cell[3]) {
  for (int d = 0; d < 3; ++d) {
    const double ext = fabs(box[d]);
    double q = floor(ext / rlist);
    if (box[d] < 0.0 && q < 1.0) q = 1.0;
    if (!(q >= (box[d] < 0.0 ? 1.0 : 3.0)) || q > 1.0e6) return OR_E_BOX;
    ncell[d] = (int32_t)q;
    inv_cell[d] = (double)ncell[d] / ext;
  }
  return OR_OK;
}

static int32_t cell_index(const double *xi, const int32_t nc[3], const double ic[3]) {
  int32_t c[3];
  for (int d = 0; d < 3; ++d) {
    double s = xi[d] * ic[d];
    int32_t k = (s > 0.0) ? (int32_t)s : 0;
    if (k > nc[d] - 1) k = nc[d] - 1;
    c[d] = k;
  }
  return (c[2] * nc[1] + c[1]) * nc[0] + c[0];
}

void or_cell_ids(int64_t n, const double *x, const int32_t ncell[3], const double inv_cell[3],
                 int32_t *cell) {
  for (int64_t i = 0; i < n; ++i) cell[i] = cell_index(x + 3 * i, ncell, inv_cell);
}

/* Stable counting sort by cell id: order[] lists atoms cell by cell, each cell
 * in increasing atom id; cell_start has ncells + 1 entries. */
void or_cell_sort(int64_t n, const int32_t *cell, int32_t ncells, int32_t *cell_start,
                  int32_t *order) {
  int32_t *fill = (int32_t *)calloc((size_t)ncells + 1, sizeof(int32_t));
  for (int64_t i = 0; i < n; ++i) fill[cell[i] + 1]++;
  for (int32_t c = 0; c < ncells; ++c) fill[c + 1] += fill[c];
  memcpy(cell_start, fill, ((size_t)ncells + 1) * sizeof(int32_t));
  for (int64_t i = 0; i < n; ++i) order[fill[cell[i]]++] = (int32_t)i;
  free(fill);
}

/* ------------------------------------------------------- neighbour lists */

/* O(N^2) list: j in N(i) iff j != i and r_ij^2 < rlist^2.  Stores at most cap
 * ids per row; cnt[i] holds the true count.  Returns max_i cnt[i]. */
int32_t or_list_brute(int64_t n, const double *x, const double box[3], double rlist, int32_t cap,
                      int32_t *cnt, int32_t *nbr) {
  const double half[3] = {0.5 * box[0], 0.5 * box[1], 0.5 * box[2]};
  const double rl2 = rlist * rlist;
  int32_t mx = 0;
#pragma omp parallel for schedule(static) reduction(max : mx)
  for (int64_t i = 0; i < n; ++i) {
    int32_t c = 0;
    double d[3];
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      if (dist2(x + 3 * i, x + 3 * j, box, half, d) < rl2) {
        if (c < cap) nbr[i * cap + c] = (int32_t)j;
        ++c;
      }
    }
    cnt[i] = c;
    if (c > mx) mx = c;
  }
  return mx;
}

/* Same list through a cell grid: candidates are the atoms of the 27 cells
 * around the atom's own cell (wrapped in periodic dimensions, cut off at the
 * grid edge in open ones), each cell in increasing id.  Falls back to brute
 * force when a periodic dimension has fewer than three cells. */
int32_t or_list_cells(int64_t n, const double *x, const double box[3], double rlist, int32_t cap,
                      int32_t *cnt, int32_t *nbr) {
  int32_t nc[3];
  double ic[3];
  if (or_cell_grid(box, rlist, nc, ic) != OR_OK)
    return or_list_brute(n, x, box, rlist, cap, cnt, nbr);
  const int32_t ncells = nc[0] * nc[1] * nc[2];
  int32_t *cell = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int32_t *start = (int32_t *)malloc(((size_t)ncells + 1) * sizeof(int32_t));
  int32_t *order = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  or_cell_ids(n, x, nc, ic, cell);
  or_cell_sort(n, cell, ncells, start, order);
  const double half[3] = {0.5 * box[0], 0.5 * box[1], 0.5 * box[2]};
  const double rl2 = rlist * rlist;
  int32_t mx = 0;
#pragma omp parallel for schedule(static) reduction(max : mx)
  for (int64_t i = 0; i < n; ++i) {
    int32_t ci = cell[i];
    int32_t cx = ci % nc[0], cy = (ci / nc[0]) % nc[1], cz = ci / (nc[0] * nc[1]);
    int32_t c = 0;
    double d[3];
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if ((box[0] < 0.0 && (cx + dx < 0 || cx + dx >= nc[0])) ||
              (box[1] < 0.0 && (cy + dy < 0 || cy + dy >= nc[1])) ||
              (box[2] < 0.0 && (cz + dz < 0 || cz + dz >= nc[2])))
            continue;
          int32_t qx = (cx + dx + nc[0]) % nc[0];
          int32_t qy = (cy + dy + nc[1]) % nc[1];
          int32_t qz = (cz + dz + nc[2]) % nc[2];
          int32_t q = (qz * nc[1] + qy) * nc[0] + qx;
          for (int32_t s = start[q]; s < start[q + 1]; ++s) {
            int32_t j = order[s];
            if (j == i) continue;
            if (dist2(x + 3 * i, x + 3 * j, box, half, d) < rl2) {
              if (c < cap) nbr[i * cap + c] = j;
              ++c;
            }
          }
        }
    cnt[i] = c;
    if (c > mx) mx = c;
  }
  free(cell);
  free(start);
  free(order);
  return mx;
}

/* ------------------------------------------------------- EAM passes */

/* rho_i = sum over listed j with r^2 < rc^2 of rho(r); F'(rho_i) and F''(rho_i).
 * Returns 1 if some rho_i lies beyond the F table (extrapolated), else 0. */
int32_t or_density(int64_t n, const double *x, const double box[3], const int32_t *cnt,
                   const int32_t *nbr, int32_t cap, double rc, const or_spline *rho,
                   const or_spline *emb, double *rho_out, double *fp_out, double *fpp_out) {
  const double half[3] = {0.5 * box[0], 0.5 * box[1], 0.5 * box[2]};
  const double rc2 = rc * rc;
  const double rmax = spl_end(emb);
  int32_t flag = 0;
#pragma omp parallel for schedule(static) reduction(| : flag)
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0, d[3];
    int32_t m = cnt[i] < cap ? cnt[i] : cap;
    for (int32_t k = 0; k < m; ++k) {
      int32_t j = nbr[i * cap + k];
      double r2 = dist2(x + 3 * i, x + 3 * j, box, half, d);
      if (r2 < rc2) acc += spl_f(rho, sqrt(r2));
    }
    rho_out[i] = acc;
    if (fp_out) fp_out[i] = spl_df(emb, acc);
    if (fpp_out) fpp_out[i] = spl_ddf(emb, acc);
    if (acc > rmax) flag |= 1;
  }
  return flag;
}

/* F_i = sum_j [(F'_i + F'_j) rho'(r) + phi'(r)] (x_j - x_i) / r. */
void or_forces(int64_t n, const double *x, const double box[3], const int32_t *cnt,
               const int32_t *nbr, int32_t cap, double rc, const or_spline *phi,
               const or_spline *rho, const double *fp, double *f) {
  const double half[3] = {0.5 * box[0], 0.5 * box[1], 0.5 * box[2]};
  const double rc2 = rc * rc;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double fx = 0.0, fy = 0.0, fz = 0.0, d[3];
    int32_t m = cnt[i] < cap ? cnt[i] : cap;
    for (int32_t k = 0; k < m; ++k) {
      int32_t j = nbr[i * cap + k];
      double r2 = dist2(x + 3 * i, x + 3 * j, box, half, d);
      if (r2 < rc2) {
        double r = sqrt(r2);
        double s = (fp[i] + fp[j]) * spl_df(rho, r) + spl_df(phi, r);
        fx += s * d[0] / r;
        fy += s * d[1] / r;
        fz += s * d[2] / r;
      }
    }
    f[3 * i + 0] = fx;
    f[3 * i + 1] = fy;
    f[3 * i + 2] = fz;
  }
}

/* Per-atom potential energy e_i = 1/2 sum_j phi(r_ij) + F(rho_i) (sums to U of
 * Eq. (potential)) and kinetic energy k_i = 1/2 m |v_i|^2 / ftm2v. */
void or_energy_atoms(int64_t n, const double *x, const double *v, const double box[3],
                     const int32_t *cnt, const int32_t *nbr, int32_t cap, double rc,
                     const or_spline *phi, const or_spline *emb, const double *rho_i, double mass,
                     double ftm2v, double *e_pot, double *e_kin) {
  const double half[3] = {0.5 * box[0], 0.5 * box[1], 0.5 * box[2]};
  const double rc2 = rc * rc;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double pair = 0.0, d[3];
    int32_t m = cnt[i] < cap ? cnt[i] : cap;
    for (int32_t k = 0; k < m; ++k) {
      int32_t j = nbr[i * cap + k];
      double r2 = dist2(x + 3 * i, x + 3 * j, box, half, d);
      if (r2 < rc2) pair += spl_f(phi, sqrt(r2));
    }
    e_pot[i] = 0.5 * pair + spl_f(emb, rho_i[i]);
    if (e_kin) {
      const double *vi = v + 3 * i;
      e_kin[i] = 0.5 * mass * ((vi[0] * vi[0] + vi[1] * vi[1]) + vi[2] * vi[2]) / ftm2v;
    }
  }
}

/* Totals in atom order (sequential). */
void or_energy(int64_t n, const double *x, const double *v, const double box[3],
               const int32_t *cnt, const int32_t *nbr, int32_t cap, double rc,
               const or_spline *phi, const or_spline *rho, const or_spline *emb, double mass,
               double ftm2v, double *pe, double *ke) {
  double *rho_i = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double *ep = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double *ek = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  or_density(n, x, box, cnt, nbr, cap, rc, rho, emb, rho_i, NULL, NULL);
  or_energy_atoms(n, x, v, box, cnt, nbr, cap, rc, phi, emb, rho_i, mass, ftm2v, ep,
                  v ? ek : NULL);
  double sp = 0.0, sk = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    sp += ep[i];
    if (v) sk += ek[i];
  }
  *pe = sp;
  if (ke) *ke = sk;
  free(rho_i);
  free(ep);
  free(ek);
}

/* ------------------------------------------------------- MD loop */

typedef struct {
  int32_t *cnt, *nbr;
  double *xref, *rho, *fp;
} md_scratch;

static int build_list(int64_t n, const double *x, const or_md_params *p, md_scratch *w,
                      or_md_stats *st) {
  int32_t mx = or_list_cells(n, x, p->box, p->r_cut + p->skin, p->cap, w->cnt, w->nbr);
  memcpy(w->xref, x, (size_t)n * 3 * sizeof(double));
  int64_t tot = 0;
  for (int64_t i = 0; i < n; ++i) tot += w->cnt[i];
  st->list_entries = tot;
  if (mx > st->max_count) st->max_count = mx;
  return mx > p->cap ? OR_E_OVERFLOW : OR_OK;
}

static int forces_now(int64_t n, const double *x, const or_md_params *p, const or_spline *phi,
                      const or_spline *rho, const or_spline *emb, md_scratch *w, double *f,
                      or_md_stats *st) {
  st->flags |= or_density(n, x, p->box, w->cnt, w->nbr, p->cap, p->r_cut, rho, emb, w->rho, w->fp,
                          NULL);
  or_forces(n, x, p->box, w->cnt, w->nbr, p->cap, p->r_cut, phi, rho, w->fp, f);
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!isfinite(f[i])) return OR_E_NONFINITE;
  return OR_OK;
}

/* Velocity-Verlet: v += dt/2 a; x += dt v; wrap; rebuild if any atom moved
 * more than skin/2 since the last build; forces; v += dt/2 a.
 * x, v are updated in place; f receives the forces at the final positions.
 * energy (optional) receives (pe, ke) at steps 0..nsteps. */
int32_t or_md_run(int64_t n, double *x, double *v, double *f, const or_md_params *p,
                  const or_spline *phi, const or_spline *rho, const or_spline *emb, int64_t nsteps,
                  double *energy, or_md_stats *st) {
  memset(st, 0, sizeof(*st));
  int32_t nc[3];
  double ic[3];
  const double rl = p->r_cut + p->skin;
  if (or_cell_grid(p->box, rl, nc, ic) != OR_OK &&
      ((p->box[0] > 0.0 && p->box[0] < 2.0 * rl) || (p->box[1] > 0.0 && p->box[1] < 2.0 * rl) ||
       (p->box[2] > 0.0 && p->box[2] < 2.0 * rl)))
    return OR_E_BOX;
  size_t nn = (size_t)(n > 0 ? n : 1);
  md_scratch w;
  w.cnt = (int32_t *)malloc(nn * sizeof(int32_t));
  w.nbr = (int32_t *)malloc(nn * (size_t)p->cap * sizeof(int32_t));
  w.xref = (double *)malloc(nn * 3 * sizeof(double));
  w.rho = (double *)malloc(nn * sizeof(double));
  w.fp = (double *)malloc(nn * sizeof(double));
  const double half[3] = {0.5 * p->box[0], 0.5 * p->box[1], 0.5 * p->box[2]};
  const double lim2 = 0.25 * p->skin * p->skin;
  const double hdt = 0.5 * p->dt;
  const double acc = p->ftm2v / p->mass;
  int rc = OR_OK;

  if (or_wrap(n, x, p->box)) rc = OR_E_LOST;
  if (rc == OR_OK) rc = build_list(n, x, p, &w, st);
  if (rc == OR_OK) rc = forces_now(n, x, p, phi, rho, emb, &w, f, st);
  if (rc == OR_OK && energy)
    or_energy(n, x, v, p->box, w.cnt, w.nbr, p->cap, p->r_cut, phi, rho, emb, p->mass, p->ftm2v,
              &energy[0], &energy[1]);
  for (int64_t s = 0; s < nsteps && rc == OR_OK; ++s) {
    for (int64_t i = 0; i < 3 * n; ++i) {
      v[i] += hdt * (f[i] * acc);
      x[i] += p->dt * v[i];
    }
    if (or_wrap(n, x, p->box)) {
      rc = OR_E_LOST;
      break;
    }
    double mx2 = 0.0, d[3];
    for (int64_t i = 0; i < n; ++i) {
      double r2 = dist2(w.xref + 3 * i, x + 3 * i, p->box, half, d);
      if (r2 > mx2) mx2 = r2;
    }
    if (mx2 > lim2) {
      rc = build_list(n, x, p, &w, st);
      st->rebuilds++;
      if (rc != OR_OK) break;
    }
    rc = forces_now(n, x, p, phi, rho, emb, &w, f, st);
    if (rc != OR_OK) break;
    for (int64_t i = 0; i < 3 * n; ++i) v[i] += hdt * (f[i] * acc);
    st->steps++;
    if (energy)
      or_energy(n, x, v, p->box, w.cnt, w.nbr, p->cap, p->r_cut, phi, rho, emb, p->mass, p->ftm2v,
                &energy[2 * (s + 1)], &energy[2 * (s + 1) + 1]);
  }
  free(w.cnt);
  free(w.nbr);
  free(w.xref);
  free(w.rho);
  free(w.fp);
  return rc;
}

/* Forces (and rho) of a configuration from scratch: list at r_cut + skin, then
 * density and force passes.  Convenience for parity checks. */
int32_t or_forces_at(int64_t n, const double *x_in, const double box[3], double rc, double skin,
                     int32_t cap, const or_spline *phi, const or_spline *rho,
                     const or_spline *emb, double *f, double *rho_out, double *fp_out,
                     double *pe) {
  size_t nn = (size_t)(n > 0 ? n : 1);
  double *x = (double *)malloc(nn * 3 * sizeof(double));
  memcpy(x, x_in, (size_t)n * 3 * sizeof(double));
  int32_t rcode = OR_OK;
  if (or_wrap(n, x, box)) rcode = OR_E_LOST;
  int32_t *cnt = (int32_t *)malloc(nn * sizeof(int32_t));
  int32_t *nbr = (int32_t *)malloc(nn * (size_t)cap * sizeof(int32_t));
  double *fp = (double *)malloc(nn * sizeof(double));
  double *rh = (double *)malloc(nn * sizeof(double));
  if (rcode == OR_OK) {
    int32_t mx = or_list_cells(n, x, box, rc + skin, cap, cnt, nbr);
    if (mx > cap) rcode = OR_E_OVERFLOW;
  }
  if (rcode == OR_OK) {
    int32_t fl = or_density(n, x, box, cnt, nbr, cap, rc, rho, emb, rh, fp, NULL);
    or_forces(n, x, box, cnt, nbr, cap, rc, phi, rho, fp, f);
    if (pe) or_energy(n, x, NULL, box, cnt, nbr, cap, rc, phi, rho, emb, 1.0, 1.0, pe, NULL);
    if (rho_out) memcpy(rho_out, rh, (size_t)n * sizeof(double));
    if (fp_out) memcpy(fp_out, fp, (size_t)n * sizeof(double));
    rcode = fl;
  }
  free(x);
  free(cnt);
  free(nbr);
  free(fp);
  free(rh);
  return rcode;
}

/* ------------------------------------------------------- analytic potential */

/* Closed-form synthetic potential: fc = (1-(r/rc)^2)^3,
 * phi = A e^{-B(r/r0-1)} fc, rho = e^{-C(r/r0-1)} fc, F = -E sqrt(rho).
 * Used for force-matching reference forces and to pin the tabulated path. */
typedef struct {
  double rc, r0, phi_a, phi_b, rho_b, emb_a;
} or_analytic;

static void an_pair(const or_analytic *a, double r, double *ph, double *dph, double *rh,
                    double *drh) {
  double u = 1.0 - (r / a->rc) * (r / a->rc);
  double f = u * u * u;
  double df = 3.0 * u * u * (-2.0 * r / (a->rc * a->rc));
  double ep = a->phi_a * exp(-a->phi_b * (r / a->r0 - 1.0));
  double er = exp(-a->rho_b * (r / a->r0 - 1.0));
  *ph = ep * f;
  *dph = ep * (-a->phi_b / a->r0) * f + ep * df;
  *rh = er * f;
  *drh = er * (-a->rho_b / a->r0) * f + er * df;
}

/* Forces and energy with the closed forms over a brute-force-free cell list. */
int32_t or_forces_analytic(int64_t n, const double *x_in, const double box[3],
                           const or_analytic *a, double *f, double *pe) {
  size_t nn = (size_t)(n > 0 ? n : 1);
  int32_t cap = 512;
  double *x = (double *)malloc(nn * 3 * sizeof(double));
  memcpy(x, x_in, (size_t)n * 3 * sizeof(double));
  or_wrap(n, x, box);
  int32_t *cnt = (int32_t *)malloc(nn * sizeof(int32_t));
  int32_t *nbr = (int32_t *)malloc(nn * (size_t)cap * sizeof(int32_t));
  double *rh = (double *)malloc(nn * sizeof(double));
  double *fp = (double *)malloc(nn * sizeof(double));
  int32_t mx = or_list_cells(n, x, box, a->rc, cap, cnt, nbr);
  if (mx > cap) {
    free(x); free(cnt); free(nbr); free(rh); free(fp);
    return OR_E_OVERFLOW;
  }
  const double half[3] = {0.5 * box[0], 0.5 * box[1], 0.5 * box[2]};
  const double rc2 = a->rc * a->rc;
  double epair = 0.0, eemb = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0, d[3], ph, dph, r1, dr1;
    for (int32_t k = 0; k < cnt[i]; ++k) {
      int32_t j = nbr[i * cap + k];
      double r2 = dist2(x + 3 * i, x + 3 * j, box, half, d);
      if (r2 < rc2) {
        an_pair(a, sqrt(r2), &ph, &dph, &r1, &dr1);
        acc += r1;
        epair += 0.5 * ph;
      }
    }
    rh[i] = acc;
    fp[i] = -0.5 * a->emb_a / sqrt(acc);
    eemb += -a->emb_a * sqrt(acc);
  }
  for (int64_t i = 0; i < n; ++i) {
    double fx = 0.0, fy = 0.0, fz = 0.0, d[3], ph, dph, r1, dr1;
    for (int32_t k = 0; k < cnt[i]; ++k) {
      int32_t j = nbr[i * cap + k];
      double r2 = dist2(x + 3 * i, x + 3 * j, box, half, d);
      if (r2 < rc2) {
        double r = sqrt(r2);
        an_pair(a, r, &ph, &dph, &r1, &dr1);
        double s = (fp[i] + fp[j]) * dr1 + dph;
        fx += s * d[0] / r;
        fy += s * d[1] / r;
        fz += s * d[2] / r;
      }
    }
    f[3 * i + 0] = fx;
    f[3 * i + 1] = fy;
    f[3 * i + 2] = fz;
  }
  if (pe) *pe = epair + eemb;
  free(x); free(cnt); free(nbr); free(rh); free(fp);
  return OR_OK;
}

/* ------------------------------------------------------- force matching */

/* Loss L = sum_c sum_i |F_i - Fref_i|^2 over n_cfg static configurations
 * (atoms of config c are [off[c], off[c+1]) in x, box c at box[3c]).
 * With grad_* non-NULL also returns dL/dcoef for the three tables (each
 * (n_knots-1)*4 doubles, same layout as coef), by reverse-mode differentiation
 * of the density and force passes:
 *   g_i = 2 (F_i - Fref_i),  u_ij = (x_j - x_i)/r,  w_ij = g_i . u_ij
 *   lambda_i = sum_j (w_ij + w_ji) rho'(r_ij),  mu_i = lambda_i F''(rho_i)
 *   dL/dphi  = sum_(i,j) w_ij dphi'(r_ij)
 *   dL/drho  = sum_(i,j) [w_ij (F'_i + F'_j) drho'(r_ij)] + sum_i mu_i sum_j drho(r_ij)
 *   dL/dF    = sum_i lambda_i dF'(rho_i)
 * where d f(s)/d c_m = t^m and d f'(s)/d c_m = m t^(m-1) alpha.
 * Per-config sums are sequential; configs are added in order. */
double or_fm_loss_grad(int32_t n_cfg, const int64_t *off, const double *x, const double *box,
                       double rc, const or_spline *phi, const or_spline *rho,
                       const or_spline *emb, const double *fref, double *grad_phi,
                       double *grad_rho, double *grad_emb, double *f_out) {
  const int want = grad_phi && grad_rho && grad_emb;
  const size_t gp = 4 * (size_t)(phi->n_knots - 1), gr = 4 * (size_t)(rho->n_knots - 1),
               ge = 4 * (size_t)(emb->n_knots - 1);
  double *loss_c = (double *)calloc((size_t)n_cfg, sizeof(double));
  double *g_all = want ? (double *)calloc((size_t)n_cfg * (gp + gr + ge), sizeof(double)) : NULL;
  const int32_t cap = 512;
  int32_t err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
  for (int32_t c = 0; c < n_cfg; ++c) {
    int64_t n = off[c + 1] - off[c];
    const double *bx = box + 3 * c;
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *xc = (double *)malloc(nn * 3 * sizeof(double));
    memcpy(xc, x + 3 * off[c], (size_t)n * 3 * sizeof(double));
    or_wrap(n, xc, bx);
    int32_t *cnt = (int32_t *)malloc(nn * sizeof(int32_t));
    int32_t *nbr = (int32_t *)malloc(nn * (size_t)cap * sizeof(int32_t));
    double *rh = (double *)malloc(nn * sizeof(double));
    double *fp = (double *)malloc(nn * sizeof(double));
    double *fpp = (double *)malloc(nn * sizeof(double));
    double *fc = (double *)malloc(nn * 3 * sizeof(double));
    double *g = (double *)malloc(nn * 3 * sizeof(double));
    double *lam = (double *)malloc(nn * sizeof(double));
    if (or_list_cells(n, xc, bx, rc, cap, cnt, nbr) > cap) err |= 1;
    else {
      const double half[3] = {0.5 * bx[0], 0.5 * bx[1], 0.5 * bx[2]};
      const double rc2 = rc * rc;
      or_density(n, xc, bx, cnt, nbr, cap, rc, rho, emb, rh, fp, fpp);
      or_forces(n, xc, bx, cnt, nbr, cap, rc, phi, rho, fp, fc);
      double l = 0.0;
      for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
          double e = fc[3 * i + a] - fref[3 * (off[c] + i) + a];
          l += e * e;
          g[3 * i + a] = 2.0 * e;
        }
      }
      loss_c[c] = l;
      if (f_out) memcpy(f_out + 3 * off[c], fc, (size_t)n * 3 * sizeof(double));
      if (want) {
        double *gph = g_all + (size_t)c * (gp + gr + ge), *grh = gph + gp, *gem = grh + gr;
        double d[3];
        /* lambda_i */
        for (int64_t i = 0; i < n; ++i) {
          double acc = 0.0;
          for (int32_t k = 0; k < cnt[i]; ++k) {
            int32_t j = nbr[i * cap + k];
            double r2 = dist2(xc + 3 * i, xc + 3 * j, bx, half, d);
            if (r2 < rc2) {
              double r = sqrt(r2);
              double wij = (g[3 * i] * d[0] + g[3 * i + 1] * d[1] + g[3 * i + 2] * d[2]) / r;
              double wji = -(g[3 * j] * d[0] + g[3 * j + 1] * d[1] + g[3 * j + 2] * d[2]) / r;
              acc += (wij + wji) * spl_df(rho, r);
            }
          }
          lam[i] = acc;
        }
        /* coefficient gradients */
        for (int64_t i = 0; i < n; ++i) {
          double mu = lam[i] * fpp[i];
          for (int32_t k = 0; k < cnt[i]; ++k) {
            int32_t j = nbr[i * cap + k];
            double r2 = dist2(xc + 3 * i, xc + 3 * j, bx, half, d);
            if (!(r2 < rc2)) continue;
            double r = sqrt(r2);
            double wij = (g[3 * i] * d[0] + g[3 * i + 1] * d[1] + g[3 * i + 2] * d[2]) / r;
            int kp;
            double tp;
            seg_of(phi, r, &kp, &tp);
            gph[4 * kp + 1] += wij * phi->inv_dx;
            gph[4 * kp + 2] += wij * 2.0 * tp * phi->inv_dx;
            gph[4 * kp + 3] += wij * 3.0 * tp * tp * phi->inv_dx;
            int kr;
            double tr;
            seg_of(rho, r, &kr, &tr);
            double wf = wij * (fp[i] + fp[j]);
            grh[4 * kr + 0] += mu;
            grh[4 * kr + 1] += wf * rho->inv_dx + mu * tr;
            grh[4 * kr + 2] += wf * 2.0 * tr * rho->inv_dx + mu * tr * tr;
            grh[4 * kr + 3] += wf * 3.0 * tr * tr * rho->inv_dx + mu * tr * tr * tr;
          }
          int ke;
          double te;
          seg_of(emb, rh[i], &ke, &te);
          if (te > 1.0) te = 1.0; /* tangent-line continuation past the last knot */
          gem[4 * ke + 1] += lam[i] * emb->inv_dx;
          gem[4 * ke + 2] += lam[i] * 2.0 * te * emb->inv_dx;
          gem[4 * ke + 3] += lam[i] * 3.0 * te * te * emb->inv_dx;
        }
      }
    }
    free(xc); free(cnt); free(nbr); free(rh); free(fp); free(fpp); free(fc); free(g); free(lam);
  }
  double loss = 0.0;
  for (int32_t c = 0; c < n_cfg; ++c) loss += loss_c[c];
  if (want) {
    memset(grad_phi, 0, gp * sizeof(double));
    memset(grad_rho, 0, gr * sizeof(double));
    memset(grad_emb, 0, ge * sizeof(double));
    for (int32_t c = 0; c < n_cfg; ++c) {
      const double *gph = g_all + (size_t)c * (gp + gr + ge), *grh = gph + gp, *gem = grh + gr;
      for (size_t q = 0; q < gp; ++q) grad_phi[q] += gph[q];
      for (size_t q = 0; q < gr; ++q) grad_rho[q] += grh[q];
      for (size_t q = 0; q < ge; ++q) grad_emb[q] += gem[q];
    }
    free(g_all);
  }
  free(loss_c);
  return err ? NAN : loss;
}

/* ------------------------------------------------------- several atom types */

/* Multi-species EAM.  Sec. II-A lets the density, embedding and pair
 * functions depend on the atoms' types (after Eq. potential):
 *   rho_i  = sum_j rho_{t_j}(r_ij)     (the density an atom of type t_j emits)
 *   U      = 1/2 sum_{i != j} phi_{t_i t_j}(r_ij) + sum_i F_{t_i}(rho_i)
 *   -dU/dx_i = sum_j [F'_i rho'_{t_j}(r) + F'_j rho'_{t_i}(r) + phi'_{t_i t_j}(r)]
 *              (x_j - x_i)/r                                  Eq. (EAMforce)
 * Tables: rho[t] and emb[t] for t < nt, phi[a*nt + b] (the caller passes the
 * same table for (a, b) and (b, a)); one mass per type.  With nt = 1 these
 * reduce to the single-species functions above. */

int32_t or_density_multi(int64_t n, const double *x, const double box[3], const int32_t *cnt,
                         const int32_t *nbr, int32_t cap, double rc, int32_t nt,
                         const int32_t *type, const or_spline *rho, const or_spline *emb,
                         double *rho_out, double *fp_out) {
  const double half[3] = {0.5 * box[0], 0.5 * box[1], 0.5 * box[2]};
  const double rc2 = rc * rc;
  int32_t flag = 0;
  (void)nt;
#pragma omp parallel for schedule(static) reduction(| : flag)
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0, d[3];
    int32_t m = cnt[i] < cap ? cnt[i] : cap;
    for (int32_t k = 0; k < m; ++k) {
      int32_t j = nbr[i * cap + k];
      double r2 = dist2(x + 3 * i, x + 3 * j, box, half, d);
      if (r2 < rc2) acc += spl_f(&rho[type[j]], sqrt(r2));
    }
    const or_spline *F = &emb[type[i]];
    rho_out[i] = acc;
    if (fp_out) fp_out[i] = spl_df(F, acc);
    if (acc > spl_end(F)) flag |= 1;
  }
  return flag;
}

void or_forces_multi(int64_t n, const double *x, const double box[3], const int32_t *cnt,
                     const int32_t *nbr, int32_t cap, double rc, int32_t nt, const int32_t *type,
                     const or_spline *phi, const or_spline *rho, const double *fp, double *f) {
  const double half[3] = {0.5 * box[0], 0.5 * box[1], 0.5 * box[2]};
  const double rc2 = rc * rc;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double fx = 0.0, fy = 0.0, fz = 0.0, d[3];
    const int32_t ti = type[i];
    int32_t m = cnt[i] < cap ? cnt[i] : cap;
    for (int32_t k = 0; k < m; ++k) {
      int32_t j = nbr[i * cap + k];
      const int32_t tj = type[j];
      double r2 = dist2(x + 3 * i, x + 3 * j, box, half, d);
      if (r2 < rc2) {
        double r = sqrt(r2);
        double s = fp[i] * spl_df(&rho[tj], r) + fp[j] * spl_df(&rho[ti], r) +
                   spl_df(&phi[ti * nt + tj], r);
        fx += s * d[0] / r;
        fy += s * d[1] / r;
        fz += s * d[2] / r;
      }
    }
    f[3 * i + 0] = fx;
    f[3 * i + 1] = fy;
    f[3 * i + 2] = fz;
  }
}

/* Totals of Eq. (potential) and the kinetic energy, summed in atom order. */
void or_energy_multi(int64_t n, const double *x, const double *v, const double box[3],
                     const int32_t *cnt, const int32_t *nbr, int32_t cap, double rc, int32_t nt,
                     const int32_t *type, const or_spline *phi, const or_spline *rho,
                     const or_spline *emb, const double *mass, double ftm2v, double *pe,
                     double *ke) {
  const double half[3] = {0.5 * box[0], 0.5 * box[1], 0.5 * box[2]};
  const double rc2 = rc * rc;
  size_t nn = (size_t)(n > 0 ? n : 1);
  double *rho_i = (double *)malloc(nn * sizeof(double));
  double *ep = (double *)malloc(nn * sizeof(double));
  double *ek = (double *)malloc(nn * sizeof(double));
  or_density_multi(n, x, box, cnt, nbr, cap, rc, nt, type, rho, emb, rho_i, NULL);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double pair = 0.0, d[3];
    const int32_t ti = type[i];
    int32_t m = cnt[i] < cap ? cnt[i] : cap;
    for (int32_t k = 0; k < m; ++k) {
      int32_t j = nbr[i * cap + k];
      double r2 = dist2(x + 3 * i, x + 3 * j, box, half, d);
      if (r2 < rc2) pair += spl_f(&phi[ti * nt + type[j]], sqrt(r2));
    }
    ep[i] = 0.5 * pair + spl_f(&emb[ti], rho_i[i]);
    if (v) {
      const double *vi = v + 3 * i;
      ek[i] = 0.5 * mass[ti] * ((vi[0] * vi[0] + vi[1] * vi[1]) + vi[2] * vi[2]) / ftm2v;
    }
  }
  double sp = 0.0, sk = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    sp += ep[i];
    if (v) sk += ek[i];
  }
  *pe = sp;
  if (ke) *ke = sk;
  free(rho_i);
  free(ep);
  free(ek);
}

static int forces_now_multi(int64_t n, const double *x, const or_md_params *p, int32_t nt,
                            const int32_t *type, const or_spline *phi, const or_spline *rho,
                            const or_spline *emb, md_scratch *w, double *f, or_md_stats *st) {
  st->flags |= or_density_multi(n, x, p->box, w->cnt, w->nbr, p->cap, p->r_cut, nt, type, rho,
                                emb, w->rho, w->fp);
  or_forces_multi(n, x, p->box, w->cnt, w->nbr, p->cap, p->r_cut, nt, type, phi, rho, w->fp, f);
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!isfinite(f[i])) return OR_E_NONFINITE;
  return OR_OK;
}

/* Velocity-Verlet as or_md_run, with the acceleration of atom i scaled by
 * 1/mass[type[i]] (p->mass is not used). */
int32_t or_md_run_multi(int64_t n, double *x, double *v, double *f, const or_md_params *p,
                        int32_t nt, const int32_t *type, const double *mass, const or_spline *phi,
                        const or_spline *rho, const or_spline *emb, int64_t nsteps,
                        double *energy, or_md_stats *st) {
  memset(st, 0, sizeof(*st));
  int32_t nc[3];
  double ic[3];
  const double rl = p->r_cut + p->skin;
  if (or_cell_grid(p->box, rl, nc, ic) != OR_OK &&
      ((p->box[0] > 0.0 && p->box[0] < 2.0 * rl) || (p->box[1] > 0.0 && p->box[1] < 2.0 * rl) ||
       (p->box[2] > 0.0 && p->box[2] < 2.0 * rl)))
    return OR_E_BOX;
  size_t nn = (size_t)(n > 0 ? n : 1);
  md_scratch w;
  w.cnt = (int32_t *)malloc(nn * sizeof(int32_t));
  w.nbr = (int32_t *)malloc(nn * (size_t)p->cap * sizeof(int32_t));
  w.xref = (double *)malloc(nn * 3 * sizeof(double));
  w.rho = (double *)malloc(nn * sizeof(double));
  w.fp = (double *)malloc(nn * sizeof(double));
  const double half[3] = {0.5 * p->box[0], 0.5 * p->box[1], 0.5 * p->box[2]};
  const double lim2 = 0.25 * p->skin * p->skin;
  const double hdt = 0.5 * p->dt;
  int rc = OR_OK;

  if (or_wrap(n, x, p->box)) rc = OR_E_LOST;
  if (rc == OR_OK) rc = build_list(n, x, p, &w, st);
  if (rc == OR_OK) rc = forces_now_multi(n, x, p, nt, type, phi, rho, emb, &w, f, st);
  if (rc == OR_OK && energy)
    or_energy_multi(n, x, v, p->box, w.cnt, w.nbr, p->cap, p->r_cut, nt, type, phi, rho, emb,
                    mass, p->ftm2v, &energy[0], &energy[1]);
  for (int64_t s = 0; s < nsteps && rc == OR_OK; ++s) {
    for (int64_t i = 0; i < n; ++i) {
      const double acc = p->ftm2v / mass[type[i]];
      for (int d = 0; d < 3; ++d) {
        v[3 * i + d] += hdt * (f[3 * i + d] * acc);
        x[3 * i + d] += p->dt * v[3 * i + d];
      }
    }
    if (or_wrap(n, x, p->box)) {
      rc = OR_E_LOST;
      break;
    }
    double mx2 = 0.0, d[3];
    for (int64_t i = 0; i < n; ++i) {
      double r2 = dist2(w.xref + 3 * i, x + 3 * i, p->box, half, d);
      if (r2 > mx2) mx2 = r2;
    }
    if (mx2 > lim2) {
      rc = build_list(n, x, p, &w, st);
      st->rebuilds++;
      if (rc != OR_OK) break;
    }
    rc = forces_now_multi(n, x, p, nt, type, phi, rho, emb, &w, f, st);
    if (rc != OR_OK) break;
    for (int64_t i = 0; i < n; ++i) {
      const double acc = p->ftm2v / mass[type[i]];
      for (int d = 0; d < 3; ++d) v[3 * i + d] += hdt * (f[3 * i + d] * acc);
    }
    st->steps++;
    if (energy)
      or_energy_multi(n, x, v, p->box, w.cnt, w.nbr, p->cap, p->r_cut, nt, type, phi, rho, emb,
                      mass, p->ftm2v, &energy[2 * (s + 1)], &energy[2 * (s + 1) + 1]);
  }
  free(w.cnt);
  free(w.nbr);
  free(w.xref);
  free(w.rho);
  free(w.fp);
  return rc;
}

/* Forces, rho, F' and potential energy of a configuration from scratch. */
int32_t or_forces_at_multi(int64_t n, const double *x_in, const double box[3], double rc,
                           double skin, int32_t cap, int32_t nt, const int32_t *type,
                           const or_spline *phi, const or_spline *rho, const or_spline *emb,
                           double *f, double *rho_out, double *fp_out, double *pe) {
  size_t nn = (size_t)(n > 0 ? n : 1);
  double *x = (double *)malloc(nn * 3 * sizeof(double));
  memcpy(x, x_in, (size_t)n * 3 * sizeof(double));
  int32_t rcode = OR_OK;
  if (or_wrap(n, x, box)) rcode = OR_E_LOST;
  int32_t *cnt = (int32_t *)malloc(nn * sizeof(int32_t));
  int32_t *nbr = (int32_t *)malloc(nn * (size_t)cap * sizeof(int32_t));
  double *fp = (double *)malloc(nn * sizeof(double));
  double *rh = (double *)malloc(nn * sizeof(double));
  if (rcode == OR_OK) {
    int32_t mx = or_list_cells(n, x, box, rc + skin, cap, cnt, nbr);
    if (mx > cap) rcode = OR_E_OVERFLOW;
  }
  if (rcode == OR_OK) {
    int32_t fl = or_density_multi(n, x, box, cnt, nbr, cap, rc, nt, type, rho, emb, rh, fp);
    or_forces_multi(n, x, box, cnt, nbr, cap, rc, nt, type, phi, rho, fp, f);
    if (pe) {
      double one[8] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0};
      or_energy_multi(n, x, NULL, box, cnt, nbr, cap, rc, nt, type, phi, rho, emb, one, 1.0, pe,
                      NULL);
    }
    if (rho_out) memcpy(rho_out, rh, (size_t)n * sizeof(double));
    if (fp_out) memcpy(fp_out, fp, (size_t)n * sizeof(double));
    rcode = fl;
  }
  free(x);
  free(cnt);
  free(nbr);
  free(fp);
  free(rh);
  return rcode;
}
