"""Error bound of the mixed form's pair terms (float32 pair arithmetic on
float64 positions), shared by the mixed-precision parity tests.

Per pair at separation r, the float32 evaluation of a tabulated g(r)
(g = rho, rho', phi') carries two kinds of error (u = 2^-24):
  - the argument: the separation rounded to float32 (|dr| <= u r), r^2 from
    two fmas (<= 1.5 u r), r from the hardware rsqrt times r^2 (<= 3 u r) and
    x = r / dx (<= u r): together |dr| <= 6.5 u r, hence |dg| <= 6.5 u r |g'(r)|;
  - the evaluation: float32 coefficients and a Horner cubic in t, at most
    7 u (|g| + dx |g'|) for these smooth tables.
So |dg| <= 8 u (|g| + r |g'|).  The density sums such terms (compensated
summation adds O(n u^2)); the force term s = F'_i rho'(r) + F'_j rho'(r) +
phi'(r) adds the float32 rounding of F' (u |F'|), its own products and sums
(3 u |s|) and the direction d/r (3 u |s|).  With a factor 2 of margin:
  |d rho_i| <= 16 u sum_j (rho + r |rho'|)
  |d F_i|   <= 16 u sum_j [(|F'_i| + |F'_j|)(|rho'| + r |rho''|) + |phi'| + r |phi''|]
over the listed partners within r_cut.  The functions are the analytic ones
(the tables are within 1e-6 of them); second derivatives by central
differences of the analytic first derivatives.
"""
import numpy as np

from workloads import potential as P

U = 2.0 ** -24


def _d2(fn, r, h=1e-5):
    return (fn(r + h) - fn(r - h)) / (2.0 * h)


def pair_bounds(x, box, fp, cnt, nbr, rc=P.RC, chunk=65536):
    """(rho bound, force bound) per atom for positions x, the oracle's F'_i and
    its neighbour list (cnt, nbr)."""
    n = x.shape[0]
    rb, fb = np.zeros(n), np.zeros(n)
    box = np.asarray(box, dtype=np.float64)
    per = box > 0
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        nb = nbr[a:b]
        valid = np.arange(nb.shape[1])[None, :] < cnt[a:b, None]
        j = np.where(valid, nb, 0)
        d = x[j] - x[a:b, None, :]
        d[..., per] -= box[per] * np.round(d[..., per] / box[per])
        r = np.sqrt((d ** 2).sum(-1))
        m = valid & (r < rc)
        rr = np.where(m, r, 1.0)
        rho, drho, ddrho = P.rho(rr), P.drho(rr), _d2(P.drho, rr)
        dphi, ddphi = P.dphi(rr), _d2(P.dphi, rr)
        t_rho = rho + rr * np.abs(drho)
        t_f = ((np.abs(fp[a:b, None]) + np.abs(fp[j])) * (np.abs(drho) + rr * np.abs(ddrho))
               + np.abs(dphi) + rr * np.abs(ddphi))
        rb[a:b] = np.where(m, t_rho, 0.0).sum(1)
        fb[a:b] = np.where(m, t_f, 0.0).sum(1)
    return 16 * U * rb, 16 * U * fb
