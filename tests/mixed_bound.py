"""Error bound of the mixed form's pair terms (float32 pair arithmetic),
shared by the mixed-precision parity tests.

Per pair at separation r, the float32 evaluation of a tabulated g(r)
(g = rho, rho', phi') carries two kinds of error (u = 2^-24):
  - the argument.  Both pair passes take the separation from the atoms'
    fixed-point positions: the difference of two quanta counts is exact, its
    conversion to float32, the float32 quantum and their product add 3 u r,
    and the two roundings to the grid add at most sqrt(3) s, with s the
    largest quantum of the box (L / 2^32 in a periodic dimension, 2^-26 A in
    an open one); write s = sigma u.  Then r^2 from two fmas (<= 1.5 u r), r
    from the hardware rsqrt times r^2 (<= 3 u r) and x = r / dx (<= u r):
    together |dr| <= 8.5 u (r + 0.21 sigma), hence |dg| <= |dr| |g'(r)|;
  - the evaluation: float32 coefficients and a Horner cubic in t, at most
    7 u (|g| + dx |g'|) for these smooth tables.
The density sums such terms (compensated summation adds O(n u^2)):
  |d rho_i| <= 20 u sum_j (rho + r' |rho'|),  r' = r + 0.21 sigma
(margins 2.3 on the argument and 2.8 on the evaluation).
The force term s = (F'_i + F'_j) rho'(r) + phi'(r) adds the error of the
form's F' (|F''(rho)| times the rho bound, plus the float32 rounding u |F'|;
counted twice, below) and its own products and sums (2 u |s|); the direction d/r adds
at most 2 |dd| / r + 4.5 u <= 10.5 u + 3.5 s / r, and the final products 2 u.
For r >= 1.5 A and sigma <= 1 A that is about 17 u |s| besides the tables'
8 u, so, with a margin of about 1.3 on the |s| terms and 3 on the argument:
  |d F_i| <= sum_j { 32 u [(|F'_i| + |F'_j|)(|rho'| + r' |rho''|) + |phi'| + r' |phi''|]
                     + 2 (dF'_i + dF'_j) |rho'| },
over the listed partners within r_cut.  The functions are
the analytic ones (the tables are within 1e-6 of them); second derivatives by
central differences of the analytic first derivatives.
"""
import numpy as np

from workloads import potential as P

U = 2.0 ** -24


def _d2(fn, r, h=1e-5):
    return (fn(r + h) - fn(r - h)) / (2.0 * h)


def quantum_sigma(box):
    """Largest fixed-point quantum of the box's dimensions, in units of u (A)."""
    box = np.asarray(box, dtype=np.float64)
    s = np.where(box > 0, np.abs(box) / 2.0 ** 32, 2.0 ** -26)
    return float(s.max() / U)


def pair_bounds(x, box, fp, cnt, nbr, rc=P.RC, chunk=65536):
    """(rho bound, force bound) per atom for positions x, the oracle's F'_i and
    its neighbour list (cnt, nbr).  The force bound also carries the error of
    the form's own F'_j = F'(rho_j): |F''(rho_j)| times rho_j's bound, plus the
    float32 rounding of F'."""
    n = x.shape[0]
    box = np.asarray(box, dtype=np.float64)
    sigma = quantum_sigma(box)
    assert sigma <= 1.0, "the bounds assume quanta of at most u A (periodic edges <= 256 A)"
    per = box > 0

    def pairs(a, b):
        nb = nbr[a:b]
        valid = np.arange(nb.shape[1])[None, :] < cnt[a:b, None]
        j = np.where(valid, nb, 0)
        d = x[j] - x[a:b, None, :]
        d[..., per] -= box[per] * np.round(d[..., per] / box[per])
        r = np.sqrt((d ** 2).sum(-1))
        m = valid & (r < rc)
        return j, m, np.where(m, r, 1.0)

    rb, rho_i = np.zeros(n), np.zeros(n)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        _, m, rr = pairs(a, b)
        rq = rr + 0.21 * sigma
        rb[a:b] = np.where(m, P.rho(rr) + rq * np.abs(P.drho(rr)), 0.0).sum(1)
        rho_i[a:b] = np.where(m, P.rho(rr), 0.0).sum(1)
    rb *= 20 * U
    dfp = np.abs(P.ddemb(rho_i)) * rb + U * np.abs(fp)
    fb = np.zeros(n)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        j, m, rr = pairs(a, b)
        drho, ddrho = P.drho(rr), _d2(P.drho, rr)
        dphi, ddphi = P.dphi(rr), _d2(P.dphi, rr)
        rq = rr + 0.21 * sigma
        t_f = 32 * U * ((np.abs(fp[a:b, None]) + np.abs(fp[j])) * (np.abs(drho) + rq * np.abs(ddrho))
                        + np.abs(dphi) + rq * np.abs(ddphi))
        t_f += 2 * (dfp[a:b, None] + dfp[j]) * np.abs(drho)
        fb[a:b] = np.where(m, t_f, 0.0).sum(1)
    return rb, fb
