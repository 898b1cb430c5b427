// Step length of the fourth-order model (Sec. VI-B, eq. fourth), shared by
// the step kernel and the host export of the same rule.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace cvo {

// The maximiser over t > 0 of P(t) = A1 t + A2 t^2 + A3 t^3 + A4 t^4 among
// its local maxima: the step is the t > 0 that maximises the quartic.
// P' = A1 + 2 A2 t + 3 A3 t^2 + 4 A4 t^3 is monotone between 0, the positive
// roots of P'' and Cauchy's bound on the roots of P'.  A local maximum of P is
// a sign change of P' from + to - inside one such piece; it is found by
// Newton's method kept inside the shrinking bracket (bisection whenever a
// Newton step leaves it or stalls).  Among the maxima the one with the
// largest P wins.  Only maxima at t <= tmax count (the model is a Taylor
// expansion, meaningful only near t = 0).  Returns false when P has no local
// maximum on (0, tmax] (P' keeps one sign, or only touches zero, or its
// maxima lie beyond tmax).  A[0] (the value at t = 0) is unused.
__host__ __device__ inline bool quartic_argmax(const double A[5], double* t_out, double tmax = INFINITY) {
  const double c[4] = {A[1], 2.0 * A[2], 3.0 * A[3], 4.0 * A[4]};  // P'
  const double scale = fabs(c[0]) + fabs(c[1]) + fabs(c[2]) + fabs(c[3]);
  if (!(scale > 0.0) || !(scale < INFINITY)) return false;
  // the highest coefficient that is not negligible fixes the degree of P'
  int deg = 3;
  while (deg > 0 && fabs(c[deg]) <= 1e-14 * scale) deg--;
  if (deg == 0) return false;  // P' is a nonzero constant: no sign change
  double bound = 0.0;
  for (int i = 0; i < deg; i++) bound = fmax(bound, fabs(c[i] / c[deg]));
  bound += 1.0;
  const double d3 = deg >= 3 ? c[3] : 0.0, d2 = deg >= 2 ? c[2] : 0.0;
  auto dP = [&](double t) { return c[0] + t * (c[1] + t * (d2 + t * d3)); };
  auto ddP = [&](double t) { return c[1] + t * (2.0 * d2 + t * 3.0 * d3); };
  auto P = [&](double t) { return t * (A[1] + t * (0.5 * c[1] + t * (d2 / 3.0 + t * 0.25 * d3))); };
  // breakpoints: 0, the positive roots of P'' = c1 + 2 c2 t + 3 c3 t^2 below
  // the bound (increasing), the bound
  double bp[4];
  int nb = 0;
  bp[nb++] = 0.0;
  double r[2];
  int nr = 0;
  const double qa = 3.0 * d3, qb = 2.0 * d2, qc = c[1];
  if (qa != 0.0) {
    const double disc = qb * qb - 4.0 * qa * qc;
    if (disc > 0.0) {
      const double sd = sqrt(disc);
      const double qq = -0.5 * (qb + (qb >= 0.0 ? sd : -sd));
      r[nr++] = qq / qa;
      if (qq != 0.0) r[nr++] = qc / qq;
    }
  } else if (qb != 0.0) {
    r[nr++] = -qc / qb;
  }
  if (nr == 2 && r[0] > r[1]) {
    const double tmp = r[0];
    r[0] = r[1];
    r[1] = tmp;
  }
  for (int i = 0; i < nr; i++)
    if (r[i] > 0.0 && r[i] < bound) bp[nb++] = r[i];
  bp[nb++] = bound;

  bool found = false;
  double best_t = 0.0, best_p = 0.0;
  for (int i = 0; i + 1 < nb; i++) {
    double lo = bp[i], hi = bp[i + 1];
    if (!(dP(lo) > 0.0 && dP(hi) <= 0.0)) continue;
    // P' > 0 at lo, <= 0 at hi, monotone in between: one crossing.  Start
    // from the quadratic model's maximiser -A1 / (2 A2) when it falls inside
    // (the usual case: few Newton steps), else from the middle.
    double t = 0.5 * (lo + hi);
    if (c[1] < 0.0) {
      const double tq = -c[0] / c[1];
      if (tq > lo && tq < hi) t = tq;
    }
    for (int it = 0; it < 100; it++) {
      const double f = dP(t);
      if (f > 0.0) lo = t;
      else hi = t;
      if (f == 0.0) break;
      const double fp = ddP(t);
      double tn = (fp != 0.0) ? t - f / fp : 0.5 * (lo + hi);
      if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);  // Newton left the bracket
      if (fabs(tn - t) <= 4e-16 * fabs(t) || !(tn > lo && tn < hi)) {
        t = tn > lo && tn < hi ? tn : t;
        break;
      }
      t = tn;
    }
    if (!(t <= tmax)) continue;
    const double pv = P(t);
    if (!found || pv > best_p) {
      found = true;
      best_t = t;
      best_p = pv;
    }
  }
  if (found) *t_out = best_t;
  return found;
}

}  // namespace cvo
