// Conical-product Gauss rules on the reference simplex.
//
// The collapsed (Duffy) coordinates map the unit simplex onto the unit cube;
// the first collapsed direction of a d-simplex carries the weight (1-s)^(d-1),
// the next (1-t)^(d-2), ...; each direction gets the n-point Gauss-Jacobi rule
// of its weight, so n points per direction integrate total degree 2n-1
// exactly.  Gauss-Jacobi nodes are the roots of the Jacobi polynomial
// P_n^(a,0) (bracketed on a grid, refined by bisection and Newton on the
// three-term recurrence); weights 2^(a+1) / ((1-x^2) P_n'(x)^2) on [-1,1].
#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "hf_internal.h"

namespace hf {
namespace {

// P_n^(a,b)(x) by the three-term recurrence
double jacobi(int n, double a, double b, double x) {
  if (n == 0) return 1.0;
  double p0 = 1.0;
  double p1 = 0.5 * (a - b + (a + b + 2.0) * x);
  for (int k = 1; k < n; ++k) {
    double c = 2.0 * k + a + b;
    double a1 = 2.0 * (k + 1) * (k + a + b + 1) * c;
    double a2 = (c + 1.0) * (a * a - b * b);
    double a3 = c * (c + 1.0) * (c + 2.0);
    double a4 = 2.0 * (k + a) * (k + b) * (c + 2.0);
    double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

double jacobi_deriv(int n, double a, double b, double x) {
  if (n == 0) return 0.0;
  return 0.5 * (n + a + b + 1.0) * jacobi(n - 1, a + 1.0, b + 1.0, x);
}

// n-point Gauss rule on [0,1] for the weight (1-s)^a, nodes ascending.
void gauss_jacobi01(int n, int a, std::vector<double> &s, std::vector<double> &w) {
  s.clear();
  w.clear();
  const int grid = 4000;
  double xl = -1.0, fl = jacobi(n, a, 0.0, xl);
  for (int g = 1; g <= grid; ++g) {
    double xr = -1.0 + 2.0 * g / grid;
    double fr = jacobi(n, a, 0.0, xr);
    if (fl == 0.0 || fl * fr < 0.0) {
      double lo = xl, hi = xr, flo = fl;
      for (int it = 0; it < 200 && hi - lo > 1e-15; ++it) {
        double mid = 0.5 * (lo + hi);
        double fm = jacobi(n, a, 0.0, mid);
        if ((fm < 0.0) == (flo < 0.0)) {
          lo = mid;
          flo = fm;
        } else {
          hi = mid;
        }
      }
      double x = 0.5 * (lo + hi);
      for (int it = 0; it < 3; ++it) x -= jacobi(n, a, 0.0, x) / jacobi_deriv(n, a, 0.0, x);
      double dp = jacobi_deriv(n, a, 0.0, x);
      double wx = std::pow(2.0, a + 1) / ((1.0 - x * x) * dp * dp);
      s.push_back(0.5 * (1.0 + x));
      w.push_back(wx * std::pow(0.5, a + 1));
    }
    xl = xr;
    fl = fr;
  }
  if ((int)s.size() != n) throw std::runtime_error("Gauss-Jacobi root bracketing failed");
}

}  // namespace

Rule simplex_rule(int dim, int n) {
  Rule r;
  r.dim = dim;
  std::vector<double> s, ws, t, wt, q, wq;
  if (dim == 1) {
    gauss_jacobi01(n, 0, s, ws);
    r.pts = s;
    r.w = ws;
  } else if (dim == 2) {
    gauss_jacobi01(n, 1, s, ws);
    gauss_jacobi01(n, 0, t, wt);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        r.pts.push_back(s[i]);
        r.pts.push_back(t[j] * (1.0 - s[i]));
        r.w.push_back(ws[i] * wt[j]);
      }
  } else if (dim == 3) {
    gauss_jacobi01(n, 2, s, ws);
    gauss_jacobi01(n, 1, t, wt);
    gauss_jacobi01(n, 0, q, wq);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) {
          r.pts.push_back(s[i]);
          r.pts.push_back(t[j] * (1.0 - s[i]));
          r.pts.push_back(q[k] * (1.0 - s[i]) * (1.0 - t[j]));
          r.w.push_back(ws[i] * wt[j] * wq[k]);
        }
  } else {
    throw std::runtime_error("simplex_rule: dim");
  }
  return r;
}

}  // namespace hf
