// Host special functions for the basis set-up (see setup_math.h).
#include "setup_math.h"

#include <algorithm>
#include <cmath>

namespace helic {

void bessel_j_all(int nmax, double x, double* out) {
  if (nmax < 0) return;
  if (x == 0.0) {
    out[0] = 1.0;
    for (int k = 1; k <= nmax; ++k) out[k] = 0.0;
    return;
  }
  // Start far enough above both the order and the argument that J_M(x) is
  // negligible against J near the turning point: the decay beyond n ~ x is
  // roughly exp(-c (n - x)^{3/2} / sqrt(x)), so a margin ~ 15 x^{1/3} + 20
  // leaves well below double precision.
  int base = std::max(nmax, (int)std::ceil(x));
  int M = base + (int)(15.0 * std::cbrt(x + 1.0)) + 24;
  if (M & 1) ++M;
  const double BIG = 1e250, SMALL = 1e-250;
  double jp1 = 0.0, j = 1e-30, sum = 0.0;
  for (int k = 0; k <= nmax; ++k) out[k] = 0.0;
  // j holds J_k (unnormalised) while k runs down from M to 1
  for (int k = M; k >= 1; --k) {
    double jm1 = (2.0 * k / x) * j - jp1;   // J_{k-1}
    jp1 = j;
    j = jm1;
    if (k - 1 <= nmax) out[k - 1] = j;
    if (((k - 1) & 1) == 0 && k - 1 > 0) sum += 2.0 * j;
    if (std::fabs(j) > BIG) {
      j *= SMALL;
      jp1 *= SMALL;
      sum *= SMALL;
      for (int q = k - 1; q <= nmax; ++q) out[q] *= SMALL;
    }
  }
  sum += j;  // J_0 term
  const double inv = 1.0 / sum;
  for (int k = 0; k <= nmax; ++k) out[k] *= inv;
}

double bessel_j(int p, double x) {
  int a = std::abs(p);
  std::vector<double> buf(a + 1);
  bessel_j_all(a, x, buf.data());
  double v = buf[a];
  return (p < 0 && (a & 1)) ? -v : v;
}

namespace {
// J_a(x) and its derivative J_a'(x) for a >= 0.
void j_and_deriv(int a, double x, double* J, double* dJ) {
  std::vector<double> buf(a + 2);
  bessel_j_all(a + 1, x, buf.data());
  *J = buf[a];
  *dJ = (a == 0) ? -buf[1] : buf[a - 1] - (a / x) * buf[a];
}
}  // namespace

std::vector<double> bessel_zeros(int p, int count) {
  std::vector<double> z;
  if (count <= 0) return z;
  const int a = std::abs(p);
  z.reserve(count);
  const double h = 0.25;   // far below the spacing of consecutive zeros (> 3)
  double x0 = std::max((double)a, 1.0);
  double f0 = bessel_j(a, x0);
  while ((int)z.size() < count) {
    double x1 = x0 + h;
    double f1 = bessel_j(a, x1);
    if (f0 == 0.0) {
      z.push_back(x0);
    } else if ((f0 < 0) != (f1 < 0) || f1 == 0.0) {
      // bracket [lo, hi] with a sign change; safeguarded Newton
      double lo = x0, hi = x1, flo = f0;
      double x = 0.5 * (lo + hi);
      for (int it = 0; it < 100; ++it) {
        double J, dJ;
        j_and_deriv(a, x, &J, &dJ);
        if (J == 0.0) break;
        if ((J < 0) == (flo < 0)) { lo = x; flo = J; } else { hi = x; }
        double xn = x - J / dJ;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        double dx = std::fabs(xn - x);
        x = xn;
        if (dx <= 1e-16 * x) break;
      }
      z.push_back(x);
    }
    x0 = x1;
    f0 = f1;
  }
  return z;
}

namespace {
// P_n^{(0,1)}(x) and P_{n-1}^{(0,1)}(x) by the three-term recurrence
// (k+1)(2k-1) P_k = ((2k+1)(2k-1) x - 1) P_{k-1} - (k-1)(2k+1) P_{k-2}.
void jacobi01(int n, double x, double* pn, double* pn1) {
  double p0 = 1.0, p1 = 0.5 * (3.0 * x - 1.0);
  if (n == 0) { *pn = 1.0; *pn1 = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double pk = (((2.0 * k + 1) * (2.0 * k - 1) * x - 1.0) * p1 - (k - 1.0) * (2.0 * k + 1) * p0) /
                ((k + 1.0) * (2.0 * k - 1));
    p0 = p1;
    p1 = pk;
  }
  *pn = p1;
  *pn1 = p0;
}

// Number of eigenvalues below x of the symmetric tridiagonal matrix T with
// diagonal d and off-diagonal e (e[i] couples i and i + 1): by Sylvester's
// law of inertia, the number of negative pivots of the LDL^T factorisation of
// T - x I, whose pivots obey p_0 = d_0 - x, p_i = d_i - x - e_{i-1}^2 / p_{i-1}
// (the Sturm-sequence count of Barth, Martin and Wilkinson, 1967).  A zero
// pivot is replaced by a tiny negative one.
int count_below(const std::vector<double>& d, const std::vector<double>& e, double x) {
  int neg = 0;
  double piv = 1.0;
  for (size_t i = 0; i < d.size(); ++i) {
    piv = (d[i] - x) - (i > 0 ? e[i - 1] * e[i - 1] / piv : 0.0);
    if (piv == 0.0) piv = -1e-300;
    neg += piv < 0.0;
  }
  return neg;
}

// All eigenvalues of that matrix, ascending, each by bisection on the count
// above inside the Gershgorin interval, down to a few units in the last
// place (the Newton step of the caller polishes them further).
std::vector<double> tridiag_eigenvalues(const std::vector<double>& d, const std::vector<double>& e) {
  const int n = (int)d.size();
  double lo = d[0], hi = d[0];
  for (int i = 0; i < n; ++i) {
    const double rad = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - rad);
    hi = std::max(hi, d[i] + rad);
  }
  std::vector<double> ev(n);
  double floor_k = lo;   // eigenvalue k is >= eigenvalue k - 1
  for (int k = 0; k < n; ++k) {
    double a = floor_k, b = hi;   // count_below(a) <= k < count_below(b)
    for (int it = 0; it < 200 && b - a > 4e-16 * std::max(std::fabs(a), std::fabs(b)); ++it) {
      const double mid = 0.5 * (a + b);
      if (mid <= a || mid >= b) break;
      if (count_below(d, e, mid) > k) b = mid; else a = mid;
    }
    ev[k] = 0.5 * (a + b);
    floor_k = a;
  }
  return ev;
}
}  // namespace

void gauss_jacobi01(int n, double* q, double* w) {
  if (n <= 0) return;
  // Jacobi matrix of the monic polynomials orthogonal for (1 + x) on [-1, 1]
  std::vector<double> d(n), e(n > 1 ? n - 1 : 0);
  for (int k = 0; k < n; ++k) d[k] = 1.0 / ((2.0 * k + 1) * (2.0 * k + 3));
  for (int k = 1; k < n; ++k) e[k - 1] = std::sqrt((double)k * (k + 1)) / (2.0 * k + 1);
  const std::vector<double> nodes = tridiag_eigenvalues(d, e);
  for (int i = 0; i < n; ++i) {
    double x = nodes[i], pn, pn1, dp = 1.0;
    for (int it = 0; it < 4; ++it) {
      jacobi01(n, x, &pn, &pn1);
      // (2n+1)(1-x^2) P_n' = n(-1 - (2n+1) x) P_n + 2 n (n+1) P_{n-1}
      dp = (n * (-1.0 - (2.0 * n + 1) * x) * pn + 2.0 * n * (n + 1.0) * pn1) /
           ((2.0 * n + 1) * (1.0 - x * x));
      double dx = pn / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    jacobi01(n, x, &pn, &pn1);
    dp = (n * (-1.0 - (2.0 * n + 1) * x) * pn + 2.0 * n * (n + 1.0) * pn1) /
         ((2.0 * n + 1) * (1.0 - x * x));
    q[i] = 0.5 * (1.0 + x);
    w[i] = 0.25 * 4.0 / ((1.0 - x * x) * dp * dp);
  }
}

int smooth_at_least(int x) {
  int n = std::max(x, 1);
  for (;; ++n) {
    int y = n;
    for (int p : {2, 3, 5})
      while (y % p == 0) y /= p;
    if (y == 1) return n;
  }
}

}  // namespace helic
