// Host special functions used by the basis set-up: Bessel functions of the
// first kind of integer order, their positive zeros, and the Gauss-Jacobi rule
// for int_0^1 f(q) q dq.  Plain double-precision C++.
#pragma once
#include <vector>

namespace helic {

// out[0..nmax] = J_0(x) .. J_nmax(x) for x >= 0 (Miller's backward recurrence
// normalised by J_0 + 2 sum_k J_2k = 1).
void bessel_j_all(int nmax, double x, double* out);

// J_p(x) for any integer p (J_{-p} = (-1)^p J_p) and x >= 0.
double bessel_j(int p, double x);

// First `count` positive zeros of J_p (p integer; zeros of J_{-p} = those of
// J_{|p|}), ascending.  Sign changes are bracketed on a fine scan starting at
// x = max(|p|, 1) (no zero of J_p lies below |p| for |p| >= 1, and the first
// zero of J_0 exceeds 2) and refined by safeguarded Newton steps.
std::vector<double> bessel_zeros(int p, int count);

// n-point Gauss rule for int_0^1 f(q) q dq: nodes ascending in (0, 1).
// Golub-Welsch eigenvalues of the Jacobi matrix for the weight (1 + x) on
// [-1, 1], polished by Newton steps on P_n^{(0,1)}; weights from
// w = 4 / ((1 - x^2) P_n'(x)^2), mapped by q = (1 + x)/2, w_q = w/4.
void gauss_jacobi01(int n, double* q, double* w);

// Smallest integer >= x whose prime factors are 2, 3 and 5 only.
int smooth_at_least(int x);

}  // namespace helic
