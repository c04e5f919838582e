// Host-side quadrature tables of the momentum discretisation (section
// "Discretization of the momentum space using quadrature rules"):
//   polar  -- Gauss-Legendre rule in xi = cos(theta) (eq. polarInt),
//   radial -- Gauss-Laguerre rule for the weight p e^{-p} (alpha = 1).
//
// Nodes: eigenvalues of the symmetric tridiagonal Jacobi matrix of the
// orthonormal polynomials (Golub-Welsch), found by implicit QL iteration and
// polished by Newton's method on the three-term recurrence.  Weights: the
// Christoffel numbers 1/sum_k ptilde_k(x)^2 of the orthonormal polynomials,
// a sum of positive terms that stays accurate near the ends of the interval.
// Everything runs in 80-bit extended precision and is rounded once.
#include <algorithm>
#include <cmath>
#include <vector>

#include "quadrature.h"

namespace rlb {
namespace {

typedef long double E;

// Eigenvalues of the symmetric tridiagonal matrix with diagonal d and
// off-diagonal e (e[k] couples k and k+1), by implicit QL with Wilkinson
// shifts.  d is overwritten with the eigenvalues (unsorted).  The iteration is
// the published tridiagonal QL algorithm (Bowdler, Martin, Reinsch and
// Wilkinson, Numer. Math. 11 (1968) 293, the "tql1" procedure, also in the
// public-domain EISPACK library), restated here for extended precision.
bool tridiagonal_eigenvalues(std::vector<E>& d, std::vector<E> e) {
  const int n = static_cast<int>(d.size());
  e.push_back(0);
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m < n - 1; ++m) {
        E dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 1e-21L * dd) break;
      }
      if (m == l) break;
      if (iter > 200) return false;
      E g = (d[l + 1] - d[l]) / (2 * e[l]);
      E r = std::hypot(g, E(1));
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      E s = 1, c = 1, p = 0;
      int i = m - 1;
      for (; i >= l; --i) {
        E f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0) {
          d[i + 1] -= p;
          e[m] = 0;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
      }
      if (r == 0 && i >= l) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0;
    }
  }
  return true;
}

// Orthonormal Legendre values ptilde_0..ptilde_{n} at x (ptilde_k = sqrt((2k+1)/2) P_k).
void legendre_all(int n, E x, std::vector<E>& P) {
  P.assign(n + 1, 0);
  P[0] = 1;
  if (n >= 1) P[1] = x;
  for (int k = 1; k < n; ++k) P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
}

void laguerre1_all(int n, E x, std::vector<E>& L) {
  L.assign(n + 1, 0);
  L[0] = 1;
  if (n >= 1) L[1] = 2 - x;
  for (int k = 1; k < n; ++k) L[k + 1] = ((2 * k + 2 - x) * L[k] - (k + 1) * L[k - 1]) / (k + 1);
}

}  // namespace

bool gauss_legendre_rule(int q, std::vector<double>& x, std::vector<double>& w) {
  if (q < 1) return false;
  // Jacobi matrix of orthonormal Legendre polynomials: zero diagonal,
  // off-diagonal k/sqrt(4k^2-1).
  std::vector<E> d(q, 0), e(q > 1 ? q - 1 : 0);
  for (int k = 1; k < q; ++k) e[k - 1] = E(k) / std::sqrt(E(4) * k * k - 1);
  if (!tridiagonal_eigenvalues(d, e)) return false;
  std::sort(d.begin(), d.end());
  std::vector<E> P;
  std::vector<E> xs(q), ws(q);
  for (int j = 0; j < q; ++j) {
    E z = d[j];
    for (int it = 0; it < 4; ++it) {  // Newton polish on P_q
      legendre_all(q, z, P);
      E dp = q * (P[q - 1] - z * P[q]) / (1 - z * z);
      z -= P[q] / dp;
    }
    legendre_all(q - 1, z, P);
    E s = 0;
    for (int k = 0; k < q; ++k) s += (2 * k + 1) * P[k] * P[k] / 2;
    xs[j] = z;
    ws[j] = 1 / s;
  }
  x.resize(q);
  w.resize(q);
  // exact symmetry; the middle node of an odd rule is exactly zero
  for (int j = 0; j < q; ++j) {
    const int m = q - 1 - j;
    E ax = (xs[m] - xs[j]) / 2, aw = (ws[m] + ws[j]) / 2;
    if (j == m) ax = 0;
    x[j] = -double(ax);
    w[j] = double(aw);
  }
  if (q % 2 == 1) x[q / 2] = 0.0;
  return true;
}

bool gauss_laguerre1_rule(int q, std::vector<double>& x, std::vector<double>& w) {
  if (q < 1) return false;
  // Jacobi matrix of orthonormal generalised Laguerre (alpha = 1):
  // diagonal 2k+2, off-diagonal sqrt(k (k+1)).
  std::vector<E> d(q), e(q > 1 ? q - 1 : 0);
  for (int k = 0; k < q; ++k) d[k] = 2 * k + 2;
  for (int k = 1; k < q; ++k) e[k - 1] = std::sqrt(E(k) * (k + 1));
  if (!tridiagonal_eigenvalues(d, e)) return false;
  std::sort(d.begin(), d.end());
  std::vector<E> L;
  x.resize(q);
  w.resize(q);
  for (int i = 0; i < q; ++i) {
    E z = d[i];
    for (int it = 0; it < 4; ++it) {  // Newton polish: z L_q' = q L_q - (q+1) L_{q-1}
      laguerre1_all(q, z, L);
      E dl = (q * L[q] - (q + 1) * L[q - 1]) / z;
      z -= L[q] / dl;
    }
    laguerre1_all(q - 1, z, L);
    E s = 0;
    for (int k = 0; k < q; ++k) s += L[k] * L[k] / (k + 1);
    x[i] = double(z);
    w[i] = double(1 / s);
  }
  return true;
}

double legendre_value(int n, double x) {
  std::vector<E> P;
  legendre_all(n, x, P);
  return double(P[n]);
}

double laguerre1_value(int n, double x) {
  std::vector<E> L;
  laguerre1_all(n, x, L);
  return double(L[n]);
}

}  // namespace rlb
