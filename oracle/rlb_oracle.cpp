// CPU reference ("oracle") for the quadrature-based relativistic lattice
// Boltzmann model of Blaga & Ambrus, "Quadrature-based Lattice Boltzmann Model
// for Relativistic Flows" (arXiv:1608.03004).
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark may load this library.  The GPU product path
// never calls it, and it shares no source with the GPU path.
//
// Everything is plain FP64, written for readability: loops over cell and
// quadrature point in the order the paper states them, no blocking, no fusion.
// The step functions are templates over the scalar type so that the very same
// code, instantiated with a dual number, yields exact forward-mode
// derivatives (the tangent-linear model) used to check the GPU adjoint.
//
// Notation (T0 = reference temperature, p = |p|/T0 the scaled momentum,
// xi = cos(theta); the azimuthal angle drops out of the 1D problem exactly):
//   F(p, xi) = 2*pi * exp(p) * f(p, xi)        weight-free distribution value
//   f_s      = w_p[i] * w_xi[j] * F(p_i, xi_j)  quadrature-weighted value
//   s        = i * Q_xi + j                      point index (radial outer)
// Moments (section "Relativistic lattice Boltzmann equation", N^mu, T^{mu nu}):
//   N0  = T0^3 sum_s w_s p_i F_s        Nz  = T0^3 sum_s w_s p_i xi_j F_s
//   T00 = T0^4 sum_s w_s p_i^2 F_s      T0z = T0^4 sum_s w_s p_i^2 xi_j F_s
//   Tzz = T0^4 sum_s w_s p_i^2 xi_j^2 F_s
// Readings of the paper where it is silent, garbled or ambiguous are marked
// "[reading]" and are listed with reasons in the design notes.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using std::sqrt;

// ---------------------------------------------------------------------------
// Dual number: value + one directional derivative.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
inline Dual sqrt(Dual a) {
  double r = std::sqrt(a.v);
  return {r, a.d / (2.0 * r)};
}
// Builds a scalar with value v and directional derivative d (d is dropped
// for plain doubles).
template <class R>
R seed(double v, double d);
template <>
inline double seed<double>(double v, double) { return v; }
template <>
inline Dual seed<Dual>(double v, double d) { return Dual(v, d); }

// ---------------------------------------------------------------------------
// Orthogonal polynomials (Gauss-Legendre and Gauss-Laguerre rules of the
// section "Discretization of the momentum space using quadrature rules").
// ---------------------------------------------------------------------------

// Legendre P_n(x) by the three-term recurrence (k+1)P_{k+1} = (2k+1)x P_k - k P_{k-1}.
template <class R>
R legendre_P(int n, R x) {
  if (n == 0) return R(1.0);
  R p0 = R(1.0), p1 = x;
  for (int k = 1; k < n; ++k) {
    R p2 = (R(2.0 * k + 1.0) * x * p1 - R(double(k)) * p0) / R(k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// Generalised Laguerre L^{(1)}_n(x):
// (n+1) L_{n+1} = (2n+2-x) L_n - (n+1) L_{n-1},  L_0 = 1, L_1 = 2 - x.
template <class T>
T laguerre1(int n, T x) {
  if (n == 0) return T(1);
  T l0 = T(1), l1 = T(2) - x;
  for (int k = 1; k < n; ++k) {
    T l2 = ((T(2 * k + 2) - x) * l1 - T(k + 1) * l0) / T(k + 1);
    l0 = l1;
    l1 = l2;
  }
  return l1;
}

// Gauss-Legendre rule of order q on [-1, 1] (polar integral).  Nodes are the
// zeros of P_q, found by Newton's method from the classical cosine guess.
// Weights follow the paper's formula with its typo corrected [reading]:
//   w_j = 2 (1 - xi_j^2) / ((q+1)^2 P_{q+1}(xi_j)^2).
// Nodes and weights are computed in 80-bit extended precision and rounded.
// The rule is made exactly symmetric; for odd q the middle node is exactly 0.
void gauss_legendre(int q, double* x, double* w) {
  typedef long double E;
  const E pi = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < (q + 1) / 2; ++j) {
    E z = std::cos(pi * (j + 0.75L) / (q + 0.5L));  // descending positive roots
    for (int it = 0; it < 100; ++it) {
      E pn = legendre_P<E>(q, z), pm = legendre_P<E>(q - 1, z);
      E dp = q * (pm - z * pn) / (1 - z * z);
      E dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    if (q % 2 == 1 && j == q / 2) z = 0;
    // P_{q+1} at a zero of P_q equals -(1 - xi^2) P_q'(xi) / (q+1); taking it
    // from the derivative (which keeps the tiny residual P_q(z) of the computed
    // node) is far better conditioned than the three-term recurrence for
    // P_{q+1}, whose error is amplified ~q^2 near xi = +-1.
    const E pq = legendre_P<E>(q, z), pqm = legendre_P<E>(q - 1, z);
    const E dpq = q * (pqm - z * pq) / (1 - z * z);
    E pq1 = -(1 - z * z) * dpq / E(q + 1);
    E wj = 2 * (1 - z * z) / (E(q + 1) * E(q + 1) * pq1 * pq1);
    x[q - 1 - j] = double(z);  // ascending order
    w[q - 1 - j] = double(wj);
    x[j] = -double(z);
    w[j] = double(wj);
  }
}

// Gauss-Laguerre rule with weight p e^{-p} (alpha = 1) of order q (radial
// integral).  Nodes are the zeros of L^{(1)}_q, bracketed by a scan and refined
// by bisection, in extended precision.  Weights as printed:
//   w_i = p_i / ((q+1) [L^{(1)}_{q+1}(p_i)]^2).
int gauss_laguerre1(int q, double* x, double* w) {
  typedef long double E;
  const E hi = 4.0L * q + 12.0L, h = 1e-3L;
  int found = 0;
  E a = 1e-12L, fa = laguerre1<E>(q, a);
  for (int step = 1; a <= hi && found < q; ++step) {
    E b = 1e-12L + step * h;
    E fb = laguerre1<E>(q, b);
    if ((fa < 0) != (fb < 0)) {
      E lo = a, up = b, flo = fa;
      for (int it = 0; it < 200; ++it) {
        E mid = (lo + up) / 2;
        E fm = laguerre1<E>(q, mid);
        if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { up = mid; }
        if (up - lo < 1e-19L * up) break;
      }
      E r = (lo + up) / 2;
      E lq1 = laguerre1<E>(q + 1, r);
      x[found] = double(r);
      w[found] = double(r / (E(q + 1) * lq1 * lq1));
      ++found;
    }
    a = b;
    fa = fb;
  }
  return found == q ? 0 : -1;
}

// ---------------------------------------------------------------------------
// Problem description (section "Riemann problem", section "Numerical results").
// ---------------------------------------------------------------------------
}  // namespace

extern "C" {
struct oracle_tube {
  int32_t nx;        // cells; cell-centred grid on [z_min, z_max]
  double z_min, z_max;
  int32_t q_xi, q_p; // Gauss-Legendre / Gauss-Laguerre(alpha=1) orders
  int32_t n_v, n_p;  // truncation orders of the equilibrium expansion
  double tau;        // relaxation time (+inf: collisionless)
  double dt;         // time step
  double T0;         // reference temperature
  double weno_eps;   // WENO epsilon, applied to the weight-free F
};
struct oracle_state {
  double P, n, u;    // pressure, density, u^z
};
}

namespace {

// Auxiliary high-order rule for the angular projection integral.
constexpr int kAuxOrder = 160;

struct Tables {
  int qx, qp, nv, np;
  std::vector<double> xi, wxi, p, wp;
  std::vector<double> Pk;    // [j][k]  P_k(xi_j)
  std::vector<double> Ll;    // [i][l]  L^{(1)}_l(p_i)
  std::vector<double> ax, aw, aPk;  // auxiliary rule and P_k at its nodes
  double T0;
  explicit Tables(const oracle_tube& t)
      : qx(t.q_xi), qp(t.q_p), nv(t.n_v), np(t.n_p), T0(t.T0) {
    xi.resize(qx); wxi.resize(qx); p.resize(qp); wp.resize(qp);
    gauss_legendre(qx, xi.data(), wxi.data());
    gauss_laguerre1(qp, p.data(), wp.data());
    Pk.resize(size_t(qx) * (nv + 1));
    for (int j = 0; j < qx; ++j)
      for (int k = 0; k <= nv; ++k) Pk[j * (nv + 1) + k] = legendre_P(k, xi[j]);
    Ll.resize(size_t(qp) * (np + 1));
    for (int i = 0; i < qp; ++i)
      for (int l = 0; l <= np; ++l) Ll[i * (np + 1) + l] = laguerre1<double>(l, p[i]);
    ax.resize(kAuxOrder); aw.resize(kAuxOrder);
    gauss_legendre(kAuxOrder, ax.data(), aw.data());
    aPk.resize(size_t(kAuxOrder) * (nv + 1));
    for (int a = 0; a < kAuxOrder; ++a)
      for (int k = 0; k <= nv; ++k) aPk[a * (nv + 1) + k] = legendre_P(k, ax[a]);
  }
  int Q() const { return qx * qp; }
};

// Macroscopic state of one cell after the Landau matching.
template <class R>
struct Macro {
  R e, v, gamma, u, n, T;
};

// Moments N0, Nz, T00, T0z, Tzz of one cell (definition of N^mu, T^{mu nu}).
template <class R>
void cell_moments(const Tables& tb, const R* F, int64_t nx, int64_t x, R m[5]) {
  for (int c = 0; c < 5; ++c) m[c] = R(0.0);
  const double t3 = tb.T0 * tb.T0 * tb.T0, t4 = t3 * tb.T0;
  for (int i = 0; i < tb.qp; ++i)
    for (int j = 0; j < tb.qx; ++j) {
      const int s = i * tb.qx + j;
      const R f = R(tb.wp[i] * tb.wxi[j]) * F[s * nx + x];
      const double pi = tb.p[i], xj = tb.xi[j];
      m[0] += R(t3 * pi) * f;
      m[1] += R(t3 * pi * xj) * f;
      m[2] += R(t4 * pi * pi) * f;
      m[3] += R(t4 * pi * pi * xj) * f;
      m[4] += R(t4 * pi * pi * xj * xj) * f;
    }
}

// Landau-Lifshitz matching T^mu_nu u^nu = -e u^mu in 1D (a 2x2 eigenproblem).
// With v = u^z/u^0 the two component equations give
//   T00 - T0z v = e,   T0z - Tzz v = e v,
// whose physical root is e = (T00 - Tzz + sqrt((T00+Tzz)^2 - 4 T0z^2))/2,
// v = T0z/(e + Tzz).  The density is n = -u_mu N^mu = gamma (N0 - v Nz) and,
// for the massless Maxwell-Juettner gas, e = 3 n T, so T = e/(3n)  [reading].
template <class R>
Macro<R> landau(const R m[5]) {
  const R a = m[2] + m[4];
  const R disc = (a - R(2.0) * m[3]) * (a + R(2.0) * m[3]);
  Macro<R> M;
  M.e = R(0.5) * (m[2] - m[4] + sqrt(disc));
  M.v = m[3] / (M.e + m[4]);
  M.gamma = R(1.0) / sqrt(R(1.0) - M.v * M.v);
  M.u = M.gamma * M.v;
  M.n = M.gamma * (m[0] - M.v * m[1]);
  M.T = M.e / (R(3.0) * M.n);
  return M;
}

// Projection coefficients of the equilibrium (eq. feqtrunc and the moment
// recovery property eq. mom_feq).  The truncated equilibrium is the orthogonal
// projection of F^eq onto span{L_l(p) P_k(xi)} under the measure p e^{-p} dp dxi:
//   C_kl = int_{-1}^{1} dxi P_k(xi) int_0^inf dp p e^{-p} F^eq(p, xi) L_l(p).
// F^eq = (n/(4T^3)) exp(p (1 - beta)), beta = T0 (gamma - xi u)/T (eq. feqMJ with
// p^alpha u_alpha = -p (u^0 - xi u^z); the sign of the printed eq. feq is taken
// from eq. feqMJ [reading]).  The radial integral is the Laplace transform
//   int_0^inf p e^{-beta p} L^{(1)}_l(p) dp = (l+1) (beta-1)^l / beta^(l+2),
// and the angular integral is done with a 160-point Gauss-Legendre rule.
// C has layout [k][l], k <= n_v, l <= n_p.
template <class R>
void feq_coefficients(const Tables& tb, R n, R T, R gamma, R u, R* C) {
  const int nv = tb.nv, np = tb.np;
  for (int c = 0; c < (nv + 1) * (np + 1); ++c) C[c] = R(0.0);
  const R pref = n / (R(4.0) * T * T * T);
  for (int a = 0; a < kAuxOrder; ++a) {
    const R beta = R(tb.T0) * (gamma - R(tb.ax[a]) * u) / T;
    const R ib = R(1.0) / beta;
    const R r = (beta - R(1.0)) * ib;  // (beta-1)/beta
    R radial = pref * ib * ib;         // l = 0 term without (l+1)
    for (int l = 0; l <= np; ++l) {
      const R A = R(l + 1.0) * radial;
      for (int k = 0; k <= nv; ++k)
        C[k * (np + 1) + l] += R(tb.aw[a] * tb.aPk[a * (nv + 1) + k]) * A;
      radial = radial * r;
    }
  }
}

// Truncated equilibrium at every quadrature node, weight-free:
//   F_trunc(p_i, xi_j) = sum_l sum_k (2k+1)/2 * 1/(l+1) * C_kl P_k(xi_j) L_l(p_i).
template <class R>
void feq_nodes(const Tables& tb, R n, R T, R gamma, R u, R* Feq) {
  const int nv = tb.nv, np = tb.np;
  std::vector<R> C((nv + 1) * (np + 1));
  feq_coefficients(tb, n, T, gamma, u, C.data());
  for (int i = 0; i < tb.qp; ++i)
    for (int j = 0; j < tb.qx; ++j) {
      R acc = R(0.0);
      for (int l = 0; l <= np; ++l)
        for (int k = 0; k <= nv; ++k)
          acc += R((2.0 * k + 1.0) / 2.0 / (l + 1.0) * tb.Pk[j * (nv + 1) + k] *
                   tb.Ll[i * (np + 1) + l]) *
                 C[k * (np + 1) + l];
      Feq[i * tb.qx + j] = acc;
    }
}

// Fifth-order WENO reconstruction of Jiang and Shu at the face between v3 and
// v4 from the upwind-biased values v1..v5 (section "Numerical results", WENO5).
template <class R>
R weno5(R v1, R v2, R v3, R v4, R v5, double eps) {
  const R q0 = (R(2.0) * v1 - R(7.0) * v2 + R(11.0) * v3) / R(6.0);
  const R q1 = (-v2 + R(5.0) * v3 + R(2.0) * v4) / R(6.0);
  const R q2 = (R(2.0) * v3 + R(5.0) * v4 - v5) / R(6.0);
  const R c13 = R(13.0 / 12.0), c14 = R(0.25);
  const R t0 = v1 - R(2.0) * v2 + v3, s0 = v1 - R(4.0) * v2 + R(3.0) * v3;
  const R t1 = v2 - R(2.0) * v3 + v4, s1 = v2 - v4;
  const R t2 = v3 - R(2.0) * v4 + v5, s2 = R(3.0) * v3 - R(4.0) * v4 + v5;
  const R b0 = c13 * t0 * t0 + c14 * s0 * s0;
  const R b1 = c13 * t1 * t1 + c14 * s1 * s1;
  const R b2 = c13 * t2 * t2 + c14 * s2 * s2;
  const R e0 = R(eps) + b0, e1 = R(eps) + b1, e2 = R(eps) + b2;
  const R a0 = R(0.1) / (e0 * e0), a1 = R(0.6) / (e1 * e1), a2 = R(0.3) / (e2 * e2);
  return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

// Open (zero-gradient outflow) boundary: the three ghost cells on each side
// repeat the edge cell [reading of the open boundaries the paper names].
inline int64_t clampx(int64_t x, int64_t nx) { return x < 0 ? 0 : (x >= nx ? nx - 1 : x); }

// Weight-free numerical flux value H at face x+1/2 for node row F (length nx),
// upwinded by the sign of xi.
template <class R>
R face_value(const R* F, int64_t nx, int64_t x, double xi, double eps) {
  auto g = [&](int64_t y) { return F[clampx(y, nx)]; };
  if (xi >= 0.0) return weno5(g(x - 2), g(x - 1), g(x), g(x + 1), g(x + 2), eps);
  return weno5(g(x + 3), g(x + 2), g(x + 1), g(x), g(x - 1), eps);
}

// Right-hand side L(F) of the 1D Boltzmann equation (eq. Boltz):
//   dF/dt = -xi dF/dz - ((u^0 - xi u^z)/tau) (F - F^eq).
// F, out: [Q][nx].  tau_inv is 1/tau (0 for the collisionless limit).
template <class R>
void rhs(const Tables& tb, const oracle_tube& t, R tau_inv, const R* F, R* out) {
  const int64_t nx = t.nx;
  const double dz = (t.z_max - t.z_min) / t.nx;
  const int Q = tb.Q();
#pragma omp parallel
  {
    std::vector<R> feq(Q);
#pragma omp for schedule(static)
    for (int64_t x = 0; x < nx; ++x) {
      R m[5];
      cell_moments(tb, F, nx, x, m);
      const Macro<R> M = landau(m);
      feq_nodes(tb, M.n, M.T, M.gamma, M.u, feq.data());
      for (int i = 0; i < tb.qp; ++i)
        for (int j = 0; j < tb.qx; ++j) {
          const int s = i * tb.qx + j;
          const double xi = tb.xi[j];
          const R* row = F + s * nx;
          const R hr = face_value(row, nx, x, xi, t.weno_eps);
          const R hl = face_value(row, nx, x - 1, xi, t.weno_eps);
          const R adv = R(-xi / dz) * (hr - hl);
          const R rate = (M.gamma - R(xi) * M.u) * tau_inv;
          out[s * nx + x] = adv - rate * (row[x] - feq[s]);
        }
    }
  }
}

// Third-order strong-stability-preserving Runge-Kutta step of Shu and Osher
// (the third-order TVD Runge-Kutta integrator named in section Numerical
// results) [reading]:
//   F1 = F + dt L(F);  F2 = 3/4 F + 1/4 (F1 + dt L(F1));
//   F' = 1/3 F + 2/3 (F2 + dt L(F2)).
template <class R>
void rk3_step(const Tables& tb, const oracle_tube& t, R tau_inv, R* F, R* F1, R* F2, R* L) {
  const int64_t N = int64_t(tb.Q()) * t.nx;
  const R dt = R(t.dt);
  rhs(tb, t, tau_inv, F, L);
  for (int64_t a = 0; a < N; ++a) F1[a] = F[a] + dt * L[a];
  rhs(tb, t, tau_inv, F1, L);
  for (int64_t a = 0; a < N; ++a) F2[a] = R(0.75) * F[a] + R(0.25) * (F1[a] + dt * L[a]);
  rhs(tb, t, tau_inv, F2, L);
  for (int64_t a = 0; a < N; ++a)
    F[a] = R(1.0 / 3.0) * F[a] + R(2.0 / 3.0) * (F2[a] + dt * L[a]);
}

// Initial condition (eq. condinit): the truncated equilibrium of the left state
// for z < 0 and of the right state otherwise.  Cells are classified by their
// centre; a centre exactly at z = 0 takes the right state [reading].
template <class R>
void init_state(const Tables& tb, const oracle_tube& t, const oracle_state* side_val,
                const oracle_state* side_dot, R* F) {
  const int64_t nx = t.nx;
  const double dz = (t.z_max - t.z_min) / t.nx;
  const int Q = tb.Q();
  std::vector<R> feq[2];
  for (int sd = 0; sd < 2; ++sd) {
    feq[sd].resize(Q);
    const R P = seed<R>(side_val[sd].P, side_dot ? side_dot[sd].P : 0.0);
    const R n = seed<R>(side_val[sd].n, side_dot ? side_dot[sd].n : 0.0);
    const R u = seed<R>(side_val[sd].u, side_dot ? side_dot[sd].u : 0.0);
    const R T = P / n;
    const R gamma = sqrt(R(1.0) + u * u);
    feq_nodes(tb, n, T, gamma, u, feq[sd].data());
  }
  for (int64_t x = 0; x < nx; ++x) {
    const double z = t.z_min + (x + 0.5) * dz;
    const int sd = z < 0.0 ? 0 : 1;
    for (int s = 0; s < Q; ++s) F[s * nx + x] = feq[sd][s];
  }
}

// Diagnostic fields per cell: N0, Nz, T00, T0z, Tzz, e, n, v, T, |N|.
template <class R>
void fields(const Tables& tb, const oracle_tube& t, const R* F, R* out) {
  const int64_t nx = t.nx;
  for (int64_t x = 0; x < nx; ++x) {
    R m[5];
    cell_moments(tb, F, nx, x, m);
    const Macro<R> M = landau(m);
    for (int c = 0; c < 5; ++c) out[c * nx + x] = m[c];
    out[5 * nx + x] = M.e;
    out[6 * nx + x] = M.n;
    out[7 * nx + x] = M.v;
    out[8 * nx + x] = M.T;
    out[9 * nx + x] = sqrt(m[0] * m[0] - m[1] * m[1]);
  }
}

bool valid(const oracle_tube* t) {
  return t && t->nx >= 1 && t->q_xi >= 1 && t->q_p >= 1 && t->n_v >= 0 && t->n_p >= 0 &&
         t->tau > 0 && t->dt > 0 && t->T0 > 0 && t->z_max > t->z_min;
}

}  // namespace

// ---------------------------------------------------------------------------
// C entry points (called from Python through ctypes).  All arrays are FP64,
// F in the [s][x] layout with s = i * q_xi + j.  Return 0 on success, -1 on an
// invalid argument.
// ---------------------------------------------------------------------------
extern "C" {

int oracle_gauss_legendre(int q, double* x, double* w) {
  if (q < 1) return -1;
  gauss_legendre(q, x, w);
  return 0;
}

int oracle_gauss_laguerre1(int q, double* x, double* w) {
  if (q < 1) return -1;
  return gauss_laguerre1(q, x, w);
}

double oracle_legendre(int n, double x) { return legendre_P<double>(n, x); }
double oracle_laguerre1(int n, double x) { return laguerre1<double>(n, x); }

double oracle_weno5(double v1, double v2, double v3, double v4, double v5, double eps) {
  return weno5(v1, v2, v3, v4, v5, eps);
}

// Landau matching: m = (N0, Nz, T00, T0z, Tzz) -> out = (e, v, gamma, u, n, T).
int oracle_landau(const double* m, double* out) {
  Macro<double> M = landau(m);
  out[0] = M.e; out[1] = M.v; out[2] = M.gamma; out[3] = M.u; out[4] = M.n; out[5] = M.T;
  return 0;
}

// Projection coefficients C[k][l] for the macroscopic state (n, T, u).
int oracle_feq_coefficients(const oracle_tube* t, double n, double T, double u, double* C) {
  if (!valid(t)) return -1;
  Tables tb(*t);
  feq_coefficients(tb, n, T, std::sqrt(1.0 + u * u), u, C);
  return 0;
}

// Truncated equilibrium at the Q nodes, weight-free (F_s, not f_s).
int oracle_feq_nodes(const oracle_tube* t, double n, double T, double u, double* F) {
  if (!valid(t)) return -1;
  Tables tb(*t);
  feq_nodes(tb, n, T, std::sqrt(1.0 + u * u), u, F);
  return 0;
}

// Quadrature tables: xi[q_xi], wxi[q_xi], p[q_p], wp[q_p].
int oracle_tables(const oracle_tube* t, double* xi, double* wxi, double* p, double* wp) {
  if (!valid(t)) return -1;
  Tables tb(*t);
  std::memcpy(xi, tb.xi.data(), sizeof(double) * tb.qx);
  std::memcpy(wxi, tb.wxi.data(), sizeof(double) * tb.qx);
  std::memcpy(p, tb.p.data(), sizeof(double) * tb.qp);
  std::memcpy(wp, tb.wp.data(), sizeof(double) * tb.qp);
  return 0;
}

int oracle_init(const oracle_tube* t, oracle_state left, oracle_state right, double* F) {
  if (!valid(t)) return -1;
  Tables tb(*t);
  oracle_state sides[2] = {left, right};
  init_state<double>(tb, *t, sides, nullptr, F);
  return 0;
}

// Advance F ([Q][nx], in place) by nsteps SSP-RK3 steps.
int oracle_step(const oracle_tube* t, double* F, int64_t nsteps) {
  if (!valid(t) || nsteps < 0) return -1;
  Tables tb(*t);
  const int64_t N = int64_t(tb.Q()) * t->nx;
  std::vector<double> F1(N), F2(N), L(N);
  const double ti = 1.0 / t->tau;
  for (int64_t n = 0; n < nsteps; ++n) rk3_step(tb, *t, ti, F, F1.data(), F2.data(), L.data());
  return 0;
}

// One evaluation of the right-hand side (for unit tests of the update).
int oracle_rhs(const oracle_tube* t, const double* F, double* out) {
  if (!valid(t)) return -1;
  Tables tb(*t);
  rhs(tb, *t, 1.0 / t->tau, F, out);
  return 0;
}

int oracle_fields(const oracle_tube* t, const double* F, double* out) {
  if (!valid(t)) return -1;
  Tables tb(*t);
  fields(tb, *t, F, out);
  return 0;
}

// Tangent-linear model: advances (F, dF) by nsteps, where dF is the derivative
// of F along a direction that also moves tau by dtau.
int oracle_step_tangent(const oracle_tube* t, double* F, double* dF, double dtau, int64_t nsteps) {
  if (!valid(t) || nsteps < 0) return -1;
  Tables tb(*t);
  const int64_t N = int64_t(tb.Q()) * t->nx;
  std::vector<Dual> G(N), G1(N), G2(N), L(N);
  for (int64_t a = 0; a < N; ++a) G[a] = Dual(F[a], dF[a]);
  // d(1/tau) = -dtau/tau^2, written out so that tau = +inf (collisionless
  // limit) gives an exact zero instead of 0 * inf in the quotient rule.
  const Dual ti = Dual(1.0 / t->tau, -dtau / (t->tau * t->tau));
  for (int64_t n = 0; n < nsteps; ++n) rk3_step(tb, *t, ti, G.data(), G1.data(), G2.data(), L.data());
  for (int64_t a = 0; a < N; ++a) { F[a] = G[a].v; dF[a] = G[a].d; }
  return 0;
}

// Tangent of the initial condition along (dleft, dright).
int oracle_init_tangent(const oracle_tube* t, oracle_state left, oracle_state right,
                        oracle_state dleft, oracle_state dright, double* F, double* dF) {
  if (!valid(t)) return -1;
  Tables tb(*t);
  const int64_t N = int64_t(tb.Q()) * t->nx;
  std::vector<Dual> G(N);
  oracle_state sides[2] = {left, right}, dots[2] = {dleft, dright};
  init_state<Dual>(tb, *t, sides, dots, G.data());
  for (int64_t a = 0; a < N; ++a) { F[a] = G[a].v; dF[a] = G[a].d; }
  return 0;
}

// Tangent of the diagnostic fields.
int oracle_fields_tangent(const oracle_tube* t, const double* F, const double* dF, double* out,
                          double* dout) {
  if (!valid(t)) return -1;
  Tables tb(*t);
  const int64_t N = int64_t(tb.Q()) * t->nx;
  std::vector<Dual> G(N), O(10 * int64_t(t->nx));
  for (int64_t a = 0; a < N; ++a) G[a] = Dual(F[a], dF[a]);
  fields(tb, *t, G.data(), O.data());
  for (int64_t a = 0; a < 10 * int64_t(t->nx); ++a) { out[a] = O[a].v; dout[a] = O[a].d; }
  return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"

// ===========================================================================
// Multi-dimensional model on a plane (x, z).
//
// The general equation (eq. Boltz_gen, with v = p/p^0 resolved in both
// directions of the plane) reads, for the weight-free F:
//   dF/dt = -v_x dF/dx - v_z dF/dz - ((u^0 - v_x u^x - v_z u^z)/tau) (F - F^eq),
// with v = (sin(theta) cos(phi), sin(theta) sin(phi), cos(theta)) and the
// full product quadrature of the section on the discretization of momentum
// space: Gauss-Laguerre in p, Gauss-Legendre in xi = cos(theta) and the
// trapezoid rule in phi (eq. azimuthInt) with nodes phi_k = 2 pi k / Q_phi
// [reading: the printed nodes are garbled; any periodic trapezoid grid is
// exact below Q_phi].  Nothing depends on y, and data with u^y = 0 stay
// symmetric under phi -> -phi, so the nodes k and Q_phi - k carry equal values
// and only k = 0 .. Q_phi/2 are evolved, with weights omega_k = m_k / Q_phi
// (m_k = 2 for a mirrored pair, 1 otherwise; sum omega_k = 1) [reading].
// F keeps the normalisation of the 1D oracle (2 pi e^p f), so a plane with no
// x dependence reproduces the 1D tube.
//
// Point s = (i * Q_xi + j) * Q_h + k, Q_h = Q_phi/2 + 1 (integer division);
// F[s][z][x].  Moments per cell (9; the y components vanish):
//   N0, Nx, Nz   = T0^3 sum w p   {1, v_x, v_z} F
//   T00, T0x, T0z, Txx, Txz, Tzz = T0^4 sum w p^2 {1, v_x, v_z, v_x^2, v_x v_z, v_z^2} F
// with w = w_p w_xi omega.
//
// The Landau frame is the timelike eigenvector of T^mu_nu (T^mu_nu u^nu =
// -e u^mu); -e is the eigenvalue of largest magnitude (the other eigenvalues
// are the principal pressures, and e >= each of them for a massless gas), so
// the power method converges to it.  With u = gamma (1, v) one power step is
//   v_i <- (T^{0i} - T^{ij} v_j) / (T^{00} - T^{0j} v_j).
//
// Equilibrium: f^eq depends on the direction only through c = v . u_hat
// (u_hat = u/|u|), so its orthogonal projection onto the polynomials of degree
// <= N_v in v (the span of the vector polynomials of eq. feqtrunc) is the
// Legendre series in c (Funk-Hecke), with the coefficients of the 1D
// projection taken at the speed |u| [reading]:
//   F_trunc(p_i, v) = sum_l sum_k (2k+1)/2 / (l+1) C_kl(|u|) P_k(c) L_l(p_i).
// ===========================================================================

extern "C" {
struct oracle_plane {
  int32_t nx, nz;           // cells along x and z, cell-centred
  double x_min, x_max, z_min, z_max;
  int32_t q_xi, q_phi, q_p; // quadrature orders
  int32_t n_v, n_p;         // truncation orders
  double tau, dt, T0, weno_eps;
};
}

namespace {

struct PlaneTables {
  Tables t1;                      // polar and radial rules, projection rule
  int qh;                         // evolved azimuthal nodes
  std::vector<double> cphi, omega, sth;
  static oracle_tube as_tube(const oracle_plane& p) {
    oracle_tube t;
    std::memset(&t, 0, sizeof t);
    t.nx = p.nx;
    t.z_min = p.z_min;
    t.z_max = p.z_max;
    t.q_xi = p.q_xi;
    t.q_p = p.q_p;
    t.n_v = p.n_v;
    t.n_p = p.n_p;
    t.tau = p.tau;
    t.dt = p.dt;
    t.T0 = p.T0;
    t.weno_eps = p.weno_eps;
    return t;
  }
  explicit PlaneTables(const oracle_plane& p) : t1(as_tube(p)), qh(p.q_phi / 2 + 1) {
    const long double pi = 3.141592653589793238462643383279502884L;
    cphi.resize(qh);
    omega.resize(qh);
    for (int k = 0; k < qh; ++k) {
      cphi[k] = double(std::cos(2.0L * pi * k / p.q_phi));
      const bool single = (k == 0) || (2 * k == p.q_phi);
      omega[k] = (single ? 1.0 : 2.0) / p.q_phi;
    }
    sth.resize(t1.qx);
    for (int j = 0; j < t1.qx; ++j) sth[j] = std::sqrt(1.0 - t1.xi[j] * t1.xi[j]);
  }
  int Q() const { return t1.qp * t1.qx * qh; }
  double vx(int j, int k) const { return sth[j] * cphi[k]; }
  double vz(int j) const { return t1.xi[j]; }
};

struct Macro2 {
  double e, vx, vz, gamma, ux, uz, n, T;
};

// Moments of one cell (s-major layout with `cells` values per point row).
void plane_moments(const PlaneTables& pt, const double* F, int64_t cells, int64_t c, double m[9]) {
  for (int a = 0; a < 9; ++a) m[a] = 0.0;
  const Tables& tb = pt.t1;
  const double t3 = tb.T0 * tb.T0 * tb.T0, t4 = t3 * tb.T0;
  for (int i = 0; i < tb.qp; ++i)
    for (int j = 0; j < tb.qx; ++j)
      for (int k = 0; k < pt.qh; ++k) {
        const int s = (i * tb.qx + j) * pt.qh + k;
        const double f = tb.wp[i] * tb.wxi[j] * pt.omega[k] * F[s * cells + c];
        const double vx = pt.vx(j, k), vz = pt.vz(j), p = tb.p[i];
        m[0] += t3 * p * f;
        m[1] += t3 * p * vx * f;
        m[2] += t3 * p * vz * f;
        m[3] += t4 * p * p * f;
        m[4] += t4 * p * p * vx * f;
        m[5] += t4 * p * p * vz * f;
        m[6] += t4 * p * p * vx * vx * f;
        m[7] += t4 * p * p * vx * vz * f;
        m[8] += t4 * p * p * vz * vz * f;
      }
}

// Landau frame of the 9 moments by the power method on T^mu_nu (extended
// precision; converged when a step changes v by less than 1e-19).
Macro2 landau2(const double m[9]) {
  typedef long double E;
  const E N0 = m[0], Nx = m[1], Nz = m[2], T00 = m[3], T0x = m[4], T0z = m[5], Txx = m[6], Txz = m[7],
          Tzz = m[8];
  E vx = 0, vz = 0;
  for (int it = 0; it < 1000000; ++it) {
    const E e = T00 - T0x * vx - T0z * vz;
    const E nx_ = (T0x - Txx * vx - Txz * vz) / e, nz_ = (T0z - Txz * vx - Tzz * vz) / e;
    const E d = std::fabs(nx_ - vx) + std::fabs(nz_ - vz);
    vx = nx_;
    vz = nz_;
    if (!(d > 1e-19L)) break;
  }
  Macro2 M;
  const E e = T00 - T0x * vx - T0z * vz;
  const E gamma = 1 / std::sqrt(1 - vx * vx - vz * vz);
  M.e = double(e);
  M.vx = double(vx);
  M.vz = double(vz);
  M.gamma = double(gamma);
  M.ux = double(gamma * vx);
  M.uz = double(gamma * vz);
  M.n = double(gamma * (N0 - vx * Nx - vz * Nz));
  M.T = double(e / (3 * gamma * (N0 - vx * Nx - vz * Nz)));
  return M;
}

// Truncated equilibrium at every point of the plane's quadrature.
void plane_feq_nodes(const PlaneTables& pt, double n, double T, double ux, double uz, double* Feq) {
  const Tables& tb = pt.t1;
  const double ua = std::sqrt(ux * ux + uz * uz), gamma = std::sqrt(1.0 + ua * ua);
  const double hx = ua > 0.0 ? ux / ua : 0.0, hz = ua > 0.0 ? uz / ua : 1.0;
  std::vector<double> C((tb.nv + 1) * (tb.np + 1));
  feq_coefficients(tb, n, T, gamma, ua, C.data());
  for (int i = 0; i < tb.qp; ++i)
    for (int j = 0; j < tb.qx; ++j)
      for (int k = 0; k < pt.qh; ++k) {
        const double c = pt.vx(j, k) * hx + pt.vz(j) * hz;
        double acc = 0.0;
        for (int l = 0; l <= tb.np; ++l)
          for (int kk = 0; kk <= tb.nv; ++kk)
            acc += (2.0 * kk + 1.0) / 2.0 / (l + 1.0) * legendre_P(kk, c) * tb.Ll[i * (tb.np + 1) + l] *
                   C[kk * (tb.np + 1) + l];
        Feq[(i * tb.qx + j) * pt.qh + k] = acc;
      }
}

// WENO value at face y+1/2 of a strided line of n values (outflow clamps),
// upwinded by the sign of the velocity component.
double face_value_line(const double* base, int64_t n, int64_t stride, int64_t y, double vel, double eps) {
  auto g = [&](int64_t q) { return base[clampx(q, n) * stride]; };
  if (vel >= 0.0) return weno5(g(y - 2), g(y - 1), g(y), g(y + 1), g(y + 2), eps);
  return weno5(g(y + 3), g(y + 2), g(y + 1), g(y), g(y - 1), eps);
}

void plane_rhs(const PlaneTables& pt, const oracle_plane& pl, const double* F, double* out) {
  const int64_t nx = pl.nx, nz = pl.nz, cells = nx * nz;
  const double dx = (pl.x_max - pl.x_min) / pl.nx, dz = (pl.z_max - pl.z_min) / pl.nz;
  const double tau_inv = 1.0 / pl.tau;
  const Tables& tb = pt.t1;
  const int Q = pt.Q();
#pragma omp parallel
  {
    std::vector<double> feq(Q);
#pragma omp for schedule(static)
    for (int64_t c = 0; c < cells; ++c) {
      const int64_t z = c / nx, x = c % nx;
      double m[9];
      plane_moments(pt, F, cells, c, m);
      const Macro2 M = landau2(m);
      plane_feq_nodes(pt, M.n, M.T, M.ux, M.uz, feq.data());
      for (int i = 0; i < tb.qp; ++i)
        for (int j = 0; j < tb.qx; ++j)
          for (int k = 0; k < pt.qh; ++k) {
            const int s = (i * tb.qx + j) * pt.qh + k;
            const double vx = pt.vx(j, k), vz = pt.vz(j);
            const double* plane = F + s * cells;
            const double hxr = face_value_line(plane + z * nx, nx, 1, x, vx, pl.weno_eps);
            const double hxl = face_value_line(plane + z * nx, nx, 1, x - 1, vx, pl.weno_eps);
            const double hzr = face_value_line(plane + x, nz, nx, z, vz, pl.weno_eps);
            const double hzl = face_value_line(plane + x, nz, nx, z - 1, vz, pl.weno_eps);
            const double adv = -vx / dx * (hxr - hxl) - vz / dz * (hzr - hzl);
            const double rate = (M.gamma - vx * M.ux - vz * M.uz) * tau_inv;
            out[s * cells + c] = adv - rate * (plane[c] - feq[s]);
          }
    }
  }
}

void plane_rk3_step(const PlaneTables& pt, const oracle_plane& pl, double* F, double* F1, double* F2, double* L) {
  const int64_t N = int64_t(pt.Q()) * pl.nx * pl.nz;
  const double dt = pl.dt;
  plane_rhs(pt, pl, F, L);
  for (int64_t a = 0; a < N; ++a) F1[a] = F[a] + dt * L[a];
  plane_rhs(pt, pl, F1, L);
  for (int64_t a = 0; a < N; ++a) F2[a] = 0.75 * F[a] + 0.25 * (F1[a] + dt * L[a]);
  plane_rhs(pt, pl, F2, L);
  for (int64_t a = 0; a < N; ++a) F[a] = (1.0 / 3.0) * F[a] + (2.0 / 3.0) * (F2[a] + dt * L[a]);
}

bool plane_valid(const oracle_plane* p) {
  return p && p->nx >= 1 && p->nz >= 1 && p->q_xi >= 1 && p->q_phi >= 1 && p->q_p >= 1 && p->n_v >= 0 &&
         p->n_p >= 0 && p->tau > 0 && p->dt > 0 && p->T0 > 0 && p->x_max > p->x_min && p->z_max > p->z_min;
}

}  // namespace

extern "C" {

// Azimuthal rule of the plane: cos(phi_k) and omega_k of the evolved nodes.
int oracle_plane_tables(const oracle_plane* p, double* cphi, double* omega) {
  if (!plane_valid(p)) return -1;
  PlaneTables pt(*p);
  for (int k = 0; k < pt.qh; ++k) {
    cphi[k] = pt.cphi[k];
    omega[k] = pt.omega[k];
  }
  return 0;
}

// Landau frame of (N0, Nx, Nz, T00, T0x, T0z, Txx, Txz, Tzz) -> e, vx, vz, gamma, n, T.
int oracle_landau2d(const double* m, double* out) {
  const Macro2 M = landau2(m);
  const double r[6] = {M.e, M.vx, M.vz, M.gamma, M.n, M.T};
  for (int a = 0; a < 6; ++a) out[a] = r[a];
  return 0;
}

int oracle_plane_feq_nodes(const oracle_plane* p, double n, double T, double ux, double uz, double* F) {
  if (!plane_valid(p)) return -1;
  PlaneTables pt(*p);
  plane_feq_nodes(pt, n, T, ux, uz, F);
  return 0;
}

// Initial distribution from per-cell states fields[4][nz][nx] = P, n, u^x, u^z.
int oracle_plane_init(const oracle_plane* p, const double* fields, double* F) {
  if (!plane_valid(p)) return -1;
  PlaneTables pt(*p);
  const int64_t cells = int64_t(p->nx) * p->nz;
  std::vector<double> feq(pt.Q());
  for (int64_t c = 0; c < cells; ++c) {
    const double P = fields[c], n = fields[cells + c], ux = fields[2 * cells + c], uz = fields[3 * cells + c];
    plane_feq_nodes(pt, n, P / n, ux, uz, feq.data());
    for (int s = 0; s < pt.Q(); ++s) F[s * cells + c] = feq[s];
  }
  return 0;
}

int oracle_plane_step(const oracle_plane* p, double* F, int64_t nsteps) {
  if (!plane_valid(p) || nsteps < 0) return -1;
  PlaneTables pt(*p);
  const size_t N = size_t(pt.Q()) * p->nx * p->nz;
  std::vector<double> F1(N), F2(N), L(N);
  for (int64_t n = 0; n < nsteps; ++n) plane_rk3_step(pt, *p, F, F1.data(), F2.data(), L.data());
  return 0;
}

int oracle_plane_rhs(const oracle_plane* p, const double* F, double* out) {
  if (!plane_valid(p)) return -1;
  PlaneTables pt(*p);
  plane_rhs(pt, *p, F, out);
  return 0;
}

// Fields per cell [14][nz][nx]: the 9 moments, e, n, v_x, v_z, T.
int oracle_plane_fields(const oracle_plane* p, const double* F, double* out) {
  if (!plane_valid(p)) return -1;
  PlaneTables pt(*p);
  const int64_t cells = int64_t(p->nx) * p->nz;
  for (int64_t c = 0; c < cells; ++c) {
    double m[9];
    plane_moments(pt, F, cells, c, m);
    const Macro2 M = landau2(m);
    for (int a = 0; a < 9; ++a) out[a * cells + c] = m[a];
    out[9 * cells + c] = M.e;
    out[10 * cells + c] = M.n;
    out[11 * cells + c] = M.vx;
    out[12 * cells + c] = M.vz;
    out[13 * cells + c] = M.T;
  }
  return 0;
}

}  // extern "C"

// ===========================================================================
// Multi-dimensional model on a box (x, y, z), any flow direction.
//
// eq. Boltz_gen with v = (sin(theta) cos(phi), sin(theta) sin(phi), cos(theta))
// resolved in all three directions:
//   dF/dt = -v_x dF/dx - v_y dF/dy - v_z dF/dz
//           - ((u^0 - v_x u^x - v_y u^y - v_z u^z)/tau) (F - F^eq),
// on the full product quadrature: Gauss-Laguerre in p, Gauss-Legendre in
// xi = cos(theta) and every node of the trapezoid rule in phi (eq.
// azimuthInt), phi_k = 2 pi k / Q_phi, k = 0 .. Q_phi - 1, weight 1/Q_phi of
// the phi-average [reading: the printed nodes are garbled; a periodic
// trapezoid grid is exact below Q_phi].  No node is collapsed: the velocity
// may point anywhere.  F keeps the 1D normalisation (2 pi e^p f), so a box
// varying along z only with u along z reproduces the tube, and one with
// ny = 1 and u^y = 0 reproduces the plane.
//
// Point s = (i * Q_xi + j) * Q_phi + k; F[s][z][y][x].  Moments per cell (14):
//   N0, Nx, Ny, Nz = T0^3 sum w p {1, v_x, v_y, v_z} F
//   T00, T0x, T0y, T0z, Txx, Txy, Txz, Tyy, Tyz, Tzz
//                  = T0^4 sum w p^2 {1, v_i, v_i v_j} F
// with w = w_p w_xi / Q_phi.  Landau frame: the timelike eigenvector of
// T^mu_nu by the power method (as for the plane, three velocity components).
// Equilibrium: the Legendre series in c = v . u_hat with the 1D coefficients
// at the speed |u| (Funk-Hecke, as for the plane) [reading].
// ===========================================================================

extern "C" {
struct oracle_box {
  int32_t nx, ny, nz;       // cells along x, y and z, cell-centred
  double x_min, x_max, y_min, y_max, z_min, z_max;
  int32_t q_xi, q_phi, q_p; // quadrature orders
  int32_t n_v, n_p;         // truncation orders
  double tau, dt, T0, weno_eps;
};
}

namespace {

struct BoxTables {
  Tables t1;
  int qf;
  std::vector<double> cphi, sphi, sth;
  static oracle_tube as_tube(const oracle_box& b) {
    oracle_tube t;
    std::memset(&t, 0, sizeof t);
    t.nx = b.nz;
    t.z_min = b.z_min;
    t.z_max = b.z_max;
    t.q_xi = b.q_xi;
    t.q_p = b.q_p;
    t.n_v = b.n_v;
    t.n_p = b.n_p;
    t.tau = b.tau;
    t.dt = b.dt;
    t.T0 = b.T0;
    t.weno_eps = b.weno_eps;
    return t;
  }
  explicit BoxTables(const oracle_box& b) : t1(as_tube(b)), qf(b.q_phi) {
    const long double pi = 3.141592653589793238462643383279502884L;
    cphi.resize(qf);
    sphi.resize(qf);
    for (int k = 0; k < qf; ++k) {
      cphi[k] = double(std::cos(2.0L * pi * k / qf));
      sphi[k] = double(std::sin(2.0L * pi * k / qf));
    }
    sth.resize(t1.qx);
    for (int j = 0; j < t1.qx; ++j) sth[j] = std::sqrt(1.0 - t1.xi[j] * t1.xi[j]);
  }
  int Q() const { return t1.qp * t1.qx * qf; }
  double vx(int j, int k) const { return sth[j] * cphi[k]; }
  double vy(int j, int k) const { return sth[j] * sphi[k]; }
  double vz(int j) const { return t1.xi[j]; }
};

struct Macro3 {
  double e, v[3], gamma, u[3], n, T;
};

// Moments of one cell: m = N0, Nx, Ny, Nz, T00, T0x, T0y, T0z, Txx, Txy, Txz,
// Tyy, Tyz, Tzz.
void box_moments(const BoxTables& bt, const double* F, int64_t cells, int64_t c, double m[14]) {
  for (int a = 0; a < 14; ++a) m[a] = 0.0;
  const Tables& tb = bt.t1;
  const double t3 = tb.T0 * tb.T0 * tb.T0, t4 = t3 * tb.T0;
  for (int i = 0; i < tb.qp; ++i)
    for (int j = 0; j < tb.qx; ++j)
      for (int k = 0; k < bt.qf; ++k) {
        const int s = (i * tb.qx + j) * bt.qf + k;
        const double f = tb.wp[i] * tb.wxi[j] / bt.qf * F[s * cells + c];
        const double v[3] = {bt.vx(j, k), bt.vy(j, k), bt.vz(j)}, p = tb.p[i];
        m[0] += t3 * p * f;
        for (int a = 0; a < 3; ++a) m[1 + a] += t3 * p * v[a] * f;
        m[4] += t4 * p * p * f;
        for (int a = 0; a < 3; ++a) m[5 + a] += t4 * p * p * v[a] * f;
        int q = 8;
        for (int a = 0; a < 3; ++a)
          for (int b = a; b < 3; ++b) m[q++] += t4 * p * p * v[a] * v[b] * f;
      }
}

// Spatial tensor T^{ab} of the 14 moments.
inline long double box_Tij(const double m[14], int a, int b) {
  if (a > b) std::swap(a, b);
  static const int idx[3][3] = {{8, 9, 10}, {9, 11, 12}, {10, 12, 13}};
  return m[idx[a][b]];
}

// Landau frame by the power method on T^mu_nu (extended precision): with
// u = gamma (1, v), one step is v_i <- (T^{0i} - T^{ij} v_j) / (T^{00} - T^{0j} v_j).
Macro3 landau3(const double m[14]) {
  typedef long double E;
  const E N0 = m[0], T00 = m[4];
  const E N[3] = {m[1], m[2], m[3]}, T0[3] = {m[5], m[6], m[7]};
  E v[3] = {0, 0, 0};
  for (int it = 0; it < 1000000; ++it) {
    const E e = T00 - T0[0] * v[0] - T0[1] * v[1] - T0[2] * v[2];
    E nv[3];
    for (int a = 0; a < 3; ++a) {
      E r = T0[a];
      for (int b = 0; b < 3; ++b) r -= box_Tij(m, a, b) * v[b];
      nv[a] = r / e;
    }
    const E d = std::fabs(nv[0] - v[0]) + std::fabs(nv[1] - v[1]) + std::fabs(nv[2] - v[2]);
    for (int a = 0; a < 3; ++a) v[a] = nv[a];
    if (!(d > 1e-19L)) break;
  }
  Macro3 M;
  const E e = T00 - T0[0] * v[0] - T0[1] * v[1] - T0[2] * v[2];
  const E gamma = 1 / std::sqrt(1 - v[0] * v[0] - v[1] * v[1] - v[2] * v[2]);
  const E n = gamma * (N0 - v[0] * N[0] - v[1] * N[1] - v[2] * N[2]);
  M.e = double(e);
  for (int a = 0; a < 3; ++a) {
    M.v[a] = double(v[a]);
    M.u[a] = double(gamma * v[a]);
  }
  M.gamma = double(gamma);
  M.n = double(n);
  M.T = double(e / (3 * n));
  return M;
}

// Truncated equilibrium at every point of the box's quadrature.
void box_feq_nodes(const BoxTables& bt, double n, double T, const double u[3], double* Feq) {
  const Tables& tb = bt.t1;
  const double ua = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]), gamma = std::sqrt(1.0 + ua * ua);
  const double h[3] = {ua > 0.0 ? u[0] / ua : 0.0, ua > 0.0 ? u[1] / ua : 0.0, ua > 0.0 ? u[2] / ua : 1.0};
  std::vector<double> C((tb.nv + 1) * (tb.np + 1));
  feq_coefficients(tb, n, T, gamma, ua, C.data());
  for (int i = 0; i < tb.qp; ++i)
    for (int j = 0; j < tb.qx; ++j)
      for (int k = 0; k < bt.qf; ++k) {
        const double c = bt.vx(j, k) * h[0] + bt.vy(j, k) * h[1] + bt.vz(j) * h[2];
        double acc = 0.0;
        for (int l = 0; l <= tb.np; ++l)
          for (int kk = 0; kk <= tb.nv; ++kk)
            acc += (2.0 * kk + 1.0) / 2.0 / (l + 1.0) * legendre_P(kk, c) * tb.Ll[i * (tb.np + 1) + l] *
                   C[kk * (tb.np + 1) + l];
        Feq[(i * tb.qx + j) * bt.qf + k] = acc;
      }
}

void box_rhs(const BoxTables& bt, const oracle_box& bx, const double* F, double* out) {
  const int64_t nx = bx.nx, ny = bx.ny, nz = bx.nz, cells = nx * ny * nz;
  const double dx = (bx.x_max - bx.x_min) / bx.nx, dy = (bx.y_max - bx.y_min) / bx.ny,
               dz = (bx.z_max - bx.z_min) / bx.nz;
  const double tau_inv = 1.0 / bx.tau;
  const Tables& tb = bt.t1;
  const int Q = bt.Q();
#pragma omp parallel
  {
    std::vector<double> feq(Q);
#pragma omp for schedule(static)
    for (int64_t c = 0; c < cells; ++c) {
      const int64_t x = c % nx, y = (c / nx) % ny, z = c / (nx * ny);
      double m[14];
      box_moments(bt, F, cells, c, m);
      const Macro3 M = landau3(m);
      box_feq_nodes(bt, M.n, M.T, M.u, feq.data());
      for (int i = 0; i < tb.qp; ++i)
        for (int j = 0; j < tb.qx; ++j)
          for (int k = 0; k < bt.qf; ++k) {
            const int s = (i * tb.qx + j) * bt.qf + k;
            const double vx = bt.vx(j, k), vy = bt.vy(j, k), vz = bt.vz(j);
            const double* pt = F + s * cells;
            const double* row_x = pt + (z * ny + y) * nx;
            const double* row_y = pt + z * nx * ny + x;
            const double* row_z = pt + y * nx + x;
            const double hxr = face_value_line(row_x, nx, 1, x, vx, bx.weno_eps);
            const double hxl = face_value_line(row_x, nx, 1, x - 1, vx, bx.weno_eps);
            const double hyr = face_value_line(row_y, ny, nx, y, vy, bx.weno_eps);
            const double hyl = face_value_line(row_y, ny, nx, y - 1, vy, bx.weno_eps);
            const double hzr = face_value_line(row_z, nz, nx * ny, z, vz, bx.weno_eps);
            const double hzl = face_value_line(row_z, nz, nx * ny, z - 1, vz, bx.weno_eps);
            const double adv = -vx / dx * (hxr - hxl) - vy / dy * (hyr - hyl) - vz / dz * (hzr - hzl);
            const double rate = (M.gamma - vx * M.u[0] - vy * M.u[1] - vz * M.u[2]) * tau_inv;
            out[s * cells + c] = adv - rate * (pt[c] - feq[s]);
          }
    }
  }
}

void box_rk3_step(const BoxTables& bt, const oracle_box& bx, double* F, double* F1, double* F2, double* L) {
  const int64_t N = int64_t(bt.Q()) * bx.nx * bx.ny * bx.nz;
  const double dt = bx.dt;
  box_rhs(bt, bx, F, L);
  for (int64_t a = 0; a < N; ++a) F1[a] = F[a] + dt * L[a];
  box_rhs(bt, bx, F1, L);
  for (int64_t a = 0; a < N; ++a) F2[a] = 0.75 * F[a] + 0.25 * (F1[a] + dt * L[a]);
  box_rhs(bt, bx, F2, L);
  for (int64_t a = 0; a < N; ++a) F[a] = (1.0 / 3.0) * F[a] + (2.0 / 3.0) * (F2[a] + dt * L[a]);
}

bool box_valid(const oracle_box* b) {
  return b && b->nx >= 1 && b->ny >= 1 && b->nz >= 1 && b->q_xi >= 1 && b->q_phi >= 1 && b->q_p >= 1 &&
         b->n_v >= 0 && b->n_p >= 0 && b->tau > 0 && b->dt > 0 && b->T0 > 0 && b->x_max > b->x_min &&
         b->y_max > b->y_min && b->z_max > b->z_min;
}

}  // namespace

extern "C" {

// Azimuthal nodes of the box: cos(phi_k), sin(phi_k).
int oracle_box_tables(const oracle_box* b, double* cphi, double* sphi) {
  if (!box_valid(b)) return -1;
  BoxTables bt(*b);
  for (int k = 0; k < bt.qf; ++k) {
    cphi[k] = bt.cphi[k];
    sphi[k] = bt.sphi[k];
  }
  return 0;
}

// Landau frame of the 14 moments -> e, v_x, v_y, v_z, gamma, n, T.
int oracle_landau3d(const double* m, double* out) {
  const Macro3 M = landau3(m);
  const double r[7] = {M.e, M.v[0], M.v[1], M.v[2], M.gamma, M.n, M.T};
  for (int a = 0; a < 7; ++a) out[a] = r[a];
  return 0;
}

int oracle_box_feq_nodes(const oracle_box* b, double n, double T, double ux, double uy, double uz, double* F) {
  if (!box_valid(b)) return -1;
  BoxTables bt(*b);
  const double u[3] = {ux, uy, uz};
  box_feq_nodes(bt, n, T, u, F);
  return 0;
}

// Initial distribution from per-cell states fields[5][nz][ny][nx] = P, n, u^x, u^y, u^z.
int oracle_box_init(const oracle_box* b, const double* fields, double* F) {
  if (!box_valid(b)) return -1;
  BoxTables bt(*b);
  const int64_t cells = int64_t(b->nx) * b->ny * b->nz;
  std::vector<double> feq(bt.Q());
  for (int64_t c = 0; c < cells; ++c) {
    const double P = fields[c], n = fields[cells + c];
    const double u[3] = {fields[2 * cells + c], fields[3 * cells + c], fields[4 * cells + c]};
    box_feq_nodes(bt, n, P / n, u, feq.data());
    for (int s = 0; s < bt.Q(); ++s) F[s * cells + c] = feq[s];
  }
  return 0;
}

int oracle_box_step(const oracle_box* b, double* F, int64_t nsteps) {
  if (!box_valid(b) || nsteps < 0) return -1;
  BoxTables bt(*b);
  const size_t N = size_t(bt.Q()) * b->nx * b->ny * b->nz;
  std::vector<double> F1(N), F2(N), L(N);
  for (int64_t n = 0; n < nsteps; ++n) box_rk3_step(bt, *b, F, F1.data(), F2.data(), L.data());
  return 0;
}

int oracle_box_rhs(const oracle_box* b, const double* F, double* out) {
  if (!box_valid(b)) return -1;
  BoxTables bt(*b);
  box_rhs(bt, *b, F, out);
  return 0;
}

// Fields per cell [20][nz][ny][nx]: the 14 moments, e, n, v_x, v_y, v_z, T.
int oracle_box_fields(const oracle_box* b, const double* F, double* out) {
  if (!box_valid(b)) return -1;
  BoxTables bt(*b);
  const int64_t cells = int64_t(b->nx) * b->ny * b->nz;
  for (int64_t c = 0; c < cells; ++c) {
    double m[14];
    box_moments(bt, F, cells, c, m);
    const Macro3 M = landau3(m);
    for (int a = 0; a < 14; ++a) out[a * cells + c] = m[a];
    out[14 * cells + c] = M.e;
    out[15 * cells + c] = M.n;
    for (int a = 0; a < 3; ++a) out[(16 + a) * cells + c] = M.v[a];
    out[19 * cells + c] = M.T;
  }
  return 0;
}

}  // extern "C"
