// Device-side arithmetic shared by the forward and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "rlb_internal.h"

namespace rlb {
namespace dev {

// Read-only kernel inputs (tube descriptors, work lists, quadrature tables) are
// read through the constant address space so that wave-uniform reads become
// scalar loads into SGPRs instead of 64-lane vector loads.
template <typename T>
using cptr = __attribute__((address_space(4))) const T*;
template <typename T>
__device__ inline cptr<T> as_const(const T* p) {
  return (cptr<T>)(p);
}

// n/d with one hardware reciprocal: FP32 takes one correction step (< 2 ulp);
// FP64 refines the reciprocal twice by Newton's method and corrects the
// quotient once, which is close to correctly rounded.
__device__ inline float fast_div(float n, float d) {
  const float r = __builtin_amdgcn_rcpf(d);
  const float q = n * r;
  return fmaf(r, fmaf(-d, q, n), q);
}
__device__ inline double fast_div(double n, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  const double q = n * r;
  return fma(r, fma(-d, q, n), q);
}

// Raw buffer resources: a scalar base and size, accessed with a 32-bit
// per-lane byte offset and a scalar byte offset, so that loads and stores carry
// no per-lane 64-bit address arithmetic.  AUX is the cache policy
// (0: default, 2: non-temporal).
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // word 3 of a raw 32-bit-format resource (gfx950)

__device__ inline Rsrc make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(bytes), kRsrcWord3);
}

template <typename Real>
struct BufIO;
template <>
struct BufIO<float> {
  template <int AUX>
  static __device__ inline float load(Rsrc r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), AUX));
  }
  template <int AUX>
  static __device__ inline void store(float v, Rsrc r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, int(voff), int(soff), AUX);
  }
};
template <>
struct BufIO<double> {
  using V2 = uint32_t __attribute__((ext_vector_type(2)));
  template <int AUX>
  static __device__ inline double load(Rsrc r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), int(soff), AUX));
  }
  template <int AUX>
  static __device__ inline void store(double v, Rsrc r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, int(voff), int(soff), AUX);
  }
};

// ---------------------------------------------------------------------------
// Small arithmetic helpers
// ---------------------------------------------------------------------------
template <typename Real>
struct Acc;  // moment accumulator over the polar nodes of one radial node

template <>
struct Acc<double> {
  double s = 0.0;
  __device__ void add(double x) { s += x; }
  __device__ double value() const { return s; }
};

// Kahan-compensated FP32 sum.
template <>
struct Acc<float> {
  float s = 0.0f, c = 0.0f;
  __device__ void add(float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ double value() const { return double(s) - double(c); }
};

// Initial condition (eq. condinit): cell x takes the left state when its
// centre z_min + (x + 1/2) dz lies below z = 0 (a centre exactly at 0 takes
// the right state).  The centre is formed with a separately rounded product
// and sum, never a fused multiply-add, so that every cell falls on the same
// side as in plain IEEE arithmetic.
__device__ inline bool left_of_split(double z_min, double dz, int x) {
#pragma clang fp contract(off)
  const double centre = z_min + (double(x) + 0.5) * dz;
  return centre < 0.0;
}
__device__ inline bool left_of_split(const TubeDev& tb, int x) { return left_of_split(tb.z_min, tb.dz, x); }

// XCD-aware work distribution.  Workgroups are dispatched round-robin over the
// 8 XCDs (workgroup b runs on XCD b % 8), and each XCD has its own L2.  The
// work list keeps a tube's tiles in ascending order; handing each XCD runs of
// kXcdRun consecutive items puts neighbouring tiles -- which read each other's
// 3-cell halos -- on the same L2, while the interleaving of runs keeps the
// cost balanced when the list is sorted by cost (batched tubes).  v is the
// workgroup's virtual index (blockIdx.x + k * gridDim.x with gridDim.x a
// multiple of 8, or plain blockIdx.x); the map is a bijection on [0, n): items
// past the last whole super-block of 8 * kXcdRun are taken in order.
constexpr int kXcds = 8;
constexpr int kXcdRun = 16;
__device__ inline int xcd_item(int v, int n) {
  constexpr int S = kXcds * kXcdRun;
  const int n_full = (n / S) * S;
  if (v >= n_full) return v;
  const int x = v % kXcds, k = v / kXcds;
  return (k / kXcdRun) * S + x * kXcdRun + (k % kXcdRun);
}

struct Macro {
  double e, v, gamma, u, n, T;
  bool ok;
};

// Landau matching T^mu_nu u^nu = -e u^mu for the 1D moments
// m = (N0, Nz, T00, T0z, Tzz) (section Relativistic LB equation).  The 2x2
// eigenproblem in the t-z block gives e = (T00 - Tzz + D)/2 and
// v = 2 T0z / (T00 + Tzz + D) with D^2 = (T00+Tzz)^2 - 4 T0z^2; the density is
// n = -u_mu N^mu and the temperature T = e/(3n) (massless gas, e = 3P = 3nT).
__device__ inline Macro landau(const double m[5]) {
  Macro M;
  const double a = m[2] + m[4];
  const double disc = (a - 2.0 * m[3]) * (a + 2.0 * m[3]);
  const double D = sqrt(disc);
  M.e = 0.5 * (m[2] - m[4] + D);
  M.v = 2.0 * m[3] / (a + D);
  M.gamma = 1.0 / sqrt((1.0 - M.v) * (1.0 + M.v));
  M.u = M.gamma * M.v;
  M.n = M.gamma * (m[0] - M.v * m[1]);
  M.T = M.e / (3.0 * M.n);
  M.ok = (disc >= 0.0) && (M.e > 0.0) && (M.n > 0.0) && (fabs(M.v) < 1.0) && isfinite(M.T);
  return M;
}

// Coefficients of the truncated equilibrium at the radial nodes:
//   F_eq(p_i, xi) = sum_{k<=n_v} D[i][k] P_k(xi),
//   D[i][k] = (2k+1)/2 int_{-1}^{1} P_k(xi) G_i(xi) dxi,
//   G_i(xi) = n/(4 T T0^2) y^2 sum_{l<=n_p} L_l(p_i) (1 - (T/T0) y)^l,
//   y = 1/(gamma - xi u),
// which is the orthogonal projection of eq. feqtrunc (the Laplace transform of
// the Laguerre polynomials done in closed form, the xi integral by a symmetric
// auxiliary Gauss-Legendre rule whose node pairs +-xi_a share one pass).
// Raw sums of the projection over the auxiliary node pairs a = a_first,
// a_first + a_step, ... (all pairs: 0, 1), before the prefactor, for the
// radial nodes i = i_first, i_first + i_step, ... (rows of other nodes are 0).
// Each row's sum runs over the pairs in the same order for any node subset.
template <typename Real, int QPT, int NVT>
__device__ inline void feq_projection_sums(Real T, Real gamma, Real u, Real T0, int qp, int np, cptr<double> itab,
                                           cptr<Real> aux, int aux_pairs, int a_first, int a_step,
                                           Real D[QPT][NVT + 1], int i_first = 0, int i_step = 1) {
#pragma unroll
  for (int i = 0; i < QPT; ++i)
#pragma unroll
    for (int k = 0; k <= NVT; ++k) D[i][k] = Real(0);
  const Real r = T / T0;
  for (int a = a_first; a < aux_pairs; a += a_step) {
    cptr<Real> A = aux + a * kAuxStride;
    const Real xa = A[0];
    const Real yp = fast_div(Real(1), gamma - xa * u);
    const Real ym = fast_div(Real(1), gamma + xa * u);
    const Real qp_ = Real(1) - r * yp, qm = Real(1) - r * ym;
    const Real yp2 = yp * yp, ym2 = ym * ym;
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
      if (i < qp && i >= i_first && (i - i_first) % i_step == 0) {
        cptr<double> L = itab + i * kIStride + 4;
        Real sp = Real(L[np]), sm = Real(L[np]);
        for (int l = np - 1; l >= 0; --l) {
          sp = sp * qp_ + Real(L[l]);
          sm = sm * qm + Real(L[l]);
        }
        const Real gp = yp2 * sp, gm = ym2 * sm;
        const Real ev = gp + gm, od = gp - gm;
#pragma unroll
        for (int k = 0; k <= NVT; ++k) D[i][k] += A[1 + k] * ((k & 1) ? od : ev);
      }
    }
  }
}

// Prefactor n / (4 T T0^2) and truncation at n_v applied to the raw sums.
template <typename Real, int QPT, int NVT>
__device__ inline void feq_scale(Real n, Real T, Real T0, int nv, Real D[QPT][NVT + 1]) {
  const Real pref = n / (Real(4) * T * T0 * T0);
#pragma unroll
  for (int i = 0; i < QPT; ++i)
#pragma unroll
    for (int k = 0; k <= NVT; ++k) D[i][k] = (k <= nv) ? D[i][k] * pref : Real(0);
}

template <typename Real, int QPT, int NVT>
__device__ inline void feq_coefficients(Real n, Real T, Real gamma, Real u, Real T0, int qp, int np, int nv,
                                        cptr<double> itab, cptr<Real> aux,
                                        int aux_pairs, Real D[QPT][NVT + 1]) {
  feq_projection_sums<Real, QPT, NVT>(T, gamma, u, T0, qp, np, itab, aux, aux_pairs, 0, 1, D);
  feq_scale<Real, QPT, NVT>(n, T, T0, nv, D);
}

// Sign bit of a value as an integer test: on a wave-uniform value held in a
// scalar register this stays on the scalar unit (a float comparison would be a
// vector instruction).
__device__ inline bool sign_bit(float x) { return (__float_as_uint(x) >> 31) != 0u; }
__device__ inline bool sign_bit(double x) { return (static_cast<uint64_t>(__double_as_longlong(x)) >> 63) != 0u; }

// Fifth-order WENO (Jiang-Shu) value at the face between v3 and v4 from the
// upwind-ordered values v1..v5:  H = sum_r w_r q_r with the candidate values
// q_r of the three 3-point stencils and the weights w_r = a_r / sum(a),
// a_r = d_r / (eps + beta_r)^2, d = (1/10, 6/10, 3/10).
//
// Evaluated in the first differences a = v2-v1, b = v3-v2, c = v4-v3,
// d = v5-v4 of the stencil, with t = (b-a, c-b, d-c) its second differences:
//   4 beta_r = 13/3 t_r^2 + s_r^2,   s = (3b - a, b + c, d - 3c),
//   q_r = v3 + P_r / 6,              P = (3b + 2 t0, b + 2c, 3c - t2).
// Numerator and denominator are multiplied by prod_r (eps + beta_r)^2 (so one
// reciprocal remains; eps4 = 4 eps) and by 10/6:
//   H = v3 + (w0 P0/6 + w1 P1 + w2 P2/2) / (w0 + 6 w1 + 3 w2),
//   w0 = e1^2 e2^2, w1 = e0^2 e2^2, w2 = e0^2 e1^2,  e_r = 4 (eps + beta_r).
// The products are fourth powers of the e_r: when the denominator comes out
// zero, subnormal, infinite or NaN (in FP32: e_r below ~1e-10 on smooth data,
// e.g. eps <= 1e-12, or above ~1e9, e.g. eps >= 1e9 or huge jumps) the face
// is evaluated again with the weights in the form w_r = (min_s e_s / e_r)^2,
// which lie in (0, 1] with at least one equal to 1 and cannot under- or
// overflow (three exact divisions; weno5_scaled).  weno5 reports through `ok`
// whether its denominator was usable; callers that batch many faces recompute
// only the rare bad ones.
__device__ inline float weno_recip(float num, float den) { return num * __builtin_amdgcn_rcpf(den); }
__device__ inline double weno_recip(double num, double den) {
  double r = __builtin_amdgcn_rcp(den);
  r = fma(r, fma(-den, r, 1.0), r);
  return num * r;
}
// positive normal number (one class test)
template <typename Real>
__device__ inline bool weno_den_ok(Real den) {
  return __builtin_isfpclass(den, 0x100);
}

// Every multiply-add below is written as an explicit fused multiply-add (and
// contraction is off), so that each inlined copy of a face -- a lane's own
// face, the tile's extra face, the plane's x and z faces -- rounds the same
// way and results do not depend on the tiling.
template <typename Real>
struct WenoTerms {
  Real e0, e1, e2, R0, R1, R2;
};

template <typename Real>
__device__ inline WenoTerms<Real> weno5_terms(Real v1, Real v2, Real v3, Real v4, Real v5, Real eps4) {
#pragma clang fp contract(off)
  const Real a = v2 - v1, b = v3 - v2, c = v4 - v3, d = v5 - v4;
  const Real t0 = b - a, t1 = c - b, t2 = d - c;
  const Real s0 = fma(b, Real(3), -a), s1 = b + c, s2 = fma(c, Real(-3), d);
  const Real k = Real(13.0 / 3.0);
  WenoTerms<Real> w;
  w.e0 = fma(t0, k * t0, fma(s0, s0, eps4));
  w.e1 = fma(t1, k * t1, fma(s1, s1, eps4));
  w.e2 = fma(t2, k * t2, fma(s2, s2, eps4));
  w.R0 = fma(Real(0.5), b, Real(1.0 / 3.0) * t0);  // P0 / 6
  w.R1 = fma(Real(2), c, b);                        // P1
  w.R2 = fma(c, Real(1.5), -(Real(0.5) * t2));      // P2 / 2
  return w;
}

// The same face value with the scaled weights (any positive eps, any data).
template <typename Real>
__device__ inline Real weno5_scaled(Real v1, Real v2, Real v3, Real v4, Real v5, Real eps4) {
#pragma clang fp contract(off)
  const WenoTerms<Real> w = weno5_terms(v1, v2, v3, v4, v5, eps4);
  const Real m = fmin(w.e0, fmin(w.e1, w.e2));
  const Real q0 = m / w.e0, q1 = m / w.e1, q2 = m / w.e2;
  const Real x0 = q0 * q0, x1 = q1 * q1, x2 = q2 * q2;
  const Real num = fma(w.R2, x2, fma(w.R0, x0, w.R1 * x1));
  const Real den = fma(Real(3), x2, fma(x1, Real(6), x0));
  return v3 + num / den;
}

// Product form; ok is cleared when its denominator is not a positive normal
// number (the value returned is then to be replaced by weno5_scaled).
template <typename Real>
__device__ inline Real weno5(Real v1, Real v2, Real v3, Real v4, Real v5, Real eps4, bool& ok) {
#pragma clang fp contract(off)
  const WenoTerms<Real> w = weno5_terms(v1, v2, v3, v4, v5, eps4);
  const Real A = w.e0 * w.e0, B = w.e1 * w.e1, C = w.e2 * w.e2;
  const Real w0 = B * C, w1 = A * C, w2 = A * B;
  const Real num = fma(w.R2, w2, fma(w.R0, w0, w.R1 * w1));
  const Real den = fma(Real(3), w2, fma(w1, Real(6), w0));
  ok = ok && weno_den_ok(den);
  return v3 + weno_recip(num, den);
}

// One face, falling back to the scaled weights in place.
template <typename Real>
__device__ inline Real weno5(Real v1, Real v2, Real v3, Real v4, Real v5, Real eps4) {
  bool ok = true;
  const Real h = weno5(v1, v2, v3, v4, v5, eps4, ok);
  if (__builtin_expect(ok, 1)) return h;
  return weno5_scaled(v1, v2, v3, v4, v5, eps4);
}

// ---------------------------------------------------------------------------
// Reverse-mode derivatives (hand-written) of the per-cell maps above.
// ---------------------------------------------------------------------------

// Adjoint of the Landau matching: given the adjoints of (e, v, gamma, u, n, T)
// at the moments m, accumulates the adjoint of m into mb.
__device__ inline void landau_adjoint(const double m[5], const Macro& M, double eb, double vb, double gb, double ub,
                                      double nb, double Tb, double mb[5]) {
  const double a = m[2] + m[4], b = m[3];
  const double D = sqrt((a - 2.0 * b) * (a + 2.0 * b));
  // T = e/(3n)
  eb += Tb / (3.0 * M.n);
  nb -= Tb * M.T / M.n;
  // n = gamma (N0 - v Nz)
  gb += nb * (m[0] - M.v * m[1]);
  mb[0] += nb * M.gamma;
  mb[1] -= nb * M.gamma * M.v;
  vb -= nb * M.gamma * m[1];
  // u = gamma v
  gb += ub * M.v;
  vb += ub * M.gamma;
  // gamma = (1 - v^2)^(-1/2)
  vb += gb * M.gamma * M.gamma * M.gamma * M.v;
  // v = 2b/(a + D)
  const double iad = 1.0 / (a + D);
  double bb = vb * 2.0 * iad;
  double ab = -vb * M.v * iad;
  double Db = -vb * M.v * iad;
  // e = (T00 - Tzz + D)/2
  mb[2] += 0.5 * eb;
  mb[4] -= 0.5 * eb;
  Db += 0.5 * eb;
  // D = sqrt(a^2 - 4b^2)
  ab += Db * a / D;
  bb -= Db * 4.0 * b / D;
  mb[2] += ab;
  mb[4] += ab;
  mb[3] += bb;
}

// Adjoint of feq_coefficients (evaluated in FP64 on the same auxiliary rule):
// given Db[i][k] = dL/dD[i][k], accumulates dL/d(n, T, gamma, u).
// Reverse sweep of the projection over the auxiliary pairs a = a_first,
// a_first + a_step, ...: accumulates the adjoints of the prefactor (prefb),
// of r = T/T0 (rb), of gamma (gb) and of u (ub).
template <int QPT, int NVT>
__device__ inline void feq_adjoint_sums(double n, double T, double gamma, double u, double T0, int qp, int np, int nv,
                                        cptr<double> itab, cptr<double> aux, int aux_pairs, int a_first, int a_step,
                                        const double Db[QPT][NVT + 1], double& prefb, double& rb, double& gb,
                                        double& ub) {
  const double pref = n / (4.0 * T * T0 * T0);
  const double r = T / T0;
  for (int a = a_first; a < aux_pairs; a += a_step) {
    cptr<double> A = aux + a * kAuxStride;
    const double xa = A[0];
    const double yp = 1.0 / (gamma - xa * u), ym = 1.0 / (gamma + xa * u);
    const double qp_ = 1.0 - r * yp, qm = 1.0 - r * ym;
    const double yp2 = yp * yp, ym2 = ym * ym;
    double ypb = 0.0, ymb = 0.0;
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
      if (i < qp) {
        cptr<double> L = itab + i * kIStride + 4;
        // P(q) = sum_l L_l q^l and P'(q) by Horner
        double sp = L[np], dsp = 0.0, sm = L[np], dsm = 0.0;
        for (int l = np - 1; l >= 0; --l) {
          dsp = dsp * qp_ + sp;
          sp = sp * qp_ + L[l];
          dsm = dsm * qm + sm;
          sm = sm * qm + L[l];
        }
        const double gp = yp2 * sp, gm = ym2 * sm;
        double ev = 0.0, od = 0.0;
#pragma unroll
        for (int k = 0; k <= NVT; ++k) {
          if (k <= nv) {
            if (k & 1) od += Db[i][k] * A[1 + k];
            else ev += Db[i][k] * A[1 + k];
          }
        }
        prefb += ev * (gp + gm) + od * (gp - gm);
        const double gpb = pref * (ev + od), gmb = pref * (ev - od);
        ypb += gpb * 2.0 * yp * sp;
        ymb += gmb * 2.0 * ym * sm;
        const double qpb = gpb * yp2 * dsp, qmb = gmb * ym2 * dsm;
        rb -= qpb * yp + qmb * ym;
        ypb -= qpb * r;
        ymb -= qmb * r;
      }
    }
    gb -= ypb * yp2 + ymb * ym2;
    ub += ypb * xa * yp2 - ymb * xa * ym2;
  }
}

// Adjoint of the prefactor: prefb, rb -> n and T.
__device__ inline void feq_adjoint_finish(double n, double T, double T0, double prefb, double rb, double& nb,
                                          double& Tb) {
  const double pref = n / (4.0 * T * T0 * T0);
  nb += prefb * pref / n;
  Tb += -prefb * pref / T + rb / T0;
}

template <int QPT, int NVT>
__device__ inline void feq_coefficients_adjoint(double n, double T, double gamma, double u, double T0, int qp, int np,
                                                int nv, cptr<double> itab, cptr<double> aux, int aux_pairs,
                                                const double Db[QPT][NVT + 1], double& nb, double& Tb, double& gb,
                                                double& ub) {
  double prefb = 0.0, rb = 0.0;
  feq_adjoint_sums<QPT, NVT>(n, T, gamma, u, T0, qp, np, nv, itab, aux, aux_pairs, 0, 1, Db, prefb, rb, gb, ub);
  feq_adjoint_finish(n, T, T0, prefb, rb, nb, Tb);
}

// Gradient of the WENO5 value with respect to its five upwind-ordered inputs.
template <typename Real>
__device__ inline void weno5_grad(Real v1, Real v2, Real v3, Real v4, Real v5, Real eps, Real g[5]) {
  const Real q0 = (Real(2) * v1 - Real(7) * v2 + Real(11) * v3) * Real(1.0 / 6.0);
  const Real q1 = (-v2 + Real(5) * v3 + Real(2) * v4) * Real(1.0 / 6.0);
  const Real q2 = (Real(2) * v3 + Real(5) * v4 - v5) * Real(1.0 / 6.0);
  const Real t0 = v1 - Real(2) * v2 + v3, s0 = v1 - Real(4) * v2 + Real(3) * v3;
  const Real t1 = v2 - Real(2) * v3 + v4, s1 = v2 - v4;
  const Real t2 = v3 - Real(2) * v4 + v5, s2 = Real(3) * v3 - Real(4) * v4 + v5;
  const Real c13 = Real(13.0 / 12.0), c14 = Real(0.25);
  const Real e0 = eps + c13 * t0 * t0 + c14 * s0 * s0;
  const Real e1 = eps + c13 * t1 * t1 + c14 * s1 * s1;
  const Real e2 = eps + c13 * t2 * t2 + c14 * s2 * s2;
  // alpha_r = d_r / e_r^2 scaled by min_s e_s^2 (the weights are unchanged;
  // no under- or overflow for any positive eps)
  const Real em = fmin(e0, fmin(e1, e2));
  const Real r0 = em / e0, r1 = em / e1, r2 = em / e2;
  const Real a0 = Real(0.1) * r0 * r0, a1 = Real(0.6) * r1 * r1, a2 = Real(0.3) * r2 * r2;
  const Real sa = a0 + a1 + a2;
  const Real w0 = a0 / sa, w1 = a1 / sa, w2 = a2 / sa;
  const Real H = w0 * q0 + w1 * q1 + w2 * q2;
  // d alpha_r = -2 alpha_r/(eps+beta_r) d beta_r ; dH/d alpha_r = (q_r - H)/sum(alpha)
  const Real c0 = -Real(2) * w0 * (q0 - H) / e0;
  const Real c1 = -Real(2) * w1 * (q1 - H) / e1;
  const Real c2 = -Real(2) * w2 * (q2 - H) / e2;
  // d beta_r / d v = (13/6) t_r dt_r + (1/2) s_r ds_r
  const Real b0t = Real(13.0 / 6.0) * t0, b0s = Real(0.5) * s0;
  const Real b1t = Real(13.0 / 6.0) * t1, b1s = Real(0.5) * s1;
  const Real b2t = Real(13.0 / 6.0) * t2, b2s = Real(0.5) * s2;
  const Real r6 = Real(1.0 / 6.0);
  g[0] = w0 * Real(2) * r6 + c0 * (b0t + b0s);
  g[1] = w0 * Real(-7) * r6 + w1 * Real(-1) * r6 + c0 * (Real(-2) * b0t - Real(4) * b0s) + c1 * (b1t + b1s);
  g[2] = w0 * Real(11) * r6 + w1 * Real(5) * r6 + w2 * Real(2) * r6 + c0 * (b0t + Real(3) * b0s) +
         c1 * (Real(-2) * b1t) + c2 * (b2t + Real(3) * b2s);
  g[3] = w1 * Real(2) * r6 + w2 * Real(5) * r6 + c1 * (b1t - b1s) + c2 * (Real(-2) * b2t - Real(4) * b2s);
  g[4] = w2 * Real(-1) * r6 + c2 * (b2t + b2s);
}

// Monomial coefficients of the Legendre polynomials, P_k(c) = sum_m L[k][m] c^m,
// from the three-term recurrence (k+1) P_{k+1} = (2k+1) c P_k - k P_{k-1}.
struct LegendreMonomials {
  double c[kMaxNv + 1][kMaxNv + 1];
};
constexpr LegendreMonomials legendre_monomials() {
  LegendreMonomials L{};
  L.c[0][0] = 1.0;
  L.c[1][1] = 1.0;
  for (int k = 1; k < kMaxNv; ++k)
    for (int m = 0; m <= k + 1; ++m)
      L.c[k + 1][m] = ((2.0 * k + 1.0) * (m > 0 ? L.c[k][m - 1] : 0.0) - k * L.c[k - 1][m]) / (k + 1.0);
  return L;
}
constexpr LegendreMonomials kLegendre = legendre_monomials();

// The truncated series sum_k D[k] P_k(c) as a polynomial in c: coefficients
// a[m] = sum_k D[k] L[k][m] (once per cell and radial node), then Horner's
// rule per point.
template <typename Real, int NVT>
__device__ inline void series_monomials(const Real D[NVT + 1], Real a[NVT + 1]) {
#pragma unroll
  for (int m = 0; m <= NVT; ++m) {
    Real acc = Real(0);
#pragma unroll
    for (int k = m; k <= NVT; ++k)
      if (kLegendre.c[k][m] != 0.0) acc += D[k] * Real(kLegendre.c[k][m]);
    a[m] = acc;
  }
}
template <typename Real, int NVT>
__device__ inline Real horner(const Real a[NVT + 1], Real c) {
  Real f = a[NVT];
#pragma unroll
  for (int m = NVT - 1; m >= 0; --m) f = f * c + a[m];
  return f;
}

}  // namespace dev
}  // namespace rlb
