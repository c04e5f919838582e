// Multi-dimensional model on an (x, z) plane: HIP kernels for gfx950.
//
// The Boltzmann equation with the particle velocity resolved in the plane
// (eq. Boltz_gen for data that do not depend on y):
//   dF/dt = -v_x dF/dx - v_z dF/dz - ((u^0 - v_x u^x - v_z u^z)/tau) (F - F^eq),
// v = (sin(theta) cos(phi), sin(theta) sin(phi), cos(theta)), on the full
// product quadrature of the section on the discretization of momentum space
// (Gauss-Laguerre in p, Gauss-Legendre in cos(theta), the trapezoid rule of
// eq. azimuthInt in phi with the mirrored nodes phi, -phi evolved once).
//
// Per cell and SSP-RK3 stage: the nine moment records of the stage input ->
// the Landau frame in FP64 (the timelike eigenvector of T^mu_nu, by Newton's
// method on the two velocity components from the 1D closed form along T^{0i})
// -> the truncated equilibrium, which depends on the direction only through
// c = v . u_hat: the coefficients of the 1D projection at the speed |u|
// (eq. feqtrunc; the projection onto polynomials of degree <= N_v on the
// sphere of a function of v . u_hat is its Legendre series in c), turned into
// a polynomial in c once per cell and radial node and evaluated by Horner's
// rule at each point -> WENO5 faces in x and z, relaxation, RK combination,
// store, and the nine moments of the output.
//
// Work decomposition: one lane per cell, stage workgroups of 64 x 8 cells
// (x contiguous in memory, one wave per row).  For every point the workgroup
// stages the cells of its tile and a 3-cell halo on each side (outflow clamps
// applied at load time) in LDS, the next point's values already in flight in
// registers; each
// lane computes the WENO value of its own left x face and lower z face (the
// tile's last row and column of faces by a wave that rotates with the
// workgroup and the point), shares them through LDS and forms the update from
// its two x and two z faces.  Two barriers per point, double buffered, with
// the point loop unrolled by two so that every LDS access of the common path
// is one per-lane offset plus an immediate; global accesses are buffer
// accesses with a scalar base per point and 32-bit per-lane offsets.  Tiles
// are ordered z-fastest within an x column and handed to the XCDs in runs, so
// the z halos of a tile come from the same L2.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "rlb_device.h"
#include "rlb_internal.h"

namespace rlb {
namespace {

using namespace dev;

struct Macro2 {
  double e, vx, vz, gamma, ux, uz, n, T;
  bool ok;
};

// Landau frame of the nine moments m = (N0, Nx, Nz, T00, T0x, T0z, Txx, Txz,
// Tzz): T^mu_nu u^nu = -e u^mu with u = gamma (1, v_x, v_z).  Its components
// give e = T00 - T0x v_x - T0z v_z and the residual
//   R_i = T^{0i} - T^{ij} v_j - e v_i = 0   (i = x, z),
// solved by Newton's method.  The start is the exact root of the 1D problem
// along the direction n of T^{0i} (T00, |T^{0.}|, n T n), which is exact when T
// is a perfect fluid; convergence is quadratic from there.
__device__ inline Macro2 landau2(const double m[9]) {
  const double N0 = m[0], Nx = m[1], Nz = m[2], T00 = m[3], T0x = m[4], T0z = m[5], Txx = m[6], Txz = m[7],
               Tzz = m[8];
  double vx = 0.0, vz = 0.0;
  const double s = sqrt(T0x * T0x + T0z * T0z);
  if (s > 0.0) {
    const double hx = T0x / s, hz = T0z / s;
    const double Tnn = hx * hx * Txx + 2.0 * hx * hz * Txz + hz * hz * Tzz;
    const double a = T00 + Tnn;
    const double D = sqrt(fmax((a - 2.0 * s) * (a + 2.0 * s), 0.0));
    const double v = 2.0 * s / (a + D);
    vx = v * hx;
    vz = v * hz;
  }
  for (int it = 0; it < 8; ++it) {
    const double e = T00 - T0x * vx - T0z * vz;
    const double rx = T0x - Txx * vx - Txz * vz - e * vx;
    const double rz = T0z - Txz * vx - Tzz * vz - e * vz;
    const double jxx = T0x * vx - Txx - e, jxz = T0z * vx - Txz;
    const double jzx = T0x * vz - Txz, jzz = T0z * vz - Tzz - e;
    const double det = jxx * jzz - jxz * jzx;
    const double dvx = (jxz * rz - jzz * rx) / det, dvz = (jzx * rx - jxx * rz) / det;
    vx += dvx;
    vz += dvz;
    if (fabs(dvx) + fabs(dvz) <= 1e-14) break;
  }
  Macro2 M;
  const double v2 = vx * vx + vz * vz;
  M.e = T00 - T0x * vx - T0z * vz;
  M.vx = vx;
  M.vz = vz;
  M.gamma = 1.0 / sqrt(1.0 - v2);
  M.ux = M.gamma * vx;
  M.uz = M.gamma * vz;
  M.n = M.gamma * (N0 - vx * Nx - vz * Nz);
  M.T = M.e / (3.0 * M.n);
  M.ok = (M.e > 0.0) && (M.n > 0.0) && (v2 < 1.0) && isfinite(M.T);
  return M;
}

// Moment sums of one radial node, in the order every kernel uses: plain
// fused sums over the azimuthal nodes of one polar node, then (Kahan in FP32)
// across polar nodes.
template <typename Real>
struct PlaneSums {
  Acc<Real> S[6];
};
template <typename Real>
__device__ inline void add_point(Real p6[6], cptr<Real> V, Real f) {
#pragma unroll
  for (int q = 0; q < 6; ++q) p6[q] = fma(V[2 + q], f, p6[q]);
}
// Adds one radial node's sums to the nine records (N from T0^3 w_p p, T from
// T0^4 w_p p^2).
template <typename Ptr>
__device__ inline void add_node9(double m[9], Ptr I, const double S[6]) {
  m[0] = fma(I[2], S[0], m[0]);
  m[1] = fma(I[2], S[1], m[1]);
  m[2] = fma(I[2], S[2], m[2]);
#pragma unroll
  for (int q = 0; q < 6; ++q) m[3 + q] = fma(I[3], S[q], m[3 + q]);
}

// Tile of a virtual workgroup index: z-fastest within x columns, XCD runs.
__device__ inline void plane_tile(int v, int nxt, int nzt, int& xt, int& zt) {
  const int item = xcd_item(v, nxt * nzt);
  xt = item / nzt;
  zt = item % nzt;
}

// LDS of one point (two buffers, alternating between points): the tile with a
// 3-cell halo (rows z0-3 .. z0+kTZ+2, columns x0-3 .. x0+66, outflow clamps
// applied at load time), then the x faces (left face of columns 0 .. 64 of
// each row) and the z faces (lower face of rows 0 .. kTZ of each column).
// All three share the row stride kLd, so that every access of the common path
// is one per-lane offset plus an immediate.
constexpr int kTZ = 8, kThreads = kPlaneTileX * kTZ;  // stage tile rows, threads
constexpr int kLd = kPlaneTileX + 8;
constexpr int kTileRows = kTZ + 6, kTileCols = kPlaneTileX + 6;
constexpr int kTileElems = kTileRows * kTileCols;
constexpr int kTileLoads = (kTileElems + kThreads - 1) / kThreads;  // per lane
constexpr int kFxOff = kTileRows * kLd, kFzOff = kFxOff + kTZ * kLd;
constexpr int kBufElems = kFzOff + (kTZ + 1) * kLd;
static_assert(kLd >= kTileCols && kLd >= kPlaneTileX + 1, "row stride");
static_assert(kPlaneTileX == 64, "one wave per tile row");

template <int B>
using BufTag = std::integral_constant<int, B>;

// WENO5 value at a face from the six cells p[0], p[ST], .. p[5 ST] around it,
// upwinded by the sign of the velocity component (cells 0 .. 4 for up,
// 5 .. 1 otherwise).  `up` is wave-uniform; the empty asm statement keeps the
// two orientations as separate branches, each reading LDS at immediate
// offsets, instead of one merged body that computes its LDS addresses.
// The product form of the weights only: the plane's epsilon is validated to
// the range in which it neither under- nor overflows for |F| up to ~1e3
// (FP32; see weno_eps_in_range).
template <typename Real, int ST>
__device__ inline Real face(const Real* p, bool up, Real eps4) {
  bool unused = true;
  if (up) return weno5(p[0], p[ST], p[2 * ST], p[3 * ST], p[4 * ST], eps4, unused);
  Real h = weno5(p[5 * ST], p[4 * ST], p[3 * ST], p[2 * ST], p[ST], eps4, unused);
  asm volatile("" : "+v"(h));
  return h;
}


// Occupancy: 6 waves per SIMD (three workgroups) for FP32 and 4 for FP64
// with Q_p <= 4, 4 for FP32 in the generic Q_p <= 8 group (the per-cell
// coefficients of the other radial nodes and a few tile constants spill,
// outside the point loop; measured 0.99 against 1.41 ms per step with the
// compiler's choice on a 512^2 plane with Q_p = 5); the FP64 generic group is
// left to the compiler (3 waves measured 29 % slower).
template <typename Real, int QPT>
constexpr int plane_waves_per_eu() {
  return QPT > 4 ? (sizeof(Real) == 4 ? 4 : 1) : (sizeof(Real) == 4 ? 6 : 4);
}

template <typename Real, int QPT, int NVT, bool HAS_FN>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(plane_waves_per_eu<Real, QPT>())))
void plane_stage_kernel(PlaneArgs<Real> a) {
  __shared__ Real lds[2 * kBufElems];
  // FP64: the nine record sums of each lane live in LDS (registers are the
  // scarce resource at four waves per SIMD); FP32 keeps them in registers
  constexpr bool kMomLds = sizeof(Real) == 8;
  __shared__ double mom_lds[kMomLds ? 9 : 1][kThreads];
  const cptr<PlaneDev> P = as_const(a.pl);
  const int nx = P->nx, nz = P->nz, ldx = P->ldx, qx = P->qx, qh = P->qh, qp = P->qp;
  const int64_t plane = P->plane;
  const uint32_t plane_bytes = uint32_t(plane * int64_t(sizeof(Real)));
  const int nxt = (nx + kPlaneTileX - 1) / kPlaneTileX, nzt = (nz + kTZ - 1) / kTZ;
  const cptr<Real> vtab = as_const(a.vtab);
  const cptr<double> itab = as_const(a.itab);
  const int stage = a.stage;
  const Real cs = stage == 1 ? Real(1) : (stage == 2 ? Real(0.25) : Real(2.0 / 3.0));
  const Real dt = Real(P->dt);
  const Real eps4 = Real(4.0 * P->weno_eps);
  const int t = threadIdx.x, tx = t % kPlaneTileX, tz = t / kPlaneTileX;
  const int lane_off = tz * kLd + tx;
  const int wave = __builtin_amdgcn_readfirstlane(tz);
  for (int v = blockIdx.x; v < nxt * nzt; v += gridDim.x) {
    int xt, zt;
    plane_tile(v, nxt, nzt, xt, zt);
    const int x0 = xt * kPlaneTileX, z0 = zt * kTZ;
    const int x = x0 + tx, z = z0 + tz;
    const bool valid = x < nx && z < nz;
    const int cell = min(z, nz - 1) * ldx + min(x, nx - 1);
    const uint32_t cell_b = uint32_t(cell) * uint32_t(sizeof(Real));
    // this lane's share of the tile loads: byte offsets in a point's plane
    // (clamped) and LDS slots
    uint32_t loff[kTileLoads];
    int lslot[kTileLoads];
#pragma unroll
    for (int q = 0; q < kTileLoads; ++q) {
      const int e = t + kThreads * q;
      const int r = min(e, kTileElems - 1) / kTileCols, c = min(e, kTileElems - 1) % kTileCols;
      const int gz = min(max(z0 - 3 + r, 0), nz - 1), gx = min(max(x0 - 3 + c, 0), nx - 1);
      loff[q] = uint32_t(gz * ldx + gx) * uint32_t(sizeof(Real));
      lslot[q] = e < kTileElems ? r * kLd + c : -1;
    }
    // Landau frame of the stage input (FP64)
    double m[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) m[c] = a.rec_in[c * plane + cell];
    const Macro2 M = landau2(m);
    if (valid && !M.ok) atomicOr(a.flag, kFlagNonphysical);
    if (valid && M.vx * M.vx + M.vz * M.vz > 0.95 * 0.95) atomicOr(a.flag, kFlagFastFlow);
    const double ua = sqrt(M.ux * M.ux + M.uz * M.uz);
    const Real hx = Real(ua > 0.0 ? M.ux / ua : 0.0), hz = Real(ua > 0.0 ? M.uz / ua : 1.0);
    Real D[QPT][NVT + 1];
    feq_coefficients<Real, QPT, NVT>(Real(M.n), Real(M.T), Real(M.gamma), Real(ua), Real(P->T0), qp, P->np, P->nv,
                                     itab, as_const(a.aux), a.aux_pairs, D);
    const Real g0 = Real(M.gamma * P->tau_inv), gx = Real(M.ux * P->tau_inv), gz = Real(M.uz * P->tau_inv);
    double mom[kMomLds ? 1 : 9];
    if constexpr (kMomLds) {
#pragma unroll
      for (int c = 0; c < 9; ++c) mom_lds[c][t] = 0.0;
    } else {
#pragma unroll
      for (int c = 0; c < 9; ++c) mom[c] = 0.0;
    }
    const int Q = qp * qx * qh;
    // first point's tile values
    Real pre[kTileLoads];
    {
      const Rsrc r0 = make_rsrc(a.fin, plane_bytes);
#pragma unroll
      for (int q = 0; q < kTileLoads; ++q) pre[q] = BufIO<Real>::template load<0>(r0, loff[q], 0);
    }
    int s = 0;
#pragma unroll 1
    for (int i = 0; i < qp; ++i) {
      Real Dc[NVT + 1];
#pragma unroll
      for (int k = 0; k <= NVT; ++k) {
        Real d = D[0][k];
#pragma unroll
        for (int ii = 1; ii < QPT; ++ii) d = i == ii ? D[ii][k] : d;
        Dc[k] = d;
      }
      Real Am[NVT + 1];
      series_monomials<Real, NVT>(Dc, Am);
      PlaneSums<Real> acc;
#pragma unroll 1
      for (int j = 0; j < qx; ++j) {
        Real p6[6] = {Real(0), Real(0), Real(0), Real(0), Real(0), Real(0)};
        // One point s = (i qx + j) qh + k with its values staged in buffer B.
        auto point = [&](auto tag, int k) {
          constexpr int B = decltype(tag)::value * kBufElems;
          Real* const L = lds + B;
          // 1. stage this point's tile, 2. prefetch the next point's values
#pragma unroll
          for (int q = 0; q < kTileLoads; ++q)
            if (lslot[q] >= 0) L[lslot[q]] = pre[q];
          if (s + 1 < Q) {
            const Rsrc rn = make_rsrc(a.fin + int64_t(s + 1) * plane, plane_bytes);
#pragma unroll
            for (int q = 0; q < kTileLoads; ++q) pre[q] = BufIO<Real>::template load<0>(rn, loff[q], 0);
          }
          const Real fnv =
              HAS_FN ? BufIO<Real>::template load<2>(make_rsrc(a.fn + int64_t(s) * plane, plane_bytes), cell_b, 0)
                     : Real(0);
          __syncthreads();
          // 3. this lane's left x face and lower z face, upwinded by the
          //    point's velocity; the tile's upper z faces and right x faces go
          //    to a wave that rotates with the workgroup and the point, so
          //    that every SIMD carries the same share of them
          const cptr<Real> V = vtab + (j * qh + k) * kVStride;
          const Real vx = V[0], vz = V[1];
          // upwind directions from the sign bits, on the scalar unit (no node
          // component is a negative zero)
          const bool ux = !sign_bit(vx), uz = !sign_bit(vz);
          const Real* T = L + lane_off;
          L[kFxOff + lane_off] = face<Real, 1>(T + 3 * kLd, ux, eps4);
          L[kFzOff + lane_off] = face<Real, kLd>(T + 3, uz, eps4);
          const int wz = (int(blockIdx.x) + s) & (kTZ - 1);
          if (wave == wz)
            L[kFzOff + kTZ * kLd + tx] = face<Real, kLd>(L + kTZ * kLd + 3 + tx, uz, eps4);
          if (wave == (wz ^ (kTZ / 2)) && tx < kTZ)
            L[kFxOff + tx * kLd + kPlaneTileX] = face<Real, 1>(L + (tx + 3) * kLd + kPlaneTileX, ux, eps4);
          __syncthreads();
          // 4. update
          const Real fr = T[3 * kLd + 3];
          const Real hxl = L[kFxOff + lane_off], hxr = L[kFxOff + lane_off + 1];
          const Real hzl = L[kFzOff + lane_off], hzr = L[kFzOff + lane_off + kLd];
          const Real feq = horner<Real, NVT>(Am, vx * hx + vz * hz);
          const Real adv = (hxr - hxl) * V[8] + (hzr - hzl) * V[9];
          const Real rate = g0 - vx * gx - vz * gz;
          const Real Lr = adv - rate * (fr - feq);
          // f^n + cs ((f_in - f^n) + dt L): one rounding at the scale of F
          const Real out = HAS_FN ? fnv + cs * ((fr - fnv) + dt * Lr) : fr + dt * Lr;
          if (valid)
            BufIO<Real>::template store<2>(out, make_rsrc(a.fout + int64_t(s) * plane, plane_bytes), cell_b, 0);
          add_point(p6, V, out);
          ++s;
        };
        int k = 0;
        for (; k + 1 < qh; k += 2) {
          point(BufTag<0>{}, k);
          point(BufTag<1>{}, k + 1);
        }
        if (k < qh) {
          point(BufTag<0>{}, k);
          __syncthreads();  // the next point reuses buffer 0
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) acc.S[q].add(p6[q]);
      }
      double S[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) S[q] = acc.S[q].value();
      if constexpr (kMomLds) {
        double mm[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) mm[c] = mom_lds[c][t];
        add_node9(mm, itab + i * kIStride, S);
#pragma unroll
        for (int c = 0; c < 9; ++c) mom_lds[c][t] = mm[c];
      } else {
        add_node9(mom, itab + i * kIStride, S);
      }
    }
    if (valid) {
#pragma unroll
      for (int c = 0; c < 9; ++c) a.rec_out[c * plane + cell] = kMomLds ? mom_lds[c][t] : mom[c];
    }
    __syncthreads();  // the next tile reuses the LDS buffers
  }
}

// Initial state: the truncated equilibrium of each cell's (P, n, u^x, u^z),
// and its records (the same sums as the stage epilogue).
template <typename Real, int QPT, int NVT>
__global__ __launch_bounds__(256) void plane_init_kernel(PlaneArgs<Real> a) {
  const cptr<PlaneDev> P = as_const(a.pl);
  const int nx = P->nx, nz = P->nz, ldx = P->ldx, qx = P->qx, qh = P->qh, qp = P->qp;
  const int64_t plane = P->plane;
  const int nxt = (nx + kPlaneTileX - 1) / kPlaneTileX, nzt = (nz + kPlaneTileZ - 1) / kPlaneTileZ;
  const cptr<Real> vtab = as_const(a.vtab);
  const cptr<double> itab = as_const(a.itab);
  for (int v = blockIdx.x; v < nxt * nzt; v += gridDim.x) {
    int xt, zt;
    plane_tile(v, nxt, nzt, xt, zt);
    const int x = xt * kPlaneTileX + int(threadIdx.x) % kPlaneTileX;
    const int z = zt * kPlaneTileZ + int(threadIdx.x) / kPlaneTileX;
    if (x >= nx || z >= nz) continue;
    const int cell = z * ldx + x;
    const int64_t dense = int64_t(z) * nx + x, cells = int64_t(nx) * nz;
    const double Pr = a.init[dense], n = a.init[cells + dense], ux = a.init[2 * cells + dense],
                 uz = a.init[3 * cells + dense];
    const double ua = sqrt(ux * ux + uz * uz), gamma = sqrt(1.0 + ua * ua);
    const Real hx = Real(ua > 0.0 ? ux / ua : 0.0), hz = Real(ua > 0.0 ? uz / ua : 1.0);
    Real D[QPT][NVT + 1];
    feq_coefficients<Real, QPT, NVT>(Real(n), Real(Pr / n), Real(gamma), Real(ua), Real(P->T0), qp, P->np, P->nv,
                                     itab, as_const(a.aux), a.aux_pairs, D);
    double mom[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
      if (i < qp) {
        Real Am[NVT + 1];
        series_monomials<Real, NVT>(D[i], Am);
        PlaneSums<Real> acc;
        for (int j = 0; j < qx; ++j) {
          Real p6[6] = {Real(0), Real(0), Real(0), Real(0), Real(0), Real(0)};
          for (int k = 0; k < qh; ++k) {
            const int64_t s = int64_t((i * qx + j) * qh + k);
            const cptr<Real> V = vtab + (j * qh + k) * kVStride;
            const Real f = horner<Real, NVT>(Am, V[0] * hx + V[1] * hz);
            a.fout[s * plane + cell] = f;
            add_point(p6, V, f);
          }
#pragma unroll
          for (int q = 0; q < 6; ++q) acc.S[q].add(p6[q]);
        }
        double S[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) S[q] = acc.S[q].value();
        add_node9(mom, itab + i * kIStride, S);
      }
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) a.rec_out[c * plane + cell] = mom[c];
  }
}

// Records of a stored state (after a state load).
template <typename Real>
__global__ __launch_bounds__(256) void plane_moments_kernel(PlaneArgs<Real> a) {
  const cptr<PlaneDev> P = as_const(a.pl);
  const int nx = P->nx, nz = P->nz, ldx = P->ldx, qx = P->qx, qh = P->qh, qp = P->qp;
  const int64_t plane = P->plane;
  const int nxt = (nx + kPlaneTileX - 1) / kPlaneTileX, nzt = (nz + kPlaneTileZ - 1) / kPlaneTileZ;
  const cptr<Real> vtab = as_const(a.vtab);
  const cptr<double> itab = as_const(a.itab);
  for (int v = blockIdx.x; v < nxt * nzt; v += gridDim.x) {
    int xt, zt;
    plane_tile(v, nxt, nzt, xt, zt);
    const int x = xt * kPlaneTileX + int(threadIdx.x) % kPlaneTileX;
    const int z = zt * kPlaneTileZ + int(threadIdx.x) / kPlaneTileX;
    if (x >= nx || z >= nz) continue;
    const int cell = z * ldx + x;
    double mom[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < qp; ++i) {
      PlaneSums<Real> acc;
      for (int j = 0; j < qx; ++j) {
        Real p6[6] = {Real(0), Real(0), Real(0), Real(0), Real(0), Real(0)};
        for (int k = 0; k < qh; ++k) {
          const int64_t s = int64_t((i * qx + j) * qh + k);
          add_point(p6, vtab + (j * qh + k) * kVStride, a.fin[s * plane + cell]);
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) acc.S[q].add(p6[q]);
      }
      double S[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) S[q] = acc.S[q].value();
      add_node9(mom, itab + i * kIStride, S);
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) a.rec_out[c * plane + cell] = mom[c];
  }
}

// Fields [14][nz][nx] from the records: the nine moments, e, n, v_x, v_z, T.
__global__ __launch_bounds__(256) void plane_fields_kernel(const PlaneDev* pl, const double* rec, double* out,
                                                           unsigned* flag) {
  const cptr<PlaneDev> P = as_const(pl);
  const int nx = P->nx, nz = P->nz, ldx = P->ldx;
  const int64_t plane = P->plane, cells = int64_t(nx) * nz;
  const int64_t dense = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (dense >= cells) return;
  const int z = int(dense / nx), x = int(dense % nx);
  const int cell = z * ldx + x;
  double m[9];
  for (int c = 0; c < 9; ++c) m[c] = rec[c * plane + cell];
  const Macro2 M = landau2(m);
  if (!M.ok) atomicOr(flag, kFlagNonphysical);
  for (int c = 0; c < 9; ++c) out[c * cells + dense] = m[c];
  out[9 * cells + dense] = M.e;
  out[10 * cells + dense] = M.n;
  out[11 * cells + dense] = M.vx;
  out[12 * cells + dense] = M.vz;
  out[13 * cells + dense] = M.T;
}

template <typename Real, int QPT, int NVT>
hipError_t stage_t(const void* args, int grid, hipStream_t s) {
  const PlaneArgs<Real>& a = *static_cast<const PlaneArgs<Real>*>(args);
  if (a.stage == 1)
    hipLaunchKernelGGL((plane_stage_kernel<Real, QPT, NVT, false>), dim3(grid), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((plane_stage_kernel<Real, QPT, NVT, true>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <typename Real>
hipError_t stage_real(int qpt, int nvt, const void* args, int grid, hipStream_t s) {
  if (qpt == 3 && nvt == 5) return stage_t<Real, 3, 5>(args, grid, s);
  if (qpt == 4 && nvt == 5) return stage_t<Real, 4, 5>(args, grid, s);
  if (qpt == 8 && nvt == 7) return stage_t<Real, 8, 7>(args, grid, s);
  return hipErrorInvalidValue;
}

template <typename Real>
hipError_t init_real(int qpt, int nvt, const void* args, int grid, hipStream_t s) {
  const PlaneArgs<Real>& a = *static_cast<const PlaneArgs<Real>*>(args);
  if (qpt == 3 && nvt == 5)
    hipLaunchKernelGGL((plane_init_kernel<Real, 3, 5>), dim3(grid), dim3(256), 0, s, a);
  else if (qpt == 4 && nvt == 5)
    hipLaunchKernelGGL((plane_init_kernel<Real, 4, 5>), dim3(grid), dim3(256), 0, s, a);
  else if (qpt == 8 && nvt == 7)
    hipLaunchKernelGGL((plane_init_kernel<Real, 8, 7>), dim3(grid), dim3(256), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

int plane_stage_grid(int nx, int nz) {
  return ((nx + kPlaneTileX - 1) / kPlaneTileX) * ((nz + kTZ - 1) / kTZ);
}

hipError_t launch_plane_stage(int prec_fp32, int qpt, int nvt, const void* args, int grid, hipStream_t stream) {
  return prec_fp32 ? stage_real<float>(qpt, nvt, args, grid, stream) : stage_real<double>(qpt, nvt, args, grid, stream);
}

hipError_t launch_plane_init(int prec_fp32, int qpt, int nvt, const void* args, int grid, hipStream_t stream) {
  return prec_fp32 ? init_real<float>(qpt, nvt, args, grid, stream) : init_real<double>(qpt, nvt, args, grid, stream);
}

hipError_t launch_plane_moments(int prec_fp32, const void* args, int grid, hipStream_t stream) {
  if (prec_fp32)
    hipLaunchKernelGGL(plane_moments_kernel<float>, dim3(grid), dim3(256), 0, stream,
                       *static_cast<const PlaneArgs<float>*>(args));
  else
    hipLaunchKernelGGL(plane_moments_kernel<double>, dim3(grid), dim3(256), 0, stream,
                       *static_cast<const PlaneArgs<double>*>(args));
  return hipGetLastError();
}

hipError_t launch_plane_fields(const PlaneDev* pl, int nx, int nz, const double* rec, double* out, unsigned* flag,
                               hipStream_t stream) {
  const int64_t cells = int64_t(nx) * nz;
  hipLaunchKernelGGL(plane_fields_kernel, dim3(unsigned((cells + 255) / 256)), dim3(256), 0, stream, pl, rec, out,
                     flag);
  return hipGetLastError();
}

}  // namespace rlb
