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
// sphere of a function of v . u_hat is its Legendre series in c) evaluated by
// the Legendre recurrence at each point -> WENO5 faces in x and z, relaxation,
// RK combination, store, and the nine moments of the output.
//
// Work decomposition: one lane per cell, workgroups of 64 x 4 cells (x
// contiguous in memory).  For every point the workgroup stages the cells of
// its tile and a 3-cell halo on each side (outflow clamps applied at load
// time) in LDS, the next point's values already in flight in registers; each
// lane computes the WENO value of its own left x face and lower z face (the
// tile's last faces by a few extra lanes), shares them through LDS and forms
// the update from its two x and two z faces.  Two barriers per point, double
// buffered.  Tiles are ordered z-fastest within an x column and handed to the
// XCDs in runs, so the z halos of a tile come from the same L2.
#include <hip/hip_runtime.h>

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

// Sum of the truncated series sum_k D[k] P_k(c), Legendre recurrence.
template <typename Real, int NVT>
__device__ inline Real legendre_series(const Real D[NVT + 1], Real c) {
  Real p0 = Real(1), p1 = c;
  Real acc = D[0] + D[1] * c;
#pragma unroll
  for (int k = 1; k < NVT; ++k) {
    const Real p2 = Real((2.0 * k + 1.0) / (k + 1.0)) * c * p1 - Real(double(k) / (k + 1.0)) * p0;
    acc += D[k + 1] * p2;
    p0 = p1;
    p1 = p2;
  }
  return acc;
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

// LDS tile of one point: rows z0-3 .. z0+6, columns x0-3 .. x0+66 (outflow
// clamps applied at load time), padded to kTileLd columns.
constexpr int kTileRows = kPlaneTileZ + 6, kTileCols = kPlaneTileX + 6, kTileLd = kTileCols + 2;
constexpr int kTileElems = kTileRows * kTileCols;
constexpr int kTileLoads = (kTileElems + 255) / 256;  // per lane

template <typename Real, int QPT, int NVT, bool HAS_FN>
__global__ __launch_bounds__(256) void plane_stage_kernel(PlaneArgs<Real> a) {
  __shared__ Real tile[2][kTileRows][kTileLd];
  __shared__ Real fxs[2][kPlaneTileZ][kPlaneTileX + 1];  // x faces: left face of column q
  __shared__ Real fzs[2][kPlaneTileZ + 1][kPlaneTileX];  // z faces: lower face of row r
  const cptr<PlaneDev> P = as_const(a.pl);
  const int nx = P->nx, nz = P->nz, ldx = P->ldx, qx = P->qx, qh = P->qh, qp = P->qp;
  const int64_t plane = P->plane;
  const int nxt = (nx + kPlaneTileX - 1) / kPlaneTileX, nzt = (nz + kPlaneTileZ - 1) / kPlaneTileZ;
  const cptr<Real> vtab = as_const(a.vtab);
  const cptr<double> itab = as_const(a.itab);
  const int stage = a.stage;
  const Real cn = stage == 1 ? Real(0) : (stage == 2 ? Real(0.75) : Real(1.0 / 3.0));
  const Real cs = stage == 1 ? Real(1) : (stage == 2 ? Real(0.25) : Real(2.0 / 3.0));
  const Real dt = Real(P->dt), cdt = cs * dt, dx_inv = Real(P->dx_inv), dz_inv = Real(P->dz_inv);
  const Real eps4 = Real(4.0 * P->weno_eps);
  const int t = threadIdx.x, tx = t % kPlaneTileX, tz = t / kPlaneTileX;
  for (int v = blockIdx.x; v < nxt * nzt; v += gridDim.x) {
    int xt, zt;
    plane_tile(v, nxt, nzt, xt, zt);
    const int x0 = xt * kPlaneTileX, z0 = zt * kPlaneTileZ;
    const int x = x0 + tx, z = z0 + tz;
    const bool valid = x < nx && z < nz;
    const int cell = min(z, nz - 1) * ldx + min(x, nx - 1);
    // this lane's share of the tile loads: plane offsets (clamped) and LDS slots
    uint32_t loff[kTileLoads];
    int lslot[kTileLoads];
#pragma unroll
    for (int q = 0; q < kTileLoads; ++q) {
      const int e = t + 256 * q;
      const int r = min(e, kTileElems - 1) / kTileCols, c = min(e, kTileElems - 1) % kTileCols;
      const int gz = min(max(z0 - 3 + r, 0), nz - 1), gx = min(max(x0 - 3 + c, 0), nx - 1);
      loff[q] = uint32_t(gz * ldx + gx);
      lslot[q] = e < kTileElems ? r * kTileLd + c : -1;
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
    double mom[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int Q = qp * qx * qh;
    // first point's tile values
    Real pre[kTileLoads];
#pragma unroll
    for (int q = 0; q < kTileLoads; ++q) pre[q] = a.fin[loff[q]];
    int buf = 0;
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
      PlaneSums<Real> acc;
      for (int j = 0; j < qx; ++j) {
        Real p6[6] = {Real(0), Real(0), Real(0), Real(0), Real(0), Real(0)};
        for (int k = 0; k < qh; ++k) {
          const int s = (i * qx + j) * qh + k;
          // 1. stage this point's tile, 2. prefetch the next point's values
#pragma unroll
          for (int q = 0; q < kTileLoads; ++q)
            if (lslot[q] >= 0) (&tile[buf][0][0])[lslot[q]] = pre[q];
          if (s + 1 < Q) {
            const Real* nrow = a.fin + int64_t(s + 1) * plane;
#pragma unroll
            for (int q = 0; q < kTileLoads; ++q) pre[q] = nrow[loff[q]];
          }
          const Real fnv = HAS_FN ? a.fn[int64_t(s) * plane + cell] : Real(0);
          __syncthreads();
          // 3. this lane's left x face and lower z face (plus the tile's last
          //    face of each row / column), upwinded by the point's velocity
          const cptr<Real> V = vtab + (j * qh + k) * kVStride;
          const Real vx = V[0], vz = V[1];
          {
            const Real* rw = &tile[buf][tz + 3][tx];  // columns tx .. tx+6 of this row
            fxs[buf][tz][tx] = vx >= Real(0) ? weno5(rw[0], rw[1], rw[2], rw[3], rw[4], eps4)
                                             : weno5(rw[5], rw[4], rw[3], rw[2], rw[1], eps4);
            const Real* cl = &tile[buf][tz][tx + 3];  // rows tz .. tz+6 of this column
            fzs[buf][tz][tx] = vz >= Real(0)
                                   ? weno5(cl[0], cl[kTileLd], cl[2 * kTileLd], cl[3 * kTileLd], cl[4 * kTileLd], eps4)
                                   : weno5(cl[5 * kTileLd], cl[4 * kTileLd], cl[3 * kTileLd], cl[2 * kTileLd],
                                           cl[kTileLd], eps4);
            if (tz == kPlaneTileZ - 1) {  // upper face of the last row
              const Real* cu = cl + kTileLd;
              fzs[buf][kPlaneTileZ][tx] =
                  vz >= Real(0) ? weno5(cu[0], cu[kTileLd], cu[2 * kTileLd], cu[3 * kTileLd], cu[4 * kTileLd], eps4)
                                : weno5(cu[5 * kTileLd], cu[4 * kTileLd], cu[3 * kTileLd], cu[2 * kTileLd],
                                        cu[kTileLd], eps4);
            }
            if (t < kPlaneTileZ) {  // right face of the last column of row t
              const Real* re = &tile[buf][t + 3][kPlaneTileX];
              fxs[buf][t][kPlaneTileX] = vx >= Real(0) ? weno5(re[0], re[1], re[2], re[3], re[4], eps4)
                                                       : weno5(re[5], re[4], re[3], re[2], re[1], eps4);
            }
          }
          __syncthreads();
          // 4. update
          const Real fr = tile[buf][tz + 3][tx + 3];
          const Real hxl = fxs[buf][tz][tx], hxr = fxs[buf][tz][tx + 1];
          const Real hzl = fzs[buf][tz][tx], hzr = fzs[buf][tz + 1][tx];
          const Real feq = legendre_series<Real, NVT>(Dc, vx * hx + vz * hz);
          const Real adv = (hxr - hxl) * (-vx * dx_inv) + (hzr - hzl) * (-vz * dz_inv);
          const Real rate = g0 - vx * gx - vz * gz;
          const Real L = adv - rate * (fr - feq);
          const Real out = HAS_FN ? cdt * L + (cs * fr + cn * fnv) : fr + dt * L;
          if (valid) a.fout[int64_t(s) * plane + cell] = out;
          add_point(p6, V, out);
          buf ^= 1;
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) acc.S[q].add(p6[q]);
      }
      double S[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) S[q] = acc.S[q].value();
      add_node9(mom, itab + i * kIStride, S);
    }
    if (valid) {
#pragma unroll
      for (int c = 0; c < 9; ++c) a.rec_out[c * plane + cell] = mom[c];
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
        PlaneSums<Real> acc;
        for (int j = 0; j < qx; ++j) {
          Real p6[6] = {Real(0), Real(0), Real(0), Real(0), Real(0), Real(0)};
          for (int k = 0; k < qh; ++k) {
            const int64_t s = int64_t((i * qx + j) * qh + k);
            const cptr<Real> V = vtab + (j * qh + k) * kVStride;
            const Real f = legendre_series<Real, NVT>(D[i], V[0] * hx + V[1] * hz);
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
    hipLaunchKernelGGL((plane_stage_kernel<Real, QPT, NVT, false>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((plane_stage_kernel<Real, QPT, NVT, true>), dim3(grid), dim3(256), 0, s, a);
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
