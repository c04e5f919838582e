// Multi-dimensional model on an (x, y, z) box: HIP kernels for gfx950.
//
// The Boltzmann equation with the particle velocity resolved in all three
// directions (eq. Boltz_gen):
//   dF/dt = -v_x dF/dx - v_y dF/dy - v_z dF/dz
//           - ((u^0 - v_x u^x - v_y u^y - v_z u^z)/tau) (F - F^eq),
// v = (sin(theta) cos(phi), sin(theta) sin(phi), cos(theta)), on the full
// product quadrature of the section on the discretization of momentum space:
// Gauss-Laguerre in p, Gauss-Legendre in cos(theta) and every node
// phi_k = 2 pi k / Q_phi of the trapezoid rule of eq. azimuthInt.  The flow
// may point anywhere, so no azimuthal node is folded onto another.
//
// Per cell and SSP-RK3 stage: the 14 moment records of the stage input -> the
// Landau frame in FP64 (the timelike eigenvector of T^mu_nu, by Newton's
// method on the three velocity components from the 1D closed form along
// T^{0i}) -> the truncated equilibrium (eq. feqtrunc), which depends on the
// direction only through c = v . u_hat: the coefficients of the 1D projection
// at the speed |u| turned into a polynomial in c once per cell and radial
// node, evaluated by Horner's rule at each point -> WENO5 faces in x, y and z,
// relaxation, RK combination, store, and the 14 moments of the output.
//
// Work decomposition: one lane per cell, workgroups of 64 x 4 cells of one z
// layer (x contiguous in memory, one wave per y row).  For every point the
// workgroup stages its cells and a 3-cell halo in x and y (outflow clamps
// applied at load time) in LDS; each lane computes its own left x face and
// lower y face (the tile's last row and column of faces by a wave that
// rotates with the workgroup and the point) and shares them through LDS.  The
// z direction is not staged: each lane loads its own column z-3 .. z+3 into
// registers (the neighbouring layers are other workgroups' tiles, handed to
// the same XCD in runs along z so that these loads hit its L2) and computes
// both of its z faces there, while the x/y tile is being written.  The next
// point's tile and column values are in flight in registers during the
// current point; two barriers per point, double-buffered LDS.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "rlb_device.h"
#include "rlb_internal.h"

namespace rlb {
namespace {

using namespace dev;

struct Macro3 {
  double e, v[3], gamma, u[3], n, T;
  bool ok;
};

// Landau frame of the 14 moments m = (N0, N^x, N^y, N^z, T00, T0x, T0y, T0z,
// Txx, Txy, Txz, Tyy, Tyz, Tzz): T^mu_nu u^nu = -e u^mu with u = gamma (1, v).
// Its time component gives e = T00 - T0j v_j and the space components the
// residual R_i = T^{0i} - T^{ij} v_j - e v_i = 0, solved by Newton's method
// with the Jacobian dR_i/dv_k = T^{0k} v_i - T^{ik} - e delta_ik.  The start
// is the exact root of the 1D problem along the direction of T^{0i}, which is
// exact for a perfect fluid.
__device__ inline Macro3 landau3(const double m[14]) {
  const double T00 = m[4];
  const double T0[3] = {m[5], m[6], m[7]};
  const double Tm[3][3] = {{m[8], m[9], m[10]}, {m[9], m[11], m[12]}, {m[10], m[12], m[13]}};
  double v[3] = {0.0, 0.0, 0.0};
  const double s = sqrt(T0[0] * T0[0] + T0[1] * T0[1] + T0[2] * T0[2]);
  if (s > 0.0) {
    const double h[3] = {T0[0] / s, T0[1] / s, T0[2] / s};
    double Tnn = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) Tnn += h[a] * Tm[a][b] * h[b];
    const double a = T00 + Tnn;
    const double D = sqrt(fmax((a - 2.0 * s) * (a + 2.0 * s), 0.0));
    const double sp = 2.0 * s / (a + D);
#pragma unroll
    for (int q = 0; q < 3; ++q) v[q] = sp * h[q];
  }
  for (int it = 0; it < 8; ++it) {
    const double e = T00 - T0[0] * v[0] - T0[1] * v[1] - T0[2] * v[2];
    double r[3], J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      r[i] = T0[i] - Tm[i][0] * v[0] - Tm[i][1] * v[1] - Tm[i][2] * v[2] - e * v[i];
#pragma unroll
      for (int k = 0; k < 3; ++k) J[i][k] = T0[k] * v[i] - Tm[i][k] - (i == k ? e : 0.0);
    }
    // J d = -r by the adjugate: d_i = -(sum_k C[k][i] r_k) / det with C the
    // cofactors of J
    const double C00 = J[1][1] * J[2][2] - J[1][2] * J[2][1], C01 = J[1][2] * J[2][0] - J[1][0] * J[2][2],
                 C02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double C10 = J[0][2] * J[2][1] - J[0][1] * J[2][2], C11 = J[0][0] * J[2][2] - J[0][2] * J[2][0],
                 C12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    const double C20 = J[0][1] * J[1][2] - J[0][2] * J[1][1], C21 = J[0][2] * J[1][0] - J[0][0] * J[1][2],
                 C22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * C00 + J[0][1] * C01 + J[0][2] * C02;
    const double d0 = -(C00 * r[0] + C10 * r[1] + C20 * r[2]) / det;
    const double d1 = -(C01 * r[0] + C11 * r[1] + C21 * r[2]) / det;
    const double d2 = -(C02 * r[0] + C12 * r[1] + C22 * r[2]) / det;
    v[0] += d0;
    v[1] += d1;
    v[2] += d2;
    if (fabs(d0) + fabs(d1) + fabs(d2) <= 1e-14) break;
  }
  Macro3 M;
  const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  M.e = T00 - T0[0] * v[0] - T0[1] * v[1] - T0[2] * v[2];
  M.gamma = 1.0 / sqrt(1.0 - v2);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    M.v[q] = v[q];
    M.u[q] = M.gamma * v[q];
  }
  M.n = M.gamma * (m[0] - v[0] * m[1] - v[1] * m[2] - v[2] * m[3]);
  M.T = M.e / (3.0 * M.n);
  M.ok = (M.e > 0.0) && (M.n > 0.0) && (v2 < 1.0) && isfinite(M.T);
  return M;
}

// Moment sums of one radial node, in the order every kernel uses: plain
// fused sums over the azimuthal nodes of one polar node, then (Kahan in FP32)
// across polar nodes.  Ten weighted factors per point (table columns 3 .. 12).
template <typename Real>
struct BoxSums {
  Acc<Real> S[10];
};
template <typename Real>
__device__ inline void add_point10(Real p[10], cptr<Real> V, Real f) {
#pragma unroll
  for (int q = 0; q < 10; ++q) p[q] = fma(V[3 + q], f, p[q]);
}
// Adds one radial node's sums to the 14 records (N from T0^3 w_p p, T from
// T0^4 w_p p^2).
template <typename Ptr, typename M>
__device__ inline void add_node14(M& m, Ptr I, const double S[10]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) m[q] = fma(I[2], S[q], double(m[q]));
#pragma unroll
  for (int q = 0; q < 10; ++q) m[4 + q] = fma(I[3], S[q], double(m[4 + q]));
}

// Tile of a virtual workgroup index: z-fastest within an (x, y) column, XCD
// runs.
__device__ inline void box_tile(int v, int nxt, int nyt, int nz, int& xt, int& yt, int& z) {
  const int item = xcd_item(v, nxt * nyt * nz);
  const int col = item / nz;
  z = item % nz;
  xt = col / nyt;
  yt = col % nyt;
}

// LDS of one point (two buffers, alternating between points): the tile with a
// 3-cell halo in x and y (rows y0-3 .. y0+6, columns x0-3 .. x0+66), then the
// x faces (left face of columns 0 .. 64 of each row) and the y faces (lower
// face of rows 0 .. 4 of each column), all with the row stride kBLd.
constexpr int kBTY = kBoxTileY, kBThreads = kBoxTileX * kBTY;
constexpr int kBLd = kBoxTileX + 8;
constexpr int kBTileRows = kBTY + 6, kBTileCols = kBoxTileX + 6;
constexpr int kBTileElems = kBTileRows * kBTileCols;
constexpr int kBTileLoads = (kBTileElems + kBThreads - 1) / kBThreads;  // per lane
constexpr int kBFxOff = kBTileRows * kBLd, kBFyOff = kBFxOff + kBTY * kBLd;
constexpr int kBBufElems = kBFyOff + (kBTY + 1) * kBLd;
static_assert(kBLd >= kBTileCols && kBLd >= kBoxTileX + 1, "row stride");
static_assert(kBoxTileX == 64 && kBTY == 4, "one wave per tile row, four rows");

template <int B>
using BufTag = std::integral_constant<int, B>;

// WENO5 value at a face from the six values p[0], p[ST], .. p[5 ST] around it
// (LDS), upwinded by the sign of the velocity component (0 .. 4 for up,
// 5 .. 1 otherwise); the empty asm statement keeps the two orientations as
// separate wave-uniform branches reading LDS at immediate offsets.
template <typename Real, int ST>
__device__ inline Real lds_face(const Real* p, bool up, Real eps4) {
  bool unused = true;
  if (up) return weno5(p[0], p[ST], p[2 * ST], p[3 * ST], p[4 * ST], eps4, unused);
  Real h = weno5(p[5 * ST], p[4 * ST], p[3 * ST], p[2 * ST], p[ST], eps4, unused);
  asm volatile("" : "+v"(h));
  return h;
}
// The same from six registers.
template <typename Real>
__device__ inline Real reg_face(Real p0, Real p1, Real p2, Real p3, Real p4, Real p5, bool up, Real eps4) {
  bool unused = true;
  return up ? weno5(p0, p1, p2, p3, p4, eps4, unused) : weno5(p5, p4, p3, p2, p1, eps4, unused);
}

// Occupancy: four waves per SIMD for FP32 with Q_p <= 4 (the LDS of four
// workgroups fills a CU; a few per-cell values spill outside the point loop;
// measured 2.45 against 3.05 ms per stage on a 128^3 box with Q = 192 with
// the compiler's three waves) and three for FP64 with Q_p <= 4 (the per-cell
// values spill, outside the point loop; 14.3 against 17.0 ms per step on that
// box with the compiler's two); the generic group is left to the compiler.
template <typename Real, int QPT>
constexpr int box_waves_per_eu() {
  return (sizeof(Real) == 4 && QPT <= 4) ? 4 : (QPT <= 4 ? 3 : 1);
}

template <typename Real, int QPT, int NVT, bool HAS_FN>
__global__ __launch_bounds__(kBThreads) __attribute__((amdgpu_waves_per_eu(box_waves_per_eu<Real, QPT>())))
void box_stage_kernel(BoxArgs<Real> a) {
  __shared__ Real lds[2 * kBBufElems];
  __shared__ double mom_lds[14][kBThreads];  // the 14 record sums of each lane
  const cptr<BoxDev> B = as_const(a.bx);
  const int nx = B->nx, ny = B->ny, nz = B->nz, ldx = B->ldx, qx = B->qx, qf = B->qf, qp = B->qp;
  const int64_t plane = B->plane;
  const int slab = int(B->slab);
  const uint32_t plane_bytes = uint32_t(plane * int64_t(sizeof(Real)));
  const uint32_t slab_bytes = uint32_t(slab) * uint32_t(sizeof(Real));
  const int nxt = (nx + kBoxTileX - 1) / kBoxTileX, nyt = (ny + kBTY - 1) / kBTY;
  const int items = nxt * nyt * nz;
  const cptr<Real> vtab = as_const(a.vtab);
  const cptr<double> itab = as_const(a.itab);
  const int stage = a.stage;
  const Real cs = stage == 1 ? Real(1) : (stage == 2 ? Real(0.25) : Real(2.0 / 3.0));
  const Real dt = Real(B->dt), dx_inv = Real(B->dx_inv), dy_inv = Real(B->dy_inv), dz_inv = Real(B->dz_inv);
  const Real eps4 = Real(4.0 * B->weno_eps);
  const int t = threadIdx.x, tx = t % kBoxTileX, ty = t / kBoxTileX;
  const int lane_off = ty * kBLd + tx;
  const int wave = __builtin_amdgcn_readfirstlane(ty);
  const int Q = qp * qx * qf;
  for (int v = blockIdx.x; v < items; v += gridDim.x) {
    int xt, yt, z;
    box_tile(v, nxt, nyt, nz, xt, yt, z);
    const int x0 = xt * kBoxTileX, y0 = yt * kBTY;
    const int x = x0 + tx, y = y0 + ty;
    const bool valid = x < nx && y < ny;
    const int cxy = min(y, ny - 1) * ldx + min(x, nx - 1);
    const int cell = z * slab + cxy;
    const uint32_t cxy_b = uint32_t(cxy) * uint32_t(sizeof(Real));
    const uint32_t cell_b = uint32_t(cell) * uint32_t(sizeof(Real));
    // byte offsets of the z layers z-3 .. z+3 (clamped; uniform)
    uint32_t zb[7];
#pragma unroll
    for (int d = 0; d < 7; ++d) zb[d] = uint32_t(min(max(z + d - 3, 0), nz - 1)) * slab_bytes;
    // this lane's share of the tile loads: byte offsets in the layer
    // (clamped) and LDS slots
    uint32_t loff[kBTileLoads];
    int lslot[kBTileLoads];
#pragma unroll
    for (int q = 0; q < kBTileLoads; ++q) {
      const int e = t + kBThreads * q;
      const int r = min(e, kBTileElems - 1) / kBTileCols, c = min(e, kBTileElems - 1) % kBTileCols;
      const int gy = min(max(y0 - 3 + r, 0), ny - 1), gx = min(max(x0 - 3 + c, 0), nx - 1);
      loff[q] = uint32_t(gy * ldx + gx) * uint32_t(sizeof(Real));
      lslot[q] = e < kBTileElems ? r * kBLd + c : -1;
    }
    // Landau frame of the stage input (FP64)
    double m[14];
#pragma unroll
    for (int c = 0; c < 14; ++c) m[c] = a.rec_in[c * plane + cell];
    const Macro3 M = landau3(m);
    if (valid && !M.ok) atomicOr(a.flag, kFlagNonphysical);
    if (valid && M.v[0] * M.v[0] + M.v[1] * M.v[1] + M.v[2] * M.v[2] > 0.95 * 0.95) atomicOr(a.flag, kFlagFastFlow);
    const double ua = sqrt(M.u[0] * M.u[0] + M.u[1] * M.u[1] + M.u[2] * M.u[2]);
    const Real hx = Real(ua > 0.0 ? M.u[0] / ua : 0.0), hy = Real(ua > 0.0 ? M.u[1] / ua : 0.0),
               hz = Real(ua > 0.0 ? M.u[2] / ua : 1.0);
    Real D[QPT][NVT + 1];
    feq_coefficients<Real, QPT, NVT>(Real(M.n), Real(M.T), Real(M.gamma), Real(ua), Real(B->T0), qp, B->np, B->nv,
                                     itab, as_const(a.aux), a.aux_pairs, D);
    const Real g0 = Real(M.gamma * B->tau_inv), gx = Real(M.u[0] * B->tau_inv), gy = Real(M.u[1] * B->tau_inv),
               gz = Real(M.u[2] * B->tau_inv);
#pragma unroll
    for (int c = 0; c < 14; ++c) mom_lds[c][t] = 0.0;
    // first point's tile and column values
    Real pre[kBTileLoads], zp[7];
    {
      const Rsrc r0 = make_rsrc(a.fin, plane_bytes);
#pragma unroll
      for (int q = 0; q < kBTileLoads; ++q) pre[q] = BufIO<Real>::template load<0>(r0, loff[q], zb[3]);
#pragma unroll
      for (int d = 0; d < 7; ++d) zp[d] = BufIO<Real>::template load<0>(r0, cxy_b, zb[d]);
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
      BoxSums<Real> acc;
#pragma unroll 1
      for (int j = 0; j < qx; ++j) {
        Real p10[10];
#pragma unroll
        for (int q = 0; q < 10; ++q) p10[q] = Real(0);
        // One point s = (i qx + j) qf + k with its tile staged in buffer B.
        auto point = [&](auto tag, int k) {
          constexpr int BO = decltype(tag)::value * kBBufElems;
          Real* const L = lds + BO;
          // 1. stage this point's tile, take its column values, prefetch the
          //    next point's
#pragma unroll
          for (int q = 0; q < kBTileLoads; ++q)
            if (lslot[q] >= 0) L[lslot[q]] = pre[q];
          Real zc[7];
#pragma unroll
          for (int d = 0; d < 7; ++d) zc[d] = zp[d];
          if (s + 1 < Q) {
            const Rsrc rn = make_rsrc(a.fin + int64_t(s + 1) * plane, plane_bytes);
#pragma unroll
            for (int q = 0; q < kBTileLoads; ++q) pre[q] = BufIO<Real>::template load<0>(rn, loff[q], zb[3]);
#pragma unroll
            for (int d = 0; d < 7; ++d) zp[d] = BufIO<Real>::template load<0>(rn, cxy_b, zb[d]);
          }
          const Real fnv =
              HAS_FN ? BufIO<Real>::template load<2>(make_rsrc(a.fn + int64_t(s) * plane, plane_bytes), cell_b, 0)
                     : Real(0);
          const cptr<Real> V = vtab + (j * qf + k) * kBoxVStride;
          const Real vx = V[0], vy = V[1], vz = V[2];
          // 2. the two z faces of this lane's cell, from its column
          const bool uz = vz >= Real(0);
          const Real hzl = reg_face(zc[0], zc[1], zc[2], zc[3], zc[4], zc[5], uz, eps4);
          const Real hzr = reg_face(zc[1], zc[2], zc[3], zc[4], zc[5], zc[6], uz, eps4);
          __syncthreads();
          // 3. this lane's left x face and lower y face; the tile's upper y
          //    faces and right x faces go to a wave that rotates with the
          //    workgroup and the point
          const bool ux = vx >= Real(0), uy = vy >= Real(0);
          const Real* T = L + lane_off;
          L[kBFxOff + lane_off] = lds_face<Real, 1>(T + 3 * kBLd, ux, eps4);
          L[kBFyOff + lane_off] = lds_face<Real, kBLd>(T + 3, uy, eps4);
          const int wy = (int(blockIdx.x) + s) & (kBTY - 1);
          if (wave == wy)
            L[kBFyOff + kBTY * kBLd + tx] = lds_face<Real, kBLd>(L + kBTY * kBLd + 3 + tx, uy, eps4);
          if (wave == (wy ^ (kBTY / 2)) && tx < kBTY)
            L[kBFxOff + tx * kBLd + kBoxTileX] = lds_face<Real, 1>(L + (tx + 3) * kBLd + kBoxTileX, ux, eps4);
          __syncthreads();
          // 4. update
          const Real fr = zc[3];
          const Real hxl = L[kBFxOff + lane_off], hxr = L[kBFxOff + lane_off + 1];
          const Real hyl = L[kBFyOff + lane_off], hyr = L[kBFyOff + lane_off + kBLd];
          const Real feq = horner<Real, NVT>(Am, vx * hx + vy * hy + vz * hz);
          const Real adv = (hxr - hxl) * (-vx * dx_inv) + (hyr - hyl) * (-vy * dy_inv) + (hzr - hzl) * (-vz * dz_inv);
          const Real rate = g0 - vx * gx - vy * gy - vz * gz;
          const Real Lr = adv - rate * (fr - feq);
          // f^n + cs ((f_in - f^n) + dt L): one rounding at the scale of F
          const Real out = HAS_FN ? fnv + cs * ((fr - fnv) + dt * Lr) : fr + dt * Lr;
          if (valid)
            BufIO<Real>::template store<2>(out, make_rsrc(a.fout + int64_t(s) * plane, plane_bytes), cell_b, 0);
          add_point10(p10, V, out);
          ++s;
        };
        int k = 0;
        for (; k + 1 < qf; k += 2) {
          point(BufTag<0>{}, k);
          point(BufTag<1>{}, k + 1);
        }
        if (k < qf) {
          point(BufTag<0>{}, k);
          __syncthreads();  // the next point reuses buffer 0
        }
#pragma unroll
        for (int q = 0; q < 10; ++q) acc.S[q].add(p10[q]);
      }
      double S[10];
#pragma unroll
      for (int q = 0; q < 10; ++q) S[q] = acc.S[q].value();
      double mm[14];
#pragma unroll
      for (int c = 0; c < 14; ++c) mm[c] = mom_lds[c][t];
      add_node14(mm, itab + i * kIStride, S);
#pragma unroll
      for (int c = 0; c < 14; ++c) mom_lds[c][t] = mm[c];
    }
    if (valid) {
#pragma unroll
      for (int c = 0; c < 14; ++c) a.rec_out[c * plane + cell] = mom_lds[c][t];
    }
    __syncthreads();  // the next tile reuses the LDS buffers
  }
}

// Cell of a lane in the init / moments kernels (the stage kernel's tiles).
__device__ inline bool box_cell(const BoxDev* B, int v, int& x, int& y, int& z) {
  const int nxt = (B->nx + kBoxTileX - 1) / kBoxTileX, nyt = (B->ny + kBTY - 1) / kBTY;
  int xt, yt;
  box_tile(v, nxt, nyt, B->nz, xt, yt, z);
  x = xt * kBoxTileX + int(threadIdx.x) % kBoxTileX;
  y = yt * kBTY + int(threadIdx.x) / kBoxTileX;
  return x < B->nx && y < B->ny;
}

// Initial state: the truncated equilibrium of each cell's (P, n, u^x, u^y,
// u^z), and its records (the same sums as the stage epilogue).
template <typename Real, int QPT, int NVT>
__global__ __launch_bounds__(256) void box_init_kernel(BoxArgs<Real> a) {
  const cptr<BoxDev> B = as_const(a.bx);
  const int nx = B->nx, ny = B->ny, nz = B->nz, ldx = B->ldx, qx = B->qx, qf = B->qf, qp = B->qp;
  const int64_t plane = B->plane, slab = B->slab;
  const int items = ((nx + kBoxTileX - 1) / kBoxTileX) * ((ny + kBTY - 1) / kBTY) * nz;
  const cptr<Real> vtab = as_const(a.vtab);
  const cptr<double> itab = as_const(a.itab);
  for (int v = blockIdx.x; v < items; v += gridDim.x) {
    int x, y, z;
    if (!box_cell(a.bx, v, x, y, z)) continue;
    const int64_t cell = z * slab + int64_t(y) * ldx + x;
    const int64_t cells = int64_t(nx) * ny * nz, dense = (int64_t(z) * ny + y) * nx + x;
    const double Pr = a.init[dense], n = a.init[cells + dense];
    const double u[3] = {a.init[2 * cells + dense], a.init[3 * cells + dense], a.init[4 * cells + dense]};
    const double ua = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]), gamma = sqrt(1.0 + ua * ua);
    const Real hx = Real(ua > 0.0 ? u[0] / ua : 0.0), hy = Real(ua > 0.0 ? u[1] / ua : 0.0),
               hz = Real(ua > 0.0 ? u[2] / ua : 1.0);
    Real D[QPT][NVT + 1];
    feq_coefficients<Real, QPT, NVT>(Real(n), Real(Pr / n), Real(gamma), Real(ua), Real(B->T0), qp, B->np, B->nv,
                                     itab, as_const(a.aux), a.aux_pairs, D);
    double mom[14];
#pragma unroll
    for (int c = 0; c < 14; ++c) mom[c] = 0.0;
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
      if (i < qp) {
        Real Am[NVT + 1];
        series_monomials<Real, NVT>(D[i], Am);
        BoxSums<Real> acc;
        for (int j = 0; j < qx; ++j) {
          Real p10[10];
#pragma unroll
          for (int q = 0; q < 10; ++q) p10[q] = Real(0);
          for (int k = 0; k < qf; ++k) {
            const int64_t s = int64_t((i * qx + j) * qf + k);
            const cptr<Real> V = vtab + (j * qf + k) * kBoxVStride;
            const Real f = horner<Real, NVT>(Am, V[0] * hx + V[1] * hy + V[2] * hz);
            a.fout[s * plane + cell] = f;
            add_point10(p10, V, f);
          }
#pragma unroll
          for (int q = 0; q < 10; ++q) acc.S[q].add(p10[q]);
        }
        double S[10];
#pragma unroll
        for (int q = 0; q < 10; ++q) S[q] = acc.S[q].value();
        add_node14(mom, itab + i * kIStride, S);
      }
    }
#pragma unroll
    for (int c = 0; c < 14; ++c) a.rec_out[c * plane + cell] = mom[c];
  }
}

// Records of a stored state (after a state load).
template <typename Real>
__global__ __launch_bounds__(256) void box_moments_kernel(BoxArgs<Real> a) {
  const cptr<BoxDev> B = as_const(a.bx);
  const int nx = B->nx, ny = B->ny, nz = B->nz, ldx = B->ldx, qx = B->qx, qf = B->qf, qp = B->qp;
  const int64_t plane = B->plane, slab = B->slab;
  const int items = ((nx + kBoxTileX - 1) / kBoxTileX) * ((ny + kBTY - 1) / kBTY) * nz;
  const cptr<Real> vtab = as_const(a.vtab);
  const cptr<double> itab = as_const(a.itab);
  for (int v = blockIdx.x; v < items; v += gridDim.x) {
    int x, y, z;
    if (!box_cell(a.bx, v, x, y, z)) continue;
    const int64_t cell = z * slab + int64_t(y) * ldx + x;
    double mom[14];
#pragma unroll
    for (int c = 0; c < 14; ++c) mom[c] = 0.0;
    for (int i = 0; i < qp; ++i) {
      BoxSums<Real> acc;
      for (int j = 0; j < qx; ++j) {
        Real p10[10];
#pragma unroll
        for (int q = 0; q < 10; ++q) p10[q] = Real(0);
        for (int k = 0; k < qf; ++k) {
          const int64_t s = int64_t((i * qx + j) * qf + k);
          add_point10(p10, vtab + (j * qf + k) * kBoxVStride, a.fin[s * plane + cell]);
        }
#pragma unroll
        for (int q = 0; q < 10; ++q) acc.S[q].add(p10[q]);
      }
      double S[10];
#pragma unroll
      for (int q = 0; q < 10; ++q) S[q] = acc.S[q].value();
      add_node14(mom, itab + i * kIStride, S);
    }
#pragma unroll
    for (int c = 0; c < 14; ++c) a.rec_out[c * plane + cell] = mom[c];
  }
}

// Fields [20][nz][ny][nx] from the records: the 14 moments, e, n, v_x, v_y,
// v_z, T.
__global__ __launch_bounds__(256) void box_fields_kernel(const BoxDev* bx, const double* rec, double* out,
                                                         unsigned* flag) {
  const cptr<BoxDev> B = as_const(bx);
  const int nx = B->nx, ny = B->ny, ldx = B->ldx;
  const int64_t plane = B->plane, slab = B->slab, cells = int64_t(nx) * ny * B->nz;
  const int64_t dense = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (dense >= cells) return;
  const int64_t x = dense % nx, y = (dense / nx) % ny, z = dense / (int64_t(nx) * ny);
  const int64_t cell = z * slab + y * ldx + x;
  double m[14];
  for (int c = 0; c < 14; ++c) m[c] = rec[c * plane + cell];
  const Macro3 M = landau3(m);
  if (!M.ok) atomicOr(flag, kFlagNonphysical);
  for (int c = 0; c < 14; ++c) out[c * cells + dense] = m[c];
  out[14 * cells + dense] = M.e;
  out[15 * cells + dense] = M.n;
  for (int q = 0; q < 3; ++q) out[(16 + q) * cells + dense] = M.v[q];
  out[19 * cells + dense] = M.T;
}

template <typename Real, int QPT, int NVT>
hipError_t stage_t(const void* args, int grid, hipStream_t s) {
  const BoxArgs<Real>& a = *static_cast<const BoxArgs<Real>*>(args);
  if (a.stage == 1)
    hipLaunchKernelGGL((box_stage_kernel<Real, QPT, NVT, false>), dim3(grid), dim3(kBThreads), 0, s, a);
  else
    hipLaunchKernelGGL((box_stage_kernel<Real, QPT, NVT, true>), dim3(grid), dim3(kBThreads), 0, s, a);
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
  const BoxArgs<Real>& a = *static_cast<const BoxArgs<Real>*>(args);
  if (qpt == 3 && nvt == 5)
    hipLaunchKernelGGL((box_init_kernel<Real, 3, 5>), dim3(grid), dim3(256), 0, s, a);
  else if (qpt == 4 && nvt == 5)
    hipLaunchKernelGGL((box_init_kernel<Real, 4, 5>), dim3(grid), dim3(256), 0, s, a);
  else if (qpt == 8 && nvt == 7)
    hipLaunchKernelGGL((box_init_kernel<Real, 8, 7>), dim3(grid), dim3(256), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

int box_grid(int nx, int ny, int nz) {
  return ((nx + kBoxTileX - 1) / kBoxTileX) * ((ny + kBTY - 1) / kBTY) * nz;
}

hipError_t launch_box_stage(int prec_fp32, int qpt, int nvt, const void* args, int grid, hipStream_t stream) {
  return prec_fp32 ? stage_real<float>(qpt, nvt, args, grid, stream) : stage_real<double>(qpt, nvt, args, grid, stream);
}

hipError_t launch_box_init(int prec_fp32, int qpt, int nvt, const void* args, int grid, hipStream_t stream) {
  return prec_fp32 ? init_real<float>(qpt, nvt, args, grid, stream) : init_real<double>(qpt, nvt, args, grid, stream);
}

hipError_t launch_box_moments(int prec_fp32, const void* args, int grid, hipStream_t stream) {
  if (prec_fp32)
    hipLaunchKernelGGL(box_moments_kernel<float>, dim3(grid), dim3(256), 0, stream,
                       *static_cast<const BoxArgs<float>*>(args));
  else
    hipLaunchKernelGGL(box_moments_kernel<double>, dim3(grid), dim3(256), 0, stream,
                       *static_cast<const BoxArgs<double>*>(args));
  return hipGetLastError();
}

hipError_t launch_box_fields(const BoxDev* bx, int64_t cells, const double* rec, double* out, unsigned* flag,
                             hipStream_t stream) {
  hipLaunchKernelGGL(box_fields_kernel, dim3(unsigned((cells + 255) / 256)), dim3(256), 0, stream, bx, rec, out, flag);
  return hipGetLastError();
}

}  // namespace rlb
