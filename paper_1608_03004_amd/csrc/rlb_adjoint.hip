// Discrete adjoint of the SSP-RK3 lattice Boltzmann step (hand-written
// reverse mode of the forward kernels in rlb_kernels.hip).
//
// For a stage input g the right-hand side is L(g) = A(g) + R(g) with
//   A_s(x) = -(xi_j/dz) (H_s(x+1/2) - H_s(x-1/2))          (WENO5 advection)
//   R_s(x) = -rho_s(x) (g_s(x) - e_s(x)),  rho = (gamma - xi u)/tau
// where gamma, u, n, T come from the Landau matching of the moments m(x) of g
// and e_s(x) is the truncated equilibrium.  Its transpose applied to K is
//   (dL/dg)^T K = A^T K - rho K + B_s . mu(x),
// with B_s the moment basis of point s and mu(x) = dR/dm^T K, obtained from a
// reduction over the points of the cell followed by the adjoints of the
// equilibrium projection and of the Landau matching.  Three parts per stage
// (the first two in one launch, adj_reduce_faces_kernel):
//   adj_reduce   per cell (four waves share a cell's sums): mu(x), the rate
//                constants and d/dtau,
//   adj_faces    one lane per (point, face): WENO5 gradient times the face
//                adjoint phi = -(xi/dz)(K_left - K_right),
//   adj_combine  one lane per (point, cell): gathers the face contributions
//                (contributions to ghost cells fold into the edge cell, the
//                transpose of the zero-gradient ghost copy) and forms the RK
//                adjoint combination.
#include <hip/hip_runtime.h>

#include "rlb_device.h"
#include "rlb_internal.h"

namespace rlb {
namespace {

using namespace dev;

// adj_reduce: a block of 256 threads holds red_cells() cells and 256 /
// red_cells() groups of red_cells() lanes, one lane per cell in each group.
// The groups split the quadrature points of the reduction and the auxiliary
// node pairs of the projection's adjoint; partial sums are combined through
// LDS in a fixed group order, so the result is deterministic.  The adjoint is
// latency-bound at its sizes, so small blocks pay: on 4096 cells x 96 points,
// 32 cells per block gave +9 % adjoint steps/s over 64 in FP64 and FP32, and
// 16 cells another +7.7 % in FP32 (but -2 % in FP64).
template <typename Real>
constexpr int red_cells() {
  return sizeof(Real) == 4 ? 16 : 32;
}

// acc[d][lane] = sum over groups (in group order) of part[d]; every group
// reads the same combined values afterwards.  Ends with a barrier.  The groups
// post kSlotVals values at a time and group g sums value g of the batch over
// the groups, so a batch costs two barriers whatever the group count.
constexpr int kSlotVals = 8;
template <int N, int kRedCells>
__device__ inline void combine_groups(double (*acc)[kRedCells], const double* part, int grp, int lane) {
  constexpr int kRedGroups = 256 / kRedCells;
  static_assert(kSlotVals <= kRedGroups, "one summing group per posted value");
  __shared__ double slots[kRedGroups][kSlotVals][kRedCells];
#pragma unroll
  for (int d0 = 0; d0 < N; d0 += kSlotVals) {
#pragma unroll
    for (int dd = 0; dd < kSlotVals; ++dd)
      if (d0 + dd < N) slots[grp][dd][lane] = part[d0 + dd];
    __syncthreads();
    if (grp < kSlotVals && d0 + grp < N) {
      double s = slots[0][grp][lane];
      for (int g = 1; g < kRedGroups; ++g) s += slots[g][grp][lane];
      acc[d0 + grp][lane] = s;
    }
    __syncthreads();
  }
}

template <typename Real, int QPT, int NVT>
__device__ inline void adj_reduce_block(const AdjArgs<Real>& a, int block) {
  constexpr int kRedCells = red_cells<Real>(), kRedGroups = 256 / kRedCells;
  constexpr int ND = QPT * (NVT + 1);
  __shared__ double acc[ND + 3][kRedCells];
  const int lane = threadIdx.x % kRedCells, grp = threadIdx.x / kRedCells;
  const TubeDev& tb = a.tubes[a.tube];
  const int nx = tb.nx;
  const int y = block * kRedCells + lane;
  const bool valid = y < nx;
  const int yc = valid ? y : nx - 1;
  const int64_t ldx = tb.ldx;
  const int qx = tb.qx, qp = tb.qp;
  const cptr<Real> jtab = as_const(a.jtab) + int64_t(tb.jrow) * kJStride;
  const cptr<double> itab = as_const(a.itab) + int64_t(tb.irow) * kIStride;
  double m[5];
  for (int c = 0; c < 5; ++c) m[c] = a.rec_g[tb.rec_off + c * ldx + yc];
  // the first kPre points of each radial node that this group reduces below
  // (j = grp + kRedGroups jj, jj < kPre): their loads go out before the Landau
  // solve and the projection, which hide their latency.  One point per node:
  // on the 4096-cell adjoint tube (Q = 32 x 3) FP32 gave 10.7e3 adjoint steps/s
  // against 9.5e3 with four (the registers of four cost a wave per SIMD of
  // the face blocks sharing the launch) and 10.0e3 with none.
  constexpr int kPre = 1;
  const Real* g = a.g + tb.f_off;
  const Real* K = a.K + tb.f_off;
  Real Kp[QPT][kPre], gp[QPT][kPre];
#pragma unroll
  for (int i = 0; i < QPT; ++i)
#pragma unroll
    for (int jj = 0; jj < kPre; ++jj) {
      const int j = grp + kRedGroups * jj;
      const bool has = i < qp && j < qx;
      const int64_t row = has ? int64_t(i * qx + j) * ldx : 0;
      Kp[i][jj] = has ? K[row + yc] : Real(0);
      gp[i][jj] = has ? g[row + yc] : Real(0);
    }
  const Macro M = landau(m);

  // 1. projection coefficients, bit for bit those of the forward stage kernel
  //    (f - f^eq is small, so the reduction below needs the forward's f^eq
  //    exactly): group grp sums the rows of radial nodes grp, grp + G, ...
  //    over all pairs in the forward's order, and the rows are exchanged
  Real D[QPT][NVT + 1];
  {
    feq_projection_sums<Real, QPT, NVT>(Real(M.T), Real(M.gamma), Real(M.u), Real(tb.T0), qp, tb.np, itab,
                                        as_const(a.aux), a.aux_pairs, 0, 1, D, grp, kRedGroups);
#pragma unroll
    for (int i = 0; i < QPT; ++i)
      if (i % kRedGroups == grp)
#pragma unroll
        for (int k = 0; k <= NVT; ++k) acc[i * (NVT + 1) + k][lane] = double(D[i][k]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < QPT; ++i)
#pragma unroll
      for (int k = 0; k <= NVT; ++k) D[i][k] = Real(acc[i * (NVT + 1) + k][lane]);
    feq_scale<Real, QPT, NVT>(Real(M.n), Real(M.T), Real(tb.T0), tb.nv, D);
    __syncthreads();  // acc is reused below
  }

  // 2. reduction over the points (group grp takes j = grp, grp + G, ...)
  const double tau_inv = tb.tau_inv;
  const Real g0 = Real(M.gamma * tau_inv), g1 = Real(M.u * tau_inv);
  double red[ND + 3];
#pragma unroll
  for (int d = 0; d < ND + 3; ++d) red[d] = 0.0;
  double& Gb = red[ND];
  double& Ub = red[ND + 1];
  double& taup = red[ND + 2];
#pragma unroll
  for (int i = 0; i < QPT; ++i) {
    if (i < qp) {
      // one point j of node i with its K and g values, in j order
      auto point = [&](int j, Real Kr, Real gr) {
        const cptr<Real> J = jtab + j * kJStride;
        const Real xi = J[0];
        const double Kv = double(Kr);
        Real e = Real(0);
#pragma unroll
        for (int k = 0; k <= NVT; ++k) e += D[i][k] * J[4 + k];
        const double diff = double(gr) - double(e);
        const double rho = double(g0 - xi * g1);
        Gb -= Kv * diff * tau_inv;
        Ub += Kv * double(xi) * diff * tau_inv;
        const double kr = Kv * rho;
#pragma unroll
        for (int k = 0; k <= NVT; ++k) red[i * (NVT + 1) + k] += kr * double(J[4 + k]);
        taup += kr * tau_inv * diff;
      };
#pragma unroll
      for (int jj = 0; jj < kPre; ++jj)
        if (grp + kRedGroups * jj < qx) point(grp + kRedGroups * jj, Kp[i][jj], gp[i][jj]);
#pragma unroll 4
      for (int j = grp + kRedGroups * kPre; j < qx; j += kRedGroups) {
        const int64_t row = int64_t(i * qx + j) * ldx;
        point(j, K[row + yc], g[row + yc]);
      }
    }
  }
  combine_groups<ND + 3, kRedCells>(acc, red, grp, lane);
  double Db[QPT][NVT + 1];
#pragma unroll
  for (int i = 0; i < QPT; ++i)
#pragma unroll
    for (int k = 0; k <= NVT; ++k) Db[i][k] = acc[i * (NVT + 1) + k][lane];
  const double Gb_all = acc[ND][lane], Ub_all = acc[ND + 1][lane], taup_all = acc[ND + 2][lane];
  __syncthreads();  // acc is reused below

  // 3. adjoint of the projection (the groups share the auxiliary pairs again)
  double part[4] = {0.0, 0.0, 0.0, 0.0};  // prefb, rb, gamma-bar, u-bar
  feq_adjoint_sums<QPT, NVT>(M.n, M.T, M.gamma, M.u, tb.T0, qp, tb.np, tb.nv, itab, as_const(a.aux_d), a.aux_pairs,
                             grp, kRedGroups, Db, part[0], part[1], part[2], part[3]);
  combine_groups<4, kRedCells>(acc, part, grp, lane);
  if (grp != 0 || !valid) return;
  double nb = 0.0, Tb = 0.0;
  feq_adjoint_finish(M.n, M.T, tb.T0, acc[0][lane], acc[1][lane], nb, Tb);
  const double gb = Gb_all + acc[2][lane], ub = Ub_all + acc[3][lane];
  double mu[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  landau_adjoint(m, M, 0.0, 0.0, gb, ub, nb, Tb, mu);
  double* cb = a.cellbuf + 7 * tb.cell_off;
  for (int c = 0; c < 5; ++c) cb[c * ldx + y] = mu[c];
  cb[5 * ldx + y] = double(g0);
  cb[6 * ldx + y] = double(g1);
  double* ta = a.tau_acc + tb.cell_off;
  ta[y] = (a.tau_init ? 0.0 : ta[y]) + a.cJ * taup_all;
}

// High-order form (n_v > 7).  The stage's equilibrium values are the
// pre-pass's (the forward's kernel on the same records, so bit for bit those
// the forward used); its adjoint runs through the even/odd tables of the
// fused projection.  Per radial node the forward forms, over the pairs b,
//   ce_j = sum_b Ze[j][b] E_b,  co_j = sum_b Zo[j][b] O_b   (j < half),
//   F_j = (ce_j + co_j)/2,  F_j' = (ce_j - co_j)/2   (j' = q_xi - 1 - j; the
//   middle node of an odd rule only F_j),
//   E_b = pref (G(x_b) + G(-x_b)),  O_b = pref (G(x_b) - G(-x_b)),
// so with W_j = dL/dF_j the pair adjoints are
//   Ebar_b = sum_j Ze[j][b] (W_j + W_j')/2,  Obar_b = sum_j Zo[j][b] (W_j - W_j')/2
// (W_j/2 for both at the middle node), and E_b, O_b go through the same chain
// to (pref, r, gamma, u) as the low-order coefficients' adjoint.  The groups
// split the points for W and the pairs for the chain; W of a node is shared
// through LDS.
template <typename Real>
__device__ inline void adj_reduce_block_high(const AdjArgs<Real>& a, int block) {
  constexpr int kRedCells = red_cells<Real>(), kRedGroups = 256 / kRedCells;
  __shared__ double wv[kMaxQxHigh][kRedCells];
  __shared__ double acc[7][kRedCells];
  const int lane = threadIdx.x % kRedCells, grp = threadIdx.x / kRedCells;
  const TubeDev& tb = a.tubes[a.tube];
  const int nx = tb.nx;
  const int y = block * kRedCells + lane;
  const bool valid = y < nx;
  const int yc = valid ? y : nx - 1;
  const int64_t ldx = tb.ldx;
  const int qx = tb.qx, qp = tb.qp, np = tb.np, half = (qx + 1) / 2;
  const cptr<Real> jtab = as_const(a.jtab) + int64_t(tb.jrow) * kJStride;
  const cptr<double> itab = as_const(a.itab) + int64_t(tb.irow) * kIStride;
  const cptr<double> zt = as_const(a.ztab) + tb.z_off;
  const int zj = tb.zj, zb = tb.zb;
  double m[5];
  for (int c = 0; c < 5; ++c) m[c] = a.rec_g[tb.rec_off + c * ldx + yc];
  const Macro M = landau(m);
  const double tau_inv = tb.tau_inv;
  const Real g0 = Real(M.gamma * tau_inv), g1 = Real(M.u * tau_inv);
  const double pref = M.n / (4.0 * M.T * tb.T0 * tb.T0), r = M.T / tb.T0;
  const Real* g = a.g + tb.f_off;
  const Real* K = a.K + tb.f_off;
  const Real* feq = a.feq + tb.f_off;
  // per-group partial sums: gamma-bar and u-bar of the rate, d/dtau, and the
  // projection's prefb, rb, gamma-bar, u-bar
  double part[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < qp; ++i) {
    for (int j = grp; j < qx; j += kRedGroups) {
      const int64_t row = int64_t(i * qx + j) * ldx;
      const Real xi = jtab[j * kJStride];
      const double Kv = double(K[row + yc]);
      const double diff = double(g[row + yc]) - double(feq[row + yc]);
      const double rho = double(g0 - xi * g1);
      part[0] -= Kv * diff * tau_inv;
      part[1] += Kv * double(xi) * diff * tau_inv;
      const double kr = Kv * rho;
      part[2] += kr * tau_inv * diff;
      wv[j][lane] = kr;
    }
    __syncthreads();
    const cptr<double> L = itab + i * kIStride + 4;
    for (int b = grp; b < zb; b += kRedGroups) {
      double ev = 0.0, od = 0.0;
      for (int j = 0; j < half; ++j) {
        const int jm = qx - 1 - j;
        const double wj = wv[j][lane];
        const double ce = jm == j ? 0.5 * wj : 0.5 * (wj + wv[jm][lane]);
        const double co = jm == j ? 0.5 * wj : 0.5 * (wj - wv[jm][lane]);
        ev += zt[j * zb + b] * ce;
        od += zt[(zj + j) * zb + b] * co;
      }
      const double xa = zt[2 * zj * zb + b];
      const double yp = 1.0 / (M.gamma - xa * M.u), ym = 1.0 / (M.gamma + xa * M.u);
      const double qpl = 1.0 - r * yp, qmi = 1.0 - r * ym;
      double sp = L[np], dsp = 0.0, sm = L[np], dsm = 0.0;
      for (int l = np - 1; l >= 0; --l) {
        dsp = dsp * qpl + sp;
        sp = sp * qpl + L[l];
        dsm = dsm * qmi + sm;
        sm = sm * qmi + L[l];
      }
      const double yp2 = yp * yp, ym2 = ym * ym;
      const double gp = yp2 * sp, gm = ym2 * sm;
      part[3] += ev * (gp + gm) + od * (gp - gm);
      const double gpb = pref * (ev + od), gmb = pref * (ev - od);
      double ypb = gpb * 2.0 * yp * sp, ymb = gmb * 2.0 * ym * sm;
      const double qpb = gpb * yp2 * dsp, qmb = gmb * ym2 * dsm;
      part[4] -= qpb * yp + qmb * ym;
      ypb -= qpb * r;
      ymb -= qmb * r;
      part[5] -= ypb * yp2 + ymb * ym2;
      part[6] += ypb * xa * yp2 - ymb * xa * ym2;
    }
    __syncthreads();  // wv is rewritten for the next node
  }
  combine_groups<7, kRedCells>(acc, part, grp, lane);
  if (grp != 0 || !valid) return;
  double nb = 0.0, Tb = 0.0;
  feq_adjoint_finish(M.n, M.T, tb.T0, acc[3][lane], acc[4][lane], nb, Tb);
  const double gb = acc[0][lane] + acc[5][lane], ub = acc[1][lane] + acc[6][lane];
  double mu[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  landau_adjoint(m, M, 0.0, 0.0, gb, ub, nb, Tb, mu);
  double* cb = a.cellbuf + 7 * tb.cell_off;
  for (int c = 0; c < 5; ++c) cb[c * ldx + y] = mu[c];
  cb[5 * ldx + y] = double(g0);
  cb[6 * ldx + y] = double(g1);
  double* ta = a.tau_acc + tb.cell_off;
  ta[y] = (a.tau_init ? 0.0 : ta[y]) + a.cJ * acc[2][lane];
}

template <typename Real>
__global__ __launch_bounds__(256) void adj_reduce_high_kernel(AdjArgs<Real> a) {
  adj_reduce_block_high<Real>(a, blockIdx.x);
}

template <typename Real>
__device__ inline void adj_faces_block(const AdjArgs<Real>& a, int bx, int s) {
  const TubeDev& tb = a.tubes[a.tube];
  const int nx = tb.nx;
  const int fx = bx * 256 + int(threadIdx.x);  // face fx sits between cells fx-1 and fx
  if (fx > nx) return;
  const int j = s % tb.qx;
  const Real xi = a.jtab[int64_t(tb.jrow + j) * kJStride];
  const Real* g = a.g + tb.f_off + int64_t(s) * tb.ldx;
  const Real* K = a.K + tb.f_off + int64_t(s) * tb.ldx;
  const int x = fx - 1;
  auto G = [&](int p) { return g[p < 0 ? 0 : (p >= nx ? nx - 1 : p)]; };
  Real gr[5];
  const Real eps = Real(tb.weno_eps);
  if (xi >= Real(0)) weno5_grad(G(x - 2), G(x - 1), G(x), G(x + 1), G(x + 2), eps, gr);
  else weno5_grad(G(x + 3), G(x + 2), G(x + 1), G(x), G(x - 1), eps, gr);
  const Real kl = (x >= 0) ? K[x] : Real(0);
  const Real kr = (x + 1 < nx) ? K[x + 1] : Real(0);
  const Real phi = -xi * Real(tb.dz_inv) * (kl - kr);
  Real* out = a.G + tb.face_off + int64_t(s) * tb.ldf + fx;
#pragma unroll
  for (int m = 0; m < 5; ++m) out[m * a.G_slot] = phi * gr[m];
}

// The per-cell reduction and the face gradients read only the stage state and
// the incoming adjoint, so one launch runs both: its first `nred` blocks are
// reduction blocks, the rest face blocks (nfx per point).  The face blocks
// fill the CUs the reduction leaves idle at the adjoint's sizes.
template <typename Real, int QPT, int NVT>
__global__ __launch_bounds__(256) void adj_reduce_faces_kernel(AdjArgs<Real> a, int nred, int nfx) {
  const int b = blockIdx.x;
  if (b < nred) {
    adj_reduce_block<Real, QPT, NVT>(a, b);
  } else {
    const int f = b - nred;
    adj_faces_block<Real>(a, f % nfx, f / nfx);
  }
}

template <typename Real>
__global__ __launch_bounds__(256) void adj_combine_kernel(AdjArgs<Real> a) {
  const TubeDev& tb = a.tubes[a.tube];
  const int nx = tb.nx;
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= nx) return;
  const int s = blockIdx.y;
  const int i = s / tb.qx, j = s % tb.qx;
  const Real* J = a.jtab + int64_t(tb.jrow + j) * kJStride;
  const double* I = a.itab + int64_t(tb.irow + i) * kIStride;
  const Real xi = J[0];
  const bool pos = xi >= Real(0);
  const Real* Gp = a.G + tb.face_off + int64_t(s) * tb.ldf;
  // sum of the face contributions aimed at (unclamped) position p
  auto at = [&](int p) {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const int fx = pos ? p + 3 - m : p - 2 + m;
      if (fx >= 0 && fx <= nx) acc += double(Gp[m * a.G_slot + fx]);
    }
    return acc;
  };
  double adv = at(y);
  if (y == 0) adv += at(-1) + at(-2) + at(-3);
  if (y == nx - 1) adv += at(nx) + at(nx + 1) + at(nx + 2);
  const int64_t ldx = tb.ldx;
  const double* cb = a.cellbuf + 7 * tb.cell_off;
  const double mu0 = cb[y], mu1 = cb[ldx + y], mu2 = cb[2 * ldx + y], mu3 = cb[3 * ldx + y], mu4 = cb[4 * ldx + y];
  const double rho = double(Real(cb[5 * ldx + y]) - xi * Real(cb[6 * ldx + y]));
  const double Bmu = double(J[1]) * (I[2] * mu0 + I[3] * mu2) + double(J[2]) * (I[2] * mu1 + I[3] * mu3) +
                     double(J[3]) * I[3] * mu4;
  const int64_t idx = tb.f_off + int64_t(s) * ldx + y;
  const double Kv = double(a.K[idx]);
  double out = a.cK * Kv + a.cJ * (adv - rho * Kv + Bmu);
  double accv = 0.0;
  if (a.add_acc || (a.cA != 0.0 && !a.acc_init)) accv = double(a.acc_in[idx]);
  if (a.add_acc) out += accv;
  if (a.cA != 0.0) a.acc_out[idx] = Real((a.acc_init ? 0.0 : accv) + a.cA * Kv);
  a.out[idx] = Real(out);
}

// dL/dtau[tube] += sum_x tau_acc[x] (fixed-order tree reduction).
__global__ __launch_bounds__(256) void tau_reduce_kernel(const TubeDev* tubes, int tube, const double* tau_acc,
                                                         double* dL_dtau) {
  __shared__ double red[256];
  const TubeDev& tb = tubes[tube];
  double s = 0.0;
  for (int x = threadIdx.x; x < tb.nx; x += blockDim.x) s += tau_acc[tb.cell_off + x];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) dL_dtau[tube] += red[0];
}

// Adjoint of the diagnostic fields (N0, Nz, T00, T0z, Tzz, e, n, v, T, |N|)
// of a state: lambda_s(x) = B_s . dL/dm(x).
template <typename Real>
__global__ __launch_bounds__(256) void fields_adjoint_kernel(const TubeDev* tubes, int tube, const Real* jtab_all,
                                                             const double* itab_all, const double* rec,
                                                             const double* dfields, int64_t ld, Real* lambda) {
  const TubeDev& tb = tubes[tube];
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= tb.nx) return;
  const int64_t ldx = tb.ldx;
  double m[5], mb[5];
  for (int c = 0; c < 5; ++c) {
    m[c] = rec[tb.rec_off + c * ldx + y];
    mb[c] = dfields[c * ld + y];
  }
  const Macro M = landau(m);
  landau_adjoint(m, M, dfields[5 * ld + y], dfields[7 * ld + y], 0.0, 0.0, dfields[6 * ld + y], dfields[8 * ld + y],
                 mb);
  const double nabs = sqrt((m[0] - m[1]) * (m[0] + m[1]));
  const double nab = dfields[9 * ld + y];
  mb[0] += nab * m[0] / nabs;
  mb[1] -= nab * m[1] / nabs;
  const Real* jtab = jtab_all + int64_t(tb.jrow) * kJStride;
  const double* itab = itab_all + int64_t(tb.irow) * kIStride;
  Real* lam = lambda + tb.f_off;
  for (int i = 0; i < tb.qp; ++i) {
    const double* I = itab + i * kIStride;
    const double c1 = I[2] * mb[0] + I[3] * mb[2], c2 = I[2] * mb[1] + I[3] * mb[3], c3 = I[3] * mb[4];
    for (int j = 0; j < tb.qx; ++j) {
      const Real* J = jtab + j * kJStride;
      lam[int64_t(i * tb.qx + j) * ldx + y] = Real(double(J[1]) * c1 + double(J[2]) * c2 + double(J[3]) * c3);
    }
  }
}

// Initial-state adjoint, pass 1: per block and side, sum over cells of
// Db[i][k] = sum_j lambda0_s(x) P_k(xi_j)  (the adjoint of the coefficients
// D[i][k] of the side's equilibrium).
template <typename Real, int QPT, int NVT>
__global__ __launch_bounds__(256) void init_adjoint_partial_kernel(const TubeDev* tubes, int tube, const Real* jtab_all,
                                                                   const Real* lambda0, double* partials) {
  __shared__ double red[2][256];
  const TubeDev& tb = tubes[tube];
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = y < tb.nx;
  const int side = valid ? (left_of_split(tb, y) ? 0 : 1) : 0;
  const Real* jtab = jtab_all + int64_t(tb.jrow) * kJStride;
  const Real* lam = lambda0 + tb.f_off;
  constexpr int NC = QPT * (NVT + 1);
  for (int c = 0; c < NC; ++c) {
    const int i = c / (NVT + 1), k = c % (NVT + 1);
    double v = 0.0;
    if (valid && i < tb.qp && k <= tb.nv)
      for (int j = 0; j < tb.qx; ++j)
        v += double(lam[int64_t(i * tb.qx + j) * tb.ldx + y]) * double(jtab[j * kJStride + 4 + k]);
    red[0][threadIdx.x] = side == 0 ? v : 0.0;
    red[1][threadIdx.x] = side == 1 ? v : 0.0;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        red[0][threadIdx.x] += red[0][threadIdx.x + w];
        red[1][threadIdx.x] += red[1][threadIdx.x + w];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      partials[(int64_t(blockIdx.x) * 2 + 0) * NC + c] = red[0][0];
      partials[(int64_t(blockIdx.x) * 2 + 1) * NC + c] = red[1][0];
    }
    __syncthreads();
  }
}

// Pass 2: one lane per side sums the block partials in order and applies the
// adjoint of the projection and of (P, n, u) -> (n, T = P/n, gamma, u).
template <int QPT, int NVT>
__global__ void init_adjoint_final_kernel(const TubeDev* tubes, int tube, const double* itab_all,
                                          const double* aux_d, int aux_pairs, const double* sides,
                                          const double* partials, int nblocks, double* grad_out) {
  const int side = threadIdx.x;
  if (side >= 2) return;
  const TubeDev& tb = tubes[tube];
  constexpr int NC = QPT * (NVT + 1);
  double Db[QPT][NVT + 1];
  for (int c = 0; c < NC; ++c) {
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) v += partials[(int64_t(b) * 2 + side) * NC + c];
    Db[c / (NVT + 1)][c % (NVT + 1)] = v;
  }
  const double* st = sides + 6 * tube + 3 * side;
  const double P = st[0], n = st[1], u = st[2];
  const double T = P / n, gamma = sqrt(1.0 + u * u);
  double nb = 0.0, Tb = 0.0, gb = 0.0, ub = 0.0;
  feq_coefficients_adjoint<QPT, NVT>(n, T, gamma, u, tb.T0, tb.qp, tb.np, tb.nv,
                                     as_const(itab_all) + int64_t(tb.irow) * kIStride, as_const(aux_d), aux_pairs,
                                     Db, nb, Tb, gb, ub);
  grad_out[3 * side + 0] = Tb / n;                  // dL/dP
  grad_out[3 * side + 1] = nb - Tb * P / (n * n);   // dL/dn
  grad_out[3 * side + 2] = ub + gb * u / gamma;     // dL/du
}

// High-order form, pass 1: per block and side the sums over the block's
// cells of lambda0 at every point (i, j), row c = i q_xi + j, in cell order.
template <typename Real>
__global__ __launch_bounds__(256) void init_adjoint_partial_high_kernel(const TubeDev* tubes, int tube,
                                                                        const Real* lambda0, double* partials,
                                                                        int part_stride) {
  const TubeDev& tb = tubes[tube];
  const int x0 = blockIdx.x * 256, x1 = min(x0 + 256, tb.nx);
  const Real* lam = lambda0 + tb.f_off;
  const int nc = tb.qp * tb.qx;
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    double v[2] = {0.0, 0.0};
    const Real* row = lam + int64_t(c) * tb.ldx;
    for (int x = x0; x < x1; ++x) v[left_of_split(tb, x) ? 0 : 1] += double(row[x]);
    partials[(int64_t(blockIdx.x) * 2 + 0) * part_stride + c] = v[0];
    partials[(int64_t(blockIdx.x) * 2 + 1) * part_stride + c] = v[1];
  }
}

// High-order form, pass 2: one workgroup per side sums the block partials in
// order into the point weights W of the side's (uniform) equilibrium, then
// applies the adjoint of the fused projection (as in the stage's reduction;
// the threads split the (node, pair) products and their partial sums are added
// in thread order) and of (P, n, u) -> (n, T = P/n, gamma, u).
__global__ __launch_bounds__(256) void init_adjoint_final_high_kernel(const TubeDev* tubes, int tube,
                                                                      const double* itab_all, const double* ztab,
                                                                      const double* sides, const double* partials,
                                                                      int nblocks, int part_stride,
                                                                      double* grad_out) {
  __shared__ double W[kMaxQp * kMaxQxHigh];
  __shared__ double red[4][256];
  const int side = blockIdx.x, t = threadIdx.x;
  const TubeDev& tb = tubes[tube];
  const int qx = tb.qx, qp = tb.qp, np = tb.np, half = (qx + 1) / 2, nc = qp * qx;
  for (int c = t; c < nc; c += blockDim.x) {
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) v += partials[(int64_t(b) * 2 + side) * part_stride + c];
    W[c] = v;
  }
  __syncthreads();
  const double* st = sides + 6 * tube + 3 * side;
  const double P = st[0], n = st[1], u = st[2];
  const double T = P / n, gamma = sqrt(1.0 + u * u);
  const double pref = n / (4.0 * T * tb.T0 * tb.T0), r = T / tb.T0;
  const double* zt = ztab + tb.z_off;
  const int zj = tb.zj, zb = tb.zb;
  double part[4] = {0.0, 0.0, 0.0, 0.0};  // prefb, rb, gamma-bar, u-bar
  for (int pb = t; pb < qp * zb; pb += blockDim.x) {
    const int i = pb / zb, b = pb % zb;
    const double* Wi = W + i * qx;
    double ev = 0.0, od = 0.0;
    for (int j = 0; j < half; ++j) {
      const int jm = qx - 1 - j;
      const double ce = jm == j ? 0.5 * Wi[j] : 0.5 * (Wi[j] + Wi[jm]);
      const double co = jm == j ? 0.5 * Wi[j] : 0.5 * (Wi[j] - Wi[jm]);
      ev += zt[j * zb + b] * ce;
      od += zt[(zj + j) * zb + b] * co;
    }
    const double* L = itab_all + int64_t(tb.irow + i) * kIStride + 4;
    const double xa = zt[2 * zj * zb + b];
    const double yp = 1.0 / (gamma - xa * u), ym = 1.0 / (gamma + xa * u);
    const double qpl = 1.0 - r * yp, qmi = 1.0 - r * ym;
    double sp = L[np], dsp = 0.0, sm = L[np], dsm = 0.0;
    for (int l = np - 1; l >= 0; --l) {
      dsp = dsp * qpl + sp;
      sp = sp * qpl + L[l];
      dsm = dsm * qmi + sm;
      sm = sm * qmi + L[l];
    }
    const double yp2 = yp * yp, ym2 = ym * ym;
    const double gp = yp2 * sp, gm = ym2 * sm;
    part[0] += ev * (gp + gm) + od * (gp - gm);
    const double gpb = pref * (ev + od), gmb = pref * (ev - od);
    double ypb = gpb * 2.0 * yp * sp, ymb = gmb * 2.0 * ym * sm;
    const double qpb = gpb * yp2 * dsp, qmb = gmb * ym2 * dsm;
    part[1] -= qpb * yp + qmb * ym;
    ypb -= qpb * r;
    ymb -= qmb * r;
    part[2] -= ypb * yp2 + ymb * ym2;
    part[3] += ypb * xa * yp2 - ymb * xa * ym2;
  }
  for (int q = 0; q < 4; ++q) red[q][t] = part[q];
  __syncthreads();
  if (t != 0) return;
  double tot[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < int(blockDim.x); ++k)
    for (int q = 0; q < 4; ++q) tot[q] += red[q][k];
  double nb = 0.0, Tb = 0.0;
  feq_adjoint_finish(n, T, tb.T0, tot[0], tot[1], nb, Tb);
  const double gb = tot[2], ub = tot[3];
  grad_out[3 * side + 0] = Tb / n;                  // dL/dP
  grad_out[3 * side + 1] = nb - Tb * P / (n * n);   // dL/dn
  grad_out[3 * side + 2] = ub + gb * u / gamma;     // dL/du
}

template <typename Real, int QPT, int NVT>
hipError_t adjoint_stage_t(int nx, int Q, const AdjArgs<Real>& a, hipStream_t s) {
  const int nred = (nx + red_cells<Real>() - 1) / red_cells<Real>(), nfx = (nx + 1 + 255) / 256;
  hipLaunchKernelGGL((adj_reduce_faces_kernel<Real, QPT, NVT>), dim3(nred + nfx * Q), dim3(256), 0, s, a, nred, nfx);
  hipLaunchKernelGGL(adj_combine_kernel<Real>, dim3((nx + 255) / 256, Q), dim3(256), 0, s, a);
  return hipGetLastError();
}

// The high-order form: its reduction in a launch of its own (up to 64 KB of
// LDS for the weights of a node), then the face blocks alone and the combine.
template <typename Real>
hipError_t adjoint_stage_high(int nx, int Q, const AdjArgs<Real>& a, hipStream_t s) {
  const int nred = (nx + red_cells<Real>() - 1) / red_cells<Real>(), nfx = (nx + 1 + 255) / 256;
  hipLaunchKernelGGL(adj_reduce_high_kernel<Real>, dim3(nred), dim3(256), 0, s, a);
  hipLaunchKernelGGL((adj_reduce_faces_kernel<Real, 3, 5>), dim3(nfx * Q), dim3(256), 0, s, a, 0, nfx);
  hipLaunchKernelGGL(adj_combine_kernel<Real>, dim3((nx + 255) / 256, Q), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename Real>
hipError_t adjoint_stage_real(int qpt, int nvt, int nx, int Q, const void* args, hipStream_t s) {
  const AdjArgs<Real>& a = *static_cast<const AdjArgs<Real>*>(args);
  if (qpt == 3 && nvt == 5) return adjoint_stage_t<Real, 3, 5>(nx, Q, a, s);
  if (qpt == 4 && nvt == 5) return adjoint_stage_t<Real, 4, 5>(nx, Q, a, s);
  if (qpt == 8 && nvt == 7) return adjoint_stage_t<Real, 8, 7>(nx, Q, a, s);
  if (nvt == kNvtHigh) return adjoint_stage_high<Real>(nx, Q, a, s);
  return hipErrorInvalidValue;
}

template <typename Real, int QPT, int NVT>
hipError_t initial_adjoint_t(const TubeDev* tubes, int tube, int nx, const void* jtab, const double* itab,
                             const double* aux_d, int aux_pairs, const double* sides, const void* lambda0,
                             double* partials, double* grad_out, hipStream_t s) {
  const int nblocks = (nx + 255) / 256;
  hipLaunchKernelGGL((init_adjoint_partial_kernel<Real, QPT, NVT>), dim3(nblocks), dim3(256), 0, s, tubes, tube,
                     static_cast<const Real*>(jtab), static_cast<const Real*>(lambda0), partials);
  hipLaunchKernelGGL((init_adjoint_final_kernel<QPT, NVT>), dim3(1), dim3(64), 0, s, tubes, tube, itab, aux_d,
                     aux_pairs, sides, partials, nblocks, grad_out);
  return hipGetLastError();
}

template <typename Real>
hipError_t initial_adjoint_real(int qpt, int nvt, const TubeDev* tubes, int tube, int nx, const void* jtab,
                                const double* itab, const double* aux_d, int aux_pairs, const double* ztab,
                                const double* sides, const void* lambda0, double* partials, int part_stride,
                                double* grad_out, hipStream_t s) {
  if (nvt == kNvtHigh) {
    const int nblocks = (nx + 255) / 256;
    hipLaunchKernelGGL(init_adjoint_partial_high_kernel<Real>, dim3(nblocks), dim3(256), 0, s, tubes, tube,
                       static_cast<const Real*>(lambda0), partials, part_stride);
    hipLaunchKernelGGL(init_adjoint_final_high_kernel, dim3(2), dim3(256), 0, s, tubes, tube, itab, ztab, sides,
                       partials, nblocks, part_stride, grad_out);
    return hipGetLastError();
  }
  if (qpt == 3 && nvt == 5)
    return initial_adjoint_t<Real, 3, 5>(tubes, tube, nx, jtab, itab, aux_d, aux_pairs, sides, lambda0, partials,
                                         grad_out, s);
  if (qpt == 4 && nvt == 5)
    return initial_adjoint_t<Real, 4, 5>(tubes, tube, nx, jtab, itab, aux_d, aux_pairs, sides, lambda0, partials,
                                         grad_out, s);
  if (qpt == 8 && nvt == 7)
    return initial_adjoint_t<Real, 8, 7>(tubes, tube, nx, jtab, itab, aux_d, aux_pairs, sides, lambda0, partials,
                                         grad_out, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_adjoint_stage(int prec_fp32, int qpt, int nvt, int nx, int Q, const void* args, hipStream_t stream) {
  return prec_fp32 ? adjoint_stage_real<float>(qpt, nvt, nx, Q, args, stream)
                   : adjoint_stage_real<double>(qpt, nvt, nx, Q, args, stream);
}

hipError_t launch_tau_reduce(const TubeDev* tubes, int tube, const double* tau_acc, double* dL_dtau,
                             hipStream_t stream) {
  hipLaunchKernelGGL(tau_reduce_kernel, dim3(1), dim3(256), 0, stream, tubes, tube, tau_acc, dL_dtau);
  return hipGetLastError();
}

hipError_t launch_fields_adjoint(int prec_fp32, const TubeDev* tubes, int tube, int nx, const void* jtab,
                                 const double* itab, const double* rec, const double* dfields, int64_t ld,
                                 void* lambda, hipStream_t stream) {
  const dim3 grid((nx + 255) / 256);
  if (prec_fp32)
    hipLaunchKernelGGL(fields_adjoint_kernel<float>, grid, dim3(256), 0, stream, tubes, tube,
                       static_cast<const float*>(jtab), itab, rec, dfields, ld, static_cast<float*>(lambda));
  else
    hipLaunchKernelGGL(fields_adjoint_kernel<double>, grid, dim3(256), 0, stream, tubes, tube,
                       static_cast<const double*>(jtab), itab, rec, dfields, ld, static_cast<double*>(lambda));
  return hipGetLastError();
}

hipError_t launch_initial_adjoint(int prec_fp32, int qpt, int nvt, const TubeDev* tubes, int tube, int nx,
                                  const void* jtab, const double* itab, const double* aux_d, int aux_pairs,
                                  const double* ztab, const double* sides, const void* lambda0, double* partials,
                                  int nblocks_max, int part_stride, double* grad_out, hipStream_t stream) {
  if ((nx + 255) / 256 > nblocks_max) return hipErrorInvalidValue;
  return prec_fp32 ? initial_adjoint_real<float>(qpt, nvt, tubes, tube, nx, jtab, itab, aux_d, aux_pairs, ztab,
                                                 sides, lambda0, partials, part_stride, grad_out, stream)
                   : initial_adjoint_real<double>(qpt, nvt, tubes, tube, nx, jtab, itab, aux_d, aux_pairs, ztab,
                                                  sides, lambda0, partials, part_stride, grad_out, stream);
}

}  // namespace rlb
