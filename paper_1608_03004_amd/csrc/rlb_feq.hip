// High-order equilibrium pre-pass (tubes with 7 < n_v <= 63, q_xi <= 64): the
// truncated expansion of the equilibrium (eq. feqtrunc, truncated at N_p and
// N_v as the section on the equilibrium expansion describes) at every
// quadrature point of every cell, for the stage kernel to read.
//
// With n_v this large a cell has about as many expansion coefficients as
// polar nodes, so the projection onto the Legendre basis and the evaluation at
// the nodes are fused into one contraction per radial node i:
//   F_eq(p_i, xi_j) = pref sum_a G_i(x_a) Z(x_a, xi_j),
//   G_i(x) = y^2 sum_{l <= n_p} L_l(p_i) (1 - r y)^l,   y = 1 / (gamma - x u),
//   Z(x, xi) = w(x) sum_{k <= n_v} (2k+1)/2 P_k(x) P_k(xi),
// with pref = n / (4 T T0^2) and r = T / T0, over an auxiliary Gauss-Legendre
// rule of 2B points +-x_b.  This is the same orthogonal projection of the
// Maxwell-Juettner distribution that the low-order kernels form as
// coefficients, with the basis sum done first.  The rule and the polar nodes
// are symmetric: with E_b = pref (G(x_b) + G(-x_b)), O_b = pref (G(x_b) -
// G(-x_b)) and j' the mirror node of j (xi_j' = -xi_j),
//   F_j + F_j' = sum_b Ze[j][b] E_b,   F_j - F_j' = sum_b Zo[j][b] O_b,
// two [ceil(q_xi/2) x B] x [B x cells] products per radial node.  They run in
// FP64 on the matrix cores (v_mfma_f64_16x16x4f64) in both precisions: the
// entries of Z grow like n_v^2 and cancel, so only the result is rounded to
// the state's precision.
//
// Work decomposition: a workgroup takes one tile of cells (and, when the grid
// has a second dimension, every gridDim.y-th radial node); its four waves take
// 16 cells at a time.  Lane l owns cell l % 16 and evaluates E_b, O_b for
// b = 4s + l / 16, which is the B-operand layout of the MFMA (B[k][n] in lane
// 16k + n); the A operands Ze, Zo (A[m][k] in lane 16k + m) are staged in LDS
// once per tile; result register r of lane l is row 4r + l / 16, column
// l % 16.
#include <hip/hip_runtime.h>

#include "rlb_device.h"
#include "rlb_internal.h"

namespace rlb {
namespace {

using namespace dev;

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kMaxS = high_aux_pairs(kMaxNvHigh) / 4;             // MFMA K-steps
constexpr int kMaxZj = high_rows(kMaxQxHigh);                      // rows of Ze, Zo
constexpr int kLdsLd = 4 * kMaxS + 1;                              // padded LDS row (doubles)

template <typename Real>
__global__ __launch_bounds__(256) void feq_kernel(FeqArgs<Real> a) {
  __shared__ double zs[2 * kMaxZj * kLdsLd + 4 * kMaxS];  // Ze rows, Zo rows, x_b
  const int t = threadIdx.x, w = t / 64, l = t % 64, col = l % 16, quarter = l / 16;
  for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
    const WorkItem wi = a.items[item];
    const TubeDev& tb = a.tubes[wi.tube];
    if (a.rec == nullptr && !a.tube_mask[wi.tube]) continue;
    if (int(blockIdx.y) >= tb.qp) continue;
    const int zj = tb.zj, zb = tb.zb, ns = zb / 4, ld = zb + 1;
    __syncthreads();  // the previous item's reads of zs are done
    const double* zt = a.ztab + tb.z_off;
    for (int e = t; e < 2 * zj * zb; e += blockDim.x) zs[(e / zb) * ld + e % zb] = zt[e];
    double* xs = zs + 2 * zj * ld;
    for (int e = t; e < zb; e += blockDim.x) xs[e] = zt[2 * zj * zb + e];
    __syncthreads();
    const int np = tb.np, qx = tb.qx, half = (qx + 1) / 2;
    const double T0 = tb.T0;
    const int64_t ldx = tb.ldx;
    Real* out = a.out + tb.f_off;
    for (int c0 = 16 * w; c0 < a.tile; c0 += 64) {
      if (wi.x0 + c0 >= tb.nx) break;  // wave-uniform
      const int x = wi.x0 + c0 + col;
      const bool valid = x < tb.nx;
      const int xc = valid ? x : tb.nx - 1;
      // macroscopic state of the cell: the Landau frame of its record, or the
      // initial state of its side
      double n, T, gam, u;
      if (a.rec != nullptr) {
        double m[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) m[c] = a.rec[tb.rec_off + c * ldx + xc];
        const Macro M = landau(m);
        n = M.n;
        T = M.T;
        gam = M.gamma;
        u = M.u;
      } else {
        const double* st = a.sides + 6 * wi.tube + (left_of_split(tb, xc) ? 0 : 3);
        n = st[1];
        T = st[0] / st[1];
        u = st[2];
        gam = sqrt(1.0 + u * u);
      }
      const double r = T / T0, pref = n / (4.0 * T * T0 * T0);
      // y at +-x_b for this lane's pairs b = 4s + quarter (shared by all nodes)
      double yp[kMaxS], ym[kMaxS];
#pragma unroll
      for (int s = 0; s < kMaxS; ++s) {
        yp[s] = 0.0;
        ym[s] = 0.0;
        if (s < ns) {
          const double xb = xs[4 * s + quarter];
          yp[s] = 1.0 / (gam - xb * u);
          ym[s] = 1.0 / (gam + xb * u);
        }
      }
      for (int node = blockIdx.y; node < tb.qp; node += gridDim.y) {
        const double* Lrow = a.itab + int64_t(tb.irow + node) * kIStride + 4;  // L_l(p_node)
        double E[kMaxS], O[kMaxS];
#pragma unroll
        for (int s = 0; s < kMaxS; ++s) {
          E[s] = 0.0;
          O[s] = 0.0;
          if (s < ns) {
            const double qpl = 1.0 - r * yp[s], qmi = 1.0 - r * ym[s];
            double sp = Lrow[np], sm = Lrow[np];
            for (int k = np - 1; k >= 0; --k) {
              sp = sp * qpl + Lrow[k];
              sm = sm * qmi + Lrow[k];
            }
            const double gp = yp[s] * yp[s] * sp, gm = ym[s] * ym[s] * sm;
            E[s] = pref * (gp + gm);
            O[s] = pref * (gp - gm);
          }
        }
        Real* orow = out + x;
        for (int jt = 0; jt < zj / 16; ++jt) {
          d4 ce = {0.0, 0.0, 0.0, 0.0}, co = {0.0, 0.0, 0.0, 0.0};
          const double* ae = zs + (jt * 16 + col) * ld + quarter;
          const double* ao = ae + zj * ld;
#pragma unroll
          for (int s = 0; s < kMaxS; ++s) {
            if (s < ns) {
              ce = __builtin_amdgcn_mfma_f64_16x16x4f64(ae[4 * s], E[s], ce, 0, 0, 0);
              co = __builtin_amdgcn_mfma_f64_16x16x4f64(ao[4 * s], O[s], co, 0, 0, 0);
            }
          }
          if (valid) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
              const int j = jt * 16 + 4 * rr + quarter;
              if (j < half) {
                const int jm = qx - 1 - j;
                orow[int64_t(node * qx + j) * ldx] = Real(0.5 * (ce[rr] + co[rr]));
                if (jm != j) orow[int64_t(node * qx + jm) * ldx] = Real(0.5 * (ce[rr] - co[rr]));
              }
            }
          }
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_feq(int prec_fp32, const LaunchShape& ls, const void* args, hipStream_t stream) {
  const dim3 grid(ls.grid, ls.nodes);
  if (prec_fp32)
    hipLaunchKernelGGL(feq_kernel<float>, grid, dim3(256), 0, stream, *static_cast<const FeqArgs<float>*>(args));
  else
    hipLaunchKernelGGL(feq_kernel<double>, grid, dim3(256), 0, stream, *static_cast<const FeqArgs<double>*>(args));
  return hipGetLastError();
}

}  // namespace rlb
