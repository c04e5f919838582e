// High-order equilibrium pre-pass (tubes with 7 < n_v < q_xi <= 256): the
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
// l % 16.  Each K-step's E_b, O_b (one reciprocal, two Horner chains over
// the node's Laguerre values, held in scalar registers for a compile-time
// N_p) are formed just before the four products that consume them.  The two
// denominators share the reciprocal: (gamma - x u)(gamma + x u) =
// 1 + u^2 (1 - x^2) (as gamma^2 = 1 + u^2), which is at least 1, so
// 1/(gamma -+ x u) = (gamma +- x u) / (1 + u^2 (1 - x^2)); the factor pref / 2
// is applied to the results instead of to every E_b, O_b.  FP64
// vector instructions do not issue while the FP64 matrix pipe is busy, so a
// step costs its products plus that vector work, and the register budget is
// capped at 128 so that four waves per SIMD keep the matrix pipe fed.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "rlb_device.h"
#include "rlb_internal.h"

namespace rlb {
namespace {

using namespace dev;

typedef double d4 __attribute__((ext_vector_type(4)));

// Three variants by the number TT of 16-row tiles of Ze, Zo (the launch's
// largest tube): TT = 2 for q_xi <= 64 (n_v <= 63, four waves per SIMD),
// TT = 4 for q_xi <= 128 (n_v <= 127; 58.8 KB of tables in LDS, two waves per
// SIMD) and TT = 8 for q_xi <= 256 (n_v <= 255): its tables (182 KB) exceed
// the LDS, so the rows are split into blocks of RT = 4 tiles over the grid's
// third dimension, each block staging its 64 rows (91.8 KB, one wave per
// SIMD) and forming the B operands itself.
template <int TT>
struct FeqShape {
  static constexpr int RT = TT < 4 ? TT : 4;                // row tiles per block
  static constexpr int kMaxNv = TT == 2 ? 63 : (TT == 4 ? 127 : kMaxNvHigh);
  static constexpr int kMaxS = high_aux_pairs(kMaxNv) / 4;  // MFMA K-steps
  static constexpr int kMaxZj = 16 * RT;                    // rows of Ze, Zo per block
  static constexpr int kLdsLd = 4 * kMaxS + 1;              // padded LDS row (doubles)
  static constexpr int kWaves = TT == 2 ? 4 : (TT == 4 ? 2 : 1);
};
static_assert(16 * 8 == high_rows(kMaxQxHigh), "the largest variant covers the polar order limit");
static_assert(FeqShape<2>::kMaxNv + 1 == 64 && FeqShape<2>::kMaxZj == high_rows(64), "the smallest variant: q_xi <= 64");

// 1/d for d > 0 (normal): hardware reciprocal refined by two Newton steps
// (the error of each step is the square of the previous one's).
__device__ inline double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return r;
}

template <typename Real, int TT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FeqShape<TT>::kWaves)))
void feq_kernel(FeqArgs<Real> a) {
  constexpr int RT = FeqShape<TT>::RT;
  constexpr int kMaxS = FeqShape<TT>::kMaxS, kMaxZj = FeqShape<TT>::kMaxZj, kLdsLd = FeqShape<TT>::kLdsLd;
  const int jt0 = RT * int(blockIdx.z);  // first row tile of this block
  __shared__ double zs[2 * kMaxZj * kLdsLd + 4 * kMaxS];  // Ze rows, Zo rows, x_b
  const int t = threadIdx.x, w = t / 64, l = t % 64, col = l % 16, quarter = l / 16;
  const cptr<WorkItem> items = as_const(a.items);
  const cptr<TubeDev> tubes = as_const(a.tubes);
  const cptr<double> itab = as_const(a.itab);
  for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
    const int wtube = items[item].tube, wx0 = items[item].x0;
    const cptr<TubeDev> tb = tubes + wtube;
    if (a.rec == nullptr && !as_const(a.tube_mask)[wtube]) continue;
    const int qp = tb->qp, nx = tb->nx;
    if (int(blockIdx.y) >= qp) continue;
    const int zj = tb->zj, zb = tb->zb, ns = zb / 4, ld = zb + 1;
    if (16 * jt0 >= zj) continue;  // the tube has no rows in this block
    // this block's rows: Ze rows 16 jt0 .. 16 jt0 + zl - 1, then the same Zo rows
    const int zl = min(kMaxZj, zj - 16 * jt0);
    __syncthreads();  // the previous item's reads of zs are done
    const double* zt = a.ztab + tb->z_off;
    for (int e = t; e < 2 * zl * zb; e += blockDim.x) {
      const int r = e / zb, b = e % zb;
      const int src = r < zl ? 16 * jt0 + r : zj + 16 * jt0 + (r - zl);
      zs[r * ld + b] = zt[src * zb + b];
    }
    double* xs = zs + 2 * zl * ld;
    for (int e = t; e < zb; e += blockDim.x) xs[e] = zt[2 * zj * zb + e];
    __syncthreads();
    const int np = tb->np, qx = tb->qx, half = (qx + 1) / 2, njt = zl / 16, irow = tb->irow;
    const double T0 = tb->T0, z_min = tb->z_min, dz = tb->dz;
    const int64_t ldx = tb->ldx, rec_off = tb->rec_off;
    Real* out = a.out + tb->f_off;
    for (int c0 = 16 * w; c0 < a.tile; c0 += 64) {
      if (wx0 + c0 >= nx) break;  // wave-uniform
      const int x = wx0 + c0 + col;
      const bool valid = x < nx;
      const int xc = valid ? x : nx - 1;
      // macroscopic state of the cell: the Landau frame of its record, or the
      // initial state of its side
      double n, T, gam, u;
      if (a.rec != nullptr) {
        double m[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) m[c] = a.rec[rec_off + c * ldx + xc];
        const Macro M = landau(m);
        n = M.n;
        T = M.T;
        gam = M.gamma;
        u = M.u;
      } else {
        const cptr<double> st = as_const(a.sides) + 6 * wtube + (left_of_split(z_min, dz, xc) ? 0 : 3);
        n = st[1];
        T = st[0] / st[1];
        u = st[2];
        gam = sqrt(1.0 + u * u);
      }
      const double r = T / T0, hpref = 0.5 * (n / (4.0 * T * T0 * T0)), u2 = u * u;
      for (int node = blockIdx.y; node < qp; node += gridDim.y) {
        const cptr<double> Lrow = itab + int64_t(irow + node) * kIStride + 4;  // L_l(p_node)
        // RT row tiles of Ze / Zo at most: 2 RT accumulators
        d4 ce[RT], co[RT];
#pragma unroll
        for (int jt = 0; jt < RT; ++jt) {
          ce[jt] = d4{0.0, 0.0, 0.0, 0.0};
          co[jt] = ce[jt];
        }
        const double* ae = zs + col * ld + quarter;
        const double* ao = ae + zl * ld;
        // the node's products for a compile-time radial order NP (the
        // Laguerre values of the node held in registers)
        auto products = [&](auto np_c) {
          constexpr int NP = decltype(np_c)::value;
          double Lv[NP + 1];
#pragma unroll
          for (int k = 0; k <= NP; ++k) Lv[k] = Lrow[k];
#pragma unroll
          for (int s = 0; s < kMaxS; ++s) {
            if (s < ns) {
              // B operands of this K-step: E_b, O_b of pair b = 4s + quarter
              const double xb = xs[4 * s + quarter];
              const double rd = recip(fma(u2, fma(-xb, xb, 1.0), 1.0));
              const double yp = fma(xb, u, gam) * rd, ym = fma(-xb, u, gam) * rd;
              const double qpl = 1.0 - r * yp, qmi = 1.0 - r * ym;
              double sp = Lv[NP], sm = Lv[NP];
#pragma unroll
              for (int k = NP - 1; k >= 0; --k) {
                sp = sp * qpl + Lv[k];
                sm = sm * qmi + Lv[k];
              }
              const double gp = yp * yp * sp, gm = ym * ym * sm;
              const double E = gp + gm, O = gp - gm;
              ce[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ae[4 * s], E, ce[0], 0, 0, 0);
              co[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ao[4 * s], O, co[0], 0, 0, 0);
#pragma unroll
              for (int jt = 1; jt < RT; ++jt) {
                if (njt > jt) {
                  ce[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ae[16 * jt * ld + 4 * s], E, ce[jt], 0, 0, 0);
                  co[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ao[16 * jt * ld + 4 * s], O, co[jt], 0, 0, 0);
                }
              }
            }
          }
        };
        switch (np) {
          case 0: products(std::integral_constant<int, 0>{}); break;
          case 1: products(std::integral_constant<int, 1>{}); break;
          case 2: products(std::integral_constant<int, 2>{}); break;
          case 3: products(std::integral_constant<int, 3>{}); break;
          case 4: products(std::integral_constant<int, 4>{}); break;
          case 5: products(std::integral_constant<int, 5>{}); break;
          case 6: products(std::integral_constant<int, 6>{}); break;
          default: products(std::integral_constant<int, 7>{}); break;
        }
        if (valid) {
          Real* orow = out + int64_t(node * qx) * ldx + x;
          auto put = [&](const d4& ce, const d4& co, int jt) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
              const int j = (jt0 + jt) * 16 + 4 * rr + quarter;
              if (j < half) {
                const int jm = qx - 1 - j;
                orow[int64_t(j) * ldx] = Real(hpref * (ce[rr] + co[rr]));
                if (jm != j) orow[int64_t(jm) * ldx] = Real(hpref * (ce[rr] - co[rr]));
              }
            }
          };
          put(ce[0], co[0], 0);
#pragma unroll
          for (int jt = 1; jt < RT; ++jt)
            if (njt > jt) put(ce[jt], co[jt], jt);
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_feq(int prec_fp32, const LaunchShape& ls, const void* args, hipStream_t stream) {
  const int rt = prec_fp32 ? static_cast<const FeqArgs<float>*>(args)->row_tiles
                           : static_cast<const FeqArgs<double>*>(args)->row_tiles;
  if (rt < 1 || rt > 8) return hipErrorInvalidValue;
  const dim3 grid(ls.grid, ls.nodes, rt <= 4 ? 1 : (rt + 3) / 4);
  auto go = [&](auto real_tag) {
    using Real = decltype(real_tag);
    const FeqArgs<Real>& a = *static_cast<const FeqArgs<Real>*>(args);
    if (rt <= 2)
      hipLaunchKernelGGL((feq_kernel<Real, 2>), grid, dim3(256), 0, stream, a);
    else if (rt <= 4)
      hipLaunchKernelGGL((feq_kernel<Real, 4>), grid, dim3(256), 0, stream, a);
    else
      hipLaunchKernelGGL((feq_kernel<Real, 8>), grid, dim3(256), 0, stream, a);
  };
  if (prec_fp32)
    go(float(0));
  else
    go(double(0));
  return hipGetLastError();
}

}  // namespace rlb
