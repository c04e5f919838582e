// HIP kernels for gfx950 (MI355X) of the relativistic lattice Boltzmann step
// (Blaga & Ambrus, arXiv:1608.03004).
//
// Data layout in HBM: structure of arrays F[s][x] per tube (s = i*q_xi + j),
// rows padded to a multiple of 64 elements so that a wavefront's 64 lanes
// (one cell each) load and store whole, aligned cache lines.  Per-cell moment
// records N0, Nz, T00, T0z, Tzz are FP64 arrays rec[5][x].
//
// One launch of `stage_kernel` is one SSP-RK3 stage for a list of (tube, tile)
// work items.  Per work item, each lane owns one cell and:
//   1. reads the FP64 moment record of the stage input (written by the
//      previous stage's epilogue -- the moments cost no extra pass over F);
//   2. solves the Landau matching in FP64;
//   3. projects the Maxwell-Juettner equilibrium onto the truncated basis with
//      an auxiliary Gauss-Legendre rule (coefficients D[i][k] in registers);
//   4. streams over the quadrature points in chunks of CJ points: the chunk's
//      F values of the tile plus a 3-cell halo go to LDS, each lane computes the
//      WENO5 value at its cell's left face (the tile's last face by CJ extra
//      lanes), then each lane forms advection + Anderson-Witting relaxation,
//      the RK combination, stores the result and accumulates the five moments
//      of the output (Kahan-compensated in FP32);
//   5. writes the output moment record.
// The outflow boundary (zero-gradient ghosts) is index clamping at load time.
#include <hip/hip_runtime.h>

#include "rlb_device.h"
#include "rlb_internal.h"

namespace rlb {
namespace {



using namespace dev;

// Points per chunk: 8 in FP32; 4 in FP64, where registers are scarcer.
template <typename Real>
constexpr int chunk_points() {
  return sizeof(Real) == 4 ? 8 : 4;
}

// Moment sums of one radial node's row of values, in the order the stage
// kernel's epilogue uses (plain sums within chunks of chunk_points() points,
// compensated across chunks), so that records computed from a stored state
// are bitwise equal to the records written while the state was produced.
template <typename Real, typename Get>
__device__ inline void row_moments(const Real* jtab, int qx, Get get, double& s0, double& s1, double& s2) {
  constexpr int CH = chunk_points<Real>();
  Acc<Real> a0, a1, a2;
  for (int j0 = 0; j0 < qx; j0 += CH) {
    Real p0 = Real(0), p1 = Real(0), p2 = Real(0);
    for (int c = 0; c < CH && j0 + c < qx; ++c) {
      const Real* J = jtab + (j0 + c) * kJStride;
      const Real v = get(j0 + c);
      p0 += J[1] * v;
      p1 += J[2] * v;
      p2 += J[3] * v;
    }
    a0.add(p0);
    a1.add(p1);
    a2.add(p2);
  }
  s0 = a0.value();
  s1 = a1.value();
  s2 = a2.value();
}

// WENO value at the face between tile positions k+2 and k+3 (left face of the
// cell stored at k+3), upwinded by the sign of xi.
template <typename Real>
__device__ inline Real face_value(const Real* row, int k, bool positive, Real eps) {
  if (positive) return weno5(row[k], row[k + 1], row[k + 2], row[k + 3], row[k + 4], eps);
  return weno5(row[k + 5], row[k + 4], row[k + 3], row[k + 2], row[k + 1], eps);
}

__device__ inline void raise_flag(unsigned* flag, unsigned bits) { atomicOr(flag, bits); }

template <typename Real>
__device__ inline void load_record(const double* rec, int64_t ldx, int x, double m[5]) {
#pragma unroll
  for (int c = 0; c < 5; ++c) m[c] = rec[c * ldx + x];
}

// ---------------------------------------------------------------------------
// Stage kernel
// ---------------------------------------------------------------------------
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

// Streaming loads of the distribution (read once per stage).
template <typename Real>
__device__ inline Real stream_load(const Real* p) {
#ifdef RLB_NT_LOADS
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

// Loads of one chunk: the tile's own cells for CH points (rows clamped to the
// last valid point, so every lane always issues the same loads) and, in
// wave 0, the 6-cell halo of all CH points with one instruction.
template <typename Real, int CH>
struct ChunkLoads {
  Real f[CH];
  Real halo;
};

template <typename Real, int TILE, int CH>
__device__ inline void issue_chunk(const Real* fin, int64_t ldx, int qx, int i, int j0, int xc, int t, int x0,
                                   int nx, ChunkLoads<Real, CH>& L) {
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int j = min(j0 + c, qx - 1);
    L.f[c] = stream_load(fin + int64_t(i * qx + j) * ldx + xc);
  }
  if (t < 64) {  // wave 0: lane h + 6c loads halo cell h of chunk point c
    const int c = min(t / 6, CH - 1), h = t % 6;
    const int j = min(j0 + c, qx - 1);
    const int hx = h < 3 ? max(x0 - 3 + h, 0) : min(x0 + TILE + (h - 3), nx - 1);
    L.halo = fin[int64_t(i * qx + j) * ldx + hx];
  }
}

// Moment sums over one radial node: plain sums within a chunk, Kahan-
// compensated across chunks in FP32 (plain FP64 sums in the FP64 form).
template <typename Real>
struct Moments3 {
  Acc<Real> a0, a1, a2;
};

template <typename Real, int TILE, int QPT, int NVT, bool HAS_FN, int CH>
__global__ __launch_bounds__(TILE) void stage_kernel(StageArgs<Real> a) {
  __shared__ Real tile[CH][TILE + 6];
  __shared__ Real faces[CH][TILE + 1];
  const int t = threadIdx.x;
  const cptr<WorkItem> items = as_const(a.items);
  const cptr<TubeDev> tubes = as_const(a.tubes);
  const bool xcd_map = (gridDim.x % kXcds) == 0 || gridDim.x == unsigned(a.nitems);
  for (int v = blockIdx.x; v < a.nitems; v += gridDim.x) {
    const int item = xcd_map ? xcd_item(v, a.nitems) : v;
    const int wtube = items[item].tube, wx0 = items[item].x0;
    const cptr<TubeDev> tbp = tubes + wtube;
    const int nx = tbp->nx, qx = tbp->qx, qp = tbp->qp;
    const int64_t ldx = tbp->ldx;
    const int x0 = wx0;
    const int x = x0 + t;
    const bool valid = x < nx;
    const int xc = valid ? x : nx - 1;
    const int64_t f_off = tbp->f_off;
    const Real* fin = a.fin + f_off;
    const Real* fn = a.fn + f_off;
    Real* fout = a.fout + f_off;
    const cptr<Real> jtab = as_const(a.jtab) + int64_t(tbp->jrow) * kJStride;
    const cptr<double> itab = as_const(a.itab) + int64_t(tbp->irow) * kIStride;

    // first chunk's loads go out before the per-cell prologue
    ChunkLoads<Real, CH> cur;
    issue_chunk<Real, TILE, CH>(fin, ldx, qx, 0, 0, xc, t, x0, nx, cur);

    // 1-2. moments of the stage input -> Landau frame (FP64)
    double m[5];
    const double* rin = a.rec_in + tbp->rec_off;
#pragma unroll
    for (int c = 0; c < 5; ++c) m[c] = rin[c * ldx + xc];
    const Macro M = landau(m);
    if (valid && !M.ok) raise_flag(a.flag, kFlagNonphysical);
    if (valid && fabs(M.v) > 0.95) raise_flag(a.flag, kFlagFastFlow);

    // 3. equilibrium coefficients and relaxation rate (gamma - xi u)/tau
    Real D[QPT][NVT + 1];
    feq_coefficients<Real, QPT, NVT>(Real(M.n), Real(M.T), Real(M.gamma), Real(M.u), Real(tbp->T0), qp, tbp->np,
                                     tbp->nv, itab, as_const(a.aux), a.aux_pairs, D);
    const double tau_inv = tbp->tau_inv;
    const Real g0 = Real(M.gamma * tau_inv), g1 = Real(M.u * tau_inv);
    const Real dt = Real(tbp->dt), dz_inv = Real(tbp->dz_inv), eps4 = Real(4.0 * tbp->weno_eps);
    const int stage = a.stage;
    // out = cn f^n + cs f_in + cs dt L
    const Real cn = stage == 1 ? Real(0) : (stage == 2 ? Real(0.75) : Real(1.0 / 3.0));
    const Real cs = stage == 1 ? Real(1) : (stage == 2 ? Real(0.25) : Real(2.0 / 3.0));
    const Real cdt = cs * dt;

    double mom[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
      if (i < qp) {
        Moments3<Real> acc;
        for (int j0 = 0; j0 < qx; j0 += CH) {
          const int cj = min(CH, qx - j0);
          // prefetch the next chunk (the next radial node's first chunk at the
          // end of this one; the very last chunk re-loads itself)
          ChunkLoads<Real, CH> nxt;
          {
            int in = i, jn = j0 + CH;
            if (jn >= qx) { in = i + 1; jn = 0; }
            if (in >= qp) { in = i; jn = j0; }
            issue_chunk<Real, TILE, CH>(fin, ldx, qx, in, jn, xc, t, x0, nx, nxt);
          }
#pragma unroll
          for (int c = 0; c < CH; ++c) tile[c][t + 3] = cur.f[c];
          if (t < 6 * CH) {
            const int c = t / 6, h = t % 6;
            tile[c][h < 3 ? h : TILE + h] = cur.halo;
          }
          __syncthreads();
          // f^n of this chunk, consumed after the faces
          Real nr[CH];
#pragma unroll
          for (int c = 0; c < CH; ++c) {
            if (HAS_FN) {
              const int j = min(j0 + c, qx - 1);
              nr[c] = stream_load(fn + int64_t(i * qx + j) * ldx + xc);
            } else {
              nr[c] = Real(0);
            }
          }
#pragma unroll
          for (int c = 0; c < CH; ++c) {
            const bool pos = jtab[min(j0 + c, qx - 1) * kJStride] >= Real(0);
            faces[c][t] = face_value(tile[c], t, pos, eps4);
          }
          if (t < CH) {  // the tile's right-most face, one chunk point per lane
            const bool pos = jtab[min(j0 + t, qx - 1) * kJStride] >= Real(0);
            faces[t][TILE] = face_value(tile[t], TILE, pos, eps4);
          }
          __syncthreads();
          Real p0 = Real(0), p1 = Real(0), p2 = Real(0);
#pragma unroll
          for (int c = 0; c < CH; ++c) {
            if (c < cj) {
              const cptr<Real> J = jtab + (j0 + c) * kJStride;
              const Real xi = J[0];
              Real feq = D[i][0];
#pragma unroll
              for (int kk = 1; kk <= NVT; ++kk) feq += D[i][kk] * J[4 + kk];
              const Real fr = cur.f[c];
              const Real adv = (faces[c][t + 1] - faces[c][t]) * (-xi * dz_inv);
              const Real rate = g0 - xi * g1;
              const Real L = adv - rate * (fr - feq);
              const Real out = HAS_FN ? cdt * L + (cs * fr + cn * nr[c]) : fr + dt * L;
              if (valid) fout[int64_t(i * qx + j0 + c) * ldx + x] = out;
              p0 += J[1] * out;
              p1 += J[2] * out;
              p2 += J[3] * out;
            }
          }
          acc.a0.add(p0);
          acc.a1.add(p1);
          acc.a2.add(p2);
          __syncthreads();
          cur = nxt;
        }
        const cptr<double> I = itab + i * kIStride;
        const double s0 = acc.a0.value(), s1 = acc.a1.value(), s2 = acc.a2.value();
        mom[0] += I[2] * s0;
        mom[1] += I[2] * s1;
        mom[2] += I[3] * s0;
        mom[3] += I[3] * s1;
        mom[4] += I[3] * s2;
      }
    }
    if (valid) {
      double* ro = a.rec_out + tbp->rec_off;
#pragma unroll
      for (int c = 0; c < 5; ++c) ro[c * ldx + x] = mom[c];
    }
  }
}

// ---------------------------------------------------------------------------
// Initial condition (eq. condinit): truncated equilibrium of the side state.
// ---------------------------------------------------------------------------
template <typename Real, int TILE, int QPT, int NVT>
__global__ __launch_bounds__(TILE) void init_kernel(InitArgs<Real> a) {
  const int t = threadIdx.x;
  for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
    const WorkItem wi = a.items[item];
    if (!a.tube_mask[wi.tube]) continue;
    const TubeDev& tb = a.tubes[wi.tube];
    const int x = wi.x0 + t;
    if (x >= tb.nx) continue;
    const double z = tb.z_min + (x + 0.5) * tb.dz;
    const double* st = a.sides + 6 * wi.tube + (z < 0.0 ? 0 : 3);
    const double P = st[0], n = st[1], u = st[2];
    const double T = P / n, gamma = sqrt(1.0 + u * u);
    const Real* jtab = a.jtab + int64_t(tb.jrow) * kJStride;
    const double* itab = a.itab + int64_t(tb.irow) * kIStride;
    Real D[QPT][NVT + 1];
    feq_coefficients<Real, QPT, NVT>(Real(n), Real(T), Real(gamma), Real(u), Real(tb.T0), tb.qp, tb.np, tb.nv,
                                     as_const(itab), as_const(a.aux), a.aux_pairs, D);
    Real* f = a.f + tb.f_off;
    double mom[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
      if (i < tb.qp) {
        Real* row = f + int64_t(i * tb.qx) * tb.ldx + x;
        for (int j = 0; j < tb.qx; ++j) {
          const Real* J = jtab + j * kJStride;
          Real F = D[i][0];
#pragma unroll
          for (int k = 1; k <= NVT; ++k) F += D[i][k] * J[4 + k];
          row[int64_t(j) * tb.ldx] = F;
        }
        double s0, s1, s2;
        row_moments<Real>(jtab, tb.qx, [&](int j) { return row[int64_t(j) * tb.ldx]; }, s0, s1, s2);
        const double* I = itab + i * kIStride;
        mom[0] += I[2] * s0;
        mom[1] += I[2] * s1;
        mom[2] += I[3] * s0;
        mom[3] += I[3] * s1;
        mom[4] += I[3] * s2;
      }
    }
    double* rec = a.rec + tb.rec_off;
#pragma unroll
    for (int c = 0; c < 5; ++c) rec[int64_t(c) * tb.ldx + x] = mom[c];
  }
}

// Moment records of an arbitrary state (after rlb_set_state).
template <typename Real>
__global__ __launch_bounds__(256) void moments_kernel(const TubeDev* tubes, const WorkItem* items, int nitems,
                                                      int tile, const Real* jtab_all, const double* itab_all,
                                                      const Real* f_all, double* rec_all) {
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const WorkItem wi = items[item];
    const TubeDev& tb = tubes[wi.tube];
    for (int t = threadIdx.x; t < tile; t += blockDim.x) {
      const int x = wi.x0 + t;
      if (x >= tb.nx) continue;
      const Real* jtab = jtab_all + int64_t(tb.jrow) * kJStride;
      const double* itab = itab_all + int64_t(tb.irow) * kIStride;
      const Real* f = f_all + tb.f_off;
      double mom[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      for (int i = 0; i < tb.qp; ++i) {
        const Real* row = f + int64_t(i * tb.qx) * tb.ldx + x;
        double s0, s1, s2;
        row_moments<Real>(jtab, tb.qx, [&](int j) { return row[int64_t(j) * tb.ldx]; }, s0, s1, s2);
        const double* I = itab + i * kIStride;
        mom[0] += I[2] * s0;
        mom[1] += I[2] * s1;
        mom[2] += I[3] * s0;
        mom[3] += I[3] * s1;
        mom[4] += I[3] * s2;
      }
      double* rec = rec_all + tb.rec_off;
      for (int c = 0; c < 5; ++c) rec[int64_t(c) * tb.ldx + x] = mom[c];
    }
  }
}

// Diagnostic fields from the moment record: N0..Tzz, e, n, v, T, |N|.
__global__ __launch_bounds__(256) void fields_kernel(const TubeDev* tubes, int tube, const double* rec_all,
                                                     double* out, int64_t ld, unsigned* flag) {
  const TubeDev& tb = tubes[tube];
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= tb.nx) return;
  double m[5];
  const double* rec = rec_all + tb.rec_off;
  for (int c = 0; c < 5; ++c) m[c] = rec[int64_t(c) * tb.ldx + x];
  const Macro M = landau(m);
  if (!M.ok) raise_flag(flag, kFlagNonphysical);
  for (int c = 0; c < 5; ++c) out[c * ld + x] = m[c];
  out[5 * ld + x] = M.e;
  out[6 * ld + x] = M.n;
  out[7 * ld + x] = M.v;
  out[8 * ld + x] = M.T;
  out[9 * ld + x] = sqrt((m[0] - m[1]) * (m[0] + m[1]));
}

// FP64 totals dz * sum_x {N0, T00, T0z} with a fixed-order tree reduction.
__global__ __launch_bounds__(256) void totals_kernel(const TubeDev* tubes, int tube, const double* rec_all,
                                                     double* out) {
  __shared__ double red[3][256];
  const TubeDev& tb = tubes[tube];
  const double* rec = rec_all + tb.rec_off;
  double s[3] = {0.0, 0.0, 0.0};
  for (int x = threadIdx.x; x < tb.nx; x += blockDim.x) {
    s[0] += rec[x];
    s[1] += rec[2 * int64_t(tb.ldx) + x];
    s[2] += rec[3 * int64_t(tb.ldx) + x];
  }
  for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) out[c] = red[c][0] * tb.dz;
}

// Plain streaming copy (16-byte vectors), for bandwidth calibration.
__global__ __launch_bounds__(256) void copy_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                   size_t n16) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n16; k += stride) dst[k] = src[k];
}

template <typename Real, int TILE, int QPT, int NVT>
hipError_t launch_stage_t(const LaunchShape& ls, const void* args, hipStream_t s) {
  const StageArgs<Real>& a = *static_cast<const StageArgs<Real>*>(args);
  constexpr int CH = chunk_points<Real>();
  if (a.stage == 1)
    hipLaunchKernelGGL((stage_kernel<Real, TILE, QPT, NVT, false, CH>), dim3(ls.grid), dim3(TILE), 0, s, a);
  else
    hipLaunchKernelGGL((stage_kernel<Real, TILE, QPT, NVT, true, CH>), dim3(ls.grid), dim3(TILE), 0, s, a);
  return hipGetLastError();
}

template <typename Real, int QPT, int NVT>
hipError_t launch_stage_tile(const LaunchShape& ls, const void* args, hipStream_t s) {
  switch (ls.tile) {
    case 128: return launch_stage_t<Real, 128, QPT, NVT>(ls, args, s);
    case 256: return launch_stage_t<Real, 256, QPT, NVT>(ls, args, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename Real>
hipError_t launch_stage_real(int qpt, int nvt, const LaunchShape& ls, const void* args, hipStream_t s) {
  if (qpt == 3 && nvt == 5) return launch_stage_tile<Real, 3, 5>(ls, args, s);
  if (qpt == 4 && nvt == 5) return launch_stage_tile<Real, 4, 5>(ls, args, s);
  if (qpt == 8 && nvt == 7) return launch_stage_tile<Real, 8, 7>(ls, args, s);
  return hipErrorInvalidValue;
}

template <typename Real, int QPT, int NVT>
hipError_t launch_init_t(const LaunchShape& ls, const void* args, hipStream_t s) {
  const InitArgs<Real>& a = *static_cast<const InitArgs<Real>*>(args);
  if (ls.tile == 128) {
    hipLaunchKernelGGL((init_kernel<Real, 128, QPT, NVT>), dim3(ls.grid), dim3(128), 0, s, a);
  } else if (ls.tile == 256) {
    hipLaunchKernelGGL((init_kernel<Real, 256, QPT, NVT>), dim3(ls.grid), dim3(256), 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_init_real(int qpt, int nvt, const LaunchShape& ls, const void* args, hipStream_t s) {
  if (qpt == 3 && nvt == 5) return launch_init_t<Real, 3, 5>(ls, args, s);
  if (qpt == 4 && nvt == 5) return launch_init_t<Real, 4, 5>(ls, args, s);
  if (qpt == 8 && nvt == 7) return launch_init_t<Real, 8, 7>(ls, args, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_stage(int prec_fp32, int qpt, int nvt, const LaunchShape& ls, const void* args,
                        hipStream_t stream) {
  return prec_fp32 ? launch_stage_real<float>(qpt, nvt, ls, args, stream)
                   : launch_stage_real<double>(qpt, nvt, ls, args, stream);
}

hipError_t launch_init(int prec_fp32, int qpt, int nvt, const LaunchShape& ls, const void* args,
                       hipStream_t stream) {
  return prec_fp32 ? launch_init_real<float>(qpt, nvt, ls, args, stream)
                   : launch_init_real<double>(qpt, nvt, ls, args, stream);
}

hipError_t launch_moments(int prec_fp32, const TubeDev* tubes, const WorkItem* items, int nitems, int tile,
                          const void* jtab, const double* itab, const void* f, double* rec, hipStream_t stream) {
  if (prec_fp32)
    hipLaunchKernelGGL(moments_kernel<float>, dim3(nitems), dim3(256), 0, stream, tubes, items, nitems, tile,
                       static_cast<const float*>(jtab), itab, static_cast<const float*>(f), rec);
  else
    hipLaunchKernelGGL(moments_kernel<double>, dim3(nitems), dim3(256), 0, stream, tubes, items, nitems, tile,
                       static_cast<const double*>(jtab), itab, static_cast<const double*>(f), rec);
  return hipGetLastError();
}

hipError_t launch_fields(const TubeDev* tubes, int tube, int nx, const double* rec, double* out, int64_t ld,
                         unsigned* flag, hipStream_t stream) {
  hipLaunchKernelGGL(fields_kernel, dim3((nx + 255) / 256), dim3(256), 0, stream, tubes, tube, rec, out, ld, flag);
  return hipGetLastError();
}

hipError_t launch_totals(const TubeDev* tubes, int tube, const double* rec, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(totals_kernel, dim3(1), dim3(256), 0, stream, tubes, tube, rec, out);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t stream) {
  const size_t n16 = bytes / 16;
  const int grid = static_cast<int>(std::min<size_t>((n16 + 255) / 256, 256 * 64));
  if (n16) {
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, stream, static_cast<uint4*>(dst),
                       static_cast<const uint4*>(src), n16);
  }
  const size_t tail = bytes - n16 * 16;
  if (tail) {
    hipError_t e = hipMemcpyAsync(static_cast<char*>(dst) + n16 * 16, static_cast<const char*>(src) + n16 * 16, tail,
                                  hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace rlb
