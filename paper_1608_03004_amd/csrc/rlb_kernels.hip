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
//      the high-order group (n_v > 7) instead streams the equilibrium values
//      that the matrix-core pre-pass of rlb_feq.hip wrote for this stage;
//   4. streams over the quadrature points in chunks of CH points: the chunk's
//      F values of the tile plus a 3-cell halo go to LDS (16-byte words of
//      consecutive chunk points of one cell), each lane computes the WENO5
//      value at its cell's left face (the tile's last face by CH extra
//      lanes), then each lane forms advection + Anderson-Witting relaxation,
//      the RK combination, stores the result and accumulates the five moments
//      of the output (Kahan-compensated in FP32);
//   5. writes the output moment record.
// Loads and stores go through raw buffer resources (scalar base and row
// offset, 32-bit lane offset).  Small problems split a launch over the radial
// nodes (one workgroup per tile and node; `combine_kernel` then forms the
// records).  The outflow boundary (zero-gradient ghosts) is index clamping at
// load time.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "rlb_device.h"
#include "rlb_internal.h"

namespace rlb {
namespace {

using namespace dev;

// Points per chunk by default: 8 in FP32; 4 in FP64, where registers are
// scarcer.  A schedule may double it (fewer barriers per point).  The moment
// sums always run in groups of chunk_points() points whatever the chunk of a
// launch, so every schedule gives the same records.
template <typename Real>
constexpr int chunk_points() {
  return sizeof(Real) == 4 ? 8 : 4;
}

// Moment sums of one radial node's row of values, in the order the stage
// kernel's epilogue uses (plain sums within groups of chunk_points() points,
// compensated across groups), so that records computed from a stored state
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

// Adds one radial node's plain sums s0 = sum w F, s1 = sum w xi F,
// s2 = sum w xi^2 F (quadrature weights of the polar rule) to the five
// moment records N0, Nz, T00, T0z, Tzz of a cell.  Every kernel that forms
// records goes through it, node by node in order, so that records of the
// same state agree to the bit.
template <typename Ptr>
__device__ inline void add_node(double m[5], Ptr I, double s0, double s1, double s2) {
  m[0] = fma(I[2], s0, m[0]);
  m[1] = fma(I[2], s1, m[1]);
  m[2] = fma(I[3], s0, m[2]);
  m[3] = fma(I[3], s1, m[3]);
  m[4] = fma(I[3], s2, m[4]);
}

// LDS layout of a chunk: value (c, p) -- chunk point c, tile position p --
// at plane[c / V][p][c % V], V = 16 / sizeof(Real), so that one lane's values
// of V consecutive chunk points are one 16-byte word and consecutive lanes
// touch consecutive words (bank-conflict free 128-bit accesses).  Every read
// of the face and update phases is then a fixed offset from a per-lane base.
template <typename Real>
struct LdsVec {
  static constexpr int V = 16 / int(sizeof(Real));
  typedef Real type __attribute__((ext_vector_type(V)));
};

// WENO value at the face between tile positions k+2 and k+3 (left face of the
// cell stored at k+3) from the six values r[k..k+5], upwinded by the sign of xi.
template <typename Real>
__device__ inline Real face_value(const Real r[6], bool positive, Real eps, bool& ok) {
  if (positive) return weno5(r[0], r[1], r[2], r[3], r[4], eps, ok);
  return weno5(r[5], r[4], r[3], r[2], r[1], eps, ok);
}
template <typename Real>
__device__ inline Real face_value_scaled(const Real r[6], bool positive, Real eps) {
  if (positive) return weno5_scaled(r[0], r[1], r[2], r[3], r[4], eps);
  return weno5_scaled(r[5], r[4], r[3], r[2], r[1], eps);
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
// Cache policies of the buffer accesses (0: default, 2: non-temporal).  f^n
// and the stage output are touched once per stage and stream past the caches;
// the stage input keeps the default policy because neighbouring tiles re-read
// its halo lines from L2 (non-temporal there measured 6 % slower).  In the
// chunk loop every access is a scalar base (per chunk), a scalar row offset and
// a 32-bit per-lane byte offset; the resource's size bounds every access to the
// chunk's rows.
constexpr int kLoadAux = 0, kFnAux = 2, kStoreAux = 2;

// The CH rows of chunk (i, j0) of one tube's distribution: rows i*qx + j0 + c,
// with rows past the last point repeating the last row (so every lane always
// issues the same loads).  `row_bytes` = ldx * sizeof(Real).
template <typename Real, int CH>
struct ChunkRows {
  Rsrc r;
  int last;  // index of the last valid row of the chunk
  __device__ inline ChunkRows(const Real* tube_f, int64_t ldx, uint32_t row_bytes, int qx, int i, int j0) {
    r = make_rsrc(tube_f + int64_t(i * qx + j0) * ldx, uint32_t(CH) * row_bytes);
    last = min(CH - 1, qx - 1 - j0);
  }
  __device__ inline uint32_t soff(int c, uint32_t row_bytes) const { return uint32_t(min(c, last)) * row_bytes; }
};

// Loads of one chunk: the tile's own cells for CH points and, in wave 0, the
// 6-cell halo of all CH points (one instruction per 64 halo values: lane l of
// instruction q loads halo cell e % 6 of chunk point e / 6, e = l + 64 q).
template <int CH>
constexpr int halo_loads() {
  return (6 * CH + 63) / 64;
}
template <typename Real, int CH>
struct ChunkLoads {
  Real f[CH];
  Real halo[halo_loads<CH>()];
};

template <typename Real, int TILE, int CH>
__device__ inline void issue_chunk(const Real* tube_f, int64_t ldx, uint32_t row_bytes, int qx, int i, int j0,
                                   uint32_t vx, int t, int x0, int nx, ChunkLoads<Real, CH>& L) {
  const ChunkRows<Real, CH> rows(tube_f, ldx, row_bytes, qx, i, j0);
#pragma unroll
  for (int c = 0; c < CH; ++c) L.f[c] = BufIO<Real>::template load<kLoadAux>(rows.r, vx, rows.soff(c, row_bytes));
  if (t < 64) {
    if constexpr (halo_loads<CH>() == 1) {  // lane h + 6c: halo cell h of chunk point c
      const int c = min(t / 6, CH - 1), h = t % 6;
      const int hx = h < 3 ? max(x0 - 3 + h, 0) : min(x0 + TILE + (h - 3), nx - 1);
      const uint32_t off = uint32_t(min(c, rows.last)) * row_bytes + uint32_t(hx) * uint32_t(sizeof(Real));
      L.halo[0] = BufIO<Real>::template load<kLoadAux>(rows.r, off, 0);
    } else {
#pragma unroll
      for (int q = 0; q < halo_loads<CH>(); ++q) {
        const int e = t + 64 * q;
        const int c = min(e / 6, CH - 1), h = e % 6;
        const int hx = h < 3 ? max(x0 - 3 + h, 0) : min(x0 + TILE + (h - 3), nx - 1);
        const uint32_t off = uint32_t(min(c, rows.last)) * row_bytes + uint32_t(hx) * uint32_t(sizeof(Real));
        L.halo[q] = BufIO<Real>::template load<kLoadAux>(rows.r, off, 0);
      }
    }
  }
}

// Moment sums over one radial node: plain sums within a chunk, Kahan-
// compensated across chunks in FP32 (plain FP64 sums in the FP64 form).
template <typename Real>
struct Moments3 {
  Acc<Real> a0, a1, a2;
};

// Waves per SIMD the register allocation must allow.  The first stage of a
// step (no f^n stream) of the Q_p <= 4 groups runs at 4 waves: in FP32 with
// every value in registers (5 waves with a few spilled registers measured 2 %
// slower), in FP64 with 148 bytes per lane spilled, which still beats 3 waves
// without spills (3.65 against 3.70 ms per FP64 step of a 2^20-cell tube with
// Q = 64 x 4); stages 2 and 3 of those groups are bandwidth-bound and keep
// every value in registers at the compiler's choice (4 waves in FP32, 3 in
// FP64, where 4 waves spill and measured 3.74 ms).  The FP32
// Q_p <= 8 group runs at 4 waves instead of the compiler's 3 (a 2^19-cell tube
// with Q = 64 x 5: 1.35 against 1.41 ms per step); its FP64 form keeps all
// its coefficients in registers (3 waves measured 18 % slower).  The
// high-order variant (NVT < 0) holds no coefficients and is left to the
// compiler.
template <typename Real, int QPT, int NVT, bool HAS_FN>
constexpr int stage_waves_per_simd() {
  return NVT < 0 ? 1
                 : QPT > 4 ? (sizeof(Real) == 4 ? 4 : 1) : (HAS_FN ? 1 : 4);
}

template <typename Real, int TILE, int QPT, int NVT, bool HAS_FN, int CH>
__global__ __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(stage_waves_per_simd<Real, QPT, NVT, HAS_FN>())))
void stage_kernel(StageArgs<Real> a) {
  constexpr int V = LdsVec<Real>::V, NH = CH / V;
  static_assert(CH % V == 0, "a chunk is a whole number of 16-byte LDS words");
  // NVT < 0: high-order group, whose equilibrium values are read from a.feq
  // (written for this stage's input by the equilibrium pre-pass) instead of
  // being evaluated from projection coefficients
  constexpr bool kHigh = NVT < 0;
  // In the pipelined stages of a high-order group the pre-pass of the next
  // piece runs beside this kernel on another stream and its matrix-core waves
  // share the SIMDs with these: a higher issue priority for the stage's
  // waves keeps its (memory-bound) loads going out while the pre-pass takes
  // the remaining issue slots.  Every wave of a launch gets the same priority,
  // so a launch that runs alone is unaffected.
  if constexpr (kHigh) __builtin_amdgcn_s_setprio(1);
  constexpr int ND = kHigh ? 1 : NVT + 1;
  using Vec = typename LdsVec<Real>::type;
  __shared__ __attribute__((aligned(16))) Real tile[NH][TILE + 6][V];
  __shared__ __attribute__((aligned(16))) Real faces[NH][TILE + 1][V];
  __shared__ double mom[5][TILE];
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
    const uint32_t row_bytes = uint32_t(ldx) * uint32_t(sizeof(Real));
    const int x0 = wx0;
    const int x = x0 + t;
    const bool valid = x < nx;
    const bool tile_full = x0 + TILE <= nx;  // uniform
    const int xc = valid ? x : nx - 1;
    const uint32_t vx = uint32_t(xc) * uint32_t(sizeof(Real));
    const int64_t f_off = tbp->f_off;
    const Real* fin = a.fin + f_off;
    const Real* fn = a.fn + f_off;
    const Real* feq_t = a.feq + f_off;
    Real* fout = a.fout + f_off;
    const cptr<Real> jtab = as_const(a.jtab) + int64_t(tbp->jrow) * kJStride;
    const cptr<double> itab = as_const(a.itab) + int64_t(tbp->irow) * kIStride;

    // radial nodes of this block: all of them, or node blockIdx.y of a split
    // launch (whose blocks beyond the tube's q_p have nothing to do)
    const bool split = a.part != nullptr;
    const int i_first = split ? int(blockIdx.y) : 0;
    if (i_first >= qp) continue;
    const int i_last = split ? i_first + 1 : qp;

    // first chunk's loads go out before the per-cell prologue
    ChunkLoads<Real, CH> bufA, bufB;
    issue_chunk<Real, TILE, CH>(fin, ldx, row_bytes, qx, i_first, 0, vx, t, x0, nx, bufA);

    // 1-2. moments of the stage input -> Landau frame (FP64)
    double m[5];
    const double* rin = a.rec_in + tbp->rec_off;
#pragma unroll
    for (int c = 0; c < 5; ++c) m[c] = rin[c * ldx + xc];
    const Macro M = landau(m);
    if (valid && !M.ok) raise_flag(a.flag, kFlagNonphysical);
    if (valid && fabs(M.v) > 0.95) raise_flag(a.flag, kFlagFastFlow);

    // 3. equilibrium coefficients
    Real D[QPT][ND];
    if constexpr (!kHigh)
      feq_coefficients<Real, QPT, NVT>(Real(M.n), Real(M.T), Real(M.gamma), Real(M.u), Real(tbp->T0), qp, tbp->np,
                                       tbp->nv, itab, as_const(a.aux), a.aux_pairs, D);
    // out = (1 - cs) f^n + cs (f_in + dt L),  L = -xi/dz (F_+ - F_-) - (gamma - xi u)/tau (f - f^eq)
    const int stage = a.stage;
    const Real cs = stage == 1 ? Real(1) : (stage == 2 ? Real(0.25) : Real(2.0 / 3.0));
    const Real dt = Real(tbp->dt), dz_inv = Real(tbp->dz_inv);
    const Real g0 = Real(M.gamma * tbp->tau_inv), g1 = Real(M.u * tbp->tau_inv);
    const Real eps4 = Real(4.0 * tbp->weno_eps);

    // One chunk: stage `cur` in LDS, prefetch the next chunk into `nxt`,
    // WENO faces, update, moment sums.
    auto chunk = [&](ChunkLoads<Real, CH>& cur, ChunkLoads<Real, CH>& nxt, int i, int j0, const Real* Dc,
                     Moments3<Real>& acc) {
      // f^n of this chunk (consumed after the faces), issued before the prefetch
      Real nr[CH];
      if (HAS_FN) {
        const ChunkRows<Real, CH> rows(fn, ldx, row_bytes, qx, i, j0);
#pragma unroll
        for (int c = 0; c < CH; ++c) nr[c] = BufIO<Real>::template load<kFnAux>(rows.r, vx, rows.soff(c, row_bytes));
      }
      Real er[kHigh ? CH : 1];
      if constexpr (kHigh) {
        const ChunkRows<Real, CH> rows(feq_t, ldx, row_bytes, qx, i, j0);
#pragma unroll
        for (int c = 0; c < CH; ++c) er[c] = BufIO<Real>::template load<kFnAux>(rows.r, vx, rows.soff(c, row_bytes));
      }
      {  // next chunk: the next radial node's first at the end of a node; the
         // very last chunk re-loads itself
        int in = i, jn = j0 + CH;
        if (jn >= qx) { in = i + 1; jn = 0; }
        if (in >= i_last) { in = i; jn = j0; }
        issue_chunk<Real, TILE, CH>(fin, ldx, row_bytes, qx, in, jn, vx, t, x0, nx, nxt);
      }
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        Vec w;
#pragma unroll
        for (int e = 0; e < V; ++e) w[e] = cur.f[h * V + e];
        *reinterpret_cast<Vec*>(&tile[h][t + 3][0]) = w;
      }
      if constexpr (halo_loads<CH>() == 1) {
        if (t < 6 * CH) {
          const int c = t / 6, h = t % 6;
          tile[c / V][h < 3 ? h : TILE + h][c % V] = cur.halo[0];
        }
      } else if (t < 64) {
#pragma unroll
        for (int q = 0; q < halo_loads<CH>(); ++q) {
          const int e = t + 64 * q;
          if (e < 6 * CH) {
            const int c = e / 6, h = e % 6;
            tile[c / V][h < 3 ? h : TILE + h][c % V] = cur.halo[q];
          }
        }
      }
      __syncthreads();
      // WENO5 value at this lane's left face and, by CH
      // lanes, at the tile's right-most face.  The six values at tile
      // positions t..t+5 cover both upwind directions; the direction is a
      // branch on the chunk's sign pattern, a wave-uniform bit mask: the polar
      // nodes are sorted and exactly symmetric (the middle node of an odd rule
      // is exactly 0), so xi_j >= 0 exactly for j >= q_xi / 2, and all points
      // of a chunk share the sign of xi except in the chunk that straddles 0.
      const int jpos = min(max(qx / 2 - j0, 0), CH);  // first chunk point with xi >= 0
      const uint32_t pos_mask = jpos >= 32 ? 0u : (~0u << jpos);
      Real own[CH];
      bool ok = true;  // every face of this lane had a usable product-form denominator
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        Vec rv[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) rv[k] = *reinterpret_cast<const Vec*>(&tile[h][t + k][0]);
        const uint32_t hm = (pos_mask >> (h * V)) & ((1u << V) - 1u);
        auto faces_of = [&](auto dir) {
#pragma unroll
          for (int e = 0; e < V; ++e) {
            Real r[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) r[k] = rv[k][e];
            const bool pos = decltype(dir)::value == 1 ? true : decltype(dir)::value == 0 ? false : ((hm >> e) & 1u);
            own[h * V + e] = face_value(r, pos, eps4, ok);
            __builtin_amdgcn_sched_barrier(0);  // one face at a time
          }
        };
        if (hm == (1u << V) - 1u)
          faces_of(std::integral_constant<int, 1>{});
        else if (hm == 0)
          faces_of(std::integral_constant<int, 0>{});
        else
          faces_of(std::integral_constant<int, 2>{});
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        Vec w;
#pragma unroll
        for (int e = 0; e < V; ++e) w[e] = own[h * V + e];
        *reinterpret_cast<Vec*>(&faces[h][t][0]) = w;
      }
      if (t < CH) {  // the tile's right-most face, one chunk point per lane
        Real r[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) r[k] = tile[t / V][TILE + k][t % V];
        bool ok_last = true;
        const Real h = face_value(r, (pos_mask >> t) & 1u, eps4, ok_last);
        faces[t / V][TILE][t % V] = ok_last ? h : face_value_scaled(r, (pos_mask >> t) & 1u, eps4);
      }
      if (__builtin_expect(!ok, 0)) {
        // rare: a face's product-form weights under- or overflowed; this
        // lane's faces of the chunk again with the scaled weights
#pragma unroll 1
        for (int c = 0; c < CH; ++c) {
          Real r[6];
          for (int k = 0; k < 6; ++k) r[k] = tile[c / V][t + k][c % V];
          faces[c / V][t][c % V] = face_value_scaled(r, (pos_mask >> c) & 1u, eps4);
        }
      }
      __syncthreads();
      const int cj = min(CH, qx - j0);
      const ChunkRows<Real, CH> orow(fout, ldx, row_bytes, qx, i, j0);
      // full: every point of the chunk belongs to the node; lanes: every lane
      // of the tile holds a cell (all tiles but the last of a tube), so that
      // the stores need no per-lane predicate (measured: 0.7 % per FP32 step
      // of the 2^20 x 256 tube, 1.7 % in FP64)
      auto update = [&](auto full, auto lanes) {
        constexpr int GP = chunk_points<Real>() / V;  // LDS planes per moment group
        static_assert(NH % GP == 0, "a chunk is a whole number of moment groups");
        Real p0 = Real(0), p1 = Real(0), p2 = Real(0);
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          // this lane's cell values and faces for V chunk points, back from LDS
          const Vec wf = *reinterpret_cast<const Vec*>(&tile[h][t + 3][0]);
          const Vec wl = *reinterpret_cast<const Vec*>(&faces[h][t][0]);
          const Vec wr = *reinterpret_cast<const Vec*>(&faces[h][t + 1][0]);
#pragma unroll
          for (int e = 0; e < V; ++e) {
            const int c = h * V + e;
            if (decltype(full)::value || c < cj) {
              const cptr<Real> J = jtab + (j0 + c) * kJStride;
              Real feq;
              if constexpr (kHigh) {
                feq = er[c];
              } else {
                feq = Dc[0];
#pragma unroll
                for (int kk = 1; kk <= NVT; ++kk) feq += Dc[kk] * J[4 + kk];
              }
              const Real fr = wf[e];
              const Real df = fr - feq;
              const Real adv = (wr[e] - wl[e]) * (-J[0] * dz_inv);
              const Real rate = g0 - J[0] * g1;
              const Real L = adv - rate * df;
              // the RK combination as f^n + cs ((f_in - f^n) + dt L): the
              // difference of two successive stage values is exact, the
              // small increment carries its own rounding and f^n is added
              // last, so only the final sum rounds at the scale of F (and a
              // state with L = 0 is reproduced exactly)
              const Real out = HAS_FN ? nr[c] + cs * ((fr - nr[c]) + dt * L) : fr + dt * L;
              if (decltype(lanes)::value || valid)
                BufIO<Real>::template store<kStoreAux>(out, orow.r, vx, uint32_t(c) * row_bytes);
              p0 += J[1] * out;
              p1 += J[2] * out;
              p2 += J[3] * out;
            }
          }
          if constexpr (NH > GP) {
            if ((h + 1) % GP == 0) {
              // one moment group of chunk_points() points, if it holds a
              // point of the node
              if (decltype(full)::value || (h + 1 - GP) * V < cj) {
                acc.a0.add(p0);
                acc.a1.add(p1);
                acc.a2.add(p2);
              }
              p0 = Real(0);
              p1 = Real(0);
              p2 = Real(0);
            }
          }
          // keep the scheduler from hoisting the next plane's reads (bounds
          // the live registers; occupancy hides the latency instead)
          __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (NH == GP) {  // the default chunk is one moment group
          acc.a0.add(p0);
          acc.a1.add(p1);
          acc.a2.add(p2);
        }
      };
      if (tile_full) {
        if (cj == CH)
          update(std::true_type{}, std::true_type{});
        else
          update(std::false_type{}, std::true_type{});
      } else {
        if (cj == CH)
          update(std::true_type{}, std::false_type{});
        else
          update(std::false_type{}, std::false_type{});
      }
      // no barrier here: the next chunk's first LDS writes (its cell values)
      // go to positions whose readers other than the writing lane all passed
      // this chunk's second barrier, and its faces are written after its own
      // first barrier, which every lane reaches only once done with this
      // chunk's update
    };

    // the five moment sums of this lane's cell live in LDS (registers are
    // the scarce resource here); each lane only touches its own column
#pragma unroll
    for (int c = 0; c < 5; ++c) mom[c][t] = 0.0;
    double* part = split ? a.part + (tbp->cell_off + xc) * a.part_stride : nullptr;
    // runtime loop over radial nodes (the node's coefficient row is selected
    // with uniform conditional moves); the chunk loop alternates the two
    // register buffers so that no in-flight load is ever copied
#pragma unroll 1
    for (int i = i_first; i < i_last; ++i) {
      Real Dc[ND] = {};
      if constexpr (!kHigh) {
#pragma unroll
        for (int k = 0; k < ND; ++k) {
          Real d = D[0][k];
#pragma unroll
          for (int ii = 1; ii < QPT; ++ii) d = i == ii ? D[ii][k] : d;
          Dc[k] = d;
        }
      }
      Moments3<Real> acc;
      for (int j0 = 0; j0 < qx; j0 += 2 * CH) {
        chunk(bufA, bufB, i, j0, Dc, acc);
        if (j0 + CH < qx)
          chunk(bufB, bufA, i, j0 + CH, Dc, acc);
        else
          bufA = bufB;  // odd number of chunks per node: the next node starts in A
      }
      const double s0 = acc.a0.value(), s1 = acc.a1.value(), s2 = acc.a2.value();
      if (split) {
        if (valid) {
          part[3 * i] = s0;
          part[3 * i + 1] = s1;
          part[3 * i + 2] = s2;
        }
      } else {
        double m5[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) m5[c] = mom[c][t];
        add_node(m5, itab + i * kIStride, s0, s1, s2);
#pragma unroll
        for (int c = 0; c < 5; ++c) mom[c][t] = m5[c];
      }
    }
    if (valid && !split) {
      double* ro = a.rec_out + tbp->rec_off;
#pragma unroll
      for (int c = 0; c < 5; ++c) ro[c * ldx + x] = mom[c][t];
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
    const double* st = a.sides + 6 * wi.tube + (left_of_split(tb, x) ? 0 : 3);
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
        add_node(mom, I, s0, s1, s2);
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
        add_node(mom, I, s0, s1, s2);
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

// Records of a split stage launch: the five moments of each cell from the
// per-node sums, in node order (the same operations as the unsplit kernel).
__global__ __launch_bounds__(256) void combine_kernel(const TubeDev* tubes, const WorkItem* items, int nitems,
                                                      int tile, const double* itab_all, const double* part,
                                                      int part_stride, double* rec_all) {
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const WorkItem wi = items[item];
    const TubeDev& tb = tubes[wi.tube];
    for (int t = threadIdx.x; t < tile; t += blockDim.x) {
      const int x = wi.x0 + t;
      if (x >= tb.nx) continue;
      const double* itab = itab_all + int64_t(tb.irow) * kIStride;
      const double* p = part + (tb.cell_off + x) * part_stride;
      double mom[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      for (int i = 0; i < tb.qp; ++i) add_node(mom, itab + i * kIStride, p[3 * i], p[3 * i + 1], p[3 * i + 2]);
      double* rec = rec_all + tb.rec_off;
#pragma unroll
      for (int c = 0; c < 5; ++c) rec[int64_t(c) * tb.ldx + x] = mom[c];
    }
  }
}

// Plain streaming copy (16-byte vectors), for bandwidth calibration.
__global__ __launch_bounds__(256) void copy_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                   size_t n16) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n16; k += stride) dst[k] = src[k];
}

// Streaming probe with the stage kernel's memory pattern and no arithmetic
// beyond one add: workgroups of 256 lanes own 256-column tiles of a [rows][ld]
// matrix (XCD-mapped like the stage kernel) and walk its rows in chunks of
// CH, the next chunk's loads issued before the current one is stored;
// out = a (+ b), with a at the default cache policy and b and out
// non-temporal, as f_k, f^n and the stage output.  The practical ceiling of
// the stage kernel's traffic: b = nullptr is stage 1 (one read, one write),
// otherwise stages 2 and 3 (two reads, one write).
template <typename Real, bool TWO>
__global__ __launch_bounds__(256) void stream_kernel(Real* out, const Real* a, const Real* b, int rows, int64_t ld,
                                                     int cols) {
  constexpr int CH = chunk_points<Real>();
  const int ntiles = (cols + 255) / 256;
  const bool xcd_map = (gridDim.x % kXcds) == 0 || int(gridDim.x) == ntiles;
  const uint32_t row_bytes = uint32_t(ld) * uint32_t(sizeof(Real));
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const int tile = xcd_map ? xcd_item(v, ntiles) : v;
    const int x = tile * 256 + int(threadIdx.x);
    const int xc = min(x, cols - 1);
    const uint32_t vx = uint32_t(xc) * uint32_t(sizeof(Real));
    Real ca[CH], cb[CH];
    auto issue = [&](int r0, Real* da, Real* db) {
      const int last = min(CH - 1, rows - 1 - r0);
      const Rsrc ra = make_rsrc(a + int64_t(r0) * ld, uint32_t(CH) * row_bytes);
#pragma unroll
      for (int c = 0; c < CH; ++c) da[c] = BufIO<Real>::template load<kLoadAux>(ra, vx, uint32_t(min(c, last)) * row_bytes);
      if (TWO) {
        const Rsrc rb = make_rsrc(b + int64_t(r0) * ld, uint32_t(CH) * row_bytes);
#pragma unroll
        for (int c = 0; c < CH; ++c) db[c] = BufIO<Real>::template load<kFnAux>(rb, vx, uint32_t(min(c, last)) * row_bytes);
      }
    };
    issue(0, ca, cb);
    for (int r0 = 0; r0 < rows; r0 += CH) {
      Real na[CH], nb[CH];
      if (r0 + CH < rows) issue(r0 + CH, na, nb);
      const Rsrc ro = make_rsrc(out + int64_t(r0) * ld, uint32_t(CH) * row_bytes);
      if (tile * 256 + 256 <= cols) {  // every lane holds a column: no per-lane predicate
#pragma unroll
        for (int c = 0; c < CH; ++c)
          if (r0 + c < rows)
            BufIO<Real>::template store<kStoreAux>(TWO ? ca[c] + cb[c] : ca[c], ro, vx, uint32_t(c) * row_bytes);
      } else {
#pragma unroll
        for (int c = 0; c < CH; ++c)
          if (r0 + c < rows && x < cols)
            BufIO<Real>::template store<kStoreAux>(TWO ? ca[c] + cb[c] : ca[c], ro, vx, uint32_t(c) * row_bytes);
      }
      if (r0 + CH < rows) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          ca[c] = na[c];
          cb[c] = nb[c];
        }
      }
    }
  }
}

// Fills n words with v (flags and counters; a kernel rather than a memset so
// that the clear can sit in captured work).
__global__ __launch_bounds__(256) void fill_u32_kernel(unsigned* p, int n, unsigned v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

template <typename Real, int TILE, int QPT, int NVT, int CH>
hipError_t launch_stage_ch(const LaunchShape& ls, const void* args, hipStream_t s) {
  const StageArgs<Real>& a = *static_cast<const StageArgs<Real>*>(args);
  const dim3 grid(ls.grid, ls.nodes);
  if (a.stage == 1)
    hipLaunchKernelGGL((stage_kernel<Real, TILE, QPT, NVT, false, CH>), grid, dim3(TILE), 0, s, a);
  else
    hipLaunchKernelGGL((stage_kernel<Real, TILE, QPT, NVT, true, CH>), grid, dim3(TILE), 0, s, a);
  return hipGetLastError();
}

template <typename Real, int TILE, int QPT, int NVT>
hipError_t launch_stage_t(const LaunchShape& ls, const void* args, hipStream_t s) {
  constexpr int CH = chunk_points<Real>();
  if (ls.chunk == CH) return launch_stage_ch<Real, TILE, QPT, NVT, CH>(ls, args, s);
  if (ls.chunk == 2 * CH) return launch_stage_ch<Real, TILE, QPT, NVT, 2 * CH>(ls, args, s);
  return hipErrorInvalidValue;
}

template <typename Real, int QPT, int NVT>
hipError_t launch_stage_tile(const LaunchShape& ls, const void* args, hipStream_t s) {
  switch (ls.tile) {
    case 64: return launch_stage_t<Real, 64, QPT, NVT>(ls, args, s);
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
  if (qpt == 8 && nvt == kNvtHigh) return launch_stage_tile<Real, 8, kNvtHigh>(ls, args, s);
  return hipErrorInvalidValue;
}

template <typename Real, int QPT, int NVT>
hipError_t launch_init_t(const LaunchShape& ls, const void* args, hipStream_t s) {
  const InitArgs<Real>& a = *static_cast<const InitArgs<Real>*>(args);
  if (ls.tile == 64) {
    hipLaunchKernelGGL((init_kernel<Real, 64, QPT, NVT>), dim3(ls.grid), dim3(64), 0, s, a);
  } else if (ls.tile == 128) {
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

hipError_t launch_combine(const TubeDev* tubes, const WorkItem* items, int nitems, int tile, const double* itab,
                          const double* part, int part_stride, double* rec_out, hipStream_t stream) {
  hipLaunchKernelGGL(combine_kernel, dim3(nitems), dim3(256), 0, stream, tubes, items, nitems, tile, itab, part,
                     part_stride, rec_out);
  return hipGetLastError();
}

hipError_t launch_stream(void* out, const void* a, const void* b, int rows, int64_t ld, int cols, int elem_bytes,
                         hipStream_t stream) {
  const int ntiles = (cols + 255) / 256;
  if (elem_bytes == 4) {
    if (b)
      hipLaunchKernelGGL((stream_kernel<float, true>), dim3(ntiles), dim3(256), 0, stream, static_cast<float*>(out),
                         static_cast<const float*>(a), static_cast<const float*>(b), rows, ld, cols);
    else
      hipLaunchKernelGGL((stream_kernel<float, false>), dim3(ntiles), dim3(256), 0, stream, static_cast<float*>(out),
                         static_cast<const float*>(a), static_cast<const float*>(b), rows, ld, cols);
  } else {
    if (b)
      hipLaunchKernelGGL((stream_kernel<double, true>), dim3(ntiles), dim3(256), 0, stream, static_cast<double*>(out),
                         static_cast<const double*>(a), static_cast<const double*>(b), rows, ld, cols);
    else
      hipLaunchKernelGGL((stream_kernel<double, false>), dim3(ntiles), dim3(256), 0, stream, static_cast<double*>(out),
                         static_cast<const double*>(a), static_cast<const double*>(b), rows, ld, cols);
  }
  return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t stream) {
  if (n > 0) hipLaunchKernelGGL(fill_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, p, n, v);
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
