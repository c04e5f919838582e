// Internal data structures shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rlb.h"

namespace rlb {

constexpr int kMaxQp = 8;   // radial (Gauss-Laguerre) order limit
constexpr int kMaxNv = 7;   // angular truncation order limit
constexpr int kMaxNp = 7;   // radial truncation order limit (n_p < q_p)

// Polar-node table row (one per Gauss-Legendre node j of a tube):
//   xi, w, w*xi, w*xi^2, P_0(xi) .. P_7(xi)
constexpr int kJStride = 12;
// Radial-node table row (one per Gauss-Laguerre node i of a tube):
//   p, w_p, T0^3 w_p p, T0^4 w_p p^2, L_0(p) .. L_7(p)   (L = L^{(1)})
constexpr int kIStride = 12;
// Auxiliary angular rule used to project the equilibrium (symmetric pairs):
//   xi_a > 0, then w_a (2k+1)/2 P_k(xi_a) for k = 0..7
constexpr int kAuxStride = 10;
constexpr int kAuxPairsFP64 = 24;  // 48-point Gauss-Legendre rule
constexpr int kAuxPairsFP32 = 12;  // 24-point Gauss-Legendre rule

// High-order equilibrium (kMaxNv < n_v <= kMaxNvHigh, q_xi <= kMaxQxHigh):
// the equilibrium of a cell is evaluated by a pre-pass on the matrix cores
// (rlb_feq.hip) as
//   F_eq(p_i, xi_j) = pref sum_a G_i(x_a) Z(x_a, xi_j),
//   Z(x, xi) = w(x) sum_{k <= n_v} (2k+1)/2 P_k(x) P_k(xi),
// over an auxiliary Gauss-Legendre rule of 2B points +-x_b, in even/odd form:
// with E_b = G(+x_b) + G(-x_b), O_b = G(+x_b) - G(-x_b) and j' the mirror node
// of j (xi_j' = -xi_j),
//   F_j + F_j' = sum_b E_b Ze[j][b],  F_j - F_j' = sum_b O_b Zo[j][b],
//   Ze[j][b] = Z(x_b, xi_j) + Z(x_b, -xi_j),  Zo[j][b] = Z(x_b, xi_j) - Z(x_b, -xi_j).
constexpr int kMaxNvHigh = 255;       // angular truncation limit of that form
constexpr int kMaxQxHigh = 256;       // polar order limit of that form
constexpr int kNvtHigh = -1;          // kernel-group tag of that form
// B: pairs of the auxiliary rule, a multiple of the MFMA's K = 4, with
// 2 (2B) - n_v >= kHighExactMargin: the rule integrates P_k G for k <= n_v
// with the margin of degree that the 48-point rule of the low-order FP64
// form has at n_v = 7 (96 - 7), so the two forms are equally accurate
constexpr int kHighExactMargin = 89;
constexpr int high_aux_pairs(int nv) { return 4 * ((nv + kHighExactMargin + 15) / 16); }
// rows of Ze, Zo: ceil(q_xi / 2) rounded up to the MFMA's M = 16 (zero rows)
constexpr int high_rows(int qx) { return 16 * (((qx + 1) / 2 + 15) / 16); }

// Range of the WENO5 epsilon.  Tubes: 4 eps must be a positive number of the
// lattice's precision with room to spare, and e_r = 4 (eps + beta_r) finite
// (the stage kernel switches to scaled weights where the product form of the
// weights under- or overflows).  Planes use the product form only, which
// needs (4 eps)^4 above the smallest normal number and e_r^4 below the
// largest: eps in [1e-10, 1e8] in FP32 (for |F| up to ~1e3), [1e-70, 1e70]
// in FP64.
inline bool weno_eps_in_range(double eps, bool fp32) {
  return eps >= (fp32 ? 1e-40 : 1e-300) && eps <= 1e30;
}
inline bool plane_weno_eps_in_range(double eps, bool fp32) {
  return fp32 ? (eps >= 1e-10 && eps <= 1e8) : (eps >= 1e-70 && eps <= 1e70);
}

// Sticky device flags.
constexpr unsigned kFlagNonphysical = 1u;
constexpr unsigned kFlagFastFlow = 2u;  // |v| > 0.95: projection rule less accurate
static_assert(kFlagNonphysical == RLB_FLAG_NONPHYSICAL && kFlagFastFlow == RLB_FLAG_FAST_FLOW,
              "device flag bits are the interface's");

struct TubeDev {
  int64_t f_off;    // element offset of the tube in a state array
  int64_t rec_off;  // double offset of the tube's moment record [5][ldx]
  int32_t nx, ldx;  // cells, row stride (elements)
  int32_t qx, qp, nv, np;
  int32_t jrow, irow;  // first row of the tube in the polar / radial tables
  double z_min, dz, dz_inv, dt, tau_inv, T0, weno_eps;
  int32_t group;    // kernel instantiation group
  int32_t ldf;      // row stride of the adjoint face buffer (>= nx + 1)
  int64_t cell_off; // offset of the tube in per-cell arrays (sum of ldx of earlier tubes)
  int64_t face_off; // element offset of the tube in one slot of the adjoint face buffer
  // high-order equilibrium table (double offset into the table buffer):
  // Ze [zj][zb], then Zo [zj][zb], then the positive nodes x_b [zb];
  // zj = high_rows(q_xi), zb = high_aux_pairs(n_v)
  int64_t z_off;
  int32_t zj, zb;
};

// Arguments of the adjoint kernels of one stage of one tube.  For the stage
// g -> out = a g_n + b (g + dt L(g)) the adjoint step forms, per point,
//   out    = cK K + cJ (dL/dg)^T K (+ acc_in if add_acc)
//   acc    = (acc_init ? 0 : acc) + cA K
// where K is the adjoint of the stage output.
template <typename Real>
struct AdjArgs {
  const TubeDev* tubes;
  int32_t tube;
  int32_t aux_pairs;
  const Real* jtab;
  const double* itab;
  const Real* aux;
  const double* aux_d;
  const Real* g;
  const double* rec_g;
  const Real* K;
  const Real* acc_in;
  Real* out;
  Real* acc_out;
  double* cellbuf;  // per cell: mu[5], gamma/tau, u/tau  ([7][ldx] per tube)
  double* tau_acc;  // per cell d/dtau partials ([ldx] per tube)
  Real* G;          // face contributions, 5 slots of the state-like face layout
  int64_t G_slot;   // elements per slot
  double cK, cJ, cA;
  int32_t add_acc, acc_init, tau_init;
  // high-order form: the pre-pass's equilibrium values of the stage input g
  // (state layout) and the even/odd projection tables
  const Real* feq;
  const double* ztab;
};

// Work item of the stage kernels: a tile of cells of one tube.
struct WorkItem {
  int32_t tube;
  int32_t x0;
};

template <typename Real>
struct StageArgs {
  const TubeDev* tubes;
  const WorkItem* items;
  int32_t nitems;
  int32_t stage;       // 1, 2, 3 (SSP-RK3 stage)
  int32_t aux_pairs;
  const Real* jtab;
  const double* itab;
  const Real* aux;
  const Real* fin;     // stage input
  const Real* fn;      // state at the start of the step (stages 2, 3)
  Real* fout;          // stage output (stage 3 may alias fn)
  const double* rec_in;
  double* rec_out;
  unsigned* flag;
  // split launch (grid.y = radial node): each block writes its node's three
  // plain sums per cell to part[(cell_off + x) * part_stride + 3 i + c] and
  // combine_kernel forms the records; nullptr: one block per item, records
  // written by the stage kernel
  double* part;
  int32_t part_stride;
  const Real* feq;  // high-order group: the stage input's equilibrium (state layout)
};

// Arguments of the high-order equilibrium pre-pass: F_eq of the state whose
// moment records are `rec` (or, with rec == nullptr, of the initial side
// states of the tubes whose tube_mask is set) into `out` (state layout).
template <typename Real>
struct FeqArgs {
  const TubeDev* tubes;
  const WorkItem* items;
  int32_t nitems;
  int32_t tile;
  const double* itab;
  const double* ztab;
  const double* rec;
  const double* sides;
  const int32_t* tube_mask;
  Real* out;
  int32_t row_tiles;  // largest zj / 16 of the launch's tubes (kernel variant: 2, 4 or 8)
};

template <typename Real>
struct InitArgs {
  const TubeDev* tubes;
  const WorkItem* items;
  int32_t nitems;
  int32_t aux_pairs;
  const Real* jtab;
  const double* itab;
  const Real* aux;
  const double* sides;  // per tube: P_L, n_L, u_L, P_R, n_R, u_R
  const int32_t* tube_mask;  // per tube: 1 = initialise
  Real* f;
  double* rec;
  unsigned* flag;
};

// Host-side launchers (defined in rlb_kernels.hip).
struct LaunchShape {
  int tile;
  int grid;
  int nodes;  // 1, or the group's radial-node bound for a split launch
  int chunk;  // quadrature points per LDS chunk of the stage kernel
};
hipError_t launch_stage(int prec_fp32, int qpt, int nvt, const LaunchShape& ls, const void* args,
                        hipStream_t stream);
hipError_t launch_init(int prec_fp32, int qpt, int nvt, const LaunchShape& ls, const void* args,
                       hipStream_t stream);
hipError_t launch_moments(int prec_fp32, const TubeDev* tubes, const WorkItem* items, int nitems, int tile,
                          const void* jtab, const double* itab, const void* f, double* rec, hipStream_t stream);
hipError_t launch_fields(const TubeDev* tubes, int tube, int nx, const double* rec, double* out, int64_t ld,
                         unsigned* flag, hipStream_t stream);
hipError_t launch_totals(const TubeDev* tubes, int tube, const double* rec, double* out, hipStream_t stream);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t stream);
hipError_t launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t stream);
hipError_t launch_stream(void* out, const void* a, const void* b, int rows, int64_t ld, int cols, int elem_bytes,
                         hipStream_t stream);
hipError_t launch_feq(int prec_fp32, const LaunchShape& ls, const void* args, hipStream_t stream);
hipError_t launch_combine(const TubeDev* tubes, const WorkItem* items, int nitems, int tile, const double* itab,
                          const double* part, int part_stride, double* rec_out, hipStream_t stream);

// ---------------------------------------------------------------------------
// Multi-dimensional model on an (x, z) plane (rlb_plane.hip, rlb_plane_api.cpp)
// ---------------------------------------------------------------------------
// Point s = (i * qx + j) * qh + k: radial node i, polar node j, evolved
// azimuthal node k = 0 .. qh - 1 (qh = q_phi / 2 + 1; the mirrored nodes
// q_phi - k carry equal values for data with u^y = 0).  State F[s][z][ldx],
// records rec[9][z][ldx] (N0, Nx, Nz, T00, T0x, T0z, Txx, Txz, Tzz).
// Velocity table row per (j, k): v_x, v_z, then the weighted moment factors
// w, w v_x, w v_z, w v_x^2, w v_x v_z, w v_z^2 with w = w_xi[j] omega[k], then
// the advection factors -v_x/dx and -v_z/dz (and two unused entries).
constexpr int kVStride = 12;
constexpr int kPlaneTileX = 64, kPlaneTileZ = 4;  // cells per workgroup (init, moments)

struct PlaneDev {
  int32_t nx, nz, ldx;
  int32_t qx, qh, qp, nv, np;
  int64_t plane;  // elements per point plane (nz * ldx)
  double dx_inv, dz_inv, dt, tau_inv, T0, weno_eps;
};

template <typename Real>
struct PlaneArgs {
  const PlaneDev* pl;
  int32_t stage;      // 1, 2, 3 (SSP-RK3 stage)
  int32_t aux_pairs;
  const Real* vtab;   // [qx * qh][kVStride]
  const double* itab; // radial rows (kIStride)
  const Real* aux;    // projection rule (kAuxStride)
  const Real* fin;
  const Real* fn;
  Real* fout;
  const double* rec_in;
  double* rec_out;
  unsigned* flag;
  const double* init;  // init kernel: per-cell P, n, u^x, u^z [4][nz][nx]
};

// Workgroups of the stage kernel's grid (its tiles are taller than kPlaneTileZ).
int plane_stage_grid(int nx, int nz);
hipError_t launch_plane_stage(int prec_fp32, int qpt, int nvt, const void* args, int grid, hipStream_t stream);
hipError_t launch_plane_init(int prec_fp32, int qpt, int nvt, const void* args, int grid, hipStream_t stream);
hipError_t launch_plane_moments(int prec_fp32, const void* args, int grid, hipStream_t stream);
hipError_t launch_plane_fields(const PlaneDev* pl, int nx, int nz, const double* rec, double* out, unsigned* flag,
                               hipStream_t stream);

// ---------------------------------------------------------------------------
// Multi-dimensional model on an (x, y, z) box (rlb_box.hip, rlb_box_api.cpp)
// ---------------------------------------------------------------------------
// Point s = (i * qx + j) * qf + k: radial node i, polar node j, azimuthal node
// k = 0 .. qf - 1 (every node of the trapezoid rule; nothing is mirrored).
// State F[s][z][y][ldx], records rec[14][z][y][ldx] (N0, Nx, Ny, Nz, T00, T0x,
// T0y, T0z, Txx, Txy, Txz, Tyy, Tyz, Tzz).  Velocity table row per (j, k):
// v_x, v_y, v_z, then the weighted moment factors w {1, v_x, v_y, v_z, v_x^2,
// v_x v_y, v_x v_z, v_y^2, v_y v_z, v_z^2} with w = w_xi[j] / qf.
constexpr int kBoxVStride = 16;
constexpr int kBoxTileX = 64, kBoxTileY = 4;  // cells per workgroup (one z layer)

struct BoxDev {
  int32_t nx, ny, nz, ldx;
  int32_t qx, qf, qp, nv, np;
  int32_t reserved;
  int64_t slab;   // elements per z layer of one point (ny * ldx)
  int64_t plane;  // elements per point (nz * slab)
  double dx_inv, dy_inv, dz_inv, dt, tau_inv, T0, weno_eps;
};

template <typename Real>
struct BoxArgs {
  const BoxDev* bx;
  int32_t stage;      // 1, 2, 3 (SSP-RK3 stage)
  int32_t aux_pairs;
  const Real* vtab;   // [qx * qf][kBoxVStride]
  const double* itab; // radial rows (kIStride)
  const Real* aux;    // projection rule (kAuxStride)
  const Real* fin;
  const Real* fn;
  Real* fout;
  const double* rec_in;
  double* rec_out;
  unsigned* flag;
  const double* init;  // init kernel: per-cell P, n, u^x, u^y, u^z [5][nz][ny][nx]
};

int box_grid(int nx, int ny, int nz);
hipError_t launch_box_stage(int prec_fp32, int qpt, int nvt, const void* args, int grid, hipStream_t stream);
hipError_t launch_box_init(int prec_fp32, int qpt, int nvt, const void* args, int grid, hipStream_t stream);
hipError_t launch_box_moments(int prec_fp32, const void* args, int grid, hipStream_t stream);
hipError_t launch_box_fields(const BoxDev* bx, int64_t cells, const double* rec, double* out, unsigned* flag,
                             hipStream_t stream);

// Adjoint launchers (defined in rlb_adjoint.hip); one tube per call.
hipError_t launch_adjoint_stage(int prec_fp32, int qpt, int nvt, int nx, int Q, const void* args, hipStream_t stream);
hipError_t launch_tau_reduce(const TubeDev* tubes, int tube, const double* tau_acc, double* dL_dtau,
                             hipStream_t stream);
hipError_t launch_fields_adjoint(int prec_fp32, const TubeDev* tubes, int tube, int nx, const void* jtab,
                                 const double* itab, const double* rec, const double* dfields, int64_t ld,
                                 void* lambda, hipStream_t stream);
// partials: nblocks_max x 2 x part_stride doubles (part_stride >= QPT (NVT + 1)
// of the low-order groups and >= q_p q_xi of a high-order tube).
hipError_t launch_initial_adjoint(int prec_fp32, int qpt, int nvt, const TubeDev* tubes, int tube, int nx,
                                  const void* jtab, const double* itab, const double* aux_d, int aux_pairs,
                                  const double* ztab, const double* sides, const void* lambda0, double* partials,
                                  int nblocks_max, int part_stride, double* grad_out, hipStream_t stream);

// Allocation-free step (rlb_noalloc.hip, host side in rlb_api.cpp): bytes of
// scratch a lattice's step needs besides its state, and the steps themselves
// with every such buffer in `scratch` (device memory of at least that size).
size_t noalloc_scratch_bytes(const rlb_lattice* L);
// Argument checks of the allocation-free step (reasons go to rlb_last_error)
// and the report of a HIP error on a lattice.
rlb_status noalloc_validate(rlb_lattice* L, const void* state, int64_t nsteps, size_t max_bytes);
rlb_status noalloc_hip_error(rlb_lattice* L, hipError_t e, const char* where);
rlb_status noalloc_steps(rlb_lattice* L, char* scratch, void* state, unsigned* flag_out, int64_t nsteps,
                         hipStream_t s);

}  // namespace rlb
