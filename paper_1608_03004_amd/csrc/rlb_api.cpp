// Host side of the C interface declared in include/rlb.h: validation, the
// momentum-quadrature tables, the device workspace layout, work lists and
// launch schedules, and the hipGraph replay of time steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/rlb.h"
#include "quadrature.h"
#include "rlb_internal.h"

using namespace rlb;

namespace {

thread_local std::string g_create_error;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Group {
  int qpt, nvt;
  int qp_max;                // largest q_p of the group's tubes
  int zj_max;                // largest high-order table rows of the group's tubes
  int item_begin, item_end;  // range in the item list
};

// Lattices up to this many cells keep a per-node sum buffer, so that stages
// of small problems can spread the radial nodes over workgroups.
constexpr int64_t kSplitMaxCells = int64_t(1) << 18;

// Pieces of the high-order group's work list per FP32 stage: the equilibrium
// pre-pass of a piece (matrix cores) runs on a side stream while the stage
// kernels of earlier pieces (bandwidth) run on the lattice's stream.  A piece
// keeps at least two tiles per CU (one tile per CU measured far slower: the
// launches no longer fill the GPU).  Measured on the 2^20 x 256, N_v = 63 FP32
// tube: 4.24 ms per step unpipelined, 3.84 with four pieces, 3.63 with eight.
// The FP64 form is not pipelined: its stage kernel needs the vector units the
// FP64 pre-pass holds, and overlapping them measured slower (7.12 against
// 6.66 ms per step with four pieces).
constexpr int kPipePieces = 8;

}  // namespace

struct rlb_lattice {
  std::vector<rlb_tube_desc> desc;
  int ntubes = 0;
  rlb_precision prec = RLB_FP64;
  uint32_t flags = 0;
  size_t rsize = 8;

  // host tables
  std::vector<TubeDev> tubes;
  std::vector<double> jtab_d, itab, aux_d;
  std::vector<float> jtab_f, aux_f;
  std::vector<double> ztab;  // high-order equilibrium tables (see high_order_table)
  bool has_high = false;
  int aux_pairs = 0;
  std::vector<std::vector<double>> xi, wxi, p, wp;  // per tube (host copies)

  // layout
  int64_t state_elems = 0, rec_elems = 0;
  int max_items = 0, max_ldx = 0;
  size_t off_F[3] = {0, 0, 0}, off_rec[3] = {0, 0, 0};
  size_t off_tubes = 0, off_jtab = 0, off_itab = 0, off_aux = 0, off_aux_d = 0, off_items = 0, off_sides = 0,
         off_mask = 0, off_flag = 0, off_fields = 0, off_totals = 0, total = 0;
  size_t off_part = 0;  // per-node sums of split launches (0: none)
  size_t off_ztab = 0, off_feq = 0;  // high-order tables and equilibrium values (0: none)
  size_t off_afeq = 0;  // the adjoint's equilibrium values (high-order with RLB_WITH_ADJOINT)
  int part_stride = 0;  // doubles per cell in that buffer
  size_t step_bytes = 0;  // bytes of the layout before f^n (see rlb_create)
  // adjoint workspace (RLB_WITH_ADJOINT)
  int64_t cell_elems = 0, face_elems = 0;
  int init_blocks_max = 0;
  int ipart_stride = kMaxQp * (kMaxNv + 1);  // doubles per block and side of the initial adjoint's partials
  size_t off_aF[2] = {0, 0}, off_arec[3] = {0, 0, 0}, off_lam2 = 0, off_lam1 = 0, off_acc = 0, off_G = 0,
         off_cellbuf = 0, off_tauacc = 0, off_ipart = 0, off_grad = 0;

  // binding
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  bool initialised = false;
  // high-order group: side stream (default priority) of the pipelined
  // equilibrium pre-pass and its events, created at the first binding on the
  // device current then
  hipStream_t side = nullptr;
  int side_device = -1;
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_pre[kPipePieces] = {};    // pre-pass of piece p done (side stream)
  hipEvent_t ev_stage[kPipePieces] = {};  // stage kernel of piece p done (lattice's stream)
  bool pipe_forked = false;  // the side stream follows the stage kernels piece by piece

  // schedule and work lists
  rlb_schedule sched = {256, 0, 4, 0, 0, -1};
  std::vector<WorkItem> items;
  std::vector<Group> groups;
  int cu_count = 0;

  // graph replay
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int graph_steps = 0;

  std::vector<double> time;
  std::vector<double> sides_h;
  std::vector<int32_t> mask_h;
  std::string err;

  // allocation-free step: the caller's state stands in for f^n and the
  // caller's word (or the scratch copy) for the flag while it runs
  void* f0_ext = nullptr;
  unsigned* flag_ext = nullptr;

  template <typename T>
  T* dev(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  void* F(int k) const { return (k == 0 && f0_ext) ? f0_ext : static_cast<void*>(ws + off_F[k]); }
  unsigned* flag() const { return flag_ext ? flag_ext : dev<unsigned>(off_flag); }
};

namespace {

// Device-to-device copy of a state: the library's 16-byte vector copy kernel
// when both ends are 16-byte aligned, the runtime's copy otherwise (caller
// buffers may be views at any element offset).
hipError_t state_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16) == 0)
    return launch_copy(dst, src, bytes, s);
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}

rlb_status fail(rlb_lattice* L, rlb_status st, const std::string& msg) {
  if (L) L->err = msg; else g_create_error = msg;
  return st;
}

rlb_status hip_fail(rlb_lattice* L, hipError_t e, const char* where) {
  return fail(L, RLB_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(L, expr)                                     \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) return hip_fail((L), _e, #expr);   \
  } while (0)

void kernel_group(int qp, int nv, int* qpt, int* nvt) {
  if (nv > kMaxNv) { *qpt = 8; *nvt = kNvtHigh; }
  else if (nv <= 5 && qp <= 3) { *qpt = 3; *nvt = 5; }
  else if (nv <= 5 && qp == 4) { *qpt = 4; *nvt = 5; }
  else { *qpt = 8; *nvt = 7; }
}

double tube_dt(const rlb_tube_desc& d) {
  const double dz = (d.z_max - d.z_min) / d.nx;
  if (d.dt > 0) return d.dt;
  return std::min(d.cfl * dz, d.dt_tau_max * d.tau);
}

// Table of the high-order equilibrium of a tube with q_xi polar nodes xi
// (ascending, symmetric) and truncation n_v: Ze and Zo [zj][zb] with
//   Ze[j][b] = 2 w_b sum_{k <= n_v even} (2k+1)/2 P_k(x_b) P_k(xi_j),
//   Zo[j][b] = 2 w_b sum_{k <= n_v odd}  (2k+1)/2 P_k(x_b) P_k(xi_j)
// for the nodes xi_j <= 0 (j < ceil(q_xi/2); the rows up to zj are zero),
// then the positive nodes x_b of the 2 zb-point Gauss-Legendre rule with
// weights w_b.  Sums in extended precision.
void high_order_table(int qx, int nv, const std::vector<double>& xi, std::vector<double>& out) {
  const int zj = high_rows(qx), zb = high_aux_pairs(nv), half = (qx + 1) / 2;
  std::vector<double> ax, aw;
  gauss_legendre_rule(2 * zb, ax, aw);
  std::vector<double> t(size_t(2 * zj + 1) * zb, 0.0);
  for (int b = 0; b < zb; ++b) {
    const long double x = ax[zb + b], w = aw[zb + b];
    t[size_t(2 * zj) * zb + b] = ax[zb + b];
    for (int j = 0; j < half; ++j) {
      const long double y = xi[j];
      long double px0 = 1.0L, px1 = x, py0 = 1.0L, py1 = y;  // P_k, P_{k+1} at x and y
      long double se = 0.0L, so = 0.0L;
      for (int k = 0; k <= nv; ++k) {
        const long double term = (2.0L * k + 1.0L) / 2.0L * px0 * py0;
        if (k & 1) so += term; else se += term;
        const long double px2 = ((2.0L * k + 3.0L) * x * px1 - (k + 1.0L) * px0) / (k + 2.0L);
        const long double py2 = ((2.0L * k + 3.0L) * y * py1 - (k + 1.0L) * py0) / (k + 2.0L);
        px0 = px1; px1 = px2;
        py0 = py1; py1 = py2;
      }
      t[size_t(j) * zb + b] = double(2.0L * w * se);
      t[size_t(zj + j) * zb + b] = double(2.0L * w * so);
    }
  }
  out.insert(out.end(), t.begin(), t.end());
}

rlb_status validate(const rlb_tube_desc& d, int k, std::string& msg) {
  char buf[256];
  auto bad = [&](const char* what) {
    std::snprintf(buf, sizeof buf, "tube %d: %s", k, what);
    msg = buf;
    return RLB_ERR_INVALID_ARG;
  };
  // the stage kernel addresses a chunk of rows with 32-bit byte offsets
  if (d.nx < 8 || d.nx > (1 << 26)) return bad("nx must be in [8, 2^26]");
  if (d.q_xi < 1 || d.q_xi > 4096) return bad("q_xi must be in [1, 4096]");
  if (d.q_p < 1 || d.q_p > kMaxQp) return bad("q_p must be in [1, 8]");
  if (d.n_v < 0 || d.n_v > kMaxNvHigh) return bad("n_v must be in [0, 255]");
  // the high-order form (n_v > 7) keeps q_xi <= 256 and, as the quadrature
  // section requires of the truncation, n_v < q_xi
  if (d.n_v > kMaxNv && (d.q_xi > kMaxQxHigh || d.n_v >= d.q_xi))
    return bad("n_v > 7 needs n_v < q_xi <= 256");
  if (d.n_p < 0 || d.n_p >= d.q_p) return bad("n_p must satisfy 0 <= n_p < q_p");
  if (d.n_p + 2 > 2 * d.q_p - 1) return bad("q_p too small to integrate T^{mu nu} of the equilibrium exactly");
  if (d.n_v + 2 > 2 * d.q_xi - 1) return bad("q_xi too small to integrate T^{mu nu} of the equilibrium exactly");
  if (!(d.z_max > d.z_min) || !std::isfinite(d.z_min) || !std::isfinite(d.z_max)) return bad("need z_min < z_max");
  if (!(d.tau > 0)) return bad("tau must be > 0 (+inf allowed)");
  if (!(d.T0 > 0) || !std::isfinite(d.T0)) return bad("T0 must be > 0");
  if (!(d.weno_eps > 0) || !std::isfinite(d.weno_eps)) return bad("weno_eps must be > 0 and finite");
  if (d.dt < 0 || !std::isfinite(d.dt)) return bad("dt must be >= 0");
  if (d.dt == 0 && !(d.cfl > 0 && std::isfinite(d.cfl))) return bad("cfl must be > 0");
  if (d.dt == 0 && !(d.dt_tau_max > 0)) return bad("dt_tau_max must be > 0");
  const double dt = tube_dt(d), dz = (d.z_max - d.z_min) / d.nx;
  if (!(dt > 0) || !std::isfinite(dt)) return bad("time step is not a positive number");
  if (dt > 1.5 * dz) {
    std::snprintf(buf, sizeof buf, "tube %d: dt/dz = %g exceeds the WENO5/RK3 stability limit 1.5", k, dt / dz);
    msg = buf;
    return RLB_ERR_UNSTABLE_DT;
  }
  if (dt > 2.5 * d.tau) {
    std::snprintf(buf, sizeof buf, "tube %d: dt/tau = %g exceeds the RK3 stability limit 2.5", k, dt / d.tau);
    msg = buf;
    return RLB_ERR_UNSTABLE_DT;
  }
  return RLB_OK;
}

void build_items(rlb_lattice* L) {
  const int tile = L->sched.tile;
  std::map<std::pair<int, int>, std::vector<int>> by_group;
  for (int t = 0; t < L->ntubes; ++t) {
    int qpt, nvt;
    kernel_group(L->desc[t].q_p, L->desc[t].n_v, &qpt, &nvt);
    by_group[{qpt, nvt}].push_back(t);
  }
  L->items.clear();
  L->groups.clear();
  for (auto& kv : by_group) {
    Group g;
    g.qpt = kv.first.first;
    g.nvt = kv.first.second;
    g.item_begin = static_cast<int>(L->items.size());
    g.qp_max = 1;
    g.zj_max = 0;
    std::vector<std::pair<int64_t, WorkItem>> tmp;
    for (int t : kv.second) {
      g.qp_max = std::max(g.qp_max, L->desc[t].q_p);
      if (L->desc[t].n_v > kMaxNv) g.zj_max = std::max(g.zj_max, high_rows(L->desc[t].q_xi));
      const int64_t cost = int64_t(L->desc[t].q_xi) * L->desc[t].q_p;
      for (int x0 = 0; x0 < L->desc[t].nx; x0 += tile) tmp.push_back({cost, WorkItem{t, x0}});
    }
    // most expensive tiles first (balances persistent grids); stable within a tube
    std::stable_sort(tmp.begin(), tmp.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    for (auto& e : tmp) L->items.push_back(e.second);
    g.item_end = static_cast<int>(L->items.size());
    L->groups.push_back(g);
  }
}

void drop_graph(rlb_lattice* L) {
  if (L->graph_exec) (void)hipGraphExecDestroy(L->graph_exec);
  if (L->graph) (void)hipGraphDestroy(L->graph);
  L->graph_exec = nullptr;
  L->graph = nullptr;
  L->graph_steps = 0;
}

rlb_status upload(rlb_lattice* L, size_t off, const void* src, size_t bytes) {
  if (!bytes) return RLB_OK;
  HIP_TRY(L, hipMemcpyAsync(L->ws + off, src, bytes, hipMemcpyHostToDevice, L->stream));
  HIP_TRY(L, hipStreamSynchronize(L->stream));
  return RLB_OK;
}

LaunchShape shape(const rlb_lattice* L, const Group& g) {
  LaunchShape ls;
  ls.tile = L->sched.tile;
  ls.chunk = L->sched.chunk > 0 ? L->sched.chunk : (L->prec == RLB_FP32 ? 8 : 4);
  const int n = g.item_end - g.item_begin;
  ls.grid = n;
  ls.nodes = 1;
  const int split_below = L->sched.split_below < 0 ? L->cu_count : L->sched.split_below;
  if (L->sched.persistent) ls.grid = std::max(1, std::min(n, L->sched.blocks_per_cu * std::max(1, L->cu_count)));
  // too few tiles to fill the GPU: one workgroup per (tile, radial node)
  else if (L->off_part && g.qp_max > 1 && n < split_below) ls.nodes = g.qp_max;
  return ls;
}

// Side stream and events of the pipelined high-order pre-pass (none on failure).
void drop_side(rlb_lattice* L) {
  for (hipEvent_t& ev : L->ev_pre)
    if (ev) (void)hipEventDestroy(ev), ev = nullptr;
  for (hipEvent_t& ev : L->ev_stage)
    if (ev) (void)hipEventDestroy(ev), ev = nullptr;
  if (L->ev_fork) (void)hipEventDestroy(L->ev_fork), L->ev_fork = nullptr;
  if (L->side) (void)hipStreamDestroy(L->side), L->side = nullptr;
  L->side_device = -1;
}
void make_side(rlb_lattice* L) {
  int dev = -1;
  bool ok = hipGetDevice(&dev) == hipSuccess && hipStreamCreateWithFlags(&L->side, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&L->ev_fork, hipEventDisableTiming) == hipSuccess;
  for (hipEvent_t& ev : L->ev_pre) ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
  for (hipEvent_t& ev : L->ev_stage) ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    drop_side(L);
    (void)hipGetLastError();
    return;
  }
  L->side_device = dev;
}

// Pieces of a high-order stage (1: no pipelining): with the side stream on the
// current device, one workgroup per tile and at least two tiles per CU in
// every piece.
int pipe_pieces(const rlb_lattice* L, const LaunchShape& ls, int nitems) {
  if (!L->side || ls.nodes > 1) return 1;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != L->side_device) return 1;
  return std::max(1, std::min(kPipePieces, nitems / (2 * std::max(1, L->cu_count))));
}

// High-order equilibrium pre-pass of one kernel group: F_eq of the state whose
// records are `rec`, or with rec == nullptr of the masked tubes' initial side
// states, into `out`.  Large groups take one workgroup per tile for all radial
// nodes (the tables are staged once per tile); small ones spread the nodes
// over a second grid dimension.  max_grid > 0 caps the workgroups (each then
// loops over several tiles).
template <typename Real>
hipError_t equilibrium_pass(rlb_lattice* L, const Group& g, const double* rec, void* out, hipStream_t s,
                            int max_grid = 0) {
  FeqArgs<Real> f;
  f.tubes = L->dev<TubeDev>(L->off_tubes);
  f.items = L->dev<WorkItem>(L->off_items) + g.item_begin;
  f.nitems = g.item_end - g.item_begin;
  f.tile = L->sched.tile;
  f.itab = L->dev<double>(L->off_itab);
  f.ztab = L->dev<double>(L->off_ztab);
  f.rec = rec;
  f.sides = L->dev<double>(L->off_sides);
  f.tube_mask = L->dev<int32_t>(L->off_mask);
  f.out = static_cast<Real*>(out);
  f.row_tiles = (g.zj_max + 15) / 16;
  LaunchShape ls;
  ls.tile = L->sched.tile;
  ls.grid = max_grid > 0 ? std::min(f.nitems, max_grid) : f.nitems;
  ls.nodes = f.nitems < 2 * std::max(1, L->cu_count) ? g.qp_max : 1;
  return launch_feq(sizeof(Real) == 4, ls, &f, s);
}

// One SSP-RK3 stage of one kernel group with explicit buffers: the stage
// kernel (after the equilibrium pre-pass for the high-order group) and, for a
// split launch, the kernel that forms the records.
template <typename Real>
hipError_t stage_group(rlb_lattice* L, const Group& g, int stage, const void* fin, const void* fn, void* fout,
                       const double* rec_in, double* rec_out, hipStream_t s) {
  const LaunchShape ls = shape(L, g);
  StageArgs<Real> a;
  a.tubes = L->dev<TubeDev>(L->off_tubes);
  a.items = L->dev<WorkItem>(L->off_items) + g.item_begin;
  a.nitems = g.item_end - g.item_begin;
  a.stage = stage;
  a.aux_pairs = L->aux_pairs;
  a.jtab = L->dev<Real>(L->off_jtab);
  a.itab = L->dev<double>(L->off_itab);
  a.aux = L->dev<Real>(L->off_aux);
  a.fin = static_cast<const Real*>(fin);
  a.fn = static_cast<const Real*>(fn);
  a.fout = static_cast<Real*>(fout);
  a.rec_in = rec_in;
  a.rec_out = rec_out;
  a.flag = L->flag();
  a.part = ls.nodes > 1 ? L->dev<double>(L->off_part) : nullptr;
  a.part_stride = L->part_stride;
  a.feq = nullptr;
  hipError_t e = hipSuccess;
  if (g.nvt == kNvtHigh) {
    a.feq = L->dev<Real>(L->off_feq);
    const int pieces = pipe_pieces(L, ls, a.nitems);
    if (pieces > 1) {
      // The pre-pass of a piece needs only the records of its own cells and
      // overwrites only its cells' equilibrium values, so it waits for the
      // previous stage's kernel of the same piece (or, first in a call, for
      // everything before on s); the stage kernel of a piece waits for its
      // piece's pre-pass, and the stage kernels keep their order on s (halos).
      // In FP64 the stage kernel is the slower of the two: a piece's pre-pass
      // then takes one workgroup per CU, looping over its tiles, which leaves
      // registers for more waves of the memory-bound stage kernel beside it
      // (in FP32 the pre-pass is the slower one and takes a workgroup per tile).
      const int pre_grid = sizeof(Real) == 8 ? std::max(1, L->cu_count) : 0;
      if (!L->pipe_forked) {
        if ((e = hipEventRecord(L->ev_fork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(L->side, L->ev_fork, 0)) != hipSuccess) return e;
      }
      for (int p = 0; p < pieces; ++p) {
        const int b = int(int64_t(a.nitems) * p / pieces), en = int(int64_t(a.nitems) * (p + 1) / pieces);
        Group gp = g;
        gp.item_begin = g.item_begin + b;
        gp.item_end = g.item_begin + en;
        if (L->pipe_forked && (e = hipStreamWaitEvent(L->side, L->ev_stage[p], 0)) != hipSuccess) return e;
        if ((e = equilibrium_pass<Real>(L, gp, rec_in, L->ws + L->off_feq, L->side, pre_grid)) != hipSuccess) return e;
        if ((e = hipEventRecord(L->ev_pre[p], L->side)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, L->ev_pre[p], 0)) != hipSuccess) return e;
        StageArgs<Real> ap = a;
        ap.items = a.items + b;
        ap.nitems = en - b;
        LaunchShape lp = ls;
        lp.grid = L->sched.persistent ? std::min(ls.grid, en - b) : en - b;
        if ((e = launch_stage(sizeof(Real) == 4, g.qpt, g.nvt, lp, &ap, s)) != hipSuccess) return e;
        if ((e = hipEventRecord(L->ev_stage[p], s)) != hipSuccess) return e;
      }
      L->pipe_forked = true;
      return hipSuccess;
    }
    e = equilibrium_pass<Real>(L, g, rec_in, L->ws + L->off_feq, s);
    if (e != hipSuccess) return e;
  }
  e = launch_stage(sizeof(Real) == 4, g.qpt, g.nvt, ls, &a, s);
  if (e == hipSuccess && ls.nodes > 1)
    e = launch_combine(a.tubes, a.items, a.nitems, ls.tile, a.itab, a.part, a.part_stride, rec_out, s);
  return e;
}

rlb_status enqueue_steps(rlb_lattice* L, hipStream_t s, int64_t nsteps) {
  const bool fp32 = L->prec == RLB_FP32;
  L->pipe_forked = false;
  for (int64_t n = 0; n < nsteps; ++n) {
    for (int stage = 1; stage <= 3; ++stage) {
      const int fin = stage == 1 ? 0 : (stage == 2 ? 1 : 2);
      const int fout = stage == 1 ? 1 : (stage == 2 ? 2 : 0);
      const int rin = fin, rout = fout;
      for (const Group& g : L->groups) {
        const void* Fin = L->F(fin);
        const void* Fn = L->F(0);
        void* Fout = L->F(fout);
        const double* Rin = L->dev<double>(L->off_rec[rin]);
        double* Rout = L->dev<double>(L->off_rec[rout]);
        const hipError_t e = fp32 ? stage_group<float>(L, g, stage, Fin, Fn, Fout, Rin, Rout, s)
                                  : stage_group<double>(L, g, stage, Fin, Fn, Fout, Rin, Rout, s);
        if (e != hipSuccess) return hip_fail(L, e, "stage kernel launch");
      }
    }
  }
  return RLB_OK;
}

rlb_status ensure_graph(rlb_lattice* L) {
  const int G = L->sched.graph_steps;
  if (L->graph_exec && L->graph_steps == G) return RLB_OK;
  drop_graph(L);
  hipStream_t cap;
  HIP_TRY(L, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cap);
    return hip_fail(L, e, "hipStreamBeginCapture");
  }
  rlb_status st = enqueue_steps(L, cap, G);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cap, &graph);
  (void)hipStreamDestroy(cap);
  if (st != RLB_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(L, e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(L, e, "hipGraphInstantiate");
  }
  L->graph = graph;
  L->graph_exec = exec;
  L->graph_steps = G;
  return RLB_OK;
}

bool check_tube(const rlb_lattice* L, int32_t tube) { return tube >= 0 && tube < L->ntubes; }

rlb_status need_ready(rlb_lattice* L, bool need_init) {
  if (!L) return RLB_ERR_INVALID_ARG;
  if (!L->ws) return fail(L, RLB_ERR_STATE, "no workspace bound (call rlb_bind)");
  if (need_init && !L->initialised) return fail(L, RLB_ERR_STATE, "no state (call rlb_set_initial_state or rlb_set_state)");
  return RLB_OK;
}

rlb_status read_flag(rlb_lattice* L) {
  unsigned flag = 0;
  HIP_TRY(L, hipMemcpyAsync(&flag, L->ws + L->off_flag, sizeof flag, hipMemcpyDeviceToHost, L->stream));
  HIP_TRY(L, hipStreamSynchronize(L->stream));
  if (flag & kFlagNonphysical)
    return fail(L, RLB_ERR_NONPHYSICAL, "a cell reached a non-physical state (e <= 0, n <= 0, |v| >= 1 or NaN)");
  return RLB_OK;
}

}  // namespace

extern "C" {

rlb_status rlb_tube_defaults(rlb_tube_desc* d) {
  if (!d) return RLB_ERR_INVALID_ARG;
  std::memset(d, 0, sizeof *d);
  d->nx = 800;
  d->q_xi = 8;
  d->q_p = 3;
  d->n_v = 5;
  d->n_p = 2;
  d->z_min = -0.5;
  d->z_max = 0.5;
  d->tau = 1e-2;
  d->cfl = 0.5;
  d->dt_tau_max = 0.5;
  d->dt = 0.0;
  d->T0 = 1.0;
  d->weno_eps = 1e-6;
  return RLB_OK;
}

rlb_status rlb_create(const rlb_tube_desc* tubes, int32_t ntubes, rlb_precision prec, uint32_t flags,
                      rlb_lattice** out) {
  if (!out) return fail(nullptr, RLB_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!tubes || ntubes < 1) return fail(nullptr, RLB_ERR_INVALID_ARG, "need ntubes >= 1 descriptors");
  if (prec != RLB_FP64 && prec != RLB_FP32) return fail(nullptr, RLB_ERR_INVALID_ARG, "unknown precision");
  if (flags & ~RLB_WITH_ADJOINT) return fail(nullptr, RLB_ERR_INVALID_ARG, "unknown flags");
  for (int k = 0; k < ntubes; ++k) {
    std::string msg;
    rlb_status st = validate(tubes[k], k, msg);
    if (st != RLB_OK) return fail(nullptr, st, msg);
    if (!rlb::weno_eps_in_range(tubes[k].weno_eps, prec == RLB_FP32))
      return fail(nullptr, RLB_ERR_INVALID_ARG,
                  "tube " + std::to_string(k) + ": weno_eps must lie in [1e-40, 1e30] (FP32) or [1e-300, 1e30] (FP64)");
  }
  rlb_lattice* L = new rlb_lattice();
  L->desc.assign(tubes, tubes + ntubes);
  L->ntubes = ntubes;
  L->prec = prec;
  L->flags = flags;
  L->rsize = prec == RLB_FP32 ? 4 : 8;
  L->time.assign(ntubes, 0.0);
  L->sides_h.assign(6 * size_t(ntubes), 0.0);
  L->mask_h.assign(ntubes, 0);

  // quadrature tables, shared between tubes with equal orders
  std::map<int, int> jrow_of;                          // q_xi -> first row
  std::map<std::tuple<int, double>, int> irow_of;      // (q_p, T0) -> first row
  std::map<std::pair<int, int>, int64_t> zoff_of;      // (q_xi, n_v) -> high-order table
  L->xi.resize(ntubes); L->wxi.resize(ntubes); L->p.resize(ntubes); L->wp.resize(ntubes);
  int64_t f_off = 0, rec_off = 0;
  for (int t = 0; t < ntubes; ++t) {
    const rlb_tube_desc& d = tubes[t];
    std::vector<double> x, w, px, pw;
    if (!gauss_legendre_rule(d.q_xi, x, w) || !gauss_laguerre1_rule(d.q_p, px, pw)) {
      delete L;
      return fail(nullptr, RLB_ERR_INVALID_ARG, "quadrature construction failed");
    }
    L->xi[t] = x; L->wxi[t] = w; L->p[t] = px; L->wp[t] = pw;
    int jrow, irow;
    auto jt = jrow_of.find(d.q_xi);
    if (jt == jrow_of.end()) {
      jrow = static_cast<int>(L->jtab_d.size() / kJStride);
      for (int j = 0; j < d.q_xi; ++j) {
        double row[kJStride];
        row[0] = x[j];
        row[1] = w[j];
        row[2] = w[j] * x[j];
        row[3] = w[j] * x[j] * x[j];
        for (int k = 0; k <= kMaxNv; ++k) row[4 + k] = legendre_value(k, x[j]);
        L->jtab_d.insert(L->jtab_d.end(), row, row + kJStride);
      }
      jrow_of[d.q_xi] = jrow;
    } else {
      jrow = jt->second;
    }
    auto key = std::make_tuple(d.q_p, d.T0);
    auto it = irow_of.find(key);
    if (it == irow_of.end()) {
      irow = static_cast<int>(L->itab.size() / kIStride);
      const double t3 = d.T0 * d.T0 * d.T0, t4 = t3 * d.T0;
      for (int i = 0; i < d.q_p; ++i) {
        double row[kIStride];
        row[0] = px[i];
        row[1] = pw[i];
        row[2] = t3 * pw[i] * px[i];
        row[3] = t4 * pw[i] * px[i] * px[i];
        for (int l = 0; l <= kMaxNp; ++l) row[4 + l] = laguerre1_value(l, px[i]);
        L->itab.insert(L->itab.end(), row, row + kIStride);
      }
      irow_of[key] = irow;
    } else {
      irow = it->second;
    }
    TubeDev td;
    std::memset(&td, 0, sizeof td);
    td.nx = d.nx;
    td.ldx = (d.nx + 63) / 64 * 64;
    td.qx = d.q_xi;
    td.qp = d.q_p;
    td.nv = d.n_v;
    td.np = d.n_p;
    td.jrow = jrow;
    td.irow = irow;
    td.z_min = d.z_min;
    td.dz = (d.z_max - d.z_min) / d.nx;
    td.dz_inv = 1.0 / td.dz;
    td.dt = tube_dt(d);
    td.tau_inv = 1.0 / d.tau;
    td.T0 = d.T0;
    td.weno_eps = d.weno_eps;
    if (d.n_v > kMaxNv) {
      const auto key = std::make_pair(d.q_xi, d.n_v);
      auto zt = zoff_of.find(key);
      if (zt == zoff_of.end()) {
        zt = zoff_of.emplace(key, int64_t(L->ztab.size())).first;
        high_order_table(d.q_xi, d.n_v, x, L->ztab);
      }
      td.z_off = zt->second;
      td.zj = high_rows(d.q_xi);
      td.zb = high_aux_pairs(d.n_v);
      L->has_high = true;
    }
    int qpt, nvt;
    kernel_group(d.q_p, d.n_v, &qpt, &nvt);
    td.group = qpt * 16 + nvt;
    td.f_off = f_off;
    td.rec_off = rec_off;
    td.cell_off = rec_off / 5;
    td.ldf = (d.nx + 1 + 63) / 64 * 64;
    td.face_off = L->face_elems;
    L->face_elems += int64_t(d.q_xi) * d.q_p * td.ldf;
    L->init_blocks_max = std::max(L->init_blocks_max, (d.nx + 255) / 256);
    if (d.n_v > kMaxNv) L->ipart_stride = std::max(L->ipart_stride, d.q_p * d.q_xi);
    f_off += int64_t(d.q_xi) * d.q_p * td.ldx;
    rec_off += 5 * int64_t(td.ldx);
    L->max_ldx = std::max(L->max_ldx, td.ldx);
    L->tubes.push_back(td);
  }
  L->state_elems = f_off;
  L->rec_elems = rec_off;
  L->cell_elems = rec_off / 5;
  L->jtab_f.assign(L->jtab_d.begin(), L->jtab_d.end());

  // auxiliary projection rule: symmetric pairs of a Gauss-Legendre rule
  const int M = prec == RLB_FP32 ? 2 * kAuxPairsFP32 : 2 * kAuxPairsFP64;
  std::vector<double> ax, aw;
  gauss_legendre_rule(M, ax, aw);
  L->aux_pairs = M / 2;
  for (int a = 0; a < M / 2; ++a) {
    const int j = M / 2 + a;  // positive nodes
    double row[kAuxStride];
    row[0] = ax[j];
    for (int k = 0; k <= kMaxNv; ++k) row[1 + k] = aw[j] * (2 * k + 1) / 2.0 * legendre_value(k, ax[j]);
    for (int k = kMaxNv + 2; k < kAuxStride; ++k) row[k] = 0.0;
    L->aux_d.insert(L->aux_d.end(), row, row + kAuxStride);
  }
  L->aux_f.assign(L->aux_d.begin(), L->aux_d.end());

  // work-list bound: smallest tile
  int64_t max_items = 0;
  for (auto& d : L->desc) max_items += (d.nx + 63) / 64;
  L->max_items = static_cast<int>(max_items);

  // workspace layout: first everything a time step uses besides the state
  // f^n (the stage arrays, records, tables, flag, buffers), up to
  // step_bytes, then f^n, then the adjoint's arrays; the allocation-free step
  // keeps the first part in its static scratch array and takes f^n from the
  // caller
  size_t o = 0;
  for (int k = 1; k < 3; ++k) { L->off_F[k] = o; o = align256(o + L->state_elems * L->rsize); }
  for (int k = 0; k < 3; ++k) { L->off_rec[k] = o; o = align256(o + L->rec_elems * 8); }
  L->off_tubes = o; o = align256(o + L->tubes.size() * sizeof(TubeDev));
  L->off_jtab = o; o = align256(o + L->jtab_d.size() * L->rsize);
  L->off_itab = o; o = align256(o + L->itab.size() * 8);
  L->off_aux = o; o = align256(o + L->aux_d.size() * L->rsize);
  L->off_aux_d = o; o = align256(o + L->aux_d.size() * 8);
  L->off_items = o; o = align256(o + size_t(L->max_items) * sizeof(WorkItem));
  L->off_sides = o; o = align256(o + L->sides_h.size() * 8);
  L->off_mask = o; o = align256(o + L->mask_h.size() * 4);
  L->off_flag = o; o = align256(o + 16);
  L->off_fields = o; o = align256(o + 10 * size_t(L->max_ldx) * 8);
  L->off_totals = o; o = align256(o + 4 * 8);
  if (L->has_high) {
    L->off_ztab = o; o = align256(o + L->ztab.size() * 8);
    L->off_feq = o; o = align256(o + L->state_elems * L->rsize);
  }
  if (L->cell_elems <= kSplitMaxCells) {
    int qp_max = 1;
    for (auto& d : L->desc) qp_max = std::max(qp_max, d.q_p);
    L->part_stride = 3 * qp_max;
    L->off_part = o; o = align256(o + size_t(L->cell_elems) * L->part_stride * 8);
  }
  L->step_bytes = o;
  L->off_F[0] = o; o = align256(o + L->state_elems * L->rsize);
  if (flags & RLB_WITH_ADJOINT) {
    for (int k = 0; k < 2; ++k) { L->off_aF[k] = o; o = align256(o + L->state_elems * L->rsize); }
    for (int k = 0; k < 3; ++k) { L->off_arec[k] = o; o = align256(o + L->rec_elems * 8); }
    L->off_lam2 = o; o = align256(o + L->state_elems * L->rsize);
    L->off_lam1 = o; o = align256(o + L->state_elems * L->rsize);
    L->off_acc = o; o = align256(o + L->state_elems * L->rsize);
    L->off_G = o; o = align256(o + 5 * size_t(L->face_elems) * L->rsize);
    L->off_cellbuf = o; o = align256(o + 7 * size_t(L->cell_elems) * 8);
    L->off_tauacc = o; o = align256(o + size_t(L->cell_elems) * 8);
    L->off_ipart = o; o = align256(o + size_t(L->init_blocks_max) * 2 * L->ipart_stride * 8);
    // a buffer of its own, so that a forward recompute on another stream
    // (the segment halves) never overwrites the values an adjoint stage reads
    if (L->has_high) { L->off_afeq = o; o = align256(o + L->state_elems * L->rsize); }
    L->off_grad = o; o = align256(o + 8 * 8);
  }
  L->total = o;

  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) L->cu_count = prop.multiProcessorCount;
  }
  // default tile: 256 cells, or 64 when 256-cell tiles would leave more than
  // half of the CUs without work (small lattices: more, shorter workgroups)
  int64_t tiles256 = 0;
  for (auto& d : L->desc) tiles256 += (d.nx + 255) / 256;
  if (L->cu_count > 0 && 2 * tiles256 < L->cu_count) L->sched.tile = 64;
  build_items(L);
  *out = L;
  return RLB_OK;
}

rlb_status rlb_destroy(rlb_lattice* L) {
  if (!L) return RLB_ERR_INVALID_ARG;
  drop_graph(L);
  drop_side(L);
  delete L;
  return RLB_OK;
}

rlb_status rlb_workspace_size(const rlb_lattice* L, size_t* bytes) {
  if (!L || !bytes) return RLB_ERR_INVALID_ARG;
  *bytes = L->total;
  return RLB_OK;
}

rlb_status rlb_bind(rlb_lattice* L, void* workspace, size_t bytes, void* hip_stream) {
  if (!L) return RLB_ERR_INVALID_ARG;
  if (!workspace) return fail(L, RLB_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(L, RLB_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (bytes < L->total) return fail(L, RLB_ERR_INVALID_ARG, "workspace too small (see rlb_workspace_size)");
  drop_graph(L);
  L->ws = static_cast<char*>(workspace);
  L->ws_bytes = bytes;
  L->stream = static_cast<hipStream_t>(hip_stream);
  L->initialised = false;
  rlb_status st;
  // the padding cells of the state rows (x >= nx) are never written by the
  // kernels: start them, and everything else, at zero so that copies of a
  // state are deterministic
  HIP_TRY(L, hipMemsetAsync(L->ws, 0, L->total, L->stream));
  if ((st = upload(L, L->off_tubes, L->tubes.data(), L->tubes.size() * sizeof(TubeDev))) != RLB_OK) return st;
  if (L->prec == RLB_FP32) {
    if ((st = upload(L, L->off_jtab, L->jtab_f.data(), L->jtab_f.size() * 4)) != RLB_OK) return st;
    if ((st = upload(L, L->off_aux, L->aux_f.data(), L->aux_f.size() * 4)) != RLB_OK) return st;
  } else {
    if ((st = upload(L, L->off_jtab, L->jtab_d.data(), L->jtab_d.size() * 8)) != RLB_OK) return st;
    if ((st = upload(L, L->off_aux, L->aux_d.data(), L->aux_d.size() * 8)) != RLB_OK) return st;
  }
  if ((st = upload(L, L->off_itab, L->itab.data(), L->itab.size() * 8)) != RLB_OK) return st;
  if ((st = upload(L, L->off_aux_d, L->aux_d.data(), L->aux_d.size() * 8)) != RLB_OK) return st;
  if ((st = upload(L, L->off_items, L->items.data(), L->items.size() * sizeof(WorkItem))) != RLB_OK) return st;
  if ((st = upload(L, L->off_ztab, L->ztab.data(), L->ztab.size() * 8)) != RLB_OK) return st;
  HIP_TRY(L, hipMemsetAsync(L->ws + L->off_flag, 0, 16, L->stream));
  HIP_TRY(L, hipStreamSynchronize(L->stream));
  if (L->has_high && !L->side) make_side(L);  // without it the pre-pass runs unpipelined
  return RLB_OK;
}

rlb_status rlb_set_stream(rlb_lattice* L, void* hip_stream) {
  if (!L) return RLB_ERR_INVALID_ARG;
  L->stream = static_cast<hipStream_t>(hip_stream);
  return RLB_OK;
}

rlb_status rlb_set_schedule(rlb_lattice* L, const rlb_schedule* s) {
  if (!L || !s) return RLB_ERR_INVALID_ARG;
  if (s->tile != 64 && s->tile != 128 && s->tile != 256)
    return fail(L, RLB_ERR_INVALID_ARG, "tile must be 64, 128 or 256");
  const int ch = L->prec == RLB_FP32 ? 8 : 4;
  if (s->chunk != 0 && s->chunk != ch && s->chunk != 2 * ch)
    return fail(L, RLB_ERR_INVALID_ARG, "chunk must be 0, the default (8 FP32, 4 FP64) or twice it");
  if (s->split_below < -1) return fail(L, RLB_ERR_INVALID_ARG, "split_below must be >= -1");
  // a chunk's rows are one buffer resource of chunk * ldx * sizeof(Real) bytes (32-bit size)
  const int64_t chunk_rows = s->chunk > 0 ? s->chunk : ch;
  if (chunk_rows * int64_t(L->max_ldx) * int64_t(L->rsize) >= (int64_t(1) << 32))
    return fail(L, RLB_ERR_INVALID_ARG, "chunk too large for the longest tube (chunk x padded row bytes >= 2^32)");
  if (s->persistent != 0 && s->persistent != 1) return fail(L, RLB_ERR_INVALID_ARG, "persistent must be 0 or 1");
  if (s->blocks_per_cu < 1 || s->blocks_per_cu > 64) return fail(L, RLB_ERR_INVALID_ARG, "blocks_per_cu in [1, 64]");
  if (s->graph_steps < 0 || s->graph_steps > 4096) return fail(L, RLB_ERR_INVALID_ARG, "graph_steps in [0, 4096]");
  const bool new_items = s->tile != L->sched.tile;
  L->sched = *s;
  drop_graph(L);
  if (new_items) {
    build_items(L);
    if (L->ws) return upload(L, L->off_items, L->items.data(), L->items.size() * sizeof(WorkItem));
  }
  return RLB_OK;
}

rlb_status rlb_get_schedule(const rlb_lattice* L, rlb_schedule* s) {
  if (!L || !s) return RLB_ERR_INVALID_ARG;
  *s = L->sched;
  return RLB_OK;
}

namespace {

bool good_state(const rlb_state& s) {
  return s.P > 0 && s.n > 0 && std::isfinite(s.P) && std::isfinite(s.n) && std::isfinite(s.u);
}

rlb_status launch_init_all(rlb_lattice* L) {
  rlb_status st;
  if ((st = upload(L, L->off_sides, L->sides_h.data(), L->sides_h.size() * 8)) != RLB_OK) return st;
  if ((st = upload(L, L->off_mask, L->mask_h.data(), L->mask_h.size() * 4)) != RLB_OK) return st;
  const bool fp32 = L->prec == RLB_FP32;
  for (const Group& g : L->groups) {
    LaunchShape ls = shape(L, g);
    hipError_t e;
    if (g.nvt == kNvtHigh) {
      // the equilibrium of the side states, then the records of the state
      // (records of unmasked tubes are recomputed from their state: equal to
      // the bit)
      void* f0 = L->ws + L->off_F[0];
      e = fp32 ? equilibrium_pass<float>(L, g, nullptr, f0, L->stream)
               : equilibrium_pass<double>(L, g, nullptr, f0, L->stream);
      if (e == hipSuccess)
        e = launch_moments(fp32 ? 1 : 0, L->dev<TubeDev>(L->off_tubes), L->dev<WorkItem>(L->off_items) + g.item_begin,
                           g.item_end - g.item_begin, L->sched.tile, L->ws + L->off_jtab, L->dev<double>(L->off_itab),
                           f0, L->dev<double>(L->off_rec[0]), L->stream);
    } else if (fp32) {
      InitArgs<float> a;
      a.tubes = L->dev<TubeDev>(L->off_tubes);
      a.items = L->dev<WorkItem>(L->off_items) + g.item_begin;
      a.nitems = g.item_end - g.item_begin;
      a.aux_pairs = L->aux_pairs;
      a.jtab = L->dev<float>(L->off_jtab);
      a.itab = L->dev<double>(L->off_itab);
      a.aux = L->dev<float>(L->off_aux);
      a.sides = L->dev<double>(L->off_sides);
      a.tube_mask = L->dev<int32_t>(L->off_mask);
      a.f = L->dev<float>(L->off_F[0]);
      a.rec = L->dev<double>(L->off_rec[0]);
      a.flag = L->dev<unsigned>(L->off_flag);
      e = launch_init(1, g.qpt, g.nvt, ls, &a, L->stream);
    } else {
      InitArgs<double> a;
      a.tubes = L->dev<TubeDev>(L->off_tubes);
      a.items = L->dev<WorkItem>(L->off_items) + g.item_begin;
      a.nitems = g.item_end - g.item_begin;
      a.aux_pairs = L->aux_pairs;
      a.jtab = L->dev<double>(L->off_jtab);
      a.itab = L->dev<double>(L->off_itab);
      a.aux = L->dev<double>(L->off_aux);
      a.sides = L->dev<double>(L->off_sides);
      a.tube_mask = L->dev<int32_t>(L->off_mask);
      a.f = L->dev<double>(L->off_F[0]);
      a.rec = L->dev<double>(L->off_rec[0]);
      a.flag = L->dev<unsigned>(L->off_flag);
      e = launch_init(0, g.qpt, g.nvt, ls, &a, L->stream);
    }
    if (e != hipSuccess) return hip_fail(L, e, "init kernel launch");
  }
  return RLB_OK;
}

}  // namespace

rlb_status rlb_set_initial_state(rlb_lattice* L, int32_t tube, rlb_state left, rlb_state right) {
  rlb_status st = need_ready(L, false);
  if (st != RLB_OK) return st;
  if (tube != -1 && !check_tube(L, tube)) return fail(L, RLB_ERR_INVALID_ARG, "tube index out of range");
  if (!good_state(left) || !good_state(right))
    return fail(L, RLB_ERR_INVALID_ARG, "initial states need P > 0, n > 0 and finite u");
  if (!L->initialised && tube != -1) return fail(L, RLB_ERR_STATE, "the first initial state must set every tube (tube = -1)");
  for (int t = 0; t < L->ntubes; ++t) {
    const bool on = tube == -1 || t == tube;
    L->mask_h[t] = on ? 1 : 0;
    if (on) {
      double* s = &L->sides_h[6 * size_t(t)];
      s[0] = left.P; s[1] = left.n; s[2] = left.u;
      s[3] = right.P; s[4] = right.n; s[5] = right.u;
      L->time[t] = 0.0;
    }
  }
  if ((st = launch_init_all(L)) != RLB_OK) return st;
  if (tube == -1) HIP_TRY(L, hipMemsetAsync(L->ws + L->off_flag, 0, 16, L->stream));
  L->initialised = true;
  return RLB_OK;
}

rlb_status rlb_set_initial_states(rlb_lattice* L, int32_t ntubes, const rlb_state* left, const rlb_state* right) {
  rlb_status st = need_ready(L, false);
  if (st != RLB_OK) return st;
  if (ntubes != L->ntubes || !left || !right) return fail(L, RLB_ERR_INVALID_ARG, "need one left/right state per tube");
  for (int t = 0; t < ntubes; ++t)
    if (!good_state(left[t]) || !good_state(right[t]))
      return fail(L, RLB_ERR_INVALID_ARG, "initial states need P > 0, n > 0 and finite u");
  for (int t = 0; t < ntubes; ++t) {
    L->mask_h[t] = 1;
    double* s = &L->sides_h[6 * size_t(t)];
    s[0] = left[t].P; s[1] = left[t].n; s[2] = left[t].u;
    s[3] = right[t].P; s[4] = right[t].n; s[5] = right[t].u;
    L->time[t] = 0.0;
  }
  if ((st = launch_init_all(L)) != RLB_OK) return st;
  HIP_TRY(L, hipMemsetAsync(L->ws + L->off_flag, 0, 16, L->stream));
  L->initialised = true;
  return RLB_OK;
}

rlb_status rlb_step(rlb_lattice* L, int64_t nsteps) {
  rlb_status st = need_ready(L, true);
  if (st != RLB_OK) return st;
  if (nsteps < 0) return fail(L, RLB_ERR_INVALID_ARG, "nsteps must be >= 0");
  int64_t done = 0;
  if (L->sched.graph_steps > 0 && nsteps >= L->sched.graph_steps) {
    if ((st = ensure_graph(L)) != RLB_OK) return st;
    for (; done + L->graph_steps <= nsteps; done += L->graph_steps)
      HIP_TRY(L, hipGraphLaunch(L->graph_exec, L->stream));
  }
  if ((st = enqueue_steps(L, L->stream, nsteps - done)) != RLB_OK) return st;
  for (int t = 0; t < L->ntubes; ++t) L->time[t] += nsteps * L->tubes[t].dt;
  return RLB_OK;
}

rlb_status rlb_fields(rlb_lattice* L, int32_t tube, double* dev_out, int64_t ld) {
  rlb_status st = need_ready(L, true);
  if (st != RLB_OK) return st;
  if (!check_tube(L, tube)) return fail(L, RLB_ERR_INVALID_ARG, "tube index out of range");
  if (!dev_out || ld < L->tubes[tube].nx) return fail(L, RLB_ERR_INVALID_ARG, "need dev_out and ld >= nx");
  hipError_t e = launch_fields(L->dev<TubeDev>(L->off_tubes), tube, L->tubes[tube].nx, L->dev<double>(L->off_rec[0]),
                               dev_out, ld, L->dev<unsigned>(L->off_flag), L->stream);
  if (e != hipSuccess) return hip_fail(L, e, "fields kernel launch");
  return RLB_OK;
}

rlb_status rlb_moments(rlb_lattice* L, int32_t tube, double* host_out, int64_t ld) {
  rlb_status st = need_ready(L, true);
  if (st != RLB_OK) return st;
  if (!check_tube(L, tube)) return fail(L, RLB_ERR_INVALID_ARG, "tube index out of range");
  const int nx = L->tubes[tube].nx;
  if (!host_out || ld < nx) return fail(L, RLB_ERR_INVALID_ARG, "need host_out and ld >= nx");
  double* scratch = L->dev<double>(L->off_fields);
  if ((st = rlb_fields(L, tube, scratch, nx)) != RLB_OK) return st;
  HIP_TRY(L, hipMemcpy2DAsync(host_out, ld * 8, scratch, size_t(nx) * 8, size_t(nx) * 8, 10, hipMemcpyDeviceToHost,
                              L->stream));
  HIP_TRY(L, hipStreamSynchronize(L->stream));
  return read_flag(L);
}

rlb_status rlb_totals(rlb_lattice* L, int32_t tube, double out[3]) {
  rlb_status st = need_ready(L, true);
  if (st != RLB_OK) return st;
  if (!check_tube(L, tube) || !out) return fail(L, RLB_ERR_INVALID_ARG, "bad tube or out");
  double* d = L->dev<double>(L->off_totals);
  hipError_t e = launch_totals(L->dev<TubeDev>(L->off_tubes), tube, L->dev<double>(L->off_rec[0]), d, L->stream);
  if (e != hipSuccess) return hip_fail(L, e, "totals kernel launch");
  HIP_TRY(L, hipMemcpyAsync(out, d, 3 * 8, hipMemcpyDeviceToHost, L->stream));
  HIP_TRY(L, hipStreamSynchronize(L->stream));
  return read_flag(L);
}

rlb_status rlb_check(rlb_lattice* L) {
  rlb_status st = need_ready(L, false);
  if (st != RLB_OK) return st;
  return read_flag(L);
}

rlb_status rlb_flags(rlb_lattice* L, uint32_t* flags) {
  rlb_status st = need_ready(L, false);
  if (st != RLB_OK) return st;
  if (!flags) return fail(L, RLB_ERR_INVALID_ARG, "flags is NULL");
  unsigned flag = 0;
  HIP_TRY(L, hipMemcpyAsync(&flag, L->ws + L->off_flag, sizeof flag, hipMemcpyDeviceToHost, L->stream));
  HIP_TRY(L, hipStreamSynchronize(L->stream));
  *flags = flag;
  return RLB_OK;
}

rlb_status rlb_state_elems(const rlb_lattice* L, int64_t* elems) {
  if (!L || !elems) return RLB_ERR_INVALID_ARG;
  *elems = L->state_elems;
  return RLB_OK;
}

rlb_status rlb_state_layout(const rlb_lattice* L, int32_t tube, int64_t* off, int64_t* ld) {
  if (!L || !off || !ld || !check_tube(L, tube)) return RLB_ERR_INVALID_ARG;
  *off = L->tubes[tube].f_off;
  *ld = L->tubes[tube].ldx;
  return RLB_OK;
}

rlb_status rlb_get_state(rlb_lattice* L, void* dst) {
  rlb_status st = need_ready(L, true);
  if (st != RLB_OK) return st;
  if (!dst) return fail(L, RLB_ERR_INVALID_ARG, "dst is NULL");
  hipError_t e = state_copy(dst, L->ws + L->off_F[0], L->state_elems * L->rsize, L->stream);
  if (e != hipSuccess) return hip_fail(L, e, "state copy");
  return RLB_OK;
}

rlb_status rlb_equilibrium(rlb_lattice* L, void* dst) {
  rlb_status st = need_ready(L, true);
  if (st != RLB_OK) return st;
  if (!dst) return fail(L, RLB_ERR_INVALID_ARG, "dst is NULL");
  if (!L->has_high) return fail(L, RLB_ERR_INVALID_ARG, "no tube of the high-order form (n_v > 7)");
  const double* rec = L->dev<double>(L->off_rec[0]);
  for (const Group& g : L->groups) {
    if (g.nvt != kNvtHigh) continue;
    const hipError_t e = L->prec == RLB_FP32 ? equilibrium_pass<float>(L, g, rec, dst, L->stream)
                                             : equilibrium_pass<double>(L, g, rec, dst, L->stream);
    if (e != hipSuccess) return hip_fail(L, e, "equilibrium kernel launch");
  }
  return RLB_OK;
}

rlb_status rlb_set_state(rlb_lattice* L, const void* src) {
  rlb_status st = need_ready(L, false);
  if (st != RLB_OK) return st;
  if (!src) return fail(L, RLB_ERR_INVALID_ARG, "src is NULL");
  hipError_t e = state_copy(L->ws + L->off_F[0], src, L->state_elems * L->rsize, L->stream);
  if (e != hipSuccess) return hip_fail(L, e, "state copy");
  const bool fp32 = L->prec == RLB_FP32;
  e = launch_moments(fp32 ? 1 : 0, L->dev<TubeDev>(L->off_tubes), L->dev<WorkItem>(L->off_items),
                     static_cast<int>(L->items.size()), L->sched.tile, L->ws + L->off_jtab,
                     L->dev<double>(L->off_itab), L->ws + L->off_F[0], L->dev<double>(L->off_rec[0]), L->stream);
  if (e != hipSuccess) return hip_fail(L, e, "moments kernel launch");
  L->initialised = true;
  return RLB_OK;
}

rlb_status rlb_set_tau(rlb_lattice* L, int32_t tube, double tau) {
  if (!L || !check_tube(L, tube)) return RLB_ERR_INVALID_ARG;
  rlb_tube_desc d = L->desc[tube];
  d.tau = tau;
  d.dt = L->tubes[tube].dt;  // the time step stays fixed
  std::string msg;
  rlb_status st = validate(d, tube, msg);
  if (st != RLB_OK) return fail(L, st, msg);
  L->desc[tube].tau = tau;
  L->tubes[tube].tau_inv = 1.0 / tau;
  if (L->ws) return upload(L, L->off_tubes + tube * sizeof(TubeDev), &L->tubes[tube], sizeof(TubeDev));
  return RLB_OK;
}

rlb_status rlb_set_time(rlb_lattice* L, int32_t tube, double time) {
  if (!L || (tube != -1 && !check_tube(L, tube))) return RLB_ERR_INVALID_ARG;
  if (!std::isfinite(time)) return fail(L, RLB_ERR_INVALID_ARG, "time must be finite");
  for (int t = 0; t < L->ntubes; ++t)
    if (tube == -1 || t == tube) L->time[t] = time;
  return RLB_OK;
}

rlb_status rlb_tube_info(const rlb_lattice* L, int32_t tube, double* dt, double* time, int32_t* Q) {
  if (!L || !check_tube(L, tube)) return RLB_ERR_INVALID_ARG;
  if (dt) *dt = L->tubes[tube].dt;
  if (time) *time = L->time[tube];
  if (Q) *Q = L->tubes[tube].qx * L->tubes[tube].qp;
  return RLB_OK;
}

rlb_status rlb_tables(const rlb_lattice* L, int32_t tube, double* xi, double* w_xi, double* p, double* w_p) {
  if (!L || !check_tube(L, tube)) return RLB_ERR_INVALID_ARG;
  if (xi) std::copy(L->xi[tube].begin(), L->xi[tube].end(), xi);
  if (w_xi) std::copy(L->wxi[tube].begin(), L->wxi[tube].end(), w_xi);
  if (p) std::copy(L->p[tube].begin(), L->p[tube].end(), p);
  if (w_p) std::copy(L->wp[tube].begin(), L->wp[tube].end(), w_p);
  return RLB_OK;
}


}  // extern "C"

namespace {

// One forward stage over every tube with explicit buffers (adjoint recompute),
// on stream s (the lattice's stream by default).
rlb_status run_stage(rlb_lattice* L, int stage, const void* fin, const void* fn, void* fout, const double* rec_in,
                     double* rec_out, hipStream_t s) {
  const bool fp32 = L->prec == RLB_FP32;
  L->pipe_forked = false;
  for (const Group& g : L->groups) {
    const hipError_t e = fp32 ? stage_group<float>(L, g, stage, fin, fn, fout, rec_in, rec_out, s)
                              : stage_group<double>(L, g, stage, fin, fn, fout, rec_in, rec_out, s);
    if (e != hipSuccess) return hip_fail(L, e, "stage kernel launch");
  }
  return RLB_OK;
}
rlb_status run_stage(rlb_lattice* L, int stage, const void* fin, const void* fn, void* fout, const double* rec_in,
                     double* rec_out) {
  return run_stage(L, stage, fin, fn, fout, rec_in, rec_out, L->stream);
}

rlb_status moments_of(rlb_lattice* L, const void* state, double* rec, hipStream_t s) {
  hipError_t e = launch_moments(L->prec == RLB_FP32 ? 1 : 0, L->dev<TubeDev>(L->off_tubes),
                                L->dev<WorkItem>(L->off_items), static_cast<int>(L->items.size()), L->sched.tile,
                                L->ws + L->off_jtab, L->dev<double>(L->off_itab), state, rec, s);
  if (e != hipSuccess) return hip_fail(L, e, "moments kernel launch");
  return RLB_OK;
}
rlb_status moments_of(rlb_lattice* L, const void* state, double* rec) { return moments_of(L, state, rec, L->stream); }

template <typename Real>
rlb_status adjoint_stage(rlb_lattice* L, int tube, int qpt, int nvt, const void* g, const double* rec_g, const void* K,
                         void* out, const void* acc_in, void* acc_out, double cK, double cJ, double cA, int add_acc,
                         int acc_init, int tau_init) {
  AdjArgs<Real> a;
  a.tubes = L->dev<TubeDev>(L->off_tubes);
  a.tube = tube;
  a.aux_pairs = L->aux_pairs;
  a.jtab = L->dev<Real>(L->off_jtab);
  a.itab = L->dev<double>(L->off_itab);
  a.aux = L->dev<Real>(L->off_aux);
  a.aux_d = L->dev<double>(L->off_aux_d);
  a.g = static_cast<const Real*>(g);
  a.rec_g = rec_g;
  a.K = static_cast<const Real*>(K);
  a.acc_in = static_cast<const Real*>(acc_in);
  a.out = static_cast<Real*>(out);
  a.acc_out = static_cast<Real*>(acc_out);
  a.cellbuf = L->dev<double>(L->off_cellbuf);
  a.tau_acc = L->dev<double>(L->off_tauacc);
  a.G = L->dev<Real>(L->off_G);
  a.G_slot = L->face_elems;
  a.cK = cK;
  a.cJ = cJ;
  a.cA = cA;
  a.add_acc = add_acc;
  a.acc_init = acc_init;
  a.tau_init = tau_init;
  a.feq = L->off_afeq ? L->dev<Real>(L->off_afeq) : nullptr;
  a.ztab = L->has_high ? L->dev<double>(L->off_ztab) : nullptr;
  const TubeDev& td = L->tubes[tube];
  hipError_t e = launch_adjoint_stage(L->prec == RLB_FP32 ? 1 : 0, qpt, nvt, td.nx, td.qx * td.qp, &a, L->stream);
  if (e != hipSuccess) return hip_fail(L, e, "adjoint kernel launch");
  return RLB_OK;
}

rlb_status need_adjoint(rlb_lattice* L) {
  rlb_status st = need_ready(L, false);
  if (st != RLB_OK) return st;
  if (!(L->flags & RLB_WITH_ADJOINT)) return fail(L, RLB_ERR_STATE, "lattice was created without RLB_WITH_ADJOINT");
  return RLB_OK;
}

}  // namespace

extern "C" {

namespace {

// The three adjoint stages of one step (f^n, its stage states f1, f2 and
// their records given) and the dL/dtau reduction: lambda goes from
// dL/df^{n+1} to dL/df^n.
rlb_status adjoint_of_step(rlb_lattice* L, const void* Fn, const void* F1, const void* F2, const double* r0,
                           const double* r1, const double* r2, void* lambda, double* dL_dtau) {
  rlb_status st;
  void* lam2 = L->ws + L->off_lam2;
  void* lam1 = L->ws + L->off_lam1;
  void* acc = L->ws + L->off_acc;
  const bool fp32 = L->prec == RLB_FP32;
  for (const Group& g : L->groups) {
    const bool high = g.nvt == kNvtHigh;
    std::vector<int> tubes;  // one pass per tube
    for (int it = g.item_begin; it < g.item_end; ++it)
      if (L->items[it].x0 == 0) tubes.push_back(L->items[it].tube);
    auto stage = [&](int t, const void* gs, const double* rec, const void* K, void* out, const void* ain, void* aout,
                     double cK, double cJ, double cA, int add_acc, int acc_init, int tau_init) {
      return fp32 ? adjoint_stage<float>(L, t, g.qpt, g.nvt, gs, rec, K, out, ain, aout, cK, cJ, cA, add_acc,
                                         acc_init, tau_init)
                  : adjoint_stage<double>(L, t, g.qpt, g.nvt, gs, rec, K, out, ain, aout, cK, cJ, cA, add_acc,
                                          acc_init, tau_init);
    };
    // the high-order group's equilibrium values of a stage's input, for all of
    // its tubes, by the forward's pre-pass (so bit for bit the forward's)
    auto equilibrium_of = [&](const double* rec) -> rlb_status {
      if (!high) return RLB_OK;
      const hipError_t e = fp32 ? equilibrium_pass<float>(L, g, rec, L->ws + L->off_afeq, L->stream)
                                : equilibrium_pass<double>(L, g, rec, L->ws + L->off_afeq, L->stream);
      return e == hipSuccess ? RLB_OK : hip_fail(L, e, "equilibrium pre-pass launch");
    };
    // f^{n+1} = 1/3 f^n + 2/3 (f2 + dt L(f2))
    if ((st = equilibrium_of(r2)) != RLB_OK) return st;
    for (int t : tubes)
      if ((st = stage(t, F2, r2, lambda, lam2, nullptr, acc, 2.0 / 3.0, 2.0 / 3.0 * L->tubes[t].dt, 1.0 / 3.0, 0, 1,
                      1)) != RLB_OK)
        return st;
    // f2 = 3/4 f^n + 1/4 (f1 + dt L(f1))
    if ((st = equilibrium_of(r1)) != RLB_OK) return st;
    for (int t : tubes)
      if ((st = stage(t, F1, r1, lam2, lam1, acc, acc, 0.25, 0.25 * L->tubes[t].dt, 0.75, 0, 0, 0)) != RLB_OK)
        return st;
    // f1 = f^n + dt L(f^n)
    if ((st = equilibrium_of(r0)) != RLB_OK) return st;
    for (int t : tubes) {
      if ((st = stage(t, Fn, r0, lam1, lambda, acc, nullptr, 1.0, L->tubes[t].dt, 0.0, 1, 0, 0)) != RLB_OK) return st;
      hipError_t e = launch_tau_reduce(L->dev<TubeDev>(L->off_tubes), t, L->dev<double>(L->off_tauacc), dL_dtau,
                                       L->stream);
      if (e != hipSuccess) return hip_fail(L, e, "tau reduction launch");
    }
  }
  return RLB_OK;
}

// Layout of one step in the segment scratch: f^n, f1, f2, then their records.
struct SegmentStep {
  size_t F[3], R[3], bytes;
};

SegmentStep segment_step(const rlb_lattice* L) {
  SegmentStep s;
  size_t o = 0;
  for (int k = 0; k < 3; ++k) { s.F[k] = o; o = align256(o + L->state_elems * L->rsize); }
  for (int k = 0; k < 3; ++k) { s.R[k] = o; o = align256(o + L->rec_elems * 8); }
  s.bytes = o;
  return s;
}

}  // namespace

rlb_status rlb_adjoint_step(rlb_lattice* L, const void* state_n, void* lambda, double* dL_dtau) {
  rlb_status st = need_adjoint(L);
  if (st != RLB_OK) return st;
  if (!state_n || !lambda || !dL_dtau) return fail(L, RLB_ERR_INVALID_ARG, "state_n, lambda and dL_dtau are required");
  if (state_n == lambda) return fail(L, RLB_ERR_INVALID_ARG, "state_n and lambda must not alias");
  void* F1 = L->ws + L->off_aF[0];
  void* F2 = L->ws + L->off_aF[1];
  double* r0 = L->dev<double>(L->off_arec[0]);
  double* r1 = L->dev<double>(L->off_arec[1]);
  double* r2 = L->dev<double>(L->off_arec[2]);
  // recompute the two intermediate stages of the step from f^n
  if ((st = moments_of(L, state_n, r0)) != RLB_OK) return st;
  if ((st = run_stage(L, 1, state_n, state_n, F1, r0, r1)) != RLB_OK) return st;
  if ((st = run_stage(L, 2, F1, state_n, F2, r1, r2)) != RLB_OK) return st;
  return adjoint_of_step(L, state_n, F1, F2, r0, r1, r2, lambda, dL_dtau);
}

rlb_status rlb_adjoint_segment_size(const rlb_lattice* L, int32_t nsteps, size_t* bytes) {
  if (!L || !bytes || nsteps < 1) return RLB_ERR_INVALID_ARG;
  *bytes = segment_step(L).bytes * size_t(nsteps);
  return RLB_OK;
}

namespace {

// Forward half of a segment: f^n, f1, f2 of every step and their records
// into the scratch, on stream s.
rlb_status segment_forward(rlb_lattice* L, const void* state0, int32_t nsteps, char* base, hipStream_t s) {
  const SegmentStep ss = segment_step(L);
  auto F = [&](int k, int i) { return static_cast<void*>(base + size_t(k) * ss.bytes + ss.F[i]); };
  auto R = [&](int k, int i) { return reinterpret_cast<double*>(base + size_t(k) * ss.bytes + ss.R[i]); };
  rlb_status st;
  hipError_t e = state_copy(F(0, 0), state0, L->state_elems * L->rsize, s);
  if (e != hipSuccess) return hip_fail(L, e, "state copy");
  if ((st = moments_of(L, F(0, 0), R(0, 0), s)) != RLB_OK) return st;
  for (int k = 0; k < nsteps; ++k) {
    if ((st = run_stage(L, 1, F(k, 0), F(k, 0), F(k, 1), R(k, 0), R(k, 1), s)) != RLB_OK) return st;
    if ((st = run_stage(L, 2, F(k, 1), F(k, 0), F(k, 2), R(k, 1), R(k, 2), s)) != RLB_OK) return st;
    if (k + 1 < nsteps && (st = run_stage(L, 3, F(k, 2), F(k, 0), F(k + 1, 0), R(k, 2), R(k + 1, 0), s)) != RLB_OK)
      return st;
  }
  return RLB_OK;
}

// Reverse half: the adjoint of every step of the segment, last step first,
// on the lattice's stream.
rlb_status segment_reverse(rlb_lattice* L, int32_t nsteps, char* base, void* lambda, double* dL_dtau) {
  const SegmentStep ss = segment_step(L);
  auto F = [&](int k, int i) { return static_cast<void*>(base + size_t(k) * ss.bytes + ss.F[i]); };
  auto R = [&](int k, int i) { return reinterpret_cast<double*>(base + size_t(k) * ss.bytes + ss.R[i]); };
  rlb_status st;
  for (int k = nsteps - 1; k >= 0; --k)
    if ((st = adjoint_of_step(L, F(k, 0), F(k, 1), F(k, 2), R(k, 0), R(k, 1), R(k, 2), lambda, dL_dtau)) != RLB_OK)
      return st;
  return RLB_OK;
}

rlb_status segment_args(rlb_lattice* L, int32_t nsteps, const void* scratch, size_t bytes) {
  if (!scratch || nsteps < 1) return fail(L, RLB_ERR_INVALID_ARG, "scratch and nsteps >= 1 are required");
  if (bytes < segment_step(L).bytes * size_t(nsteps))
    return fail(L, RLB_ERR_INVALID_ARG, "scratch smaller than rlb_adjoint_segment_size");
  return RLB_OK;
}

}  // namespace

rlb_status rlb_adjoint_segment(rlb_lattice* L, const void* state0, int32_t nsteps, void* scratch, size_t bytes,
                               void* lambda, double* dL_dtau) {
  rlb_status st = need_adjoint(L);
  if (st != RLB_OK) return st;
  if (!state0 || !lambda || !dL_dtau) return fail(L, RLB_ERR_INVALID_ARG, "state0, lambda and dL_dtau are required");
  if ((st = segment_args(L, nsteps, scratch, bytes)) != RLB_OK) return st;
  char* base = static_cast<char*>(scratch);
  if ((st = segment_forward(L, state0, nsteps, base, L->stream)) != RLB_OK) return st;
  return segment_reverse(L, nsteps, base, lambda, dL_dtau);
}

rlb_status rlb_adjoint_segment_forward(rlb_lattice* L, const void* state0, int32_t nsteps, void* scratch, size_t bytes,
                                       void* hip_stream) {
  rlb_status st = need_adjoint(L);
  if (st != RLB_OK) return st;
  if (!state0) return fail(L, RLB_ERR_INVALID_ARG, "state0 is required");
  if ((st = segment_args(L, nsteps, scratch, bytes)) != RLB_OK) return st;
  hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : L->stream;
  return segment_forward(L, state0, nsteps, static_cast<char*>(scratch), s);
}

rlb_status rlb_adjoint_segment_reverse(rlb_lattice* L, int32_t nsteps, const void* scratch, size_t bytes,
                                       void* lambda, double* dL_dtau) {
  rlb_status st = need_adjoint(L);
  if (st != RLB_OK) return st;
  if (!lambda || !dL_dtau) return fail(L, RLB_ERR_INVALID_ARG, "lambda and dL_dtau are required");
  if ((st = segment_args(L, nsteps, scratch, bytes)) != RLB_OK) return st;
  return segment_reverse(L, nsteps, static_cast<char*>(const_cast<void*>(scratch)), lambda, dL_dtau);
}

rlb_status rlb_fields_adjoint(rlb_lattice* L, int32_t tube, const void* state, const double* dL_dfields, int64_t ld,
                              void* lambda) {
  rlb_status st = need_adjoint(L);
  if (st != RLB_OK) return st;
  if (!check_tube(L, tube)) return fail(L, RLB_ERR_INVALID_ARG, "tube index out of range");
  if (!state || !dL_dfields || !lambda || ld < L->tubes[tube].nx)
    return fail(L, RLB_ERR_INVALID_ARG, "need state, dL_dfields, lambda and ld >= nx");
  double* r0 = L->dev<double>(L->off_arec[0]);
  if ((st = moments_of(L, state, r0)) != RLB_OK) return st;
  hipError_t e = launch_fields_adjoint(L->prec == RLB_FP32 ? 1 : 0, L->dev<TubeDev>(L->off_tubes), tube,
                                       L->tubes[tube].nx, L->ws + L->off_jtab, L->dev<double>(L->off_itab), r0,
                                       dL_dfields, ld, lambda, L->stream);
  if (e != hipSuccess) return hip_fail(L, e, "fields adjoint launch");
  return RLB_OK;
}

rlb_status rlb_initial_state_adjoint(rlb_lattice* L, int32_t tube, const void* lambda0, double grad_left[3],
                                     double grad_right[3]) {
  rlb_status st = need_adjoint(L);
  if (st != RLB_OK) return st;
  if (!check_tube(L, tube) || !lambda0 || !grad_left || !grad_right)
    return fail(L, RLB_ERR_INVALID_ARG, "bad tube or NULL argument");
  if (!L->initialised) return fail(L, RLB_ERR_STATE, "no initial state has been set");
  int qpt, nvt;
  kernel_group(L->desc[tube].q_p, L->desc[tube].n_v, &qpt, &nvt);
  double* grad = L->dev<double>(L->off_grad);
  hipError_t e = launch_initial_adjoint(L->prec == RLB_FP32 ? 1 : 0, qpt, nvt, L->dev<TubeDev>(L->off_tubes), tube,
                                        L->tubes[tube].nx, L->ws + L->off_jtab, L->dev<double>(L->off_itab),
                                        L->dev<double>(L->off_aux_d), L->aux_pairs, L->dev<double>(L->off_ztab),
                                        L->dev<double>(L->off_sides), lambda0, L->dev<double>(L->off_ipart),
                                        L->init_blocks_max, L->ipart_stride, grad, L->stream);
  if (e != hipSuccess) return hip_fail(L, e, "initial-state adjoint launch");
  double h[6];
  HIP_TRY(L, hipMemcpyAsync(h, grad, sizeof h, hipMemcpyDeviceToHost, L->stream));
  HIP_TRY(L, hipStreamSynchronize(L->stream));
  for (int k = 0; k < 3; ++k) {
    grad_left[k] = h[k];
    grad_right[k] = h[3 + k];
  }
  return RLB_OK;
}

}  // extern "C"

namespace rlb {

size_t noalloc_scratch_bytes(const rlb_lattice* L) { return L->step_bytes; }

rlb_status noalloc_validate(rlb_lattice* L, const void* state, int64_t nsteps, size_t max_bytes) {
  if (!L) return RLB_ERR_INVALID_ARG;
  if (!state) return fail(L, RLB_ERR_INVALID_ARG, "state is NULL");
  if (reinterpret_cast<uintptr_t>(state) % L->rsize)
    return fail(L, RLB_ERR_INVALID_ARG, "state must be aligned to its element size");
  if (nsteps < 0) return fail(L, RLB_ERR_INVALID_ARG, "nsteps must be >= 0");
  if (L->step_bytes > max_bytes) {
    char buf[200];
    std::snprintf(buf, sizeof buf,
                  "the lattice's step needs %zu bytes of scratch; the allocation-free step holds at most %zu",
                  L->step_bytes, max_bytes);
    return fail(L, RLB_ERR_INVALID_ARG, buf);
  }
  return RLB_OK;
}

rlb_status noalloc_hip_error(rlb_lattice* L, hipError_t e, const char* where) { return hip_fail(L, e, where); }

// Time steps of a caller-owned state with every other device buffer of the
// step (stage arrays, records, tables, work lists, node-split sums, the
// high-order equilibrium values and, unless the caller passes its own word,
// the flag) placed in `scratch` at the lattice's workspace offsets.  The
// lattice's own binding is left as it was.
rlb_status noalloc_steps(rlb_lattice* L, char* scratch, void* state, unsigned* flag_out, int64_t nsteps,
                         hipStream_t s) {
  struct Restore {
    rlb_lattice* L;
    char* ws;
    hipStream_t stream;
    ~Restore() {
      L->ws = ws;
      L->stream = stream;
      L->f0_ext = nullptr;
      L->flag_ext = nullptr;
    }
  } restore{L, L->ws, L->stream};
  L->ws = scratch;
  L->stream = s;
  L->f0_ext = state;
  L->flag_ext = flag_out;
  auto put = [&](size_t off, const void* src, size_t bytes) {
    return bytes ? hipMemcpyAsync(scratch + off, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
  };
  const bool fp32 = L->prec == RLB_FP32;
  HIP_TRY(L, put(L->off_tubes, L->tubes.data(), L->tubes.size() * sizeof(TubeDev)));
  HIP_TRY(L, fp32 ? put(L->off_jtab, L->jtab_f.data(), L->jtab_f.size() * 4)
                  : put(L->off_jtab, L->jtab_d.data(), L->jtab_d.size() * 8));
  HIP_TRY(L, fp32 ? put(L->off_aux, L->aux_f.data(), L->aux_f.size() * 4)
                  : put(L->off_aux, L->aux_d.data(), L->aux_d.size() * 8));
  HIP_TRY(L, put(L->off_itab, L->itab.data(), L->itab.size() * 8));
  HIP_TRY(L, put(L->off_aux_d, L->aux_d.data(), L->aux_d.size() * 8));
  HIP_TRY(L, put(L->off_items, L->items.data(), L->items.size() * sizeof(WorkItem)));
  HIP_TRY(L, put(L->off_ztab, L->ztab.data(), L->ztab.size() * 8));
  // the scratch keeps the previous call's contents: only the flag must start
  // at zero (a fill kernel, no memset node); every record, stage value and
  // node sum is written before it is read
  HIP_TRY(L, launch_fill_u32(L->flag(), 1, 0u, s));
  rlb_status st = moments_of(L, state, L->dev<double>(L->off_rec[0]));
  if (st != RLB_OK) return st;
  return enqueue_steps(L, s, nsteps);
}

}  // namespace rlb

extern "C" {

rlb_status rlb_device_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if ((!dst || !src) && bytes) return RLB_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16) return RLB_ERR_INVALID_ARG;
  hipError_t e = launch_copy(dst, src, bytes, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? RLB_OK : RLB_ERR_HIP;
}

rlb_status rlb_device_stream(void* out, const void* a, const void* b, int64_t rows, int64_t ld, int32_t cols,
                             int32_t elem_bytes, void* hip_stream) {
  if (!out || !a || rows < 1 || cols < 1 || ld < cols || (elem_bytes != 4 && elem_bytes != 8)) return RLB_ERR_INVALID_ARG;
  // one chunk of rows is addressed with 32-bit byte offsets, as in the stage kernel
  if (rows > (int64_t(1) << 24) || ld * elem_bytes * 8 > (int64_t(1) << 31)) return RLB_ERR_INVALID_ARG;
  const uintptr_t al = reinterpret_cast<uintptr_t>(out) | reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b);
  if (al % uintptr_t(elem_bytes)) return RLB_ERR_INVALID_ARG;
  const hipError_t e = launch_stream(out, a, b, int(rows), ld, cols, elem_bytes, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? RLB_OK : RLB_ERR_HIP;
}

const char* rlb_status_string(rlb_status st) {
  switch (st) {
    case RLB_OK: return "ok";
    case RLB_ERR_INVALID_ARG: return "invalid argument";
    case RLB_ERR_NONPHYSICAL: return "non-physical state";
    case RLB_ERR_HIP: return "HIP runtime error";
    case RLB_ERR_STATE: return "call out of order";
    case RLB_ERR_UNSTABLE_DT: return "unstable time step";
  }
  return "unknown status";
}

const char* rlb_last_error(const rlb_lattice* L) {
  if (!L) return g_create_error.c_str();
  return L->err.c_str();
}

}  // extern "C"
