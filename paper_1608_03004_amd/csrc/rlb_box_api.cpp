// Host side of the box (x, y, z) interface declared in include/rlb.h:
// validation, the velocity / radial / projection tables, the workspace layout
// and the stage sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rlb.h"
#include "quadrature.h"
#include "rlb_internal.h"

using namespace rlb;

namespace {

thread_local std::string g_box_create_error;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Spacing {
  double dx, dy, dz;
  double inv_sum() const { return 1.0 / dx + 1.0 / dy + 1.0 / dz; }
};

Spacing spacing(const rlb_box_desc& d) {
  return {(d.x_max - d.x_min) / d.nx, (d.y_max - d.y_min) / d.ny, (d.z_max - d.z_min) / d.nz};
}

// The time step: explicit, or the CFL bound of the sum of the three inverse
// spacings, capped at dt_tau_max tau.
double box_dt(const rlb_box_desc& d) {
  if (d.dt > 0) return d.dt;
  return std::min(d.cfl / spacing(d).inv_sum(), d.dt_tau_max * d.tau);
}

}  // namespace

struct rlb_box {
  rlb_box_desc desc;
  rlb_precision prec = RLB_FP64;
  size_t rsize = 8;
  BoxDev bd;
  int qpt = 3, nvt = 5, grid = 1;
  std::vector<double> vtab_d, itab, aux_d;
  std::vector<float> vtab_f, aux_f;
  int aux_pairs = 0;
  int64_t state_elems = 0, cells = 0;
  size_t off_F[3] = {0, 0, 0}, off_rec[3] = {0, 0, 0};
  size_t off_bd = 0, off_vtab = 0, off_itab = 0, off_aux = 0, off_flag = 0, total = 0;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  bool initialised = false;
  double time = 0.0;
  std::string err;
  template <typename T>
  T* dev(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

namespace {

// Device-to-device copy of a state: the library's 16-byte vector copy kernel
// when both ends are 16-byte aligned, the runtime's copy otherwise.
hipError_t state_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16) == 0)
    return launch_copy(dst, src, bytes, s);
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}

rlb_status bfail(rlb_box* X, rlb_status st, const std::string& msg) {
  if (X) X->err = msg; else g_box_create_error = msg;
  return st;
}

rlb_status bhip(rlb_box* X, hipError_t e, const char* where) {
  return bfail(X, RLB_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define BHIP_TRY(X, expr)                                   \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) return bhip((X), _e, #expr);      \
  } while (0)

rlb_status validate_box(const rlb_box_desc& d, std::string& msg) {
  auto bad = [&](const char* what) {
    msg = std::string("box: ") + what;
    return RLB_ERR_INVALID_ARG;
  };
  if (d.nx < 1 || d.ny < 1 || d.nz < 1) return bad("nx, ny and nz must be >= 1");
  if (int64_t(d.nx) * d.ny * d.nz > (int64_t(1) << 26)) return bad("nx * ny * nz must be <= 2^26");
  if (int64_t((d.nx + 63) / 64 * 64) * d.ny * d.nz > (int64_t(1) << 27))
    return bad("the padded box (nx rounded up to 64) * ny * nz must be <= 2^27 cells");
  if (d.q_xi < 1 || d.q_xi > 1024) return bad("q_xi must be in [1, 1024]");
  if (d.q_p < 1 || d.q_p > kMaxQp) return bad("q_p must be in [1, 8]");
  if (d.n_v < 0 || d.n_v > kMaxNv) return bad("n_v must be in [0, 7]");
  if (d.n_p < 0 || d.n_p >= d.q_p) return bad("n_p must satisfy 0 <= n_p < q_p");
  if (d.n_p + 2 > 2 * d.q_p - 1) return bad("q_p too small to integrate T^{mu nu} of the equilibrium exactly");
  if (d.n_v + 2 > 2 * d.q_xi - 1) return bad("q_xi too small to integrate T^{mu nu} of the equilibrium exactly");
  if (d.q_phi < d.n_v + 3 || d.q_phi > 64) return bad("q_phi must satisfy n_v + 3 <= q_phi <= 64");
  if (!(d.x_max > d.x_min) || !(d.y_max > d.y_min) || !(d.z_max > d.z_min) ||
      !std::isfinite(d.x_min + d.x_max + d.y_min + d.y_max + d.z_min + d.z_max))
    return bad("need x_min < x_max, y_min < y_max and z_min < z_max");
  if (!(d.tau > 0)) return bad("tau must be > 0 (+inf allowed)");
  if (!(d.T0 > 0) || !std::isfinite(d.T0)) return bad("T0 must be > 0");
  if (!(d.weno_eps > 0) || !std::isfinite(d.weno_eps)) return bad("weno_eps must be > 0 and finite");
  if (d.dt < 0 || !std::isfinite(d.dt)) return bad("dt must be >= 0");
  if (d.dt == 0 && !(d.cfl > 0 && std::isfinite(d.cfl))) return bad("cfl must be > 0");
  if (d.dt == 0 && !(d.dt_tau_max > 0)) return bad("dt_tau_max must be > 0");
  const double dt = box_dt(d);
  if (!(dt > 0) || !std::isfinite(dt)) return bad("time step is not a positive number");
  if (dt * spacing(d).inv_sum() > 1.5) {
    msg = "box: dt (1/dx + 1/dy + 1/dz) exceeds the WENO5/RK3 stability limit 1.5";
    return RLB_ERR_UNSTABLE_DT;
  }
  if (dt > 2.5 * d.tau) {
    msg = "box: dt/tau exceeds the RK3 stability limit 2.5";
    return RLB_ERR_UNSTABLE_DT;
  }
  return RLB_OK;
}

rlb_status ready(rlb_box* X, bool need_init) {
  if (!X) return RLB_ERR_INVALID_ARG;
  if (!X->ws) return bfail(X, RLB_ERR_STATE, "no workspace bound (call rlb_box_bind)");
  if (need_init && !X->initialised)
    return bfail(X, RLB_ERR_STATE, "no state (call rlb_box_set_initial_fields or rlb_box_set_state)");
  return RLB_OK;
}

template <typename Real>
BoxArgs<Real> box_args(const rlb_box* X) {
  BoxArgs<Real> a;
  std::memset(&a, 0, sizeof a);
  a.bx = X->dev<BoxDev>(X->off_bd);
  a.aux_pairs = X->aux_pairs;
  a.vtab = X->dev<Real>(X->off_vtab);
  a.itab = X->dev<double>(X->off_itab);
  a.aux = X->dev<Real>(X->off_aux);
  a.flag = X->dev<unsigned>(X->off_flag);
  return a;
}

template <typename Real>
hipError_t box_stage(rlb_box* X, int stage, size_t fin, size_t fout, size_t rin, size_t rout) {
  BoxArgs<Real> a = box_args<Real>(X);
  a.stage = stage;
  a.fin = X->dev<Real>(fin);
  a.fn = X->dev<Real>(X->off_F[0]);
  a.fout = X->dev<Real>(fout);
  a.rec_in = X->dev<double>(rin);
  a.rec_out = X->dev<double>(rout);
  return launch_box_stage(sizeof(Real) == 4, X->qpt, X->nvt, &a, X->grid, X->stream);
}

template <typename Real>
hipError_t box_records(rlb_box* X) {
  BoxArgs<Real> a = box_args<Real>(X);
  a.fin = X->dev<Real>(X->off_F[0]);
  a.rec_out = X->dev<double>(X->off_rec[0]);
  return launch_box_moments(sizeof(Real) == 4, &a, X->grid, X->stream);
}

template <typename Real>
hipError_t box_init(rlb_box* X, const double* fields) {
  BoxArgs<Real> a = box_args<Real>(X);
  a.init = fields;
  a.fout = X->dev<Real>(X->off_F[0]);
  a.rec_out = X->dev<double>(X->off_rec[0]);
  return launch_box_init(sizeof(Real) == 4, X->qpt, X->nvt, &a, X->grid, X->stream);
}

}  // namespace

extern "C" {

rlb_status rlb_box_defaults(rlb_box_desc* d) {
  if (!d) return RLB_ERR_INVALID_ARG;
  std::memset(d, 0, sizeof *d);
  d->nx = 32;
  d->ny = 32;
  d->nz = 32;
  d->q_xi = 8;
  d->q_phi = 8;
  d->q_p = 3;
  d->n_v = 5;
  d->n_p = 2;
  d->x_min = -0.5;
  d->x_max = 0.5;
  d->y_min = -0.5;
  d->y_max = 0.5;
  d->z_min = -0.5;
  d->z_max = 0.5;
  d->tau = 1e-2;
  d->cfl = 0.5;
  d->dt_tau_max = 0.5;
  d->T0 = 1.0;
  d->weno_eps = 1e-6;
  return RLB_OK;
}

rlb_status rlb_box_create(const rlb_box_desc* desc, rlb_precision prec, rlb_box** out) {
  if (!out) return bfail(nullptr, RLB_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!desc) return bfail(nullptr, RLB_ERR_INVALID_ARG, "desc is NULL");
  if (prec != RLB_FP64 && prec != RLB_FP32) return bfail(nullptr, RLB_ERR_INVALID_ARG, "unknown precision");
  std::string msg;
  const rlb_status st = validate_box(*desc, msg);
  if (st != RLB_OK) return bfail(nullptr, st, msg);
  if (!rlb::plane_weno_eps_in_range(desc->weno_eps, prec == RLB_FP32))
    return bfail(nullptr, RLB_ERR_INVALID_ARG, "weno_eps must lie in [1e-10, 1e8] (FP32) or [1e-70, 1e70] (FP64)");
  const rlb_box_desc& d = *desc;
  std::vector<double> xi, wxi, p, wp;
  if (!gauss_legendre_rule(d.q_xi, xi, wxi) || !gauss_laguerre1_rule(d.q_p, p, wp))
    return bfail(nullptr, RLB_ERR_INVALID_ARG, "quadrature construction failed");
  rlb_box* X = new rlb_box();
  X->desc = d;
  X->prec = prec;
  X->rsize = prec == RLB_FP32 ? 4 : 8;
  // velocity table per (j, k): v_x, v_y, v_z and the weighted moment factors
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < d.q_xi; ++j) {
    const long double vz = xi[j], st_ = std::sqrt(1.0L - vz * vz);
    for (int k = 0; k < d.q_phi; ++k) {
      const long double ang = 2.0L * pi * k / d.q_phi;
      const long double vx = st_ * std::cos(ang), vy = st_ * std::sin(ang);
      const long double w = (long double)wxi[j] / d.q_phi;
      const long double row[kBoxVStride] = {vx,          vy,          vz,          w,           w * vx,      w * vy,
                                            w * vz,      w * vx * vx, w * vx * vy, w * vx * vz, w * vy * vy, w * vy * vz,
                                            w * vz * vz, 0.0L,        0.0L,        0.0L};
      for (int q = 0; q < kBoxVStride; ++q) X->vtab_d.push_back(double(row[q]));
    }
  }
  X->vtab_f.assign(X->vtab_d.begin(), X->vtab_d.end());
  // radial rows (as for a tube)
  const double t3 = d.T0 * d.T0 * d.T0, t4 = t3 * d.T0;
  for (int i = 0; i < d.q_p; ++i) {
    double row[kIStride];
    row[0] = p[i];
    row[1] = wp[i];
    row[2] = t3 * wp[i] * p[i];
    row[3] = t4 * wp[i] * p[i] * p[i];
    for (int l = 0; l <= kMaxNp; ++l) row[4 + l] = laguerre1_value(l, p[i]);
    X->itab.insert(X->itab.end(), row, row + kIStride);
  }
  // projection rule: symmetric pairs of a Gauss-Legendre rule
  const int M = prec == RLB_FP32 ? 2 * kAuxPairsFP32 : 2 * kAuxPairsFP64;
  std::vector<double> ax, aw;
  gauss_legendre_rule(M, ax, aw);
  X->aux_pairs = M / 2;
  for (int a = 0; a < M / 2; ++a) {
    const int j = M / 2 + a;
    double row[kAuxStride];
    row[0] = ax[j];
    for (int k = 0; k <= kMaxNv; ++k) row[1 + k] = aw[j] * (2 * k + 1) / 2.0 * legendre_value(k, ax[j]);
    for (int k = kMaxNv + 2; k < kAuxStride; ++k) row[k] = 0.0;
    X->aux_d.insert(X->aux_d.end(), row, row + kAuxStride);
  }
  X->aux_f.assign(X->aux_d.begin(), X->aux_d.end());
  // device descriptor
  BoxDev& bd = X->bd;
  std::memset(&bd, 0, sizeof bd);
  bd.nx = d.nx;
  bd.ny = d.ny;
  bd.nz = d.nz;
  bd.ldx = (d.nx + 63) / 64 * 64;
  bd.qx = d.q_xi;
  bd.qf = d.q_phi;
  bd.qp = d.q_p;
  bd.nv = d.n_v;
  bd.np = d.n_p;
  bd.slab = int64_t(d.ny) * bd.ldx;
  bd.plane = int64_t(d.nz) * bd.slab;
  bd.dx_inv = d.nx / (d.x_max - d.x_min);
  bd.dy_inv = d.ny / (d.y_max - d.y_min);
  bd.dz_inv = d.nz / (d.z_max - d.z_min);
  bd.dt = box_dt(d);
  bd.tau_inv = 1.0 / d.tau;
  bd.T0 = d.T0;
  bd.weno_eps = d.weno_eps;
  if (d.n_v <= 5 && d.q_p <= 3) { X->qpt = 3; X->nvt = 5; }
  else if (d.n_v <= 5 && d.q_p == 4) { X->qpt = 4; X->nvt = 5; }
  else { X->qpt = 8; X->nvt = 7; }
  X->grid = box_grid(d.nx, d.ny, d.nz);
  X->cells = int64_t(d.nx) * d.ny * d.nz;
  X->state_elems = int64_t(d.q_p) * d.q_xi * d.q_phi * bd.plane;
  // workspace layout
  size_t o = 0;
  for (int k = 0; k < 3; ++k) { X->off_F[k] = o; o = align256(o + X->state_elems * X->rsize); }
  for (int k = 0; k < 3; ++k) { X->off_rec[k] = o; o = align256(o + 14 * size_t(bd.plane) * 8); }
  X->off_bd = o; o = align256(o + sizeof(BoxDev));
  X->off_vtab = o; o = align256(o + X->vtab_d.size() * X->rsize);
  X->off_itab = o; o = align256(o + X->itab.size() * 8);
  X->off_aux = o; o = align256(o + X->aux_d.size() * X->rsize);
  X->off_flag = o; o = align256(o + 16);
  X->total = o;
  *out = X;
  return RLB_OK;
}

rlb_status rlb_box_destroy(rlb_box* X) {
  if (!X) return RLB_ERR_INVALID_ARG;
  delete X;
  return RLB_OK;
}

rlb_status rlb_box_workspace_size(const rlb_box* X, size_t* bytes) {
  if (!X || !bytes) return RLB_ERR_INVALID_ARG;
  *bytes = X->total;
  return RLB_OK;
}

rlb_status rlb_box_bind(rlb_box* X, void* workspace, size_t bytes, void* hip_stream) {
  if (!X) return RLB_ERR_INVALID_ARG;
  if (!workspace) return bfail(X, RLB_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return bfail(X, RLB_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (bytes < X->total) return bfail(X, RLB_ERR_INVALID_ARG, "workspace too small (see rlb_box_workspace_size)");
  X->ws = static_cast<char*>(workspace);
  X->stream = static_cast<hipStream_t>(hip_stream);
  X->initialised = false;
  BHIP_TRY(X, hipMemsetAsync(X->ws, 0, X->total, X->stream));
  BHIP_TRY(X, hipMemcpyAsync(X->ws + X->off_bd, &X->bd, sizeof(BoxDev), hipMemcpyHostToDevice, X->stream));
  if (X->prec == RLB_FP32) {
    BHIP_TRY(X, hipMemcpyAsync(X->ws + X->off_vtab, X->vtab_f.data(), X->vtab_f.size() * 4, hipMemcpyHostToDevice, X->stream));
    BHIP_TRY(X, hipMemcpyAsync(X->ws + X->off_aux, X->aux_f.data(), X->aux_f.size() * 4, hipMemcpyHostToDevice, X->stream));
  } else {
    BHIP_TRY(X, hipMemcpyAsync(X->ws + X->off_vtab, X->vtab_d.data(), X->vtab_d.size() * 8, hipMemcpyHostToDevice, X->stream));
    BHIP_TRY(X, hipMemcpyAsync(X->ws + X->off_aux, X->aux_d.data(), X->aux_d.size() * 8, hipMemcpyHostToDevice, X->stream));
  }
  BHIP_TRY(X, hipMemcpyAsync(X->ws + X->off_itab, X->itab.data(), X->itab.size() * 8, hipMemcpyHostToDevice, X->stream));
  BHIP_TRY(X, hipStreamSynchronize(X->stream));
  return RLB_OK;
}

rlb_status rlb_box_set_initial_fields(rlb_box* X, const double* fields) {
  rlb_status st = ready(X, false);
  if (st != RLB_OK) return st;
  if (!fields) return bfail(X, RLB_ERR_INVALID_ARG, "fields_device is NULL");
  const hipError_t e = X->prec == RLB_FP32 ? box_init<float>(X, fields) : box_init<double>(X, fields);
  if (e != hipSuccess) return bhip(X, e, "box init kernel launch");
  BHIP_TRY(X, launch_fill_u32(X->dev<unsigned>(X->off_flag), 4, 0u, X->stream));
  X->time = 0.0;
  X->initialised = true;
  return RLB_OK;
}

rlb_status rlb_box_step(rlb_box* X, int64_t nsteps) {
  rlb_status st = ready(X, true);
  if (st != RLB_OK) return st;
  if (nsteps < 0) return bfail(X, RLB_ERR_INVALID_ARG, "nsteps must be >= 0");
  const bool fp32 = X->prec == RLB_FP32;
  for (int64_t n = 0; n < nsteps; ++n) {
    for (int stage = 1; stage <= 3; ++stage) {
      const int fin = stage == 1 ? 0 : (stage == 2 ? 1 : 2);
      const int fout = stage == 1 ? 1 : (stage == 2 ? 2 : 0);
      const hipError_t e =
          fp32 ? box_stage<float>(X, stage, X->off_F[fin], X->off_F[fout], X->off_rec[fin], X->off_rec[fout])
               : box_stage<double>(X, stage, X->off_F[fin], X->off_F[fout], X->off_rec[fin], X->off_rec[fout]);
      if (e != hipSuccess) return bhip(X, e, "box stage kernel launch");
    }
  }
  X->time += nsteps * X->bd.dt;
  return RLB_OK;
}

rlb_status rlb_box_fields(rlb_box* X, double* out) {
  rlb_status st = ready(X, true);
  if (st != RLB_OK) return st;
  if (!out) return bfail(X, RLB_ERR_INVALID_ARG, "out_device is NULL");
  const hipError_t e = launch_box_fields(X->dev<BoxDev>(X->off_bd), X->cells, X->dev<double>(X->off_rec[0]), out,
                                         X->dev<unsigned>(X->off_flag), X->stream);
  if (e != hipSuccess) return bhip(X, e, "box fields kernel launch");
  return RLB_OK;
}

rlb_status rlb_box_layout(const rlb_box* X, int64_t* state_elems, int64_t* ldx) {
  if (!X || !state_elems || !ldx) return RLB_ERR_INVALID_ARG;
  *state_elems = X->state_elems;
  *ldx = X->bd.ldx;
  return RLB_OK;
}

rlb_status rlb_box_get_state(rlb_box* X, void* dst) {
  rlb_status st = ready(X, true);
  if (st != RLB_OK) return st;
  if (!dst) return bfail(X, RLB_ERR_INVALID_ARG, "dst is NULL");
  const hipError_t e = state_copy(dst, X->ws + X->off_F[0], X->state_elems * X->rsize, X->stream);
  if (e != hipSuccess) return bhip(X, e, "state copy");
  return RLB_OK;
}

rlb_status rlb_box_set_state(rlb_box* X, const void* src) {
  rlb_status st = ready(X, false);
  if (st != RLB_OK) return st;
  if (!src) return bfail(X, RLB_ERR_INVALID_ARG, "src is NULL");
  hipError_t e = state_copy(X->ws + X->off_F[0], src, X->state_elems * X->rsize, X->stream);
  if (e == hipSuccess) e = X->prec == RLB_FP32 ? box_records<float>(X) : box_records<double>(X);
  if (e != hipSuccess) return bhip(X, e, "state load");
  X->initialised = true;
  return RLB_OK;
}

rlb_status rlb_box_info(const rlb_box* X, double* dt, double* time, int32_t* Q) {
  if (!X) return RLB_ERR_INVALID_ARG;
  if (dt) *dt = X->bd.dt;
  if (time) *time = X->time;
  if (Q) *Q = X->bd.qp * X->bd.qx * X->bd.qf;
  return RLB_OK;
}

rlb_status rlb_box_check(rlb_box* X) {
  rlb_status st = ready(X, false);
  if (st != RLB_OK) return st;
  unsigned flag = 0;
  BHIP_TRY(X, hipMemcpyAsync(&flag, X->ws + X->off_flag, sizeof flag, hipMemcpyDeviceToHost, X->stream));
  BHIP_TRY(X, hipStreamSynchronize(X->stream));
  if (flag & kFlagNonphysical)
    return bfail(X, RLB_ERR_NONPHYSICAL, "a cell reached a non-physical state (e <= 0, n <= 0, |v| >= 1 or NaN)");
  return RLB_OK;
}

rlb_status rlb_box_flags(rlb_box* X, uint32_t* flags) {
  rlb_status st = ready(X, false);
  if (st != RLB_OK) return st;
  if (!flags) return bfail(X, RLB_ERR_INVALID_ARG, "flags is NULL");
  unsigned flag = 0;
  BHIP_TRY(X, hipMemcpyAsync(&flag, X->ws + X->off_flag, sizeof flag, hipMemcpyDeviceToHost, X->stream));
  BHIP_TRY(X, hipStreamSynchronize(X->stream));
  *flags = flag;
  return RLB_OK;
}

const char* rlb_box_last_error(const rlb_box* X) {
  if (!X) return g_box_create_error.c_str();
  return X->err.c_str();
}

}  // extern "C"
