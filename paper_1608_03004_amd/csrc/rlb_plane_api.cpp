// Host side of the plane (x, z) interface declared in include/rlb.h:
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

thread_local std::string g_plane_create_error;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

double plane_dt(const rlb_plane_desc& d) {
  if (d.dt > 0) return d.dt;
  const double dx = (d.x_max - d.x_min) / d.nx, dz = (d.z_max - d.z_min) / d.nz;
  return std::min(d.cfl / (1.0 / dx + 1.0 / dz), d.dt_tau_max * d.tau);
}

}  // namespace

struct rlb_plane {
  rlb_plane_desc desc;
  rlb_precision prec = RLB_FP64;
  size_t rsize = 8;
  PlaneDev pd;
  int qpt = 3, nvt = 5, grid = 1, stage_grid = 1;
  std::vector<double> vtab_d, itab, aux_d;
  std::vector<float> vtab_f, aux_f;
  int aux_pairs = 0;
  int64_t state_elems = 0;
  size_t off_F[3] = {0, 0, 0}, off_rec[3] = {0, 0, 0};
  size_t off_pd = 0, off_vtab = 0, off_itab = 0, off_aux = 0, off_flag = 0, total = 0;
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
// when both ends are 16-byte aligned, the runtime's copy otherwise (caller
// buffers may be views at any element offset).
hipError_t state_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16) == 0)
    return launch_copy(dst, src, bytes, s);
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}

rlb_status pfail(rlb_plane* P, rlb_status st, const std::string& msg) {
  if (P) P->err = msg; else g_plane_create_error = msg;
  return st;
}

rlb_status phip(rlb_plane* P, hipError_t e, const char* where) {
  return pfail(P, RLB_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define PHIP_TRY(P, expr)                                   \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) return phip((P), _e, #expr);      \
  } while (0)

rlb_status validate_plane(const rlb_plane_desc& d, std::string& msg) {
  auto bad = [&](const char* what) {
    msg = std::string("plane: ") + what;
    return RLB_ERR_INVALID_ARG;
  };
  if (d.nx < 8 || d.nz < 8) return bad("nx and nz must be >= 8");
  if (int64_t(d.nx) * d.nz > (int64_t(1) << 26)) return bad("nx * nz must be <= 2^26");
  if (int64_t((d.nx + 63) / 64 * 64) * d.nz > (int64_t(1) << 27))
    return bad("the padded plane (nx rounded up to 64) * nz must be <= 2^27 cells");
  if (d.q_xi < 1 || d.q_xi > 4096) return bad("q_xi must be in [1, 4096]");
  if (d.q_p < 1 || d.q_p > kMaxQp) return bad("q_p must be in [1, 8]");
  if (d.n_v < 0 || d.n_v > kMaxNv) return bad("n_v must be in [0, 7]");
  if (d.n_p < 0 || d.n_p >= d.q_p) return bad("n_p must satisfy 0 <= n_p < q_p");
  if (d.n_p + 2 > 2 * d.q_p - 1) return bad("q_p too small to integrate T^{mu nu} of the equilibrium exactly");
  if (d.n_v + 2 > 2 * d.q_xi - 1) return bad("q_xi too small to integrate T^{mu nu} of the equilibrium exactly");
  if (d.q_phi < d.n_v + 3 || d.q_phi > 64) return bad("q_phi must satisfy n_v + 3 <= q_phi <= 64");
  if (!(d.x_max > d.x_min) || !(d.z_max > d.z_min) || !std::isfinite(d.x_min + d.x_max + d.z_min + d.z_max))
    return bad("need x_min < x_max and z_min < z_max");
  if (!(d.tau > 0)) return bad("tau must be > 0 (+inf allowed)");
  if (!(d.T0 > 0) || !std::isfinite(d.T0)) return bad("T0 must be > 0");
  if (!(d.weno_eps > 0) || !std::isfinite(d.weno_eps)) return bad("weno_eps must be > 0 and finite");
  if (d.dt < 0 || !std::isfinite(d.dt)) return bad("dt must be >= 0");
  if (d.dt == 0 && !(d.cfl > 0 && std::isfinite(d.cfl))) return bad("cfl must be > 0");
  if (d.dt == 0 && !(d.dt_tau_max > 0)) return bad("dt_tau_max must be > 0");
  const double dt = plane_dt(d);
  const double dx = (d.x_max - d.x_min) / d.nx, dz = (d.z_max - d.z_min) / d.nz;
  if (!(dt > 0) || !std::isfinite(dt)) return bad("time step is not a positive number");
  if (dt * (1.0 / dx + 1.0 / dz) > 1.5) {
    msg = "plane: dt (1/dx + 1/dz) exceeds the WENO5/RK3 stability limit 1.5";
    return RLB_ERR_UNSTABLE_DT;
  }
  if (dt > 2.5 * d.tau) {
    msg = "plane: dt/tau exceeds the RK3 stability limit 2.5";
    return RLB_ERR_UNSTABLE_DT;
  }
  return RLB_OK;
}

rlb_status ready(rlb_plane* P, bool need_init) {
  if (!P) return RLB_ERR_INVALID_ARG;
  if (!P->ws) return pfail(P, RLB_ERR_STATE, "no workspace bound (call rlb_plane_bind)");
  if (need_init && !P->initialised)
    return pfail(P, RLB_ERR_STATE, "no state (call rlb_plane_set_initial_fields or rlb_plane_set_state)");
  return RLB_OK;
}

template <typename Real>
PlaneArgs<Real> plane_args(const rlb_plane* P) {
  PlaneArgs<Real> a;
  std::memset(&a, 0, sizeof a);
  a.pl = P->dev<PlaneDev>(P->off_pd);
  a.aux_pairs = P->aux_pairs;
  a.vtab = P->dev<Real>(P->off_vtab);
  a.itab = P->dev<double>(P->off_itab);
  a.aux = P->dev<Real>(P->off_aux);
  a.flag = P->dev<unsigned>(P->off_flag);
  return a;
}

template <typename Real>
hipError_t plane_stage(rlb_plane* P, int stage, size_t fin, size_t fout, size_t rin, size_t rout) {
  PlaneArgs<Real> a = plane_args<Real>(P);
  a.stage = stage;
  a.fin = P->dev<Real>(fin);
  a.fn = P->dev<Real>(P->off_F[0]);
  a.fout = P->dev<Real>(fout);
  a.rec_in = P->dev<double>(rin);
  a.rec_out = P->dev<double>(rout);
  return launch_plane_stage(sizeof(Real) == 4, P->qpt, P->nvt, &a, P->stage_grid, P->stream);
}

template <typename Real>
hipError_t plane_records(rlb_plane* P) {
  PlaneArgs<Real> a = plane_args<Real>(P);
  a.fin = P->dev<Real>(P->off_F[0]);
  a.rec_out = P->dev<double>(P->off_rec[0]);
  return launch_plane_moments(sizeof(Real) == 4, &a, P->grid, P->stream);
}

template <typename Real>
hipError_t plane_init(rlb_plane* P, const double* fields) {
  PlaneArgs<Real> a = plane_args<Real>(P);
  a.init = fields;
  a.fout = P->dev<Real>(P->off_F[0]);
  a.rec_out = P->dev<double>(P->off_rec[0]);
  return launch_plane_init(sizeof(Real) == 4, P->qpt, P->nvt, &a, P->grid, P->stream);
}

}  // namespace

extern "C" {

rlb_status rlb_plane_defaults(rlb_plane_desc* d) {
  if (!d) return RLB_ERR_INVALID_ARG;
  std::memset(d, 0, sizeof *d);
  d->nx = 64;
  d->nz = 64;
  d->q_xi = 8;
  d->q_phi = 8;
  d->q_p = 3;
  d->n_v = 5;
  d->n_p = 2;
  d->x_min = -0.5;
  d->x_max = 0.5;
  d->z_min = -0.5;
  d->z_max = 0.5;
  d->tau = 1e-2;
  d->cfl = 0.5;
  d->dt_tau_max = 0.5;
  d->T0 = 1.0;
  d->weno_eps = 1e-6;
  return RLB_OK;
}

rlb_status rlb_plane_create(const rlb_plane_desc* desc, rlb_precision prec, rlb_plane** out) {
  if (!out) return pfail(nullptr, RLB_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!desc) return pfail(nullptr, RLB_ERR_INVALID_ARG, "desc is NULL");
  if (prec != RLB_FP64 && prec != RLB_FP32) return pfail(nullptr, RLB_ERR_INVALID_ARG, "unknown precision");
  std::string msg;
  const rlb_status st = validate_plane(*desc, msg);
  if (st != RLB_OK) return pfail(nullptr, st, msg);
  if (!rlb::plane_weno_eps_in_range(desc->weno_eps, prec == RLB_FP32))
    return pfail(nullptr, RLB_ERR_INVALID_ARG, "weno_eps must lie in [1e-10, 1e8] (FP32) or [1e-70, 1e70] (FP64)");
  const rlb_plane_desc& d = *desc;
  std::vector<double> xi, wxi, p, wp;
  if (!gauss_legendre_rule(d.q_xi, xi, wxi) || !gauss_laguerre1_rule(d.q_p, p, wp))
    return pfail(nullptr, RLB_ERR_INVALID_ARG, "quadrature construction failed");
  rlb_plane* P = new rlb_plane();
  P->desc = d;
  P->prec = prec;
  P->rsize = prec == RLB_FP32 ? 4 : 8;
  const int qh = d.q_phi / 2 + 1;
  // velocity table: v_x, v_z, the weighted moment factors and the advection
  // factors -v_x/dx, -v_z/dz per (j, k)
  const long double pi = 3.141592653589793238462643383279502884L;
  const long double adv_x = -(long double)d.nx / ((long double)d.x_max - d.x_min),
                    adv_z = -(long double)d.nz / ((long double)d.z_max - d.z_min);
  for (int j = 0; j < d.q_xi; ++j) {
    for (int k = 0; k < qh; ++k) {
      const long double c = std::cos(2.0L * pi * k / d.q_phi);
      const long double vz = xi[j], vx = std::sqrt(1.0L - vz * vz) * c;
      const bool single = (k == 0) || (2 * k == d.q_phi);
      const long double w = (long double)wxi[j] * (single ? 1.0L : 2.0L) / d.q_phi;
      const long double row[kVStride] = {vx, vz, w, w * vx, w * vz, w * vx * vx, w * vx * vz, w * vz * vz,
                                         adv_x * vx, adv_z * vz, 0.0L, 0.0L};
      for (int q = 0; q < kVStride; ++q) P->vtab_d.push_back(double(row[q]));
    }
  }
  P->vtab_f.assign(P->vtab_d.begin(), P->vtab_d.end());
  // radial rows (as for a tube)
  const double t3 = d.T0 * d.T0 * d.T0, t4 = t3 * d.T0;
  for (int i = 0; i < d.q_p; ++i) {
    double row[kIStride];
    row[0] = p[i];
    row[1] = wp[i];
    row[2] = t3 * wp[i] * p[i];
    row[3] = t4 * wp[i] * p[i] * p[i];
    for (int l = 0; l <= kMaxNp; ++l) row[4 + l] = laguerre1_value(l, p[i]);
    P->itab.insert(P->itab.end(), row, row + kIStride);
  }
  // projection rule: symmetric pairs of a Gauss-Legendre rule
  const int M = prec == RLB_FP32 ? 2 * kAuxPairsFP32 : 2 * kAuxPairsFP64;
  std::vector<double> ax, aw;
  gauss_legendre_rule(M, ax, aw);
  P->aux_pairs = M / 2;
  for (int a = 0; a < M / 2; ++a) {
    const int j = M / 2 + a;
    double row[kAuxStride];
    row[0] = ax[j];
    for (int k = 0; k <= kMaxNv; ++k) row[1 + k] = aw[j] * (2 * k + 1) / 2.0 * legendre_value(k, ax[j]);
    for (int k = kMaxNv + 2; k < kAuxStride; ++k) row[k] = 0.0;
    P->aux_d.insert(P->aux_d.end(), row, row + kAuxStride);
  }
  P->aux_f.assign(P->aux_d.begin(), P->aux_d.end());
  // device descriptor
  PlaneDev& pd = P->pd;
  std::memset(&pd, 0, sizeof pd);
  pd.nx = d.nx;
  pd.nz = d.nz;
  pd.ldx = (d.nx + 63) / 64 * 64;
  pd.qx = d.q_xi;
  pd.qh = qh;
  pd.qp = d.q_p;
  pd.nv = d.n_v;
  pd.np = d.n_p;
  pd.plane = int64_t(d.nz) * pd.ldx;
  pd.dx_inv = d.nx / (d.x_max - d.x_min);
  pd.dz_inv = d.nz / (d.z_max - d.z_min);
  pd.dt = plane_dt(d);
  pd.tau_inv = 1.0 / d.tau;
  pd.T0 = d.T0;
  pd.weno_eps = d.weno_eps;
  if (d.n_v <= 5 && d.q_p <= 3) { P->qpt = 3; P->nvt = 5; }
  else if (d.n_v <= 5 && d.q_p == 4) { P->qpt = 4; P->nvt = 5; }
  else { P->qpt = 8; P->nvt = 7; }
  P->grid = ((d.nx + kPlaneTileX - 1) / kPlaneTileX) * ((d.nz + kPlaneTileZ - 1) / kPlaneTileZ);
  P->stage_grid = plane_stage_grid(d.nx, d.nz);
  P->state_elems = int64_t(d.q_p) * d.q_xi * qh * pd.plane;
  // workspace layout
  size_t o = 0;
  for (int k = 0; k < 3; ++k) { P->off_F[k] = o; o = align256(o + P->state_elems * P->rsize); }
  for (int k = 0; k < 3; ++k) { P->off_rec[k] = o; o = align256(o + 9 * size_t(pd.plane) * 8); }
  P->off_pd = o; o = align256(o + sizeof(PlaneDev));
  P->off_vtab = o; o = align256(o + P->vtab_d.size() * P->rsize);
  P->off_itab = o; o = align256(o + P->itab.size() * 8);
  P->off_aux = o; o = align256(o + P->aux_d.size() * P->rsize);
  P->off_flag = o; o = align256(o + 16);
  P->total = o;
  *out = P;
  return RLB_OK;
}

rlb_status rlb_plane_destroy(rlb_plane* P) {
  if (!P) return RLB_ERR_INVALID_ARG;
  delete P;
  return RLB_OK;
}

rlb_status rlb_plane_workspace_size(const rlb_plane* P, size_t* bytes) {
  if (!P || !bytes) return RLB_ERR_INVALID_ARG;
  *bytes = P->total;
  return RLB_OK;
}

rlb_status rlb_plane_bind(rlb_plane* P, void* workspace, size_t bytes, void* hip_stream) {
  if (!P) return RLB_ERR_INVALID_ARG;
  if (!workspace) return pfail(P, RLB_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return pfail(P, RLB_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (bytes < P->total) return pfail(P, RLB_ERR_INVALID_ARG, "workspace too small (see rlb_plane_workspace_size)");
  P->ws = static_cast<char*>(workspace);
  P->stream = static_cast<hipStream_t>(hip_stream);
  P->initialised = false;
  PHIP_TRY(P, hipMemsetAsync(P->ws, 0, P->total, P->stream));
  PHIP_TRY(P, hipMemcpyAsync(P->ws + P->off_pd, &P->pd, sizeof(PlaneDev), hipMemcpyHostToDevice, P->stream));
  if (P->prec == RLB_FP32) {
    PHIP_TRY(P, hipMemcpyAsync(P->ws + P->off_vtab, P->vtab_f.data(), P->vtab_f.size() * 4, hipMemcpyHostToDevice, P->stream));
    PHIP_TRY(P, hipMemcpyAsync(P->ws + P->off_aux, P->aux_f.data(), P->aux_f.size() * 4, hipMemcpyHostToDevice, P->stream));
  } else {
    PHIP_TRY(P, hipMemcpyAsync(P->ws + P->off_vtab, P->vtab_d.data(), P->vtab_d.size() * 8, hipMemcpyHostToDevice, P->stream));
    PHIP_TRY(P, hipMemcpyAsync(P->ws + P->off_aux, P->aux_d.data(), P->aux_d.size() * 8, hipMemcpyHostToDevice, P->stream));
  }
  PHIP_TRY(P, hipMemcpyAsync(P->ws + P->off_itab, P->itab.data(), P->itab.size() * 8, hipMemcpyHostToDevice, P->stream));
  PHIP_TRY(P, hipStreamSynchronize(P->stream));
  return RLB_OK;
}

rlb_status rlb_plane_set_initial_fields(rlb_plane* P, const double* fields) {
  rlb_status st = ready(P, false);
  if (st != RLB_OK) return st;
  if (!fields) return pfail(P, RLB_ERR_INVALID_ARG, "fields_device is NULL");
  const hipError_t e = P->prec == RLB_FP32 ? plane_init<float>(P, fields) : plane_init<double>(P, fields);
  if (e != hipSuccess) return phip(P, e, "plane init kernel launch");
  PHIP_TRY(P, hipMemsetAsync(P->ws + P->off_flag, 0, 16, P->stream));
  P->time = 0.0;
  P->initialised = true;
  return RLB_OK;
}

rlb_status rlb_plane_step(rlb_plane* P, int64_t nsteps) {
  rlb_status st = ready(P, true);
  if (st != RLB_OK) return st;
  if (nsteps < 0) return pfail(P, RLB_ERR_INVALID_ARG, "nsteps must be >= 0");
  const bool fp32 = P->prec == RLB_FP32;
  for (int64_t n = 0; n < nsteps; ++n) {
    for (int stage = 1; stage <= 3; ++stage) {
      const int fin = stage == 1 ? 0 : (stage == 2 ? 1 : 2);
      const int fout = stage == 1 ? 1 : (stage == 2 ? 2 : 0);
      const hipError_t e =
          fp32 ? plane_stage<float>(P, stage, P->off_F[fin], P->off_F[fout], P->off_rec[fin], P->off_rec[fout])
               : plane_stage<double>(P, stage, P->off_F[fin], P->off_F[fout], P->off_rec[fin], P->off_rec[fout]);
      if (e != hipSuccess) return phip(P, e, "plane stage kernel launch");
    }
  }
  P->time += nsteps * P->pd.dt;
  return RLB_OK;
}

rlb_status rlb_plane_fields(rlb_plane* P, double* out) {
  rlb_status st = ready(P, true);
  if (st != RLB_OK) return st;
  if (!out) return pfail(P, RLB_ERR_INVALID_ARG, "out_device is NULL");
  const hipError_t e = launch_plane_fields(P->dev<PlaneDev>(P->off_pd), P->pd.nx, P->pd.nz,
                                           P->dev<double>(P->off_rec[0]), out, P->dev<unsigned>(P->off_flag), P->stream);
  if (e != hipSuccess) return phip(P, e, "plane fields kernel launch");
  return RLB_OK;
}

rlb_status rlb_plane_layout(const rlb_plane* P, int64_t* state_elems, int64_t* ldx) {
  if (!P || !state_elems || !ldx) return RLB_ERR_INVALID_ARG;
  *state_elems = P->state_elems;
  *ldx = P->pd.ldx;
  return RLB_OK;
}

rlb_status rlb_plane_get_state(rlb_plane* P, void* dst) {
  rlb_status st = ready(P, true);
  if (st != RLB_OK) return st;
  if (!dst) return pfail(P, RLB_ERR_INVALID_ARG, "dst is NULL");
  const hipError_t e = state_copy(dst, P->ws + P->off_F[0], P->state_elems * P->rsize, P->stream);
  if (e != hipSuccess) return phip(P, e, "state copy");
  return RLB_OK;
}

rlb_status rlb_plane_set_state(rlb_plane* P, const void* src) {
  rlb_status st = ready(P, false);
  if (st != RLB_OK) return st;
  if (!src) return pfail(P, RLB_ERR_INVALID_ARG, "src is NULL");
  hipError_t e = state_copy(P->ws + P->off_F[0], src, P->state_elems * P->rsize, P->stream);
  if (e == hipSuccess) e = P->prec == RLB_FP32 ? plane_records<float>(P) : plane_records<double>(P);
  if (e != hipSuccess) return phip(P, e, "state load");
  P->initialised = true;
  return RLB_OK;
}

rlb_status rlb_plane_info(const rlb_plane* P, double* dt, double* time, int32_t* Q) {
  if (!P) return RLB_ERR_INVALID_ARG;
  if (dt) *dt = P->pd.dt;
  if (time) *time = P->time;
  if (Q) *Q = P->pd.qp * P->pd.qx * P->pd.qh;
  return RLB_OK;
}

rlb_status rlb_plane_check(rlb_plane* P) {
  rlb_status st = ready(P, false);
  if (st != RLB_OK) return st;
  unsigned flag = 0;
  PHIP_TRY(P, hipMemcpyAsync(&flag, P->ws + P->off_flag, sizeof flag, hipMemcpyDeviceToHost, P->stream));
  PHIP_TRY(P, hipStreamSynchronize(P->stream));
  if (flag & kFlagNonphysical)
    return pfail(P, RLB_ERR_NONPHYSICAL, "a cell reached a non-physical state (e <= 0, n <= 0, |v| >= 1 or NaN)");
  return RLB_OK;
}

rlb_status rlb_plane_flags(rlb_plane* P, uint32_t* flags) {
  rlb_status st = ready(P, false);
  if (st != RLB_OK) return st;
  if (!flags) return pfail(P, RLB_ERR_INVALID_ARG, "flags is NULL");
  unsigned flag = 0;
  PHIP_TRY(P, hipMemcpyAsync(&flag, P->ws + P->off_flag, sizeof flag, hipMemcpyDeviceToHost, P->stream));
  PHIP_TRY(P, hipStreamSynchronize(P->stream));
  *flags = flag;
  return RLB_OK;
}

const char* rlb_plane_last_error(const rlb_plane* P) {
  if (!P) return g_plane_create_error.c_str();
  return P->err.c_str();
}

}  // extern "C"
