/*
 * rlb.h -- C interface of the MI355X (gfx950) implementation of the
 * quadrature-based finite-difference relativistic lattice Boltzmann model for
 * massless particles of Blaga & Ambrus, "Quadrature-based Lattice Boltzmann
 * Model for Relativistic Flows" (arXiv:1608.03004).
 *
 * One time step advances, for every cell and every point of the momentum
 * quadrature, the 1D Boltzmann equation with the Anderson-Witting collision
 * term (section "Relativistic lattice Boltzmann equation", eq. Boltz):
 *   moments N^mu, T^{mu nu} -> Landau frame (e, u^mu, n, T) -> truncated
 *   Maxwell-Juettner equilibrium (eq. feqtrunc) -> WENO5 upwind advection and
 *   relaxation -> third-order SSP Runge-Kutta (section "Numerical results").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All functions return an rlb_status; 0 is success, negative is an error.
 *   Argument errors are detected synchronously on the host before any device
 *   work is queued; the lattice is then unchanged.  rlb_last_error() gives a
 *   human-readable reason for the last failure on a lattice.
 * - Device pointers are plain HIP device addresses.  The caller owns the
 *   workspace (rlb_bind) and every state/adjoint buffer it passes in; the
 *   library owns only the opaque handle and its host-side tables.  The library
 *   never allocates device memory; its only device memory of its own is the
 *   static scratch array of rlb_step_noalloc (see there).
 * - Work is queued asynchronously on the HIP stream given to rlb_bind (NULL
 *   means the legacy default stream).  Calls documented as "synchronizes" wait
 *   for that stream.  A lattice must not be used from two threads at once.
 *   A lattice with a high-order tube (n_v > 7) also owns one side stream
 *   (default priority, created by its first rlb_bind on the device current
 *   then) on which the equilibrium pre-pass of a stage runs piece by piece,
 *   ordered with events against the stage kernels on the lattice's stream; a
 *   step's work on the side stream is complete when the lattice's stream
 *   reaches the step's end.
 * - A non-physical cell state met on the device (e <= 0, n <= 0, |v| >= 1 or
 *   NaN in the Landau matching) sets a sticky flag; the next synchronizing call
 *   (rlb_moments, rlb_totals, rlb_check) returns RLB_ERR_NONPHYSICAL.
 *
 * Layouts
 * -------
 * Quadrature point s = i*q_xi + j, with i the Gauss-Laguerre (|p|) node and j
 * the Gauss-Legendre (xi = cos theta) node, both in ascending order.  The
 * azimuthal angle drops out of the 1D problem exactly and is not stored.
 * A state buffer holds, for every tube, the weight-free distribution values
 *   F_s(x) = 2*pi * exp(p_i) * f(p_i, xi_j; z_x)      (p in units of T0)
 * in rows of ld_x >= nx elements: element (s, x) of tube t is at
 *   state + off[t] + s*ld[t] + x, in FP64 or FP32 as chosen at creation.
 * rlb_state_layout() returns off[t] and ld[t] (in elements).  The quadrature-
 * weighted distribution of the paper is f_s = w^p_i w^xi_j F_s.
 */
#ifndef RLB_H
#define RLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RLB_OK = 0,
  RLB_ERR_INVALID_ARG = -1, /* an argument is out of range; nothing was done  */
  RLB_ERR_NONPHYSICAL = -2, /* the sticky device flag is set (see above)       */
  RLB_ERR_HIP = -3,         /* a HIP runtime call failed                        */
  RLB_ERR_STATE = -4,       /* call out of order (e.g. step before bind/init)   */
  RLB_ERR_UNSTABLE_DT = -5  /* dt*|rate| outside the explicit RK3 stability box */
} rlb_status;

typedef enum { RLB_FP64 = 0, RLB_FP32 = 1 } rlb_precision;

/* Creation flags. */
#define RLB_WITH_ADJOINT 1u /* reserve workspace for rlb_adjoint_step */

/*
 * One shock tube, following the problem statement of the paper:
 *   grid      -- the unit-length domain of 1 x 1 x L_z nodes of section
 *                Numerical results: cell-centred cells on [z_min, z_max],
 *                dz = (z_max - z_min)/nx, 8 <= nx <= 2^26;
 *   q_xi, q_p -- quadrature orders (section "Discretization of the momentum
 *                space"; Q_p = 3 suffices for N^mu and T^{mu nu}, section
 *                Riemann problem); q_p <= 8;
 *   n_v, n_p  -- truncation orders of eq. feqtrunc (the paper uses 5 and 2);
 *                n_p < q_p;  n_v <= 7, or 7 < n_v < q_xi <= 256 (the
 *                high-order form: the equilibrium is evaluated by a
 *                matrix-core pre-pass into one more state-sized buffer, and
 *                RLB_WITH_ADJOINT adds one for the adjoint's own pre-pass);
 *                N^mu and T^{mu nu} of the equilibrium are exact
 *                when n_p + 2 <= 2 q_p - 1 and n_v + 2 <= 2 q_xi - 1, both
 *                required;
 *   tau       -- constant relaxation time (section Relativistic LB equation);
 *                +INFINITY gives the collisionless (ballistic) limit;
 *   dt        -- > 0: explicit time step; 0: min(cfl*dz, dt_tau_max*tau)
 *                (CFL with the speed of light, section Numerical results);
 *   T0        -- reference temperature of eq. feq (results do not depend on
 *                it in exact arithmetic);
 *   weno_eps  -- WENO5 epsilon applied to the weight-free F; in
 *                [1e-40, 1e30] for FP32 lattices, [1e-300, 1e30] for FP64.
 * rlb_tube_defaults() fills the paper's values (nx 800, q_xi 8, q_p 3,
 * n_v 5, n_p 2, tau 1e-2, z in [-0.5, 0.5], cfl 0.5, dt_tau_max 0.5, T0 1,
 * weno_eps 1e-6).
 */
typedef struct {
  int32_t nx;
  int32_t q_xi, q_p;
  int32_t n_v, n_p;
  int32_t reserved0;
  double z_min, z_max;
  double tau;
  double cfl;
  double dt_tau_max;
  double dt;
  double T0;
  double weno_eps;
} rlb_tube_desc;

/* Macroscopic state (pressure P, density n, velocity u^z) of one side of the
 * Riemann problem (section Riemann problem, eq. condinit). */
typedef struct {
  double P, n, u;
} rlb_state;

/* Launch schedule of the stage kernels (chosen by the autotuner).  Every
 * schedule gives bit-identical states and records.  Default after rlb_create:
 * tile 256 (64 when 256-cell tiles would number fewer than half the CUs),
 * no persistent grid, no graph replay, default chunk, split below the CU
 * count. */
typedef struct {
  int32_t tile;        /* cells per workgroup: 64, 128 or 256                   */
  int32_t persistent;  /* 1: grid sized to the device, blocks loop over tiles   */
  int32_t blocks_per_cu; /* persistent grid = blocks_per_cu * CU count           */
  int32_t graph_steps; /* >0: replay time steps from a captured hipGraph of this many steps */
  int32_t chunk;       /* quadrature points staged per LDS chunk: 0 (default: 8 in FP32, 4 in FP64)
                          or twice the default                                  */
  int32_t split_below; /* a kernel group with fewer work items than this spreads each stage over
                          its radial nodes (one workgroup per tile and node, then a combine
                          kernel); -1: the device's CU count (default), 0: never */
} rlb_schedule;

typedef struct rlb_lattice rlb_lattice;

rlb_status rlb_tube_defaults(rlb_tube_desc* desc);

/* Validates the tubes and builds the host tables; no device work.  The
 * tables are the momentum quadrature of the section "Discretization of the
 * momentum space": Gauss-Legendre nodes and weights in xi = cos(theta)
 * (eq. polarInt, with the weight 2(1 - xi^2)/((Q+1)^2 P_{Q+1}(xi)^2)) and
 * Gauss-Laguerre (alpha = 1) nodes and weights in p (the radial rule of the
 * same section); the grid and time step follow section Numerical results.
 * tubes: ntubes >= 1 descriptors (copied).  prec: arithmetic of the
 * distribution (the Landau matching and the moment records are always FP64).
 * flags: RLB_WITH_ADJOINT or 0 (with RLB_WITH_ADJOINT the workspace also
 * holds the adjoint's buffers, for every tube form).  *out receives the
 * handle. */
rlb_status rlb_create(const rlb_tube_desc* tubes, int32_t ntubes, rlb_precision prec, uint32_t flags,
                      rlb_lattice** out);
rlb_status rlb_destroy(rlb_lattice* lat);

/* Bytes of device workspace the lattice needs (256-byte aligned base). */
rlb_status rlb_workspace_size(const rlb_lattice* lat, size_t* bytes);
/* Attaches caller-owned device memory and the stream, clears it and uploads
 * the tables (synchronizes the stream).  May be called again to move the
 * lattice; the state must then be set again. */
rlb_status rlb_bind(rlb_lattice* lat, void* workspace, size_t bytes, void* hip_stream);
rlb_status rlb_set_stream(rlb_lattice* lat, void* hip_stream);
rlb_status rlb_set_schedule(rlb_lattice* lat, const rlb_schedule* sched);
rlb_status rlb_get_schedule(const rlb_lattice* lat, rlb_schedule* sched);

/* Initial condition of eq. condinit: the truncated equilibrium of `left` for
 * cell centres z < 0 and of `right` otherwise.  tube = -1 sets every tube.
 * Resets the tube's time to 0.  Requires P > 0, n > 0. */
rlb_status rlb_set_initial_state(rlb_lattice* lat, int32_t tube, rlb_state left, rlb_state right);

/* Per-tube initial states in one call: left[t], right[t] for t < ntubes
 * (ntubes must equal the lattice's tube count). */
rlb_status rlb_set_initial_states(rlb_lattice* lat, int32_t ntubes, const rlb_state* left, const rlb_state* right);

/* Advances every tube by nsteps time steps of eq. Boltz (advection with the
 * fifth-order WENO scheme and Anderson-Witting relaxation towards the
 * truncated equilibrium of eq. feqtrunc in the Landau frame) with the
 * third-order Runge-Kutta integrator of section Numerical results (three
 * stage launches per step; the moments, Landau frame and equilibrium are
 * recomputed at every stage).  Asynchronous. */
rlb_status rlb_step(rlb_lattice* lat, int64_t nsteps);

/* Per-cell fields of one tube, FP64, 10 rows of ld >= nx:
 * N0, Nz, T00, T0z, Tzz, e, n, v, T, |N| = sqrt(N0^2 - Nz^2): the moments
 * N^mu and T^{mu nu} as quadrature sums (section Relativistic LB equation,
 * the definitions of N^mu and T^{mu nu}), the Landau-frame energy density,
 * density, velocity and temperature (T^mu_nu u^nu = -e u^mu, n = -u_mu N^mu,
 * e = 3nT), and |N|, the density of the free-streaming profile eq. ballistic.
 * rlb_fields writes a device buffer asynchronously; rlb_moments writes a host
 * buffer, synchronizes, and reports the sticky flag. */
rlb_status rlb_fields(rlb_lattice* lat, int32_t tube, double* dev_out, int64_t ld);
rlb_status rlb_moments(rlb_lattice* lat, int32_t tube, double* host_out, int64_t ld);
/* FP64 totals dz*sum(N0), dz*sum(T00), dz*sum(T0z) -- the integrals of N^0
 * and T^{0 mu} that the method conserves (section Relativistic LB equation:
 * the collision term conserves N^mu and T^{mu nu} in the Landau frame) up to
 * the boundary fluxes; synchronizes. */
rlb_status rlb_totals(rlb_lattice* lat, int32_t tube, double out[3]);
/* Synchronizes and reports the sticky flag; RLB_OK if clear. */
rlb_status rlb_check(rlb_lattice* lat);
/* Sticky flag bits (rlb_flags, rlb_plane_flags, rlb_step_noalloc). */
#define RLB_FLAG_NONPHYSICAL 1u /* e <= 0, n <= 0, |v| >= 1 or NaN met          */
#define RLB_FLAG_FAST_FLOW 2u   /* |v| > 0.95 met: the projection of the
                                   equilibrium (auxiliary Gauss-Legendre rule of
                                   48 points in FP64, 24 in FP32) loses accuracy
                                   there (about 1e-6 relative at |v| = 0.99 in
                                   FP64); results are still computed */
/* Synchronizes and returns in *flags every sticky bit raised since the last
 * initial state (the non-physical bit also makes rlb_check fail). */
rlb_status rlb_flags(rlb_lattice* lat, uint32_t* flags);

/* State buffers: element count of a full state and each tube's placement. */
rlb_status rlb_state_elems(const rlb_lattice* lat, int64_t* elems);
rlb_status rlb_state_layout(const rlb_lattice* lat, int32_t tube, int64_t* off, int64_t* ld);
/* Copies the current state to / from a caller device buffer (asynchronous).
 * rlb_set_state also recomputes the moment records. */
rlb_status rlb_get_state(rlb_lattice* lat, void* dst_device);
rlb_status rlb_set_state(rlb_lattice* lat, const void* src_device);

/* Truncated equilibrium (eq. feqtrunc, truncated at N_p and N_v) of the
 * current state, in the Landau frame of each cell's moments, for the tubes
 * of the high-order form (n_v > 7): dst_device (device memory, state layout
 * and precision of the lattice, rlb_state_elems elements, caller-owned)
 * receives F_eq at every quadrature point of those tubes' cells; the entries
 * of other tubes and of padding cells are left untouched.  It is the pre-pass
 * that each stage runs on its input (matrix cores, FP64 arithmetic, rounded
 * to the lattice's precision).  Asynchronous on the lattice's stream.
 * RLB_ERR_INVALID_ARG if dst_device is NULL or no tube has n_v > 7;
 * RLB_ERR_STATE without a bound workspace and a state. */
rlb_status rlb_equilibrium(rlb_lattice* lat, void* dst_device);

/* Per-tube parameters and time.  rlb_set_time sets the elapsed time that
 * rlb_tube_info reports (tube = -1: every tube), e.g. after restoring a saved
 * state with rlb_set_state, which leaves the clocks as they are. */
rlb_status rlb_set_tau(rlb_lattice* lat, int32_t tube, double tau);
rlb_status rlb_set_time(rlb_lattice* lat, int32_t tube, double time);
rlb_status rlb_tube_info(const rlb_lattice* lat, int32_t tube, double* dt, double* time, int32_t* Q);

/* Quadrature tables of a tube as used on the device (host copies):
 * xi[q_xi], w_xi[q_xi], p[q_p], w_p[q_p]. */
rlb_status rlb_tables(const rlb_lattice* lat, int32_t tube, double* xi, double* w_xi, double* p, double* w_p);

/*
 * Discrete adjoint (reverse mode) of the time step, for gradients of a loss on
 * the final fields with respect to tau and the initial states, for every tube
 * form: in the high-order form (n_v > 7) an adjoint stage re-evaluates its
 * input's equilibrium with the forward's pre-pass and applies the transposed
 * even/odd projection tables.  The lattice must have been created with
 * RLB_WITH_ADJOINT.  All buffers are device memory in the state layout (see
 * above); all calls are asynchronous unless noted.
 *
 * rlb_adjoint_step: lambda holds dL/df^{n+1} on entry and dL/df^n on return,
 *   where f^{n+1} is the step (3 stages) applied to state_n = f^n.  The two
 *   intermediate stages are recomputed from state_n.  dL_dtau[t] (device, one
 *   double per tube) is incremented by the step's contribution to dL/dtau_t at
 *   fixed time step.  state_n and lambda must not overlap.
 * rlb_adjoint_segment: the reverse sweep over one checkpoint segment of
 *   nsteps >= 1 steps starting from state0 = f^n (the sqrt(N) checkpointing of
 *   the adjoint): recomputes the segment's states f^{n+k} and their stage
 *   states f1, f2 into `scratch` (device, caller-owned, at least
 *   rlb_adjoint_segment_size bytes), then applies the adjoint step to each
 *   step in reverse order, so lambda goes from dL/df^{n+nsteps} to dL/df^n
 *   and dL_dtau accumulates.  The result equals, bit for bit, nsteps calls of
 *   rlb_adjoint_step on the same states; the stage states are computed once
 *   instead of twice.  The lattice's own state is not touched.  state0,
 *   scratch and lambda must not overlap.
 * rlb_fields_adjoint: writes into tube's rows of lambda the gradient dL/df of a
 *   loss on the fields of `state` (the rows of rlb_fields: N0, Nz, T00, T0z,
 *   Tzz, e, n, v, T, |N|), given dL_dfields [10][ld] (device, FP64).
 * rlb_initial_state_adjoint: given lambda0 = dL/df(t = 0), returns on the host
 *   dL/d(P, n, u) of the left and right states of eq. condinit; synchronizes.
 */
rlb_status rlb_adjoint_step(rlb_lattice* lat, const void* state_n, void* lambda, double* dL_dtau);
rlb_status rlb_adjoint_segment_size(const rlb_lattice* lat, int32_t nsteps, size_t* bytes);
rlb_status rlb_adjoint_segment(rlb_lattice* lat, const void* state0, int32_t nsteps, void* scratch, size_t bytes,
                               void* lambda, double* dL_dtau);
/* The two halves of rlb_adjoint_segment, for callers that overlap the
 * recomputation of one segment with the reverse sweep of the next one in
 * reverse order (two scratch buffers, two streams; both halves are small,
 * latency-bound launches that leave most of the GPU idle).
 * rlb_adjoint_segment_forward recomputes the states of the nsteps steps from
 * state0 into scratch on hip_stream (NULL: the lattice's stream);
 * rlb_adjoint_segment_reverse applies the adjoint of those steps, last first,
 * on the lattice's stream.  The caller orders them with events: a reverse
 * sweep after the forward half that filled its scratch, and a forward half
 * into a scratch after the reverse sweep that last read it.  The forward half
 * uses none of the buffers of the reverse sweep, so the two may run at the
 * same time; no rlb_step may run meanwhile.  Results equal rlb_adjoint_segment
 * bit for bit. */
rlb_status rlb_adjoint_segment_forward(rlb_lattice* lat, const void* state0, int32_t nsteps, void* scratch,
                                       size_t bytes, void* hip_stream);
rlb_status rlb_adjoint_segment_reverse(rlb_lattice* lat, int32_t nsteps, const void* scratch, size_t bytes,
                                       void* lambda, double* dL_dtau);
rlb_status rlb_fields_adjoint(rlb_lattice* lat, int32_t tube, const void* state, const double* dL_dfields, int64_t ld,
                              void* lambda);
rlb_status rlb_initial_state_adjoint(rlb_lattice* lat, int32_t tube, const void* lambda0, double grad_left[3],
                                     double grad_right[3]);

/*
 * Allocation-free time steps, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Advances the caller's state (device memory, state layout and
 * precision of the lattice: input f^n, output f^{n+nsteps}, in place) by
 * nsteps SSP-RK3 steps with the lattice's tubes, time steps and schedule
 * (without graph replay), on hip_stream; asynchronous.  The lattice needs no
 * workspace (rlb_bind is not required) and its own state, time and flag are
 * not touched.  The moment records are recomputed from `state` first, so the
 * result equals, bit for bit, rlb_set_state(state) followed by
 * rlb_step(nsteps) on a bound lattice.
 * Every other buffer of the step (stage arrays, moment records, tables, work
 * list, node-split sums, high-order equilibrium values) lives in a static
 * device array of RLB_NOALLOC_SCRATCH_BYTES per GPU, held from the first call
 * on a GPU until the process ends; the call makes no allocation.  A lattice
 * whose step needs more is rejected with RLB_ERR_INVALID_ARG (the reason is
 * in rlb_last_error).  Calls on one GPU share the array and must not overlap
 * (they race); consecutive calls on one stream are fine, whatever lattice
 * they use.
 * flags_device: NULL, or one device word that receives the sticky flag bits
 * raised during this call (bit 0: non-physical state, bit 1: |v| > 0.95); it
 * is cleared at the start of the call.  state must not overlap flags_device.
 */
#define RLB_NOALLOC_SCRATCH_BYTES (64u << 20)
rlb_status rlb_step_noalloc(rlb_lattice* lat, void* state, int64_t nsteps, uint32_t* flags_device, void* hip_stream);

/* Plain device copy kernel (bandwidth calibration); asynchronous. */
rlb_status rlb_device_copy(void* dst, const void* src, size_t bytes, void* hip_stream);
/* Streaming probe with the stage kernel's memory pattern (256-column tiles
 * walking the rows of [rows][ld] matrices in chunks, the same cache policies
 * and buffer accesses) and no arithmetic but one add: out = a + b, or out = a
 * when b is NULL (the one-read, one-write pattern of the first Runge-Kutta
 * stage).  The practical HBM ceiling of the stage kernel; elem_bytes 4 or 8;
 * device buffers, caller-owned; asynchronous. */
rlb_status rlb_device_stream(void* out, const void* a, const void* b, int64_t rows, int64_t ld, int32_t cols,
                             int32_t elem_bytes, void* hip_stream);

const char* rlb_status_string(rlb_status st);
const char* rlb_last_error(const rlb_lattice* lat);

/*
 * Multi-dimensional model on an (x, z) plane: eq. Boltz_gen with the particle
 * velocity v = (sin(theta) cos(phi), sin(theta) sin(phi), cos(theta)) resolved
 * in the plane, for data independent of y, on the full product quadrature of
 * the section "Discretization of the momentum space": q_p Gauss-Laguerre x
 * q_xi Gauss-Legendre x the q_phi-node trapezoid rule of eq. azimuthInt
 * (phi_k = 2 pi k / q_phi).  With u^y = 0 the nodes phi and -phi carry equal
 * values, so q_p * q_xi * (q_phi/2 + 1) points are evolved per cell.  The
 * Landau frame is the timelike eigenvector of T^mu_nu; the truncated
 * equilibrium (eq. feqtrunc) is the Legendre series of order n_v in v . u/|u|.
 * Cells are cell-centred on [x_min, x_max] x [z_min, z_max]; every edge is an
 * outflow (zero-gradient) boundary.
 *
 *   nx, nz     -- cells, 8 <= each, nx * nz <= 2^26 and, with rows padded
 *                 to 64 cells, ceil(nx/64)*64 * nz <= 2^27 (one point's plane
 *                 is addressed with 32-bit byte offsets);
 *   q_xi, q_phi, q_p, n_v, n_p -- as for a tube (n_v <= 7), plus
 *                 n_v + 3 <= q_phi <= 64 (the azimuthal rule integrates the
 *                 moments of the equilibrium exactly);
 *   tau, T0    -- as for a tube;
 *   weno_eps   -- as for a tube, in [1e-10, 1e8] for FP32 planes and
 *                 [1e-70, 1e70] for FP64 (the plane's weights are always
 *                 taken in product form, which needs this range; in FP32 the
 *                 weight-free F should also stay below ~1e3 in magnitude,
 *                 beyond which the products overflow and the cell is flagged
 *                 non-physical);
 *   dt         -- > 0: explicit; 0: min(cfl / (1/dx + 1/dz), dt_tau_max tau).
 *                 dt (1/dx + 1/dz) <= 1.5 and dt <= 2.5 tau are required.
 *
 * State layout (rlb_plane_layout): F[s][z][ldx], s = (i q_xi + j) (q_phi/2+1)
 * + k, precision of the plane, ldx >= nx.  Ownership as for a lattice: the
 * caller owns the workspace (rlb_plane_workspace_size bytes, 256-byte aligned)
 * and the stream; calls are asynchronous on that stream except where noted.
 */
typedef struct {
  int32_t nx, nz;
  int32_t q_xi, q_phi, q_p;
  int32_t n_v, n_p;
  int32_t reserved0;
  double x_min, x_max, z_min, z_max;
  double tau;
  double cfl;
  double dt_tau_max;
  double dt;
  double T0;
  double weno_eps;
} rlb_plane_desc;

typedef struct rlb_plane rlb_plane;

/* Defaults: 64 x 64 cells on [-0.5, 0.5]^2, q_xi 8, q_phi 8, q_p 3, n_v 5,
 * n_p 2, tau 1e-2, cfl 0.5, dt_tau_max 0.5, T0 1, weno_eps 1e-6. */
rlb_status rlb_plane_defaults(rlb_plane_desc* desc);
/* Validates the descriptor and builds the host tables; no device work. */
rlb_status rlb_plane_create(const rlb_plane_desc* desc, rlb_precision prec, rlb_plane** out);
rlb_status rlb_plane_destroy(rlb_plane* pl);
rlb_status rlb_plane_workspace_size(const rlb_plane* pl, size_t* bytes);
/* Binds the caller's device workspace and stream, clears it and uploads the
 * tables (synchronizes). */
rlb_status rlb_plane_bind(rlb_plane* pl, void* workspace, size_t bytes, void* hip_stream);
/* Initial state: every cell takes the truncated equilibrium of its state
 * fields_device[4][nz][nx] (FP64 device memory: P, n, u^x, u^z; P, n > 0),
 * which must stay valid until the stream reaches this call.  Time restarts at
 * 0 and the sticky flag is cleared. */
rlb_status rlb_plane_set_initial_fields(rlb_plane* pl, const double* fields_device);
/* nsteps SSP-RK3 steps (three stage launches each). */
rlb_status rlb_plane_step(rlb_plane* pl, int64_t nsteps);
/* Fields [14][nz][nx] (FP64 device memory): N0, Nx, Nz, T00, T0x, T0z, Txx,
 * Txz, Tzz, e, n, v_x, v_z, T of the current state.  A non-physical cell sets
 * the sticky flag. */
rlb_status rlb_plane_fields(rlb_plane* pl, double* out_device);
rlb_status rlb_plane_layout(const rlb_plane* pl, int64_t* state_elems, int64_t* ldx);
/* Copy the current state out of / into the workspace (device buffers of
 * state_elems elements); setting a state recomputes its records. */
rlb_status rlb_plane_get_state(rlb_plane* pl, void* dst_device);
rlb_status rlb_plane_set_state(rlb_plane* pl, const void* src_device);
/* Time step, elapsed time and evolved points per cell (host values). */
rlb_status rlb_plane_info(const rlb_plane* pl, double* dt, double* time, int32_t* Q);
/* Synchronizes and reports the sticky non-physical flag. */
rlb_status rlb_plane_check(rlb_plane* pl);
/* Synchronizes and returns the sticky flag bits (RLB_FLAG_*). */
rlb_status rlb_plane_flags(rlb_plane* pl, uint32_t* flags);
const char* rlb_plane_last_error(const rlb_plane* pl);

/*
 * Multi-dimensional model on an (x, y, z) box: eq. Boltz_gen with the particle
 * velocity v = (sin(theta) cos(phi), sin(theta) sin(phi), cos(theta)) resolved
 * in all three directions, on the full product quadrature of the section
 * "Discretization of the momentum space": q_p Gauss-Laguerre x q_xi
 * Gauss-Legendre x every node phi_k = 2 pi k / q_phi (k = 0 .. q_phi - 1) of
 * the trapezoid rule of eq. azimuthInt, weight 1/q_phi.  The flow may point
 * anywhere: q_p * q_xi * q_phi points are evolved per cell.  The Landau frame
 * is the timelike eigenvector of T^mu_nu (three velocity components); the
 * truncated equilibrium (eq. feqtrunc) is the Legendre series of order n_v in
 * c = v . u/|u| with the coefficients of the 1D projection at the speed |u|.
 * Cells are cell-centred on [x_min, x_max] x [y_min, y_max] x [z_min, z_max];
 * every face is an outflow (zero-gradient) boundary.  A box with ny = 1 and
 * u^y = 0 evolves like a plane; one varying along z only with u along z like
 * a tube.
 *
 *   nx, ny, nz -- cells, >= 1 each, nx * ny * nz <= 2^26 and, with rows
 *                 padded to 64 cells, ceil(nx/64)*64 * ny * nz <= 2^27;
 *   q_xi (<= 1024), q_phi, q_p, n_v, n_p -- as for a plane
 *                 (n_v + 3 <= q_phi <= 64, any parity);
 *   tau, T0, weno_eps -- as for a plane (the same weno_eps ranges);
 *   dt         -- > 0: explicit; 0: min(cfl / (1/dx + 1/dy + 1/dz),
 *                 dt_tau_max tau).  dt (1/dx + 1/dy + 1/dz) <= 1.5 and
 *                 dt <= 2.5 tau are required.
 *
 * State layout (rlb_box_layout): F[s][z][y][ldx], s = (i q_xi + j) q_phi + k,
 * precision of the box, ldx >= nx.  Ownership as for a plane: the caller owns
 * the workspace (rlb_box_workspace_size bytes, 256-byte aligned) and the
 * stream; calls are asynchronous on that stream except where noted.
 */
typedef struct {
  int32_t nx, ny, nz;
  int32_t q_xi, q_phi, q_p;
  int32_t n_v, n_p;
  double x_min, x_max, y_min, y_max, z_min, z_max;
  double tau;
  double cfl;
  double dt_tau_max;
  double dt;
  double T0;
  double weno_eps;
} rlb_box_desc;

typedef struct rlb_box rlb_box;

/* Defaults: 32^3 cells on [-0.5, 0.5]^3, q_xi 8, q_phi 8, q_p 3, n_v 5,
 * n_p 2, tau 1e-2, cfl 0.5, dt_tau_max 0.5, T0 1, weno_eps 1e-6. */
rlb_status rlb_box_defaults(rlb_box_desc* desc);
/* Validates the descriptor and builds the host tables; no device work. */
rlb_status rlb_box_create(const rlb_box_desc* desc, rlb_precision prec, rlb_box** out);
rlb_status rlb_box_destroy(rlb_box* bx);
rlb_status rlb_box_workspace_size(const rlb_box* bx, size_t* bytes);
/* Binds the caller's device workspace and stream, clears it and uploads the
 * tables (synchronizes). */
rlb_status rlb_box_bind(rlb_box* bx, void* workspace, size_t bytes, void* hip_stream);
/* Initial state: every cell takes the truncated equilibrium of its state
 * fields_device[5][nz][ny][nx] (FP64 device memory: P, n, u^x, u^y, u^z;
 * P, n > 0), which must stay valid until the stream reaches this call.  Time
 * restarts at 0 and the sticky flag is cleared. */
rlb_status rlb_box_set_initial_fields(rlb_box* bx, const double* fields_device);
/* nsteps SSP-RK3 steps (three stage launches each). */
rlb_status rlb_box_step(rlb_box* bx, int64_t nsteps);
/* Fields [20][nz][ny][nx] (FP64 device memory): N0, Nx, Ny, Nz, T00, T0x,
 * T0y, T0z, Txx, Txy, Txz, Tyy, Tyz, Tzz, e, n, v_x, v_y, v_z, T of the
 * current state.  A non-physical cell sets the sticky flag. */
rlb_status rlb_box_fields(rlb_box* bx, double* out_device);
rlb_status rlb_box_layout(const rlb_box* bx, int64_t* state_elems, int64_t* ldx);
/* Copy the current state out of / into the workspace (device buffers of
 * state_elems elements); setting a state recomputes its records. */
rlb_status rlb_box_get_state(rlb_box* bx, void* dst_device);
rlb_status rlb_box_set_state(rlb_box* bx, const void* src_device);
/* Time step, elapsed time and evolved points per cell (host values). */
rlb_status rlb_box_info(const rlb_box* bx, double* dt, double* time, int32_t* Q);
/* Synchronizes and reports the sticky non-physical flag. */
rlb_status rlb_box_check(rlb_box* bx);
/* Synchronizes and returns the sticky flag bits (RLB_FLAG_*). */
rlb_status rlb_box_flags(rlb_box* bx, uint32_t* flags);
const char* rlb_box_last_error(const rlb_box* bx);

#ifdef __cplusplus
}
#endif
#endif /* RLB_H */
