/*
 * ib.h - C ABI of the MI355X immersed-boundary acoustic finite-difference library.
 *
 * Method: Caunt, Nelson, Luporini, Gorman, "A Novel Immersed Boundary Approach for
 * Irregular Topography with Acoustic Wave Equations" (arXiv 2309.03600).
 *   - Grid nodes near an irregular surface use modified second-derivative stencils whose
 *     weights come from N-D Taylor extrapolants fitted, in hyperspherical support
 *     regions, to interior data and to boundary conditions imposed at surface points
 *     (sections "Constructing Finite-Difference Approximations", "Imposition of
 *     Boundaries", "Approximating Boundary Conditions", "Reconciliation with the Interior
 *     Numerical Discretization").
 *   - Time stepping is the explicit centred scheme of the second-order acoustic wave
 *     equation (section "Application to the 2nd-Order Acoustic Wave Equation"), with a
 *     damping layer on the outer faces (mentioned in the 2D free-surface example).
 *
 * Conventions
 *   - Axis order (x, [y,] z); z is depth, positive downward.  Every 3D array is stored
 *     [z][y][x], every 2D array [z][x] (x fastest), heightfields [y][x] or [x].
 *   - Lateral axes are periodic; above and below the box the field is zero.
 *   - "device" pointers are HIP device memory on the current device; "host" pointers
 *     are ordinary host memory.  Streams are hipStream_t passed as void* (NULL = the
 *     default stream).  Device buffers passed in are borrowed for the call only and
 *     stay owned by the caller; opaque handles are owned by the library and freed only
 *     by the matching *_free call.
 *   - Every call returns ib_status; IB_OK is 0, errors are negative.  Argument errors
 *     are detected on the host before anything is enqueued; the message is available
 *     from ib_last_error() (thread-local, valid until the next failing call).  Work is
 *     enqueued on the given stream; faults inside kernels surface at the next
 *     synchronising call (ib_build_weights synchronises the stream it is given).
 */
#ifndef IBWAVE_IB_H
#define IBWAVE_IB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IB_ABI_VERSION 4

typedef enum {
  IB_OK = 0,
  IB_ERR_ARG = -1,            /* invalid argument, unsupported combination or size      */
  IB_ERR_HIP = -2,            /* a HIP runtime call failed                             */
  IB_ERR_OOM = -3,            /* device allocation failed                              */
  IB_ERR_UNCONSTRAINED = -4,  /* an IB point stayed rank deficient after the radius
                                 growth and basis-order reduction of the rank rule     */
  IB_ERR_NONFINITE = -5,      /* the watchdog saw a non-finite pressure or one above its
                                 limit (ib_state_set_watchdog)                          */
  IB_ERR_STATE = -6           /* call not valid for this handle / state                */
} ib_status;

typedef enum { IB_FORM_P2 = 0,  /* second-order pressure form                                  */
               IB_FORM_PV1 = 1  /* first-order pressure-velocity form on a staggered grid (free
                                   surface: section "The Particle Velocity Free-Surface"; in 3D
                                   space_order <= 4, the order of the paper's examples) */
} ib_form;
typedef enum { IB_SURF_FREE = 0, IB_SURF_RIGID = 1, IB_SURF_ROBIN = 2 } ib_surface;
typedef enum { IB_METHOD_ND = 0, IB_METHOD_1D = 1 } ib_method;
typedef enum { IB_F32 = 0, IB_F64 = 1 } ib_precision;

/* Regular grid.  n[0] = nx, n[1] = ny (3D) , n[ndim-1] = nz.  h = grid increment in
 * metres, equal on every axis. */
typedef struct {
  int32_t ndim;        /* 2 or 3 */
  int32_t reserved;
  int64_t n[3];
  double h;
} ib_grid;

/* Boundary treatment parameters.
 *   space_order      M, even, 2..8: order of the interior stencil and of the Taylor basis.
 *   surface          IB_SURF_FREE: p = 0, lap p = 0, lap^2 p = 0, ... (section
 *                    "Free-Surface Boundary Constraints");  IB_SURF_RIGID: zero normal
 *                    velocity, i.e. n.grad(lap^q p) = 0 (rigid-surface examples);
 *                    IB_SURF_ROBIN: p + a(x_b) dp/dn = 0 with n the normal pointing out of
 *                    the physical domain and a coefficient that varies along the surface
 *                    (section "Approximating Boundary Conditions" lets the coefficients
 *                    vary with the boundary point), and its members
 *                    lap^q p + a n.grad(lap^q p) = 0 obtained through the wave equation,
 *                    q = 0 .. M_b/2 (a = 0 is the free surface).  Second-order form, N-D
 *                    method.
 *   eta              exclusion cut-off: interior nodes with a boundary point strictly
 *                    inside their node-centred box of half-width eta*h are not used as
 *                    data (section "Approximating Boundary Conditions"; 0.5 in the
 *                    paper's examples).
 *   max_radius_steps support radius starts at (M_b+1)/2 cells and grows by one cell up
 *                    to this many times before the basis order M_b drops by one.
 *   min_basis_order  lowest basis order tried (basis-order reduction).
 *   rank_rtol        numerical-rank tolerance relative to sigma_max; <= 0 selects
 *                    max(rows, cols) * 2^-52.
 *   physical_below   1: the physical domain is below the surface (z > H); 0: above.
 *   eta_v            exclusion cut-off of the velocity nodes (first-order form; the paper
 *                    uses 0: no velocity node is excluded).
 *   method           IB_METHOD_ND: the N-D Taylor extrapolants over hyperspherical supports
 *                    (the paper's method); IB_METHOD_1D: one 1D extrapolation per truncated
 *                    side of each axis stencil, from the free-surface conditions where the
 *                    axis line crosses the surface and the M/2 nearest interior nodes of the
 *                    line farther than eta from it (section "Reduction to 1D"; second-order
 *                    form, free surface).
 *   keep_bc_weights  1: also keep, per IB point, the weights of the boundary-condition
 *                    values (the entries of y on the condition rows: the columns of B A^+
 *                    that multiply g, section "Reconciliation with the Interior Numerical
 *                    Discretization"), needed for non-zero boundary values
 *                    (ib_state_set_forcing).  Second-order form, N-D method only.  0: drop
 *                    them (homogeneous conditions; the paper's examples).
 *   robin_dev        IB_SURF_ROBIN only: device float64 samples of a (metres, >= 0 for an
 *                    energy-stable condition) at the node columns, laid out like the
 *                    heightfield; a(x_b) is their periodic bilinear (2D: linear)
 *                    interpolation at the boundary point's lateral position.  Borrowed for
 *                    the call.  NULL for the other surfaces.
 */
typedef struct {
  int32_t form;
  int32_t surface;
  int32_t space_order;
  int32_t max_radius_steps;
  int32_t min_basis_order;
  int32_t physical_below;
  double eta;
  double rank_rtol;
  double eta_v;
  int32_t method;
  int32_t keep_bc_weights;
  const double *robin_dev;
} ib_params;

typedef struct {
  int64_t n_nodes;           /* grid nodes                                              */
  int64_t n_interior;        /* interior (physical-side) nodes                          */
  int64_t n_boundary_points; /* hosted boundary points                                  */
  int64_t n_ib;              /* IB points (interior nodes whose axis stencils reach an
                                exterior node)                                          */
  int64_t sum_nw;            /* total extrapolation weights                             */
  int64_t max_nw;
  int64_t radius_hist[8];    /* IB points per radius step k (0..7)                      */
  int64_t order_hist[17];    /* IB points per final basis order                         */
  double max_cond;           /* largest estimated sigma_max/sigma_min over accepted points */
  double min_margin;         /* smallest (sigma_min/sigma_max)/tolerance over accepted    */
  int64_t table_bytes_f32;   /* bytes of the FP32 stencil records (masks + weights)      */
  int64_t table_bytes_f64;
  int64_t max_ball;          /* largest support ball (lattice points) used               */
  double build_ms;           /* wall time of ib_build_weights                            */
  int64_t dense_weights;     /* entries of the dense-range records (>= sum_nw; zeros fill
                                non-data lattice points between a support's first and
                                last data point)                                        */
  int64_t col_weights;       /* entries of the column-run records streamed by the 3D tiled
                                patch kernel (the data nodes' weights of the supports of
                                radius <= 4.5, plus zeros at the rare non-data node inside
                                a column's run)                                         */
} ib_stats;

typedef struct ib_weights ib_weights;
typedef struct ib_state ib_state;
typedef struct ib_checkpoints ib_checkpoints;   /* time checkpoints of one forward run */

int32_t ib_abi_version(void);
const char *ib_last_error(void);

/* Build the immersed-boundary stencils for one topography.
 *   height_dev: device, float64 [ny][nx] (3D) or [nx] (2D), surface depth in metres at
 *     each node column; the surface between columns is the periodic Catmull-Rom cubic
 *     through these samples and the nodes' signed distance is measured to it (the
 *     paper's discretised signed-distance function).  Borrowed.
 *   Produces (on the device): node classes, boundary points (closest surface point of
 *   each node whose one-cell box contains it), the eta-exclusion mask, the IB-point
 *   list and, per IB point, the FP64 least-squares extrapolation weights
 *   y = (A^+)^T c with A the Taylor/boundary-condition rows and c the exterior part of
 *   the interior Laplacian stencil, plus an FP32 copy.  Synchronises ``stream``.
 * Errors: IB_ERR_ARG (shape, order, surface too close to the top/bottom of the box),
 *   IB_ERR_UNCONSTRAINED, IB_ERR_OOM, IB_ERR_HIP. */
ib_status ib_build_weights(const ib_grid *grid, const double *height_dev, const ib_params *params,
                           void *stream, ib_weights **out);
ib_status ib_weights_stats(const ib_weights *w, ib_stats *out);
void ib_weights_free(ib_weights *w);

/* Copy one array of a built table to host memory (for inspection and tests).
 *   IB_FIELD_NODE_CLASS  uint8 [n_nodes], memory order: bit0 interior, bit1 excluded
 *                        by eta, bit2 IB point, bit3 hosts a boundary point.
 *   IB_FIELD_BPOINTS     float64 [n_boundary_points][7]: host node (x,y,z) as doubles,
 *                        boundary point (x,y,z) in grid units (2D: y = 0), the mixed
 *                        surface's coefficient a(x_b) in metres (0 for the others).
 *   IB_FIELD_IB_NODES    int64 [n_ib]: memory-order node index of each IB point.
 *   IB_FIELD_IB_META     int32 [n_ib][4]: radius step k, basis order M_b, weight count,
 *                        first weight index.
 *   IB_FIELD_WEIGHTS_F64 float64 [sum_nw]: weights of each point in the lattice order
 *                        of its support ball (z, then y, then x), data nodes only.
 *   IB_FIELD_SIGMA       float64 [n_ib]: estimated sigma_min/sigma_max of accepted A.
 * Built with keep_bc_weights = 1 only:
 *   IB_FIELD_BC_COUNTS   int32 [n_ib]: condition-value weights of each IB point.
 *   IB_FIELD_BC_ENTRIES  float64 [sum][3]: boundary point (index into IB_FIELD_BPOINTS),
 *                        condition q of the hierarchy, weight (grid units: the value of
 *                        a condition of derivative order o enters as h^o g); IB points in
 *                        order, each point's entries by boundary point, then q.
 * First-order form only:
 *   IB_FIELD_PV_ROWS     int64 [n_rows][3]: family (n < ndim: d/dx_n p at a v_n node,
 *                        ndim: div v at a p node), memory-order node, number of weights.
 *   IB_FIELD_PV_ENTRIES  float64 [sum][3]: data field (-1 p, n: v_n along the n-th
 *                        velocity axis), memory-order node, weight; rows in order.
 *   IB_FIELD_VCLASS      uint8 [ndim][n_nodes]: classes of the v_n nodes (bit0 interior,
 *                        bit1 excluded).
 * dst_bytes must be at least the field size. */
typedef enum {
  IB_FIELD_NODE_CLASS = 0, IB_FIELD_BPOINTS = 1, IB_FIELD_IB_NODES = 2,
  IB_FIELD_IB_META = 3, IB_FIELD_WEIGHTS_F64 = 4, IB_FIELD_SIGMA = 5,
  IB_FIELD_PV_ROWS = 6, IB_FIELD_PV_ENTRIES = 7, IB_FIELD_VCLASS = 8,
  IB_FIELD_BC_COUNTS = 9, IB_FIELD_BC_ENTRIES = 10
} ib_field;
ib_status ib_weights_copy(const ib_weights *w, int32_t field, void *dst_host, int64_t dst_bytes);

/* Create a time-stepping state for ``nshots`` simultaneous shots over one topography.
 *   vel_dev:  device float64 [nz][ny][nx] (or [nz][nx]) velocity in m/s.  Borrowed.
 *   dt:       time step (s).  The caller chooses it (e.g. half the interior limit).
 *   damp_width, damp_R: damping layer of ``damp_width`` cells on the lateral faces and
 *             the bottom, d = d_max (l/W)^2 with l the depth into the layer in cells,
 *             d_max = 3 c_max ln(1/R) / (W h) in the second-order form (damping term
 *             d p_t) and half of it in the first-order form (d on each field), so that a
 *             wave crossing the layer and back keeps the amplitude fraction R (WKB);
 *             0 disables it.
 *   prec:     IB_F32 or IB_F64 wavefields (weights rounded from the FP64 master).
 *   src_pos_host: host float64 [nshots][ndim], one point source per shot (metres),
 *             spread multilinearly over the 2^d surrounding nodes, amplitude
 *             dt^2 * wavelet / h^d (the paper's f~ = f dt^2).
 *   rec_pos_host: host float64 [nrec][ndim] receivers (metres), sampled multilinearly;
 *             shared by all shots.
 * First-order form (weights built with IB_FORM_PV1): the state holds p and the staggered
 *   velocities v_n (rho = 1); the source amplitude is dt * wavelet / h^d; ndim times the padded
 *   grid (x rounded up to 32) must stay below 2^32 nodes.
 * Wavefields start at zero; the step counter at 0.
 * Errors: IB_ERR_ARG (positions outside the box or touching exterior nodes, nshots < 1),
 *   IB_ERR_OOM, IB_ERR_HIP. */
ib_status ib_state_create(const ib_weights *w, const double *vel_dev, double dt, int32_t damp_width,
                          double damp_R, int32_t prec, int32_t nshots, const double *src_pos_host,
                          int32_t nrec, const double *rec_pos_host, void *stream, ib_state **out);
void ib_state_free(ib_state *st);

/* Advance every shot by ``nsteps`` leapfrog steps:
 *   p^{n+1} = [2 p^n - (1 - s) p^{n-1} + K (L p^n) + dt^2 f^n] / (1 + s),
 *   which FP32 states evaluate in increment form: with d^n = p^n - p^{n-1} kept in place
 *   of p^{n-1}, d^{n+1} = [(1 - s) d^n + K (L p^n) + dt^2 f^n] / (1 + s) and
 *   p^{n+1} = p^n + d^{n+1} (the same recurrence; single-precision rounding of p^{n+1} then
 *   does not build up as an error of the time difference).  FP64 states keep p^{n-1}.
 *   K = (c dt / h)^2 at interior nodes (0 elsewhere), s = d dt / 2, L the grid-unit
 *   Laplacian with the immersed-boundary rows.
 *   wavelet_dev: device [nshots][wavelet_stride] in the state precision; step n uses
 *     sample t of the state's step counter (t = 0, 1, ...).  Must cover t + nsteps.
 *   traces_dev:  device [nshots][nsteps][nrec] in the state precision; receives
 *     p^{n+1} sampled at the receivers after each step.  May be NULL when nrec = 0.
 * First-order form: each step is
 *   v_n^{n+1/2} = [(1 - s) v_n^{n-1/2} + (dt / h) D+_n p^n] / (1 + s)       (interior v_n nodes)
 *   p^{n+1}     = [(1 - s) p^n + (dt c^2 / h) D-.v^{n+1/2} + dt f^n] / (1 + s)  (interior p nodes)
 *   with the staggered M-th order differences and the immersed-boundary rows of both
 *   families; the traces sample p^{n+1}.
 * When use_graph is non-zero the per-step kernels are captured into HIP graphs of two and
 * of sixteen steps (even/odd buffers), replayed as the call's length allows (the rest is
 * launched eagerly); results are identical to eager launch.
 * The watchdog (ib_state_set_watchdog) scans p^n after every ``every`` steps on the
 * stream; a scan that finds a bad value makes the next call on the state (this one's
 * successor, or ib_state_status) return IB_ERR_NONFINITE.
 * Errors: IB_ERR_ARG, IB_ERR_NONFINITE (a scan of an earlier call tripped; nothing is
 *   enqueued), IB_ERR_HIP. */
ib_status ib_step(ib_state *st, int32_t nsteps, const void *wavelet_dev, int64_t wavelet_stride,
                  void *traces_dev, int32_t use_graph, void *stream);

/* Forward modelling with time checkpoints, for a later ib_adjoint.  Restarts every shot
 * from rest (step counter 0), runs ``nt`` steps exactly as ib_step (eager launches), and
 * keeps (p^n, p^{n-1}) at every multiple of ``ckpt_every`` inside the state (device
 * memory, 2 * nshots * grid * ceil(nt / ckpt_every) values; the increment form keeps d^n
 * in place of p^{n-1}).  The watchdog runs as in ib_step.
 *   traces_dev: device [nshots][nt][nrec] in the state precision (may be NULL if nrec = 0). */
ib_status ib_forward(ib_state *st, int32_t nt, const void *wavelet_dev, int64_t wavelet_stride, void *traces_dev,
                     int32_t ckpt_every, void *stream);

/* ib_forward into a checkpoint handle held by the caller, so that the checkpoints of
 * several forward runs (other wavelets or receivers' residuals later) can live side by
 * side and outlive the next ib_forward.
 *   ckpt: in/out.  *ckpt == NULL: a new handle is created and stored there.  Otherwise an
 *     earlier handle is reused (reallocated only if its size differs) and taken over by
 *     this state.  Free it with ib_checkpoints_free (after the stream is done with it).
 * Errors: as ib_forward; on error a handle created by the call is freed and *ckpt is left
 *   unchanged. */
ib_status ib_forward_ckpt(ib_state *st, int32_t nt, const void *wavelet_dev, int64_t wavelet_stride,
                          void *traces_dev, int32_t ckpt_every, ib_checkpoints **ckpt, void *stream);
void ib_checkpoints_free(ib_checkpoints *ckpt);

/* Gradient of a misfit J with respect to the velocity, by the discrete adjoint of the
 * stepper (not a result of the paper: full-waveform inversion is its motivation).
 *   residual_dev: device [nshots][nt][nrec] (state precision) = dJ/d traces of the last
 *     ib_forward (for J = 1/2 sum (d - d_obs)^2 it is d - d_obs).
 *   grad_dev: device float64 [nz][ny][nx], overwritten with dJ/dc summed over shots (zero
 *     at exterior nodes).  The damping profile is held fixed.
 * Each checkpoint segment is recomputed forward and kept (ckpt_every fields) while the
 * adjoint steps back through it; the adjoint of the IB rows uses a transposed stencil
 * table (per receiving node) built on the first call.
 * Errors: IB_ERR_STATE without a previous ib_forward or with boundary values set
 *   (ib_state_set_forcing); IB_ERR_ARG for the first-order form
 *   (ib_forward and ib_adjoint cover the second-order form only). */
ib_status ib_adjoint(ib_state *st, const void *residual_dev, const void *wavelet_dev, int64_t wavelet_stride,
                     double *grad_dev, void *stream);

/* ib_adjoint from the checkpoints of an ib_forward_ckpt call by the same state (same
 * arguments otherwise: residual_dev is dJ/d traces of that forward run).
 * Errors: as ib_adjoint; IB_ERR_STATE for checkpoints written by another state. */
ib_status ib_adjoint_ckpt(ib_state *st, const ib_checkpoints *ckpt, const void *residual_dev,
                          const void *wavelet_dev, int64_t wavelet_stride, double *grad_dev, void *stream);

/* ib_adjoint without any device allocation, for callers that cannot allocate (code under
 * stream capture, serving loops, hosts that forbid hipMalloc).  Same arguments, same result
 * as ib_adjoint.  Its work space is a fixed 64 MiB device array per device (held until the
 * process ends) instead of a fresh allocation: the two lambda fields (three in the
 * increment form), the recomputed segment (ckpt_every + 2 fields of nshots * grid values)
 * and an FP64 grid must fit, else IB_ERR_ARG (ib_adjoint has no such limit).  The adjoint
 * tables are built by ib_forward, so no host-device copy is made either.  The work is
 * enqueued on ``stream`` and the call returns without waiting: grad_dev is ready when
 * the stream is.  Every call on one device shares that array (each call clears what it
 * needs), so calls that overlap on one device, from any state or stream, race.
 * Errors: as ib_adjoint, plus IB_ERR_ARG when the work space does not fit. */
ib_status ib_adjoint_noalloc(ib_state *st, const void *residual_dev, const void *wavelet_dev,
                             int64_t wavelet_stride, double *grad_dev, void *stream);

/* Read or write the current wavefields of one shot (layout [nz][ny][nx] or [nz][nx],
 * state precision, device memory):  which = 0: p^n (newest), 1: p^{n-1}.
 * First-order form: which = 0: p^n, 2 + k: v_k^{n-1/2} (k < ndim; in 2D k = 1 is the
 * vertical velocity), 1 is invalid.
 * direction 0 copies out of the state, 1 copies into it.  Values written at exterior
 * nodes (velocity fields: exterior v_k nodes) are replaced by zero: the method takes the
 * wavefield as zero outside the physical domain.
 * FP32 states of the second-order form keep d^n = p^n - p^{n-1} (increment form, see
 * ib_step) instead of p^{n-1}: reading which = 1 returns p^n - d^n, writing it sets
 * d^n = p^n - (the given p^{n-1}) from the current p^n, so write p^n first. */
ib_status ib_state_field(ib_state *st, int32_t which, int32_t shot, void *dev_buf, int32_t direction,
                         void *stream);
int64_t ib_state_step_count(const ib_state *st);

/* Non-zero boundary values (inhomogeneous conditions; section "Approximating Boundary
 * Conditions" lets each condition equal a value g(x_b), and section "Reconciliation with
 * the Interior Numerical Discretization" keeps the columns of B A^+ that multiply it).
 * Second-order form, weights built with keep_bc_weights = 1.
 *   The conditions of the surface get right-hand sides, condition q of the hierarchy
 *     free:  lap^q p (x_b) = g_q(x_b) s_q(t),   rigid:  n.grad(lap^q p)(x_b) = g_q(x_b) s_q(t),
 *     robin: lap^q p + a n.grad(lap^q p) = g_q(x_b) s_q(t),
 *   so step n adds K (sum_q s_q(t_n) sum_b v_ibq h^{o_q} g_q(x_b)) / (1 + s) at each IB
 *   point i (o_q = 2q free and robin, 2q + 1 rigid; v the condition-value weights).
 *   g_dev:   device float64 [n_boundary_points][nq] (IB_FIELD_BPOINTS order), physical
 *            units (Pa / m^{o_q}).  Borrowed: contracted with the weights during the call.
 *   s_host:  host float64 [nq][s_len]: step t uses s_q[t] (t = the state's step counter);
 *            copied into the state.
 *   nq:      1 .. conditions at full order (M/2 + 1 free and robin, (M - 1)/2 + 1 rigid); conditions
 *            beyond nq stay homogeneous.
 *   g_dev = NULL clears the forcing.  The same values drive every shot.  ib_step then
 *   needs s_len >= step counter + nsteps; ib_forward and ib_adjoint refuse a forced state
 *   (the boundary values are not differentiated).
 * Errors: IB_ERR_ARG (nq, s_len, null s_host), IB_ERR_STATE (first-order form, weights
 *   without condition-value weights), IB_ERR_OOM, IB_ERR_HIP. */
ib_status ib_state_set_forcing(ib_state *st, const double *g_dev, int32_t nq, const double *s_host, int64_t s_len,
                               void *stream);

/* Watchdog against instability (the paper introduces the support parameter eta to keep
 * the scheme stable, section "Approximating Boundary Conditions"; a growing mode shows as
 * values that blow up).  After every ``every`` steps of ib_step and ib_forward a kernel
 * scans p^n of every shot; a value that is NaN, infinite or above ``limit`` in magnitude
 * trips it.  Its flags come back to the host behind the scan without a wait; the next
 * call on the state sees them and returns IB_ERR_NONFINITE, as does every call that
 * steps or differentiates the state after it, until this function is called again.
 * Defaults: every = 100, limit = 1e30 (FP32 states cap it at the largest float).
 *   every: steps between scans, 0 turns the scans off; odd values are rounded up so that
 *     the scans fall between graph launches.
 *   limit > 0.
 * Waits for a scan still in flight, then clears the flags (on ``stream``).
 * Errors: IB_ERR_ARG. */
ib_status ib_state_set_watchdog(ib_state *st, int32_t every, double limit, void *stream);

/* IB_OK, or IB_ERR_NONFINITE if a watchdog scan has tripped.  wait != 0 waits for the
 * last scan enqueued; wait = 0 reads only what has come back. */
ib_status ib_state_status(ib_state *st, int32_t wait);

/* Measurement aid: enqueue ``count`` launches of one kernel of the step on ``stream``
 * with the current buffers (which = 0: interior stencil, 1: IB patch), rotating the
 * buffers as a step would, without sources, receivers or the step counter.  Used to
 * time each kernel on its own; it changes the wavefields.  Second-order form only. */
ib_status ib_state_run_kernel(ib_state *st, int32_t which, int32_t count, void *stream);

/* Tuning knobs of the 3D eighth-order step kernels.
 *   variant (interior stencil): 0 (one plane per barrier pair), 1 (software-pipelined,
 *     64x16 tiles), 2 (pipelined, 64x32 tiles, 8 rows per thread), 3 (pipelined, 64x32
 *     tiles, 512 threads), 4 (pipelined, 64x16 tiles, 512 threads, 2 rows per thread);
 *   zchunk: depth planes per interior workgroup (0 = automatic: enough workgroups to fill
 *     the device);
 *   patch_variant (tiled IB patch): 0-3 dense-range records, point records read per
 *     wavefront (bit 0 as scalar loads, bit 1 DPP wavefront sums); 4-6 dense-range records,
 *     point records staged in LDS per tile, 1-3 groups of two points' weights in flight;
 *     7 compact records (bit masks and the data nodes' weights only); 8 column-run records
 *     (the data nodes' weights, one ball column per lane; the default), 9 the same with two
 *     FP32 shots per pass (the default for FP32 states of several shots); -1 keeps the
 *     current one.
 * Results do not depend on the interior knobs; the patch variants differ only in the
 * summation order of each point's weighted sum. */
ib_status ib_state_set_tuning(ib_state *st, int32_t variant, int32_t zchunk, int32_t patch_variant);

#ifdef __cplusplus
}
#endif
#endif
