/*
 * fslbm.h -- C interface of the MI355X free-surface lattice Boltzmann library.
 *
 * One time step (Bogner, Ammer, Ruede, "Boundary Conditions for Free Interfaces
 * with the Lattice Boltzmann Method"):
 *   - D3Q19 two-relaxation-time stream/collide, Eq. (lbe1), (lbe2), with the
 *     equilibria Eq. (eqEven), (eqOdd) and the body force through
 *     u_eq = U - F/lambda_- (section 2.1);
 *   - halfway bounce-back at every non-periodic domain face (section 4.3),
 *     with the momentum of moving faces (section 4.1), and solid cells with
 *     the linear-interpolation wall closure at any wall distance (section 4.2,
 *     fslbm_set_walls);
 *   - reconstruction of every population that streams in from a gas cell by the
 *     general linear closure Eq. (closure) with the FSK row of Table 1 (the rule
 *     of Eq. (koerner)) or the FSL row (Eq. (fsli1)-(fsli4), alpha_+ = 1), with
 *     S^b = 0 or with the boundary shear term D of Eq. (bterm) taken from the
 *     bulk or prescribed (sections 3.3, 3.4; the rule argument of fslbm_step);
 *     optionally the Laplace pressure P_b - sigma kappa (Eq. freeboundary) and
 *     the PLIC interface position for the FSL link distance (section 5);
 *   - mass exchange, fill-level update and interface <-> liquid / gas cell
 *     conversion with excess-mass redistribution (the interface tracking of the
 *     free-surface LBM that section 2.3 describes and section 4.4 cites);
 *   - the adjoint of windows of such steps with frozen cell classes.
 *
 * Memory: every device buffer is allocated by the caller (e.g. as torch
 * tensors) and borrowed by the library until fslbm_destroy; the library never
 * frees caller memory.  The library owns only its host-side context.
 *
 * Streams: fslbm_step enqueues work on the stream given at init and returns
 * without synchronising.  Functions documented as "synchronises" wait for that
 * stream.
 *
 * Errors: every entry point returns a status; no C++ exception crosses this
 * interface.  fslbm_last_error gives a message for the last failure on a
 * context.  HIP runtime failures map to FSLBM_E_DEVICE.
 *
 * Layout: a cell (x, y, z) has linear index idx = x + nx*(y + ny*z); population
 * q of cell idx is element q*N + idx of a population buffer (N = nx*ny*nz).
 * The population order is: q = 0 rest; 1..6 the axis links (+x, -x, +y, -y,
 * +z, -z); 7..18 the diagonals (+x+y, -x-y, +x-y, -x+y, +x+z, -x-z, +x-z,
 * -x+z, +y+z, -y-z, +y-z, -y+z); odd q has its opposite at q + 1.
 */
#ifndef FSLBM_H
#define FSLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FSLBM_ABI_VERSION 5

typedef struct fslbm_ctx fslbm_ctx;

typedef enum {
  FSLBM_OK = 0,
  FSLBM_E_INVALID = 1,      /* bad argument, size or cell-class pattern */
  FSLBM_E_UNSUPPORTED = 2,  /* valid but not supported (e.g. FSL at tau = 1) */
  FSLBM_E_DEVICE = 3,       /* HIP runtime error */
  FSLBM_E_UNSTABLE = 4,     /* a health check found a NaN, a non-positive density or |u| > u_max */
  FSLBM_E_INVARIANT = 5,    /* a health check found a liquid cell next to a gas cell or an
                                unknown cell class */
  FSLBM_E_CAPACITY = 6      /* an output array, or the static workspace, is too small */
} fslbm_status;

/* Gas-side reconstruction rule (Table 1).  FSK and FSL use the boundary value
 * term of Eq. (bterm) with S^b = 0 (D = 0).  The _STRESS variants add its
 * shear-rate part D c_a c_b S^b_ab with D = -alpha_+ Lambda_+ w_q / c_s^2
 * (Table 1, column D; section 3.4): S is taken from the non-equilibrium of the
 * liquid neighbour opposite the surface normal, and S^b keeps its tangential
 * block, has zero tangential-normal entries (Eq. proj2) and normal entry
 * S_nn / 3 (Eq. proj1 with sigma = 0). */
enum {
  FSLBM_RULE_FSK = 0,
  FSLBM_RULE_FSL = 1,
  FSLBM_RULE_FSK_STRESS = 2,
  FSLBM_RULE_FSL_STRESS = 3,
  /* the same D term with S^b given in fslbm_params.shear_b (section 4.2) */
  FSLBM_RULE_FSK_SHEAR = 4,
  FSLBM_RULE_FSL_SHEAR = 5
};

/* Precision forms.  FP64: populations f stored and computed in double.
 * FP32: shifted populations f - w_q stored and computed in float.
 * FP16S: shifted populations scaled by 2^fp16_scale_log2 stored as IEEE
 * binary16 (round to nearest even), computed in float.  Mass, fill level and
 * excess-mass redistribution are double in every form. */
enum { FSLBM_FP64 = 0, FSLBM_FP32 = 1, FSLBM_FP16S = 2 };

/* Cell classes stored in the flags array. */
enum { FSLBM_GAS = 0, FSLBM_INTERFACE = 1, FSLBM_LIQUID = 2 };

typedef struct {
  int32_t abi_version;      /* FSLBM_ABI_VERSION */
  int32_t nx, ny, nz;       /* lattice size, each >= 1, 19*nx*ny*nz < 2^32 */
  int32_t periodic[3];      /* nonzero: periodic axis; zero: bounce-back walls */
  int32_t precision;        /* FSLBM_FP64, FSLBM_FP32 or FSLBM_FP16S */
  double tau;               /* symmetric relaxation time, lambda_+ = -1/tau; > 1/2 */
  double magic;             /* Lambda = Lambda_+ Lambda_- (section 3.1); > 0 */
  int32_t incompressible;   /* nonzero: rho_0 = 1; zero: rho_0 = rho (section 2.1) */
  int32_t stokes;           /* nonzero: drop the quadratic term N_q of e+ */
  double g[3];              /* body acceleration (force F = rho_0 g) */
  double rho_gas;           /* gas density rho_b, pressure P_b = rho_b / 3 */
  double conv_eps;          /* conversion margin: filled m > (1+eps) rho, emptied m < -eps rho */
  int32_t fp16_scale_log2;  /* FP16S scale exponent k (storage 2^k (f - w)); 0..24 */
  int32_t freeze;           /* nonzero: frozen flag topology, no conversions */
  double wall_u[6][3];      /* velocity of each wall face, in the order x-, x+, y-, y+, z-, z+
                               (ignored on periodic axes).  Halfway bounce-back off a moving
                               wall adds 2 w_q (c_q . u_w) / c_s^2 (rho_w = 1); a link leaving
                               through an edge takes the first crossed face in x, y, z order */
  double shear_b[6];        /* prescribed boundary shear rate S^b = [xx, yy, zz, xy, xz, yz]
                               of the FSLBM_RULE_*_SHEAR rules (section 4.2) */
  double sigma;             /* surface tension coefficient (>= 0).  The boundary term takes the
                               gas pressure P_b - sigma kappa (Eq. freeboundary) with kappa =
                               -div n from the fill field's gradient and Hessian by central
                               differences over the D3Q19 neighbourhood; not supported by the
                               adjoint window */
  int32_t plic;             /* 0, 1 or 2.  1: the FSL rules (FSL, FSL_STRESS, FSL_SHEAR) take the
                               link distance delta = d / (c_q . n) from the plane n.(x - x_node)
                               = d that cuts the cell's fill fraction phi (PLIC, the second-order
                               interface position asked for in section 5) instead of d = phi -
                               1/2.  2: the same with the normal from height functions (3 x 3
                               columns of 7 cells along the dominant axis, exact for planes of
                               slope <= 1) where every column is complete, else the central-
                               difference normal; with sigma != 0 the Laplace pressure then also
                               takes the height-function curvature of the same columns (any
                               rule), where they are not complete the mean of those of the
                               D3Q19 interface neighbours that have one, else the central-
                               difference one (the workspace then holds 8 N more bytes).  Not
                               supported by the adjoint window */
  int32_t check_every;      /* health check every K steps of fslbm_step (0: none; the
                               environment variable FSLBM_CHECK_EVERY overrides it): after every
                               K-th step the library checks every fluid cell and synchronises
                               (see fslbm_step) */
  double u_max;             /* |u| bound of the health check (lattice units, >= 0; 0 selects 0.4,
                               below the lattice speed of sound 1/sqrt 3) */
  int32_t hold_fill;        /* nonzero: the fill levels and interface masses keep
                               their values, so the surface stays where the caller put it (an
                               interface position known exactly, as for the steady films of
                               section 4.3); the cell classes are frozen as with freeze; the
                               populations evolve as usual */
} fslbm_params;

typedef struct {
  void* f[2];               /* 2 buffers of 19*N elements of the storage type
                               (double, float or binary16) */
  uint8_t* flags;           /* N cell classes; filled by the caller before init */
  double* mass;             /* N interface mass values */
  double* phi[2];           /* 2 buffers of N fill levels */
  void* workspace;          /* fslbm_workspace_size bytes, 256-byte aligned */
  size_t workspace_bytes;
  void* stream;             /* hipStream_t, or NULL for the null stream */
} fslbm_buffers;

/* Bytes of workspace a context from fslbm_init with these parameters needs
 * (in the FP32 and FP64 forms including a cell -> list-entry map and a
 * list-ordered population buffer of N/8 entries, at least 32768, for the
 * interface-first step of fslbm_step). */
fslbm_status fslbm_workspace_size(const fslbm_params* p, size_t* bytes);

/* Validate parameters and buffers, check the cell classes on the device (every
 * class in {GAS, INTERFACE, LIQUID}; no liquid cell has a gas cell among its 18
 * neighbours, walls excluded) and create a context.  Rejects: dims < 1, too
 * many cells, tau <= 1/2, magic <= 0, an unknown precision, NULL buffers, a
 * short workspace.  Synchronises.  Populations are undefined until
 * fslbm_set_equilibrium or fslbm_set_state. */
fslbm_status fslbm_init(const fslbm_params* p, const fslbm_buffers* b, fslbm_ctx** out);

/* Size of the library's static workspace of fslbm_init_static (64 MiB per
 * device: about 880,000 cells without surface tension; a static context needs
 * less than fslbm_workspace_size, as it always runs the interface kernel after
 * the sweep). */
#define FSLBM_STATIC_WORKSPACE_BYTES (64u << 20)

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): the same as
 * fslbm_init, but b->workspace and b->workspace_bytes are ignored -- the
 * context's workspace is an array of FSLBM_STATIC_WORKSPACE_BYTES inside the
 * library on the current device, which each device that uses it holds until
 * the process ends.  No device memory is allocated, by this call or by the
 * calls on the context.  The caller still passes every other buffer.
 * FSLBM_E_CAPACITY if its workspace exceeds the array.  One context
 * per device may hold the array at a time: while one exists, a second call
 * on the same device is FSLBM_E_INVALID (contexts sharing it would race);
 * fslbm_destroy releases it.  The array keeps the contents of the previous
 * context; everything a step needs cleared is cleared here, as by
 * fslbm_init.  Synchronises. */
fslbm_status fslbm_init_static(const fslbm_params* p, const fslbm_buffers* b, fslbm_ctx** out);

/* Initial state from macroscopic fields (device pointers, double): rho[N],
 * u[3*N] (u[a*N + idx]) and fill[N].  Every non-gas cell gets the
 * post-collision state of a resting-frame equilibrium, e+(rho,u) +
 * e-(rho_0, u + g/2); interface cells get m = fill * rho.  Synchronises. */
fslbm_status fslbm_set_equilibrium(fslbm_ctx* c, const double* rho, const double* u, const double* fill);

/* Initial state given directly (device pointers, double): post-collision
 * populations f[19*N] (unshifted), mass[N] and fill[N] (read at interface
 * cells), and the reservoir value.  Synchronises. */
fslbm_status fslbm_set_state(fslbm_ctx* c, const double* f, const double* mass, const double* fill,
                             double reservoir);

/* Enqueue n time steps with one of the FSLBM_RULE_* rules.  Every rule but
 * FSK with tau = 1 is FSLBM_E_UNSUPPORTED (n+ cannot be recovered from the
 * post-collision state).  Asynchronous, except with a health check
 * (params.check_every = K > 0): after every step whose count of steps done
 * is a multiple of K the health check of fslbm_stats runs and the call waits
 * for it; on failure it returns FSLBM_E_UNSTABLE or FSLBM_E_INVARIANT (the
 * message names the count of bad cells and the step) and enqueues no further
 * step of this call.  A context from fslbm_init also bounds how far the host
 * may run ahead: the sweep launches only the rows within the fluid's extent,
 * measured on the device every 16 steps and read back without a wait, and
 * when the extent in use is 32 steps old the call waits for the next one
 * (so the device has at most 32 steps queued).  The environment variable
 * FSLBM_EXTENT_EVERY at init sets the 16 (0: every row, never a wait).  In
 * the FP32 form the plain step (no moving wall, surface tension, PLIC, solid
 * cells or prescribed surface) runs the interface kernel before the sweep,
 * which stores the interface populations with its whole rows; the results
 * are the same bits as with the interface kernel after the sweep.  The
 * environment variable FSLBM_REORDER at init (0 / 1) selects either order for
 * the FP32 and FP64 forms; FP16 storage always runs the interface kernel
 * after the sweep.  The classes change
 * only through the steps: a caller that writes the flags buffer between steps
 * calls fslbm_set_state or fslbm_set_equilibrium afterwards, which also make
 * the next step measure the extent again and rebuild the interface list.
 * Steps are not for HIP graph capture: each call passes host-side state into
 * its launches (which population buffer is current, the step count that
 * stamps the conversion marks, and for a context from fslbm_init the row box
 * and the interface list), so a captured step would replay stale arguments. */
fslbm_status fslbm_step(fslbm_ctx* c, int32_t n, int32_t rule);

/* Field export into caller device buffers.  mask selects fields by bit; dst[i]
 * is the destination of bit i (unused entries may be NULL):
 *   bit 0 rho     double[N]   density from the current populations (gas: 0)
 *   bit 1 u       double[3N]  velocity u = U + g/2 of time t (gas: 0)
 *   bit 2 phi     double[N]   fill level: liquid 1, gas 0, interface m/rho
 *   bit 3 flags   uint8[N]    cell classes
 *   bit 4 f       double[19N] post-collision populations, unshifted
 *   bit 5 mass    double[N]   interface mass (meaningful at interface cells)
 *   bit 6 rho_c   double[N]   density of the last collision (interface cells)
 *   bit 7 u_c     double[3N]  velocity of the last collision (interface cells)
 * Synchronises. */
fslbm_status fslbm_fields(fslbm_ctx* c, uint32_t mask, void* const* dst);

/* Diagnostics (host outputs).  total_mass = sum over liquid cells of sum_q f +
 * sum over interface cells of m + reservoir (double).  counts: [0] filled,
 * [1] emptied, [2] emptied and converted, [3] new interface from gas, [4] new
 * interface from liquid (all of the last step), [5] interface cells now,
 * [6] liquid cells now, [7] steps done.  Health check of the current state
 * (the interface tracking keeps a layer of interface cells between liquid and
 * gas, section 2.3): FSLBM_E_INVARIANT if a cell class is unknown or a liquid
 * cell has a gas cell among its 18 neighbours; else FSLBM_E_UNSTABLE if a
 * liquid or interface cell has a NaN or non-positive density or a velocity
 * |u| above params.u_max (all outputs are still written).  Synchronises. */
fslbm_status fslbm_stats(fslbm_ctx* c, double* total_mass, double* reservoir, int64_t counts[8]);

/* Conversion lists of the last step into host arrays, ascending cell index:
 * out[0] filled, out[1] emptied, out[2] emptied and converted, out[3] new
 * interface from gas, out[4] new interface from liquid.  n_out[i] receives each
 * length; FSLBM_E_CAPACITY if a length exceeds cap (the first cap entries are
 * still written).  Synchronises. */
fslbm_status fslbm_conversions(fslbm_ctx* c, int32_t* const* out, int32_t cap, int32_t n_out[5]);

/* Kernel timing of the stream/collide sweep (the kernel that moves the
 * populations).  enable = 1 clears the record and starts bracketing every
 * sweep launch of fslbm_step with a pair of HIP events on the context's
 * stream; enable = 0 stops recording.  In both cases, when sweep_ms / sweeps
 * are non-NULL, they receive the summed event-to-event time (milliseconds) and
 * the number of sweeps recorded so far (synchronises). */
fslbm_status fslbm_timing(fslbm_ctx* c, int32_t enable, double* sweep_ms, int64_t* sweeps);

/* Set the body acceleration g and the gas density rho_b (P_b = rho_b / 3) used
 * by the steps enqueued from now on (the parameters of the boundary term of
 * Eq. (bterm) and of the force of section 2.1).  Host arguments; no device
 * work. */
fslbm_status fslbm_set_forcing(fslbm_ctx* c, const double g[3], double rho_gas);

/* Solid walls at arbitrary distances from the nodes (the rotated channels of
 * section 4.2).  Cells of class 3 in the flags are solid: they hold no fluid,
 * never convert, and are walls to their fluid neighbours (no mass exchange,
 * the cell's own fill in the interface geometry).  A population pulled from a
 * solid cell takes the linear-interpolation closure for the link p towards
 * the wall point x + delta c_p: the closure of Eq. (closure) whose
 * coefficients satisfy the fitting conditions of Eq. (fitting, cl1) with no
 * pressure term and the wall momentum to first order (C = 0, a0 = 1):
 *   f_q(x,t+1) = ft_p(x) + kappa (ft_p(x - c_p) - ft_q(x))
 *                + 2/(1 + 2 delta) * 2 w_q (c_q . u_w) / c_s^2,
 * kappa = (1 - 2 delta)/(1 + 2 delta), q = pbar, rho_w = 1; halfway
 * bounce-back (delta = 1/2) where x - c_p is not a fluid cell.
 *   n       number of listed cells;
 *   cells   int32[n], device: every non-solid cell with a D3Q19 link into a
 *           solid cell, strictly ascending, nothing else;
 *   delta   double[19][n], device: delta[p*n + i] in (0, 1] for each link p
 *           of cells[i] whose neighbour x + c_p is solid (other entries not
 *           read);
 *   wall_u  double[3][19][n], device: velocity of that wall point,
 *           wall_u[(a*19 + p)*n + i] (finite).
 * The arrays stay owned by the caller and are read by every later step: keep
 * them alive and unchanged until the next call or fslbm_destroy.  The table
 * is validated on the device (then synchronises the stream); FSLBM_E_INVALID
 * names the first violation.  Required before fslbm_step when the flags hold
 * solid cells; not supported by the adjoint window. */
fslbm_status fslbm_set_walls(fslbm_ctx* c, int32_t n, const int32_t* cells, const double* delta,
                             const double* wall_u);

/* A prescribed surface plane for every interface cell (section 2.2: a
 * boundary node x_b with boundary links meeting the surface at x_b + delta
 * c_q, 0 <= delta <= 1), for surfaces whose position is known exactly (the
 * steady films of section 4.3).  Requires params.hold_fill.  The FSL rules
 * then take the link distances delta = offset / (n . c_o) (clamped to
 * [0, 1]) and the rules with a D term the local basis from this plane
 * instead of the fill field.
 *   normal  double[3][N], device: unit normal towards the gas,
 *           normal[a*N + idx] (read at interface cells);
 *   offset  double[N], device: signed distance of the plane from the node
 *           along the normal (positive: the node is on the liquid side).
 * The arrays stay owned by the caller and are read by every later step; NULL
 * removes the surface.  Not supported by the adjoint window.  No device
 * work. */
fslbm_status fslbm_set_surface(fslbm_ctx* c, const double* normal, const double* offset);

/* ---------------------------------------------------------------------------
 * Adjoint window: gradients through T steps with frozen cell classes.
 *
 * Over a window the cell classes stay fixed (no conversions), so a step is a
 * piecewise-smooth map of the state (ft, m, phi): pull (Eq. lbe1), mass
 * exchange, the normal from the fill gradient and the link distance delta
 * (section 3.3), FSK / FSL reconstruction (Eq. closure; Table 1 or Eq.
 * fsli1-fsli4), TRT collision (Eq. lbe2), phi = m / rho.  The window's
 * backward pass is the exact reverse-mode derivative of that map (the branches
 * of the forward run: delta clamps, the FSK fallback), written by hand; states
 * are kept by checkpointing: every K-th state is stored during the forward
 * pass, and each segment's states are recomputed from its checkpoint during
 * the backward pass (the last segment's are kept from the forward pass).  K =
 * 0 selects the default: K = T (every step's record kept, no recomputation)
 * when that workspace fits in half the device memory free at
 * fslbm_window_workspace_size, else K = ceil(sqrt T) (sqrt(T)
 * checkpointing).  Between checkpoints only a compact record
 * per step is kept: the collision velocity of the liquid cells and the inputs
 * of the interface cells.  All work runs on the context's stream.
 * Supported: FP64 and FP32 forms, the incompressible equilibrium with its
 * quadratic term (otherwise FSLBM_E_UNSUPPORTED).  The caller owns the window workspace; it must stay
 * allocated, and the context alive, until fslbm_window_destroy. */
typedef struct fslbm_window fslbm_window;

/* Bytes of window workspace for T steps with checkpoint spacing K (0: the
 * default) for the current cell classes of c.  Synchronises. */
fslbm_status fslbm_window_workspace_size(fslbm_ctx* c, int32_t T, int32_t K, size_t* bytes);

/* Forward pass: T steps with rule FSK or FSL (the rules with a D term, surface
 * tension, the PLIC option and solid cells are FSLBM_E_UNSUPPORTED here; the
 * FP16 storage form, the compressible equilibrium and the Stokes equilibrium
 * too) from the current state of c,
 * conversions disabled, storing checkpoints in the workspace (device memory,
 * 256-byte aligned, at least fslbm_window_workspace_size bytes).  On return the
 * state of c is that of time T (read it with fslbm_fields) and *out is the
 * window.  Synchronises once (to size the interface-cell list), then enqueues
 * the steps. */
fslbm_status fslbm_window_forward(fslbm_ctx* c, int32_t T, int32_t K, int32_t rule, void* workspace,
                                  size_t workspace_bytes, fslbm_window** out);

/* Backward pass.  Inputs (device, double; any may be NULL = zero): dL_df[19N]
 * = dL/d(post-collision populations of time T, unshifted; read at non-gas
 * cells), dL_dm[N] and dL_dphi[N] = dL/d(mass, fill of time T; read at
 * interface cells).  Outputs (device, double; any may be NULL = not written):
 * dL_df0[19N] (zero at gas cells), dL_dm0[N] and dL_dphi0[N] (zero outside
 * interface cells) for the state of time 0; host grads[4] = {dL/drho_b,
 * dL/dg_x, dL/dg_y, dL/dg_z} with dL/dP_b = 3 dL/drho_b.  Parameter gradients
 * are summed in FP64 in a fixed order.  May be called more than once.
 * Synchronises. */
fslbm_status fslbm_window_backward(fslbm_window* w, const double* dL_df, const double* dL_dm, const double* dL_dphi,
                                   double* dL_df0, double* dL_dm0, double* dL_dphi0, double grads[4]);

/* info = {T, K, number of checkpoints, interface cells}. */
fslbm_status fslbm_window_info(const fslbm_window* w, int32_t info[4]);

/* Wait for the window's work, then release its host state (not the
 * workspace).  Synchronises. */
fslbm_status fslbm_window_destroy(fslbm_window* w);

/* Release the context (not the caller's buffers).  Synchronises. */
fslbm_status fslbm_destroy(fslbm_ctx* c);

/* Message of the last failure on c, or of the last failed fslbm_init when c is
 * NULL.  Valid until the next call on the same context. */
const char* fslbm_last_error(const fslbm_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* FSLBM_H */
