/*
 * vanse.h -- C ABI of libvanse, the MI355X (gfx950) implementation of the
 * D2Q9 time step of the consistent multiple-relaxation-time lattice
 * Boltzmann method for the volume-averaged Navier-Stokes equations
 * (MRTLB-VANSE) of Liu, Zhang, Min & Wu, arXiv:2409.02964.
 *
 * Problem statement (Sec. 2.1-2.3): given a void-fraction field phi(x) in
 * (0, 1], a body force F^B, relaxation rates (the paper's tau_*, which are
 * RATES: Sec. 2.2, Eq. A11), the provisional equation-of-state constant
 * kappa (Eq. 13) and boundary conditions, advance Eq. (16) -- moment-space
 * MRT relaxation with the adjusted equilibrium (Eq. 14/18), Guo forcing
 * (Eq. 6/19) carrying F = F^p (Eq. 13) + F^B and the penalty source C
 * (Eq. 20) -- followed by streaming, and report rho, u, p (Eq. 7).
 *
 * Conventions shared by every call:
 *  - Every function returns VANSE_OK (0) or a negative VANSE_ERR_* code and
 *    never throws; vanse_last_error() returns a thread-local detail string.
 *  - Field arrays passed in or out are DEVICE pointers to dense row-major
 *    float64 arrays of shape [ny][nx] (index y*nx + x).  Populations are
 *    [9][ny][nx] in the D2Q9 order of Eq. (5): e_0 = (0,0), e_1..4 =
 *    (1,0),(0,1),(-1,0),(0,-1), e_5..8 = (1,1),(-1,1),(-1,-1),(1,-1).
 *    Inputs are borrowed for the duration of the call only (copied into the
 *    workspace); outputs are written by the call.
 *  - `stream` is a hipStream_t (NULL: the legacy default stream).  All work
 *    is enqueued on it; calls returning host data synchronize it.
 *  - A handle must not be used by two host threads at once.
 *  - The library allocates no device memory: all device state lives in a
 *    caller-owned workspace of vanse_workspace_bytes() bytes that must
 *    outlive the handle.
 */
#ifndef VANSE_H
#define VANSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define VANSE_OK 0
#define VANSE_ERR_INVALID_ARG (-1) /* bad size, rate, kappa, phi, pointer */
#define VANSE_ERR_WORKSPACE (-2)   /* workspace missing, too small, misaligned */
#define VANSE_ERR_HIP (-3)         /* a HIP runtime call failed */
#define VANSE_ERR_STATE (-4)       /* step/read before phi, params and init */
#define VANSE_ERR_DIVERGED (-5)    /* non-finite populations were observed */
#define VANSE_ERR_UNSUPPORTED (-6) /* a variant that is not built */

/* ---- precision of arithmetic and of the stored populations --------------
 * The step always works on deviations g_i = f_i - f_i^rest from the rest
 * state f^rest = f^eq(rho0, u = 0) of Eq. (14) (rest_0 = (phi - 5 kappa/9)
 * rho0, rest_i = w_i kappa rho0).  "Shifted" storage keeps g in memory, the
 * others keep f. */
#define VANSE_F64 0         /* FP64 arithmetic, FP64 f                 152 B/node */
#define VANSE_F32 1         /* FP32 arithmetic, FP32 f                  76 B/node */
#define VANSE_F32_SHIFTED 2 /* FP32 arithmetic, FP32 g                  76 B/node */
#define VANSE_F16_SHIFTED 3 /* FP32 arithmetic, FP16 g * 2^storage_exp  40 B/node */

/* ---- boundaries ---------------------------------------------------------- */
#define VANSE_PERIODIC 0
#define VANSE_WALL 1 /* half-way bounce-back walls on both faces (Sec. 3.1) */

typedef struct vanse_lattice vanse_lattice;

typedef struct {
  int32_t nx, ny;          /* nodes; nx >= 2, 2 <= ny <= 65535 */
  int32_t precision;       /* VANSE_F64 | VANSE_F32 | ..._SHIFTED */
  int32_t bc_x;            /* VANSE_PERIODIC | VANSE_WALL; walls in x step with the
                              solid-node kernel, one step per launch */
  int32_t bc_y;            /* VANSE_PERIODIC | VANSE_WALL */
  int32_t has_force_field; /* 1: a per-node force field is added to F^B */
  int32_t has_drag;        /* 1: a per-node linear drag acts (vanse_set_drag) */
  int32_t has_mask;        /* 1: solid nodes given by vanse_set_mask */
  int32_t dynamic_phi;     /* 1: phi may change in time (vanse_set_void_fraction_next) */
} vanse_desc;

/* Diagonal of Gamma in Eq. (16), each in (0, 2):
 * Gamma = diag(s_c, s_e, s_eps, s_c, s_q, s_c, s_q, s_nu, s_nu).
 * nu = (1/s_nu - 1/2)/3 and nu_e = (1/s_e - 1/2)/3 (Eq. A11).  s_c acts on
 * conserved moments only and drops out of the update (their relaxation
 * leaves phi*rho and j + F unchanged, Eq. 17). */
typedef struct {
  double s_c, s_e, s_eps, s_q, s_nu;
} vanse_rates;

/* Bytes of device workspace the lattice described by *d needs (256-byte
 * aligned).  Layout: two population buffers, phi, optional phi(t+1),
 * solid-flag, force and drag planes, a density scratch plane and reduction
 * space.  VANSE_ERR_INVALID_ARG for a lattice whose population buffer (nine
 * planes of the storage type, rows padded to 64 nodes) would reach 4 GiB --
 * the step kernels address it with 32-bit offsets -- or with more than 65535
 * rows (set-up and read-out kernels put one row per grid row). */
int vanse_workspace_bytes(const vanse_desc *d, size_t *bytes);

/* Create a lattice whose device state lives in `workspace` (device pointer,
 * 256-byte aligned, >= vanse_workspace_bytes).  The caller keeps ownership
 * of the workspace; the handle is host memory freed by vanse_destroy. */
int vanse_create(const vanse_desc *d, void *workspace, size_t bytes,
                 vanse_lattice **out);
int vanse_destroy(vanse_lattice *h);

/* kappa in [0, 1] (Eq. 13: constant of the provisional equation of state,
 * best close to the minimum of phi) and the relaxation rates. */
int vanse_set_params(vanse_lattice *h, double kappa, const vanse_rates *r);

/* ---- scheme variants (Sec. 2.3 below Eq. 20, Appendix B) ----------------- */
#define VANSE_MODEL_A 0 /* the consistent VANSE of Eq. (1): -phi grad p, div(phi tau) */
#define VANSE_MODEL_B 1 /* model B (set I): -grad p, div(tau) */

/* Choose the scheme: model VANSE_MODEL_A (default) or VANSE_MODEL_B --
 * F^p = (kappa - 1) cs^2 grad rho in place of Eq. (13) and "kappa - phi"
 * replaced by "kappa - 1" in the source term -- and the equilibrium order:
 * 3 (default; Eq. 14, moments Eq. 18, penalty Eq. 20) or 2 (the truncated
 * equilibrium of Appendix B, Eq. B1, moments B2, penalty B3 with twelve
 * derivatives).  Only before the populations are set. */
int vanse_set_scheme(vanse_lattice *h, int model, int equilibrium_order);

/* Tangential (x) velocities of the walls on the faces y = -1/2 (u_lo) and
 * y = ny - 1/2 (u_hi); default 0.  A population crossing a moving wall
 * returns less the odd part of the equilibrium (Eq. 14, or B1) at
 * (phi(x), rho0, u_w), and the Eq. (10) stand-ins across the wall carry
 * 2 u_w - u.  This moving form of half-way bounce-back is an alternative to
 * the paper's own velocity condition for Couette flow (Sec. 3.1 imposes it
 * by non-equilibrium extrapolation: vanse_set_velocity_rows); it keeps every
 * row a fluid row and a closed box's lid on the face.  Needs bc_y =
 * VANSE_WALL; only before the populations are set. */
int vanse_set_wall_velocity(vanse_lattice *h, double u_lo, double u_hi);

/* Velocity boundary rows: the moving-wall condition of Couette flow in
 * Sec. 3.1 (Eq. 22 II), imposed by non-equilibrium extrapolation (the
 * paper's ref. [47]).  `faces` is VANSE_FACE_LO and/or VANSE_FACE_HI: the
 * first (y = 0) and/or last (y = ny - 1) row becomes a row of boundary nodes
 * lying on a wall that moves with x velocity u_lo / u_hi.  Such a node is not
 * evolved by the scheme.  After every collision its post-collision
 * populations are set from the fluid node x_f next to it across the row:
 *   f+_i(x_b) = f^eq_i(phi(x_b), rho(x_f), u_w) + f+_i(x_f) - f^eq_i(phi(x_f), rho(x_f), u(x_f))
 * with f^eq of Eq. (14), or B1 with the Appendix B equilibrium; the density
 * is extrapolated as rho(x_b) = rho(x_f).  The Eq. (10) stencils of x_f see
 * rho(x_f) and u_w at x_b.  vanse_read_moments reports rho(x_f), u_w and
 * rho(x_f)/3 on the row; it is left out of vanse_observe and
 * vanse_residual (mass is not conserved through it).  The face beyond the
 * row stays a half-way wall, which no population crossing it reaches a fluid
 * node through.  With a velocity row on the upper face only, the walls of a
 * channel are ny - 1/2 apart.  Needs bc_y = VANSE_WALL, ny >= 3, bc_x =
 * VANSE_PERIODIC and no mask (VANSE_ERR_UNSUPPORTED otherwise), no half-way
 * wall velocity on the same face; only before the populations are set.
 * faces = 0 removes the rows.  One step per launch, in the step-kernel
 * instance that carries every optional input; batches do not take such
 * lattices (VANSE_ERR_UNSUPPORTED). */
#define VANSE_FACE_LO 1
#define VANSE_FACE_HI 2
int vanse_set_velocity_rows(vanse_lattice *h, int faces, double u_lo, double u_hi);

/* Uniform external acceleration G: F^B = phi*G (scale_by_phi = 1, the form
 * F^B = phi(G - ...) of Sec. 3.1 and Eq. 23) or F^B = G (scale_by_phi = 0).
 * Defaults: G = 0, scale_by_phi = 1. */
int vanse_set_body_force(vanse_lattice *h, double gx, double gy,
                         int scale_by_phi);

/* Void fraction phi: device float64 [ny][nx], each value in (0, 1]
 * (checked; VANSE_ERR_INVALID_ARG otherwise).  Synchronizes the stream. */
int vanse_set_void_fraction(vanse_lattice *h, const double *phi, void *stream);

/* Time-varying void fraction (Sec. 2.3, Eq. 20): phi(x, t+1) for the next
 * step, device float64 [ny][nx] in (0, 1] (solid nodes excepted).  The next
 * vanse_step call must advance exactly one step; it evaluates the d_t phi
 * term of C_a with the forward difference phi(t+1) - phi(t) and then makes
 * phi(t+1) the current void fraction.  Without a pending phi(t+1) the void
 * fraction is held constant.  Needs dynamic_phi; synchronizes the stream. */
int vanse_set_void_fraction_next(vanse_lattice *h, const double *phi_next,
                                 void *stream);

/* Time-varying void fraction over the next two steps (Sec. 2.3, Eq. 20;
 * the moving particles of Eq. 23), for two steps per launch
 * (vanse_set_steps_per_pass): phi(x, t+1) and phi(x, t+2), device float64
 * [ny][nx] each in (0, 1].  The second step's drag coefficient beta_next
 * (needs has_drag) and force field fx_next, fy_next (both or neither; needs
 * has_force_field) are optional, device float64 [ny][nx]: without them the
 * current ones serve both steps; the current ones serve the first step.
 * The next vanse_step calls advance these two steps (one call of two steps,
 * or two calls of one); the first takes d_t phi = phi(t+1) - phi(t), the
 * second phi(t+2) - phi(t+1).  Afterwards phi(t+2) and the second step's
 * force field and drag coefficient are the current ones.  The caller keeps
 * ownership of the inputs (copied before the call returns).  Needs
 * dynamic_phi and no pending void fraction (VANSE_ERR_STATE); synchronizes
 * the stream. */
int vanse_set_void_fraction_next2(vanse_lattice *h, const double *phi_next,
                                  const double *phi_next2, const double *beta_next,
                                  const double *fx_next, const double *fy_next,
                                  void *stream);

/* Solid nodes (Sec. 2.3 and Sec. 3.1: half-way bounce-back on their faces):
 * device uint8 [ny][nx], nonzero = solid.  A fluid node pulls the opposite
 * population of its own post-collision state from a solid neighbour's
 * direction, and the Eq. (10) stencils use the centre node's value for a
 * solid neighbour (negated for velocity-like fields); solid nodes report
 * zero moments and populations and are left out of the observables.  Their
 * phi is not used (any value is accepted there).  Needs has_mask; only
 * before the populations are set; synchronizes the stream. */
int vanse_set_mask(vanse_lattice *h, const uint8_t *mask, void *stream);

/* Per-node force added to F^B (e.g. the manufactured-solution forces of
 * Appendix C): device float64 [ny][nx] each.  Needs has_force_field. */
int vanse_set_force_field(vanse_lattice *h, const double *fx, const double *fy,
                          void *stream);

/* Linear drag towards a solid velocity u_s: F^B gains -phi*beta*(u - u_s),
 * and u of Eq. (7) is solved in closed form from
 * u = (j + F/2)/(phi rho).  This is the Darcy term of Eq. (21) (beta =
 * phi nu / k0) and the particle drag of Eq. (23) (beta = phi (1 - phi)).
 * beta: device float64 [ny][nx].  Needs has_drag. */
int vanse_set_drag(vanse_lattice *h, const double *beta, double usx, double usy,
                   void *stream);

/* t = 0 with f(0) = f^eq(rho0, u0) of Eq. (14) at every node.  rho0 is also
 * the reference density of the rest state used by the deviation form. */
int vanse_init_equilibrium(vanse_lattice *h, double rho0, double ux0,
                           double uy0, void *stream);

/* t = 0 with the given post-streaming populations f(0): device float64
 * [9][ny][nx].  The rest-state reference density is rho0. */
int vanse_set_populations(vanse_lattice *h, const double *f, double rho0,
                          void *stream);

/* Advance nsteps >= 0 time steps (collision of Eq. 16, then streaming with
 * bounce-back).  Enqueued only; does not synchronize -- unless a check
 * interval is set (below). */
int vanse_step(vanse_lattice *h, int64_t nsteps, void *stream);

/* Divergence check inside vanse_step: with k > 0, every time t that is a
 * multiple of k reached during a vanse_step call is followed by the FP64
 * observables of vanse_observe (enqueued between the launches; the record
 * of the last one is what vanse_observe would return at that time), and the
 * call ends with one synchronizing read: VANSE_ERR_DIVERGED, with the first
 * checked time in vanse_last_error(), when one of them counted a non-finite
 * node.  With two steps per launch a check follows the launch that reaches
 * the multiple of k (at t or t + 1), so the launches, and the results, are
 * those of the unchecked call.
 * The steps run to the end of the call either way (t advances by nsteps).
 * k = 0 (the default) turns the check off.  Batches do not run it. */
int vanse_set_check_interval(vanse_lattice *h, int64_t k);

/* rho = sum f / phi, u = (sum e f + F/2) / sum f, p = rho/3 (Eq. 7, with
 * F = F^p + F^B of Eq. 13) of the populations at the current t.  Device
 * float64 [ny][nx] outputs; any of ux, uy, p may be NULL. */
int vanse_read_moments(vanse_lattice *h, double *rho, double *ux, double *uy,
                       double *p, void *stream);

/* Post-streaming populations f_i(x, t) at the current t: device float64
 * [9][ny][nx]. */
int vanse_read_populations(vanse_lattice *h, double *f, void *stream);

/* Observables of the current state, reduced in FP64 on the device in a
 * fixed order: out[0] = total mass sum_x sum_i f_i, out[1] = sum_x |u|^2,
 * out[2] = max_x |u|, out[3] = number of nodes with a non-finite value.
 * `out` is HOST memory (4 doubles); synchronizes the stream.  Returns
 * VANSE_ERR_DIVERGED (after filling out) when out[3] > 0. */
int vanse_observe(vanse_lattice *h, double *out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * observables of vanse_observe, bitwise the same values, computed without
 * the lattice workspace's scratch -- the density of every node and of its
 * neighbours is formed again from the populations, and the FP64 block
 * partials and the reduction records live in a static device array of the
 * library (about 5.3 MB, held by every device the library runs on until the
 * process ends).  Allocates nothing.  Limit: ceil(nx/256) * ny <= 131072
 * (for example 4096 x 8192 or 8192 x 4096); larger lattices get
 * VANSE_ERR_INVALID_ARG before any device work.  Calls that overlap on one
 * device share the array and race: serialize them (one stream, or events).
 * `out` is HOST memory (4 doubles); synchronizes the stream; returns
 * VANSE_ERR_DIVERGED (after filling out) when out[3] > 0. */
int vanse_observe_noalloc(vanse_lattice *h, double *out, void *stream);

/* Steady-state residual support: out[0] = sum_x |u(t) - u(t')|^2 where t'
 * is the time of the previous vanse_residual call on this lattice (-1 on
 * the first call after initialisation), out[1] = sum_x |u(t)|^2, out[2] =
 * number of non-finite nodes.  u(t) is kept for the next call.  The
 * relative residual of two consecutive steps is sqrt(out[0] / out[1]).
 * `out` is HOST memory (3 doubles); synchronizes the stream. */
int vanse_residual(vanse_lattice *h, double *out, void *stream);

/* Launch shape of the step kernel: threads per workgroup (64, 128, 256 or
 * 512; a workgroup owns threads-4 columns) and rows swept per workgroup
 * (>= 1).  threads = 0 or rows = 0 restores the size-based default. */
int vanse_set_tiling(vanse_lattice *h, int threads, int rows);
int vanse_get_tiling(const vanse_lattice *h, int *threads, int *rows,
                     int *workgroups);

/* Time steps per launch of the step with any of the force field, the linear
 * drag, and solid nodes or a moving phi (vanse_set_void_fraction_next2) or
 * a scheme variant (model B, the Appendix B equilibrium, or both; also
 * with solid nodes), with no walls in x, wall velocity or velocity rows: 1
 * (the
 * default) or 2.  With 2, vanse_step advances pairs of steps with one
 * launch each: a workgroup's first half runs step t -> t+1 into an LDS ring
 * and its second half step t+1 -> t+2 from it, so the populations cross HBM
 * once per two steps; an odd step count ends with one single step.  Each
 * half computes the same scheme as the single step (its Eq. 10 sums in the
 * stencil's separable form, so the roundings differ); the intermediate
 * state stays in deviations of the arithmetic type (FP32, or FP64 for
 * VANSE_F64), so FP32-shifted and FP64 storage match the single-step
 * results to rounding and the other storage formats skip one storage
 * rounding.  Halves of 256 lanes in FP32 arithmetic and of 128 in FP64
 * (half that for solid nodes with the drag, a moving phi and the Appendix B
 * equilibrium).  Other
 * lattices keep one step per launch.  rows: rows per workgroup of the
 * two-step kernel (0: one full round of resident workgroups). */
int vanse_set_steps_per_pass(vanse_lattice *h, int steps, int rows);
/* Whether the two-step launch is in use (*active), and its rows per
 * workgroup and workgroups per launch. */
int vanse_get_fused_tiling(const vanse_lattice *h, int *active, int *rows,
                           int *workgroups);

/* Exponent e of the storage scale 2^e of VANSE_F16_SHIFTED (default 12):
 * memory holds g * 2^e in FP16.  Only before init. */
int vanse_set_storage_exponent(vanse_lattice *h, int e);

/* Measurement helper, not part of the method: n launches of a kernel with
 * the step's exact memory pattern (pull of the nine populations with the
 * same shifts and bounce-back at y-walls, written back unchanged to the
 * other buffer; 9 reads + 9 writes per node, no arithmetic; x always wraps).  It is the speed-of-light
 * reference for the step's HBM traffic and the calibration kernel for
 * memory counters.  It permutes the stored state; t is not advanced. */
int vanse_stream_copy(vanse_lattice *h, int64_t n, void *stream);

/* ---- batches -------------------------------------------------------------
 * Many independent lattices advanced together: every call to
 * vanse_batch_step launches ONE kernel per time step (or per two, see
 * vanse_batch_create_ex) whose workgroups cover the tiles of all member
 * lattices (tile = strip of threads-4 columns x `rows` rows of one lattice).  Each member's arithmetic is exactly that of
 * vanse_step (results are bitwise identical).  Members must share precision,
 * boundary types, force field, drag, mask and scheme variant (VANSE_ERR_INVALID_ARG
 * otherwise), be fully set up, and stay alive
 * while the batch exists.  The batch keeps a table of the members'
 * parameters and buffer parity in a caller-owned device workspace; it is
 * written again automatically when a member changed or was stepped on its
 * own.  Member handles stay usable (vanse_time, vanse_read_*).  Lattices with
 * a time-varying void fraction or velocity rows are not batched, nor
 * lattices combining a scheme variant (model B, the Appendix B equilibrium,
 * moving walls) with solid nodes or walls in x (VANSE_ERR_UNSUPPORTED). */
typedef struct vanse_batch vanse_batch;

/* Workspace bytes for a batch of n lattices with the given workgroup width
 * (64, 128 or 256) and rows per workgroup (0: about two rounds of resident
 * workgroups over the batch). */
int vanse_batch_workspace_bytes(vanse_lattice *const *lats, int n, int threads,
                                int rows, size_t *bytes);
int vanse_batch_create(vanse_lattice *const *lats, int n, int threads, int rows,
                       void *workspace, size_t bytes, vanse_batch **out);
int vanse_batch_destroy(vanse_batch *b);

/* As the two calls above, with steps_per_pass time steps per launch (1 or
 * 2).  With 2 every launch applies the two-step kernel of
 * vanse_set_steps_per_pass to all members, which must share its instance
 * (VANSE_ERR_INVALID_ARG otherwise; model B alone and the Appendix B
 * equilibrium do not): threads is then the width of each half of a
 * workgroup of 2 x threads lanes, at most the half width of that instance
 * (256 in FP32 arithmetic, 128 in FP64, half that for solid nodes with the
 * drag and for the Appendix B equilibrium; VANSE_ERR_UNSUPPORTED beyond), a
 * tile is a strip of threads-10 columns, and rows = 0 gives about four
 * rounds of resident workgroups.  Each member's results are bitwise those
 * of stepping it alone with two steps per launch; an odd step count ends
 * with one step of each member on its own. */
int vanse_batch_workspace_bytes_ex(vanse_lattice *const *lats, int n, int threads,
                                   int rows, int steps_per_pass, size_t *bytes);
int vanse_batch_create_ex(vanse_lattice *const *lats, int n, int threads, int rows,
                          int steps_per_pass, void *workspace, size_t bytes,
                          vanse_batch **out);

/* Capture the step loop in hipGraphs of this many time steps (> 0 and a
 * multiple of 2 x steps per pass, so that a replay covers an even number of
 * launches; 0 turns graphs off).  Graph launches run on a stream owned by
 * the batch, ordered after and before the caller's stream with events. */
int vanse_batch_set_graph(vanse_batch *b, int steps_per_graph);

/* Advance every member nsteps time steps.  Enqueued on `stream`. */
int vanse_batch_step(vanse_batch *b, int64_t nsteps, void *stream);

/* vanse_residual of every member, with one copy to the host and one
 * synchronization for the whole batch: out is HOST memory of 3 doubles per
 * member, in member order (sum |u(t) - u(t')|^2 or -1 on a member's first
 * call, sum |u(t)|^2, non-finite count); each member keeps u(t) for its next
 * vanse_residual or vanse_batch_residual call.  VANSE_ERR_DIVERGED (after
 * filling out) when a member holds a non-finite node. */
int vanse_batch_residual(vanse_batch *b, double *out, void *stream);

/* Tiles (workgroups per launch) and rows per workgroup of the batch. */
int vanse_batch_tiles(const vanse_batch *b, int *tiles, int *rows);

/* Current time step t. */
int64_t vanse_time(const vanse_lattice *h);

const char *vanse_error_string(int code);
const char *vanse_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VANSE_H */
