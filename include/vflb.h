/*
 * vflb.h -- C ABI of libvflb, the MI355X (gfx950) implementation of the
 * fluctuating lattice Boltzmann method for Oldroyd-B viscoelastic flows
 * (Wang, Liu, Wang, Yu, Ji, arXiv 2506.13072).
 *
 * One time step of the method on a D2Q9 or D3Q19 lattice, fused into a
 * single pass over the populations:
 *   - pull streaming of the velocity populations f_i and the conformation
 *     populations h_abi (left-hand sides of the evolution equations of
 *     Sec. 2.2 and Sec. 2.3), periodic or halfway bounce-back;
 *   - moments: A = sum_i h_abi (Sec. 2.3), tau_p = (mu_p/lambda)(A - I)
 *     (Sec. 2.1), u = sum c_i f_i + F/2 and the pressure (Sec. 2.2, App. B);
 *   - the polymer-stress fluctuation term f^B from the pseudo-inverse
 *     closed forms (Sec. 2.2 for D2Q9, App. A for D3Q19);
 *   - the BGK collision with f^eq, the Guo forcing term and f^B (Sec. 2.2);
 *   - the Oldroyd-B source chi = -(A - I)/lambda + A.grad u + grad u^T.A
 *     from the velocity gradient at the same time level, its distribution
 *     chi_abi and the collision of h with tau_h (Sec. 2.3).
 *
 * Conventions.
 *   - C linkage only; every call returns a vflb_status.  A failing call
 *     leaves the simulation unchanged and records a message readable with
 *     vflb_last_error().
 *   - Device memory is owned by the caller.  vflb_query_buffers() reports
 *     the sizes of the VFLB_NBUF device buffers a simulation needs; the
 *     caller allocates them (any allocator, 256-byte aligned) and hands
 *     them over with vflb_bind_buffers().  The library never frees them.
 *     Handles and small host-side metadata are owned by the library.
 *   - Work is enqueued on the HIP stream given at creation, in call order.
 *     vflb_reduce(), vflb_set_force(), vflb_save() and vflb_load()
 *     synchronise that stream; every other call only enqueues.
 *   - Fields are node-major with x fastest: node n = (z*ny + y)*nx + x.
 *     Symmetric tensors use the component order (xx, xy, yy) in 2D and
 *     (xx, yy, zz, xy, xz, yz) in 3D.
 *   - Lattice units: dx = dt = 1, c_s^2 = 1/3, rho0 = 1.
 */
#ifndef VFLB_H
#define VFLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vflb_sim vflb_sim;
typedef struct vflb_batch vflb_batch;
typedef struct vflb_mlp vflb_mlp;

typedef enum {
  VFLB_OK = 0,
  VFLB_EINVAL = 1,    /* bad argument; nothing was changed            */
  VFLB_ENOMEM = 2,    /* a buffer is missing or too small             */
  VFLB_EDEVICE = 3,   /* a HIP call failed                            */
  VFLB_EUNSTABLE = 4, /* non-finite values found by vflb_reduce       */
  VFLB_ESTATE = 5     /* call out of order (e.g. step before init)    */
} vflb_status;

typedef enum { VFLB_D2Q9 = 2, VFLB_D3Q19 = 3 } vflb_lattice;

/* Storage of the populations.  Arithmetic is FP64 for VFLB_F64 and FP32
 * otherwise.  The conformation populations are stored shifted by their rest
 * value w_i delta_ab (so A - I is their plain sum); the velocity populations
 * have rest value 0 in this incompressible model.  The 16-bit storages are
 * anchored: every node also keeps an FP32 anchor (A - I, pressure and
 * velocity of its last update), and a stored population is the 16-bit
 * deviation of the value from the equilibrium-form reference built from
 * the anchor of the node that wrote it, so that A and u live in FP32.
 * VFLB_F16S stores the deviations times a power of two
 * (vflb_set_storage_scale), VFLB_BF16S stores them unscaled; both round to
 * nearest even.  With 16-bit storage, D3Q19 runs 32 x 4 tiles.  D3Q19
 * takes VFLB_F16S but not VFLB_BF16S: BF16's 8-bit mantissa leaves u and tau
 * 2e-3 .. 7e-3 (relative L2) away from the FP64 iteration on coarse D3Q19
 * lattices, above the 1e-3 accuracy of 16-bit storage, so vflb_create
 * returns VFLB_EINVAL for it. */
typedef enum {
  VFLB_F64 = 0,
  VFLB_F32 = 1,
  VFLB_F16S = 2,
  VFLB_BF16S = 3
} vflb_storage;

/* Body force kinds (lattice units):
 *   NONE       F = 0
 *   CONST      F = amp
 *   FOUR_ROLL  F = (amp[0] sin(kx x) cos(ky y), amp[1] cos(kx x) sin(ky y), 0),
 *              kx = 2 pi/nx, ky = 2 pi/ny, x, y the node indices
 *              (simplified four-roll mill, Sec. 3.1)
 *   COS_T      F = amp cos(omega t), t the step index (Womersley, Sec. 3.3)
 * The force of step t is evaluated at time level t, in the velocity moment
 * and in the forcing term alike. */
enum {
  VFLB_FORCE_NONE = 0,
  VFLB_FORCE_CONST = 1,
  VFLB_FORCE_FOUR_ROLL = 2,
  VFLB_FORCE_COS_T = 3
};

/* Boundary kind per axis: periodic, or halfway bounce-back walls half a
 * lattice spacing outside the first and the last node of that axis (for f
 * and for h alike).  Next to a wall the normal derivative of u uses the
 * parabola through the wall value 0 and the first two nodes. */
enum { VFLB_PERIODIC = 0, VFLB_WALLS = 1 };

/* How the polymer stress enters the velocity populations:
 *   FLUCTUATING        the paper's method: the fluctuation term f^B of the
 *                      pseudo-inverse closed forms (Sec. 2.2, App. A);
 *   STRESS_DIVERGENCE  the scheme the paper measures its method against
 *                      (Sec. 3, performance tables of the Poiseuille and
 *                      Taylor-Green tests; described in words in the
 *                      Introduction): no f^B, and div tau_p(t) added to the
 *                      body force in the forcing term, the velocity moment
 *                      and the pressure.  Its stencil is not given in the
 *                      paper; here second-order central differences of
 *                      tau_p(t), one-sided second order (-3 t0 + 4 t1 -
 *                      t2)/2 normal to a wall.  D2Q9 and D3Q19 with FP32
 *                      or FP64 storage; tau_p and div tau_p occupy NC + D
 *                      more words per node of the AUX buffer (5 in 2D, 9
 *                      in 3D).
 * The conformation equation (Sec. 2.3) is the same in both. */
enum { VFLB_SCHEME_FLUCTUATING = 0, VFLB_SCHEME_STRESS_DIVERGENCE = 1 };

/* Constitutive model of the polymer: the relaxation term R(E), E = A - I,
 * of the conformation equation chi = -R(E)/lambda + A.grad u + grad u^T.A
 * (Sec. 2.1, 2.3; the paper's method is built on Oldroyd-B and names the
 * Giesekus and Phan-Thien-Tanner models as the next ones):
 *   OLDROYD_B  R = E                               (default; param ignored)
 *   GIESEKUS   R = E + alpha E.E,  alpha = param in [0, 1/2]
 *   LPTT       R = (1 + eps tr E) E,   eps = param >= 0
 *   EPTT       R = exp(eps tr E) E,    eps = param >= 0
 * The polymer stress stays tau_p = (eta_p/lambda) E, so f^B and the
 * stress-divergence force are unchanged. */
enum {
  VFLB_MODEL_OLDROYD_B = 0,
  VFLB_MODEL_GIESEKUS = 1,
  VFLB_MODEL_LPTT = 2,
  VFLB_MODEL_EPTT = 3
};

/* Device buffers of one simulation (sizes from vflb_query_buffers).  Their
 * internal layout is private to the library (it differs between lattices
 * and storages); read fields through vflb_read and move whole states through
 * vflb_save / vflb_load. */
enum {
  VFLB_BUF_POP0 = 0, /* all populations, ping                              */
  VFLB_BUF_POP1 = 1, /* all populations, pong (256 bytes, unused, in place)*/
  VFLB_BUF_AUX = 2,  /* chi(t-1) and u(t-1), arithmetic type               */
  VFLB_BUF_SNAP = 3, /* residual snapshot of u and tau, arithmetic type    */
  VFLB_BUF_WORK = 4, /* force tables, reduction partials                   */
  VFLB_NBUF = 5
};

/* Read-back fields (vflb_read).  FIELD_U .. FIELD_H are moments of the
 * pre-collision state at the current time level t, with the force F(t);
 * CHI_PREV and U_PREV are the auxiliary state kept for the backward
 * difference of the source term (chi and u of time level t-1). */
enum {
  VFLB_FIELD_U = 0,   /* [D][N]  velocity                                  */
  VFLB_FIELD_P = 1,   /* [N]     pressure (App. B)                         */
  VFLB_FIELD_RHO = 2, /* [N]     rho0 + p / c_s^2 (the model has no density) */
  VFLB_FIELD_A = 3,   /* [NC][N] conformation tensor                       */
  VFLB_FIELD_TAU = 4, /* [NC][N] polymer stress                            */
  VFLB_FIELD_F = 5,   /* [Q][N]  pre-collision f populations               */
  VFLB_FIELD_H = 6,   /* [NC][Q][N] pre-collision h populations, unshifted */
  VFLB_FIELD_CHI_PREV = 7, /* [NC][N] stored source tensor of the last step */
  VFLB_FIELD_U_PREV = 8    /* [D][N]  stored velocity of the last step      */
};

/* Dimensionless parameters (Sec. 3): beta = nu_s/(nu_s + nu_p),
 * Wi = lambda U/L, Re = U L/(nu_s + nu_p).  Mapped to lattice units as
 * nu = U0 L / Re, nu_s = beta nu, nu_p = (1 - beta) nu,
 * tau_f = nu_s/c_s^2 + 1/2 (Sec. 2.2), lambda = Wi L / U0 unless
 * lambda > 0 is given, eta_p = nu_p.  tau_h <= 0 selects the paper's 0.501.
 * Valid: Re > 0, U0 > 0, L > 0, 0 < beta <= 1, tau_f > 1/2, tau_h > 1/2,
 * lambda > 0.  beta = 1 is the Newtonian limit (eta_p = 0, f^B = 0). */
typedef struct {
  double Re, Wi, beta, U0, L;
  double lambda; /* > 0 overrides Wi L / U0 */
  double tau_h;  /* <= 0: 0.501             */
} vflb_params;

/* Derived lattice-unit parameters (vflb_get_lattice_params). */
typedef struct {
  double nu_s, nu_p, tau_f, tau_h, lambda, eta_p;
} vflb_lattice_params;

/* Create a simulation of nx*ny*nz nodes (nz = 1 for D2Q9) whose work is
 * enqueued on hip_stream (a hipStream_t; NULL is the null stream).
 * *out receives a library-owned handle.  EINVAL for a bad lattice, storage
 * (BF16S on D3Q19 included) or size. */
vflb_status vflb_create(int lattice, int nx, int ny, int nz, int storage,
                        void *hip_stream, vflb_sim **out);

/* vflb_create with the scheme (VFLB_SCHEME_*; vflb_create is
 * VFLB_SCHEME_FLUCTUATING).  EINVAL for an unknown scheme, or for
 * STRESS_DIVERGENCE with 16-bit storage. */
vflb_status vflb_create_scheme(int lattice, int nx, int ny, int nz, int storage, int scheme,
                               void *hip_stream, vflb_sim **out);

/* Options of vflb_create_ex.
 *   VFLB_OPT_INPLACE  one population buffer instead of two (AA streaming):
 *     a step at even t reads a node's pre-collision populations from its
 *     own slots and writes the post-collision ones back into them under the
 *     opposite directions; a step at odd t reads them where their writers
 *     left them and writes into the slots of the readers of the next step.
 *     The same-time velocity gradient then needs u of the neighbours before
 *     they are overwritten: a velocity pass per step writes u(t) (D more
 *     words per node of AUX).  D2Q9: results equal the two-buffer step's
 *     bit for bit.  D3Q19: the z-march with the in-place maps, its
 *     velocity ring read from u(t) instead of pulled from the neighbours'
 *     slots; the same iteration up to rounding (the velocity sums in
 *     another order).  FP32 or FP64 storage, single lattices; no
 *     settling.  The
 *     population layout alternates with the parity of t; checkpoints record
 *     it (vflb_load refuses a checkpoint of the other layout). */
enum { VFLB_OPT_INPLACE = 1 };

/* vflb_create_scheme with options (VFLB_OPT_* bits; 0 is vflb_create_scheme).
 * EINVAL for unknown bits or an option on a lattice or storage that does
 * not support it. */
vflb_status vflb_create_ex(int lattice, int nx, int ny, int nz, int storage, int scheme,
                           int options, void *hip_stream, vflb_sim **out);

/* Constitutive model (VFLB_MODEL_*) and its parameter; takes effect from the
 * next step.  EINVAL for an unknown model or a parameter out of range. */
vflb_status vflb_set_model(vflb_sim *sim, int model, double param);

/* Sizes in bytes of the VFLB_NBUF device buffers. */
vflb_status vflb_query_buffers(const vflb_sim *sim, size_t bytes[VFLB_NBUF]);

/* Hand over the caller-owned device buffers (one pointer per buffer, each at
 * least the queried size).  EINVAL on a NULL pointer. */
vflb_status vflb_bind_buffers(vflb_sim *sim, void *const dev_ptrs[VFLB_NBUF]);

/* Set the physical parameters (see vflb_params).  EINVAL when the derived
 * lattice parameters are out of range. */
vflb_status vflb_set_params(vflb_sim *sim, const vflb_params *p);

/* Lattice-unit parameters derived by vflb_set_params. */
vflb_status vflb_get_lattice_params(const vflb_sim *sim,
                                    vflb_lattice_params *out);

/* Set the body force (kind and lattice-unit amplitude amp[3]; omega for
 * COS_T).  Needs bound buffers (the four-roll tables live in the work
 * buffer).  EINVAL for an unknown kind.  FOUR_ROLL on D3Q19 is the same
 * z-independent field. */
vflb_status vflb_set_force(vflb_sim *sim, int kind, const double amp[3],
                           double omega);

/* Boundary kind per axis (VFLB_PERIODIC or VFLB_WALLS); a wall axis needs
 * at least 2 nodes. */
vflb_status vflb_set_boundaries(vflb_sim *sim, const int kind_per_axis[3]);

/* Power-of-two scales of the VFLB_F16S storage: f is stored as
 * f * 2^log2_f, the shifted h as (h - w delta) * 2^log2_h.  Defaults are
 * chosen from U0 by vflb_set_params.  Ignored for other storages. */
vflb_status vflb_set_storage_scale(vflb_sim *sim, int log2_f, int log2_h);

/* Equilibrium-only initial state from FP64 device fields u [D][N],
 * tau [NC][N] (polymer stress) and p [N]; NULL means zero.  Sets
 * f = f^eq(p, u), h = h^eq(A, u) with A = I + lambda tau / eta_p, and the
 * time level t = 0.  Needs bound buffers and parameters. */
vflb_status vflb_init_fields(vflb_sim *sim, const double *u_dev,
                             const double *tau_dev, const double *p_dev);

/* Advance nsteps >= 0 time steps (nsteps fused stream-collide launches,
 * replayed from a captured HIP graph when nsteps is large). */
vflb_status vflb_step(vflb_sim *sim, int64_t nsteps);

/* Current time level (host copy; no synchronisation). */
int64_t vflb_time(const vflb_sim *sim);

/* FP64 reductions over the pre-collision state at time t (synchronises):
 *   out[0]  R: max over q in {u, tau} of ||q - q_snap||_2 / ||q||_2, where
 *           q_snap is the state at the previous vflb_reduce call (+inf on
 *           the first call); the snapshot is then replaced
 *   out[1]  M  = sum of all f (stays 0 from an equilibrium start)
 *   out[2..4] P = sum of c_i f_i (x, y, z)
 *   out[5]  KE = (1/N) sum |u|^2 / 2,  out[6] PE = (1/N) sum tr(tau)/2
 *           (Sec. 3.4)
 *   out[7]  number of nodes with a non-finite moment
 *   out[8..13] sum over nodes of the NC components of A
 * Returns VFLB_EUNSTABLE when out[7] > 0 (out is still filled). */
vflb_status vflb_reduce(vflb_sim *sim, double out[14]);

/* vflb_reduce for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels, values and snapshot update as vflb_reduce, but the
 * per-block partial sums and the results live in a static device array of
 * the library (17 x 1024 + 17 doubles, 139 KB, one copy per GPU, held until
 * the process ends) instead of the VFLB_BUF_WORK buffer.  It calls no
 * hipMalloc/hipFree.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (several host threads, or streams of different
 * simulations running concurrently) race and must be serialised by the
 * caller.  EINVAL if a reduction ever needed more partials than the array
 * holds (it cannot with the library's launch shape); otherwise as
 * vflb_reduce, which it synchronises like. */
vflb_status vflb_reduce_noalloc(vflb_sim *sim, double out[14]);

/* Write a read-back field (VFLB_FIELD_*) as FP64 into the caller's device
 * array of n doubles (n must equal the field size). */
vflb_status vflb_read(vflb_sim *sim, int field, double *dev_dst, size_t n);

/* vflb_read restricted to a box of size[0] x size[1] x size[2] nodes with
 * origin lo (size[2] = 1, lo[2] = 0 in 2D): component-major, x fastest
 * within the box; n = width of the field x box nodes.  Coordinates wrap on
 * periodic axes; on a wall axis the box must lie inside the lattice
 * (EINVAL otherwise). */
vflb_status vflb_read_box(vflb_sim *sim, int field, const int lo[3],
                          const int size[3], double *dev_dst, size_t n);

/* Checkpoint: vflb_state_size() bytes describe the full state (populations,
 * auxiliary fields, time level).  vflb_save copies it into a caller device
 * blob, vflb_load restores it (same lattice, size and storage). */
vflb_status vflb_state_size(const vflb_sim *sim, size_t *bytes);
vflb_status vflb_save(vflb_sim *sim, void *dev_blob, size_t n);
vflb_status vflb_load(vflb_sim *sim, const void *dev_blob, size_t n);

/* Block height of the step kernel: D2Q9 tiles of 64 x tile_y nodes,
 * tile_y in {4, 8, 16}; D3Q19 columns of 32 x tile_y nodes, tile_y in
 * {4, 8} (4 only with 16-bit storage).  0 restores the built-in choice.
 * EINVAL for other values.  Results do not depend on it (bitwise for
 * D2Q9). */
vflb_status vflb_set_tile(vflb_sim *sim, int tile_y);

/* Bandwidth probe: copies nbytes (a multiple of 16) from src to dst, both
 * device pointers 16-byte aligned, with a plain streaming kernel on
 * hip_stream.  Not part of the method: it measures the achievable HBM copy
 * rate and calibrates hardware byte counters against a transfer of known
 * size.  EINVAL on bad sizes or alignment. */
vflb_status vflb_stream_copy(const void *src, void *dst, size_t nbytes,
                             void *hip_stream);

/* Counter calibration copies: copies nbytes from src to dst (device
 * pointers) on hip_stream with one access kind of the step kernels, so that
 * hardware byte counters can be converted into bytes per kind.  kind 0:
 * non-temporal 16-byte loads and stores (vflb_stream_copy); 1: plain
 * 16-byte loads and stores; 2: plain 4-byte loads and stores; 3: 16-byte
 * loads through LDS-DMA (global_load_lds), non-temporal 16-byte stores.
 * nbytes and both pointers must be multiples of 16 (of 4 for kind 2).
 * Not part of the method.  EINVAL on a bad kind, size or alignment. */
vflb_status vflb_copy_probe(const void *src, void *dst, size_t nbytes, int kind,
                            void *hip_stream);

/* Settling towards prescribed fields (D2Q9): nsteps steps in which every
 * collision takes the FP32 device fields u [2][N] and tau [3][N], stored
 * back to back at dev_targets, in place of the state's own moment u (flags
 * VFLB_SETTLE_U) and/or A (VFLB_SETTLE_A); the pressure follows from the
 * populations.  After an equilibrium-only initialisation this builds the
 * non-equilibrium parts of f and h and a consistent pressure before the
 * real run (with both flags: the iterative initialisation of Mei, Luo,
 * Lallemand and d'Humieres, 2006, which needs a divergence-free u; with A
 * alone the flow adjusts to the prescribed stress).  The time level
 * advances by nsteps.  On a batch instance only right after its
 * initialisation.  EINVAL for other flags or a D3Q19 lattice. */
enum { VFLB_SETTLE_U = 1, VFLB_SETTLE_A = 2 };
vflb_status vflb_settle(vflb_sim *sim, const float *dev_targets,
                        int64_t nsteps, int flags);

/* Release the handle (not the caller's buffers).  Ignored for the
 * instances of a batch, which the batch owns. */
void vflb_destroy(vflb_sim *sim);

/* Message of the last failed call on sim (or of the last failed
 * vflb_create when sim is NULL); never NULL. */
const char *vflb_last_error(const vflb_sim *sim);

/* ------------------------------------------------------------------ batches
 * An ensemble of independent D2Q9 lattices of different sizes and
 * parameters advanced together: every step is one persistent launch whose
 * workgroups walk a flattened table of (instance, 64 x tile_y tile)
 * entries, so small lattices do not each pay a launch and the GPU stays
 * full.  Each tile runs the same per-node arithmetic as vflb_step, so an
 * instance takes bitwise the values it would take alone.  Instances are
 * configured, initialised and read through vflb_sim handles
 * (vflb_batch_instance) with the single-lattice calls; stepping belongs to
 * the batch.  Every call enqueues on the batch's stream.
 */

/* Outcome per instance of vflb_batch_run_until. */
enum {
  VFLB_RUN_ACTIVE = 0,    /* still running (not returned by run_until)       */
  VFLB_RUN_CONVERGED = 1, /* residual fell below tol                         */
  VFLB_RUN_CAPPED = 2,    /* reached its step cap first                      */
  VFLB_RUN_UNSTABLE = 3,  /* a non-finite moment appeared                    */
  VFLB_RUN_SKIPPED = 4    /* was inactive when run_until started             */
};

/* Create a batch of n D2Q9 lattices; dims holds n triples (nx, ny, nz),
 * nz ignored.  Storage as for vflb_create.  EINVAL for another lattice or a
 * bad size. */
vflb_status vflb_batch_create(int lattice, int n, const int *dims, int storage,
                              void *hip_stream, vflb_batch **out);

/* Sizes of the VFLB_NBUF device buffers of the whole batch (each holds the
 * instances' buffers back to back plus the batch's tables). */
vflb_status vflb_batch_query_buffers(const vflb_batch *batch,
                                     size_t bytes[VFLB_NBUF]);

/* Hand over the caller-owned buffers; binds every instance to its slice.
 * Instances must be initialised again afterwards. */
vflb_status vflb_batch_bind_buffers(vflb_batch *batch,
                                    void *const dev_ptrs[VFLB_NBUF]);

/* Handle of instance i (owned by the batch; NULL when out of range).  Use
 * it with vflb_set_params, vflb_set_force (not COS_T), vflb_set_boundaries,
 * vflb_set_storage_scale, vflb_init_fields, vflb_reduce, vflb_read,
 * vflb_save and vflb_load; vflb_step, vflb_bind_buffers and vflb_set_tile
 * on it fail. */
vflb_sim *vflb_batch_instance(vflb_batch *batch, int i);

/* Number of instances. */
int vflb_batch_size(const vflb_batch *batch);

/* Tile height of the batched step (4, 8 or 16; 0: built-in 8), and the
 * height in use. */
vflb_status vflb_batch_set_tile(vflb_batch *batch, int tile_y);
int vflb_batch_get_tile(const vflb_batch *batch);

/* Include (active = 1) or leave out (0) instance i from the steps and
 * reductions; a left-out instance keeps its state and time level. */
vflb_status vflb_batch_set_active(vflb_batch *batch, int i, int active);
int vflb_batch_is_active(const vflb_batch *batch, int i);

/* Advance every active instance by nsteps.  The active instances must be
 * initialised and at the same time level (ESTATE otherwise); COS_T forcing
 * is not batched (EINVAL). */
vflb_status vflb_batch_step(vflb_batch *batch, int64_t nsteps);

/* vflb_reduce for every active instance in one pass (synchronises).  out
 * holds 14 doubles per instance, instance-major, laid out as for
 * vflb_reduce; an inactive instance keeps the values of its last
 * reduction (NaN before any).  Non-finite moments are reported in
 * out[14 i + 7], not as an error. */
vflb_status vflb_batch_reduce(vflb_batch *batch, double *out);

/* Run the active instances towards a steady state: a first reduction takes
 * a fresh residual snapshot; then every check_every steps (fewer when a cap
 * is closer) reduce and leave out each instance whose residual R
 * (vflb_reduce out[0], the relative change of u and tau over the interval)
 * fell below tol over a full interval of check_every steps, whose step
 * count reached max_steps[i], or that became non-finite; repeat until none
 * is active.  An interval shortened to stop another instance at its cap
 * never counts as convergence.  The tile table shrinks as instances leave.
 * Per instance: steps_out[i] its time level, resid_out[i] its residual over
 * the last full interval (+inf when none completed; for a skipped instance
 * its last reduction), status_out[i] a VFLB_RUN_* code. */
vflb_status vflb_batch_run_until(vflb_batch *batch, double tol,
                                 int64_t check_every, const int64_t *max_steps,
                                 int64_t *steps_out, double *resid_out,
                                 int *status_out);

/* Choose the tile height of the batched step for the active set: looked up
 * in the text cache file cache_path (NULL: the file named by the
 * environment variable VFLB_AUTOTUNE_CACHE; no file: no cache), keyed by
 * storage, size class, number of active instances and GPU architecture;
 * otherwise measured by timing the candidates 4, 8 and 16, and appended to
 * the cache.  Measuring overwrites the populations: the instances must be
 * initialised afterwards.  *tile_y_out (may be NULL) receives the choice. */
vflb_status vflb_batch_autotune(vflb_batch *batch, const char *cache_path,
                                int *tile_y_out);

/* Release the batch and its instance handles (not the caller's buffers). */
void vflb_batch_destroy(vflb_batch *batch);

/* Message of the last failed call on batch (or of the last failed
 * vflb_batch_create when batch is NULL); never NULL. */
const char *vflb_batch_last_error(const vflb_batch *batch);

/* ---------------------------------------------------------- warm start
 * A learned initial guess for steady states: a Fourier-feature network
 * maps (x/nx, y/ny, ln Wi, beta, ln Re) to the normalised steady fields
 * (u/U, v/U, txx/S, txy/S, tyy/S); vflb_init_from_mlp evaluates it at every
 * node and starts the lattice from the equilibrium of those fields, after
 * which the method itself runs to the steady state.  The network:
 * phi(x) = [sin(2 pi B x), cos(2 pi B x)] with n_freq fixed Gaussian
 * frequencies B (standard deviation sigma), `hidden` tanh layers of
 * `width`, a linear output layer.  Products run on the matrix cores in BF16
 * with FP32 accumulation; master weights and Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8) are FP32; the loss is the mean squared error.  Not part of the
 * paper: a way to reach the steady states faster.
 */
typedef struct {
  int in_dim;     /* inputs per point, 1..8 (5 for the warm start)          */
  int n_freq;     /* Fourier frequencies, multiple of 32 in [32, 256]        */
  int width;      /* hidden width, multiple of 64 in [64, 1024]              */
  int hidden;     /* hidden layers, 1..16                                    */
  int out_dim;    /* outputs per point, 1..64 (5 for the warm start)         */
  int max_batch;  /* rows per train / gradient call, multiple of 64          */
  double sigma;   /* standard deviation of the frequencies                   */
} vflb_mlp_cfg;

enum {
  VFLB_MLP_BUF_PARAMS = 0, /* frequencies, weights, Adam moments, gradients */
  VFLB_MLP_BUF_WORK = 1,   /* activations of max_batch rows, partial sums    */
  VFLB_MLP_NBUF = 2
};

/* Create a network (EINVAL for a configuration outside the ranges above);
 * work is enqueued on hip_stream. */
vflb_status vflb_mlp_create(const vflb_mlp_cfg *cfg, void *hip_stream,
                            vflb_mlp **out);
vflb_status vflb_mlp_query_buffers(const vflb_mlp *mlp,
                                   size_t bytes[VFLB_MLP_NBUF]);
/* Caller-owned device buffers (256-byte aligned); parameters must be set
 * (vflb_mlp_init or vflb_mlp_set_params) afterwards. */
vflb_status vflb_mlp_bind_buffers(vflb_mlp *mlp,
                                  void *const dev_ptrs[VFLB_MLP_NBUF]);

/* Number of parameters in the flat host order used below: the
 * frequencies [n_freq][in_dim], then per layer W [out][in] and b [out]. */
size_t vflb_mlp_param_count(const vflb_mlp *mlp);

/* Seeded initial parameters (SplitMix64): frequencies N(0, sigma^2),
 * Glorot-uniform weights, zero biases; resets Adam. */
vflb_status vflb_mlp_init(vflb_mlp *mlp, uint64_t seed);

/* Host copies of the parameters (n = vflb_mlp_param_count); set resets
 * Adam.  Both synchronise. */
vflb_status vflb_mlp_set_params(vflb_mlp *mlp, const float *host, size_t n);
vflb_status vflb_mlp_get_params(vflb_mlp *mlp, float *host, size_t n);

/* Network outputs y [n][out_dim] for inputs x [n][in_dim] (FP32 device
 * arrays; any n, processed max_batch rows at a time). */
vflb_status vflb_mlp_forward(vflb_mlp *mlp, const float *dev_x, float *dev_y,
                             int64_t n);

/* Gradient of the loss on n <= max_batch rows (targets t [n][out_dim]),
 * in the flat parameter order (zeros for the frequencies, which are not
 * trained), and the loss; no update.  Synchronises. */
vflb_status vflb_mlp_grad(vflb_mlp *mlp, const float *dev_x, const float *dev_t,
                          int64_t n, float *host_grad, double *loss);

/* One Adam step on n <= max_batch rows with learning rate lr; *loss_out
 * (may be NULL, then nothing synchronises) receives the loss before the
 * step. */
vflb_status vflb_mlp_train_step(vflb_mlp *mlp, const float *dev_x,
                                const float *dev_t, int64_t n, float lr,
                                double *loss_out);

/* Train on a data set in device memory: iters Adam steps, each on `rows`
 * (<= max_batch) samples of X [n][in_dim], T [n][out_dim] (FP32) drawn with
 * replacement (sample floor(z n / 2^64) for z the SplitMix64 output at
 * position it * rows + r of the stream seeded with `seed`), learning rate
 * lr (1 + cos(pi it / iters))/2, floored at lr/1000.  The targets are
 * standardised per output (mean and standard deviation over all n samples,
 * FP64) for training, and the standardisation is folded into the output
 * layer at the end, so that the network predicts T itself; the Adam moments
 * are then reset.  With log_every > 0, losses[k] receives the standardised
 * loss of step k * log_every, and one more entry the last step's when
 * (iters - 1) is not a multiple of log_every ((iters - 1)/log_every + 2
 * entries at most).  Synchronises. */
vflb_status vflb_mlp_train(vflb_mlp *mlp, const float *dev_X, const float *dev_T,
                           int64_t n, int64_t rows, int64_t iters, float lr,
                           uint64_t seed, int64_t log_every, double *losses);

/* Initialise a D2Q9 simulation from the network: inputs (x/nx, y/ny,
 * extra[0], extra[1], extra[2]) at every node, u = u_scale (y0, y1),
 * tau = tau_scale (y2, y3, y4), pressure 0.  On a lattice periodic on every
 * axis (sides <= 512), u is projected onto the fields without central
 * divergence (the step's gradient stencil), without mean and without the
 * Nyquist lines kx = pi, ky = pi: a periodic lattice conserves the total
 * momentum (the force permitting) and, up to sign, the momentum of the
 * alternating (-1)^x and (-1)^y components, so a start from rest has none of
 * either.  With walls, the alternating component along each periodic axis
 * of even length is removed (its momentum is kept up to sign there too).
 * The conformation tensor A = I + lambda tau / eta_p is kept positive
 * definite (eigenvalues raised to at least 0.05).  Then as vflb_init_fields,
 * followed by settle_steps settling steps towards those fields with
 * settle_flags (as vflb_settle; ignored when settle_steps is 0).  The
 * simulation's residual snapshot buffer serves as scratch; both handles must
 * use the same stream. */
vflb_status vflb_init_from_mlp(vflb_sim *sim, vflb_mlp *mlp,
                               const double extra[3], double u_scale,
                               double tau_scale, int64_t settle_steps,
                               int settle_flags);

void vflb_mlp_destroy(vflb_mlp *mlp);
const char *vflb_mlp_last_error(const vflb_mlp *mlp);

#ifdef __cplusplus
}
#endif
#endif /* VFLB_H */
