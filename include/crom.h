/*
 * crom.h - C interface of the MI355X (gfx950) library for the latent time
 * step of Continuous Reduced-Order Modeling (CROM, Chen et al., ICLR 2023,
 * arXiv 2206.02607).
 *
 * The method represents a PDE field f(x, t) by a neural field g(x, q(t)):
 * an MLP over the concatenation of a spatial point x (m values) and a latent
 * vector q (r values) with `depth` hidden ELU layers of equal `width` and a
 * linear output layer of d values (Sec. "Manifold Construction", Sec.
 * "Network Details").  One latent step q_n -> q_{n+1} has three stages
 * (Sec. "Method: Latent Space Dynamics", Alg. "Latent-space dynamics"):
 *   1. network inference at a small set of integration samples, with the
 *      spatial derivatives and the latent Jacobian dg/dq taken through the
 *      network by the forward chain rule (Alg. "Network gradient");
 *   2. explicit time stepping of the exact PDE at the samples
 *      (eqs. "discrete-time", "time-integration");
 *   3. network inversion: q_{n+1} minimises sum_j |g(y_j, q) - f_{n+1}(y_j)|^2
 *      (eq. "invert") by Gauss-Newton with backtracking line search
 *      (Sec. "Network Inversion") or by one linearised normal-equation solve
 *      (Sec. "Linearization").
 *
 * Conventions for every call below
 *   - Array pointers are DEVICE pointers owned by the caller unless a
 *     parameter says "host".  Nothing here allocates device memory; scratch
 *     space comes from a caller-owned workspace sized by a *_workspace call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call only enqueues work on it and returns; none synchronises,
 *     so the calls can be captured into a HIP graph.
 *   - Argument errors (bad sizes, unsupported shapes, NULL pointers where
 *     one is required, too small a workspace) are detected on the host and
 *     returned before anything is enqueued; crom_last_error() then holds a
 *     message.  A failed launch returns CROM_ERR_HIP.  Numerical outcomes of
 *     the inversion (singular system, non-finite values, line-search
 *     failure) are reported per instance in device memory (crom_step_info).
 *   - Layouts are row-major and fully packed; the indices are listed with
 *     each argument, slowest first.
 *   - Supported decoder shapes (m, r, d, width): (1, 3, 1, 32),
 *     (2, 8, 1, 128), (2, 16, 1, 128), (3, 16, 3, 256); depth >= 1.  Other
 *     shapes return CROM_ERR_UNSUPPORTED.
 */
#ifndef CROM_H
#define CROM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CROM_OK = 0,
  CROM_ERR_INVALID_ARG = 1,
  CROM_ERR_UNSUPPORTED = 2,
  CROM_ERR_WORKSPACE = 3,
  CROM_ERR_HIP = 4
} crom_status;

/* Arithmetic of the hidden-to-hidden layers.
 *   FP32       FP32 operands and accumulation.
 *   BF16       matrix-core products with FP32 accumulation.  Latent-tangent
 *              columns (dg/dq) use bfloat16 operands (round to nearest
 *              even).  Value, x-tangent and second-derivative columns, and
 *              the decoder differences the inversion's line search
 *              evaluates, carry each operand as a sum of two bfloat16
 *              numbers (hi + lo) and take three products (hi*hi + hi*lo +
 *              lo*hi), about 16 significant bits: the Laplacian feeds the
 *              PDE update and the line search compares nearby values.
 *   BF16_PURE  every column with plain bfloat16 operands (precision study;
 *              values then carry errors of order 1e-2).
 *   BF16X3     every column with split hi + lo operands.
 * The input layer, the ELU epilogues, the derivative recurrences and the
 * output layer are FP32 in every mode; the latent fold q -> W1q q + b1 is
 * accumulated in FP64.  Inside crom_step, dg/dq comes from an adjoint pass
 * (one column per output back through the layers, transposed weights) for
 * depths 2..6, in the latent-tangent arithmetic above; each layer's ELU
 * slope is kept for it in FP32 (FP32, BF16X3) or as a half-precision value
 * (BF16, BF16_PURE: relative error below 2^-10).  The decode calls form
 * dg/dq by forward tangent columns. */
enum { CROM_PREC_FP32 = 0, CROM_PREC_BF16 = 1, CROM_PREC_BF16_PURE = 2, CROM_PREC_BF16X3 = 3 };

/* Second spatial derivatives requested from crom_decode_jac. */
enum {
  CROM_D2_NONE = 0,      /* none                                           */
  CROM_D2_LAPLACIAN = 1, /* sum_i d2g/dx_i^2 : [P][d]                      */
  CROM_D2_HESSIAN = 2    /* upper triangle i <= j, row-major : [P][d][m(m+1)/2] */
};

/* Decoder description.
 * params: FP32, natural layout, layer by layer for l = 1 .. depth+1:
 *   W_l [n_l][n_{l-1}] row-major, then b_l [n_l], with n_0 = m + r
 *   (input order [x; q]: x first), n_1..n_depth = width, n_{depth+1} = d.
 *   The output layer is linear.
 * act: the hidden layers' activation (Sec. "Network Details": ELU or
 *   SIREN):
 *   CROM_ACT_ELU   ELU with alpha = 1 (ELU(z) = z for z > 0, e^z - 1
 *                  otherwise; z = 0 takes the exponential branch)
 *   CROM_ACT_SINE  sin(z), the SIREN layer with its frequency omega_0
 *                  folded into W_l and b_l (sin(omega_0 (W a + b)) is
 *                  sin(W' a + b') with W' = omega_0 W, b' = omega_0 b).
 *                  Supported by the decode calls and the heat step for
 *                  the (1, 3, 1, 32) and (2, 8, 1, 128) shapes in FP32 and
 *                  BF16, and by the training calls in the bfloat16 modes
 *                  (the forward stores cos(z) beside sin(z) for the
 *                  backward); other calls return CROM_ERR_UNSUPPORTED.
 * packed: the fragment-ordered copy of the hidden-to-hidden weights, and
 *   of their transposes (for the reverse pass of the latent Jacobian), that
 *   crom_net_pack writes (crom_net_packed_bytes long).  It must be
 *   refreshed after params change. */
enum { CROM_ACT_ELU = 0, CROM_ACT_SINE = 1 };
typedef struct {
  int32_t m, r, d, width, depth, precision, act, _pad;
  const float* params;
  const void* packed;
} crom_net;

/* Number of FP32 values in `params` for the given shape. */
size_t crom_net_param_count(int32_t m, int32_t r, int32_t d, int32_t width, int32_t depth);

/* Bytes of the packed buffer for net->precision (0 on invalid shape). */
size_t crom_net_packed_bytes(const crom_net* net);

/* Write the packed hidden-layer weights of net->params into `packed`
 * (device, crom_net_packed_bytes bytes) in net->precision. */
crom_status crom_net_pack(const crom_net* net, void* packed, void* stream);

/* Decoder values g(x_p, q) (Sec. "Step 1: Network Inference").
 * x [P][m] FP32 points, q [r] FP64 latent, g [P][d] FP32 out.  P >= 0. */
crom_status crom_decode(const crom_net* net, const float* x, int64_t P, const double* q,
                        float* g, void* stream);

/* Values with any subset of the derivative columns, all from one forward
 * pass of value and tangents through the layers (Alg. "Network gradient",
 * extended to second order in x and to the latent directions):
 *   g    [P][d]                values (required)
 *   dgdx [P][d][m]             dg/dx (NULL = not computed)
 *   d2g  per d2_mode           see CROM_D2_* (NULL iff d2_mode == NONE)
 *   dgdq [P][d][r]             latent Jacobian dg/dq (NULL = not computed)
 * d2_mode != NONE needs dgdx's columns internally but dgdx may still be NULL. */
crom_status crom_decode_jac(const crom_net* net, const float* x, int64_t P, const double* q,
                            int32_t d2_mode, float* g, float* dgdx, float* d2g, float* dgdq,
                            void* stream);

/* Spatial derivatives only: crom_decode_jac with dgdq = NULL. */
crom_status crom_decode_jac_x(const crom_net* net, const float* x, int64_t P, const double* q,
                              int32_t d2_mode, float* g, float* dgdx, float* d2g, void* stream);

/* Latent Jacobian only (the matrix J of Sec. "Linearization"):
 * crom_decode_jac with d2_mode = NONE and dgdx = NULL. */
crom_status crom_decode_jac_q(const crom_net* net, const float* x, int64_t P, const double* q,
                              float* g, float* dgdq, void* stream);

/* ---------------------------------------------------------------------------
 * Latent step for a batch of independent instances.
 * ------------------------------------------------------------------------- */

enum { CROM_PDE_HEAT = 0, CROM_PDE_NEOHOOKEAN = 1, CROM_PDE_COROTATED_FE = 2, CROM_PDE_PROJECT = 3 };

/* Finite-element stencil of the samples for CROM_PDE_COROTATED_FE (appendix,
 * Sec. "Solid Mechanics / Reduced-order Model": the forces on a sample come
 * from the linear tetrahedra incident on it, so the decoder is evaluated at
 * their vertices, the samples' one-ring).  All arrays are device memory
 * owned by the caller; the host struct is read during the call only.
 *   n_ring        ring vertices of all instances together
 *   max_ring      the largest instance's ring size (sizes the ring decode's
 *                 grid; a larger ring makes its instance NONFINITE)
 *   ring_offsets  [n_inst+1] int64 CSR: instance i's ring vertices are
 *                 ring_offsets[i] .. ring_offsets[i+1]-1 (the samples'
 *                 own vertices included)
 *   ring_X        [n_ring][3] FP32 rest positions (the decoder's inputs)
 *   n_inc         (sample, incident tetrahedron) pairs of all samples
 *   inc_offsets   [total_samples+1] int64 CSR: sample p's pairs are
 *                 inc_offsets[p] .. inc_offsets[p+1]-1; every sample needs
 *                 all of its incident tetrahedra (the lumped mass is their
 *                 volume) and at least one
 *   inc_tets      [n_inc][4] int32: the tetrahedron's vertices as indices
 *                 into its instance's ring range (0 .. ring size - 1), in
 *                 the mesh's vertex order
 *   inc_corner    [n_inc] int8: which of the four is the sample's vertex
 *   ring_u        [n_ring][3] FP32 out: u = g(X, q_n) at the ring vertices
 * Stencil data that breaks these rules (a range that is not CSR, an index
 * outside the ring, a corner outside 0..3) is caught in the kernels and
 * makes the instance NONFINITE; nothing outside the arrays is read. */
typedef struct {
  int64_t n_ring, max_ring, n_inc;
  const int64_t* ring_offsets;
  const float* ring_X;
  const int64_t* inc_offsets;
  const int32_t* inc_tets;
  const int8_t* inc_corner;
  float* ring_u;
} crom_fe_mesh;

/* Builds the stencil of crom_fe_mesh on the host (the same section): for
 * each sample vertex, every tetrahedron that contains it (ascending index),
 * and for each instance its ring, the sorted vertices of those tetrahedra.
 *   n_vert, n_tet, tets  the mesh: tets [n_tet][4] int32 vertex indices
 *   n_inst, sample_offsets [n_inst+1] int64 CSR (sample_offsets[0] = 0),
 *   sample_vert [total] int32  each instance's sample vertices
 * Outputs (host): n_ring, max_ring, n_inc; and, when ring_offsets is not
 * NULL, ring_offsets [n_inst+1], ring_vert [n_ring] (mesh vertex of each
 * ring entry, so ring_X = X[ring_vert]), inc_offsets [total+1], inc_tets
 * [n_inc][4] (ring-local indices) and inc_corner [n_inc].  Call once with
 * ring_offsets = NULL for the sizes, then with arrays of those sizes.
 * Errors: CROM_ERR_INVALID_ARG for an index out of range, a tetrahedron
 * with a repeated vertex, offsets that are not CSR, or a sample vertex that
 * no tetrahedron contains. */
crom_status crom_fe_stencil(int64_t n_vert, int64_t n_tet, const int32_t* tets, int32_t n_inst,
                            const int64_t* sample_offsets, const int32_t* sample_vert, int64_t* n_ring,
                            int64_t* max_ring, int64_t* n_inc, int64_t* ring_offsets, int32_t* ring_vert,
                            int64_t* inc_offsets, int32_t* inc_tets, int8_t* inc_corner);

/* PDE of the instances.
 * HEAT: u_t = nu * Laplacian(u) with forward Euler,
 *   f_{n+1}(y) = g(y, q_n) + dt * nu * Laplacian_x g(y, q_n); coef = nu
 *   [n_inst] FP64 (device).  Needs d == 1.
 * NEOHOOKEAN: elastodynamics rho0 phi_tt = div P(F) + rho0 B of the
 *   displacement u = g(X, q) (phi = X + u, Sec. "Solid Mechanics"), with
 *   F = I + du/dX, P = mu (F - F^-T) + lam ln(det F) F^-T, div P taken
 *   through the decoder's x-Hessian, the velocity from the tangent space
 *   v_n = (dg/dq)(q_n - q_prev)/dt (q_prev NULL: at rest), and symplectic
 *   Euler at the samples: v+ = v_n + dt (div P / rho0 + B), target
 *   u+ = u + dt v+.  coef [n_inst][6] FP64 = lam, mu, rho0, Bx, By, Bz.
 *   Needs m == 3 and d == 3 (the (3, 16, 3, 256) decoder).  A sample with
 *   det F <= 0 makes its instance NONFINITE.
 * COROTATED_FE: the same elastodynamics with corotated linear elasticity
 *   and finite-element forces (appendix, Sec. "Solid Mechanics"): the
 *   decoder gives the deformed positions x = X + g(X, q_n) of the ring
 *   vertices (`mesh`); per incident tetrahedron D_m = [X_a - X_4], F =
 *   I + [u_a - u_4] D_m^-1, R the rotation of the polar decomposition
 *   F = R S, P = 2 mu (F - R) + lam (tr(R^T F) - 3) R (the derivative of the
 *   corotated energy mu |F - R|^2 + lam/2 tr(R^T F - I)^2), vertex forces
 *   [f_1 f_2 f_3] = -(|det D_m| / 6) P D_m^-T, f_4 = -(f_1 + f_2 + f_3);
 *   the force on a sample is the sum over its incident tetrahedra, its
 *   lumped mass rho0 / 4 of their volume; then v+ = v_n + dt (f / m + B)
 *   and u+ = u + dt v+ as for NEOHOOKEAN.  coef [n_inst][6] FP64 = lam,
 *   mu, rho0, Bx, By, Bz.  Needs the (3, 16, 3, 256) decoder and at most
 *   65535 instances.  A tetrahedron with det F <= 0 makes its instance
 *   NONFINITE.
 * PROJECT: no time stepping: the targets are given, coef [total_samples]
 *   FP64 = f(y) at the samples, and the step is the inversion alone (eq.
 *   "invert", Sec. "Network Inversion"): q_{n+1} = argmin |g(Y, q) - f|^2
 *   from q_n (dt is ignored).  Needs d == 1 and m <= 2 (the heat shapes). */
typedef struct {
  int32_t kind, _pad;
  double dt;
  const double* coef;
  const crom_fe_mesh* mesh; /* COROTATED_FE: host pointer; ignored otherwise */
} crom_pde;

/* Inversion options (host struct).
 *   max_iter   >= 1 Gauss-Newton iterations (accepted steps) at most
 *   linearized 1: one normal-equation solve with unit step (Sec.
 *              "Linearization"); 0: Gauss-Newton with line search
 *   ls_max     the line search tries alpha = 1, s, s^2, ..., s^ls_max
 *   tol_step   stop when |alpha delta| or |delta| <= tol_step (1 + |q|)
 *   armijo_c   accept alpha when phi(q + alpha delta) <= phi(q) - c alpha b.delta
 *   ls_shrink  s in (0, 1)
 *   max_rounds evaluation rounds after the first, 0 = enough for max_iter
 *              iterations that each need the longest line search (at most
 *              256).  A round evaluates one line-search trial (or
 *              re-linearises after a shortened step); an instance still
 *              running after the last round ends with CROM_FLAG_MAXITER.
 * The step runs as one persistent kernel whose grid fits on the GPU at
 * once; it loops until every instance has finished. */
typedef struct {
  int32_t max_iter, linearized, ls_max, max_rounds;
  double tol_step, armijo_c, ls_shrink;
} crom_gn_opts;

enum {
  CROM_FLAG_MAXITER = 1,   /* iteration budget used up                      */
  CROM_FLAG_SINGULAR = 2,  /* Cholesky pivot <= 1e-14 * max diag(J^T J)     */
  CROM_FLAG_NONFINITE = 4, /* NaN/Inf in the residual or normal equations   */
  CROM_FLAG_LS_FAIL = 8,   /* no trial step satisfied the Armijo condition  */
  CROM_FLAG_ABORTED = 16,  /* the step kernel gave up waiting on a phase (an
                              internal error; q_next holds the last iterate) */
  CROM_FLAG_INVERTED = 32  /* elastic kinds: det F <= 0 at a sample that is not
                              clamped (no stress there; NONFINITE follows from
                              its NaN targets and q_next = q_n) */
};

/* Per-instance outcome (device memory, written by crom_step). */
typedef struct {
  int32_t flags;    /* CROM_FLAG_* bits                                       */
  int32_t iters;    /* accepted Gauss-Newton steps                            */
  int32_t ls_evals; /* line-search trials examined, in order, up to acceptance */
  int32_t rounds;   /* evaluation rounds after the first that this instance used */
  double obj_first, obj_last; /* 1/2 |f_{n+1} - g(Y, q)|^2 at q_n and at q_{n+1} */
} crom_step_info;

/* Workspace bytes for crom_step with n_inst instances and total_samples
 * samples (host out-parameter `bytes`). */
crom_status crom_step_workspace(const crom_net* net, int32_t n_inst, int64_t total_samples,
                                size_t* bytes);

/* One latent step q_n -> q_{n+1} for every instance.
 *   offsets [n_inst+1] int64  CSR offsets of each instance's samples in y
 *                             (device; non-decreasing, offsets[0] = 0,
 *                             offsets[n_inst] = total_samples, and every
 *                             instance needs r <= d * S_i samples)
 *   y       [total_samples][m] FP32 sample points
 *   clamp   NULL or [total_samples] uint8: 1 = Dirichlet sample, target 0
 *   q_prev  NEOHOOKEAN, COROTATED_FE: NULL or [n_inst][r] FP64, the previous
 *           step's latent (ignored for HEAT)
 *   q_n     [n_inst][r] FP64;  q_next [n_inst][r] FP64 out (must not alias q_n)
 *   info    [n_inst] crom_step_info out
 *   ws      workspace of at least crom_step_workspace bytes, 256-byte aligned
 * The target values f_{n+1} are kept in the workspace and are readable with
 * crom_step_targets after the step. On SINGULAR / NONFINITE / LS_FAIL the
 * instance's q_next holds the last accepted iterate. */
crom_status crom_step(const crom_net* net, const crom_pde* pde, int32_t n_inst,
                      const int64_t* offsets, int64_t total_samples, const float* y,
                      const uint8_t* clamp, const double* q_prev, const double* q_n, double* q_next,
                      const crom_gn_opts* opts, crom_step_info* info, void* ws, size_t ws_bytes,
                      void* stream);

/* crom_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same step with the same kernels and results, its
 * workspace a library-owned device array of crom_step_static_capacity()
 * bytes (64 MiB) that each GPU the library runs on holds until the process
 * ends.  A step whose crom_step_workspace exceeds it returns
 * CROM_ERR_WORKSPACE before anything is enqueued.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * other host threads) race and must be serialised by the caller; a call
 * needs nothing cleared from the previous one.  The targets and increments
 * of the last step are not exposed (crom_step_targets needs a caller
 * workspace). */
size_t crom_step_static_capacity(void);
crom_status crom_step_static(const crom_net* net, const crom_pde* pde, int32_t n_inst, const int64_t* offsets,
                             int64_t total_samples, const float* y, const uint8_t* clamp, const double* q_prev,
                             const double* q_n, double* q_next, const crom_gn_opts* opts, crom_step_info* info,
                             void* stream);

/* crom_step with a second candidate starting point for the Gauss-Newton
 * inversion (Sec. "Initial Guess for the Nonlinear Solver": where the field
 * changes a lot over one step, a latent from an encoder of the updated field
 * can start the solver closer to the minimum than q_n).
 *   q_init  [n_inst][r] FP64 device, one guess per instance (NULL: crom_step);
 *           must not alias q_next
 * After the first evaluation at q_n, an instance whose Gauss-Newton step at
 * q_n is computable and not negligible spends one evaluation round on its
 * guess (the value and J there); a strictly smaller objective makes the
 * guess the start, otherwise the line search from q_n proceeds exactly as in
 * crom_step (the result is then bit-identical, with one more round).  The
 * linearised variant ignores the guess.  info.obj_first stays the objective
 * at q_n; an accepted guess is not counted in info.iters. */
crom_status crom_step_guess(const crom_net* net, const crom_pde* pde, int32_t n_inst,
                            const int64_t* offsets, int64_t total_samples, const float* y,
                            const uint8_t* clamp, const double* q_prev, const double* q_n,
                            const double* q_init, double* q_next, const crom_gn_opts* opts,
                            crom_step_info* info, void* ws, size_t ws_bytes, void* stream);

/* Device pointer to the FP64 targets f_{n+1} [total_samples][d] inside a
 * workspace used by crom_step (NULL on invalid arguments). */
const double* crom_step_targets(const crom_net* net, int32_t n_inst, int64_t total_samples,
                                const void* ws);

/* Device pointer to the FP64 increments rho_0 = f_{n+1} - g(q_n)
 * [total_samples][d] of the last crom_step in this workspace, formed
 * directly (heat: dt nu Laplacian g; neo-Hookean: dt v_{n+1}; a clamped
 * sample: -g).  NULL on invalid arguments. */
const double* crom_step_increments(const crom_net* net, int32_t n_inst, int64_t total_samples,
                                   const void* ws);

/* ---------------------------------------------------------------------------
 * Full-order FP64 finite-difference heat solver: the snapshot generator, the
 * judge of reduced-order rollouts and the fallback for failed steps (Sec.
 * "Thermodynamics / Full-order Model" and "Image Processing / Full-order
 * Model": 3-point / 5-point Laplacian, forward Euler, boundary held at 0).
 *   dim      1 or 2
 *   shape    host [dim]: nodes per axis (nx) or (nx, ny), boundary included
 *   n_grid   independent fields, stored one after another:
 *            u [n_grid][nx] or [n_grid][nx][ny] (index [i_x][i_y]), FP64
 *   nu       diffusivity: [n_grid] (nu_per_node = 0) or one per node (1)
 *   dx, dt   node spacing (both axes) and substep
 *   steps    substeps; each is u <- u + (dt nu) * Lap_h u on interior nodes,
 *            evaluated in that order without fused multiply-add, and 0 on
 *            the boundary (input boundary values are ignored)
 *   u        in/out; scratch: a second buffer of the same size
 * Stability (nu dt / dx^2 <= 1/2 in 1D, 1/4 in 2D) is the caller's
 * responsibility. */
crom_status crom_fd_heat(int32_t dim, const int64_t* shape, int64_t n_grid, const double* nu,
                         int32_t nu_per_node, double dx, double dt, int64_t steps, double* u,
                         double* scratch, void* stream);

/* ---------------------------------------------------------------------------
 * Training of the manifold parameterisation (Sec. "Manifold Construction",
 * eq. "loss"; Sec. "Training Details").  A batch holds B snapshots u_b of P
 * points with d values each, at the shared points x [P][m].  The encoder
 * maps a snapshot to its latent, q_b = E2 ELU(E1 u_b + c1) + c2, the decoder
 * is evaluated at every (snapshot, point) pair, and the loss is
 *   L = mean over b, p, o of (g(x_p, q_b)_o - u_b(x_p)_o)^2.
 * Gradients are the exact reverse-mode derivatives of L (written out layer
 * by layer, no tape).  In CROM_PREC_FP32 every product is FP32; in the
 * bfloat16 modes the hidden-layer products, the encoder's first layer and
 * the stored activations use bfloat16 operands with FP32 accumulation, and
 * the first and output layers, the loss and every sum over points are
 * FP32/FP64.  Sums run in a fixed order: results are deterministic.
 * The decoder must have one of the compiled shapes; the packed weights are
 * not used (crom_train_step refreshes them when given a buffer).
 * ------------------------------------------------------------------------- */

/* Encoder description: n_in = P * d (a snapshot [P][d], point-major), r =
 * the net's r, params FP32.
 * CROM_ENC_DENSE: q = E2 ELU(E1 u + c1) + c2, params
 *   E1 [hidden][n_in], c1 [hidden], E2 [r][hidden], c2 [r].
 * CROM_ENC_CONV (Sec. "Network Details"): the snapshot as a 1D vector of
 *   P points with d channels; 1D convolutions of kernel 6 and stride 4 with
 *   d output channels (no padding, L -> (L - 6) / 4 + 1, ELU) applied while
 *   the result keeps at least 32 values (L d >= 32); the last one's output
 *   flattened channel-major (value (c, j) at c L + j); then
 *   h = ELU(E1 . + c1) of `hidden` values (the paper's 32) and
 *   q = E2 h + c2.  Params: per convolution W [d][d][6], b [d]; then
 *   E1 [hidden][L d], c1 [hidden], E2 [r][hidden], c2 [r].  Needs room for
 *   one convolution.  Its arithmetic is FP32 in every precision mode. */
enum { CROM_ENC_DENSE = 0, CROM_ENC_CONV = 1 };
typedef struct {
  int32_t n_in, hidden, r, kind;
  float* params;
} crom_encoder;

/* Number of FP32 values in a dense encoder's params (0 on invalid sizes). */
size_t crom_encoder_param_count(int32_t n_in, int32_t hidden, int32_t r);

/* Number of FP32 values in a convolutional encoder's params for P points
 * with d channels (0 on invalid sizes or when no convolution fits). */
size_t crom_conv_encoder_param_count(int64_t P, int32_t d, int32_t hidden, int32_t r);

/* Workspace bytes for crom_train_grads / crom_train_step with B snapshots
 * (host out-parameter). */
crom_status crom_train_workspace(const crom_net* net, const crom_encoder* enc, int32_t B,
                                 size_t* bytes);

/* Loss and gradients for one batch.
 *   u         [B][P][d] FP32 snapshots;  x [P][m] FP32 points
 *   grad_dec  [crom_net_param_count] out, the decoder's natural layout
 *   grad_enc  [crom_encoder_param_count] out, the encoder's layout
 *   loss      [1] FP32 out;  q_out NULL or [B][r] FP32 out (the latents)
 *   ws        workspace of crom_train_workspace bytes */
crom_status crom_train_grads(const crom_net* net, const crom_encoder* enc, const float* u,
                             const float* x, int32_t B, float* grad_dec, float* grad_enc,
                             float* loss, float* q_out, void* ws, size_t ws_bytes, void* stream);

/* Adam (Kingma & Ba) with bias correction on n FP32 values, step t >= 1:
 *   m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
 *   p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * m and v start at 0 (caller-owned, n values each). */
crom_status crom_adam_step(float* params, const float* grad, float* m, float* v, int64_t n,
                           int64_t t, float lr, float beta1, float beta2, float eps,
                           void* stream);

/* One training step: crom_train_grads, then Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8) on the FP32 master parameters of the decoder (net->params, which
 * this call updates in place) and of the encoder, then, when `packed` is not
 * NULL, crom_net_pack into it.  dec_grad/enc_grad are caller buffers of the
 * gradient sizes; dec_m, dec_v, enc_m, enc_v are the Adam moments. */
crom_status crom_train_step(const crom_net* net, void* packed, float* dec_grad, float* dec_m,
                            float* dec_v, const crom_encoder* enc, float* enc_grad, float* enc_m,
                            float* enc_v, int64_t t, const float* u, const float* x, int32_t B,
                            float lr, float* loss, void* ws, size_t ws_bytes, void* stream);

/* Standardization of the training data (Sec. "Training Details": the
 * training fields have zero mean and unit variance, and the coordinates of
 * ELU networks are standardized as well).  Population moments: the mean and
 * the root mean squared deviation over every value.  Device struct. */
typedef struct {
  double u_mean, u_std;        /* over every value of every snapshot           */
  double x_mean[3], x_std[3];  /* per coordinate axis over the nodes; axes past
                                  m hold 0 and 1                             */
} crom_standardization;

/* Moments of the snapshots u [n_u] FP64 (any layout: every value counts
 * alike) and of the nodes x [P][m] FP32, written to s (device).  One
 * workgroup, fixed summation order (deterministic). */
crom_status crom_standardization_of(const double* u, int64_t n_u, const float* x, int64_t P, int32_t m,
                                    crom_standardization* s, void* stream);

/* u_s [n_u] FP32 = (u - u_mean) / u_std and x_s [P][m] FP32 =
 * (x - x_mean) / x_std, evaluated in FP64 and rounded once.  Either part may
 * be skipped with n_u = 0 or P = 0. */
crom_status crom_standardize(const crom_standardization* s, const double* u, int64_t n_u, float* u_s,
                             const float* x, int64_t P, int32_t m, float* x_s, void* stream);

/* Fold the standardization into networks trained on standardized data, in
 * place, so that they act on physical points and fields:
 *   g(x, q) = u_std g_s((x - x_mean) / x_std, q) + u_mean,   e(u) = e_s((u - u_mean) / u_std).
 * The decoder's layer 1 coordinate columns divide by x_std and its bias
 * loses W1x (x_mean / x_std); the output layer's weights and bias scale by
 * u_std and the bias gains u_mean; the encoder's first layer (dense E1, or
 * the first convolution) divides by u_std and its bias loses
 * u_mean / u_std times the sum of each output's weights.  net->params (FP32)
 * and enc->params are updated in place (enc may be NULL: decoder only); the
 * packed weights must be refreshed with crom_net_pack afterwards. */
crom_status crom_fold_standardization(const crom_net* net, const crom_encoder* enc, const crom_standardization* s,
                                      void* stream);

/* The whole training state in one caller-owned device blob, so that a
 * training run is checkpointed and resumed by copying it (together with the
 * Adam step t, which the caller keeps): the FP32 decoder parameters (the
 * natural layout), their gradient buffer and Adam moments m and v, then the
 * same four for the encoder, each section starting on a 256-byte boundary
 * at the offsets below.  The blob is 256-byte aligned. */
typedef struct {
  size_t dec_params, dec_grad, dec_m, dec_v, enc_params, enc_grad, enc_m, enc_v, total;
} crom_train_state_layout;

/* Section offsets of the blob for this decoder and encoder (host out). */
crom_status crom_train_state_offsets(const crom_net* net, const crom_encoder* enc, crom_train_state_layout* out);

/* Bytes of the blob (0 on invalid arguments). */
size_t crom_train_state_bytes(const crom_net* net, const crom_encoder* enc);

/* crom_train_step on a state blob: the parameters, gradients and moments
 * are the blob's sections (net->params and enc->params are ignored); packed
 * (NULL or crom_net_packed_bytes) receives the packed decoder weights. */
crom_status crom_train_step_state(const crom_net* net, const crom_encoder* enc, void* state, void* packed, int64_t t,
                                  const float* u, const float* x, int32_t B, float lr, float* loss, void* ws,
                                  size_t ws_bytes, void* stream);

/* Encoder forward only: q [B][r] FP32 = E2 ELU(E1 u_b + c1) + c2 for
 * snapshots u [B][P][d], in the arithmetic crom_train_grads uses for the
 * net's precision (the latent of an initial field, Sec. "Manifold
 * Construction").  ws: crom_encode_workspace bytes. */
crom_status crom_encode_workspace(const crom_net* net, const crom_encoder* enc, int32_t B,
                                  size_t* bytes);
crom_status crom_encode(const crom_net* net, const crom_encoder* enc, const float* u, int32_t B,
                        float* q, void* ws, size_t ws_bytes, void* stream);

/* Encoder-based initial guess for the heat step (Sec. "Initial Guess for
 * the Nonlinear Solver"): the updated field at every node,
 * f_i = g(x, q_n,i) + dt nu_i Laplacian g(x, q_n,i), FP32, passed through the
 * training encoder (crom_encode's arithmetic), as FP64 latents for
 * crom_step_guess.
 *   nodes [P][m] FP32, the full node set the encoder was trained on (its
 *   n_in = P * d); q_n [n_inst][r] FP64; nu [n_inst] FP64 (device);
 *   q_guess [n_inst][r] FP64 out; ws: crom_heat_guess_workspace bytes.
 * Needs d == 1 and m <= 2. */
crom_status crom_heat_guess_workspace(const crom_net* net, const crom_encoder* enc, int32_t n_inst, int64_t P,
                                      size_t* bytes);
crom_status crom_heat_guess(const crom_net* net, const crom_encoder* enc, const float* nodes, int64_t P,
                            int32_t n_inst, const double* q_n, const double* nu, double dt, double* q_guess,
                            void* ws, size_t ws_bytes, void* stream);

/* Full-order fallback for failed heat steps (Sec. "Thermodynamics /
 * Full-order Model", "Image Processing / Full-order Model"): for each listed
 * instance, its last good latent q_last is decoded at every node of the
 * (nx, ny) grid, the field is advanced by `substeps` steps of crom_fd_heat
 * with that instance's diffusivity, and the result is projected back onto
 * the decoder at every node by the method's own inversion (crom_step with
 * CROM_PDE_PROJECT from q_last, Gauss-Newton with `opts`), giving q_next
 * (FP64).  Other instances are not touched.
 *   nodes    [nx * ny][2] FP32, node (i_x, i_y) at index i_x * ny + i_y;
 *            boundary nodes are held at 0
 *   inst     HOST [n_fail] distinct instance indices in [0, n_inst)
 *   q_last   [n_inst][r] FP64, nu [n_inst] FP64, q_next [n_inst][r] FP64
 *   info     NULL or [n_inst] crom_step_info: the listed instances' entries
 *            receive the projection's outcome
 *   ws       crom_heat_fallback_workspace bytes
 * Needs m == 2 and d == 1.  The caller picks the instances from
 * crom_step_info (SINGULAR, NONFINITE, LS_FAIL), which makes the fallback a
 * host decision (one read of the flags). */
crom_status crom_heat_fallback_workspace(const crom_net* net, int32_t n_fail, int64_t nx, int64_t ny, size_t* bytes);
crom_status crom_heat_fallback(const crom_net* net, const float* nodes, int64_t nx, int64_t ny, double dx,
                               int32_t n_inst, int32_t n_fail, const int32_t* inst, const double* q_last,
                               const double* nu, double dt_fd, int64_t substeps, const crom_gn_opts* opts,
                               double* q_next, crom_step_info* info, void* ws, size_t ws_bytes, void* stream);

/* Vector-Jacobian product of the decoder (the backward of crom_decode over
 * B latents): with G[b][p][o] = g(x_p, q_b)_o and a cotangent dg [B][P][d],
 *   grad_params = sum dg . dG/dparams   (natural layout, overwritten)
 *   grad_q [B][r] = sum over p, o of dg . dG/dq_b.
 * q [B][r] FP32.  The forward activations are recomputed, in the net's
 * precision, into the workspace (crom_decode_vjp_workspace bytes). */
crom_status crom_decode_vjp_workspace(const crom_net* net, int32_t B, int64_t P, size_t* bytes);
crom_status crom_decode_vjp(const crom_net* net, const float* x, int64_t P, const float* q,
                            int32_t B, const float* dg, float* grad_params, float* grad_q,
                            void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Robust selection of the integration samples (Appendix "Robust Sampling",
 * Alg. "Robust sampling"): a greedy precomputation that grows a set M of
 * integration samples, drawn from the P nodes x_i of the full-order
 * discretisation, until the latent dynamics run with M reproduce the
 * full-order solution of every training parameter mu_k at the final time.
 *
 * Residual vector of a set (the algorithm's Calculate_Residual): with
 * q_end(mu_k) the latent after the rollout of parameter k with samples M,
 *   res[i] = sum_k | g(x_i, q_end(mu_k)) - f(x_i, t_end; mu_k) |_2
 * and its metric (the algorithm's Metric) mean_i res[i] + max_i res[i].
 * Rankings: a NaN residual or metric ranks above every number in the
 * largest-residual ranking and below every number in the smallest-metric
 * choice; ties go to the lower node index and to the earlier candidate. */

/* Residual vectors and metrics of n_set sample sets whose final latents are
 * given (the decode of every node and the comparison run fused in one
 * kernel; the decoded fields are not stored).
 *   nodes  [P][m] FP32 node coordinates
 *   q      [n_set][n_mu][r] FP64 final latents (set s, parameter k)
 *   ref    [n_mu][P][d] FP64 full-order field at the final time
 *   res    [n_set][P] FP64 out, metric [n_set] FP64 out (may be NULL)
 * Sum over k in increasing order; P >= 1, n_set >= 1, n_mu >= 1. */
crom_status crom_sampling_residual(const crom_net* net, const float* nodes, int64_t P, int32_t n_set,
                                   int32_t n_mu, const double* q, const double* ref, double* res,
                                   double* metric, void* stream);

/* The n nodes outside the set with the largest residuals (the algorithm's
 * Max_Indices), in ranking order.
 *   res    [P] FP64 residual vector
 *   member NULL or [P] uint8: 1 = node already in the set (never a candidate)
 *   cand   [n] int32 out; entries past the number of eligible nodes are -1
 * 1 <= n <= CROM_SAMPLING_MAX_TRY. */
enum { CROM_SAMPLING_MAX_TRY = 64 };
crom_status crom_sampling_candidates(const double* res, int64_t P, const uint8_t* member, int32_t n,
                                     int32_t* cand, void* stream);

/* Options of the greedy loop (host struct).
 *   n_try        candidates per round, 1 .. CROM_SAMPLING_MAX_TRY (the
 *                appendix uses 10)
 *   max_samples  the loop also stops when the set holds this many nodes
 *                (n_init <= max_samples <= P)
 *   n_steps      latent steps from the initial latents to the final time
 *   target       the loop stops once the metric is below this value */
typedef struct {
  int32_t n_try, max_samples;
  int64_t n_steps;
  double target;
} crom_sampling_opts;

/* Outcome of crom_robust_sampling (host struct). */
typedef struct {
  int32_t n_samples; /* nodes in the returned set                          */
  int32_t reached;   /* 1 when its metric is below the target              */
  int32_t rounds;    /* greedy rounds run (nodes added)                    */
  int32_t _pad;
  double metric;     /* metric of the returned set                         */
} crom_sampling_result;

/* Workspace bytes of crom_robust_sampling (host out-parameter `bytes`). */
crom_status crom_sampling_workspace(const crom_net* net, int32_t pde_kind, int32_t n_mu, int64_t P,
                                    const crom_sampling_opts* opts, size_t* bytes);

/* The greedy loop.  Each round runs, as one batch of crom_step calls, the
 * rollouts of n_try x n_mu instances (candidate c with parameter k), each
 * with the samples M + {candidate}, then their residual vectors; the host
 * reads the n_try metrics back (one synchronisation per round) and appends
 * the best candidate.  The residual vector of the chosen set is kept as the
 * next round's (it is the same computation).
 *   pde         kind, dt and coef [n_mu][n_coef] per training parameter
 *               (as for crom_step; every instance of parameter k uses row k)
 *   nodes       [P][m] FP32;  node_clamp NULL or [P] uint8 (Dirichlet node:
 *               target 0 when it is a sample)
 *   ref         [n_mu][P][d] FP64 full-order field at step n_steps
 *   q0          [n_mu][r] FP64 initial latents (neo-Hookean: at rest)
 *   gn          inversion options of every step (host)
 *   samples     host [max_samples] int32: in, the first n_init entries are
 *               the initial set (distinct node indices); out, the set in the
 *               order the nodes joined it
 *   result      host out
 *   trace_cand, trace_metric  NULL or host [max_samples - n_init][n_try]:
 *               each round's candidates and their metrics (-1 / NaN past
 *               the round's candidate count)
 * The initial set needs r <= d * n_init.  A rollout step that fails keeps
 * its last iterate (crom_step's convention); the residual then measures
 * it.  Unlike the other calls this one synchronises the stream every
 * round. */
crom_status crom_robust_sampling(const crom_net* net, const crom_pde* pde, int32_t n_mu, const float* nodes,
                                 int64_t P, const uint8_t* node_clamp, const double* ref, const double* q0,
                                 const crom_gn_opts* gn, const crom_sampling_opts* opts, int32_t* samples,
                                 int32_t n_init, crom_sampling_result* result, int32_t* trace_cand,
                                 double* trace_metric, void* ws, size_t ws_bytes, void* stream);

/* Benchmark support.  crom_kernel_timer(1) starts a record on the calling
 * host thread (releasing any earlier one): every later crom_step on this
 * thread then records a pair of HIP events on its stream that brackets the
 * step's compute kernels: the persistent step kernel, every round of the
 * batched Gauss-Newton path, or the linearised path's evaluation kernel
 * (its small solve kernel is left out).  The set-up launch is never inside
 * a pair.  crom_kernel_timer(0) stops recording.  crom_kernel_timer_read
 * waits for the recorded events, returns the summed milliseconds of the
 * pairs and their number, and, when recording has stopped, destroys the
 * events. */
crom_status crom_kernel_timer(int32_t on);
crom_status crom_kernel_timer_read(double* total_ms, int64_t* count);

/* Message describing the last error returned on the calling thread. */
const char* crom_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CROM_H */
