/*
 * liblbm -- semi-Lagrangian off-lattice Boltzmann time step on AMD Instinct
 * MI355X (gfx950).  C ABI.
 *
 * The method is the one of Wilde, Kraemer, Bedrunka, Reith, Foysi, "Cubature
 * rules for weakly and fully compressible off-lattice Boltzmann methods"
 * (arXiv 2101.03982), Sec. 3:
 *   1. streaming: every population f_i is interpolated at its departure point
 *      x - xi_i dt (eq. sl_streaming).  This library interpolates on a uniform
 *      grid with a tensor product of 1D Lagrange polynomials through n
 *      neighbouring nodes per axis (the n nodes around the departure point for
 *      even n; for odd n the n nodes centred on the nearest node, the arrival
 *      side winning an exact tie);
 *   2. moments: rho = sum f_i, rho u = sum xi_i f_i (eqs. density, momentum)
 *      and, in the compressible model, 2 rho C_v theta =
 *      sum(|xi_i - u|^2 f_i / T0 + g_i) with T0 = c_s^2;
 *   3. equilibrium: the Hermite expansion of App. A truncated at order N,
 *      g^eq = theta (2 C_v - D) f^eq;
 *   4. BGK relaxation f <- f - (f - f^eq)/tau (lattice Boltzmann equation),
 *      tau = 1/2 + (tau_ref - 1/2)/(rho theta) in the compressible model
 *      (tau = mu/(c_s^2 dt P) + 1/2 with P = rho theta).
 * Velocity sets: D2Q9, D2Q19, D2Q25, D3Q13, D3Q21, D3Q27, D3V27, D3Q45
 * (Table tab:sets, Tables tab:d3q13 and tab:d3q21, Apps. C-E).
 *
 * Conventions shared by every call:
 *  - Return value: LBM_OK (0) or a negative lbm_status.  No call throws or
 *    aborts; lbm_strerror() names the code and lbm_last_error() gives the
 *    message of the most recent failure on the calling thread.
 *  - Population buffers are caller-owned device memory in the layout
 *    [A*Q][nz][ny][nx], x fastest, f populations then g populations (A = 2
 *    only in the compressible model), element type by storage: LBM_F64
 *    double holding f_i; LBM_F32 float, LBM_BF16DEV bfloat16 and LBM_F16DEV
 *    IEEE half holding the deviation f_i - r_i from the reference
 *    r_i = w_i (f) or (2 C_v - D) w_i (g), which keeps the storage precision
 *    on the part of f_i that varies.  lbm_state_bytes() gives the size.
 *  - Macroscopic fields (rho, u, theta) are device arrays of the compute type:
 *    double for LBM_F64 storage, float otherwise; u is [D][nz][ny][nx] in the
 *    physical units of dx and dt.
 *  - Device work is enqueued on the context's stream and returns at once;
 *    only lbm_moments() (and lbm_sync()) wait.  Asynchronous kernel failures
 *    surface in the next synchronizing call as LBM_EHIP.  A context is not
 *    thread-safe; use one context per stream.
 *  - Population index order: rows of the printed tables in order, sign
 *    patterns of the non-zero components in lexicographic order with + before
 *    -, first component outermost; "(cyc)" rows expand to (a,b,c), (c,a,b),
 *    (b,c,a); product sets enumerate 1D nodes (0, +a, -a, +b, -b), first axis
 *    outermost.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lbm_status {
  LBM_OK = 0,
  LBM_EINVAL = -1,        /* bad argument: null pointer, size, range, grid too small */
  LBM_ENOMEM = -2,        /* device or host allocation failed */
  LBM_EHIP = -3,          /* HIP runtime error (launch or asynchronous fault) */
  LBM_EUNSUPPORTED = -4,  /* combination not built: set/order/stencil/storage */
  LBM_EDIVERGED = -5      /* NaN, rho <= 0 or theta <= 0 found by lbm_moments */
} lbm_status;

typedef enum lbm_set {
  LBM_D2Q9 = 0, LBM_D2Q19 = 1, LBM_D2Q25 = 2, LBM_D3Q13 = 3,
  LBM_D3Q21 = 4, LBM_D3Q27 = 5, LBM_D3V27 = 6, LBM_D3Q45 = 7
} lbm_set;

typedef enum lbm_storage {
  LBM_F64 = 0,      /* double populations, double arithmetic */
  LBM_F32 = 1,      /* float deviations f - r, float arithmetic */
  LBM_BF16DEV = 2,  /* bfloat16 deviations f - r, float arithmetic */
  LBM_F16DEV = 3    /* IEEE half deviations f - r, float arithmetic */
} lbm_storage;

/* Streaming support (Sec. 3, eq. sl_streaming).  LBM_UNIFORM: equally spaced
 * nodes, a stencil of `stencil` Lagrange nodes around every departure point.
 * LBM_GLC: the paper's own form: every axis is cut into cells of p + 1
 * Gauss-Lobatto-Chebyshev support points, p = stencil - 1, at
 * (c + (1 - cos(pi k / p)) / 2) p dx for node c p + k (neighbouring cells
 * share their end points; dx is the mean node spacing); each node's
 * departure point is interpolated with the polynomial through the points of
 * the cell that holds it.  Built for p = 4 (stencil 5), the weakly
 * compressible model with D2Q9, D3Q13, D3Q21, D3Q27, D3V27 at their
 * workload orders (N = 2; N = 3 for D3V27), LBM_F64 / LBM_F32, periodic axes
 * whose extents are multiples of p, forward steps (no adjoint);
 * LBM_EUNSUPPORTED otherwise. */
typedef enum lbm_support {
  LBM_UNIFORM = 0,
  LBM_GLC = 1
} lbm_support;

typedef enum lbm_boundary {
  LBM_PERIODIC = 0,     /* node indices wrap around */
  LBM_EXTRAPOLATE = 1   /* zeroth-order extrapolation: indices clamp to the edge */
} lbm_boundary;

/* How 16-bit storage rounds each stored value. */
typedef enum lbm_rounding {
  LBM_ROUND_NEAREST = 0,    /* to nearest, ties to even (default) */
  LBM_ROUND_STOCHASTIC = 1  /* 16-bit storage (LBM_EUNSUPPORTED otherwise): up or down with
                               probabilities given by the distance to the two neighbouring
                               values, so the rounding error has mean zero.  The random bits are
                               a hash of the cell, the array, the context's count of steps
                               taken (every lbm_step step and lbm_step_into call advances it)
                               and `seed`: a run repeats exactly from the same state, step
                               count and seed.  Not a method of the paper: a storage
                               choice of this library's reduced-precision form. */
} lbm_rounding;

typedef struct lbm_options {
  int32_t storage;       /* lbm_storage */
  int32_t stencil;       /* Lagrange nodes per axis n, 1..5 (LBM_GLC: p + 1 points per cell edge) */
  int32_t compressible;  /* 0: f only, theta = 1; 1: f and g (Sec. 3) */
  int32_t boundary[3];   /* lbm_boundary per axis x, y, z */
  int32_t energy_f64;    /* 16-bit storage, compressible: sum the energy moment in FP64
                            (LBM_EUNSUPPORTED with any other storage or model) */
  int32_t support;       /* lbm_support: where the nodes sit and how streaming interpolates */
  double dx;             /* grid spacing (> 0; LBM_GLC: the mean node spacing, cell width p dx) */
  double dt;             /* time step (> 0) */
  double cs;             /* speed of sound the set is scaled to; <= 0: the table's own */
  double gamma;          /* heat capacity ratio (compressible; C_v = 1/(gamma - 1)) */
  void *stream;          /* hipStream_t for all work of the context; NULL = null stream */
  double prandtl;        /* compressible model: Prandtl number (default 1: plain BGK).  Other
                            values relax the heat fluxes of f and g, taken in the frame moving
                            with the fluid, at 1/tau_q, tau_q = 1/2 + (tau - 1/2)/Pr, through
                            a quasi-equilibrium (Sec. 3 names the approach; reading in the
                            design notes), every other moment at 1/tau.  Built for D3Q45 with
                            n = 4 and D2Q19 / D2Q25 with n = 5, LBM_F64 / LBM_F32 storage
                            (LBM_EUNSUPPORTED otherwise). */
  int32_t rounding;      /* lbm_rounding of the stored values (default LBM_ROUND_NEAREST) */
  uint32_t seed;         /* LBM_ROUND_STOCHASTIC: seed of the random bits */
} lbm_options;

typedef struct lbm_diag {
  double mass;           /* sum over cells of rho */
  double momentum[3];    /* sum over cells of rho u */
  double ke;             /* mean over cells of |u|^2 / 2 (Sec. 4.2, unweighted) */
  double energy;         /* sum over cells of sum_i (|xi_i|^2 f_i / T0 + g_i) / 2 */
  double min_rho;        /* smallest rho */
  double min_theta;      /* smallest theta (1 in the weakly compressible model) */
  int32_t nonfinite;     /* number of cells whose rho, u or theta is not finite */
  int32_t reserved;
} lbm_diag;

typedef struct lbm_ctx lbm_ctx;

/* Fills opt with defaults: F32 storage, n = 4, periodic, dx = dt = 1,
 * cs = table's own, gamma = 1.4, Pr = 1, uniform support, null stream. */
void lbm_default_options(lbm_options *opt);

/* Creates a context for velocity set `set` on the grid grid[0] x grid[1] x
 * grid[2] (nx, ny, nz; nz must be 1 for the 2D sets), relaxation time `tau`
 * (at rho theta = 1 in the compressible model; must exceed 1/2) and Hermite
 * truncation order `order` (App. A; 2 <= order and 2 * order <= degree of the
 * set, so that the equilibrium's moments up to order N are exact, Sec. 2).
 * Computes the per-direction stencil (offsets and Lagrange weights) on the
 * host in FP64 and uploads it; allocates small device scratch for reductions.
 * The grid must hold the stencil: along every periodic axis of N nodes
 * every first-node offset o satisfies -N <= o and o + n <= N + 1.  Size
 * limits (LBM_EINVAL): fewer than 2^31 cells, and one population plus one
 * xy plane below 4 GiB (kernels use 32-bit byte offsets within a
 * population).  The context uses the current HIP device.  On failure *out is
 * NULL.  Ownership: the caller destroys the context with lbm_destroy(). */
int lbm_create(lbm_ctx **out, int32_t set, const int64_t grid[3], double tau, int32_t order,
               const lbm_options *opt);

/* Releases the context's own device and host memory (never the caller's
 * buffers).  Waits for the context's stream first.  NULL is accepted. */
int lbm_destroy(lbm_ctx *ctx);

/* Bytes of one population buffer: A * Q * nx * ny * nz * element size. */
size_t lbm_state_bytes(const lbm_ctx *ctx);

/* Hands the context two caller-owned device buffers of lbm_state_bytes()
 * bytes each (ping-pong pair; they must not overlap).  buf0 becomes the
 * current state.  The caller keeps ownership and must keep them alive while
 * the context uses them. */
int lbm_bind(lbm_ctx *ctx, void *buf0, void *buf1);

/* Device pointer of the buffer that holds the current state. */
void *lbm_state(lbm_ctx *ctx);

/* Writes f = f^eq(rho, u, theta) (and g = g^eq) into the current buffer:
 * the Hermite equilibrium of Sec. 3 truncated at the context's order N, with
 * the moments and Hermite tensors of App. A (T0 = c_s^2), and in the
 * compressible model g^eq = theta (2 C_v - D) f^eq (Sec. 3).  rho [cells],
 * u [D][cells] (physical units), theta [cells] or NULL (theta = 1), all
 * device arrays of the compute type, read on the context's stream.
 * LBM_EINVAL: null rho or u, or no buffers bound. */
int lbm_init_equilibrium(lbm_ctx *ctx, const void *rho, const void *u, const void *theta);

/* Checkpoint and resume: copies the current state (lbm_state_bytes() bytes,
 * the population layout above, as stored) to dst, or from src into the
 * current buffer.  dst/src may be device memory or host memory (pinned or
 * pageable); the copy is ordered on the context's stream after all work
 * enqueued before it, and the call returns once it has completed, so a host
 * buffer is ready (get) or reusable (set) on return.  A state saved with
 * lbm_get_state and restored with lbm_set_state into a context created with
 * the same arguments steps on bit for bit as the original.  The caller owns
 * dst/src.  LBM_EINVAL: null pointer or no buffers bound; LBM_EHIP: copy
 * failure (including earlier asynchronous faults). */
int lbm_get_state(lbm_ctx *ctx, void *dst);
int lbm_set_state(lbm_ctx *ctx, const void *src);

/* Advances the bound state by n >= 0 time steps (stream, then collide); each
 * step reads the current buffer and writes the other one, which then becomes
 * current.  n = 0 does nothing.  With float arithmetic (all storages but
 * LBM_F64) the collision also restores the momentum, and with LBM_F32 in the
 * compressible model the mass and the energy, that the float-rounded set
 * constants would miss (sum_i w_i xi_i xi_i equals c_s^2 I only to ~1e-8
 * there), so that these collision invariants (Sec. 3) hold to rounding as in
 * FP64.  Buffers need the element type's alignment; an even-element alignment
 * is faster. */
int lbm_step(lbm_ctx *ctx, int64_t n);

/* One time step from src to dst (caller device buffers of lbm_state_bytes(),
 * not overlapping); the bound pair is neither used nor changed. */
int lbm_step_into(lbm_ctx *ctx, const void *src, void *dst);

/* Per-cell rho, u, theta of `state` (NULL: the current buffer) into the
 * optional device arrays rho/u/theta (any may be NULL), and global
 * diagnostics into *diag (may be NULL).  The stored state is post-collision;
 * its rho, rho u and energy equal the pre-collision ones because the collision
 * conserves them (Sec. 3).  Synchronizes the context's stream.  Returns
 * LBM_EDIVERGED (with *diag filled) if a cell holds a non-finite value,
 * rho <= 0 or theta <= 0. */
int lbm_moments(lbm_ctx *ctx, const void *state, void *rho, void *u, void *theta, lbm_diag *diag);

/* lbm_moments for callers that cannot allocate memory (HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same kernels,
 * results and errors, but the block sums go to a static device array of the
 * library (1025 x 9 doubles, 73.8 KB per device, held until the process
 * ends) instead of the context's scratch, and the nine global sums come back
 * through a buffer on the caller's stack; the call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine).  Every call on one
 * device shares that array: calls that overlap on one device (several
 * streams or threads) race and must be serialized by the caller.  Nothing in
 * the array needs to start at zero: each call writes every element it reads.
 * LBM_EINVAL if the reduction would need more than the array holds (it
 * cannot with the current block count; checked). */
int lbm_moments_noalloc(lbm_ctx *ctx, const void *state, void *rho, void *u, void *theta, lbm_diag *diag);

/* Enstrophy E = <|curl u|^2> of a velocity field (Sec. 4.2: the squared
 * vorticity integrated over the domain and divided by its volume; on the
 * uniform periodic grid, the mean over the nodes), written to *enstrophy
 * (host memory).  u is a device array [D][nz][ny][nx] of the compute type in
 * the units lbm_moments() writes (physical velocity, lengths in units of dx's
 * length); derivatives are central differences of even order `order`
 * (2, 4, 6 or 8) with spacing dx, wrapped periodically.  In 2D the vorticity
 * has only its z component d_x u_y - d_y u_x.  For an incompressible flow
 * nu E is the physical dissipation rate of the kinetic energy, so its
 * difference from -dK/dt measures the scheme's numerical dissipation.  FP64
 * arithmetic.  LBM_EUNSUPPORTED unless every axis is periodic; LBM_EINVAL for
 * a null pointer or another order.  Synchronizes the context's stream. */
int lbm_enstrophy(lbm_ctx *ctx, const void *u, int32_t order, double *enstrophy);

/* Waits for the context's stream; reports asynchronous HIP errors. */
int lbm_sync(lbm_ctx *ctx);

/* Changes the stream used by later calls. */
int lbm_set_stream(lbm_ctx *ctx, void *stream);

/* ---- Adjoint (reverse-mode derivative of the time step; not in the paper).
 * Weakly compressible model with LBM_F64 or LBM_F32 storage only
 * (LBM_EUNSUPPORTED otherwise).  One time step is f' = C(S f) with S the
 * linear streaming and C the per-cell collision.  All arrays are device
 * arrays of the compute type in the population layout [Q][cells]. ---- */

/* nu = J_C(S f_prev)^T lam : adjoint of the collision of the step that
 * starts from f_prev, applied to lam = dL/df' (the step's output). */
int lbm_adjoint_collide(lbm_ctx *ctx, const void *f_prev, const void *lam, void *nu);

/* dst = S src : streaming alone, without the collision (forward stencil),
 * for diagnostics and tests; same availability as the adjoint calls. */
int lbm_stream(lbm_ctx *ctx, const void *src, void *dst);

/* lam = S^T nu : adjoint of streaming (a gather with mirrored offsets and
 * reversed weights), giving dL/df_prev. */
int lbm_adjoint_stream(lbm_ctx *ctx, const void *nu, void *lam);

/* nu_out = J_C(S f_prev)^T S^T nu_in : one fused reverse step.  With
 * nu_in = nu_{t+1} (the collision adjoint of step t+1) and f_prev = f_{t-1}
 * it returns nu_t; the chain starts with lbm_adjoint_collide and ends with
 * lbm_adjoint_stream. */
int lbm_adjoint_step(lbm_ctx *ctx, const void *f_prev, const void *nu_in, void *nu_out);

/* lam = dK/df for the mean kinetic energy K = <|u|^2/2> of state f. */
int lbm_ke_adjoint(lbm_ctx *ctx, const void *f, void *lam);

/* grad_u = (d f^eq(rho, u, 1)/d u)^T lam0, per cell: the gradient with
 * respect to the initial velocity through lbm_init_equilibrium. */
int lbm_init_equilibrium_adjoint(lbm_ctx *ctx, const void *rho, const void *u, const void *lam0,
                                 void *grad_u);

/* ---- Host-only helpers (no GPU needed) ---- */

/* The per-direction stencil of the semi-Lagrangian streaming (Sec. 3, eq.
 * sl_streaming: f_i at the departure point x - xi_i dt, as a sum of node
 * values times interpolation polynomials), computed on the host: for every
 * population i and axis a, offsets[3*i + a] is the offset of the first
 * stencil node from the arrival node and weights[(3*i + a)*n + k] the
 * Lagrange weight of node k at the departure point, for a set scaled to
 * speed of sound cs (<= 0: the table's own) with time step dt and spacing dx.  An axis along which xi_i has no
 * component gets offset 0 and the single weight 1 followed by zeros.  The
 * weights are exact FP64 Lagrange weights (not the quantized ones the kernels
 * use).  Arrays hold Q*3 and Q*3*n entries. */
int lbm_stencil(int32_t set, double dt, double dx, double cs, int32_t n, int32_t *offsets, double *weights);

/* The library's velocity set table: Q, D, degree, table speed of sound,
 * weights w[Q] and abscissae xi[Q][3] in table units. */
int lbm_set_table(int32_t set, int32_t *Q, int32_t *D, int32_t *degree, double *cs, double *w, double *xi);

/* The 30 coefficients with which the float (LBM_F32) compressible collision
 * restores the equilibrium's mass (lbm_step): the defects of the set's
 * moments, with its weights, abscissae and |xh|^2 rounded to float, against
 * the Gaussian moments they replace (degree 0, 2 and 4, in table units
 * xh = xi / c_s), each times the multiplicity of its monomial.  out[0]:
 * sum w - 1; out[1..6]: quadratic moments, monomials xx yy zz xy xz yz;
 * out[7]: sum w |xh|^2 - D; out[8..13]: |xh|^2-weighted quadratic moments
 * minus (D + 2) times the Gaussian ones, same monomials; out[14]:
 * sum w |xh|^4 - D (D + 2); out[15..29]: quartic moments, monomials xxxx
 * yyyy zzzz xxxy xxxz yyyx yyyz zzzx zzzy xxyy xxzz yyzz xxyz yyxz zzxy.
 * Monomials along axes the set lacks are 0.  Host-only; out holds 30. */
int lbm_float_moment_defects(int32_t set, double *out);

const char *lbm_strerror(int status);
const char *lbm_last_error(void);

/* Version of the ABI described by this header (3: lbm_options.rounding and seed). */
int32_t lbm_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
