/*
 * helm.h -- C ABI of the MI355X three-grid IOFD Helmholtz library.
 *
 * The library applies the matrix-free 27-point IOFD operator with PML
 * stretching on the h, 2h and 4h grids (Sec. 2.2, eq. iofd-shell-form,
 * eq. pml-second-difference, Sec. 3.1), the complex-shifted 2h-4h auxiliary
 * cycle (eq. shifted-auxiliary-cycle), restriction and prolongation
 * (eq. full-weighting, eq. linear-prolongation), the unshifted 2h solve
 * (eq. unshifted-middle-solve), the fine smoother and Algorithm 1, and the
 * outer FGMRES (Sec. 3.3) to a relative residual (eq. relative-residual).
 *
 * Conventions (all entry points)
 *   Grid sizes   Physical intervals nx, ny, nz; n_pml cells per face; the total
 *                grid has N_a = n_a + 2 n_pml intervals per axis, each N_a
 *                divisible by 4 and >= 8.  Level l in {0, 1, 2} (spacing
 *                2^l h) has N_a / 2^l intervals and (N_a/2^l + 1) nodes.
 *   Layout       Grid functions are [z][y][x], x fastest, all nodes including
 *                the boundary, complex interleaved (re, im): complex128 in
 *                HELM_FP64 mode, complex64 in HELM_FP32 and HELM_MIXED modes
 *                (the "precision vector type" below).  Nodes with an index 0 or N on any axis
 *                are boundary nodes (u = 0, eq. helmholtz-pml): operators read
 *                them as zero and write zero there.
 *   Pointers     Grid functions, the velocity and the workspace are DEVICE
 *                pointers owned by the caller; iters/relres and dot results are
 *                HOST pointers.  The library owns only the opaque hierarchy.
 *   Streams      All device work is enqueued on options.stream (a hipStream_t;
 *                NULL = default stream).  Entry points that return host values
 *                (helm_solve, helm_vec_dots, helm_setup's velocity check)
 *                synchronise that stream; the others return without waiting.
 *   Errors       Arguments are validated on the host before any device work;
 *                nothing throws across the ABI.  helm_last_error() returns the
 *                message of the last failing call (per hierarchy, or per thread
 *                for calls that had no hierarchy).
 *   Threads      A hierarchy must not be used by two threads at once, and two
 *                calls on one hierarchy must not overlap on different streams
 *                (they share the workspace).
 */
#ifndef HELM_H
#define HELM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct helm_hierarchy helm_hierarchy;

typedef enum {
    HELM_OK = 0,
    HELM_NOT_CONVERGED = 1, /* warning: outputs written, max_outer reached */
    HELM_EINVAL = -1,       /* invalid argument (nothing was enqueued) */
    HELM_EWORKSPACE = -2,   /* workspace too small or misaligned */
    HELM_EHIP = -3,         /* a HIP runtime call failed */
    HELM_BREAKDOWN = -4,    /* non-finite Krylov quantity (NaN/Inf in the data) */
    HELM_ENOTIMPL = -5
} helm_status;

/* Arithmetic of the hot path (Sec. 5, arithmetic precision).  In every mode the
 * outer FGMRES keeps its iterate, right-hand side and true residual in FP64 and
 * sums every inner product in FP64.
 *   HELM_FP64   complex128 vectors, FP64 arithmetic throughout.
 *   HELM_FP32   complex64 vectors, FP32 stencil and vector arithmetic.
 *   HELM_MIXED  as HELM_FP32, except that the vectors inside the 2h-4h cycle
 *               (its Jacobi iterates and residual, the 4h basis, its Jacobi
 *               images and correction) and K_2h's preconditioned vectors are
 *               stored in IEEE half precision, scaled by the inverse norm of the
 *               cycle's input and a fixed per-level factor (arithmetic stays
 *               FP32).  Requires nJ_2h = nJ_4h = 2. */
typedef enum { HELM_FP64 = 0, HELM_FP32 = 1, HELM_MIXED = 2 } helm_precision;

/* Level operators accepted by helm_apply */
typedef enum {
    HELM_OP_A = 0,      /* A_l = L_l - M_l, unshifted (eq. physical-iofd-levels) */
    HELM_OP_B = 1,      /* B_l = L_l - (1 + i sigma) M_l (eq. shifted-iofd-levels) */
    HELM_OP_Q = 2,      /* amplitude correction Q_h, level 0 only (eq. q-operator) */
    HELM_OP_DIAG_A = 3, /* y = diag(A_l) x */
    HELM_OP_DIAG_B = 4, /* y = diag(B_l) x */
    HELM_OP_AT = 5,     /* y = A_l^T x (transpose, not conjugate transpose) */
    HELM_OP_BT = 6,     /* y = B_l^T x */
    HELM_OP_QT = 7,     /* y = Q_h^T x, level 0 only */
    HELM_OP_DA = 8,     /* y_i = (d A_h / d m_i x)_i, m = 1/c^2 at node i, level 0 only */
    HELM_OP_DQ = 9      /* y_i = (d Q_h / d m_i x)_i, level 0 only */
} helm_op;

/* Solver configuration.  helm_default_options() fills the fixed
 * configuration of the paper's performance table: sigma 0.9; omega_h 0.8,
 * omega_2h 0.8, omega_4h 0.2; gamma_max 1.119058; nJ_h = nJ_2h = nJ_4h = 2;
 * m_h 2; c_2h 2; m_2h 10; m_4h 4; m_out 5. */
typedef struct {
    int struct_size;          /* sizeof(helm_options) */
    helm_precision precision; /* arithmetic and vector type of the hot path */
    double sigma, omega_h, omega_2h, omega_4h, gamma_max;
    int nJ_h, nJ_2h, nJ_4h;   /* Jacobi sweeps per level, 1..8 */
    int m_h, c_2h, m_2h, m_4h, m_out; /* m_h, m_2h, m_out in 1..12; m_4h in 1..8; c_2h in 1..8 */
    int max_outer;            /* preconditioner calls per right-hand side (<= 0: 1000) */
    const double *iofd_table; /* HOST, (K+1)*8*2 doubles: [node k][function f][value, slope],
                                 f = alpha1..alpha5, beta1..beta3, nodes eta_k = 0.4 k / K.
                                 Required (the paper takes these values as given data);
                                 copied during helm_setup. */
    int iofd_K;               /* number of table intervals, 1..128 */
    void *stream;             /* hipStream_t */
    /* Stencil tiling per level (performance only, results do not depend on it
     * beyond rounding of the fused norms).  helm_setup times the candidates
     * that are not fixed here on options.stream and keeps the fastest. */
    int tile_tz;              /* z planes per wavefront: 0 = timed; else 2..64 */
    int tile_split;           /* -1 = timed; 0 = one launch per stencil; 1 = an interior launch plus
                                 a border launch where the PML layout allows it */
    int lanes;                /* right-hand sides helm_solve runs concurrently (1..8; 0 = 1), each on
                                 its own copy of the solver's vectors and its own stream; the
                                 workspace grows by one copy per lane */
    int pml_variant;          /* reading of eq. pml-profile / eq. pml-second-difference (default 0):
                                 0 = gamma at the nodes from the distance d to the physical box with
                                     L_pml = n_pml h (gamma_max at the Dirichlet nodes), half-node gamma
                                     the mean of the two node values;
                                 1 = as 0, but half-node gamma from the half-node distance;
                                 2 = as 0, but the profile reaches gamma_max one fine cell earlier
                                     (denominator L_pml - h) and stays there.
                                 1 and 2 exist to study the Green-function error; the hot path is the same. */
    int batch;                /* right-hand sides each lane advances together in one set of launches
                                 (1..8; 0 = 1): every kernel of the solve runs once for all of them
                                 (the slot is the grid's y index), each with its own vectors and Krylov
                                 states; the workspace grows by one solver copy per slot and lane.
                                 Results equal, bit for bit, those of solving each right-hand side
                                 alone with the same stencil tiling (setup times the tiling with all
                                 slots running, so a batch may get other z depths than batch 1, and
                                 the fused norms then round in another order). */
} helm_options;

/* Fill *opt with the defaults above (table NULL, stream NULL, FP32, pml_variant 0, lanes 1,
 * batch 1). */
helm_status helm_default_options(helm_options *opt);

/* Bytes of device workspace helm_setup needs for this grid and options
 * (host-only computation, no device call). */
helm_status helm_workspace_size(int nx, int ny, int nz, int n_pml, const helm_options *opt, size_t *bytes);

/* Build the operator hierarchy (Sec. 3.1): the velocity is extended into the
 * PML by its nearest physical value (Sec. 2.1) and sampled at the nodes of
 * each level; the per-axis PML factors (eq. pml-profile, half nodes averaged
 * before inversion) and the table are uploaded.  The stencil tilings not fixed
 * by the options are timed on the first setup of a level shape and precision
 * in the process (per device) and reused by later setups of that shape. 
 *   velocity  DEVICE float[(nz+1)(ny+1)(nx+1)], physical nodes, m/s, finite > 0
 *   h, omega  fine spacing (m) and angular frequency (rad/s), finite > 0
 *   workspace DEVICE, >= helm_workspace_size() bytes, 256-byte aligned, owned by
 *             the caller and kept alive until helm_destroy
 * Returns HELM_EINVAL for a non-positive or non-finite velocity value. */
helm_status helm_setup(const float *velocity, int nx, int ny, int nz, double h, double omega, int n_pml,
                       const helm_options *opt, void *workspace, size_t ws_bytes, helm_hierarchy **out);

/* Solve A_h v = Q_h f and return u = Q_h v for nrhs right-hand sides
 * (eq. iofd-complete-system) with outer FGMRES(m_out) right preconditioned by
 * Algorithm 1, from v = 0, until ||A_h v - b|| / ||b|| <= tol recomputed with
 * FP64 arithmetic (eq. relative-residual).  The right-hand sides are taken in
 * groups of options.batch; options.lanes groups run concurrently.
 *   f, u    DEVICE [nrhs][total grid] precision vectors (may not alias)
 *   iters   HOST int[nrhs]: preconditioner calls per right-hand side
 *   relres  HOST double[nrhs]: final true relative residual
 * Returns HELM_NOT_CONVERGED (u still written) if a right-hand side spent
 * max_outer preconditioner calls. */
helm_status helm_solve(helm_hierarchy *H, const void *f, int nrhs, double tol, void *u, int *iters,
                       double *relres);

/* helm_solve that also keeps the forward solutions v (A_h v = Q_h f, u = Q_h v)
 * in FP64 for a later helm_grad (checkpointed forward wavefields):
 *   v  DEVICE complex128 [nrhs][total grid], written (must not alias f or u)
 * Other arguments and returns as helm_solve. */
helm_status helm_solve_checkpoint(helm_hierarchy *H, const void *f, int nrhs, double tol, void *u, void *v,
                                  int *iters, double *relres);

/* Gradient of a real misfit J(u) of the solutions u = Q_h v, A_h v = Q_h f
 * (eq. iofd-complete-system), with respect to the squared slowness m = 1/c^2
 * at the physical nodes, by the adjoint state.  Each row of A_h and Q_h takes
 * its coefficients at its own node (Sec. 2.2: kappa and eta* at the row
 * centre), so with A_h^T mu = Q_h^T conj(s),
 *   dJ/dm_i = Re[ conj(s_i) (d_i Q_h v)_i + mu_i ((d_i Q_h f)_i - (d_i A_h v)_i) ],
 * and a PML node, which takes the velocity of its nearest physical node
 * (Sec. 2.1), adds its term onto that node.  Per right-hand side: one forward
 * solve (skipped when v_fwd is given) and one adjoint solve (outer FGMRES with
 * A_h^T, the same preconditioner), each to the true relative residual tol.
 *   f, adj_src DEVICE [nrhs][total grid] precision vectors: sources, and the
 *              adjoint sources s defined by dJ = Re sum_i conj(s_i) du_i
 *              (for J = 1/2 ||u - d||^2: s = u - d)
 *   v_fwd      DEVICE complex128 [nrhs][total grid]: the forward solutions as
 *              helm_solve_checkpoint returns them for the same f, or NULL to
 *              solve the forward problems here (then iters/relres report them;
 *              with v_fwd their forward entries are 0)
 *   grad_m     DEVICE float[(nz+1)(ny+1)(nx+1)], physical nodes: dJ/dm summed
 *              over the right-hand sides (overwritten)
 *   workspace  DEVICE, >= helm_grad_workspace_size() bytes, 256-byte aligned
 *   iters, relres HOST [2 nrhs]: preconditioner calls and final true relative
 *              residuals, forward then adjoint, per right-hand side
 * Returns HELM_NOT_CONVERGED (gradient still written) if a solve spent
 * max_outer preconditioner calls. */
helm_status helm_grad_workspace_size(const helm_hierarchy *H, size_t *bytes);

/* grad_c = grad_m * dm/dc = grad_m * (-2 / c^3): a gradient with respect to the squared
 * slowness (as helm_grad returns it) turned into one with respect to the velocity c the
 * hierarchy was built from.  Both DEVICE float[(nz+1)(ny+1)(nx+1)], physical nodes; may alias. */
helm_status helm_grad_to_velocity(helm_hierarchy *H, const float *grad_m, float *grad_c);
helm_status helm_grad(helm_hierarchy *H, const void *f, const void *adj_src, const void *v_fwd, int nrhs, double tol,
                      float *grad_m, void *workspace, size_t ws_bytes, int *iters, double *relres);

void helm_destroy(helm_hierarchy *H);

/* Message of the last failing call on H (H == NULL: of this thread). */
const char *helm_last_error(const helm_hierarchy *H);

/* Total intervals (Nx, Ny, Nz) of level 0..2. */
helm_status helm_dims(const helm_hierarchy *H, int level, int dims[3]);

/* ---- Steps of the hot path (same kernels as helm_solve; used by the tests
 *      and the benchmark).  All vectors are DEVICE precision vectors of the
 *      named level; inputs must have zero boundary entries where stated. ---- */

/* y = op x on level (helm_op; HELM_OP_Q, QT, DA, DQ only on level 0).  x, y must differ. */
helm_status helm_apply(helm_hierarchy *H, int level, int op, const void *x, void *y);


/* r = g - op x (op = HELM_OP_A or HELM_OP_B); boundary entries of r are zero. */
helm_status helm_residual(helm_hierarchy *H, int level, int op, const void *g, const void *x, void *r);

/* y = J_nJ(op, g; omega): nJ damped Jacobi sweeps from zero (eq. jacobi-map),
 * diagonal of the same operator (PML and shift included). */
helm_status helm_jacobi(helm_hierarchy *H, int level, int op, const void *g, int nJ, double omega, void *y);

/* coarse = R fine (full weighting), fine on `level` (0 or 1), coarse on level+1. */
helm_status helm_restrict(helm_hierarchy *H, int level, const void *fine, void *coarse);

/* coarse = R (g - op x): the residual on `level` (0 or 1) restricted by full
 * weighting to level+1 in one fused pass over the fine grid plus a small pass
 * over a quarter-size intermediate held in the workspace (eq. full-weighting
 * applied to the residual, as in steps 2 of Algorithm 1 and of
 * eq. shifted-auxiliary-cycle).  op = HELM_OP_A or HELM_OP_B; g, x on level,
 * coarse on level+1 (boundary entries written as zero); coarse must not alias
 * g or x.  Returns HELM_EINVAL for other levels or ops. */
helm_status helm_residual_restrict(helm_hierarchy *H, int level, int op, const void *g, const void *x, void *coarse);

/* fine += P coarse (trilinear), coarse on `level` (1 or 2), fine on level-1. */
helm_status helm_prolong_add(helm_hierarchy *H, int level, const void *coarse, void *fine);

/* e = C_4h(q): m_4h CA-GMRES steps on B_4h from zero, right preconditioned by
 * J_nJ4h(B_4h; omega_4h) (Sec. 3.2).  q, e on level 2, zero boundary.  In
 * HELM_MIXED mode q is stored in half precision in units of its own norm, as
 * inside the cycle, and e is returned in complex64. */
helm_status helm_bottom(helm_hierarchy *H, const void *q, void *e);

/* y = V^sigma_2h(q), one shifted 2h-4h cycle (eq. shifted-auxiliary-cycle).
 * In HELM_MIXED mode the cycle runs in units of the norm of q (a zero q gives
 * a zero y) and y is returned in complex64. */
helm_status helm_vcycle(helm_hierarchy *H, const void *q, void *y);

/* e = K_2h(r): c_2h FGMRES(m_2h) cycles on A_2h from zero, right
 * preconditioned by V^sigma_2h (eq. unshifted-middle-solve). */
helm_status helm_coarse_solve(helm_hierarchy *H, const void *r, void *e);

/* x = S_h(g; x0): one GMRES(m_h) cycle on A_h from x0 (NULL = zero), right
 * preconditioned by J_nJh(A_h; omega_h) (Sec. 3.3).  x may equal x0. */
helm_status helm_smooth(helm_hierarchy *H, const void *g, const void *x0, void *x);

/* z = M_h^{-1} r, Algorithm 1.  r with zero boundary; z must not alias r. */
helm_status helm_precond(helm_hierarchy *H, const void *r, void *z);

/* Krylov vector kernel: out[j] = sum_i conj(V_j[i]) w[i] for j < k, and
 * out[k] = ||w||^2 (imaginary part 0), accumulated in FP64.
 *   V   HOST array of k DEVICE pointers (level vectors), 0 <= k <= 12
 *   out HOST double[2*(k+1)] (complex pairs)
 * Returns HELM_EINVAL for k outside 0..12. */
helm_status helm_vec_dots(helm_hierarchy *H, int level, int k, const void *const *V, const void *w, double *out);

/* One Arnoldi orthogonalisation step (classical Gram-Schmidt, two passes):
 * w <- (w - V h) / ||w - V h||, with h = V^* w accumulated over both passes.
 *   V   HOST array of k DEVICE pointers (orthonormal level vectors), 1 <= k <= 12
 *   out HOST double[2*(k+1)]: h_0..h_{k-1} then ||w - V h||
 * Returns HELM_EINVAL for k outside 1..12.  If w lies in the span of V (w - V h
 * vanishes exactly), w is set to zero. */
helm_status helm_vec_orthonormalize(helm_hierarchy *H, int level, int k, const void *const *V, void *w,
                                    double *out);

/* Tile choices that helm_setup has timed in this process (per GPU architecture, precision, level
 * shape, kernel family and batch slots: the z depth of the stencil wavefronts and whether a stencil
 * runs as one launch or two), written to or read from a text file, so that a later process reuses them instead of
 * timing again (the timing is most of a first setup).  Performance only: results depend on the
 * choices no more than through the rounding order of fused norms.
 *   helm_tiles_save  writes every choice made or loaded so far in this process to `path` (a header
 *                    line, then one line per choice).
 *   helm_tiles_load  adds the choices in `path` whose architecture is that of a visible GPU to this
 *                    process's table, for every such GPU, replacing equal keys; `n_loaded` (optional,
 *                    HOST int) receives the number of entries added or replaced.
 * Both return HELM_EINVAL (message in helm_last_error(NULL)) for a NULL path, a file that cannot be
 * opened or written, or (load) a file that is not a tile-choice file or has a malformed line; choices
 * read before a malformed line stay loaded. */
helm_status helm_tiles_save(const char *path);
helm_status helm_tiles_load(const char *path, int *n_loaded);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): helm_vec_dots on plain
 * vectors, without a hierarchy, with the result left in device memory.  The
 * reduction's per-block partial sums and its completion counter live in a
 * library-owned static device array of at most 192 KiB per GPU, held from the
 * first call on that GPU until the process ends; the call performs no hipMalloc,
 * hipFree or other allocation and does not synchronise.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (different streams or
 * threads) race and give wrong sums.
 *   precision HELM_FP32 (complex64 vectors) or HELM_FP64 (complex128 vectors)
 *   n         entries per vector, 1 <= n <= 2^40
 *   k         0 <= k <= 12
 *   V         HOST array of k DEVICE pointers (n entries each)
 *   w         DEVICE vector of n entries
 *   out       DEVICE double[2*(k+1)]: conj(V_j) . w for j < k, then ||w||^2 (imaginary
 *             part 0), accumulated in FP64 (the sums of helm_vec_dots for the same n)
 *   stream    hipStream_t the work is enqueued on (NULL = default stream)
 * Returns HELM_EINVAL (message in helm_last_error(NULL)) for a bad precision, n
 * or k, or a NULL pointer, before any device work. */
helm_status helm_vec_dots_static(int precision, long long n, int k, const void *const *V, const void *w,
                                 double *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HELM_H */
