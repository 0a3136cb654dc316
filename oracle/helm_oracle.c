/*
 * helm_oracle.c -- plain, slow FP64 reference implementation of the
 * three-grid IOFD Helmholtz preconditioner and its outer solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU library: it is written directly from the paper's equations, one
 * function per definition, with no blocking, fusion or reordering beyond what
 * the definitions state.
 *
 * Conventions
 *   - Grid functions are complex double, interleaved (re, im), laid out
 *     [z][y][x] with x fastest, on nodes 0..n_a of every axis a.
 *   - Nodes with an index 0 or n_a on any axis lie on the outer boundary,
 *     where u = 0 (eq. helmholtz-pml).  Every operator reads them as zero and
 *     writes zero there; the unknowns are the interior nodes.
 *   - Level s in {1, 2, 4} (spacing ell = s h) has n_a / s intervals per axis.
 *
 * Parity status: every function below is pinned by a CPU test (symbol, DST
 * diagonalisation, Kronecker special case, transfer identities, minimal
 * residual property, dense direct solve, Green function), see the test files.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef double complex cplx;

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -2

/* Operators handed to or_apply */
enum { OP_A = 0, OP_B = 1, OP_Q = 2, OP_DIAG_A = 3, OP_DIAG_B = 4 };

/* Solver parameters (Table "Fixed discretization and three-grid parameters") */
typedef struct {
    double sigma, omega_h, omega_2h, omega_4h, gamma_max;
    int nJ_h, nJ_2h, nJ_4h, m_h, c_2h, m_2h, m_4h, m_out;
    int pml_variant;   /* 0: the reading used throughout; 1, 2: alternatives (pml_gamma) */
} or_params;

typedef struct {
    int n[3];            /* intervals per axis (x, y, z) */
    double ell;          /* level spacing */
    double *c;           /* velocity on level nodes */
    cplx *xin[3];        /* 1/xi at nodes, n[a]+1 entries */
    cplx *xih[3];        /* 1/xi at half nodes j+1/2, n[a] entries */
    size_t nn;           /* number of nodes */
} or_level;

typedef struct {
    or_level lev[3];
    double h, omega;
    int n_pml;
    int nphys[3];        /* physical intervals per axis (the velocity grid) */
    const double *tab;   /* [node][function][value, slope] */
    int K;
    double eta_max;
    or_params p;
} or_hier;

/* ------------------------------------------------------------------ */
/* small vector helpers (all entries, boundary included)              */
/* ------------------------------------------------------------------ */

static cplx *vnew(size_t n) { return (cplx *)calloc(n ? n : 1, sizeof(cplx)); }

static void vcopy(size_t n, const cplx *a, cplx *b) { memcpy(b, a, n * sizeof(cplx)); }

static void vzero(size_t n, cplx *a) { memset(a, 0, n * sizeof(cplx)); }

/* Sum of conj(a_i) b_i.  Each thread sums a fixed contiguous chunk and the
 * chunks are added in order, so a fixed thread count gives a fixed result. */
static cplx vdot(size_t n, const cplx *a, const cplx *b)
{
    int nt = omp_get_max_threads();
    cplx *part = (cplx *)calloc((size_t)nt, sizeof(cplx));
#pragma omp parallel num_threads(nt)
    {
        int t = omp_get_thread_num(), T = omp_get_num_threads();
        size_t lo = n * (size_t)t / (size_t)T, hi = n * (size_t)(t + 1) / (size_t)T;
        cplx s = 0;
        for (size_t i = lo; i < hi; ++i) s += conj(a[i]) * b[i];
        part[t] = s;
    }
    cplx s = 0;
    for (int t = 0; t < nt; ++t) s += part[t];
    free(part);
    return s;
}

static double vnorm(size_t n, const cplx *a) { return sqrt(creal(vdot(n, a, a))); }

/* b += alpha a */
static void vaxpy(size_t n, cplx alpha, const cplx *a, cplx *b)
{
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < n; ++i) b[i] += alpha * a[i];
}

static void vscale(size_t n, cplx alpha, cplx *a)
{
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < n; ++i) a[i] *= alpha;
}

/* c = a - b */
static void vsub(size_t n, const cplx *a, const cplx *b, cplx *c)
{
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < n; ++i) c[i] = a[i] - b[i];
}

static inline size_t idx3(const int n[3], int x, int y, int z)
{
    return ((size_t)z * (size_t)(n[1] + 1) + (size_t)y) * (size_t)(n[0] + 1) + (size_t)x;
}

static inline int on_boundary(const int n[3], int x, int y, int z)
{
    return x == 0 || y == 0 || z == 0 || x == n[0] || y == n[1] || z == n[2];
}

/* ------------------------------------------------------------------ */
/* IOFD coefficient functions: cubic Hermite interpolation (Sec. 2.2)  */
/* ------------------------------------------------------------------ */

/* Value of tabulated function f (0..7 = alpha1..5, beta1..3) at eta in
 * [0, eta_max]; nodes eta_k = k * eta_max / K carry a value and a slope. */
static double hermite(const or_hier *H, int f, double eta)
{
    const double de = H->eta_max / H->K;
    int k = (int)floor(eta / de);
    if (k < 0) k = 0;
    if (k > H->K - 1) k = H->K - 1;
    double t = (eta - k * de) / de;
    double p0 = H->tab[(k * 8 + f) * 2 + 0], m0 = H->tab[(k * 8 + f) * 2 + 1];
    double p1 = H->tab[((k + 1) * 8 + f) * 2 + 0], m1 = H->tab[((k + 1) * 8 + f) * 2 + 1];
    double h00 = 2 * t * t * t - 3 * t * t + 1;
    double h10 = t * t * t - 2 * t * t + t;
    double h01 = -2 * t * t * t + 3 * t * t;
    double h11 = t * t * t - t * t;
    return h00 * p0 + h10 * de * m0 + h01 * p1 + h11 * de * m1;
}

/* Row-centre quantities at a node with velocity c on spacing ell
 * (eq. iofd-clamped-coordinate): kappa = k ell (physical, for the mass term)
 * and eta* = min(kappa / 2pi, 0.4) (for the tables). */
static void row_coeffs(const or_hier *H, double c, double ell, double *kappa, double a[5])
{
    double k = H->omega / c;
    *kappa = k * ell;
    double eta = *kappa / (2.0 * M_PI);
    if (eta > 0.4) eta = 0.4;
    for (int f = 0; f < 5; ++f) a[f] = hermite(H, f, eta);
}

/* ------------------------------------------------------------------ */
/* PML stretching (eq. pml-profile)                                    */
/* ------------------------------------------------------------------ */

/* gamma(d) = gamma_max (1 - cos(pi d / (2 L_pml))), d the distance from the physical box
 * into the layer, L_pml = n_pml h.  Alternative readings (pml_variant): 2 = the profile
 * reaches gamma_max at d = L_pml - h and stays there; 1 only changes the half nodes
 * (level_init). */
static double pml_gamma(const or_hier *H, int axis, double x)
{
    double Lpml = H->n_pml * H->h;
    if (Lpml <= 0) return 0.0;
    double L = H->lev[0].n[axis] * H->h;         /* total box length on this axis */
    double Lp = (H->p.pml_variant == 2) ? Lpml - H->h : Lpml;
    double d = 0.0;
    if (x < Lpml) d = Lpml - x;
    if (x > L - Lpml) d = x - (L - Lpml);
    if (d > Lp) d = Lp;
    return H->p.gamma_max * (1.0 - cos(M_PI * d / (2.0 * Lp)));
}

static int level_init(or_hier *H, int li, const double *vel_phys, const int nphys[3])
{
    or_level *L = &H->lev[li];
    int s = 1 << li;
    for (int a = 0; a < 3; ++a) L->n[a] = H->lev[0].n[a] / s;
    L->ell = s * H->h;
    L->nn = (size_t)(L->n[0] + 1) * (L->n[1] + 1) * (L->n[2] + 1);
    L->c = (double *)malloc(L->nn * sizeof(double));
    if (!L->c) return OR_ENOMEM;
    /* velocity sampled at the level nodes (injection), extended into the PML
     * by its nearest physical value (Sec. 2.1) */
    for (int z = 0; z <= L->n[2]; ++z)
        for (int y = 0; y <= L->n[1]; ++y)
            for (int x = 0; x <= L->n[0]; ++x) {
                int fi[3] = {x * s, y * s, z * s}, pi[3];
                for (int a = 0; a < 3; ++a) {
                    int q = fi[a] - H->n_pml;
                    if (q < 0) q = 0;
                    if (q > nphys[a]) q = nphys[a];
                    pi[a] = q;
                }
                L->c[idx3(L->n, x, y, z)] =
                    vel_phys[((size_t)pi[2] * (nphys[1] + 1) + pi[1]) * (nphys[0] + 1) + pi[0]];
            }
    /* 1/xi at nodes and at half nodes; the half-node gamma is the average of the
     * two adjacent node values, inverted afterwards (Sec. 2.2; pml_variant 1: gamma
     * at the half node itself) */
    for (int a = 0; a < 3; ++a) {
        int n = L->n[a];
        L->xin[a] = vnew((size_t)n + 1);
        L->xih[a] = vnew((size_t)n);
        if (!L->xin[a] || !L->xih[a]) return OR_ENOMEM;
        for (int j = 0; j <= n; ++j) L->xin[a][j] = 1.0 / (1.0 + I * pml_gamma(H, a, j * L->ell));
        for (int j = 0; j < n; ++j) {
            double g = (H->p.pml_variant == 1)
                           ? pml_gamma(H, a, (j + 0.5) * L->ell)
                           : 0.5 * (pml_gamma(H, a, j * L->ell) + pml_gamma(H, a, (j + 1) * L->ell));
            L->xih[a][j] = 1.0 / (1.0 + I * g);
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Level operators                                                     */
/* ------------------------------------------------------------------ */

/* The 27 row coefficients of H_mu = L - mu M at interior node (x,y,z), times
 * ell^2, from the tensor-product form (Sec. 2.2): for each axis j, the PML
 * second difference weights w_j(delta_j) times the transverse weight for the
 * other two offsets (a4, a5/4, (1-a4-a5)/4 by their number of nonzeros), minus
 * mu kappa^2 times the mass weight (a1, a2/6, a3/12, (1-a1-a2-a3)/8) of the
 * shell |delta|_1.  Index of delta: (dz+1)*9 + (dy+1)*3 + (dx+1). */
static void row_stencil(const or_hier *H, const or_level *L, int x, int y, int z, cplx mu, cplx Kst[27])
{
    double kappa, a[5];
    row_coeffs(H, L->c[idx3(L->n, x, y, z)], L->ell, &kappa, a);
    double T[3] = {a[3], a[4] / 4.0, (1.0 - a[3] - a[4]) / 4.0};
    double Mw[4] = {a[0], a[1] / 6.0, a[2] / 12.0, (1.0 - a[0] - a[1] - a[2]) / 8.0};
    int pos[3] = {x, y, z};
    cplx w[3][3];                                  /* w[axis][delta+1] */
    for (int j = 0; j < 3; ++j) {
        int i = pos[j];
        cplx xn = L->xin[j][i], xp = L->xih[j][i], xm = L->xih[j][i - 1];
        w[j][0] = -xn * xm;
        w[j][1] = xn * (xp + xm);
        w[j][2] = -xn * xp;
    }
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int d[3] = {dx, dy, dz};
                cplx k = 0;
                for (int j = 0; j < 3; ++j) {
                    int nz = 0;
                    for (int q = 0; q < 3; ++q)
                        if (q != j && d[q] != 0) ++nz;
                    k += w[j][d[j] + 1] * T[nz];
                }
                int shell = abs(dx) + abs(dy) + abs(dz);
                k -= mu * kappa * kappa * Mw[shell];
                Kst[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] = k;
            }
}

static cplx op_mu(const or_hier *H, int op)
{
    return (op == OP_B || op == OP_DIAG_B) ? (1.0 + I * H->p.sigma) : 1.0;
}

static cplx apply_row(const or_hier *H, const or_level *L, int op, const cplx *xv, int x, int y, int z)
{
    if (on_boundary(L->n, x, y, z)) return 0;
    cplx mu = op_mu(H, op);
    if (op == OP_DIAG_A || op == OP_DIAG_B) {
        cplx Kst[27];
        row_stencil(H, L, x, y, z, mu, Kst);
        return Kst[13] / (L->ell * L->ell) * xv[idx3(L->n, x, y, z)];
    }
    if (op == OP_Q) {
        /* amplitude correction, eq. q-operator: shell weights from beta at the
         * fine-grid eta*, no PML form, no ell^-2 */
        double kappa = H->omega / L->c[idx3(L->n, x, y, z)] * L->ell;
        double eta = kappa / (2.0 * M_PI);
        if (eta > 0.4) eta = 0.4;
        double b1 = hermite(H, 5, eta), b2 = hermite(H, 6, eta), b3 = hermite(H, 7, eta);
        double Qm[4] = {b1, b2 / 6.0, b3 / 12.0, (1.0 - b1 - b2 - b3) / 8.0};
        cplx s = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int xx = x + dx, yy = y + dy, zz = z + dz;
                    if (on_boundary(L->n, xx, yy, zz)) continue;
                    s += Qm[abs(dx) + abs(dy) + abs(dz)] * xv[idx3(L->n, xx, yy, zz)];
                }
        return s;
    }
    cplx Kst[27];
    row_stencil(H, L, x, y, z, mu, Kst);
    cplx s = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int xx = x + dx, yy = y + dy, zz = z + dz;
                if (on_boundary(L->n, xx, yy, zz)) continue;
                s += Kst[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] * xv[idx3(L->n, xx, yy, zz)];
            }
    return s / (L->ell * L->ell);
}

/* y = op x on level L (A_l, B_l, Q_h, or the diagonal of A_l / B_l times x) */
static void level_apply(const or_hier *H, const or_level *L, int op, const cplx *xv, cplx *yv)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z <= L->n[2]; ++z)
        for (int y = 0; y <= L->n[1]; ++y)
            for (int x = 0; x <= L->n[0]; ++x) yv[idx3(L->n, x, y, z)] = apply_row(H, L, op, xv, x, y, z);
}

/* diagonal D of A_l (op = OP_A) or B_l (op = OP_B) at an interior node */
static cplx level_diag(const or_hier *H, const or_level *L, int op, int x, int y, int z)
{
    cplx Kst[27];
    row_stencil(H, L, x, y, z, op_mu(H, op), Kst);
    return Kst[13] / (L->ell * L->ell);
}

/* r = g - op x */
static void level_residual(const or_hier *H, const or_level *L, int op, const cplx *g, const cplx *xv, cplx *r)
{
    level_apply(H, L, op, xv, r);
#pragma omp parallel for schedule(static)
    for (int z = 0; z <= L->n[2]; ++z)
        for (int y = 0; y <= L->n[1]; ++y)
            for (int x = 0; x <= L->n[0]; ++x) {
                size_t i = idx3(L->n, x, y, z);
                r[i] = on_boundary(L->n, x, y, z) ? 0 : g[i] - r[i];
            }
}

/* ------------------------------------------------------------------ */
/* Transposes and derivatives with respect to m = 1/c^2 (adjoint-state  */
/* gradient of a misfit of u = Q_h v, A_h v = Q_h f)                    */
/* ------------------------------------------------------------------ */

/* d alpha_f / d eta of the Hermite interpolant of hermite() */
static double hermite_deta(const or_hier *H, int f, double eta)
{
    const double de = H->eta_max / H->K;
    int k = (int)floor(eta / de);
    if (k < 0) k = 0;
    if (k > H->K - 1) k = H->K - 1;
    double t = (eta - k * de) / de;
    double p0 = H->tab[(k * 8 + f) * 2 + 0], m0 = H->tab[(k * 8 + f) * 2 + 1];
    double p1 = H->tab[((k + 1) * 8 + f) * 2 + 0], m1 = H->tab[((k + 1) * 8 + f) * 2 + 1];
    double d00 = 6 * t * t - 6 * t;           /* derivatives in t of the four basis cubics */
    double d10 = 3 * t * t - 4 * t + 1;
    double d01 = -6 * t * t + 6 * t;
    double d11 = 3 * t * t - 2 * t;
    return (d00 * p0 + d10 * de * m0 + d01 * p1 + d11 * de * m1) / de;
}

/* At a node with velocity c on spacing ell: kappa = omega ell / c = omega ell sqrt(m);
 * eta = min(kappa / 2pi, 0.4).  d eta / d m = kappa c^2 / (4 pi) below the clamp, 0 on it;
 * d kappa^2 / d m = kappa^2 c^2. */
static double deta_dm(double c, double kappa)
{
    double eta = kappa / (2.0 * M_PI);
    return eta >= 0.4 ? 0.0 : kappa * c * c / (4.0 * M_PI);
}

/* d/dm of the 27 row coefficients of row_stencil (mu = 1) at interior node (x,y,z), times ell^2:
 * the transverse weights (a4, a5/4, (1-a4-a5)/4) and mass weights (a1, a2/6, a3/12,
 * (1-a1-a2-a3)/8) differentiated through alpha(eta), and kappa^2 differentiated directly. */
static void row_stencil_dm(const or_hier *H, const or_level *L, int x, int y, int z, cplx Kd[27])
{
    double c = L->c[idx3(L->n, x, y, z)];
    double kappa, a[5], da[5];
    row_coeffs(H, c, L->ell, &kappa, a);
    double eta = kappa / (2.0 * M_PI);
    if (eta > 0.4) eta = 0.4;
    double de = deta_dm(c, kappa);
    for (int f = 0; f < 5; ++f) da[f] = hermite_deta(H, f, eta) * de;
    double k2 = kappa * kappa, dk2 = kappa * kappa * c * c;
    double dT[3] = {da[3], da[4] / 4.0, -(da[3] + da[4]) / 4.0};
    double Mw[4] = {a[0], a[1] / 6.0, a[2] / 12.0, (1.0 - a[0] - a[1] - a[2]) / 8.0};
    double dMw[4] = {da[0], da[1] / 6.0, da[2] / 12.0, -(da[0] + da[1] + da[2]) / 8.0};
    int pos[3] = {x, y, z};
    cplx w[3][3];
    for (int j = 0; j < 3; ++j) {
        int i = pos[j];
        cplx xn = L->xin[j][i], xp = L->xih[j][i], xm = L->xih[j][i - 1];
        w[j][0] = -xn * xm;
        w[j][1] = xn * (xp + xm);
        w[j][2] = -xn * xp;
    }
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int d[3] = {dx, dy, dz};
                cplx k = 0;
                for (int j = 0; j < 3; ++j) {
                    int nz = 0;
                    for (int q = 0; q < 3; ++q)
                        if (q != j && d[q] != 0) ++nz;
                    k += w[j][d[j] + 1] * dT[nz];
                }
                int shell = abs(dx) + abs(dy) + abs(dz);
                k -= dk2 * Mw[shell] + k2 * dMw[shell];
                Kd[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] = k;
            }
}

/* shell weights of Q_h at a fine node (eq. q-operator) and their derivatives in m */
static void q_weights(const or_hier *H, const or_level *L, int x, int y, int z, double Qm[4], double dQm[4])
{
    double c = L->c[idx3(L->n, x, y, z)];
    double kappa = H->omega / c * L->ell;
    double eta = kappa / (2.0 * M_PI);
    if (eta > 0.4) eta = 0.4;
    double b[3], db[3], de = deta_dm(c, kappa);
    for (int f = 0; f < 3; ++f) {
        b[f] = hermite(H, 5 + f, eta);
        db[f] = hermite_deta(H, 5 + f, eta) * de;
    }
    Qm[0] = b[0];
    Qm[1] = b[1] / 6.0;
    Qm[2] = b[2] / 12.0;
    Qm[3] = (1.0 - b[0] - b[1] - b[2]) / 8.0;
    dQm[0] = db[0];
    dQm[1] = db[1] / 6.0;
    dQm[2] = db[2] / 12.0;
    dQm[3] = -(db[0] + db[1] + db[2]) / 8.0;
}

/* y = op^T x on level L (op A or B on any level, Q on level 0): by definition of the
 * transpose, every interior row i adds (row i, column j) * x_i to y_j for each interior
 * neighbour j.  Serial, so the scatter has no races. */
static void level_apply_t(const or_hier *H, const or_level *L, int op, const cplx *xv, cplx *yv)
{
    vzero(L->nn, yv);
    for (int z = 1; z < L->n[2]; ++z)
        for (int y = 1; y < L->n[1]; ++y)
            for (int x = 1; x < L->n[0]; ++x) {
                cplx xi = xv[idx3(L->n, x, y, z)];
                cplx Kst[27];
                double Qm[4], dQm[4];
                if (op == OP_Q)
                    q_weights(H, L, x, y, z, Qm, dQm);
                else
                    row_stencil(H, L, x, y, z, op_mu(H, op), Kst);
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            int xx = x + dx, yy = y + dy, zz = z + dz;
                            if (on_boundary(L->n, xx, yy, zz)) continue;
                            cplx coef = (op == OP_Q) ? Qm[abs(dx) + abs(dy) + abs(dz)]
                                                     : Kst[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] /
                                                           (L->ell * L->ell);
                            yv[idx3(L->n, xx, yy, zz)] += coef * xi;
                        }
            }
}

/* y_i = (d_i op x)_i on level 0: row i of op differentiated with respect to m_i (the
 * squared slowness at node i; every row depends on its own node only), op A or Q */
static void level_apply_dm(const or_hier *H, int op, const cplx *xv, cplx *yv)
{
    const or_level *L = &H->lev[0];
#pragma omp parallel for schedule(static)
    for (int z = 0; z <= L->n[2]; ++z)
        for (int y = 0; y <= L->n[1]; ++y)
            for (int x = 0; x <= L->n[0]; ++x) {
                size_t i = idx3(L->n, x, y, z);
                if (on_boundary(L->n, x, y, z)) {
                    yv[i] = 0;
                    continue;
                }
                cplx Kd[27];
                double Qm[4], dQm[4];
                if (op == OP_Q)
                    q_weights(H, L, x, y, z, Qm, dQm);
                else
                    row_stencil_dm(H, L, x, y, z, Kd);
                cplx s = 0;
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            int xx = x + dx, yy = y + dy, zz = z + dz;
                            if (on_boundary(L->n, xx, yy, zz)) continue;
                            cplx coef = (op == OP_Q) ? dQm[abs(dx) + abs(dy) + abs(dz)]
                                                     : Kd[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] /
                                                           (L->ell * L->ell);
                            s += coef * xv[idx3(L->n, xx, yy, zz)];
                        }
                yv[i] = s;
            }
}

/* ------------------------------------------------------------------ */
/* Grid transfers (eq. linear-prolongation, eq. full-weighting)        */
/* ------------------------------------------------------------------ */

/* coarse = R fine: full weighting (1/4, 1/2, 1/4) per axis, tensorised */
static void restrict_fw(const or_level *F, const or_level *C, const cplx *fine, cplx *coarse)
{
    static const double w1[3] = {0.25, 0.5, 0.25};
#pragma omp parallel for schedule(static)
    for (int Z = 0; Z <= C->n[2]; ++Z)
        for (int Y = 0; Y <= C->n[1]; ++Y)
            for (int X = 0; X <= C->n[0]; ++X) {
                size_t o = idx3(C->n, X, Y, Z);
                if (on_boundary(C->n, X, Y, Z)) {
                    coarse[o] = 0;
                    continue;
                }
                cplx s = 0;
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            int x = 2 * X + dx, y = 2 * Y + dy, z = 2 * Z + dz;
                            if (on_boundary(F->n, x, y, z)) continue;
                            s += w1[dx + 1] * w1[dy + 1] * w1[dz + 1] * fine[idx3(F->n, x, y, z)];
                        }
                coarse[o] = s;
            }
}

/* fine = P coarse: (Pw)_{2j} = w_j, (Pw)_{2j+1} = (w_j + w_{j+1})/2 per axis */
static void prolong_lin(const or_level *C, const or_level *F, const cplx *coarse, cplx *fine)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z <= F->n[2]; ++z)
        for (int y = 0; y <= F->n[1]; ++y)
            for (int x = 0; x <= F->n[0]; ++x) {
                int p[3] = {x, y, z};
                int lo[3], hi[3];
                double wl[3], wh[3];
                for (int a = 0; a < 3; ++a) {
                    if (p[a] % 2 == 0) {
                        lo[a] = hi[a] = p[a] / 2;
                        wl[a] = 1.0;
                        wh[a] = 0.0;
                    } else {
                        lo[a] = (p[a] - 1) / 2;
                        hi[a] = (p[a] + 1) / 2;
                        wl[a] = wh[a] = 0.5;
                    }
                }
                cplx s = 0;
                for (int cz = 0; cz < 2; ++cz)
                    for (int cy = 0; cy < 2; ++cy)
                        for (int cx = 0; cx < 2; ++cx) {
                            int X = cx ? hi[0] : lo[0], Y = cy ? hi[1] : lo[1], Z = cz ? hi[2] : lo[2];
                            double w = (cx ? wh[0] : wl[0]) * (cy ? wh[1] : wl[1]) * (cz ? wh[2] : wl[2]);
                            if (w == 0.0 || on_boundary(C->n, X, Y, Z)) continue;
                            s += w * coarse[idx3(C->n, X, Y, Z)];
                        }
                fine[idx3(F->n, x, y, z)] = on_boundary(F->n, x, y, z) ? 0 : s;
            }
}

/* ------------------------------------------------------------------ */
/* Damped Jacobi from zero (eq. jacobi-map)                            */
/* ------------------------------------------------------------------ */

static void jacobi(const or_hier *H, const or_level *L, int op, const cplx *g, int nJ, double wJ, cplx *y)
{
    size_t n = L->nn;
    cplx *r = vnew(n);
    vzero(n, y);
    for (int it = 0; it < nJ; ++it) {
        level_residual(H, L, op, g, y, r);
#pragma omp parallel for schedule(static)
        for (int z = 1; z < L->n[2]; ++z)
            for (int yy = 1; yy < L->n[1]; ++yy)
                for (int x = 1; x < L->n[0]; ++x) {
                    size_t i = idx3(L->n, x, yy, z);
                    y[i] += wJ * r[i] / level_diag(H, L, op, x, yy, z);
                }
    }
    free(r);
}

/* ------------------------------------------------------------------ */
/* Flexible GMRES (Saad 1993), right preconditioned, modified Gram-Schmidt  */
/* ------------------------------------------------------------------ */

typedef void (*or_linop)(const or_hier *H, void *ctx, const cplx *in, cplx *out);

/* x <- result of `cycles` restarted cycles of length m for op x = g started at
 * x (x holds x0 on entry), right preconditioned by prec (stored Z vectors).
 * A cycle ends early on a happy breakdown: the new direction w = op(prec(v_k))
 * lies in the Krylov space, h_{k+1,k} = ||w - V h|| <= 1e-14 ||w|| (a
 * scale-free test: the iterate scales with g).  Returns
 * the number of Arnoldi steps done. */
static int fgmres(const or_hier *H, size_t n, or_linop op, void *opctx, or_linop prec, void *pctx,
                  const cplx *g, cplx *x, int m, int cycles, int x0_is_zero)
{
    cplx **V = (cplx **)calloc((size_t)m + 1, sizeof(cplx *));
    cplx **Z = (cplx **)calloc((size_t)m, sizeof(cplx *));
    for (int j = 0; j <= m; ++j) V[j] = vnew(n);
    for (int j = 0; j < m; ++j) Z[j] = vnew(n);
    cplx *w = vnew(n);
    cplx *Hm = (cplx *)calloc((size_t)(m + 1) * m, sizeof(cplx)); /* Hm[i*m + k] */
    double *cs = (double *)calloc((size_t)m, sizeof(double));
    cplx *sn = (cplx *)calloc((size_t)m, sizeof(cplx));
    cplx *gv = (cplx *)calloc((size_t)m + 1, sizeof(cplx));
    cplx *yv = (cplx *)calloc((size_t)m, sizeof(cplx));
    int steps = 0;
    for (int cyc = 0; cyc < cycles; ++cyc) {
        if (cyc == 0 && x0_is_zero) {
            vcopy(n, g, V[0]);
        } else {
            op(H, opctx, x, w);
            vsub(n, g, w, V[0]);
        }
        double beta = vnorm(n, V[0]);
        if (beta == 0.0) break;
        vscale(n, 1.0 / beta, V[0]);
        memset(gv, 0, sizeof(cplx) * (size_t)(m + 1));
        gv[0] = beta;
        int kk = 0;
        for (int k = 0; k < m; ++k) {
            prec(H, pctx, V[k], Z[k]);
            op(H, opctx, Z[k], w);
            double wn = vnorm(n, w);
            for (int j = 0; j <= k; ++j) {
                cplx hjk = vdot(n, V[j], w);
                Hm[j * m + k] = hjk;
                vaxpy(n, -hjk, V[j], w);
            }
            double hk1 = vnorm(n, w);
            Hm[(k + 1) * m + k] = hk1;
            /* previous Givens rotations on column k */
            for (int j = 0; j < k; ++j) {
                cplx a = Hm[j * m + k], b = Hm[(j + 1) * m + k];
                Hm[j * m + k] = cs[j] * a + sn[j] * b;
                Hm[(j + 1) * m + k] = -conj(sn[j]) * a + cs[j] * b;
            }
            /* new rotation annihilating H[k+1][k] */
            cplx a = Hm[k * m + k];
            double b = creal(Hm[(k + 1) * m + k]);
            double r = sqrt(creal(a * conj(a)) + b * b);
            if (r == 0.0) {
                cs[k] = 1.0;
                sn[k] = 0.0;
            } else if (cabs(a) == 0.0) {
                cs[k] = 0.0;
                sn[k] = 1.0;
            } else {
                cs[k] = cabs(a) / r;
                sn[k] = (a / cabs(a)) * b / r;
            }
            Hm[k * m + k] = cs[k] * a + sn[k] * b;
            Hm[(k + 1) * m + k] = 0.0;
            gv[k + 1] = -conj(sn[k]) * gv[k];
            gv[k] = cs[k] * gv[k];
            kk = k + 1;
            ++steps;
            if (hk1 <= 1e-14 * wn) break;
            vcopy(n, w, V[k + 1]);
            vscale(n, 1.0 / hk1, V[k + 1]);
        }
        /* back substitution R y = g */
        for (int i = kk - 1; i >= 0; --i) {
            cplx s = gv[i];
            for (int j = i + 1; j < kk; ++j) s -= Hm[i * m + j] * yv[j];
            yv[i] = (Hm[i * m + i] == 0.0) ? 0.0 : s / Hm[i * m + i];
        }
        for (int j = 0; j < kk; ++j) vaxpy(n, yv[j], Z[j], x);
    }
    for (int j = 0; j <= m; ++j) free(V[j]);
    for (int j = 0; j < m; ++j) free(Z[j]);
    free(V);
    free(Z);
    free(w);
    free(Hm);
    free(cs);
    free(sn);
    free(gv);
    free(yv);
    return steps;
}

/* ------------------------------------------------------------------ */
/* The nested maps (Sec. 3.2, 3.3)                                      */
/* ------------------------------------------------------------------ */

typedef struct {
    int level, op;
} lvl_op;

typedef struct {
    int level, op, nJ;
    double w;
} jac_ctx;

static void lin_level_op(const or_hier *H, void *ctx, const cplx *in, cplx *out)
{
    lvl_op *c = (lvl_op *)ctx;
    level_apply(H, &H->lev[c->level], c->op, in, out);
}

static void lin_jacobi(const or_hier *H, void *ctx, const cplx *in, cplx *out)
{
    jac_ctx *c = (jac_ctx *)ctx;
    jacobi(H, &H->lev[c->level], c->op, in, c->nJ, c->w, out);
}

/* C_4h(g): m_4h GMRES steps on B_4h e = g from zero, right preconditioned by
 * J_{nJ,4h}(B_4h; omega_4h).  (The paper computes these steps in
 * communication-avoiding form; in exact arithmetic the iterate is the same
 * minimal-residual solution.) */
static void bottom_solve(const or_hier *H, const cplx *g, cplx *e)
{
    lvl_op o = {2, OP_B};
    jac_ctx j = {2, OP_B, H->p.nJ_4h, H->p.omega_4h};
    vzero(H->lev[2].nn, e);
    fgmres(H, H->lev[2].nn, lin_level_op, &o, lin_jacobi, &j, g, e, H->p.m_4h, 1, 1);
}

/* V^sigma_2h(q), eq. shifted-auxiliary-cycle */
static void vcycle(const or_hier *H, const cplx *q, cplx *out)
{
    const or_level *L2 = &H->lev[1], *L4 = &H->lev[2];
    size_t n2 = L2->nn, n4 = L4->nn;
    cplx *y = vnew(n2), *r = vnew(n2), *q4 = vnew(n4), *e4 = vnew(n4), *pe = vnew(n2), *j2 = vnew(n2);
    jacobi(H, L2, OP_B, q, H->p.nJ_2h, H->p.omega_2h, y);       /* y = J(B, q) */
    level_residual(H, L2, OP_B, q, y, r);                       /* q - B y */
    restrict_fw(L2, L4, r, q4);                                 /* q4 = R(q - B y) */
    bottom_solve(H, q4, e4);                                    /* e4 = C_4h(q4) */
    prolong_lin(L4, L2, e4, pe);
    vaxpy(n2, 1.0, pe, y);                                      /* y~ = y + P e4 */
    level_residual(H, L2, OP_B, q, y, r);                       /* q - B y~ */
    jacobi(H, L2, OP_B, r, H->p.nJ_2h, H->p.omega_2h, j2);
    vcopy(n2, y, out);
    vaxpy(n2, 1.0, j2, out);                                    /* y~ + J(B, q - B y~) */
    free(y);
    free(r);
    free(q4);
    free(e4);
    free(pe);
    free(j2);
}

static void lin_vcycle(const or_hier *H, void *ctx, const cplx *in, cplx *out)
{
    (void)ctx;
    vcycle(H, in, out);
}

/* K_2h(r), eq. unshifted-middle-solve: c_2h restarted FGMRES(m_2h) cycles on
 * A_2h from zero, right preconditioned by V^sigma_2h */
static void k2h(const or_hier *H, const cplx *r, cplx *e)
{
    lvl_op o = {1, OP_A};
    vzero(H->lev[1].nn, e);
    fgmres(H, H->lev[1].nn, lin_level_op, &o, lin_vcycle, NULL, r, e, H->p.m_2h, H->p.c_2h, 1);
}

/* S_h(g; x0): one GMRES(m_h) cycle on A_h from x0, right preconditioned by
 * J_{nJ,h}(A_h; omega_h) */
static void smooth(const or_hier *H, const cplx *g, const cplx *x0, int x0_zero, cplx *x)
{
    lvl_op o = {0, OP_A};
    jac_ctx j = {0, OP_A, H->p.nJ_h, H->p.omega_h};
    vcopy(H->lev[0].nn, x0, x);
    fgmres(H, H->lev[0].nn, lin_level_op, &o, lin_jacobi, &j, g, x, H->p.m_h, 1, x0_zero);
}

/* Algorithm 1: z = M_h^{-1} r */
static void precond(const or_hier *H, const cplx *r, cplx *z)
{
    const or_level *L1 = &H->lev[0], *L2 = &H->lev[1];
    size_t n1 = L1->nn, n2 = L2->nn;
    cplx *zpre = vnew(n1), *t = vnew(n1), *r2 = vnew(n2), *e2 = vnew(n2), *pe = vnew(n1);
    smooth(H, r, t, 1, zpre);                              /* 1: z_pre = S_h(r; 0) (t is zero) */
    level_residual(H, L1, OP_A, r, zpre, t);               /* 2: r_2h = R(r - A z_pre) */
    restrict_fw(L1, L2, t, r2);
    k2h(H, r2, e2);                                        /* 3: e_2h = K_2h(r_2h) */
    prolong_lin(L2, L1, e2, pe);                           /* 4: z~ = z_pre + P e_2h */
    vaxpy(n1, 1.0, pe, zpre);
    smooth(H, r, zpre, 0, z);                              /* 5: z = S_h(r; z~) */
    free(zpre);
    free(t);
    free(r2);
    free(e2);
    free(pe);
}

/* ------------------------------------------------------------------ */
/* Exported C API (loaded with ctypes by the tests)                    */
/* ------------------------------------------------------------------ */

/* params: sigma, omega_h, omega_2h, omega_4h, gamma_max, nJ_h, nJ_2h, nJ_4h,
 *         m_h, c_2h, m_2h, m_4h, m_out, pml_variant  (14 doubles) */
int or_create(const float *vel_phys, int nx, int ny, int nz, double h, double omega, int n_pml,
              const double *table, int K, double eta_max, const double *params, void **out)
{
    if (!vel_phys || !table || !out || K < 1 || n_pml < 0 || h <= 0 || omega <= 0) return OR_EINVAL;
    int N[3] = {nx + 2 * n_pml, ny + 2 * n_pml, nz + 2 * n_pml};
    for (int a = 0; a < 3; ++a)
        if (N[a] % 4 != 0 || N[a] < 4) return OR_EINVAL;
    or_hier *H = (or_hier *)calloc(1, sizeof(or_hier));
    H->h = h;
    H->omega = omega;
    H->n_pml = n_pml;
    H->K = K;
    H->eta_max = eta_max;
    double *tab = (double *)malloc(sizeof(double) * (size_t)(K + 1) * 16);
    memcpy(tab, table, sizeof(double) * (size_t)(K + 1) * 16);
    H->tab = tab;
    H->p.sigma = params[0];
    H->p.omega_h = params[1];
    H->p.omega_2h = params[2];
    H->p.omega_4h = params[3];
    H->p.gamma_max = params[4];
    H->p.nJ_h = (int)params[5];
    H->p.nJ_2h = (int)params[6];
    H->p.nJ_4h = (int)params[7];
    H->p.m_h = (int)params[8];
    H->p.c_2h = (int)params[9];
    H->p.m_2h = (int)params[10];
    H->p.m_4h = (int)params[11];
    H->p.m_out = (int)params[12];
    H->p.pml_variant = (int)params[13];
    for (int a = 0; a < 3; ++a) H->lev[0].n[a] = N[a];
    int nphys[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) H->nphys[a] = nphys[a];
    size_t nv = (size_t)(nx + 1) * (ny + 1) * (nz + 1);
    double *vd = (double *)malloc(nv * sizeof(double));
    for (size_t i = 0; i < nv; ++i) vd[i] = (double)vel_phys[i];
    for (int l = 0; l < 3; ++l) {
        if (level_init(H, l, vd, nphys) != OR_OK) {
            free(vd);
            return OR_ENOMEM;
        }
    }
    free(vd);
    *out = H;
    return OR_OK;
}

void or_destroy(void *p)
{
    or_hier *H = (or_hier *)p;
    if (!H) return;
    for (int l = 0; l < 3; ++l) {
        free(H->lev[l].c);
        for (int a = 0; a < 3; ++a) {
            free(H->lev[l].xin[a]);
            free(H->lev[l].xih[a]);
        }
    }
    free((void *)H->tab);
    free(H);
}

int or_dims(void *p, int level, int dims[3])
{
    or_hier *H = (or_hier *)p;
    if (level < 0 || level > 2) return OR_EINVAL;
    for (int a = 0; a < 3; ++a) dims[a] = H->lev[level].n[a];
    return OR_OK;
}

/* velocity on the nodes of a level (FP64 copy of the extended, injected field) */
int or_level_velocity(void *p, int level, double *out)
{
    or_hier *H = (or_hier *)p;
    if (level < 0 || level > 2) return OR_EINVAL;
    memcpy(out, H->lev[level].c, H->lev[level].nn * sizeof(double));
    return OR_OK;
}

/* 1/xi at nodes (n+1) and half nodes (n) of one axis of one level */
int or_level_xi(void *p, int level, int axis, double *node, double *half)
{
    or_hier *H = (or_hier *)p;
    if (level < 0 || level > 2 || axis < 0 || axis > 2) return OR_EINVAL;
    const or_level *L = &H->lev[level];
    memcpy(node, L->xin[axis], sizeof(cplx) * (size_t)(L->n[axis] + 1));
    memcpy(half, L->xih[axis], sizeof(cplx) * (size_t)L->n[axis]);
    return OR_OK;
}

int or_apply(void *p, int level, int op, const double *x, double *y)
{
    or_hier *H = (or_hier *)p;
    if (level < 0 || level > 2 || op < 0 || op > 4 || (op == OP_Q && level != 0)) return OR_EINVAL;
    level_apply(H, &H->lev[level], op, (const cplx *)x, (cplx *)y);
    return OR_OK;
}

/* rows at selected flat node indices only (for sampled checks on big grids) */
int or_apply_at(void *p, int level, int op, const double *x, const long long *nodes, long long npts, double *y)
{
    or_hier *H = (or_hier *)p;
    if (level < 0 || level > 2 || op < 0 || op > 4 || (op == OP_Q && level != 0)) return OR_EINVAL;
    const or_level *L = &H->lev[level];
#pragma omp parallel for schedule(static)
    for (long long q = 0; q < npts; ++q) {
        long long i = nodes[q];
        int x0 = (int)(i % (L->n[0] + 1));
        int y0 = (int)((i / (L->n[0] + 1)) % (L->n[1] + 1));
        int z0 = (int)(i / ((long long)(L->n[0] + 1) * (L->n[1] + 1)));
        ((cplx *)y)[q] = apply_row(H, L, op, (const cplx *)x, x0, y0, z0);
    }
    return OR_OK;
}

int or_residual(void *p, int level, int op, const double *g, const double *x, double *r)
{
    or_hier *H = (or_hier *)p;
    if (level < 0 || level > 2 || (op != OP_A && op != OP_B)) return OR_EINVAL;
    level_residual(H, &H->lev[level], op, (const cplx *)g, (const cplx *)x, (cplx *)r);
    return OR_OK;
}

/* coarse = R_level fine, fine on `level`, coarse on level+1 */
int or_restrict(void *p, int level, const double *fine, double *coarse)
{
    or_hier *H = (or_hier *)p;
    if (level < 0 || level > 1) return OR_EINVAL;
    restrict_fw(&H->lev[level], &H->lev[level + 1], (const cplx *)fine, (cplx *)coarse);
    return OR_OK;
}

/* fine = P coarse, coarse on `level` (1 or 2), fine on level-1 */
int or_prolong(void *p, int level, const double *coarse, double *fine)
{
    or_hier *H = (or_hier *)p;
    if (level < 1 || level > 2) return OR_EINVAL;
    prolong_lin(&H->lev[level], &H->lev[level - 1], (const cplx *)coarse, (cplx *)fine);
    return OR_OK;
}

int or_jacobi(void *p, int level, int op, const double *g, int nJ, double wJ, double *y)
{
    or_hier *H = (or_hier *)p;
    if (level < 0 || level > 2 || (op != OP_A && op != OP_B) || nJ < 0) return OR_EINVAL;
    jacobi(H, &H->lev[level], op, (const cplx *)g, nJ, wJ, (cplx *)y);
    return OR_OK;
}

/* Generic right-preconditioned GMRES on one level (operator op, Jacobi
 * preconditioner J_nJ(op; wJ), or the identity when nJ == 0), started from x
 * (x0 on entry).  Returns the number of Arnoldi steps. */
static void lin_identity(const or_hier *H, void *ctx, const cplx *in, cplx *out)
{
    lvl_op *c = (lvl_op *)ctx;
    vcopy(H->lev[c->level].nn, in, out);
}

int or_gmres(void *p, int level, int op, int nJ, double wJ, const double *g, double *x, int m, int cycles)
{
    or_hier *H = (or_hier *)p;
    if (level < 0 || level > 2 || (op != OP_A && op != OP_B) || m < 1 || cycles < 1 || nJ < 0) return OR_EINVAL;
    size_t n = H->lev[level].nn;
    lvl_op o = {level, op};
    jac_ctx j = {level, op, nJ, wJ};
    int zero = 1;
    for (size_t i = 0; i < 2 * n; ++i)
        if (x[i] != 0.0) {
            zero = 0;
            break;
        }
    if (nJ == 0)
        return fgmres(H, n, lin_level_op, &o, lin_identity, &o, (const cplx *)g, (cplx *)x, m, cycles, zero);
    return fgmres(H, n, lin_level_op, &o, lin_jacobi, &j, (const cplx *)g, (cplx *)x, m, cycles, zero);
}

int or_bottom(void *p, const double *g, double *e)
{
    bottom_solve((or_hier *)p, (const cplx *)g, (cplx *)e);
    return OR_OK;
}

int or_vcycle(void *p, const double *q, double *y)
{
    vcycle((or_hier *)p, (const cplx *)q, (cplx *)y);
    return OR_OK;
}

int or_k2h(void *p, const double *r, double *e)
{
    k2h((or_hier *)p, (const cplx *)r, (cplx *)e);
    return OR_OK;
}

int or_smooth(void *p, const double *g, const double *x0, double *x)
{
    or_hier *H = (or_hier *)p;
    size_t n = H->lev[0].nn;
    int zero = 1;
    for (size_t i = 0; i < 2 * n; ++i)
        if (x0[i] != 0.0) {
            zero = 0;
            break;
        }
    smooth(H, (const cplx *)g, (const cplx *)x0, zero, (cplx *)x);
    return OR_OK;
}

int or_precond(void *p, const double *r, double *z)
{
    precond((or_hier *)p, (const cplx *)r, (cplx *)z);
    return OR_OK;
}

/* A_h (transposed = 0) or A_h^T (transposed = 1) on level 0 */
static void outer_apply(const or_hier *H, int transposed, const cplx *x, cplx *y)
{
    if (transposed)
        level_apply_t(H, &H->lev[0], OP_A, x, y);
    else
        level_apply(H, &H->lev[0], OP_A, x, y);
}

/* v <- outer FGMRES(m_out) for (A_h or A_h^T) v = b from v = 0, right preconditioned by
 * M_h^{-1} (Algorithm 1).  Each cycle ends when the Arnoldi estimate of the relative
 * residual drops to tol; convergence is decided on the recomputed residual
 * ||b - A v|| / ||b|| (eq. relative-residual).  Returns 0 when converged, 1 when
 * max_outer preconditioner calls were spent first.  max_outer <= 0 means no limit. */
static int outer_fgmres(const or_hier *H, int transposed, const cplx *b, cplx *v, double tol, int max_outer,
                        int *iters, double *relres)
{
    const or_level *L = &H->lev[0];
    size_t n = L->nn;
    int m = H->p.m_out;
    cplx *r = vnew(n), *w = vnew(n);
    cplx **V = (cplx **)calloc((size_t)m + 1, sizeof(cplx *));
    cplx **Z = (cplx **)calloc((size_t)m, sizeof(cplx *));
    for (int j = 0; j <= m; ++j) V[j] = vnew(n);
    for (int j = 0; j < m; ++j) Z[j] = vnew(n);
    cplx *Hm = (cplx *)calloc((size_t)(m + 1) * m, sizeof(cplx));
    double *cs = (double *)calloc((size_t)m, sizeof(double));
    cplx *sn = (cplx *)calloc((size_t)m, sizeof(cplx));
    cplx *gv = (cplx *)calloc((size_t)m + 1, sizeof(cplx));
    cplx *yv = (cplx *)calloc((size_t)m, sizeof(cplx));
    vzero(n, v);
    double bn = vnorm(n, b);
    int its = 0, status = 0;
    double rel = 0.0;
    if (bn > 0.0) {
        for (;;) {
            outer_apply(H, transposed, v, r);   /* r = b - A v, zero on the boundary */
            for (int z = 0; z <= L->n[2]; ++z)
                for (int y = 0; y <= L->n[1]; ++y)
                    for (int x = 0; x <= L->n[0]; ++x) {
                        size_t i = idx3(L->n, x, y, z);
                        r[i] = on_boundary(L->n, x, y, z) ? 0 : b[i] - r[i];
                    }
            double beta = vnorm(n, r);
            rel = beta / bn;
            if (rel <= tol) break;
            if (max_outer > 0 && its >= max_outer) {
                status = 1;
                break;
            }
            vcopy(n, r, V[0]);
            vscale(n, 1.0 / beta, V[0]);
            memset(gv, 0, sizeof(cplx) * (size_t)(m + 1));
            gv[0] = beta;
            int kk = 0;
            for (int k = 0; k < m; ++k) {
                precond(H, V[k], Z[k]);
                ++its;
                outer_apply(H, transposed, Z[k], w);
                double wn = vnorm(n, w);
                for (int j = 0; j <= k; ++j) {
                    cplx hjk = vdot(n, V[j], w);
                    Hm[j * m + k] = hjk;
                    vaxpy(n, -hjk, V[j], w);
                }
                double hk1 = vnorm(n, w);
                Hm[(k + 1) * m + k] = hk1;
                for (int j = 0; j < k; ++j) {
                    cplx a = Hm[j * m + k], bb = Hm[(j + 1) * m + k];
                    Hm[j * m + k] = cs[j] * a + sn[j] * bb;
                    Hm[(j + 1) * m + k] = -conj(sn[j]) * a + cs[j] * bb;
                }
                cplx a = Hm[k * m + k];
                double bb = hk1;
                double rr = sqrt(creal(a * conj(a)) + bb * bb);
                if (rr == 0.0) {
                    cs[k] = 1.0;
                    sn[k] = 0.0;
                } else if (cabs(a) == 0.0) {
                    cs[k] = 0.0;
                    sn[k] = 1.0;
                } else {
                    cs[k] = cabs(a) / rr;
                    sn[k] = (a / cabs(a)) * bb / rr;
                }
                Hm[k * m + k] = cs[k] * a + sn[k] * bb;
                Hm[(k + 1) * m + k] = 0.0;
                gv[k + 1] = -conj(sn[k]) * gv[k];
                gv[k] = cs[k] * gv[k];
                kk = k + 1;
                if (cabs(gv[k + 1]) / bn <= tol || hk1 <= 1e-14 * wn) break;
                if (max_outer > 0 && its >= max_outer) break;
                vcopy(n, w, V[k + 1]);
                vscale(n, 1.0 / hk1, V[k + 1]);
            }
            for (int i = kk - 1; i >= 0; --i) {
                cplx s = gv[i];
                for (int j = i + 1; j < kk; ++j) s -= Hm[i * m + j] * yv[j];
                yv[i] = (Hm[i * m + i] == 0.0) ? 0.0 : s / Hm[i * m + i];
            }
            for (int j = 0; j < kk; ++j) vaxpy(n, yv[j], Z[j], v);
        }
    }
    *iters = its;
    *relres = rel;
    for (int j = 0; j <= m; ++j) free(V[j]);
    for (int j = 0; j < m; ++j) free(Z[j]);
    free(V);
    free(Z);
    free(Hm);
    free(cs);
    free(sn);
    free(gv);
    free(yv);
    free(r);
    free(w);
    return status;
}

/* Outer FGMRES(m_out) for A_h v = Q_h f (eq. iofd-complete-system), right preconditioned by
 * M_h^{-1} (Algorithm 1), from v = 0 (see outer_fgmres).  Writes u = Q_h v.  Returns 0
 * when converged, 1 when max_outer preconditioner calls were spent first. */
int or_solve(void *p, const double *f, double tol, int max_outer, double *u, int *iters, double *relres)
{
    or_hier *H = (or_hier *)p;
    const or_level *L = &H->lev[0];
    size_t n = L->nn;
    cplx *b = vnew(n), *v = vnew(n);
    level_apply(H, L, OP_Q, (const cplx *)f, b);
    int status = outer_fgmres(H, 0, b, v, tol, max_outer, iters, relres);
    level_apply(H, L, OP_Q, v, (cplx *)u);
    free(b);
    free(v);
    return status;
}

/* y = op^T x (op A or B on any level, Q on level 0) */
int or_apply_t(void *p, int level, int op, const double *x, double *y)
{
    or_hier *H = (or_hier *)p;
    if (level < 0 || level > 2 || (op != OP_A && op != OP_B && op != OP_Q) || (op == OP_Q && level != 0))
        return OR_EINVAL;
    level_apply_t(H, &H->lev[level], op, (const cplx *)x, (cplx *)y);
    return OR_OK;
}

/* y_i = (d_i op x)_i on level 0, op A or Q (derivative of row i in m_i = 1/c_i^2) */
int or_apply_dm(void *p, int op, const double *x, double *y)
{
    or_hier *H = (or_hier *)p;
    if (op != OP_A && op != OP_Q) return OR_EINVAL;
    level_apply_dm(H, op, (const cplx *)x, (cplx *)y);
    return OR_OK;
}

/* Gradient of a misfit J(u), u = Q_h v, A_h v = Q_h f, with respect to the squared slowness
 * m = 1/c^2 at the physical nodes, for the adjoint source s (dJ = Re sum_i conj(s_i) du_i).
 * Differentiating the state equation: du = dQ v + Q dv and A dv = dQ f - dA v, so with
 * A^T mu = Q^T conj(s),
 *   dJ = Re sum_i dm_i [ conj(s_i) (d_i Q v)_i + mu_i ((d_i Q f)_i - (d_i A v)_i) ],
 * every row depending on the m of its own node.  A PML node carries the m of its nearest
 * physical node, so its term adds onto that node.  Both solves run to tol.  iters and
 * relres receive the forward then the adjoint counts. */
int or_grad(void *p, const double *f, const double *s, double tol, double *grad_phys, int *iters, double *relres)
{
    or_hier *H = (or_hier *)p;
    const or_level *L = &H->lev[0];
    size_t n = L->nn;
    const cplx *fv = (const cplx *)f, *sv = (const cplx *)s;
    cplx *b = vnew(n), *v = vnew(n), *mu = vnew(n), *sc = vnew(n);
    cplx *dAv = vnew(n), *dQv = vnew(n), *dQf = vnew(n);
    level_apply(H, L, OP_Q, fv, b);
    int st = outer_fgmres(H, 0, b, v, tol, 0, &iters[0], &relres[0]);
    for (size_t i = 0; i < n; ++i) sc[i] = conj(sv[i]);
    level_apply_t(H, L, OP_Q, sc, b);                   /* Q^T conj(s) */
    st |= outer_fgmres(H, 1, b, mu, tol, 0, &iters[1], &relres[1]);
    level_apply_dm(H, OP_A, v, dAv);
    level_apply_dm(H, OP_Q, v, dQv);
    level_apply_dm(H, OP_Q, fv, dQf);
    const int *np = H->nphys;
    memset(grad_phys, 0, sizeof(double) * (size_t)(np[0] + 1) * (np[1] + 1) * (np[2] + 1));
    for (int z = 1; z < L->n[2]; ++z)
        for (int y = 1; y < L->n[1]; ++y)
            for (int x = 1; x < L->n[0]; ++x) {
                size_t i = idx3(L->n, x, y, z);
                double gi = creal(conj(sv[i]) * dQv[i] + mu[i] * (dQf[i] - dAv[i]));
                int q[3] = {x - H->n_pml, y - H->n_pml, z - H->n_pml};
                for (int a = 0; a < 3; ++a) {
                    if (q[a] < 0) q[a] = 0;
                    if (q[a] > np[a]) q[a] = np[a];
                }
                grad_phys[((size_t)q[2] * (np[1] + 1) + q[1]) * (np[0] + 1) + q[0]] += gi;
            }
    free(b);
    free(v);
    free(mu);
    free(sc);
    free(dAv);
    free(dQv);
    free(dQf);
    return st;
}
