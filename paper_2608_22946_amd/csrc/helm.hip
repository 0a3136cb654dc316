// Operator hierarchy, nested Krylov drivers and the C ABI (include/helm.h).
//
// Everything a solve does is enqueued on the caller's stream: the level
// operators, transfers and vector kernels run on the GPU and the small dense
// work (Givens rotations, back substitution, the s-step Gram solve) runs in
// the last block of the reduction kernels, so a preconditioner application
// (Algorithm 1) needs no host synchronisation.  The host reads one Krylov
// state per outer Arnoldi step for the convergence test.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "helm_internal.h"

using namespace helm;

namespace {
thread_local std::string g_thread_error;
}

constexpr int kMaxLanes = 8;   // right-hand sides solved concurrently by helm_solve
constexpr int kMaxBatch = 8;   // right-hand sides one lane advances together (slots)
static_assert(sizeof(KState) % sizeof(double) == 0, "KState strides are counted in doubles");
constexpr int kKStateDoubles = (int)(sizeof(KState) / sizeof(double));
// device and pinned host scratch of a lane: EPI_STORE results of every slot (2 kRedSlots doubles each)
constexpr int kScratchDoubles = 2 * kRedSlots * kMaxBatch > 256 ? 2 * kRedSlots * kMaxBatch : 256;

// Everything one solve writes: Krylov vectors of the three levels, solver
// states, reduction buffers, pinned host copies and the stream it runs on.
struct Lane {
    void *Vout[kMMax + 1], *Zout[kMMax];
    void *Vs[kMMax + 1], *Zs[kMMax];
    c64 *x64, *b64;
    void *V2[kMMax + 1], *Z2[kMMax];
    void *e2, *r2, *vy, *vr;
    void *P4[kM4Max + 1], *Z4[kM4Max];
    void *e4;
    void *tmp[3];
    void *wrest[2];       // x/z-restricted residual rows (fused residual + full weighting from level l)
    KState *st_outer, *st_smooth, *st_k2h, *st_bottom, *st_hook;
    RedBuf rb;
    double *dscratch;     // small device result buffer (dots, velocity check)
    KState *host_state;   // pinned host copies of the Krylov states of the lane's slots
    double *host_scratch; // pinned host doubles
    int nslot;            // right-hand sides the lane advances together (helm_options.batch)
    long long pstride;    // doubles of reduction partials per slot
    hipStream_t s;        // lane 0: the caller's stream; others: created by helm_setup (default priority)
    bool own_stream;
    std::string err;
};

struct helm_hierarchy {
    helm_options opt;
    helm_precision prec;
    int nphys[3];
    int n_pml;
    double h, omega;
    double cmin, cmax;   // velocity range (the level velocities lie inside it)
    hipStream_t s;
    Geom geom[3];
    LevelArgs<float> Lf[3];
    LevelArgs<double> Ld[3];
    // device buffers carved from the caller's workspace: shared, read-only during solves
    float *vel[3];
    float *svel[3];      // FP32 mode: the scaled interpolation coordinate per node (LevelArgs::s)
    void *dinv[3][2];    // D^-1 of A_l and B_l per level, in the working precision
    float *wf[3][3];
    double *wd[3][3];
    float *atab_f, *btab_f, *ctab_f;
    double *atab_d, *btab_d;
    // HELM_MIXED: FP16-stored vectors hold v * f * qs (helm_internal.h), f = fres[l] for
    // residual-like vectors (the cycle input, residuals, the bottom basis P) and fsol[l]
    // for correction-like ones (Jacobi iterates, corrections, Z); d_one is the qs of
    // normalised cycle inputs
    float fres[3], fsol[3];
    double *d_one;
    int nlanes;
    Lane lane[kMaxLanes];
    std::string err;
};

namespace helm {
helm_status thread_error(helm_status st, const char *msg) {
    g_thread_error = msg;
    return st;
}
}  // namespace helm

namespace {

std::mutex g_err_mutex;   // lanes of one helm_solve may report errors concurrently

helm_status fail(helm_hierarchy *H, helm_status st, const std::string &msg) {
    if (H) {
        std::lock_guard<std::mutex> lock(g_err_mutex);
        H->err = msg;
    } else {
        g_thread_error = msg;
    }
    return st;
}

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail(H, HELM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define HIP_CHK(expr)                         \
    do {                                      \
        hipError_t e_ = (expr);               \
        if (e_ != hipSuccess) return e_;      \
    } while (0)

// ---------------------------------------------------------------------------
// Workspace layout
// ---------------------------------------------------------------------------
struct Carver {
    char *base;
    size_t off = 0;
    template <typename X>
    X *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        X *p = base ? reinterpret_cast<X *>(base + off) : nullptr;
        off += count * sizeof(X);
        return p;
    }
};

void level_geom(const int N[3], int l, double h, Geom &g) {
    const int s = 1 << l;
    for (int a = 0; a < 3; ++a) g.n[a] = N[a] / s;
    g.sx = g.n[0] + 1;
    g.sy = (long long)(g.n[0] + 1) * (g.n[1] + 1);
    g.nn = g.sy * (g.n[2] + 1);
    g.ell = s * h;
}

// Lay out (or size, when base == nullptr) every device buffer.
size_t carve(helm_hierarchy *H, char *base, const int N[3], const helm_options &o, int K) {
    Carver c{base};
    Geom g[3];
    for (int l = 0; l < 3; ++l) level_geom(N, l, 1.0, g[l]);
    const size_t es = (o.precision == HELM_FP64) ? sizeof(c64) : sizeof(c32);
    auto vec = [&](int l) { return c.take<char>(es * (size_t)g[l].nn); };
    // the preconditioner's inner vectors: FP16-stored in HELM_MIXED
    const size_t es16 = (o.precision == HELM_MIXED) ? sizeof(c16) : es;
    // a lane's vectors hold one copy per batched slot, slot s at s times the vector's length
    const int B = (o.batch > 1) ? o.batch : 1;
    auto lvec = [&](int l) { return c.take<char>(es * (size_t)g[l].nn * B); };
    auto lvec16 = [&](int l) { return c.take<char>(es16 * (size_t)g[l].nn * B); };
    helm_hierarchy dummy;
    helm_hierarchy *Hp = H ? H : &dummy;
    for (int l = 0; l < 3; ++l) {
        Hp->vel[l] = c.take<float>(g[l].nn);
        Hp->svel[l] = (o.precision == HELM_FP64) ? nullptr : c.take<float>(g[l].nn);
        for (int sh = 0; sh < 2; ++sh) Hp->dinv[l][sh] = vec(l);
        for (int a = 0; a < 3; ++a) {
            Hp->wf[l][a] = c.take<float>(6 * (size_t)(g[l].n[a] + 1));
            Hp->wd[l][a] = c.take<double>(6 * (size_t)(g[l].n[a] + 1));
        }
    }
    Hp->atab_f = c.take<float>(20 * (size_t)K);
    Hp->btab_f = c.take<float>(12 * (size_t)K);
    Hp->ctab_f = c.take<float>(24 * (size_t)(K + 1));
    Hp->d_one = c.take<double>(1);
    Hp->atab_d = c.take<double>(20 * (size_t)K);
    Hp->btab_d = c.take<double>(12 * (size_t)K);
    const int nl = (o.lanes > 1) ? o.lanes : 1;
    if (H) H->nlanes = nl;
    for (int li = 0; li < nl; ++li) {
        Lane &Ln = Hp->lane[li];
        for (int j = 0; j <= o.m_out; ++j) Ln.Vout[j] = lvec(0);
        for (int j = 0; j < o.m_out; ++j) Ln.Zout[j] = lvec(0);
        for (int j = 0; j <= o.m_h; ++j) Ln.Vs[j] = lvec(0);
        for (int j = 0; j < o.m_h; ++j) Ln.Zs[j] = lvec(0);
        Ln.x64 = c.take<c64>(g[0].nn * B);
        Ln.b64 = c.take<c64>(g[0].nn * B);
        for (int j = 0; j <= o.m_2h; ++j) Ln.V2[j] = lvec(1);
        for (int j = 0; j < o.m_2h; ++j) Ln.Z2[j] = lvec16(1);
        Ln.e2 = lvec(1);
        Ln.r2 = lvec(1);
        Ln.vy = lvec16(1);
        Ln.vr = lvec16(1);
        for (int j = 0; j <= o.m_4h; ++j) Ln.P4[j] = lvec16(2);
        for (int j = 0; j < o.m_4h; ++j) Ln.Z4[j] = lvec16(2);
        Ln.e4 = lvec16(2);
        for (int l = 0; l < 3; ++l) Ln.tmp[l] = lvec(l);
        for (int l = 0; l < 2; ++l)
            Ln.wrest[l] = c.take<char>(es * (size_t)(g[l].n[2] / 2 + 1) * (g[l].n[1] + 1) * (g[l].n[0] / 2 + 1) * B);
        Ln.st_outer = c.take<KState>(B);
        Ln.st_smooth = c.take<KState>(B);
        Ln.st_k2h = c.take<KState>(B);
        Ln.st_bottom = c.take<KState>(B);
        Ln.st_hook = c.take<KState>(1);
        size_t np = (size_t)kRedBlocks * 2 * 48;
        for (int l = 0; l < 3; ++l)
            np = std::max(np, (size_t)stencil_blocks(g[l].n[0], g[l].n[1], g[l].n[2], kTzMin));
        Ln.rb.partials = c.take<double>(np * B);
        Ln.nslot = B;
        Ln.pstride = (long long)np;
        Ln.rb.counter = c.take<unsigned>(64);
        // small results: 256 doubles, or 2 kRedSlots per slot for the batched norms of the outer solve
        Ln.dscratch = c.take<double>(kScratchDoubles);
    }
    return c.off + 256;
}

// Per-axis stretching of one level (eq. pml-profile): gamma at the nodes,
// averaged to the half nodes before inversion; second-difference weights
// wm = -xi_a^-1 xi_{a-1/2}^-1, wc = xi_a^-1 (xi_{a+1/2}^-1 + xi_{a-1/2}^-1),
// wp = -xi_a^-1 xi_{a+1/2}^-1 (eq. pml-second-difference).
// gamma of eq. pml-profile at coordinate x of an axis of length L (helm_options.pml_variant:
// 2 = the profile reaches gamma_max at d = Lpml - h)
double pml_gamma(double x, double L, double Lpml, double h, double gmax, int variant) {
    if (Lpml <= 0) return 0.0;
    double d = std::max(0.0, std::max(Lpml - x, x - (L - Lpml)));
    const double Lp = (variant == 2) ? Lpml - h : Lpml;
    d = std::min(d, Lp);
    return gmax * (1.0 - std::cos(M_PI * d / (2.0 * Lp)));
}

void axis_weights(int n, double ell, double L, double Lpml, double h, double gmax, int variant,
                  std::vector<double> &w, int &lo, int &hi) {
    std::vector<double> gam(n + 1);
    for (int j = 0; j <= n; ++j) gam[j] = pml_gamma(j * ell, L, Lpml, h, gmax, variant);
    // half-node gamma: the mean of the node values (variant 1: at the half-node distance)
    auto half = [&](int j) {   // between nodes j and j + 1
        return (variant == 1) ? pml_gamma((j + 0.5) * ell, L, Lpml, h, gmax, variant)
                              : 0.5 * (gam[j] + gam[j + 1]);
    };
    auto inv = [](double g, double &re, double &im) {   // 1 / (1 + i g)
        const double den = 1.0 + g * g;
        re = 1.0 / den;
        im = -g / den;
    };
    w.assign(6 * (size_t)(n + 1), 0.0);
    for (int j = 1; j <= n - 1; ++j) {
        double nr, ni, pr, pi, mr, mi;
        inv(gam[j], nr, ni);
        inv(half(j), pr, pi);
        inv(half(j - 1), mr, mi);
        double *o = &w[6 * j];
        o[0] = -(nr * mr - ni * mi);
        o[1] = -(nr * mi + ni * mr);
        o[2] = nr * (pr + mr) - ni * (pi + mi);
        o[3] = nr * (pi + mi) + ni * (pr + mr);
        o[4] = -(nr * pr - ni * pi);
        o[5] = -(nr * pi + ni * pr);
    }
    lo = n;
    hi = 0;
    for (int j = 1; j <= n - 1; ++j)
        if (gam[j - 1] == 0.0 && gam[j] == 0.0 && gam[j + 1] == 0.0) {
            lo = std::min(lo, j);
            hi = std::max(hi, j);
        }
}

// Hermite nodes (value, slope) -> monomial coefficients in t on each interval
void hermite_monomials(const double *tab, int K, int f0, int nf, std::vector<double> &out) {
    const double de = 0.4 / K;
    out.assign((size_t)K * nf * 4, 0.0);
    for (int k = 0; k < K; ++k)
        for (int f = 0; f < nf; ++f) {
            const double p0 = tab[(k * 8 + f0 + f) * 2], m0 = de * tab[(k * 8 + f0 + f) * 2 + 1];
            const double p1 = tab[((k + 1) * 8 + f0 + f) * 2], m1 = de * tab[((k + 1) * 8 + f0 + f) * 2 + 1];
            double *c = &out[((size_t)k * nf + f) * 4];
            c[0] = p0;
            c[1] = m0;
            c[2] = -3 * p0 - 2 * m0 + 3 * p1 - m1;
            c[3] = 2 * p0 + m0 - 2 * p1 + m1;
        }
}

// The unshifted shell coefficients (eq. iofd-shell-coefficients with mu = 1) as quintics in
// the local coordinate t of each table interval: with a_j(t) the cubic Hermite pieces (monomial
// form `at`, K intervals) and kappa^2 = (2 pi deta (k + t))^2,
//   C_0 = 6 a4 - kappa^2 a1,  C_1 = a5 - a4 - kappa^2 a2 / 6,
//   C_2 = (1 - a4 - a5) / 2 - a5 / 2 - kappa^2 a3 / 12,
//   C_3 = -3 (1 - a4 - a5) / 4 - kappa^2 (1 - a1 - a2 - a3) / 8;
// interval K is the clamped range eta* = 0.4 (a_j at the last node, s = K + t).
void shell_quintics(const std::vector<double> &at, int K, std::vector<double> &out) {
    out.assign((size_t)(K + 1) * 24, 0.0);
    const double w = 2.0 * M_PI * 0.4 / K;
    for (int k = 0; k <= K; ++k) {
        double a[5][4];   // a_j as cubics in t
        for (int j = 0; j < 5; ++j)
            for (int d = 0; d < 4; ++d) {
                if (k < K) {
                    a[j][d] = at[((size_t)k * 5 + j) * 4 + d];
                } else {   // value at the end of the last interval, constant in t
                    const double *p = &at[((size_t)(K - 1) * 5 + j) * 4];
                    a[j][d] = d == 0 ? p[0] + p[1] + p[2] + p[3] : 0.0;
                }
            }
        const double k2[3] = {w * w * k * k, 2.0 * w * w * k, w * w};   // kappa^2 in t
        double stiff[4][4] = {}, mass[4][4] = {};
        for (int d = 0; d < 4; ++d) {
            const double q = (d == 0 ? 1.0 : 0.0) - a[3][d] - a[4][d];
            stiff[0][d] = 6.0 * a[3][d];
            stiff[1][d] = a[4][d] - a[3][d];
            stiff[2][d] = 0.5 * q - 0.5 * a[4][d];
            stiff[3][d] = -0.75 * q;
            mass[0][d] = a[0][d];
            mass[1][d] = a[1][d] / 6.0;
            mass[2][d] = a[2][d] / 12.0;
            mass[3][d] = ((d == 0 ? 1.0 : 0.0) - a[0][d] - a[1][d] - a[2][d]) / 8.0;
        }
        for (int m = 0; m < 4; ++m) {
            double *c = &out[((size_t)k * 4 + m) * 6];
            for (int d = 0; d < 4; ++d) {
                c[d] += stiff[m][d];
                for (int e = 0; e < 3; ++e) c[d + e] -= k2[e] * mass[m][d];
            }
        }
    }
}

template <typename R>
void fill_level_args(helm_hierarchy *H, int l, LevelArgs<R> &L, const R *wx, const R *wy, const R *wz, const R *at,
                     const R *bt) {
    const Geom &g = H->geom[l];
    L.nx = g.n[0];
    L.ny = g.n[1];
    L.nz = g.n[2];
    L.sx = g.sx;
    L.sy = g.sy;
    L.lox = g.lo[0]; L.hix = g.hi[0];
    L.loy = g.lo[1]; L.hiy = g.hi[1];
    L.loz = g.lo[2]; L.hiz = g.hi[2];
    L.c = H->vel[l];
    L.wx = wx;
    L.wy = wy;
    L.wz = wz;
    L.atab = at;
    L.btab = bt;
    L.K = H->opt.iofd_K;
    L.inv_deta = (R)(H->opt.iofd_K / 0.4);
    L.omega_ell = (R)(H->omega * g.ell);
    L.inv_ell2 = (R)(1.0 / (g.ell * g.ell));
    L.sigma = (R)H->opt.sigma;
    L.tz[0] = L.tz[1] = 0;
    L.split[0] = L.split[1] = 0;
    // D^-1 exists in the working precision only (the other LevelArgs serve the
    // FP64 outer residual and Q_h, which do not use it)
    const bool own = (sizeof(R) == sizeof(double)) == (H->prec == HELM_FP64);
    for (int sh = 0; sh < 2; ++sh) L.dinv[sh] = own ? static_cast<const R *>(H->dinv[l][sh]) : nullptr;
    const bool fp32 = sizeof(R) == sizeof(float) && H->prec != HELM_FP64;
    L.s = fp32 ? H->svel[l] : nullptr;
    L.ctab = fp32 ? reinterpret_cast<const R *>(H->ctab_f) : nullptr;
    L.kap_s = (R)(2.0 * M_PI * 0.4 / H->opt.iofd_K);
    // table window: the interval of a node is monotone in its velocity, so the velocity
    // range [cmin, cmax] bounds it; the same formulas as the kernels (locate / locate_s,
    // shell_at_s), widened by one interval each side against rounding
    const int K = H->opt.iofd_K;
    auto clampi = [](int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); };
    int ka, kz, ca = 0, cz = K;
    if (fp32) {
        const double factor = H->omega * g.ell * K / (0.4 * 2.0 * M_PI);
        const float slo = (float)(factor / H->cmax), shi = (float)(factor / H->cmin);
        auto kof = [&](float sv) { return clampi((int)std::min(sv, (float)K), 0, K - 1); };
        ka = kof(slo);
        kz = kof(shi);
        ca = clampi((int)slo, 0, K);
        cz = clampi((int)shi, 0, K);
    } else {
        auto kof = [&](double c) {
            double eta = (H->omega * g.ell * (1.0 / c)) * 0.15915494309189533577;
            eta = eta < 0.4 ? eta : 0.4;
            return clampi((int)(eta * (K / 0.4)), 0, K - 1);
        };
        ka = kof(H->cmax);
        kz = kof(H->cmin);
    }
    L.kb = clampi(ka - 1, 0, K - 1);
    L.nk = clampi(kz + 1, 0, K - 1) - L.kb + 1;
    L.cb = clampi(ca - 1, 0, K);
    L.nck = clampi(cz + 1, 0, K) - L.cb + 1;
}

// ---------------------------------------------------------------------------
// Precision-specific drivers
// ---------------------------------------------------------------------------
template <typename T>
struct Eng {
    using R = decltype(T{}.re);
    helm_hierarchy *H;
    Lane *Ln;
    hipStream_t s;

    bool transposed = false;   // outer solve with A_h^T (adjoint); r64: its FP64 residual buffer;
    c64 *r64 = nullptr;        // xin, u: PML node factors and a vector for the preconditioner Xi M(Xi^-1 .)
    const c64 *xin = nullptr;   // 1/xi_j then xi_j per axis (launch_xi_scale)
    T *u_t = nullptr;

    explicit Eng(helm_hierarchy *h, int lane = 0) : H(h), Ln(&h->lane[lane]), s(h->lane[lane].s) {}

    const LevelArgs<R> &L(int l) const;
    long long nn(int l) const { return H->geom[l].nn; }
    T *v(void *p) const { return static_cast<T *>(p); }

    hipError_t stencil(int l, int mode, bool shifted, double wJ, const void *x, const void *g, const void *base,
                       void *y, bool norm = false, KState *st = nullptr) {
        StencilCall c{mode, shifted ? 1 : 0, wJ, x, g, base, y, norm, EPI_NORM_INIT, st, 0};
        return launch_stencil<R, T, T, T>(L(l), c, Ln->rb, s);
    }

    // coarse = R (g - op x) from level l to l+1 (eq. full-weighting fused with the residual)
    hipError_t resid_restrict(int l, bool shifted, const T *x, const T *g, T *coarse) {
        HIP_CHK(stencil(l, M_RESID_R, shifted, 0.0, x, g, nullptr, Ln->wrest[l]));
        return launch_restrict_y<T>(H->geom[l], H->geom[l + 1], static_cast<const T *>(Ln->wrest[l]), coarse, s);
    }

    // y = J_nJ(op, g; w) from zero; tmp is a scratch vector of the level
    hipError_t jacobi(int l, bool shifted, int nJ, double w, const T *g, T *y) {
        if (nJ == 1) return launch_jac1<R, T>(L(l), shifted, w, g, y, s);
        HIP_CHK(stencil(l, M_JAC2, shifted, w, nullptr, g, nullptr, y));
        T *a = y, *b = v(Ln->tmp[l]);
        for (int it = 2; it < nJ; ++it) {
            HIP_CHK(stencil(l, M_JSWEEP, shifted, w, a, g, nullptr, b));
            std::swap(a, b);
        }
        if (a != y) HIP_CHK((launch_convert<T, T>(a, y, nn(l), s)));
        return hipSuccess;
    }

    // Arnoldi step: V[k+1] <- A Z[k] orthonormalised against V[0..k] (CGS2), Givens update of column k
    // Classical Gram-Schmidt with a second pass only where the first one left
    // less than kReorthEta of ||w||^2 (decided on the device: the second-pass
    // kernel returns at once otherwise).  The last step of a cycle (last = true) stops
    // after the Hessenberg column: the next basis vector is never used, so it is
    // neither written nor normalised.
    hipError_t arnoldi(int l, T **V, int k, KState *st, bool last) {
        HIP_CHK(launch_dots<T>((const T *const *)V, k + 1, V[k + 1], true, nn(l), EPI_ARNOLDI_SEL, st, k, nullptr,
                               Ln->rb, s));
        HIP_CHK(launch_axpy_dots<T>((const T *const *)V, k + 1, V[k + 1], nn(l), st, Ln->rb, s, !last));
        if (!last) HIP_CHK(launch_axpy_scale<T>((const T *const *)V, k + 1, V[k + 1], nn(l), st, s));
        return hipSuccess;
    }

    // `cycles` restarted right-preconditioned (F)GMRES(m) cycles for op x = g on level l
    template <typename Prec>
    hipError_t gmres(int l, bool shifted, Prec prec, const T *g, T *x, bool x0_zero, int m, int cycles, KState *st,
                     void **Vv, void **Zv) {
        T *V[kMMax + 1], *Zp[kMMax];
        for (int j = 0; j <= m; ++j) V[j] = v(Vv[j]);
        for (int j = 0; j < m; ++j) Zp[j] = v(Zv[j]);
        for (int cyc = 0; cyc < cycles; ++cyc) {
            // The first basis vector is the residual itself, unnormalised (the
            // state keeps its 1/beta for the projections): g from zero, else
            // g - op x.  Its preconditioned image is then beta times larger, so
            // Hessenberg column 0 and y_0 carry the factor and x = Z y is unchanged.
            const bool from_zero = (cyc == 0 && x0_zero);
            if (from_zero) {
                V[0] = const_cast<T *>(g);   // read only
                HIP_CHK(launch_dots<T>(nullptr, 0, g, true, nn(l), EPI_NORM_INIT, st, 0, nullptr, Ln->rb, s));
            } else {
                V[0] = v(Vv[0]);
                HIP_CHK(stencil(l, M_RESID, shifted, 0.0, x, g, nullptr, V[0], true, st));
            }
            for (int k = 0; k < m; ++k) {
                HIP_CHK(prec(V[k], Zp[k]));
                HIP_CHK(stencil(l, M_APPLY, shifted, 0.0, Zp[k], nullptr, nullptr, V[k + 1]));
                HIP_CHK(arnoldi(l, V, k, st, k == m - 1));
            }
            HIP_CHK((launch_combine<T, T>(x, (const T *const *)Zp, m, nn(l), st, true, from_zero, s)));
        }
        return hipSuccess;
    }

    // C_4h: m_4h s-step (CA-GMRES) steps on B_4h from zero, right preconditioned by
    // J_nJ4h(B_4h; omega_4h).  Basis P_0 = q, P_{j+1} = B_4h J(P_j); the iterate
    // sum_j y_j J(P_j) minimises ||q - sum_j y_j P_{j+1}|| (normal equations of the
    // FP64 Gram matrix, Cholesky).
    hipError_t bottom(const T *q, T *e) {
        const int m = H->opt.m_4h;
        T *P[kM4Max + 1], *Zb[kM4Max];
        P[0] = const_cast<T *>(q);
        for (int j = 1; j <= m; ++j) P[j] = v(Ln->P4[j]);
        for (int j = 0; j < m; ++j) Zb[j] = v(Ln->Z4[j]);
        for (int j = 0; j < m; ++j) {
            HIP_CHK(jacobi(2, true, H->opt.nJ_4h, H->opt.omega_4h, P[j], Zb[j]));
            HIP_CHK(stencil(2, M_APPLY, true, 0.0, Zb[j], nullptr, nullptr, P[j + 1]));
        }
        HIP_CHK(launch_gram<T>((const T *const *)P, m + 1, nn(2), Ln->st_bottom, Ln->rb, s));
        HIP_CHK((launch_combine<T, T>(e, (const T *const *)Zb, m, nn(2), Ln->st_bottom, false, true, s)));
        return hipSuccess;
    }

    // V^sigma_2h(q), eq. shifted-auxiliary-cycle
    hipError_t vcycle(const T *q, T *out) {
        const helm_options &o = H->opt;
        T *y = v(Ln->vy), *r = v(Ln->vr), *q4 = v(Ln->P4[0]), *e4 = v(Ln->e4);
        HIP_CHK(jacobi(1, true, o.nJ_2h, o.omega_2h, q, y));                 // y = J(B_2h, q)
        HIP_CHK(resid_restrict(1, true, y, q, q4));                          // q_4h = R(q - B y)
        HIP_CHK(bottom(q4, e4));                                             // e_4h = C_4h(q_4h)
        HIP_CHK(launch_prolong_add<T>(H->geom[2], H->geom[1], e4, y, s));   // y~ = y + P e_4h
        HIP_CHK(stencil(1, M_RESID, true, 0.0, y, q, nullptr, r));           // q - B y~
        if (o.nJ_2h == 2) {
            HIP_CHK(stencil(1, M_JAC2_ADD, true, o.omega_2h, nullptr, r, y, out));   // y~ + J(B, q - B y~)
        } else {
            HIP_CHK(jacobi(1, true, o.nJ_2h, o.omega_2h, r, out));
            HIP_CHK(launch_add<T>(y, out, nn(1), s));
        }
        return hipSuccess;
    }

    // K_2h(r), eq. unshifted-middle-solve
    hipError_t k2h(const T *r, T *e) {
        if constexpr (std::is_same<T, c32>::value)
            if (H->prec == HELM_MIXED) return k2h_mixed(r, e);
        auto prec = [this](const T *in, T *out) { return vcycle(in, out); };
        return gmres(1, false, prec, r, e, true, H->opt.m_2h, H->opt.c_2h, Ln->st_k2h, Ln->V2, Ln->Z2);
    }

    // ---- HELM_MIXED (FP32 arithmetic, FP16-stored inner vectors; Sec. 5 "Arithmetic Precision") ----
    // The V-cycle's iterates y and r, the 4h basis P, Z and correction e, and K_2h's
    // preconditioned vectors Z are stored as c16 with the scales of helm_hierarchy::fres /
    // fsol times qs, the inverse norm of the cycle's input (the K_2h state's vs0 for its
    // unnormalised first basis vector, 1 for the others).  Every V-cycle map is homogeneous
    // of degree one in its input, so these units keep the stored values near unit size.
    // qs is a Krylov state's vs0 (one per batched slot) or the shared constant 1
    int qstride(const double *qs) const { return qs == H->d_one ? 0 : kKStateDoubles; }
    Scale sres(int l, const double *qs) const { return {H->fres[l], qs, qstride(qs)}; }
    Scale ssol(int l, const double *qs) const { return {H->fsol[l], qs, qstride(qs)}; }
    static c16 *h16(void *p) { return static_cast<c16 *>(p); }

    template <typename TX, typename TG, typename TY>
    hipError_t st16(int l, int mode, bool shifted, double wJ, const void *x, const void *g, const void *base, void *y,
                    Scale sx, Scale sg, Scale sb, Scale sy) {
        StencilCall c{mode, shifted ? 1 : 0, wJ, x, g, base, y, false, EPI_NORM_INIT, nullptr, 0};
        c.sx = sx;
        c.sg = sg;
        c.sb = sb;
        c.sy = sy;
        return launch_stencil<R, TX, TG, TY>(L(l), c, Ln->rb, s);
    }

    // C_4h on FP16-stored vectors: basis P (residual units), Z = J(P) and e (correction units);
    // the Gram solve and the combination are invariant to the common scales
    hipError_t bottom_mixed(const c16 *q, const double *qs, c16 *e) {
        const int m = H->opt.m_4h;
        c16 *P[kM4Max + 1], *Zb[kM4Max];
        P[0] = const_cast<c16 *>(q);
        for (int j = 1; j <= m; ++j) P[j] = h16(Ln->P4[j]);
        for (int j = 0; j < m; ++j) Zb[j] = h16(Ln->Z4[j]);
        const Scale sr = sres(2, qs), ss = ssol(2, qs);
        for (int j = 0; j < m; ++j) {
            HIP_CHK((st16<c16, c16, c16>(2, M_JAC2, true, H->opt.omega_4h, nullptr, P[j], nullptr, Zb[j], sr, sr, ss,
                                         ss)));
            HIP_CHK((st16<c16, c16, c16>(2, M_APPLY, true, 0.0, Zb[j], nullptr, nullptr, P[j + 1], ss, sr, ss, sr)));
        }
        HIP_CHK(launch_gram<c16>((const c16 *const *)P, m + 1, nn(2), Ln->st_bottom, Ln->rb, s));
        return launch_combine<c16, c16>(e, (const c16 *const *)Zb, m, nn(2), Ln->st_bottom, false, true, s);
    }

    // V^sigma_2h(q) with FP16-stored iterates; q in FP32 (true values), out = Z in correction units
    hipError_t vcycle_mixed(const T *q, const double *qs, c16 *out) {
        const helm_options &o = H->opt;
        c16 *y = h16(Ln->vy), *r = h16(Ln->vr), *q4 = h16(Ln->P4[0]), *e4 = h16(Ln->e4);
        const Scale one = {1.0f, nullptr}, s1 = ssol(1, qs), r1 = sres(1, qs), r2 = sres(2, qs), s2 = ssol(2, qs);
        HIP_CHK((st16<c32, c32, c16>(1, M_JAC2, true, o.omega_2h, nullptr, q, nullptr, y, one, one, one, s1)));   // y = J(B, q)
        HIP_CHK((st16<c16, c32, c32>(1, M_RESID_R, true, 0.0, y, q, nullptr, Ln->wrest[1], s1, one, one, one)));
        HIP_CHK((launch_restrict_y<c32, c16>(H->geom[1], H->geom[2], static_cast<const c32 *>(Ln->wrest[1]), q4, s,
                                             r2)));                                                   // q4 = R(q - B y)
        HIP_CHK(bottom_mixed(q4, qs, e4));                                                             // e4 = C_4h(q4)
        HIP_CHK((launch_prolong_add<c16, c16>(H->geom[2], H->geom[1], e4, y, s, s2, s1)));            // y~ = y + P e4
        HIP_CHK((st16<c16, c32, c16>(1, M_RESID, true, 0.0, y, q, nullptr, r, s1, one, one, r1)));    // r = q - B y~
        return st16<c16, c16, c16>(1, M_JAC2_ADD, true, o.omega_2h, nullptr, r, y, out, r1, r1, s1, s1);   // y~ + J(B, r)
    }

    // helm_vcycle / helm_bottom on caller vectors: in HELM_MIXED the input's own inverse
    // norm gives the FP16 units, and the result is returned in FP32
    hipError_t vcycle_hook(const T *q, T *y) {
        if constexpr (std::is_same<T, c32>::value)
            if (H->prec == HELM_MIXED) {
                KState *st = Ln->st_hook;
                c16 *z = h16(Ln->Z2[0]);
                HIP_CHK(launch_dots<T>(nullptr, 0, q, true, nn(1), EPI_NORM_INIT, st, 0, nullptr, Ln->rb, s));
                HIP_CHK(vcycle_mixed(q, &st->vs0, z));
                return launch_convert_scaled<c16, c32>(z, y, nn(1), ssol(1, &st->vs0), Scale{1.0f, nullptr}, s);
            }
        return vcycle(q, y);
    }
    hipError_t bottom_hook(const T *q, T *e) {
        if constexpr (std::is_same<T, c32>::value)
            if (H->prec == HELM_MIXED) {
                KState *st = Ln->st_hook;
                c16 *q4 = h16(Ln->P4[0]), *e4 = h16(Ln->e4);
                const Scale one = {1.0f, nullptr};
                HIP_CHK(launch_dots<T>(nullptr, 0, q, true, nn(2), EPI_NORM_INIT, st, 0, nullptr, Ln->rb, s));
                HIP_CHK((launch_convert_scaled<c32, c16>(q, q4, nn(2), one, sres(2, &st->vs0), s)));
                HIP_CHK(bottom_mixed(q4, &st->vs0, e4));
                return launch_convert_scaled<c16, c32>(e4, e, nn(2), ssol(2, &st->vs0), one, s);
            }
        return bottom(q, e);
    }

    // K_2h with FP16-stored Z: FGMRES on A_2h (FP32 basis, FP64 sums), V-cycle on each basis vector
    hipError_t k2h_mixed(const T *r, T *e) {
        const int m = H->opt.m_2h;
        KState *st = Ln->st_k2h;
        T *V[kMMax + 1];
        c16 *Zp[kMMax];
        for (int j = 0; j <= m; ++j) V[j] = v(Ln->V2[j]);
        for (int j = 0; j < m; ++j) Zp[j] = h16(Ln->Z2[j]);
        const Scale one = {1.0f, nullptr};
        for (int cyc = 0; cyc < H->opt.c_2h; ++cyc) {
            const bool from_zero = (cyc == 0);
            if (from_zero) {
                V[0] = const_cast<T *>(r);   // read only
                HIP_CHK(launch_dots<T>(nullptr, 0, r, true, nn(1), EPI_NORM_INIT, st, 0, nullptr, Ln->rb, s));
            } else {
                V[0] = v(Ln->V2[0]);
                HIP_CHK(stencil(1, M_RESID, false, 0.0, e, r, nullptr, V[0], true, st));
            }
            for (int k = 0; k < m; ++k) {
                const double *qs = (k == 0) ? &st->vs0 : H->d_one;   // V_0 is kept unnormalised
                HIP_CHK(vcycle_mixed(V[k], qs, Zp[k]));
                HIP_CHK((st16<c16, c16, c32>(1, M_APPLY, false, 0.0, Zp[k], nullptr, nullptr, V[k + 1], ssol(1, qs), one,
                                             one, one)));
                HIP_CHK(arnoldi(1, V, k, st, k == m - 1));
            }
            HIP_CHK((launch_combine<c32, c16>(e, (const c16 *const *)Zp, m, nn(1), st, true, from_zero, s,
                                             H->fsol[1])));
        }
        return hipSuccess;
    }

    // S_h(g; x0) -> x (in place when x0 == x): one GMRES(m_h) cycle right-preconditioned by J_nJh(A_h).
    // For m_h <= kSstepMax the minimal-residual iterate over the same Krylov space is
    // computed from the s-step basis P_0 = r_0, P_{j+1} = A_h J(P_j) and the FP64 Gram
    // matrix (as in the bottom solver): two vector passes per step fewer than Arnoldi's
    // projections, with a basis of at most three vectors, well conditioned in FP64 even
    // where A_h J is close to the identity.  Longer cycles use Arnoldi.
    hipError_t smooth(const T *g, T *x, bool x0_zero) {
        const int m = H->opt.m_h;
        if (m > kSstepMax) {
            auto prec = [this](const T *in, T *out) {
                return jacobi(0, false, H->opt.nJ_h, H->opt.omega_h, in, out);
            };
            return gmres(0, false, prec, g, x, x0_zero, m, 1, Ln->st_smooth, Ln->Vs, Ln->Zs);
        }
        T *P[kSstepMax + 1], *Zp[kSstepMax];
        for (int j = 1; j <= m; ++j) P[j] = v(Ln->Vs[j]);
        for (int j = 0; j < m; ++j) Zp[j] = v(Ln->Zs[j]);
        if (x0_zero) {
            P[0] = const_cast<T *>(g);   // read only
        } else {
            P[0] = v(Ln->Vs[0]);
            HIP_CHK(stencil(0, M_RESID, false, 0.0, x, g, nullptr, P[0]));   // r_0 = g - A_h x_0
        }
        for (int j = 0; j < m; ++j) {
            HIP_CHK(jacobi(0, false, H->opt.nJ_h, H->opt.omega_h, P[j], Zp[j]));
            HIP_CHK(stencil(0, M_APPLY, false, 0.0, Zp[j], nullptr, nullptr, P[j + 1]));
        }
        HIP_CHK(launch_gram<T>((const T *const *)P, m + 1, nn(0), Ln->st_smooth, Ln->rb, s));
        return launch_combine<T, T>(x, (const T *const *)Zp, m, nn(0), Ln->st_smooth, false, x0_zero, s);
    }

    // Algorithm 1: z = M_h^{-1} r
    hipError_t precond(const T *r, T *z) {
        T *r2 = v(Ln->r2), *e2 = v(Ln->e2);
        HIP_CHK(smooth(r, z, true));                                          // 1: z_pre = S_h(r; 0)
        HIP_CHK(resid_restrict(0, false, z, r, r2));                         // 2: r_2h = R(r - A z_pre)
        HIP_CHK(k2h(r2, e2));                                                 // 3: e_2h = K_2h(r_2h)
        HIP_CHK(launch_prolong_add<T>(H->geom[1], H->geom[0], e2, z, s));    // 4: z~ = z_pre + P e_2h
        HIP_CHK(smooth(r, z, false));                                         // 5: z = S_h(r; z~)
        return hipSuccess;
    }

    hipError_t read_state(const KState *st) {
        HIP_CHK(hipMemcpyAsync(Ln->host_state, st, sizeof(KState), hipMemcpyDeviceToHost, s));
        return hipStreamSynchronize(s);
    }

    // Outer FGMRES(m_out) for one right-hand side (Sec. 3.3); x and b in FP64:
    // b = Q_h f, solve A_h v = b, u = Q_h v (u may be null: v stays in x64);
    // v_out (optional) receives a copy of v.
    helm_status solve_one(const T *f, T *u, double tol, int *iters, double *relres, c64 *v_out = nullptr) {
        HIP_TRY((launch_qapply<double, T, c64>(H->Ld[0], f, Ln->b64, s)));   // b = Q_h f
        const helm_status status = solve_b64(tol, iters, relres);
        if (status < 0) return status;
        if (u) HIP_TRY((launch_qapply<double, c64, T>(H->Ld[0], Ln->x64, u, s)));   // u = Q_h v
        if (v_out) HIP_TRY((launch_convert<c64, c64>(Ln->x64, v_out, nn(0), s)));
        HIP_TRY(hipStreamSynchronize(s));
        return status;
    }

    // Several right-hand sides (nb <= the lane's slots) in one set of launches: slot s solves
    // f_s in its own copy of every vector and state.  The slots advance in lockstep through the
    // outer FGMRES steps; a slot whose residual estimate reaches tol (or that breaks down or
    // reaches max_outer) leaves the launch mask for the rest of the cycle, and a converged slot
    // leaves it for good, so each slot performs exactly the arithmetic of a solve on its own.
    helm_status solve_batch(const T *f, T *u, int nb, double tol, int *iters, double *relres, c64 *v_out) {
        if (nb == 1) return solve_one(f, u, tol, iters, relres, v_out);
        if (nb < 1 || nb > Ln->nslot || transposed) return fail(H, HELM_EINVAL, "invalid batch");
        Batch bt;
        bt.n = nb;
        bt.mask = (1u << nb) - 1u;
        bt.pstride = Ln->pstride;
        BatchScope scope(bt);
        HIP_TRY((launch_qapply<double, T, c64>(H->Ld[0], f, Ln->b64, s)));   // b = Q_h f
        const helm_status status = solve_b64_batch(nb, tol, iters, relres);
        cur_batch().mask = bt.mask;
        if (status < 0) return status;
        if (u) HIP_TRY((launch_qapply<double, c64, T>(H->Ld[0], Ln->x64, u, s)));   // u = Q_h v
        if (v_out) HIP_TRY((launch_convert<c64, c64>(Ln->x64, v_out, nn(0), s)));
        HIP_TRY(hipStreamSynchronize(s));
        return status;
    }

    hipError_t read_states(const KState *st, int nb) {
        HIP_CHK(hipMemcpyAsync(Ln->host_state, st, nb * sizeof(KState), hipMemcpyDeviceToHost, s));
        return hipStreamSynchronize(s);
    }

    helm_status solve_b64_batch(int nb, double tol, int *iters, double *relres) {
        const helm_options &o = H->opt;
        const long long n = nn(0);
        T *V[kMMax + 1], *Zp[kMMax];
        for (int j = 0; j <= o.m_out; ++j) V[j] = v(Ln->Vout[j]);
        for (int j = 0; j < o.m_out; ++j) Zp[j] = v(Ln->Zout[j]);
        KState *st = Ln->st_outer;
        const int max_outer = o.max_outer > 0 ? o.max_outer : 1000;
        const unsigned all = cur_batch().mask;
        auto use = [](unsigned m) { cur_batch().mask = m; };
        // ||b|| of every slot (EPI_STORE: 2 kRedSlots doubles per slot)
        HIP_TRY(launch_dots<c64>(nullptr, 0, Ln->b64, true, n, EPI_STORE, nullptr, 0, Ln->dscratch, Ln->rb, s));
        HIP_TRY(hipMemcpyAsync(Ln->host_scratch, Ln->dscratch, nb * 2 * kRedSlots * sizeof(double),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        double bn[kMaxBatch];
        int its[kMaxBatch], kk[kMaxBatch];
        helm_status stat[kMaxBatch];
        unsigned active = 0;
        for (int q = 0; q < nb; ++q) {
            bn[q] = std::sqrt(Ln->host_scratch[q * 2 * kRedSlots]);
            its[q] = 0;
            stat[q] = HELM_OK;
            iters[q] = 0;
            relres[q] = 0.0;
            if (!(bn[q] == bn[q]) || bn[q] > 1e300) return fail(H, HELM_BREAKDOWN, "non-finite right-hand side");
            if (bn[q] > 0.0) active |= 1u << q;
        }
        HIP_TRY(launch_fill_zero<c64>(Ln->x64, n, s));
        while (active) {
            // true residuals in FP64 arithmetic: r = b - A x
            use(active);
            HIP_TRY(outer_residual(V[0], st));
            HIP_TRY(read_states(st, nb));
            unsigned cyc = 0;
            for (int q = 0; q < nb; ++q) {
                if (!(active >> q & 1u)) continue;
                const KState &hs = Ln->host_state[q];
                if (hs.nonfinite) return fail(H, HELM_BREAKDOWN, "non-finite residual");
                relres[q] = hs.beta / bn[q];
                iters[q] = its[q];
                if (relres[q] <= tol) continue;
                if (its[q] >= max_outer) {
                    stat[q] = HELM_NOT_CONVERGED;
                    continue;
                }
                cyc |= 1u << q;
            }
            active = cyc;
            if (!cyc) break;
            unsigned inc = cyc;   // slots still stepping in this cycle
            for (int q = 0; q < nb; ++q) kk[q] = 0;
            for (int k = 0; k < o.m_out && inc; ++k) {
                use(inc);
                HIP_TRY(precond(V[k], Zp[k]));
                HIP_TRY(stencil(0, M_APPLY, false, 0.0, Zp[k], nullptr, nullptr, V[k + 1]));
                HIP_TRY(arnoldi(0, V, k, st, k == o.m_out - 1));
                HIP_TRY(read_states(st, nb));
                for (int q = 0; q < nb; ++q) {
                    if (!(inc >> q & 1u)) continue;
                    ++its[q];
                    kk[q] = k + 1;
                    const KState &hs = Ln->host_state[q];
                    if (hs.nonfinite) return fail(H, HELM_BREAKDOWN, "non-finite Krylov quantity");
                    const double est = std::hypot(hs.g[k + 1][0], hs.g[k + 1][1]) / bn[q];
                    if (est <= tol || hs.breakdown || its[q] >= max_outer) inc &= ~(1u << q);
                }
            }
            // x += Z y per slot (each with its own number of columns)
            for (int q = 0; q < nb; ++q) {
                if (!(cyc >> q & 1u)) continue;
                use(1u << q);
                HIP_TRY((launch_combine<c64, T>(Ln->x64, (const T *const *)Zp, kk[q], n, st, true, false, s)));
            }
        }
        use(all);
        helm_status worst = HELM_OK;
        for (int q = 0; q < nb; ++q)
            if (stat[q] == HELM_NOT_CONVERGED) worst = HELM_NOT_CONVERGED;
        return worst;
    }

    // FP64 true residual r = b - op x64 into V0 (working precision), its norm into the state
    hipError_t outer_residual(T *V0, KState *st) {
        if (!transposed) {
            StencilCall c{M_RESID, 0, 0.0, Ln->x64, Ln->b64, nullptr, V0, true, EPI_NORM_INIT, st, 0};
            return launch_stencil<double, c64, c64, T>(H->Ld[0], c, Ln->rb, s);
        }
        HIP_CHK((launch_apply_t<double, c64, c64, c64>(H->Ld[0], 0, Ln->x64, Ln->b64, r64, s)));
        HIP_CHK(launch_dots<c64>(nullptr, 0, r64, true, nn(0), EPI_NORM_INIT, st, 0, nullptr, Ln->rb, s));
        return launch_convert<c64, T>(r64, V0, nn(0), s);
    }

    // Outer FGMRES(m_out) for op x64 = b64 from x64 = 0 (op = A_h, or A_h^T when transposed),
    // right preconditioned by Algorithm 1, until the FP64 true relative residual <= tol.
    helm_status solve_b64(double tol, int *iters, double *relres) {
        const helm_options &o = H->opt;
        const long long n = nn(0);
        T *V[kMMax + 1], *Zp[kMMax];
        for (int j = 0; j <= o.m_out; ++j) V[j] = v(Ln->Vout[j]);
        for (int j = 0; j < o.m_out; ++j) Zp[j] = v(Ln->Zout[j]);
        KState *st = Ln->st_outer;
        const int max_outer = o.max_outer > 0 ? o.max_outer : 1000;
        HIP_TRY(launch_dots<c64>(nullptr, 0, Ln->b64, true, n, EPI_STORE, nullptr, 0, Ln->dscratch, Ln->rb, s));
        HIP_TRY(hipMemcpyAsync(Ln->host_scratch, Ln->dscratch, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const double bn = std::sqrt(Ln->host_scratch[0]);
        HIP_TRY(launch_fill_zero<c64>(Ln->x64, n, s));
        int its = 0;
        double rel = 0.0;
        helm_status status = HELM_OK;
        if (!(bn == bn) || bn > 1e300) return fail(H, HELM_BREAKDOWN, "non-finite right-hand side");
        if (bn == 0.0) {
            *iters = 0;
            *relres = 0.0;
            return HELM_OK;
        }
        for (;;) {
            // true residual in FP64 arithmetic: r = b - op x
            HIP_TRY(outer_residual(V[0], st));
            HIP_TRY(read_state(st));
            if (Ln->host_state->nonfinite) return fail(H, HELM_BREAKDOWN, "non-finite residual");
            rel = Ln->host_state->beta / bn;
            if (rel <= tol) break;
            if (its >= max_outer) {
                status = HELM_NOT_CONVERGED;
                break;
            }
            int kk = 0;   // V[0] = r stays unnormalised (the state holds 1/beta)
            for (int k = 0; k < o.m_out; ++k) {
                if (transposed && xin) {
                    // A_h^T is close to Xi A_h Xi^-1 (the PML row factors move to the columns), so
                    // Xi M_h^-1 Xi^-1 approximates its inverse
                    HIP_TRY(launch_xi_scale<T>(H->geom[0], xin, V[k], u_t, false, s));
                    HIP_TRY(precond(u_t, Zp[k]));
                    HIP_TRY(launch_xi_scale<T>(H->geom[0], xin, Zp[k], Zp[k], true, s));
                } else {
                    HIP_TRY(precond(V[k], Zp[k]));
                }
                ++its;
                if (transposed)
                    HIP_TRY((launch_apply_t<R, T, T, T>(L(0), 0, Zp[k], (const T *)nullptr, V[k + 1], s)));
                else
                    HIP_TRY(stencil(0, M_APPLY, false, 0.0, Zp[k], nullptr, nullptr, V[k + 1]));
                HIP_TRY(arnoldi(0, V, k, st, k == o.m_out - 1));
                HIP_TRY(read_state(st));
                kk = k + 1;
                const KState &hs = *Ln->host_state;
                if (hs.nonfinite) return fail(H, HELM_BREAKDOWN, "non-finite Krylov quantity");
                const double est = std::hypot(hs.g[k + 1][0], hs.g[k + 1][1]) / bn;
                if (est <= tol || hs.breakdown || its >= max_outer) break;
            }
            HIP_TRY((launch_combine<c64, T>(Ln->x64, (const T *const *)Zp, kk, n, st, true, false, s)));
        }
        *iters = its;
        *relres = rel;
        return status;
    }
};

template <>
const LevelArgs<float> &Eng<c32>::L(int l) const { return H->Lf[l]; }
template <>
const LevelArgs<double> &Eng<c64>::L(int l) const { return H->Ld[l]; }

// pinned host buffers and the streams helm_setup created for lanes 1..
void release_lanes(helm_hierarchy *H) {
    for (int li = 0; li < kMaxLanes; ++li) {
        Lane &Ln = H->lane[li];
        if (Ln.host_state) (void)hipHostFree(Ln.host_state);
        if (Ln.host_scratch) (void)hipHostFree(Ln.host_scratch);
        if (Ln.own_stream) {
            (void)hipStreamSynchronize(Ln.s);
            (void)hipStreamDestroy(Ln.s);
        }
        Ln.host_state = nullptr;
        Ln.host_scratch = nullptr;
        Ln.own_stream = false;
    }
}

helm_status check_options(const helm_options *o, std::string &msg) {
    if (!o) { msg = "options pointer is NULL"; return HELM_EINVAL; }
    if (o->struct_size != (int)sizeof(helm_options)) { msg = "options.struct_size mismatch"; return HELM_EINVAL; }
    if (o->precision != HELM_FP64 && o->precision != HELM_FP32 && o->precision != HELM_MIXED) {
        msg = "unknown precision";
        return HELM_EINVAL;
    }
    if (o->precision == HELM_MIXED && (o->nJ_2h != 2 || o->nJ_4h != 2)) {
        msg = "HELM_MIXED runs the fused two-sweep Jacobi on the 2h and 4h levels: nJ_2h and nJ_4h must be 2";
        return HELM_EINVAL;
    }
    if (!(o->sigma >= 0) || !(o->omega_h > 0) || !(o->omega_2h > 0) || !(o->omega_4h > 0) || !(o->gamma_max >= 0) ||
        !std::isfinite(o->sigma) || !std::isfinite(o->gamma_max)) {
        msg = "sigma, Jacobi weights and gamma_max must be finite (weights > 0)";
        return HELM_EINVAL;
    }
    auto in = [](int v, int lo, int hi) { return v >= lo && v <= hi; };
    if (!in(o->nJ_h, 1, 8) || !in(o->nJ_2h, 1, 8) || !in(o->nJ_4h, 1, 8)) { msg = "nJ must be in 1..8"; return HELM_EINVAL; }
    if (!in(o->m_h, 1, kMMax) || !in(o->m_2h, 1, kMMax) || !in(o->m_out, 1, kMMax)) {
        msg = "m_h, m_2h and m_out must be in 1..12";
        return HELM_EINVAL;
    }
    if (!in(o->m_4h, 1, kM4Max) || !in(o->c_2h, 1, 8)) { msg = "m_4h must be in 1..8 and c_2h in 1..8"; return HELM_EINVAL; }
    if (!in(o->iofd_K, 1, kKMax)) { msg = "iofd_K must be in 1..128"; return HELM_EINVAL; }
    if (o->tile_tz != 0 && !in(o->tile_tz, kTzMin, kTzMax)) { msg = "tile_tz must be 0 or in 2..64"; return HELM_EINVAL; }
    if (!in(o->tile_split, -1, 1)) { msg = "tile_split must be -1, 0 or 1"; return HELM_EINVAL; }
    if (!in(o->lanes, 0, kMaxLanes)) { msg = "lanes must be in 0..8"; return HELM_EINVAL; }
    if (!in(o->pml_variant, 0, 2)) { msg = "pml_variant must be 0, 1 or 2"; return HELM_EINVAL; }
    if (!in(o->batch, 0, kMaxBatch)) { msg = "batch must be in 0..8"; return HELM_EINVAL; }
    return HELM_OK;
}

helm_status check_dims(int nx, int ny, int nz, int n_pml, int N[3], std::string &msg) {
    if (nx < 1 || ny < 1 || nz < 1 || n_pml < 0) { msg = "grid sizes must be positive and n_pml >= 0"; return HELM_EINVAL; }
    const int n[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        const long long t = (long long)n[a] + 2LL * n_pml;
        if (t % 4 != 0 || t < 8 || t > 4096) {
            msg = "total intervals per axis (n + 2 n_pml) must be a multiple of 4 in [8, 4096]";
            return HELM_EINVAL;
        }
        N[a] = (int)t;
    }
    return HELM_OK;
}

template <typename F>
helm_status dispatch(helm_hierarchy *H, F &&f) {
    hipError_t e = (H->prec == HELM_FP64) ? f(Eng<c64>(H)) : f(Eng<c32>(H));
    if (e != hipSuccess) return fail(H, HELM_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return HELM_OK;
}

bool level_ok(int l) { return l >= 0 && l <= 2; }

// Pick, per level and kernel family, the number of z planes each stencil
// wavefront marches through and whether the stencils run as one launch or as
// interior + border launches: time the family's kernel (an operator apply, or a
// fused two-sweep Jacobi; six launches) with HIP events on the caller's stream
// and keep the fastest.  Long marches amortise the plane pipeline; short ones
// give small grids enough workgroups, and depths between the powers of two
// let the last round of workgroups fill the chip.  Every candidate depth is
// timed as one launch, then the interior + border split (a second launch, but
// interior tiles at higher occupancy) at the two fastest depths.
template <typename T>
hipError_t tune_level_tiles(helm_hierarchy *H, int l, int fam) {
    Eng<T> E(H);
    // working-precision vectors large enough for the level (the V-cycle ones are FP16 in HELM_MIXED)
    T *x = static_cast<T *>(H->lane[0].tmp[l]);
    T *y = static_cast<T *>(l == 0 ? H->lane[0].Vs[0] : (l == 1 ? H->lane[0].V2[1] : H->lane[0].Vs[1]));
    HIP_CHK(launch_fill_zero<T>(x, E.nn(l), H->s));
    hipEvent_t a, b;
    HIP_CHK(hipEventCreate(&a));
    HIP_CHK(hipEventCreate(&b));
    // every slot of the lane runs, as in a batched solve (more workgroups per launch favour
    // longer marches)
    Batch tb;
    tb.n = H->lane[0].nslot;
    tb.mask = (1u << tb.n) - 1u;
    tb.pstride = H->lane[0].pstride;
    BatchScope tscope(tb);
    auto run = [&]() -> hipError_t {
        return fam == 0 ? E.stencil(l, M_APPLY, l > 0, 0.0, x, nullptr, nullptr, y)
                        : E.stencil(l, M_JAC2, l > 0, H->opt.omega_h, nullptr, x, nullptr, y);
    };
    auto time_one = [&](int tz, int split, float &ms) -> hipError_t {
        H->Lf[l].tz[fam] = H->Ld[l].tz[fam] = tz;
        H->Lf[l].split[fam] = H->Ld[l].split[fam] = split;
        HIP_CHK(run());
        ms = 1e30f;
        if (l > 0) {
            // Coarse levels fit the last-level cache when timed back to back, but inside a
            // solve the Krylov bases stream through it in between: time each launch after
            // writing a full fine-level vector (lane 0's outer basis, free during setup).
            float tot = 0.f;
            for (int r = 0; r < 6; ++r) {
                {
                    BatchScope one{Batch{}};   // one fine vector is enough to evict the coarse level
                    HIP_CHK(launch_fill_zero<T>(static_cast<T *>(H->lane[0].Vout[1]), E.nn(0), H->s));
                }
                HIP_CHK(hipEventRecord(a, H->s));
                HIP_CHK(run());
                HIP_CHK(hipEventRecord(b, H->s));
                HIP_CHK(hipEventSynchronize(b));
                float t = 0.f;
                HIP_CHK(hipEventElapsedTime(&t, a, b));
                tot += t;
            }
            ms = tot;
        } else {
            for (int trial = 0; trial < 2; ++trial) {
                HIP_CHK(hipEventRecord(a, H->s));
                for (int r = 0; r < 6; ++r) HIP_CHK(run());
                HIP_CHK(hipEventRecord(b, H->s));
                HIP_CHK(hipEventSynchronize(b));
                float t = 0.f;
                HIP_CHK(hipEventElapsedTime(&t, a, b));
                ms = std::min(ms, t);
            }
        }
        return hipSuccess;
    };
    const long long nn = H->geom[l].nn;
    const int first_split = H->opt.tile_split >= 0 ? H->opt.tile_split : 0;
    float best = 1e30f, t1 = 1e30f, t2 = 1e30f;   // fastest overall; fastest two depths of the first pass
    int best_tz = 0, best_split = 0, tz1 = 0, tz2 = 0;
    hipError_t err = hipSuccess;
    for (int tz : kTzCandidates) {
        if (H->opt.tile_tz != 0) {
            if (tz != kTzCandidates[0]) break;
            tz = H->opt.tile_tz;
        } else {
            const int planes = H->geom[l].n[2] + 1;
            if (tz > planes && tz != kTzCandidates[0]) break;
            // short marches pay the plane pipeline's start every few planes: never the fastest on
            // large levels (unless the level is too thin for longer ones)
            if ((tz < 4 && nn > (1LL << 20) && planes >= 4) || (tz < 8 && nn > (1LL << 23) && planes >= 8)) continue;
        }
        float ms = 0.f;
        if ((err = time_one(tz, first_split, ms)) != hipSuccess) break;
        if (ms < best) best = ms, best_tz = tz, best_split = first_split;
        if (ms < t1) t2 = t1, tz2 = tz1, t1 = ms, tz1 = tz;
        else if (ms < t2) t2 = ms, tz2 = tz;
    }
    if (err == hipSuccess && H->opt.tile_split < 0)
        for (int tz : {tz1, tz2}) {
            if (tz == 0) continue;
            float ms = 0.f;
            if ((err = time_one(tz, 1, ms)) != hipSuccess) break;
            if (ms < best) best = ms, best_tz = tz, best_split = 1;
        }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    H->Lf[l].tz[fam] = H->Ld[l].tz[fam] = best_tz;
    H->Lf[l].split[fam] = H->Ld[l].split[fam] = best_split;
    return err;
}

// Tile choices already timed in this process, per device, precision, level shape, kernel
// family and batch slots (and the options that restrict the candidates): a later setup of
// the same shape reuses them instead of timing again.
struct TileKey {
    int dev, prec, fam, tz_opt, split_opt, slots, n[3];
    bool operator<(const TileKey &o) const {
        return std::memcmp(this, &o, sizeof(TileKey)) < 0;
    }
};
std::mutex g_tile_mutex;
std::map<TileKey, std::pair<int, int>> g_tile_cache;

hipError_t tune_tiles(helm_hierarchy *H) {
    if (H->opt.tile_tz != 0 && H->opt.tile_split >= 0) {
        for (int l = 0; l < 3; ++l)
            for (int f = 0; f < 2; ++f) {
                H->Lf[l].tz[f] = H->Ld[l].tz[f] = H->opt.tile_tz;
                H->Lf[l].split[f] = H->Ld[l].split[f] = H->opt.tile_split;
            }
        return hipSuccess;
    }
    int dev = 0;
    HIP_CHK(hipGetDevice(&dev));
    for (int l = 0; l < 3; ++l)
        for (int f = 0; f < 2; ++f) {
            TileKey key;
            std::memset(&key, 0, sizeof(key));
            key.dev = dev;
            key.prec = H->prec;
            key.fam = f;
            key.tz_opt = H->opt.tile_tz;
            key.split_opt = H->opt.tile_split;
            key.slots = H->lane[0].nslot;
            for (int a = 0; a < 3; ++a) key.n[a] = H->geom[l].n[a];
            {
                std::lock_guard<std::mutex> lock(g_tile_mutex);
                auto it = g_tile_cache.find(key);
                if (it != g_tile_cache.end()) {
                    H->Lf[l].tz[f] = H->Ld[l].tz[f] = it->second.first;
                    H->Lf[l].split[f] = H->Ld[l].split[f] = it->second.second;
                    continue;
                }
            }
            hipError_t e = (H->prec == HELM_FP64) ? tune_level_tiles<c64>(H, l, f) : tune_level_tiles<c32>(H, l, f);
            if (e != hipSuccess) return e;
            std::lock_guard<std::mutex> lock(g_tile_mutex);
            g_tile_cache[key] = {H->Lf[l].tz[f], H->Lf[l].split[f]};
        }
    return hipSuccess;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

helm_status helm_default_options(helm_options *o) {
    if (!o) return fail(nullptr, HELM_EINVAL, "options pointer is NULL");
    std::memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(helm_options);
    o->precision = HELM_FP32;
    o->sigma = 0.9;
    o->omega_h = 0.8;
    o->omega_2h = 0.8;
    o->omega_4h = 0.2;
    o->gamma_max = 1.119058;
    o->nJ_h = o->nJ_2h = o->nJ_4h = 2;
    o->m_h = 2;
    o->c_2h = 2;
    o->m_2h = 10;
    o->m_4h = 4;
    o->m_out = 5;
    o->max_outer = 1000;
    o->iofd_table = nullptr;
    o->iofd_K = 0;
    o->stream = nullptr;
    o->tile_tz = 0;
    o->tile_split = -1;
    o->lanes = 1;
    o->batch = 1;
    return HELM_OK;
}

helm_status helm_workspace_size(int nx, int ny, int nz, int n_pml, const helm_options *opt, size_t *bytes) {
    std::string msg;
    int N[3];
    helm_status st = check_options(opt, msg);
    if (st == HELM_OK) st = check_dims(nx, ny, nz, n_pml, N, msg);
    if (st == HELM_OK && !bytes) { msg = "bytes pointer is NULL"; st = HELM_EINVAL; }
    if (st != HELM_OK) return fail(nullptr, st, msg);
    *bytes = carve(nullptr, nullptr, N, *opt, opt->iofd_K);
    return HELM_OK;
}

helm_status helm_setup(const float *velocity, int nx, int ny, int nz, double h, double omega, int n_pml,
                       const helm_options *opt, void *workspace, size_t ws_bytes, helm_hierarchy **out) {
    std::string msg;
    int N[3];
    helm_status st = check_options(opt, msg);
    if (st == HELM_OK) st = check_dims(nx, ny, nz, n_pml, N, msg);
    if (st == HELM_OK && opt->pml_variant == 2 && n_pml < 2) {
        msg = "pml_variant 2 needs n_pml >= 2";
        st = HELM_EINVAL;
    }
    if (st == HELM_OK && (!velocity || !out)) { msg = "velocity and out must not be NULL"; st = HELM_EINVAL; }
    if (st == HELM_OK && (!(h > 0) || !(omega > 0) || !std::isfinite(h) || !std::isfinite(omega))) {
        msg = "h and omega must be finite and positive";
        st = HELM_EINVAL;
    }
    if (st == HELM_OK && !opt->iofd_table) { msg = "options.iofd_table is required"; st = HELM_EINVAL; }
    if (st == HELM_OK) {
        for (int i = 0; i < (opt->iofd_K + 1) * 16; ++i)
            if (!std::isfinite(opt->iofd_table[i])) { msg = "iofd_table holds a non-finite value"; st = HELM_EINVAL; break; }
    }
    if (st != HELM_OK) return fail(nullptr, st, msg);
    const size_t need = carve(nullptr, nullptr, N, *opt, opt->iofd_K);
    if (!workspace || ws_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255u))
        return fail(nullptr, HELM_EWORKSPACE, "workspace missing, smaller than helm_workspace_size() or not 256-byte aligned");

    helm_hierarchy *H = new helm_hierarchy();
    H->opt = *opt;
    H->prec = opt->precision;
    H->nphys[0] = nx; H->nphys[1] = ny; H->nphys[2] = nz;
    H->n_pml = n_pml;
    H->h = h;
    H->omega = omega;
    H->s = static_cast<hipStream_t>(opt->stream);
    carve(H, static_cast<char *>(workspace), N, *opt, opt->iofd_K);
    H->opt.iofd_table = nullptr;   // copied below, not retained

    auto bail = [&](helm_status code, const std::string &m) {
        g_thread_error = m;
        release_lanes(H);
        delete H;
        return code;
    };
    hipError_t e;
    hipStream_t s = H->s;
    for (int li = 0; li < H->nlanes; ++li) {
        Lane &Ln = H->lane[li];
        Ln.s = s;
        if (li > 0) {
            if ((e = hipStreamCreateWithFlags(&Ln.s, hipStreamNonBlocking)) != hipSuccess)
                return bail(HELM_EHIP, std::string("lane stream: ") + hipGetErrorString(e));
            Ln.own_stream = true;
        }
        if ((e = hipHostMalloc((void **)&Ln.host_state, sizeof(KState) * kMaxBatch)) != hipSuccess ||
            (e = hipHostMalloc((void **)&Ln.host_scratch, kScratchDoubles * sizeof(double))) != hipSuccess)
            return bail(HELM_EHIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
        // reduction counters start at zero
        if ((e = hipMemsetAsync(Ln.rb.counter, 0, 64 * sizeof(unsigned), s)) != hipSuccess)
            return bail(HELM_EHIP, hipGetErrorString(e));
    }
    // velocity must be finite and positive
    const long long nphys = (long long)(nx + 1) * (ny + 1) * (nz + 1);
    if ((e = launch_velocity_check(velocity, nphys, H->lane[0].rb, H->lane[0].dscratch, s)) != hipSuccess ||
        (e = hipMemcpyAsync(H->lane[0].host_scratch, H->lane[0].dscratch, 3 * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return bail(HELM_EHIP, std::string("velocity check: ") + hipGetErrorString(e));
    if (H->lane[0].host_scratch[2] != 0.0 || !(H->lane[0].host_scratch[0] > 0.0))
        return bail(HELM_EINVAL, "velocity must be finite and positive everywhere");
    H->cmin = H->lane[0].host_scratch[0];
    H->cmax = H->lane[0].host_scratch[1];

    const double Lpml = n_pml * h;
    std::vector<double> w;
    std::vector<float> wfv;
    for (int l = 0; l < 3; ++l) {
        Geom &g = H->geom[l];
        level_geom(N, l, h, g);
        for (int a = 0; a < 3; ++a) {
            axis_weights(g.n[a], g.ell, N[a] * h, Lpml, h, opt->gamma_max, opt->pml_variant, w, g.lo[a], g.hi[a]);
            wfv.assign(w.begin(), w.end());
            if ((e = hipMemcpyAsync(H->wd[l][a], w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess ||
                (e = hipMemcpyAsync(H->wf[l][a], wfv.data(), wfv.size() * sizeof(float), hipMemcpyHostToDevice, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return bail(HELM_EHIP, std::string("upload: ") + hipGetErrorString(e));
        }
        if ((e = launch_extend_velocity(velocity, H->nphys, n_pml, 1 << l, g, H->vel[l], s)) != hipSuccess)
            return bail(HELM_EHIP, hipGetErrorString(e));
    }
    std::vector<double> at, bt, ct;
    hermite_monomials(opt->iofd_table, opt->iofd_K, 0, 5, at);
    hermite_monomials(opt->iofd_table, opt->iofd_K, 5, 3, bt);
    shell_quintics(at, opt->iofd_K, ct);
    std::vector<float> atf(at.begin(), at.end()), btf(bt.begin(), bt.end()), ctf(ct.begin(), ct.end());
    if (H->prec != HELM_FP64) {
        if ((e = hipMemcpyAsync(H->ctab_f, ctf.data(), ctf.size() * sizeof(float), hipMemcpyHostToDevice, s)) !=
            hipSuccess)
            return bail(HELM_EHIP, std::string("table upload: ") + hipGetErrorString(e));
        for (int l = 0; l < 3; ++l) {
            const double factor = omega * H->geom[l].ell * opt->iofd_K / (0.4 * 2.0 * M_PI);
            if ((e = launch_scaled_eta(H->vel[l], H->geom[l].nn, factor, H->svel[l], s)) != hipSuccess)
                return bail(HELM_EHIP, hipGetErrorString(e));
        }
    }
    if ((e = hipMemcpyAsync(H->atab_d, at.data(), at.size() * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(H->btab_d, bt.data(), bt.size() * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(H->atab_f, atf.data(), atf.size() * sizeof(float), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(H->btab_f, btf.data(), btf.size() * sizeof(float), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return bail(HELM_EHIP, std::string("table upload: ") + hipGetErrorString(e));
    for (int l = 0; l < 3; ++l) {
        // FP16 units: a cycle input of unit norm has entries of RMS 1/64; D^-1 ~ ell^2 / 4
        H->fres[l] = (float)(std::sqrt((double)H->geom[l].nn) / 64.0);
        H->fsol[l] = (float)(H->fres[l] * 4.0 / (H->geom[l].ell * H->geom[l].ell));
    }
    {
        static const double one = 1.0;
        if ((e = hipMemcpyAsync(H->d_one, &one, sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return bail(HELM_EHIP, std::string("upload: ") + hipGetErrorString(e));
    }
    for (int l = 0; l < 3; ++l) {
        fill_level_args<float>(H, l, H->Lf[l], H->wf[l][0], H->wf[l][1], H->wf[l][2], H->atab_f, H->btab_f);
        fill_level_args<double>(H, l, H->Ld[l], H->wd[l][0], H->wd[l][1], H->wd[l][2], H->atab_d, H->btab_d);
    }
    for (int l = 0; l < 3; ++l)
        for (int sh = 0; sh < 2; ++sh) {
            e = (H->prec == HELM_FP64) ? launch_dinv<double>(H->Ld[l], sh, static_cast<double *>(H->dinv[l][sh]), s)
                                       : launch_dinv<float>(H->Lf[l], sh, static_cast<float *>(H->dinv[l][sh]), s);
            if (e != hipSuccess) return bail(HELM_EHIP, std::string("diagonal: ") + hipGetErrorString(e));
        }
    if ((e = tune_tiles(H)) != hipSuccess) return bail(HELM_EHIP, std::string("tile tuning: ") + hipGetErrorString(e));
    *out = H;
    return HELM_OK;
}

static helm_status solve_impl(helm_hierarchy *H, const void *f, int nrhs, double tol, void *u, void *v, int *iters,
                              double *relres) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    if (!f || !u || !iters || !relres || nrhs < 0 || !(tol > 0) || !std::isfinite(tol))
        return fail(H, HELM_EINVAL, "invalid solve arguments");
    if (f == u || v == f || v == u) return fail(H, HELM_EINVAL, "f, u and v must not alias");
    const size_t es = (H->prec == HELM_FP64) ? sizeof(c64) : sizeof(c32);
    const long long n = H->geom[0].nn;
    // right-hand sides r .. r + cnt - 1 on one lane, cnt <= the lane's slots
    auto one = [&](int lane, int r, int cnt) {
        const char *fr = static_cast<const char *>(f) + (size_t)r * n * es;
        char *ur = static_cast<char *>(u) + (size_t)r * n * es;
        c64 *vr = v ? static_cast<c64 *>(v) + (size_t)r * n : nullptr;
        return (H->prec == HELM_FP64)
                   ? Eng<c64>(H, lane).solve_batch((const c64 *)fr, (c64 *)ur, cnt, tol, iters + r, relres + r, vr)
                   : Eng<c32>(H, lane).solve_batch((const c32 *)fr, (c32 *)ur, cnt, tol, iters + r, relres + r, vr);
    };
    const int B = H->lane[0].nslot;
    const int chunks = (nrhs + B - 1) / B;
    const int L = std::min(H->nlanes, chunks);
    if (L <= 1) {
        helm_status worst = HELM_OK;
        for (int r = 0; r < nrhs; r += B) {
            helm_status st = one(0, r, std::min(B, nrhs - r));
            if (st < 0) return st;
            if (st == HELM_NOT_CONVERGED) worst = st;
        }
        return worst;
    }
    // Lanes 1.. start after the work already queued on the caller's stream (lane 0);
    // each lane takes the next right-hand side until none is left.  Every solve
    // ends by synchronising its lane's stream, so all results are in place on return.
    hipEvent_t ready;
    HIP_TRY(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ready, H->s);
    for (int li = 1; li < L && e == hipSuccess; ++li) e = hipStreamWaitEvent(H->lane[li].s, ready, 0);
    int dev = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        (void)hipEventDestroy(ready);
        return fail(H, HELM_EHIP, std::string("lane start: ") + hipGetErrorString(e));
    }
    std::atomic<int> next(0);
    std::vector<helm_status> lane_st(L, HELM_OK);
    std::vector<std::thread> pool;
    for (int li = 0; li < L; ++li)
        pool.emplace_back([&, li] {
            if (li > 0 && hipSetDevice(dev) != hipSuccess) {
                lane_st[li] = fail(H, HELM_EHIP, "lane thread could not select the device");
                return;
            }
            for (int c = next++; c < chunks; c = next++) {
                const int r = c * B;
                helm_status st = one(li, r, std::min(B, nrhs - r));
                if (st < 0) {
                    lane_st[li] = st;
                    next = chunks;   // stop handing out work
                    return;
                }
                if (st == HELM_NOT_CONVERGED) lane_st[li] = st;
            }
        });
    for (auto &t : pool) t.join();
    (void)hipEventDestroy(ready);
    helm_status worst = HELM_OK;
    for (helm_status st : lane_st) {
        if (st < 0) return st;
        if (st == HELM_NOT_CONVERGED) worst = st;
    }
    return worst;
}

helm_status helm_solve(helm_hierarchy *H, const void *f, int nrhs, double tol, void *u, int *iters, double *relres) {
    return solve_impl(H, f, nrhs, tol, u, nullptr, iters, relres);
}

helm_status helm_solve_checkpoint(helm_hierarchy *H, const void *f, int nrhs, double tol, void *u, void *v, int *iters,
                                  double *relres) {
    if (!v) return fail(H, HELM_EINVAL, "v must not be NULL");
    return solve_impl(H, f, nrhs, tol, u, v, iters, relres);
}

// Gradient workspace: v (c64), the adjoint residual (c64), the FP64 per-node sums, one
// working-precision vector and the per-axis PML node factors 1/xi (c64).
static size_t grad_ws_bytes(const helm_hierarchy *H) {
    const size_t n = (size_t)H->geom[0].nn;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t es = (H->prec == HELM_FP64) ? sizeof(c64) : sizeof(c32);
    const Geom &g = H->geom[0];
    return 2 * up(n * sizeof(c64)) + up(n * sizeof(double)) + up(n * es) +
           up(2 * (size_t)(g.n[0] + g.n[1] + g.n[2] + 3) * sizeof(c64));
}

helm_status helm_grad_workspace_size(const helm_hierarchy *H, size_t *bytes) {
    if (!H || !bytes) return fail(const_cast<helm_hierarchy *>(H), HELM_EINVAL, "invalid workspace-size arguments");
    *bytes = grad_ws_bytes(H);
    return HELM_OK;
}

helm_status helm_grad(helm_hierarchy *H, const void *f, const void *adj_src, const void *v_fwd, int nrhs, double tol,
                      float *grad_m, void *workspace, size_t ws_bytes, int *iters, double *relres) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    if (!f || !adj_src || !grad_m || !workspace || !iters || !relres || nrhs < 1 || !(tol > 0) ||
        !std::isfinite(tol))
        return fail(H, HELM_EINVAL, "invalid gradient arguments");
    if (ws_bytes < grad_ws_bytes(H) || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return fail(H, HELM_EWORKSPACE, "gradient workspace too small or not 256-byte aligned");
    const long long n = H->geom[0].nn;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *w = static_cast<char *>(workspace);
    c64 *v64 = reinterpret_cast<c64 *>(w);
    c64 *r64 = reinterpret_cast<c64 *>(w + up(n * sizeof(c64)));
    double *gacc = reinterpret_cast<double *>(w + 2 * up(n * sizeof(c64)));
    const size_t es = (H->prec == HELM_FP64) ? sizeof(c64) : sizeof(c32);
    void *u_t = w + 2 * up(n * sizeof(c64)) + up(n * sizeof(double));
    c64 *xin = reinterpret_cast<c64 *>(w + 2 * up(n * sizeof(c64)) + up(n * sizeof(double)) + up(n * es));
    {   // 1/xi_j, then xi_j, at the fine nodes of each axis (eq. pml-profile), x then y then z
        const Geom &g = H->geom[0];
        const double Lpml = H->n_pml * H->h;
        std::vector<c64> hx;
        for (int q = 0; q < 2; ++q)
        for (int a = 0; a < 3; ++a) {
            const double L = g.n[a] * H->h;
            for (int j = 0; j <= g.n[a]; ++j) {
                const double xj = j * H->h;
                double gam = 0.0;
                if (Lpml > 0) {
                    const double d = std::min(Lpml, std::max(0.0, std::max(Lpml - xj, xj - (L - Lpml))));
                    gam = H->opt.gamma_max * (1.0 - std::cos(M_PI * d / (2.0 * Lpml)));
                }
                const double den = 1.0 + gam * gam;
                hx.push_back(q == 0 ? c64{1.0 / den, -gam / den} : c64{1.0, gam});
            }
        }
        HIP_TRY(hipMemcpyAsync(xin, hx.data(), hx.size() * sizeof(c64), hipMemcpyHostToDevice, H->s));
        HIP_TRY(hipStreamSynchronize(H->s));
    }
    helm_status worst = HELM_OK;
    auto run = [&](auto E, auto *tag) -> helm_status {
        using TT = typename std::remove_pointer<decltype(tag)>::type;
        HIP_TRY((launch_fill_zero<c64>(reinterpret_cast<c64 *>(gacc), n / 2, E.s)));   // n doubles
        if (n & 1) HIP_TRY(hipMemsetAsync(gacc + n - 1, 0, sizeof(double), E.s));
        for (int r = 0; r < nrhs; ++r) {
            const TT *fr = reinterpret_cast<const TT *>(static_cast<const char *>(f) + (size_t)r * n * es);
            const TT *sr = reinterpret_cast<const TT *>(static_cast<const char *>(adj_src) + (size_t)r * n * es);
            const c64 *vr = v64;
            helm_status st = HELM_OK;
            if (v_fwd) {
                // checkpointed forward solution (helm_solve_checkpoint): no forward solve
                vr = static_cast<const c64 *>(v_fwd) + (size_t)r * n;
                iters[2 * r] = 0;
                relres[2 * r] = 0.0;
            } else {
                // forward: A_h v = Q_h f (v kept in FP64)
                st = E.solve_one(fr, nullptr, tol, iters + 2 * r, relres + 2 * r);
                if (st < 0) return st;
                if (st == HELM_NOT_CONVERGED) worst = st;
                HIP_TRY((launch_convert<c64, c64>(E.Ln->x64, v64, n, E.s)));
            }
            // adjoint: A_h^T mu = Q_h^T conj(s)
            HIP_TRY((launch_qapply_t<double, TT, c64>(H->Ld[0], sr, true, E.Ln->b64, E.s)));
            E.transposed = true;
            E.r64 = r64;
            E.xin = xin;
            E.u_t = static_cast<TT *>(u_t);
            st = E.solve_b64(tol, iters + 2 * r + 1, relres + 2 * r + 1);
            E.transposed = false;
            if (st < 0) return st;
            if (st == HELM_NOT_CONVERGED) worst = st;
            HIP_TRY((launch_grad_node<TT>(H->Ld[0], vr, E.Ln->x64, sr, fr, gacc, E.s)));
        }
        HIP_TRY(launch_grad_phys(gacc, H->geom[0], H->n_pml, H->nphys, grad_m, E.s));
        HIP_TRY(hipStreamSynchronize(E.s));
        return HELM_OK;
    };
    helm_status st = (H->prec == HELM_FP64) ? run(Eng<c64>(H, 0), (c64 *)nullptr) : run(Eng<c32>(H, 0), (c32 *)nullptr);
    return st < 0 ? st : worst;
}

void helm_destroy(helm_hierarchy *H) {
    if (!H) return;
    release_lanes(H);
    delete H;
}

const char *helm_last_error(const helm_hierarchy *H) { return H ? H->err.c_str() : g_thread_error.c_str(); }

// Tile-choice file: a header line, then one line per choice:
//   <arch> <precision> <family> <tile_tz option> <tile_split option> <slots> <n0> <n1> <n2> <z depth> <split>
// <arch> is the GPU's architecture name up to its first ':' (e.g. gfx950).
static const char *const kTileHeader = "# helm tile choices v2";

static std::string device_arch(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return std::string();
    std::string a(p.gcnArchName);
    return a.substr(0, a.find(':'));
}

helm_status helm_tiles_save(const char *path) {
    if (!path) return fail(nullptr, HELM_EINVAL, "path is NULL");
    std::vector<std::pair<TileKey, std::pair<int, int>>> entries;
    {
        std::lock_guard<std::mutex> lock(g_tile_mutex);
        entries.assign(g_tile_cache.begin(), g_tile_cache.end());
    }
    FILE *fp = std::fopen(path, "w");
    if (!fp) return fail(nullptr, HELM_EINVAL, std::string("cannot write ") + path);
    bool ok = std::fprintf(fp, "%s\n", kTileHeader) > 0;
    for (const auto &e : entries) {
        const TileKey &k = e.first;
        const std::string arch = device_arch(k.dev);
        if (arch.empty()) continue;
        ok = ok && std::fprintf(fp, "%s %d %d %d %d %d %d %d %d %d %d\n", arch.c_str(), k.prec, k.fam, k.tz_opt,
                                k.split_opt, k.slots, k.n[0], k.n[1], k.n[2], e.second.first, e.second.second) > 0;
    }
    ok = (std::fclose(fp) == 0) && ok;
    if (!ok) return fail(nullptr, HELM_EINVAL, std::string("error writing ") + path);
    return HELM_OK;
}

helm_status helm_tiles_load(const char *path, int *n_loaded) {
    if (n_loaded) *n_loaded = 0;
    if (!path) return fail(nullptr, HELM_EINVAL, "path is NULL");
    FILE *fp = std::fopen(path, "r");
    if (!fp) return fail(nullptr, HELM_EINVAL, std::string("cannot read ") + path);
    // visible GPUs by architecture (none without a GPU: the file is still checked)
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
    std::vector<std::string> archs;
    for (int d = 0; d < ndev; ++d) archs.push_back(device_arch(d));
    char line[512];
    int lineno = 0, added = 0;
    helm_status st = HELM_OK;
    std::string msg;
    while (std::fgets(line, sizeof line, fp)) {
        ++lineno;
        if (lineno == 1) {
            if (std::strncmp(line, kTileHeader, std::strlen(kTileHeader)) != 0) {
                st = HELM_EINVAL;
                msg = std::string(path) + ": not a tile-choice file";
                break;
            }
            continue;
        }
        char arch[64];
        int v[10], tail = 0;
        const int got = std::sscanf(line, "%63s %d %d %d %d %d %d %d %d %d %d %n", arch, &v[0], &v[1], &v[2],
                                    &v[3], &v[4], &v[5], &v[6], &v[7], &v[8], &v[9], &tail);
        const bool valid = got == 11 && line[tail] == '\0' && v[0] >= HELM_FP64 && v[0] <= HELM_MIXED &&
                           (v[1] == 0 || v[1] == 1) && (v[2] == 0 || (v[2] >= kTzMin && v[2] <= kTzMax)) &&
                           v[3] >= -1 && v[3] <= 1 && v[4] >= 1 && v[4] <= kMaxBatch && v[5] >= 2 && v[6] >= 2 &&
                           v[7] >= 2 && v[8] >= kTzMin && v[8] <= kTzMax && (v[9] == 0 || v[9] == 1);
        if (!valid) {
            st = HELM_EINVAL;
            msg = std::string(path) + ": malformed line " + std::to_string(lineno);
            break;
        }
        for (int d = 0; d < ndev; ++d) {
            if (archs[d] != arch) continue;
            TileKey key;
            std::memset(&key, 0, sizeof(key));
            key.dev = d;
            key.prec = v[0];
            key.fam = v[1];
            key.tz_opt = v[2];
            key.split_opt = v[3];
            key.slots = v[4];
            for (int a = 0; a < 3; ++a) key.n[a] = v[5 + a];
            std::lock_guard<std::mutex> lock(g_tile_mutex);
            g_tile_cache[key] = {v[8], v[9]};
            ++added;
        }
    }
    std::fclose(fp);
    if (n_loaded) *n_loaded = added;
    if (st == HELM_OK && lineno == 0) {
        st = HELM_EINVAL;
        msg = std::string(path) + ": empty file";
    }
    return st == HELM_OK ? HELM_OK : fail(nullptr, st, msg);
}

helm_status helm_dims(const helm_hierarchy *H, int level, int dims[3]) {
    if (!H || !dims || !level_ok(level)) return fail(const_cast<helm_hierarchy *>(H), HELM_EINVAL, "invalid arguments");
    for (int a = 0; a < 3; ++a) dims[a] = H->geom[level].n[a];
    return HELM_OK;
}

helm_status helm_grad_to_velocity(helm_hierarchy *H, const float *grad_m, float *grad_c) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    if (!grad_m || !grad_c) return fail(H, HELM_EINVAL, "invalid gradient-conversion arguments");
    HIP_TRY(launch_grad_to_velocity(grad_m, H->vel[0], H->geom[0], H->n_pml, H->nphys, grad_c, H->s));
    return HELM_OK;
}

helm_status helm_apply(helm_hierarchy *H, int level, int op, const void *x, void *y) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    const bool fine_only = op == HELM_OP_Q || op == HELM_OP_QT || op == HELM_OP_DA || op == HELM_OP_DQ;
    if (!level_ok(level) || op < 0 || op > HELM_OP_DQ || (fine_only && level != 0) || !x || !y || x == y)
        return fail(H, HELM_EINVAL, "invalid apply arguments");
    return dispatch(H, [&](auto E) -> hipError_t {
        using T = typename std::remove_reference<decltype(E)>::type;
        using V = decltype(*E.v(nullptr));
        using TT = typename std::remove_reference<V>::type;
        using RR = typename T::R;
        if (op == HELM_OP_AT || op == HELM_OP_BT)
            return launch_apply_t<RR, TT, TT, TT>(E.L(level), op == HELM_OP_BT, (const TT *)x, (const TT *)nullptr,
                                                  (TT *)y, E.s);
        if (op == HELM_OP_QT) return launch_qapply_t<RR, TT, TT>(E.L(0), (const TT *)x, false, (TT *)y, E.s);
        if (op == HELM_OP_DA || op == HELM_OP_DQ)
            return launch_apply_dm<RR, TT>(E.L(0), op == HELM_OP_DQ, (const TT *)x, (TT *)y, E.s);
        if (op == HELM_OP_A || op == HELM_OP_B)
            return E.stencil(level, M_APPLY, op == HELM_OP_B, 0.0, x, nullptr, nullptr, y);
        if (op == HELM_OP_Q)
            return launch_qapply<typename T::R, TT, TT>(E.L(0), (const TT *)x, (TT *)y, E.s);
        return launch_diag<typename T::R, TT>(E.L(level), op == HELM_OP_DIAG_B, (const TT *)x, (TT *)y, E.s);
    });
}

helm_status helm_residual(helm_hierarchy *H, int level, int op, const void *g, const void *x, void *r) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    if (!level_ok(level) || (op != HELM_OP_A && op != HELM_OP_B) || !g || !x || !r || r == x || r == g)
        return fail(H, HELM_EINVAL, "invalid residual arguments");
    return dispatch(H, [&](auto E) { return E.stencil(level, M_RESID, op == HELM_OP_B, 0.0, x, g, nullptr, r); });
}

helm_status helm_residual_restrict(helm_hierarchy *H, int level, int op, const void *g, const void *x, void *coarse) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    if (level < 0 || level > 1 || (op != HELM_OP_A && op != HELM_OP_B) || !g || !x || !coarse || coarse == x ||
        coarse == g)
        return fail(H, HELM_EINVAL, "invalid residual-restrict arguments");
    return dispatch(H, [&](auto E) {
        using TT = typename std::remove_reference<decltype(*E.v(nullptr))>::type;
        return E.resid_restrict(level, op == HELM_OP_B, (const TT *)x, (const TT *)g, (TT *)coarse);
    });
}

helm_status helm_jacobi(helm_hierarchy *H, int level, int op, const void *g, int nJ, double omega, void *y) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    if (!level_ok(level) || (op != HELM_OP_A && op != HELM_OP_B) || !g || !y || g == y || nJ < 1 || nJ > 64 ||
        !std::isfinite(omega))
        return fail(H, HELM_EINVAL, "invalid jacobi arguments");
    return dispatch(H, [&](auto E) {
        using TT = typename std::remove_reference<decltype(*E.v(nullptr))>::type;
        return E.jacobi(level, op == HELM_OP_B, nJ, omega, (const TT *)g, (TT *)y);
    });
}

helm_status helm_restrict(helm_hierarchy *H, int level, const void *fine, void *coarse) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    if (level < 0 || level > 1 || !fine || !coarse) return fail(H, HELM_EINVAL, "invalid restrict arguments");
    return dispatch(H, [&](auto E) {
        using TT = typename std::remove_reference<decltype(*E.v(nullptr))>::type;
        return launch_restrict<TT>(H->geom[level], H->geom[level + 1], (const TT *)fine, (TT *)coarse, E.s);
    });
}

helm_status helm_prolong_add(helm_hierarchy *H, int level, const void *coarse, void *fine) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    if (level < 1 || level > 2 || !fine || !coarse) return fail(H, HELM_EINVAL, "invalid prolong arguments");
    return dispatch(H, [&](auto E) {
        using TT = typename std::remove_reference<decltype(*E.v(nullptr))>::type;
        return launch_prolong_add<TT>(H->geom[level], H->geom[level - 1], (const TT *)coarse, (TT *)fine, E.s);
    });
}

helm_status helm_bottom(helm_hierarchy *H, const void *q, void *e) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    if (!q || !e || q == e) return fail(H, HELM_EINVAL, "invalid bottom arguments");
    return dispatch(H, [&](auto E) {
        using TT = typename std::remove_reference<decltype(*E.v(nullptr))>::type;
        return E.bottom_hook((const TT *)q, (TT *)e);
    });
}

helm_status helm_vcycle(helm_hierarchy *H, const void *q, void *y) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    if (!q || !y || q == y) return fail(H, HELM_EINVAL, "invalid vcycle arguments");
    return dispatch(H, [&](auto E) {
        using TT = typename std::remove_reference<decltype(*E.v(nullptr))>::type;
        return E.vcycle_hook((const TT *)q, (TT *)y);
    });
}

helm_status helm_coarse_solve(helm_hierarchy *H, const void *r, void *e) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    if (!r || !e || r == e) return fail(H, HELM_EINVAL, "invalid coarse-solve arguments");
    return dispatch(H, [&](auto E) {
        using TT = typename std::remove_reference<decltype(*E.v(nullptr))>::type;
        return E.k2h((const TT *)r, (TT *)e);
    });
}

helm_status helm_smooth(helm_hierarchy *H, const void *g, const void *x0, void *x) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    if (!g || !x || g == x) return fail(H, HELM_EINVAL, "invalid smooth arguments");
    return dispatch(H, [&](auto E) -> hipError_t {
        using TT = typename std::remove_reference<decltype(*E.v(nullptr))>::type;
        if (x0 && x0 != x) HIP_CHK((launch_convert<TT, TT>((const TT *)x0, (TT *)x, E.nn(0), E.s)));
        return E.smooth((const TT *)g, (TT *)x, x0 == nullptr);
    });
}

helm_status helm_precond(helm_hierarchy *H, const void *r, void *z) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    if (!r || !z || r == z) return fail(H, HELM_EINVAL, "invalid precond arguments");
    return dispatch(H, [&](auto E) {
        using TT = typename std::remove_reference<decltype(*E.v(nullptr))>::type;
        return E.precond((const TT *)r, (TT *)z);
    });
}

helm_status helm_vec_dots(helm_hierarchy *H, int level, int k, const void *const *V, const void *w, double *out) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    if (!level_ok(level) || k < 0 || k > kMMax || (k > 0 && !V) || !w || !out)
        return fail(H, HELM_EINVAL, "invalid dots arguments");
    helm_status st = dispatch(H, [&](auto E) {
        using TT = typename std::remove_reference<decltype(*E.v(nullptr))>::type;
        return launch_dots<TT>((const TT *const *)V, k, (const TT *)w, true, E.nn(level), EPI_STORE, nullptr, 0,
                               H->lane[0].dscratch, H->lane[0].rb, E.s);
    });
    if (st != HELM_OK) return st;
    HIP_TRY(hipMemcpyAsync(H->lane[0].host_scratch, H->lane[0].dscratch, 2 * (k + 1) * sizeof(double), hipMemcpyDeviceToHost, H->s));
    HIP_TRY(hipStreamSynchronize(H->s));
    std::memcpy(out, H->lane[0].host_scratch, 2 * (k + 1) * sizeof(double));
    return HELM_OK;
}

helm_status helm_vec_orthonormalize(helm_hierarchy *H, int level, int k, const void *const *V, void *w, double *out) {
    if (!H) return fail(nullptr, HELM_EINVAL, "hierarchy is NULL");
    if (!level_ok(level) || k < 1 || k > kMMax || !V || !w || !out)
        return fail(H, HELM_EINVAL, "invalid orthonormalize arguments");
    HIP_TRY(hipMemsetAsync(H->lane[0].st_hook, 0, sizeof(KState), H->s));
    static const double one = 1.0;   // the caller's V_0 is normalised
    HIP_TRY(hipMemcpyAsync(&H->lane[0].st_hook->vs0, &one, sizeof(double), hipMemcpyHostToDevice, H->s));
    helm_status st = dispatch(H, [&](auto E) -> hipError_t {
        using TT = typename std::remove_reference<decltype(*E.v(nullptr))>::type;
        const TT *const *VV = (const TT *const *)V;
        HIP_CHK(launch_dots<TT>(VV, k, (const TT *)w, false, E.nn(level), EPI_ARNOLDI1, H->lane[0].st_hook, 0, nullptr, H->lane[0].rb,
                                E.s));
        HIP_CHK(launch_axpy_dots<TT>(VV, k, (TT *)w, E.nn(level), H->lane[0].st_hook, H->lane[0].rb, E.s));
        return launch_axpy_scale<TT>(VV, k, (TT *)w, E.nn(level), H->lane[0].st_hook, E.s);
    });
    if (st != HELM_OK) return st;
    HIP_TRY(hipMemcpyAsync(H->lane[0].host_state, H->lane[0].st_hook, sizeof(KState), hipMemcpyDeviceToHost, H->s));
    HIP_TRY(hipStreamSynchronize(H->s));
    for (int j = 0; j < k; ++j) {
        out[2 * j] = H->lane[0].host_state->h1[j][0] + H->lane[0].host_state->h2[j][0];
        out[2 * j + 1] = H->lane[0].host_state->h1[j][1] + H->lane[0].host_state->h2[j][1];
    }
    out[2 * k] = H->lane[0].host_state->hk1;
    out[2 * k + 1] = 0.0;
    return HELM_OK;
}

}  // extern "C"
