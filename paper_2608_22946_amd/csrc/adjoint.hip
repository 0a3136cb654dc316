// Adjoint-state gradient of a misfit of u = Q_h v, A_h v = Q_h f, with respect
// to the squared slowness m = 1/c^2 (Sec. 2.2 fixes that every row of A_h and
// Q_h takes its coefficients at its own node, so d/dm_i touches row i only):
//   transposed operators A^T, B^T (any level; rows staged plane by plane in LDS) and
//   Q_h^T, gathered per output node from the rows of its 27 neighbours (tensor form);
//   the derivative of row i in m_i applied to a vector;
//   the gradient terms conj(s_i)(d_i Q v)_i + mu_i ((d_i Q f)_i - (d_i A v)_i)
//   accumulated in FP64, then summed onto the physical nodes (a PML node takes
//   the velocity of its nearest physical node, Sec. 2.1).
// Apart from A^T, these kernels run once per gradient: one thread per node, every
// coefficient evaluated where it is needed.
#include "helm_internal.h"

namespace helm {
namespace {

template <typename T>
using real_of = decltype(T{}.re);

template <typename R>
struct Zc {
    R r, i;
};

constexpr int kTX = 64, kTY = 4;

dim3 node_grid3(const Geom &g) {
    return dim3((unsigned)((g.n[0] + kTX) / kTX), (unsigned)((g.n[1] + kTY) / kTY), (unsigned)(g.n[2] + 1));
}

template <typename R, typename T>
__device__ __forceinline__ Zc<R> load(const T *p, long long i) {
    const T v = p[i];
    return {(R)v.re, (R)v.im};
}

// Coefficient functions at a node with velocity c on the level of L:
// kappa = omega ell / c, eta = min(kappa / 2pi, 0.4) (eq. iofd-clamped-coordinate),
// the Hermite interval k and local variable t.  de = d eta / d m (0 on the clamp).
template <typename R>
struct Loc {
    R kappa, t, de;
    int k;
};

template <typename R>
__device__ __forceinline__ Loc<R> locate_at(const LevelArgs<R> &L, float c) {
    Loc<R> o;
    const R cc = (R)c;
    o.kappa = L.omega_ell / cc;
    R eta = o.kappa * (R)0.15915494309189533577;   // 1 / (2 pi)
    const bool clamped = !(eta < (R)0.4);
    if (clamped) eta = (R)0.4;
    // kappa = omega ell sqrt(m): d kappa / d m = kappa c^2 / 2
    o.de = clamped ? (R)0 : o.kappa * cc * cc * (R)0.07957747154594766788;   // / (4 pi)
    const R u = eta * L.inv_deta;
    int k = (int)u;
    k = k < L.K - 1 ? k : L.K - 1;
    k = k > 0 ? k : 0;
    o.k = k;
    o.t = u - (R)k;
    return o;
}

template <typename R>
__device__ __forceinline__ R hval(const R *p, R t) { return ((p[3] * t + p[2]) * t + p[1]) * t + p[0]; }

// The five coefficient functions and kappa^2 of the row of node i, from the block's LDS copy
// `tab` of the level's window of table intervals (kb .. kb + nk - 1).  FP32 levels read the
// per-node scaled coordinate s (eta* = min(s, K) 0.4 / K, kappa = s kap_s) as their forward
// stencils do; FP64 levels the velocity.
template <typename R>
__device__ __forceinline__ void row_coefs(const LevelArgs<R> &L, const R *tab, long long i, R (&a)[5], R &k2) {
    R kappa, t;
    int k;
    if constexpr (sizeof(R) == sizeof(float)) {
        const float sv = L.s[i];
        kappa = (R)sv * L.kap_s;
        const R u = (R)sv < (R)L.K ? (R)sv : (R)L.K;
        k = (int)u;
        k = k < L.K - 1 ? k : L.K - 1;
        t = u - (R)k;
    } else {
        const Loc<R> q = locate_at(L, L.c[i]);
        kappa = q.kappa;
        k = q.k;
        t = q.t;
    }
    k = k < L.kb ? L.kb : (k > L.kb + L.nk - 1 ? L.kb + L.nk - 1 : k);
    const R *p = tab + (k - L.kb) * 20;
#pragma unroll
    for (int f = 0; f < 5; ++f) a[f] = hval(p + 4 * f, t);
    k2 = kappa * kappa;
}
template <typename R>
__device__ __forceinline__ R hdt(const R *p, R t) { return ((R)3 * p[3] * t + (R)2 * p[2]) * t + p[1]; }

// transverse weights T[nz] (a4, a5/4, (1-a4-a5)/4) and mass weights M[shell]
// (a1, a2/6, a3/12, (1-a1-a2-a3)/8) of row i, kappa^2 of row i
template <typename R>
struct RowW {
    R T[3], M[4], k2;
};

template <typename R>
__device__ __forceinline__ RowW<R> row_weights(const LevelArgs<R> &L, float c) {
    const Loc<R> q = locate_at(L, c);
    const R *p = L.atab + q.k * 20;
    R a[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) a[f] = hval(p + 4 * f, q.t);
    RowW<R> w;
    w.T[0] = a[3];
    w.T[1] = a[4] * (R)0.25;
    w.T[2] = ((R)1 - a[3] - a[4]) * (R)0.25;
    w.M[0] = a[0];
    w.M[1] = a[1] * (R)(1.0 / 6);
    w.M[2] = a[2] * (R)(1.0 / 12);
    w.M[3] = ((R)1 - a[0] - a[1] - a[2]) * (R)0.125;
    w.k2 = q.kappa * q.kappa;
    return w;
}

// derivatives in m of the same weights (dk2 = d kappa^2 / dm = kappa^2 c^2) and the
// Q_h shell weights' derivatives (b1, b2/6, b3/12, (1-b1-b2-b3)/8)
template <typename R>
struct RowD {
    R dT[3], dM[4], M[4], k2, dk2, dQ[4];
};

template <typename R>
__device__ __forceinline__ RowD<R> row_derivs(const LevelArgs<R> &L, float c) {
    const Loc<R> q = locate_at(L, c);
    const R *p = L.atab + q.k * 20;
    const R *pb = L.btab + q.k * 12;
    const R dt = L.inv_deta * q.de;   // d t / d m
    R a[5], da[5], db[3];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        a[f] = hval(p + 4 * f, q.t);
        da[f] = hdt(p + 4 * f, q.t) * dt;
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) db[f] = hdt(pb + 4 * f, q.t) * dt;
    RowD<R> d;
    d.dT[0] = da[3];
    d.dT[1] = da[4] * (R)0.25;
    d.dT[2] = -(da[3] + da[4]) * (R)0.25;
    d.M[0] = a[0];
    d.M[1] = a[1] * (R)(1.0 / 6);
    d.M[2] = a[2] * (R)(1.0 / 12);
    d.M[3] = ((R)1 - a[0] - a[1] - a[2]) * (R)0.125;
    d.dM[0] = da[0];
    d.dM[1] = da[1] * (R)(1.0 / 6);
    d.dM[2] = da[2] * (R)(1.0 / 12);
    d.dM[3] = -(da[0] + da[1] + da[2]) * (R)0.125;
    d.k2 = q.kappa * q.kappa;
    const R cc = (R)c;
    d.dk2 = d.k2 * cc * cc;
    d.dQ[0] = db[0];
    d.dQ[1] = db[1] * (R)(1.0 / 6);
    d.dQ[2] = db[2] * (R)(1.0 / 12);
    d.dQ[3] = -(db[0] + db[1] + db[2]) * (R)0.125;
    return d;
}

// second-difference weight of axis j at node coordinate a for offset d in {-1, 0, 1}
template <typename R>
__device__ __forceinline__ Zc<R> axis_w(const R *w, int a, int d) {
    const R *p = w + 6 * a + 2 * (d + 1);
    return {p[0], p[1]};
}

template <typename R>
__device__ __forceinline__ bool inside(const LevelArgs<R> &L, int x, int y, int z) {
    return x >= 1 && x <= L.nx - 1 && y >= 1 && y <= L.ny - 1 && z >= 1 && z <= L.nz - 1;
}

// y = op^T x (op A, or B with SHIFT), optionally y = g - op^T x (RESID; zero on the boundary).
// Entry (i, k) of op, i = k + delta, is row i's coefficient for the offset -delta:
//   sum_j w_j(i_j, -delta_j) T_i[nonzeros of delta off axis j] - mu kappa_i^2 M_i[|delta|_1].
// A block owns 64 x 4 output nodes of kTZ consecutive planes and marches in z, staging one
// plane at a time in LDS: every staged node holds x and the weights of its own row, from the
// coefficient functions evaluated once per staging (about 1.7 times per node with the halos):
// T = (a4, a5/4, (1-a4-a5)/4) and kappa^2 M = kappa^2 (a1, a2/6, a3/12, (1-a1-a2-a3)/8).
// A staged plane p holds the neighbour rows of the outputs in planes p - 1, p and p + 1, so
// each thread reads its 9 in-plane neighbours once and adds their terms to three running
// sums; the sum of plane p - 1 is complete and stored after plane p.
constexpr int kTZ = 16;
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHN = kHX * kHY;   // staged plane incl. halo

template <typename R, typename TX>
__device__ __forceinline__ void stage_plane(const LevelArgs<R> &L, const R *tab, const TX *__restrict__ x, int X0,
                                            int Y0, int z, R (*S)[kHN]) {   // S: 9 arrays of kHN
    const int tid = threadIdx.y * kTX + threadIdx.x;
    for (int e = tid; e < kHN; e += kTX * kTY) {
        const int c = e % kHX, r = e / kHX;
        const int xi = X0 - 1 + c, yi = Y0 - 1 + r;
        R v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (inside(L, xi, yi, z)) {   // rows exist at interior nodes only; x is zero elsewhere
            const long long i = (long long)z * L.sy + (long long)yi * L.sx + xi;
            const Zc<R> xv = load<R>(x, i);
            R a[5], k2;
            row_coefs(L, tab, i, a, k2);
            v[0] = xv.r;
            v[1] = xv.i;
            v[2] = a[3];
            v[3] = a[4] * (R)0.25;
            v[4] = ((R)1 - a[3] - a[4]) * (R)0.25;
            v[5] = k2 * a[0];
            v[6] = k2 * a[1] * (R)(1.0 / 6);
            v[7] = k2 * a[2] * (R)(1.0 / 12);
            v[8] = k2 * ((R)1 - a[0] - a[1] - a[2]) * (R)0.125;
        }
#pragma unroll
        for (int f = 0; f < 9; ++f) S[f][e] = v[f];
    }
}

// Blocks whose staged rows are all free of stretching (eq. iofd-shell-form): row i has the
// coefficient C_m(i) (minus i sigma kappa_i^2 M_m(i) when shifted) on its shell-m neighbours, so
// (op^T x)_j = ell^-2 sum_m sum_{i in shell m of j} C_m(i) x_i.  Each staged node then holds
// u_m = C_m(i) x_i (m = 0..3) and the outputs are plain shell sums of the u_m, with no
// per-neighbour coefficient arithmetic.
template <typename R, typename TX, bool SHIFT>
__device__ __forceinline__ void stage_plane_shell(const LevelArgs<R> &L, const R *tab, const TX *__restrict__ x,
                                                  int X0, int Y0, int z, R (*S)[kHN]) {
    const int tid = threadIdx.y * kTX + threadIdx.x;
    for (int e = tid; e < kHN; e += kTX * kTY) {
        const int c = e % kHX, r = e / kHX;
        const int xi = X0 - 1 + c, yi = Y0 - 1 + r;
        const long long i = (long long)z * L.sy + (long long)yi * L.sx + xi;   // an interior node
        const Zc<R> xv = load<R>(x, i);
        R a[5], k2;
        row_coefs(L, tab, i, a, k2);
        const R qq = (R)1 - a[3] - a[4];
        const R M[4] = {a[0], a[1] * (R)(1.0 / 6), a[2] * (R)(1.0 / 12), ((R)1 - a[0] - a[1] - a[2]) * (R)0.125};
        const R C[4] = {(R)6 * a[3] - k2 * M[0], (a[4] - a[3]) - k2 * M[1], (R)0.5 * (qq - a[4]) - k2 * M[2],
                        (R)-0.75 * qq - k2 * M[3]};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const R ci = SHIFT ? -L.sigma * k2 * M[m] : (R)0;
            S[2 * m][e] = C[m] * xv.r - ci * xv.i;
            S[2 * m + 1][e] = C[m] * xv.i + ci * xv.r;
        }
    }
}

template <typename R, typename TX, typename TG, typename TY, bool SHIFT, bool RESID>
__global__ void __launch_bounds__(256) k_apply_t(LevelArgs<R> L, const TX *__restrict__ x, const TG *__restrict__ g,
                                                TY *__restrict__ y) {
    __shared__ R S[9][kHN];   // [x.re, x.im, T0..T2, kappa^2 M0..M3][node] of the staged plane
    extern __shared__ unsigned char smem_raw[];
    R *tab = reinterpret_cast<R *>(smem_raw);   // the level's window of table intervals
    for (int e = threadIdx.y * kTX + threadIdx.x; e < L.nk * 20; e += kTX * kTY) tab[e] = L.atab[L.kb * 20 + e];
    __syncthreads();
    const int X0 = blockIdx.x * kTX, Y0 = blockIdx.y * kTY, Zb = blockIdx.z * kTZ;
    const int X = X0 + threadIdx.x, Y = Y0 + threadIdx.y;
    const int Ze = min(Zb + kTZ, L.nz + 1);
    const bool col = X <= L.nx && Y <= L.ny;
    const bool inxy = X >= 1 && X <= L.nx - 1 && Y >= 1 && Y <= L.ny - 1;
    // axis weights w_j(k_j + d, -d) of the neighbour rows, d = -1, 0, 1 (x and y fixed per thread)
    Zc<R> Wx[3], Wy[3];
#pragma unroll
    for (int d = -1; d <= 1; ++d) {
        Wx[d + 1] = inxy ? axis_w(L.wx, X + d, -d) : Zc<R>{0, 0};
        Wy[d + 1] = inxy ? axis_w(L.wy, Y + d, -d) : Zc<R>{0, 0};
    }
    // every row the block stages (x X0-1..X0+64, y Y0-1..Y0+4, planes Zb-1..Ze) free of stretching
    const bool shell = X0 - 1 >= L.lox && X0 + kTX <= L.hix && Y0 - 1 >= L.loy && Y0 + kTY <= L.hiy &&
                       Zb - 1 >= L.loz && Ze <= L.hiz;
    // acc[0], acc[1], acc[2]: running sums of the outputs in planes p - 1, p, p + 1
    Zc<R> acc[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int p = Zb - 1; p <= Ze; ++p) {
        if (shell) {
            stage_plane_shell<R, TX, SHIFT>(L, tab, x, X0, Y0, p, S);
            __syncthreads();
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int e = (threadIdx.y + 1 + dy) * kHX + threadIdx.x + 1 + dx;
                    const int m = (dx != 0) + (dy != 0);   // shell of this neighbour in its own plane
                    const R u0r = S[2 * m][e], u0i = S[2 * m + 1][e];           // same plane: shell m
                    const R u1r = S[2 * m + 2][e], u1i = S[2 * m + 3][e];       // planes p -+ 1: shell m + 1
                    acc[1].r += u0r;
                    acc[1].i += u0i;
                    acc[0].r += u1r;
                    acc[0].i += u1i;
                    acc[2].r += u1r;
                    acc[2].i += u1i;
                }
        } else {
        stage_plane(L, tab, x, X0, Y0, p, S);
        __syncthreads();
        if (inxy && p >= 1 && p <= L.nz - 1) {   // only interior planes hold rows
            // z weights of row plane p seen from output plane p - dz: w_z(p, -dz)
            Zc<R> Wz[3];
#pragma unroll
            for (int dz = -1; dz <= 1; ++dz) Wz[dz + 1] = axis_w(L.wz, p, -dz);
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int e = (threadIdx.y + 1 + dy) * kHX + threadIdx.x + 1 + dx;
                    const R xr = S[0][e], xi = S[1][e];
                    const R T[3] = {S[2][e], S[3][e], S[4][e]};
                    const R KM[4] = {S[5][e], S[6][e], S[7][e], S[8][e]};
                    const int sxy = (dx != 0) + (dy != 0);
                    const Zc<R> wx = Wx[dx + 1], wy = Wy[dy + 1];
#pragma unroll
                    for (int dz = -1; dz <= 1; ++dz) {   // contribution to output plane p - dz
                        const int nzz = dz != 0;
                        const R tx = T[(dy != 0) + nzz], ty = T[(dx != 0) + nzz], tz = T[sxy];
                        const R km = KM[sxy + nzz];
                        const Zc<R> wz = Wz[dz + 1];
                        Zc<R> cf = {wx.r * tx + wy.r * ty + wz.r * tz - km, wx.i * tx + wy.i * ty + wz.i * tz};
                        if (SHIFT) cf.i -= L.sigma * km;
                        Zc<R> &a = acc[1 - dz];
                        a.r += cf.r * xr - cf.i * xi;
                        a.i += cf.r * xi + cf.i * xr;
                    }
                }
        }
        }
        const int z = p - 1;   // all three neighbour planes of output plane p - 1 are in
        if (col && z >= Zb && z < Ze) {
            const bool in = inxy && z >= 1 && z <= L.nz - 1;
            const long long k = (long long)z * L.sy + (long long)Y * L.sx + X;
            const Zc<R> v = in ? Zc<R>{acc[0].r * L.inv_ell2, acc[0].i * L.inv_ell2} : Zc<R>{0, 0};
            TY o;
            if (RESID) {
                const Zc<R> gv = in ? load<R>(g, k) : Zc<R>{0, 0};
                o.re = (real_of<TY>)(gv.r - v.r);
                o.im = (real_of<TY>)(gv.i - v.i);
            } else {
                o.re = (real_of<TY>)v.r;
                o.im = (real_of<TY>)v.i;
            }
            y[k] = o;
        }
        acc[0] = acc[1];
        acc[1] = acc[2];
        acc[2] = Zc<R>{0, 0};
        __syncthreads();   // the staged plane is overwritten next
    }
}

// y = Q_h^T w (CONJ: of conj(w)); row i of Q_h has the shell weights of its own node
// (eq. q-operator) on its interior neighbours.
template <typename R, typename TI, typename TO, bool CONJ>
__global__ void __launch_bounds__(256) k_qapply_t(LevelArgs<R> L, const TI *__restrict__ w, TO *__restrict__ y) {
    const int X = blockIdx.x * kTX + threadIdx.x, Y = blockIdx.y * kTY + threadIdx.y, Zz = blockIdx.z;
    if (X > L.nx || Y > L.ny) return;
    const long long k = (long long)Zz * L.sy + (long long)Y * L.sx + X;
    Zc<R> acc = {0, 0};
    if (inside(L, X, Y, Zz)) {
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (!inside(L, X + dx, Y + dy, Zz + dz)) continue;
                    const long long i = k + dx + (long long)dy * L.sx + (long long)dz * L.sy;
                    const Loc<R> q = locate_at(L, L.c[i]);
                    const R *pb = L.btab + q.k * 12;
                    const R b1 = hval(pb, q.t), b2 = hval(pb + 4, q.t), b3 = hval(pb + 8, q.t);
                    const int sh = (dx != 0) + (dy != 0) + (dz != 0);
                    const R qm = sh == 0 ? b1 : sh == 1 ? b2 * (R)(1.0 / 6)
                                              : sh == 2 ? b3 * (R)(1.0 / 12) : ((R)1 - b1 - b2 - b3) * (R)0.125;
                    Zc<R> v = load<R>(w, i);
                    if (CONJ) v.i = -v.i;
                    acc.r += qm * v.r;
                    acc.i += qm * v.i;
                }
    }
    TO o;
    o.re = (real_of<TO>)acc.r;
    o.im = (real_of<TO>)acc.i;
    y[k] = o;
}

// (d_i A x)_i and (d_i Q x)_i at an interior node
template <typename R, typename T>
__device__ __forceinline__ Zc<R> row_dA(const LevelArgs<R> &L, const RowD<R> &d, int X, int Y, int Zz, long long k,
                                        const T *x) {
    Zc<R> acc = {0, 0};
    const int pos[3] = {X, Y, Zz};
    const R *ws[3] = {L.wx, L.wy, L.wz};
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!inside(L, X + dx, Y + dy, Zz + dz)) continue;
                const int dd[3] = {dx, dy, dz};
                Zc<R> cf = {0, 0};
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const int nz = (j != 0 && dx != 0) + (j != 1 && dy != 0) + (j != 2 && dz != 0);
                    const Zc<R> wj = axis_w(ws[j], pos[j], dd[j]);
                    cf.r += wj.r * d.dT[nz];
                    cf.i += wj.i * d.dT[nz];
                }
                const int sh = (dx != 0) + (dy != 0) + (dz != 0);
                cf.r -= d.dk2 * d.M[sh] + d.k2 * d.dM[sh];
                const Zc<R> xv = load<R>(x, k + dx + (long long)dy * L.sx + (long long)dz * L.sy);
                acc.r += cf.r * xv.r - cf.i * xv.i;
                acc.i += cf.r * xv.i + cf.i * xv.r;
            }
    acc.r *= L.inv_ell2;
    acc.i *= L.inv_ell2;
    return acc;
}

template <typename R, typename T>
__device__ __forceinline__ Zc<R> row_dQ(const LevelArgs<R> &L, const RowD<R> &d, int X, int Y, int Zz, long long k,
                                        const T *x) {
    Zc<R> acc = {0, 0};
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!inside(L, X + dx, Y + dy, Zz + dz)) continue;
                const R qm = d.dQ[(dx != 0) + (dy != 0) + (dz != 0)];
                const Zc<R> xv = load<R>(x, k + dx + (long long)dy * L.sx + (long long)dz * L.sy);
                acc.r += qm * xv.r;
                acc.i += qm * xv.i;
            }
    return acc;
}

// y_i = (d_i op x)_i (op A: WHICH 0, Q_h: WHICH 1) on level 0; zero on the boundary
template <typename R, typename T, int WHICH>
__global__ void __launch_bounds__(256) k_apply_dm(LevelArgs<R> L, const T *__restrict__ x, T *__restrict__ y) {
    const int X = blockIdx.x * kTX + threadIdx.x, Y = blockIdx.y * kTY + threadIdx.y, Zz = blockIdx.z;
    if (X > L.nx || Y > L.ny) return;
    const long long k = (long long)Zz * L.sy + (long long)Y * L.sx + X;
    Zc<R> v = {0, 0};
    if (inside(L, X, Y, Zz)) {
        const RowD<R> d = row_derivs(L, L.c[k]);
        v = WHICH == 0 ? row_dA(L, d, X, Y, Zz, k, x) : row_dQ(L, d, X, Y, Zz, k, x);
    }
    T o;
    o.re = (real_of<T>)v.r;
    o.im = (real_of<T>)v.i;
    y[k] = o;
}

// gacc_i += Re[ conj(s_i) (d_i Q v)_i + mu_i ((d_i Q f)_i - (d_i A v)_i) ] at interior nodes
template <typename TS>
__global__ void __launch_bounds__(256) k_grad_node(LevelArgs<double> L, const c64 *__restrict__ v,
                                                  const c64 *__restrict__ mu, const TS *__restrict__ s,
                                                  const TS *__restrict__ f, double *__restrict__ gacc) {
    const int X = blockIdx.x * kTX + threadIdx.x, Y = blockIdx.y * kTY + threadIdx.y, Zz = blockIdx.z;
    if (X > L.nx || Y > L.ny || !inside(L, X, Y, Zz)) return;
    const long long k = (long long)Zz * L.sy + (long long)Y * L.sx + X;
    const RowD<double> d = row_derivs(L, L.c[k]);
    const Zc<double> dAv = row_dA(L, d, X, Y, Zz, k, v);
    const Zc<double> dQv = row_dQ(L, d, X, Y, Zz, k, v);
    const Zc<double> dQf = row_dQ(L, d, X, Y, Zz, k, f);
    const Zc<double> si = load<double>(s, k), mi = load<double>(mu, k);
    const double tr = dQf.r - dAv.r, ti = dQf.i - dAv.i;
    gacc[k] += (si.r * dQv.r + si.i * dQv.i) + (mi.r * tr - mi.i * ti);
}

// out = in * prod_j f_j(i_j) with f the per-axis node factors 1/xi_j (inverse = 0) or xi_j
// (inverse = 1): the diagonal Xi = prod_j xi_j(i_j) of the PML node factors, which relates
// A^T to A (in one dimension the stretched second difference L = Xi^-1 K with K symmetric,
// so L^T = Xi L Xi^-1).  Xi is 1 off the PML: with in == out those nodes are not touched.
template <typename R, typename T>
__global__ void __launch_bounds__(256) k_xi_scale(Geom F, const c64 *__restrict__ fac, const T *in, T *out,
                                                 int inverse) {
    const int X = blockIdx.x * kTX + threadIdx.x, Y = blockIdx.y * kTY + threadIdx.y, Zz = blockIdx.z;
    if (X > F.n[0] || Y > F.n[1]) return;
    const long long i = (long long)Zz * F.sy + (long long)Y * F.sx + X;
    const int plane = (F.n[0] + F.n[1] + F.n[2] + 3) * inverse;   // factors: 1/xi, then xi
    const c64 a = fac[plane + X], b = fac[plane + F.n[0] + 1 + Y], c = fac[plane + F.n[0] + F.n[1] + 2 + Zz];
    const bool one = a.im == 0.0 && b.im == 0.0 && c.im == 0.0;   // gamma = 0 on all three axes
    if (one && in == out) return;
    const R ar = (R)a.re, ai = (R)a.im, br = (R)b.re, bi = (R)b.im, cr = (R)c.re, ci = (R)c.im;
    const R fr0 = ar * br - ai * bi, fi0 = ar * bi + ai * br;
    const R fr = fr0 * cr - fi0 * ci, fi = fr0 * ci + fi0 * cr;
    const T v = in[i];
    T o;
    o.re = (real_of<T>)((R)v.re * fr - (R)v.im * fi);
    o.im = (real_of<T>)((R)v.re * fi + (R)v.im * fr);
    out[i] = o;
}

// out_p = sum of gacc over the total-grid nodes whose nearest physical node is p
__global__ void __launch_bounds__(256) k_grad_phys(const double *__restrict__ gacc, Geom F, int n_pml, int nxp,
                                                  int nyp, int nzp, float *__restrict__ out) {
    const int px = blockIdx.x * kTX + threadIdx.x, py = blockIdx.y * kTY + threadIdx.y, pz = blockIdx.z;
    if (px > nxp || py > nyp || pz > nzp) return;
    auto range = [n_pml](int p, int np, int &lo, int &hi) {
        lo = p == 0 ? 0 : p + n_pml;
        hi = p == np ? np + 2 * n_pml : p + n_pml;
    };
    int x0, x1, y0, y1, z0, z1;
    range(px, nxp, x0, x1);
    range(py, nyp, y0, y1);
    range(pz, nzp, z0, z1);
    double sacc = 0.0;
    for (int z = z0; z <= z1; ++z)
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) sacc += gacc[(long long)z * F.sy + (long long)y * F.sx + x];
    out[((long long)pz * (nyp + 1) + py) * (nxp + 1) + px] = (float)sacc;
}

}  // namespace

template <typename R, typename TX, typename TG, typename TY>
hipError_t launch_apply_t(const LevelArgs<R> &L, int shifted, const TX *x, const TG *g, TY *y, hipStream_t s) {
    const dim3 grid((unsigned)((L.nx + kTX) / kTX), (unsigned)((L.ny + kTY) / kTY), (unsigned)((L.nz + kTZ) / kTZ));
    const dim3 blk(kTX, kTY);
    const size_t shm = sizeof(R) * L.nk * 20;
#define HELM_AT(SH, RS) hipLaunchKernelGGL((k_apply_t<R, TX, TG, TY, SH, RS>), grid, blk, shm, s, L, x, g, y)
    if (g) {
        if (shifted) HELM_AT(true, true); else HELM_AT(false, true);
    } else {
        if (shifted) HELM_AT(true, false); else HELM_AT(false, false);
    }
#undef HELM_AT
    return hipGetLastError();
}

template <typename R, typename TI, typename TO>
hipError_t launch_qapply_t(const LevelArgs<R> &L, const TI *w, bool conj_in, TO *y, hipStream_t s) {
    Geom gm{};
    gm.n[0] = L.nx;
    gm.n[1] = L.ny;
    gm.n[2] = L.nz;
    if (conj_in)
        hipLaunchKernelGGL((k_qapply_t<R, TI, TO, true>), node_grid3(gm), dim3(kTX, kTY), 0, s, L, w, y);
    else
        hipLaunchKernelGGL((k_qapply_t<R, TI, TO, false>), node_grid3(gm), dim3(kTX, kTY), 0, s, L, w, y);
    return hipGetLastError();
}

template <typename R, typename T>
hipError_t launch_apply_dm(const LevelArgs<R> &L, int which, const T *x, T *y, hipStream_t s) {
    Geom gm{};
    gm.n[0] = L.nx;
    gm.n[1] = L.ny;
    gm.n[2] = L.nz;
    if (which == 0)
        hipLaunchKernelGGL((k_apply_dm<R, T, 0>), node_grid3(gm), dim3(kTX, kTY), 0, s, L, x, y);
    else
        hipLaunchKernelGGL((k_apply_dm<R, T, 1>), node_grid3(gm), dim3(kTX, kTY), 0, s, L, x, y);
    return hipGetLastError();
}

template <typename TS>
hipError_t launch_grad_node(const LevelArgs<double> &L, const c64 *v, const c64 *mu, const TS *s_, const TS *f,
                            double *gacc, hipStream_t s) {
    Geom gm{};
    gm.n[0] = L.nx;
    gm.n[1] = L.ny;
    gm.n[2] = L.nz;
    hipLaunchKernelGGL((k_grad_node<TS>), node_grid3(gm), dim3(kTX, kTY), 0, s, L, v, mu, s_, f, gacc);
    return hipGetLastError();
}

// grad_c = grad_m * dm/dc = grad_m * (-2 / c^3) at the physical nodes; c from the fine-level velocity,
// whose node p + n_pml (per axis) is physical node p
__global__ void __launch_bounds__(256) k_grad_to_velocity(const float *grad_m, const float *__restrict__ vel, Geom F,
                                                         int n_pml, int nxp, int nyp, int nzp, float *grad_c) {
    const int px = blockIdx.x * kTX + threadIdx.x, py = blockIdx.y * kTY + threadIdx.y, pz = blockIdx.z;
    if (px > nxp || py > nyp || pz > nzp) return;
    const double c = vel[(long long)(pz + n_pml) * F.sy + (long long)(py + n_pml) * F.sx + px + n_pml];
    const long long p = ((long long)pz * (nyp + 1) + py) * (nxp + 1) + px;
    grad_c[p] = (float)((double)grad_m[p] * (-2.0 / (c * c * c)));
}

hipError_t launch_grad_to_velocity(const float *grad_m, const float *vel, const Geom &fine, int n_pml,
                                   const int nphys[3], float *grad_c, hipStream_t s) {
    const dim3 grid((unsigned)((nphys[0] + kTX) / kTX), (unsigned)((nphys[1] + kTY) / kTY), (unsigned)(nphys[2] + 1));
    hipLaunchKernelGGL(k_grad_to_velocity, grid, dim3(kTX, kTY), 0, s, grad_m, vel, fine, n_pml, nphys[0], nphys[1],
                       nphys[2], grad_c);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_xi_scale(const Geom &F, const c64 *fac, const T *in, T *out, bool inverse, hipStream_t s) {
    using R = real_of<T>;
    hipLaunchKernelGGL((k_xi_scale<R, T>), node_grid3(F), dim3(kTX, kTY), 0, s, F, fac, in, out, inverse ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_grad_phys(const double *gacc, const Geom &fine, int n_pml, const int nphys[3], float *out,
                            hipStream_t s) {
    const dim3 grid((unsigned)((nphys[0] + kTX) / kTX), (unsigned)((nphys[1] + kTY) / kTY), (unsigned)(nphys[2] + 1));
    hipLaunchKernelGGL(k_grad_phys, grid, dim3(kTX, kTY), 0, s, gacc, fine, n_pml, nphys[0], nphys[1], nphys[2], out);
    return hipGetLastError();
}

template hipError_t launch_apply_t<float, c32, c32, c32>(const LevelArgs<float> &, int, const c32 *, const c32 *,
                                                         c32 *, hipStream_t);
template hipError_t launch_apply_t<double, c64, c64, c64>(const LevelArgs<double> &, int, const c64 *, const c64 *,
                                                          c64 *, hipStream_t);
template hipError_t launch_qapply_t<double, c32, c64>(const LevelArgs<double> &, const c32 *, bool, c64 *,
                                                      hipStream_t);
template hipError_t launch_qapply_t<double, c64, c64>(const LevelArgs<double> &, const c64 *, bool, c64 *,
                                                      hipStream_t);
template hipError_t launch_qapply_t<float, c32, c32>(const LevelArgs<float> &, const c32 *, bool, c32 *, hipStream_t);
template hipError_t launch_apply_dm<float, c32>(const LevelArgs<float> &, int, const c32 *, c32 *, hipStream_t);
template hipError_t launch_apply_dm<double, c64>(const LevelArgs<double> &, int, const c64 *, c64 *, hipStream_t);
template hipError_t launch_xi_scale<c32>(const Geom &, const c64 *, const c32 *, c32 *, bool, hipStream_t);
template hipError_t launch_xi_scale<c64>(const Geom &, const c64 *, const c64 *, c64 *, bool, hipStream_t);
template hipError_t launch_grad_node<c32>(const LevelArgs<double> &, const c64 *, const c64 *, const c32 *,
                                          const c32 *, double *, hipStream_t);
template hipError_t launch_grad_node<c64>(const LevelArgs<double> &, const c64 *, const c64 *, const c64 *,
                                          const c64 *, double *, hipStream_t);

}  // namespace helm
