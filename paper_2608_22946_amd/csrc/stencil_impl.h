// Implementation of the stencil kernels and their launcher templates, included by the
// translation units that instantiate them (stencil.hip: FP32 / FP64 operands;
// stencil_mixed.hip: the FP16-stored operands of the mixed-precision cycle).
// Matrix-free 27-point IOFD level operator and its fused variants.
//
// Row i of H_mu = L - mu M (mu = 1 for A_l, 1 + i sigma for B_l; Sec. 2.2 and
// eq. shifted-iofd-levels) is, with a = alpha(eta*_i), kappa_i = omega ell / c_i:
//   ell^2 (H v)_i = sum_j sum_d w_j(i_j, d_j) T(d_perp) v_{i+d} - mu kappa_i^2 sum_d Mw(|d|_1) v_{i+d}
// with the stretched second-difference weights w_j (eq. pml-second-difference),
// transverse weights T = a4, a5/4, (1-a4-a5)/4 and mass weights
// Mw = a1, a2/6, a3/12, (1-a1-a2-a3)/8.  Where no stretching is present the row
// collapses to the shell form (eq. iofd-shell-form, eq. iofd-shell-coefficients).
//
// Work decomposition (CDNA wave64): one wavefront covers 64 consecutive x nodes
// of one y row; lanes 1..62 produce outputs, lanes 0 and 63 only supply the x
// halo.  x neighbours come from DPP wave shifts (no LDS), the y neighbours are
// the rows y-1 and y+1 loaded by the same lane, and the wave marches in z over a
// chunk of planes keeping per-plane partial sums in registers, so each input
// value is fetched from HBM once (plus L2-resident halo re-reads).  Workgroups
// of 4 waves cover 4 adjacent rows; the block index is remapped so that each of
// the 8 XCDs walks a contiguous range of tiles and shares halos in its own L2.
// Per-node coefficients are evaluated on the fly from the velocity: one
// reciprocal, the clamped interpolation coordinate and five cubic polynomials
// read from an LDS copy of the table, so the only per-node data read besides
// the operand is the FP32 velocity.
#pragma once

#include <algorithm>

#include "helm_internal.h"

namespace helm {
namespace {

template <typename R>
struct Z {
    R r, i;
};

template <typename R>
__device__ __forceinline__ Z<R> zadd(Z<R> a, Z<R> b) { return {a.r + b.r, a.i + b.i}; }
template <typename R>
__device__ __forceinline__ Z<R> zsub(Z<R> a, Z<R> b) { return {a.r - b.r, a.i - b.i}; }
template <typename R>
__device__ __forceinline__ Z<R> zscale(R s, Z<R> a) { return {s * a.r, s * a.i}; }
template <typename R>
__device__ __forceinline__ Z<R> zmul(Z<R> a, Z<R> b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
template <typename R>
__device__ __forceinline__ Z<R> zfma(Z<R> a, Z<R> b, Z<R> acc) {  // acc + a*b
    return {acc.r + a.r * b.r - a.i * b.i, acc.i + a.r * b.i + a.i * b.r};
}
template <typename R>
__device__ __forceinline__ Z<R> zdiv(Z<R> a, Z<R> d) {
    R inv = R(1) / (d.r * d.r + d.i * d.i);
    return {(a.r * d.r + a.i * d.i) * inv, (a.i * d.r - a.r * d.i) * inv};
}

// value from the lane holding x-1 (wave_shr:1) and from the lane holding x+1 (wave_shl:1)
__device__ __forceinline__ float from_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double from_left(double v) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x138, 0xf, 0xf, false);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double from_right(double v) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x130, 0xf, 0xf, false);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <typename R>
__device__ __forceinline__ Z<R> zleft(Z<R> v) { return {from_left(v.r), from_left(v.i)}; }
template <typename R>
__device__ __forceinline__ Z<R> zright(Z<R> v) { return {from_right(v.r), from_right(v.i)}; }

template <typename R, typename T>
__device__ __forceinline__ Z<R> ld(const T *p, long long i) {
    T v = p[i];
    return {(R)v.re, (R)v.im};
}

// FP16-stored operands (c16): true value = stored value / (f qs), see helm_internal.h
template <typename R, typename T>
__device__ __forceinline__ Z<R> dq(T v, R inv) {
    Z<R> o = {(R)v.re, (R)v.im};
    if (is_half<T>()) {
        o.r *= inv;
        o.i *= inv;
    }
    return o;
}
template <typename T, typename R>
__device__ __forceinline__ T qz(Z<R> v, R s) { return to_stored<T, R>(v.r, v.i, s); }
struct Scales {
    Scale x, g, b, y;
};

__device__ __forceinline__ float recip(float c) { return __builtin_amdgcn_rcpf(c); }
__device__ __forceinline__ double recip(double c) { return 1.0 / c; }

// Interpolation coordinate and the five coefficient functions at a node
// (eq. iofd-clamped-coordinate); the table holds, per interval, the monomial
// coefficients of the cubic Hermite interpolant in the local variable t.
template <typename R>
struct Coef {
    R a1, a2, a3, a4, a5, k2;
};

template <typename R>
__device__ __forceinline__ void locate(const LevelArgs<R> &L, float c, R &kappa, int &k, R &t) {
    kappa = L.omega_ell * recip((R)c);
    R eta = kappa * (R)0.15915494309189533577;   // 1 / (2 pi)
    eta = eta < (R)0.4 ? eta : (R)0.4;
    R u = eta * L.inv_deta;
    k = (int)u;
    k = k < L.K - 1 ? k : L.K - 1;
    k = k > 0 ? k : 0;
    t = u - (R)k;
}

template <typename R>
__device__ __forceinline__ R horner(const R *p, R t) { return ((p[3] * t + p[2]) * t + p[1]) * t + p[0]; }
template <typename R>
__device__ __forceinline__ R horner5(const R *p, R t) {
    return ((((p[5] * t + p[4]) * t + p[3]) * t + p[2]) * t + p[1]) * t + p[0];
}

// FP32 levels read the scaled coordinate s = omega ell K / (0.4 * 2 pi c) per node instead of
// c (LevelArgs::s): the same interval and local coordinate as `locate`, and kappa = s kap_s.
template <typename R>
constexpr bool scaled_coordinate() { return sizeof(R) == sizeof(float); }

template <typename R>
__device__ __forceinline__ void locate_s(const LevelArgs<R> &L, float s, R &kappa, int &k, R &t) {
    kappa = (R)s * L.kap_s;
    const R u = (R)s < (R)L.K ? (R)s : (R)L.K;   // eta* clamped at 0.4
    k = (int)u;
    k = k < L.K - 1 ? k : L.K - 1;
    t = u - (R)k;
}

// the five coefficient functions and kappa^2 at a node; v is the per-node value the level
// stores (s on FP32 levels, the velocity c on FP64 ones)
template <typename R>
__device__ __forceinline__ Coef<R> coef_at(const LevelArgs<R> &L, const R *stab, float v) {
    R kappa, t;
    int k;
    if (scaled_coordinate<R>())
        locate_s(L, v, kappa, k, t);
    else
        locate(L, v, kappa, k, t);
    // stab holds the intervals kb .. kb + nk - 1 (the level's window)
    k = k < L.kb ? L.kb : (k > L.kb + L.nk - 1 ? L.kb + L.nk - 1 : k);
    const R *p = stab + (k - L.kb) * 20;
    Coef<R> o;
    o.a1 = horner(p + 0, t);
    o.a2 = horner(p + 4, t);
    o.a3 = horner(p + 8, t);
    o.a4 = horner(p + 12, t);
    o.a5 = horner(p + 16, t);
    o.k2 = kappa * kappa;
    return o;
}

// unshifted shell coefficients C_0..C_3 at a node of an FP32 level from the quintic table
// (LDS copy `ctab`): interval min(floor(s), K), the last one unbounded in t
template <typename R>
__device__ __forceinline__ void shell_at_s(const LevelArgs<R> &L, const R *ctab, float s, R &c0, R &c1, R &c2,
                                           R &c3) {
    int k = (int)s;
    k = k < L.K ? k : L.K;
    const R t = (R)s - (R)k;
    // ctab holds the intervals cb .. cb + nck - 1 (the level's window)
    const int kw = k < L.cb ? L.cb : (k > L.cb + L.nck - 1 ? L.cb + L.nck - 1 : k);
    const R *p = ctab + (kw - L.cb) * 24;
    c0 = horner5(p, t);
    c1 = horner5(p + 6, t);
    c2 = horner5(p + 12, t);
    c3 = horner5(p + 18, t);
}

// per-node value a level's coefficient evaluation reads
template <typename R>
__device__ __forceinline__ const float *node_values(const LevelArgs<R> &L) {
    return scaled_coordinate<R>() ? L.s : L.c;
}

// diagonal entry ell^2 D = a4 (wxc + wyc + wzc) - mu kappa^2 a1
template <typename R, bool SHIFT>
__device__ __forceinline__ Z<R> diag_of(const LevelArgs<R> &L, R a1, R a4, R k2, Z<R> wsum) {
    Z<R> d = zscale(a4, wsum);
    d.r -= k2 * a1;
    if (SHIFT) d.i -= L.sigma * k2 * a1;
    return zscale(L.inv_ell2, d);
}

template <typename R>
struct Plane {
    Z<R> p0, p1, p2;   // centre, 4 in-plane face neighbours, 4 in-plane corners
    Z<R> ea, eb;       // x/y stiffness partials (tensor form only)
    Z<R> gc;           // right-hand side at the centre (residual / Jacobi modes)
    Z<R> dc;           // D^-1 at the centre (Jacobi modes)
    Z<R> bc;           // base value at the centre (fused Jacobi + base)
    float cc;          // per-node value at the centre (s on FP32 levels, c on FP64 ones)
};

// In-plane partial sums of one z plane from the rows y-1 (a), y (b), y+1 (c)
// at this lane's x; x neighbours come from the adjacent lanes.  XI / YI: the
// x / y stretching of this wave is the identity (weights -1, 2, -1).
template <typename R, bool XI, bool YI>
__device__ __forceinline__ void plane_partials(Z<R> a, Z<R> b, Z<R> c, const Z<R> *wx, const Z<R> *wy,
                                               Plane<R> &P) {
    const Z<R> col = zadd(a, c);
    const Z<R> bL = zleft(b), bR = zright(b);
    P.p0 = b;
    if (XI && YI) {
        P.p1 = zadd(col, zadd(bL, bR));
        P.p2 = zadd(zleft(col), zright(col));
        return;
    }
    const Z<R> aL = zleft(a), aR = zright(a), cL = zleft(c), cR = zright(c);
    const Z<R> colL = zadd(aL, cL), colR = zadd(aR, cR);
    const Z<R> rsm = zadd(aL, aR), rs0 = zadd(bL, bR), rsp = zadd(cL, cR);
    P.p1 = zadd(col, rs0);
    P.p2 = zadd(rsm, rsp);
    Z<R> ea, eb;
    if (XI) {            // -1, 2, -1 along x
        ea = zsub(zscale((R)2, b), rs0);
        eb = zsub(zscale((R)2, col), zadd(colL, colR));
    } else {
        ea = zmul(wx[0], bL);
        ea = zfma(wx[1], b, ea);
        ea = zfma(wx[2], bR, ea);
        eb = zmul(wx[0], colL);
        eb = zfma(wx[1], col, eb);
        eb = zfma(wx[2], colR, eb);
    }
    if (YI) {            // -1, 2, -1 along y
        ea = zadd(ea, zsub(zscale((R)2, b), col));
        eb = zadd(eb, zsub(zscale((R)2, rs0), zadd(rsm, rsp)));
    } else {
        ea = zfma(wy[0], a, ea);
        ea = zfma(wy[1], b, ea);
        ea = zfma(wy[2], c, ea);
        eb = zfma(wy[0], rsm, eb);
        eb = zfma(wy[1], rs0, eb);
        eb = zfma(wy[2], rsp, eb);
    }
    P.ea = ea;
    P.eb = eb;
}

// H v at the centre of plane "o" from planes m (z-1), o (z), p (z+1); the row's coefficients
// come from the per-node value o.cc (s or c).  Unshifted rows of an FP32 level free of
// stretching take the shell coefficients from the quintic table (one Horner per
// coefficient); every other row evaluates alpha_1..alpha_5 (eq. iofd-shell-coefficients,
// or the tensor-product form in the PML).
template <typename R, bool XYI, bool SHIFT>
__device__ __forceinline__ Z<R> row_value(const LevelArgs<R> &L, const R *stab, const R *ctab, const Plane<R> &m,
                                          const Plane<R> &o, const Plane<R> &p, bool zint, const Z<R> *wz) {
    // shell sums S_m over the 1 / 6 / 12 / 8 neighbours
    const Z<R> S0 = o.p0;
    const Z<R> S1 = zadd(o.p1, zadd(m.p0, p.p0));
    const Z<R> S2 = zadd(o.p2, zadd(m.p1, p.p1));
    const Z<R> S3 = zadd(m.p2, p.p2);
    if (scaled_coordinate<R>() && !SHIFT && XYI && zint) {
        R c0, c1, c2, c3;
        shell_at_s(L, ctab, o.cc, c0, c1, c2, c3);
        Z<R> out;
        out.r = c0 * S0.r + c1 * S1.r + c2 * S2.r + c3 * S3.r;
        out.i = c0 * S0.i + c1 * S1.i + c2 * S2.i + c3 * S3.i;
        return zscale(L.inv_ell2, out);
    }
    const Coef<R> cf = coef_at(L, stab, o.cc);
    const R a1 = cf.a1, a2 = cf.a2, a3 = cf.a3, a4 = cf.a4, a5 = cf.a5;
    const R q = (R)1 - a4 - a5;
    const R m0 = a1, m1 = a2 * (R)(1.0 / 6), m2 = a3 * (R)(1.0 / 12), m3 = ((R)1 - a1 - a2 - a3) * (R)0.125;
    if (XYI && zint) {
        // eq. iofd-shell-coefficients: C_m = stiffness_m - mu kappa^2 mass_m, then sum_m C_m S_m
        const R k2 = cf.k2;
        const R c0 = (R)6 * a4 - k2 * m0, c1 = (a5 - a4) - k2 * m1, c2 = (R)0.5 * (q - a5) - k2 * m2,
                c3 = (R)-0.75 * q - k2 * m3;
        Z<R> out;
        out.r = c0 * S0.r + c1 * S1.r + c2 * S2.r + c3 * S3.r;
        out.i = c0 * S0.i + c1 * S1.i + c2 * S2.i + c3 * S3.i;
        if (SHIFT) {   // - i sigma kappa^2 sum_m mass_m S_m
            const R sk = L.sigma * k2;
            const R mr = m0 * S0.r + m1 * S1.r + m2 * S2.r + m3 * S3.r;
            const R mi = m0 * S0.i + m1 * S1.i + m2 * S2.i + m3 * S3.i;
            out.r += sk * mi;
            out.i -= sk * mr;
        }
        return zscale(L.inv_ell2, out);
    }
    Z<R> Mass = zscale(m0, S0);
    Mass = zadd(Mass, zscale(m1, S1));
    Mass = zadd(Mass, zscale(m2, S2));
    Mass = zadd(Mass, zscale(m3, S3));
    Z<R> St;
    {
        const R t0 = a4, t1 = a5 * (R)0.25, t2 = q * (R)0.25;
        Z<R> eam, ebm, eao, ebo, eap, ebp;
        if (XYI) {   // unit x/y stretching: Ea = 4 P0 - P1, Eb = 2 P1 - 2 P2
            eam = zsub(zscale((R)4, m.p0), m.p1);
            ebm = zscale((R)2, zsub(m.p1, m.p2));
            eao = zsub(zscale((R)4, o.p0), o.p1);
            ebo = zscale((R)2, zsub(o.p1, o.p2));
            eap = zsub(zscale((R)4, p.p0), p.p1);
            ebp = zscale((R)2, zsub(p.p1, p.p2));
        } else {
            eam = m.ea; ebm = m.eb; eao = o.ea; ebo = o.eb; eap = p.ea; ebp = p.eb;
        }
        St = zscale(t0, eao);
        St = zadd(St, zscale(t1, zadd(ebo, zadd(eam, eap))));
        St = zadd(St, zscale(t2, zadd(ebm, ebp)));
        // z-direction second difference with transverse weights
        Z<R> z0, z1, z2;
        if (zint) {   // unit z stretching: -1, 2, -1
            z0 = zsub(zscale((R)2, o.p0), zadd(m.p0, p.p0));
            z1 = zsub(zscale((R)2, o.p1), zadd(m.p1, p.p1));
            z2 = zsub(zscale((R)2, o.p2), zadd(m.p2, p.p2));
        } else {
            z0 = zmul(wz[1], o.p0);
            z0 = zfma(wz[0], m.p0, z0);
            z0 = zfma(wz[2], p.p0, z0);
            z1 = zmul(wz[1], o.p1);
            z1 = zfma(wz[0], m.p1, z1);
            z1 = zfma(wz[2], p.p1, z1);
            z2 = zmul(wz[1], o.p2);
            z2 = zfma(wz[0], m.p2, z2);
            z2 = zfma(wz[2], p.p2, z2);
        }
        St = zadd(St, zscale(t0, z0));
        St = zadd(St, zscale(t1, z1));
        St = zadd(St, zscale(t2, z2));
    }
    Z<R> out;
    out.r = St.r - cf.k2 * Mass.r;
    out.i = St.i - cf.k2 * Mass.i;
    if (SHIFT) {   // - i sigma kappa^2 Mass
        out.r += L.sigma * cf.k2 * Mass.i;
        out.i -= L.sigma * cf.k2 * Mass.r;
    }
    return zscale(L.inv_ell2, out);
}

__device__ __forceinline__ void block_reduce_store(double v, double *dst) {
    // wavefront sum (DPP), then across the workgroup's waves through LDS
    v = wave_sum_f64(v);
    __shared__ double red[kWavesY];
    int w = threadIdx.y, l = threadIdx.x;
    if (l == 0) red[w] = v;
    __syncthreads();
    if (w == 0 && l == 0) {
        double s = 0;
        for (int i = 0; i < kWavesY; ++i) s += red[i];
        partial_store(dst, s);
        stores_done();
    }
}

// Last-block epilogue of a stencil with fused ||y||^2: beta, state reset.
__device__ void norm_epilogue(const RedBuf &rb, int nblocks, KState *st) {
    constexpr int nt = 64 * kWavesY;   // threads of a stencil workgroup
    static_assert((nt & (nt - 1)) == 0, "the tree sum needs a power-of-two workgroup");
    __shared__ bool last;
    __shared__ double red[nt];
    const int tid = threadIdx.x + 64 * threadIdx.y;
    if (tid == 0) last = take_ticket(rb.counter, nblocks);
    __syncthreads();
    if (!last) return;
    double s = 0;
#pragma unroll 8
    for (int b = tid; b < nblocks; b += nt) s += partial_load(rb.partials + b);
    red[tid] = s;
    __syncthreads();
    for (int off = nt / 2; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
    }
    if (tid == 0) {
        double beta = sqrt(red[0]);
        st->beta = beta;
        st->scale = (beta > 0.0) ? 1.0 / beta : 0.0;
        st->vs0 = st->scale;
        st->kk = 0;
        st->breakdown = 0;
        st->nonfinite = !(beta == beta && beta < 1e300);
        for (int j = 0; j <= kMMax; ++j) st->g[j][0] = st->g[j][1] = 0.0;
        st->g[0][0] = beta;
        reset_ticket(rb.counter);
    }
}

// Stencil outputs are stored with the non-temporal hint: the fine-level apply at 352^3 ran
// 3% faster (0.279 -> 0.271 ms) with the solve unchanged.  Choosing the hint per level at
// run time made every stencil slower (code generation of the march), so it is unconditional.
__device__ __forceinline__ void st_nt(c32 *p, c32 v) {
    const long long b = ((long long)__float_as_int(v.im) << 32) | (unsigned)__float_as_int(v.re);
    __builtin_nontemporal_store(b, reinterpret_cast<long long *>(p));
}
__device__ __forceinline__ void st_nt(c64 *p, c64 v) {
    __builtin_nontemporal_store(v.re, &p->re);
    __builtin_nontemporal_store(v.im, &p->im);
}
__device__ __forceinline__ void st_nt(c16 *p, c16 v) {
    const unsigned b = (unsigned)__builtin_bit_cast(unsigned short, v.re) |
                       ((unsigned)__builtin_bit_cast(unsigned short, v.im) << 16);
    __builtin_nontemporal_store(b, reinterpret_cast<unsigned *>(p));
}

template <typename T>
__device__ __forceinline__ const T *plane_ptr(const T *base, long long plane_stride, int z) {
    return base + (long long)z * plane_stride;
}
template <typename T>
__device__ __forceinline__ T at_byte(const T *plane, unsigned off) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(plane) + off);
}

// One wavefront: rows y-1, y, y+1 at 64 consecutive x, marching planes z0..z1-1.
// Every load reads an in-bounds node (indices clamped to the grid) and
// boundary / out-of-box values are masked to zero afterwards, so the loads
// carry no branches; the per-lane byte offsets inside a plane are fixed and the
// plane base is wave-uniform (scalar registers).
template <typename R, typename TX, typename TG, typename TY, int MODE, bool SHIFT, bool NORM, bool XI, bool YI>
__device__ __forceinline__ void march(const LevelArgs<R> &L, const R *stab, const TX *__restrict__ x,
                                      const TG *__restrict__ g, const TY *__restrict__ base, TY *__restrict__ y,
                                      R omegaJ, const R (&mul)[4], int xg, int yg, int z0, int z1, bool out_lane,
                                      double &nrm, int Z0 = 0) {
    // mul: multipliers of the c16 operands (x, g, base loads; y store), 1 for the others
    const R mx = mul[0], mg = mul[1], mb = mul[2], my = mul[3];
    constexpr bool JAC = (MODE == M_JAC2 || MODE == M_JAC2_ADD);
    constexpr bool RESTRICT = (MODE == M_RESID_R);
    constexpr bool NEED_G = (MODE != M_APPLY);
    const bool x_int = (xg >= 1 && xg <= L.nx - 1);
    const int xc = min(max(xg, 0), L.nx);
    const int ym = max(yg - 1, 0), yp = min(yg + 1, L.ny);
    const unsigned e0 = (unsigned)(yg * (int)L.sx + xc), em = (unsigned)(ym * (int)L.sx + xc),
                   ep = (unsigned)(yp * (int)L.sx + xc);
    const unsigned bx0 = e0 * sizeof(TX), bxm = em * sizeof(TX), bxp = ep * sizeof(TX);
    const unsigned bg0 = e0 * sizeof(TG), bgm = em * sizeof(TG), bgp = ep * sizeof(TG);
    const unsigned bc0 = e0 * 4u;
    const bool rm_ok = x_int && (yg - 1 >= 1);
    const bool r0_ok = x_int && (yg >= 1) && (yg <= L.ny - 1);
    const bool rp_ok = x_int && (yg + 1 <= L.ny - 1);

    Z<R> wx[3] = {{0, 0}, {0, 0}, {0, 0}}, wy[3] = {{0, 0}, {0, 0}, {0, 0}};
    {
        const R *w = L.wx + 6 * xc;
        wx[0] = {w[0], w[1]}; wx[1] = {w[2], w[3]}; wx[2] = {w[4], w[5]};
        const R *v = L.wy + 6 * yg;
        wy[0] = {v[0], v[1]}; wy[1] = {v[2], v[3]}; wy[2] = {v[4], v[5]};
    }
    const Z<R> zero = {0, 0};

    // Raw loads of one plane (issued one plane ahead of their use).
    using DT = cplx<R>;
    struct Raw {
        TX va, vb, vc;     // operand rows (or the right-hand side rows in the Jacobi modes)
        TG gb;             // right-hand side at the centre
        DT da, db, dc;     // D^-1 rows (Jacobi modes; db alone in the sweep mode)
        TY bb;             // base at the centre (fused Jacobi + base)
        float cb;          // velocity at the centre
        int zp;
    };
    constexpr bool SWEEP = (MODE == M_JSWEEP);
    const DT *dinv = reinterpret_cast<const DT *>(L.dinv[SHIFT ? 1 : 0]);
    const unsigned bd0 = e0 * (unsigned)sizeof(DT), bdm = em * (unsigned)sizeof(DT), bdp = ep * (unsigned)sizeof(DT);
    // Planes past the tile's last plane z1 are re-read from z1 (a cache hit):
    // the prefetch is then issued unconditionally, which keeps the count of
    // outstanding loads the same on every path through the loop, so waiting
    // for one plane never waits for the planes issued after it.
    const int zlast = min(z1, L.nz);
    const float *vnode = node_values(L);
    auto issue = [&](int zp, Raw &r) {
        const int zc = min(max(zp, 0), zlast);
        r.zp = zp;
        const float *cp = plane_ptr(vnode, L.sy, zc);
        r.cb = at_byte(cp, bc0);
        if constexpr (!JAC) {
            const TX *xp = plane_ptr(x, L.sy, zc);
            r.va = at_byte(xp, bxm);
            r.vb = at_byte(xp, bx0);
            r.vc = at_byte(xp, bxp);
            if (NEED_G) r.gb = at_byte(plane_ptr(g, L.sy, zc), bg0);
            if (SWEEP) r.db = at_byte(plane_ptr(dinv, L.sy, zc), bd0);
        } else {
            const TG *gp = plane_ptr(g, L.sy, zc);
            r.va = at_byte(gp, bgm);
            r.vb = at_byte(gp, bg0);
            r.vc = at_byte(gp, bgp);
            const DT *dp = plane_ptr(dinv, L.sy, zc);
            r.da = at_byte(dp, bdm);
            r.db = at_byte(dp, bd0);
            r.dc = at_byte(dp, bdp);
            if (MODE == M_JAC2_ADD) r.bb = at_byte(plane_ptr(base, L.sy, zc), e0 * (unsigned)sizeof(TY));
        }
    };
    // mask boundary / out-of-box values and form the plane partials
    auto finish = [&](const Raw &r, Plane<R> &P) {
        const int zp = r.zp;
        const bool zok = (zp >= 1 && zp <= L.nz - 1);
        Z<R> a, b, c;
        Z<R> gc = zero;
        if constexpr (!JAC) {
            a = dq<R>(r.va, mx);
            b = dq<R>(r.vb, mx);
            c = dq<R>(r.vc, mx);
            if (NEED_G) gc = dq<R>(r.gb, mg);
        } else {
            a = dq<R>(r.va, mg);   // the loaded rows are g
            b = dq<R>(r.vb, mg);
            c = dq<R>(r.vc, mg);
            // fused two-sweep Jacobi: the operand is y1 = omega D^-1 g at every loaded node
            gc = b;
            a = zscale(omegaJ, zmul(Z<R>{r.da.re, r.da.im}, a));
            b = zscale(omegaJ, zmul(Z<R>{r.db.re, r.db.im}, b));
            c = zscale(omegaJ, zmul(Z<R>{r.dc.re, r.dc.im}, c));
        }
        if (!(zok && rm_ok)) a = zero;
        if (!(zok && r0_ok)) b = zero;
        if (!(zok && rp_ok)) c = zero;
        P.cc = r.cb;
        P.gc = gc;
        if (JAC || SWEEP) P.dc = Z<R>{r.db.re, r.db.im};
        if (MODE == M_JAC2_ADD) P.bc = dq<R>(r.bb, mb);
        plane_partials<R, XI, YI>(a, b, c, wx, wy, P);
    };

    const bool yint = (yg >= 1 && yg <= L.ny - 1);
    // M_RESID_R: x/z-restricted residual rows w[coarse z][fine y][coarse x]
    const int nxc = L.nx >> 1, nzc = L.nz >> 1;
    const long long wsx = nxc + 1, wsy = (long long)(L.ny + 1) * wsx;
    const int lane = threadIdx.x;
    const bool rstore = RESTRICT && (lane & 1) && lane >= 3 && lane <= 61 && yint && (xg >> 1) >= 1 && (xg >> 1) <= nxc - 1;
    Z<R> rcur = zero;
    // output plane z from planes m, o, p
    auto emit = [&](int z, const Plane<R> &m, const Plane<R> &o, const Plane<R> &p) {
        Z<R> res = zero;
        const bool interior = x_int && yint && z >= 1 && z <= L.nz - 1;
        if (interior) {
            const bool zint = (z >= L.loz && z <= L.hiz);
            const R *wzp = L.wz + 6 * z;
            const Z<R> wz[3] = {{wzp[0], wzp[1]}, {wzp[2], wzp[3]}, {wzp[4], wzp[5]}};
            const Z<R> Hv = row_value<R, XI && YI, SHIFT>(L, stab, stab + 20 * L.nk, m, o, p, zint, wz);
            if (MODE == M_APPLY) {
                res = Hv;
            } else if (MODE == M_RESID || RESTRICT) {
                res = zsub(o.gc, Hv);
            } else {
                res = zadd(o.p0, zscale(omegaJ, zmul(o.dc, zsub(o.gc, Hv))));   // p0: operand / y1
            }
        }
        if (RESTRICT) {
            // full weighting along x (this lane's fine x is even on the storing
            // lanes) and along z (running sums over the coarse planes), stored per
            // fine row; the y weights follow in a second pass
            const Z<R> rl = zleft(res), rr = zright(res);
            const Z<R> rx = {(R)0.25 * (rl.r + rr.r) + (R)0.5 * res.r, (R)0.25 * (rl.i + rr.i) + (R)0.5 * res.i};
            if (z & 1) {   // odd fine plane: completes coarse plane (z-1)/2, starts (z+1)/2
                rcur.r += (R)0.25 * rx.r;
                rcur.i += (R)0.25 * rx.i;
                const int Zc = (z - 1) >> 1;
                if (rstore && z >= 2 * Z0 + 1 && Zc >= 1 && Zc <= nzc - 1)
                    y[(long long)Zc * wsy + (long long)yg * wsx + (xg >> 1)] = qz<TY>(rcur, my);
                rcur = {(R)0.25 * rx.r, (R)0.25 * rx.i};
            } else {
                rcur.r += (R)0.5 * rx.r;
                rcur.i += (R)0.5 * rx.i;
            }
            return;
        }
        TY *yp_ = const_cast<TY *>(plane_ptr(y, L.sy, z));
        if (MODE == M_JAC2_ADD) {
            res.r += o.bc.r;
            res.i += o.bc.i;
        }
        if (out_lane) {
            st_nt(reinterpret_cast<TY *>(reinterpret_cast<char *>(yp_) + e0 * (unsigned)sizeof(TY)), qz<TY>(res, my));
            if (NORM) nrm += (double)res.r * (double)res.r + (double)res.i * (double)res.i;
        }
    };

    // Two planes of loads stay in flight: a step issues plane z+3, forms the
    // output of plane z, then turns the already-arrived plane z+2 into partial
    // sums.  Plane slots rotate with period 3 and load buffers with period 2.
    Plane<R> P0, P1, P2;
    Raw ra, rb;
    issue(z0 - 1, ra);
    issue(z0, rb);
    finish(ra, P0);
    issue(z0 + 1, ra);
    finish(rb, P1);
    issue(z0 + 2, rb);
    finish(ra, P2);
    auto step = [&](int z, const Plane<R> &m, const Plane<R> &o, const Plane<R> &p, Plane<R> &slot,
                    const Raw &arrived, Raw &next) -> bool {
        issue(z + 3, next);
        emit(z, m, o, p);
        if (z + 1 >= z1) return false;
        finish(arrived, slot);   // slot (held plane z-1) now holds plane z+2
        return true;
    };
    for (int z = z0;; z += 6) {
        if (!step(z, P0, P1, P2, P0, rb, ra)) break;
        if (!step(z + 1, P1, P2, P0, P1, ra, rb)) break;
        if (!step(z + 2, P2, P0, P1, P2, rb, ra)) break;
        if (!step(z + 3, P0, P1, P2, P0, ra, rb)) break;
        if (!step(z + 4, P1, P2, P0, P1, rb, ra)) break;
        if (!step(z + 5, P2, P0, P1, P2, ra, rb)) break;
    }
}

// Edge strips of kEdge output columns each (x = 0..29 and nx-29..nx) share one
// wavefront when both x-PML strips fit inside them.
constexpr int kEdge = 30;

template <typename R>
__host__ __device__ __forceinline__ bool split_edges(const LevelArgs<R> &L) {
    return L.nx >= 2 * kEdge && L.lox >= 1 && L.lox <= kEdge && L.hix >= L.nx - kEdge;
}

template <typename R>
int x_tiles(const LevelArgs<R> &L) {
    return split_edges(L) ? 1 + ceil_div(L.nx - 2 * kEdge + 1, kTileX) : ceil_div(L.nx + 1, kTileX);
}

// Grid of one stencil launch.  PART 0 covers every tile.  With split edges the
// tiles divide into an interior set (x tiles 1.. and y tiles whose four rows
// all lie between the y-PML strips, PART 1), which needs no x/y stretching
// and so compiles to fewer registers, and the remaining border set (PART 2).
// The two parts are launched back to back; a fused norm spans both through
// block_offset / total_blocks.
struct TileMap {
    int ntx, nty, tz;
    int yt_lo, nyi;        // interior y tiles: yt_lo .. yt_lo + nyi - 1
    int block_offset;      // index of this launch's first block among all blocks of the call
    int total_blocks;      // blocks over all launches of the call
};

template <typename R, typename TX, typename TG, typename TY, int MODE, bool SHIFT, bool NORM, int PART>
__global__ void __launch_bounds__(64 * kWavesY) k_stencil(LevelArgs<R> L, const TX *__restrict__ x, const TG *__restrict__ g,
                                                 const TY *__restrict__ base, TY *__restrict__ y, R omegaJ, TileMap M,
                                                 RedBuf rb, KState *st, Scales sc, Batch bt) {
    // XCD-aware order of (tile, slot) pairs: block b runs on XCD b % 8; each XCD takes a
    // contiguous range of u = tile * slots + slot, so the slots of one tile run back to
    // back on one XCD and share the tile's per-node values and D^-1 through its L2.
    const int nb = gridDim.x, b = blockIdx.x;
    const int per = nb / 8, rem = nb % 8, xcd = b % 8, idx = b / 8;
    const int u = (xcd < rem) ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
    const int sl = u % bt.n;   // batched right-hand side: its own vectors, state and partials
    int t = u / bt.n;
    const int tile = t;
    if (slot_off(bt, sl)) return;
    {
        const long long nn = (long long)(L.nz + 1) * L.sy;
        x = slot_ptr(x, nn, sl);
        g = slot_ptr(g, nn, sl);
        base = slot_ptr(base, nn, sl);
        // M_RESID_R writes the x/z-restricted rows [coarse z][fine y][coarse x]
        y = slot_ptr(y, MODE == M_RESID_R ? (long long)((L.nz >> 1) + 1) * (L.ny + 1) * ((L.nx >> 1) + 1) : nn, sl);
        st = slot_ptr(st, 1, sl);
        rb = slot_rb(rb, bt, sl);
        sc.x = slot_scale(sc.x, sl);
        sc.g = slot_scale(sc.g, sl);
        sc.b = slot_scale(sc.b, sl);
        sc.y = slot_scale(sc.y, sl);
    }
    const R mul[4] = {load_mul<R, TX>(sc.x), load_mul<R, TG>(sc.g), load_mul<R, TY>(sc.b), store_mul<R, TY>(sc.y)};
    extern __shared__ unsigned char smem_raw[];
    R *stab = reinterpret_cast<R *>(smem_raw);   // alpha pieces, then (FP32) the shell quintics
    const int tid = threadIdx.x + 64 * threadIdx.y;
    // the level's window of table intervals only (at 4h almost every node is in the clamped one)
    for (int i = tid; i < L.nk * 20; i += 64 * kWavesY) stab[i] = L.atab[L.kb * 20 + i];
    if (scaled_coordinate<R>())
        for (int i = tid; i < L.nck * 24; i += 64 * kWavesY) stab[L.nk * 20 + i] = L.ctab[L.cb * 24 + i];
    __syncthreads();

    const int ntx = M.ntx, nty = M.nty;
    int xt, yt, zc;
    if (PART == 0) {
        xt = t % ntx;
        t /= ntx;
        yt = t % nty;
        zc = t / nty;
    } else if (PART == 1) {
        const int nxi = ntx - 1;
        xt = 1 + t % nxi;
        t /= nxi;
        yt = M.yt_lo + t % M.nyi;
        zc = t / M.nyi;
    } else {
        // per z chunk: the edge x tile of every y tile, then the inner x tiles of the y tiles outside the interior
        const int per_z = nty + (nty - M.nyi) * (ntx - 1);
        zc = t / per_z;
        int u = t - zc * per_z;
        if (u < nty) {
            xt = 0;
            yt = u;
        } else {
            u -= nty;
            xt = 1 + u % (ntx - 1);
            const int yo = u / (ntx - 1);
            yt = yo < M.yt_lo ? yo : yo + M.nyi;
        }
    }
    const int lane = threadIdx.x;
    const int yg = yt * kWavesY + threadIdx.y;
    if (MODE == M_RESID_R) {
        // Fused residual + full weighting, first pass: x tiles of 60 fine columns
        // (lanes 0..63 hold x = 60 xt - 1 .. 60 xt + 62; the residual is valid on
        // lanes 1..62, so the odd lanes 3..61 hold the 30 coarse columns whose
        // three fine neighbours are all valid); z chunks of M.tz coarse planes,
        // marching fine planes 2 Z0 - 1 .. 2 Z1 - 1 (one odd plane shared with
        // the next chunk).
        const int xg = 60 * xt - 1 + lane;
        const int xa = max(1, 60 * xt), xb = min(60 * xt + 61, L.nx - 1);
        const bool xi = (xa > xb) || (xa >= L.lox && xb <= L.hix);
        const int Z0 = zc * M.tz, Z1 = min(Z0 + M.tz, L.nz >> 1);
        double nrm = 0.0;
        if (yg <= L.ny) {
            const bool yi = (yg >= L.loy && yg <= L.hiy) || yg < 1 || yg > L.ny - 1;
            if (xi && yi)
                march<R, TX, TG, TY, MODE, SHIFT, false, true, true>(L, stab, x, g, base, y, omegaJ, mul, xg, yg, 2 * Z0 - 1,
                                                                     2 * Z1, false, nrm, Z0);
            else if (xi)
                march<R, TX, TG, TY, MODE, SHIFT, false, true, false>(L, stab, x, g, base, y, omegaJ, mul, xg, yg, 2 * Z0 - 1,
                                                                      2 * Z1, false, nrm, Z0);
            else if (yi)
                march<R, TX, TG, TY, MODE, SHIFT, false, false, true>(L, stab, x, g, base, y, omegaJ, mul, xg, yg, 2 * Z0 - 1,
                                                                      2 * Z1, false, nrm, Z0);
            else
                march<R, TX, TG, TY, MODE, SHIFT, false, false, false>(L, stab, x, g, base, y, omegaJ, mul, xg, yg,
                                                                       2 * Z0 - 1, 2 * Z1, false, nrm, Z0);
        }
        return;
    }
    const int z0 = zc * M.tz;
    const int z1 = min(z0 + M.tz, L.nz + 1);
    // x tiling: with split edges, tile 0 holds both x edge strips (lanes 0..31:
    // x = -1..30, lanes 32..63: x = nx-30..nx+1; lanes 31 and 32 are halo only),
    // so every other tile is free of x stretching; otherwise 62-column tiles.
    int xg;
    bool out_lane, xi;
    if (split_edges(L)) {
        if (xt == 0) {
            xg = lane < 32 ? lane - 1 : L.nx - kEdge + (lane - 32);
            out_lane = (lane >= 1 && lane <= kEdge) || (lane >= 33 && lane <= 62);
            xi = (L.lox <= 1 && L.hix >= L.nx - 1);
        } else {
            xg = kEdge - 1 + (xt - 1) * kTileX + lane;
            out_lane = (lane >= 1 && lane <= kTileX && xg <= L.nx - kEdge);
            xi = true;
        }
    } else {
        xg = xt * kTileX - 1 + lane;
        out_lane = (lane >= 1 && lane <= kTileX && xg <= L.nx);
        const int xa = max(1, xt * kTileX), xb = min(xt * kTileX + kTileX - 1, L.nx - 1);
        xi = (xa > xb) || (xa >= L.lox && xb <= L.hix);
    }
    double nrm = 0.0;
    if (PART == 1) {   // interior tiles: unit x/y weights on every row by construction
        march<R, TX, TG, TY, MODE, SHIFT, NORM, true, true>(L, stab, x, g, base, y, omegaJ, mul, xg, yg, z0, z1, out_lane,
                                                            nrm);
    } else if (yg <= L.ny) {
        const bool yi = (yg >= L.loy && yg <= L.hiy) || yg < 1 || yg > L.ny - 1;
        if (xi && yi)
            march<R, TX, TG, TY, MODE, SHIFT, NORM, true, true>(L, stab, x, g, base, y, omegaJ, mul, xg, yg, z0, z1,
                                                                out_lane, nrm);
        else if (xi)
            march<R, TX, TG, TY, MODE, SHIFT, NORM, true, false>(L, stab, x, g, base, y, omegaJ, mul, xg, yg, z0, z1,
                                                                 out_lane, nrm);
        else if (yi)
            march<R, TX, TG, TY, MODE, SHIFT, NORM, false, true>(L, stab, x, g, base, y, omegaJ, mul, xg, yg, z0, z1,
                                                                 out_lane, nrm);
        else
            march<R, TX, TG, TY, MODE, SHIFT, NORM, false, false>(L, stab, x, g, base, y, omegaJ, mul, xg, yg, z0, z1,
                                                                  out_lane, nrm);
    }
    if (NORM) {
        block_reduce_store(nrm, rb.partials + M.block_offset + tile);
        norm_epilogue(rb, M.total_blocks, st);
    }
}

// Amplitude correction Q_h (eq. q-operator): row i takes the shell weights of its own node
// (from beta at the fine-grid eta*) on its interior neighbours, with no stretching and no
// ell^-2.  One wavefront per row y at 64 consecutive x (outputs on lanes 1..62, neighbours
// x -+ 1 through DPP), marching kQZ planes in z: every plane gives its in-plane shell sums of
// the interior values, S0 (centre), S1 (four faces) and S2 (four corners), and output plane z
// takes Q0 S0(z) + Q1 (S1(z) + S0(z-+1)) + Q2 (S2(z) + S1(z-+1)) + Q3 S2(z-+1).  The loads of
// plane p + 1 are issued before plane p is summed.
constexpr int kQZ = 16, kQX = 62;

template <typename R>
struct QSums {
    Z<R> s0, s1, s2;
};

template <typename R, typename TI, typename TO>
__global__ void __launch_bounds__(256) k_qapply(LevelArgs<R> L, const TI *__restrict__ x, TO *__restrict__ y,
                                               Batch bt) {
    const int sl = blockIdx.z;   // batched right-hand side
    if (slot_off(bt, sl)) return;
    const long long nn = (long long)(L.nz + 1) * L.sy;
    x = slot_ptr(x, nn, sl);
    y = slot_ptr(y, nn, sl);
    extern __shared__ unsigned char smem_raw[];
    R *btab = reinterpret_cast<R *>(smem_raw);
    for (int i = threadIdx.x + 64 * threadIdx.y; i < L.K * 12; i += 256) btab[i] = L.btab[i];
    __syncthreads();
    const int ntx = (L.nx + kQX) / kQX;   // x tiles covering nodes 0..nx
    const int xt = blockIdx.x % ntx, yt = blockIdx.x / ntx;
    const int lane = threadIdx.x, yg = yt * 4 + threadIdx.y;
    const int xg = xt * kQX - 1 + lane;
    if (yg > L.ny) return;   // whole wavefronts leave; no barrier follows
    const int z0 = blockIdx.y * kQZ, z1 = min(z0 + kQZ, L.nz + 1);
    const bool x_int = xg >= 1 && xg <= L.nx - 1;
    const bool out_lane = lane >= 1 && lane <= kQX && xg <= L.nx;
    const int xc = min(max(xg, 0), L.nx);
    const int ym = max(yg - 1, 0), yp = min(yg + 1, L.ny);
    const bool rm_ok = x_int && yg - 1 >= 1, r0_ok = x_int && yg >= 1 && yg <= L.ny - 1, rp_ok = x_int && yg + 1 <= L.ny - 1;
    const long long om = (long long)ym * L.sx + xc, o0 = (long long)yg * L.sx + xc, op = (long long)yp * L.sx + xc;
    const Z<R> zero = {0, 0};
    struct Raw {
        TI a, b, c;
    };
    auto issue = [&](int p, Raw &r) {
        const long long base = (long long)min(max(p, 0), L.nz) * L.sy;
        r.a = x[base + om];
        r.b = x[base + o0];
        r.c = x[base + op];
    };
    auto sums = [&](int p, const Raw &r) {
        const bool zok = p >= 1 && p <= L.nz - 1;
        const Z<R> a = (zok && rm_ok) ? Z<R>{(R)r.a.re, (R)r.a.im} : zero;
        const Z<R> b = (zok && r0_ok) ? Z<R>{(R)r.b.re, (R)r.b.im} : zero;
        const Z<R> c = (zok && rp_ok) ? Z<R>{(R)r.c.re, (R)r.c.im} : zero;
        const Z<R> col = zadd(a, c);
        QSums<R> q;
        q.s0 = b;
        q.s1 = zadd(col, zadd(zleft(b), zright(b)));
        q.s2 = zadd(zleft(col), zright(col));
        return q;
    };
    auto emit = [&](int z, const QSums<R> &m, const QSums<R> &o, const QSums<R> &p) {
        if (!out_lane || z < z0 || z >= z1) return;
        Z<R> acc = zero;
        if (r0_ok && z >= 1 && z <= L.nz - 1) {
            R kappa, t;
            int k;
            locate(L, L.c[(long long)z * L.sy + o0], kappa, k, t);
            const R *bp = btab + k * 12;
            const R b1 = horner(bp, t), b2 = horner(bp + 4, t), b3 = horner(bp + 8, t);
            const R Q[4] = {b1, b2 * (R)(1.0 / 6), b3 * (R)(1.0 / 12), ((R)1 - b1 - b2 - b3) * (R)0.125};
            acc = zscale(Q[0], o.s0);
            acc = zadd(acc, zscale(Q[1], zadd(o.s1, zadd(m.s0, p.s0))));
            acc = zadd(acc, zscale(Q[2], zadd(o.s2, zadd(m.s1, p.s1))));
            acc = zadd(acc, zscale(Q[3], zadd(m.s2, p.s2)));
        }
        TO v;
        v.re = acc.r;
        v.im = acc.i;
        y[(long long)z * L.sy + o0] = v;
    };
    // window of plane sums: m (z - 1), o (z), p (z + 1); output plane z after plane z + 1 is summed
    Raw ra, rb;
    issue(z0 - 1, ra);
    issue(z0, rb);
    QSums<R> m = sums(z0 - 1, ra);
    issue(z0 + 1, ra);
    QSums<R> o = sums(z0, rb);
    for (int z = z0; z < z1; z += 2) {
        issue(z + 2, rb);
        const QSums<R> p = sums(z + 1, ra);   // plane z + 1 (issued one step earlier)
        emit(z, m, o, p);
        m = o;
        o = p;
        if (z + 1 >= z1) break;
        issue(z + 3, ra);
        const QSums<R> p2 = sums(z + 2, rb);
        emit(z + 1, m, o, p2);
        m = o;
        o = p2;
    }
}

// y = diag(H) x (test and diagnostics hook)
template <typename R, typename T, bool SHIFT>
__global__ void __launch_bounds__(256) k_diag(LevelArgs<R> L, const T *__restrict__ x, T *__restrict__ y) {
    extern __shared__ unsigned char smem_raw[];
    R *stab = reinterpret_cast<R *>(smem_raw);
    for (int i = threadIdx.x; i < L.nk * 20; i += blockDim.x) stab[i] = L.atab[L.kb * 20 + i];
    __syncthreads();
    const long long nn = (long long)(L.nz + 1) * L.sy;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn; i += (long long)gridDim.x * blockDim.x) {
        const int xi = (int)(i % L.sx);
        const int yi = (int)((i / L.sx) % (L.ny + 1));
        const int zi = (int)(i / L.sy);
        Z<R> r = {0, 0};
        if (xi >= 1 && xi <= L.nx - 1 && yi >= 1 && yi <= L.ny - 1 && zi >= 1 && zi <= L.nz - 1) {
            Coef<R> cf = coef_at(L, stab, node_values(L)[i]);
            Z<R> ws = {L.wx[6 * xi + 2] + L.wy[6 * yi + 2] + L.wz[6 * zi + 2],
                       L.wx[6 * xi + 3] + L.wy[6 * yi + 3] + L.wz[6 * zi + 3]};
            r = zmul(diag_of<R, SHIFT>(L, cf.a1, cf.a4, cf.k2, ws), ld<R>(x, i));
        }
        T o;
        o.re = r.r;
        o.im = r.i;
        y[i] = o;
    }
}

// one Jacobi sweep from zero: y = omega D^-1 g (eq. jacobi-map with n_J = 1)
template <typename R, typename T>
__global__ void __launch_bounds__(256) k_jac1(const R *__restrict__ dinv, const T *__restrict__ g, T *__restrict__ y,
                                              long long nn, R omegaJ, Batch bt) {
    if (slot_off(bt, blockIdx.y)) return;
    g = slot_ptr(g, nn, blockIdx.y);
    y = slot_ptr(y, nn, blockIdx.y);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn; i += (long long)gridDim.x * blockDim.x) {
        const Z<R> r = zscale(omegaJ, zmul(Z<R>{dinv[2 * i], dinv[2 * i + 1]}, ld<R>(g, i)));
        T o;
        o.re = r.r;
        o.im = r.i;
        y[i] = o;
    }
}

// D^-1 at every node of a level (zero on the boundary): the diagonal depends
// only on the velocity, the stretching and the shift, so the Jacobi kernels
// read it instead of evaluating the coefficients of every neighbour row.
template <typename R, bool SHIFT>
__global__ void __launch_bounds__(256) k_dinv(LevelArgs<R> L, R *__restrict__ out) {
    extern __shared__ unsigned char smem_raw[];
    R *stab = reinterpret_cast<R *>(smem_raw);
    for (int i = threadIdx.x; i < L.nk * 20; i += blockDim.x) stab[i] = L.atab[L.kb * 20 + i];
    __syncthreads();
    const long long nn = (long long)(L.nz + 1) * L.sy;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn; i += (long long)gridDim.x * blockDim.x) {
        const int xi = (int)(i % L.sx);
        const int yi = (int)((i / L.sx) % (L.ny + 1));
        const int zi = (int)(i / L.sy);
        Z<R> r = {0, 0};
        if (xi >= 1 && xi <= L.nx - 1 && yi >= 1 && yi <= L.ny - 1 && zi >= 1 && zi <= L.nz - 1) {
            Coef<R> cf = coef_at(L, stab, node_values(L)[i]);
            Z<R> ws = {L.wx[6 * xi + 2] + L.wy[6 * yi + 2] + L.wz[6 * zi + 2],
                       L.wx[6 * xi + 3] + L.wy[6 * yi + 3] + L.wz[6 * zi + 3]};
            r = zdiv(Z<R>{1, 0}, diag_of<R, SHIFT>(L, cf.a1, cf.a4, cf.k2, ws));
        }
        out[2 * i] = r.r;
        out[2 * i + 1] = r.i;
    }
}

int pick_tz(int ntx, int nty, int nz1) {
    long long work = (long long)ntx * nty * nz1;
    long long tz = (work + 4095) / 4096;
    if (tz < 4) tz = 4;
    if (tz > 64) tz = 64;
    return (int)tz;
}

// Modes each operand-type combination is built for: all of them for FP32 / FP64 operands;
// for FP16-stored ones (HELM_MIXED) only those the mixed-precision cycle uses, without the
// fused norm: the V-cycle's first Jacobi y = J(B, q) (c32 -> c16), the fused residual +
// restriction and the residual from y (c16 x), the bottom basis steps and the V-cycle's
// last Jacobi + base (all c16), and K_2h's A_2h Z (c16 -> c32).
template <typename TX, typename TG, typename TY>
constexpr bool mode_built(int mode, bool shifted, bool norm) {
    constexpr bool hx = is_half<TX>(), hg = is_half<TG>(), hy = is_half<TY>();
    if (!hx && !hg && !hy) return true;
    if (norm) return false;
    if (!hx && !hg && hy) return mode == M_JAC2 && shifted;
    if (hx && hg && hy) return (mode == M_JAC2 || mode == M_APPLY || mode == M_JAC2_ADD) && shifted;
    if (hx && !hg && !hy) return mode == M_RESID_R && shifted;
    if (hx && !hg && hy) return mode == M_RESID && shifted;
    if (hx && hg && !hy) return mode == M_APPLY && !shifted;
    return false;
}

}  // namespace

template <typename R, typename TX, typename TG, typename TY, int PART>
hipError_t launch_stencil_part(const LevelArgs<R> &L, const StencilCall &c, const RedBuf &rb, const TileMap &M,
                               int blocks, hipStream_t s) {
    const dim3 blk(64, kWavesY);
    const size_t shm = sizeof(R) * (L.nk * 20 + (scaled_coordinate<R>() ? L.nck * 24 : 0));
    const TX *x = (const TX *)c.x;
    const TG *g = (const TG *)c.g;
    const TY *base = (const TY *)c.base;
    TY *y = (TY *)c.y;
    const R om = (R)c.omegaJ;
    const Scales sc = {c.sx, c.sg, c.sb, c.sy};
    const Batch &bt = cur_batch();
#define HELM_LAUNCH(MODE, SH, NRM)                                                                                  \
    do {                                                                                                            \
        if constexpr (mode_built<TX, TG, TY>(MODE, SH, NRM))                                                        \
            hipLaunchKernelGGL((k_stencil<R, TX, TG, TY, MODE, SH, NRM, PART>), dim3(blocks * bt.n), blk, shm, s, L, \
                               x, g, base, y, om, M, rb, c.st, sc, bt);                                             \
        else                                                                                                        \
            return hipErrorInvalidValue;                                                                            \
    } while (0)
    if (c.norm) {
        if (c.mode != M_RESID) return hipErrorInvalidValue;
        if (c.shifted)
            HELM_LAUNCH(M_RESID, true, true);
        else
            HELM_LAUNCH(M_RESID, false, true);
        return hipGetLastError();
    }
    switch (c.mode) {
    case M_APPLY:
        if (c.shifted) HELM_LAUNCH(M_APPLY, true, false); else HELM_LAUNCH(M_APPLY, false, false);
        break;
    case M_RESID:
        if (c.shifted) HELM_LAUNCH(M_RESID, true, false); else HELM_LAUNCH(M_RESID, false, false);
        break;
    case M_JSWEEP:
        if (c.shifted) HELM_LAUNCH(M_JSWEEP, true, false); else HELM_LAUNCH(M_JSWEEP, false, false);
        break;
    case M_JAC2:
        if (c.shifted) HELM_LAUNCH(M_JAC2, true, false); else HELM_LAUNCH(M_JAC2, false, false);
        break;
    case M_JAC2_ADD:
        if (c.shifted) HELM_LAUNCH(M_JAC2_ADD, true, false); else HELM_LAUNCH(M_JAC2_ADD, false, false);
        break;
    case M_RESID_R:
        if constexpr (PART == 0) {
            if (c.shifted) HELM_LAUNCH(M_RESID_R, true, false); else HELM_LAUNCH(M_RESID_R, false, false);
        } else {
            return hipErrorInvalidValue;
        }
        break;
    default:
        return hipErrorInvalidValue;
    }
#undef HELM_LAUNCH
    return hipGetLastError();
}

template <typename R, typename TX, typename TG, typename TY>
hipError_t launch_stencil(const LevelArgs<R> &L, const StencilCall &c, const RedBuf &rb, hipStream_t s) {
    if (scaled_coordinate<R>() && (!L.s || !L.ctab)) return hipErrorInvalidValue;   // FP32 levels read s
    // the Jacobi modes read the stored D^-1 of the operator
    if ((c.mode == M_JSWEEP || c.mode == M_JAC2 || c.mode == M_JAC2_ADD) && !L.dinv[c.shifted ? 1 : 0])
        return hipErrorInvalidValue;
    TileMap M;
    if (c.mode == M_RESID_R) {
        if (c.norm) return hipErrorInvalidValue;
        M.ntx = std::max(1, ceil_div((L.nx >> 1) - 1, 30));
        M.nty = ceil_div(L.ny + 1, kWavesY);
        M.tz = std::max(1, (L.tz[0] > 0 ? L.tz[0] : pick_tz(M.ntx, M.nty, L.nz + 1)) / 2);   // coarse planes per chunk
        M.yt_lo = M.nyi = 0;
        M.block_offset = 0;
        M.total_blocks = M.ntx * M.nty * ceil_div(L.nz >> 1, M.tz);
        return launch_stencil_part<R, TX, TG, TY, 0>(L, c, rb, M, M.total_blocks, s);
    }
    M.ntx = x_tiles(L);
    M.nty = ceil_div(L.ny + 1, kWavesY);
    const int fam = (c.mode == M_JAC2 || c.mode == M_JAC2_ADD) ? 1 : 0;
    M.tz = L.tz[fam] > 0 ? L.tz[fam] : pick_tz(M.ntx, M.nty, L.nz + 1);
    const int nzc = ceil_div(L.nz + 1, M.tz);
    const int blocks = M.ntx * M.nty * nzc;
    // interior y tiles: all kWavesY rows inside [loy, hiy]
    M.yt_lo = ceil_div(L.loy, kWavesY);
    M.nyi = std::max(0, (L.hiy + 1) / kWavesY - M.yt_lo);
    M.block_offset = 0;
    M.total_blocks = blocks;
    if (L.split[fam] && split_edges(L) && M.ntx > 1 && M.nyi > 0) {
        const int bi = (M.ntx - 1) * M.nyi * nzc;
        const int bb = blocks - bi;
        hipError_t e = launch_stencil_part<R, TX, TG, TY, 2>(L, c, rb, M, bb, s);
        if (e != hipSuccess) return e;
        M.block_offset = bb;
        return launch_stencil_part<R, TX, TG, TY, 1>(L, c, rb, M, bi, s);
    }
    M.yt_lo = M.nyi = 0;
    return launch_stencil_part<R, TX, TG, TY, 0>(L, c, rb, M, blocks, s);
}

}  // namespace helm
