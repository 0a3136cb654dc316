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
__device__ __forceinline__ Coef<R> coef_at(const LevelArgs<R> &L, const R *stab, float c) {
    R kappa, t;
    int k;
    locate(L, c, kappa, k, t);
    const R *p = stab + k * 20;
    Coef<R> o;
    o.a1 = horner(p + 0, t);
    o.a2 = horner(p + 4, t);
    o.a3 = horner(p + 8, t);
    o.a4 = horner(p + 12, t);
    o.a5 = horner(p + 16, t);
    o.k2 = kappa * kappa;
    return o;
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
};

template <typename R>
struct Rows {
    Z<R> a, b, c;      // rows y-1, y, y+1 at this lane's x
};

// in-plane partial sums of one z plane (x neighbours from adjacent lanes)
template <typename R, bool XYI>
__device__ __forceinline__ Plane<R> plane_partials(const Rows<R> &v, const Z<R> *wx, const Z<R> *wy) {
    Plane<R> P;
    Z<R> col = zadd(v.a, v.c);
    if (XYI) {
        P.p0 = v.b;
        P.p1 = zadd(col, zadd(zleft(v.b), zright(v.b)));
        P.p2 = zadd(zleft(col), zright(col));
        P.ea = P.eb = Z<R>{0, 0};
    } else {
        Z<R> aL = zleft(v.a), aR = zright(v.a), bL = zleft(v.b), bR = zright(v.b), cL = zleft(v.c),
             cR = zright(v.c);
        Z<R> colL = zadd(aL, cL), colR = zadd(aR, cR);
        Z<R> rsm = zadd(aL, aR), rs0 = zadd(bL, bR), rsp = zadd(cL, cR);
        P.p0 = v.b;
        P.p1 = zadd(col, rs0);
        P.p2 = zadd(rsm, rsp);
        Z<R> ea = zmul(wx[0], bL);
        ea = zfma(wx[1], v.b, ea);
        ea = zfma(wx[2], bR, ea);
        ea = zfma(wy[0], v.a, ea);
        ea = zfma(wy[1], v.b, ea);
        ea = zfma(wy[2], v.c, ea);
        Z<R> eb = zmul(wx[0], colL);
        eb = zfma(wx[1], col, eb);
        eb = zfma(wx[2], colR, eb);
        eb = zfma(wy[0], rsm, eb);
        eb = zfma(wy[1], rs0, eb);
        eb = zfma(wy[2], rsp, eb);
        P.ea = ea;
        P.eb = eb;
    }
    return P;
}

// ell^2 (H v) at the centre of plane "o" from planes m (z-1), o (z), p (z+1)
template <typename R, bool XYI, bool SHIFT>
__device__ __forceinline__ Z<R> row_value(const LevelArgs<R> &L, const Coef<R> &cf, const Plane<R> &m,
                                          const Plane<R> &o, const Plane<R> &p, bool zint, const Z<R> *wz) {
    // shell sums S_m over the 1 / 6 / 12 / 8 neighbours
    Z<R> S0 = o.p0;
    Z<R> S1 = zadd(o.p1, zadd(m.p0, p.p0));
    Z<R> S2 = zadd(o.p2, zadd(m.p1, p.p1));
    Z<R> S3 = zadd(m.p2, p.p2);
    const R a1 = cf.a1, a2 = cf.a2, a3 = cf.a3, a4 = cf.a4, a5 = cf.a5;
    const R q = (R)1 - a4 - a5;
    const R mass0 = a1, mass1 = a2 * (R)(1.0 / 6), mass2 = a3 * (R)(1.0 / 12), mass3 = ((R)1 - a1 - a2 - a3) * (R)0.125;
    Z<R> Mass = zscale(mass0, S0);
    Mass = zadd(Mass, zscale(mass1, S1));
    Mass = zadd(Mass, zscale(mass2, S2));
    Mass = zadd(Mass, zscale(mass3, S3));
    Z<R> St;
    if (XYI && zint) {
        // eq. iofd-shell-coefficients, stiffness parts
        St = zscale((R)6 * a4, S0);
        St = zadd(St, zscale(a5 - a4, S1));
        St = zadd(St, zscale((R)0.5 * (q - a5), S2));
        St = zadd(St, zscale((R)-0.75 * q, S3));
    } else {
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
        Z<R> z0 = zmul(wz[1], o.p0);
        z0 = zfma(wz[0], m.p0, z0);
        z0 = zfma(wz[2], p.p0, z0);
        Z<R> z1 = zmul(wz[1], o.p1);
        z1 = zfma(wz[0], m.p1, z1);
        z1 = zfma(wz[2], p.p1, z1);
        Z<R> z2 = zmul(wz[1], o.p2);
        z2 = zfma(wz[0], m.p2, z2);
        z2 = zfma(wz[2], p.p2, z2);
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
    // wave64 butterfly then across the 4 waves through LDS
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __shared__ double red[kWavesY];
    int w = threadIdx.y, l = threadIdx.x;
    if (l == 0) red[w] = v;
    __syncthreads();
    if (w == 0 && l == 0) {
        double s = 0;
        for (int i = 0; i < kWavesY; ++i) s += red[i];
        *dst = s;
    }
}

// Last-block epilogue of a stencil with fused ||y||^2: beta, state reset.
__device__ void norm_epilogue(const RedBuf &rb, int nblocks, KState *st) {
    __shared__ bool last;
    __shared__ double red[256];
    const int tid = threadIdx.x + 64 * threadIdx.y;
    __threadfence();
    if (tid == 0) last = (atomicAdd(rb.counter, 1u) == (unsigned)nblocks - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    double s = 0;
    for (int b = tid; b < nblocks; b += 256)
        s += __hip_atomic_load(rb.partials + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    red[tid] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
    }
    if (tid == 0) {
        double beta = sqrt(red[0]);
        st->beta = beta;
        st->scale = (beta > 0.0) ? 1.0 / beta : 0.0;
        st->kk = 0;
        st->breakdown = 0;
        st->nonfinite = !(beta == beta && beta < 1e300);
        for (int j = 0; j <= kMMax; ++j) st->g[j][0] = st->g[j][1] = 0.0;
        st->g[0][0] = beta;
        *rb.counter = 0u;
    }
}

template <typename R, typename TX, typename TG, typename TY, int MODE, bool SHIFT, bool NORM, bool XYI>
__device__ __forceinline__ void march(const LevelArgs<R> &L, const R *stab, const TX *__restrict__ x,
                                      const TG *__restrict__ g, const TY *__restrict__ base, TY *__restrict__ y,
                                      R omegaJ, int xg, int yg, int z0, int z1, bool out_lane, double &nrm) {
    const bool x_int = (xg >= 1 && xg <= L.nx - 1);
    const long long rowoff = (long long)yg * L.sx + xg;
    Z<R> wx[3] = {{0, 0}, {0, 0}, {0, 0}}, wy[3] = {{0, 0}, {0, 0}, {0, 0}};
    Z<R> wyc_m = {0, 0}, wyc_p = {0, 0};
    if (x_int) {
        const R *w = L.wx + 6 * xg;
        wx[0] = {w[0], w[1]}; wx[1] = {w[2], w[3]}; wx[2] = {w[4], w[5]};
    }
    {
        const R *w = L.wy + 6 * yg;
        wy[0] = {w[0], w[1]}; wy[1] = {w[2], w[3]}; wy[2] = {w[4], w[5]};
        if (MODE == M_JAC2 || MODE == M_JAC2_ADD) {
            if (yg - 1 >= 1) wyc_m = {L.wy[6 * (yg - 1) + 2], L.wy[6 * (yg - 1) + 3]};
            if (yg + 1 <= L.ny - 1) wyc_p = {L.wy[6 * (yg + 1) + 2], L.wy[6 * (yg + 1) + 3]};
        }
    }
    const bool rm_ok = x_int && (yg - 1 >= 1);
    const bool r0_ok = x_int && (yg >= 1) && (yg <= L.ny - 1);
    const bool rp_ok = x_int && (yg + 1 <= L.ny - 1);
    constexpr bool JAC = (MODE == M_JAC2 || MODE == M_JAC2_ADD);

    // per plane: values (operand, or omega D^-1 g for the fused two-sweep Jacobi)
    auto load_plane = [&](int zp, Rows<R> &v, float &cc, Z<R> &gc) {
        v.a = v.b = v.c = Z<R>{0, 0};
        cc = 1.0f;
        gc = Z<R>{0, 0};
        if (zp < 1 || zp > L.nz - 1) return;
        const long long pz = (long long)zp * L.sy + rowoff;
        if (r0_ok) cc = L.c[pz];
        if (!JAC) {
            if (rm_ok) v.a = ld<R>(x, pz - L.sx);
            if (r0_ok) v.b = ld<R>(x, pz);
            if (rp_ok) v.c = ld<R>(x, pz + L.sx);
            if (MODE == M_RESID || MODE == M_JSWEEP) {
                if (r0_ok) gc = ld<R>(g, pz);
            }
        } else {
            const R *wzp = L.wz + 6 * zp;
            Z<R> wzc = {wzp[2], wzp[3]};
            Z<R> wxc = wx[1];
            if (rm_ok) {
                Z<R> gv = ld<R>(g, pz - L.sx);
                Coef<R> cf = coef_at(L, stab, L.c[pz - L.sx]);
                Z<R> D = diag_of<R, SHIFT>(L, cf.a1, cf.a4, cf.k2, zadd(wxc, zadd(wyc_m, wzc)));
                v.a = zscale(omegaJ, zdiv(gv, D));
            }
            if (r0_ok) {
                gc = ld<R>(g, pz);
                Coef<R> cf = coef_at(L, stab, cc);
                Z<R> D = diag_of<R, SHIFT>(L, cf.a1, cf.a4, cf.k2, zadd(wxc, zadd(wy[1], wzc)));
                v.b = zscale(omegaJ, zdiv(gc, D));
            }
            if (rp_ok) {
                Z<R> gv = ld<R>(g, pz + L.sx);
                Coef<R> cf = coef_at(L, stab, L.c[pz + L.sx]);
                Z<R> D = diag_of<R, SHIFT>(L, cf.a1, cf.a4, cf.k2, zadd(wxc, zadd(wyc_p, wzc)));
                v.c = zscale(omegaJ, zdiv(gv, D));
            }
        }
    };

    const bool yint = (yg >= 1 && yg <= L.ny - 1);
    Plane<R> Pm, Po, Pp;
    float cm = 1.f, co = 1.f, cp = 1.f;
    Z<R> gm = {0, 0}, go = {0, 0}, gp = {0, 0};
    Rows<R> cur, nxt;
    float cnx;
    Z<R> gnx;
    load_plane(z0 - 1, cur, cm, gm);
    Pm = plane_partials<R, XYI>(cur, wx, wy);
    load_plane(z0, cur, co, go);
    load_plane(z0 + 1, nxt, cnx, gnx);
    Po = plane_partials<R, XYI>(cur, wx, wy);
    for (int z = z0; z < z1; ++z) {
        cur = nxt;
        cp = cnx;
        gp = gnx;
        if (z + 2 <= z1) load_plane(z + 2, nxt, cnx, gnx);   // prefetch the plane after next
        Pp = plane_partials<R, XYI>(cur, wx, wy);
        // ---- output plane z ----
        if (out_lane) {
            const long long oi = (long long)z * L.sy + rowoff;
            const bool interior = x_int && yint && z >= 1 && z <= L.nz - 1;
            Z<R> res = {0, 0};
            if (interior) {
                Coef<R> cf = coef_at(L, stab, co);
                const bool zint = (z >= L.loz && z <= L.hiz);
                Z<R> wz[3];
                const R *wzp = L.wz + 6 * z;
                wz[0] = {wzp[0], wzp[1]}; wz[1] = {wzp[2], wzp[3]}; wz[2] = {wzp[4], wzp[5]};
                Z<R> Hv = row_value<R, XYI, SHIFT>(L, cf, Pm, Po, Pp, zint, wz);
                if (MODE == M_APPLY) {
                    res = Hv;
                } else if (MODE == M_RESID) {
                    res = zsub(go, Hv);
                } else {
                    Z<R> D = diag_of<R, SHIFT>(L, cf.a1, cf.a4, cf.k2, zadd(wx[1], zadd(wy[1], wz[1])));
                    Z<R> upd = zscale(omegaJ, zdiv(zsub(go, Hv), D));
                    res = zadd(Po.p0, upd);   // p0 holds the operand (JSWEEP) or omega D^-1 g (JAC2)
                }
            }
            if (MODE == M_JAC2_ADD) res = zadd(res, ld<R>(base, oi));
            TY o;
            o.re = res.r;
            o.im = res.i;
            y[oi] = o;
            if (NORM) nrm += (double)res.r * (double)res.r + (double)res.i * (double)res.i;
        }
        Pm = Po;
        Po = Pp;
        co = cp;
        go = gp;
        (void)cm;
        (void)gm;
    }
}

template <typename R, typename TX, typename TG, typename TY, int MODE, bool SHIFT, bool NORM>
__global__ void __launch_bounds__(256) k_stencil(LevelArgs<R> L, const TX *__restrict__ x, const TG *__restrict__ g,
                                                 const TY *__restrict__ base, TY *__restrict__ y, R omegaJ, int ntx,
                                                 int nty, int tz, RedBuf rb, KState *st) {
    extern __shared__ unsigned char smem_raw[];
    R *stab = reinterpret_cast<R *>(smem_raw);
    const int tid = threadIdx.x + 64 * threadIdx.y;
    for (int i = tid; i < L.K * 20; i += 256) stab[i] = L.atab[i];
    __syncthreads();

    // XCD-aware tile order: block b runs on XCD b % 8; give each XCD a contiguous tile range
    const int nb = gridDim.x, b = blockIdx.x;
    const int per = nb / 8, rem = nb % 8, xcd = b % 8, idx = b / 8;
    int t = (xcd < rem) ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
    const int xt = t % ntx;
    t /= ntx;
    const int yt = t % nty;
    const int zc = t / nty;
    const int lane = threadIdx.x;
    const int xg = xt * kTileX - 1 + lane;
    const int yg = yt * kWavesY + threadIdx.y;
    const int z0 = zc * tz;
    const int z1 = min(z0 + tz, L.nz + 1);
    double nrm = 0.0;
    if (yg <= L.ny) {
        const bool out_lane = (lane >= 1 && lane <= kTileX && xg <= L.nx);
        // whole wave free of x/y stretching?
        const int xa = max(1, xt * kTileX), xb = min(xt * kTileX + kTileX - 1, L.nx - 1);
        const bool xyi = (yg >= L.loy && yg <= L.hiy) && (xa > xb || (xa >= L.lox && xb <= L.hix));
        if (xyi)
            march<R, TX, TG, TY, MODE, SHIFT, NORM, true>(L, stab, x, g, base, y, omegaJ, xg, yg, z0, z1, out_lane,
                                                          nrm);
        else
            march<R, TX, TG, TY, MODE, SHIFT, NORM, false>(L, stab, x, g, base, y, omegaJ, xg, yg, z0, z1, out_lane,
                                                           nrm);
    }
    if (NORM) {
        block_reduce_store(nrm, rb.partials + blockIdx.x);
        norm_epilogue(rb, gridDim.x, st);
    }
}

// Amplitude correction Q_h (eq. q-operator): shell weights from beta at the
// fine-grid eta*, no stretching and no ell^-2.  Used twice per solve, so a
// plain one-thread-per-node gather is enough.
template <typename R, typename TI, typename TO>
__global__ void __launch_bounds__(256) k_qapply(LevelArgs<R> L, const TI *__restrict__ x, TO *__restrict__ y) {
    extern __shared__ unsigned char smem_raw[];
    R *btab = reinterpret_cast<R *>(smem_raw);
    for (int i = threadIdx.x; i < L.K * 12; i += blockDim.x) btab[i] = L.btab[i];
    __syncthreads();
    const long long nn = (long long)(L.nz + 1) * L.sy;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn; i += (long long)gridDim.x * blockDim.x) {
        const int xi = (int)(i % L.sx);
        const int yi = (int)((i / L.sx) % (L.ny + 1));
        const int zi = (int)(i / L.sy);
        Z<R> acc = {0, 0};
        if (xi >= 1 && xi <= L.nx - 1 && yi >= 1 && yi <= L.ny - 1 && zi >= 1 && zi <= L.nz - 1) {
            R kappa, t;
            int k;
            locate(L, L.c[i], kappa, k, t);
            const R *p = btab + k * 12;
            const R b1 = horner(p, t), b2 = horner(p + 4, t), b3 = horner(p + 8, t);
            const R Q[4] = {b1, b2 * (R)(1.0 / 6), b3 * (R)(1.0 / 12), ((R)1 - b1 - b2 - b3) * (R)0.125};
            Z<R> S[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int xx = xi + dx, yy = yi + dy, zz = zi + dz;
                        if (xx < 1 || xx > L.nx - 1 || yy < 1 || yy > L.ny - 1 || zz < 1 || zz > L.nz - 1) continue;
                        const int sh = (dx != 0) + (dy != 0) + (dz != 0);
                        S[sh] = zadd(S[sh], ld<R>(x, i + dx + dy * L.sx + dz * L.sy));
                    }
            for (int m = 0; m < 4; ++m) acc = zadd(acc, zscale(Q[m], S[m]));
        }
        TO o;
        o.re = acc.r;
        o.im = acc.i;
        y[i] = o;
    }
}

// y = diag(H) x (test and diagnostics hook)
template <typename R, typename T, bool SHIFT>
__global__ void __launch_bounds__(256) k_diag(LevelArgs<R> L, const T *__restrict__ x, T *__restrict__ y) {
    extern __shared__ unsigned char smem_raw[];
    R *stab = reinterpret_cast<R *>(smem_raw);
    for (int i = threadIdx.x; i < L.K * 20; i += blockDim.x) stab[i] = L.atab[i];
    __syncthreads();
    const long long nn = (long long)(L.nz + 1) * L.sy;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn; i += (long long)gridDim.x * blockDim.x) {
        const int xi = (int)(i % L.sx);
        const int yi = (int)((i / L.sx) % (L.ny + 1));
        const int zi = (int)(i / L.sy);
        Z<R> r = {0, 0};
        if (xi >= 1 && xi <= L.nx - 1 && yi >= 1 && yi <= L.ny - 1 && zi >= 1 && zi <= L.nz - 1) {
            Coef<R> cf = coef_at(L, stab, L.c[i]);
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
template <typename R, typename T, bool SHIFT>
__global__ void __launch_bounds__(256) k_jac1(LevelArgs<R> L, const T *__restrict__ g, T *__restrict__ y, R omegaJ) {
    extern __shared__ unsigned char smem_raw[];
    R *stab = reinterpret_cast<R *>(smem_raw);
    for (int i = threadIdx.x; i < L.K * 20; i += blockDim.x) stab[i] = L.atab[i];
    __syncthreads();
    const long long nn = (long long)(L.nz + 1) * L.sy;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn; i += (long long)gridDim.x * blockDim.x) {
        const int xi = (int)(i % L.sx);
        const int yi = (int)((i / L.sx) % (L.ny + 1));
        const int zi = (int)(i / L.sy);
        Z<R> r = {0, 0};
        if (xi >= 1 && xi <= L.nx - 1 && yi >= 1 && yi <= L.ny - 1 && zi >= 1 && zi <= L.nz - 1) {
            Coef<R> cf = coef_at(L, stab, L.c[i]);
            Z<R> ws = {L.wx[6 * xi + 2] + L.wy[6 * yi + 2] + L.wz[6 * zi + 2],
                       L.wx[6 * xi + 3] + L.wy[6 * yi + 3] + L.wz[6 * zi + 3]};
            r = zscale(omegaJ, zdiv(ld<R>(g, i), diag_of<R, SHIFT>(L, cf.a1, cf.a4, cf.k2, ws)));
        }
        T o;
        o.re = r.r;
        o.im = r.i;
        y[i] = o;
    }
}

int pick_tz(int ntx, int nty, int nz1) {
    long long work = (long long)ntx * nty * nz1;
    long long tz = (work + 4095) / 4096;
    if (tz < 4) tz = 4;
    if (tz > 64) tz = 64;
    return (int)tz;
}

}  // namespace

template <typename R, typename TX, typename TG, typename TY>
hipError_t launch_stencil(const LevelArgs<R> &L, const StencilCall &c, const RedBuf &rb, hipStream_t s) {
    const int ntx = ceil_div(L.nx + 1, kTileX);
    const int nty = ceil_div(L.ny + 1, kWavesY);
    const int tz = pick_tz(ntx, nty, L.nz + 1);
    const int nzc = ceil_div(L.nz + 1, tz);
    const int blocks = ntx * nty * nzc;
    const dim3 blk(64, kWavesY);
    const size_t shm = sizeof(R) * L.K * 20;
    const TX *x = (const TX *)c.x;
    const TG *g = (const TG *)c.g;
    const TY *base = (const TY *)c.base;
    TY *y = (TY *)c.y;
    const R om = (R)c.omegaJ;
#define HELM_LAUNCH(MODE, SH, NRM)                                                                              \
    hipLaunchKernelGGL((k_stencil<R, TX, TG, TY, MODE, SH, NRM>), dim3(blocks), blk, shm, s, L, x, g, base, y, om, \
                       ntx, nty, tz, rb, c.st)
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
    default:
        return hipErrorInvalidValue;
    }
#undef HELM_LAUNCH
    return hipGetLastError();
}

int stencil_blocks(int nx, int ny, int nz) {
    const int ntx = ceil_div(nx + 1, kTileX);
    const int nty = ceil_div(ny + 1, kWavesY);
    const int tz = pick_tz(ntx, nty, nz + 1);
    return ntx * nty * ceil_div(nz + 1, tz);
}

template <typename R, typename TI, typename TO>
hipError_t launch_qapply(const LevelArgs<R> &L, const TI *x, TO *y, hipStream_t s) {
    const long long nn = (long long)(L.nz + 1) * L.sy;
    int blocks = (int)std::min<long long>((nn + 255) / 256, 65536);
    hipLaunchKernelGGL((k_qapply<R, TI, TO>), dim3(blocks), dim3(256), sizeof(R) * L.K * 12, s, L, x, y);
    return hipGetLastError();
}

template <typename R, typename T>
hipError_t launch_diag(const LevelArgs<R> &L, int shifted, const T *x, T *y, hipStream_t s) {
    const long long nn = (long long)(L.nz + 1) * L.sy;
    int blocks = (int)std::min<long long>((nn + 255) / 256, 65536);
    if (shifted)
        hipLaunchKernelGGL((k_diag<R, T, true>), dim3(blocks), dim3(256), sizeof(R) * L.K * 20, s, L, x, y);
    else
        hipLaunchKernelGGL((k_diag<R, T, false>), dim3(blocks), dim3(256), sizeof(R) * L.K * 20, s, L, x, y);
    return hipGetLastError();
}

template <typename R, typename T>
hipError_t launch_jac1(const LevelArgs<R> &L, int shifted, double omegaJ, const T *g, T *y, hipStream_t s) {
    const long long nn = (long long)(L.nz + 1) * L.sy;
    int blocks = (int)std::min<long long>((nn + 255) / 256, 65536);
    if (shifted)
        hipLaunchKernelGGL((k_jac1<R, T, true>), dim3(blocks), dim3(256), sizeof(R) * L.K * 20, s, L, g, y, (R)omegaJ);
    else
        hipLaunchKernelGGL((k_jac1<R, T, false>), dim3(blocks), dim3(256), sizeof(R) * L.K * 20, s, L, g, y,
                           (R)omegaJ);
    return hipGetLastError();
}

template hipError_t launch_jac1<float, c32>(const LevelArgs<float> &, int, double, const c32 *, c32 *, hipStream_t);
template hipError_t launch_jac1<double, c64>(const LevelArgs<double> &, int, double, const c64 *, c64 *, hipStream_t);
template hipError_t launch_stencil<float, c32, c32, c32>(const LevelArgs<float> &, const StencilCall &, const RedBuf &,
                                                         hipStream_t);
template hipError_t launch_stencil<double, c64, c64, c64>(const LevelArgs<double> &, const StencilCall &,
                                                          const RedBuf &, hipStream_t);
template hipError_t launch_stencil<double, c64, c64, c32>(const LevelArgs<double> &, const StencilCall &,
                                                          const RedBuf &, hipStream_t);
template hipError_t launch_qapply<double, c32, c64>(const LevelArgs<double> &, const c32 *, c64 *, hipStream_t);
template hipError_t launch_qapply<double, c64, c32>(const LevelArgs<double> &, const c64 *, c32 *, hipStream_t);
template hipError_t launch_qapply<double, c64, c64>(const LevelArgs<double> &, const c64 *, c64 *, hipStream_t);
template hipError_t launch_qapply<float, c32, c32>(const LevelArgs<float> &, const c32 *, c32 *, hipStream_t);
template hipError_t launch_diag<float, c32>(const LevelArgs<float> &, int, const c32 *, c32 *, hipStream_t);
template hipError_t launch_diag<double, c64>(const LevelArgs<double> &, int, const c64 *, c64 *, hipStream_t);

}  // namespace helm
