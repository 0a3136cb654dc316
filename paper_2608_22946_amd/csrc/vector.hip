// Krylov vector kernels of the nested (F)GMRES iterations (Sec. 3.2, 3.3):
// multi-dot products, the two classical Gram-Schmidt passes of one Arnoldi
// step, normalisation, the final combination x += Z y, and the Gram matrix of
// the s-step basis of the bottom solver.  All sums are accumulated in FP64 and
// reduced deterministically: every block writes its partial sums, the last
// block to finish (atomic ticket) adds them in a fixed order and runs the
// small dense epilogue (Givens rotation, back substitution, Cholesky) in FP64,
// so that no host synchronisation is needed inside a preconditioner call.
#include <algorithm>
#include <type_traits>

#include "helm_internal.h"

namespace helm {

constexpr int kSlots = kRedSlots;

namespace {
thread_local Batch g_batch;
}
Batch &cur_batch() { return g_batch; }

namespace {

template <typename T>
using real_of = decltype(T{}.re);

struct D2 {
    double r, i;
};

__device__ __forceinline__ D2 operator+(D2 a, D2 b) { return {a.r + b.r, a.i + b.i}; }

template <typename T>
__device__ __forceinline__ D2 cdot(T a, T b) {   // conj(a) * b
    const double ar = a.re, ai = a.im, br = b.re, bi = b.im;
    return {ar * br + ai * bi, ar * bi - ai * br};
}

__device__ __forceinline__ double wave_sum(double v) { return wave_sum_f64(v); }

// Krylov basis vectors (V_j in the projections and updates, Z_j in the combination) are
// loaded with the non-temporal hint: at 2h the K_2h basis alone is up to 0.5 GB, and
// streaming it through the last-level cache evicted the velocity, D^-1 and V-cycle vectors
// the next preconditioner call reads (352^3 solve: 0.2512 -> 0.2468 s).
__device__ __forceinline__ c32 ldnt(const c32 *p) {
    const long long v = __builtin_nontemporal_load(reinterpret_cast<const long long *>(p));
    c32 o;
    o.re = __int_as_float((int)v);
    o.im = __int_as_float((int)(v >> 32));
    return o;
}
__device__ __forceinline__ c16 ldnt(const c16 *p) {
    const unsigned v = __builtin_nontemporal_load(reinterpret_cast<const unsigned *>(p));
    c16 o;
    o.re = __builtin_bit_cast(_Float16, (unsigned short)(v & 0xffffu));
    o.im = __builtin_bit_cast(_Float16, (unsigned short)(v >> 16));
    return o;
}
__device__ __forceinline__ c64 ldnt(const c64 *p) {
    c64 o;
    o.re = __builtin_nontemporal_load(&p->re);
    o.im = __builtin_nontemporal_load(&p->im);
    return o;
}

// Elementwise kernels run one thread per element over a full grid: measured on
// fine-level vectors this streams faster than any grid-stride loop, with or
// without several elements in flight per thread, because the blocks then sweep
// memory in order.  Reductions keep a grid-stride loop over a fixed number of
// blocks (one element per step: unrolled steps measured slower).
__device__ __forceinline__ long long elem_index() { return blockIdx.x * (long long)blockDim.x + threadIdx.x; }

// Block-reduce NS complex sums, store them as this block's partials, then
// return true in the last block to arrive (which may read every block's partials).
constexpr int kRedThreads = 1024;      // threads per reduction block (16 wavefronts)
constexpr int kRedWaves = kRedThreads / 64;

template <int NS>
__device__ bool reduce_partials(D2 (&acc)[NS], const RedBuf &rb) {
    __shared__ double red[kRedWaves][2 * kSlots];
    __shared__ bool last;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        double r = wave_sum(acc[s].r), i = wave_sum(acc[s].i);
        if (lane == 0) {
            red[w][2 * s] = r;
            red[w][2 * s + 1] = i;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * NS) {
        double v = 0.0;
        for (int k = 0; k < kRedWaves; ++k) v += red[k][threadIdx.x];
        partial_store(rb.partials + (size_t)blockIdx.x * 2 * kSlots + threadIdx.x, v);
        stores_done();
    }
    __syncthreads();
    if (threadIdx.x == 0) last = take_ticket(rb.counter, gridDim.x);
    __syncthreads();
    return last;
}

// In the last block: total of every slot over all blocks, in a fixed order.
// Thread t owns slot q = t % (2 NS) and the blocks b = t / (2 NS) + k * G
// (G = blockDim / (2 NS) groups); its loads are independent and unrolled, then
// the G group sums are added in order.
template <int NS>
__device__ void sum_partials(const RedBuf &rb, D2 *out) {
    constexpr int NQ = 2 * NS;
    constexpr int G = kRedThreads / NQ > 0 ? kRedThreads / NQ : 1;
    __shared__ double grp[kRedThreads];
    const int nb = gridDim.x;
    const int t = threadIdx.x;
    double v = 0.0;
    if (t < G * NQ) {
        const int q = t % NQ, g0 = t / NQ;
#pragma unroll 8
        for (int b = g0; b < nb; b += G) v += partial_load(rb.partials + (size_t)b * 2 * kSlots + q);
    }
    grp[t] = v;
    __syncthreads();
    if (t < NQ) {
        double s = 0.0;
        for (int g = 0; g < G; ++g) s += grp[g * NQ + t];
        if (t & 1)
            out[t >> 1].i = s;
        else
            out[t >> 1].r = s;
    }
    __syncthreads();
}

__device__ void state_init(KState *st, double beta) {
    st->beta = beta;
    st->scale = (beta > 0.0) ? 1.0 / beta : 0.0;
    st->vs0 = st->scale;   // the residual itself stays the stored first basis vector
    st->kk = 0;
    st->breakdown = 0;
    st->nonfinite = !(beta == beta && beta < 1e300);
    for (int j = 0; j <= kMMax; ++j) st->g[j][0] = st->g[j][1] = 0.0;
    st->g[0][0] = beta;
}

// Column k of the Hessenberg matrix: cr (k+1 entries, rotated in place) and
// h_{k+1,k}; apply the previous rotations, build the one annihilating h_{k+1,k},
// rotate g.  One thread runs it; cr lives in LDS so that the loops with a
// run-time bound need no private (scratch) array and add nothing to the
// register budget of the streaming loop that precedes the epilogue.
__device__ void givens_column(KState *st, int k, double (*cr)[2], double hk1) {
    for (int j = 0; j < k; ++j) {
        const double c = st->cs[j], sr = st->sn[j][0], si = st->sn[j][1];
        const double ar = cr[j][0], ai = cr[j][1], br = cr[j + 1][0], bi = cr[j + 1][1];
        // [c s; -conj(s) c] [a; b]
        cr[j][0] = c * ar + (sr * br - si * bi);
        cr[j][1] = c * ai + (sr * bi + si * br);
        cr[j + 1][0] = -(sr * ar + si * ai) + c * br;
        cr[j + 1][1] = -(sr * ai - si * ar) + c * bi;
    }
    const double ar = cr[k][0], ai = cr[k][1];
    const double aa = sqrt(ar * ar + ai * ai);
    const double rr = sqrt(aa * aa + hk1 * hk1);
    double c, sr, si;
    if (rr == 0.0) {
        c = 1.0; sr = 0.0; si = 0.0;
    } else if (aa == 0.0) {
        c = 0.0; sr = 1.0; si = 0.0;
    } else {
        c = aa / rr;
        sr = (ar / aa) * hk1 / rr;
        si = (ai / aa) * hk1 / rr;
    }
    st->cs[k] = c;
    st->sn[k][0] = sr;
    st->sn[k][1] = si;
    cr[k][0] = c * ar + sr * hk1;
    cr[k][1] = c * ai + si * hk1;
    for (int j = 0; j <= k; ++j) {
        st->H[j][k][0] = cr[j][0];
        st->H[j][k][1] = cr[j][1];
    }
    const double gr = st->g[k][0], gi = st->g[k][1];
    st->g[k + 1][0] = -(sr * gr + si * gi);
    st->g[k + 1][1] = -(sr * gi - si * gr);
    st->g[k][0] = c * gr;
    st->g[k][1] = c * gi;
    st->kk = k + 1;
    st->hk1 = hk1;
    // h_{k+1,k} and ||w|| carry the same scale (also in column 0, built from the
    // unnormalised first vector), so the test is scale-free
    const bool ok = hk1 > kBreakdown * st->wn;
    st->scale = ok ? 1.0 / hk1 : 0.0;
    if (!ok) st->breakdown = 1;
    if (!(hk1 == hk1) || !(st->g[k + 1][0] == st->g[k + 1][0])) st->nonfinite = 1;
}

// ---------------------------------------------------------------------------

template <typename T, int NV>
struct Ptrs {
    const T *v[NV > 0 ? NV : 1];
};

// sums conj(V_j) w (j < NV) and optionally ||w||^2
template <typename T, int NV, bool NORM, int EPI>
__global__ void __launch_bounds__(1024) k_dots(Ptrs<T, NV> P, const T *__restrict__ w, long long n, KState *st,
                                             double *out, RedBuf rb, Batch bt) {
    const int sl = blockIdx.y;
    if (slot_off(bt, sl)) return;
#pragma unroll
    for (int j = 0; j < NV; ++j) P.v[j] = slot_ptr(P.v[j], n, sl);
    w = slot_ptr(w, n, sl);
    st = slot_ptr(st, 1, sl);
    out = slot_ptr(out, 2 * kSlots, sl);
    rb = slot_rb(rb, bt, sl);
    constexpr int NS0 = NV + (NORM ? 1 : 0);
    constexpr int NS = NS0 > 0 ? NS0 : 1;
    D2 acc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] = {0, 0};
    for (long long i = elem_index(); i < n; i += (long long)gridDim.x * blockDim.x) {
        const T wi = w[i];
#pragma unroll
        for (int j = 0; j < NV; ++j) acc[j] = acc[j] + cdot(ldnt(P.v[j] + i), wi);
        if (NORM) acc[NV] = acc[NV] + D2{(double)wi.re * wi.re + (double)wi.im * wi.im, 0.0};
    }
    if (!reduce_partials<NS>(acc, rb)) return;
    __shared__ D2 tot[kSlots];
    sum_partials<NS>(rb, tot);
    if (threadIdx.x == 0) {
        if (EPI == EPI_STORE) {
            for (int s = 0; s < NS; ++s) {
                out[2 * s] = tot[s].r;
                out[2 * s + 1] = tot[s].i;
            }
        } else if (EPI == EPI_ARNOLDI1) {
            if (NV > 0) tot[0] = {tot[0].r * st->vs0, tot[0].i * st->vs0};   // onto the normalised V_0
            for (int j = 0; j < NV; ++j) {
                st->h1[j][0] = tot[j].r;
                st->h1[j][1] = tot[j].i;
            }
            st->reorth = 1;
            st->wn = 0.0;   // no norm in this pass: only an exactly vanishing w - V h counts as breakdown
        } else if (EPI == EPI_ARNOLDI_SEL && NV > 0) {
            // selective second pass: if the first projection keeps at least
            // kReorthEta of ||w||^2, w - V h1 is orthogonal to a few units of
            // roundoff and the second pass is skipped.
            __shared__ double col[kMMax + 1][2];
            tot[0] = {tot[0].r * st->vs0, tot[0].i * st->vs0};   // onto the normalised V_0
            double c2 = 0.0;
            for (int j = 0; j < NV; ++j) {
                st->h1[j][0] = col[j][0] = tot[j].r;
                st->h1[j][1] = col[j][1] = tot[j].i;
                c2 += tot[j].r * tot[j].r + tot[j].i * tot[j].i;
            }
            const double w2 = tot[NS - 1].r, r2 = w2 - c2;
            st->wn = sqrt(w2);
            if (r2 >= kReorthEta * w2) {
                for (int j = 0; j < NV; ++j) {
                    st->h2[j][0] = tot[j].r;
                    st->h2[j][1] = tot[j].i;
                }
                st->reorth = 0;
                givens_column(st, NV - 1, col, sqrt(r2));
            } else {
                st->reorth = 1;
            }
        } else if (EPI == EPI_NORM_INIT) {
            state_init(st, sqrt(tot[NS - 1].r));
        }
        reset_ticket(rb.counter);
    }
}

// w <- w - sum_j h1_j V_j; then conj(V_j) w and ||w||^2; Givens update of column NV-1.
// Without STORE the corrected w is not written back: the last Arnoldi step of a
// cycle needs only the Hessenberg column and h_{k+1,k}, not the next basis vector.
template <typename T, int NV, bool STORE>
__global__ void __launch_bounds__(1024) k_axpy_dots(Ptrs<T, NV> P, T *__restrict__ w, long long n, KState *st,
                                                  RedBuf rb, Batch bt) {
    const int sl = blockIdx.y;
    if (slot_off(bt, sl)) return;
    st = slot_ptr(st, 1, sl);
    if (!st->reorth) return;   // the first pass was enough (the slot's blocks return; no ticket is taken)
#pragma unroll
    for (int j = 0; j < NV; ++j) P.v[j] = slot_ptr(P.v[j], n, sl);
    w = slot_ptr(w, n, sl);
    rb = slot_rb(rb, bt, sl);
    __shared__ double hs[NV][2];
    if (threadIdx.x < NV) {   // coefficients of the stored vectors (V_0 is stored unnormalised)
        const double f = threadIdx.x == 0 ? st->vs0 : 1.0;
        hs[threadIdx.x][0] = st->h1[threadIdx.x][0] * f;
        hs[threadIdx.x][1] = st->h1[threadIdx.x][1] * f;
    }
    __syncthreads();
    real_of<T> hr[NV], hi[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        hr[j] = (real_of<T>)hs[j][0];
        hi[j] = (real_of<T>)hs[j][1];
    }
    D2 acc[NV + 1];
#pragma unroll
    for (int s = 0; s <= NV; ++s) acc[s] = {0, 0};
    for (long long i = elem_index(); i < n; i += (long long)gridDim.x * blockDim.x) {
        T v[NV];
        T wi = w[i];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            v[j] = ldnt(P.v[j] + i);
            wi.re -= hr[j] * v[j].re - hi[j] * v[j].im;
            wi.im -= hr[j] * v[j].im + hi[j] * v[j].re;
        }
        if (STORE) w[i] = wi;
#pragma unroll
        for (int j = 0; j < NV; ++j) acc[j] = acc[j] + cdot(v[j], wi);
        acc[NV] = acc[NV] + D2{(double)wi.re * wi.re + (double)wi.im * wi.im, 0.0};
    }
    if (!reduce_partials<NV + 1>(acc, rb)) return;
    __shared__ D2 tot[kSlots];
    sum_partials<NV + 1>(rb, tot);
    if (threadIdx.x == 0) {
        __shared__ double col[kMMax + 1][2];
        tot[0] = {tot[0].r * st->vs0, tot[0].i * st->vs0};   // onto the normalised V_0
        double c2 = 0.0;
        for (int j = 0; j < NV; ++j) {
            st->h2[j][0] = tot[j].r;
            st->h2[j][1] = tot[j].i;
            col[j][0] = st->h1[j][0] + tot[j].r;
            col[j][1] = st->h1[j][1] + tot[j].i;
            c2 += tot[j].r * tot[j].r + tot[j].i * tot[j].i;
        }
        // ||w - V h2||^2 = ||w||^2 - ||h2||^2 for orthonormal V
        const double hk1 = sqrt(fmax(tot[NV].r - c2, 0.0));
        givens_column(st, NV - 1, col, hk1);
        reset_ticket(rb.counter);
    }
}

// w <- (w - sum_j h2_j V_j) * scale
template <typename T, int NV>
__global__ void __launch_bounds__(256) k_axpy_scale(Ptrs<T, NV> P, T *__restrict__ w, long long n, const KState *st,
                                                   Batch bt) {
    const int sl = blockIdx.y;
    if (slot_off(bt, sl)) return;
#pragma unroll
    for (int j = 0; j < NV; ++j) P.v[j] = slot_ptr(P.v[j], n, sl);
    w = slot_ptr(w, n, sl);
    st = slot_ptr(st, 1, sl);
    __shared__ double hs[NV + 1][2];
    if (threadIdx.x < NV) {   // coefficients of the stored vectors (V_0 is stored unnormalised)
        const double f = threadIdx.x == 0 ? st->vs0 : 1.0;
        hs[threadIdx.x][0] = st->h2[threadIdx.x][0] * f;
        hs[threadIdx.x][1] = st->h2[threadIdx.x][1] * f;
    }
    if (threadIdx.x == 0) hs[NV][0] = st->scale;
    __syncthreads();
    real_of<T> hr[NV], hi[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        hr[j] = (real_of<T>)hs[j][0];
        hi[j] = (real_of<T>)hs[j][1];
    }
    const real_of<T> sc = (real_of<T>)hs[NV][0];
    const long long i = elem_index();
    if (i >= n) return;
    T wi = w[i];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const T v = ldnt(P.v[j] + i);
        wi.re -= hr[j] * v.re - hi[j] * v.im;
        wi.im -= hr[j] * v.im + hi[j] * v.re;
    }
    wi.re *= sc;
    wi.im *= sc;
    w[i] = wi;
}

// y = R^{-1} g: back substitution of the rotated Hessenberg over its kk columns
// (guarded zero pivots), y_j = 0 beyond; one thread.
__global__ void __launch_bounds__(64) k_backsolve(KState *st, int nv, Batch bt) {
    if (threadIdx.x != 0 || slot_off(bt, blockIdx.y)) return;
    st = slot_ptr(st, 1, blockIdx.y);
    const int kk = st->kk < nv ? st->kk : nv;
    for (int j = kk; j < kMMax; ++j) st->y[j][0] = st->y[j][1] = 0.0;
    for (int i = kk - 1; i >= 0; --i) {
        double sr = st->g[i][0], si = st->g[i][1];
        for (int j = i + 1; j < kk; ++j) {
            const double hr = st->H[i][j][0], hi = st->H[i][j][1];
            sr -= hr * st->y[j][0] - hi * st->y[j][1];
            si -= hr * st->y[j][1] + hi * st->y[j][0];
        }
        const double dr = st->H[i][i][0], di = st->H[i][i][1];
        const double d2 = dr * dr + di * di;
        if (d2 == 0.0) {
            st->y[i][0] = st->y[i][1] = 0.0;
        } else {
            st->y[i][0] = (sr * dr + si * di) / d2;
            st->y[i][1] = (si * dr - sr * di) / d2;
        }
    }
}

// x (+)= sum_j y_j Z_j with y from st->y (written by k_backsolve or by the
// s-step Gram solve)
template <typename TX, typename TZ, int NV>
__global__ void __launch_bounds__(256) k_combine(TX *__restrict__ x, Ptrs<TZ, NV> Zp, long long n, const KState *st,
                                                int overwrite, float zf, Batch bt) {
    const int sl = blockIdx.y;
    if (slot_off(bt, sl)) return;
#pragma unroll
    for (int j = 0; j < NV; ++j) Zp.v[j] = slot_ptr(Zp.v[j], n, sl);
    x = slot_ptr(x, n, sl);
    st = slot_ptr(st, 1, sl);
    using RA = std::conditional_t<is_half<TX>(), float, real_of<TX>>;   // FP16-stored x adds in FP32
    __shared__ double ys[NV][2];
    if (threadIdx.x < NV) {
        // c16 Z into a c32 / c64 x: the coefficient takes Z_j's inverse scale 1 / (zf qs_j)
        double w = 1.0;
        if (is_half<TZ>() && !is_half<TX>()) {
            const double d = (double)zf * (threadIdx.x == 0 ? st->vs0 : 1.0);
            w = d != 0.0 ? 1.0 / d : 0.0;
        }
        ys[threadIdx.x][0] = st->y[threadIdx.x][0] * w;
        ys[threadIdx.x][1] = st->y[threadIdx.x][1] * w;
    }
    __syncthreads();
    RA yr[NV], yi[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        yr[j] = (RA)ys[j][0];
        yi[j] = (RA)ys[j][1];
    }
    const long long i = elem_index();
    if (i >= n) return;
    RA ar = 0, ai = 0;
    if (!overwrite) {
        const TX v = x[i];
        ar = (RA)v.re;
        ai = (RA)v.im;
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const TZ z = ldnt(Zp.v[j] + i);
        const RA zr = (RA)z.re, zi = (RA)z.im;
        ar += yr[j] * zr - yi[j] * zi;
        ai += yr[j] * zi + yi[j] * zr;
    }
    x[i] = to_stored<TX, RA>(ar, ai, (RA)1);
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_convert_scaled(const TI *__restrict__ x, TO *__restrict__ y, long long n,
                                                       Scale si, Scale so, Batch bt) {
    const int sl = blockIdx.y;
    if (slot_off(bt, sl)) return;
    x = slot_ptr(x, n, sl);
    y = slot_ptr(y, n, sl);
    si = slot_scale(si, sl);
    so = slot_scale(so, sl);
    using RA = std::conditional_t<is_half<TO>(), float, real_of<TO>>;
    const long long i = elem_index();
    if (i >= n) return;
    const RA mi = load_mul<RA, TI>(si), mo = store_mul<RA, TO>(so);
    const TI v = x[i];
    y[i] = to_stored<TO, RA>((RA)v.re * mi, (RA)v.im * mi, mo);
}

// Gram matrix G_ij = <P_i, P_j> (i <= j) of the s-step basis P_0..P_{NP-1}, then
// the least-squares coefficients y of min ||P_0 - [P_1..P_{NP-1}] y|| from the
// normal equations by Cholesky (truncated at a vanishing pivot).
template <typename T, int NP>
__global__ void __launch_bounds__(1024) k_gram(Ptrs<T, NP> P, long long n, KState *st, RedBuf rb, Batch bt) {
    const int sl = blockIdx.y;
    if (slot_off(bt, sl)) return;
#pragma unroll
    for (int a = 0; a < NP; ++a) P.v[a] = slot_ptr(P.v[a], n, sl);
    st = slot_ptr(st, 1, sl);
    rb = slot_rb(rb, bt, sl);
    constexpr int NS = NP * (NP + 1) / 2;
    D2 acc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] = {0, 0};
    for (long long i = elem_index(); i < n; i += (long long)gridDim.x * blockDim.x) {
        T v[NP];
#pragma unroll
        for (int a = 0; a < NP; ++a) v[a] = P.v[a][i];
        int s = 0;
#pragma unroll
        for (int a = 0; a < NP; ++a)
#pragma unroll
            for (int b = a; b < NP; ++b) {
                acc[s] = acc[s] + cdot(v[a], v[b]);
                ++s;
            }
    }
    if (!reduce_partials<NS>(acc, rb)) return;
    __shared__ D2 tot[kSlots];
    sum_partials<NS>(rb, tot);
    // the small dense solve runs on one thread with its arrays in LDS
    // (dynamically indexed arrays in registers would go to scratch memory)
    constexpr int m = NP - 1;
    __shared__ double G[NP][NP][2];
    __shared__ double Lr[m][m], Li[m][m], ur[m], ui[m];
    if (threadIdx.x == 0) {
        int s = 0;
        for (int a = 0; a < NP; ++a)
            for (int b = a; b < NP; ++b) {
                G[a][b][0] = tot[s].r;
                G[a][b][1] = tot[s].i;
                G[b][a][0] = tot[s].r;
                G[b][a][1] = -tot[s].i;
                ++s;
            }
        int rank = m;
        for (int j = 0; j < m && rank == m; ++j) {
            double d = G[j + 1][j + 1][0];
            for (int k = 0; k < j; ++k) d -= Lr[j][k] * Lr[j][k] + Li[j][k] * Li[j][k];
            if (!(d > 1e-24 * G[j + 1][j + 1][0])) {
                rank = j;
                break;
            }
            const double ljj = sqrt(d);
            Lr[j][j] = ljj;
            Li[j][j] = 0.0;
            for (int i = j + 1; i < m; ++i) {
                double ar = G[i + 1][j + 1][0], ai = G[i + 1][j + 1][1];
                for (int k = 0; k < j; ++k) {   // - L_ik conj(L_jk)
                    ar -= Lr[i][k] * Lr[j][k] + Li[i][k] * Li[j][k];
                    ai -= Li[i][k] * Lr[j][k] - Lr[i][k] * Li[j][k];
                }
                Lr[i][j] = ar / ljj;
                Li[i][j] = ai / ljj;
            }
        }
        for (int i = 0; i < rank; ++i) {   // L u = rhs, rhs_i = <P_{i+1}, P_0>
            double ar = G[i + 1][0][0], ai = G[i + 1][0][1];
            for (int k = 0; k < i; ++k) {
                ar -= Lr[i][k] * ur[k] - Li[i][k] * ui[k];
                ai -= Lr[i][k] * ui[k] + Li[i][k] * ur[k];
            }
            ur[i] = ar / Lr[i][i];
            ui[i] = ai / Lr[i][i];
        }
        for (int j = 0; j < kMMax; ++j) st->y[j][0] = st->y[j][1] = 0.0;
        for (int i = rank - 1; i >= 0; --i) {   // L^H y = u
            double ar = ur[i], ai = ui[i];
            for (int k = i + 1; k < rank; ++k) {   // - conj(L_ki) y_k
                ar -= Lr[k][i] * st->y[k][0] + Li[k][i] * st->y[k][1];
                ai -= Lr[k][i] * st->y[k][1] - Li[k][i] * st->y[k][0];
            }
            st->y[i][0] = ar / Lr[i][i];
            st->y[i][1] = ai / Lr[i][i];
        }
        if (!(G[0][0][0] == G[0][0][0]) || !(G[0][0][0] < 1e300)) st->nonfinite = 1;
        reset_ticket(rb.counter);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_fill_zero(T *x, long long n, Batch bt) {
    if (slot_off(bt, blockIdx.y)) return;
    x = slot_ptr(x, n, blockIdx.y);
    const long long i = elem_index();
    if (i >= n) return;
    T z;
    z.re = 0;
    z.im = 0;
    x[i] = z;
}

template <typename T>
__global__ void __launch_bounds__(256) k_add(const T *__restrict__ x, T *__restrict__ y, long long n, Batch bt) {
    if (slot_off(bt, blockIdx.y)) return;
    x = slot_ptr(x, n, blockIdx.y);
    y = slot_ptr(y, n, blockIdx.y);
    const long long i = elem_index();
    if (i >= n) return;
    T v = y[i];
    const T a = x[i];
    v.re += a.re;
    v.im += a.im;
    y[i] = v;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_convert(const TI *__restrict__ x, TO *__restrict__ y, long long n, Batch bt) {
    if (slot_off(bt, blockIdx.y)) return;
    x = slot_ptr(x, n, blockIdx.y);
    y = slot_ptr(y, n, blockIdx.y);
    const long long i = elem_index();
    if (i >= n) return;
    TO o;
    o.re = (real_of<TO>)x[i].re;
    o.im = (real_of<TO>)x[i].im;
    y[i] = o;
}

// velocity on the nodes of one level: nearest physical value in the PML
// (Sec. 2.1), sampled at every stride-th fine node (Sec. 3.1)
__global__ void __launch_bounds__(256) k_extend_velocity(const float *__restrict__ phys, int nxp, int nyp, int nzp,
                                                        int n_pml, int stride, Geom g, float *__restrict__ out) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.nn; i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % g.sx);
        const int y = (int)((i / g.sx) % (g.n[1] + 1));
        const int z = (int)(i / g.sy);
        const int px = min(max(x * stride - n_pml, 0), nxp);
        const int py = min(max(y * stride - n_pml, 0), nyp);
        const int pz = min(max(z * stride - n_pml, 0), nzp);
        out[i] = phys[((long long)pz * (nyp + 1) + py) * (nxp + 1) + px];
    }
}

__global__ void __launch_bounds__(256) k_scaled_eta(const float *__restrict__ c, long long n, double factor,
                                                   float *__restrict__ out) {
    const long long i = elem_index();
    if (i < n) out[i] = (float)(factor / (double)c[i]);
}

// min, max and the count of non-finite values of the velocity
__global__ void __launch_bounds__(256) k_velocity_check(const float *__restrict__ v, long long n, RedBuf rb,
                                                       double *out) {
    double mn = 1e300, mx = -1e300, bad = 0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float c = v[i];
        if (!(c == c) || c > 3.0e38f || c < -3.0e38f) {
            bad += 1;
        } else {
            mn = fmin(mn, (double)c);
            mx = fmax(mx, (double)c);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        mn = fmin(mn, __shfl_xor(mn, off, 64));
        mx = fmax(mx, __shfl_xor(mx, off, 64));
        bad += __shfl_xor(bad, off, 64);
    }
    __shared__ double red[4][3];
    __shared__ bool last;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red[w][0] = mn;
        red[w][1] = mx;
        red[w][2] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; ++k) {
            red[0][0] = fmin(red[0][0], red[k][0]);
            red[0][1] = fmax(red[0][1], red[k][1]);
            red[0][2] += red[k][2];
        }
        partial_store(rb.partials + 3 * blockIdx.x + 0, red[0][0]);
        partial_store(rb.partials + 3 * blockIdx.x + 1, red[0][1]);
        partial_store(rb.partials + 3 * blockIdx.x + 2, red[0][2]);
        stores_done();
        last = take_ticket(rb.counter, gridDim.x);
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        double a = 1e300, b = -1e300, c = 0;
        for (unsigned k = 0; k < gridDim.x; ++k) {
            a = fmin(a, partial_load(rb.partials + 3 * k));
            b = fmax(b, partial_load(rb.partials + 3 * k + 1));
            c += partial_load(rb.partials + 3 * k + 2);
        }
        out[0] = a;
        out[1] = b;
        out[2] = c;
        reset_ticket(rb.counter);
    }
}

// blocks of a reduction: at least ~4 elements per thread, so that small (cache
// resident) vectors spend their time on loads rather than on block reductions
int red_blocks(long long n) {
    long long b = (n + 4 * kRedThreads - 1) / (4 * kRedThreads);
    if (b < 1) b = 1;
    if (b > kRedMaxBlocks) b = kRedMaxBlocks;
    return (int)b;
}

// blocks of an elementwise kernel: one thread per element, 256 per block
unsigned stream_blocks(long long n) {
    long long b = (n + 255) / 256;
    if (b < 1) b = 1;
    return (unsigned)b;
}

template <typename T, int NV>
Ptrs<T, NV> pack(const T *const *V) {
    Ptrs<T, NV> p{};
    for (int j = 0; j < NV; ++j) p.v[j] = V[j];
    return p;
}

}  // namespace

template <typename T>
hipError_t launch_dots(const T *const *V, int nv, const T *w, bool norm, long long n, int epi, KState *st, int k,
                       double *out, const RedBuf &rb, hipStream_t s) {
    (void)k;
    const int nb = red_blocks(n);
#define HELM_DOTS(NV)                                                                                               \
    case NV:                                                                                                        \
        if (norm) {                                                                                                 \
            if (epi == EPI_STORE)                                                                                   \
                hipLaunchKernelGGL((k_dots<T, NV, true, EPI_STORE>), dim3(nb, cur_batch().n), dim3(kRedThreads), 0, s, pack<T, NV>(V), w, n, \
                                   st, out, rb, cur_batch());                                                                    \
            else if (epi == EPI_NORM_INIT)                                                                          \
                hipLaunchKernelGGL((k_dots<T, NV, true, EPI_NORM_INIT>), dim3(nb, cur_batch().n), dim3(kRedThreads), 0, s, pack<T, NV>(V), \
                                   w, n, st, out, rb, cur_batch());                                                              \
            else if (epi == EPI_ARNOLDI_SEL && NV > 0)                                                              \
                hipLaunchKernelGGL((k_dots<T, NV, true, EPI_ARNOLDI_SEL>), dim3(nb, cur_batch().n), dim3(kRedThreads), 0, s,         \
                                   pack<T, NV>(V), w, n, st, out, rb, cur_batch());                                              \
            else                                                                                                    \
                return hipErrorInvalidValue;                                                                        \
        } else {                                                                                                    \
            if (epi == EPI_STORE)                                                                                   \
                hipLaunchKernelGGL((k_dots<T, NV, false, EPI_STORE>), dim3(nb, cur_batch().n), dim3(kRedThreads), 0, s, pack<T, NV>(V), w, \
                                   n, st, out, rb, cur_batch());                                                                 \
            else if (epi == EPI_ARNOLDI1)                                                                           \
                hipLaunchKernelGGL((k_dots<T, NV, false, EPI_ARNOLDI1>), dim3(nb, cur_batch().n), dim3(kRedThreads), 0, s, pack<T, NV>(V), \
                                   w, n, st, out, rb, cur_batch());                                                              \
            else                                                                                                    \
                return hipErrorInvalidValue;                                                                        \
        }                                                                                                           \
        break;
    switch (nv) {
        HELM_DOTS(0) HELM_DOTS(1) HELM_DOTS(2) HELM_DOTS(3) HELM_DOTS(4) HELM_DOTS(5) HELM_DOTS(6) HELM_DOTS(7)
        HELM_DOTS(8) HELM_DOTS(9) HELM_DOTS(10) HELM_DOTS(11) HELM_DOTS(12)
    default:
        return hipErrorInvalidValue;
    }
#undef HELM_DOTS
    return hipGetLastError();
}

template <typename T>
hipError_t launch_axpy_dots(const T *const *V, int nv, T *w, long long n, KState *st, const RedBuf &rb,
                            hipStream_t s, bool store) {
    const int nb = red_blocks(n);
#define HELM_AD(NV)                                                                                                \
    case NV:                                                                                                       \
        if (store)                                                                                                 \
            hipLaunchKernelGGL((k_axpy_dots<T, NV, true>), dim3(nb, cur_batch().n), dim3(kRedThreads), 0, s, pack<T, NV>(V), w, n, \
                               st, rb, cur_batch());                                                               \
        else                                                                                                       \
            hipLaunchKernelGGL((k_axpy_dots<T, NV, false>), dim3(nb, cur_batch().n), dim3(kRedThreads), 0, s, pack<T, NV>(V), w,  \
                               n, st, rb, cur_batch());                                                            \
        break;
    switch (nv) {
        HELM_AD(1) HELM_AD(2) HELM_AD(3) HELM_AD(4) HELM_AD(5) HELM_AD(6) HELM_AD(7) HELM_AD(8) HELM_AD(9)
        HELM_AD(10) HELM_AD(11) HELM_AD(12)
    default:
        return hipErrorInvalidValue;
    }
#undef HELM_AD
    return hipGetLastError();
}

template <typename T>
hipError_t launch_axpy_scale(const T *const *V, int nv, T *w, long long n, KState *st, hipStream_t s) {
    const unsigned nb = stream_blocks(n);
#define HELM_AS(NV) \
    case NV: hipLaunchKernelGGL((k_axpy_scale<T, NV>), dim3(nb, cur_batch().n), dim3(256), 0, s, pack<T, NV>(V), w, n, st, cur_batch()); break;
    switch (nv) {
        HELM_AS(1) HELM_AS(2) HELM_AS(3) HELM_AS(4) HELM_AS(5) HELM_AS(6) HELM_AS(7) HELM_AS(8) HELM_AS(9)
        HELM_AS(10) HELM_AS(11) HELM_AS(12)
    default:
        return hipErrorInvalidValue;
    }
#undef HELM_AS
    return hipGetLastError();
}

template <typename TX, typename TZ>
hipError_t launch_combine(TX *x, const TZ *const *Z, int nz, long long n, KState *st, bool from_backsolve,
                          bool overwrite, hipStream_t s, float zf) {
    if (nz < 1 || nz > kMMax) return hipErrorInvalidValue;
    if (from_backsolve) {
        hipLaunchKernelGGL(k_backsolve, dim3(1, cur_batch().n), dim3(64), 0, s, st, nz, cur_batch());
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const unsigned nb = stream_blocks(n);
#define HELM_CB(NV)                                                                                            \
    case NV:                                                                                                   \
        hipLaunchKernelGGL((k_combine<TX, TZ, NV>), dim3(nb, cur_batch().n), dim3(256), 0, s, x, pack<TZ, NV>(Z), n, st,       \
                           (int)overwrite, zf, cur_batch());                                                                \
        break;
    switch (nz) {
        HELM_CB(1) HELM_CB(2) HELM_CB(3) HELM_CB(4) HELM_CB(5) HELM_CB(6) HELM_CB(7) HELM_CB(8) HELM_CB(9)
        HELM_CB(10) HELM_CB(11) HELM_CB(12)
    default:
        return hipErrorInvalidValue;
    }
#undef HELM_CB
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gram(const T *const *P, int np, long long n, KState *st, const RedBuf &rb, hipStream_t s) {
    const int nb = red_blocks(n);
#define HELM_GR(NP) \
    case NP: hipLaunchKernelGGL((k_gram<T, NP>), dim3(nb, cur_batch().n), dim3(kRedThreads), 0, s, pack<T, NP>(P), n, st, rb, cur_batch()); break;
    switch (np) {
        HELM_GR(2) HELM_GR(3) HELM_GR(4) HELM_GR(5) HELM_GR(6) HELM_GR(7) HELM_GR(8) HELM_GR(9)
    default:
        return hipErrorInvalidValue;
    }
#undef HELM_GR
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_zero(T *x, long long n, hipStream_t s) {
    hipLaunchKernelGGL((k_fill_zero<T>), dim3(stream_blocks(n), cur_batch().n), dim3(256), 0, s, x, n, cur_batch());
    return hipGetLastError();
}

template <typename T>
hipError_t launch_add(const T *x, T *y, long long n, hipStream_t s) {
    hipLaunchKernelGGL((k_add<T>), dim3(stream_blocks(n), cur_batch().n), dim3(256), 0, s, x, y, n, cur_batch());
    return hipGetLastError();
}

template <typename TI, typename TO>
hipError_t launch_convert(const TI *x, TO *y, long long n, hipStream_t s) {
    hipLaunchKernelGGL((k_convert<TI, TO>), dim3(stream_blocks(n), cur_batch().n), dim3(256), 0, s, x, y, n, cur_batch());
    return hipGetLastError();
}

hipError_t launch_extend_velocity(const float *phys, const int nphys[3], int n_pml, int stride, const Geom &g,
                                  float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_extend_velocity, dim3(stream_blocks(g.nn)), dim3(256), 0, s, phys, nphys[0], nphys[1],
                       nphys[2], n_pml, stride, g, out);
    return hipGetLastError();
}

hipError_t launch_scaled_eta(const float *c, long long n, double factor, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_scaled_eta, dim3(stream_blocks(n)), dim3(256), 0, s, c, n, factor, out);
    return hipGetLastError();
}

hipError_t launch_velocity_check(const float *v, long long n, const RedBuf &rb, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_velocity_check, dim3(red_blocks(n)), dim3(256), 0, s, v, n, rb, out);
    return hipGetLastError();
}

#define HELM_INST(T)                                                                                              \
    template hipError_t launch_dots<T>(const T *const *, int, const T *, bool, long long, int, KState *, int,     \
                                       double *, const RedBuf &, hipStream_t);                                    \
    template hipError_t launch_axpy_dots<T>(const T *const *, int, T *, long long, KState *, const RedBuf &,      \
                                            hipStream_t, bool);                                                   \
    template hipError_t launch_axpy_scale<T>(const T *const *, int, T *, long long, KState *, hipStream_t);       \
    template hipError_t launch_gram<T>(const T *const *, int, long long, KState *, const RedBuf &, hipStream_t); \
    template hipError_t launch_fill_zero<T>(T *, long long, hipStream_t);                                      \
    template hipError_t launch_add<T>(const T *, T *, long long, hipStream_t);
HELM_INST(c32)
HELM_INST(c64)
#undef HELM_INST
template hipError_t launch_combine<c32, c32>(c32 *, const c32 *const *, int, long long, KState *, bool, bool,
                                             hipStream_t, float);
template hipError_t launch_combine<c64, c64>(c64 *, const c64 *const *, int, long long, KState *, bool, bool,
                                             hipStream_t, float);
template hipError_t launch_combine<c64, c32>(c64 *, const c32 *const *, int, long long, KState *, bool, bool,
                                             hipStream_t, float);
template hipError_t launch_combine<c32, c16>(c32 *, const c16 *const *, int, long long, KState *, bool, bool,
                                             hipStream_t, float);
template hipError_t launch_combine<c16, c16>(c16 *, const c16 *const *, int, long long, KState *, bool, bool,
                                             hipStream_t, float);
template hipError_t launch_gram<c16>(const c16 *const *, int, long long, KState *, const RedBuf &, hipStream_t);

template <typename TI, typename TO>
hipError_t launch_convert_scaled(const TI *x, TO *y, long long n, Scale si, Scale so, hipStream_t s) {
    if ((is_half<TI>() && !si.qs) || (is_half<TO>() && !so.qs)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_convert_scaled<TI, TO>), dim3(stream_blocks(n), cur_batch().n), dim3(256), 0, s, x, y, n, si,
                       so, cur_batch());
    return hipGetLastError();
}
template hipError_t launch_convert_scaled<c32, c16>(const c32 *, c16 *, long long, Scale, Scale, hipStream_t);
template hipError_t launch_convert_scaled<c16, c32>(const c16 *, c32 *, long long, Scale, Scale, hipStream_t);
template hipError_t launch_convert<c32, c64>(const c32 *, c64 *, long long, hipStream_t);
template hipError_t launch_convert<c64, c32>(const c64 *, c32 *, long long, hipStream_t);
template hipError_t launch_convert<c32, c32>(const c32 *, c32 *, long long, hipStream_t);
template hipError_t launch_convert<c64, c64>(const c64 *, c64 *, long long, hipStream_t);

}  // namespace helm
