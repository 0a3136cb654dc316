// Grid transfers between consecutive levels (Sec. 3.1):
//   full weighting  (R v)_j = v_{2j-1}/4 + v_{2j}/2 + v_{2j+1}/4 per axis (eq. full-weighting)
//   trilinear       (P w)_{2j} = w_j, (P w)_{2j+1} = (w_j + w_{j+1})/2 per axis (eq. linear-prolongation)
// Coarse interior nodes only touch fine interior nodes, boundary values read as
// zero, boundary outputs are zero (restriction) or left unchanged (prolong-add).
#include <algorithm>

#include "helm_internal.h"

namespace helm {
namespace {

template <typename T>
using real_of = decltype(T{}.re);

// Both kernels run on a 3D grid: 64 x-consecutive nodes per wavefront, four
// rows (wavefronts) per block along y, one plane per block along z, so node
// coordinates come from the launch indices without integer division.
constexpr int kTX = 64, kTY = 4;

// one thread per coarse node; the 27 fine values are read through the cache hierarchy
template <typename T>
__global__ void __launch_bounds__(256) k_restrict(Geom F, Geom C, const T *__restrict__ f, T *__restrict__ c) {
    const int X = blockIdx.x * kTX + threadIdx.x, Y = blockIdx.y * kTY + threadIdx.y, Zc = blockIdx.z;
    if (X > C.n[0] || Y > C.n[1]) return;
    real_of<T> sr = 0, si = 0;
    if (X >= 1 && X <= C.n[0] - 1 && Y >= 1 && Y <= C.n[1] - 1 && Zc >= 1 && Zc <= C.n[2] - 1) {
        const long long fc = (long long)(2 * Zc) * F.sy + (long long)(2 * Y) * F.sx + 2 * X;
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const long long row = fc + dz * F.sy + dy * F.sx;
                const T a = f[row - 1], b = f[row], d = f[row + 1];
                // (1/4, 1/2, 1/4) along x, times the y and z weights: 1/16 for dy = dz = 0
                const real_of<T> w = (real_of<T>)((dz ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * 0.0625);
                sr += w * (a.re + 2 * b.re + d.re);
                si += w * (a.im + 2 * b.im + d.im);
            }
    }
    T o;
    o.re = sr;
    o.im = si;
    c[(long long)Zc * C.sy + (long long)Y * C.sx + X] = o;
}

// Second pass of the fused residual + full weighting: w[Z][y][X] holds the
// residual already weighted along x and z; coarse node (X, Y, Z) takes the
// fine rows 2Y-1, 2Y, 2Y+1 with weights 1/4, 1/2, 1/4.  Coarse boundary nodes
// are written as zero.
template <typename T>
__global__ void __launch_bounds__(256) k_restrict_y(Geom F, Geom C, const T *__restrict__ w, T *__restrict__ c) {
    const int X = blockIdx.x * kTX + threadIdx.x, Y = blockIdx.y * kTY + threadIdx.y, Zc = blockIdx.z;
    if (X > C.n[0] || Y > C.n[1]) return;
    real_of<T> sr = 0, si = 0;
    if (X >= 1 && X <= C.n[0] - 1 && Y >= 1 && Y <= C.n[1] - 1 && Zc >= 1 && Zc <= C.n[2] - 1) {
        const long long wsx = C.n[0] + 1, wsy = (long long)(F.n[1] + 1) * wsx;
        const T *p = w + (long long)Zc * wsy + (long long)(2 * Y) * wsx + X;
        const T a = p[-wsx], b = p[0], d = p[wsx];
        sr = (real_of<T>)0.25 * (a.re + d.re) + (real_of<T>)0.5 * b.re;
        si = (real_of<T>)0.25 * (a.im + d.im) + (real_of<T>)0.5 * b.im;
    }
    T o;
    o.re = sr;
    o.im = si;
    c[(long long)Zc * C.sy + (long long)Y * C.sx + X] = o;
}

// one thread per fine node: fine += P coarse.  Along each axis a fine node
// 2j takes coarse node j with weight 1 and a fine node 2j+1 takes j and j+1
// with weight 1/2 each; coarse boundary nodes contribute zero.
template <typename T>
__global__ void __launch_bounds__(256) k_prolong_add(Geom C, Geom F, const T *__restrict__ c, T *__restrict__ f) {
    const int x = blockIdx.x * kTX + threadIdx.x, y = blockIdx.y * kTY + threadIdx.y, z = blockIdx.z;
    if (x < 1 || x > F.n[0] - 1 || y < 1 || y > F.n[1] - 1 || z < 1 || z > F.n[2] - 1) return;
    const int xa = x >> 1, xb = (x + 1) >> 1, ya = y >> 1, yb = (y + 1) >> 1, za = z >> 1, zb = (z + 1) >> 1;
    const real_of<T> hx = (x & 1) ? (real_of<T>)0.5 : (real_of<T>)1, hy = (y & 1) ? (real_of<T>)0.5 : (real_of<T>)1,
                     hz = (z & 1) ? (real_of<T>)0.5 : (real_of<T>)1;
    real_of<T> sr = 0, si = 0;
#pragma unroll
    for (int cz = 0; cz < 2; ++cz) {
        const int Zc = cz ? zb : za;
        if ((cz && zb == za) || Zc < 1 || Zc > C.n[2] - 1) continue;
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
            const int Yc = cy ? yb : ya;
            if ((cy && yb == ya) || Yc < 1 || Yc > C.n[1] - 1) continue;
            const T *row = c + (long long)Zc * C.sy + (long long)Yc * C.sx;
            real_of<T> rr = 0, ri = 0;
            if (xa >= 1 && xa <= C.n[0] - 1) {
                const T v = row[xa];
                rr += v.re;
                ri += v.im;
            }
            if (xb != xa && xb >= 1 && xb <= C.n[0] - 1) {
                const T v = row[xb];
                rr += v.re;
                ri += v.im;
            }
            sr += rr;
            si += ri;
        }
    }
    const real_of<T> w = hx * hy * hz;
    const long long i = (long long)z * F.sy + (long long)y * F.sx + x;
    T o = f[i];
    o.re += w * sr;
    o.im += w * si;
    f[i] = o;
}

}  // namespace

namespace {
dim3 node_grid(const Geom &g) {
    return dim3((unsigned)((g.n[0] + kTX) / kTX), (unsigned)((g.n[1] + kTY) / kTY), (unsigned)(g.n[2] + 1));
}
}  // namespace

template <typename T>
hipError_t launch_restrict(const Geom &fine, const Geom &coarse, const T *f, T *c, hipStream_t s) {
    hipLaunchKernelGGL((k_restrict<T>), node_grid(coarse), dim3(kTX, kTY), 0, s, fine, coarse, f, c);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_y(const Geom &fine, const Geom &coarse, const T *w, T *c, hipStream_t s) {
    hipLaunchKernelGGL((k_restrict_y<T>), node_grid(coarse), dim3(kTX, kTY), 0, s, fine, coarse, w, c);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(const Geom &coarse, const Geom &fine, const T *c, T *f, hipStream_t s) {
    hipLaunchKernelGGL((k_prolong_add<T>), node_grid(fine), dim3(kTX, kTY), 0, s, coarse, fine, c, f);
    return hipGetLastError();
}

template hipError_t launch_restrict<c32>(const Geom &, const Geom &, const c32 *, c32 *, hipStream_t);
template hipError_t launch_restrict<c64>(const Geom &, const Geom &, const c64 *, c64 *, hipStream_t);
template hipError_t launch_restrict_y<c32>(const Geom &, const Geom &, const c32 *, c32 *, hipStream_t);
template hipError_t launch_restrict_y<c64>(const Geom &, const Geom &, const c64 *, c64 *, hipStream_t);
template hipError_t launch_prolong_add<c32>(const Geom &, const Geom &, const c32 *, c32 *, hipStream_t);
template hipError_t launch_prolong_add<c64>(const Geom &, const Geom &, const c64 *, c64 *, hipStream_t);

}  // namespace helm
