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

// one thread per coarse node; fine rows are read through the cache hierarchy
template <typename T>
__global__ void __launch_bounds__(256) k_restrict(Geom F, Geom C, const T *__restrict__ f, T *__restrict__ c) {
    const long long nn = C.nn;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn; i += (long long)gridDim.x * blockDim.x) {
        const int X = (int)(i % C.sx);
        const int Y = (int)((i / C.sx) % (C.n[1] + 1));
        const int Zc = (int)(i / C.sy);
        real_of<T> sr = 0, si = 0;
        if (X >= 1 && X <= C.n[0] - 1 && Y >= 1 && Y <= C.n[1] - 1 && Zc >= 1 && Zc <= C.n[2] - 1) {
            const long long fc = (long long)(2 * Zc) * F.sy + (long long)(2 * Y) * F.sx + 2 * X;
            for (int dz = -1; dz <= 1; ++dz)
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
        c[i] = o;
    }
}

// one thread per fine node: fine += P coarse
template <typename T>
__global__ void __launch_bounds__(256) k_prolong_add(Geom C, Geom F, const T *__restrict__ c, T *__restrict__ f) {
    const long long nn = F.nn;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn; i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % F.sx);
        const int y = (int)((i / F.sx) % (F.n[1] + 1));
        const int z = (int)(i / F.sy);
        if (x < 1 || x > F.n[0] - 1 || y < 1 || y > F.n[1] - 1 || z < 1 || z > F.n[2] - 1) continue;
        const int p[3] = {x, y, z};
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = p[a] >> 1;
            hi[a] = (p[a] + 1) >> 1;
        }
        real_of<T> sr = 0, si = 0;
        for (int cz = 0; cz < 2; ++cz) {
            const int Zc = cz ? hi[2] : lo[2];
            if (cz && hi[2] == lo[2]) continue;
            if (Zc < 1 || Zc > C.n[2] - 1) continue;
            for (int cy = 0; cy < 2; ++cy) {
                const int Yc = cy ? hi[1] : lo[1];
                if (cy && hi[1] == lo[1]) continue;
                if (Yc < 1 || Yc > C.n[1] - 1) continue;
                for (int cx = 0; cx < 2; ++cx) {
                    const int Xc = cx ? hi[0] : lo[0];
                    if (cx && hi[0] == lo[0]) continue;
                    if (Xc < 1 || Xc > C.n[0] - 1) continue;
                    const real_of<T> w =
                        (real_of<T>)(((p[0] & 1) ? 0.5 : 1.0) * ((p[1] & 1) ? 0.5 : 1.0) * ((p[2] & 1) ? 0.5 : 1.0));
                    const T v = c[(long long)Zc * C.sy + (long long)Yc * C.sx + Xc];
                    sr += w * v.re;
                    si += w * v.im;
                }
            }
        }
        T o = f[i];
        o.re += sr;
        o.im += si;
        f[i] = o;
    }
}

}  // namespace

template <typename T>
hipError_t launch_restrict(const Geom &fine, const Geom &coarse, const T *f, T *c, hipStream_t s) {
    int blocks = (int)std::min<long long>((coarse.nn + 255) / 256, 65536);
    hipLaunchKernelGGL((k_restrict<T>), dim3(blocks), dim3(256), 0, s, fine, coarse, f, c);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(const Geom &coarse, const Geom &fine, const T *c, T *f, hipStream_t s) {
    int blocks = (int)std::min<long long>((fine.nn + 255) / 256, 65536);
    hipLaunchKernelGGL((k_prolong_add<T>), dim3(blocks), dim3(256), 0, s, coarse, fine, c, f);
    return hipGetLastError();
}

template hipError_t launch_restrict<c32>(const Geom &, const Geom &, const c32 *, c32 *, hipStream_t);
template hipError_t launch_restrict<c64>(const Geom &, const Geom &, const c64 *, c64 *, hipStream_t);
template hipError_t launch_prolong_add<c32>(const Geom &, const Geom &, const c32 *, c32 *, hipStream_t);
template hipError_t launch_prolong_add<c64>(const Geom &, const Geom &, const c64 *, c64 *, hipStream_t);

}  // namespace helm
