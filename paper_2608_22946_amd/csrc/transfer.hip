// Grid transfers between consecutive levels (Sec. 3.1):
//   full weighting  (R v)_j = v_{2j-1}/4 + v_{2j}/2 + v_{2j+1}/4 per axis (eq. full-weighting)
//   trilinear       (P w)_{2j} = w_j, (P w)_{2j+1} = (w_j + w_{j+1})/2 per axis (eq. linear-prolongation)
// Coarse interior nodes only touch fine interior nodes, boundary values read as
// zero, boundary outputs are zero (restriction) or left unchanged (prolong-add).
#include <algorithm>
#include <type_traits>

#include "helm_internal.h"

namespace helm {
namespace {

template <typename T>
using real_of = decltype(T{}.re);

// The kernels run on 3D grids: 64 x-consecutive nodes per wavefront, four
// rows (wavefronts) per block along y, one plane per block along z, so node
// coordinates come from the launch indices without integer division (the
// prolongation's blocks may instead be 32 cells wide and eight rows deep).
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
template <typename T, typename TO>
__global__ void __launch_bounds__(256) k_restrict_y(Geom F, Geom C, const T *__restrict__ w, TO *__restrict__ c,
                                                   Scale so, Batch bt) {
    // batched slots follow each other along z: slot sl covers planes sl (nc + 1) ..
    const int sl = blockIdx.z / (C.n[2] + 1);
    if (slot_off(bt, sl)) return;
    const int X = blockIdx.x * kTX + threadIdx.x, Y = blockIdx.y * kTY + threadIdx.y, Zc = blockIdx.z % (C.n[2] + 1);
    if (X > C.n[0] || Y > C.n[1]) return;
    w = slot_ptr(w, (long long)(C.n[2] + 1) * (F.n[1] + 1) * (C.n[0] + 1), sl);
    c = slot_ptr(c, C.nn, sl);
    so = slot_scale(so, sl);
    const real_of<T> ms = store_mul<real_of<T>, TO>(so);
    real_of<T> sr = 0, si = 0;
    if (X >= 1 && X <= C.n[0] - 1 && Y >= 1 && Y <= C.n[1] - 1 && Zc >= 1 && Zc <= C.n[2] - 1) {
        const long long wsx = C.n[0] + 1, wsy = (long long)(F.n[1] + 1) * wsx;
        const T *p = w + (long long)Zc * wsy + (long long)(2 * Y) * wsx + X;
        const T a = p[-wsx], b = p[0], d = p[wsx];
        sr = (real_of<T>)0.25 * (a.re + d.re) + (real_of<T>)0.5 * b.re;
        si = (real_of<T>)0.25 * (a.im + d.im) + (real_of<T>)0.5 * b.im;
    }
    c[(long long)Zc * C.sy + (long long)Y * C.sx + X] = to_stored<TO>(sr, si, ms);
}

// fine += P coarse, one thread per coarse cell (X, Y, Z), X in [0, nc): it
// updates the fine nodes 2X + i, 2Y + j, 2Z + k (i, j, k in {0, 1}) from the
// eight coarse nodes X + a, Y + b, Z + c (a, b, c in {0, 1}).  Along each axis
// a fine node 2X takes coarse X with weight 1 and a fine node 2X + 1 takes X
// and X + 1 with weight 1/2 each; coarse boundary nodes contribute zero and
// fine boundary nodes are left unchanged.  Each coarse value is loaded once per
// cell instead of once per fine node, and the two x-neighbouring fine nodes of
// a cell are adjacent in memory.
template <typename T, typename TF>
__global__ void __launch_bounds__(256) k_prolong_add(Geom C, Geom F, const T *__restrict__ c, TF *__restrict__ f,
                                                    Scale sc, Scale sf, Batch bt) {
    using R = std::conditional_t<is_half<TF>(), float, real_of<TF>>;   // FP16-stored vectors add in FP32
    const int sl = blockIdx.z / C.n[2];   // batched slots follow each other along z
    if (slot_off(bt, sl)) return;
    const int X = blockIdx.x * blockDim.x + threadIdx.x, Y = blockIdx.y * blockDim.y + threadIdx.y, Z = blockIdx.z % C.n[2];
    if (X >= C.n[0] || Y >= C.n[1]) return;
    c = slot_ptr(c, C.nn, sl);
    f = slot_ptr(f, F.nn, sl);
    sc = slot_scale(sc, sl);
    sf = slot_scale(sf, sl);
    // c16 operands: coarse values to true units, fine values through the fine scale
    const R mc = load_mul<R, T>(sc), mfl = load_mul<R, TF>(sf), mfs = store_mul<R, TF>(sf);
    // coarse corner values, zero outside the coarse interior
    R cr[2][2][2], ci[2][2][2];
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                const int Xc = X + cx, Yc = Y + cy, Zc = Z + cz;
                const bool in = Xc >= 1 && Xc <= C.n[0] - 1 && Yc >= 1 && Yc <= C.n[1] - 1 && Zc >= 1 &&
                                Zc <= C.n[2] - 1;
                T v;
                v.re = 0;
                v.im = 0;
                if (in) v = c[(long long)Zc * C.sy + (long long)Yc * C.sx + Xc];
                cr[cz][cy][cx] = (R)v.re * mc;
                ci[cz][cy][cx] = (R)v.im * mc;
            }
    const R half = (R)0.5;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int z = 2 * Z + k;
        if (z < 1) continue;   // z <= 2 (nc - 1) + 1 = F.n[2] - 1 always
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int y = 2 * Y + j;
            if (y < 1) continue;
            // the four coarse values of this fine row, weighted along z and y
            R pr[2], pi[2];
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                R zr[2], zi[2];
#pragma unroll
                for (int cy = 0; cy < 2; ++cy) {
                    zr[cy] = k ? half * (cr[0][cy][cx] + cr[1][cy][cx]) : cr[0][cy][cx];
                    zi[cy] = k ? half * (ci[0][cy][cx] + ci[1][cy][cx]) : ci[0][cy][cx];
                }
                pr[cx] = j ? half * (zr[0] + zr[1]) : zr[0];
                pi[cx] = j ? half * (zi[0] + zi[1]) : zi[0];
            }
            TF *row = f + (long long)z * F.sy + (long long)y * F.sx + 2 * X;
            if (X >= 1) {   // fine node 2X (x = 0 is a boundary node)
                const TF o = row[0];
                row[0] = to_stored<TF, R>((R)o.re * mfl + pr[0], (R)o.im * mfl + pi[0], mfs);
            }
            const TF o = row[1];   // fine node 2X + 1
            row[1] = to_stored<TF, R>((R)o.re * mfl + half * (pr[0] + pr[1]), (R)o.im * mfl + half * (pi[0] + pi[1]), mfs);
        }
    }
}

}  // namespace

namespace {
// one thread per node of g (z planes repeated for each batched slot)
dim3 node_grid(const Geom &g, int slots = 1) {
    return dim3((unsigned)((g.n[0] + kTX) / kTX), (unsigned)((g.n[1] + kTY) / kTY), (unsigned)(g.n[2] + 1) * slots);
}
// one thread per cell of g: n[0] x n[1] x n[2] (z repeated for each batched slot), in blocks of
// bx x (256 / bx) threads
dim3 cell_grid(const Geom &g, int bx, int slots = 1) {
    const int by = 256 / bx;
    return dim3((unsigned)((g.n[0] + bx - 1) / bx), (unsigned)((g.n[1] + by - 1) / by), (unsigned)g.n[2] * slots);
}
// x extent of the prolongation's blocks: 64 cells (a wavefront per row, the widest fine
// segments), or 32 where that leaves fewer idle lanes (88 cells: 96 lanes against 128)
int cell_block_x(const Geom &g) {
    return (g.n[0] + 31) / 32 * 32 < (g.n[0] + 63) / 64 * 64 ? 32 : 64;
}
}  // namespace

template <typename T>
hipError_t launch_restrict(const Geom &fine, const Geom &coarse, const T *f, T *c, hipStream_t s) {
    hipLaunchKernelGGL((k_restrict<T>), node_grid(coarse), dim3(kTX, kTY), 0, s, fine, coarse, f, c);
    return hipGetLastError();
}

template <typename T, typename TO>
hipError_t launch_restrict_y(const Geom &fine, const Geom &coarse, const T *w, TO *c, hipStream_t s, Scale so) {
    if (is_half<TO>() && !so.qs) return hipErrorInvalidValue;
    const Batch &bt = cur_batch();
    hipLaunchKernelGGL((k_restrict_y<T, TO>), node_grid(coarse, bt.n), dim3(kTX, kTY), 0, s, fine, coarse, w, c, so, bt);
    return hipGetLastError();
}

template <typename T, typename TF>
hipError_t launch_prolong_add(const Geom &coarse, const Geom &fine, const T *c, TF *f, hipStream_t s, Scale sc,
                              Scale sf) {
    if (fine.n[0] != 2 * coarse.n[0] || fine.n[1] != 2 * coarse.n[1] || fine.n[2] != 2 * coarse.n[2])
        return hipErrorInvalidValue;
    if ((is_half<T>() && !sc.qs) || (is_half<TF>() && !sf.qs)) return hipErrorInvalidValue;
    const Batch &bt = cur_batch();
    const int bx = cell_block_x(coarse);
    hipLaunchKernelGGL((k_prolong_add<T, TF>), cell_grid(coarse, bx, bt.n), dim3(bx, 256 / bx), 0, s, coarse, fine, c, f,
                       sc, sf, bt);
    return hipGetLastError();
}

template hipError_t launch_restrict<c32>(const Geom &, const Geom &, const c32 *, c32 *, hipStream_t);
template hipError_t launch_restrict<c64>(const Geom &, const Geom &, const c64 *, c64 *, hipStream_t);
template hipError_t launch_restrict_y<c32, c32>(const Geom &, const Geom &, const c32 *, c32 *, hipStream_t, Scale);
template hipError_t launch_restrict_y<c64, c64>(const Geom &, const Geom &, const c64 *, c64 *, hipStream_t, Scale);
template hipError_t launch_restrict_y<c32, c16>(const Geom &, const Geom &, const c32 *, c16 *, hipStream_t, Scale);
template hipError_t launch_prolong_add<c32, c32>(const Geom &, const Geom &, const c32 *, c32 *, hipStream_t, Scale,
                                                 Scale);
template hipError_t launch_prolong_add<c64, c64>(const Geom &, const Geom &, const c64 *, c64 *, hipStream_t, Scale,
                                                 Scale);
template hipError_t launch_prolong_add<c16, c16>(const Geom &, const Geom &, const c16 *, c16 *, hipStream_t, Scale,
                                                 Scale);

}  // namespace helm
