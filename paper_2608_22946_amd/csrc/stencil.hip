// Level-operator kernels: instantiations for FP32 and FP64 operands, the operator
// hooks (Q_h, diag, one Jacobi sweep) and D^-1 (the stencil itself is in stencil_impl.h).
#include "stencil_impl.h"

namespace helm {

int stencil_blocks(int nx, int ny, int nz, int tz) {
    const int ntx = 1 + ceil_div(nx + 1, kTileX);   // upper bound for both x tilings
    const int nty = ceil_div(ny + 1, kWavesY);
    if (tz <= 0) tz = pick_tz(ntx, nty, nz + 1);
    return ntx * nty * ceil_div(nz + 1, tz);
}

template <typename R, typename TI, typename TO>
hipError_t launch_qapply(const LevelArgs<R> &L, const TI *x, TO *y, hipStream_t s) {
    const int ntx = ceil_div(L.nx + 1, kQX), nty = ceil_div(L.ny + 1, 4), nzc = ceil_div(L.nz + 1, kQZ);
    hipLaunchKernelGGL((k_qapply<R, TI, TO>), dim3(ntx * nty, nzc, cur_batch().n), dim3(64, 4), sizeof(R) * L.K * 12, s,
                       L, x, y, cur_batch());
    return hipGetLastError();
}

template <typename R, typename T>
hipError_t launch_diag(const LevelArgs<R> &L, int shifted, const T *x, T *y, hipStream_t s) {
    const long long nn = (long long)(L.nz + 1) * L.sy;
    int blocks = (int)std::min<long long>((nn + 255) / 256, 65536);
    if (shifted)
        hipLaunchKernelGGL((k_diag<R, T, true>), dim3(blocks), dim3(256), sizeof(R) * L.nk * 20, s, L, x, y);
    else
        hipLaunchKernelGGL((k_diag<R, T, false>), dim3(blocks), dim3(256), sizeof(R) * L.nk * 20, s, L, x, y);
    return hipGetLastError();
}

template <typename R, typename T>
hipError_t launch_jac1(const LevelArgs<R> &L, int shifted, double omegaJ, const T *g, T *y, hipStream_t s) {
    const R *dinv = L.dinv[shifted ? 1 : 0];
    if (!dinv) return hipErrorInvalidValue;
    const long long nn = (long long)(L.nz + 1) * L.sy;
    int blocks = (int)std::min<long long>((nn + 255) / 256, 65536);
    hipLaunchKernelGGL((k_jac1<R, T>), dim3(blocks, cur_batch().n), dim3(256), 0, s, dinv, g, y, nn, (R)omegaJ,
                       cur_batch());
    return hipGetLastError();
}

template <typename R>
hipError_t launch_dinv(const LevelArgs<R> &L, int shifted, R *out, hipStream_t s) {
    const long long nn = (long long)(L.nz + 1) * L.sy;
    int blocks = (int)std::min<long long>((nn + 255) / 256, 65536);
    if (shifted)
        hipLaunchKernelGGL((k_dinv<R, true>), dim3(blocks), dim3(256), sizeof(R) * L.nk * 20, s, L, out);
    else
        hipLaunchKernelGGL((k_dinv<R, false>), dim3(blocks), dim3(256), sizeof(R) * L.nk * 20, s, L, out);
    return hipGetLastError();
}
template hipError_t launch_dinv<float>(const LevelArgs<float> &, int, float *, hipStream_t);
template hipError_t launch_dinv<double>(const LevelArgs<double> &, int, double *, hipStream_t);

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
