// Internal declarations of the MI355X IOFD Helmholtz library (device types,
// per-level kernel arguments, Krylov state and the kernel launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "helm.h"

namespace helm {

constexpr int kMMax = 12;       // longest Krylov restart supported (m_h, m_2h, m_out)
constexpr int kM4Max = 8;       // longest bottom (s-step) basis
constexpr int kSstepMax = 2;    // longest fine-level smoothing cycle computed with an s-step basis
constexpr int kKMax = 128;      // most table intervals
constexpr int kTileX = 62;      // output nodes per wavefront along x (64 lanes, 1-node halo each side)
constexpr int kWavesY = 4;      // wavefronts (rows y) per workgroup
constexpr int kRedBlocks = 1024;
constexpr int kRedStride = kMMax + 2;   // partial-sum slots per block (dots + norm)
constexpr int kRedMaxBlocks = 256;      // most blocks of a vector reduction (red_blocks)
// complex partial-sum slots per reduction block: the larger of the s-step Gram
// matrix's (kM4Max + 1)(kM4Max + 2)/2 entries and the dots' kRedStride
constexpr int kRedSlots = (kM4Max + 1) * (kM4Max + 2) / 2 > kRedStride ? (kM4Max + 1) * (kM4Max + 2) / 2 : kRedStride;
// Happy breakdown: the newest direction w = op(prec(v_k)) lies in the Krylov space,
// h_{k+1,k} = ||w - V h|| <= kBreakdown ||w|| (scale-free: a scaled right-hand side
// gives the scaled iterate)
constexpr double kBreakdown = 1e-14;
// Selective reorthogonalisation: the second classical Gram-Schmidt pass runs only
// when the first left less than this fraction of ||w||^2, i.e. ||w - V h|| <
// ||w|| / 32.  One pass then keeps the new vector orthogonal to about 32 units
// of roundoff (2e-6 in FP32), below what the inner FP32 solves resolve; the
// stricter 1/2 of Kahan and Parlett (orthogonal to working accuracy) gave the
// same iteration counts and residuals at 5% more solve time.
constexpr double kReorthEta = 1.0 / 1024;

template <typename R>
struct cplx {
    R re, im;
};
using c32 = cplx<float>;
using c64 = cplx<double>;
// FP16-stored complex (HELM_MIXED): the preconditioner's inner vectors in 4 B per node.
// A stored vector holds v * f * (*qs) for its true value v: f a level constant, *qs the
// inverse norm of the cycle's input (device memory), so stored values stay near unit size
// whatever the grid spacing and the source strength.
using c16 = cplx<_Float16>;
struct Scale {
    float f;             // constant factor
    const double *qs;    // device scalar; null for vectors stored in FP32 / FP64
    int qstride = 0;     // doubles between the scalars of batched slots (0: one scalar for all)
};
constexpr float kHalfMax = 65504.0f;   // largest finite FP16 value

template <typename T>
constexpr bool is_half() { return sizeof(T{}.re) == 2; }
template <typename R>
__device__ __forceinline__ R sat_half(R a) {   // keeps NaN, clamps to the finite FP16 range
    return a > (R)kHalfMax ? (R)kHalfMax : (a < -(R)kHalfMax ? -(R)kHalfMax : a);
}
// element of type T from a true value (c16: times the store multiplier s, saturated)
template <typename T, typename R>
__device__ __forceinline__ T to_stored(R re, R im, R s) {
    T o;
    if constexpr (is_half<T>()) {
        o.re = (_Float16)sat_half(re * s);
        o.im = (_Float16)sat_half(im * s);
    } else {
        o.re = re;
        o.im = im;
    }
    return o;
}
// multipliers of a kernel's operands: 1 / (f qs) after a c16 load, f qs before a c16 store, else 1.
// qs = 0 (the inverse norm of a zero input) stores zeros, which load as zeros.
template <typename R, typename T>
__device__ __forceinline__ R load_mul(const Scale &s) {
    if constexpr (is_half<T>()) {
        const double d = (double)s.f * *s.qs;
        return d != 0.0 ? (R)(1.0 / d) : (R)0;
    }
    return (R)1;
}
template <typename R, typename T>
__device__ __forceinline__ R store_mul(const Scale &s) {
    if constexpr (is_half<T>()) return (R)((double)s.f * *s.qs);
    return (R)1;
}

// ---------------------------------------------------------------------------
// Geometry and per-level kernel arguments
// ---------------------------------------------------------------------------
struct Geom {
    int n[3];            // intervals per axis on this level
    long long sx, sy;    // node strides of y and z
    long long nn;        // nodes
    int lo[3], hi[3];    // nodes a with unit stretching at a, a-1/2, a+1/2 (weights exactly -1, 2, -1)
    double ell;
};

template <typename R>
struct LevelArgs {
    int nx, ny, nz;
    long long sx, sy;
    int lox, hix, loy, hiy, loz, hiz;
    const float *c;      // velocity at the level nodes
    const R *wx, *wy, *wz;  // per node: (wm.re, wm.im, wc.re, wc.im, wp.re, wp.im)
    const R *atab;       // [K][5][4] monomial coefficients of alpha1..5 in t on each interval
    const R *btab;       // [K][3][4] same for beta1..3
    int K;
    R inv_deta;          // K / 0.4
    R omega_ell;         // omega * ell
    R inv_ell2;
    R sigma;
    // stencil tiling per kernel family ([0] apply / residual / sweep, [1] fused two-sweep Jacobi)
    int tz[2];           // z planes per wavefront (0: default rule)
    int split[2];        // 1: an interior launch plus a border launch where the tiling allows
    const R *dinv[2];    // per node D^-1 of A_l ([0]) and B_l ([1]), complex interleaved; 0 on the boundary
    // FP32 levels: the interpolation coordinate before the clamp at eta* = 0.4, per node,
    // s = omega ell K / (0.4 * 2 pi c) (formed in FP64 at setup), read instead of c by the
    // stencils: eta* = min(s, K) 0.4 / K and kappa = s kap_s, without a reciprocal per node;
    // and the unshifted shell coefficients C_0..C_3 (eq. iofd-shell-coefficients, mu = 1) as
    // quintics in the local coordinate t of each table interval, interval K standing for
    // the clamped range s >= K (t = s - K unbounded there).  Null in FP64 arguments.
    const float *s;
    const R *ctab;       // [K + 1][4][6] monomial coefficients in t
    R kap_s;             // kappa per unit of s: 0.4 * 2 pi / K
    // table intervals the stencils stage in LDS: the alpha pieces kb .. kb + nk - 1 and the
    // shell quintics cb .. cb + nck - 1, every interval a node of this level can reach
    // (from the velocity range, one interval of margin each side)
    int kb, nk, cb, nck;
};

// ---------------------------------------------------------------------------
// Krylov state kept in device memory (one per nested solver)
// ---------------------------------------------------------------------------
struct KState {
    double H[kMMax + 1][kMMax][2];   // rotated Hessenberg (upper triangle = R factor)
    double cs[kMMax];
    double sn[kMMax][2];
    double g[kMMax + 1][2];          // rotated beta e1
    double h1[kMMax + 1][2];         // first Gram-Schmidt pass coefficients
    double h2[kMMax + 1][2];         // second pass coefficients
    double y[kMMax][2];              // combination coefficients (bottom solver)
    double beta;                     // initial residual norm of the cycle
    double scale;                    // multiplier that normalises the newest basis vector
    double vs0;                      // the first basis vector is kept unnormalised: V_0 = vs0 * (stored vector)
    double hk1;                      // last subdiagonal entry
    double wn;                       // ||w|| of the newest column before orthogonalisation
    int kk;                          // Arnoldi columns in the current cycle
    int breakdown;
    int nonfinite;
    int reorth;                      // 1: the newest column needs the second Gram-Schmidt pass
};

struct RedBuf {
    double *partials;    // [kRedBlocks][kRedStride][2]
    unsigned *counter;   // zero between kernels
};

// Right-hand sides batched in one launch (helm_options.batch).  Slot s = blockIdx.y
// owns its own copy of every vector (at s times the vector's length from the pointer
// passed), its own Krylov state (st + s), reduction partials (partials + s * pstride)
// and completion counter (counter + s).  Blocks of a slot outside the mask return at
// once, before any barrier or ticket, so a slot that has converged costs nothing.
struct Batch {
    int n = 1;               // slots (gridDim.y)
    unsigned mask = 1u;      // bit s set: slot s runs
    long long pstride = 0;   // doubles between the slots' reduction partials
};
// The batch of the calling host thread's launches (1 slot unless a BatchScope is active):
// the launchers read it, so the solver's code is the same for one and for several slots.
Batch &cur_batch();
struct BatchScope {
    Batch saved;
    explicit BatchScope(const Batch &b) : saved(cur_batch()) { cur_batch() = b; }
    ~BatchScope() { cur_batch() = saved; }
    BatchScope(const BatchScope &) = delete;
    BatchScope &operator=(const BatchScope &) = delete;
};

// slot index sl: blockIdx.y in the 1-D and 2-D kernels, from blockIdx.z in the transfers
__device__ __forceinline__ bool slot_off(const Batch &b, int sl) { return !((b.mask >> sl) & 1u); }
__device__ __forceinline__ RedBuf slot_rb(RedBuf rb, const Batch &b, int sl) {
    rb.partials += (long long)sl * b.pstride;
    rb.counter += sl;
    return rb;
}
template <typename T>
__device__ __forceinline__ T *slot_ptr(T *p, long long stride, int sl) {
    return p ? p + (long long)sl * stride : p;
}
__device__ __forceinline__ Scale slot_scale(Scale s, int sl) {
    if (s.qs) s.qs += (long long)sl * s.qstride;
    return s;
}

// M_RESID_R: residual restricted in x and z on the fly (first pass of the fused
// residual + full weighting; launch_restrict_y finishes it)
enum Mode { M_APPLY = 0, M_RESID = 1, M_JSWEEP = 2, M_JAC2 = 3, M_JAC2_ADD = 4, M_RESID_R = 5 };

enum Epi {
    EPI_STORE = 0,       // write sums to out
    EPI_NORM_INIT = 1,   // beta = sqrt(norm); reset the Krylov state; scale = 1/beta
    EPI_ARNOLDI1 = 2,    // h1 = dots
    EPI_ARNOLDI2 = 3,    // h = h1 + h2, subdiagonal, Givens update of column k
    EPI_GRAM = 4,        // s-step Gram matrix -> least-squares coefficients y
    EPI_ARNOLDI_SEL = 5  // h1 = dots with ||w||^2; one pass suffices when ||w - V h1||^2 >= kReorthEta ||w||^2
                         // (then Givens update now, h2 = h1, reorth = 0), else reorth = 1
};

// ---------------------------------------------------------------------------
// Launchers (stencil.hip, transfer.hip, vector.hip)
// ---------------------------------------------------------------------------
struct StencilCall {
    int mode;            // Mode
    int shifted;         // 0: A (mu = 1), 1: B (mu = 1 + i sigma)
    double omegaJ;       // Jacobi weight (JSWEEP, JAC2)
    const void *x;       // operand (APPLY, RESID, JSWEEP)
    const void *g;       // right-hand side (RESID, JSWEEP, JAC2)
    const void *base;    // JAC2_ADD: y = base + J2(g)
    void *y;
    bool norm;           // accumulate ||y||^2 into the reduction epilogue
    int epi;
    KState *st;
    int k;
    Scale sx = {1.0f, nullptr}, sg = {1.0f, nullptr}, sb = {1.0f, nullptr}, sy = {1.0f, nullptr};   // c16 operands
};

// R = arithmetic type, TX/TG/TY = element types of x, g, y (c32 or c64)
template <typename R, typename TX, typename TG, typename TY>
hipError_t launch_stencil(const LevelArgs<R> &L, const StencilCall &c, const RedBuf &rb, hipStream_t s);

template <typename R, typename TI, typename TO>
hipError_t launch_qapply(const LevelArgs<R> &L, const TI *x, TO *y, hipStream_t s);

template <typename R, typename T>
hipError_t launch_diag(const LevelArgs<R> &L, int shifted, const T *x, T *y, hipStream_t s);

template <typename T>
hipError_t launch_restrict(const Geom &fine, const Geom &coarse, const T *f, T *c, hipStream_t s);

// second pass of the fused residual + full weighting: coarse = y-weights of the
// x/z-restricted residual rows w ([coarse z][fine y][coarse x]); zero on the coarse boundary
template <typename T, typename TO = T>
hipError_t launch_restrict_y(const Geom &fine, const Geom &coarse, const T *w, TO *c, hipStream_t s,
                             Scale so = {1.0f, nullptr});
template <typename T, typename TF = T>
hipError_t launch_prolong_add(const Geom &coarse, const Geom &fine, const T *c, TF *f, hipStream_t s,
                              Scale sc = {1.0f, nullptr}, Scale sf = {1.0f, nullptr});

template <typename T>
hipError_t launch_dots(const T *const *V, int nv, const T *w, bool norm, long long n, int epi, KState *st, int k,
                       double *out, const RedBuf &rb, hipStream_t s);

template <typename T>
hipError_t launch_axpy_dots(const T *const *V, int nv, T *w, long long n, KState *st, const RedBuf &rb,
                            hipStream_t s, bool store = true);

template <typename T>
hipError_t launch_axpy_scale(const T *const *V, int nv, T *w, long long n, KState *st, hipStream_t s);


// x (+)= sum_j y_j Z_j with y from the state: back substitution of the
// rotated Hessenberg (from_backsolve) or the stored s-step coefficients.  With
// c16 Z and a c32 / c64 x, Z_j is stored with the scale zf * qs_j, qs_0 = st->vs0
// (the cycle's first basis vector kept unnormalised) and qs_j = 1 for j >= 1;
// with c16 Z and c16 x both carry the same scale (no conversion).
template <typename TX, typename TZ>
hipError_t launch_combine(TX *x, const TZ *const *Z, int nz, long long n, KState *st, bool from_backsolve,
                          bool overwrite, hipStream_t s, float zf = 1.0f);
// y = x with the scales of c16 operands applied (true values in, true values out)
template <typename TI, typename TO>
hipError_t launch_convert_scaled(const TI *x, TO *y, long long n, Scale si, Scale so, hipStream_t s);

template <typename T>
hipError_t launch_gram(const T *const *P, int np, long long n, KState *st, const RedBuf &rb, hipStream_t s);

template <typename T>
hipError_t launch_fill_zero(T *x, long long n, hipStream_t s);

template <typename T>
hipError_t launch_add(const T *x, T *y, long long n, hipStream_t s);   // y += x

template <typename R, typename T>
hipError_t launch_jac1(const LevelArgs<R> &L, int shifted, double omegaJ, const T *g, T *y, hipStream_t s);
template <typename R>
hipError_t launch_dinv(const LevelArgs<R> &L, int shifted, R *out, hipStream_t s);   // out = D^-1 per node

// Adjoint gradient (adjoint.hip): y = [g -] op^T x (op A, or B when shifted; g == nullptr:
// no residual), y = Q_h^T w (of conj(w) when conj_in), y_i = (d_i op x)_i in m = 1/c^2
// (which 0: A, 1: Q_h), the per-node gradient terms accumulated into gacc, and their sum
// onto the physical nodes.
template <typename R, typename TX, typename TG, typename TY>
hipError_t launch_apply_t(const LevelArgs<R> &L, int shifted, const TX *x, const TG *g, TY *y, hipStream_t s);
template <typename R, typename TI, typename TO>
hipError_t launch_qapply_t(const LevelArgs<R> &L, const TI *w, bool conj_in, TO *y, hipStream_t s);
template <typename R, typename T>
hipError_t launch_apply_dm(const LevelArgs<R> &L, int which, const T *x, T *y, hipStream_t s);
template <typename TS>
hipError_t launch_grad_node(const LevelArgs<double> &L, const c64 *v, const c64 *mu, const TS *s_, const TS *f,
                            double *gacc, hipStream_t s);
// out = in * Xi^-1 (inverse false) or in * Xi (inverse true), Xi = prod_j xi_j(i_j); fac = the per-axis
// node factors 1/xi_j concatenated (x, y, z; n_j + 1 each), followed by xi_j in the same layout;
// in may equal out (then nodes off the PML are not touched)
template <typename T>
hipError_t launch_xi_scale(const Geom &F, const c64 *fac, const T *in, T *out, bool inverse, hipStream_t s);
hipError_t launch_grad_to_velocity(const float *grad_m, const float *vel, const Geom &fine, int n_pml,
                                   const int nphys[3], float *grad_c, hipStream_t s);
hipError_t launch_grad_phys(const double *gacc, const Geom &fine, int n_pml, const int nphys[3], float *out,
                            hipStream_t s);

int stencil_blocks(int nx, int ny, int nz, int tz);   // grid size of launch_stencil on a level (tz 0: default)
// z planes per stencil wavefront: any depth kTzMin..kTzMax may be fixed; setup times the candidates
constexpr int kTzMin = 2, kTzMax = 64;
constexpr int kTzCandidates[] = {2, 3, 4, 5, 6, 8, 10, 12, 14, 16, 20, 24, 32, 40, 48, 64};

template <typename TI, typename TO>
hipError_t launch_convert(const TI *x, TO *y, long long n, hipStream_t s);

hipError_t launch_extend_velocity(const float *phys, const int nphys[3], int n_pml, int stride_fine,
                                  const Geom &g, float *out, hipStream_t s);
// out_i = factor / c_i in FP64, rounded to FP32 (the scaled interpolation coordinate s of LevelArgs)
hipError_t launch_scaled_eta(const float *c, long long n, double factor, float *out, hipStream_t s);

hipError_t launch_velocity_check(const float *v, long long n, const RedBuf &rb, double *out, hipStream_t s);

inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// record the message helm_last_error(NULL) returns on this thread; returns st
helm_status thread_error(helm_status st, const char *msg);

// Cross-block completion ticket without device-wide cache maintenance.
// Partial results are written with agent-scope atomic stores (write-through
// to the device coherence point, past the per-XCD L2), every store is
// waited for (s_waitcnt) before the block takes a ticket with an agent-scope
// atomic add, and the last block reads the partials with agent-scope atomic
// loads.  A __threadfence() here would write back and invalidate the whole
// L2 of the XCD in every block, evicting the operands other blocks stream.
__device__ __forceinline__ void partial_store(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double partial_load(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stores_done() {
    __builtin_amdgcn_s_waitcnt(0);          // vmcnt/expcnt/lgkmcnt = 0: this thread's stores are performed
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
// returns true in exactly one block: the last to arrive (call from one thread)
__device__ __forceinline__ bool take_ticket(unsigned *counter, unsigned nblocks) {
    return __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == nblocks - 1;
}
__device__ __forceinline__ void reset_ticket(unsigned *counter) {
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of a double over the 64 lanes of a wavefront, returned in every lane, in
// a fixed order.  Lane exchanges use DPP on the two 32-bit halves: xor 1 and
// xor 2 inside each quad, then rotations by 4 and 8 inside each 16-lane row
// (every lane then holds its row sum), and the four row sums are read out.
// All 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_double<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_double<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_double<0x124>(v);   // row_ror:4
    v += dpp_double<0x128>(v);   // row_ror:8
    const long long b = __double_as_longlong(v);
    double r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int lo = __builtin_amdgcn_readlane((int)b, 16 * q), hi = __builtin_amdgcn_readlane((int)(b >> 32), 16 * q);
        r[q] = __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    }
    return (r[0] + r[1]) + (r[2] + r[3]);
}

}  // namespace helm
