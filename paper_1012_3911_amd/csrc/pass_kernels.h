// Row (x) and column (strided) line passes of the Schroedinger step, as
// templates over the tile shape so that the planner can pick, per line
// length and precision, how many lines a work-group holds, the register
// radix and an occupancy hint.  Included by the per-precision instantiation
// units sfo_row.hip and sfo_col.hip.
#pragma once
#include <utility>

#include "sfo_impl.h"

namespace sfo {

template <typename R> using VStore = typename std::conditional<sizeof(R) == 4, float, double>::type;

// sin and cos of |x| <= 1/8 by their Taylor series to x^11 / x^10
// (truncation below 3e-20 relative); used for potential phases the host has
// bounded by 1/8.
__device__ __forceinline__ void sincos_small(double x, double &s, double &c)
{
    const double x2 = x * x;
    double ps = -2.5052108385441718775e-08;                  // -1/11!
    ps = __builtin_fma(ps, x2, 2.7557319223985890653e-06);   // 1/9!
    ps = __builtin_fma(ps, x2, -1.9841269841269841270e-04);  // -1/7!
    ps = __builtin_fma(ps, x2, 8.3333333333333333333e-03);   // 1/5!
    ps = __builtin_fma(ps, x2, -1.6666666666666666667e-01);  // -1/3!
    s = __builtin_fma(ps * x2, x, x);
    double pc = -2.7557319223985890653e-07;                  // -1/10!
    pc = __builtin_fma(pc, x2, 2.4801587301587301587e-05);   // 1/8!
    pc = __builtin_fma(pc, x2, -1.3888888888888888889e-03);  // -1/6!
    pc = __builtin_fma(pc, x2, 4.1666666666666666667e-02);   // 1/4!
    pc = __builtin_fma(pc, x2, -0.5);
    c = __builtin_fma(pc, x2, 1.0);
}

template <int N, int RAD, int THREADS> struct RowTile {
    using Sh = LineShape<N, RAD>;
    static constexpr int ROWS = THREADS / Sh::T > 0 ? THREADS / Sh::T : 1;
    static constexpr int NT = ROWS * Sh::T;
};

// --------------------------------------------------------------- row pass --
// One work-group holds ROWS rows of N points; thread t of a row owns the
// cyclic elements x = t + m T.  Global access is contiguous along the row.
// The potential factor exp(-i sgn [aV V0(x) + e.x]) is built from a per-point
// exp(-i sgn aV V0) and the separable field factor exp(-i sgn e.x), whose
// x-dependence along the thread's elements is a geometric sequence (ratio
// exp(-i sgn e_x T dx)) advanced by FP64 complex multiplication.
template <typename R, int N, int RAD, int THREADS, int WPE>
__global__ void __launch_bounds__((RowTile<N, RAD, THREADS>::NT)) __attribute__((amdgpu_waves_per_eu(WPE)))
k_xpass(cx<R> *__restrict__ psi, int ny, const VStore<R> *__restrict__ V0, const TwEntry<R> *__restrict__ tw,
        PhaseArgs ph, int mode)
{
    using Sh = LineShape<N, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV, ROWS = RowTile<N, RAD, THREADS>::ROWS;
    using Map = RowMap<R, RAD>;
    __shared__ cx<R> lds[ROWS * Map::slots(N)];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int64_t row = (int64_t)blockIdx.x * ROWS + line;
    cx<R> *p = psi + row * N;
    cx<R> *sh = lds + line * Map::slots(N);
    cx<R> v[RV];
    VStore<R> vv[RV];
#pragma unroll
    for (int m = 0; m < RV; ++m) v[m] = p[t + m * T];
    if (mode & M_PHASE) {
        // issue the potential loads now; they complete under the inverse transform
        const VStore<R> *vr = V0 + row * N;
#pragma unroll
        for (int m = 0; m < RV; ++m) vv[m] = vr[t + m * T];
    }
    if (mode & M_INV) fft_line<R, N, RAD, +1, Map>(v, sh, t, tw);
    if (mode & M_PHASE) {
        const int64_t y = row % ny, z = row / ny;
        const double sg = (double)ph.sgn;
        const double base = ph.e[1] * (ph.xmin[1] + (double)y * ph.dx[1]) +
                            ph.e[2] * (ph.xmin[2] + (double)z * ph.dx[2]);
        if (sizeof(R) == 4 && ph.small32) {
            // |theta| <= 1/8 everywhere: theta in FP64, then exp(-i theta) = 1 + (cm - i s)
            // with cm = cos - 1 and s = sin in FP32, and psi + psi (cm - i s): the only
            // rounding at the size of psi is the final addition.
            const double x0 = ph.xmin[0] + (double)t * ph.dx[0], xs = (double)T * ph.dx[0];
#pragma unroll
            for (int m = 0; m < RV; ++m) {
                const double th = sg * (ph.aV * (double)vv[m] + ph.e[0] * (x0 + (double)m * xs) + base);
                const float x = (float)th, x2 = x * x;
                float ps = __builtin_fmaf(x2, -1.0f / 5040.0f, 1.0f / 120.0f);
                ps = __builtin_fmaf(ps, x2, -1.0f / 6.0f);
                const float sn = __builtin_fmaf(ps * x2, x, x);
                float pc = __builtin_fmaf(x2, 1.0f / 40320.0f, -1.0f / 720.0f);
                pc = __builtin_fmaf(pc, x2, 1.0f / 24.0f);
                pc = __builtin_fmaf(pc, x2, -0.5f);
                const float cm = pc * x2;
                const float a = (float)v[m].re, b = (float)v[m].im;
                const float dr = __builtin_fmaf(a, cm, b * sn);
                const float di = __builtin_fmaf(b, cm, -(a * sn));
                v[m].re = (R)(a + dr);
                v[m].im = (R)(b + di);
            }
        } else {
            double s0, c0, s1, c1;
            sincos_fp64(sg * (ph.e[0] * (ph.xmin[0] + (double)t * ph.dx[0]) + base), s0, c0);
            sincos_fp64(sg * ph.e[0] * ((double)T * ph.dx[0]), s1, c1);
            double fr = c0, fi = -s0;  // exp(-i sg e.x) at x = t
            const double wr = c1, wi = -s1;
#pragma unroll
            for (int m = 0; m < RV; ++m) {
                const double th = sg * ph.aV * (double)vv[m];
                double sv, cv;
                if (ph.small) sincos_small(th, sv, cv);
                else sincos_fp64(th, sv, cv);
                // (cv - i sv) (fr + i fi)
                v[m] = mul_phase(v[m], cv * fr + sv * fi, cv * fi - sv * fr);
                const double nr = fr * wr - fi * wi;
                fi = fr * wi + fi * wr;
                fr = nr;
                if ((m & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bound the interleaving
            }
        }
    }
    if (mode & M_FWD) fft_line<R, N, RAD, -1, Map>(v, sh, t, tw);
#pragma unroll
    for (int m = 0; m < RV; ++m) p[t + m * T] = v[m];
}

// ------------------------------------------------------------ column pass --
// Lines run along a strided axis (stride elements apart); one work-group
// holds C adjacent lines so that each global access moves C contiguous
// values.  Thread (t, c) owns elements t + m T of line c.  Work-groups are
// dispatched round-robin over the 8 XCDs; the group index is remapped so
// that consecutive column groups, which share cache lines, run on the same
// XCD (and so share its L2) at about the same time.
template <typename R, int N, int RAD, int C, int WPE>
__global__ void __launch_bounds__((C * LineShape<N, RAD>::T)) __attribute__((amdgpu_waves_per_eu(WPE)))
k_colpass(cx<R> *__restrict__ psi, int64_t stride, int64_t slab_stride, const TwEntry<R> *__restrict__ tw,
          KinArgs kin, int mode)
{
    using Sh = LineShape<N, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV;
    using Map = ColMap<C>;
    __shared__ cx<R> lds[Map::slots(N)];
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const unsigned G = gridDim.x * gridDim.y;
    unsigned L = blockIdx.x + gridDim.x * blockIdx.y;
    if ((G & 7u) == 0) L = (L & 7u) * (G >> 3) + (L >> 3);
    const unsigned gx = L % gridDim.x, slab = L / gridDim.x;
    const int64_t col = (int64_t)gx * C + c;
    cx<R> *p = psi + (int64_t)slab * slab_stride + col;
    cx<R> *sh = lds + c;
    cx<R> v[RV];
#pragma unroll
    for (int m = 0; m < RV; ++m) v[m] = p[(int64_t)(t + m * T) * stride];
    if (mode & M_FWD) fft_line<R, N, RAD, -1, Map>(v, sh, t, tw);
    if (mode & M_KIN) {
        const double2 a = kin.kA[col % kin.nA], b = kin.kB[col / kin.nA];
        const double kcr = a.x * b.x - a.y * b.y, kci = a.x * b.y + a.y * b.x;
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const double2 l = kin.kL[t + m * T];
            const double kr = kcr * l.x - kci * l.y, ki = kcr * l.y + kci * l.x;
            v[m] = mul_phase(v[m], kr, (double)kin.sgn * ki);
        }
    }
    if (mode & M_INV) fft_line<R, N, RAD, +1, Map>(v, sh, t, tw);
#pragma unroll
    for (int m = 0; m < RV; ++m) p[(int64_t)(t + m * T) * stride] = v[m];
}

// ------------------------------------------------------ variant dispatch --
template <typename R, int N, int V> constexpr bool row_variant_ok()
{
    constexpr RowVariant rv = kRowVariants[V];
    using Tl = RowTile<N, rv.rad, rv.threads>;
    if (N < 256 && V != 0) return false;  // short rows: default shape only
    return Tl::NT <= 1024 && Tl::ROWS * RowMap<R, rv.rad>::slots(N) * (int)sizeof(cx<R>) <= 160 * 1024;
}

template <typename R, int N, int V>
hipError_t row_launch(cx<R> *psi, int64_t nrows, int ny, const void *V0, const void *const *tws,
                      const PhaseArgs &ph, int mode, hipStream_t st)
{
    if constexpr (!row_variant_ok<R, N, V>()) {
        return hipErrorInvalidValue;
    } else {
        constexpr RowVariant rv = kRowVariants[V];
        const void *tw = tws[rv.rad == 8 ? 0 : 1];
        using Tl = RowTile<N, rv.rad, rv.threads>;
        if (nrows % Tl::ROWS) {
            // fewer rows than a work-group holds (a single 1-D line): one row per group
            hipLaunchKernelGGL((k_xpass<R, N, rv.rad, LineShape<N, rv.rad>::T, 0>), dim3((unsigned)nrows),
                               dim3(LineShape<N, rv.rad>::T), 0, st, psi, ny, (const VStore<R> *)V0,
                               (const TwEntry<R> *)tw, ph, mode);
        } else {
            hipLaunchKernelGGL((k_xpass<R, N, rv.rad, rv.threads, rv.wpe>), dim3((unsigned)(nrows / Tl::ROWS)),
                               dim3(Tl::NT), 0, st, psi, ny, (const VStore<R> *)V0, (const TwEntry<R> *)tw, ph,
                               mode);
        }
        return hipGetLastError();
    }
}

template <typename R, int N, size_t... I>
hipError_t row_dispatch(int var, cx<R> *psi, int64_t nrows, int ny, const void *V0, const void *const *tw,
                        const PhaseArgs &ph, int mode, hipStream_t st, std::index_sequence<I...>)
{
    hipError_t r = hipErrorInvalidValue;
    ((var == (int)I ? (r = row_launch<R, N, (int)I>(psi, nrows, ny, V0, tw, ph, mode, st), 0) : 0), ...);
    return r;
}

template <typename R, int N, int V> constexpr bool col_variant_ok()
{
    constexpr ColVariant cv = kColVariants[V];
    if (N < 256 && V != 0) return false;
    return cv.cols * LineShape<N, cv.rad>::T <= 1024 &&
           ColMap<cv.cols>::slots(N) * (int)sizeof(cx<R>) <= 160 * 1024;
}

template <typename R, int N, int V>
hipError_t col_launch(cx<R> *psi, int64_t ncols, int64_t stride, int nslab, int64_t slab_stride,
                      const void *const *tws, const KinArgs &kin, int mode, hipStream_t st)
{
    if constexpr (!col_variant_ok<R, N, V>()) {
        return hipErrorInvalidValue;
    } else {
        constexpr ColVariant cv = kColVariants[V];
        const void *tw = tws[cv.rad == 8 ? 0 : 1];
        if (ncols % cv.cols) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_colpass<R, N, cv.rad, cv.cols, cv.wpe>), dim3((unsigned)(ncols / cv.cols), (unsigned)nslab),
                           dim3(cv.cols * LineShape<N, cv.rad>::T), 0, st, psi, stride, slab_stride,
                           (const TwEntry<R> *)tw, kin, mode);
        return hipGetLastError();
    }
}

template <typename R, int N, size_t... I>
hipError_t col_dispatch(int var, cx<R> *psi, int64_t ncols, int64_t stride, int nslab, int64_t slab_stride,
                        const void *const *tw, const KinArgs &kin, int mode, hipStream_t st, std::index_sequence<I...>)
{
    hipError_t r = hipErrorInvalidValue;
    ((var == (int)I ? (r = col_launch<R, N, (int)I>(psi, ncols, stride, nslab, slab_stride, tw, kin, mode, st), 0)
                    : 0),
     ...);
    return r;
}

#define SFO_SWITCH_PASS_N(N_, CALL)   \
    switch (N_) {                     \
    case 64: return CALL(64);         \
    case 128: return CALL(128);       \
    case 256: return CALL(256);       \
    case 512: return CALL(512);       \
    case 1024: return CALL(1024);     \
    case 2048: return CALL(2048);     \
    case 4096: return CALL(4096);     \
    default: return hipErrorInvalidValue; \
    }

}  // namespace sfo
