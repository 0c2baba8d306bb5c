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

// Sum of v over the work-group (all threads), FP64, deterministic order;
// every thread returns the total.  red: 16 x 3 doubles of LDS.
__device__ __forceinline__ void block_sum3(double (&v)[3], double (*red)[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
        for (int off = 32; off > 0; off >>= 1) v[a] += __shfl_xor(v[a], off, 64);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) red[w][a] = v[a];
    __syncthreads();
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int i = 0; i < nw; ++i) s += red[i][a];
        v[a] = s;
    }
    __syncthreads();
}

// Work-group partial moments -> part[blockIdx.x]; the last group to finish
// sums all partials in a fixed order into out[0..2] and re-arms the counter.
__device__ __forceinline__ void grid_sum3(double (&v)[3], double (*red)[3], double *part, unsigned *count,
                                          double *out)
{
    block_sum3(v, red);
    __shared__ unsigned last;
    if (threadIdx.x == 0) {
        for (int a = 0; a < 3; ++a) part[3 * blockIdx.x + a] = v[a];
        __threadfence();
        last = atomicAdd(count, 1u) == gridDim.x * gridDim.y - 1 ? 1u : 0u;
    }
    __syncthreads();
    if (last) {
        __threadfence();
        const unsigned nb = gridDim.x * gridDim.y;
        double s[3] = {0.0, 0.0, 0.0};
        for (unsigned i = threadIdx.x; i < nb; i += blockDim.x)
            for (int a = 0; a < 3; ++a) s[a] += __builtin_nontemporal_load(part + 3 * i + a);
        block_sum3(s, red);
        if (threadIdx.x == 0) {
            for (int a = 0; a < 3; ++a) out[a] = s[a];
            *count = 0u;
        }
    }
}

// --------------------------------------------------------------- row pass --
// One work-group holds ROWS rows of N points of each of NS states (NS = 2:
// the state and its adjoint, walked back together); thread t of a row owns
// the cyclic elements x = t + m T.  Global access is contiguous along the
// row.  The potential factor exp(-i sgn [aV V0(x) + e.x]) is computed once
// per point and applied to every state.  In FP64 it is a per-point
// exp(-i sgn aV V0) times the separable field factor exp(-i sgn e.x), whose
// x-dependence along the thread's elements is a geometric sequence (ratio
// exp(-i sgn e_x T dx)) advanced by FP64 complex multiplication.
// M_GRAD (NS = 2) additionally forms b = Im(conj(g) psi) at this step
// boundary in real space: acc += w b (the dL/dV0 accumulator) and the
// moments sum_x (x b, y b, z b) reduced over the grid into ga.mom.
template <typename R, int N, int RAD, int THREADS, int WPE, int NS>
__global__ void __launch_bounds__((RowTile<N, RAD, THREADS>::NT)) __attribute__((amdgpu_waves_per_eu(WPE)))
k_xpass(StatePtrs<R> S, int ny, const VStore<R> *__restrict__ V0, const TwEntry<R> *__restrict__ tw,
        PhaseArgs ph, GradArgs ga, int mode)
{
    using Sh = LineShape<N, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV, ROWS = RowTile<N, RAD, THREADS>::ROWS;
    using Map = RowMap<R, RAD>;
    __shared__ cx<R> lds[ROWS * Map::slots(N)];
    __shared__ double red[16][3];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int64_t row = (int64_t)blockIdx.x * ROWS + line;
    cx<R> *sh = lds + line * Map::slots(N);
    cx<R> v[NS][RV];
    VStore<R> vv[RV];
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) v[q][m] = S.p[q][row * N + t + m * T];
    if (mode & M_PHASE) {
        // issue the potential loads now; they complete under the inverse transform
        const VStore<R> *vr = V0 + row * N;
#pragma unroll
        for (int m = 0; m < RV; ++m) vv[m] = vr[t + m * T];
    }
    if (mode & M_INV)
#pragma unroll
        for (int q = 0; q < NS; ++q) fft_line<R, N, RAD, +1, Map>(v[q], sh, t, tw);
    const int64_t y = row % ny, z = row / ny;
    if (mode & M_PHASE) {
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
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    const float a = (float)v[q][m].re, b = (float)v[q][m].im;
                    const float dr = __builtin_fmaf(a, cm, b * sn);
                    const float di = __builtin_fmaf(b, cm, -(a * sn));
                    v[q][m].re = (R)(a + dr);
                    v[q][m].im = (R)(b + di);
                }
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
                const double tr = cv * fr + sv * fi, ti = cv * fi - sv * fr;
#pragma unroll
                for (int q = 0; q < NS; ++q) v[q][m] = mul_phase(v[q][m], tr, ti);
                const double nr = fr * wr - fi * wi;
                fi = fr * wi + fi * wr;
                fr = nr;
                if ((m & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bound the interleaving
            }
        }
    }
    if (NS == 2 && (mode & M_GRAD)) {
        double mom[3] = {0.0, 0.0, 0.0};
        double sb = 0.0;
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const int x = t + m * T;
            const cx<R> ps = v[0][m], gq = v[NS - 1][m];
            const double b = (double)gq.re * (double)ps.im - (double)gq.im * (double)ps.re;
            if (ga.acc) {
                double *ap = ga.acc + row * N + x;
                *ap = (ga.acc_init ? 0.0 : *ap) + ga.wacc * b;
            }
            sb += b;
            mom[0] += (ph.xmin[0] + (double)x * ph.dx[0]) * b;
        }
        mom[1] = (ph.xmin[1] + (double)y * ph.dx[1]) * sb;
        mom[2] = (ph.xmin[2] + (double)z * ph.dx[2]) * sb;
        grid_sum3(mom, red, ga.part, ga.count, ga.mom);
    }
    if (mode & M_FWD)
#pragma unroll
        for (int q = 0; q < NS; ++q) fft_line<R, N, RAD, -1, Map>(v[q], sh, t, tw);
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) S.p[q][row * N + t + m * T] = v[q][m];
}

// ------------------------------------------------------------ column pass --
// Lines run along a strided axis (stride elements apart); one work-group
// holds C adjacent lines (of each of NS states) so that each global access
// moves C contiguous values.  Thread (t, c) owns elements t + m T of line c.
// Work-groups are dispatched round-robin over the 8 XCDs; the group index is
// remapped so that consecutive column groups, which share cache lines, run
// on the same XCD (and so share its L2) at about the same time.
template <typename R, int N, int RAD, int C, int WPE, int NS>
__global__ void __launch_bounds__((C * LineShape<N, RAD>::T)) __attribute__((amdgpu_waves_per_eu(WPE)))
k_colpass(StatePtrs<R> S, int64_t stride, int64_t slab_stride, const TwEntry<R> *__restrict__ tw, KinArgs kin,
          int mode)
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
    const int64_t off = (int64_t)slab * slab_stride + col;
    cx<R> *sh = lds + c;
    cx<R> v[NS][RV];
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) v[q][m] = S.p[q][off + (int64_t)(t + m * T) * stride];
    if (mode & M_FWD)
#pragma unroll
        for (int q = 0; q < NS; ++q) fft_line<R, N, RAD, -1, Map>(v[q], sh, t, tw);
    if (mode & M_KIN) {
        const double2 a = kin.kA[col % kin.nA], b = kin.kB[col / kin.nA];
        const double kcr = a.x * b.x - a.y * b.y, kci = a.x * b.y + a.y * b.x;
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const double2 l = kin.kL[t + m * T];
            const double kr = kcr * l.x - kci * l.y, ki = kcr * l.y + kci * l.x;
#pragma unroll
            for (int q = 0; q < NS; ++q) v[q][m] = mul_phase(v[q][m], kr, (double)kin.sgn * ki);
        }
    }
    if (mode & M_INV)
#pragma unroll
        for (int q = 0; q < NS; ++q) fft_line<R, N, RAD, +1, Map>(v[q], sh, t, tw);
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) S.p[q][off + (int64_t)(t + m * T) * stride] = v[q][m];
}

// ------------------------------------------------------ variant dispatch --
template <typename R, int N, int V> constexpr bool row_variant_ok()
{
    constexpr RowVariant rv = kRowVariants[V];
    using Tl = RowTile<N, rv.rad, rv.threads>;
    if (N < 256 && V != 0) return false;  // short rows: default shape only
    return Tl::NT <= 1024 && Tl::ROWS * RowMap<R, rv.rad>::slots(N) * (int)sizeof(cx<R>) <= 160 * 1024;
}

template <typename R, int N, int V, int NS>
hipError_t row_launch(const StatePtrs<R> &S, int64_t nrows, int ny, const void *V0, const void *const *tws,
                      const PhaseArgs &ph, const GradArgs &ga, int mode, hipStream_t st)
{
    if constexpr (!row_variant_ok<R, N, V>()) {
        return hipErrorInvalidValue;
    } else {
        constexpr RowVariant rv = kRowVariants[V];
        const void *tw = tws[rv.rad == 8 ? 0 : 1];
        using Tl = RowTile<N, rv.rad, rv.threads>;
        if (nrows % Tl::ROWS) {
            // fewer rows than a work-group holds (a single 1-D line): one row per group
            hipLaunchKernelGGL((k_xpass<R, N, rv.rad, LineShape<N, rv.rad>::T, 1, NS>), dim3((unsigned)nrows),
                               dim3(LineShape<N, rv.rad>::T), 0, st, S, ny, (const VStore<R> *)V0,
                               (const TwEntry<R> *)tw, ph, ga, mode);
        } else {
            hipLaunchKernelGGL((k_xpass<R, N, rv.rad, rv.threads, rv.wpe, NS>), dim3((unsigned)(nrows / Tl::ROWS)),
                               dim3(Tl::NT), 0, st, S, ny, (const VStore<R> *)V0, (const TwEntry<R> *)tw, ph, ga,
                               mode);
        }
        return hipGetLastError();
    }
}

template <typename R, int N, int NS, size_t... I>
hipError_t row_dispatch(int var, const StatePtrs<R> &S, int64_t nrows, int ny, const void *V0,
                        const void *const *tw, const PhaseArgs &ph, const GradArgs &ga, int mode, hipStream_t st,
                        std::index_sequence<I...>)
{
    hipError_t r = hipErrorInvalidValue;
    ((var == (int)I ? (r = row_launch<R, N, (int)I, NS>(S, nrows, ny, V0, tw, ph, ga, mode, st), 0) : 0), ...);
    return r;
}

template <typename R, int N, int V> constexpr bool col_variant_ok()
{
    constexpr ColVariant cv = kColVariants[V];
    if (N < 256 && V != 0) return false;
    return cv.cols * LineShape<N, cv.rad>::T <= 1024 &&
           ColMap<cv.cols>::slots(N) * (int)sizeof(cx<R>) <= 160 * 1024;
}

template <typename R, int N, int V, int NS>
hipError_t col_launch(const StatePtrs<R> &S, int64_t ncols, int64_t stride, int nslab, int64_t slab_stride,
                      const void *const *tws, const KinArgs &kin, int mode, hipStream_t st)
{
    if constexpr (!col_variant_ok<R, N, V>()) {
        return hipErrorInvalidValue;
    } else {
        constexpr ColVariant cv = kColVariants[V];
        const void *tw = tws[cv.rad == 8 ? 0 : 1];
        if (ncols % cv.cols) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_colpass<R, N, cv.rad, cv.cols, cv.wpe, NS>),
                           dim3((unsigned)(ncols / cv.cols), (unsigned)nslab), dim3(cv.cols * LineShape<N, cv.rad>::T),
                           0, st, S, stride, slab_stride, (const TwEntry<R> *)tw, kin, mode);
        return hipGetLastError();
    }
}

template <typename R, int N, int NS, size_t... I>
hipError_t col_dispatch(int var, const StatePtrs<R> &S, int64_t ncols, int64_t stride, int nslab,
                        int64_t slab_stride, const void *const *tw, const KinArgs &kin, int mode, hipStream_t st,
                        std::index_sequence<I...>)
{
    hipError_t r = hipErrorInvalidValue;
    ((var == (int)I ? (r = col_launch<R, N, (int)I, NS>(S, ncols, stride, nslab, slab_stride, tw, kin, mode, st), 0)
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
