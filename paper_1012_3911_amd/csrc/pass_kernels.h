// Row (x) and column (strided) line passes of the Schroedinger step, as
// templates over the tile shape so that the planner can pick, per line
// length and precision, how many lines a work-group holds, the register
// radix and an occupancy hint.  Included by the per-precision instantiation
// units sfo_row.hip and sfo_col.hip.
#pragma once
#include <utility>

#include <hip/hip_ext.h>

#include "sfo_impl.h"

namespace sfo {

template <typename R> using VStore = typename std::conditional<sizeof(R) == 4, float, double>::type;
template <typename VT> __device__ __forceinline__ double ldv(const VT *p) { return (double)*p; }

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

// Potential factor of a grouped row pass for problem P, covering the half
// steps sa and sb (-1: absent); the same arguments the host forms for a
// single grid (phase_args in sfo_api.hip).
template <typename R>
__device__ __forceinline__ PhaseArgs group_phase(const BatchProb<R> &P, int64_t sa, int64_t sb, int sgn)
{
    PhaseArgs ph{};
    const int halves = (sa >= 0) + (sb >= 0);
    ph.aV = P.aV_half * halves;
    double bound = ph.aV * P.v0max;
    for (int a = 0; a < 3; ++a) {
        double e = 0.0;
        if (a < P.ndim && P.ebar) {
            if (sa >= 0) e += P.ebar[sa * P.ndim + a];
            if (sb >= 0) e += P.ebar[sb * P.ndim + a];
        }
        ph.e[a] = e * P.inv_2hbar;
        ph.xmin[a] = a < P.ndim ? P.xmin[a] : 0.0;
        ph.dx[a] = a < P.ndim ? P.dx[a] : 0.0;
        if (a < P.ndim) bound += fabs(ph.e[a]) * P.xabs[a];
    }
    ph.sgn = sgn;
    ph.small = ph.aV * P.v0max <= 0.125 ? 1 : 0;
    ph.small32 = bound <= 0.125 ? 1 : 0;
    return ph;
}

// The arguments of a grouped row pass for this work-group's problem.
template <typename R, int NS>
__device__ __forceinline__ void group_row_args(const GroupArgs<R> &grp, StatePtrs<R> &S,
                                               const VStore<R> *__restrict__ &V0, PhaseArgs &ph, GradArgs &ga)
{
    const BatchProb<R> &P = grp.probs[grp.ids[blockIdx.y]];
    S.p[0] = P.psi;
    S.p[1] = NS == 2 ? P.gadj : nullptr;
    V0 = P.V0;
    ph = group_phase(P, grp.sa, grp.sb, ph.sgn);
    if (NS == 2) {
        ga.acc = P.dV;
        ga.wacc = grp.wmul * P.aV_half;
        ga.acc_init = grp.acc_init;
        ga.part = P.part + 3 * (int64_t)gridDim.x * grp.jmom;
    }
}

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

// Work-group moment partials -> part[3 blockIdx.x + a]; the slots are summed
// by a later kernel, so no fence or counter is needed here.
__device__ __forceinline__ void block_part3(double (&v)[3], double (*red)[3], double *part)
{
    block_sum3(v, red);
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) part[3 * blockIdx.x + a] = v[a];
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
// moments sum_x (x b, y b, z b), summed over the work-group into ga.part.
//
// Row tile addressing: the base of element m of the tile's first row is
// uniform and is kept in scalar registers (scalar_base: an opaque copy stops
// the compiler from folding it into a 64-bit vector address); a thread adds
// its own 32-bit offset (line * N + t) * size.  scalar_base is only for
// values uniform over the work-group.
template <typename P> __device__ __forceinline__ P scalar_base(P p)
{
    __asm__ __volatile__("" : "+s"(p));
    return p;
}

template <typename R, int N, int RAD, int NS, int NV>
__device__ __forceinline__ void row_load(cx<R> (&v)[NS][NV], const StatePtrs<R> &S, int64_t row0,
                                         uint32_t lt)
{
    static_assert(NV == LineShape<N, RAD>::RV, "register array size must match the line shape");
    constexpr int T = LineShape<N, RAD>::T, RV = LineShape<N, RAD>::RV;
    const uint32_t tb = lt * (uint32_t)sizeof(cx<R>);
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const char *b = scalar_base((const char *)(S.p[q] + row0 * N + m * T));
            v[q][m] = gload((const cx<R> *)(b + tb));
        }
}

template <typename R, int N, int RAD, int NS, int NV>
__device__ __forceinline__ void row_store(const cx<R> (&v)[NS][NV], const StatePtrs<R> &S,
                                          int64_t row0, uint32_t lt)
{
    static_assert(NV == LineShape<N, RAD>::RV, "register array size must match the line shape");
    constexpr int T = LineShape<N, RAD>::T, RV = LineShape<N, RAD>::RV;
    const uint32_t tb = lt * (uint32_t)sizeof(cx<R>);
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            char *b = scalar_base((char *)(S.p[q] + row0 * N + m * T));
            gstore((cx<R> *)(b + tb), v[q][m]);
        }
}

template <typename R, int N, int RAD, int NV>
__device__ __forceinline__ void row_load_v0(VStore<R> (&vv)[NV], const VStore<R> *__restrict__ V0,
                                            int64_t row0, uint32_t lt)
{
    static_assert(NV == LineShape<N, RAD>::RV, "register array size must match the line shape");
    constexpr int T = LineShape<N, RAD>::T, RV = LineShape<N, RAD>::RV;
    const uint32_t tb = lt * (uint32_t)sizeof(VStore<R>);
#pragma unroll
    for (int m = 0; m < RV; ++m) {
        const char *b = scalar_base((const char *)(V0 + row0 * N + m * T));
        vv[m] = gload1((const VStore<R> *)(b + tb));
    }
}

// The register part of a row tile: inverse x-transform, potential factor,
// gradient partials (mom accumulates this row's moments), forward
// x-transform.  sh: this row's LDS exchange region; tw: twiddle table
// (global or an LDS copy).
// PRE (complex128; complex64 radix-16 rows always do it): the stage factors
// are formed from wb, each stage's W^k read with the line.
template <typename R, int N, int RAD, int NS, bool PAD, bool PRE = false, int NV>
__device__ __forceinline__ void row_body(cx<R> (&v)[NS][NV],
                                         VStore<R> (&vv)[NV], int64_t row0, int line, int ny, cx<R> *sh, int t,
                                         const TwEntry<R> *__restrict__ tw, const TwBase<N, RAD> &wb, const PhaseArgs &ph,
                                         const GradArgs &ga, int mode, double (&mom)[3],
                                         const VStore<R> *__restrict__ V0late = nullptr)
{
    static_assert(NV == LineShape<N, RAD>::RV, "register array size must match the line shape");
    // everything below is derived from an opaque copy of t: in a persistent
    // loop the compiler would otherwise keep every tile-invariant value (16
    // x coordinates, exchange addresses) live across all tiles
    __asm__ __volatile__("" : "+v"(t));
    using Sh = LineShape<N, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV;
    using Map = RowMap<R, RAD, PAD>;
    if (mode & M_INV)
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            if constexpr (PRE)
                fft_line_pre<R, N, RAD, +1, Map>(v[q], sh, t, tw, wb);
            else if constexpr (RAD == 16)
                fft_line<R, N, RAD, +1, Map>(v[q], sh, t, tw, wb);
            else
                fft_line<R, N, RAD, +1, Map>(v[q], sh, t, tw);
        }
    // potential loaded here rather than before the transform: fewer registers held through it
    const int64_t row = row0 + line;
    const uint32_t lt = (uint32_t)(line * N + t);
    if (V0late && (mode & M_PHASE)) row_load_v0<R, N, RAD>(vv, V0late, row0, lt);
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
                // the factor does not depend on psi; pinning its input here keeps
                // the compiler from computing all of them during the transform
                VStore<R> vm = vv[m];
                __asm__ __volatile__("" : "+v"(vm));
                const double th = sg * (ph.aV * (double)vm + ph.e[0] * (x0 + (double)m * xs) + base);
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
            // one straight loop per series (the choice is uniform): a branch per
            // point would split the loop into blocks and keep every value live
            // across them
            auto sweep = [&](auto sincos) {
#pragma unroll
                for (int m = 0; m < RV; ++m) {
                    // pin this point's values here; the conversions to FP64 are
                    // common to both loops and would otherwise all be hoisted
                    // above the choice, holding 16 points in FP64 registers
#pragma unroll
                    for (int q = 0; q < NS; ++q) __asm__ __volatile__("" : "+v"(v[q][m].re), "+v"(v[q][m].im));
                    VStore<R> vm = vv[m];
                    __asm__ __volatile__("" : "+v"(vm));
                    const double th = sg * ph.aV * (double)vm;
                    double sv, cv;
                    sincos(th, sv, cv);
                    // (cv - i sv) (fr + i fi)
                    const double tr = cv * fr + sv * fi, ti = cv * fi - sv * fr;
#pragma unroll
                    for (int q = 0; q < NS; ++q) v[q][m] = mul_phase(v[q][m], tr, ti);
                    const double nr = fr * wr - fi * wi;
                    fi = fr * wi + fi * wr;
                    fr = nr;
                    if ((m & 1) == 1) __builtin_amdgcn_sched_barrier(0);  // bound the interleaving
                }
            };
            if (ph.small)
                sweep([](double x, double &sn, double &cs) { sincos_small(x, sn, cs); });
            else
                sweep([](double x, double &sn, double &cs) { sincos_fp64(x, sn, cs); });
        }
    }
    if (NS == 2 && (mode & M_GRAD)) {
        double sb = 0.0;
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const int x = t + m * T;
            const cx<R> ps = v[0][m], gq = v[NS - 1][m];
            const double b = (double)gq.re * (double)ps.im - (double)gq.im * (double)ps.re;
            if (ga.acc) {
                double *ap = (double *)(scalar_base((char *)(ga.acc + row0 * N + m * T)) + lt * sizeof(double));
                gstore1(ap, (ga.acc_init ? 0.0 : gload1(ap)) + ga.wacc * b);
            }
            sb += b;
            mom[0] += (ph.xmin[0] + (double)x * ph.dx[0]) * b;
        }
        mom[1] += (ph.xmin[1] + (double)y * ph.dx[1]) * sb;
        mom[2] += (ph.xmin[2] + (double)z * ph.dx[2]) * sb;
    }
    if (mode & M_FWD)
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            if constexpr (PRE)
                fft_line_pre<R, N, RAD, -1, Map>(v[q], sh, t, tw, wb);
            else if constexpr (RAD == 16)
                fft_line<R, N, RAD, -1, Map>(v[q], sh, t, tw, wb);
            else
                fft_line<R, N, RAD, -1, Map>(v[q], sh, t, tw);
        }
}

template <typename R, int N, int RAD, int ROWS, int NS, bool PAD = (RAD == 16), bool LATE = false, bool PRE = false>
__device__ __forceinline__ void row_tile(const StatePtrs<R> &S, int64_t row0, int ny, const VStore<R> *__restrict__ V0,
                                         const TwEntry<R> *__restrict__ tw, const PhaseArgs &ph, const GradArgs &ga,
                                         int mode, cx<R> *lds, double (*red)[3], int tid)
{
    using Sh = LineShape<N, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV;
    const int line = tid / T, t = tid % T;
    cx<R> *sh = lds + line * RowMap<R, RAD, PAD>::slots(N);
    cx<R> v[NS][RV];
    VStore<R> vv[RV];
    uint32_t lt = (uint32_t)(line * N + t);
    // complex64 radix-16 rows read their stage twiddles here, with the line
    // (measured: faster for these; radix-8 rows and columns read them per stage)
    TwBase<N, RAD> wb;
    if constexpr ((std::is_same<R, float>::value && RAD == 16) || PRE) tw_base_load(wb, tw, t);
    row_load<R, N, RAD, NS>(v, S, row0, lt);
    // the potential loads complete under the inverse transform (or, LATE, are issued after it)
    if (!LATE && (mode & M_PHASE)) row_load_v0<R, N, RAD>(vv, V0, row0, lt);
    double mom[3] = {0.0, 0.0, 0.0};
    row_body<R, N, RAD, NS, PAD, PRE>(v, vv, row0, line, ny, sh, t, tw, wb, ph, ga, mode, mom, LATE ? V0 : nullptr);
    // the offset is recomputed rather than held through the transforms
    __asm__ __volatile__("" : "+v"(lt));
    row_store<R, N, RAD, NS>(v, S, row0, lt);
    if (NS == 2 && (mode & M_GRAD)) block_part3(mom, red, ga.part);
}

template <typename R, int N, int RAD, int THREADS, int WPE, int NS, bool PAD = (RAD == 16), bool LATE = false,
          bool PRE = false>
__global__ void __launch_bounds__((RowTile<N, RAD, THREADS>::NT)) __attribute__((amdgpu_waves_per_eu(WPE)))
k_xpass(StatePtrs<R> S, int ny, const VStore<R> *__restrict__ V0, const TwEntry<R> *__restrict__ tw,
        PhaseArgs ph, GradArgs ga, int mode, GroupArgs<R> grp)
{
    constexpr int ROWS = RowTile<N, RAD, THREADS>::ROWS;
    if (grp.probs) group_row_args<R, NS>(grp, S, V0, ph, ga);
    __shared__ cx<R> lds[ROWS * RowMap<R, RAD, PAD>::slots(N)];
    __shared__ double red[16][3];
    row_tile<R, N, RAD, ROWS, NS, PAD, LATE, PRE>(S, (int64_t)blockIdx.x * ROWS, ny, V0, tw, ph, ga, mode, lds, red,
                                                  threadIdx.x);
}

// ------------------------------------------------------------ column pass --
// Lines run along a strided axis (stride elements apart); one work-group
// holds C adjacent lines (of each of NS states) so that each global access
// moves C contiguous values.  Thread (t, c) owns elements t + m T of line c.
// Work-groups are dispatched round-robin over the 8 XCDs; the group index is
// remapped so that consecutive column groups, which share cache lines, run
// on the same XCD (and so share its L2) at about the same time.
// Addresses: the work-group's base (slab, first line) and the distance
// between a thread's elements are uniform and live in scalar registers; a
// thread adds only its own 32-bit byte offset tb = (t stride + c) * size, so
// each access is a scalar-base + vector-offset load or store with no 64-bit
// vector arithmetic (the launcher checks that tb fits 32 bits).
template <typename R, int N, int RAD, int NS, int NV>
__device__ __forceinline__ void col_load(cx<R> (&v)[NS][NV], const StatePtrs<R> &S, int64_t ubase,
                                         int64_t stride, uint32_t tb)
{
    static_assert(NV == LineShape<N, RAD>::RV, "register array size must match the line shape");
    constexpr int T = LineShape<N, RAD>::T, RV = LineShape<N, RAD>::RV;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const char *b = (const char *)(S.p[q] + ubase);
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            // opaque scalar base: keeps the compiler from folding the uniform
            // part into a 64-bit vector address
            const char *bm = b + (int64_t)m * T * stride * (int64_t)sizeof(cx<R>);
            __asm__ __volatile__("" : "+s"(bm));
            v[q][m] = gload((const cx<R> *)(bm + tb));
        }
    }
}
// elements m in [M0, M1) of each line only (a load issued in parts)
template <typename R, int N, int RAD, int M0, int M1, int NV>
__device__ __forceinline__ void col_load_part(cx<R> (&v)[1][NV], const StatePtrs<R> &S, int64_t ubase,
                                              int64_t stride, uint32_t tb)
{
    constexpr int T = LineShape<N, RAD>::T;
    const char *b = (const char *)(S.p[0] + ubase);
#pragma unroll
    for (int m = M0; m < M1; ++m) {
        const char *bm = b + (int64_t)m * T * stride * (int64_t)sizeof(cx<R>);
        __asm__ __volatile__("" : "+s"(bm));
        v[0][m] = gload((const cx<R> *)(bm + tb));
    }
}
template <typename R, int N, int RAD, int NS, int NV>
__device__ __forceinline__ void col_store(const cx<R> (&v)[NS][NV], const StatePtrs<R> &S,
                                          int64_t ubase, int64_t stride, uint32_t tb)
{
    static_assert(NV == LineShape<N, RAD>::RV, "register array size must match the line shape");
    constexpr int T = LineShape<N, RAD>::T, RV = LineShape<N, RAD>::RV;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        char *b = (char *)(S.p[q] + ubase);
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            char *bm = b + (int64_t)m * T * stride * (int64_t)sizeof(cx<R>);
            __asm__ __volatile__("" : "+s"(bm));
            gstore((cx<R> *)(bm + tb), v[q][m]);
        }
    }
}

// Forward transform, kinetic factor kc[q] * kL[j] (kc[q]: the factor of
// state q's line from the other axes), inverse transform.  kL: global table
// or an LDS copy.
// PRE: the stage factors are formed from wb (each stage's W^k, read once per
// work-group) instead of being read from the table in every stage.
template <typename R, int N, int RAD, int C, int NS, bool PRE = false, int NV>
__device__ __forceinline__ void col_body(cx<R> (&v)[NS][NV], const double (&kcr)[NS], const double (&kci)[NS],
                                         int sgn, const double2 *kL, cx<R> *sh, int t,
                                         const TwEntry<R> *__restrict__ tw, int mode,
                                         const TwBase<N, RAD> *wb = nullptr)
{
    static_assert(NV == LineShape<N, RAD>::RV, "register array size must match the line shape");
    __asm__ __volatile__("" : "+v"(t));  // see row_body
    constexpr int T = LineShape<N, RAD>::T, RV = LineShape<N, RAD>::RV;
    using Map = ColMap<C>;
    auto transform = [&](auto dir, cx<R>(&x)[NV]) {
        constexpr int D = decltype(dir)::value;
        if constexpr (PRE)
            fft_line_pre<R, N, RAD, D, Map>(x, sh, t, tw, *wb);
        else
            fft_line<R, N, RAD, D, Map>(x, sh, t, tw);
    };
    if (mode & M_FWD)
#pragma unroll
        for (int q = 0; q < NS; ++q) transform(std::integral_constant<int, -1>{}, v[q]);
    if (mode & M_KIN) {
        // index laundered after the transform: the table loads stay here
        // instead of being hoisted above it (16 FP64 pairs held through it)
        uint32_t tk = (uint32_t)t * (uint32_t)sizeof(double2);
        __asm__ __volatile__("" : "+v"(tk));
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const cx<double> l = gload((const cx<double> *)((const char *)kL + m * T * (int)sizeof(double2) + tk));
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const double kr = kcr[q] * l.re - kci[q] * l.im, ki = kcr[q] * l.im + kci[q] * l.re;
                v[q][m] = mul_phase(v[q][m], kr, (double)sgn * ki);
            }
            // complex64: four points at a time; complex128 issues every table
            // load at once (measured faster; its register budget allows it)
            constexpr int KG = sizeof(R) == 8 ? 16 : 4;
            if ((m & (KG - 1)) == KG - 1) __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (mode & M_INV)
#pragma unroll
        for (int q = 0; q < NS; ++q) transform(std::integral_constant<int, +1>{}, v[q]);
}

template <typename R, int N, int RAD, int C, int NS, bool CHI, bool VGRAD = false, bool PRE = false>
__device__ __forceinline__ void col_tile(const StatePtrs<R> &S, int64_t gx, int64_t slab, int64_t stride,
                                         int64_t slab_stride, const TwEntry<R> *__restrict__ tw, const KinArgs &kin,
                                         int mode, cx<R> *lds, double (*red)[3], int tid)
{
    constexpr int RV = LineShape<N, RAD>::RV;
    constexpr int W = C;  // lines per work-group
    const int c = tid % C, t = tid / C;
    const int64_t ubase = slab * slab_stride + gx * W;
    uint32_t tb = ((uint32_t)t * (uint32_t)stride + (uint32_t)c) * (uint32_t)sizeof(cx<R>);
    cx<R> v[NS][RV];
    col_load<R, N, RAD, NS>(v, S, ubase, stride, tb);
    double kcr[NS], kci[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        kcr[q] = 1.0;
        kci[q] = 0.0;
        if (mode & M_KIN) {
            const int64_t col = gx * W + c;
            const cx<double> a = gload((const cx<double> *)kin.kA + col % kin.nA),
                             b = gload((const cx<double> *)kin.kB + col / kin.nA);
            kcr[q] = a.re * b.re - a.im * b.im;
            kci[q] = a.re * b.im + a.im * b.re;
        }
    }
    if constexpr (CHI) {
        // overlap of the transformed state with the reference (same layout), between the
        // forward transform and the kinetic factor (a kernel of its own: the
        // extra code would otherwise cost the plain pass registers)
        col_body<R, N, RAD, C, NS>(v, kcr, kci, kin.sgn, kin.kL, lds + c, t, tw, mode & M_FWD);
        constexpr int T = LineShape<N, RAD>::T;
        const char *rb = (const char *)((const cx<R> *)kin.chi_ref + ubase);
        double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const cx<R> r = gload((const cx<R> *)(rb + (int64_t)m * T * stride * (int64_t)sizeof(cx<R>) + tb));
            const cx<R> a = v[0][m];
            acc[0] += (double)r.re * (double)a.re + (double)r.im * (double)a.im;
            acc[1] += (double)r.re * (double)a.im - (double)r.im * (double)a.re;
        }
        block_sum3(acc, red);
        if (tid == 0) {
            const int64_t slot = (int64_t)blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
            gstore1(kin.chi_part + 2 * slot, acc[0]);
            gstore1(kin.chi_part + 2 * slot + 1, acc[1]);
        }
        col_body<R, N, RAD, C, NS>(v, kcr, kci, kin.sgn, kin.kL, lds + c, t, tw, mode & (M_KIN | M_INV));
    } else if constexpr (VGRAD) {
        // velocity-gauge gradient partials of the reverse sweep: with psi~ and g~
        // the states right after the forward transform (k-space), the sums of
        // (kA, kB, kL, 1) Im(conj(g~) psi~) over the work-group's points (a
        // kernel of its own, like the overlap above)
        static_assert(NS == 2, "gradient partials need the state and its adjoint");
        col_body<R, N, RAD, C, NS>(v, kcr, kci, kin.sgn, kin.kL, lds + c, t, tw, mode & M_FWD);
        constexpr int T = LineShape<N, RAD>::T;
        const int64_t col = gx * W + c;
        const double ka = kin.kvA[col % kin.nA], kb = kin.kvB ? kin.kvB[col / kin.nA] : 0.0;
        double s1 = 0.0, sl = 0.0;
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const double b = (double)v[1][m].re * (double)v[0][m].im - (double)v[1][m].im * (double)v[0][m].re;
            s1 += b;
            sl += kin.kvL[t + m * T] * b;
        }
        double acc[3] = {ka * s1, kb * s1, sl}, acc2[3] = {s1, 0.0, 0.0};
        block_sum3(acc, red);
        block_sum3(acc2, red);
        if (tid == 0) {
            const int64_t slot = (int64_t)blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
            for (int a = 0; a < 3; ++a) gstore1(kin.vpart + 4 * slot + a, acc[a]);
            gstore1(kin.vpart + 4 * slot + 3, acc2[0]);
        }
        col_body<R, N, RAD, C, NS>(v, kcr, kci, kin.sgn, kin.kL, lds + c, t, tw, mode & (M_KIN | M_INV));
    } else if constexpr (PRE) {
        TwBase<N, RAD> wb;
        tw_base_load(wb, tw, t);
        col_body<R, N, RAD, C, NS, true>(v, kcr, kci, kin.sgn, kin.kL, lds + c, t, tw, mode, &wb);
    } else {
        col_body<R, N, RAD, C, NS>(v, kcr, kci, kin.sgn, kin.kL, lds + c, t, tw, mode);
    }
    // the offset is recomputed rather than held through the transforms
    __asm__ __volatile__("" : "+v"(tb));
    col_store<R, N, RAD, NS>(v, S, ubase, stride, tb);
}

template <typename R, int N, int RAD, int C, int WPE, int NS, bool CHI = false, bool VGRAD = false, bool PRE = false>
__global__ void __launch_bounds__((C * LineShape<N, RAD>::T)) __attribute__((amdgpu_waves_per_eu(WPE)))
k_colpass(StatePtrs<R> S, int64_t stride, int64_t slab_stride, const TwEntry<R> *__restrict__ tw, KinArgs kin,
          int mode, GroupArgs<R> grp)
{
    __shared__ cx<R> lds[ColMap<C>::slots(N)];
    __shared__ double red[16][3];
    if (grp.probs) {
        const BatchProb<R> &P = grp.probs[grp.ids[blockIdx.z]];
        S.p[0] = P.psi;
        S.p[1] = NS == 2 ? P.gadj : nullptr;
        kin.kA = P.kin_x;
        kin.kB = P.one;
        kin.kL = P.kin_y;
        kin.nA = P.nx;
    }
    const unsigned G = gridDim.x * gridDim.y;
    unsigned L = blockIdx.x + gridDim.x * blockIdx.y;
    if ((G & 7u) == 0) L = (L & 7u) * (G >> 3) + (L >> 3);
    col_tile<R, N, RAD, C, NS, CHI, VGRAD, PRE>(S, L % gridDim.x, L / gridDim.x, stride, slab_stride, tw, kin, mode,
                                                lds, red, threadIdx.x);
}

// ------------------------------------------------- pipelined column pass --
// The k-space pass of a step (forward transform, kinetic factor, inverse
// transform; one state) with each work-group walking column groups
// w, w + G, w + 2G, ... (G = the grid size): the next group's loads are
// issued while the current group transforms, so that on each CU a group's
// memory traffic overlaps the previous group's arithmetic instead of all
// work-groups loading, transforming and storing in lockstep.  Vector-memory
// loads complete in order, so the transforms read no table while the
// prefetch is in flight (a wait for a table load would also wait for every
// load issued before it): the stage factors are formed in FP64 from each
// stage's W^k, read once per work-group (see tw_dft), and the kinetic
// factors of the group are requested before the prefetch.
// ORDER 0: kinetic factors and the prefetch at the start of the group (the
// prefetch overlaps both transforms); ORDER 1: both after the forward
// transform (fewer registers held through it); ORDER 2: the kinetic factors
// issued in parts between the stages of the forward transform and the
// prefetch in parts between those of the inverse transform (a wave that
// issues all its loads at once waits for the address unit to take them, and
// then does no arithmetic).
template <typename R, int N, int RAD, int C, int WPE, int ORDER>
__global__ void __launch_bounds__((C * LineShape<N, RAD>::T)) __attribute__((amdgpu_waves_per_eu(WPE)))
k_colpipe(StatePtrs<R> S, int64_t stride, int64_t ngroups, const TwEntry<R> *__restrict__ tw, KinArgs kin,
          GroupArgs<R> grp)
{
    using Sh = LineShape<N, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV;
    __shared__ cx<R> lds[ColMap<C>::slots(N)];
    if (grp.probs) {
        const BatchProb<R> &P = grp.probs[grp.ids[blockIdx.z]];
        S.p[0] = P.psi;
        kin.kA = P.kin_x;
        kin.kB = P.one;
        kin.kL = P.kin_y;
        kin.nA = P.nx;
    }
    const int64_t nwg = gridDim.x;
    int64_t w = blockIdx.x;
    if ((nwg & 7) == 0) w = (w & 7) * (nwg >> 3) + (w >> 3);  // consecutive groups on one XCD (see k_colpass)
    if (w >= ngroups) return;
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    cx<R> *sh = lds + c;
    uint32_t tb = ((uint32_t)t * (uint32_t)stride + (uint32_t)c) * (uint32_t)sizeof(cx<R>);
    TwBase<N, RAD> wb;
    tw_base_load(wb, tw, t);
    uint32_t tk = (uint32_t)t * (uint32_t)sizeof(double2);
    const double sg = (double)kin.sgn;
    cx<R> a[1][RV], b[1][RV];
    col_load<R, N, RAD, 1>(a, S, w * C, stride, tb);
    int64_t j = w;
    // one group; NEXT: the next group's loads are issued into b.  The last
    // group is a separate instance so that no path through a group lacks the
    // prefetch: where two paths meet, the compiler's wait for the kinetic
    // table would count only the loads common to both and so wait for the
    // whole prefetch.
    auto group = [&](auto next) {
        constexpr bool NEXT = decltype(next)::value;
        const int64_t jn = j + nwg;
        const int64_t col = j * C + c;
        const cx<double> ka = gload((const cx<double> *)kin.kA + col % kin.nA),
                         kb = gload((const cx<double> *)kin.kB + col / kin.nA);
        cx<double> kl[RV];
        // kinetic factors of elements [M0, M1) of the thread's line
        auto load_kl = [&](auto m0, auto m1) {
            constexpr int M0 = decltype(m0)::value, M1 = decltype(m1)::value;
            __asm__ __volatile__("" : "+v"(tk));
#pragma unroll
            for (int m = M0; m < M1; ++m)
                kl[m] = gload((const cx<double> *)((const char *)kin.kL + m * T * (int)sizeof(double2) + tk));
        };
        using Z = std::integral_constant<int, 0>;
        using F = std::integral_constant<int, RV>;
        auto prefetch = [&] {
            if constexpr (NEXT) col_load<R, N, RAD, 1>(b, S, jn * C, stride, tb);
        };
        if constexpr (ORDER == 0) {
            load_kl(Z{}, F{});
            __builtin_amdgcn_sched_barrier(0);
            prefetch();
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (ORDER == 2) {
            // part k of NST - 1 parts of the factors after stage k of the forward transform
            // (none after the last stage: the factors are used right after it)
            constexpr int NST = LineShape<N, RAD>::NST, NP = NST > 1 ? NST - 1 : 1, P = (RV + NP - 1) / NP;
            auto part = [&](auto st) {
                constexpr int K = decltype(st)::value;
                constexpr int M0 = K * P < RV ? K * P : RV, M1 = (K + 1) * P < RV ? (K + 1) * P : RV;
                if constexpr (M0 < M1) {
                    __builtin_amdgcn_sched_barrier(0);
                    load_kl(std::integral_constant<int, M0>{}, std::integral_constant<int, M1>{});
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            fft_line_pre<R, N, RAD, -1, ColMap<C>>(a[0], sh, t, tw, wb, part);
        } else {
            fft_line_pre<R, N, RAD, -1, ColMap<C>>(a[0], sh, t, tw, wb);
        }
        if constexpr (ORDER == 1) {
            __builtin_amdgcn_sched_barrier(0);
            load_kl(Z{}, F{});
            __builtin_amdgcn_sched_barrier(0);
            prefetch();
            __builtin_amdgcn_sched_barrier(0);
        }
        const double kcr = ka.re * kb.re - ka.im * kb.im, kci = ka.re * kb.im + ka.im * kb.re;
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const double kr = kcr * kl[m].re - kci * kl[m].im, ki = kcr * kl[m].im + kci * kl[m].re;
            a[0][m] = mul_phase(a[0][m], kr, sg * ki);
        }
        if constexpr (ORDER == 2 && NEXT) {
            // part k of NST parts of the prefetch: before the transform (k = 0) and after each
            // stage but the last
            constexpr int NST = LineShape<N, RAD>::NST, P = (RV + NST - 1) / NST;
            auto part = [&](auto st) {
                constexpr int K = decltype(st)::value + 1;
                constexpr int M0 = K * P < RV ? K * P : RV, M1 = (K + 1) * P < RV ? (K + 1) * P : RV;
                if constexpr (M0 < M1) {
                    __builtin_amdgcn_sched_barrier(0);
                    col_load_part<R, N, RAD, M0, M1>(b, S, jn * C, stride, tb);
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            part(std::integral_constant<int, -1>{});
            fft_line_pre<R, N, RAD, +1, ColMap<C>>(a[0], sh, t, tw, wb, part);
        } else {
            fft_line_pre<R, N, RAD, +1, ColMap<C>>(a[0], sh, t, tw, wb);
        }
        __asm__ __volatile__("" : "+v"(tb));
        col_store<R, N, RAD, 1>(a, S, j * C, stride, tb);
        if constexpr (NEXT) {
#pragma unroll
            for (int m = 0; m < RV; ++m) a[0][m] = b[0][m];
            j = jn;
        }
    };
    for (; j + nwg < ngroups;) group(std::true_type{});
    group(std::false_type{});
}

// ---------------------------------------------------------------- 1-D run --
// One work-group per problem keeps its line in registers (cyclic layout) for
// all steps; V0 of the thread's points is held in registers as well.  Steps
// are visited forward (dir = +1) or backward with conjugated factors
// (dir = -1, the exact inverse).  Consecutive half steps are merged:
//   P_first, then per step: F, K, F^-1, P_s P_next (or P_s at the end).
// MODE 1 (autocorrelation): at the top of step s the registers hold P psi_s
// (P the first half factor, the same every step without a field), so
// chi_s = dv sum conj(P psi_0)(P psi_s); each thread keeps its own points of
// P psi_0 in a.ref (written at s = 0, read back by the same thread) and the
// FP64 sum over the work-group is written by thread 0.  MODE 2 (windowed
// eigenfunction): each thread accumulates tau w_s exp(i E s tau/hbar) P psi_s
// of its points in FP64 (a.eig_acc, same-thread access), and after the run
// writes P^-1 of the sum, exp(+i aV_half V0) acc, to a.eig_out.
template <typename R, typename VT, int N, int RAD, int MODE = 0>
__device__ __forceinline__ void run1d_tile(cx<R> *__restrict__ p, const VT *__restrict__ vp,
                                           const TwEntry<R> *__restrict__ tw, const Run1DArgs &a, cx<R> *sh, int tid,
                                           double (*red)[3] = nullptr)
{
    using Sh = LineShape<N, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV;
    // threads beyond T (a work-group sized for a longer line) only keep step with the barriers
    const bool act = tid < T;
    const int t = act ? tid : 0;
    cx<R> v[RV];
    if (act)
#pragma unroll
        for (int m = 0; m < RV; ++m) v[m] = p[t + m * T];
    const double sg = (double)a.dir;
    auto step_of = [&](int64_t s) { return a.dir > 0 ? a.step0 + s : a.step0 + a.nsteps - 1 - s; };
    auto field = [&](int64_t st) { return a.ebar ? a.ebar[st] : 0.0; };
    // V0, x and the kinetic table are re-read each step (L1/L2 hits) rather
    // than held in registers, which keeps the line itself spill-free.
    auto potential = [&](double av, double e) {
        if (!act) return;
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const int x = t + m * T;
            v[m] = mul_expmi(v[m], sg * (av * ldv(vp + x) + e * (a.xmin + (double)x * a.dx)));
            if ((m & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bound the interleaving
        }
    };
    if (a.nsteps > 0) potential(a.aV_half, field(step_of(0)) * a.inv_2hbar);
#pragma unroll 1
    for (int64_t s = 0; s < a.nsteps; ++s) {
        // keep the table loads inside the loop: hoisting every twiddle, kinetic
        // factor and potential value of all steps out of it exhausts registers
        __asm__ __volatile__("" ::: "memory");
        if constexpr (MODE == 1) {
            cx<R> *ref = (cx<R> *)a.ref;
            double acc[3] = {0.0, 0.0, 0.0};
            if (act)
#pragma unroll
                for (int m = 0; m < RV; ++m) {
                    cx<R> r;
                    if (s == 0) {
                        ref[t + m * T] = v[m];
                        r = v[m];
                    } else {
                        r = ref[t + m * T];
                    }
                    acc[0] += (double)r.re * (double)v[m].re + (double)r.im * (double)v[m].im;
                    acc[1] += (double)r.re * (double)v[m].im - (double)r.im * (double)v[m].re;
                }
            block_sum3(acc, red);
            if (tid == 0) {
                a.chi[2 * s] = acc[0] * a.dv;
                a.chi[2 * s + 1] = acc[1] * a.dv;
            }
        }
        if constexpr (MODE == 2) {
            const double w = a.tau * (1.0 - cospi(2.0 * (double)s / (double)a.nsteps));
            double sn, cs;
            sincos_fp64(a.eig_E * (double)s * a.tau / a.hbar, sn, cs);
            const double cr = w * cs, ci = w * sn;
            if (act)
#pragma unroll
                for (int m = 0; m < RV; ++m) {
                    double2 *q = a.eig_acc + t + m * T;
                    const double2 o = s == 0 ? double2{0.0, 0.0} : *q;
                    const double vr = (double)v[m].re, vi = (double)v[m].im;
                    *q = double2{o.x + cr * vr - ci * vi, o.y + cr * vi + ci * vr};
                }
        }
        fft_line<R, N, RAD, -1, RowMap<R, RAD>>(v, sh, t, tw, act);
        if (act) {
            const double2 *kin = a.kin + step_of(s) * a.kin_stride;
#pragma unroll
            for (int m = 0; m < RV; ++m) {
                const double2 k = kin[t + m * T];
                v[m] = mul_phase(v[m], k.x, sg * k.y);
            }
        }
        fft_line<R, N, RAD, +1, RowMap<R, RAD>>(v, sh, t, tw, act);
        const bool more = s + 1 < a.nsteps;
        potential(a.aV_half * (more ? 2.0 : 1.0),
                  (field(step_of(s)) + (more ? field(step_of(s + 1)) : 0.0)) * a.inv_2hbar);
    }
    if (act)
#pragma unroll
        for (int m = 0; m < RV; ++m) p[t + m * T] = v[m];
    if constexpr (MODE == 2) {
        cx<R> *out = (cx<R> *)a.eig_out;
        if (act)
#pragma unroll
            for (int m = 0; m < RV; ++m) {
                const int x = t + m * T;
                const double2 o = a.nsteps > 0 ? a.eig_acc[x] : double2{0.0, 0.0};
                double sn, cs;
                sincos_fp64(a.aV_half * ldv(vp + x), sn, cs);
                out[x] = cx<R>{(R)(o.x * cs - o.y * sn), (R)(o.x * sn + o.y * cs)};
            }
    }
}

// Reverse sweep of a 1-D run: the state psi and its adjoint g are walked back
// together with the exact inverse step (conjugated factors, last step first),
// as run1d_tile does with dir = -1.  At every step boundary n (psi_n, g_n in
// real space) it forms b_n = Im(conj(g_n) psi_n): the dL/dV0 accumulator
// (registers) gains w_n b_n and mom[n] receives sum_x x b_n.
template <typename R, typename VT, int N, int RAD>
__device__ __forceinline__ void adj1d_tile(cx<R> *__restrict__ psi, cx<R> *__restrict__ gv,
                                           const VT *__restrict__ V0, const TwEntry<R> *__restrict__ tw,
                                           const Run1DArgs &a, double wbase, double *acc_out, double *mom, cx<R> *sh,
                                           double (*red)[3], int tid)
{
    using Sh = LineShape<N, RAD>;
    using Map = RowMap<R, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV;
    const bool act = tid < T;
    const int t = act ? tid : 0;
    cx<R> v[2][RV];
    double acc[RV];
#pragma unroll
    for (int m = 0; m < RV; ++m) {
        v[0][m] = act ? psi[t + m * T] : cx<R>{};
        v[1][m] = act ? gv[t + m * T] : cx<R>{};
        acc[m] = 0.0;
    }
    auto step_of = [&](int64_t s) { return a.step0 + a.nsteps - 1 - s; };
    auto field = [&](int64_t st) { return a.ebar ? a.ebar[st] : 0.0; };
    auto grad = [&](int64_t bidx, double w) {
        double mo[3] = {0.0, 0.0, 0.0};
        if (act)
#pragma unroll
            for (int m = 0; m < RV; ++m) {
                const double b = (double)v[1][m].re * (double)v[0][m].im - (double)v[1][m].im * (double)v[0][m].re;
                acc[m] += w * b;
                mo[0] += (a.xmin + (double)(t + m * T) * a.dx) * b;
            }
        block_sum3(mo, red);
        if (tid == 0)
            for (int q = 0; q < 3; ++q) mom[3 * bidx + q] = mo[q];
    };
    auto potential = [&](double av, double e) {
        if (!act) return;
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const int x = t + m * T;
            const double th = -(av * (double)V0[x] + e * (a.xmin + (double)x * a.dx));
            double sn, cs;
            sincos_fp64(th, sn, cs);
            v[0][m] = mul_phase(v[0][m], cs, -sn);
            v[1][m] = mul_phase(v[1][m], cs, -sn);
        }
    };
    grad(a.nsteps, wbase);
    if (a.nsteps > 0) potential(a.aV_half, field(step_of(0)) * a.inv_2hbar);
#pragma unroll 1
    for (int64_t s = 0; s < a.nsteps; ++s) {
        __asm__ __volatile__("" ::: "memory");
        for (int q = 0; q < 2; ++q) fft_line<R, N, RAD, -1, Map>(v[q], sh, t, tw, act);
        if (a.vmom) {
            // velocity gauge: sum_k (k, 1) Im(conj(g~) psi~) of this step in k-space
            double mo[3] = {0.0, 0.0, 0.0};
            if (act)
#pragma unroll
                for (int m = 0; m < RV; ++m) {
                    const double b = (double)v[1][m].re * (double)v[0][m].im - (double)v[1][m].im * (double)v[0][m].re;
                    mo[0] += a.kv[t + m * T] * b;
                    mo[1] += b;
                }
            block_sum3(mo, red);
            if (tid == 0) {
                double *o = a.vmom + 4 * (step_of(s) - a.step0);
                o[0] = 0.0;
                o[1] = 0.0;
                o[2] = mo[0];
                o[3] = mo[1];
            }
        }
        const double2 *kin = a.kin + step_of(s) * a.kin_stride;
        for (int q = 0; q < 2; ++q) {
            if (act)
#pragma unroll
                for (int m = 0; m < RV; ++m) {
                    const double2 k = kin[t + m * T];
                    v[q][m] = mul_phase(v[q][m], k.x, -k.y);
                }
            fft_line<R, N, RAD, +1, Map>(v[q], sh, t, tw, act);
        }
        const bool more = s + 1 < a.nsteps;
        potential(a.aV_half * (more ? 2.0 : 1.0),
                  (field(step_of(s)) + (more ? field(step_of(s + 1)) : 0.0)) * a.inv_2hbar);
        grad(a.nsteps - 1 - s, (more ? 2.0 : 1.0) * wbase);
    }
    if (act)
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            psi[t + m * T] = v[0][m];
            gv[t + m * T] = v[1][m];
            if (acc_out) acc_out[t + m * T] = acc[m];
        }
}

// ------------------------------------------------------ variant dispatch --
// A kernel launch; ev != null: an event pair that the dispatch itself
// timestamps at its start and end (no packet between launches).
template <typename K, typename... A>
void launch_kernel(K kernel, dim3 grid, dim3 block, hipStream_t st, const hipEvent_t *ev, A... args)
{
    if (ev)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, ev[0], ev[1], 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
}

template <typename R, int N, int V> constexpr bool row_variant_ok()
{
    constexpr RowVariant rv = kRowVariants[V];
    using Tl = RowTile<N, rv.rad, rv.threads>;
    if (N < 256 && V != 0) return false;  // short rows: default shape only
    // 1 KiB stays free for the reduction buffer and static LDS of the kernel
    return Tl::NT <= 1024 && Tl::ROWS * RowMap<R, rv.rad, rv.pad>::slots(N) * (int)sizeof(cx<R>) <= 159 * 1024;
}

template <typename R, int N, int V, int NS>
hipError_t row_launch(const StatePtrs<R> &S, int64_t nrows, int ny, const void *V0, const void *const *tws,
                      const PhaseArgs &ph, const GradArgs &ga, int mode, hipStream_t st, const GroupArgs<R> &grp,
                      int ngroup, const hipEvent_t *ev)
{
    if constexpr (!row_variant_ok<R, N, V>()) {
        return hipErrorInvalidValue;
    } else {
        constexpr RowVariant rv = kRowVariants[V];
        const void *tw = tws[rv.rad == 8 ? 0 : 1];
        using Tl = RowTile<N, rv.rad, rv.threads>;
        if (nrows % Tl::ROWS) {
            // fewer rows than a work-group holds (a single 1-D line): one row per group
            launch_kernel(k_xpass<R, N, rv.rad, LineShape<N, rv.rad>::T, 1, NS, rv.pad>,
                          dim3((unsigned)nrows, (unsigned)ngroup), dim3(LineShape<N, rv.rad>::T), st, ev, S, ny,
                          (const VStore<R> *)V0, (const TwEntry<R> *)tw, ph, ga, mode, grp);
        } else {
            launch_kernel(k_xpass<R, N, rv.rad, rv.threads, rv.wpe, NS, rv.pad, rv.late, rv.pre && sizeof(R) == 8>,
                          dim3((unsigned)(nrows / Tl::ROWS), (unsigned)ngroup), dim3(Tl::NT), st, ev, S, ny,
                          (const VStore<R> *)V0, (const TwEntry<R> *)tw, ph, ga, mode, grp);
        }
        return hipGetLastError();
    }
}

template <typename R, int N, int NS, size_t... I>
hipError_t row_dispatch(int var, const StatePtrs<R> &S, int64_t nrows, int ny, const void *V0,
                        const void *const *tw, const PhaseArgs &ph, const GradArgs &ga, int mode, hipStream_t st,
                        const GroupArgs<R> &grp, int ngroup, const hipEvent_t *ev, std::index_sequence<I...>)
{
    hipError_t r = hipErrorInvalidValue;
    ((var == (int)I ? (r = row_launch<R, N, (int)I, NS>(S, nrows, ny, V0, tw, ph, ga, mode, st, grp, ngroup, ev), 0)
                    : 0),
     ...);
    return r;
}

template <typename R, int N, int V> constexpr bool col_variant_ok()
{
    constexpr ColVariant cv = kColVariants[V];
    if (N < 256 && V != 0) return false;
    return cv.cols * LineShape<N, cv.rad>::T <= 1024 && ColMap<cv.cols>::slots(N) * (int)sizeof(cx<R>) <= 159 * 1024;
}


template <typename R, int N, int V, int NS>
hipError_t col_launch(const StatePtrs<R> &S, int64_t ncols, int64_t stride, int nslab, int64_t slab_stride,
                      const void *const *tws, const KinArgs &kin, int mode, hipStream_t st, const GroupArgs<R> &grp,
                      int ngroup, const hipEvent_t *ev)
{
    if constexpr (!col_variant_ok<R, N, V>()) {
        return hipErrorInvalidValue;
    } else {
        constexpr ColVariant cv = kColVariants[V];
        const void *tw = tws[cv.rad == 8 ? 0 : 1];
        const bool chi = NS == 1 && (mode & M_CHI);
        if (ncols % cv.cols) return hipErrorInvalidValue;
        // per-thread byte offsets within a work-group's lines are 32-bit
        if (((int64_t)(LineShape<N, cv.rad>::T - 1) * stride + cv.cols) * (int64_t)sizeof(cx<R>) > (int64_t)UINT32_MAX)
            return hipErrorInvalidValue;
        const dim3 grid((unsigned)(ncols / cv.cols), (unsigned)nslab, (unsigned)ngroup);
        const dim3 block(cv.cols * LineShape<N, cv.rad>::T);
        if constexpr (NS == 1) {
            if (chi) {
                launch_kernel(k_colpass<R, N, cv.rad, cv.cols, cv.wpe, 1, true>, grid, block, st, ev, S, stride,
                              slab_stride, (const TwEntry<R> *)tw, kin, mode, grp);
                return hipGetLastError();
            }
        }
        if constexpr (cv.pipe > 0 && NS == 1) {
            // the k-space pass of a forward step; other modes run the plain shape
            if (mode == (M_FWD | M_KIN | M_INV) && nslab == 1 && !chi) {
                const int64_t ngroups = ncols / cv.cols;
                const dim3 pgrid((unsigned)((ngroups + cv.pipe - 1) / cv.pipe), 1, (unsigned)ngroup);
                launch_kernel(k_colpipe<R, N, cv.rad, cv.cols, cv.wpe, cv.order>, pgrid, block, st, ev, S, stride,
                              ngroups, (const TwEntry<R> *)tw, kin, grp);
                return hipGetLastError();
            }
        }
        if constexpr (NS == 2) {
            if (mode & M_VGRAD) {
                launch_kernel(k_colpass<R, N, cv.rad, cv.cols, cv.wpe, 2, false, true>, grid, block, st, ev, S, stride,
                              slab_stride, (const TwEntry<R> *)tw, kin, mode, grp);
                return hipGetLastError();
            }
        }
        if constexpr (cv.pre) {
            launch_kernel(k_colpass<R, N, cv.rad, cv.cols, cv.wpe, NS, false, false, true>, grid, block, st, ev, S,
                          stride, slab_stride, (const TwEntry<R> *)tw, kin, mode, grp);
        } else {
            launch_kernel(k_colpass<R, N, cv.rad, cv.cols, cv.wpe, NS>, grid, block, st, ev, S, stride, slab_stride,
                          (const TwEntry<R> *)tw, kin, mode, grp);
        }
        return hipGetLastError();
    }
}

template <typename R, int N, int NS, size_t... I>
hipError_t col_dispatch(int var, const StatePtrs<R> &S, int64_t ncols, int64_t stride, int nslab,
                        int64_t slab_stride, const void *const *tw, const KinArgs &kin, int mode, hipStream_t st,
                        const GroupArgs<R> &grp, int ngroup, const hipEvent_t *ev, std::index_sequence<I...>)
{
    hipError_t r = hipErrorInvalidValue;
    ((var == (int)I
          ? (r = col_launch<R, N, (int)I, NS>(S, ncols, stride, nslab, slab_stride, tw, kin, mode, st, grp, ngroup, ev),
             0)
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
