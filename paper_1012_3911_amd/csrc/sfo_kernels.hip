// Schroedinger split-step kernels: row (x) passes, strided column passes,
// the 1-D whole-run kernel and the FP64 reductions.
//
// A 2-D step costs two passes over HBM: a row pass (inverse x-transform,
// merged potential factor of two consecutive half steps, forward
// x-transform) and a column pass (forward y-transform, kinetic factor,
// inverse y-transform).  A 3-D step adds a forward and an inverse y-pass
// around the z-pass that carries the kinetic factor.  A 1-D line of up to
// 8192 points stays in one work-group's registers and LDS for the whole run.
#include <algorithm>
#include <type_traits>

#include "pass_kernels.h"

namespace sfo {

template <typename VT> __device__ __forceinline__ double ldv(const VT *p) { return (double)*p; }

// ---------------------------------------------------------------- 1-D run --
// One work-group per problem keeps its line in registers (cyclic layout) for
// all steps; V0 of the thread's points is held in registers as well.  Steps
// are visited forward (dir = +1) or backward with conjugated factors
// (dir = -1, the exact inverse).  Consecutive half steps are merged:
//   P_first, then per step: F, K, F^-1, P_s P_next (or P_s at the end).
template <typename R, typename VT, int N, int RAD>
__global__ void __launch_bounds__((LineShape<N, RAD>::T))
    k_1d_run(cx<R> *__restrict__ psi, int64_t prob_stride, const VT *__restrict__ V0,
             const TwEntry<R> *__restrict__ tw, Run1DArgs a)
{
    using Sh = LineShape<N, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV;
    __shared__ cx<R> sh[RowMap<R, RAD>::slots(N)];
    const int t = threadIdx.x;
    cx<R> *p = psi + (int64_t)blockIdx.x * prob_stride;
    const VT *vp = V0 + (int64_t)blockIdx.x * prob_stride;
    cx<R> v[RV];
#pragma unroll
    for (int m = 0; m < RV; ++m) v[m] = p[t + m * T];
    const double sg = (double)a.dir;
    auto step_of = [&](int64_t s) { return a.dir > 0 ? a.step0 + s : a.step0 + a.nsteps - 1 - s; };
    auto field = [&](int64_t st) { return a.ebar ? a.ebar[st] : 0.0; };
    // V0, x and the kinetic table are re-read each step (L1/L2 hits) rather
    // than held in registers, which keeps the line itself spill-free.
    auto potential = [&](double av, double e) {
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
        fft_line<R, N, RAD, -1, RowMap<R, RAD>>(v, sh, t, tw);
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const double2 k = a.kin[t + m * T];
            v[m] = mul_phase(v[m], k.x, sg * k.y);
        }
        fft_line<R, N, RAD, +1, RowMap<R, RAD>>(v, sh, t, tw);
        const bool more = s + 1 < a.nsteps;
        potential(a.aV_half * (more ? 2.0 : 1.0),
                  (field(step_of(s)) + (more ? field(step_of(s + 1)) : 0.0)) * a.inv_2hbar);
    }
#pragma unroll
    for (int m = 0; m < RV; ++m) p[t + m * T] = v[m];
}

// ------------------------------------------------------------ 1-D adjoint --
// Reverse sweep of a 1-D run: the state psi and its adjoint g are walked back
// together with the exact inverse step (conjugated factors, last step first),
// as the forward whole-run kernel does with dir = -1.  At every step boundary
// n (psi_n, g_n in real space) it forms b_n = Im(conj(g_n) psi_n): the dL/dV0
// accumulator (registers) gains w_n b_n and mom[n] receives sum_x x b_n.
template <typename R, typename VT, int N, int RAD>
__global__ void __launch_bounds__((LineShape<N, RAD>::T))
    k_1d_adjoint(cx<R> *__restrict__ psi, cx<R> *__restrict__ gv, const VT *__restrict__ V0,
                 const TwEntry<R> *__restrict__ tw, Run1DArgs a, double wbase, double *acc_out, double *mom)
{
    using Sh = LineShape<N, RAD>;
    using Map = RowMap<R, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV;
    __shared__ cx<R> sh[Map::slots(N)];
    __shared__ double red[16][3];
    const int t = threadIdx.x;
    cx<R> v[2][RV];
    double acc[RV];
#pragma unroll
    for (int m = 0; m < RV; ++m) {
        v[0][m] = psi[t + m * T];
        v[1][m] = gv[t + m * T];
        acc[m] = 0.0;
    }
    auto step_of = [&](int64_t s) { return a.step0 + a.nsteps - 1 - s; };
    auto field = [&](int64_t st) { return a.ebar ? a.ebar[st] : 0.0; };
    auto grad = [&](int64_t bidx, double w) {
        double mo[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const double b = (double)v[1][m].re * (double)v[0][m].im - (double)v[1][m].im * (double)v[0][m].re;
            acc[m] += w * b;
            mo[0] += (a.xmin + (double)(t + m * T) * a.dx) * b;
        }
        block_sum3(mo, red);
        if (t == 0)
            for (int q = 0; q < 3; ++q) mom[3 * bidx + q] = mo[q];
    };
    auto potential = [&](double av, double e) {
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
        for (int q = 0; q < 2; ++q) {
            fft_line<R, N, RAD, -1, Map>(v[q], sh, t, tw);
#pragma unroll
            for (int m = 0; m < RV; ++m) {
                const double2 k = a.kin[t + m * T];
                v[q][m] = mul_phase(v[q][m], k.x, -k.y);
            }
            fft_line<R, N, RAD, +1, Map>(v[q], sh, t, tw);
        }
        const bool more = s + 1 < a.nsteps;
        potential(a.aV_half * (more ? 2.0 : 1.0),
                  (field(step_of(s)) + (more ? field(step_of(s + 1)) : 0.0)) * a.inv_2hbar);
        grad(a.nsteps - 1 - s, (more ? 2.0 : 1.0) * wbase);
    }
#pragma unroll
    for (int m = 0; m < RV; ++m) {
        psi[t + m * T] = v[0][m];
        gv[t + m * T] = v[1][m];
        if (acc_out) acc_out[t + m * T] = acc[m];
    }
}

__global__ void k_ebar_grad(const double *mom, int64_t nsteps, int ndim, double scale, double *out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nsteps * ndim; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / ndim;
        const int a = (int)(i % ndim);
        out[i] = (mom[3 * (s + 1) + a] + mom[3 * s + a]) * scale;
    }
}

// ------------------------------------------------------------- reductions --
template <typename R>
__global__ void __launch_bounds__(256) k_norm_partial(const cx<R> *__restrict__ a, int64_t n, double *part)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double re = a[i].re, im = a[i].im;
        acc += re * re + im * im;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

template <typename R>
__global__ void __launch_bounds__(256) k_overlap_partial(const cx<R> *__restrict__ a, const cx<R> *__restrict__ b,
                                                         int64_t n, double *part)
{
    __shared__ double sr[256], si[256];
    double ar = 0.0, ai = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double xr = a[i].re, xi = a[i].im, yr = b[i].re, yi = b[i].im;
        ar += xr * yr + xi * yi;
        ai += xr * yi - xi * yr;
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sr[threadIdx.x] += sr[threadIdx.x + w];
            si[threadIdx.x] += si[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sr[0];
        part[2 * blockIdx.x + 1] = si[0];
    }
}

// Sum `count` interleaved groups of `width` partials in a fixed order.
__global__ void __launch_bounds__(256) k_sum_partials(const double *part, int count, int width, double *out)
{
    __shared__ double s[2][256];
    for (int w = 0; w < width; ++w) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < count; i += 256) acc += part[i * width + w];
        s[w][threadIdx.x] = acc;
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int w = 0; w < width; ++w) s[w][threadIdx.x] += s[w][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int w = 0; w < width; ++w) out[w] = s[w][0];
}

__global__ void __launch_bounds__(256) k_absmax_partial(const double *__restrict__ a, int64_t n, double *part)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        acc = fmax(acc, fabs(a[i]));
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(256) k_max_partials(const double *part, int count, double *out)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += 256) acc = fmax(acc, part[i]);
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

__global__ void k_convert_v0(const double *__restrict__ src, void *dst, int to_fp64, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (to_fp64)
            ((double *)dst)[i] = src[i];
        else
            ((float *)dst)[i] = (float)src[i];
    }
}

// ------------------------------------------------------------ host helpers --
void line_stages(int N, int RAD, int *radix, int *span, int *nst)
{
    const int RV = N < RAD ? N : RAD;
    const int LOGR = ilog2(RV);
    const int NFULL = LOGR ? ilog2(N) / LOGR : 0;
    const int REM = N >> (NFULL * LOGR);
    int n = 0, L = 1;
    if (REM > 1) { radix[n] = REM; span[n] = L; L *= REM; ++n; }
    for (int i = 0; i < NFULL; ++i) { radix[n] = RV; span[n] = L; L *= RV; ++n; }
    *nst = n;
}
static_assert(LineShape<2048, 16>::TW_SIZE == 15 * 8 + 15 * 128, "stage table layout");
static_assert(LineShape<2048, 8>::TW_SIZE == 7 * 4 + 7 * 32 + 7 * 256, "stage table layout");

// -------------------------------------------------------------- launchers --
constexpr int kRad = 16;

#define SFO_SWITCH_1D_N(N_, CALL)                     \
    switch (N_) {                                     \
    case 64: return CALL(64);                         \
    case 128: return CALL(128);                       \
    case 256: return CALL(256);                       \
    case 512: return CALL(512);                       \
    case 1024: return CALL(1024);                     \
    case 2048: return CALL(2048);                     \
    case 4096: return CALL(4096);                     \
    case 8192: return CALL(8192);                     \
    default: return hipErrorInvalidValue;             \
    }

template <typename R, typename VT, int N>
static hipError_t run1d_n(cx<R> *psi, int nprob, int64_t prob_stride, const void *V0, const void *tw,
                          const Run1DArgs &a, hipStream_t st)
{
    constexpr int threads = LineShape<N, kRad>::T;
    hipLaunchKernelGGL((k_1d_run<R, VT, N, kRad>), dim3((unsigned)nprob), dim3(threads), 0, st, psi, prob_stride,
                       (const VT *)V0, (const TwEntry<R> *)tw, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_1d(int N, cx<R> *psi, int nprob, int64_t prob_stride, const void *V0, const void *tw,
                     const Run1DArgs &a, hipStream_t st)
{
    using VT = typename std::conditional<sizeof(R) == 4, float, double>::type;
#define CALL(n) run1d_n<R, VT, n>(psi, nprob, prob_stride, V0, tw, a, st)
    SFO_SWITCH_1D_N(N, CALL)
#undef CALL
}

template <typename R, typename VT, int N>
static hipError_t adj1d_n(cx<R> *psi, cx<R> *gv, const void *V0, const void *tw, const Run1DArgs &a, double wbase,
                          double *acc, double *mom, hipStream_t st)
{
    constexpr int threads = LineShape<N, kRad>::T;
    hipLaunchKernelGGL((k_1d_adjoint<R, VT, N, kRad>), dim3(1), dim3(threads), 0, st, psi, gv, (const VT *)V0,
                       (const TwEntry<R> *)tw, a, wbase, acc, mom);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_1d_adjoint(int N, cx<R> *psi, cx<R> *gv, const void *V0, const void *tw, const Run1DArgs &a,
                             double wbase, double *acc, double *mom, hipStream_t st)
{
    using VT = typename std::conditional<sizeof(R) == 4, float, double>::type;
#define CALL(n) adj1d_n<R, VT, n>(psi, gv, V0, tw, a, wbase, acc, mom, st)
    SFO_SWITCH_1D_N(N, CALL)
#undef CALL
}

hipError_t launch_ebar_grad(const double *mom, int64_t nsteps, int ndim, double scale, double *out, hipStream_t st)
{
    if (nsteps <= 0) return hipSuccess;
    const int64_t n = nsteps * ndim;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_ebar_grad, dim3(blocks), dim3(256), 0, st, mom, nsteps, ndim, scale, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_norm(const cx<R> *a, int64_t n, double *partials, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_norm_partial<R>, dim3(kReduceBlocks), dim3(256), 0, st, a, n, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, (const double *)partials, kReduceBlocks, 1, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_overlap(const cx<R> *a, const cx<R> *b, int64_t n, double *partials, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_overlap_partial<R>, dim3(kReduceBlocks), dim3(256), 0, st, a, b, n, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, (const double *)partials, kReduceBlocks, 2, out);
    return hipGetLastError();
}

hipError_t launch_absmax(const double *src, int64_t n, double *partials, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_absmax_partial, dim3(kReduceBlocks), dim3(256), 0, st, src, n, partials);
    hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(256), 0, st, (const double *)partials, kReduceBlocks, out);
    return hipGetLastError();
}

hipError_t launch_convert_v0(const double *src, void *dst, bool to_fp64, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_convert_v0, dim3(1024), dim3(256), 0, st, src, dst, to_fp64 ? 1 : 0, n);
    return hipGetLastError();
}

template hipError_t launch_1d<float>(int, cx<float> *, int, int64_t, const void *, const void *, const Run1DArgs &,
                                     hipStream_t);
template hipError_t launch_1d<double>(int, cx<double> *, int, int64_t, const void *, const void *, const Run1DArgs &,
                                      hipStream_t);
template hipError_t launch_1d_adjoint<float>(int, cx<float> *, cx<float> *, const void *, const void *,
                                             const Run1DArgs &, double, double *, double *, hipStream_t);
template hipError_t launch_1d_adjoint<double>(int, cx<double> *, cx<double> *, const void *, const void *,
                                              const Run1DArgs &, double, double *, double *, hipStream_t);
template hipError_t launch_norm<float>(const cx<float> *, int64_t, double *, double *, hipStream_t);
template hipError_t launch_norm<double>(const cx<double> *, int64_t, double *, double *, hipStream_t);
template hipError_t launch_overlap<float>(const cx<float> *, const cx<float> *, int64_t, double *, double *,
                                          hipStream_t);
template hipError_t launch_overlap<double>(const cx<double> *, const cx<double> *, int64_t, double *, double *,
                                           hipStream_t);

}  // namespace sfo
