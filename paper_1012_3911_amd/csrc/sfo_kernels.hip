// Schroedinger split-step kernels: row (x) passes, strided column passes,
// the 1-D whole-run kernel and the FP64 reductions.
//
// A 2-D step costs two passes over HBM: a row pass (inverse x-transform,
// merged potential factor of two consecutive half steps, forward
// x-transform) and a column pass (forward y-transform, kinetic factor,
// inverse y-transform).  A 3-D step adds a forward and an inverse y-pass
// around the z-pass that carries the kinetic factor.  A 1-D line of up to
// 8192 points stays in one work-group's registers and LDS for the whole run.
#include "sfo_impl.h"

namespace sfo {

template <typename VT> __device__ __forceinline__ double ldv(const VT *p) { return (double)*p; }

// --------------------------------------------------------------- row pass --
// One work-group holds ROWS rows of N points; thread t of a row owns the
// cyclic elements t + m T.  Global access is contiguous along the row.
template <typename R, typename VT, int N, int RAD, int ROWS>
__global__ void __launch_bounds__((ROWS * LineShape<N, RAD>::T))
    k_xpass(cx<R> *__restrict__ psi, int ny, const VT *__restrict__ V0,
            const TwEntry<R> *__restrict__ tw, PhaseArgs ph, int mode)
{
    using Sh = LineShape<N, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV;
    __shared__ cx<R> lds[ROWS * Sh::LDS];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int64_t row = (int64_t)blockIdx.x * ROWS + line;
    cx<R> *p = psi + row * N;
    cx<R> *sh = lds + line * Sh::LDS;
    cx<R> v[RV];
#pragma unroll
    for (int m = 0; m < RV; ++m) v[m] = p[t + m * T];
    if (mode & M_INV) fft_line<R, N, RAD, +1>(v, sh, t, tw);
    if (mode & M_PHASE) {
        const int64_t y = row % ny, z = row / ny;
        const double base = ph.e[1] * (ph.xmin[1] + (double)y * ph.dx[1]) +
                            ph.e[2] * (ph.xmin[2] + (double)z * ph.dx[2]);
        const VT *vr = V0 + row * N;
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const int x = t + m * T;
            double th = ph.aV * ldv(vr + x) + ph.e[0] * (ph.xmin[0] + (double)x * ph.dx[0]) + base;
            v[m] = mul_expmi(v[m], (double)ph.sgn * th);
            if ((m & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bound the interleaving
        }
    }
    if (mode & M_FWD) fft_line<R, N, RAD, -1>(v, sh, t, tw);
#pragma unroll
    for (int m = 0; m < RV; ++m) p[t + m * T] = v[m];
}

// ------------------------------------------------------------ column pass --
// Lines run along a strided axis (stride elements apart); one work-group
// holds C adjacent lines so that each global access moves C contiguous
// values.  Thread (t, c) owns elements t + m T of line c.
template <typename R, int N, int RAD, int C>
__global__ void __launch_bounds__((C * LineShape<N, RAD>::T))
    k_colpass(cx<R> *__restrict__ psi, int64_t stride, int64_t slab_stride,
              const TwEntry<R> *__restrict__ tw, KinArgs kin, int mode)
{
    using Sh = LineShape<N, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV;
    __shared__ cx<R> lds[C * Sh::LDS];
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int64_t col = (int64_t)blockIdx.x * C + c;
    cx<R> *p = psi + (int64_t)blockIdx.y * slab_stride + col;
    cx<R> *sh = lds + c * Sh::LDS;
    cx<R> v[RV];
#pragma unroll
    for (int m = 0; m < RV; ++m) v[m] = p[(int64_t)(t + m * T) * stride];
    if (mode & M_FWD) fft_line<R, N, RAD, -1>(v, sh, t, tw);
    if (mode & M_KIN) {
        const double2 a = kin.kA[col % kin.nA], b = kin.kB[col / kin.nA];
        const double kcr = a.x * b.x - a.y * b.y, kci = a.x * b.y + a.y * b.x;
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const double2 l = kin.kL[t + m * T];
            double kr = kcr * l.x - kci * l.y, ki = kcr * l.y + kci * l.x;
            v[m] = mul_phase(v[m], kr, (double)kin.sgn * ki);
        }
    }
    if (mode & M_INV) fft_line<R, N, RAD, +1>(v, sh, t, tw);
#pragma unroll
    for (int m = 0; m < RV; ++m) p[(int64_t)(t + m * T) * stride] = v[m];
}

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
    __shared__ cx<R> sh[Sh::LDS];
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
        fft_line<R, N, RAD, -1>(v, sh, t, tw);
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const double2 k = a.kin[t + m * T];
            v[m] = mul_phase(v[m], k.x, sg * k.y);
        }
        fft_line<R, N, RAD, +1>(v, sh, t, tw);
        const bool more = s + 1 < a.nsteps;
        potential(a.aV_half * (more ? 2.0 : 1.0),
                  (field(step_of(s)) + (more ? field(step_of(s + 1)) : 0.0)) * a.inv_2hbar);
    }
#pragma unroll
    for (int m = 0; m < RV; ++m) p[t + m * T] = v[m];
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

__global__ void k_convert_v0(const double *__restrict__ src, void *dst, int to_fp64, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (to_fp64)
            ((double *)dst)[i] = src[i];
        else
            ((float *)dst)[i] = (float)src[i];
    }
}

// -------------------------------------------------------------- launchers --
constexpr int kRad = 16;

template <int N> constexpr int rows_for() { return LineShape<N, kRad>::T >= 256 ? 1 : 256 / LineShape<N, kRad>::T; }

template <typename R, int N> constexpr int cols_for()
{
    constexpr int T = LineShape<N, kRad>::T;
    constexpr int per_line = LineShape<N, kRad>::LDS * (int)sizeof(cx<R>);
    int c = sizeof(R) == 4 ? 8 : 4;
    while (c > 1 && (c * T > 1024 || c * per_line > 160 * 1024)) c /= 2;
    return c;
}

template <typename R, typename VT, int N>
static hipError_t xpass_n(cx<R> *psi, int64_t nrows, int ny, const void *V0, const void *tw,
                          const PhaseArgs &ph, int mode, hipStream_t st)
{
    constexpr int ROWS = rows_for<N>();
    constexpr int threads = ROWS * LineShape<N, kRad>::T;
    if (nrows % ROWS) {
        // fewer rows than one work-group holds (a single 1-D line): one row per group
        hipLaunchKernelGGL((k_xpass<R, VT, N, kRad, 1>), dim3((unsigned)nrows), dim3(LineShape<N, kRad>::T), 0,
                           st, psi, ny, (const VT *)V0, (const TwEntry<R> *)tw, ph, mode);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_xpass<R, VT, N, kRad, ROWS>), dim3((unsigned)(nrows / ROWS)), dim3(threads), 0, st,
                       psi, ny, (const VT *)V0, (const TwEntry<R> *)tw, ph, mode);
    return hipGetLastError();
}

#define SFO_SWITCH_PASS_N(N_, CALL)                   \
    switch (N_) {                                     \
    case 64: return CALL(64);                         \
    case 128: return CALL(128);                       \
    case 256: return CALL(256);                       \
    case 512: return CALL(512);                       \
    case 1024: return CALL(1024);                     \
    case 2048: return CALL(2048);                     \
    case 4096: return CALL(4096);                     \
    default: return hipErrorInvalidValue;             \
    }

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

template <typename R>
hipError_t launch_xpass(int N, cx<R> *psi, int64_t nrows, int ny, const void *V0, bool v0_fp64,
                        const void *tw, const PhaseArgs &ph, int mode, hipStream_t st)
{
    if (v0_fp64) {
#define CALL(n) xpass_n<R, double, n>(psi, nrows, ny, V0, tw, ph, mode, st)
        SFO_SWITCH_PASS_N(N, CALL)
#undef CALL
    } else {
#define CALL(n) xpass_n<R, float, n>(psi, nrows, ny, V0, tw, ph, mode, st)
        SFO_SWITCH_PASS_N(N, CALL)
#undef CALL
    }
}

template <typename R, int N>
static hipError_t colpass_n(cx<R> *psi, int64_t ncols, int64_t stride, int nslab, int64_t slab_stride,
                            const void *tw, const KinArgs &kin, int mode, hipStream_t st)
{
    constexpr int C = cols_for<R, N>();
    constexpr int threads = C * LineShape<N, kRad>::T;
    if (ncols % C) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_colpass<R, N, kRad, C>), dim3((unsigned)(ncols / C), (unsigned)nslab), dim3(threads), 0,
                       st, psi, stride, slab_stride, (const TwEntry<R> *)tw, kin, mode);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_colpass(int N, cx<R> *psi, int64_t ncols, int64_t stride, int nslab, int64_t slab_stride,
                          const void *tw, const KinArgs &kin, int mode, hipStream_t st)
{
#define CALL(n) colpass_n<R, n>(psi, ncols, stride, nslab, slab_stride, tw, kin, mode, st)
    SFO_SWITCH_PASS_N(N, CALL)
#undef CALL
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
hipError_t launch_1d(int N, cx<R> *psi, int nprob, int64_t prob_stride, const void *V0, bool v0_fp64,
                     const void *tw, const Run1DArgs &a, hipStream_t st)
{
    if (v0_fp64) {
#define CALL(n) run1d_n<R, double, n>(psi, nprob, prob_stride, V0, tw, a, st)
        SFO_SWITCH_1D_N(N, CALL)
#undef CALL
    } else {
#define CALL(n) run1d_n<R, float, n>(psi, nprob, prob_stride, V0, tw, a, st)
        SFO_SWITCH_1D_N(N, CALL)
#undef CALL
    }
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

hipError_t launch_convert_v0(const double *src, void *dst, bool to_fp64, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_convert_v0, dim3(1024), dim3(256), 0, st, src, dst, to_fp64 ? 1 : 0, n);
    return hipGetLastError();
}

template hipError_t launch_xpass<float>(int, cx<float> *, int64_t, int, const void *, bool, const void *,
                                        const PhaseArgs &, int, hipStream_t);
template hipError_t launch_xpass<double>(int, cx<double> *, int64_t, int, const void *, bool, const void *,
                                         const PhaseArgs &, int, hipStream_t);
template hipError_t launch_colpass<float>(int, cx<float> *, int64_t, int64_t, int, int64_t, const void *,
                                          const KinArgs &, int, hipStream_t);
template hipError_t launch_colpass<double>(int, cx<double> *, int64_t, int64_t, int, int64_t, const void *,
                                           const KinArgs &, int, hipStream_t);
template hipError_t launch_1d<float>(int, cx<float> *, int, int64_t, const void *, bool, const void *,
                                     const Run1DArgs &, hipStream_t);
template hipError_t launch_1d<double>(int, cx<double> *, int, int64_t, const void *, bool, const void *,
                                      const Run1DArgs &, hipStream_t);
template hipError_t launch_norm<float>(const cx<float> *, int64_t, double *, double *, hipStream_t);
template hipError_t launch_norm<double>(const cx<double> *, int64_t, double *, double *, hipStream_t);
template hipError_t launch_overlap<float>(const cx<float> *, const cx<float> *, int64_t, double *, double *,
                                          hipStream_t);
template hipError_t launch_overlap<double>(const cx<double> *, const cx<double> *, int64_t, double *, double *,
                                           hipStream_t);

}  // namespace sfo
