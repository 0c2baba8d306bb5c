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


// ---------------------------------------------------------------- 1-D run --
// 1-D whole-run arguments of problem P of a grouped launch.
template <typename R> __device__ __forceinline__ void group_1d_args(const BatchProb<R> &P, Run1DArgs &a)
{
    a.kin = P.kin_x;
    a.ebar = P.ebar;
    a.aV_half = P.aV_half;
    a.inv_2hbar = P.inv_2hbar;
    a.xmin = P.xmin[0];
    a.dx = P.dx[0];
}

template <typename R, typename VT, int N, int RAD>
__global__ void __launch_bounds__((LineShape<N, RAD>::T))
    k_1d_run(cx<R> *__restrict__ psi, int64_t prob_stride, const VT *__restrict__ V0,
             const TwEntry<R> *__restrict__ tw, Run1DArgs a, GroupArgs<R> grp)
{
    __shared__ cx<R> sh[RowMap<R, RAD>::slots(N)];
    if (grp.probs) {
        const BatchProb<R> &P = grp.probs[grp.ids[blockIdx.x]];
        group_1d_args(P, a);
        run1d_tile<R, VT, N, RAD>(P.psi, (const VT *)P.V0, tw, a, sh, threadIdx.x);
        return;
    }
    run1d_tile<R, VT, N, RAD>(psi + (int64_t)blockIdx.x * prob_stride, V0 + (int64_t)blockIdx.x * prob_stride, tw, a,
                              sh, threadIdx.x);
}

// 1-D eigenstate run of one line: MODE 1 autocorrelation, MODE 2 windowed
// eigenfunction (see run1d_tile).
template <typename R, typename VT, int N, int RAD, int MODE>
__global__ void __launch_bounds__((LineShape<N, RAD>::T))
    k_1d_eigen(cx<R> *__restrict__ psi, const VT *__restrict__ V0, const TwEntry<R> *__restrict__ tw, Run1DArgs a)
{
    __shared__ cx<R> sh[RowMap<R, RAD>::slots(N)];
    __shared__ double red[16][3];
    run1d_tile<R, VT, N, RAD, MODE>(psi, V0, tw, a, sh, threadIdx.x, red);
}

// ------------------------------------------------------------ 1-D adjoint --
template <typename R, typename VT, int N, int RAD>
__global__ void __launch_bounds__((LineShape<N, RAD>::T))
    k_1d_adjoint(cx<R> *__restrict__ psi, cx<R> *__restrict__ gv, const VT *__restrict__ V0,
                 const TwEntry<R> *__restrict__ tw, Run1DArgs a, double wbase, double *acc_out, double *mom,
                 GroupArgs<R> grp)
{
    __shared__ cx<R> sh[RowMap<R, RAD>::slots(N)];
    __shared__ double red[16][3];
    if (grp.probs) {
        const BatchProb<R> &P = grp.probs[grp.ids[blockIdx.x]];
        group_1d_args(P, a);
        adj1d_tile<R, VT, N, RAD>(P.psi, P.gadj, (const VT *)P.V0, tw, a, P.aV_half, P.dV, P.part, sh, red,
                                  threadIdx.x);
        return;
    }
    adj1d_tile<R, VT, N, RAD>(psi, gv, V0, tw, a, wbase, acc_out, mom, sh, red, threadIdx.x);
}

__global__ void k_ebar_grad(const double *part, int nslots, int64_t nsteps, int ndim, double scale, double *out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nsteps * ndim; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / ndim;
        const int a = (int)(i % ndim);
        double m1 = 0.0, m0 = 0.0;
        for (int k = 0; k < nslots; ++k) {
            m1 += part[((s + 1) * nslots + k) * 3 + a];
            m0 += part[(s * nslots + k) * 3 + a];
        }
        out[i] = (m1 + m0) * scale;
    }
}

// Velocity-gauge gradient: per step j and axis a (one thread each; the
// step's A2bar derivative by the thread of axis 0), the slots summed in slot
// order (see launch_vgrad_sum).
__global__ void k_vgrad_sum(const double *part, int nslots, int64_t nsteps, int ndim, double sA, double sA2, double *dA,
                            double *dA2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nsteps * ndim; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = i / ndim;
        const int a = (int)(i % ndim);
        // partial index of axis a: the moment along the line is entry 2
        const int idx = a == ndim - 1 ? 2 : a;
        double m = 0.0, m1 = 0.0;
        for (int k = 0; k < nslots; ++k) {
            m += part[(j * nslots + k) * 4 + idx];
            m1 += part[(j * nslots + k) * 4 + 3];
        }
        if (dA) dA[i] = m * sA;
        if (dA2 && a == 0) dA2[j] = m1 * sA2;
    }
}

// Autocorrelation: chi_j = scale * sum over the slots of step j (slot order).
__global__ void k_chi_sum(const double *part, int nslots, int64_t nsteps, double scale, double *chi)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nsteps; j += (int64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k < nslots; ++k) {
            re += part[(j * nslots + k) * 2];
            im += part[(j * nslots + k) * 2 + 1];
        }
        chi[2 * j] = re * scale;
        chi[2 * j + 1] = im * scale;
    }
}

// Windowed transform of the autocorrelation, one energy per thread: the sum
// over steps in step order, window 1 - cos(2 pi j / nsteps), phase j dt E /
// hbar (range-reduced FP64 sine and cosine).
__global__ void k_spectrum(const double *chi, int64_t nsteps, double dt, double hbar, const double *E, int nE,
                           double *out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nE) return;
    const double w0 = 2.0 * 3.14159265358979323846 / (double)nsteps, a = dt * E[e] / hbar;
    double re = 0.0, im = 0.0;
    for (int64_t j = 0; j < nsteps; ++j) {
        double sw, cw, s, c;
        sincos_fp64(w0 * (double)j, sw, cw);
        sincos_fp64(a * (double)j, s, c);
        const double w = 1.0 - cw, xr = chi[2 * j], xi = chi[2 * j + 1];
        re += w * (xr * c - xi * s);
        im += w * (xr * s + xi * c);
    }
    out[2 * e] = dt * re;
    out[2 * e + 1] = dt * im;
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

// max that keeps a NaN (fmax would return the other operand), so a NaN
// anywhere in the input reaches the result and the host's finiteness check
__device__ inline double max_keep_nan(double acc, double v) { return (v != v || v > acc) ? v : acc; }

__global__ void __launch_bounds__(256) k_absmax_partial(const double *__restrict__ a, int64_t n, double *part)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        acc = max_keep_nan(acc, fabs(a[i]));
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] = max_keep_nan(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(256) k_max_partials(const double *part, int count, double *out)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += 256) acc = max_keep_nan(acc, part[i]);
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] = max_keep_nan(s[threadIdx.x], s[threadIdx.x + h]);
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

// Windowed eigenfunction: acc += (cr + i ci) s in FP64, and the final
// rounding of the accumulator to the state's precision.
template <typename R>
__global__ void k_eig_axpy(const cx<R> *__restrict__ s, double2 *__restrict__ acc, int64_t n, double cr, double ci)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double a = (double)s[i].re, b = (double)s[i].im;
        double2 r = acc[i];
        r.x += cr * a - ci * b;
        r.y += cr * b + ci * a;
        acc[i] = r;
    }
}

template <typename R> __global__ void k_acc_to_state(const double2 *__restrict__ acc, cx<R> *__restrict__ out, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = {(R)acc[i].x, (R)acc[i].y};
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
                          const Run1DArgs &a, hipStream_t st, const GroupArgs<R> &grp)
{
    constexpr int threads = LineShape<N, kRad>::T;
    hipLaunchKernelGGL((k_1d_run<R, VT, N, kRad>), dim3((unsigned)nprob), dim3(threads), 0, st, psi, prob_stride,
                       (const VT *)V0, (const TwEntry<R> *)tw, a, grp);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_1d(int N, cx<R> *psi, int nprob, int64_t prob_stride, const void *V0, const void *tw,
                     const Run1DArgs &a, hipStream_t st, const GroupArgs<R> &grp)
{
    using VT = typename std::conditional<sizeof(R) == 4, float, double>::type;
#define CALL(n) run1d_n<R, VT, n>(psi, nprob, prob_stride, V0, tw, a, st, grp)
    SFO_SWITCH_1D_N(N, CALL)
#undef CALL
}

template <typename R, typename VT, int N>
static hipError_t eig1d_n(cx<R> *psi, const void *V0, const void *tw, const Run1DArgs &a, hipStream_t st)
{
    constexpr int threads = LineShape<N, kRad>::T;
    if (a.chi)
        hipLaunchKernelGGL((k_1d_eigen<R, VT, N, kRad, 1>), dim3(1), dim3(threads), 0, st, psi, (const VT *)V0,
                           (const TwEntry<R> *)tw, a);
    else
        hipLaunchKernelGGL((k_1d_eigen<R, VT, N, kRad, 2>), dim3(1), dim3(threads), 0, st, psi, (const VT *)V0,
                           (const TwEntry<R> *)tw, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_1d_eigen(int N, cx<R> *psi, const void *V0, const void *tw, const Run1DArgs &a, hipStream_t st)
{
    using VT = typename std::conditional<sizeof(R) == 4, float, double>::type;
    if ((!a.chi && !a.eig_acc) || (a.chi && !a.ref) || (a.eig_acc && !a.eig_out) || a.dir != 1 || a.ebar)
        return hipErrorInvalidValue;
#define CALL(n) eig1d_n<R, VT, n>(psi, V0, tw, a, st)
    SFO_SWITCH_1D_N(N, CALL)
#undef CALL
}

template <typename R, typename VT, int N>
static hipError_t adj1d_n(cx<R> *psi, cx<R> *gv, const void *V0, const void *tw, const Run1DArgs &a, double wbase,
                          double *acc, double *mom, hipStream_t st, const GroupArgs<R> &grp, int ngroup)
{
    constexpr int threads = LineShape<N, kRad>::T;
    hipLaunchKernelGGL((k_1d_adjoint<R, VT, N, kRad>), dim3((unsigned)ngroup), dim3(threads), 0, st, psi, gv,
                       (const VT *)V0, (const TwEntry<R> *)tw, a, wbase, acc, mom, grp);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_1d_adjoint(int N, cx<R> *psi, cx<R> *gv, const void *V0, const void *tw, const Run1DArgs &a,
                             double wbase, double *acc, double *mom, hipStream_t st, const GroupArgs<R> &grp,
                             int ngroup)
{
    using VT = typename std::conditional<sizeof(R) == 4, float, double>::type;
#define CALL(n) adj1d_n<R, VT, n>(psi, gv, V0, tw, a, wbase, acc, mom, st, grp, ngroup)
    SFO_SWITCH_1D_N(N, CALL)
#undef CALL
}

hipError_t launch_ebar_grad(const double *part, int nslots, int64_t nsteps, int ndim, double scale, double *out,
                            hipStream_t st)
{
    if (nsteps <= 0) return hipSuccess;
    const int64_t n = nsteps * ndim;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_ebar_grad, dim3(blocks), dim3(256), 0, st, part, nslots, nsteps, ndim, scale, out);
    return hipGetLastError();
}

hipError_t launch_vgrad_sum(const double *part, int nslots, int64_t nsteps, int ndim, double sA, double sA2,
                            double *dA, double *dA2, hipStream_t st)
{
    if (nsteps <= 0 || (!dA && !dA2)) return hipSuccess;
    const int64_t n = nsteps * ndim;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_vgrad_sum, dim3(blocks), dim3(256), 0, st, part, nslots, nsteps, ndim, sA, sA2, dA, dA2);
    return hipGetLastError();
}

hipError_t launch_chi_sum(const double *part, int nslots, int64_t nsteps, double scale, double *chi, hipStream_t st)
{
    if (nsteps <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>((nsteps + 255) / 256, 4096);
    hipLaunchKernelGGL(k_chi_sum, dim3(blocks), dim3(256), 0, st, part, nslots, nsteps, scale, chi);
    return hipGetLastError();
}

hipError_t launch_spectrum(const double *chi, int64_t nsteps, double dt, double hbar, const double *E, int nE,
                           double *out, hipStream_t st)
{
    if (nE <= 0 || nsteps <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_spectrum, dim3((unsigned)(((int64_t)nE + 63) / 64)), dim3(64), 0, st, chi, nsteps, dt, hbar, E, nE,
                       out);
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

template <typename R>
hipError_t launch_eig_axpy(const cx<R> *s, double2 *acc, int64_t n, double cr, double ci, hipStream_t st)
{
    hipLaunchKernelGGL(k_eig_axpy<R>, dim3(2048), dim3(256), 0, st, s, acc, n, cr, ci);
    return hipGetLastError();
}

template <typename R> hipError_t launch_acc_to_state(const double2 *acc, cx<R> *out, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_acc_to_state<R>, dim3(2048), dim3(256), 0, st, acc, out, n);
    return hipGetLastError();
}

template hipError_t launch_eig_axpy<float>(const cx<float> *, double2 *, int64_t, double, double, hipStream_t);
template hipError_t launch_eig_axpy<double>(const cx<double> *, double2 *, int64_t, double, double, hipStream_t);
template hipError_t launch_acc_to_state<float>(const double2 *, cx<float> *, int64_t, hipStream_t);
template hipError_t launch_acc_to_state<double>(const double2 *, cx<double> *, int64_t, hipStream_t);

hipError_t launch_convert_v0(const double *src, void *dst, bool to_fp64, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_convert_v0, dim3(1024), dim3(256), 0, st, src, dst, to_fp64 ? 1 : 0, n);
    return hipGetLastError();
}

template hipError_t launch_1d_eigen<float>(int, cx<float> *, const void *, const void *, const Run1DArgs &,
                                           hipStream_t);
template hipError_t launch_1d_eigen<double>(int, cx<double> *, const void *, const void *, const Run1DArgs &,
                                            hipStream_t);
template hipError_t launch_1d<float>(int, cx<float> *, int, int64_t, const void *, const void *, const Run1DArgs &,
                                     hipStream_t, const GroupArgs<float> &);
template hipError_t launch_1d<double>(int, cx<double> *, int, int64_t, const void *, const void *, const Run1DArgs &,
                                      hipStream_t, const GroupArgs<double> &);
template hipError_t launch_1d_adjoint<float>(int, cx<float> *, cx<float> *, const void *, const void *,
                                             const Run1DArgs &, double, double *, double *, hipStream_t,
                                             const GroupArgs<float> &, int);
template hipError_t launch_1d_adjoint<double>(int, cx<double> *, cx<double> *, const void *, const void *,
                                              const Run1DArgs &, double, double *, double *, hipStream_t,
                                              const GroupArgs<double> &, int);
template hipError_t launch_norm<float>(const cx<float> *, int64_t, double *, double *, hipStream_t);
template hipError_t launch_norm<double>(const cx<double> *, int64_t, double *, double *, hipStream_t);
template hipError_t launch_overlap<float>(const cx<float> *, const cx<float> *, int64_t, double *, double *,
                                          hipStream_t);
template hipError_t launch_overlap<double>(const cx<double> *, const cx<double> *, int64_t, double *, double *,
                                           hipStream_t);

}  // namespace sfo
