// Split-step passes of the 2-D Dirac equation for a 4-spinor stored as four
// planes [4][ny][nx] (Sec. 2.3 of the paper, Dirac representation).
//
// Row pass: inverse x-transform of the four planes, the real-space factor
//   exp(-i sgn aV V0) [cos a + i sin a alpha_2],  a(x) = sgn q c Abar_y(x) / (2 hbar)
// (eq. exp_alpha with the single component A_y; i alpha_2 maps
// (p1, p2, p3, p4) to (p4, -p3, p2, -p1), so the factor is real apart from the
// scalar phase), forward x-transform.  Consecutive half steps merge: both the
// scalar phases and the alpha_2 rotations add.
// Column pass: forward y-transform, the momentum-space factor
//   U(k) = cos(E tau/hbar) - i sgn sin(E tau/hbar) H(hbar k) / E,
//   H = c (alpha_1 p_x + alpha_2 p_y) + m c^2 beta,  E = sqrt(m^2 c^4 + c^2 p^2)
// (eq. U_A_2_DE evaluated through H^2 = E^2), times 1/N_tot, inverse transform.
// In the Dirac representation H couples (1,4) and (2,3):
//   H = [[mc2, 0, 0, w], [0, mc2, wb, 0], [0, w, -mc2, 0], [wb, 0, 0, -mc2]],
//   w = c (p_x - i p_y), wb = c (p_x + i p_y).
// The spinor factors are evaluated in FP64 and applied in FP64.
#include <type_traits>

#include "pass_kernels.h"

namespace sfo {

template <typename R> __device__ __forceinline__ void dirac_rotate(cx<R> (&p)[4], double c, double s, double fr, double fi)
{
    // p <- (fr + i fi) (c p + s (p4, -p3, p2, -p1)) in FP64
    const double r0 = c * (double)p[0].re + s * (double)p[3].re, i0 = c * (double)p[0].im + s * (double)p[3].im;
    const double r1 = c * (double)p[1].re - s * (double)p[2].re, i1 = c * (double)p[1].im - s * (double)p[2].im;
    const double r2 = c * (double)p[2].re + s * (double)p[1].re, i2 = c * (double)p[2].im + s * (double)p[1].im;
    const double r3 = c * (double)p[3].re - s * (double)p[0].re, i3 = c * (double)p[3].im - s * (double)p[0].im;
    p[0] = {(R)(fr * r0 - fi * i0), (R)(fr * i0 + fi * r0)};
    p[1] = {(R)(fr * r1 - fi * i1), (R)(fr * i1 + fi * r1)};
    p[2] = {(R)(fr * r2 - fi * i2), (R)(fr * i2 + fi * r2)};
    p[3] = {(R)(fr * r3 - fi * i3), (R)(fr * i3 + fi * r3)};
}

template <typename R, int N, int RAD>
__global__ void __launch_bounds__((RowTile<N, RAD, 256>::NT))
    k_dirac_xpass(cx<R> *__restrict__ psi, int64_t plane, const VStore<R> *__restrict__ V0,
                  const TwEntry<R> *__restrict__ tw, DiracPhaseArgs ph, int mode)
{
    using Sh = LineShape<N, RAD>;
    using Map = RowMap<R, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV, ROWS = RowTile<N, RAD, 256>::ROWS;
    __shared__ cx<R> lds[ROWS * Map::slots(N)];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int64_t row0 = (int64_t)blockIdx.x * ROWS, row = row0 + line;
    cx<R> *sh = lds + line * Map::slots(N);
    // addresses: the work-group's uniform base of plane q, element m (scalar
    // registers) plus the thread's 32-bit byte offset (see row_load)
    uint32_t lt = (uint32_t)(line * N + t) * (uint32_t)sizeof(cx<R>);
    auto at = [&](int q, int m) {
        char *b = scalar_base((char *)(psi + q * plane + row0 * N + m * T));
        return (cx<R> *)(b + lt);
    };
    // stage factors formed from each stage's W^k, read once with the line (no
    // table reads inside the transforms)
    TwBase<N, RAD> wb;
    tw_base_load(wb, tw, t);
    cx<R> v[4][RV];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) v[q][m] = gload(at(q, m));
    if (mode & M_INV)
#pragma unroll
        for (int q = 0; q < 4; ++q) fft_line_pre<R, N, RAD, +1, Map>(v[q], sh, t, tw, wb);
    if (mode & M_PHASE) {
        const double sg = (double)ph.sgn;
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const int x = t + m * T;
            double s, c;
            sincos_fp64(sg * ph.aV * (double)gload1(V0 + row * N + x), s, c);
            double ab = 0.0;
            if (ph.abar_a) ab += ph.ca * ph.abar_a[x];
            if (ph.abar_b) ab += ph.cb * ph.abar_b[x];
            double sa, ca;
            sincos_fp64(sg * ph.aA * ab, sa, ca);
            cx<R> p[4] = {v[0][m], v[1][m], v[2][m], v[3][m]};
            dirac_rotate(p, ca, sa, c, -s);
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q][m] = p[q];
        }
    }
    if (mode & M_FWD)
#pragma unroll
        for (int q = 0; q < 4; ++q) fft_line_pre<R, N, RAD, -1, Map>(v[q], sh, t, tw, wb);
    // the offset is recomputed rather than held through the transforms
    __asm__ __volatile__("" : "+v"(lt));
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) gstore(at(q, m), v[q][m]);
}

template <typename R, int N, int RAD, int C>
__global__ void __launch_bounds__((C * LineShape<N, RAD>::T))
    k_dirac_colpass(cx<R> *__restrict__ psi, int64_t plane, int nx, const TwEntry<R> *__restrict__ tw,
                    DiracKinArgs kin, int mode)
{
    using Sh = LineShape<N, RAD>;
    using Map = ColMap<C>;
    constexpr int T = Sh::T, RV = Sh::RV;
    __shared__ cx<R> lds[Map::slots(N)];
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const unsigned G = gridDim.x;
    unsigned L = blockIdx.x;
    if ((G & 7u) == 0) L = (L & 7u) * (G >> 3) + (L >> 3);
    const int64_t col = (int64_t)L * C + c;
    cx<R> *sh = lds + c;
    // addresses: uniform base of plane q, element m (scalar registers) plus the
    // thread's 32-bit byte offset (t nx + c) (see col_load; the launcher checks the range)
    uint32_t tb = ((uint32_t)t * (uint32_t)nx + (uint32_t)c) * (uint32_t)sizeof(cx<R>);
    auto at = [&](int q, int m) {
        char *b = (char *)(psi + q * plane + (int64_t)m * T * nx + (int64_t)L * C);
        __asm__ __volatile__("" : "+s"(b));
        return (cx<R> *)(b + tb);
    };
    TwBase<N, RAD> wb;  // stage factors formed from W^k (see k_dirac_xpass)
    tw_base_load(wb, tw, t);
    cx<R> v[4][RV];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) v[q][m] = gload(at(q, m));
    if (mode & M_FWD)
#pragma unroll
        for (int q = 0; q < 4; ++q) fft_line_pre<R, N, RAD, -1, Map>(v[q], sh, t, tw, wb);
    if (mode & M_KIN) {
        const double px = kin.hbar * kin.kx[col];
        const double sg = (double)kin.sgn;
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            const double py = kin.hbar * kin.ky[t + m * T];
            const double E = sqrt(kin.mc2 * kin.mc2 + kin.c * kin.c * (px * px + py * py));
            double sE, cE;
            sincos_fp64(E * kin.tau_over_hbar, sE, cE);
            const double sig = sg * sE / E;
            // U = C - i sig H, scaled by 1/Ntot
            const double Cn = cE * kin.inv_ntot, sgn_ = sig * kin.inv_ntot;
            const double am = sgn_ * kin.mc2;              // diag: Cn -+ i am
            const double wr = kin.c * px, wi = -kin.c * py; // w = c (px - i py)
            // off-diagonal coefficient -i sig w = (sig wi) - i (sig wr)  [times 1/Ntot]
            const double owr = sgn_ * wi, owi = -sgn_ * wr;     // -i sig w
            const double obr = -sgn_ * wi, obi = -sgn_ * wr;    // -i sig wb, wb = conj(w)
            double a[4][2];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q][0] = (double)v[q][m].re;
                a[q][1] = (double)v[q][m].im;
            }
            auto mul = [](double xr, double xi, double yr, double yi, double &zr, double &zi) {
                zr = xr * yr - xi * yi;
                zi = xr * yi + xi * yr;
            };
            double t0r, t0i, t1r, t1i;
            // psi1' = (Cn - i am) psi1 + (-i sig w) psi4
            mul(Cn, -am, a[0][0], a[0][1], t0r, t0i);
            mul(owr, owi, a[3][0], a[3][1], t1r, t1i);
            const double n0r = t0r + t1r, n0i = t0i + t1i;
            // psi4' = (-i sig wb) psi1 + (Cn + i am) psi4
            mul(obr, obi, a[0][0], a[0][1], t0r, t0i);
            mul(Cn, am, a[3][0], a[3][1], t1r, t1i);
            const double n3r = t0r + t1r, n3i = t0i + t1i;
            // psi2' = (Cn - i am) psi2 + (-i sig wb) psi3
            mul(Cn, -am, a[1][0], a[1][1], t0r, t0i);
            mul(obr, obi, a[2][0], a[2][1], t1r, t1i);
            const double n1r = t0r + t1r, n1i = t0i + t1i;
            // psi3' = (-i sig w) psi2 + (Cn + i am) psi3
            mul(owr, owi, a[1][0], a[1][1], t0r, t0i);
            mul(Cn, am, a[2][0], a[2][1], t1r, t1i);
            const double n2r = t0r + t1r, n2i = t0i + t1i;
            v[0][m] = {(R)n0r, (R)n0i};
            v[1][m] = {(R)n1r, (R)n1i};
            v[2][m] = {(R)n2r, (R)n2i};
            v[3][m] = {(R)n3r, (R)n3i};
        }
    }
    if (mode & M_INV)
#pragma unroll
        for (int q = 0; q < 4; ++q) fft_line_pre<R, N, RAD, +1, Map>(v[q], sh, t, tw, wb);
    __asm__ __volatile__("" : "+v"(tb));
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) gstore(at(q, m), v[q][m]);
}

// Tile shapes: radix 8 (four planes in registers), rows filling 256 threads;
// columns: 4 adjacent lines (64-byte row segments of complex128), within 1024
// threads and 160 KiB of LDS.  Complex128 holds about 240 VGPRs per thread,
// so it keeps 4 columns only while a group stays within 512 threads (two
// waves per SIMD) and takes 2 beyond that.
constexpr int kDiracRad = 8;
template <typename R, int N> constexpr int dirac_cols()
{
    constexpr int T = LineShape<N, kDiracRad>::T;
    int c = (sizeof(R) == 4 || 4 * T <= 512) ? 4 : 2;
    while (c > 1 && (c * T > 1024 || ColMap<1>::slots(N) * c * (int)sizeof(cx<R>) > 160 * 1024))
        c /= 2;
    return c;
}

template <typename R, int N>
static hipError_t dirac_x_n(cx<R> *psi, int ny, int64_t plane, const void *V0, const void *tw, const DiracPhaseArgs &ph,
                            int mode, hipStream_t st)
{
    using Tl = RowTile<N, kDiracRad, 256>;
    if (ny % Tl::ROWS) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_dirac_xpass<R, N, kDiracRad>), dim3((unsigned)(ny / Tl::ROWS)), dim3(Tl::NT), 0, st, psi,
                       plane, (const VStore<R> *)V0, (const TwEntry<R> *)tw, ph, mode);
    return hipGetLastError();
}

template <typename R, int N>
static hipError_t dirac_c_n(cx<R> *psi, int nx, int64_t plane, const void *tw, const DiracKinArgs &kin, int mode,
                            hipStream_t st)
{
    constexpr int C = dirac_cols<R, N>();
    if (nx % C) return hipErrorInvalidValue;
    // per-thread byte offsets within a work-group's columns are 32-bit
    if (((int64_t)(LineShape<N, kDiracRad>::T - 1) * nx + C) * (int64_t)sizeof(cx<R>) > (int64_t)UINT32_MAX)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_dirac_colpass<R, N, kDiracRad, C>), dim3((unsigned)(nx / C)),
                       dim3(C * LineShape<N, kDiracRad>::T), 0, st, psi, plane, nx, (const TwEntry<R> *)tw, kin, mode);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_dirac_xpass(int N, cx<R> *psi, int ny, int64_t plane, const void *V0, const void *tw,
                              const DiracPhaseArgs &ph, int mode, hipStream_t st)
{
#define CALL(n) dirac_x_n<R, n>(psi, ny, plane, V0, tw, ph, mode, st)
    SFO_SWITCH_PASS_N(N, CALL)
#undef CALL
}

template <typename R>
hipError_t launch_dirac_colpass(int N, cx<R> *psi, int nx, int64_t plane, const void *tw, const DiracKinArgs &kin,
                                int mode, hipStream_t st)
{
#define CALL(n) dirac_c_n<R, n>(psi, nx, plane, tw, kin, mode, st)
    SFO_SWITCH_PASS_N(N, CALL)
#undef CALL
}

// ------------------------------------------------------------- 1-D Dirac --
// The whole run of one line in one work-group: both components in registers
// (cyclic layout), transformed one after the other through the same LDS
// region; the real-space factor exp(-i th) (cos a + i sin a sigma_x) and the
// momentum-space 2x2 factor are applied in FP64 with one rounding.
template <typename R, typename VT, int N, int RAD>
__global__ void __launch_bounds__((LineShape<N, RAD>::T))
    k_dirac1d_run(cx<R> *__restrict__ psi, const VT *__restrict__ V0, const TwEntry<R> *__restrict__ tw,
                  Dirac1DArgs a)
{
    using Sh = LineShape<N, RAD>;
    constexpr int T = Sh::T, RV = Sh::RV;
    __shared__ cx<R> sh[RowMap<R, RAD>::slots(N)];
    const int t = threadIdx.x;
    cx<R> v[2][RV];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) v[q][m] = gload(psi + (int64_t)q * N + t + m * T);
    auto abar = [&](int64_t st, int x) { return a.abar ? a.abar[st * N + x] : 0.0; };
    // halves of steps sa and sb (sb < 0: one half)
    auto potential = [&](int64_t sa, int64_t sb) {
        const double w = sb >= 0 ? 2.0 : 1.0;
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            // an opaque index pins this point's table reads here (they do not
            // depend on the state; the compiler would issue them all at once)
            int x = t + m * T;
            __asm__ __volatile__("" : "+v"(x));
            const double th = w * a.aV_half * ldv(V0 + x);
            const double aa = a.aA * (abar(sa, x) + (sb >= 0 ? abar(sb, x) : 0.0));
            double s, c, sa_, ca;
            sincos_fp64(th, s, c);
            sincos_fp64(aa, sa_, ca);
            const double ur = v[0][m].re, ui = v[0][m].im, vr = v[1][m].re, vi = v[1][m].im;
            // (cos a u + i sin a v, i sin a u + cos a v), then times exp(-i th) = (c - i s)
            const double pr = ca * ur - sa_ * vi, pi = ca * ui + sa_ * vr;
            const double qr = ca * vr - sa_ * ui, qi = ca * vi + sa_ * ur;
            v[0][m] = {(R)(c * pr + s * pi), (R)(c * pi - s * pr)};
            v[1][m] = {(R)(c * qr + s * qi), (R)(c * qi - s * qr)};
            if ((m & 1) == 1) __builtin_amdgcn_sched_barrier(0);
        }
    };
    if (a.nsteps > 0) potential(a.step0, -1);
#pragma unroll 1
    for (int64_t s = 0; s < a.nsteps; ++s) {
        __asm__ __volatile__("" ::: "memory");
#pragma unroll
        for (int q = 0; q < 2; ++q) fft_line<R, N, RAD, -1, RowMap<R, RAD>>(v[q], sh, t, tw);
#pragma unroll
        for (int m = 0; m < RV; ++m) {
            int k = t + m * T;
            __asm__ __volatile__("" : "+v"(k));
            const double2 u00 = a.u[3 * k], u01 = a.u[3 * k + 1], u11 = a.u[3 * k + 2];
            const double ur = v[0][m].re, ui = v[0][m].im, vr = v[1][m].re, vi = v[1][m].im;
            v[0][m] = {(R)(u00.x * ur - u00.y * ui + u01.x * vr - u01.y * vi),
                       (R)(u00.x * ui + u00.y * ur + u01.x * vi + u01.y * vr)};
            v[1][m] = {(R)(u01.x * ur - u01.y * ui + u11.x * vr - u11.y * vi),
                       (R)(u01.x * ui + u01.y * ur + u11.x * vi + u11.y * vr)};
            if ((m & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) fft_line<R, N, RAD, +1, RowMap<R, RAD>>(v[q], sh, t, tw);
        const bool more = s + 1 < a.nsteps;
        potential(a.step0 + s, more ? a.step0 + s + 1 : -1);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int m = 0; m < RV; ++m) gstore(psi + (int64_t)q * N + t + m * T, v[q][m]);
}

// tws[0], tws[1]: the line's stage twiddles for radix 8 and 16.  Long lines
// use radix 8 (more threads, half the registers per thread for the two
// components).
template <typename R, int N>
static hipError_t dirac1d_n(cx<R> *psi, const void *V0, const void *const *tws, const Dirac1DArgs &a,
                            hipStream_t st)
{
    using VT = typename std::conditional<sizeof(R) == 4, float, double>::type;
    constexpr int RAD = N >= 4096 ? 8 : 16;
    hipLaunchKernelGGL((k_dirac1d_run<R, VT, N, RAD>), dim3(1), dim3(LineShape<N, RAD>::T), 0, st, psi,
                       (const VT *)V0, (const TwEntry<R> *)tws[RAD == 8 ? 0 : 1], a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_dirac1d(int N, cx<R> *psi, const void *V0, const void *const *tw, const Dirac1DArgs &a,
                          hipStream_t st)
{
    switch (N) {
    case 64: return dirac1d_n<R, 64>(psi, V0, tw, a, st);
    case 128: return dirac1d_n<R, 128>(psi, V0, tw, a, st);
    case 256: return dirac1d_n<R, 256>(psi, V0, tw, a, st);
    case 512: return dirac1d_n<R, 512>(psi, V0, tw, a, st);
    case 1024: return dirac1d_n<R, 1024>(psi, V0, tw, a, st);
    case 2048: return dirac1d_n<R, 2048>(psi, V0, tw, a, st);
    case 4096: return dirac1d_n<R, 4096>(psi, V0, tw, a, st);
    case 8192: return dirac1d_n<R, 8192>(psi, V0, tw, a, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_dirac1d<float>(int, cx<float> *, const void *, const void *const *,
                                          const Dirac1DArgs &, hipStream_t);
template hipError_t launch_dirac1d<double>(int, cx<double> *, const void *, const void *const *,
                                           const Dirac1DArgs &, hipStream_t);

template hipError_t launch_dirac_xpass<float>(int, cx<float> *, int, int64_t, const void *, const void *,
                                              const DiracPhaseArgs &, int, hipStream_t);
template hipError_t launch_dirac_xpass<double>(int, cx<double> *, int, int64_t, const void *, const void *,
                                               const DiracPhaseArgs &, int, hipStream_t);
template hipError_t launch_dirac_colpass<float>(int, cx<float> *, int, int64_t, const void *, const DiracKinArgs &,
                                                int, hipStream_t);
template hipError_t launch_dirac_colpass<double>(int, cx<double> *, int, int64_t, const void *, const DiracKinArgs &,
                                                 int, hipStream_t);

}  // namespace sfo
