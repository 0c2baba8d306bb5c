// Internal interface between the C ABI layer (sfo_api.hip) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "fft_engine.h"
#include "sfo_validate.h"

namespace sfo {

// Pass modes: which operations a line pass applies, in this order.
enum : int {
    M_INV = 1,    // inverse transform along the pass axis (first)
    M_PHASE = 2,  // real-space potential factor (row passes only)
    M_KIN = 8,    // momentum-space factor (column passes only)
    M_FWD = 4,    // forward transform along the pass axis (last for rows, first for columns)
    M_GRAD = 16,  // adjoint partials at a step boundary (row passes with two states)
    M_CHI = 32,   // overlap with a reference k-space state after the forward transform (column passes)
    M_VGRAD = 64, // velocity-gauge gradient partials in k-space after the forward transform (two-state k-space passes)
};

// The states a pass transforms together: p[0] alone, or the state p[0] and
// its adjoint p[1] during the reverse sweep.
template <typename R> struct StatePtrs {
    cx<R> *p[2];
};

// Gradient partials of a row pass at one step boundary (see k_xpass).
struct GradArgs {
    double *acc;       // dL/dV0 accumulator (FP64, one per point) or null
    double wacc;       // weight of this boundary in acc
    int acc_init;      // 1: overwrite acc instead of adding
    double *part;      // this boundary's moment partials: 3 per work-group (slot = blockIdx.x)
};

// Real-space phase of a row pass: theta(x) = aV * V0(x) + e . x, applied as
// exp(-i sgn theta) (sgn = -1 for the inverse step).
struct PhaseArgs {
    double aV;
    double e[3];
    double xmin[3];
    double dx[3];
    int sgn;
    int small;    // |aV V0| <= 1/8 everywhere: short FP64 sin/cos series suffice
    int small32;  // |aV V0 + e.x| <= 1/8 everywhere: complex64 may form the factor in FP32
};

// Momentum-space factor of a column pass, for element e of column `col`:
//   K = kA[col % nA] * kB[col / nA] * kL[e]   (conjugated if sgn < 0).
// M_CHI: chi_part[2 slot + {0, 1}] = sum over the work-group's points of
// conj(chi_ref) psi~ (FP64) right after the forward transform, slot = the
// work-group's linear index; chi_ref has the state's layout.
struct KinArgs {
    const double2 *kA;
    const double2 *kB;
    const double2 *kL;
    int nA;
    int sgn;
    const void *chi_ref = nullptr;
    double *chi_part = nullptr;
    // M_VGRAD (two states psi~, g~ in k-space): wave numbers of the line's
    // other axes, kvA[col % nA] and kvB[col / nA] (kvB null: 0), and along the
    // line, kvL[e]; vpart[4 slot + {0, 1, 2, 3}] = sum over the work-group's
    // points of (kA, kB, kL, 1) Im(conj(g~) psi~), slot = the work-group's
    // linear index
    const double *kvA = nullptr, *kvB = nullptr, *kvL = nullptr;
    double *vpart = nullptr;
};

// Dirac real-space factor of a row pass (4 planes):
//   exp(-i sgn aV V0) [cos a + i sin a alpha_2],  a = sgn * aA * Abar_y(x),
// with Abar_y(x) = ca * abar[step_a][x] + cb * abar[step_b][x].
struct DiracPhaseArgs {
    double aV;
    double aA;
    const double *abar_a;
    const double *abar_b;
    double ca, cb;
    int sgn;
};

// Dirac momentum-space factor: (1/Ntot) [cos(E tau/hbar) - i sgn sin(E tau/hbar) H/E],
// H = c alpha.(hbar k) + m c^2 beta; k from per-axis wave-number tables.
struct DiracKinArgs {
    const double *kx;  // nx wave numbers (FFT order)
    const double *ky;  // ny wave numbers
    double c, mc2, hbar, tau_over_hbar, inv_ntot;
    int sgn;
};

// 1-D whole-run kernel arguments (one work-group per problem).
struct Run1DArgs {
    const double2 *kin;  // N kinetic factors (1/N folded in); step st uses kin + st * kin_stride
    const double *ebar;  // per-step field integrals (1 per step) or null
    int64_t step0, nsteps;
    double aV_half;   // tau / (2 hbar)
    double inv_2hbar; // 1 / (2 hbar)
    double xmin, dx;
    int dir;          // +1 forward steps, -1 inverse steps (last first)
    int64_t kin_stride = 0;  // velocity gauge: per-step kinetic tables, N apart (0: one table)
    // velocity-gauge reverse sweep: wave numbers of the line (kv) and, per
    // step s of the run, vmom[4 s + {2, 3}] = sum_k (k, 1) Im(conj(g~) psi~)
    // in k-space after the forward transforms ({0, 1} are set to 0)
    const double *kv = nullptr;
    double *vmom = nullptr;
    // eigenstate runs (time-independent potential, dir = +1): chi[2 s + {0, 1}]
    // = dv sum conj(psi_0) psi_s with ref (a state-sized buffer) keeping
    // P psi_0; or the windowed eigenfunction, accumulated in FP64 in eig_acc
    // and written to eig_out (see run1d_tile)
    double *chi = nullptr;
    void *ref = nullptr;
    double2 *eig_acc = nullptr;
    void *eig_out = nullptr;
    double eig_E = 0.0, tau = 0.0, hbar = 1.0, dv = 1.0;
};

// One problem of a batch (device memory).  A grouped launch covers every
// problem of one grid shape: the problem of a work-group is
// probs[ids[slice]], slice = blockIdx.y (row passes), blockIdx.z (column
// passes) or blockIdx.x (1-D whole runs).
template <typename R> struct BatchProb {
    int ndim, nx, ny;                  // 1-D: nx points; 2-D: nx x ny
    cx<R> *psi;                        // state (caller's buffer)
    cx<R> *gadj;                       // adjoint state (reverse sweep) or null
    const double *ebar;                // per-step field integrals, ndim per step, or null
    const double2 *kin_x, *kin_y;      // per-axis kinetic factors (1/N_tot in kin_x)
    const double2 *one;                // {1, 0}
    double xmin[3], dx[3], xabs[3];    // box; xabs = max |x| per axis
    double aV_half, inv_2hbar, v0max;  // tau/(2 hbar), 1/(2 hbar), max |V0|
    typename std::conditional<sizeof(R) == 4, const float, const double>::type *V0;
    double *dV;                        // dL/dV0 (N points) or null
    double *dE;                        // dL/dEbar (nsteps x ndim) or null
    double *part;                      // moment partials: (nsteps + 1) boundaries x gslots x 3
    int gslots;                        // partial slots per boundary (row work-groups; 1 for 1-D)
};

// Per-launch part of a grouped pass (probs == null: an ordinary launch).
template <typename R> struct GroupArgs {
    const BatchProb<R> *probs;
    const int *ids;
    int64_t sa, sb;   // row passes: half steps of the potential factor (-1: absent)
    int64_t jmom;     // reverse sweep: step boundary of the gradient partials
    double wmul;      // its weight (1 at the ends, 2 inside)
    int acc_init;     // first boundary of the sweep: overwrite dL/dV0
};

// Tile shapes the planner chooses from (index = variant number).  Row
// passes: register radix, threads per work-group (rows = threads / (N/radix)),
// minimum waves per SIMD the register allocation must allow.  Column
// passes: register radix, adjacent lines per work-group, waves per SIMD.
struct RowVariant {
    int rad, threads, wpe;
    bool pad;   // padded LDS map with immediate offsets (else the XOR swizzle)
    bool late;  // potential loaded after the inverse transform (fewer registers held)
    bool pre = false;  // complex128: stage factors formed from each stage's W^k, read with the line
};
struct ColVariant {
    int rad, cols, wpe;
    int pipe = 0;        // > 0: a forward step's k-space pass walks this many column groups per work-group,
                         // the next group's loads in flight while the current one transforms (k_colpipe)
    int order = 0;       // k_colpipe: where the kinetic factors and the prefetch are issued (0: both at the group
                         // start, 1: both after the forward transform, 2: in parts between the stages of the
                         // forward (factors) and inverse (prefetch) transforms)
    bool pre = false;    // stage factors formed from each stage's W^k, read once per work-group (no table per stage)
};
constexpr RowVariant kRowVariants[] = {
    {16, 256, 1, true, false}, {16, 128, 1, true, false}, {16, 512, 1, true, false}, {16, 256, 3, true, false},
    {16, 256, 4, true, false}, {8, 256, 1, false, false},  {8, 512, 1, false, false},  {8, 256, 4, false, false},
    {8, 256, 1, true, false},  {8, 512, 1, true, false},  {16, 256, 4, true, true},  {16, 128, 4, true, true},
    {16, 256, 1, true, true},  {8, 256, 1, false, true},
    // complex128 with the stage factors formed from W^k (for complex64 these equal shapes 0, 11, 12 and 13)
    {16, 256, 1, true, false, true}, {16, 128, 4, true, true, true}, {16, 256, 1, true, true, true},
    {8, 256, 1, false, true, true},
    // radix 16 through the XOR-swizzled LDS map (an address per element; other bank pattern)
    {16, 128, 4, false, true, true}, {16, 256, 1, false, true, true}};
constexpr ColVariant kColVariants[] = {
    {16, 8, 1}, {16, 4, 1}, {16, 2, 1}, {16, 16, 1}, {16, 4, 2}, {16, 2, 4}, {8, 8, 1}, {8, 4, 1}, {8, 2, 4},
    // pipelined k-space pass: 2, 4 or 8 column groups per work-group, prefetch at the group start (order 0)
    // or after the forward transform (order 1)
    {16, 4, 2, 2, 0}, {16, 4, 2, 2, 1}, {16, 4, 2, 4, 0}, {16, 4, 2, 4, 1},
    {16, 2, 2, 4, 0}, {16, 2, 2, 4, 1}, {16, 2, 2, 8, 0}, {16, 2, 2, 8, 1},
    // plain shapes with the stage factors formed from W^k
    {16, 8, 1, 0, 0, true}, {16, 4, 1, 0, 0, true}, {16, 4, 2, 0, 0, true}, {16, 2, 1, 0, 0, true},
    {16, 2, 4, 0, 0, true},
    // pipelined, the kinetic factors and the prefetch issued in parts between the transforms' stages
    {16, 4, 2, 2, 2}};
constexpr int kNumRowVariants = sizeof(kRowVariants) / sizeof(kRowVariants[0]);
constexpr int kNumColVariants = sizeof(kColVariants) / sizeof(kColVariants[0]);

// tw[0], tw[1]: the stage twiddle tables of the line length for radix 8 and 16.
// grp / ngroup: a grouped launch over ngroup problems of the same shape
// (S, V0, the phase and gradient arguments then come from the descriptors).
// ev: null, or an event pair the dispatch timestamps at its start and end.
template <typename R>
hipError_t launch_xpass(int variant, int N, int ns, const StatePtrs<R> &S, int64_t nrows, int ny,
                        const void *V0, const void *const *tw, const PhaseArgs &ph, const GradArgs &ga,
                        int mode, hipStream_t st, const GroupArgs<R> &grp = GroupArgs<R>{}, int ngroup = 1,
                        const hipEvent_t *ev = nullptr);

template <typename R>
hipError_t launch_colpass(int variant, int N, int ns, const StatePtrs<R> &S, int64_t ncols, int64_t stride,
                          int nslab, int64_t slab_stride, const void *const *tw, const KinArgs &kin, int mode,
                          hipStream_t st, const GroupArgs<R> &grp = GroupArgs<R>{}, int ngroup = 1,
                          const hipEvent_t *ev = nullptr);

template <typename R>
hipError_t launch_1d_adjoint(int N, cx<R> *psi, cx<R> *gv, const void *V0, const void *tw, const Run1DArgs &a,
                             double wbase, double *acc, double *mom, hipStream_t st,
                             const GroupArgs<R> &grp = GroupArgs<R>{}, int ngroup = 1);

// dL/dEbar[s][a] = (M[s+1][a] + M[s][a]) * scale for s < nsteps, where
// M[j][a] = sum over the nslots partials part[(j nslots + i) 3 + a], summed in
// slot order (deterministic).
hipError_t launch_ebar_grad(const double *part, int nslots, int64_t nsteps, int ndim, double scale, double *out,
                            hipStream_t st);

// Velocity-gauge gradient from the k-space partials of the reverse sweep
// (4 per slot and step, see KinArgs): for step j < nsteps and axis a < ndim,
// dA[j ndim + a] = sA * sum_slots part[(j nslots + slot) 4 + idx(a)] with
// idx = {2} (1-D), {0, 2} (2-D), {0, 1, 2} (3-D), and
// dA2[j] = sA2 * sum_slots part[(j nslots + slot) 4 + 3]; slot order.
hipError_t launch_vgrad_sum(const double *part, int nslots, int64_t nsteps, int ndim, double sA, double sA2,
                            double *dA, double *dA2, hipStream_t st);

// chi[2 j + {0, 1}] = scale * sum over the nslots partials of step j, in slot
// order (deterministic), j < nsteps.
hipError_t launch_chi_sum(const double *part, int nslots, int64_t nsteps, double scale, double *chi, hipStream_t st);

// out[2 e + {0, 1}] = sum_j dt chi_j (1 - cos(2 pi j / nsteps)) exp(i j dt E_e / hbar), e < nE.
hipError_t launch_spectrum(const double *chi, int64_t nsteps, double dt, double hbar, const double *E, int nE,
                           double *out, hipStream_t st);

// acc[i] += (cr + i ci) s[i] (FP64 accumulator); out[i] = acc[i] rounded to R.
template <typename R>
hipError_t launch_eig_axpy(const cx<R> *s, double2 *acc, int64_t n, double cr, double ci, hipStream_t st);
template <typename R> hipError_t launch_acc_to_state(const double2 *acc, cx<R> *out, int64_t n, hipStream_t st);

// Number of work-groups (= gradient partial slots) of a row pass launch.
template <typename R> int xpass_groups(int variant, int N, int64_t nrows);

// Host copy of the stage layout of LineShape<N, RAD>: (radix, span) per stage.
void line_stages(int N, int RAD, int *radix, int *span, int *nst);

// Whether a variant exists for this line length and precision (and, for
// columns, divides the number of lines).
template <typename R> bool xpass_variant_ok(int variant, int N);
// Scratch (spill) bytes per lane of the kernel a shape launches with ns
// states, -1 if the shape does not exist; the autotuner skips shapes > 0.
template <typename R> int xpass_scratch(int variant, int N, int ns);
template <typename R> int colpass_scratch(int variant, int N, int ns);
template <typename R> bool colpass_variant_ok(int variant, int N, int64_t ncols, int ns = 1);

template <typename R>
hipError_t launch_1d(int N, cx<R> *psi, int nprob, int64_t prob_stride, const void *V0,
                     const void *tw, const Run1DArgs &a, hipStream_t st, const GroupArgs<R> &grp = GroupArgs<R>{});

// One 1-D line's eigenstate run (a.chi: autocorrelation; a.eig_acc: windowed
// eigenfunction), dir = +1, no field table.
template <typename R>
hipError_t launch_1d_eigen(int N, cx<R> *psi, const void *V0, const void *tw, const Run1DArgs &a, hipStream_t st);

// 2-D Dirac pass tile shapes: radix, planes per work-group (4, or 2: one of
// the pairs (1,4), (2,3) that every factor maps to itself), for the column
// pass adjacent lines per work-group, for the row pass threads per
// work-group (whole rows).
struct DiracVariant {
    int rad, planes, cols;
    int threads = 256;
};
constexpr DiracVariant kDiracRowVariants[] = {{8, 4, 0},       {16, 2, 0},      {8, 2, 0},
                                             {16, 2, 0, 128}, {8, 2, 0, 128},  {16, 2, 0, 64}};
constexpr DiracVariant kDiracColVariants[] = {{8, 4, 4}, {8, 4, 2}, {16, 2, 4}, {16, 2, 2}, {8, 2, 4}};
constexpr int kNumDiracRowVariants = sizeof(kDiracRowVariants) / sizeof(kDiracRowVariants[0]);
constexpr int kNumDiracColVariants = sizeof(kDiracColVariants) / sizeof(kDiracColVariants[0]);
template <typename R> bool dirac_row_variant_ok(int variant, int N, int64_t ny);
template <typename R> bool dirac_col_variant_ok(int variant, int N, int64_t nx);

// tw[0], tw[1]: the stage twiddle tables of the line length for radix 8 and 16.
template <typename R>
hipError_t launch_dirac_xpass(int variant, int N, cx<R> *psi, int ny, int64_t plane, const void *V0,
                              const void *const *tw, const DiracPhaseArgs &ph, int mode, hipStream_t st);

template <typename R>
hipError_t launch_dirac_colpass(int variant, int N, cx<R> *psi, int nx, int64_t plane, const void *const *tw,
                                const DiracKinArgs &kin, int mode, hipStream_t st);

// 1-D two-component Dirac run (one work-group per line; alpha_1 = sigma_x,
// beta = sigma_z).  Per k, u[3 k + {0, 1, 2}] = U00, U01 (= U10), U11 of
// exp(-i tau H(p) / hbar) / N.  Real space, half step of step s:
// exp(-i aV_half V0) (cos a + i sin a sigma_x), a = aA * abar[s N + x]
// (aA = q c / (2 hbar); abar null: a = 0); consecutive halves merge.
struct Dirac1DArgs {
    const double2 *u;
    const double *abar;
    int64_t step0, nsteps;
    double aV_half, aA;
};
template <typename R>
hipError_t launch_dirac1d(int N, cx<R> *psi, const void *V0, const void *const *tw, const Dirac1DArgs &a,
                          hipStream_t st);

// FP64 reductions over n complex values: sum |a|^2 -> out[0]; or sum conj(a) b -> out[0..1].
template <typename R>
hipError_t launch_norm(const cx<R> *a, int64_t n, double *partials, double *out, hipStream_t st);
template <typename R>
hipError_t launch_overlap(const cx<R> *a, const cx<R> *b, int64_t n, double *partials, double *out,
                          hipStream_t st);

hipError_t launch_convert_v0(const double *src, void *dst, bool to_fp64, int64_t n, hipStream_t st);

// max |src| over n values into *out (device), for the potential-phase bound.
hipError_t launch_absmax(const double *src, int64_t n, double *partials, double *out, hipStream_t st);

constexpr int kReduceBlocks = 1024;

}  // namespace sfo
