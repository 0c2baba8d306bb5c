/*
 * sfo.h - C ABI of the Fourier split-operator library for AMD MI355X (gfx950).
 *
 * The library propagates a wave function by the split-operator method of
 * Bauke & Keitel, "Accelerating the Fourier split operator method via
 * graphics processing units":  each step is the Strang factorisation
 *
 *     w(t+tau) = U_A1(1/2) F^-1 { U~_A2(1) F { U_A1(1/2) w(t) } }
 *
 * (Sec. 2.1, eqs. U_split and step_t_to_t+dt_F), with
 *   - Schroedinger (Sec. 2.2, dipole approximation in the length gauge):
 *     U_A1(1/2) = exp(-i [tau V0(x) + x.Ebar_n] / (2 hbar)),
 *     U~_A2(1)  = exp(-i hbar tau |k|^2 / (2 m));
 *   - Dirac, d = 2, 4-spinor in the Dirac representation (Sec. 2.3):
 *     U_A1(1/2) = exp(-i tau V0/(2 hbar)) [cos a + i sin a alpha_2],
 *                 a = q c Abar_y(x)/(2 hbar)              (eq. exp_alpha),
 *     U~_A2(1)  = cos(E tau/hbar) - i sin(E tau/hbar) H(hbar k)/E,
 *                 H = c alpha.p + m c^2 beta, E = sqrt(m^2c^4 + c^2 p^2)
 *                 (eq. U_A_2_DE, closed form of its diagonalisation);
 *   - Dirac, d = 1, 2-spinor (alpha_1 = sigma_x, beta = sigma_z): the same
 *     with alpha_1 and a = q c Abar_1(x)/(2 hbar), Abar_1 the step integral
 *     of the line's vector potential A_1(x, t).
 * Ebar_n = Int_{t_n}^{t_n+tau} E(t') dt' and Abar_n = Int A_y dt' are step
 * integrals supplied by the caller; both half steps of step n use the same
 * integral (eq. U_split).  The DFT is unnormalised forward,
 * exp(-2 pi i j m/N), with 1/N on the inverse; k_m = 2 pi m / L for
 * m in [-N/2, N/2) in FFT order (the Nyquist mode is negative).
 *
 * Conventions shared by every entry point
 *   - Units are the caller's; atomic units give hbar = m = 1, q = -1.
 *   - A state is a contiguous device array, layout [comp][z][y][x] with x
 *     fastest (n[0] is the x size), complex64 (interleaved float re, im)
 *     or complex128 (interleaved double re, im) per desc.dtype; comp = 4
 *     for 2-D Dirac, 2 for 1-D Dirac, 1 otherwise.  The caller owns every state buffer.
 *   - x_j = xmin + j dx, dx = (xmax - xmin)/n: the box is periodic and the
 *     right end is excluded.
 *   - All work is enqueued on the stream given at creation and is
 *     asynchronous, except sfo_norm and sfo_overlap, which return values
 *     to the host and therefore synchronise that stream.
 *   - Every function returns an sfo_status; on failure nothing has been
 *     enqueued and sfo_last_error() describes the reason.  No exception
 *     crosses the ABI.  A grid handle is not thread-safe.
 */
#ifndef SFO_H
#define SFO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfo_grid_s *sfo_grid;
typedef struct sfo_batch_s *sfo_batch;

typedef enum {
    SFO_OK = 0,
    SFO_E_INVALID = -1,     /* bad argument: null pointer, size, index, table too short */
    SFO_E_UNSUPPORTED = -2, /* valid request the library does not implement */
    SFO_E_NOMEM = -3,       /* device allocation failed */
    SFO_E_HIP = -4,         /* HIP runtime error (no device, launch failure) */
    SFO_E_STATE = -5,       /* call out of order (e.g. no potential set) */
    SFO_E_NUMERIC = -6      /* sfo_norm / sfo_overlap: a non-finite value in a state, or the
                               norm left the band set by sfo_set_norm_watch */
} sfo_status;

enum { SFO_SCHRODINGER = 0, SFO_DIRAC = 1 };
enum { SFO_C64 = 0, SFO_C128 = 1 };

/* flags */
enum {
    SFO_UNFUSED = 1u << 1  /* run the paper's five-launch step (phase kernel, FFT, kinetic
                              kernel, inverse FFT, phase kernel) instead of the fused passes;
                              a reference configuration of the same kernels */
};

typedef struct {
    int32_t ndim;      /* 1, 2 or 3 (Dirac: 1 or 2) */
    int64_t n[3];      /* points per axis, x first; powers of two, 1-D 64..8192, 2-D/3-D 64..4096,
                          at most 2^35 bytes (32 GiB) per state component */
    double xmin[3];    /* box per axis, x first */
    double xmax[3];
    int32_t equation;  /* SFO_SCHRODINGER or SFO_DIRAC */
    int32_t dtype;     /* SFO_C64 or SFO_C128 */
    double dt;         /* tau */
    double mass;       /* m (a.u.: 1) */
    double charge;     /* q (a.u. electron: -1); used by the Dirac vector-potential factor */
    double c;          /* speed of light (a.u.: 137.036); Dirac only */
    double hbar;       /* (a.u.: 1) */
    uint32_t flags;
} sfo_grid_desc;

/* Create a grid handle: validates desc, allocates the library's device
 * tables (twiddles, kinetic factors, V0 storage, reduction scratch) on the
 * current HIP device, and binds the handle to `hip_stream` (a hipStream_t,
 * NULL = default stream).  V0 starts at zero and the field tables empty.
 * Errors: SFO_E_INVALID (desc), SFO_E_UNSUPPORTED (size or equation/ndim
 * combination), SFO_E_HIP (no device), SFO_E_NOMEM. */
sfo_status sfo_create_grid(const sfo_grid_desc *desc, void *hip_stream, sfo_grid *out);

/* Release every library-owned buffer of the handle (waits for its stream). */
sfo_status sfo_destroy_grid(sfo_grid g);

/* Copy the static potential energy V0(x) (FP64, N_points values, device
 * pointer, layout [z][y][x]) into the handle, which keeps it in FP32 for
 * complex64 states and in FP64 for complex128 states (the phase argument is
 * always formed in FP64).  Synchronises the stream (it also records max|V0|,
 * which selects the shorter sin/cos series when every potential phase of a
 * step is below 1/8 rad).  Errors: SFO_E_INVALID for a non-finite value,
 * checked before anything is copied (the previous potential stays). */
sfo_status sfo_set_potential(sfo_grid g, const double *V0_dev);

/* Copy the per-step field integrals Ebar[step][axis] (host, FP64,
 * nsteps x ndim, axis x first) into a device table indexed by absolute step
 * number.  Steps beyond the table are an error at propagation time; with no
 * table the field is zero.  Also releases velocity-gauge tables
 * (sfo_set_vector_field).  Schroedinger only.  At most 2^28 steps
 * (SFO_E_UNSUPPORTED beyond).  Errors leave the previous table in place:
 * SFO_E_INVALID for a non-finite value, SFO_E_NOMEM when the host or device
 * copy cannot be allocated.  Synchronises the stream before the old table is
 * released. */
sfo_status sfo_set_field(sfo_grid g, const double *ebar_host, int64_t nsteps);

/* Velocity gauge of the dipole approximation (the split's momentum-space
 * operator, eq. SE_K: exp(-(i/hbar) int (p - q A(t'))^2 / (2m) dt') per step,
 * the potential half steps with tau V0 only).  abar_host: nsteps x ndim
 * step integrals int A_a dt' (x first); a2bar_host: nsteps step integrals of
 * |A|^2; FP64 host arrays, copied: the library builds per-step, per-axis
 * kinetic tables (nsteps x (n[0] + n[1] + n[2]) complex FP64 on the device,
 * at most 1 GiB and 2^28 steps: SFO_E_UNSUPPORTED beyond).  Replaces a
 * length-gauge field table; sfo_set_field (any nsteps) in turn releases these
 * tables.  nsteps = 0 clears.  Arguments are checked (SFO_E_INVALID for a
 * non-finite value) before anything changes; a failed allocation
 * (SFO_E_NOMEM) leaves the grid with no field at all.  Schroedinger grids of any dimension (on a 1-D
 * grid the whole-run kernel reads step st's row of the table);
 * sfo_step / sfo_propagate use it and sfo_adjoint_velocity differentiates
 * it; sfo_adjoint, sfo_autocorrelation and batches refuse a grid that has it
 * (SFO_E_UNSUPPORTED). */
sfo_status sfo_set_vector_field(sfo_grid g, const double *abar_host, const double *a2bar_host, int64_t nsteps);

/* Copy the per-step vector-potential integrals Abar_y[step][ix] (host,
 * FP64, nsteps x n[0]) of a field A = A_y(x, t) y_hat (2-D; in 1-D the
 * line's own component A_1(x, t)).  Dirac only.  At most 1 GiB of table
 * (SFO_E_UNSUPPORTED beyond).  Errors leave the previous table in place:
 * SFO_E_INVALID for a non-finite value, SFO_E_NOMEM when a copy cannot be
 * allocated.  Synchronises the stream before the old table is released. */
sfo_status sfo_set_vector_potential(sfo_grid g, const double *abar_y_host, int64_t nsteps);

/* One un-merged Strang step number `step_index` applied in place to psi. */
sfo_status sfo_step(sfo_grid g, void *psi_dev, int64_t step_index);

/* Steps step0 .. step0+nsteps-1 in place.  Consecutive half steps of the
 * potential are merged into one factor (exact up to rounding); the result
 * equals nsteps calls of sfo_step to rounding. */
sfo_status sfo_propagate(sfo_grid g, void *psi_dev, int64_t step0, int64_t nsteps);

/* Autocorrelation run of the eigenstate method (the paper's eigenstate
 * section, first equation): advances psi in place by nsteps steps of the
 * time-independent potential and writes chi_j = dV sum_x conj(psi_0(x))
 * psi_j(x), j = 0..nsteps-1 (psi_0 the state on entry, psi_j after j steps)
 * to chi_dev as FP64 (re, im) pairs: 2 * nsteps doubles of device memory the
 * caller owns (may be NULL when nsteps is 0).  chi_j is formed inside the k-space pass of step j from its
 * state right after the forward transform and the stored transform of the
 * entry state (Parseval; exact because every step's first half factor is
 * the same unitary diagonal), summed in FP64 in a fixed order; on a 1-D grid
 * the whole run is one work-group that forms chi_j from its registers at
 * the start of each step.  Schroedinger grids (SFO_E_UNSUPPORTED otherwise)
 * with no field table set (SFO_E_UNSUPPORTED: clear it with
 * sfo_set_field(g, NULL, 0)).  The library keeps a state-sized reference
 * buffer on the handle.  Asynchronous. */
sfo_status sfo_autocorrelation(sfo_grid g, void *psi_dev, int64_t nsteps, double *chi_dev);

/* Windowed eigenfunction of the eigenstate method (the eigenstate section,
 * third equation) as the rectangle rule over t_j = j dt, T = nsteps dt:
 * advances psi in place by nsteps steps of the time-independent potential
 * and writes out = sum_j dt (1 - cos(2 pi j / nsteps)) exp(i E j dt / hbar)
 * psi_j, j < nsteps (unnormalised; psi_j the state after j steps), in the
 * state's dtype and layout.  The sum is accumulated in FP64 between the
 * passes of each step (a state-sized complex128 buffer the library keeps on
 * the handle) and brought to real space once at the end (1-D: each point
 * accumulated by the thread that owns it in the whole-run kernel).
 * Schroedinger grids with no field table set (SFO_E_UNSUPPORTED otherwise);
 * psi and out distinct device buffers the caller owns.  Asynchronous. */
sfo_status sfo_eigenfunction(sfo_grid g, void *psi_dev, int64_t nsteps, double energy, void *out_dev);

/* Windowed Fourier transform of an autocorrelation (the eigenstate section,
 * second equation) as the rectangle rule over t_j = j dt, T = nsteps dt:
 * out[2e], out[2e+1] = re, im of sum_j dt chi_j (1 - cos(2 pi j / nsteps))
 * exp(i j dt E_e / hbar), e < nE, with dt and hbar of the grid.  chi_dev:
 * 2 * nsteps doubles, energies_dev: nE doubles, out_dev: 2 * nE doubles, all
 * device memory the caller owns; FP64.  Peaks of |out| mark eigenenergies.
 * nE = 0 does nothing; more than 2^30 energies: SFO_E_UNSUPPORTED.
 * Asynchronous on the grid's stream. */
sfo_status sfo_spectrum(sfo_grid g, const double *chi_dev, int64_t nsteps, const double *energies_dev, int32_t nE,
                        double *out_dev);

/* Reverse-mode gradient through sfo_propagate(g, psi0, step0, nsteps)
 * (Schroedinger only).  On entry psi holds psi(T) = the forward result and
 * g_vec holds 2 dL/dconj(psi(T)) (the complex-autograd convention) for a
 * real loss L.  The states are walked back with the exact inverse step (no
 * stored trajectory); on return psi holds the recomputed psi(0) and g_vec
 * holds 2 dL/dconj(psi(0)).  dL_debar_dev (device, FP64, nsteps x ndim,
 * row s for step step0+s) receives dL/dEbar; dL_dV0_dev (device, FP64,
 * N_points, may be NULL) receives dL/dV0.  Both are overwritten. */
sfo_status sfo_adjoint(sfo_grid g, void *psi_dev, void *g_dev, int64_t step0, int64_t nsteps,
                       double *dL_debar_dev, double *dL_dV0_dev);

/* Reverse-mode gradient through a velocity-gauge run (Schroedinger grids
 * with a table set by sfo_set_vector_field; Sec. 2.2, eq. SE_K: step n's
 * kinetic factor exp(-i/(2 m hbar) [tau p^2 - 2 q p.Abar_n + q^2 A2bar_n])).
 * psi and g_vec as for sfo_adjoint (psi(T) and 2 dL/dconj(psi(T)) in,
 * recomputed psi(0) and 2 dL/dconj(psi(0)) out).  Outputs, device FP64, each
 * may be NULL, overwritten: dL_dabar_dev (nsteps x ndim, row s for step
 * step0+s) = dL/dAbar_{s,a}; dL_da2bar_dev (nsteps) = dL/dA2bar_s; dL_dV0_dev
 * (N points) = dL/dV0.  The gradient with respect to the step integrals is
 * formed in momentum space inside the reverse sweep's k-space pass: with
 * psi~ and g~ the transforms of P^-1 psi_{s+1} and P^-1 g_{s+1} there,
 * dL/dAbar_{s,a} = -(q / (m N)) sum_k k_a Im(conj(g~) psi~) and
 * dL/dA2bar_s = (q^2 / (2 m hbar N)) sum_k Im(conj(g~) psi~), summed in FP64
 * per work-group and then in a fixed order.  SFO_E_STATE without a
 * vector-field table; sfo_adjoint refuses such a grid.  Asynchronous. */
sfo_status sfo_adjoint_velocity(sfo_grid g, void *psi_dev, void *g_dev, int64_t step0, int64_t nsteps,
                                double *dL_dabar_dev, double *dL_da2bar_dev, double *dL_dV0_dev);

/* sfo_adjoint without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * sfo_adjoint (bit for bit); the reverse sweep's moment partials live in a
 * static 16 MiB scratch array that each device holds until the process ends
 * (looked up once per device by sfo_create_grid) instead of a buffer the
 * handle allocates.  The run must fit it: 3 x (row work-groups of the
 * two-state row pass, 1 for 1-D) x (nsteps + 1) doubles at most 2^21 (a
 * 2048^2 grid with 1024 row work-groups fits 681 steps), else
 * SFO_E_UNSUPPORTED before anything is enqueued.  Every call on one device
 * shares that array: calls that overlap on one GPU (other streams, other
 * threads, other handles) race and give wrong gradients.  Kernel timing
 * (sfo_profile_enable) does not cover this call.  SFO_E_HIP if the array
 * has no device address on the grid's device.  Asynchronous. */
sfo_status sfo_adjoint_noalloc(sfo_grid g, void *psi_dev, void *g_dev, int64_t step0, int64_t nsteps,
                               double *dL_debar_dev, double *dL_dV0_dev);

/* ||psi||^2 = dV sum |psi|^2 over all points and components, accumulated in
 * FP64; written to *out_host (also when the status is SFO_E_NUMERIC).
 * SFO_E_NUMERIC: the state holds a NaN or Inf (the sum is then not finite),
 * or a norm watch is set and |norm / reference - 1| exceeds its tolerance.  Every factor of the step (Sec. 2.1, eq.
 * U_split) is unitary, so this is the quantity a run conserves; the
 * rectangle rule over the periodic grid is the discrete form of the L2 norm
 * of the wave function.  Synchronises the stream. */
sfo_status sfo_norm(sfo_grid g, const void *psi_dev, double *out_host);

/* Norm watch of the handle (failure detection): from now on sfo_norm
 * returns SFO_E_NUMERIC when |norm / reference - 1| > tolerance.  The step is
 * unitary (Sec. 2.1), so the norm of a propagated state may only drift by
 * rounding; a drift beyond what the precision allows (about 1e-6 over a
 * complex64 run, 1e-12 for complex128) signals a broken run.  reference = 0
 * switches the watch off.  SFO_E_INVALID for a negative or non-finite value. */
sfo_status sfo_set_norm_watch(sfo_grid g, double reference, double tolerance);

/* <a|b> = dV sum conj(a) b in FP64; out_host[0] = real, out_host[1] = imaginary
 * (SFO_E_NUMERIC, with the values written, when either is not finite).
 * With a = the state at t = 0 and b = the state at t this is the
 * autocorrelation chi(t) of the eigenstate method (Sec. 5.2, first equation),
 * rectangle rule over the grid; sfo_autocorrelation forms the same sum for
 * every step of a run inside the momentum-space pass.  Synchronises the
 * stream. */
sfo_status sfo_overlap(sfo_grid g, const void *a_dev, const void *b_dev, double *out_host);

/* Unnormalised n-dimensional DFT of every component of psi in place,
 * exp(sign 2 pi i j m / N) along each axis, sign = -1 or +1: the transforms F
 * (sign -1) and N F^-1 (sign +1) of eq. step_t_to_t+dt_F (Sec. 2.1), which
 * the paper's GPU code takes from a vendor FFT library (Sec. 3.3) and which
 * the passes here carry out with their own transforms.  Exposed for
 * diagnostics; the step itself never calls it. */
sfo_status sfo_fft(sfo_grid g, void *psi_dev, int32_t sign);

/* Batched runs (Schroedinger, 1-D and 2-D).  The step of Sec. 2.1 (eq.
 * step_t_to_t+dt_F) and the reverse sweep of sfo_adjoint for many problems
 * at once; the paper propagates one wave function per run (Sec. 4.2), so
 * the batching itself is this library's.  Many independent problems of
 * uneven size, each described by its own grid handle (its own box, time
 * step, potential, field table and tile shapes), advance together: problems
 * of one shape form a group, and each pass of the split step (Sec. 2.1, eq.
 * step_t_to_t+dt_F) is launched once per group with the problem as a grid
 * dimension, the 1-D whole runs on a parallel branch.  The launch sequence is
 * captured once per (direction, step0, nsteps) in a HIP graph and replayed.
 * The per-problem result equals sfo_propagate / sfo_adjoint on that grid
 * to rounding (bit for bit when the grids of a shape share tile shapes).
 *
 * sfo_create_batch: `grids` (count >= 1, not owned, must outlive the batch)
 * all of one dtype, Schroedinger, 1-D or 2-D (SFO_E_UNSUPPORTED otherwise).
 * The batch launches on `hip_stream` (NULL = default stream), not on the
 * grids' streams.  States are the caller's: psi_devs[i] (and g_devs[i]) are
 * device pointers laid out as for grid i.  While a batched call is in
 * flight, nothing else may touch these states or grids.
 *
 * sfo_propagate_batch: steps step0 .. step0+nsteps-1 of every problem.
 * sfo_adjoint_batch: the reverse sweep of sfo_adjoint for every problem;
 * dL_debar_devs[i] (nsteps x ndim) and dL_dV0_devs[i] (N points) are device
 * pointers or NULL, and either array itself may be NULL.
 * Both calls are asynchronous.  A changed list of state pointers (or a
 * changed grid table) makes the call wait for the batch's earlier launches
 * before it uploads the new problem descriptors.
 *
 * sfo_batch_set_graph: on = 0 launches the kernels directly instead of
 * replaying graphs.
 * sfo_batch_check: waits for the batch's stream; SFO_E_HIP if a launch
 * failed.
 * sfo_batch_autotune: chooses the tile shapes of the grouped launches (a
 * group's launch covers all its problems, so the shapes that suit one grid
 * need not suit the group) by timing `reps` steps of each 2-D group's
 * sequence, forward and in the reverse sweep, in every row shape, then
 * every column shape, on scratch states it allocates and frees (it may grow
 * the batch's partial-slot buffer); the member grids' own plans are
 * unchanged, and results differ from those of the member grids' shapes by
 * rounding only.  Synchronises the stream; reps in 1..10000, else
 * SFO_E_INVALID. */
sfo_status sfo_create_batch(const sfo_grid *grids, int32_t count, void *hip_stream, sfo_batch *out);
sfo_status sfo_destroy_batch(sfo_batch b);
sfo_status sfo_propagate_batch(sfo_batch b, void *const *psi_devs, int64_t step0, int64_t nsteps);
sfo_status sfo_adjoint_batch(sfo_batch b, void *const *psi_devs, void *const *g_devs, int64_t step0, int64_t nsteps,
                             double *const *dL_debar_devs, double *const *dL_dV0_devs);
sfo_status sfo_batch_set_graph(sfo_batch b, int32_t on);
sfo_status sfo_batch_autotune(sfo_batch b, int32_t reps);
sfo_status sfo_batch_check(sfo_batch b);

/* Tile-shape planning.  The line passes carry the transforms F and F^-1
 * of eq. step_t_to_t+dt_F (Sec. 2.1); the paper leaves their schedule to its
 * vendor FFT library (Sec. 3.3), here it is chosen by measurement.  Each
 * line pass exists in several shapes (lines per work-group, register radix,
 * occupancy hint).  sfo_autotune times every
 * shape of every pass of this grid on a scratch state the call allocates and
 * frees (2-D and 3-D Schroedinger: `reps` whole steps of the propagation's
 * pass sequence, x shapes first with the current others, then each further
 * axis; the reverse sweep's two-state passes likewise; otherwise `reps`
 * launches of each pass), keeps the fastest, and remembers the choice for later
 * grids of the same shape, precision and equation in this process and, if
 * the environment variable SFO_TUNE_CACHE names a file, in that file.
 * Synchronises the stream.  sfo_get_plan / sfo_set_plan read and force the
 * three shape numbers (x pass, y pass, z pass); setting a shape that does not
 * exist for the grid is SFO_E_INVALID. */
sfo_status sfo_autotune(sfo_grid g, int32_t reps);
sfo_status sfo_get_plan(sfo_grid g, int32_t *plan3);
sfo_status sfo_set_plan(sfo_grid g, const int32_t *plan3);

/* Kernel timing (diagnostics): the per-task times of the paper's
 * performance section (Sec. 4.2: transforms with the position-space factor,
 * transforms with the momentum-space factor).  While enabled, every pass the handle launches
 * is bracketed by a pair of HIP events recorded on the handle's stream;
 * enabling clears what was collected.  sfo_profile_read synchronises the
 * stream and returns, for one kernel kind, the number of launches and their
 * summed duration in milliseconds. */
enum {
    SFO_KERNEL_ROW = 0,    /* contiguous x-axis pass (transform, potential factor) */
    SFO_KERNEL_COLUMN = 1, /* strided y-axis pass (2-D: transform, kinetic factor) */
    SFO_KERNEL_ZCOLUMN = 2,/* strided z-axis pass (3-D: transform, kinetic factor) */
    SFO_KERNEL_LINE1D = 3, /* whole-run 1-D kernel */
    SFO_KERNEL_KINDS = 4
};
sfo_status sfo_profile_enable(sfo_grid g, int32_t on);
sfo_status sfo_profile_read(sfo_grid g, int32_t kind, int64_t *count, double *total_ms);

/* Average duration in milliseconds of one launch of the grid's current
 * shape of a pass (SFO_KERNEL_ROW: inverse x-transform, potential factor,
 * forward x-transform; SFO_KERNEL_COLUMN / ZCOLUMN: transform, kinetic
 * factor, inverse transform), on a scratch state (allocated and freed by the
 * call).  By default from `reps` back-to-back launches of that pass between
 * two HIP events on the grid's stream: each launch then reads what the
 * previous launch of the same pass wrote, partly from cache.  With
 * SFO_TIME_IN_STEP or'ed into kind: `reps` (at most 4096) steps of the pass
 * sequence a propagation runs (row pass, then the other axes), each launch
 * of the pass timestamped by its own dispatch (hipExtLaunchKernelGGL start
 * and stop events; a timestamped dispatch ends with a wider release, which
 * adds about a microsecond to its own duration); for SFO_KERNEL_COLUMN in
 * 3-D, the y-forward pass.
 * Unlike sfo_profile_read, no event packet sits between launches.  2-D and
 * 3-D Schroedinger grids; synchronises the stream. */
enum { SFO_TIME_IN_STEP = 16 };
sfo_status sfo_time_pass(sfo_grid g, int32_t kind, int32_t reps, double *avg_ms);

/* Description of the last failure on the calling thread ("" if none). */
const char *sfo_last_error(void);

/* Library version string. */
const char *sfo_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SFO_H */
