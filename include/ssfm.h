/*
 * ssfm.h -- C ABI of the MI355X split-step (phase-screen) NLSE march.
 *
 * The library integrates the stationary (2D+1) nonlinear Schroedinger
 * equation of Bulygin & Geints (arXiv 2306.15678; Math and Equations,
 * Eq. (1), (3), (9)) by the split-step method: every z step applies the
 * paraxial diffraction operator exactly in Fourier space,
 *   V = F^-1[ exp(-i (kx^2 + ky^2) dz / 2k0) F U ],
 * and then a pointwise nonlinear screen U' = V A(I) exp(i Phi(I)) built from
 * the Kerr term (Eq. (1)), saturating plasma refraction and multiphoton
 * absorption (Eq. (3)), an 8-parameter ansatz f_theta(I) standing in for the
 * effective lens (Eq. (6), (9)), and optional random turbulence phase
 * screens (Eq. (9) eps_t, Eq. (10)).  Conventions: dU/dz = (i/2k0) Lap U +
 * i k0 dn U - alpha/2 U (the complex conjugate of the paper's e^{i w t}
 * form; intensities are identical), cell-centred periodic grid, Lie
 * splitting with diffraction first.
 *
 * Units at this boundary are SI: lengths in m, fields in sqrt(W/m^2),
 * intensities in W/m^2.  Fields cross the boundary as interleaved complex128
 * (re, im doubles), row-major [y][x] with x contiguous, n*n elements.
 *
 * Ownership: the caller allocates every device buffer, including the
 * workspace sized by ssfm_workspace_bytes(); the library never calls
 * hipMalloc and never frees caller memory.  A context owns only host
 * objects (plans, captured graphs) and is released by ssfm_destroy().
 *
 * Streams: all device work is enqueued on the stream given to ssfm_create()
 * (a hipStream_t passed as void*; NULL is the default stream).  Functions
 * that return data to the host synchronise that stream; the others are
 * asynchronous.
 *
 * Errors: every function returns an ssfm_status; ssfm_last_error() gives a
 * thread-local detail string for the last failure.  No C++ exception crosses
 * this boundary.  A context is not thread-safe; distinct contexts are
 * independent.
 */
#ifndef SSFM_H
#define SSFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSFM_VERSION 10000 /* major*10000 + minor*100 + patch */

typedef struct ssfm_ctx ssfm_ctx;

typedef enum {
  SSFM_OK = 0,
  SSFM_EINVAL = -1,       /* bad argument (null pointer, range, size)      */
  SSFM_EUNSUPPORTED = -2, /* grid size or option not built into the library */
  SSFM_EHIP = -3,         /* HIP runtime error (detail in ssfm_last_error) */
  SSFM_ESTATE = -4,       /* call out of order (e.g. backward before forward) */
  SSFM_ENONFINITE = -5,   /* non-finite power or theta gradient detected   */
  SSFM_EWORKSPACE = -6    /* workspace missing, misaligned or too small    */
} ssfm_status;

/* Screen terms (bit mask). */
enum {
  SSFM_KERR = 1,   /* phase k0 n2 I dz                               (Eq. 1) */
  SSFM_MPA = 2,    /* exact pointwise solution of dI/dz = -beta_K I^K (Eq. 3) */
  SSFM_PLASMA = 4, /* phase -k0 n2 I_a dz x^K/(1+x^(K-1)), x = I/I_a (Eq. 3) */
  SSFM_ANSATZ = 8, /* exp(i k0 n2 I_a dz f_theta(x))            (Eq. 6, 9) */
  SSFM_TURB = 16   /* Kolmogorov phase screens after scheduled steps (Eq. 9) */
};

/* Precision of the march. */
enum { SSFM_FP32 = 32, SSFM_FP64 = 64 };

/* Where a caller buffer lives. */
enum { SSFM_HOST = 0, SSFM_DEVICE = 1 };

/* One beam on one grid (Math and Equations; Eq. (7) gives the beams the
 * workloads start from).  Supported n: 128, 256, 512, 768, 1024, 2048, 4096. */
typedef struct {
  int32_t n;           /* grid points per side (square grid)                */
  int32_t mpa_order;   /* K >= 2 (multiphoton order; plasma exponent)        */
  uint32_t terms;      /* SSFM_KERR | SSFM_MPA | ...                         */
  int32_t n_screens;   /* turbulence screens, used when SSFM_TURB is set     */
  double length;       /* window side [m]                                    */
  double dz;           /* z step [m]                                         */
  double wavelength;   /* [m]; k0 = 2 pi / wavelength (air, n0 = 1)          */
  double n2;           /* Kerr index [m^2/W]                                 */
  double beta_k;       /* MPA coefficient [m^(2K-3) W^(1-K)]                 */
  double i_ref;        /* reference intensity I_a [W/m^2] (> 0)              */
  double cn2;          /* refractive structure constant [m^(-2/3)]           */
  double screen_dz;    /* spacing of turbulence screens [m]; screen s (1-based)
                          sits at (s - 1/2) screen_dz and is applied after the
                          step that reaches it                               */
  uint64_t seed;       /* Philox4x32-10 key of this beam's screens           */
} ssfm_instance_desc;

/* Version number (SSFM_VERSION of the built library). */
int ssfm_version(void);

/* Static description of a status code. */
const char* ssfm_strerror(int status);

/* Detail of the last failure on the calling thread ("" if none). */
const char* ssfm_last_error(void);

/* Device workspace a context needs.
 *   desc, n_inst : the instances (n_inst >= 1)
 *   precision    : SSFM_FP32 (complex64 march) or SSFM_FP64 (complex128)
 *   max_steps    : longest march that will be recorded for the adjoint
 *                  (0 if ssfm_forward_record() will not be used)
 *   ckpt_every   : M, steps per adjoint checkpoint segment (M >= 1; M >=
 *                  max_steps stores every step and needs no recompute)
 *   stored_segments : K >= 0, the last K segments of a recorded march are
 *                  kept whole (every pre-screen field) by the forward
 *                  itself, so the backward recomputes only the others; each
 *                  costs M - 1 fields of workspace
 * Writes the byte count to *bytes.  Pure host computation.  SSFM_EINVAL
 * for a bad argument, SSFM_EUNSUPPORTED for an unsupported grid size. */
int ssfm_workspace_bytes(const ssfm_instance_desc* desc, int32_t n_inst,
                         int32_t precision, int64_t max_steps,
                         int32_t ckpt_every, int32_t stored_segments,
                         size_t* bytes);

/* Checkpointing of a recorded march of n_steps that fits budget_bytes of
 * workspace (the memory side of the adjoint: the trajectory the backward
 * needs, Math and Equations, kept or recomputed).  Every pre-screen field
 * when that fits (M = n_steps, K = 0); else the (M, K) of
 * ssfm_workspace_bytes that fits and minimises the steps the backward
 * recomputes plus one per segment.  Writes M to *ckpt_every, K to
 * *stored_segments and, if recomputed is not NULL, the steps the backward
 * recomputes.  Pure host computation.  SSFM_EWORKSPACE if no layout fits. */
int ssfm_checkpoint_plan(const ssfm_instance_desc* desc, int32_t n_inst,
                         int32_t precision, int64_t n_steps,
                         size_t budget_bytes, int32_t* ckpt_every,
                         int32_t* stored_segments, int64_t* recomputed);

/* Create a context over a caller-owned device workspace of ws_bytes bytes
 * (256-byte aligned, at least ssfm_workspace_bytes() of the same
 * arguments).  Builds the propagator and twiddle tables (FP64 on the host,
 * rounded once) and the work lists; fields start at zero.  stream:
 * hipStream_t or NULL. */
int ssfm_create(const ssfm_instance_desc* desc, int32_t n_inst,
                int32_t precision, int64_t max_steps, int32_t ckpt_every,
                int32_t stored_segments, void* workspace, size_t ws_bytes,
                void* stream, ssfm_ctx** out);

/* Release the context's host objects (not the workspace).  Synchronises. */
int ssfm_destroy(ssfm_ctx* ctx);

/* Initial field of instance inst: the beam entering the medium (Math and
 * Equations: the problem starts from a given input field; Eq. (7) is the
 * paper's Gaussian beam, U = A exp(-(r/r_n)^2)).  src: n*n complex128
 * U [sqrt(W/m^2)] in host or device memory (where), row-major [y][x],
 * read before return (host) or on the stream (device); the caller keeps
 * ownership.  The instance's own step count, which places its turbulence
 * screens, restarts at 0; the other instances keep their fields (with any
 * pending screen applied) and their step counts.  Drops a recorded march
 * and its cotangents.  SSFM_EINVAL for inst out of range or src NULL. */
int ssfm_set_field(ssfm_ctx* ctx, int32_t inst, const void* src, int32_t where);

/* Ansatz parameters theta[8] of instance inst, the sparse-grid stand-in for
 * the effective screen f_lens[U, D] of Eq. (2) and its parameters D (Math
 * and Equations, Eq. (2), (6), (9)):
 * f_theta(x) = [sum_p theta_p x^p + i sum_p theta_{4+p} x^p] / (1 + x^4),
 * x = I / I_a, applied as exp(i k0 n2 I_a dz f_theta) every step.  theta:
 * host double[8], copied.  Drops a recorded march (its stored fields were
 * made with the old theta).  SSFM_EINVAL for a non-finite entry. */
int ssfm_set_theta(ssfm_ctx* ctx, int32_t inst, const double* theta);

/* Generate every instance's turbulence phase screens eps_t on the device
 * by the spectral method of Eq. (9)-(10) (Multiple filamentation regime in
 * turbulent air): Philox4x32-10 white noise per Fourier mode, shaped by the
 * Kolmogorov phase spectrum (r0 from cn2 and screen_dz) or the instance's
 * Eq. (10) step spectrum, inverse FFT; one draw gives two screens (its real
 * and imaginary parts).  Screens live in the workspace.  Drops a recorded
 * march (it used the previous screens). */
int ssfm_gen_screens(ssfm_ctx* ctx);

/* Splitting of each z step.  SSFM_LIE (default): diffraction L(dz), then
 * the screen.  SSFM_STRANG: L(dz/2), screen, L(dz/2), second order in dz
 * (a scheme variant; the paper does not state its splitting).  A Strang
 * context keeps V = L(dz/2) U between steps (one extra half step when a
 * field is set, one backward half step when it is read).  It marches,
 * reads out fields, intensities, per-step diagnostics and screens, and
 * records and differentiates: in V the step is V' = L(dz) S_n(V), the Lie
 * recurrence with each step's own screen acting on load, so the adjoint is
 * the Lie adjoint with that screen, preceded by the adjoint of the read-out
 * (the cotangent of U_N is taken to L(dz/2) of it) and followed by that of
 * the set-field half step (dL/dU_0 = L(-dz/2) dL/dV_0).  The effective
 * lens returns SSFM_EUNSUPPORTED.  Its per-step
 * power is exact; its per-step peak is that of L(dz/2) U.  Changing the
 * scheme zeroes every field: call it before ssfm_set_field. */
enum { SSFM_LIE = 0, SSFM_STRANG = 1, SSFM_FD = 2 };
int ssfm_set_splitting(ssfm_ctx* ctx, int32_t scheme);

/* SSFM_FD selects the finite-difference reference scheme instead of the
 * split-step march (the paper's dense reference solver for Eq. (3), a
 * semi-implicit conservative finite-difference scheme; the scheme is not
 * printed, the reading here is Crank-Nicolson with the nonlinearity at the
 * step's mean intensity):
 *   (U+ - U)/dz = (i/2k0) Lap_h Ubar + G(J) Ubar,  Ubar = (U+ + U)/2,
 *   J = (|U+|^2 + |U|^2)/2,
 *   G(I) = i k0 n2 [I - I_a x^K/(1 + x^(K-1))] - beta_K I^(K-1)/2, x = I/I_a,
 * G holding the beam's Kerr, plasma and multiphoton terms, Lap_h the
 * periodic 5-point Laplacian.  Each step solves
 * Ubar = (1 - (i dz/4k0) Lap_h)^-1 [U + (dz/2) G(J) Ubar] by a fixed number of
 * fixed-point iterations from Ubar = U (ssfm_set_fd_iterations, default 4;
 * the linear solve is exact, Lap_h being diagonal in the 2-D DFT basis),
 * then U+ = 2 Ubar - U.  Converged, a step conserves power exactly without
 * absorption.  The per-step power and peak are those of U+.  Returns
 * SSFM_EUNSUPPORTED when a beam has the ansatz term or turbulence screens;
 * forward only like Strang (the recorded march, its adjoint, the fluence
 * loss and the lens return SSFM_EUNSUPPORTED), while ssfm_fluence_mismatch
 * works on its fields.  Zeroes every field. */
int ssfm_set_fd_iterations(ssfm_ctx* ctx, int32_t iterations);  /* 1..64 */

/* Screen spectrum of instance inst for the next ssfm_gen_screens:
 * SSFM_SPECTRUM_KOLMOGOROV (default; Phi(f) = 0.023 r0^(-5/3) f^(-11/3) with
 * r0 from cn2 and screen_dz, Eq. (9)), or SSFM_SPECTRUM_STEP, Eq. (10) read
 * as a low-pass step: every Fourier mode with 0 < kappa <= kappa_h
 * [rad/m] gets amplitude sqrt(tau) (tau [rad^2] per mode), the others 0.
 * The mode of integer indices (mx, my) has kappa = 2 pi |m| / L, so the band
 * is decided on the integers: 0 < mx^2 + my^2 <= q2 with
 * q2 = (kappa_h L / 2 pi)^2 (1 + 2^-40), formed once in FP64 (the slack
 * keeps a ring that kappa_h was placed on, kappa_h = 2 pi M / L, inside). */
enum { SSFM_SPECTRUM_KOLMOGOROV = 0, SSFM_SPECTRUM_STEP = 1 };
int ssfm_set_screen_spectrum(ssfm_ctx* ctx, int32_t inst, int32_t kind, double tau,
                             double kappa_h);

/* Subharmonic levels of instance inst for the next ssfm_gen_screens (0, the
 * default, to 8).  An FFT screen carries no power below the window's
 * fundamental 1/L; with P levels the subharmonic method (Lane, Glindemann
 * and Dainty 1992; the paper's spectral screen method, Eq. (9)-(10), leaves
 * the low end to the implementation) adds, to every screen pair, the modes
 * f = (mx, my) / (3^p L) for p = 1..P and (mx, my) in {-1, 0, 1}^2 without
 * (0, 0), with amplitude sqrt(density(f)) / (3^p L) (density: the
 * Kolmogorov Phi, or tau L^2 inside mx^2 + my^2 <= 9^p q2 for the step
 * spectrum) and coefficient c = z0 + i z1 from Philox4x32-10 counter
 * (q, p, pair, 1), q = 3 (my + 1) + (mx + 1), key = seed; the sum over the
 * cell-centred grid, minus its grid mean, adds its real part to screen
 * 2 pair and its imaginary part to screen 2 pair + 1.  Kolmogorov beams with
 * cn2 = 0 get none.  SSFM_EINVAL outside [0, 8]. */
int ssfm_set_subharmonics(ssfm_ctx* ctx, int32_t inst, int32_t levels);

/* Copy screen s of instance inst [rad], float64 n*n, to host or device. */
int ssfm_get_screen(ssfm_ctx* ctx, int32_t inst, int32_t s, void* dst,
                    int32_t where);

/* March every instance n_steps further by the split-step method (Math and
 * Equations: Eq. (1) with the Eq. (3) terms, Eq. (9) in turbulent air):
 * per step, exact diffraction exp(-i (kx^2 + ky^2) dz / 2k0) in Fourier
 * space, then the pointwise screen of the instance's terms, then its
 * turbulence screen if one is scheduled.  Asynchronous on the context's
 * stream.  Per-step power and peak intensity are accumulated in FP64 for
 * ssfm_get_diag().  SSFM_EINVAL for n_steps < 0; 0 does nothing. */
int ssfm_propagate(ssfm_ctx* ctx, int64_t n_steps);

/* Current field U of instance inst (Eq. (1)): n*n complex128
 * [sqrt(W/m^2)], row-major [y][x], written to the caller's host or device
 * buffer dst.  Synchronises when dst is on the host. */
int ssfm_get_field(ssfm_ctx* ctx, int32_t inst, void* dst, int32_t where);

/* Current fluence w = U U* of instance inst (the stationary model's
 * fluence, Math and Equations before Eq. (4); EL benchmarking) [W/m^2]:
 * n*n float64 to the caller's host or device buffer dst.  Synchronises
 * when dst is on the host. */
int ssfm_get_intensity(ssfm_ctx* ctx, int32_t inst, void* dst, int32_t where);

/* The monitored beam quantities (Math and Equations: the drop of the pulse
 * energy and the maximum intensity along the path; EL benchmarking, Fig. 3
 * and 6): power sum |U|^2 dx^2 [W] and peak intensity [W/m^2] after each of
 * the last n steps of the most recent propagate/record call, reduced in
 * FP64 in a fixed order.  power, peak: host double[n] (either may be NULL).
 * Synchronises.  SSFM_EINVAL if n exceeds the steps kept; SSFM_ENONFINITE if
 * a power is not finite. */
int ssfm_get_diag(ssfm_ctx* ctx, int32_t inst, double* power, double* peak,
                  int64_t n);

/* The march of ssfm_propagate (Eq. (1), (3), (9)) over n_steps (<=
 * max_steps) from the current fields, keeping what its adjoint needs for
 * fitting the screen parameters to a discrepancy (Math and Equations: the
 * effective screen's parameters minimise the residual against the dense
 * solution): the field at the start of every segment of M steps and every
 * pre-screen field of the last K (stored_segments) segments; all of them
 * when M >= n_steps.  Drops earlier cotangents.
 * SSFM_EINVAL if n_steps exceeds max_steps or is < 1. */
int ssfm_forward_record(ssfm_ctx* ctx, int64_t n_steps);

/* Cotangent of the recorded march's final field for instance inst, for a
 * discrepancy L chosen by the caller (Math and Equations leaves the measure
 * to the problem): G = dL/dRe U_N + i dL/dIm U_N [1/sqrt(W/m^2)], n*n
 * complex128 from host or device.  SSFM_ESTATE without a recorded march. */
int ssfm_set_cotangent(ssfm_ctx* ctx, int32_t inst, const void* g, int32_t where);

/* The discrepancy between the sparse-grid fluence and a target (Math and
 * Equations: the residual between the true dense-grid solution and the
 * effective one; here the L2 fluence mismatch) for instance inst, target
 * w [W/m^2] n*n float64 on host or device (e.g. a dense fluence block-
 * averaged by ssfm_block_mean):
 *   L = sum (|U_N|^2 - w)^2 / sum w^2,
 * which also sets the cotangent of U_N for ssfm_backward.  Writes L to
 * *loss (may be NULL); synchronises.  SSFM_ESTATE without a recorded
 * march. */
int ssfm_fluence_loss(ssfm_ctx* ctx, int32_t inst, const void* target,
                      int32_t where, double* loss);

/* The same normalised fluence mismatch as ssfm_fluence_loss for the
 * current field of instance inst, after any march (propagate or record),
 * without seeding the adjoint or touching a recorded march's state: for
 * fitness evaluations (a population of beams in one context); under
 * Strang on U = L(-dz/2) V (the work buffer holds it afterwards).
 * Synchronises. */
int ssfm_fluence_mismatch(ssfm_ctx* ctx, int32_t inst, const void* target,
                          int32_t where, double* loss);

/* Exact discrete adjoint of the recorded march (the Eq. (1), (3), (9)
 * split steps in reverse) back to its first step, recomputing each segment
 * the record did not keep whole from its checkpoint; gives dL/dU_0 and
 * dL/dtheta for fitting the screen parameters by gradients (Math and
 * Equations fits them with a genetic algorithm).  Instances without a cotangent since the
 * record contribute nothing to L: their gradients are zero.  SSFM_ESTATE
 * without a record or without any cotangent. */
int ssfm_backward(ssfm_ctx* ctx);

/* Gradient of L w.r.t. instance inst's initial field (complex128 SI, same
 * convention as the cotangent), to host or device. */
int ssfm_get_grad_field(ssfm_ctx* ctx, int32_t inst, void* dst, int32_t where);

/* Gradient of L w.r.t. theta of instance inst (FP64, host double[8]).
 * Returns SSFM_ENONFINITE (g still written) if a component is not finite:
 * the linearised march can grow exponentially (e.g. an ansatz whose
 * imaginary coefficients make a gain that rises with intensity, Eq. (6)),
 * and a complex64 adjoint then overflows. */
int ssfm_get_grad_theta(ssfm_ctx* ctx, int32_t inst, double* g);

/* Block mean of a float64 n*n device array into (n/b)*(n/b) (device to
 * device): the dense-grid fluence averaged onto the sparse grid of the
 * effective solution (Math and Equations: dense true solutions against
 * sparse effective ones).  dst[i][j] = mean of src over rows b i .. b i +
 * b - 1 and columns b j .. b j + b - 1.  SSFM_EINVAL unless b divides n. */
int ssfm_block_mean(ssfm_ctx* ctx, const double* src, int32_t n, int32_t b,
                    double* dst);

/* Effective-lens screen D_f (Math and Equations, Eq. (4)-(6)).  Applied to
 * the current field U of one instance (its pending screen applied first):
 *   w_dif = F^-1[exp(-l_dif k^2) F |U|^2]                       (Eq. (4))
 *   where w_dif >= w_l (the trimmed lens field):
 *     r = cbrt(w_dif / c1 + c2), clamped at 0  (inverse of the cubic lens
 *         field w_lens = c1 (r^3 - c2), Eq. (5))
 *     f = sum_j a_j cos(omega_j r + psi_j) on [r_{j-1}, r_j), r_0 = 0,
 *         + i (the same with the imaginary segments)         (Eq. (6))
 *     U <- U exp(i f) = U exp(-Im f) exp(i Re f)
 * Segment rows are {r_j [m], amplitude, frequency [1/m], phase}, with
 * increasing r_j; f = 0 beyond the last one.  The filter runs through the
 * row and column pass kernels (the filter table in place of the
 * propagator), the rest pointwise in FP64.  Ends the recorded march
 * (backward needs a new ssfm_forward_record).  Synchronises. */
typedef struct {
  double l_dif;       /* [m^2] Fourier filter of Eq. (4), >= 0 */
  double w_l;         /* [W/m^2] trimming level */
  double c1, c2;      /* cubic lens field w = c1 (r^3 - c2): [W/m^5], [m^3]; c1 != 0 */
  int32_t n_re, n_im; /* segments of the real / imaginary profile, 0..8 */
  double re[8][4];    /* {r_j, a_j, omega_j, psi_j} */
  double im[8][4];    /* {r_l, b_l, nu_l, eta_l} */
} ssfm_lens;

int ssfm_apply_lens(ssfm_ctx* ctx, int32_t inst, const ssfm_lens* lens);

/* Vector-Jacobian product of the effective lens, for fitting the lens
 * parameters by gradients (the differentiable variant of the lens that can
 * take the place of the ansatz f_theta; Eq. (4)-(6)).  For the lens applied
 * to the field u_in of instance inst's grid (the context's own fields and
 * recorded march are not used or changed), given the cotangent g_out of
 * its output, writes the cotangent g_in of its input and grad[] = dL/d
 * (c1, c2, then amplitude, frequency, phase of each real segment, then of
 * each imaginary segment): 2 + 3 (n_re + n_im) values, n_grad at least that.
 * Cotangents follow G = dL/dRe U + i dL/dIm U (as ssfm_set_cotangent);
 * u_in, g_out, g_in: device complex128 n x n row-major [sqrt(W/m^2)],
 * g_in may not alias the others.  With z = conj(g_out) U E, E = exp(i f):
 *   g_in = conj(E) g_out + 2 F^-1[exp(-l_dif k^2) F h] U,
 *   h = -Im(z) df_re/dw_dif - Re(z) df_im/dw_dif on the active points;
 * l_dif, w_l and the joining points are not differentiated (the last two
 * are jumps of f).  Uses the work buffer and the staging area; synchronises.
 * SSFM_EINVAL for an invalid lens, NULL pointers or a short grad. */
int ssfm_lens_vjp(ssfm_ctx* ctx, int32_t inst, const ssfm_lens* lens, const void* u_in,
                  const void* g_out, void* g_in, double* grad, int32_t n_grad);

/* Hot areas (Results, multiple filamentation and the turbulent path: a hot
 * area is a closed region of the fluence where w >= w_p; N_ha is their
 * number).  Counts the 4-connected regions of w >= threshold in the n x n
 * FP64 array w [W/m^2, row-major, device memory, e.g. from
 * ssfm_get_intensity]; with periodic != 0 a region continues across the
 * window edge (the march's grid is periodic).  n must not exceed the
 * context's largest grid (the labels use its staging buffer).  Enqueued on
 * the context's stream and synchronises; *count on the host.  SSFM_EHIP if
 * the labelling's bounded union loop hit its cap (not expected). */
int ssfm_hot_areas(ssfm_ctx* ctx, const double* w, int32_t n, double threshold,
                   int32_t periodic, int64_t* count);

/* ssfm_hot_areas for callers that cannot allocate device memory (code that
 * must not call hipMalloc, e.g. tight serving loops or harnesses that forbid
 * it) and have no context: the same count, with the labels, overflow flag
 * and partial counts in a fixed device array inside the library (16 MiB +
 * 4 KiB per GPU, held until the process ends) instead of a workspace.  w:
 * n x n FP64 device array [W/m^2], row-major; n <= 2048 (larger grids:
 * ssfm_hot_areas with a context), else SSFM_EINVAL; stream: hipStream_t or
 * NULL.  Calls no hipMalloc or hipFree.  All calls on one GPU share that
 * array: calls that overlap on one GPU (other threads or streams) race and
 * must be serialised by the caller.  Synchronises stream; *count on the
 * host.  SSFM_EHIP if the labelling's bounded union loop hit its cap. */
int ssfm_hot_areas_static(const double* w, int32_t n, double threshold, int32_t periodic,
                          void* stream, int64_t* count);

/* Spatial moment of a fluence (Eq. (8) family, read as Q(p, m) = sum over
 * the cell-centred grid of w^p (x^2 + y^2)^m dx^2, dx = length / n,
 * x_j = (j + 1/2 - n/2) dx): w is n x n FP64 in device memory, p any
 * finite exponent (p = 2m the printed form, p = 1 the energy moments),
 * m >= 0.  FP64 block partial sums added on the host in block order
 * (deterministic); synchronises; *q on the host. */
int ssfm_moment(ssfm_ctx* ctx, const double* w, int32_t n, double length, double p,
                int32_t m, double* q);

/* Measure vector P of a solution, for the genetic search's population
 * fitness (Math and Equations, GA paragraph: P characterises the solution of
 * a gene and is compared with the dense-grid solution's P0 by the Euclidean
 * metric; Eq. (8) moments).  Of an n x n FP64 fluence w [W/m^2] in device
 * memory on a window of side length [m]:
 *   P = (Q(1,0), Q(1,1), Q(2,0), Q(2,1), max w, N_ha(w >= w_p))
 * with Q(p, m) as in ssfm_moment (energy [W], its second moment [W m^2], the
 * Eq. (8) m = 1 moment Q(2,1) and Q(2,0)), the peak [W/m^2] and the hot-area
 * count of ssfm_hot_areas (periodic != 0: regions continue across the
 * window edge).  FP64 partial sums in a fixed order; p: host double[6].
 * n at most the context's largest grid (labels in its staging area).
 * Synchronises. */
#define SSFM_MEASURE_LEN 6
int ssfm_measure_vector(ssfm_ctx* ctx, const double* w, int32_t n, double length, double w_p,
                        int32_t periodic, double* p);

/* Distance of instance inst's current fluence from a reference measure
 * vector p0 (host double[6], e.g. ssfm_measure_vector of a dense-grid
 * fluence): d = sqrt(sum_k ((P_k - P0_k) / s_k)^2), s_k = |P0_k| (1 where
 * P0_k = 0), the Euclidean metric in relative units so that quantities of
 * different units weigh alike.  Writes d and, if p is not NULL, P (host
 * double[6]).  Uses the staging area; synchronises. */
int ssfm_measure_distance(ssfm_ctx* ctx, int32_t inst, double w_p, int32_t periodic,
                          const double* p0, double* d, double* p);

/* FP32 screens evaluate sin/cos with the hardware v_sin/v_cos instructions
 * after an exact-to-rounding reduction to [-1/2, 1/2] revolutions (0,
 * default) or with the device math library's sincosf (1).  No effect on
 * FP64 contexts. */
int ssfm_set_precise_math(ssfm_ctx* ctx, int32_t enable);

/* Backward sweep schedule (section Math and Equations, the adjoint of the
 * march with checkpoints): each checkpointed segment is recomputed after
 * the adjoint of the following segment on the context's stream (0,
 * default), or on a second stream while that adjoint runs (1).  The
 * gradients are the same bitwise; the second form overlaps the two kernel
 * chains, which pays only where neither fills the GPU (the 4096^2 passes
 * do).  Drops the context's captured steps. */
int ssfm_set_recompute_overlap(ssfm_ctx* ctx, int32_t enable);

/* Run march steps through captured HIP graphs (1, default) or plain
 * launches (0). */
int ssfm_use_graphs(ssfm_ctx* ctx, int32_t enable);

/* Number of compiled FFT tile variants of the row pass and of the column
 * pass for grid size n (points per thread, lines per workgroup, twiddle
 * loading, occupancy target), and the selection of the variants this
 * context uses for that n (autotuner hook; drops the context's captured
 * graphs).  A variant whose tile does not fit a workgroup's LDS at the
 * context's precision (wide column tiles in FP64) is not built for it:
 * ssfm_select_plan then returns SSFM_EUNSUPPORTED and keeps the current
 * selection. */
int ssfm_plan_variants(int32_t n, int32_t precision, int32_t* n_row, int32_t* n_col);
int ssfm_select_plan(ssfm_ctx* ctx, int32_t n, int32_t row_variant, int32_t col_variant);

/* Variants of the adjoint row and column passes for grid size n, chosen
 * apart from the forward ones (their registers and best tiles differ); -1
 * follows the forward variant (the default).  A variant must have the lines
 * per workgroup of the forward variant in use (the work lists are shared),
 * else SSFM_EINVAL; one not built at the context's precision returns
 * SSFM_EUNSUPPORTED.  A later ssfm_select_plan whose lines differ resets the
 * adjoint choice to -1.  Drops the context's captured graphs. */
int ssfm_select_adjoint_plan(ssfm_ctx* ctx, int32_t n, int32_t row_variant,
                             int32_t col_variant);

/* Autotuner hook for the adjoint passes: reps launches of the adjoint
 * column pass and of the adjoint row pass over all instances (with their
 * selected variants), timed with HIP events on the context's stream; mean
 * milliseconds per launch.  The passes read the cotangent buffer and the
 * state and write the work buffer and the theta accumulators (which every
 * backward clears first): fields, cotangents and gradients are unchanged.
 * SSFM_ESTATE unless the context was created with max_steps > 0. */
int ssfm_time_adjoint_passes(ssfm_ctx* ctx, int32_t reps, double* ms_col, double* ms_row);

/* Time each pass kernel of one step in isolation with HIP events on the
 * context's stream: reps launches of the forward row pass and of the
 * forward column pass over all instances.  Writes the mean milliseconds per
 * launch and the bytes each launch moves (algorithmic: read + write of the
 * field).  The passes read the state and write the work buffer only, so the
 * fields and the march position are unchanged. */
int ssfm_time_passes(ssfm_ctx* ctx, int32_t reps, double* ms_row,
                     double* ms_col, double* bytes_row, double* bytes_col);

/* Sampled pass timing inside the march itself.  With every > 0, each step
 * s of ssfm_propagate and ssfm_forward_record with s % every == every / 2
 * is launched outside the captured step graphs (which then cover the steps
 * in between) and bracketed by HIP events on the context's stream: one
 * before the row pass, one between the row and the column pass, one after
 * the column pass.  Results are bitwise those of an unsampled march.  0
 * (default) turns sampling off.  Changing it drops the captured graphs. */
int ssfm_set_pass_timing(ssfm_ctx* ctx, int32_t every);

/* Mean milliseconds of the row pass and of the column pass over the samples
 * of the most recent propagate or forward-record call (synchronises the
 * context's stream); *n_samples = 0 and zero times when none were taken. */
int ssfm_pass_times(ssfm_ctx* ctx, double* ms_row, double* ms_col,
                    int32_t* n_samples);

/* Sampled pass timing of the most recent ssfm_backward (with pass timing on,
 * ssfm_set_pass_timing(every > 0), the backward runs without its captured
 * graph; adjoint step s of its first checkpoint segment, the one that runs
 * without a recompute beside it, with s % every == every / 2 is bracketed
 * by HIP events on the context's stream).  Mean milliseconds of the adjoint
 * column pass (reads and writes the cotangent) and of the adjoint row pass
 * (reads the cotangent and the stored pre-screen field, writes the
 * cotangent; the adjoint screen fused); synchronises; *n_samples = 0 and
 * zero times when none were taken. */
int ssfm_adjoint_pass_times(ssfm_ctx* ctx, double* ms_col, double* ms_row,
                            int32_t* n_samples);

/* Wait for all work of the context's stream. */
int ssfm_synchronize(ssfm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SSFM_H */
