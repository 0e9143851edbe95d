/*
 * libomm: dense orbital minimization method (OMM) on one AMD Instinct MI355X (gfx950).
 *
 * The library minimizes the OMM functional of Corsetti, "The orbital minimization method for
 * electronic structure calculations with finite-range atomic basis sets" (arXiv:1312.1549):
 *
 *     E[C] = 4 Tr{HW} - 2 Tr{SW HW},   HW = C Hs C^T,  SW = C S C^T,  Hs = H - eta S
 *
 * (Sec. 2.1, Eq. 8, with the eigenspectrum shift of Sec. 2.2, Eq. 9) by conjugate gradients with
 * exact quartic line searches (Sec. 2.3, Eqs. 12-16) and the kinetic-energy preconditioner
 * P = (S + T/tau)^-1 (Sec. 2.4, Eq. 17), stopping on the relative energy change (Sec. 2.5.2,
 * Eq. 18, taken with absolute values).
 *
 * Conventions shared by every entry point:
 *  - All matrices are FP64, row-major, dense. H, S, T are N x N and symmetric. C is M x N with
 *    one row per Wannier function (the paper's m x n column matrix C^mu_i holds the same
 *    numbers), so N = number of basis orbitals (the paper's m), M = number of Wannier functions
 *    (the paper's n), 0 < M <= N.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device memory on the
 *    context's device. Host inputs are copied in; device inputs are read during the call only
 *    (stream-ordered on the context's stream). Outputs go to caller-allocated buffers.
 *  - A context owns all of its device memory; it is not thread-safe; one context uses one
 *    HIP stream.
 *  - Return value: 0 = OMM_OK, > 0 warning, < 0 error. omm_last_error() returns the message of
 *    the last non-zero status of that context.
 */
#ifndef OMM_H_
#define OMM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  OMM_OK = 0,
  OMM_W_MAXITER = 1,      /* max_iter line searches done without meeting tol */
  OMM_E_ARG = -1,         /* invalid argument (sizes, null pointers, tol < 0, missing T, ...) */
  OMM_E_STATE = -2,       /* call out of order (no H/S yet, no C to resume from, ...) */
  OMM_E_ALLOC = -3,       /* device allocation failed */
  OMM_E_HIP = -4,         /* HIP runtime error */
  OMM_E_NONFINITE = -5,   /* NaN/Inf in an input or in the iteration */
  OMM_E_PRECON = -6,      /* S + T/tau (or S) could not be inverted */
  OMM_E_NO_LINE_MIN = -7, /* the quartic along D has no local minimum (Sec. 2.2: eta too low) */
  OMM_E_DIVERGED = -8,    /* Tr SW exceeded 16 M: the iterate left the basin of the minimum */
  OMM_E_ASYMMETRIC = -9   /* H, S or T is not symmetric */
};

/* Arithmetic of the cubic-scaling products (the trace reductions, quartic coefficients and line
 * minimum are always FP64). */
enum {
  OMM_FP64 = 0,   /* FP64 MFMA, FP64 storage */
  OMM_FP32 = 1,   /* FP32 MFMA, FP32 storage of the M x N and N x N operands */
  OMM_BF16X3 = 2  /* BF16 MFMA on bf16 hi/lo splits with FP32 accumulation: operands with two
                     planes (x = hi + lo) give products exact to ~2^-17 relative per term.
                     MFMA passes per product: the gradient 3 (lo*hi + hi*lo + hi*hi); every
                     product with the search direction 2 (D is rounded to bf16 when it is
                     formed, so its lo plane is zero); the preconditioning PG = G~ P~ 1 (both
                     G and P applied as their bf16 roundings; OMM_PG_SPLIT=1 in the environment
                     makes it 2, with G split hi/lo) */
};

typedef struct omm_ctx omm_ctx;

/* Create a context for N basis orbitals and M Wannier functions (0 < M <= N) on the current
 * HIP device. *out is set to NULL on failure. */
int omm_create(int64_t N, int64_t M, omm_ctx **out);
int omm_destroy(omm_ctx *ctx);

/* Select the arithmetic of the products (OMM_FP64 default). fp64_refine != 0 with a mixed mode:
 *  - OMM_BF16X3: the CG state (C, HC, SC, HW, SW) is kept in FP64 while every cubic product runs
 *    on bf16 planes; every omm_set_resync() line searches HC, SC, HW, SW and the energy are
 *    recomputed exactly in FP64 from C, and the stopping rule (Eq. 18) is applied to consecutive
 *    exact energies (scaled by the number of line searches between them); omm_minimize ends
 *    with a resynchronization, so its final energy and state are FP64-exact functions of C;
 *  - OMM_FP32: an FP32 minimization to omm_set_mixed_tol() followed by an FP64 one from its C.
 * fp64_refine == 0: the whole minimization runs in the mixed arithmetic with FP32 storage. */
int omm_set_precision(omm_ctx *ctx, int mode, int fp64_refine);

/* Stopping threshold of the FP32 phase of OMM_FP32 + refinement (default 1e-9). */
int omm_set_mixed_tol(omm_ctx *ctx, double tol);

/* Line searches between FP64 resynchronizations of OMM_BF16X3 + refinement (default 80). */
int omm_set_resync(omm_ctx *ctx, int every);

/* Flavours of the minimization (Sec. 2.4 and the flavours compared in Sec. 3.1). */
enum {
  OMM_FLAVOUR_DENSE = 0,    /* the generalized problem with the preconditioner chosen by tau */
  OMM_FLAVOUR_CHOLESKY = 1  /* Cholesky-reduced: S = L L^T, minimize over C~ = C L with
                               H~ = L^-1 (H - eta S) L^-T and S~ = I (no S products, no P product);
                               the iterates are those of the S^-1-preconditioned dense flavour */
};

/* Select the flavour (OMM_FLAVOUR_DENSE default). With OMM_FLAVOUR_CHOLESKY omm_minimize ignores
 * tau, factorizes S once per omm_set_HS (OMM_E_PRECON if S is not positive definite), and
 * transforms C0 in and C out: omm_get_C, omm_density, omm_edm and omm_backward_device work in the
 * original basis, omm_get_subspace and the energy are basis independent. Changing the flavour
 * ends the active minimization; the next omm_minimize needs a C0. */
int omm_set_flavour(omm_ctx *ctx, int flavour);

/* Block-sparse operator products (the sparse x dense products of Secs. 2.6 and 3, applied to
 * every product with Hs or S of OMM_BF16X3 in the dense flavour: [HD | SD] = D [Hs | S] in each
 * line search, and C [Hs | S] in FP64 when a phase starts and at each resynchronization; default
 * off). The finite-range basis leaves most of Hs and S zero: for every 256-column tile of the
 * product the library lists the 32-deep K blocks in which the operator is not all zero (built
 * once per Hs and S) and multiplies over those only. The skipped blocks contribute exact zeros,
 * so the results are the dense products (up to the sign of zero) and the iterates do not change.
 * Other modes and the Cholesky flavour (whose H~ is dense) ignore it. */
int omm_set_sparse(omm_ctx *ctx, int on);
/* Fraction of K blocks listed for Hs (density[0]) and S (density[1]) after a minimization with
 * sparse products on; OMM_E_STATE otherwise. */
int omm_sparse_density(omm_ctx *ctx, double *density);

/* Use `hip_stream` (a hipStream_t) for all work; NULL restores the context's own stream. */
int omm_set_stream(omm_ctx *ctx, void *hip_stream);

/* Hamiltonian, overlap and (nullable) kinetic matrices of the generalized eigenproblem
 * H c = eps S c (Sec. 2.1, Eq. 1). Host pointers, N*N each, copied in. T is needed only for a
 * finite tau > 0 (Eq. 17). Checked for finite values and symmetry (relative 1e-10):
 * OMM_E_NONFINITE / OMM_E_ASYMMETRIC (the previous inputs then stay; a HIP failure while copying
 * leaves the context without inputs, OMM_E_STATE until the next successful call). Ends the active
 * minimization and drops the cached shift Hs = H - eta S and everything derived from it. When
 * S and T are bit for bit those of the previous call (an SCF step at a fixed geometry, Sec. 3),
 * what derives from them alone is kept: the preconditioner P, the Cholesky factor of the
 * reduced flavour, the bf16 planes, FP32 copy and K-block list of S; a new S or T drops those
 * too. */
int omm_set_HS(omm_ctx *ctx, const double *H, const double *S, const double *T);
/* Same with device pointers (validated on the device, then copied device-to-device). */
int omm_set_HS_device(omm_ctx *ctx, const double *dH, const double *dS, const double *dT);

/* CG minimization of Eq. 8 from C0 (host, M*N; NULL resumes from the context's current C).
 *   eta       eigenspectrum shift (Sec. 2.2); must exceed the M-th eigenvalue for the minimum to
 *             describe the occupied subspace;
 *   tau       > 0 finite: P = (S + T/tau)^-1; +INFINITY: P = S^-1; <= 0: no preconditioning
 *             (Sec. 2.4, Eq. 17). P is factorized once and reused while S, T, tau are unchanged;
 *   tol       stop when |2 (E_new - E)| <= tol |E_new + E| after a line search (Eq. 18);
 *   max_iter  maximum number of line searches (per phase in mixed precision).
 * Returns OMM_OK, OMM_W_MAXITER, or an error. */
int omm_minimize(omm_ctx *ctx, const double *C0, double eta, double tau, double tol,
                 int max_iter);
/* Same with C0 a device pointer (M*N FP64; NULL resumes). */
int omm_minimize_device(omm_ctx *ctx, const double *dC0, double eta, double tau, double tol,
                        int max_iter);

/* Continue the CG of the last minimization (same precision phase, same direction history) for
 * up to `count` more line searches, stopping early when Eq. 18 holds for `tol` (tol = 0 never
 * stops early). No setup work is repeated. In OMM_BF16X3 + refinement the FP64
 * resynchronizations stay on the schedule of omm_set_resync() counted across calls (every
 * `every` line searches since the last one, which omm_minimize's end also performs): a call
 * that stops between two leaves the incrementally updated FP64 state, whose energy (omm_energy,
 * the trace) carries the products' rounding since the last resynchronization, and the stopping
 * rule is only tested at resynchronizations. Returns OMM_OK (converged), OMM_W_MAXITER (count
 * line searches done) or an error; OMM_E_STATE if no minimization is active (new H/S invalidate
 * it). */
int omm_iterate(omm_ctx *ctx, int count, double tol);

/* Functional value (Eq. 8, shifted Hamiltonian) at the current C. The unshifted band energy
 * is E + 2 M eta. */
int omm_energy(omm_ctx *ctx, double *E);

/* rho = 2 C^T (2I - SW) C (N*N, host): the derivative of E with respect to H; at the minimum
 * (SW = I) the density matrix 2 sum_i c_i c_i^T of the occupied subspace (Sec. 2.1). */
int omm_density(omm_ctx *ctx, double *rho);
int omm_density_device(omm_ctx *ctx, double *d_rho);

/* EDM = 2 C^T HW C (N*N, host): the energy-density matrix; dE/dS = -EDM - eta rho. */
int omm_edm(omm_ctx *ctx, double *edm);
int omm_edm_device(omm_ctx *ctx, double *d_edm);

/* Reverse-mode derivative of E: d_gH = gE * rho and d_gS = gE * (-EDM - eta rho) (device N*N
 * each, FP64), evaluated at the current C (exact derivatives of the minimum at convergence). */
int omm_backward_device(omm_ctx *ctx, double gE, double *d_gH, double *d_gS);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * or training loops, harnesses that forbid allocation): omm_backward_device's results (same
 * arguments, layout and ownership, equal to rounding: the C^T X C sums run over chunks of C's
 * rows) with no hipMalloc/hipFree and no use of the context's scratch buffers. Its only
 * scratch is a 16 MiB array in the library's static device memory, one copy per GPU held
 * until the process ends; calls that overlap on one GPU race on it (serialize them). Limits:
 * N <= 32768 (N <= 2^21 / min(M, 64)); larger N -> OMM_E_ARG. The Cholesky flavour ->
 * OMM_E_STATE (use omm_backward_device). */
int omm_backward_device_noalloc(omm_ctx *ctx, double gE, double *d_gH, double *d_gS);

/* Current C (host M*N), HW and SW (host M*M each; either may be NULL). */
int omm_get_C(omm_ctx *ctx, double *C);
int omm_get_subspace(omm_ctx *ctx, double *HW, double *SW);
/* Preconditioner of the last minimization (host N*N), kept across omm_set_HS calls that leave S
 * and T unchanged; OMM_E_STATE if none was used or a new S or T dropped it. */
int omm_get_preconditioner(omm_ctx *ctx, double *P);

/* Line searches of the last minimize call (both phases) and the last relative change. */
int omm_stats(omm_ctx *ctx, int *iters, double *last_rel_change);
/* Line searches of the last minimize call split by phase: mixed precision, then FP64 (an FP64
 * run reports all of them as FP64). The energy trace holds mixed_iters + 1 entries of the mixed
 * phase followed by fp64_iters + 1 entries of the FP64 phase (when both ran). */
int omm_phase_stats(omm_ctx *ctx, int *mixed_iters, int *fp64_iters);
/* FP64-exact energies of the OMM_BF16X3 + refinement scheme: the line-search index and energy
 * at the start and at every resynchronization (up to cap; *n = total). */
int omm_checkpoints(omm_ctx *ctx, int *iters, double *energies, int cap, int *n);
/* Complex Hermitian problems (a general k-point: the Hermitian forms of Secs. 2.1-2.4). The
 * context holds the exact real embedding: N x N Hermitian X = A + iB (A symmetric, B
 * antisymmetric) acts on row vectors [Re c, Im c] as the real symmetric 2N x 2N [[A, B],
 * [-B, A]], and every complex Wannier function c becomes the two real rows [Re c, Im c] and
 * [-Im c, Re c] (the real problem has 2M rows; each complex eigenvalue appears twice). The
 * iterates are the complex iterates; omm_energy, omm_energy_trace and omm_checkpoints report the
 * complex problem's energy (half the real one). omm_get_C and omm_get_subspace return the real
 * embedding (2M x 2N, 2M x 2M); omm_density_complex the complex density.
 * omm_create_complex: N, M are the complex sizes (0 < M <= N). */
int omm_create_complex(int64_t N, int64_t M, omm_ctx **out);
/* Host pointers, N*N row-major each: the real and imaginary parts of H, S and (nullable) T;
 * a null imaginary part is zero. Hermiticity is checked (OMM_E_ASYMMETRIC otherwise). */
int omm_set_HS_complex(omm_ctx *ctx, const double *H_re, const double *H_im,
                       const double *S_re, const double *S_im, const double *T_re,
                       const double *T_im);
/* C0 (M x N, host, row i = the conjugated coefficients of Wannier function i, i.e. the paper's
 * C^H) as real and (nullable) imaginary parts; C0_re == NULL resumes. Other arguments and the
 * return value as omm_minimize. */
int omm_minimize_complex(omm_ctx *ctx, const double *C0_re, const double *C0_im, double eta,
                         double tau, double tol, int max_iter);
/* rho = 2 C^H (2I - SW) C (N x N Hermitian, host): real and imaginary parts. */
int omm_density_complex(omm_ctx *ctx, double *rho_re, double *rho_im);

/* Energies E_0, E_1, ... of the last minimize call (phase 1 then refinement), up to cap. */
int omm_energy_trace(omm_ctx *ctx, double *buf, int cap, int *n);

/* Diagnostics: with profiling on, every line search records HIP events on the context's stream
 * around its 7 stages (gradient GEMM, P GEMM, Polak-Ribiere + direction, [HD|SD] GEMM alone,
 * projection GEMM with the bf16 splits of HD and SD, coefficients + line minimum, updates +
 * energy). Line searches replayed from a captured graph are not profiled: profiling turns graph
 * replay off. Turning it on (or off) resets
 * the sums. omm_stage_times writes min(cap, 7) accumulated stage times in ms and the number of
 * profiled line searches, and returns the number of stages (7). */
int omm_set_profiling(omm_ctx *ctx, int on);
int omm_stage_times(omm_ctx *ctx, double *ms, int cap, int *iters);

const char *omm_last_error(const omm_ctx *ctx);

/* ---- many independent systems of uneven size in one set of launches ----
 * Every CG stage is one grouped launch over the tiles of all live systems; converged systems
 * drop out of the tile lists. FP32 (default) or FP64 MFMA products, FP64 reductions. */
typedef struct omm_batch omm_batch;

int omm_batch_create(int nsys, const int64_t *N, const int64_t *M, omm_batch **out);
int omm_batch_destroy(omm_batch *b);
/* Arithmetic of the batched minimization: OMM_FP32 (default: FP32 products and M x N state) or
 * OMM_FP64; any other mode is OMM_E_ARG. fp64_refine != 0 with OMM_FP32: each system first
 * runs the FP32 phase to the tolerance of omm_batch_set_mixed_tol() (default 1e-9; the larger
 * of it and the call's tol), then an FP64 phase from that C to the call's tol, also in grouped
 * launches; energies, C and the stopping rule then come from the FP64 phase. */
int omm_batch_set_precision(omm_batch *b, int mode, int fp64_refine);
int omm_batch_set_mixed_tol(omm_batch *b, double tol);
/* Line searches of the last omm_batch_minimize per system (nsys entries each, either pointer
 * nullable): in the FP32 phase and in the FP64 phase. */
int omm_batch_phase_iterations(omm_batch *b, int *iters32, int *iters64);
/* System i: host H, S, T (N_i*N_i each; T nullable as for omm_set_HS). The system keeps its
 * preconditioner when S and T are bit for bit those of its previous call. */
int omm_batch_set_HS(omm_batch *b, int i, const double *H, const double *S, const double *T);
/* Same with device pointers, validated on the device (OMM_E_NONFINITE / OMM_E_ASYMMETRIC), then
 * copied device-to-device on the batch's own stream: the caller's writes to them must be
 * complete before the call; they are no longer read when it returns. */
int omm_batch_set_HS_device(omm_batch *b, int i, const double *dH, const double *dS,
                            const double *dT);
/* C0[i]: host M_i*N_i start of system i (NULL entry: resume from its current C). eta, tau:
 * arrays of nsys values; max_iter bounds each phase. Returns OMM_OK if every system converged,
 * OMM_W_MAXITER if some did not, or the first error. */
int omm_batch_minimize(omm_batch *b, const double *const *C0, const double *eta,
                       const double *tau, double tol, int max_iter);
int omm_batch_energy(omm_batch *b, double *E /* nsys */);
int omm_batch_iterations(omm_batch *b, int *iters /* nsys */);
int omm_batch_get_C(omm_batch *b, int i, double *C /* host M_i*N_i */);
const char *omm_batch_last_error(const omm_batch *b);

/* k-point batches: complex Hermitian systems (N[i], M[i] the complex sizes, 0 < M <= N <= 32768)
 * held as their exact real embeddings (see omm_create_complex) and solved together by the
 * grouped launches above. omm_batch_energy reports the complex energies; omm_batch_get_C
 * returns the real embedding (2M x 2N) of system i. A warm start across k passes the previous
 * k-point's C as C0. */
int omm_batch_create_complex(int nsys, const int64_t *N, const int64_t *M, omm_batch **out);
int omm_batch_set_HS_complex(omm_batch *b, int i, const double *H_re, const double *H_im,
                             const double *S_re, const double *S_im, const double *T_re,
                             const double *T_im);
int omm_batch_minimize_complex(omm_batch *b, const double *const *C0_re,
                               const double *const *C0_im, const double *eta, const double *tau,
                               double tol, int max_iter);

#ifdef __cplusplus
}
#endif

#endif /* OMM_H_ */
