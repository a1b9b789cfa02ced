/*
 * fnocc.h -- C ABI of the MI355X (gfx950) FNO-EOM-CCSDT library.
 *
 * What the library computes (arXiv 2509.14157):
 *   - Section 1.2, eqs (8)-(10): MP2 amplitudes t_ij^ab = <ab||ij>/e_ij^ab,
 *     the virtual-virtual MP2 density D_ab, its natural orbitals and the
 *     frozen-natural-orbital truncation of the virtual space, followed by
 *     semicanonicalisation of the kept virtual block.
 *   - Section 1.1, eqs (5)-(7): ground-state CCSDT, 0 = <Phi^n|e^{-T} H e^{T}|Phi_0>
 *     for n = 1..3 and E = <Phi_0|e^{-T} H e^{T}|Phi_0>.
 *   - Section 1.1, eqs (1)-(4): EOM-CCSDT right eigenstates for the ionized
 *     (IP: 1h, 2h1p, 3h2p), doubly ionized (DIP: 2h, 3h1p, 4h2p), electron
 *     attached (EA: 1p, 2p1h, 3p2h) and doubly attached (DEA: 2p, 3p1h, 4p2h)
 *     operator spaces.
 * All of it runs in the (truncated) spin-orbital space on one GPU.
 *
 * Conventions
 *   - Spin-orbitals, occupied orbitals first.  Energies in hartree.
 *   - Every call returns an int status: FNO_OK or a negative error code;
 *     fno_last_error() then describes the failure.
 *   - Inputs are copied; outputs are caller-allocated host arrays.
 *   - Call order: fno_load_hamiltonian -> [fno_truncate] -> fno_ccsdt -> fno_eom.
 *     An out-of-order call returns FNO_ESTATE.  One context per host thread.
 *   - Packed amplitude layout (fno_get/set_amplitudes): each antisymmetric
 *     index group holds strictly increasing tuples in colexicographic order
 *     (tuple x0<x1<..<x{g-1} at sum_t C(x_t, t+1)); groups are row-major with
 *     the hole group first.  T1 is the dense o x v array.
 */
#ifndef FNOCC_H
#define FNOCC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FNO_OK = 0,
  FNO_EINVAL = -1,     /* bad argument, bad input symmetry, size out of range */
  FNO_ENOMEM = -2,     /* device or host allocation failed */
  FNO_EDEVICE = -3,    /* HIP runtime error or missing gfx950 device */
  FNO_ENOCONV = -4,    /* solver reached max_iter without meeting its tolerances */
  FNO_ENONFINITE = -5, /* NaN or Inf in an input or during the iterations */
  FNO_ESTATE = -6      /* call out of order (e.g. fno_eom before fno_ccsdt) */
};

typedef struct fno_ctx fno_ctx;

/* Create a context on HIP device `hip_device` (owns all device memory). */
int fno_create(int hip_device, fno_ctx **out);
void fno_destroy(fno_ctx *ctx);
/* Message of the last failing call on ctx; valid until the next call. */
const char *fno_last_error(const fno_ctx *ctx);
/* Run all device work on this hipStream_t (NULL = the default stream). */
int fno_set_stream(fno_ctx *ctx, void *hip_stream);

/*
 * Load the problem (Section 1.2: canonical orbitals, orbital energies f_pp and
 * antisymmetrized integrals).
 *   fock : n x n row-major Fock matrix, n = nocc + nvir; |f_ov| must be < 1e-10.
 *   eri  : n^4 row-major <pq||rs>; must satisfy <pq||rs> = -<qp||rs> = -<pq||sr>
 *          = <rs||pq> to 1e-10 relative.
 *   e_nuc: constant added to every total energy.
 * Errors: FNO_EINVAL (sizes, symmetry), FNO_ENONFINITE, FNO_ENOMEM.
 */
int fno_load_hamiltonian(fno_ctx *ctx, int nocc, int nvir, const double *fock, const double *eri, double e_nuc);

/*
 * FNO truncation (Section 1.2): MP2 amplitudes (eq 8) with denominators
 * (eq 9), virtual density (eq 10), natural orbitals sorted by descending
 * occupation, truncation, semicanonicalisation of the kept block and
 * transformation of f and <pq||rs>.
 *   occt      : cumulative-occupation threshold in (0, 1]; the smallest k
 *               with sum_{l<=k} n_l >= occt * sum_l n_l is kept (1 keeps all).
 *   nvir_keep : > 0 keeps exactly this many natural orbitals (overrides occt).
 *   nvir_kept : out, number of kept virtuals (may be NULL).
 *   e_mp2     : out, MP2 correlation energy of the full space (may be NULL).
 *   occ       : out, nvir occupation numbers in descending order (may be NULL).
 */
int fno_truncate(fno_ctx *ctx, double occt, int nvir_keep, int *nvir_kept, double *e_mp2, double *occ);

typedef enum { FNO_FP64 = 0, FNO_FP32 = 1, FNO_BF16X3 = 2 } fno_prec;

/* Options of the ground-state solver (Jacobi steps t += r/D with DIIS). */
typedef struct {
  int max_iter;     /* default 100 */
  double r_tol;     /* converged when ||r||_2 over unique amplitudes < r_tol ... */
  double e_tol;     /* ... and |Delta E| < e_tol */
  int diis_n;       /* DIIS history length (0 disables), default 8 */
  int diis_start;   /* first iteration that extrapolates, default 3 */
  fno_prec prec;    /* precision of the triples contractions; solver stays FP64 */
  int guess;        /* 0 = zero amplitudes (first step gives MP2); 1 = learned T3 guess
                       (needs fno_set_guess_model; see below) */
} fno_cc_opts;
void fno_cc_opts_default(fno_cc_opts *o);

/*
 * Ground-state CCSDT (eqs 5-7) in the current (possibly truncated) space.
 *   e_corr, e_tot: correlation and total energy (e_tot = E_ref + e_corr + e_nuc).
 *   iters, res_norm: iterations used and final residual norm.
 * Converged: res_norm < r_tol and |Delta E| < e_tol.  With FP32 or split-BF16
 * triples products the residual has a floor set by the products' rounding
 * (about 2e-7 for FP32 and 1e-5 for split-BF16 at o=10, v=59); such a solve
 * has also converged when |Delta E| < e_tol, res_norm < 100 r_tol and the
 * last four residual norms lie within 25% of each other (res_norm then
 * reports the floor; fno_last_trace gives the history).
 * Returns FNO_ENOCONV (results still written) when max_iter is reached.
 */
int fno_ccsdt(fno_ctx *ctx, const fno_cc_opts *opts, double *e_corr, double *e_tot, int *iters, double *res_norm);

typedef enum { FNO_IP = 1, FNO_DIP = 2, FNO_EA = 3, FNO_DEA = 4 } fno_eom_kind;

typedef struct {
  int nroots;       /* number of roots (lowest real parts) */
  int max_iter;     /* Davidson iterations, default 60 */
  int max_sub;      /* subspace size before a thick restart (the Ritz vectors of this
                       and the previous iteration are kept), default 8 * nroots */
  double e_tol;     /* |Delta omega| tolerance */
  double r_tol;     /* residual-norm tolerance */
  fno_prec prec;    /* precision of the R3 sigma contractions */
  int guess;        /* 0 = unit vectors on the lowest principal-block diagonal */
  int precond;      /* 0 = (omega - D)^-1, D the one-body H-bar diagonal (dressed
                       Fock diagonal at the CC amplitudes, particles minus holes) */
  int block;        /* sigma vectors evaluated together (the R-derived tensors hold a
                       block of vectors; every contraction covers the block in one
                       GEMM); 0 = nroots, at most 16 */
} fno_eom_opts;
void fno_eom_opts_default(fno_eom_opts *o);

/*
 * EOM-CCSDT roots of `kind` on top of the converged ground state.
 *   omega   : nroots excitation energies E_target - E_CCSDT, ascending real part
 *             (IP/DIP: ionization energies; EA/DEA: minus the attachment energy).
 *   e_tot   : nroots total energies (may be NULL).
 *   res_norm: nroots final residual norms (may be NULL).
 */
int fno_eom(fno_ctx *ctx, fno_eom_kind kind, const fno_eom_opts *opts, double *omega, double *e_tot,
            double *res_norm, int *iters);

/*
 * EOM roots of `kind` for n independent problems (batching of uneven-size
 * instances).  Every context must hold a converged fno_ccsdt; they may differ
 * in size; none may appear twice.  The Davidson solvers advance in lockstep:
 * each iteration issues the sigma work of every instance on its own context
 * stream (replayed from hipGraphs once recorded) before any instance waits
 * for its results, so the instances' kernels overlap on the device.  Each
 * instance computes exactly what fno_eom would on that context.
 *   omega    : n * nroots excitation energies, instance-major.
 *   res_norm : n * nroots residual norms (may be NULL).
 *   iters    : n iteration counts (may be NULL).
 * Returns FNO_OK if every instance converged, FNO_ENOCONV if some did not
 * (results still written), another status on error (fno_last_error of the
 * first context names the failing instance).
 */
int fno_batch_eom(int n, fno_ctx *const *ctxs, fno_eom_kind kind, const fno_eom_opts *opts, double *omega,
                  double *res_norm, int *iters);

/*
 * The same solve as fno_batch_eom for callers that batch many small
 * instances, with one persistent grouped launch per contraction: each sigma
 * round takes one block of pending vectors of every instance and, term by
 * term, issues every instance's operand expansions, then the GEMMs of all
 * instances as one persistent launch per kernel instantiation (workgroups
 * take (instance, term, tile) items from a device work queue; the block's
 * roots are inside each GEMM), then every instance's fold, on one batch
 * stream.  Every GEMM runs with its default tile and without split-K, so
 * each instance's roots are bit-identical to those of a grouped batch that
 * holds that instance alone (they differ from fno_eom's in the last bits).
 * All contexts must be on one device.  Arguments, results and errors as for
 * fno_batch_eom.
 */
int fno_batch_eom_grouped(int n, fno_ctx *const *ctxs, fno_eom_kind kind, const fno_eom_opts *opts, double *omega,
                          double *res_norm, int *iters);

/*
 * MP2 correlation energies (eqs 8-9) of the full virtual space and of the
 * truncated space of the last fno_truncate (the kept semicanonical
 * natural orbitals).  Either output may be NULL.
 * Errors: FNO_ESTATE before fno_truncate.
 */
int fno_mp2_energies(const fno_ctx *ctx, double *e_full, double *e_trunc);

/*
 * Extrapolated FNO (XFNO, Computational Details: the M3 values of the result
 * tables).  At each of npts occupation thresholds the problem is truncated
 * (fno_truncate), the ground state solved (fno_ccsdt) and, when kind is an
 * fno_eom_kind, nroots target states found (fno_eom); every total energy is
 * then fitted by a least-squares line in OCCT and the line evaluated at
 * OCCT = 1.  The paper computes its M3 values from the thresholds 0.999,
 * 0.9975 and 0.995 and leaves the extrapolation formula to its supplement;
 * the linear fit in OCCT is this library's reading of it.
 *   occt    : npts distinct thresholds in (0, 1], 2 <= npts <= 16.
 *   cc, eom : solver options (NULL = defaults); kind = 0 skips the EOM part.
 *   kept    : out, npts kept virtual counts (may be NULL).
 *   e_cc    : out, npts ground-state total energies.
 *   e_eom   : out, npts x nroots target total energies, threshold-major (kind != 0).
 *   e_cc_x, e_eom_x : out, the extrapolated ground-state and nroots target
 *             total energies.
 * The context is left truncated at the last threshold, holding its solution.
 * Errors: FNO_EINVAL (thresholds, outputs), those of fno_truncate, fno_ccsdt
 * and fno_eom; FNO_ENOCONV when a solve did not converge (with kind != 0 a
 * ground state that did not converge stops the run).
 */
int fno_xfno(fno_ctx *ctx, int npts, const double *occt, const fno_cc_opts *cc, int kind, const fno_eom_opts *eom,
             int *kept, double *e_cc, double *e_eom, double *e_cc_x, double *e_eom_x);

/* Orbital-space sizes of the current problem (after truncation). */
int fno_sizes(const fno_ctx *ctx, int *nocc, int *nvir, int *nvir_full);

/*
 * Amplitude access in packed layout.  block: 1, 2, 3 = T1, T2, T3.
 * len must equal the packed size (FNO_EINVAL otherwise): o*v, C(o,2)C(v,2),
 * C(o,3)C(v,3).
 */
int fno_get_amplitudes(fno_ctx *ctx, int block, double *buf, size_t len);
int fno_set_amplitudes(fno_ctx *ctx, int block, const double *buf, size_t len);
size_t fno_amplitude_size(const fno_ctx *ctx, int block);

/*
 * One evaluation of the CCSDT residual at the amplitudes currently held
 * (set with fno_set_amplitudes, or the converged ones), in the precision
 * `prec`.  r1/r2/r3 receive the packed residual blocks (each may be NULL),
 * e_corr the energy eq (6) at those amplitudes.  Used for parity checks and
 * benchmarks of one pass of the hot path.
 */
int fno_cc_residual(fno_ctx *ctx, fno_prec prec, double *r1, double *r2, double *r3, double *e_corr);

/*
 * One EOM sigma evaluation sigma = <mu|(H-bar R)_C|0> for the R vector given
 * in packed unique layout (blocks concatenated in rank order, e.g. IP:
 * 1h, 2h1p, 3h2p), on top of the amplitudes currently held.
 * len = fno_eom_size(ctx, kind).
 */
size_t fno_eom_size(const fno_ctx *ctx, fno_eom_kind kind);
int fno_eom_sigma(fno_ctx *ctx, fno_eom_kind kind, fno_prec prec, const double *r, double *sigma, size_t len);

/*
 * Left-hand EOM sigma sigma^T = l^T (H-bar - E_CC) over the same R space
 * (the transpose of fno_eom_sigma in the packed basis), the product that the
 * left EOM vectors L1..L3 (Introduction: L3 among the rate-determining
 * six-index quantities) are found with.  Layout and length as fno_eom_sigma.
 */
int fno_eom_sigma_left(fno_ctx *ctx, fno_eom_kind kind, fno_prec prec, const double *l, double *sigma, size_t len);

/*
 * EOM-CCSDT roots of `kind` with their eigenvectors: right vectors
 * (H-bar - E_CC) r = omega r (left = 0), or left vectors
 * l^T (H-bar - E_CC) = omega l^T (left = 1), by the same block Davidson as
 * fno_eom applied to the corresponding sigma.  Both sides have the same
 * eigenvalues; a left vector and a right vector of different roots are
 * orthogonal.
 *   omega   : nroots eigenvalues, ascending real part.
 *   vectors : nroots * fno_eom_size(ctx, kind) doubles, root-major, each of
 *             unit 2-norm (a biorthonormal pair is l / (l.r), r).
 *   res_norm, iters : as fno_eom (may be NULL).
 * Errors: as fno_eom.
 */
int fno_eom_vectors(fno_ctx *ctx, fno_eom_kind kind, const fno_eom_opts *opts, int left, double *omega,
                    double *vectors, double *res_norm, int *iters);

/*
 * Device-pointer variants of the calls above.  Every d_ buffer is device
 * memory on the context's device (caller-owned, same packed layouts and
 * lengths as the host versions); copies and kernels are enqueued on the
 * context's stream (fno_set_stream), so a caller whose buffers come from
 * another stream orders them with that stream first.  The calls return when
 * the work is enqueued, except fno_cc_residual_dev and fno_eom_sigma_dev,
 * which synchronize the stream before returning (e_corr is read back; the
 * EOM setup of the intermediates needs it).  Device amplitudes are not
 * checked for NaN / Inf on entry (a non-finite residual later makes
 * fno_ccsdt return FNO_ENONFINITE).  Errors as for the host versions.
 */
int fno_get_amplitudes_dev(fno_ctx *ctx, int block, double *d_buf, size_t len);
int fno_set_amplitudes_dev(fno_ctx *ctx, int block, const double *d_buf, size_t len);
int fno_cc_residual_dev(fno_ctx *ctx, fno_prec prec, double *d_r1, double *d_r2, double *d_r3, double *e_corr);
int fno_eom_sigma_dev(fno_ctx *ctx, fno_eom_kind kind, fno_prec prec, const double *d_r, double *d_sigma,
                      size_t len);

/*
 * The fused triples residual (the triples projection of eq 5 in its
 * T1-dressed form: pp-ladder, hh-ladder, ring, one-body and T2 driver terms)
 * without a context, on caller device buffers of device hip_device:
 *   R3 += sum of those terms,
 * with T3 [C(o,3)][C(v,3)] and T2 [C(o,2)][C(v,2)] packed (colex, holes
 * slow); the dressed intermediates W3_vvvv [C(v,2)(bc)][C(v,2)(ef)],
 * F3_vv [v][v], W3_ovvo [o][v][v][o] (m a e i), W3_vvvo [o (k)][v (e)][C(v,2) (bc)],
 * W3_ovoo [o (m)][v (c)][C(o,2) (jk)], W3_oooo [C(o,2)(mn)][C(o,2)(ij)] and
 * F3_oo [o (m)][o (i)], all FP64 (the intermediates a context builds from
 * T1, T2, T3; fno_debug_tensor shows them).  3 <= nocc, nvir <= 64; prec
 * FNO_FP64, FNO_FP32 or FNO_BF16X3 (products; R3 accumulates in FP64).  Work runs on
 * `stream` (NULL: the device's null stream); the call allocates its working
 * buffers (about 2 C(o,3) v C(v,2) values of the product type) for its own
 * duration and returns after the stream has finished.  Inputs are read only,
 * R3 is caller-owned.  Errors: FNO_EINVAL (sizes, precision, null buffer),
 * FNO_EDEVICE, FNO_ENOMEM; fno_dev_last_error() gives the message (per host
 * thread).
 */
int fno_triples_residual_dev(int hip_device, int nocc, int nvir, fno_prec prec, const double *T3, const double *T2,
                             const double *W3_vvvv, const double *F3_vv, const double *W3_ovvo,
                             const double *W3_vvvo, const double *W3_ovoo, const double *W3_oooo,
                             const double *F3_oo, double *R3, void *stream);
const char *fno_dev_last_error(void);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): fno_triples_residual_dev
 * with its working buffers in a static per-device array of 256 MiB (held from
 * the first call on a device until the process ends) instead of allocated
 * memory.  Same arguments, layouts and results; the call allocates nothing
 * (no hipMalloc / hipFree, no allocating library routine), enqueues the work
 * on `stream` and returns without waiting.  The first call on a device looks
 * up the array and fills two small index tables (a device synchronization).
 * Sizes whose working buffers exceed 256 MiB (about 2 C(o,3) v C(v,2)
 * elements of the product type plus small parts; o=10, v=59 and o=12, v=48
 * fit in FP64) return FNO_ENOMEM with the required size in
 * fno_dev_last_error().  Every call on a device shares that device's array,
 * which keeps the last call's contents: calls that overlap on one device
 * (other streams, other host threads) race and give wrong results; order
 * them on one stream or synchronize between them.
 */
int fno_triples_residual_dev_noalloc(int hip_device, int nocc, int nvir, fno_prec prec, const double *T3,
                                     const double *T2, const double *W3_vvvv, const double *F3_vv,
                                     const double *W3_ovvo, const double *W3_vvvo, const double *W3_ovoo,
                                     const double *W3_oooo, const double *F3_oo, double *R3, void *stream);

/* Algorithmic GEMM flops (packed forms) of the triples contractions and of all
 * terms: of one residual evaluation after fno_ccsdt / fno_cc_residual, of the
 * sigma sweep after fno_eom_sigma, and summed over every sigma sweep of the
 * solve after fno_eom / fno_batch_eom (per context). */
int fno_last_flops(const fno_ctx *ctx, double *triples_flops, double *all_flops);

/* Convergence history of the last fno_ccsdt call: for each iteration k
 * (k < *n), energies[k] = E_corr after the update of iteration k+1 and
 * res_norms[k] = the Euclidean norm of that iteration's residual over the
 * unique amplitudes (the quantities the stopping test of fno_ccsdt uses).
 * At most cap entries are written; *n receives the number of iterations
 * recorded.  Either array may be NULL.  Host arrays, caller-owned.
 * Returns FNO_OK, or FNO_EINVAL for a null context or n. */
int fno_last_trace(const fno_ctx *ctx, double *energies, double *res_norms, int cap, int *n);

/*
 * Diagnostics.
 * fno_debug_tensor copies the whole storage (packed layout, FP64) of the named
 * device tensor of the current problem (e.g. "T3", "R3", "W3_vvvv", "Gd") to
 * buf; len must equal fno_debug_tensor_size (0 when the name is unknown).
 * fno_debug_gemm runs one device GEMM C = alpha*A*B + beta*C on host arrays:
 * A is M x K (a_kfast: row-major, else column-major), B is K x N (b_nfast:
 * row-major, else column-major), C is M x N row-major; prec selects the MFMA
 * path (operands are rounded to it on the device), tile a tile shape index
 * (-1 = default heuristic).  Used to validate the kernels and by the tile
 * autotuner.
 */
/*
 * Kernel timing with HIP events on the context's stream.  fno_profile(ctx, 1)
 * starts recording every expansion, GEMM and fold launch; fno_profile_report
 * writes a JSON text (per kernel name: launches, total_ms, algorithmic GEMM
 * flops, operand bytes; per term: the same for the GEMM) into buf (len bytes,
 * NUL-terminated, FNO_EINVAL if too small) and clears the records.  A GEMM's
 * name is its kernel followed by its shape, e.g.
 * "fno::gemm_k4v_kernel<double, 128, 128, true, true> [590x76995x590]" (M x N x K),
 * so terms that share an instantiation are reported apart.
 */
/*
 * Diagnostics: with the environment variable FNO_TRACE set, the library
 * prints to stderr each Davidson iteration's Ritz
 * values and residual norms, the autotuner's time for every tile of every
 * shape it tunes, and the shape (groups, combos, shuffles, outputs) of every
 * fold it launches.
 */
int fno_profile(fno_ctx *ctx, int on);
int fno_profile_report(fno_ctx *ctx, char *buf, size_t len);
/*
 * Restrict timing to the kernels whose name (with a GEMM's shape, as in
 * fno_profile_report) contains `substr` (NULL or "" = all kernels).  With a filter set, the residual and sigma sweeps are still
 * replayed from hipGraphs: the selected GEMMs are bracketed by event-record
 * nodes inside the graph, read after every replay (in fno_ccsdt, where the
 * next sweep is enqueued before the host waits for the energy, after the
 * following synchronization).  FNO_EINVAL on a null context.
 */
int fno_profile_filter(fno_ctx *ctx, const char *substr);

/*
 * Launch mode of the CCSDT residual sweep (the loop of fno_ccsdt, and the
 * ground-state intermediates of fno_eom / fno_eom_sigma / fno_cc_residual).
 * on = 1 (default): once a sweep has run without allocating device memory, the
 * next one is recorded into a hipGraph (by stream capture on the context's
 * stream and, for the concurrent part of the residual, a side stream joined
 * back into it) and later sweeps replay it; any new allocation in the context
 * discards the recording.
 * on = 0: every launch is issued from the host.  Results are identical in both
 * modes (same kernels, same order).  In either mode fno_ccsdt enqueues the next
 * iteration's sweep before it waits for the current energy; when the loop
 * stops before max_iter, that last sweep's residual is not used.
 */
int fno_set_graphs(fno_ctx *ctx, int on);

/*
 * Ground-state triples residual path (on by default).  With on = 1 every term
 * of the CCSDT triples projection (eq 5 on the triples; the pp-ladder, the
 * hh-ladder, the ring, the one-body and the two T2 driver terms) runs through
 * one fused pass per sweep: each occupied triple's products with the three
 * occupied placements concatenated along K, computed by one MFMA GEMM whose
 * operand tiles are gathered from packed T3/T2 into LDS, followed by one
 * P(a/bc) fold into R3 and one occupied-only operator applied to packed T3.
 * Used for FP64 and FP32 triples products when 3 <= nvir <= 64 (after
 * truncation) and nocc >= 3.  With on = 0, with split-BF16 products, or
 * outside those sizes, every term runs as its own expand / GEMM / fold
 * sequence.  Both paths compute the same residual (to rounding); the EOM
 * sigma vectors always use the per-term path.  Returns FNO_OK.
 */
int fno_set_fused(fno_ctx *ctx, int on);

/*
 * GEMM tile autotuner (off by default).  With on = 1, the first host-launched
 * contraction GEMM of every (precision, M, N, K, operand layout) times each
 * MFMA tile configuration on a scratch output and keeps the fastest for that
 * shape in this context; fno_profile_report lists the choices under "tuned".
 * Tiles change the tiling and split-K slicing, not the k order within a
 * slice, so results agree with the untuned run to rounding.  The setting
 * survives fno_load_hamiltonian and fno_truncate; the tuned choices do not
 * (they belong to the problem's shapes).
 */
int fno_set_autotune(fno_ctx *ctx, int on);

size_t fno_debug_tensor_size(fno_ctx *ctx, const char *name);
int fno_debug_tensor(fno_ctx *ctx, const char *name, double *buf, size_t len);
int fno_debug_gemm(fno_ctx *ctx, fno_prec prec, int tile, long M, long N, long K, int a_kfast, int b_nfast,
                   double alpha, double beta, const double *A, const double *B, double *Cmat);

/*
 * Learned initial guess (CCSDT starting amplitudes).
 *
 * A small network (9 -> 256 -> 256 -> 2, SiLU) maps per-element features of
 * the MP-style T3 guess x (two Jacobi steps from zero: T2 = MP2, T3 from its
 * drivers) -- x and |x| in units of their RMS, the denominator, the six
 * orbital energies -- to a correction of the guess (t3 = x + rms(x) y0) and a
 * shift y1 of that element's Jacobi denominator (kept within [2D, D/2]).
 * With fno_cc_opts.guess = 1 and a model set on the context, fno_ccsdt applies
 * it after its second iteration and evaluates the residual at both starts
 * (that extra evaluation counts as an iteration); the start with the smaller
 * residual norm is kept, so a poor network falls back to the plain guess.
 * Training (FP32, Adam) and inference (single-BF16 operands, FP32
 * accumulation) run on the device with the library's kernels.
 */
typedef struct fno_mlp fno_mlp;
long fno_mlp_num_params(void);                      /* float parameters of the network */
int fno_mlp_create(int hip_device, fno_mlp **out);  /* deterministic initial weights */
void fno_mlp_destroy(fno_mlp *net);
const char *fno_mlp_last_error(const fno_mlp *net);
/* append up to max_samples T3 elements (evenly strided) of a context holding
 * a converged fno_ccsdt: features and targets (converged T3 and dressed
 * one-body diagonal); the context's amplitudes are left as they were */
int fno_mlp_collect(fno_mlp *net, fno_ctx *ctx, long max_samples);
long fno_mlp_samples(const fno_mlp *net);
/* minibatch Adam on the collected samples; loss = mean of the last 20 steps */
int fno_mlp_train(fno_mlp *net, int steps, int batch, double lr, unsigned long seed, double *loss);
int fno_mlp_save(fno_mlp *net, const char *path);   /* raw little-endian float32 with a header */
int fno_mlp_load(fno_mlp *net, const char *path);
/* copy the parameters out (set = 0) or in (set = 1); len = fno_mlp_num_params() */
int fno_mlp_params(fno_mlp *net, float *buf, size_t len, int set);
/* loss and parameter gradient of one batch (host arrays X[B][9], T[B][2]), FP32 */
int fno_mlp_loss_grad(fno_mlp *net, const float *X, const float *T, long B, float *grad, double *loss);
/* outputs Y[n][2] of the BF16 inference path for host features X[n][9] */
int fno_mlp_predict(fno_mlp *net, const float *X, long n, float *Y);
/* copy the first n collected samples out (host arrays X[n][9], T[n][2]) */
int fno_mlp_dataset(fno_mlp *net, float *X, float *T, long n);
/* network used by fno_ccsdt with guess = 1 (not owned; NULL clears) */
int fno_set_guess_model(fno_ctx *ctx, fno_mlp *net);
/* 1 if the last fno_ccsdt kept the learned guess, 0 if not (or none was tried) */
int fno_last_guess_accepted(const fno_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* FNOCC_H */
