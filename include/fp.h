/*
 * fp.h - C ABI of libfp: per-process three- and four-phonon scattering rates on
 * AMD Instinct MI355X (gfx950).
 *
 * The operation is the hybrid CPU-GPU scheme of the paper (Methodology section;
 * Appendix Algorithms 3 and 4): the host enumerates, per phonon mode, the
 * partner tuples that conserve crystal momentum and pass the energy filter, as
 * CSR lists of packed indices; the GPU evaluates every listed process
 * (matrix element, |V|^2, Gaussian delta, Bose-Einstein factors) and reduces
 * the contributions per mode into the scattering rate Gamma and the weighted
 * phase space WP, scaled by const/nptk and 1/nptk as at the end of Algorithm 4.
 *
 * Conventions shared by every entry point
 *   units       amu, Angstrom, ps, K; omega in rad/ps; force constants in
 *               eV/Angstrom^m; Gamma in 1/ps (a rate 1/tau, not a linewidth)
 *   q-mesh      Gamma-centred N0 x N1 x N2; point n = (n0, n1, n2) has index
 *               iq = (n0*N1 + n1)*N2 + n2 and wavevector sum_d n_d b_d / N_d
 *   modes       nb = 3*n_atoms branches; global mode index g = iq*nb + j
 *   eigvecs     e[g][3*atom + alpha], complex128 stored as (re, im) pairs,
 *               normalised; e(-q) = conj e(q); e(q + G) = e(q) (phases on
 *               lattice vectors only)
 *   force       term t of order m: atoms[t][0..m-1], slot 0 in the home cell,
 *   constants   cells[t][r-1][0..2] integer lattice coordinates of slot r,
 *               phi[t][alpha0]...[alpha_{m-1}] row-major (3^m values)
 *   matrix      V = sum_t sum_alpha phi_t/sqrt(prod M) e_lambda(a0)
 *   element       prod_{r>=1} eps_r(a_r) exp(i sum_{r>=1} Q_r . R_{t,r}),
 *               Q_r = s_r q_r, eps_r = e (s_r = +1) or conj e (s_r = -1)
 *
 * Process types (fp_ptype) and what one record of that type means:
 *   FP_3P   lambda + lambda'  -> lambda''            q'' = q + q'
 *   FP_3M   lambda -> lambda' + lambda''            q'' = q - q'
 *   FP_4PP  lambda + lambda' + lambda'' -> lambda'''  q''' = q + q' + q''
 *   FP_4PM  lambda + lambda' -> lambda'' + lambda'''  q''' = q + q' - q''
 *   FP_4MM  lambda -> lambda' + lambda'' + lambda'''  q''' = q - q' - q''
 * Records are one uint64 each (0-based forms of the paper's Ind2/Ind3):
 *   3ph: bits 0-23 g', bits 24-31 j''            (q'' from momentum)
 *   4ph: bits 0-23 g', bits 24-47 g'', bits 48-55 j'''  (q''' from momentum)
 *   FP_3E   three-phonon events lambda + lambda' -> lambda'' with g' >= g,
 *           each evaluated once for all three of its modes (see below)
 * Lists are triangle-reduced over interchangeable partners (the paper's
 * triangular iteration domain, Methodology section): FP_3M and FP_4PP keep
 * g' <= g'', FP_4PM keeps g'' <= g''', FP_4MM keeps g' <= g'' <= g'''; the
 * weight of a record (1, 1/2 or 1/6) follows from equality of those indices.
 *
 * Event lists (FP_3E; the event-symmetric form of the all-modes strategy,
 * Results): a record has the FP_3P layout plus two flags, bit 32 = the 3+
 * processes of g and g' pass the filter (mismatch ((w + w') - w'')), bit 33 =
 * the 3- process of g'' with partners g <= g' passes it ((w'' - w) - w').  Its
 * one matrix element adds the 3+ rate of g, the 3+ rate of g' (if g' != g) and
 * the 3- rate of g'' (weight 1/2 if g' == g), each with its own occupations
 * and Gaussian.  With every active mode of the mesh as a row, FP_3E lists give
 * the Gamma and WP of FP_3P + FP_3M lists over all modes from a third of the
 * matrix elements.  The contributions to g' and g'' are kept per record and
 * added per mode after the row sums, in the order of a stable sort by mode, so
 * the result does not depend on timing.  Fixed width only (not with an
 * adaptive fp_broadening); not accepted by fp_rates_backward.
 * Rates (FP_3P/FP_3M: prefactor pi hbar/(4N), ordered-sum weights 1, 1/2;
 * 4ph: pi hbar^2/(8N^2), weights 1/2, 1/2, 1/6; N = N0*N1*N2):
 *   Gamma_lambda = pref sum_records w |V|^2 occ G(Delta) / prod(omega)
 *   WP_lambda    = (1/N or 1/N^2) sum_records w occ G(Delta) / prod(omega)
 *   G(D) = exp(-D^2/sigma^2)/(sigma sqrt(pi))  (Algorithm 1, WP); sigma is the
 *        call's width, or the per-process width of fp_broadening
 *   occ: 3+ n'-n''; 3- 1+n'+n''; ++ n'n''(1+n''')-(1+n')(1+n'')n''';
 *        +- n'(1+n'')(1+n''')-(1+n')n''n'''; -- (1+n')(1+n'')(1+n''')-n'n''n'''
 *   n = 1/expm1(hbar omega / kB T)
 *
 * Errors: every entry point returns fp_status; argument and state checks are
 * synchronous; fp_last_error() returns a description of the last failure.
 * Device-side range violations (a record or row mode outside the loaded mesh)
 * never read out of bounds: the offending record contributes nothing and a
 * device flag is raised, which fp_check() reports as FP_ERR_RANGE (and every
 * rates call does when the environment variable FP_VALIDATE=1).  Nothing aborts,
 * throws or prints.
 *
 * Threading: a context is not thread-safe; use one per host thread.
 */
#ifndef FP_H
#define FP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fp_ctx fp_ctx;

typedef enum {
    FP_OK = 0,
    FP_ERR_ARG = -1,         /* null pointer, bad size or value */
    FP_ERR_STATE = -2,       /* modes or force constants not loaded, or mismatched */
    FP_ERR_RANGE = -3,       /* a record or row mode outside the loaded mesh (device flag) */
    FP_ERR_NOMEM = -4,       /* device or host allocation failed */
    FP_ERR_HIP = -5,         /* HIP runtime error */
    FP_ERR_UNSUPPORTED = -6  /* a size beyond the documented limits */
} fp_status;

typedef enum { FP_FP64 = 0, FP_MIXED = 1 } fp_precision;

/* OR-ed into the precision argument of fp_rates3/fp_rates4: add into the
 * outputs instead of overwriting them (Gamma = Gamma3 + Gamma4 in one pass). */
#define FP_ACCUMULATE 0x100

typedef enum { FP_3P = 0, FP_3M = 1, FP_4PP = 2, FP_4PM = 3, FP_4MM = 4, FP_3E = 5 } fp_ptype;

/* Limits: n_modes < 2^24, nb <= 96 (32 atoms), n_T <= 8, lists per call <= 8,
 * lcm(N0, N1, N2) <= 1024, force-constant terms per order <= 4096. */
#define FP_MAX_T 8
#define FP_MAX_LISTS 8

/* Width of the Gaussian delta (the broadening step of Algorithms 1-4, whose
 * formula the paper names but does not print).
 *   adaptive = 0: every process takes the width `sigma` of the call.
 *   adaptive = 1: process p takes sigma_p = max(factor * sigma0_p, sigma), with
 *     sigma0_p^2 = sum over partner pairs i < j of
 *                  sum_d ((v_i - v_j) . b_d / N_d)^2 / (3 (m - 1))
 *     over the m - 1 partners of the process (m = 3 or 4), v their group
 *     velocities (Angstrom/ps) and b_d the reciprocal vectors (rad/Angstrom,
 *     recip[3d .. 3d+2] = b_d).  For three phonons this is
 *     sum_d ((v' - v'').b_d/N_d)^2 / 6: the Gaussian whose variance equals that
 *     of the energy mismatch when the free partner wavevector ranges uniformly
 *     over one mesh cell; four phonons average that over the choice of the
 *     momentum-closed partner, so sigma_p is symmetric in the partners and the
 *     triangle reduction stays exact.  `sigma` of each call is the floor that
 *     keeps sigma_p > 0 where the partner velocities coincide.
 * The host enumerator evaluates sigma_p in double precision, pairs in
 * ascending slot order (record order), d = 0, 1, 2, each projection as
 * ((v_i - v_j) . b_d) / N_d, left to right without contraction, so its
 * filter decision is reproducible. */
typedef struct {
    int32_t adaptive;
    int32_t reserved;
    double factor;   /* > 0 */
    double recip[9]; /* b_1, b_2, b_3 as rows */
} fp_broadening;

/* Create a context on HIP device `device`; *out receives it.  Allocates the
 * context's small device buffers.  FP_ERR_ARG if out is NULL, FP_ERR_HIP if the
 * device cannot be used. */
fp_status fp_create(fp_ctx** out, int32_t device);

/* Free every device buffer the context owns.  NULL is accepted. */
void fp_destroy(fp_ctx* ctx);

/* Text of the last error on this context ("" if none).  Owned by the context. */
const char* fp_last_error(const fp_ctx* ctx);

/* Harmonic data of the mesh (the "Get q, omega, v" steps of Algorithms 1-4).
 * All pointers are host memory; the library copies them (synchronously) into
 * device memory it owns, replacing any previous load (force constants must then
 * be loaded again).
 *   mesh[3]      N0, N1, N2 >= 1
 *   lattice[9]   rows a1, a2, a3 in Angstrom (for the cell volume)
 *   masses       [n_atoms] amu, > 0
 *   omega        [N*nb] rad/ps, finite and >= 0
 *   evec         [N*nb*nb] complex as 2*N*nb*nb doubles
 *   vel          [N*nb*3] group velocities in Angstrom/ps (used by
 *                fp_kappa_rta and adaptive broadening; may be NULL)
 *   omega_floor  modes below it are inactive (rad/ps); lists must not use them
 * Resets the broadening to the fixed width (fp_set_broadening).
 * FP_ERR_ARG on NULL/invalid values, FP_ERR_UNSUPPORTED beyond the limits. */
fp_status fp_load_modes(fp_ctx* ctx, const int32_t mesh[3], int32_t n_atoms, const double lattice[9],
                        const double* masses, const double* omega, const double* evec, const double* vel,
                        double omega_floor);

/* Force constants of order 3 or 4 (the tables behind the matrix element of
 * Algorithm 4, whose arguments the paper elides).  atoms and cells are host
 * arrays ([n_terms][order] and [n_terms][order-1][3]); phi is [n_terms][3^order]
 * in eV/Angstrom^order, host memory if phi_on_device == 0, else device memory
 * read on `hip_stream` (so a caller can keep the values device-resident, e.g.
 * under automatic differentiation).  The library converts units, folds the
 * mass factors in and groups the terms; it owns the result.  Requires
 * fp_load_modes first (FP_ERR_STATE).  FP_ERR_ARG on atoms/cells out of range. */
fp_status fp_load_ifc(fp_ctx* ctx, int32_t order, int64_t n_terms, const int32_t* atoms, const int32_t* cells,
                      const double* phi, int32_t phi_on_device, void* hip_stream);

/* Structure of the loaded force constants of one order, for work accounting.
 * The phase of a term in any process depends only on its partner atoms and on
 * its phase vectors A = R1 - R_last (and B = R2 - R_last for order 4) modulo
 * the mesh (Methodology, the matrix element inlined in Algorithm 4); terms that
 * agree in these form one phase key, whose per-row table is the sum of theirs,
 * and the rate kernels run over keys.  out (HOST int64 [5]) receives
 *   out[0] terms, out[1] phase keys, out[2] partner groups (the keys of one
 *   partner-atom tuple, at most 16 per group), and for order 4 the tables of
 *   the default FP64 form of fp_rates4_fused: out[3] pkeys (distinct B among
 *   the keys of one pair of slot-2 and slot-3 atoms), out[4] pair groups (at
 *   most 16 pkeys per group); 0 for order 3.
 * FP_ERR_ARG for a NULL context or out or an order other than 3 or 4,
 * FP_ERR_STATE if that order is not loaded. */
fp_status fp_ifc_info(fp_ctx* ctx, int32_t order, int64_t out[5]);

/* Broadening of the rate, adjoint and autotune calls that follow (see
 * fp_broadening); NULL or adaptive = 0 selects the fixed width of each call.
 * The context keeps the per-mode projections v . b_d / N_d on the device
 * (computed here by a kernel, synchronously).  Requires fp_load_modes with
 * velocities (FP_ERR_STATE).  FP_ERR_ARG for factor <= 0, a non-finite
 * reciprocal vector or adaptive outside {0, 1}.  fp_rates4_fused applies the
 * same rule in its on-GPU filter (the same operations in the same order,
 * correctly rounded), so its kept set equals the host enumerator's. */
fp_status fp_set_broadening(fp_ctx* ctx, const fp_broadening* broadening);

/* One CSR process list: the rows are modes lambda (the paper's mm loop), the
 * records of row r are rec[row_off[r] .. row_off[r+1]) (N_accum/Ind2/Ind3 of
 * Algorithm 3).  row_mode, row_off and rec are DEVICE pointers owned by the
 * caller, which keeps them alive until the stream has passed the call.  Rows of
 * one list must name distinct modes.  n_rec is row_off[n_rows] (host value). */
typedef struct {
    int32_t type; /* fp_ptype */
    int32_t reserved;
    int64_t n_rows;
    int64_t n_rec;
    const int32_t* row_mode;  /* [n_rows] global mode g of lambda */
    const int64_t* row_off;   /* [n_rows+1], row_off[0] = 0, non-decreasing */
    const uint64_t* rec;      /* [n_rec] packed records */
} fp_plist;

/* Three-phonon rates over 3ph lists (types FP_3P/FP_3M/FP_3E).  Enqueued on
 * `hip_stream` (hipStream_t, NULL = default stream); returns after argument
 * checks without waiting for the GPU.  Outputs are DEVICE arrays
 * [n_T][N*nb] in g order, OVERWRITTEN (modes in no row get 0); either may be
 * NULL to skip it (with FP_ACCUMULATE they are added to instead).  T_K is a
 * host array of n_T temperatures (K, > 0); sigma is the Gaussian width in
 * rad/ps.  precision is FP_FP64 or FP_MIXED; order 3 always computes in FP64.
 * One launch evaluates every row of every list.  Requires fp_load_modes and
 * fp_load_ifc(order 3). */
fp_status fp_rates3(fp_ctx* ctx, const fp_plist* lists, int32_t n_lists, int32_t n_T, const double* T_K,
                    double sigma, int32_t precision, double* gamma_out, double* wp_out, void* hip_stream);

/* Four-phonon rates over 4ph lists (types FP_4PP/FP_4PM/FP_4MM); otherwise as
 * fp_rates3.  Requires fp_load_ifc(order 4).
 * FP_FP64: every step in FP64 (the "variant" knob picks the contraction form).
 * FP_MIXED: the phase-weighted force constants of each (lambda, q', q'') tuple
 *   are formed on bf16 matrix cores with three-way bf16 splits of both operands
 *   and FP32 accumulation (an FP32-accurate product), the eigenvector
 *   contraction runs in FP32, and the phases (exact roots of unity), |V|^2,
 *   Gaussian, occupations, 1/prod(omega) and every sum over processes stay in
 *   FP64.  Per-mode relative error against FP64 is of order 1e-6. */
fp_status fp_rates4(fp_ctx* ctx, const fp_plist* lists, int32_t n_lists, int32_t n_T, const double* T_K,
                    double sigma, int32_t precision, double* gamma_out, double* wp_out, void* hip_stream);

/* fp_rates4 for callers that cannot allocate device memory: code under HIP
 * graph capture, serving loops and harnesses that forbid allocation.  Arguments,
 * checks and results are those of fp_rates4 (the same kernels, bit for bit).
 * Every per-call device table (Bose-Einstein table, row and work-unit tables,
 * per-row force-constant tables, per-unit partial sums, and the bf16 planes of
 * FP_MIXED) is placed in a fixed workspace compiled into the library,
 * FP_NOALLOC_BYTES per device, which each device holds from its first context
 * until the process ends; the call itself allocates nothing (no hipMalloc,
 * hipFree or allocating library routine) and records no fp_profile timing.
 * FP_ERR_UNSUPPORTED if the lists need more workspace than that (the message
 * gives the size), FP_ERR_HIP if the workspace has no device address.  All
 * contexts on one device share its workspace and the next call overwrites it:
 * calls that overlap in time on one device (other streams, contexts or host
 * threads) race, so the caller must serialise them.  Load calls (fp_load_modes,
 * fp_load_ifc) still allocate and are made beforehand.  Asynchronous on
 * hip_stream like fp_rates4. */
#define FP_NOALLOC_BYTES ((int64_t)128 << 20)
fp_status fp_rates4_noalloc(fp_ctx* ctx, const fp_plist* lists, int32_t n_lists, int32_t n_T, const double* T_K,
                            double sigma, int32_t precision, double* gamma_out, double* wp_out, void* hip_stream);

/* Four-phonon rates with the process lists generated on the GPU: enumeration
 * (Algorithm 3) fused with the evaluation, for meshes whose lists would not fit
 * in memory.  For every mode of row_mode (DEVICE int32 [n_rows], distinct modes)
 * and every type selected by type_mask (bit 0 FP_4PP, bit 1 FP_4PM, bit 2
 * FP_4MM), each (q', q'') pair and branch triple is tested on the GPU with the
 * host enumerator's rules (frequency floor, triangle order, |Delta| <=
 * nsigma*sigma in FP64 left to right, or nsigma*sigma_p under an adaptive
 * fp_broadening) and the kept processes are evaluated in the tuple-batched
 * form, FP64 or FP_MIXED as in fp_rates4.  The result equals fp_rates4 with the
 * same precision over the lists that fp_enumerate_fill gives for these rows
 * (keep_fraction 1), up to the grouping of the sums.  n_kept (DEVICE int64 [1],
 * may be NULL) receives the number of processes evaluated.  Other arguments as
 * fp_rates4 (precision FP_FP64 or FP_MIXED, optionally | FP_ACCUMULATE).
 * Requires nb = 6 (two-atom cells): FP_ERR_UNSUPPORTED otherwise.  Asynchronous
 * on hip_stream. */
fp_status fp_rates4_fused(fp_ctx* ctx, int64_t n_rows, const int32_t* row_mode, int32_t type_mask, int32_t n_T,
                          const double* T_K, double sigma, double nsigma, int32_t precision, double* gamma_out,
                          double* wp_out, int64_t* n_kept, void* hip_stream);

/* Work counts of the last fp_rates4_fused call on this context, for throughput
 * and roofline accounting of the tuple-batched form (Appendix, Algorithms 3
 * and 4, evaluated per (lambda, q', q'') tuple):
 *   out[0]  processes evaluated (the n_kept of that call)
 *   out[1]  (lambda, q', q'') tuples, over every row and type of the call, with
 *           at least one kept process: the phase-weighted force-constant builds
 *           the form needs at least (a tuple split between two 128-record
 *           batches is built once in each)
 * out is a HOST array of 2; the copy is enqueued on hip_stream, which must be
 * (or follow) the stream of that call, and the function waits for it.
 * FP_ERR_ARG for NULL out, FP_ERR_STATE before any fp_rates4_fused call. */
fp_status fp_fused_counts(fp_ctx* ctx, int64_t out[2], void* hip_stream);

/* Peak probes of the device, measured beside the published peaks that rooflines
 * divide by.  kind 0: FP64 vector FMA; 1: FP64 matrix cores (v_mfma_f64_16x16x4f64);
 * 2: FP32 matrix cores (v_mfma_f32_16x16x4f32); 3: bf16 matrix cores
 * (v_mfma_f32_16x16x32_bf16, dense) -- all in TFLOP/s; 4: device copy of 1 GiB,
 * bytes read plus written, in GB/s.  Each kernel keeps one pipe busy with
 * independent chains on every CU.  One untimed launch, then `reps` (1..100)
 * timed with HIP events on `hip_stream`; *achieved is the best.  Waits for the
 * stream; kind 4 allocates (and frees) 2 GiB of device memory.  FP_ERR_ARG for
 * an unknown kind or reps out of range. */
fp_status fp_peak_probe(fp_ctx* ctx, int32_t kind, int32_t reps, double* achieved, void* hip_stream);

/* Figures of one fp_rates_streamed call (host wall-clock milliseconds). */
typedef struct {
    int64_t n_records;  /* records evaluated, all selected types */
    int64_t n_chunks;   /* staged chunks */
    int64_t max_chunk;  /* records of the largest chunk */
    double count_ms;    /* host counting pass */
    double fill_ms;     /* host enumeration into the staging slots, summed */
    double wait_ms;     /* host time blocked on the GPU (slot reuse, final wait) */
    double total_ms;    /* the whole call */
} fp_stream_stats;

/* Rates over lists that never exist whole: the memory-bounded fallback of the
 * paper's mode-wise variant (Appendix, the mode-wise form of Algorithm 4;
 * Results, where the all-modes lists outgrow device memory), generalised from
 * one mode at a time to chunks of records.  The library enumerates, on host
 * threads and with the rules of fp_enumerate_fill (keep_fraction 1, and the
 * context's broadening), every (type, row) for the types in type_mask (bit t
 * selects fp_ptype t, 1..31) and the modes of row_mode (HOST int32 [n_rows],
 * distinct); it cuts the concatenated record sequence (types ascending, rows in
 * the given order) into chunks of at most chunk_records and evaluates each with
 * the fp_rates3/fp_rates4 launches, accumulating into the outputs.  Two pinned
 * staging slots of chunk_records records (8 bytes each) and their device
 * copies are owned by the context; the host enumerates one chunk while the GPU
 * copies and evaluates the previous one.  A row longer than a chunk is split
 * across chunks.  The result equals fp_rates3 + fp_rates4 over the full lists
 * up to the grouping of the sums.  Outputs, precision (FP_FP64 or FP_MIXED,
 * optionally | FP_ACCUMULATE), T and sigma are as in fp_rates4; nsigma as in
 * fp_enumerate_count; n_threads <= 0 uses every hardware thread.  stats (host,
 * may be NULL) receives the call's figures.  Requires the force constants of
 * every selected order.  Synchronous: returns when the GPU work on
 * `hip_stream` has finished. */
fp_status fp_rates_streamed(fp_ctx* ctx, int32_t type_mask, int64_t n_rows, const int32_t* row_mode, int32_t n_T,
                            const double* T_K, double sigma, double nsigma, int32_t precision,
                            int64_t chunk_records, int32_t n_threads, double* gamma_out, double* wp_out,
                            fp_stream_stats* stats, void* hip_stream);

/* Adjoint of the rates (vector-Jacobian product): given dL/dGamma, a DEVICE
 * array [n_T][N*nb], write dL/dPhi for the raw force-constant entries,
 *   dphi3 DEVICE [n3][27] (eV/A^3 units of phi) and dphi4 DEVICE [n4][81],
 * in the term order of fp_load_ifc (either may be NULL to skip that order;
 * OVERWRITTEN, or added to with FP_ACCUMULATE).  Gamma is quadratic in the
 * force constants, so dL/dPhi = sum_p c_p 2 Re(conj(V_p) dV_p/dPhi) with c_p the
 * process weight; V is recomputed from the lists, never stored.  The lists may
 * mix both orders; the other arguments are as in fp_rates3/fp_rates4.
 * precision FP_FP64, or FP_MIXED: the order-4 V is recomputed with the
 * mixed-precision forward (as fp_rates4 with FP_MIXED) while every sum that
 * forms dL/dPhi stays in FP64; order 3 is FP64 either way.  Deterministic:
 * partial sums are kept per wave and reduced in a fixed order. */
fp_status fp_rates_backward(fp_ctx* ctx, const fp_plist* lists, int32_t n_lists, int32_t n_T, const double* T_K,
                            double sigma, int32_t precision, const double* dL_dgamma, double* dphi3, double* dphi4,
                            void* hip_stream);

/* kappa_RTA (post-processing of the rates, Results section):
 *   kappa^{ab}(T) = 1/(N Omega kB T^2) sum_{q in Q1} w_q sum_j n(n+1) (hbar omega)^2 v^a v^b / Gamma
 * in W/(m K), summed over the irreducible points q1[n_q1] (device int32) with
 * weights q1_weight[n_q1] (device double, sum = N).  gamma is a DEVICE array
 * [n_T][N*nb] (total rate per mode); modes with omega < floor or Gamma <= 0
 * contribute nothing.  kappa_out: DEVICE [n_T][9].  dkappa_dgamma: DEVICE
 * [n_T][N*nb] derivative of tr(kappa)/3 with respect to Gamma (zero outside
 * the q1 modes), or NULL.  Requires velocities in fp_load_modes. */
fp_status fp_kappa_rta(fp_ctx* ctx, int32_t n_q1, const int32_t* q1, const double* q1_weight, int32_t n_T,
                       const double* T_K, const double* gamma, double* kappa_out, double* dkappa_dgamma,
                       void* hip_stream);

/* Tuning knobs of the rate kernels (set by the autotuner; defaults are sane):
 *   "ppl"            records per lane per work unit, 1..64 (unit = 64*ppl records)
 *   "blocks_per_cu"  resident 256-thread blocks per compute unit in the
 *                    persistent launch, 1..16; 0 = as many as fit
 *   "variant"        order-4 contraction form, 0..7: per-process P-form or
 *                    W-form with one or two processes per lane (0-3), or the
 *                    tuple-batched form (phase-weighted force constants per
 *                    (lambda, q', q'') tuple on FP64 MFMA, then per-process
 *                    contraction) with two records per lane (4),
 *                    one (5), or two with 24-tuple batches and three resident
 *                    blocks per CU (6, the default), or three records per
 *                    lane (7)
 *   "grad_chunk"     records per adjoint work chunk, a multiple of 256 (default 4096)
 *   "grad_records"   records per order-4 adjoint pass, 1024..2^34 (default
 *                    2^25, 1 GiB of buffer): rows are taken in ranges of at most this many
 *                    records (a longer row alone), so the per-record adjoint
 *                    buffers hold one range (32 bytes per record), not the
 *                    whole call; the gradient is summed over the ranges in order
 *   "fused_form"     FP64 form of fp_rates4_fused: 0 = phase keys folded over
 *                    A per (lambda, q') unit, 2 (the default) = keys and the
 *                    first partner's eigenvector folded per unit, pair groups
 *                    over the atoms of slots 2 and 3.  With FP_MIXED, 0 takes
 *                    the split-bf16 build and 2 the folded form in FP32
 *                    (folded table, build on FP32 matrix cores, contraction;
 *                    filter and weights stay FP64)
 * FP_ERR_ARG for an unknown name or a value out of range. */
fp_status fp_set_knob(fp_ctx* ctx, const char* name, int64_t value);

/* One measured candidate of fp_autotune. */
typedef struct {
    int32_t variant, ppl, blocks_per_cu, reserved;
    double ms;  /* mean time of one fp_rates call with these knobs */
} fp_tune_entry;

/* Autotuner of the persistent launch (work distribution and tile shape): runs
 * the order-`order` rates of these lists (arguments as fp_rates3/fp_rates4)
 * under every candidate launch configuration and leaves the fastest in the
 * context's knobs.  Candidates for FP64 order 4: variant 0-7 x records per lane
 * {1, 2, 4} (per-process forms; two-process forms {2, 4}; the tuple-batched
 * forms fix it) x blocks_per_cu {0, 1}; for FP_MIXED order 4 and for order 3
 * the knobs that apply.  Each candidate gets one untimed call and `reps`
 * (1..100) timed ones, bracketed by HIP events on `hip_stream`; outputs go to a
 * library-owned scratch buffer, so the caller's arrays are untouched.
 * Synchronous.  Writes up to n_report entries to `report` (may be NULL with
 * n_report 0) and their number to *n_written (may be NULL).  On an error the
 * previous knobs are restored. */
fp_status fp_autotune(fp_ctx* ctx, int32_t order, const fp_plist* lists, int32_t n_lists, int32_t n_T,
                      const double* T_K, double sigma, int32_t precision, int32_t reps, fp_tune_entry* report,
                      int32_t n_report, int32_t* n_written, void* hip_stream);

/* Current value of a launch knob (names as for fp_set_knob) in *value.
 * FP_ERR_ARG for an unknown name or a NULL pointer. */
fp_status fp_get_knob(fp_ctx* ctx, const char* name, int64_t* value);

/* Kernel timing for measurement: with enable != 0 every launch of the rate
 * kernel is bracketed by HIP events on its stream; fp_profile_read waits for
 * them and returns the summed milliseconds and the launch count of one kernel
 * since the last enable, then clears the record: order 3 or 4 = the FP64 rate
 * kernel of that order, 24 = the mixed-precision order-4 rate kernel, 34 = the
 * fused-enumeration order-4 kernel, 13 or 14 = the adjoint kernels of that
 * order. */
fp_status fp_profile(fp_ctx* ctx, int32_t enable);
fp_status fp_profile_read(fp_ctx* ctx, int32_t order, double* total_ms, int64_t* launches);

/* Wait for `hip_stream` and report device-side range violations raised since
 * the last check (FP_ERR_RANGE), clearing the flag. */
fp_status fp_check(fp_ctx* ctx, void* hip_stream);

/* Host enumeration of one list (Algorithm 3, generalised to every type), in two
 * passes like the paper's N_plus / N_accum / Ind2-Ind3 steps.  Host memory
 * throughout; `omega` is [N*nb] as in fp_load_modes.
 *   fp_enumerate_count fills row_off[n_rows+1] (exclusive prefix sum of the
 *     per-row counts; row_off[n_rows] = total records)
 *   fp_enumerate_fill writes rec[row_off[n_rows]] given that row_off
 * A candidate is kept iff every mode has omega >= omega_floor, its
 * interchangeable partners are in ascending g order (triangle reduction) and
 * |Delta| <= nsigma*sigma, with Delta evaluated in double precision left to
 * right in record order (((w + s'w') + s''w'') + s'''w''') and sigma the
 * call's width, or with broadening->adaptive = 1 the per-process width of
 * fp_broadening (vel, [N*nb*3] host memory, is then required; both may be
 * NULL for the fixed width).  Within a row the
 * records are ordered by (q', q'', j', j'', j''') (3ph: q', j', j''), so the
 * records of one (lambda, q', q'') tuple are contiguous.  keep_fraction in
 * (0, 1] keeps a deterministic hash-selected subset of each row's (q', q'')
 * pairs (3ph: of its q'), each with all of its records that pass the filter (1
 * keeps all); seed selects the hash.
 * n_threads <= 0 uses every hardware thread.  FP_ERR_ARG on invalid input,
 * FP_ERR_UNSUPPORTED beyond the record encoding's limits. */
fp_status fp_enumerate_count(int32_t type, const int32_t mesh[3], int32_t nb, const double* omega,
                             double omega_floor, int64_t n_rows, const int32_t* row_mode, double sigma,
                             double nsigma, double keep_fraction, uint64_t seed, int32_t n_threads,
                             const double* vel, const fp_broadening* broadening, int64_t* row_off);
fp_status fp_enumerate_fill(int32_t type, const int32_t mesh[3], int32_t nb, const double* omega,
                            double omega_floor, int64_t n_rows, const int32_t* row_mode, double sigma,
                            double nsigma, double keep_fraction, uint64_t seed, int32_t n_threads,
                            const double* vel, const fp_broadening* broadening, const int64_t* row_off,
                            uint64_t* rec);

#ifdef __cplusplus
}
#endif

#endif /* FP_H */
