/*
 * tdgrad.h -- C ABI of the MI355X (gfx950) library for the two-electron part
 * of the TDA-TDDFT nuclear gradient with range-separated hybrid functionals.
 *
 * The library computes (paper section II.A, eq dE_ao, fourth and fifth terms)
 *
 *   G[A][x] = sum_{mu nu lam sig} Gamma_{mu nu lam sig}    d(mu nu|lam sig)   /dA_x
 *                               + Gamma^lr_{mu nu lam sig} d(mu nu|lam sig)_lr/dA_x
 *
 * with the two-particle densities of eq gamma,
 *   Gamma    = 2 R_{nu mu} R_{lam sig} - alpha R_{sig mu} R_{lam nu}
 *              + 1/2 ( D_{mu nu} P_{lam sig} - alpha/2 D_{mu sig} P_{lam nu} )
 *   Gamma^lr = - beta R_{sig mu} R_{lam nu} - beta/4 D_{mu sig} P_{lam nu},
 * where P is the ground-state density P0, D = P0 + 2 PDelta, R the TDA
 * transition density, (..|..) the Coulomb ERI of eq eri_j and (..|..)_lr the
 * erf(omega r)/r ERI of eq lreri_k, over contracted Cartesian Gaussians of
 * eq cartG with l <= 2 (d shells optionally as real solid harmonics, see
 * tdg_basis_t.spherical).  The derivative of each quartet follows eqs deri,
 * deriv, ti and eriupdate (section II.C); the integrals are evaluated by Rys
 * quadrature in hand-written HIP kernels.  Units: hartree/bohr; the output is
 * dE/dA (the gradient, not the force).
 *
 * It also builds the two-electron part of the Fock-type matrices of the
 * Z-vector equations (section II.B, eqs G_2e and zfock): tdg_fock.
 *
 * Conventions
 *   - Every Cartesian component is normalised to one (primitive, contraction
 *     and angular factor).  Components of a shell are ordered lx descending,
 *     then ly descending: p = x,y,z; d = xx,xy,xz,yy,yz,zz.
 *   - Density matrices are FP64, row-major n_bf x n_bf, in the AO order given
 *     by shell_ao_off (n_bf counts 5 functions per d shell of a spherical basis).
 *     P0 and PDelta must be symmetric (only their symmetric part enters); R is
 *     general.
 *   - All entry points return TDG_OK (0) or a negative tdg_status; they never
 *     abort or throw.  tdg_last_error() returns a thread-local message.
 *   - On error no partial result is written to grad.
 *
 * Ownership
 *   - The caller owns every input and output buffer; the library never frees them.
 *   - A plan owns its device tables and work buffers; free it with tdg_plan_destroy.
 *   - ptr_kind = 1: densities and grad are device pointers on the plan's device;
 *     all work is queued on hip_stream and the gradient is written there, so the caller
 *     synchronises the stream before reading it.  The call itself is not fully
 *     asynchronous: it waits once on the stream (after screening) to read the task
 *     counts that size the class launches, and again when stats are requested, so it
 *     cannot be captured into a HIP graph.
 *     ptr_kind = 0: host pointers; the call returns after the result is copied.
 *   - Calls on one plan must not overlap (a plan holds one set of work buffers).
 */
#ifndef TDGRAD_H
#define TDGRAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TDG_OK = 0,
    TDG_EINVAL = -1,        /* null pointer, negative size, index out of range */
    TDG_EUNSUPPORTED = -2,  /* l > 2, too many primitives, unsupported option */
    TDG_ENOMEM = -3,        /* device or host allocation failed */
    TDG_EDEVICE = -4,       /* a HIP runtime call failed */
    TDG_ESTATE = -5         /* plan in an unusable state */
} tdg_status;

typedef struct tdg_plan tdg_plan_t; /* opaque */
typedef struct tdg_mlp tdg_mlp_t;   /* opaque: quartet-contribution estimator */

/* Basis and geometry (host pointers, copied by tdg_plan_create). */
typedef struct {
    int32_t n_atoms;
    const double *coords;          /* [n_atoms][3], bohr */
    int32_t n_shells;
    const int32_t *shell_atom;     /* [n_shells] atom index */
    const int32_t *shell_l;        /* [n_shells] angular momentum, 0..2 */
    const int32_t *shell_nprim;    /* [n_shells] contraction degree, 1..TDG_MAX_NPRIM */
    const int32_t *shell_prim_off; /* [n_shells] offset into exps/coefs */
    const int32_t *shell_ao_off;   /* [n_shells] first AO index of the shell */
    int32_t n_prims;
    const double *exps;            /* [n_prims] Gaussian exponents zeta > 0 */
    const double *coefs;           /* [n_prims] contraction coefficients of unnormalised primitives */
    int32_t spherical;             /* 0: Cartesian functions, ncart(l) per shell (eq cartG);
                                      1: d shells as the five real solid harmonics (section II.C
                                      names both forms), order xy, yz, z^2, xz, x^2-y^2 (m = -2..2),
                                      each normalised to one; s and p shells are the same in both.
                                      shell_ao_off, the density and the Fock-type matrix then count
                                      2l+1 functions per d shell; the library works on the Cartesian
                                      functions internally (densities transformed on entry, the
                                      Fock-type matrix on exit; the gradient is unchanged by it) */
} tdg_basis_t;

#define TDG_MAX_NPRIM 16

/* Method parameters (section II.A: alpha is the short-range HF fraction,
 * alpha + beta the long-range one, omega the range-separation parameter;
 * section II.E: density-multiplied Schwarz threshold). */
typedef struct {
    double omega;       /* bohr^-1, > 0 when terms has bit 4 */
    double alpha;       /* full-range exchange fraction */
    double beta;        /* long-range exchange fraction */
    double schwarz_tol; /* skip a quartet when Q_ab Q_cd M_abcd < schwarz_tol; 0 = no screening */
    int32_t precision;  /* 0: FP64 throughout; 1: mixed -- 2D integrals, derivative products and
                           per-primitive partial sums in FP32 for quartets routed to FP32; Rys
                           roots, weights, prefactors and all accumulation in FP64.  A quartet
                           is routed to FP32 when bound * f_ab * f_cd < mixed_tau64 and every
                           primitive exponent sum is < mixed_p64, with f the square root of
                           the pair's largest primitive exponent (the scale a centre
                           derivative adds to an integral); classes where FP64 measures faster
                           run their FP32-routed quartets in FP64 (see autotune) */
    int32_t terms;      /* bit 1: Coulomb-type (J) terms, bit 2: full-range exchange (alpha),
                           bit 4: long-range exchange (beta); 7 = all */
    int32_t autotune;   /* 1: on the plan's first tdg_grad_jk call, time the kernel variants
                           of each angular class on that call's tasks (every k-th task of a
                           class holding more than 2^21) and keep the fastest, then the launch
                           shape of the kept variant (4, 8, 16 or 32 blocks per compute unit);
                           in mixed mode also run a class's FP32-routed quartets in FP64 (one
                           launch for the class) when that measures faster than the split */
    int32_t kernel_variant; /* -1: per-class default or autotuned choice; 0: team-per-quartet
                               kernels (FP64: vertical recursion + transfers; FP32: direct
                               four-centre derivative tables); 1: wavefront-per-quartet kernels;
                               2: team-per-quartet kernels with direct four-centre base tables
                               and the collapsed contraction; 3, 4: as 0, 2 with one lane per
                               (quartet, range) looping over the Rys roots, for classes with
                               <= 27 components (elsewhere 0, 2 run).  The transfer form (0, 3)
                               is offered only for classes without p or d functions on B and D
                               (its A->B and C->D transfers lose accuracy for tight exponents)
                               and whose kernel needs no scratch memory; elsewhere 2 (4) runs
                               instead.  Stats report the variant that ran. */
    double mixed_tau64; /* mixed mode: FP32 only when bound * f_ab * f_cd is below this (the
                           Python binding's default is 0.1); INFINITY routes on class timing
                           alone, which is fastest but leaves the error unbounded by the
                           router: it scales with the largest quartet contributions */
    double mixed_p64;   /* mixed mode: pairs with a primitive exponent sum >= this stay FP64
                           (INFINITY: no exponent cap; the Python binding's default is 1e4) */
    int64_t max_tasks;  /* screened quartets held at once (chunking of large systems); 0 = 2^31 */
    int32_t screening;  /* 0: density-multiplied Schwarz bound only (section II.E); an attached
                           estimator is ignored.  1: the same bound, then the learned veto of the
                           estimator attached with tdg_plan_set_screen_model (a call without one
                           attached fails with TDG_ESTATE) */
    int32_t deterministic; /* 1: bitwise repeatable gradients: tasks in a fixed order (no fused
                              screening), per-class default kernel variants (no autotuning; an
                              explicit kernel_variant still applies), each quartet's twelve values
                              reduced over its lanes in a fixed order and summed per atom in task
                              order (fixed blocks of tasks, then the blocks in order) instead of by
                              floating-point atomics.  Slower; single-molecule calls of a batch run
                              one after another.  0: atomics (default) */
    int32_t ml_min_components; /* screening = 1: the learned veto applies only to classes with at
                                  least this many Cartesian components (their quartets cost far
                                  more than one network evaluation); 0 = every class */
    int32_t streams;    /* the class kernels of a call run side by side on this many HIP streams
                           (the caller's stream and streams - 1 of the plan's, joined back into
                           the caller's stream before the call's last step); 1 = all on the
                           caller's stream, 0 = 4 (the maximum) */
} tdg_params_t;

/* Per-call statistics (optional output). */
typedef struct {
    int64_t quartets;          /* shell quartets evaluated after screening */
    int64_t prim_quartets;     /* primitive quartets of those */
    int64_t candidates;        /* shell quartets tested by the exact screening bound */
    int64_t class_quartets[21];/* per angular class, in the library's class order */
    int64_t class_prim_quartets[21];
    double class_ms[21];       /* derivative-kernel time per class (HIP events on the call's stream) */
    int32_t class_variant[21]; /* kernel variant per class (kernel_variant numbering): bits 0-2
                                  the FP64 list's, bits 3-5 the FP32 list's; bit 6 set: the
                                  FP32-routed quartets ran in FP64; bits 8-15 and 16-23: the
                                  launch shape of the FP64 and FP32 kernels, blocks per compute
                                  unit (chosen by the autotuner among 4, 8, 16, 32; default 16) */
    int64_t fp32_quartets;     /* mixed mode: quartets evaluated with FP32 2D integrals (those
                                  routed to FP32 in classes that run the FP32 kernels) */
    int64_t ml_skipped;        /* quartets vetoed by the contribution estimator */
    int64_t chunks;            /* number of task-list chunks the call was split into */
    int64_t class_fp32_quartets[21];
    double ms_total;           /* wall time of the call (host clock, synchronised) */
    double ms_kernels;         /* summed derivative-kernel time (HIP events), all chunks */
} tdg_stats_t;

/* Build a plan for one geometry and basis on HIP device `device` (section II.C: the
 * contracted Cartesian functions of eq cartG and the presorted shell-pair lists of the
 * paper's design; section II.E: the Schwarz factors of the screening bound):
 * normalisation, shell-pair tables, Schwarz factors Q_ab = sqrt(max (mu nu|mu nu)),
 * pair lists sorted by class, contraction degree and Q.  The plan copies the basis.
 * Errors: TDG_EINVAL (bad pointers/indices), TDG_EUNSUPPORTED (l > 2 or
 * nprim > TDG_MAX_NPRIM), TDG_ENOMEM, TDG_EDEVICE. */
int tdg_plan_create(const tdg_basis_t *basis, const tdg_params_t *params, int device,
                    tdg_plan_t **out);

/* Two-electron gradient for one set of densities (section II.A, eq dE_ao terms 4-5 with
 * the densities of eq gamma; derivatives per section II.C eqs deri, deriv, ti,
 * eriupdate; screening per section II.E).
 * P0, PDelta, R: [n_bf][n_bf] FP64 row-major; grad: [n_atoms][3] FP64,
 * overwritten.  ptr_kind 0: host pointers (synchronous); 1: device pointers on
 * hip_stream (a hipStream_t, NULL = default stream; see Ownership for the one wait
 * on the stream inside the call).  stats may be NULL; when given, the call
 * synchronises the stream to fill it.
 * Errors: TDG_EINVAL, TDG_ENOMEM, TDG_EDEVICE, TDG_ESTATE. */
int tdg_grad_jk(tdg_plan_t *plan, const double *P0, const double *PDelta, const double *R,
                int32_t ptr_kind, void *hip_stream, double *grad, tdg_stats_t *stats);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): tdg_grad_jk with device pointers (P0, PDelta, R,
 * grad on the plan's device, work queued on hip_stream) that calls no hipMalloc, hipFree or
 * other allocating routine.  The screened task list of each chunk goes to a static device
 * buffer of 8,388,608 tasks (64 MiB, one per GPU the library runs on, held until the process
 * ends); a larger task list runs as several chunks.  The plan's current kernel variants are
 * used (tuned by an earlier tdg_grad_jk call, else the per-class defaults): no autotuning and
 * no fused screening here.  Calls on one GPU share its buffer, whatever the plan: calls that
 * overlap on one GPU race (the caller serialises them).  Like tdg_grad_jk it waits once on
 * the stream to read the task counts.
 * Errors: TDG_EINVAL (null pointers); TDG_EUNSUPPORTED for a deterministic plan, a plan with
 * screening = 1, or when the survivors of one bra pair in one class exceed the buffer;
 * TDG_EDEVICE. */
int tdg_grad_jk_noalloc(tdg_plan_t *plan, const double *P0, const double *PDelta, const double *R,
                        void *hip_stream, double *grad, tdg_stats_t *stats);

/* Gradients of n molecules in one pass (the computation of tdg_grad_jk for each):
 * per molecule density preparation and the screening count pass, one host
 * synchronisation for all task counts, the fill passes into one task list, then one
 * launch graph of the (molecule, class) kernel items, largest expected work first, spread
 * over the lead plan's streams (see streams) so that the GPU runs small items beside large
 * ones.  plans[m] with densities P0[m], PDelta[m], R[m] writes grad[m] ([n_atoms(m)][3]).
 * All plans must share device, omega, alpha, beta, terms, precision and deterministic, and
 * appear once.  Work buffers of the batch belong to plans[0]; its kernel variants for
 * batched calls (autotuned on the molecule with the most quartets of each class) are kept
 * separately from single calls.  Deterministic plans run one molecule after another.
 * Errors: as tdg_grad_jk. */
int tdg_grad_jk_batch(int32_t n, tdg_plan_t *const *plans, const double *const *P0,
                      const double *const *PDelta, const double *const *R, int32_t ptr_kind,
                      void *hip_stream, double *const *grad, tdg_stats_t *stats);

/* ---------------------------------------------------------------------------
 * Learned screening.  A 10 -> 64 -> 64 -> 1 ReLU network predicts, from features of
 * a shell quartet that passed the density-multiplied Schwarz bound (log Q_ab,
 * log Q_cd, log of the density-block product, extreme primitive exponent sums of
 * both pairs, pair distance, angular momentum, bond lengths), log10 of the largest
 * of its twelve gradient contributions (scaled by 1/10).  Forward and backward
 * passes use BF16 matrix-core instructions with FP32 accumulation; weights are
 * FP32 (tdg_mlp_nweights() floats: W1[64][16], b1[64], W2[64][64], b2[64],
 * W3[64], b3).  Used as a veto on top of the Schwarz screening, for the callers
 * that train it on contributions this library generates (tdg_collect).
 * ------------------------------------------------------------------------- */
int tdg_mlp_create(int device, uint64_t seed, tdg_mlp_t **out);   /* seeded initial weights */
int tdg_mlp_destroy(tdg_mlp_t *model);
int tdg_mlp_nweights(void);
int tdg_mlp_set_weights(tdg_mlp_t *model, const float *w_host);   /* resets the Adam state */
int tdg_mlp_get_weights(const tdg_mlp_t *model, float *w_host);
/* predictions for n samples: X device [n][16] FP32, out device [n] FP32 (async on stream) */
int tdg_mlp_forward(const tdg_mlp_t *model, const float *X, int64_t n, float *out, void *hip_stream);
/* loss mean((pred - Y)^2) and its gradient (host [nweights]) for n device samples; no update */
int tdg_mlp_grad(tdg_mlp_t *model, const float *X, const float *Y, int64_t n, float *grad_host,
                 float *loss_host, void *hip_stream);
/* one Adam step (beta 0.9/0.999) on a batch of n device samples; loss_host may be NULL */
int tdg_mlp_train_step(tdg_mlp_t *model, const float *X, const float *Y, int64_t n, float lr,
                       float *loss_host, void *hip_stream);

/* Attach an estimator to a plan (NULL detaches): a screened quartet is skipped when the
 * predicted log10 contribution is below log10_threshold and its screening bound is below
 * tau_hi (the rigorous bound keeps large quartets).  The model must outlive its use.
 * Applies to tdg_grad_jk (not to batched calls). */
int tdg_plan_set_screen_model(tdg_plan_t *plan, const tdg_mlp_t *model, double log10_threshold,
                              double tau_hi);

/* Training data generated by the method itself: screens the quartets of one FP64 plan,
 * evaluates every surviving quartet's twelve gradient contributions, and writes features
 * (device [cap][16]) and targets (device [cap], log10 of the largest contribution / 10)
 * of every stride-th surviving quartet; *n_out = samples written (<= cap). */
int tdg_collect(tdg_plan_t *plan, const double *P0, const double *PDelta, const double *R,
                int32_t ptr_kind, void *hip_stream, float *feat, float *target, int64_t cap,
                int64_t stride, int64_t *n_out);

/* Move the plan to a new geometry (same basis, shells on the same atoms): coords
 * [n_atoms][3] bohr, host.  Rebuilds every geometry-dependent table (primitive-pair
 * centres and factors, Schwarz factors and the sorted pair lists, section II.C/II.E) and
 * keeps the kernel variants chosen by the autotuner, the learned region capacities of
 * the fused screening and an attached estimator.  For finite-difference checks and
 * geometry steps.  Errors: TDG_EINVAL (null pointers, non-finite coordinates),
 * TDG_ENOMEM, TDG_EDEVICE; on error the plan is unchanged. */
int tdg_plan_update_coords(tdg_plan_t *plan, const double *coords);

/* Verification of the screening (section II.E): the shell quartets that pass the
 * density-multiplied Schwarz bound for these densities, as the class kernels would
 * receive them (learned veto not applied).  quartets: host [cap][4] int32, caller shell
 * indices (a, b | c, d) of every stride-th surviving unique quartet (stride >= 1) in the
 * library's canonical orientation (l_a >= l_b, l_c >= l_d, pair class of ab >= that of
 * cd).  Order: the list is built in chunks of bra pairs (each holding at most 2^27
 * survivors; one chunk for all but large systems); within a chunk by class, then the
 * precision list of the route (FP64, FP32; one list unless the plan is mixed), bra pair,
 * ket pair.  *n_out = the number of survivors; at most cap are written, and cap = 0 only
 * counts them.  Densities as in tdg_grad_jk.  Synchronous.
 * Errors: TDG_EINVAL, TDG_ENOMEM, TDG_EDEVICE. */
int tdg_screen_list(tdg_plan_t *plan, const double *P0, const double *PDelta, const double *R,
                    int32_t ptr_kind, void *hip_stream, int32_t *quartets, int64_t cap, int64_t stride,
                    int64_t *n_out);

/* Verification of the class kernels one quartet at a time (eq dE_ao terms 4-5 restricted
 * to one unique shell quartet, with its permutation degeneracy): for n shell quartets
 * quartets [n][4] (host int32, caller shell indices in any order within and between
 * the two pairs) writes out [n][4][3] (host FP64): the contributions to the gradient
 * of the atoms of shells a, b, c, d as listed (hartree/bohr).  No screening.
 * precision 0: FP64 kernels; 1: the FP32-table kernels of the mixed route.  Each
 * quartet runs in the plan's kernel variant of its class.  Synchronous.
 * Errors: TDG_EINVAL (bad indices), TDG_ENOMEM, TDG_EDEVICE. */
int tdg_quartet_contribs(tdg_plan_t *plan, const double *P0, const double *PDelta, const double *R,
                         int32_t ptr_kind, void *hip_stream, int64_t n, const int32_t *quartets,
                         int32_t precision, double *out);

/* Two-electron part of the Fock-type matrix of section II.B (eq G_2e; eq zfock for the
 * Z-vector and CPHF products), for the plan's basis and geometry:
 *   F_{mu nu} = sum_{lam sig} Bs_{lam sig} [ cJ (mu nu|lam sig) + cK (mu lam|nu sig)
 *                                            + cKlr (mu lam|nu sig)_lr ],
 * Bs = (B + B^T)/2, (|)_lr the erf(omega r)/r integral of eq lreri_k with the plan's omega.
 * eq G_2e is (cJ, cK, cKlr) = (2, -alpha, -beta) with B = PDelta (symmetric); eq zfock is
 * (4, -2 alpha, -2 beta), its two exchange orderings summing to twice K(Bs).  The
 * exchange-correlation kernel term of both equations is not part of this call.
 * B, F: [n_bf][n_bf] FP64 row-major (F overwritten, symmetric).  ptr_kind 0: host
 * pointers (synchronous); 1: device pointers on hip_stream (the call waits once on the
 * stream to read the screening counts).  Screening: a unique shell quartet is skipped when
 * Q_ab Q_cd times the largest |Bs| element of the six blocks it is contracted with is
 * below the plan's schwarz_tol (0: no screening); one-centre quartets are kept.
 * relative = 1 screens as if B were first scaled to a largest |Bs| element of one and F
 * scaled back (the threshold becomes schwarz_tol max|Bs|): the normalisation of the
 * Krylov vectors before the Fock build discussed in section III.B, which keeps the shrinking
 * vectors of late Z-vector iterations from being screened away; 0 = absolute.  FP64
 * throughout, whatever the plan's precision.  The class kernels run side by side on the
 * plan's streams as in tdg_grad_jk (joined back into hip_stream before the last step).
 * The matrix is summed with FP64 atomics, so it is not bitwise repeatable (the plan's
 * deterministic setting applies to gradients only).
 * stats may be NULL; when given, quartets,
 * prim_quartets, candidates, class_quartets, class_prim_quartets, class_ms (each Fock class
 * kernel timed alone on hip_stream: the call waits after every launch), chunks, ms_kernels
 * and ms_total are filled.
 * Errors: TDG_EINVAL (null pointers, non-finite coefficients, cKlr != 0 with omega <= 0,
 * relative not 0 or 1),
 * TDG_ENOMEM, TDG_EDEVICE. */
int tdg_fock(tdg_plan_t *plan, const double *B, int32_t ptr_kind, void *hip_stream, double cJ,
             double cK, double cKlr, int32_t relative, double *F, tdg_stats_t *stats);

/* Z-vector (coupled-perturbed) equations of section II.B, eq cphf: (d - A) Z = L with
 * d_ai = eps_i - eps_a and A of eq cphf_a without its exchange-correlation kernel term,
 * solved by the Krylov subspace method of the same section: b0 = d^-1 L, orthonormal
 * subspace vectors (each normalised before its Fock build), the products
 * A b = C_v^T F(C_v b C_o^T) C_o of eqs sigma and zfock with F = tdg_fock(B; cJ, cK, cKlr,
 * relative) -- eq zfock is (cJ, cK, cKlr) = (4, -2 alpha, -2 beta) -- and the subspace
 * equations (delta_ij - b_i . d^-1 A b_j) a_j = delta_i0 |b0| solved on the host, until
 * |d^-1 L - (I - d^-1 A) Z| <= tol |d^-1 L| or max_iter products.
 * C_occ [n_bf][n_occ], C_vir [n_bf][n_vir]: orbital coefficients in the plan's functions,
 * row-major; eps_occ [n_occ], eps_vir [n_vir] with every occupied energy below every virtual
 * one; L, Z [n_vir][n_occ] row-major.  Host pointers; synchronous (the plan's device, its
 * default stream); *iterations = products evaluated, *residual = the final relative
 * residual (either may be NULL).  Errors: TDG_EINVAL, TDG_ENOMEM, TDG_EDEVICE, TDG_ESTATE
 * (singular subspace matrix). */
int tdg_zvector(tdg_plan_t *plan, int32_t n_occ, int32_t n_vir, const double *C_occ,
                const double *C_vir, const double *eps_occ, const double *eps_vir, const double *L,
                double cJ, double cK, double cKlr, int32_t relative, double tol, int32_t max_iter,
                double *Z, int32_t *iterations, double *residual);

/* Release a plan and its device memory (NULL is accepted). */
int tdg_plan_destroy(tdg_plan_t *plan);

/* Number of streams the class kernels of later calls spread over: 1 .. the plan's streams
 * parameter (e.g. 1 to time every kernel alone).  Errors: TDG_EINVAL. */
int tdg_plan_set_streams(tdg_plan_t *plan, int32_t streams);

/* Number of basis functions and atoms of a plan (for callers sizing buffers). */
int tdg_plan_dims(const tdg_plan_t *plan, int32_t *n_bf, int32_t *n_atoms, int32_t *n_shells);

/* Schwarz factor of every shell pair, copied to host: Q[a*(a+1)/2 + b] for a >= b
 * (shell indices of the caller's basis).  Q must hold n_shells*(n_shells+1)/2 doubles. */
int tdg_plan_schwarz(const tdg_plan_t *plan, double *Q);

/* Rys quadrature rule used by the kernels (for verification): for n roots
 * (1..5) and argument T >= 0, u[i] (= t_i^2, ascending) and w[i].  Evaluated
 * on the device of the plan-less default device 0; u and w are host arrays of n. */
int tdg_rys_rule(int32_t n, double T, double *u, double *w);

/* Thread-local description of the last failure ("" if none). */
const char *tdg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TDGRAD_H */
