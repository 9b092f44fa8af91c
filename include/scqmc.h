/*
 * scqmc.h -- C ABI of the MI355X (gfx950) stochastic SC-MRCI / SC-NEVPT2
 * local-energy engine.
 *
 * Method: Mahajan, Blunt, Sabzevari, Sharma, "Multireference configuration
 * interaction and perturbation theory without reduced density matrices"
 * (arXiv:1909.06935).  The library samples the strongly contracted (SC) wave
 * function  psi_SC = sum_{k,l} c_l^(k) |psi_l^(k)>,  |psi_l^(k)> = P_l^(k) H |phi0>
 * (Theory, "Overview of contraction schemes"; the state from S_0^(0) is phi0
 * itself) with a rejection-free continuous-time walk over Slater determinants
 * ("SC-MRCI(s)"), evaluating for every walker the local energy of eq:locE and,
 * in NEVPT2 mode, the Dyall-Hamiltonian local energy needed by eq:nevpt.
 *
 * Conventions
 *  - Spatial orbitals are ordered [core | active | virtual]; N <= 128,
 *    n_act <= 32, at most 2*n_virt <= 65534 virtual spin-orbitals.
 *  - A determinant is two spin strings, alpha then beta, each of
 *    words = ceil(N/64) little-endian uint64 words; bit i of word w is orbital
 *    64*w + i.  Arrays of determinants are [n][2][words].
 *  - Core orbitals are doubly occupied in every determinant the method uses
 *    (frozen core, "Implementation" section); at most two electrons sit in
 *    virtual orbitals (the first-order interacting space).
 *  - Class (the subspace S_l^(k), l = occupied virtual spin-orbitals): 0 for
 *    the active space; virtual spin-orbital s = a + sigma*V (a in [0,V),
 *    sigma = 0 alpha / 1 beta); one virtual electron: 1 + s; two, s1 < s2:
 *    1 + 2V + s1*2V - s1*(s1+1)/2 + (s2 - s1 - 1).  n_classes = 1 + 2V + C(2V,2).
 *  - Hamiltonian  H = e_const + sum h_pq a+_p a_q + 1/2 sum (pq|rs) a+_p a+_r a_s a_q
 *    (chemist notation, real orbitals, 8-fold symmetric (pq|rs)).
 *  - Phases: a single p->q has sign <m|a+_q a_p|n>; a double removing P1<P2
 *    and adding Q1<Q2 (spin-orbital order: all alpha, then all beta) has sign
 *    <m|a+_Q1 a+_Q2 a_P2 a_P1|n>.
 *
 * Ownership: host arrays are read during the call and copied; the library
 * keeps no caller pointer.  Device pointers (eval_snapshot) must live on the
 * context's device and are written asynchronously on the context's stream.
 * Errors: every function returns scqmc_status; SCQMC_OK == 0.  The message of
 * the last failure on a context is scqmc_last_error().  No exception crosses
 * the ABI.  One context per host thread; contexts share nothing.
 *
 * Call order: set_space -> set_integrals_* -> set_reference -> set_sc_coeffs
 * -> [set_dyall] -> [set_options] -> init_walkers -> sample / read_* ...
 * Calling out of order returns SCQMC_E_STATE.
 */
#ifndef SCQMC_H
#define SCQMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SCQMC_OK = 0,
    SCQMC_E_INVALID_ARG = -1,  /* bad size, bad determinant, wrong length, ... */
    SCQMC_E_STATE = -2,        /* called out of order */
    SCQMC_E_UNSUPPORTED = -3,  /* outside the supported sizes */
    SCQMC_E_OOM = -4,          /* device allocation failed */
    SCQMC_E_DEVICE = -5,       /* HIP runtime error */
    SCQMC_E_NUMERIC = -6       /* non-finite input, or a non-finite / zero-rate walker */
} scqmc_status;

typedef struct scqmc_ctx scqmc_ctx;

typedef struct {
    int32_t n_orb, n_core, n_act;
    int32_t n_elec_a, n_elec_b;   /* total alpha / beta electrons (core included) */
} scqmc_space;

typedef struct {
    double eps_screen;    /* doubles with |<rs||pq>| <= eps_screen are left out of the
                             neighbour set ("heat-bath" screening, Implementation
                             section); 0 = keep every double */
    int32_t mode;         /* 0: local energy (SC-MRCI); 1: also the Dyall local energy and
                             the per-class NEVPT2 sums of eq:nevpt (needs set_dyall) */
    int32_t precision;    /* 0: FP64.  1: precision form -- the off-diagonal Slater-Condon
                             elements and the terms of every overlap psi(m) are computed
                             in FP32 from FP32 copies of the integrals (made on first use)
                             and summed in FP64; H_nn, psi(n) of the walker, the
                             accumulators and the estimators stay FP64.  Changing it
                             invalidates placed walkers.  Other values -> INVALID_ARG. */
    int64_t burn_in;      /* global step index from which estimators accumulate */
    int64_t block_len;    /* steps per kernel launch inside scqmc_sample (0 = all) */
} scqmc_options;

typedef struct {
    double e_var, e_var_err;    /* eq:vmc: sum t E_L / sum t; delete-one jackknife over min(W, 256)
                                   groups of consecutive walkers */
    double a0_sq, a0_sq_err;    /* CAS residence fraction (Davidson section) */
    double e_ref;               /* E_0^(0) as given to set_dyall (0 if not given) */
    double davidson;            /* (1 - a0^2)(e_var - e_ref), Davidson correction equation */
    double e2, e2_err;          /* SC-NEVPT2 E^(2) (eq:nevpt2e2) from the sampled class sums;
                                   error: delete-one jackknife over min(W, 16) groups of
                                   consecutive walkers, each with its own class sums (NaN
                                   when W = 1 or a leave-one-out estimate is undefined) */
    int64_t n_steps_accumulated, n_walkers;
} scqmc_estimates;

/* Stochastic optimisation of the SC coefficients ("SC-MRCI(s)": AMSGrad on
 * the sampled energy gradient).  With rho the walk's distribution,
 *   g_l = < [class(n) = l] (E_L(n) - E) >_rho / c_l
 * (the derivative overlap <n|psi_l>/<n|psi> is [class(n) = l]/c_l), which
 * needs only the per-class sums of t and t*E_L the walk accumulates.  c0 is
 * held fixed (the energy does not depend on the overall scale); classes with
 * c_l = 0 stay at 0.  AMSGrad (Reddi, Kale, Kumar 2018): m <- b1 m + (1-b1) g,
 * v <- b2 v + (1-b2) g^2, vmax <- max(vmax, v), c <- c - lr m/(sqrt(vmax)+eps). */
typedef struct {
    double lr, beta1, beta2, eps;
    int64_t steps_per_iter;     /* walk steps whose samples make one gradient */
    int64_t equil_steps;        /* steps walked, not sampled, after each update */
} scqmc_amsgrad;

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to
 * enqueue on, or NULL for a stream the context creates and owns. */
scqmc_status scqmc_create(int device, void *hip_stream, scqmc_ctx **out);
void scqmc_destroy(scqmc_ctx *ctx);
const char *scqmc_last_error(const scqmc_ctx *ctx);

/* Orbital partition and electron counts.  Requires n_core <= n_elec_a,b,
 * n_elec_a,b - n_core < n_act (a hole must exist), N <= 128, n_act <= 32. */
scqmc_status scqmc_set_space(scqmc_ctx *ctx, const scqmc_space *space);

/* Integrals in Cholesky form: h1 [N*N] (symmetric), chol [n_chol][N][N]
 * (each slice symmetric), (pq|rs) = sum_L chol[L][p][q] chol[L][r][s].
 * The library forms the core-folded one-body operator
 * h_eff_pq = h_pq + sum_i (2(pq|ii) - (pi|iq)), the core energy, and the
 * two-electron integrals over active+virtual orbitals on the device. */
scqmc_status scqmc_set_integrals_chol(scqmc_ctx *ctx, const double *h1, const double *chol, int32_t n_chol,
                                      double e_const);
/* Same with a dense [N^4] chemist-notation tensor (pq|rs) at eri[((p*N+q)*N+r)*N+s]. */
scqmc_status scqmc_set_integrals_dense(scqmc_ctx *ctx, const double *h1, const double *eri, double e_const);

/* Active-space reference phi0 (selected CI / CASCI, the "Implementation"
 * section): n_det determinants [n_det][2][words] and coefficients.  Each
 * determinant must have a full core, no virtual electron and the right
 * electron counts; duplicates are rejected.  phi0 need not be normalised.
 * The library builds a device hash table of the determinants (constant-time
 * overlap, "SC-MRCI(s)") and two derived tables that list, for every
 * determinant with one or two active electrons removed, the reference
 * determinants it came from. */
scqmc_status scqmc_set_reference(scqmc_ctx *ctx, int64_t n_det, const uint64_t *dets, const double *coeff);

/* SC coefficients: c0 for phi0 and c_cls[n] for classes 1..n_classes-1, in
 * class-id order (n must equal n_classes - 1, else SCQMC_E_INVALID_ARG).
 * Zero coefficients are allowed (the class is then never visited). */
scqmc_status scqmc_set_sc_coeffs(scqmc_ctx *ctx, double c0, const double *c_cls, int64_t n);

/* Dyall Hamiltonian of "SC-NEVPT2(s)": virtual orbital energies eps_virt[V]
 * (the orbitals are taken as the semicanonical virtuals, so the virtual part
 * of H_D is diagonal) and E_0^(0).  H_D = sum_a eps_a n_a + H_0, where H_0 is
 * the core-averaged active-space Hamiltonian (e_const and core energy
 * included, so <phi0|H_D|phi0> = <phi0|H|phi0>).  Required for mode 1. */
scqmc_status scqmc_set_dyall(scqmc_ctx *ctx, const double *eps_virt, double e0_ref);

/* E_0^(0) = <phi0|H|phi0> / <phi0|phi0>, the zeroth-order energy of
 * "SC-NEVPT2(s)", evaluated on the device (the local energy of every reference
 * determinant over its active-space neighbours, summed on the host with
 * weights phi0(d)^2 in reference order).  Needs set_reference; writes *e0.
 * SCQMC_E_NUMERIC if a local energy is not finite. */
scqmc_status scqmc_reference_energy(scqmc_ctx *ctx, double *e0);

/* Spin-summed active one-particle density of phi0, normalised:
 * gamma[t*n_act + u] = sum_sigma <phi0|a+_{t sigma} a_{u sigma}|phi0> / <phi0|phi0>
 * (t, u active orbitals counted from the first active one).  The density
 * enters the generalized Fock operator of the Dyall Hamiltonian
 * ("SC-NEVPT2(s)").  Caller-owned gamma[n_act * n_act].  Needs set_reference. */
scqmc_status scqmc_reference_rdm1(scqmc_ctx *ctx, double *gamma);

/* Semicanonical virtual orbitals for Dyall's Hamiltonian ("SC-NEVPT2(s)": the
 * virtual orbital energies come from diagonalising the virtual generalized
 * Fock operator).  Builds
 *   F_ab = h_ab + sum_{i core} [2(ab|ii) - (ai|ib)] + sum_{tu} gamma_tu [(ab|tu) - 1/2 (at|ub)]
 * on the device, diagonalises it on the host (cyclic Jacobi; eigenvalues
 * ascending, each eigenvector's largest-|component| positive), rotates the
 * context's integrals to the new virtual orbitals phi'_b = sum_a phi_a U[a][b],
 * and sets the Dyall Hamiltonian as set_dyall would with eps_virt = the
 * eigenvalues and e0_ref = E_0^(0).  The reference (active space) is
 * unchanged; class coefficients refer to the rotated orbitals.  Outputs,
 * both optional (NULL): eps_virt[V], u[V*V] row-major U[a][b].  Needs
 * set_reference; invalidates placed walkers (call init_walkers afterwards). */
scqmc_status scqmc_semicanonicalize(scqmc_ctx *ctx, double *eps_virt, double *u);

scqmc_status scqmc_set_options(scqmc_ctx *ctx, const scqmc_options *opt);

/* Place n_walkers walkers on the given determinants (host [W][2][words]); the
 * global walker id of row w is w.  seed keys the Philox4x32-10 counter
 * generator.  Resets the step counter and every accumulator.  Fails with
 * INVALID_ARG if a determinant is outside the allowed space or has psi = 0. */
scqmc_status scqmc_init_walkers(scqmc_ctx *ctx, int64_t n_walkers, const uint64_t *dets, uint64_t seed);

/* Advance every walker by n_steps continuous-time steps (enqueued on the
 * context stream; returns after launch).  Each step evaluates E_L (and in
 * mode 1 the Dyall local energy), the rates |psi(m)/psi(n)| over the
 * neighbour set, accumulates the estimators with residence weight
 * t = 1/sum of rates once the global step index reaches burn_in, and moves
 * the walker by the two-level first-reaction method (group of neighbours
 * sharing an active part, then one neighbour within it).  Before every
 * launch the walkers are put in a dispatch order (costliest class first,
 * grouped by virtual orbitals); a walker's chain depends only on its id, the
 * seed and the step, so the order never changes a result. */
scqmc_status scqmc_sample(scqmc_ctx *ctx, int64_t n_steps);
scqmc_status scqmc_synchronize(scqmc_ctx *ctx);

/* Host finalisation of the accumulated sums (synchronises). */
scqmc_status scqmc_read_estimates(scqmc_ctx *ctx, scqmc_estimates *out);
/* The E_var part of read_estimates alone (E_var, its jackknife error, a0^2),
 * from the per-walker sums only -- cheap enough to poll (serving loops). */
scqmc_status scqmc_read_energy(scqmc_ctx *ctx, double *e_var, double *e_var_err, double *a0_sq);
/* Small-norm perturber screen of "SC-NEVPT2(s)" (end of that section):
 * classes whose sampled relative norm N_l/N_0 is below tau are left out of
 * E^(2) (read_estimates) and of the first-order wave function
 * (read_first_order gives them coefficient 0).  tau = 0 (the default) keeps
 * every class.  tau must be finite and >= 0, else INVALID_ARG. */
scqmc_status scqmc_set_nevpt2_screen(scqmc_ctx *ctx, double tau);
/* SC-NEVPT2 first-order wave function (first equation of "SC-NEVPT2(s)"):
 *   psi1 = sum_{l != 0} coef_l P_l H phi0,  coef_l = 1 / (E_0^(0) - E_l),
 * for the unnormalised perturbers P_l H phi0 of a normalised phi0, with the
 * perturber energies E_l = D_l / N_l of eq:nevpt from the sampled class sums
 * (so that E^(2) = sum_l coef_l N_l / N_0).  Outputs, each [n] with
 * n = n_classes - 1 in class-id order (classes 1 ..) and each optional
 * (NULL): coef (NaN for a class never visited, 0 for a screened one),
 * coef_err (delete-one jackknife over the walker groups of the class sums,
 * NaN where undefined), e_l, rel_norm = N_l / N_0.  Needs mode 1; synchronises. */
scqmc_status scqmc_read_first_order(scqmc_ctx *ctx, double *coef, double *coef_err, double *e_l, double *rel_norm,
                                    int64_t n);
/* Per-class sums (n == n_classes): t_l = sum t, te_l = sum t E_L,
 * n_l = sum t / c_l^2, d_l = sum t E_D,L / c_l^2 (synchronises). */
scqmc_status scqmc_read_class_sums(scqmc_ctx *ctx, double *n_l, double *d_l, double *t_l, double *te_l, int64_t n);
/* Per-walker sums (n == n_walkers): sum t, sum t E_L, sum t [class 0] (synchronises). */
scqmc_status scqmc_read_walker_sums(scqmc_ctx *ctx, double *sum_t, double *sum_te, double *sum_t0, int64_t n);
/* Current walker determinants [n][2][words] and psi(n) (synchronises). */
scqmc_status scqmc_read_walkers(scqmc_ctx *ctx, uint64_t *dets, double *psi, int64_t n);
/* Steps taken since init_walkers and the count of walker-steps whose rates
 * summed to zero or whose local energy was not finite. */
scqmc_status scqmc_read_counters(scqmc_ctx *ctx, int64_t *steps, int64_t *bad_steps);

/* n_iter AMSGrad iterations on the placed walkers: per iteration the walkers'
 * psi(n) is recomputed with the current coefficients, equil_steps steps are
 * walked, the class sums are cleared, steps_per_iter steps are sampled, the
 * energy and gradient are formed on the host and the coefficients updated.
 * The moment estimates persist across calls (reset by set_sc_coeffs).
 * Optional outputs: e_trace[n_iter] (sampled E of each iteration),
 * g_trace[n_iter] (gradient 2-norm).  Synchronous.  Afterwards the walker and
 * class sums hold the last iteration's samples and read_class_sums /
 * set_sc_coeffs see the optimised coefficients (read them with
 * scqmc_read_sc_coeffs). */
scqmc_status scqmc_optimize(scqmc_ctx *ctx, const scqmc_amsgrad *opt, int64_t n_iter, double *e_trace,
                            double *g_trace);
/* Current SC coefficients: *c0 and c_cls[n], n = n_classes - 1. */
scqmc_status scqmc_read_sc_coeffs(scqmc_ctx *ctx, double *c0, double *c_cls, int64_t n);

/* Parity / debug.  Local energies of n determinants d_dets [n][2][words]
 * (device) without moving: E_L, psi, Gamma = sum_m |psi(m)/psi(n)|, the Dyall
 * local energy (mode 1, NaN for class 0; pass NULL to skip) and the class.
 * A determinant outside the allowed space or with psi = 0 gets NaN. */
scqmc_status scqmc_eval_snapshot(scqmc_ctx *ctx, int64_t n, const uint64_t *d_dets, double *d_eloc, double *d_psi,
                                 double *d_gamma, double *d_eloc_dyall, int32_t *d_class);
/* Allocation-free variant of scqmc_eval_snapshot, for callers that cannot
 * allocate device memory or wait on the device: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments and
 * results (bit for bit: the same kernels); it calls no allocator and never
 * synchronises -- everything is enqueued on the context stream.  Its scratch
 * -- the compacted copy of the determinants (SCQMC_NOALLOC_MAX_DETS entries
 * of 16 B = 1 MiB) and the evaluation kernel's per-wave Fock tables
 * (SCQMC_NOALLOC_FTAB_BYTES = 16 MiB; fewer waves run when a table is large)
 * -- lives in a fixed device array of the library (one per GPU, 17 MiB, held
 * until the process ends) that every call on that GPU shares: calls that
 * overlap on one GPU (other streams, other threads, other contexts) race;
 * serialise them.
 * n > SCQMC_NOALLOC_MAX_DETS -> INVALID_ARG.  In the precision form the FP32
 * integral copies must exist (any earlier sample / eval_snapshot call after
 * set_options makes them), else SCQMC_E_STATE. */
#define SCQMC_NOALLOC_MAX_DETS 65536
#define SCQMC_NOALLOC_FTAB_BYTES (16u << 20)
scqmc_status scqmc_eval_snapshot_noalloc(scqmc_ctx *ctx, int64_t n, const uint64_t *d_dets, double *d_eloc,
                                         double *d_psi, double *d_gamma, double *d_eloc_dyall, int32_t *d_class);
/* Neighbour set M(n) of one host determinant: up to cap entries of
 * determinant [2][words], phase (+-1), <m|H|n>, psi(m) (host arrays);
 * *out_count receives |M(n)|.  Order is unspecified. */
scqmc_status scqmc_debug_neighbors(scqmc_ctx *ctx, const uint64_t *det, int64_t cap, uint64_t *out_dets,
                                   int8_t *out_phase, double *out_hnm, double *out_psi, int64_t *out_count);

/* Checkpoint: walker state, step counter, seed and every accumulator, as an
 * opaque byte buffer (host).  *used receives the size; cap too small ->
 * INVALID_ARG with *used set.  load_state requires the same space, reference
 * and options; a walk resumed from it continues bit for bit. */
scqmc_status scqmc_save_state(scqmc_ctx *ctx, void *buf, int64_t cap, int64_t *used);
scqmc_status scqmc_load_state(scqmc_ctx *ctx, const void *buf, int64_t len);

/* ------------------------------------------------------------------------
 * Batched form: several contexts (independent systems of any sizes, each with
 * placed walkers, all on one device and in one precision) walked by one
 * launch per group of steps.  A schedule maps workgroups to (system, walker);
 * a walker's chain depends only on its own id and its system's step counter,
 * so the results equal those of the systems walked one by one, bit for bit.
 * The launch and the step advance are captured in a HIP graph and replayed
 * (with the persistent hand-out, the work counter is cleared by the step
 * advance, so replays need no memset).
 * The batch keeps pointers to the contexts (which must outlive it) and reads
 * their current state at every call.
 * ------------------------------------------------------------------------ */
typedef struct scqmc_batch scqmc_batch;

scqmc_status scqmc_batch_create(scqmc_ctx *const *ctxs, int32_t n, scqmc_batch **out);
void scqmc_batch_destroy(scqmc_batch *batch);
const char *scqmc_batch_last_error(const scqmc_batch *batch);
/* n_steps steps of every system (synchronous); each context's step counter
 * advances by n_steps. */
scqmc_status scqmc_batch_sample(scqmc_batch *batch, int64_t n_steps);
/* Schedule: order 0 = systems one after another, 1 = walkers of all systems
 * interleaved, 2 = costliest systems first; steps_per_launch 1..1024. */
scqmc_status scqmc_batch_set_schedule(scqmc_batch *batch, int32_t order, int32_t steps_per_launch);
/* Hand-out of the schedule's slots: bin = 0 lets the hardware dispatch one
 * workgroup per slot; bin >= 1 launches a persistent grid (sixteen
 * workgroups per compute unit) whose waves take work items of bin
 * consecutive slots from a device counter until the schedule is exhausted.
 * Results are the same either way.  bin 0..4096, else INVALID_ARG. */
scqmc_status scqmc_batch_set_queue(scqmc_batch *batch, int32_t bin);
/* Kernel variant of the hardware-dispatched launch: walkers (waves) per
 * workgroup and the minimum waves per SIMD the kernel's register budget is
 * compiled for.  Supported pairs: (1, 3), (1, 4) [default], (1, 5), (2, 4),
 * (4, 4); others -> INVALID_ARG.  The precision form has (1, 4) only (a batch
 * in the precision form with another pair fails at launch with
 * UNSUPPORTED).  Results do not depend on the variant. */
scqmc_status scqmc_batch_set_kernel(scqmc_batch *batch, int32_t walkers_per_group, int32_t waves_per_simd);
scqmc_status scqmc_batch_get_kernel(const scqmc_batch *batch, int32_t *walkers_per_group, int32_t *waves_per_simd);
/* Autotuner: times trial_steps steps (real steps of every system) for each
 * order 0..2, 1, 2, 4 steps per launch and hand-out bin 0 (hardware), 1, 4
 * (persistent) with the default kernel variant, then -- if the hardware
 * hand-out won and the batch is FP64 -- each other kernel variant of
 * scqmc_batch_set_kernel at that schedule, and keeps the fastest; outputs the
 * schedule and its time per step (each optional); the kernel variant chosen
 * is read with scqmc_batch_get_kernel. */
scqmc_status scqmc_batch_tune(scqmc_batch *batch, int64_t trial_steps, int32_t *order, int32_t *steps_per_launch,
                              int32_t *bin, double *ms_per_step);

#ifdef __cplusplus
}
#endif
#endif /* SCQMC_H */
