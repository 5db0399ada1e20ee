/*
 * ascc.h -- C ABI of libascc: the closed-shell CCSD-form T1/T2 residual, energy, Jacobi
 * update and DIIS that Aufbau-suppressed coupled cluster (ASCC) shares with ground-state
 * CCSD, on AMD Instinct MI355X (gfx950).
 *
 * What is computed (Tuckman, Ma, Neuscamman, arXiv:2501.10515):
 *   energy    E = <phi_0| e^{-T} Hbar e^{T} |phi_0>              (Sec. II.A, Eq. (eqn:energy))
 *   residual  R_mu = <mu| e^{-T} Hbar e^{T} |phi_0>, mu = singles and doubles
 *                                                                (Sec. II.A, Eq. (eqn:amp))
 *   with T = T1 + T2 (Sec. II.B) in the spin-adapted closed-shell form (Supporting
 *   Information S1): t1[i][a] = t_{i_alpha}^{a_alpha}, t2[i][j][a][b] = t_{i_alpha j_beta}^{a_alpha b_beta},
 *   and R1[i][a], R2[i][j][a][b] the matching alpha / alpha-beta projections.  The integrals
 *   are density fitted, (pq|rs) = sum_Q B[Q][p][q] B[Q][r][s], so Hbar is given through B and
 *   the reference Fock matrix; with S = 0 (ground state) Hbar = H (Eq. (eqn: sim)).
 *   The update is the diagonal approximate Jacobian with DIIS (Sec. III.B); the convergence
 *   test is max|R| and |dE| (Sec. III.A), optionally the residual 2-norm.
 *   For a 1-CSF excited state, ascc_build_ints_hbar forms Hbar = e^{S^dagger} H e^{-S^dagger}
 *   (Sec. II.A) and ascc_initial_guess the guess T^P(0) = beta S + gamma S^2; ascc_set_plascc
 *   switches to the partially linearised equations (Sec. II.C); ascc_two_ansatz solves both
 *   ansatz choices of Sec. II.D.  The mixed triples T^M_3' of Sec. II.B.1 are not provided.
 *
 * Conventions shared by every call:
 *   - no = occupied orbitals, nv = virtual orbitals, naux = fitting functions, n = no + nv;
 *     orbitals are ordered occupied first.  All arrays are C-order (row-major), contiguous.
 *   - Pointers named d_* are DEVICE memory on the current HIP device, owned by the caller,
 *     and must stay valid until the stream work that uses them has finished.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Every call
 *     except ascc_build_ints(_hbar), ascc_diis_create, ascc_solve, ascc_two_ansatz and
 *     ascc_reference_energy is asynchronous on it (ascc_set_plascc issues no stream work).
 *   - Amplitude and residual arrays are double precision.  `precision` selects the arithmetic
 *     of the large contractions only; energies, norms, the update and DIIS are always FP64.
 *   - Every function returns ASCC_OK (0) or a negative ASCC_E_* code and never throws, exits
 *     or aborts; ascc_last_error() returns a message for the last failure on this thread.
 *   - Device memory: ascc_build_ints(_hbar), ascc_batch_reserve, ascc_set_plascc and
 *     ascc_diis_create allocate the library's own device memory (integrals, work arrays, DIIS
 *     history, batch buffers, PLASCC buffers; ascc_workspace_bytes, ascc_batch_workspace_bytes and
 *     ascc_plascc_workspace_bytes report the amounts); ascc_*_free releases it.  Their *_ws forms
 *     carve the same arrays from a caller workspace instead and allocate nothing.  ascc_solve and ascc_two_ansatz allocate their own
 *     state and free it before returning.  No other call allocates device memory.
 *   - A handle is not re-entrant: calls that share an ascc_ints (its work arrays) or an
 *     ascc_diis must be ordered on one stream.
 *   - Check mode: with ASCC_CHECK_BOUNDS=1 in the environment (read once per process) every
 *     call verifies, before it launches, that each device range it touches lies inside a
 *     buffer it was given or owns (failing with ASCC_E_HIP and a message instead), and the
 *     integral builds verify that the largest occupied orbital energy lies below the smallest
 *     virtual one (ASCC_E_ARG otherwise: the Jacobi denominators must stay negative).
 *   - Low-precision contractions whose last 256-row tile holds at most 64 rows compute those rows
 *     in a launch of 64-row tail tiles when that takes fewer rounds of workgroups; the rows are
 *     bit for bit those of the full-tile launch, which ASCC_NO_TAIL_TILES=1 (read once per
 *     process) selects instead.
 */
#ifndef ASCC_H
#define ASCC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ASCC_OK = 0,
  ASCC_E_ARG = -1,           /* NULL pointer or invalid option value                    */
  ASCC_E_SHAPE = -2,         /* no, nv or naux out of range                             */
  ASCC_E_NOMEM = -3,         /* device allocation failed                                */
  ASCC_E_HIP = -4,           /* a HIP runtime call or kernel launch failed              */
  ASCC_E_NONFINITE = -5,     /* a NaN or Inf appeared in the residual or the energy     */
  ASCC_E_NOT_CONVERGED = -6, /* maxiter reached; results are the last iterate           */
  ASCC_E_STATE = -7          /* handles do not belong together (sizes differ)           */
};

enum {
  ASCC_PREC_FP64 = 0,  /* every contraction in FP64 on the FP64 matrix cores                    */
  ASCC_PREC_FP32 = 1,  /* the N^6 contractions (pp ladder, W/Z, rings) on FP32 matrix cores     */
  ASCC_PREC_BF16X3 = 2 /* the same on bf16 matrix cores with x = hi + lo splits: hi*hi + hi*lo  */
                       /* + lo*hi.  Both low modes accumulate in FP32 within K chunks of 8192  */
                       /* and in FP64 across chunks; everything else                         */
                       /* stays FP64                                                          */
};

enum {
  ASCC_VVVV_FULL = 0,  /* particle-particle ladder over the full (ac|bd) matrix, v^2 x v^2 */
  ASCC_VVVV_PACKED = 1 /* ladder over the (ab) / (cd) symmetric and antisymmetric halves   */
};

typedef struct ascc_ints ascc_ints; /* integrals of one Hamiltonian + residual work arrays */
typedef struct ascc_diis ascc_diis; /* DIIS history and solver state of one amplitude set  */

/* Device bytes of an integral set (`ints_bytes`: integrals, residual work arrays and the largest
 * build-time temporary, as carved by ascc_build_ints_ws) and of a DIIS state with m = diis_size
 * (`diis_bytes`, as carved by ascc_diis_create_ws).  Host-only, synchronous.
 * Errors: ASCC_E_SHAPE, ASCC_E_ARG. */
int ascc_workspace_bytes(int no, int nv, int naux, int precision, int vvvv_mode, int diis_size,
                         size_t* ints_bytes, size_t* diis_bytes);

/* Build the integral set for one Hamiltonian (Sec. II.A: the integrals of Hbar).
 *   d_B        [naux][n][n]  density-fitting factors; the residual is exact for the
 *                            integrals sum_Q B[Q][p][q] B[Q][r][s] (B need not be symmetric in
 *                            p,q: a one-body similarity transform makes it non-symmetric)
 *   d_fock     [n] (fock_is_diag = 1: orbital energies) or [n][n] (fock_is_diag = 0): the Fock
 *                            matrix of the reference determinant; its diagonal gives the
 *                            Jacobi denominators
 *   precision  ASCC_PREC_FP64, or a low precision (ASCC_PREC_FP32 / ASCC_PREC_BF16X3): the
 *              handle then also holds FP32 copies of the constant operands and can switch
 *              between FP64 and low precision (ascc_set_precision)
 *   vvvv_mode  ASCC_VVVV_FULL or ASCC_VVVV_PACKED (storage of the (ac|bd) block)
 * Copies what it needs from d_B / d_fock (they may be freed after the call), forms the
 * constant integral blocks on `stream`, and synchronises `stream` before returning.
 * On success *out owns the device memory until ascc_ints_free.
 * Errors: ASCC_E_ARG, ASCC_E_SHAPE (no, nv, naux < 1), ASCC_E_NOMEM, ASCC_E_HIP. */
int ascc_build_ints(const double* d_B, const double* d_fock, int fock_is_diag, int no, int nv, int naux,
                    int precision, int vvvv_mode, void* stream, ascc_ints** out);

/* Arithmetic of the N^6 contractions in the following ascc_residual calls on this handle:
 * ASCC_PREC_FP64 always; ASCC_PREC_FP32 / ASCC_PREC_BF16X3 only if the handle was built with a
 * low precision (it then holds FP32 copies of the constant operands).  ascc_build_ints starts
 * the handle in the precision it was built with.  Host-only.
 * Errors: ASCC_E_ARG, ASCC_E_STATE (low precision requested on an FP64-only handle). */
int ascc_set_precision(ascc_ints* ints, int precision);
int ascc_get_precision(const ascc_ints* ints);

/* ascc_build_ints carving every device array, build-time temporaries included, from the
 * caller's workspace d_workspace (256-byte aligned, ws_bytes >= the ints_bytes that
 * ascc_workspace_bytes reports) instead of allocating: for callers that admit work by memory
 * footprint or must not call the allocator.  Unlike ascc_build_ints it does not synchronise:
 * the build is queued on `stream` (d_B and d_fock must stay valid until it has run; later work
 * on the same stream is ordered after it).  The workspace must outlive the handle.
 * Errors: as ascc_build_ints, ASCC_E_NOMEM if ws_bytes is too small. */
int ascc_build_ints_ws(const double* d_B, const double* d_fock, int fock_is_diag, int no, int nv, int naux,
                       int precision, int vvvv_mode, void* d_workspace, size_t ws_bytes, void* stream,
                       ascc_ints** out);

/* The integral set of the ASCC transformed Hamiltonian of a 1-CSF state (Sec. II.A):
 * Hbar = e^{S^dagger} H e^{-S^dagger} (Eq. (eqn: sim)) with S = (s/sqrt 2)(p_up^dagger h_up +
 * p_dn^dagger h_dn) (Eq. (eqn:1CSF-S)), where H is given exactly as for ascc_build_ints.
 *   hole      the orbital h (occupied: 0 <= hole < no)
 *   particle  the orbital p (virtual: no <= particle < no + nv, a full orbital index)
 *   s_sign    s = +1: S as the paper writes it; s = -1: the same S after flipping the sign of the
 *             hole orbital, which the second ansatz of Sec. II.D uses (see ascc_two_ansatz).
 * S^dagger is one-body with the spatial matrix K = s E_hp / sqrt 2 (K^2 = 0), so Hbar stays two-body:
 * on the device every index pair of the DF factors and of the one-electron operator transforms as
 * x -> (1 + K) x (1 - K) before the constant blocks are formed (Bbar is then not symmetric in p,q).
 * The Jacobi denominators keep the diagonal of d_fock; the energy's f_ia is that of Hbar.  Every
 * other call then works on this handle unchanged (the amplitude equations of Hbar are those of
 * the ground state, Eq. (eqn:amp)); start it from ascc_initial_guess.  Synchronises `stream`.
 * Errors: as ascc_build_ints; ASCC_E_ARG for a hole or particle out of range or s_sign not +-1. */
int ascc_build_ints_hbar(const double* d_B, const double* d_fock, int fock_is_diag, int no, int nv, int naux,
                         int precision, int vvvv_mode, int hole, int particle, int s_sign, void* stream,
                         ascc_ints** out);

/* The initial cluster operator T^P(0) = beta S + gamma S^2 of Eq. (eqn:TP-guess) (the paper's
 * values: beta = 1, gamma = -1/2), written as closed-shell amplitudes into caller-owned device
 * arrays d_t1 [no][nv] and d_t2 [no][no][nv][nv]: every entry 0 except t1[hole][particle - no] =
 * beta / sqrt 2 and t2[hole][hole][particle - no][particle - no] = gamma (S^2 has only the
 * opposite-spin pair excitation).  With beta = 1 and gamma = -1/2, e^{-S^dagger} e^{T} |phi_0> is
 * the 1-CSF reference S |phi_0> of Eq. (eqn: 1csf).  Asynchronous on `stream` (a kernel, no memset).
 * Errors: ASCC_E_ARG, ASCC_E_HIP. */
int ascc_initial_guess(double* d_t1, double* d_t2, int no, int nv, int hole, int particle, double beta, double gamma,
                       void* stream);

/* Residual and energy at the given amplitudes (Eqs. (eqn:energy), (eqn:amp)).
 *   d_t1 [no][nv], d_t2 [no][no][nv][nv] with t2[i][j][a][b] == t2[j][i][b][a] (read only)
 *   d_r1 [no][nv], d_r2 [no][no][nv][nv]  (written; R2 has the same pair symmetry)
 *   d_e  [1]  correlation energy E - E_ref at (t1, t2) (written)
 * Asynchronous.  Errors: ASCC_E_ARG, ASCC_E_HIP. */
int ascc_residual(ascc_ints* ints, const double* d_t1, const double* d_t2, double* d_r1, double* d_r2,
                  double* d_e, void* stream);

/* Capacity for batched residuals of up to max_states amplitude sets on this integral set:
 * allocates the stacked ladder operands and one ladder result per state (device memory;
 * freed by ascc_ints_free; a larger later request reallocates; the same as
 * ascc_batch_reserve_ws(ints, max_states, 1, NULL, 0)).  Synchronous.
 * Errors: ASCC_E_ARG, ASCC_E_NOMEM. */
int ascc_batch_reserve(ascc_ints* ints, int max_states);

/* Exact device bytes of a batch capacity (ascc_batch_reserve_ws with the same max_states and
 * group) for an integral set of this shape, precision and vvvv_mode.  Host-only.
 * Errors: ASCC_E_SHAPE, ASCC_E_ARG. */
int ascc_batch_workspace_bytes(int no, int nv, int naux, int precision, int vvvv_mode, int max_states, int group,
                               size_t* bytes);

/* Batch capacity of max_states states whose residual terms other than the pp ladder run `group`
 * states at a time as one batched pass (every contraction one launch over the group's states
 * against the shared integrals, 1 <= group <= max_states; group = 1: state by state): the stacked
 * ladder operands and results plus `group` copies of the residual work arrays (about the integral
 * set's own work arrays each; ascc_batch_workspace_bytes gives the total).  d_workspace != NULL:
 * carved from it (256-byte aligned, >= that size; it must outlive the handle; no allocation);
 * NULL: allocated (freed by ascc_ints_free).  Replaces any earlier capacity.  Host-only.
 * Errors: ASCC_E_ARG, ASCC_E_NOMEM. */
int ascc_batch_reserve_ws(ascc_ints* ints, int max_states, int group, void* d_workspace, size_t ws_bytes);

/* Residuals and energies of nstates amplitude sets that share this integral set (several
 * states of one Hamiltonian).  d_t1[k], d_t2[k], d_r1[k], d_r2[k] are host arrays of device
 * pointers with the shapes of ascc_residual; d_e is a device array [nstates].  The particle-
 * particle ladders of all states are one launch over the shared vvvv block (its tiles are
 * streamed once for the batch).  With a capacity of group > 1 and evenly spaced state arrays
 * (d_t1[k] = d_t1[0] + k (d_t1[1] - d_t1[0]), likewise d_t2, d_r1, d_r2) every other term runs
 * `group` states per batched pass; otherwise state by state (and always with the PLASCC removal).
 * Each state's result is the one ascc_residual gives for it alone (the same arithmetic in the same
 * order).  Asynchronous.
 * Errors: ASCC_E_ARG, ASCC_E_STATE (nstates above the reserved capacity), ASCC_E_HIP. */
int ascc_residual_batch(ascc_ints* ints, int nstates, const double* const* d_t1, const double* const* d_t2,
                        double* const* d_r1, double* const* d_r2, double* d_e, void* stream);

/* DIIS state for one amplitude set of `ints`' shape: up to `max_vectors` (1..16) stored pairs
 * of (amplitudes after the Jacobi step, the step itself); pairs are stored from 0-based
 * update call `start` on.  Allocates device memory; synchronous.
 * Errors: ASCC_E_ARG, ASCC_E_NOMEM, ASCC_E_HIP. */
int ascc_diis_create(const ascc_ints* ints, int max_vectors, int start, ascc_diis** out);

/* ascc_diis_create carving from a caller workspace (256-byte aligned, >= the diis_bytes of
 * ascc_workspace_bytes for the same max_vectors); no allocation.  Errors: as ascc_diis_create. */
int ascc_diis_create_ws(const ascc_ints* ints, int max_vectors, int start, void* d_workspace, size_t ws_bytes,
                        ascc_diis** out);

/* Return the DIIS state to empty (no stored pairs, no previous energy).  Asynchronous. */
int ascc_diis_reset(ascc_diis* diis, void* stream);

/* One diagonal approximate-Jacobian step with DIIS (Sec. III.B), in place on (t1, t2):
 *   t <- t + R / D,  D_i^a = f_ii - f_aa,  D_ij^ab = f_ii + f_jj - f_aa - f_bb (+ level shift),
 * then, once two pairs are stored, t <- sum_k c_k t_k with the DIIS coefficients.  Reads the
 * residual (d_r1, d_r2) and energy d_e produced by ascc_residual at the same t.
 *   d_stats [8] doubles (written): E, dE (vs the previous call; +inf on the first), max|R|,
 *           |R|_2 over r1 (+) r2, number of stored DIIS pairs, flags (bit 0: non-finite
 *           residual or energy; bit 1: the DIIS system was ill-conditioned and old pairs were
 *           dropped), update index, level shift.
 * Asynchronous.  Errors: ASCC_E_ARG, ASCC_E_STATE, ASCC_E_HIP. */
int ascc_update(ascc_ints* ints, ascc_diis* diis, double* d_t1, double* d_t2, const double* d_r1,
                const double* d_r2, const double* d_e, double level_shift, double* d_stats, void* stream);

typedef struct ascc_opts {
  double tol_rnorm;   /* converged when |R|_2 <= tol_rnorm      (<= 0: test not used) */
  double tol_rmax;    /* ... and max|R| <= tol_rmax               (<= 0: not used)    */
  double tol_de;      /* ... and |dE| < tol_de                    (<= 0: not used)    */
  int maxiter;        /* >= 1                                                          */
  int diis_size;      /* 1..16 (1 disables extrapolation)                             */
  int diis_start;     /* first 0-based iteration whose pair is stored                 */
  double level_shift; /* added to |D| (D - shift); 0 for the plain Jacobi step         */
  /* FP64 refinement of a low-precision solve: when the handle's precision is FP32 or BF16X3,
   * the iteration first runs in that precision until its statistics pass the tests above, or
   * |R|_2 <= lowp_rnorm, or lowp_maxiter iterations (<= 0: that bound unused), or |R|_2 has not
   * set a new minimum (by 1%) for 8 iterations (the rounding floor of the low precision); then
   * the same amplitudes are evaluated in FP64: if the tests pass there (with the energy change of
   * the last low-precision iteration) the solve ends, else DIIS restarts from that FP64 residual
   * and the iteration continues in FP64 until the tests pass.  A solve never ends on a
   * low-precision residual.  The handle's precision is restored. */
  double lowp_rnorm;
  int lowp_maxiter;
} ascc_opts;

typedef struct ascc_result {
  double e_corr;   /* energy at the returned amplitudes                     */
  double rnorm;    /* |R|_2 at the returned amplitudes                      */
  double rmax;     /* max|R| at the returned amplitudes                     */
  double de;       /* last energy change                                    */
  int iterations;  /* residual evaluations made                             */
  int converged;   /* 1 if every requested test passed                      */
  int lowp_iterations; /* of which in low precision                         */
  int stalled;     /* not converged, but near it: the last energy change below the energy test
                      (tol_de, or 1e-7 Eh when tol_de is unused) and each residual test missed by
                      less than a factor 10 -- the paper keeps such states, marked (Sec. III.A) */
} ascc_result;

/* Iterate residual -> convergence test -> update from the amplitudes in (d_t1, d_t2)
 * (in place) until converged or opts->maxiter residual evaluations.  Allocates its DIIS
 * state internally (freed before returning) and synchronises `stream` once per iteration to
 * read the 8-double statistics block.  On return (t1, t2) hold the amplitudes the reported
 * energy and residual norms belong to.
 * Errors: ASCC_E_ARG, ASCC_E_NOMEM, ASCC_E_HIP, ASCC_E_NONFINITE (res filled up to the
 * failing iteration), ASCC_E_NOT_CONVERGED (res and amplitudes are the last iterate;
 * res->stalled marks a solve that stopped near convergence). */
int ascc_solve(ascc_ints* ints, const ascc_opts* opts, double* d_t1, double* d_t2, ascc_result* res,
               void* stream);

/* ascc_solve for callers that cannot allocate device memory -- code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc: the same iteration, arguments, results and errors
 * as ascc_solve, with its DIIS state, residual, trial amplitudes and statistics carved from a fixed
 * 64 MiB device array of the library instead of allocated (each GPU that runs the library holds one
 * until the process ends) and the statistics read into host stack memory.  No hipMalloc, hipFree
 * or other allocating routine is called.  The solver state must fit: (2 m + 2)(no nv + no^2 nv^2)
 * doubles plus a few KiB, m = opts->diis_size (with m = 8 up to about no = 8, nv = 72); larger
 * requests fail with ASCC_E_NOMEM before any work.  Every call on one GPU shares that GPU's array
 * and leaves its last contents there: calls that overlap on one GPU (other threads, other streams)
 * race and must not be made.  Synchronises `stream` once per iteration, as ascc_solve does.
 * Errors: as ascc_solve; ASCC_E_NOMEM when the solver state exceeds the fixed array. */
int ascc_solve_noalloc(ascc_ints* ints, const ascc_opts* opts, double* d_t1, double* d_t2, ascc_result* res,
                       void* stream);

/* ---- Request server: many independent solves on one GPU --------------------------------
 * A request is one Hamiltonian (DF tensor + orbital energies, diagonal Fock) solved from T = 0
 * with opts.solve.  The server owns one device slab of hbm_budget bytes (allocated at creation)
 * and carves each admitted request's complete working set from it, admitting queued requests in
 * arrival order whenever the head of the queue fits and fewer than max_active are running.
 * Ground-state requests of one shape (no, nv, naux) are bucketed: a bucket is a slab region of
 * up to 8 equal slots (as many as a quarter of the budget holds; 1 if the budget is tighter), and
 * one iteration of all its running slots is one batched pass -- every contraction one launch over
 * the slots, the Jacobi/DIIS update one launch set -- for the slots in low precision and for those
 * in FP64, captured once per slot set into a hipGraph (use_graphs = 1) and replayed.  Excited-state
 * and PLASCC requests run in buckets of one slot.  Every bucket has its own stream, and each
 * ascc_server_step launches the next iteration of every bucket whose previous one has finished,
 * so buckets overlap on the device and requests join or leave between iterations.  Each request's
 * results are those it gets alone (a slot's contractions take the same kernels and summation order
 * in a batch as alone).  With a low `precision` the bulk iterations run in it and the last ones in
 * FP64 (opts.solve.lowp_*).  All calls are host-side and never wait for the device except
 * ascc_server_free (and short waits on an idle bucket stream when a request changes precision or
 * finishes). */
typedef struct ascc_server ascc_server;

typedef struct ascc_server_opts {
  size_t hbm_budget; /* bytes of device memory for all requests together           */
  int max_active;    /* requests running at once (one stream each)                  */
  int precision;     /* ASCC_PREC_*: arithmetic of the bulk iterations             */
  int vvvv_mode;     /* ASCC_VVVV_FULL or ASCC_VVVV_PACKED                         */
  int use_graphs;    /* 1: replay a captured hipGraph per iteration                */
  ascc_opts solve;   /* tolerances, maxiter, DIIS, FP64-refinement switch          */
} ascc_server_opts;

typedef struct ascc_request_info {
  int id, no, nv, naux;
  int status; /* 1 queued, 2 running, ASCC_OK converged, or a negative ASCC_E_* code */
  int iterations, lowp_iterations;
  double e_corr, rnorm, rmax; /* of the last completed iteration                     */
  double t_submit, t_admit, t_done; /* caller clock values (ascc_server_submit/step) */
  size_t bytes;                     /* HBM footprint                                  */
  double e_ref;      /* <phi_0|H|phi_0> of the request's integral set (of Hbar for a state), once
                        the request has finished; e_ref + e_corr is its total energy         */
  int hole, particle; /* the 1-CSF state of ascc_server_submit_state, or -1, -1           */
  int bucket, slot;   /* the size bucket and slot the request ran in (-1 while queued or
                         after it finished: the last ones it held are kept)              */
} ascc_request_info;

/* Errors: ASCC_E_ARG, ASCC_E_NOMEM (slab allocation). */
int ascc_server_create(const ascc_server_opts* opts, ascc_server** out);
/* Queue a request; h_B [naux][n][n] and h_eps [n] are host arrays, copied before returning.
 * Errors: ASCC_E_ARG, ASCC_E_SHAPE, ASCC_E_NOMEM (larger than the whole budget). */
int ascc_server_submit(ascc_server* srv, const double* h_B, const double* h_eps, int no, int nv, int naux,
                       double t_submit, int* id);
/* Queue an ASCC 1-CSF excited-state request (Sec. II.A): its integral set is Hbar of the state
 * (hole, particle, s_sign as for ascc_build_ints_hbar) and its amplitudes start from T^P(0) =
 * beta s S - (beta^2 / 2) S^2 (ascc_initial_guess; beta = 1 is Eq. (eqn:TP-guess)); with plascc = 1 its
 * residuals leave out the terms quadratic in the mixed doubles (ascc_set_plascc_ws: its work
 * buffers are part of the request's footprint, carved from the slab and cleared on the request's
 * stream); otherwise it is served exactly like a ground-state request, with the same footprint.  Both ansatz of Sec. II.D are two requests
 * (s_sign = +1 and -1 with their beta).
 * Errors: as ascc_server_submit; ASCC_E_ARG for a hole or particle out of range, s_sign not +-1 or
 * beta <= 0. */
int ascc_server_submit_state(ascc_server* srv, const double* h_B, const double* h_eps, int no, int nv, int naux,
                             int hole, int particle, int s_sign, double beta, int plascc, double t_submit, int* id);
/* Retire finished requests, admit queued ones, launch the next iterations; `now` is the caller's
 * clock, recorded as admission / completion times.  Errors: ASCC_E_ARG, ASCC_E_HIP. */
int ascc_server_step(ascc_server* srv, double now, int* n_queued, int* n_running, int* n_done);
int ascc_server_info(const ascc_server* srv, int id, ascc_request_info* info);
void ascc_server_free(ascc_server* srv); /* waits for the device, then releases everything */

void ascc_ints_free(ascc_ints* ints); /* NULL is a no-op; waits for the device first unless the
                                         handle was carved from a caller workspace */
void ascc_diis_free(ascc_diis* diis); /* NULL is a no-op; synchronises the device first */

/* Per-phase timing of ascc_residual / ascc_update on a handle, with HIP events recorded on the
 * caller's stream around each phase (pp_ladder is the particle-particle ladder contraction,
 * etc.; names from ascc_phase_name).  ascc_timing_enable(ints, 1) starts recording;
 * ascc_timing_read waits for the recorded events, returns per phase the summed milliseconds
 * and the number of recorded intervals (arrays of at least ascc_phase_count() entries), and
 * clears the record.  Timing adds two event records per phase and no synchronisation.
 * Errors: ASCC_E_ARG, ASCC_E_HIP. */
int ascc_phase_count(void);
const char* ascc_phase_name(int k);
int ascc_timing_enable(ascc_ints* ints, int enable);
int ascc_timing_read(ascc_ints* ints, double* ms, int* counts, int n);

/* Partial linearisation, PLASCC (paper Sec. II.C): later residuals of this integral set leave out
 * every term that carries two or more powers of the mixed doubles T^M, the amplitudes whose index
 * set holds both a primary orbital (the hole or the particle of S) and a non-primary one
 * (Sec. II.B, Eq. (eqn: pnm split)); singles count for nothing here (kept to all orders).  The
 * doubles residual is of degree two in T2, so exactly its part quadratic in T^M is removed; the
 * singles residual and the energy are unchanged.  The paper applies the same removal, with the
 * same primaries, to the ground-state equations: call this on an ascc_build_ints set too.
 *   hole      occupied orbital index in [0, no), or < 0 to return to the full equations.
 *   particle  virtual orbital index in [no, no + nv) (full orbital numbering).
 * The first call with hole >= 0 allocates the removal's device work buffers (compact slabs along
 * the primary crosses; their exact size is what ascc_plascc_workspace_bytes reports, up to
 * even padding 8 m no nv + 3 m^2 + naux (no nv + 2 m) + 2 (2 no - 1) nv^2 + 3 no^2 (2 nv - 1) +
 * 2 no^2 (2 no - 1) doubles, m = no + nv - 1), clears
 * them and waits for the clears (released by ascc_ints_free).  The removal costs N^5 work per
 * residual.  Synchronous.  Errors: ASCC_E_ARG (NULL handle, indices out of range), ASCC_E_NOMEM,
 * ASCC_E_HIP. */
int ascc_set_plascc(ascc_ints* ints, int hole, int particle);

/* Exact device bytes of the PLASCC work buffers of an integral set of this shape (the workspace
 * ascc_set_plascc_ws needs).  Host-only.  Errors: ASCC_E_SHAPE, ASCC_E_ARG. */
int ascc_plascc_workspace_bytes(int no, int nv, int naux, size_t* bytes);

/* ascc_set_plascc carving its work buffers from the caller's workspace d_workspace (256-byte
 * aligned, ws_bytes >= ascc_plascc_workspace_bytes) instead of allocating: for callers that admit
 * work by memory footprint (the request server) or must not call the allocator.  The buffers are
 * cleared by a kernel queued on `stream` (no memset, no synchronisation); residuals of this handle
 * must run on `stream` or be ordered after it.  The workspace must outlive the handle; a handle
 * keeps the buffers of its first call (a later call with another workspace is ASCC_E_STATE).
 * hole < 0 returns to the full equations (d_workspace may then be NULL).
 * Errors: as ascc_set_plascc; ASCC_E_NOMEM if ws_bytes is too small. */
int ascc_set_plascc_ws(ascc_ints* ints, int hole, int particle, void* d_workspace, size_t ws_bytes, void* stream);

/* The two ansatz choices of Sec. II.D for a 1-CSF state whose reference has the Aufbau coefficient
 * alpha, alpha |phi_0> + S |phi_0> (Eq. (eqn:ref-with-nz-aufbau)), |alpha| < 1: the guess of
 * Eq. (eqn:TP-guess) with gamma = -beta^2/2 reaches it for (1 - beta)/beta = alpha, and, with the
 * hole orbital's sign flipped (S -> -S, s_sign = -1), for (1 - beta)/beta = -alpha.  Both are solved
 * (ascc_build_ints_hbar, ascc_initial_guess with beta s and gamma, ascc_solve) one after the other,
 * each on an integral set that is freed before the next is built; the reported energy is the mean
 * of the two total energies.  For alpha = 0 both have beta = 1.  A solve counts when it converged
 * or stalled near convergence (ascc_result.stalled); when only one of the two counts, its energy
 * alone is reported (Sec. III.A: the paper keeps the single converged solution, and stalled
 * states marked); when neither does, the state has no energy (ASCC_E_NOT_CONVERGED).  A solve whose
 * iteration becomes non-finite (ASCC_E_NONFINITE from ascc_solve) is such a failed solve: it is
 * recorded in res->solve with converged = 0 and the other ansatz is still solved.
 *   d_B, d_fock, fock_is_diag, no, nv, naux, precision, vvvv_mode, hole, particle: as for
 *             ascc_build_ints_hbar; opts: as for ascc_solve (its low-precision hand-over applies
 *             to both solves).
 *   d_t1[2], d_t2[2]: caller-owned device arrays [no][nv] and [no][no][nv][nv] that receive the
 *             amplitudes of the two solves ([0]: s = +1, [1]: s = -1).
 *   res       host struct (written).
 * Synchronises `stream`.  Errors: as the calls above; ASCC_E_ARG for |alpha| >= 1;
 * ASCC_E_NOT_CONVERGED if neither solve converges (res still written). */
typedef struct ascc_two_ansatz_result {
  double e_total[2];  /* total energies: [0] s = +1, beta = 1/(1 + alpha); [1] s = -1, beta = 1/(1 - alpha) */
  double e_mean;      /* the reported ASCC energy: the mean of the converged solves' total energies     */
  double beta[2];
  ascc_result solve[2];
  int used;           /* which solves e_mean averages: bit 0 = [0], bit 1 = [1] (0: neither converged)  */
} ascc_two_ansatz_result;
int ascc_two_ansatz(const double* d_B, const double* d_fock, int fock_is_diag, int no, int nv, int naux, int precision,
                    int vvvv_mode, int hole, int particle, double alpha, const ascc_opts* opts, double* const* d_t1,
                    double* const* d_t2, ascc_two_ansatz_result* res, void* stream);

/* The workspace form of ascc_build_ints_hbar (arguments as there and as for ascc_build_ints_ws:
 * the integral set is carved from d_workspace, asynchronous on `stream`). */
int ascc_build_ints_hbar_ws(const double* d_B, const double* d_fock, int fock_is_diag, int no, int nv, int naux,
                            int precision, int vvvv_mode, int hole, int particle, int s_sign, void* d_workspace,
                            size_t ws_bytes, void* stream, ascc_ints** out);

/* Reference energy <phi_0|H|phi_0> of an integral set (paper Eq. (eqn:energy): the total energy
 * is this plus the correlation energy that ascc_residual / ascc_solve report), formed at build time
 * as sum_{i<no} (h_ii + f_ii) from the core Hamiltonian h = f - sum_k [2 (pq|kk) - (pk|kq)] and the
 * reference Fock matrix f.  For a set from ascc_build_ints_hbar both are the transformed ones
 * (hbar, fbar of Eq. (eqn: sim)), so <phi_0|Hbar|phi_0> + e_corr is the ASCC total energy of the
 * state and its difference from the ground-state total is the excitation energy.
 *   e0      HOST pointer to one double (written).
 *   stream  the stream the handle was built on (or 0): waited for before reading.
 * Errors: ASCC_E_ARG for NULL arguments, ASCC_E_HIP if the copy fails.  A dry run writes 0. */
int ascc_reference_energy(const ascc_ints* ints, double* e0, void* stream);

/* Shape queries on a built handle (host-only). */
int ascc_ints_shape(const ascc_ints* ints, int* no, int* nv, int* naux);

/* Message for the last non-zero status returned on this thread ("" if none). */
const char* ascc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ASCC_H */
