/*
 * ctm.h -- C ABI of the MI355X (gfx950) CTMRG environment library.
 *
 * What it computes (arXiv:1906.02220, Sec. III and Fig. 4): the thermal state
 * of a hexagonal-lattice model is a purification with two sublattice tensors
 * A and B (Fig. 3(a)).  Fusing each A-B pair across one bond type gamma gives
 * a composite tensor on a rhombic, i.e. square, lattice (Fig. 4(b)).  The
 * ket and bra layers of the composite are contracted into a double-layer site
 * tensor a[u,l,d,r] with legs of dimension d = D^2 (Fig. 4(a,b)).  The corner
 * transfer matrix renormalisation group replaces the infinite network around
 * one site by four corner tensors C and four edge tensors T of bond dimension
 * chi (Fig. 4(c)); the environment of the fused gamma bond then gives the
 * full-update bond metric, the norm per site and local expectation values
 * (Sec. III, last paragraph).
 *
 * Conventions.  All arrays are real IEEE double, row-major, C-contiguous.
 *   A, B      [s=2][a=2][x][y][z]: pseudospin, ancilla, then the three bond
 *             legs; the gamma leg has dimension D_gamma, the others D.
 *   a         [u][l][d][r], each leg of dimension d.
 *   environment, clockwise from the top-left: C1 T1 C2 T2 C3 T3 C4 T4.
 *             C[a][b] (chi x chi): a on the counter-clockwise side.
 *             T[a][m][b] (chi x d x chi): m points into the lattice.
 *   composite physical index p = (s_A, a_A, s_B, a_B), 16 values.
 *   double-layer leg index  = k * D + b (k ket, b bra).
 *
 * Memory and ownership.  Host pointers passed in are read during the call
 * only; output buffers are caller-owned and written before return.  Device
 * memory is allocated by the library (hipMalloc) at environment creation and
 * released by ctm_env_destroy.  Every call on one context is serialised on
 * the context's stream; a context is not thread-safe.
 *
 * Errors.  Every entry point returns a status code; nothing throws across
 * the ABI.  The message of the last failure is kept per context and is read
 * with ctm_last_error.  Argument errors leave the environment unchanged.
 */
#ifndef CTM_H
#define CTM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define CTM_OK        0   /* success */
#define CTM_ENOTCONV  1   /* warning: max_sweeps reached before tol; env valid */
#define CTM_EINVAL   -1   /* bad argument (shape, length, index, null) */
#define CTM_ENOMEM   -2   /* device allocation failed */
#define CTM_EDEVICE  -3   /* HIP runtime error or no usable gfx950 device */
#define CTM_ENUMERIC -4   /* NaN/Inf in the environment or SVD failure */

/* Arithmetic used for the dense contractions (projector SVD and the norm
 * normalisation always stay in FP64). */
#define CTM_PREC_F64     0  /* FP64 MFMA */
#define CTM_PREC_F32     1  /* one FP32 MFMA product, FP64 storage */
#define CTM_PREC_BF16X3  3  /* FP64 operands split into 3 BF16 slices */
#define CTM_PREC_BF16X4  4  /* ... 4 slices */
/* Any other value (2, 5, 6, ...) is rejected with CTM_EINVAL. */

typedef struct ctm_context ctm_context;
typedef struct ctm_env ctm_env;

typedef struct ctm_opts {
  int precision;          /* CTM_PREC_*; default CTM_PREC_F64 */
  double eps_cut;         /* singular values below eps_cut * s_1 get S^-1/2 := 0
                             (shapes kept); default 1e-12 */
  int svd_block;          /* subspace size b (chi <= b <= 128) of the truncated
                             projector SVD; 0 = automatic (see svd_oversample).
                             A cut matrix with chi*d <= 128 rows gets a full
                             Jacobi SVD instead. */
  int svd_iters;          /* subspace iterations per move when warm-started;
                             0 = automatic: 2 for the first 8 warm moves of
                             each direction after a random start, then 1 */
  int svd_iters_cold;     /* iterations from a random start; 0 = automatic (5) */
  unsigned long long seed;/* seed of the counter-based generator for cold
                             starts; default 0x5eed */
  const double* boundary; /* length-d boundary vector of the initial edges, or
                             NULL: e_0 for ctm_env_init_tensor, vec(I_D) for
                             ctm_env_init_purification */
  int svd_oversample;     /* with svd_block = 0: b = min(chi*d, chi + svd_oversample,
                             128); 0 = automatic, b = min(chi*d, 128,
                             max(88, chi + max(16, ceil(chi / 4)))) */
  double svd_tol;         /* > 0: after each truncated SVD's fixed iterations, iterate
                             again from its vectors (at most 8 more times) until
                             max_i ||M u_i - s_i v_i|| / s_1 over the kept chi
                             triplets is at most svd_tol; every check waits for
                             the device, so such sweeps are never replayed from
                             graphs.  < 0: fixed iteration counts only.  0 =
                             automatic: fixed counts for sweeps, 1e-12 for the
                             gradient calls (the adjoint assumes exact SVDs). */
  int move_order[4];      /* directions of the four moves of a sweep, a permutation
                             of 0 (left), 1 (up), 2 (right), 3 (down): the move in
                             direction k is the left move of the lattice rotated
                             k times by 90 degrees.  All zero = default
                             {0, 2, 1, 3}: left, right, up, down. */
} ctm_opts;

/* Fill *opts with the defaults listed above. */
void ctm_opts_default(ctm_opts* opts);

/* Create a context on HIP device `device` (must be gfx950).  Owns one HIP
 * stream (default priority) and the timing events.  Returns CTM_EDEVICE if
 * the device is missing or not gfx950. */
int ctm_context_create(int device, ctm_context** out);
void ctm_context_destroy(ctm_context* ctx);
/* Message of the most recent failure on this context ("" if none).  The
 * string is owned by the context and valid until the next call on it. */
const char* ctm_last_error(const ctm_context* ctx);
/* Use an external HIP stream (e.g. a torch stream) for all further work of
 * this context; NULL restores the context's own stream. */
int ctm_context_set_stream(ctm_context* ctx, void* hip_stream);

/* Autotune the tile shape of the large FP64 and FP32 products (on != 0;
 * default off): the first product of each shape on this context runs every
 * candidate tiling (96 x 96, 128 x 128, 64 x 64 output tiles) three times,
 * keeps the fastest, and later products of that shape use it.  The
 * candidates accumulate in the same order, so results do not depend on the
 * choice. */
int ctm_context_set_autotune(ctm_context* ctx, int on);

/* Replay warm sweeps from HIP graphs (on != 0; default off).  Once every
 * projector SVD of an environment runs from a warm start and one such sweep
 * has run normally, the next sweep is captured into a graph (the four moves
 * and the corner-spectrum delta) and later sweeps replay it, which removes
 * the per-kernel launch cost.  The counter-based generator that refills
 * numerically dependent subspace columns then repeats its counters from
 * sweep to sweep.  Sweeps with kernel timing switched on run normally. */
int ctm_context_set_graphs(ctm_context* ctx, int on);

/* Environment of a user-supplied site tensor a[u][l][d][r] (d^4 doubles,
 * host memory), chi >= 1, d >= 1.  Initial corners C = [[1]] and edges
 * T[0,:,0] = boundary (zero-padded to chi): after k sweeps in which no
 * singular value of a cut matrix falls below the cutoff (nothing truncated)
 * the environment is the (2k+1)^2 open lattice with that boundary vector.
 * (Fig. 4(c): the corner and edge tensors of the square lattice.) */
int ctm_env_init_tensor(ctm_context* ctx, const double* a, int d, int chi,
                        const ctm_opts* opts, ctm_env** out);

/* Environment of the rhombic lattice of an A-B purification pair (Sec. III,
 * Figs. 3(a), 4(a,b)).  Builds the composite tensor K[p,u,l,d,r] of A and B
 * fused across bond `gamma` (0=x, 1=y, 2=z; its dimension is D_gamma, D or
 * 4D after a gate as in Fig. 3(b)), with u = A.beta, l = A.alpha,
 * d = B.beta, r = B.alpha where (alpha, beta) are the two other bond types in
 * cyclic order after gamma; then the double layer a = sum_p K_p (x) K_p; then
 * the initial environment as for ctm_env_init_tensor with boundary vec(I_D).
 * A and B: host arrays of 4 * D * D * D_gamma doubles. */
int ctm_env_init_purification(ctm_context* ctx, const double* A, const double* B,
                              int D, int D_gamma, int gamma, int chi,
                              const ctm_opts* opts, ctm_env** out);

/* The same two constructors with the tensors in device memory (for example
 * torch-owned): a, A and B are device pointers on the context's device, in
 * the layouts above.  They are read by kernels on the context's stream
 * (ctm_context_set_stream), so the caller makes them ready there first; the
 * library does not keep them after the call returns.  Returns CTM_EINVAL if
 * a pointer is not device memory (hipMalloc-type, not host or managed) of
 * that device or the allocation it lies in ends before the tensor does. */
int ctm_env_init_tensor_dev(ctm_context* ctx, const double* a, int d, int chi,
                            const ctm_opts* opts, ctm_env** out);
int ctm_env_init_purification_dev(ctm_context* ctx, const double* A, const double* B,
                                  int D, int D_gamma, int gamma, int chi,
                                  const ctm_opts* opts, ctm_env** out);
void ctm_env_destroy(ctm_env* env);

/* CTMRG sweeps (Fig. 4(c)).  One sweep is the left, right, up and down
 * absorption move, each built from the four enlarged corners and a
 * projector pair from the truncated SVD of the product of the two half
 * systems.  After every sweep delta = max over the four corners of
 * ||s_hat - s_hat_old||_2 with s_hat the corner singular values normalised to
 * unit 2-norm.  Stops after max_sweeps, or earlier once delta < tol when
 * tol > 0.  sweeps_done and delta may be NULL.  Returns CTM_ENOTCONV (> 0,
 * environment valid) if tol > 0 was not reached, CTM_ENUMERIC on NaN/Inf or
 * an SVD failure. */
int ctm_sweep(ctm_env* env, int max_sweeps, double tol, int* sweeps_done, double* delta);

/* Sweeps of several independent environments at once (for example a scan
 * over couplings or temperatures, Sec. III's CTMRG run per state).  Every
 * round enqueues one sweep of each environment that has not converged, then
 * waits for them: environments created on different contexts run
 * concurrently on their contexts' streams, environments sharing a context
 * run in turn.  Per environment the semantics are those of ctm_sweep.
 * envs: count distinct environments; sweeps_done, delta: arrays of count
 * (may be NULL).  Returns CTM_ENOTCONV if tol > 0 was not reached by every
 * environment; on an error the message (kept on the first environment's
 * context) names the environment, and every stream has drained. */
int ctm_sweep_batch(ctm_env* const* envs, int count, int max_sweeps, double tol,
                    int* sweeps_done, double* delta);

/* The same sweeps in lock-step (Sec. III's CTMRG run per state, many states
 * at once): each move direction of a round takes the enlarged corners of
 * every unconverged environment on its own stream, then the two half-system
 * products and the cut matrix (the n x n x n contractions of the absorption
 * move) of all of them as one persistent grouped launch per kernel kind on
 * the first environment's context stream, whose workgroups claim tiles from a
 * device counter, then the projector SVDs and absorptions again on each
 * environment's stream.  Products are grouped only where ctm_sweep would run
 * the same FP64 or FP32 tile kernel without split-K (other products, such as
 * those of the BF16 slice modes, run on the environment's own stream), so the
 * results are bit-identical to ctm_sweep.  Every environment must live on the
 * first one's device; a captured sweep graph of an environment is dropped.
 * Arguments, return codes and error reporting as ctm_sweep_batch. */
int ctm_sweep_batch_grouped(ctm_env* const* envs, int count, int max_sweeps, double tol,
                            int* sweeps_done, double* delta);

/* One absorption move: direction 0 left, 1 up, 2 right, 3 down. */
int ctm_move(ctm_env* env, int direction);

/* Norm per site of the rhombic lattice (one composite = two hexagonal
 * sites): kappa = Z_site Z_0 / (Z_row Z_col), where Z_site closes the ring of
 * all eight environment tensors around a, Z_0 is the ring of the corners,
 * and Z_row (Z_col) inserts only the top and bottom (left and right) edges
 * with their inner legs joined. */
int ctm_norm(ctm_env* env, double* kappa);

/* log|Z| and sign of the ring closed around a, with every scale divided
 * out during the sweeps added back (the finite-lattice value for untruncated
 * sweeps). */
int ctm_log_z(ctm_env* env, double* log_abs, double* sign);

/* Full-update bond metric of the fused gamma bond (Sec. III, last
 * paragraph; Fig. 3(b)): the environment E of the composite site, normalised
 * so that <E, a> = 1.  Purification environments: len must be D^8, layout
 * [u_k][l_k][d_k][r_k][u_b][l_b][d_b][r_b] (ket legs, then bra legs).
 * Tensor environments: len must be d^4, layout [u][l][d][r].
 * CTM_EINVAL on a wrong len. */
int ctm_bond_metric(ctm_env* env, double* E, size_t len);

/* <O> = <psi|O|psi> / <psi|psi> for a real operator on the composite's
 * physical index (purification environments only).  op_dim 4: op is a 4x4
 * row-major matrix on (s_A, s_B) x (s_A', s_B') with the identity on the
 * ancillas; op_dim 16: op is 16x16 on p = (s_A, a_A, s_B, a_B).  Real states
 * make the imaginary part of a Hermitian operator contribute nothing, so the
 * caller passes its real part. */
int ctm_expect(ctm_env* env, const double* op, int op_dim, double* value);

/* ctm_expect for callers that cannot allocate device memory (serving loops
 * that evaluate many operators on one converged environment, code that must
 * not call hipMalloc): the same <O>, computed without any allocation.  The
 * per-call buffers (the D^4 x 16 partial contraction, rho, the operator,
 * reduction and split-K partial sums) live in a fixed device array of 8 MiB
 * that the library holds on every GPU it runs on until the process ends.
 * op, op_dim, value: as for ctm_expect (op is host memory, read during the
 * call; value is written before return).
 * Requirements: the environment's ring must be current, i.e. ctm_norm,
 * ctm_expect, ctm_log_z or ctm_bond_metric has run once since the last sweep
 * or move (contracting the ring needs workspace this call does not
 * allocate); D <= 8 (16 D^4 + 1344 doubles must fit the array).  Either
 * failure returns CTM_EINVAL and runs nothing.  Every call on one GPU shares
 * that GPU's array and leaves its contents behind (nothing in it needs to
 * start at zero): calls that overlap on one GPU, from several threads or
 * streams, race. */
int ctm_expect_noalloc(ctm_env* env, const double* op, int op_dim, double* value);

/* <E, a_imp> / <E, a> for an impurity site tensor a_imp[u][l][d][r] (d^4
 * doubles, host), any environment. */
int ctm_expect_tensor(ctm_env* env, const double* a_imp, double* value);

/* The four corner spectra s_hat (each normalised to unit 2-norm, descending,
 * zero-padded): len must be 4 * chi. */
int ctm_corner_spectra(ctm_env* env, double* s, size_t len);

/* Copy the environment out / in: C 4*chi*chi, T 4*chi*d*chi (host arrays,
 * C1..C4 then T1..T4 in the layout above), logs 8 (log scales of C1..C4,
 * T1..T4).  ctm_env_set also resets the warm starts of the projector SVD. */
int ctm_env_get(ctm_env* env, double* C, double* T, double* logs);
int ctm_env_set(ctm_env* env, const double* C, const double* T, const double* logs);

/* Checkpoint of the environment (C, T, logs, chi, d, sweep count) to a
 * binary file, and restore into an environment of the same chi and d. */
int ctm_env_save(ctm_env* env, const char* path);
int ctm_env_load(ctm_env* env, const char* path);

/* Shape queries. */
int ctm_env_dims(const ctm_env* env, int* chi, int* d, int* D, int* sweeps);

/* Accuracy of the truncated projector SVD (Sec. III, the CTMRG truncation
 * of Fig. 4(c)).  calls: truncated SVDs computed by subspace iteration so far
 * (cut matrices of at most 128 rows get a full Jacobi SVD and are not
 * counted); iterations: their subspace iterations in total; last_residual:
 * max_i ||M u_i - s_i v_i|| / s_1 over the kept chi triplets of the last
 * move's cut matrix M (0 before the first move), computed on request, which
 * waits for the device.  Any pointer may be NULL. */
int ctm_svd_stats(ctm_env* env, long long* calls, long long* iterations, double* last_residual);

/* Debugging aid, process-wide: on != 0 fills every device buffer the library
 * allocates from now on (environments, context workspaces, gradient tapes)
 * with all-ones bytes, a NaN as a double and -1 as an int, and places it
 * between two 64 KiB guard bands of a fixed pattern, so that a kernel reading
 * memory the library never wrote shows up in the results and one writing
 * past either end of a buffer is caught when the buffer is freed (the bands
 * are checked then, after waiting for the device; each damaged band is
 * counted and reported on stderr).  on = 0 stops it for later allocations.
 * *previous (may be NULL) gets the old state.  The environment variable
 * CTM_POISON_ALLOC (set and not "0") turns it on at load.  Slows every
 * allocation and free; results do not change.  Always CTM_OK. */
int ctm_debug_poison_allocations(int on, int* previous);

/* Number of damaged guard bands found so far (see above); CTM_EINVAL if
 * count is NULL. */
int ctm_debug_guard_violations(long long* count);

/* Statistics of the last gradient call. */
typedef struct ctm_grad_info {
  int moves;                 /* absorption moves differentiated */
  int cg_iters_max;          /* most conjugate-gradient steps of one move */
  long long cg_iters_total;  /* over all moves */
  double ms_forward;         /* first forward pass, with checkpoints */
  double ms_recompute;       /* forward re-runs of the checkpointed segments */
  double ms_backward;        /* reverse pass */
  double tape_bytes;         /* device memory of the per-move records */
  double checkpoint_bytes;   /* device memory of the checkpoints */
} ctm_grad_info;

/* Gradient of L = w_log_kappa ln(kappa) + w_expect <O> with respect to the
 * purification tensors A and B (reverse mode, written by hand), where kappa
 * and <O> are those of ctm_norm and ctm_expect after `sweeps` sweeps from the
 * boundary environment of the composite of A and B (Sec. III, Fig. 4).
 * Inputs as ctm_env_init_purification; op / op_dim as ctm_expect (op may be
 * null when w_expect = 0; *expect is then 0).  Outputs (host, caller-owned):
 * *log_kappa, *expect, grad_A and grad_B (4 D^2 D_gamma each, the layout of
 * A and B), *info when not null.
 * The derivative is that of the fixed-sweep map with exact truncated SVDs
 * of the cut matrices (the adjoint of the top-chi SVD includes the terms of
 * the discarded subspace); the forward SVD is the subspace iteration of
 * ctm_sweep, so raise svd_iters when the forward must match the exact SVD
 * closely.  The environment state is checkpointed every checkpoint_every
 * sweeps (<= 0: once at the start) and each segment is recomputed for the
 * reverse pass; the result does not depend on checkpoint_every.  Device
 * memory: about 4 (chi^2 (1 + d) + 2 n chi) doubles per move of a segment,
 * n = chi d.  Needs precision CTM_PREC_F64 (CTM_EINVAL otherwise);
 * CTM_ENUMERIC if a sweep fails as in ctm_sweep or kappa is not positive. */
int ctm_grad_purification(ctm_context* ctx, const double* A, const double* B, int D, int D_gamma,
                          int gamma, int chi, const ctm_opts* opts, int sweeps,
                          int checkpoint_every, const double* op, int op_dim,
                          double w_log_kappa, double w_expect, double* log_kappa,
                          double* expect, double* grad_A, double* grad_B, ctm_grad_info* info);

/* The same for a site tensor a (d^4, [u][l][d][r], as ctm_env_init_tensor):
 * L = w_log_kappa ln(kappa) + w_expect <E, a_imp> / <E, a> with an impurity
 * tensor a_imp (d^4; null when w_expect = 0), gradient dL/da in grad_a (d^4);
 * a_imp is held fixed. */
int ctm_grad_tensor(ctm_context* ctx, const double* a, int d, int chi, const ctm_opts* opts,
                    int sweeps, int checkpoint_every, const double* a_imp, double w_log_kappa,
                    double w_expect, double* log_kappa, double* expect, double* grad_a,
                    ctm_grad_info* info);

/* The same two gradients with A, B (a) and grad_A, grad_B (grad_a) in device
 * memory of the context's device, for callers whose tensors already live
 * there (torch autograd): nothing crosses PCIe but the scalars and, when
 * given, the small host arrays op (16 x 16 or 4 x 4) and a_imp.  The inputs
 * are read and the gradients written on the context's stream, and the call
 * returns after that stream has drained, so the caller must have finished
 * writing the inputs (on any stream) before the call.  Each device pointer
 * must lie in one device allocation of the context's device holding the
 * whole array (CTM_EINVAL otherwise, nothing written; an allocator that
 * sub-allocates, like torch's caching allocator, is seen as its underlying
 * segment, so only overruns past that segment are caught); the layouts are
 * those of the host calls. */
int ctm_grad_purification_dev(ctm_context* ctx, const double* A, const double* B, int D,
                              int D_gamma, int gamma, int chi, const ctm_opts* opts, int sweeps,
                              int checkpoint_every, const double* op, int op_dim,
                              double w_log_kappa, double w_expect, double* log_kappa,
                              double* expect, double* grad_A, double* grad_B,
                              ctm_grad_info* info);
int ctm_grad_tensor_dev(ctm_context* ctx, const double* a, int d, int chi, const ctm_opts* opts,
                        int sweeps, int checkpoint_every, const double* a_imp, double w_log_kappa,
                        double w_expect, double* log_kappa, double* expect, double* grad_a,
                        ctm_grad_info* info);

/* One bond update of the exact-environment full update (Sec. III,
 * Fig. 3(b), Fig. 4).  The gate exp(-tau H/2) of the real 4 x 4 bond term H
 * (row-major, index (s_A s_B)(s_A' s_B'), acting on the pseudospins) is
 * split by SVD into two gate tensors joined by an index of dimension 4 and
 * contracted with A and B, so that the gamma bond grows to 4D.  The
 * environment of the gated composite A'-B' (the 4D bond hidden inside it)
 * comes from `sweeps` CTMRG sweeps at chi with opts, as the bond metric E of
 * the composite's outer legs.  Then `als_iters` rounds of alternating least
 * squares (A'' with B'' fixed, then B'' with A'' fixed, from A'' = A,
 * B'' = B) minimise the error of the purification in that metric,
 *   d = sum_p <K'_p - K''_p, E (K'_p - K''_p)>,  K = composite over gamma,
 * with E symmetrised and a ridge of 1e-12 tr(N)/dim(N) on each normal
 * matrix.  A, B, A_out, B_out: host [2][2][D][D][D], every bond D <= 8;
 * errors (host, als_iters + 1 entries, may be null): d / <K', E K'> at the
 * start and after each round.  CTM_ENUMERIC if a sweep fails or a normal
 * matrix is not positive definite. */
int ctm_fu_bond_update(ctm_context* ctx, const double* A, const double* B, int D, int gamma,
                       const double* H, double tau, int chi, const ctm_opts* opts, int sweeps,
                       int als_iters, double* A_out, double* B_out, double* errors);

/* One second-order Trotter step of the imaginary-time evolution (Sec. III):
 * the bond updates G_x(dbeta/2) G_y(dbeta/2) G_z(dbeta) G_y(dbeta/2)
 * G_x(dbeta/2), applied right to left, where G_gamma(t) uses the gate
 * exp(-t H_gamma / 2) on every gamma bond.  H: three 4 x 4 bond terms
 * (x, y, z) one after the other.  A and B (host [2][2][D][D][D]) are
 * updated in place.  errors (host, 5 (als_iters + 1) entries, may be null):
 * the error history of each of the five bond updates. */
int ctm_fu_trotter_step(ctm_context* ctx, double* A, double* B, int D, const double* H,
                        double dbeta, int chi, const ctm_opts* opts, int sweeps, int als_iters,
                        double* errors);

/* Leading eigenvalues of the transfer matrix of the environment, for the
 * correlation length (Sec. IV quotes xi in lattice constants of the rhombic
 * lattice).  direction 0: one column, v'[x',r,y'] = sum T1[x,m,x']
 * a[m,l,n,r] T3[y',n,y] v[x,l,y]; direction 1: one row (T2, a rotated by
 * 90 degrees, T4); site = 0 leaves the site tensor out (T1 and T3 joined over
 * their inner leg).  `krylov` Arnoldi steps (2..64, capped at the dimension)
 * from a start drawn with opts' seed of the environment; the nev leading
 * Ritz values by decreasing magnitude go to re, im (host, nev entries,
 * 1 <= nev <= krylov; missing ones are 0) and *xi = -1/ln|lambda_2/lambda_1|
 * (0 if lambda_2 vanishes; may be null).  CTM_ENUMERIC if the Hessenberg QR
 * does not converge. */
int ctm_transfer_spectrum(ctm_env* env, int direction, int site, int nev, int krylov, double* re,
                          double* im, double* xi);

/* Kernel timing over the calls since the last reset, measured with HIP
 * events on the context's stream around every launch of one kernel class.
 * cls 0: FP64 GEMMs of the n x n x n half-system and cut products;
 * cls 1: all dense contraction kernels; cls 2: a whole move.
 * Returns count of launches, their summed milliseconds and summed
 * algorithmic flops.  ctm_timing_enable(ctx, 1) switches recording on. */
int ctm_timing_enable(ctm_context* ctx, int on);
int ctm_timing_reset(ctm_context* ctx);
int ctm_timing_get(ctm_context* ctx, int cls, long long* count, double* ms, double* flops);

#ifdef __cplusplus
}
#endif
#endif /* CTM_H */
