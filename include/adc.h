/*
 * adc.h -- C ABI of the MI355X library for spin-adapted, density-fitted
 * EA/IP-ADC(n), n = 2 or 3 (closed-shell reference).
 *
 * The library computes the lowest charged excitations of a closed-shell
 * system from its orbital energies and density-fitting factors:
 *   * electron attachment (EA): matrix M+ of Eq. 7, eigenvalues
 *     omega = E(N+1) - E(N) (the vertical attachment energy is -omega);
 *   * ionisation (IP): the negative of M- of Eq. 9, eigenvalues
 *     omega = E(N-1) - E(N) > 0 (ionisation energies);
 * by the five steps of Sec. III.A: integrals from B (Eq. 38), amplitudes
 * (Eqs. 13-14), the 1p-1p / 1h-1h block, the sigma = M Y product with an
 * iterative (Davidson) eigensolver, and spectroscopic factors (Eqs. 16-17,
 * 46-50).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Sizes: O = nocc, V = nvir, N = O + V, Q = naux.
 * Orbital energies eps[N]: occupied first; Fock matrix = diag(eps).
 * DF factors B[Q][N][N], row-major, symmetric in the last two indices:
 *   (pq|rs) = sum_Q B[Q][p][q] B[Q][r][s]                       (Eq. 38)
 * Vectors live in the orthonormal spin-adapted basis Z = S^{1/2} Y, where Y
 * are the spin-adapted amplitudes of Eqs. 36-37 (and their EA analogue) and
 * S = 1 (+) (2 - P_swap) is the metric behind the norm of Eq. 48
 * (symmetric square root; P_swap exchanges the two like indices).  In this
 * basis M is symmetric and a unit vector gives the renormalised amplitudes
 * of Eqs. 46-48.  A vector of length dim is laid out as
 *   EA: dim = V + O*V*V:  Z1[a] (V entries), then Z2[i][a][b], where a is
 *       the attached alpha electron and (b, i) a spin-conserving pair;
 *   IP: dim = O + V*O*O:  Z1[i] (O entries), then Z2[a][i][j], where i is
 *       the removed alpha electron and (j, a) a spin-conserving pair.
 * Blocks of vectors are row-major [nvec][dim].
 *
 * Memory and streams: pointers documented as "device" are HIP device
 * pointers on the current device (for example torch tensors' data_ptr());
 * "host" pointers are ordinary host memory.  All caller arrays stay owned by
 * the caller; the library never frees them.  adc_setup copies what it needs,
 * so eps and B may be freed after it returns.  Everything the library
 * allocates is released by adc_destroy.  A context is bound to one HIP
 * stream (the null stream unless adc_set_stream is called); calls on one
 * context must not overlap.
 *
 * Errors: every int-returning call returns ADC_OK (0) on success, a negative
 * ADC_E_* code on failure, or ADC_E_NOCONV (1) when a solve ran out of
 * iterations (its outputs then hold the best current estimates).  Arguments
 * are validated on the host before any device work; a message describing
 * the last failure is available from adc_last_error (per context) or
 * adc_last_error(NULL) (failures before a context exists).  No C++
 * exception crosses this interface.
 */
#ifndef ADC_H
#define ADC_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct adc_ctx adc_ctx;

enum { ADC_IP = 0, ADC_EA = 1 };

enum {
    ADC_OK = 0,
    ADC_E_ARG = -1,      /* invalid argument (checked on the host)           */
    ADC_E_OOM = -2,      /* device allocation failed or workspace limit hit  */
    ADC_E_HIP = -3,      /* HIP / rocBLAS runtime error                      */
    ADC_E_STATE = -4,    /* call not valid in the context's current state    */
    ADC_E_NUMERIC = -5,  /* non-finite values met (residual or sigma)        */
    ADC_E_NOCONV = 1     /* solver stopped at max_iter; outputs are estimates */
};

/* Steps 1-3 of Sec. III.A.  Stages eps ([N]) and B ([Q][N][N]), each either
 * device memory or host memory (host B is copied in blocks of auxiliary
 * functions, so the caller's B need not occupy the GPU), into the library's
 * layouts, computes the MP amplitudes
 * (t2 first order; for order 3 also the second-order singles and doubles
 * and third-order singles, Eqs. 13-14) and the 1p-1p (EA) or 1h-1h (IP)
 * block through order `order`, and keeps everything resident on the device.
 * Setup always runs in FP64 (the amplitudes define M).
 * order: 2 or 3.  kind: ADC_IP or ADC_EA.  On success *out receives a new
 * context.  Errors: ADC_E_ARG (nocc < 1, nvir < 1, naux < 1, bad order or
 * kind, NULL pointer), ADC_E_OOM, ADC_E_HIP. */
int adc_setup(const double* eps, const double* B, int nocc, int nvir, int naux,
              int order, int kind, adc_ctx** out);

/* Unrestricted (open-shell) reference: the paper's UADC code (Sec. II; the
 * open-shell radical of Sec. V.B), EA/IP-ADC(2).  Inputs per spin: orbital
 * energies eps_a, eps_b ([nmo] each, occupied first, each block ascending)
 * and density-fitting factors B_a, B_b ([naux][nmo][nmo], symmetric in the
 * orbital pair; (pq|rs) for spins s, t is sum_Q B_s^Q_pq B_t^Q_rs, Eq. 38),
 * device or host memory (host inputs are copied to the device whole);
 * nocc_a alpha and nocc_b beta electrons occupy the lowest orbitals of
 * their spin, whose Fock matrices are diag(eps_s).  order must be 2.
 * Setup (FP64): first-order doubles of the three spin blocks, second-order
 * singles, the 1p-1p (EA) or 1h-1h (IP) block of each spin through second
 * order, and the exact diagonal.
 * Vectors hold both spin sectors (the matrix is block diagonal in them),
 * dim = n1 + the four 2p1h (EA) / 2h1p (IP) blocks, in this order:
 *   EA: Y alpha [Va], Y beta [Vb], (i a b) spins aaa [Oa][a<b], bab
 *       [Ob][Va][Vb], aab [Oa][Va][Vb], bbb [Ob][a<b];
 *   IP: Y alpha [Oa], Y beta [Ob], (a i j) spins aaa [Va][i<j], bab
 *       [Vb][Oa][Ob], aab [Va][Oa][Ob], bbb [Vb][i<j];
 * (Va = nmo - nocc_a, Vb = nmo - nocc_b; packed pairs p < q row-major).  The
 * element of a block is the coefficient of a_b^+ a_a^+ a_i |Phi> (EA) or
 * a_a^+ a_j a_i |Phi> (IP) with the two like indices in that order (in the
 * mixed blocks the alpha one first).  The other entry points then work on
 * the context as on a closed-shell one, with these differences: sigma runs
 * in FP64 at every precision level; adc_spec_factors and the solver's
 * factors are P = sum_p X_p^2 over the 2 nmo spin orbitals (Eq. 17; X rows:
 * alpha orbitals, then beta) instead of the spin-adapted Eq. 50; the
 * learned preconditioner and its training records are not available
 * (ADC_E_STATE).  Errors: ADC_E_ARG (NULL pointer, nocc_a or nocc_b outside
 * [1, nmo), naux < 1, order != 2, bad kind), ADC_E_OOM, ADC_E_HIP. */
int adc_setup_u(const double* eps_a, const double* eps_b, const double* B_a, const double* B_b,
                int nocc_a, int nocc_b, int nmo, int naux, int order, int kind, adc_ctx** out);

/* Options taken by later adc_setup calls of the calling thread (the setup
 * runs before any adc_set_option can reach the context):
 *   "slice_budget"  elements per operand slice of the setup's large
 *                   contractions (four-index products are evaluated in slices
 *                   of this size or less, so that the setup's temporaries stay
 *                   bounded; default 0 = 2^28); results do not depend on it
 *                   beyond the order of floating-point sums;
 *   "m11_onthefly"  1: skip the precomputation of the 1p-1p (EA) / 1h-1h (IP)
 *                   block (step 3 of Sec. III.A); every sigma applies it to
 *                   the trial vectors on the fly through intermediates (the
 *                   alternative the paper describes there: no O^2 V^4 block
 *                   build, at most O^3 V^2 or V^2 Naux work per vector, in
 *                   FP64 at every precision level), keeping u, D u, Lambda and
 *                   the small P intermediates resident.  adc_diag then gives
 *                   that block's diagonal through second order only (the
 *                   Davidson correction and guesses use it as it is);
 *                   0 (default): the block is precomputed;
 *   "verbose"       1: one line on stderr per setup phase and per block of
 *                   its long loops, with the seconds since adc_setup began
 *                   (each line synchronises the stream); 0 (default): silent.
 * Errors: ADC_E_ARG for an unknown key or a bad value. */
int adc_set_setup_option(const char* key, double value);

/* Options (numeric values):
 *   "precision"   0 = FP64 sigma (default); 1 = mixed: sigma contractions
 *                 with BF16 products and FP32 sums (FP32 storage), FP64
 *                 subspace, then FP64 refinement iterations; 2 = as 1 with a
 *                 phase of FP32 products (FP32 storage and sums) between the
 *                 BF16 and FP64 phases.  adc_sigma runs at the selected level
 *                 (2: FP32 products)
 *   "block"       trial vectors per sigma launch in adc_davidson (default:
 *                 max(nroots, 8))
 *   "max_space"   Davidson subspace limit (default 8 * block, lowered to what
 *                 fits in a quarter of the free device memory, but at least
 *                 3 * block)
 *   "max_iter"    Davidson iteration limit (default 300)
 *   "tol_e"       eigenvalue change tolerance in Eh (default 1e-8)
 *   "tol_r"       residual norm tolerance, in units of max(1, |theta|) for
 *                 each root (default sqrt(tol_e))
 *   "verbose"     1: per-iteration line on stderr; 2: also the solver's
 *                 wall time per phase (synchronising after each phase)
 *   "eigensolver" projected Rayleigh-Ritz eigenproblem: 0 = automatic
 *                 (default: 2 up to 64 basis vectors, else 3), 1 = rocSOLVER
 *                 cyclic Jacobi, 2 = Householder tridiagonalisation and
 *                 implicit QR on the host, where the projected matrix is
 *                 assembled (3 if its sweeps do not converge), 3 = rocSOLVER
 *                 divide and conquer
 *   "pp_slab_mb"  size bound in MiB of the rebuilt four-virtual slab of the
 *                 particle-particle term (default: the larger of 16 GiB and a
 *                 third of the device memory free for it, at most 64 GiB); a
 *                 smaller slab means more, smaller rebuild blocks
 *   "pp_blocks"   minimum number of blocks of a in that rebuild (default 0:
 *                 min(24, V/8) in FP64 and FP32, min(12, V/8) in BF16);
 *                 block k rebuilds only the pairs b >= its first a, so more
 *                 blocks mean fewer rebuilt flops but smaller products
 *   "pp_group"    blocks of that rebuild contracted together in one product
 *                 (default 0: 8, bounded by the slab size)
 *   "workspace_limit"  bytes the context may allocate in total
 *   "graph"       1 = replay sigma from HIP graphs captured per (vector
 *                 count, precision) after an eager warm-up call (default 0)
 *   "record"      keep up to this many Davidson iterates for training pairs
 *   "precond"     0 = diagonal preconditioner, 1 = the installed network
 *   "autotune"    GEMM tile choice: 0 = fixed heuristic, 1 = time the tile
 *                 configurations on the first call of each shape and keep
 *                 the fastest (default), 2 = as 1 and log the choices
 *   "ea_layout"   EA sigma: 1 = keep the amplitudes and integrals of the
 *                 2p1h rows also in product-ready layouts (six extra
 *                 O^2 V^2 FP64 tensors, seven BF16 ones in the mixed mode,
 *                 and two O V Naux matrices that fold t~ into the coupling)
 *                 so that each large contraction is one matrix-core product,
 *                 0 = generic contractions (permute per call), 2 = the same
 *                 products as 1 with each product-ready operand built per
 *                 call, one block of its leading index at a time, from the
 *                 resident t, (ov|ov) and (oo|vv) (for systems whose extra
 *                 tensors do not fit: t~ is then released and t~ + u~ of the
 *                 spectroscopic amplitudes kept in pinned host memory), -1 = 1
 *                 when the extra tensors fit in half of the free device
 *                 memory, else 2 (default)
 *   "ctr_log"     1 = time each generic contraction with HIP events and
 *                 print its product shape on stderr (sigma then runs eagerly)
 *   "bvv_host"    EA only.  1 = keep the vv block of the DF factors (V^2 Naux,
 *                 the largest input tensor) and its FP32 / BF16 copies in
 *                 pinned host memory instead of the device (the out-of-core
 *                 storage mode of Sec. III.A): every sigma product that reads
 *                 it stages the rows it needs, one block at a time; 0 = back
 *                 on the device (default).  Needs ea_layout -1, 1 or 2
 *   "gemm_config" -1 = tile configuration of each matrix-core product chosen
 *                 by the autotuner or heuristic (default); 0..8 = that
 *                 configuration forced on every product of this context (ids
 *                 from adc_gemm_configs; one not compiled for a product's
 *                 type runs as 0)
 * Errors: ADC_E_ARG for an unknown key or out-of-range value. */
int adc_set_option(adc_ctx* ctx, const char* key, double value);

/* Bind later calls of this context to a HIP stream (hipStream_t). */
int adc_set_stream(adc_ctx* ctx, void* hip_stream);

/* Dimension of the ADC matrix (see the layout above); -1 for NULL. */
long long adc_dim(const adc_ctx* ctx);

/* Exact diagonal of M in the Z basis (with the setup option "m11_onthefly":
 * the 1p-1p / 1h-1h part through second order) (the diagonal that the Davidson
 * correction of Sec. III.A, step 4, divides by; the paper does not say which
 * diagonal its solver uses, and this one is exact: the 1p-1p / 1h-1h block's
 * diagonal through order n and, in the 2p1h / 2h1p block, the zeroth-order
 * orbital-energy differences plus, for n = 3, the first-order diagonal terms
 * such as (aa|bb), in the Z basis of the layout above).
 * d: device [dim] (written; caller-owned).  Errors: ADC_E_ARG for a NULL
 * context or output, ADC_E_HIP for a failed copy. */
int adc_diag(adc_ctx* ctx, double* d);

/* sigma = M X for a block of vectors (step 4, Eqs. 36-37 and their EA
 * analogue).  X: device [nvec][dim] (read), Y: device [nvec][dim] (written);
 * X and Y must not overlap.  Runs in the precision selected by
 * "precision" (FP64 by default).  nvec >= 1. */
int adc_sigma(adc_ctx* ctx, const double* X, double* Y, int nvec);

/* Lowest `nroots` eigenpairs by block Davidson-Liu in an FP64 subspace
 * (steps 4-5): initial guesses are unit vectors at the smallest diagonal
 * entries unless adc_set_guess provided vectors; the diagonal
 * preconditioner (theta - D)^-1 corrects the residuals.  Converged when
 * every root changes by <= max(tol_e, 8 eps |theta|) (eps = 2^-52: changes
 * below the FP64 resolution of theta are rounding) and has residual norm
 * <= tol_r max(1, |theta|).
 * energies, spec_factors: host [nroots] (written; spec_factors may be NULL);
 * P = 2 sum_p |X_p|^2 (Eq. 50, the sum over both spin components;
 * unrestricted contexts: the sum over spin orbitals, see adc_spec_factors).
 * vecs: device [nroots][dim] (written) or NULL.  n_iter: host, may be NULL.
 * Returns ADC_OK, ADC_E_NOCONV (estimates written), or an error. */
int adc_davidson(adc_ctx* ctx, int nroots, double* energies, double* spec_factors,
                 double* vecs, int* n_iter);

/* Spectroscopic factors P = 2 sum_p X_p^2 with X = T Y (Eqs. 16, 46-50)
 * for normalised Z-basis vectors.  vecs: device [nvec][dim];
 * P: host [nvec].  X (optional, device [nvec][N], may be NULL) receives
 * the spectroscopic amplitudes X_p (occupied orbitals first).  Unrestricted
 * contexts (adc_setup_u): X is [nvec][2N] (alpha orbitals, then beta) and
 * P = sum_p X_p^2 over those 2N spin orbitals. */
int adc_spec_factors(adc_ctx* ctx, const double* vecs, int nvec, double* P, double* X);

/* Spectra from the solver's outputs (no context; device pointers on
 * `stream`, a hipStream_t or NULL; caller-owned; synchronises the stream).
 * adc_spectral_function: the density of states / photoelectron spectrum of
 * Sec. IV (the ADC density of states of Sec. II with broadening eta):
 *   A[k] = -(1/pi) Im sum_mu P[mu] / (omega[k] - energies[mu] + i eta)
 *        = (1/pi) sum_mu P[mu] eta / ((omega[k] - energies[mu])^2 + eta^2)
 * omega [nomega], energies and P [nroots] (for example adc_davidson's outputs
 * copied to the device), A [nomega] (written).  With P from Eq. 50 (both spin
 * components) this is -(1/pi) Im of the trace of G over spin orbitals.
 * adc_propagator_diag: the diagonal of the ADC propagator of Sec. II,
 *   G_pp(omega[k] + i eta) = sum_mu X[mu][p]^2 / (omega[k] - energies[mu] + i eta)
 * for the spectroscopic amplitudes X [nroots][norb] of adc_spec_factors (one
 * spin component; these amplitudes are also the coefficients of the Dyson
 * orbitals of Sec. IV in the reference orbitals), written to
 * G [nomega][norb][2] as (real, imaginary).
 * Errors: ADC_E_ARG (NULL pointer, sizes < 1, eta <= 0), ADC_E_HIP. */
int adc_spectral_function(const double* omega, int nomega, const double* energies, const double* P,
                          int nroots, double eta, double* A, void* stream);
int adc_propagator_diag(const double* omega, int nomega, const double* energies, const double* X,
                        int nroots, int norb, double eta, double* G, void* stream);

/* Warm start: the next adc_davidson starts from these nvec vectors
 * (device [nvec][dim], copied). */
int adc_set_guess(adc_ctx* ctx, const double* V0, int nvec);

/* Convergence history of the last adc_davidson call: for each iteration k <
 * min(count, max_entries): seconds[k] since the call started (host wall
 * clock after the iteration's Ritz values were known), theta[k*nroots + r]
 * and rnorm[k*nroots + r] for the lowest nroots Ritz pairs, and mixed[k] =
 * the sigma level of the iteration (0 FP64, 1 BF16 products, 2 FP32
 * products).  Any output may be NULL.  Returns the
 * number of recorded iterations (>= 0) or a negative error code. */
int adc_history(const adc_ctx* ctx, int max_entries, double* seconds, double* theta,
                double* rnorm, int* mixed);

/* Algorithmic cost model of one adc_sigma call on nvec vectors (Table I
 * scaling with the constants of this implementation; 2 flops per
 * multiply-add).  total: every contraction of the call; pp: the
 * particle-particle / hole-hole term alone (EA-ADC(3): the rebuild of the
 * unique (ac|bd), Naux V^2 (V^2+1), plus 2 O V^4 nvec; IP-ADC(3):
 * 2 V O^4 nvec; 0 for ADC(2)).  Host outputs; never touches the device. */
int adc_sigma_flops(const adc_ctx* ctx, int nvec, double* total, double* pp);

/* adc_sigma with timing: HIP events recorded on the context's stream
 * around the particle-particle kernel(s) and around the whole call.
 * ms_pp, ms_total: host outputs in milliseconds (either may be NULL). */
int adc_sigma_timed(adc_ctx* ctx, const double* X, double* Y, int nvec, double* ms_pp,
                    double* ms_total);

/* Message describing the last failure of ctx (or of a call that had no
 * context when ctx is NULL).  Never NULL; owned by the library. */
const char* adc_last_error(const adc_ctx* ctx);

/* Release everything the context owns.  NULL is ignored. */
void adc_destroy(adc_ctx* ctx);

/* Statistics of the last adc_davidson call: iterations, sigma calls
 * (vectors), mixed-precision iterations, wall seconds.  host arrays. */
int adc_last_stats(const adc_ctx* ctx, int* iters, long long* sigma_vectors,
                   int* mixed_iters, double* seconds);

/* Device memory of the context (not in the paper: planning aid for large
 * systems): bytes it holds now and the most it has held at once since
 * adc_setup began (amplitudes, integrals, operand copies, Davidson space,
 * scratch).  used, peak: host pointers, either may be NULL.  ADC_E_ARG for a
 * NULL context. */
int adc_workspace(const adc_ctx* ctx, long long* used, long long* peak);

/* Several systems solved together (not in the paper: batching of its step 4
 * over independent systems).  ctxs: nsys distinct contexts, each set up and
 * configured as for adc_davidson.  flags:
 *   bit 0 (1): sigma replayed from each system's own captured graphs (one per
 *              vector count and precision, reused across iterations);
 *   bit 1 (2): concurrent instead of lockstep: host threads each run the
 *              single-system solver on the next unsolved system, on a
 *              stream of its own when the context uses the null stream, so
 *              that the host work of one solve overlaps the device work of
 *              the others;
 *   bit 2 (4): stats has 5 entries (see below);
 *   bits 8-15: number of those threads, 1..64 (0: 8).
 * Without bit 1 the solvers advance in lockstep and each iteration applies
 * sigma to the new trial vectors of every active system; with bit 0 as one
 * launch of a graph holding every ready system's sigma graph as a child node
 * (with the copies of its vectors in and out; independent branches, so the
 * systems run side by side; instantiated again only when the set of systems,
 * vector counts or precisions changes), a system whose graph is not yet
 * captured running its own sigma (and capture) over a few default-priority
 * streams.  Results equal those of adc_davidson on each context.
 * energies, spec_factors: host [nsys][nroots] (spec_factors may be NULL);
 * n_iter, status: host [nsys] (may be NULL; status per system as
 * adc_davidson returns it; the message of a failed system is its context's
 * adc_last_error); stats: host [3] (or [5] with flag bit 2) or NULL: lockstep
 * iterations (concurrent: the largest iteration count), sigma graph replays
 * (one per system and iteration), graph captures; then launches of the
 * combined graph and the number of times it was instantiated (lockstep with
 * graphs only; 0 otherwise).
 * Returns ADC_OK when every system converged, else the first non-OK status;
 * ADC_E_ARG for bad arguments (message in adc_last_error(NULL)). */
int adc_batch_davidson(adc_ctx* const* ctxs, int nsys, int nroots, int flags,
                       double* energies, double* spec_factors, int* n_iter, int* status,
                       long long* stats);

/* The same batched solve over a batch object that owns its contexts
 * (step 4 of Sec. III.A over many independent systems; not in the paper).
 * adc_system_desc: the arguments of adc_setup for one system (eps, B device
 * pointers, read during adc_setup_batch only).  adc_setup_batch sets up nsys
 * systems one after another (each as adc_setup; every system's tensors stay
 * resident, so the batch must fit in device memory together) and returns a
 * batch that owns them; on any failure it releases the systems already made
 * and returns that failure's code (message in adc_last_error(NULL)).
 * adc_batch_set_option applies one option to every system.
 * adc_davidson_batch solves every system as adc_batch_davidson does on the
 * batch's contexts (same flags and outputs).  adc_batch_context returns the
 * k-th context (owned by the batch; NULL when k is out of range), for per-system
 * options or queries.  adc_batch_destroy releases the batch and its
 * contexts (NULL is ignored). */
typedef struct adc_batch adc_batch;
typedef struct adc_system_desc {
    const double* eps;   /* device [nocc + nvir]                 */
    const double* B;     /* device [naux][nocc+nvir][nocc+nvir]  */
    int nocc, nvir, naux, order, kind;
} adc_system_desc;
int adc_setup_batch(int nsys, const adc_system_desc* sys, adc_batch** out);
int adc_batch_set_option(adc_batch* batch, const char* key, double value);
int adc_davidson_batch(adc_batch* batch, int nroots, int flags, double* energies,
                       double* spec_factors, int* n_iter, int* status, long long* stats);
adc_ctx* adc_batch_context(adc_batch* batch, int k);
void adc_batch_destroy(adc_batch* batch);

/* The matrix-core product under every contraction of the library, on its
 * own (not in the paper: exposed so that each compiled tile configuration
 * can be checked against a reference product):
 *   C = alpha op(A) op(B) + beta C
 * ta = 0: A is [M][K] row-major (lda >= K), ta = 1: A is [K][M] (lda >= M);
 * tb = 1: B is [N][K] (ldb >= K), tb = 0: B is [K][N] (ldb >= N).
 * dtype: 0 = FP64 throughout; 1 = FP32 operands, products and sums; 2 = FP32
 * operands rounded to BF16 (nearest even) while staged, BF16 products, FP32
 * sums; 3 = BF16 operands (A, B as raw 16-bit BF16), FP32 sums.  C: FP64 for
 * dtype 0, else FP32.  A, B, C: device pointers on `stream` (a hipStream_t,
 * NULL: the null stream); caller-owned; C must not overlap A or B.
 * map: NULL for a row-major C with leading dimension ldc, else 6 values
 * {rsplit, rs1, rs2, csplit, cs1, cs2}: element (m, n) is stored at
 *   (m / rsplit) rs1 + (m % rsplit) rs2 + (n / csplit) cs1 + (n % csplit) cs2
 * (a split of 0 means no split: m rs2, n cs2); the caller guarantees every
 * such offset lies inside C and that distinct (m, n) map to distinct offsets.
 * config: a tile configuration id from adc_gemm_configs, or -1 for the
 * library's own choice.  Configuration 8 (the BF16 256x256 tile whose operands
 * are loaded straight into LDS) applies to BF16 storage (dtype 3) in the NT
 * form (ta = 0, tb = 1) with 16-byte aligned rows; other products given 8 run
 * as 7.  Synchronises the stream before returning.
 * Errors: ADC_E_ARG (bad dtype, sizes, leading dimensions, map or config),
 * ADC_E_HIP.  adc_gemm_configs writes the configuration ids compiled for a
 * dtype into ids (at most 8) and returns their count (ADC_E_ARG for a bad
 * dtype or NULL ids). */
int adc_gemm(int dtype, int ta, int tb, long long M, long long N, long long K, double alpha,
             const void* A, long long lda, const void* B, long long ldb, double beta, void* C,
             long long ldc, const long long* map, int config, void* stream);
int adc_gemm_configs(int dtype, int* ids);

/* Number of sigma graph replays so far (option "graph"); -1 for NULL. */
long long adc_graph_launches(const adc_ctx* ctx);

/* ---- learned preconditioner --------------------------------------------
 * Not in the paper: an extension of its Davidson correction (Sec. III.A,
 * step 4).  The diagonal correction r / (theta - D) is multiplied element
 * by element by (1 + y), y the output of a 3-layer perceptron (width 256,
 * tanh) fed with 7 local features of the element (theta - D, the
 * normalised residual, the element's orbital energies, theta, the block);
 * the exact definitions, the FP32 parameter layout and the training target
 * are in csrc/mlp.hip.  The diagonal preconditioner stays the fallback. */

/* Number of FP32 parameters of the network (68097). */
long long adc_mlp_nparams(void);

/* Install a network for later adc_davidson calls of ctx (params: device
 * [adc_mlp_nparams()] FP32, copied) and select it; NULL restores the
 * diagonal preconditioner.  A solve whose learned corrections turn
 * non-finite, or whose residuals stop falling (four iterations without a
 * 10% decrease), goes
 * on with the diagonal one (counted by adc_mlp_status).  Option "precond"
 * (0/1) switches between an installed network and the diagonal. */
int adc_precond_mlp(adc_ctx* ctx, const float* params, long long nparams);
int adc_mlp_status(const adc_ctx* ctx, int* installed, int* fallbacks);

/* Training pairs for nidx sampled elements (idx: device [nidx], each in
 * [0, dim)) of one Davidson iterate: x its Ritz vector and r its residual
 * (device [dim]), theta its Ritz value, xstar the converged eigenvector of
 * the same root (device [dim]).  Writes F: device [nidx][7] features,
 * a: device [nidx] rhat*q (the diagonal correction of the normalised
 * residual), t: device [nidx] target.  ADC_E_ARG for a zero vector. */
int adc_mlp_pairs(adc_ctx* ctx, const double* x, const double* r, double theta,
                  const double* xstar, const long long* idx, long long nidx, float* F,
                  float* a, float* t);

/* y[n] = network output for features F[n][7] (device).  bf16 != 0: the
 * hidden 256x256 layer multiplies in BF16 with FP32 sums (inference);
 * else FP32 throughout. */
int adc_mlp_forward(adc_ctx* ctx, const float* params, const float* F, long long n, int bf16,
                    float* y);

/* adc_mlp_forward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): no context, no allocation.  The hidden activations of the
 * network live in a static device array the library holds on each GPU it
 * runs on until the process ends (8192 rows x 3 x 256 FP32 = 24 MiB); the
 * first call on a device looks its address up (not a stream operation, but
 * make that first call outside a capture).  params: device
 * [adc_mlp_nparams()] FP32; F: device [n][7] FP32; y: device [n] FP32
 * (written); all caller-owned.  bf16 as in adc_mlp_forward.  The work is
 * enqueued on `stream` (hipStream_t, NULL: the null stream) and the call
 * returns without synchronising.  1 <= n <= 8192, else ADC_E_ARG; ADC_E_HIP
 * on a launch failure (messages in adc_last_error(NULL)).  Calls that
 * overlap on one GPU (other streams or threads) share the array and race. */
int adc_mlp_forward_noalloc(const float* params, const float* F, long long n, int bf16, float* y,
                            void* stream);

/* loss = 0.5 mean_e (a_e (1 + y_e) - t_e)^2 over n pairs (host output) and
 * its gradient grad[adc_mlp_nparams()] (device) with respect to params,
 * FP32 forward and backward. */
int adc_mlp_loss_grad(adc_ctx* ctx, const float* params, const float* F, const float* a,
                      const float* t, long long n, float* grad, double* loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; step >= 1)
 * on params with first/second moments m, v (all device FP32 vectors of
 * adc_mlp_nparams() entries, updated in place). */
int adc_mlp_adam(adc_ctx* ctx, float* params, const float* grad, float* m, float* v, int step,
                 double lr);

/* Iterates recorded by the last adc_davidson call (option "record" = how
 * many, 0 by default): count, and entry i: Ritz vector x and residual r
 * (device [dim] outputs, either may be NULL), Ritz value and root index
 * (host outputs, may be NULL). */
int adc_record_count(const adc_ctx* ctx);
int adc_record_get(adc_ctx* ctx, int i, double* x, double* r, double* theta, int* root);

#ifdef __cplusplus
}
#endif

#endif /* ADC_H */
