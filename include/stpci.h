/*
 * stpci.h -- C ABI of the MI355X categorical STP-DAS configuration-interaction
 * library (libstpci.so).
 *
 * The library computes sigma = H c for a CI Hamiltonian over a categorically
 * compressed small-tensor-product distributed-active-space (STP-DAS)
 * wavefunction, and runs the Davidson eigensolver that calls it.  The
 * operations follow the Methods section of arXiv:2505.20375: the categorical
 * vector C = (+)_B C^B (Results, categorical compression), the sigma build of
 * Eqs. sigmaL / sigmaL1e / sigmaL2e, the Davidson solver with the
 * preconditioner of Eq. sparsePreconditioner, and the residual-based
 * convergence test.
 *
 * Conventions shared by every call
 * --------------------------------
 * Hamiltonian.  H = e_core + sum_pq h_pq a+_p a_q
 *                 + 1/2 sum_pqrs (pq|rs) a+_p a+_r a_s a_q,
 *   with two-electron integrals in chemists' (Mulliken) order,
 *   g[p][q][r][s] = (pq|rs).  h must be Hermitian; g must satisfy
 *   (pq|rs) = (rs|pq) and (pq|rs) = conj((qp|sr)).
 * Space.  The M spin-orbitals are split into n_sub contiguous subspaces
 *   (distributed active spaces) of sizes sub_size[k]; a determinant belongs to
 *   the space when its electron count in subspace k lies in the inclusive
 *   window [win_lo[k], win_hi[k]].  A category is one occupation tuple
 *   (n_1..n_K) of the space.  Determinant |b> = a+_{i1}...a+_{iN}|0>,
 *   i1 < ... < iN (bit p of b set <=> spin-orbital p occupied).
 * Vector layout.  A CI vector is the concatenation of one dense block per
 *   category, categories in lexicographic order of (n_1..n_K); inside a block
 *   the element of local strings (s_1..s_K) sits at row-major position
 *   sum_k rank(s_k) * stride_k (subspace 1 slowest), rank = colexicographic
 *   rank of the local occupation mask among masks of equal popcount (the
 *   ascending order of the mask values).  n_vec vectors are stored one after
 *   the other ([n_vec][n_dets]).  Complex values are interleaved (re, im)
 *   doubles, the layout of torch.complex128.
 * Memory.  Host arrays passed in are copied; the caller keeps ownership.
 *   Device pointers (suffix _dev) are caller-owned HIP device allocations on
 *   the context's device; the library never frees them.  The context owns its
 *   tables, integrals, solver vectors and workspace and frees them in
 *   stpci_destroy.
 * Streams.  All device work of a context runs in order on the stream given
 *   to stpci_create (NULL: the default stream).  Calls returning results to
 *   host memory synchronise that stream; stpci_sigma does not.
 * Errors.  Every call returns a status; nothing aborts, throws or exits
 *   across the ABI.  stpci_last_error() describes the last failure on a
 *   context.  A context is used by one host thread at a time.
 */
#ifndef STPCI_H
#define STPCI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stpci_ctx stpci_ctx;

typedef enum {
    STPCI_OK = 0,
    STPCI_EINVAL = -1,   /* invalid argument: shape, symmetry, empty space, NULL pointer */
    STPCI_ENOMEM = -2,   /* device memory budget exceeded or allocation failed */
    STPCI_EHIP = -3,     /* a HIP runtime call failed */
    STPCI_ENOCONV = -4,  /* Davidson reached max_iter (results hold the last iterate) */
    STPCI_ESTATE = -5    /* call order: integrals/space missing, or host-only context */
} stpci_status;

typedef enum { STPCI_REAL64 = 0, STPCI_COMPLEX128 = 1 } stpci_scalar;

/* Arithmetic of the category-block contractions (sigma build).  The Davidson
 * residual, orthogonalisation and subspace problem are always FP64.
 *  STPCI_FP64: FP64 throughout.
 *  STPCI_FP32: integrals, coefficients and products in FP32, sums over the
 *    contraction in FP32 and FP64, sigma FP64 (tile and pair kernels).
 *  STPCI_BF16: pair kernel only; each batch of 16 / n pair intermediates
 *    (n = vectors per pass, 1 or 2) is contracted as one dense product over
 *    all pairs on the matrix cores (bfloat16 integrals and coefficients, FP32
 *    accumulation), the per-target sums in FP64.  Relative sigma error of
 *    the order of the bfloat16 rounding (2^-9); requires the workgroup's LDS
 *    slice (pair table width rounded to 32, 16 / n intermediates) to fit
 *    160 KB, else STPCI_EINVAL.  Not in the paper (which is FP64 throughout). */
typedef enum { STPCI_FP64 = 0, STPCI_FP32 = 1, STPCI_BF16 = 2 } stpci_precision;

/* Create a context on HIP device `hip_device` issuing work on `hip_stream`
 * (a hipStream_t, NULL for the default stream).  hip_device = -1 creates a
 * host-only context: space and table queries work, device calls return
 * STPCI_ESTATE. */
stpci_status stpci_create(stpci_ctx** out, int hip_device, void* hip_stream);

/* Free every allocation made by the context.  NULL-safe. */
void stpci_destroy(stpci_ctx* ctx);

/* Text of the last error on ctx (valid until the next call on ctx). */
const char* stpci_last_error(const stpci_ctx* ctx);

/* Set the Hamiltonian (the inputs h'_pq and g_pqrs of Eqs. sigmaL1e/sigmaL2e
 * are derived from it: h'_pq = h_pq - 1/2 sum_r (pr|rq)).
 * n_orb: number of spin-orbitals, or of spatial orbitals when spin_free = 1
 *   (then the space is built over 2*n_orb spin-orbitals, alpha block first,
 *   with h_so = h (x) 1 and (ps qs'|rt st') = (pq|rs) d_ss' d_tt').
 * h: [n_orb][n_orb], g: [n_orb]^4 in the scalar type given.
 * Returns STPCI_EINVAL if h is not Hermitian or g breaks the symmetries
 * above (tolerance 1e-12 relative to the largest element). */
stpci_status stpci_set_integrals(stpci_ctx* ctx, int n_orb, stpci_scalar scalar, int spin_free,
                                 const void* h, const void* g, double e_core);

/* Set the distributed-active-space partition and the occupation windows
 * (Results: STP-DAS partition and categories).  n_sub <= 8, each subspace at
 * most 32 spin-orbitals, at most 64 in total.  An empty space is
 * STPCI_EINVAL.  The partition must cover the spin-orbitals of the
 * integrals (checked when both are set). */
stpci_status stpci_set_space(stpci_ctx* ctx, int n_elec, int n_sub, const int* sub_size, const int* win_lo,
                             const int* win_hi);

/* Space summary.  Any output pointer may be NULL.
 * n_dets: determinants; n_cat: categories; bytes_per_vec: bytes of one CI
 * vector; w_sigma_macs: multiply-adds of one sigma build in the resolution
 * over intermediate determinants, W1 + W2 with W1 = sum_B |B| deg(B),
 * W2 = sum_C |C| deg(C)^2 (deg = one-electron moves into the space);
 * nnz_h: nonzero couplings <L|H|K> allowed between space determinants. */
stpci_status stpci_space_info(const stpci_ctx* ctx, int64_t* n_dets, int* n_cat, int64_t* bytes_per_vec,
                              double* w_sigma_macs, double* nnz_h);

/* Algorithmic work of one sigma build for one vector, split as in the
 * two-electron resolution: w1 = sum_B |B| deg(B) one-electron multiply-adds
 * (Eq. sigmaL1e), w2 = sum_C |C| deg(C)^2 two-electron multiply-adds over the
 * intermediate categories C (Eq. sigmaL2e), n_intermediate = number of
 * intermediate determinants, max_deg = largest move count of a determinant.
 * Any output may be NULL. */
stpci_status stpci_work_counts(const stpci_ctx* ctx, double* w1, double* w2, int64_t* n_intermediate,
                               int* max_deg);

/* Category `cat` (0-based, lexicographic): occupation tuple occ[n_sub],
 * offset of its block in the vector, and its number of determinants. */
stpci_status stpci_category(const stpci_ctx* ctx, int cat, int* occ, int64_t* offset, int64_t* n_dets);

/* Global occupation bitstring of the determinant at vector address addr. */
stpci_status stpci_address_to_det(const stpci_ctx* ctx, int64_t addr, uint64_t* occ_bits);

/* Pair-resolved work of one sigma build for one vector (the default kernel):
 * the two-electron operator, with the one-electron part folded in, resolved
 * over (N-2)-electron intermediates K' (the resolution of Eq. sigmaL2e taken
 * two electrons down): w_pair = sum_K' deg(K')^2 multiply-adds, deg = pair
 * creations p < r from K' into the space; n_pair_intermediate = number of K';
 * max_pair_deg = largest deg.  Zero for N < 2.  Any output may be NULL. */
stpci_status stpci_pair_counts(const stpci_ctx* ctx, double* w_pair, int64_t* n_pair_intermediate,
                               int* max_pair_deg);

/* Select the sigma kernel used from the next device call on: "pair" (pair
 * intermediates, the default where N >= 2 and the largest pair degree fits the
 * per-wavefront LDS slice; each pair contribution is stored once and summed
 * per target in a fixed order, so sigma is deterministic, when that workspace
 * -- n_dets * N (N - 1) / 2 * 2 scalars -- fits a quarter of the free device
 * memory or 1 GB, else contributions are added with device atomics; FP64
 * products run on the matrix cores when the pair table (16 or 8 bytes per
 * pair-pair entry) fits 4 MB, the L2 of one XCD, else on the vector ALUs with
 * Hermitian tiles; in a space of one subspace, with at least three electrons
 * and target indices below 2^30, the intermediates that add one electron to a
 * common (N-3)-electron core are contracted eight (or four) at a time against
 * one block of the pair table on the matrix cores, FP64 or, for
 * STPCI_FP32, FP32; in a space of several subspaces whose pair table exceeds
 * 4 MB, with at most 31 orbitals in the last subspace and M <= 64, the
 * products of all intermediates that share a pair category and the strings
 * of subspaces 1..K-1 are batched over the last subspace's strings into
 * 16 x 16 x 4 matrix-core products (FP64, or for STPCI_FP32 FP32 with FP64
 * sums), contributions added with device atomics),
 * "pair_atomic" (the same with device atomics),
 * "pair_mf64" and "pair_valu" (the pair form with the FP64 products forced
 * onto the matrix cores one intermediate at a time, or onto the vector ALUs),
 * "pair_grp" (the grouped form, one subspace only), "pair_sb" (the batched
 * form of spaces of several subspaces), "tile" (one-move intermediates
 * of Eq. sigmaL2e, Hermitian tiles, one- and two-electron parts fused),
 * "rowtile" (row-tiled one-move form, any degree: the fallback beyond the
 * tile kernel's limits), or "auto".  All compute the same sigma; an unknown
 * name is STPCI_EINVAL, and a kernel that cannot handle the space makes the
 * next device call fail with STPCI_EINVAL.  stpci_sigma_kernel reports the
 * kernel in use after the first device call (static string): "pair_grp",
 * "pair_mf64", "pair_valu" (store-and-reduce scatter), "pair_sb",
 * "pair_grp_atomic",
 * "pair_mf64_atomic", "pair_valu_atomic", "tile" or "rowtile". */
stpci_status stpci_set_sigma_kernel(stpci_ctx* ctx, const char* name);
stpci_status stpci_sigma_kernel(const stpci_ctx* ctx, const char** name);

/* sigma_dev = H c_dev for n_vec vectors, H including e_core (Eq. sigmaL:
 * one-electron part Eq. sigmaL1e plus two-electron part Eq. sigmaL2e, the
 * latter resolved over every intermediate one or two electrons away from the
 * space, including occupations outside the windows).  Device pointers,
 * [n_vec][n_dets] in the scalar type of the integrals; c_dev and sigma_dev
 * must not overlap.  prec: contraction arithmetic (stpci_precision).
 * Asynchronous on the context stream. */
stpci_status stpci_sigma(stpci_ctx* ctx, const void* c_dev, void* sigma_dev, int n_vec, stpci_precision prec);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sigma as stpci_sigma, same arguments, kernels and results, without any
 * device allocation.  The store-and-reduce workspace of the pair kernels
 * comes from a static device array of stpci_sigma_noalloc_max_bytes() bytes
 * (256 MiB) that each device holds from the first context created on it
 * until the process ends; every table must already be on the device, so
 * call stpci_sigma (with the same precision) or stpci_diagonal once after
 * the last stpci_set_integrals / stpci_set_space, else STPCI_ESTATE.  A space
 * whose workspace (n_dets * N (N - 1) / 2 * 2 scalars, when the context's
 * kernel uses the store-and-reduce scatter) exceeds the array: STPCI_EINVAL
 * with the sizes in stpci_last_error.  No profiling events are recorded.  All
 * calls on one device share the array and it keeps the last call's contents
 * (each sigma writes the part it reads in full before reading it): calls
 * that overlap on one device, on two streams or from two threads, race. */
stpci_status stpci_sigma_noalloc(stpci_ctx* ctx, const void* c_dev, void* sigma_dev, int n_vec,
                                 stpci_precision prec);
int64_t stpci_sigma_noalloc_max_bytes(void);

/* Categorical compression (Results, categorical compression): a vector as,
 * per space category B in order, the nonzero coefficients V^B and their
 * local addresses A^B (position inside the category's dense block),
 * ascending -- the CSC pair (V, A) of the paper.  Device arrays: cat_ptr
 * [n_cat + 1] int64 (entries of category B at cat_ptr[B] .. cat_ptr[B+1]-1),
 * a uint32 local addresses, v values in the scalar type of the integrals.
 *
 * stpci_csc_compress: compress the dense vector x_dev ([n_dets]), keeping
 *   the entries with |x_i| >= thresh (and != 0): thresh = 0 keeps every
 *   nonzero, thresh = eps ||x|| applies the drop of Eq. sparsePreconditioner.
 *   Writes cat_ptr_dev always, a_dev / v_dev up to `capacity` entries; *nnz =
 *   entries of the compressed vector; more than capacity: STPCI_ENOMEM (call
 *   again with arrays of *nnz entries).  Synchronises the context stream.
 * stpci_csc_expand: the dense vector of a compressed one (zeros elsewhere).
 * stpci_sigma_csc: sigma_dev = H c (dense, [n_dets], e_core included) for c
 *   given compressed, by the compression-compatible sigma build of Alg.
 *   sigmaBuild: only the (N-2)-electron pair intermediates reached from a
 *   nonzero coefficient are visited; each one's sorted pair lists are
 *   intersected with the categories' address lists by the exponential search
 *   of that algorithm, and only the matched coefficients are contracted, so
 *   the work follows the number of nonzeros, not the size of the space.
 *   FP64, device atomics (not bitwise deterministic); one vector.  Needs the
 *   pair form (N >= 2; STPCI_EINVAL otherwise).  A, V must be exactly as
 *   stpci_csc_compress writes them (ascending within each category, in
 *   range); the call reads cat_ptr_dev[n_cat] (synchronising the stream) and
 *   allocates its work arrays on first use. */
stpci_status stpci_csc_compress(stpci_ctx* ctx, const void* x_dev, double thresh, int64_t* cat_ptr_dev,
                                uint32_t* a_dev, void* v_dev, int64_t capacity, int64_t* nnz);
stpci_status stpci_csc_expand(stpci_ctx* ctx, const int64_t* cat_ptr_dev, const uint32_t* a_dev, const void* v_dev,
                              void* x_dev);
stpci_status stpci_sigma_csc(stpci_ctx* ctx, const int64_t* cat_ptr_dev, const uint32_t* a_dev, const void* v_dev,
                             void* sigma_dev);

/* diag_dev[i] = <i|H|i> (real, n_dets doubles).  The solver itself never
 * stores the diagonal; this call exists for checks. */
stpci_status stpci_diagonal(stpci_ctx* ctx, double* diag_dev);

/* Davidson options.  k: roots; max_iter: iterations; max_subspace: basis
 * vectors before a restart (0: max(8k, 32); capped at 64 and at n_dets, at
 * least 2k, and lowered when device memory is short); the restart keeps the
 * k Ritz vectors and the previous iteration's Ritz vectors (GD+k), so below
 * 3k vectors only some roots keep their previous iterate and convergence can
 * slow down or stall;
 * tol_residual: stop when every ||H x - E x|| <= tol_residual; eps_drop: the
 * epsilon of Eq. sparsePreconditioner in [0, 1): each correction s (the
 * residual divided by theta - H_ii, 0 where |theta - H_ii| < 1e-12) keeps only
 * its entries with |s_i| >= eps_drop ||s||; 0 gives the traditional Davidson
 * update with the 1e-12 guard (Eq. davidsonPreconditioner); the Results
 * section finds eps <~ 10 / sqrt(n_dets) safe.  precision: sigma arithmetic
 * inside the iteration; refine_tol_energy (>= 0; 0: off): with precision !=
 * FP64, the run carries one root more than k and the FP64 refinement phase
 * also ends, as converged, once every requested root's gap-theorem bound
 * ||r_j||^2 / gamma_j^- (stpci_dav_certificate) is below this value (the
 * residuals of that iteration are reported as they are; like any residual
 * bound it presumes that no eigenvalue below the Ritz values was missed);
 * guess_dev: k
 * starting vectors ([k][n_dets], device) or NULL for unit vectors at the k
 * lowest diagonal elements.  Out-of-range eps_drop or refine_tol_energy:
 * STPCI_EINVAL. */
typedef struct {
    int k;
    int max_iter;
    int max_subspace;
    double tol_residual;
    double eps_drop;
    stpci_precision precision;
    double refine_tol_energy;
    const void* guess_dev;
    int certify;   /* 1: converge one root more than k internally (to tol_residual), so
                    * that stpci_dav_certificate bounds every requested root; 0: off */
} stpci_dav_opts;

/* Lowest k eigenpairs (Results: Davidson with residual-norm convergence).
 * energies, resid: host arrays of k doubles (Ritz values and residual norms);
 * vecs_dev: device [k][n_dets] for the Ritz vectors or NULL; n_iter: host int
 * or NULL.  Returns STPCI_ENOCONV when max_iter is reached. */
stpci_status stpci_davidson(stpci_ctx* ctx, const stpci_dav_opts* opts, double* energies, double* resid,
                            void* vecs_dev, int* n_iter);

/* Error bounds of the roots of the last Davidson run (Methods, Eigenvalue
 * Bound Analysis): for root j < k, gamma_lower[j] is a lower bound of the gap
 * from E_j to the nearest other eigenvalue, from the Ritz values and
 * residual norms of the neighbouring roots -- (E_1 - ||r_1||) - E_0 for the
 * lowest root (Eq. gammaLowerBound), and for j > 0 also
 * E_j - (E_{j-1} + ||r_{j-1}||) -- and bound[j] = ||r_j||^2 / gamma_lower[j]
 * bounds |E_j - exact| by the gap theorem (infinity when gamma_lower[j] <= 0,
 * e.g. degenerate roots).  The last root run has no neighbour above: run
 * with certify = 1 to bound all k requested roots, otherwise root k - 1 gets
 * NaN.  The bounds hold when no eigenvalue lies between the computed ones.
 * Host arrays of k doubles (either may be NULL); STPCI_ESTATE before any run. */
stpci_status stpci_dav_certificate(const stpci_ctx* ctx, double* gamma_lower, double* bound);

/* Step-wise Davidson: the same solver as stpci_davidson cut into the steps a
 * caller needs to drive several problems side by side on one device (its own
 * admission and batching loop; stpci_server_* is such a loop):
 *   stpci_footprint_bytes(ctx, opts): device bytes the context holds during
 *     such a run -- tables, integrals (with the FP32 or bfloat16 copies the
 *     precision needs), the Davidson vectors and workspace; the pair kernels'
 *     store-and-reduce workspace is counted when it is at most 1 GB (a larger
 *     one is used only if it fits a quarter of the free device memory when
 *     the tables are built).  -1 for NULL arguments, missing integrals or
 *     space, or k out of range.  Host-only computation.
 *   stpci_dav_begin(ctx, opts): validate the options (as stpci_davidson),
 *     build the tables, allocate the vectors and set up the starting guess;
 *     its products become pending.
 *   stpci_dav_sigma_batched(ctxs, n): compute the pending sigma products of
 *     the n contexts (distinct, one device; contexts without pending products
 *     are skipped): each context's products with its own kernel on its own
 *     stream, launched back to back so that they overlap on the device
 *     (asynchronous: stpci_dav_finish_step orders after them on the
 *     context's stream).  On failure: the status of the first failing
 *     context (its stpci_last_error says why).
 *   stpci_dav_finish_step(ctx, done): one Davidson iteration on the computed
 *     products (Rayleigh-Ritz, residuals, convergence test, preconditioner,
 *     orthogonalisation, restart) on ctx's stream; *done = 1 when the run
 *     has ended (converged, max_iter or stagnation), else its next products
 *     are pending.  STPCI_ESTATE without a run in progress or before its
 *     products were computed.
 *   stpci_dav_result(ctx, energies, resid, vecs_dev, n_iter): results of the
 *     finished run as stpci_davidson returns them (STPCI_ENOCONV when it
 *     ended unconverged); STPCI_ESTATE before the run has ended.  The gap
 *     certificate is then available from stpci_dav_certificate. */
int64_t stpci_footprint_bytes(const stpci_ctx* ctx, const stpci_dav_opts* opts);
stpci_status stpci_dav_begin(stpci_ctx* ctx, const stpci_dav_opts* opts);
stpci_status stpci_dav_sigma_batched(stpci_ctx* const* ctxs, int n);
stpci_status stpci_dav_finish_step(stpci_ctx* ctx, int* done);
stpci_status stpci_dav_result(stpci_ctx* ctx, double* energies, double* resid, void* vecs_dev, int* n_iter);

/* Per-iteration record of the last Davidson run: iteration count, and for
 * iteration i < cap the Ritz values energies[i*k + j] and residual norms
 * resid[i*k + j].  Either array may be NULL. */
stpci_status stpci_dav_history(const stpci_ctx* ctx, int* n_iter, int cap, double* energies, double* resid);

/* Largest coefficient change of each Ritz vector per iteration of the last
 * Davidson run (Results: reported per iteration beside the energies and
 * residual norms): dc[i*k + j] = max_a |x_j[a] - ph x_j'[a]| for iteration
 * i < cap, x_j' the Ritz vector of the previous iteration and ph the unit
 * phase of <x_j'|x_j> (Ritz vectors are defined up to a phase); NaN on the
 * first iteration of a run and of the FP64 phase after a reduced-precision
 * one.  dc: host array of cap * k doubles. */
stpci_status stpci_dav_history_dc(const stpci_ctx* ctx, int cap, double* dc);

/* Sigma products spent by the last Davidson run, counted in vectors: with
 * precision STPCI_FP32 (STPCI_BF16) the run first iterates with FP32 (BF16)
 * contractions to a residual of max(tol_residual, 1e-4) (BF16:
 * max(tol_residual, 2e-2), or until its largest residual has not dropped by
 * 10 % over 8 iterations), then refines from those Ritz vectors with FP64
 * contractions to tol_residual (the reported energies and residuals are
 * always those of the FP64 phase).  sigma_fp32 counts the reduced-precision
 * products of either kind; stpci_dav_sigma_count splits them by precision. */
stpci_status stpci_dav_stats(const stpci_ctx* ctx, int* sigma_fp64, int* sigma_fp32);
stpci_status stpci_dav_sigma_count(const stpci_ctx* ctx, stpci_precision prec, int* n_vectors);

/* Kernel timing with HIP events on the context stream.  enable != 0 starts
 * recording every kernel launch of the sigma build; stpci_kernel_time
 * returns, for kernel `name`, the number of recorded launches and their
 * summed duration in milliseconds (synchronises).  Names: "sigma" (alias
 * "sigma2e": the FP64 one-pass sigma kernel -- the pair kernel, or the fused
 * one-move kernel), "sigma_fp32" (the same with the FP32 contraction),
 * "sigma_bf16" (the matrix-core pair kernel of the BF16 contraction),
 * "sigma_reduce" (the per-target sum of the pair kernel's store-and-reduce
 * scatter), "sigma1e" (the separate one-electron kernel of the earlier
 * one-move forms). */
stpci_status stpci_profile(stpci_ctx* ctx, int enable);
stpci_status stpci_kernel_time(stpci_ctx* ctx, const char* name, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* STPCI_H */
