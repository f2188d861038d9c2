/*
 * stpci_testing.h -- test hooks of libstpci (not part of the solver API).
 */
#ifndef STPCI_TESTING_H
#define STPCI_TESTING_H

#include "stpci.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Eigen-decomposition of a Hermitian n x n matrix with the host eigensolver
 * solver that the Davidson driver uses for its projected problem.
 * A: host [n][n] complex (interleaved), read only; w: n eigenvalues
 * ascending; V: [n][n] complex, eigenvectors as columns.  Host memory only;
 * returns STPCI_EINVAL for n < 1 or NULL pointers. */
stpci_status stpci_test_heev(int n, const double* A, double* w, double* V);

/* Run, on the host, the move enumeration and sign/address arithmetic that the
 * sigma kernels use, for up to max_dets_per_cat determinants of every
 * intermediate category (evenly spaced), and verify each move against the
 * global sign rule and the address-to-determinant map.  n_checked: moves
 * checked; n_bad: moves whose target address is outside the space, holds the
 * wrong determinant, or carries the wrong sign. */
stpci_status stpci_test_moves(const stpci_ctx* ctx, int64_t max_dets_per_cat, int64_t* n_checked,
                              int64_t* n_bad);

/* The same for the pair kernel: for up to max_dets_per_cat (N-2)-electron
 * intermediates K' of every pair category, run the kernel's pair-slot
 * arithmetic on the host and verify that every slot's target address holds
 * K' + {p, r} (p < r both empty in K', the pair the slot reports) with the
 * sign of a+_p a+_r |K'> from the global occupation bits.  n_checked: slots
 * checked; n_bad: slots that fail. */
stpci_status stpci_test_pairs(const stpci_ctx* ctx, int64_t max_dets_per_cat, int64_t* n_checked,
                              int64_t* n_bad);

/* Build, on the host, the items of the grouped pair kernel (spaces of one
 * subspace: up to `unit` (N-2)-electron intermediates that each add one
 * electron to a shared (N-3)-electron core) and verify them: every
 * intermediate in exactly one item, every member the core plus one electron,
 * 1..unit members per item.  n_items: items built; n_bad: violations; unit:
 * intermediates per item the kernel takes (8 or 4, by the LDS its slice
 * needs).  Returns STPCI_EINVAL when the grouped kernel does not apply to the
 * space (more than one subspace, fewer than three electrons). */
stpci_status stpci_test_pair_groups(const stpci_ctx* ctx, int64_t* n_items, int64_t* n_bad, int* unit);

/* Work of the spectator-batched pair kernel for an n_vec-vector sigma (for
 * reports): the matrix-core flops its launches execute, padding included
 * (per item: row tiles x steps x column groups x 2048 flop per
 * v_mfma_f64_16x16x4f64, twice for complex integrals), and the number of
 * items.  STPCI_EINVAL when the kernel does not apply to the space. */
stpci_status stpci_sb_counts(const stpci_ctx* ctx, int n_vec, double* mfma_flops, int64_t* items);

/* The Davidson corrections of Eq. sparsePreconditioner as the solver forms
 * them: for q < n, s_q,i = r_q,i / (theta[q] - H_ii) where |theta[q] - H_ii|
 * >= 1e-12 (H_ii computed on the fly from the occupation bits), else 0; then
 * with eps > 0, t_q,i = s_q,i where |s_q,i| >= eps ||s_q||, else 0.
 * r_dev, t_dev: device [n][n_dets] in the scalar type of the integrals;
 * theta: host, n values; n in [1, 16]; eps in [0, 1) (else STPCI_EINVAL).
 * Synchronises the context stream. */
stpci_status stpci_test_precond(stpci_ctx* ctx, const void* r_dev, void* t_dev, int n, const double* theta,
                                double eps);

/* Classical Gram-Schmidt passes against the basis made by the last Davidson
 * run (one or two per iteration that added directions: the second only where
 * the first removed more than half of a correction's squared norm). */
stpci_status stpci_test_dav_cgs_passes(const stpci_ctx* ctx, int* passes);

/* The solver's fused Rayleigh-Ritz pass on given vectors: V (m consecutive
 * basis vectors) and W (m vectors; in the solver W = H V), coefficients Y and
 * optional coefficient changes Z (m x k, row-major) and Ritz values theta:
 *   x_j = V y_j, r_j = W y_j - theta_j x_j,
 *   t_j,i = r_j,i / (theta_j - H_ii) where |theta_j - H_ii| >= 1e-12, else 0
 *   (Eq. sparsePreconditioner before its eps drop; H_ii on the fly),
 * x_j to x_dev and t_j to t_dev ([k][n_dets] each); red[3 j], red[3 j + 1],
 * red[3 j + 2] = ||r_j||^2, ||t_j||^2 and max_i |(V z_j)_i|^2 (0 when z is
 * NULL).  Vectors on the device in the scalar type of the integrals; y, z
 * and theta on the host, complex entries as (re, im) pairs; m in [1, 64], k
 * in [1, 16] (else STPCI_EINVAL).  Synchronises the context stream. */
stpci_status stpci_test_ritz(stpci_ctx* ctx, const void* v_dev, const void* w_dev, int m, const double* y,
                             const double* z, int k, const double* theta, void* x_dev, void* t_dev, double* red);

/* Build, on the host, the plan of the spectator-batched pair kernel (spaces
 * of several subspaces: the pair intermediates of a pair category that share
 * their strings on subspaces 1..K-1 form a group, contracted over a padded
 * pair list that holds every orbital of the last subspace) and run the
 * kernel's row and entry arithmetic for up to max_groups groups of every
 * pair category (evenly spaced), every padded row and every member: an entry
 * must vanish exactly when its pair meets an orbital occupied in the member,
 * and otherwise address K' + {p, r} in the space with the sign of
 * a+_p a+_r |K'> from the global occupation bits; each member must meet
 * every pair that leads from it into the space exactly once.  n_checked:
 * entries checked; n_bad: violations.  Returns STPCI_EINVAL when the kernel
 * does not apply (one subspace, fewer than two electrons, a last subspace of
 * more than 31 spin-orbitals). */
stpci_status stpci_test_sb(const stpci_ctx* ctx, int64_t max_groups, int64_t* n_checked, int64_t* n_bad);

/* The exponential search of Alg. sigmaBuild (subroutine exponentialSearch)
 * as the compressed sigma build runs it: the lowest j in [i, n) with
 * a[j] >= x, or n, for a ascending on [i, n) (host arrays).  -1 for invalid
 * arguments (a NULL, n < 0, i outside [0, n]). */
int64_t stpci_test_exp_search(const uint32_t* a, int64_t n, int64_t i, uint32_t x);

/* The same search on the device: out_dev[t] = search(a_dev, n, starts_dev[t],
 * xs_dev[t]) for t < m, one thread each, on `stream` (a hipStream_t, NULL:
 * the default stream); starts must lie in [0, n].  Device arrays. */
stpci_status stpci_test_exp_search_dev(const uint32_t* a_dev, int64_t n, const int64_t* starts_dev,
                                       const uint32_t* xs_dev, int64_t* out_dev, int64_t m, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* STPCI_TESTING_H */
