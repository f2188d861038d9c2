// Host-side launchers of the HIP kernels.
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <vector>

#include "stp_internal.hpp"

namespace stp {

hipError_t launch_sigma1e(const DevSpace& S, bool cplx, const void* hp, const void* c, void* sigma, int n_vec,
                          hipStream_t st);
size_t sigma2e_tiled_lds(const Sigma2eSched& P, int nv, bool cplx);
hipError_t launch_sigma2e_tiled(const DevSpace& S, const Sigma2eSched& P, bool cplx, const void* gT, const void* c,
                                void* sigma, int n_vec, hipStream_t st);
bool symtile_supported(int deg_max, bool cplx);
// sigma = H c in one pass, Hermitian 4x4 tiles per intermediate determinant
// f32: integrals gT/hp are FP32 (complex FP32 when cplx); c and sigma stay FP64.
hipError_t launch_sigma_symtile(const DevSpace& S, int deg_max, bool cplx, bool f32, const void* gT, const void* hp,
                                const void* c, void* sigma, int n_vec, double e_core, hipStream_t st);
// sigma = H c in one pass over the (N-2)-electron pair intermediates; A is the
// pair-pair table A[(q,s)-pair * npairs + (p,r)-pair] (FP32 when f32)
bool pair_supported(int n_elec, int deg_max, bool cplx);
size_t pair_slice_bytes(int deg_max, int nv, bool cplx, bool f32);
// E: NULL (accumulate with device atomics) or pair_store_bytes of workspace
// (each pair contribution stored once, then summed per target: deterministic)
size_t pair_store_bytes(const DevSpace& S, bool cplx);
// optional callback around each launch (what: 0 the pair kernel, 1 the reduce)
struct LaunchMarks {
    void (*fn)(void* user, int what, bool start);
    void* user;
};
// sigma = e_core c + the stored pair contributions E (nv = 1 or 2 vectors of
// the store layout), summed in a fixed order.
hipError_t launch_pair_reduce(const DevSpace& S, bool cplx, int nv, void* sigma, const void* c, const void* E,
                              int n_vec, double e_core, hipStream_t st);
// BF16 matrix-core form of the pair sigma build: Ab holds the pair-pair table
// in bfloat16, row-major [P][Q] with npp (a multiple of 32) columns; complex:
// three matrices (real part, imaginary part, negated imaginary part).
// E non-null: store-and-reduce scatter, else device atomics.
// FP64 matrix-core form of the pair sigma build (v_mfma_f64_4x4x4f64), same
// arguments and scatter modes as launch_sigma_pair with the FP64 table.
bool pair_mf64_supported(int n_elec, int deg_max);
size_t pair_mf64_slice_bytes(int deg_max);
hipError_t launch_sigma_pair_mf64(const DevSpace& S, int deg_max, bool cplx, const void* A, const void* c,
                                  void* sigma, void* E, int n_vec, double e_core, const LaunchMarks* mk,
                                  hipStream_t st);
bool pair_mfma_supported(const DevSpace& S, int deg_max, bool cplx);
int pair_mfma_npp(int npairs);
hipError_t launch_sigma_pair_mfma(const DevSpace& S, int deg_max, bool cplx, const void* Ab, const void* c,
                                  void* sigma, void* E, int n_vec, double e_core, const LaunchMarks* mk,
                                  hipStream_t st);
hipError_t launch_sigma_pair(const DevSpace& S, int deg_max, bool cplx, bool f32, const void* A, const void* c,
                             void* sigma, void* E, int n_vec, double e_core, const LaunchMarks* mk, hipStream_t st);
// Grouped FP64 matrix-core form for spaces of one subspace: items of four
// intermediates sharing an (N-3)-electron core (build_pair_groups) take one
// 16-column product per table read; same scatter modes as launch_sigma_pair.
// f32: A is the FP32 table; products and accumulation in FP32.
struct HostSpace;
bool pair_grp_supported(const Space& sp);
int pair_grp_unit(const Space& sp);   // intermediates per item (8 or 4), 0: unsupported
size_t pair_grp_slice_bytes(const Space& sp);
bool build_pair_groups(const HostSpace& H, std::vector<GrpItem>& items);
hipError_t launch_sigma_pair_grp(const DevSpace& S, const GrpItem* items_dev, int nitems, bool cplx, bool f32,
                                 const void* A, const void* c, void* sigma, void* E, int n_vec, double e_core,
                                 const LaunchMarks* mk, hipStream_t st);
// Spectator-batched matrix-core form for spaces of several subspaces: the
// pair intermediates of a pair category that share the strings of subspaces
// 1..K-1 are contracted as one product over their padded pair list
// (build_sb_plan); contributions are added with device atomics.  f32: A is
// the FP32 table; products and accumulation in FP32.
bool pair_sb_supported(const Space& sp);
struct SbHostPlan {
    std::vector<SbCat> cats;
    std::vector<uint32_t> rows;
    std::vector<SbStream> streams;
    int cap = 0, nlmax = 0;
    int32_t sbegin[3][9] = {};
    int64_t nitems[3][8] = {};
};
bool build_sb_plan(const HostSpace& H, SbHostPlan& plan);
void sb_plan_counts(const SbHostPlan& plan, bool cplx, int nv, double* flops, int64_t* items);
size_t pair_sb_lds_bytes(int cap, int nlmax);
hipError_t launch_sigma_pair_sb(const DevSpace& S, const SbPlan& plan, bool cplx, bool f32, const void* A,
                                const void* c, void* sigma, int n_vec, double e_core, const LaunchMarks* mk,
                                hipStream_t st);
int64_t check_sb_host(const DevSpace& S, const SbHostPlan& plan, int64_t max_groups, int64_t* n_checked,
                      bool (*to_bits)(const void*, int64_t, uint64_t*), const void* user);
// sigma <- e_core * c (zero when e_core == 0)
hipError_t launch_fill_init(bool cplx, void* sigma, const void* c, double e_core, int64_t n, hipStream_t st);
// sigma += e_core * c
hipError_t launch_axpy_core(bool cplx, void* sigma, const void* c, double e_core, int64_t n, hipStream_t st);
int waves_per_group(size_t per_wave);
hipError_t launch_diag(const DevSpace& S, const double* hd, const double* JK, double e_core, double* out,
                       hipStream_t st);
// t_q = r_{root[q]} / (theta[q] - H_ii) (0 where |theta[q] - H_ii| < guard)
// for q < n <= PRE_MAX; r and t hold consecutive vectors of ld scalars
constexpr int PRE_MAX = 16;
hipError_t launch_precond(const DevSpace& S, bool cplx, const double* hd, const double* JK, double e_core,
                          const void* r, void* t, int64_t ld, int n, const int* root, const double* theta,
                          double guard, hipStream_t st);
// t_q <- 0 where |t_q,i| < eps ||t_q|| (Eq. sparsePreconditioner), ||t_q||^2
// read on the device at nrm2[slot[q] * stride] (real part), q < n <= PRE_MAX
hipError_t launch_eps_drop(bool cplx, void* t, int64_t ld, int64_t nd, int n, const int* slot, const double* nrm2,
                           int stride, double eps, hipStream_t st);
int topk_blocks(const DevSpace& S);
hipError_t launch_diag_topk(const DevSpace& S, const double* hd, const double* JK, double e_core, int k,
                            double* vals, int64_t* idx, hipStream_t st);
int dots_blocks(int64_t n);
// out[t * m + i] = <V_i | W_t> for i < m, t < nw (V_i = Vb + i ld, W_t = W +
// t ld); partial holds dots_blocks(n) * m * nw scalars
hipError_t launch_dots(bool cplx, const void* Vb, int64_t ld, int m, const void* W, int nw, int64_t n,
                       void* partial, void* out, hipStream_t st);
// Davidson Rayleigh-Ritz step for k <= PRE_MAX Ritz pairs (coefficients Y,
// m x k row-major; Z: coefficient changes or NULL; theta on the device):
// X = V Y, T = the preconditioned residuals (W Y - X theta) / (theta - H_ii)
// (0 where |theta - H_ii| < guard); out[12 (j / 4) + 4 q + j % 4] =
// ||r_j||^2, ||t_j||^2, max |(V Z)_j|^2 for q = 0, 1, 2 (12 ceil(k / 4)
// doubles); partial holds ritz_blocks(n, k) * 12 doubles
int ritz_blocks(int64_t n, int k);
hipError_t launch_ritz(const DevSpace& S, bool cplx, const double* hd, const double* JK, double e_core,
                       const void* V, const void* W, int64_t ld, int m, const void* Y, const void* Z, int k,
                       const double* theta, double guard, void* X, void* T, int64_t n, double* partial, double* out,
                       hipStream_t st);
// nx <= 4 vectors X_t from m vectors A_i (mode 0: X_t = sum_i A_i Y[i nx + t];
// mode 3: X_t -= sum_i A_i Y[t m + i]) and the Gram matrix of the results,
// gout[2 (4 t + s) + c] = real (c = 0) and imaginary (c = 1) part of
// <X_s | X_t> (a 4 x 4 block of complex slots; real vectors: c = 1 is 0);
// partial holds comb_gram_blocks(n) * 32 doubles
int comb_gram_blocks(int64_t n);
hipError_t launch_comb_gram(bool cplx, const void* A, int64_t ld, int m, const void* Y, void* X, int nx, int64_t n,
                            int mode, double* partial, double* gout, hipStream_t st);
// X_j <- sum_i X_i Y[i kk + j], j < kk <= min(32, m), i < m, in place
hipError_t launch_combine_inplace(bool cplx, void* X, int64_t ld, int m, const void* Y, int kk, int64_t n,
                                  hipStream_t st);
hipError_t launch_combine(bool cplx, const void* A, const void* B, int64_t ld, int m, const void* Y, int k,
                          const double* theta, void* X, void* R, int64_t n, int mode, hipStream_t st);
hipError_t launch_scale(bool cplx, void* x, double s, int64_t n, hipStream_t st);
int64_t check_moves_host(const DevSpace& S, int64_t max_dets_per_cat, int64_t* n_checked,
                         bool (*to_bits)(const void*, int64_t, uint64_t*), const void* user);
hipError_t launch_unit(bool cplx, void* x, int64_t n, int64_t at, hipStream_t st);
int64_t check_pairs_host(const DevSpace& S, int64_t max_dets_per_cat, int64_t* n_checked,
                         bool (*to_bits)(const void*, int64_t, uint64_t*), const void* user);

// categorical compression (csc.hip)
void build_csc_pcat_of(const HostSpace& H, std::vector<int32_t>& out);
size_t csc_slice_bytes(int deg_max, bool cplx);
hipError_t launch_csc_compress(const DevSpace& S, bool cplx, const void* x, double thresh, const int64_t* cat_off,
                               int64_t* cnt, int64_t* cat_ptr, uint32_t* A, void* V, int64_t cap, hipStream_t st);
hipError_t launch_csc_expand(const DevSpace& S, bool cplx, const int64_t* cat_ptr, const int64_t* cat_off,
                             const uint32_t* A, const void* V, void* x, hipStream_t st);
hipError_t launch_csc_sigma(const DevSpace& S, bool cplx, const int64_t* cat_ptr, const uint32_t* A, const void* V,
                            const void* pA, const int32_t* pcat_of, double e_core, int deg_max, uint32_t* bitmap,
                            int64_t nwords, int64_t* list, unsigned long long* count, int64_t cap, void* sigma,
                            hipStream_t st);
hipError_t launch_csc_search_test(const uint32_t* A, int64_t n, const int64_t* starts, const uint32_t* xs,
                                  int64_t* out, int64_t m, hipStream_t st);
int64_t csc_exp_search_host(const uint32_t* A, int64_t n, int64_t i, uint32_t x);

}  // namespace stp
