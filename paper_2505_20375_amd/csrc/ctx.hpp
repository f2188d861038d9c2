// Internal state of one stpci context.
#pragma once
#include <hip/hip_runtime_api.h>

#include <complex>
#include <string>
#include <vector>

#include "../../include/stpci.h"
#include "space.hpp"

namespace stp {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    void free_() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

struct KernelEvent {
    int kind;  // 0 sigma1e, 1 sigma2e
    hipEvent_t a, b;
};

struct DavRecord {
    std::vector<double> e, r;
    std::vector<double> dc;   // max |x_j - phase x_j(previous iteration)|, NaN on a run's first iteration
    int precision = 0;
};

// State of one Davidson run (see davidson.cpp).
struct DavState {
    stpci_dav_opts opts{};
    stpci_precision prec = STPCI_FP64;
    double tol = 0, final_tol = 0;
    int pidx = 0, kr_max = 0, mmax = 0, max_iter = 0;
    int m = 0;    // vectors in V with their W known
    int nv = 0;   // pending: W[m..m+nv) = H V[m..m+nv)
    int it = 0, it_prev = 0;
    double best_rn = -1.0;   // BF16 phase: smallest largest-residual so far
    int stall = 0;           // iterations since it last dropped by 10 %
    bool converged = false, done = false, active = false;
    std::vector<std::complex<double>> G;
    std::vector<double> theta, rn;
    int k_req = 0;                    // roots requested (opts.k may hold one more, see certify)
    std::vector<double> theta_prev;   // Ritz values of the previous iteration of this phase
    bool energy_stop = false;         // the FP64 refinement ended on refine_tol_energy
    bool products_ready = false;      // step-wise runs: the pending products were computed
    int cgs_passes = 0;               // Gram-Schmidt passes against V over the run
    // coordinates, in the current basis V, of the previous iteration's Ritz
    // vectors ([prev_rows][k], row-major; prev_rows <= m), for the restart and
    // the coefficient change
    std::vector<std::complex<double>> prev_coef;
    int prev_rows = 0;
};

}  // namespace stp

struct stpci_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    bool host_only = true;
    std::string err;

    // integrals (spin-orbital basis)
    bool have_ints = false;
    bool cplx = true;
    int M = 0;
    double e_core = 0.0;
    std::vector<double> h, g;      // interleaved if complex
    std::vector<double> hprime;    // h' = h - 1/2 sum_r (pr|rq)
    std::vector<double> gT;        // gT[(y*M + x)*M*M + (y'*M + x')] = (x' y' | y x)
    std::vector<double> hd, JK;    // Re h_ii ; (ii|jj) - (ij|ji)
    std::vector<float> gT32, hp32; // FP32 copies for the FP32 contraction
    std::vector<double> pA;        // pair-pair table of the pair kernel (built with the space)
    std::vector<float> pA32;
    std::vector<uint16_t> pAbf;   // bfloat16 pair-pair table of the matrix-core form

    // space
    bool have_space = false;
    stp::HostSpace hs;

    // device copies
    bool prepared = false;
    stp::DevBuf d_cats, d_tabs, d_bits, d_ann, d_cre, d_work_cat, d_work_begin, d_space_begin;
    stp::DevBuf d_hp, d_gT, d_hd, d_JK;
    stp::DevBuf d_gT32, d_hp32;
    bool have32 = false;
    bool have_bf = false;
    stp::DevBuf d_pcats, d_pwork, d_pslot, d_pA, d_pA32, d_pAbf;
    stp::DevBuf d_E;         // pair contributions of the store-and-reduce scatter
    stp::DevBuf d_csc_cnt, d_csc_pcat, d_csc_bitmap, d_csc_list, d_csc_count;   // compressed-vector work
    // pinned host staging of the solver's small transfers (coefficients up,
    // dot products down): copies from it are asynchronous, so an upload does
    // not wait for the stream; regions are reused after the next stream sync
    void* pin = nullptr;
    size_t pin_bytes = 0, pin_off = 0;
    bool csc_pcat_ready = false;
    bool pair_store = false; // pair kernel: store-and-reduce (true) or device atomics
    bool pair_mf64 = false;   // FP64 pair products on the matrix cores (else the vector-ALU tiles)
    bool pair_grp = false;    // FP64 pair products of grouped intermediates (spaces of one subspace)
    std::vector<stp::GrpItem> grp_items;
    stp::DevBuf d_grp;
    bool pair_sb = false;     // spectator-batched matrix-core products (spaces of several subspaces)
    stp::SbPlan sb_plan{};
    stp::DevBuf d_sbcats, d_sbrows, d_sbstreams;
    int kernel_req = -1;   // requested sigma kernel (stpci_set_sigma_kernel), -1: automatic
    stp::DevSpace dev{};

    // schedule of the tiled two-electron kernel
    stp::DevBuf d_s2blocks, d_ygroup;
    stp::Sigma2eSched s2{};
    // sigma kernel: 0 simple per-determinant, 1 row-tiled, 2 wavefront, 3 Hermitian tiles over
    // one-move intermediates, 4 Hermitian tiles over pair intermediates
    int s2_kernel = 4;

    // Davidson workspace
    stp::DevBuf d_V, d_W, d_X, d_T, d_partial, d_small, d_topv, d_topi;
    std::vector<stp::DavRecord> history;
    int hist_k = 0;
    int nsigma[3] = {0, 0, 0};   // sigma builds of the last Davidson run: FP64, FP32, BF16 (vectors)
    int cert_k = 0;              // roots of the last collected run, with their gap bounds
    std::vector<double> cert_gamma, cert_bound;
    stp::DavState dav;

    // profiling
    bool profile = false;
    std::vector<stp::KernelEvent> events;

    ~stpci_ctx();
};

namespace stp {
stpci_status set_err(stpci_ctx* c, stpci_status s, const std::string& msg);
stpci_status hip_check(stpci_ctx* c, hipError_t e, const char* what);
stpci_status prepare(stpci_ctx* c);
stpci_status ensure(stpci_ctx* c, DevBuf& b, size_t bytes, const char* what);
// ws: the pair kernels' store-and-reduce workspace to use instead of the
// context's own (NULL: the context's, allocated on first use)
stpci_status sigma_impl(stpci_ctx* c, const void* cin, void* sout, int n_vec, stpci_precision prec,
                        void* ws = nullptr);
hipError_t scratch_setup(int device);   // noalloc.hip
stpci_status ensure32(stpci_ctx* c);  // upload the FP32 integral copies once
stpci_status ensure_bf16(stpci_ctx* c);  // upload the bfloat16 pair table once
int select_kernel(const stpci_ctx* c);
int64_t device_table_bytes(const stpci_ctx* c, bool f32);
size_t scalar_bytes(const stpci_ctx* c);
// step-wise Davidson (davidson.cpp)
stpci_status dav_begin(stpci_ctx* c, const stpci_dav_opts* o);
int64_t dav_device_bytes(const stpci_ctx* c, const stpci_dav_opts& o);
bool dav_pending(stpci_ctx* c, const void** in, void** out, int* n, stpci_precision* prec);
stpci_status dav_step_after_sigma(stpci_ctx* c, int* finished);
stpci_status dav_collect(stpci_ctx* c, double* energies, double* resid, void* vecs_dev, int* n_iter);
}  // namespace stp
