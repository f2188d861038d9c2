// C ABI of the categorical compression: dense <-> compressed vectors and
// sigma from a compressed vector (kernels in csc.hip).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <sstream>
#include <vector>

#include "../../include/stpci.h"
#include "../../include/stpci_testing.h"
#include "ctx.hpp"
#include "kernels.hpp"

using namespace stp;

static stpci_status csc_ready(stpci_ctx* c) {
    if (!c) return STPCI_EINVAL;
    stpci_status s = prepare(c);
    if (s) return s;
    return hip_check(c, hipSetDevice(c->device), "hipSetDevice");
}

extern "C" {

stpci_status stpci_csc_compress(stpci_ctx* c, const void* x_dev, double thresh, int64_t* cat_ptr_dev,
                                uint32_t* a_dev, void* v_dev, int64_t capacity, int64_t* nnz) {
    stpci_status s = csc_ready(c);
    if (s) return s;
    if (!x_dev || !cat_ptr_dev || !nnz || capacity < 0 || (capacity > 0 && (!a_dev || !v_dev)))
        return set_err(c, STPCI_EINVAL, "bad compression arguments");
    if (!(thresh >= 0.0) || !std::isfinite(thresh)) return set_err(c, STPCI_EINVAL, "thresh must be finite and >= 0");
    const int64_t nb = (c->hs.sp.ndets + 1023) / 1024;
    if ((s = ensure(c, c->d_csc_cnt, (size_t)(nb + 1) * 8, "compression block counts"))) return s;
    hipError_t e = launch_csc_compress(c->dev, c->cplx, x_dev, thresh, c->dev.space_begin, (int64_t*)c->d_csc_cnt.p,
                                       cat_ptr_dev, a_dev, v_dev, capacity, c->stream);
    if ((s = hip_check(c, e, "compression launch"))) return s;
    int64_t tot = 0;
    e = hipMemcpyAsync(&tot, cat_ptr_dev + c->hs.sp.nspace, 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if ((s = hip_check(c, e, "compression count"))) return s;
    *nnz = tot;
    if (tot > capacity) {
        std::ostringstream o;
        o << "the compressed vector has " << tot << " entries, more than the capacity " << capacity;
        return set_err(c, STPCI_ENOMEM, o.str());
    }
    return STPCI_OK;
}

stpci_status stpci_csc_expand(stpci_ctx* c, const int64_t* cat_ptr_dev, const uint32_t* a_dev, const void* v_dev,
                              void* x_dev) {
    stpci_status s = csc_ready(c);
    if (s) return s;
    if (!cat_ptr_dev || !x_dev) return set_err(c, STPCI_EINVAL, "bad expansion arguments");
    const size_t bytes = (size_t)c->hs.sp.ndets * scalar_bytes(c);
    hipError_t e = hipMemsetAsync(x_dev, 0, bytes, c->stream);
    if (e == hipSuccess) e = launch_csc_expand(c->dev, c->cplx, cat_ptr_dev, c->dev.space_begin, a_dev, v_dev, x_dev,
                                               c->stream);
    return hip_check(c, e, "expansion launch");
}

stpci_status stpci_sigma_csc(stpci_ctx* c, const int64_t* cat_ptr_dev, const uint32_t* a_dev, const void* v_dev,
                             void* sigma_dev) {
    stpci_status s = csc_ready(c);
    if (s) return s;
    if (!cat_ptr_dev || !sigma_dev) return set_err(c, STPCI_EINVAL, "bad sigma arguments");
    if (c->s2_kernel != 4 || !c->d_pA.p)
        return set_err(c, STPCI_EINVAL, "sigma of a compressed vector needs the pair form (N >= 2, pair kernel)");
    const int deg = c->hs.pmax_deg;
    const size_t lds = 4 * csc_slice_bytes(deg, c->cplx);
    if (lds > 160 * 1024) return set_err(c, STPCI_EINVAL, "pair degree too large for the compressed sigma kernel");
    if (!c->csc_pcat_ready) {
        std::vector<int32_t> tab;
        build_csc_pcat_of(c->hs, tab);
        s = ensure(c, c->d_csc_pcat, tab.size() * 4, "compressed-sigma pair-category table");
        if (!s) s = hip_check(c, hipMemcpy(c->d_csc_pcat.p, tab.data(), tab.size() * 4, hipMemcpyHostToDevice),
                              "pair-category table upload");
        if (s) return s;
        c->csc_pcat_ready = true;
    }
    // the number of entries bounds the marked intermediates
    int64_t nnz = 0;
    hipError_t e = hipMemcpyAsync(&nnz, cat_ptr_dev + c->hs.sp.nspace, 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if ((s = hip_check(c, e, "compressed vector size"))) return s;
    if (nnz < 0) return set_err(c, STPCI_EINVAL, "cat_ptr is not a valid prefix");
    const int64_t npw = c->hs.sp.npwork_dets;
    const int64_t npairs_occ = (int64_t)c->hs.sp.N * (c->hs.sp.N - 1) / 2;
    const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(npw, nnz * npairs_occ));
    const int64_t nwords = (npw + 31) / 32;
    if ((s = ensure(c, c->d_csc_bitmap, (size_t)nwords * 4, "intermediate bitmap")) ||
        (s = ensure(c, c->d_csc_list, (size_t)cap * 8, "intermediate list")) ||
        (s = ensure(c, c->d_csc_count, 8, "intermediate count")))
        return s;
    const size_t bytes = (size_t)c->hs.sp.ndets * scalar_bytes(c);
    e = hipMemsetAsync(sigma_dev, 0, bytes, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->d_csc_bitmap.p, 0, (size_t)nwords * 4, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->d_csc_count.p, 0, 8, c->stream);
    if (e == hipSuccess && nnz > 0)
        e = launch_csc_sigma(c->dev, c->cplx, cat_ptr_dev, a_dev, v_dev, c->d_pA.p, (const int32_t*)c->d_csc_pcat.p,
                             c->e_core, deg, (uint32_t*)c->d_csc_bitmap.p, nwords, (int64_t*)c->d_csc_list.p,
                             (unsigned long long*)c->d_csc_count.p, cap, sigma_dev, c->stream);
    return hip_check(c, e, "compressed sigma launch");
}

int64_t stpci_test_exp_search(const uint32_t* a, int64_t n, int64_t i, uint32_t x) {
    if (!a || n < 0 || i < 0 || i > n) return -1;
    return csc_exp_search_host(a, n, i, x);
}

stpci_status stpci_test_exp_search_dev(const uint32_t* a_dev, int64_t n, const int64_t* starts_dev,
                                       const uint32_t* xs_dev, int64_t* out_dev, int64_t m, void* stream) {
    if (n < 0 || m < 0 || (m > 0 && (!a_dev || !starts_dev || !xs_dev || !out_dev))) return STPCI_EINVAL;
    hipError_t e = launch_csc_search_test(a_dev, n, starts_dev, xs_dev, out_dev, m, (hipStream_t)stream);
    return e == hipSuccess ? STPCI_OK : STPCI_EHIP;
}

}  // extern "C"
