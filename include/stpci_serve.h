/*
 * stpci_serve.h -- continuous-batching request server of libstpci.
 *
 * Serving many CI solves of different sizes on one device is not part of
 * arXiv:2505.20375; each request is the paper's problem (integrals, an
 * STP-DAS space, k lowest roots by Davidson with residual-norm convergence,
 * Results and Methods), solved with the same sigma kernels and solver as
 * stpci_davidson.  The server adds the scheduling around them:
 *
 *  - stpci_server_submit copies a request's integrals and space, builds its
 *    host tables and computes its exact device footprint (tables, integrals,
 *    Davidson vectors and workspace; for requests whose products take the
 *    sigma kernel's own workspace: the store-and-reduce workspace where it
 *    fits 1 GB -- larger ones use device atomics -- and the item list of the
 *    grouped kernel, counted as one item per intermediate).  Requests wait
 *    in FIFO order.
 *  - stpci_server_tick admits waiting requests, oldest first, while fewer
 *    than max_active are active and their footprints fit mem_budget_bytes
 *    (admission stops at the first request that does not fit, so later ones
 *    never overtake it); then launches the pending sigma products of all
 *    active requests, each with the request's own kernel on the request's
 *    own stream, back to back, so that they overlap on the device; then
 *    advances each active request by one
 *    Davidson iteration and retires the finished ones, releasing their
 *    device memory.  A request's vectors stay on the device from admission
 *    to retirement.
 *  - Results and timings (submission, admission, completion; host monotonic
 *    clock in seconds) remain readable after retirement.
 *
 * A request's result does not depend on its co-tenants except through the
 * summation order of floating-point atomics inside the sigma kernel: energies
 * alone and in a mix agree to rounding (far below 1e-9 Eh).
 *
 * Memory: the server copies everything a request needs at submission; the
 * caller keeps ownership of its arrays.  Device memory of a request is
 * allocated by the server on admission and freed on retirement or
 * cancellation.  The server is used by one host thread at a time.  Each
 * active request's work (sigma products and Davidson vector algebra) runs on
 * a stream the server owns (default priority, reused across requests); the
 * Davidson iterations are advanced by up to 8 host worker threads inside
 * stpci_server_tick.  The stream given at creation is the one the requests'
 * host-side setup uses.
 * Errors: every call returns a status; stpci_server_last_error() describes
 * the last server-level failure.  A request that fails on the device is
 * retired with its status (STPCI_ENOCONV counts as finished, with the
 * energies and residuals reached).
 */
#ifndef STPCI_SERVE_H
#define STPCI_SERVE_H

#include "stpci.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stpci_server stpci_server;

/* One solve request.  n_orb, scalar, spin_free, h, g, e_core: as for
 * stpci_set_integrals; n_elec, n_sub, sub_size, win_lo, win_hi: as for
 * stpci_set_space; opts: Davidson options (guess_dev is ignored). */
typedef struct {
    int n_orb;
    stpci_scalar scalar;
    int spin_free;
    const void* h;
    const void* g;
    double e_core;
    int n_elec;
    int n_sub;
    const int* sub_size;
    const int* win_lo;
    const int* win_hi;
    const stpci_dav_opts* opts;
} stpci_request;

typedef enum {
    STPCI_REQ_QUEUED = 0,
    STPCI_REQ_ACTIVE = 1,
    STPCI_REQ_DONE = 2,
    STPCI_REQ_FAILED = 3,
    STPCI_REQ_CANCELLED = 4
} stpci_request_state;

/* Create a server on HIP device hip_device and stream hip_stream (NULL: the
 * default stream).  mem_budget_bytes bounds the summed footprints of active
 * requests; max_active bounds their number (>= 1). */
stpci_status stpci_server_create(stpci_server** out, int hip_device, void* hip_stream, int64_t mem_budget_bytes,
                                 int max_active);
void stpci_server_destroy(stpci_server* srv);
const char* stpci_server_last_error(const stpci_server* srv);

/* Queue a request; *id receives its number (0, 1, ... in submission order).
 * STPCI_EINVAL for inconsistent inputs (as the context calls report them,
 * or k outside [1, min(16, n_dets)]); STPCI_ENOMEM when the request's
 * footprint alone exceeds the budget. */
stpci_status stpci_server_submit(stpci_server* srv, const stpci_request* req, int* id);

/* Remove a queued or active request and free its device memory; finished
 * requests are left as they are. */
stpci_status stpci_server_cancel(stpci_server* srv, int id);

/* One scheduling step (admission, the sigma products of the active
 * requests, one Davidson iteration per active request, retirement).
 * n_pending: requests queued or active after the step; n_finished: requests
 * retired during it.  Request streams may still hold the tail of their
 * iteration's work, which their next products follow in stream order. */
stpci_status stpci_server_tick(stpci_server* srv, int* n_pending, int* n_finished);

/* State, results and timings of request id.  energies, resid: host arrays of
 * k doubles (filled once the request is done); any output may be NULL.
 * Returns the request's failure status when it failed, else STPCI_OK. */
stpci_status stpci_server_result(const stpci_server* srv, int id, int* state, double* energies, double* resid,
                                 int* n_iter, double* t_submit, double* t_admit, double* t_done);

/* Size and cost of request id: determinants, structural nonzeros of H, the
 * device footprint used for admission, and the sigma products (vectors) its
 * solve used (known once retired). */
stpci_status stpci_server_request_info(const stpci_server* srv, int id, int64_t* n_dets, double* nnz_h,
                                       int64_t* footprint_bytes, int* sigma_vectors);

/* Server counters: footprint bytes now active and the peak over all ticks,
 * the peak number of simultaneously active requests, ticks run and the
 * requests' sigma products launched (one per request and tick). */
stpci_status stpci_server_stats(const stpci_server* srv, int64_t* used_bytes, int64_t* peak_bytes, int* peak_active,
                                int64_t* ticks, int64_t* sigma_launches);

/* Wall seconds the server's ticks spent so far in their three phases:
 * admission (including each admitted request's Davidson start), launching
 * the sigma products, and the Davidson iterations of the stepped requests
 * (which wait for their products on their streams). */
stpci_status stpci_server_phase_times(const stpci_server* srv, double* admit_s, double* sigma_s, double* step_s);

#ifdef __cplusplus
}
#endif
#endif /* STPCI_SERVE_H */
