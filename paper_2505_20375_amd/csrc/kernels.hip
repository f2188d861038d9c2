// HIP kernels of the categorical STP-DAS sigma build and the Davidson vector
// algebra, written for gfx950 (64-wide wavefronts).
//
// sigma = 1e-sigma + 2e-sigma (Eq. sigmaL):
//   1e: sigma_L += sum_pq h'_pq <L|E_pq|K> C_K          (Eq. sigmaL1e)
//   2e: sigma_L += 1/2 sum_J sum_pqrs <L|E_pq|J> (pq|rs) <J|E_rs|K> C_K   (Eq. sigmaL2e)
// with h'_pq = h_pq - 1/2 sum_r (pr|rq).  A "move" from a determinant D is
// the pair (x created, y annihilated) of E_xy applied to D; its target is the
// determinant reached and its sign that of E_xy D.  For an intermediate J the
// moves (x, y) give
//   D side:  K = E_xy J,  <J|E_rs|K> = sign  with (r, s) = (y, x)
//   E side:  L = E_xy J,  <L|E_pq|J> = sign  with (p, q) = (x, y)
// so the 2e update of J is e = G_J d with G_J[m', m] = (x' y' | y x) over
// the moves m', m of J, followed by sigma[target(m')] += 1/2 sign(m') e[m'].
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "stp_device.hpp"

namespace stp {

// ---------------------------------------------------------------------------
// 1e sigma: owner-computes over target determinants (writes every sigma_L)
// ---------------------------------------------------------------------------
template <bool CPLX>
__global__ __launch_bounds__(256) void k_sigma1e(DevSpace S, const typename VT<CPLX>::T* __restrict__ hp,
                                                 const typename VT<CPLX>::T* __restrict__ c,
                                                 typename VT<CPLX>::T* __restrict__ sigma, int n_vec) {
    using V = VT<CPLX>;
    using T = typename V::T;
    const int64_t nd = S.sp.ndets;
    const int M = S.sp.M;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < nd; L += (int64_t)gridDim.x * blockDim.x) {
        int a = find_segment(S.space_begin, S.sp.nspace, L);
        const Cat& A = S.cats[a];
        Det d;
        decode(S, A, L - A.offset, d);
        for (int v = 0; v < n_vec; ++v) {
            const T* cv = c + (int64_t)v * nd;
            T acc = V::zero();
            for (int slot = 0; slot < A.deg; ++slot) {
                int cls, xs, ys, lx, ly, sg;
                slot_move(S, A, d, slot, cls, xs, ys, lx, ly);
                int64_t t = apply_move(S, A, cls, xs, ys, lx, ly, d, sg);
                int x = S.sp.sub_off[xs] + lx, y = S.sp.sub_off[ys] + ly;
                // p = y, q = x
                acc = V::mad(V::scale(hp[y * M + x], (double)sg), cv[t], acc);
            }
            sigma[(int64_t)v * nd + L] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// Diagonal of H, computed on the fly (never stored by the solver):
//   H_LL = e_core + sum_{i in L} h_ii + sum_{i<j in L} [(ii|jj) - (ij|ji)]
// ---------------------------------------------------------------------------
__device__ __forceinline__ double diag_elem(const DevSpace& S, const double* __restrict__ hd,
                                            const double* __restrict__ JK, double e_core, int64_t L) {
    int a = find_segment(S.space_begin, S.sp.nspace, L);
    const Cat& A = S.cats[a];
    Det d;
    decode(S, A, L - A.offset, d);
    // occupied spin-orbitals as one mask (subspaces are contiguous, so the
    // bits ascend with the global index); walked in ascending order without
    // an index list, which would live in scratch memory
    uint64_t occ = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
        if (k < S.sp.K) occ |= (uint64_t)d.s[k] << S.sp.sub_off[k];
    const int M = S.sp.M;
    double e = e_core;
    for (uint64_t a = occ; a; ) {
        const int i = __builtin_ctzll(a);
        a &= a - 1;
        e += hd[i];
        const double* row = JK + i * M;
        for (uint64_t b = a; b; b &= b - 1) e += row[__builtin_ctzll(b)];
    }
    return e;
}

__global__ __launch_bounds__(256) void k_diag(DevSpace S, const double* hd, const double* JK, double e_core,
                                              double* out) {
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < S.sp.ndets;
         L += (int64_t)gridDim.x * blockDim.x)
        out[L] = diag_elem(S, hd, JK, e_core, L);
}

// Davidson preconditioner (Eq. sparsePreconditioner with eps = 0), for
// several roots at once (the diagonal element is formed once per determinant):
//   t_q,i = r_root(q),i / (theta_q - H_ii) if |theta_q - H_ii| >= guard, else 0.
struct PrecondRoots {
    int n;
    int root[PRE_MAX];
    double theta[PRE_MAX];
};
template <bool CPLX>
__global__ __launch_bounds__(256) void k_precond(DevSpace S, const double* hd, const double* JK, double e_core,
                                                 const typename VT<CPLX>::T* __restrict__ r,
                                                 typename VT<CPLX>::T* __restrict__ t, int64_t ld, PrecondRoots P,
                                                 double guard) {
    using V = VT<CPLX>;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < S.sp.ndets;
         L += (int64_t)gridDim.x * blockDim.x) {
        const double h = diag_elem(S, hd, JK, e_core, L);
        // (a fixed trip count: the argument arrays are indexed by constants)
#pragma unroll
        for (int q = 0; q < PRE_MAX; ++q) {
            if (q >= P.n) break;
            const double den = P.theta[q] - h;
            t[(int64_t)q * ld + L] =
                (fabs(den) >= guard) ? V::scale(r[(int64_t)P.root[q] * ld + L], 1.0 / den) : V::zero();
        }
    }
}

// Second step of Eq. sparsePreconditioner for several corrections at once:
// t_q,i = s_q,i if |s_q,i| >= eps ||s_q||, else 0, with ||s_q||^2 read on the
// device (the real part of the double at nrm2 + slot[q] * stride).
struct DropRoots {
    int n;
    int slot[PRE_MAX];
};
template <bool CPLX>
__global__ __launch_bounds__(256) void k_eps_drop(typename VT<CPLX>::T* __restrict__ t, int64_t ld, int64_t nd,
                                                  DropRoots D, const double* __restrict__ nrm2, int stride,
                                                  double eps) {
    using V = VT<CPLX>;
    double thr2[PRE_MAX];
#pragma unroll
    for (int q = 0; q < PRE_MAX; ++q) thr2[q] = (q < D.n) ? eps * eps * fmax(nrm2[(int64_t)D.slot[q] * stride], 0.0) : 0.0;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < nd; L += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int q = 0; q < PRE_MAX; ++q) {
            if (q >= D.n) break;
            typename V::T* x = t + (int64_t)q * ld + L;
            // |s| >= eps ||s||  <=>  |s|^2 >= eps^2 ||s||^2 (both sides non-negative)
            if (V::abs2(*x) < thr2[q]) *x = V::zero();
        }
    }
}

// Lowest-k diagonal entries (value, address), ties to the lower address.
constexpr int TOPK = 16;
__global__ __launch_bounds__(256) void k_diag_topk(DevSpace S, const double* hd, const double* JK, double e_core,
                                                   int k, double* out_val, int64_t* out_idx) {
    double bv[TOPK];
    int64_t bi[TOPK];
    for (int i = 0; i < TOPK; ++i) { bv[i] = 1e300; bi[i] = INT64_MAX; }
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < S.sp.ndets;
         L += (int64_t)gridDim.x * blockDim.x) {
        double e = diag_elem(S, hd, JK, e_core, L);
        if (e < bv[k - 1] || (e == bv[k - 1] && L < bi[k - 1])) {
            int p = k - 1;
            while (p > 0 && (e < bv[p - 1] || (e == bv[p - 1] && L < bi[p - 1]))) {
                bv[p] = bv[p - 1];
                bi[p] = bi[p - 1];
                --p;
            }
            bv[p] = e;
            bi[p] = L;
        }
    }
    __shared__ double sv[256 * TOPK];
    __shared__ int64_t si[256 * TOPK];
    for (int i = 0; i < k; ++i) { sv[threadIdx.x * k + i] = bv[i]; si[threadIdx.x * k + i] = bi[i]; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double rv[TOPK];
        int64_t ri[TOPK];
        for (int i = 0; i < k; ++i) { rv[i] = 1e300; ri[i] = INT64_MAX; }
        for (int q = 0; q < (int)blockDim.x * k; ++q) {
            double e = sv[q];
            int64_t L = si[q];
            if (e < rv[k - 1] || (e == rv[k - 1] && L < ri[k - 1])) {
                int p = k - 1;
                while (p > 0 && (e < rv[p - 1] || (e == rv[p - 1] && L < ri[p - 1]))) {
                    rv[p] = rv[p - 1];
                    ri[p] = ri[p - 1];
                    --p;
                }
                rv[p] = e;
                ri[p] = L;
            }
        }
        for (int i = 0; i < k; ++i) { out_val[blockIdx.x * k + i] = rv[i]; out_idx[blockIdx.x * k + i] = ri[i]; }
    }
}

// ---------------------------------------------------------------------------
// Vector algebra (memory-bound; wavefront + block reductions, fixed order)
// ---------------------------------------------------------------------------
// Davidson vector algebra with its reductions fused into the passes that
// produce the vectors.  A kernel accumulates per-thread sums (or maxima) of a
// few scalars over its elements and reduces them over the workgroup in a
// fixed order into partial[workgroup][slot]; a small second launch (k_fold)
// folds the workgroups' partials in a fixed order, one wavefront per output.
// The results do not depend on timing.  (A fold by the workgroup that
// finishes last would need a device-scope release fence in every workgroup,
// which writes the XCD's L2 back to memory: far slower here than a launch.)
// ---------------------------------------------------------------------------

// per-thread v[0..NS) -> part[0..NS): wavefront butterfly, then the four
// wavefronts in order; the slots whose bit is set in MAXMASK take the maximum
// (of non-negative values), the others the sum (256 threads)
template <int NS, uint64_t MAXMASK>
__device__ __forceinline__ void wg_partials(const double (&v)[NS], double* __restrict__ part) {
    __shared__ double red[4][NS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        constexpr uint64_t one = 1;
        const bool mx = (MAXMASK >> s) & one;
        double x = v[s];
        for (int off = 32; off > 0; off >>= 1) {
            const double y = __shfl_xor(x, off, 64);
            x = mx ? fmax(x, y) : x + y;
        }
        if (lane == 0) red[w][s] = x;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < NS; s += blockDim.x) {
        const bool mx = (MAXMASK >> s) & (uint64_t)1;
        part[s] = mx ? fmax(fmax(red[0][s], red[1][s]), fmax(red[2][s], red[3][s]))
                     : (red[0][s] + red[1][s]) + (red[2][s] + red[3][s]);
    }
}

// out[q] = fold over b < nblk of partial[b * stride + q], q < nout, one
// wavefront per output (lanes take b in order, then a butterfly): the sum,
// or for q % period >= max_from the maximum (of non-negative values)
__global__ __launch_bounds__(256) void k_fold(const double* __restrict__ partial, int nblk, int stride, int nout,
                                              int period, int max_from, double* __restrict__ out) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + w;
    if (q >= nout) return;
    const bool mx = (q % period) >= max_from;
    double x = 0.0;
    for (int b = lane; b < nblk; b += 64) {
        const double y = partial[(int64_t)b * stride + q];
        x = mx ? fmax(x, y) : x + y;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double y = __shfl_xor(x, off, 64);
        x = mx ? fmax(x, y) : x + y;
    }
    if (lane == 0) out[q] = x;
}

static hipError_t launch_fold(const double* partial, int nblk, int stride, int nout, int period, int max_from,
                              double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_fold, dim3((nout + 3) / 4), dim3(256), 0, st, partial, nblk, stride, nout, period, max_from,
                       out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
constexpr int DOTV = 8;   // vectors V_i per workgroup
constexpr int DOTW = 2;   // vectors W_t per workgroup

// partial[range][t * m + i] = sum over the element range of conj(V_i) W_t,
// for i < m, t < nw (V_i = Vb + i ld, W_t = W + t ld); k_fold adds the ranges.
// blockIdx.x: group of DOTV vectors V, blockIdx.y: element range, blockIdx.z:
// group of DOTW vectors W.  Each V element is read once per W group, each W
// element once per V group.
template <bool CPLX>
__global__ __launch_bounds__(256) void k_dots(const typename VT<CPLX>::T* __restrict__ Vb, int64_t ld, int m,
                                              const typename VT<CPLX>::T* __restrict__ W, int nw, int64_t n,
                                              typename VT<CPLX>::T* __restrict__ partial) {
    using V = VT<CPLX>;
    using T = typename V::T;
    const int i0 = blockIdx.x * DOTV;
    const int t0 = blockIdx.z * DOTW;
    T acc[DOTW][DOTV];
#pragma unroll
    for (int t = 0; t < DOTW; ++t)
#pragma unroll
        for (int i = 0; i < DOTV; ++i) acc[t][i] = V::zero();
    // DOTE elements per trip (stride apart), all read before any is added;
    // the sums still take the elements in the order of one per trip
    constexpr int DOTE = 2;
    const int64_t stride = (int64_t)gridDim.y * blockDim.x;
    for (int64_t e0 = blockIdx.y * (int64_t)blockDim.x + threadIdx.x; e0 < n; e0 += DOTE * stride) {
        T wv[DOTE][DOTW], a[DOTE][DOTV];
#pragma unroll
        for (int u = 0; u < DOTE; ++u) {
            const int64_t e = e0 + u * stride;
            const bool in = e < n;
#pragma unroll
            for (int t = 0; t < DOTW; ++t) wv[u][t] = (in && t0 + t < nw) ? W[(int64_t)(t0 + t) * ld + e] : V::zero();
#pragma unroll
            for (int i = 0; i < DOTV; ++i) a[u][i] = (in && i0 + i < m) ? Vb[(int64_t)(i0 + i) * ld + e] : V::zero();
        }
#pragma unroll
        for (int u = 0; u < DOTE; ++u) {
            if (e0 + u * stride >= n) break;
#pragma unroll
            for (int i = 0; i < DOTV; ++i)
                if (i0 + i < m) {
#pragma unroll
                    for (int t = 0; t < DOTW; ++t) acc[t][i] = V::cmad(a[u][i], wv[u][t], acc[t][i]);
                }
        }
    }
    // wavefront sums (fixed butterfly), then the 4 wavefronts in order
    __shared__ T red[4][DOTW * DOTV];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < DOTW; ++t)
#pragma unroll
        for (int i = 0; i < DOTV; ++i) {
            T x = acc[t][i];
            for (int off = 32; off > 0; off >>= 1) x = V::add(x, V::shfl_xor(x, off));
            if (lane == 0) red[wv][t * DOTV + i] = x;
        }
    __syncthreads();
    const int j = threadIdx.x;
    if (j < DOTW * DOTV) {
        const int t = j / DOTV, i = j % DOTV;
        if (t0 + t < nw && i0 + i < m) {
            const T x = V::add(V::add(red[0][j], red[1][j]), V::add(red[2][j], red[3][j]));
            partial[(int64_t)blockIdx.y * m * nw + (int64_t)(t0 + t) * m + i0 + i] = x;
        }
    }
}

// out_j = sum_i A_i * Y[i][j]  (+ beta_j * out_j when accumulate)   for j < k
// optionally R_j = sum_i B_i * Y[i][j] - theta_j * out_j
template <bool CPLX>
__global__ __launch_bounds__(256) void k_combine(const typename VT<CPLX>::T* __restrict__ A,
                                                 const typename VT<CPLX>::T* __restrict__ B, int64_t ld, int m,
                                                 const typename VT<CPLX>::T* __restrict__ Y, int k,
                                                 const double* __restrict__ theta,
                                                 typename VT<CPLX>::T* __restrict__ X,
                                                 typename VT<CPLX>::T* __restrict__ R, int64_t n, int mode) {
    // mode 0: X = A Y ; mode 1: X = A Y, R = B Y - X theta ; mode 2: X -= A Y (Y: m x k, row-major)
    // mode 3: X -= A Y with Y stored column by column (Y[j m + i], as the dot products lie)
    // Up to CB output columns per pass over A (and B), so that each element of
    // A is read once per CB columns; every sum runs over i in ascending order.
    using V = VT<CPLX>;
    using T = typename V::T;
    constexpr int CB = 4;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        for (int j0 = 0; j0 < k; j0 += CB) {
            T xs[CB], rs[CB];
#pragma unroll
            for (int jj = 0; jj < CB; ++jj) xs[jj] = rs[jj] = V::zero();
#pragma unroll 4
            for (int i = 0; i < m; ++i) {
                const T a = A[(int64_t)i * ld + e];
                const T b = (mode == 1) ? B[(int64_t)i * ld + e] : V::zero();
#pragma unroll
                for (int jj = 0; jj < CB; ++jj)
                    if (j0 + jj < k) {
                        const T y = (mode == 3) ? Y[(j0 + jj) * m + i] : Y[i * k + j0 + jj];
                        xs[jj] = V::mad(a, y, xs[jj]);
                        if (mode == 1) rs[jj] = V::mad(b, y, rs[jj]);
                    }
            }
#pragma unroll
            for (int jj = 0; jj < CB; ++jj) {
                const int j = j0 + jj;
                if (j >= k) break;
                if (mode >= 2) {
                    X[(int64_t)j * ld + e] = V::sub(X[(int64_t)j * ld + e], xs[jj]);
                } else {
                    X[(int64_t)j * ld + e] = xs[jj];
                    if (mode == 1) R[(int64_t)j * ld + e] = V::sub(rs[jj], V::scale(xs[jj], theta[j]));
                }
            }
        }
    }
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_scale(typename VT<CPLX>::T* __restrict__ x, double s, int64_t n) {
    using V = VT<CPLX>;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        x[e] = V::scale(x[e], s);
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_unit(typename VT<CPLX>::T* __restrict__ x, int64_t n, int64_t at) {
    using V = VT<CPLX>;
    typename V::T one = V::zero();
    *reinterpret_cast<double*>(&one) = 1.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        x[e] = (e == at) ? one : V::zero();
}

// Rayleigh-Ritz step for Ritz columns j0 .. j0 + 3 (j0 = 4 blockIdx.y):
//   x_j = V y_j,  r_j = W y_j - theta_j x_j,
//   t_j = r_j / (theta_j - H_ii), 0 where |theta_j - H_ii| < guard (the
//   preconditioner of Eq. sparsePreconditioner before its eps drop, the
//   diagonal formed once per determinant),
//   d_j = V z_j (with Z: z_j = y_j - ph_j yp_j, the change of the Ritz vector
//   since the previous iteration),
// x_j and t_j written; the workgroup's sums of |r_j|^2 and |t_j|^2 and its
// maximum of |d_j|^2 (0 without Z) go to partial[wg][12 (j / 4) + 4 q + j % 4]
// for q = 0, 1, 2 (wg over blockIdx.x).  Y, Z: m x k row-major.
constexpr int RZ_CB = 4;
constexpr int RZ_NS = 3 * RZ_CB;
template <bool CPLX>
__global__ __launch_bounds__(256) void k_ritz(DevSpace S, const double* __restrict__ hd,
                                              const double* __restrict__ JK, double e_core,
                                              const typename VT<CPLX>::T* __restrict__ V,
                                              const typename VT<CPLX>::T* __restrict__ W, int64_t ld, int m,
                                              const typename VT<CPLX>::T* __restrict__ Y,
                                              const typename VT<CPLX>::T* __restrict__ Z, int k,
                                              const double* __restrict__ theta, double guard,
                                              typename VT<CPLX>::T* __restrict__ X,
                                              typename VT<CPLX>::T* __restrict__ Tc, int64_t n,
                                              double* __restrict__ partial) {
    using Vt = VT<CPLX>;
    using T = typename Vt::T;
    const int j0 = blockIdx.y * RZ_CB;
    double acc[RZ_NS];
#pragma unroll
    for (int s = 0; s < RZ_NS; ++s) acc[s] = 0.0;
    double th[RZ_CB];
#pragma unroll
    for (int jj = 0; jj < RZ_CB; ++jj) th[jj] = (j0 + jj < k) ? theta[j0 + jj] : 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const double h = diag_elem(S, hd, JK, e_core, e);
        T xs[RZ_CB], rs[RZ_CB], ds[RZ_CB];
#pragma unroll
        for (int jj = 0; jj < RZ_CB; ++jj) xs[jj] = rs[jj] = ds[jj] = Vt::zero();
#pragma unroll 4
        for (int i = 0; i < m; ++i) {
            const T a = V[(int64_t)i * ld + e];
            const T b = W[(int64_t)i * ld + e];
#pragma unroll
            for (int jj = 0; jj < RZ_CB; ++jj)
                if (j0 + jj < k) {
                    const T y = Y[i * k + j0 + jj];
                    xs[jj] = Vt::mad(a, y, xs[jj]);
                    rs[jj] = Vt::mad(b, y, rs[jj]);
                    if (Z) ds[jj] = Vt::mad(a, Z[i * k + j0 + jj], ds[jj]);
                }
        }
#pragma unroll
        for (int jj = 0; jj < RZ_CB; ++jj) {
            const int j = j0 + jj;
            if (j >= k) break;
            X[(int64_t)j * ld + e] = xs[jj];
            const T r = Vt::sub(rs[jj], Vt::scale(xs[jj], th[jj]));
            const double den = th[jj] - h;
            const T t = (fabs(den) >= guard) ? Vt::scale(r, 1.0 / den) : Vt::zero();
            Tc[(int64_t)j * ld + e] = t;
            acc[jj] += Vt::abs2(r);
            acc[RZ_CB + jj] += Vt::abs2(t);
            acc[2 * RZ_CB + jj] = fmax(acc[2 * RZ_CB + jj], Vt::abs2(ds[jj]));
        }
    }
    constexpr uint64_t kMax = ((uint64_t)((1 << RZ_CB) - 1)) << (2 * RZ_CB);
    wg_partials<RZ_NS, kMax>(acc, partial + ((int64_t)blockIdx.x * gridDim.y + blockIdx.y) * RZ_NS);
}

// One pass over nx <= 4 vectors X_t (t < nx) with the Gram matrix of the
// results: the workgroup's sums of conj(X_s) X_t go to partial[wg][2 (4 t + s)
// + c] (c = 0 real, 1 imaginary part; a 4 x 4 block whatever nx):
//   mode 0: X_t = sum_i A_i Y[i nx + t]        (Y: m x nx row-major)
//   mode 3: X_t <- X_t - sum_i A_i Y[t m + i]  (Y as the dot products lie)
// A and X are distinct vectors; every sum runs over i in ascending order.
constexpr int CG_NX = 4;
constexpr int CG_NS = 2 * CG_NX * CG_NX;
template <bool CPLX>
__global__ __launch_bounds__(256) void k_comb_gram(const typename VT<CPLX>::T* __restrict__ A, int64_t ld, int m,
                                                   const typename VT<CPLX>::T* __restrict__ Y,
                                                   typename VT<CPLX>::T* __restrict__ X, int nx, int64_t n, int mode,
                                                   double* __restrict__ partial) {
    using Vt = VT<CPLX>;
    using T = typename Vt::T;
    T g[CG_NX][CG_NX];
#pragma unroll
    for (int t = 0; t < CG_NX; ++t)
#pragma unroll
        for (int s = 0; s < CG_NX; ++s) g[t][s] = Vt::zero();
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        T xs[CG_NX];
#pragma unroll
        for (int t = 0; t < CG_NX; ++t) xs[t] = Vt::zero();
#pragma unroll 4
        for (int i = 0; i < m; ++i) {
            const T a = A[(int64_t)i * ld + e];
#pragma unroll
            for (int t = 0; t < CG_NX; ++t)
                if (t < nx) xs[t] = Vt::mad(a, (mode == 3) ? Y[t * m + i] : Y[i * nx + t], xs[t]);
        }
#pragma unroll
        for (int t = 0; t < CG_NX; ++t) {
            if (t >= nx) break;
            T* dst = X + (int64_t)t * ld + e;
            if (mode == 3) xs[t] = Vt::sub(*dst, xs[t]);
            *dst = xs[t];
        }
#pragma unroll
        for (int t = 0; t < CG_NX; ++t)
#pragma unroll
            for (int s = 0; s < CG_NX; ++s)
                if (t < nx && s < nx) g[t][s] = Vt::cmad(xs[s], xs[t], g[t][s]);
    }
    double v[CG_NS];
#pragma unroll
    for (int t = 0; t < CG_NX; ++t)
#pragma unroll
        for (int s = 0; s < CG_NX; ++s) {
            const double* q = reinterpret_cast<const double*>(&g[t][s]);
            v[2 * (t * CG_NX + s)] = q[0];
            v[2 * (t * CG_NX + s) + 1] = CPLX ? q[1] : 0.0;
        }
    wg_partials<CG_NS, 0>(v, partial + (int64_t)blockIdx.x * CG_NS);
}

// X_j <- sum_i X_i Y[i kk + j] for j < kk <= KR, i < m, in place: every
// element's m inputs are read before any of its outputs is written
template <bool CPLX, int KR>
__global__ __launch_bounds__(256) void k_combine_inplace(typename VT<CPLX>::T* X, int64_t ld, int m,
                                                         const typename VT<CPLX>::T* __restrict__ Y, int kk,
                                                         int64_t n) {
    using Vt = VT<CPLX>;
    using T = typename Vt::T;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        T acc[KR];
#pragma unroll
        for (int j = 0; j < KR; ++j) acc[j] = Vt::zero();
        for (int i = 0; i < m; ++i) {
            const T a = X[(int64_t)i * ld + e];
#pragma unroll
            for (int j = 0; j < KR; ++j)
                if (j < kk) acc[j] = Vt::mad(a, Y[i * kk + j], acc[j]);
        }
#pragma unroll
        for (int j = 0; j < KR; ++j)
            if (j < kk) X[(int64_t)j * ld + e] = acc[j];
    }
}

// ---------------------------------------------------------------------------
// Host-side check of the move machinery used by the kernels: for every
// checked determinant and every move slot, the target address must lie in the
// space, hold the determinant E_xy D, and carry the sign of the global rule
// (-1)^(#occupied below y in D) * (-1)^(#occupied below x in D - y).
// ---------------------------------------------------------------------------
int64_t check_moves_host(const DevSpace& S, int64_t max_dets_per_cat, int64_t* n_checked,
                         bool (*to_bits)(const void*, int64_t, uint64_t*), const void* user) {
    int64_t bad = 0, checked = 0;
    const int K = S.sp.K;
    for (int w = 0; w < S.sp.nwork; ++w) {
        const Cat& C = S.cats[S.work_cat[w]];
        int64_t step = C.size <= max_dets_per_cat ? 1 : C.size / max_dets_per_cat;
        for (int64_t j = 0; j < C.size; j += step) {
            Det d;
            decode(S, C, j, d);
            uint64_t Jb = 0;
            for (int k = 0; k < K; ++k) Jb |= (uint64_t)d.s[k] << S.sp.sub_off[k];
            for (int slot = 0; slot < C.deg; ++slot) {
                int cls, xs, ys, lx, ly, sg;
                slot_move(S, C, d, slot, cls, xs, ys, lx, ly);
                int64_t t = apply_move(S, C, cls, xs, ys, lx, ly, d, sg);
                ++checked;
                int x = S.sp.sub_off[xs] + lx, y = S.sp.sub_off[ys] + ly;
                uint64_t want = (Jb & ~(1ULL << y)) | (1ULL << x);
                int par = __builtin_popcountll(Jb & ((1ULL << y) - 1ULL)) +
                          __builtin_popcountll((Jb & ~(1ULL << y)) & ((1ULL << x) - 1ULL));
                int want_sign = (par & 1) ? -1 : 1;
                uint64_t got = 0;
                if (t < 0 || t >= S.sp.ndets || !to_bits(user, t, &got) || got != want || sg != want_sign) ++bad;
            }
        }
    }
    if (n_checked) *n_checked = checked;
    return bad;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline int grid_for(int64_t n, int block, int cap = 65536) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_sigma1e(const DevSpace& S, bool cplx, const void* hp, const void* c, void* sigma, int n_vec,
                          hipStream_t st) {
    int g = grid_for(S.sp.ndets, 256);
    if (cplx)
        hipLaunchKernelGGL(k_sigma1e<true>, dim3(g), dim3(256), 0, st, S, (const cd*)hp, (const cd*)c, (cd*)sigma,
                           n_vec);
    else
        hipLaunchKernelGGL(k_sigma1e<false>, dim3(g), dim3(256), 0, st, S, (const double*)hp, (const double*)c,
                           (double*)sigma, n_vec);
    return hipGetLastError();
}

hipError_t launch_diag(const DevSpace& S, const double* hd, const double* JK, double e_core, double* out,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_diag, dim3(grid_for(S.sp.ndets, 256)), dim3(256), 0, st, S, hd, JK, e_core, out);
    return hipGetLastError();
}

hipError_t launch_precond(const DevSpace& S, bool cplx, const double* hd, const double* JK, double e_core,
                          const void* r, void* t, int64_t ld, int n, const int* root, const double* theta,
                          double guard, hipStream_t st) {
    if (n < 1) return hipSuccess;
    if (n > PRE_MAX) return hipErrorInvalidValue;
    PrecondRoots P{};
    P.n = n;
    for (int q = 0; q < n; ++q) {
        P.root[q] = root[q];
        P.theta[q] = theta[q];
    }
    int g = grid_for(S.sp.ndets, 256);
    if (cplx)
        hipLaunchKernelGGL(k_precond<true>, dim3(g), dim3(256), 0, st, S, hd, JK, e_core, (const cd*)r, (cd*)t,
                           ld, P, guard);
    else
        hipLaunchKernelGGL(k_precond<false>, dim3(g), dim3(256), 0, st, S, hd, JK, e_core, (const double*)r,
                           (double*)t, ld, P, guard);
    return hipGetLastError();
}

int topk_blocks(const DevSpace& S) { return grid_for(S.sp.ndets, 256, 1024); }

hipError_t launch_diag_topk(const DevSpace& S, const double* hd, const double* JK, double e_core, int k,
                            double* vals, int64_t* idx, hipStream_t st) {
    hipLaunchKernelGGL(k_diag_topk, dim3(topk_blocks(S)), dim3(256), 0, st, S, hd, JK, e_core, k, vals, idx);
    return hipGetLastError();
}

int dots_blocks(int64_t n) { return grid_for(n, 256, 256); }

hipError_t launch_dots(bool cplx, const void* Vb, int64_t ld, int m, const void* W, int nw, int64_t n,
                       void* partial, void* out, hipStream_t st) {
    if (m <= 0 || nw <= 0) return hipSuccess;
    const int nb = dots_blocks(n);
    const dim3 grid((m + DOTV - 1) / DOTV, nb, (nw + DOTW - 1) / DOTW);
    if (cplx)
        hipLaunchKernelGGL(k_dots<true>, grid, dim3(256), 0, st, (const cd*)Vb, ld, m, (const cd*)W, nw, n,
                           (cd*)partial);
    else
        hipLaunchKernelGGL(k_dots<false>, grid, dim3(256), 0, st, (const double*)Vb, ld, m, (const double*)W, nw, n,
                           (double*)partial);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nout = m * nw * (cplx ? 2 : 1);
    return launch_fold((const double*)partial, nb, nout, nout, nout, nout, (double*)out, st);
}

static int ritz_wgs(int64_t n) { return grid_for(n, 256, 1024); }
int ritz_blocks(int64_t n, int k) { return ritz_wgs(n) * ((k + RZ_CB - 1) / RZ_CB); }

hipError_t launch_ritz(const DevSpace& S, bool cplx, const double* hd, const double* JK, double e_core,
                       const void* V, const void* W, int64_t ld, int m, const void* Y, const void* Z, int k,
                       const double* theta, double guard, void* X, void* T, int64_t n, double* partial, double* out,
                       hipStream_t st) {
    if (k < 1 || k > PRE_MAX || m < 1) return hipErrorInvalidValue;
    const int gy = (k + RZ_CB - 1) / RZ_CB;
    const dim3 grid(ritz_wgs(n), gy);
    if (cplx)
        hipLaunchKernelGGL(k_ritz<true>, grid, dim3(256), 0, st, S, hd, JK, e_core, (const cd*)V, (const cd*)W, ld,
                           m, (const cd*)Y, (const cd*)Z, k, theta, guard, (cd*)X, (cd*)T, n, partial);
    else
        hipLaunchKernelGGL(k_ritz<false>, grid, dim3(256), 0, st, S, hd, JK, e_core, (const double*)V,
                           (const double*)W, ld, m, (const double*)Y, (const double*)Z, k, theta, guard, (double*)X,
                           (double*)T, n, partial);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_fold(partial, grid.x, gy * RZ_NS, gy * RZ_NS, RZ_NS, 2 * RZ_CB, out, st);
}

int comb_gram_blocks(int64_t n) { return grid_for(n, 256, 1024); }

hipError_t launch_comb_gram(bool cplx, const void* A, int64_t ld, int m, const void* Y, void* X, int nx, int64_t n,
                            int mode, double* partial, double* gout, hipStream_t st) {
    if (nx < 1 || nx > CG_NX || m < 1 || (mode != 0 && mode != 3)) return hipErrorInvalidValue;
    const int g = comb_gram_blocks(n);
    if (cplx)
        hipLaunchKernelGGL(k_comb_gram<true>, dim3(g), dim3(256), 0, st, (const cd*)A, ld, m, (const cd*)Y, (cd*)X,
                           nx, n, mode, partial);
    else
        hipLaunchKernelGGL(k_comb_gram<false>, dim3(g), dim3(256), 0, st, (const double*)A, ld, m,
                           (const double*)Y, (double*)X, nx, n, mode, partial);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_fold(partial, g, CG_NS, CG_NS, CG_NS, CG_NS, gout, st);
}

template <bool CPLX>
static hipError_t launch_inplace_t(void* X, int64_t ld, int m, const void* Y, int kk, int64_t n, hipStream_t st) {
    using T = typename VT<CPLX>::T;
    const int g = grid_for(n, 256, 8192);
    if (kk <= 4)
        hipLaunchKernelGGL((k_combine_inplace<CPLX, 4>), dim3(g), dim3(256), 0, st, (T*)X, ld, m, (const T*)Y, kk, n);
    else if (kk <= 8)
        hipLaunchKernelGGL((k_combine_inplace<CPLX, 8>), dim3(g), dim3(256), 0, st, (T*)X, ld, m, (const T*)Y, kk, n);
    else if (kk <= 16)
        hipLaunchKernelGGL((k_combine_inplace<CPLX, 16>), dim3(g), dim3(256), 0, st, (T*)X, ld, m, (const T*)Y, kk,
                           n);
    else
        hipLaunchKernelGGL((k_combine_inplace<CPLX, 32>), dim3(g), dim3(256), 0, st, (T*)X, ld, m, (const T*)Y, kk,
                           n);
    return hipGetLastError();
}

hipError_t launch_combine_inplace(bool cplx, void* X, int64_t ld, int m, const void* Y, int kk, int64_t n,
                                  hipStream_t st) {
    if (kk < 1 || kk > 32 || kk > m) return hipErrorInvalidValue;
    return cplx ? launch_inplace_t<true>(X, ld, m, Y, kk, n, st) : launch_inplace_t<false>(X, ld, m, Y, kk, n, st);
}

hipError_t launch_combine(bool cplx, const void* A, const void* B, int64_t ld, int m, const void* Y, int k,
                          const double* theta, void* X, void* R, int64_t n, int mode, hipStream_t st) {
    int g = grid_for(n, 256, 8192);
    if (cplx)
        hipLaunchKernelGGL(k_combine<true>, dim3(g), dim3(256), 0, st, (const cd*)A, (const cd*)B, ld, m,
                           (const cd*)Y, k, theta, (cd*)X, (cd*)R, n, mode);
    else
        hipLaunchKernelGGL(k_combine<false>, dim3(g), dim3(256), 0, st, (const double*)A, (const double*)B, ld, m,
                           (const double*)Y, k, theta, (double*)X, (double*)R, n, mode);
    return hipGetLastError();
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_axpy_core(typename VT<CPLX>::T* __restrict__ y,
                                                  const typename VT<CPLX>::T* __restrict__ x, double a, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = VT<CPLX>::add(y[e], VT<CPLX>::scale(x[e], a));
}

hipError_t launch_axpy_core(bool cplx, void* sigma, const void* c, double e_core, int64_t n, hipStream_t st) {
    const int g = grid_for(n, 256, 8192);
    if (cplx)
        hipLaunchKernelGGL(k_axpy_core<true>, dim3(g), dim3(256), 0, st, (cd*)sigma, (const cd*)c, e_core, n);
    else
        hipLaunchKernelGGL(k_axpy_core<false>, dim3(g), dim3(256), 0, st, (double*)sigma, (const double*)c, e_core,
                           n);
    return hipGetLastError();
}

hipError_t launch_eps_drop(bool cplx, void* t, int64_t ld, int64_t nd, int n, const int* slot, const double* nrm2,
                           int stride, double eps, hipStream_t st) {
    if (n < 1) return hipSuccess;
    if (n > PRE_MAX) return hipErrorInvalidValue;
    DropRoots D{};
    D.n = n;
    for (int q = 0; q < n; ++q) D.slot[q] = slot[q];
    const int g = grid_for(nd, 256);
    if (cplx)
        hipLaunchKernelGGL(k_eps_drop<true>, dim3(g), dim3(256), 0, st, (cd*)t, ld, nd, D, nrm2, stride, eps);
    else
        hipLaunchKernelGGL(k_eps_drop<false>, dim3(g), dim3(256), 0, st, (double*)t, ld, nd, D, nrm2, stride, eps);
    return hipGetLastError();
}

hipError_t launch_scale(bool cplx, void* x, double s, int64_t n, hipStream_t st) {
    int g = grid_for(n, 256, 8192);
    if (cplx)
        hipLaunchKernelGGL(k_scale<true>, dim3(g), dim3(256), 0, st, (cd*)x, s, n);
    else
        hipLaunchKernelGGL(k_scale<false>, dim3(g), dim3(256), 0, st, (double*)x, s, n);
    return hipGetLastError();
}

hipError_t launch_unit(bool cplx, void* x, int64_t n, int64_t at, hipStream_t st) {
    int g = grid_for(n, 256, 8192);
    if (cplx)
        hipLaunchKernelGGL(k_unit<true>, dim3(g), dim3(256), 0, st, (cd*)x, n, at);
    else
        hipLaunchKernelGGL(k_unit<false>, dim3(g), dim3(256), 0, st, (double*)x, n, at);
    return hipGetLastError();
}

}  // namespace stp
