// Two-electron sigma (Eq. sigmaL2e), tiled form for gfx950.
//
// For an intermediate determinant J with moves m = (x created, y annihilated)
// into the space, the update is e = G_J d,
//   d[m]      = sign(m) C[target(m)]                       (<J|E_rs|K> C_K, (r,s) = (y,x))
//   G_J[m',m] = (x' y' | y x)                              (g_pqrs, (p,q) = (x',y'))
//   sigma[target(m')] += 1/2 sign(m') e[m'].
// A workgroup owns a block of determinants of one intermediate category and
// one group of annihilated orbitals y' (the rows of G_J).  Workgroups are
// dispatched round-robin over the 8 XCDs, and the row group is blockIdx mod
// the number of groups, so each XCD only ever reads the slice of the
// integrals gT[(y x)][(y' x')] whose y' lies in its group: that slice stays
// resident in the XCD's L2.  Both Davidson vectors of a launch share every
// integral load.
//
// Phase 1 enumerates the moves of every determinant of the block (pair index,
// sign, target) and gathers d for all vectors into LDS; it also builds, in
// slot order, the list of rows whose y' is in the group (a block-wide scan),
// so consecutive threads take consecutive x' of one y' and their integral
// loads coalesce.  Phase 2 gives each thread one row: a dot product over all
// moves of its determinant, then one atomic update of sigma per vector.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"
#include "stp_device.hpp"

namespace stp {

constexpr int S2_THREADS = 256;

template <bool CPLX, int NV>
__global__ __launch_bounds__(S2_THREADS) void k_sigma2e_tiled(DevSpace S, Sigma2eSched P,
                                                             const typename VT<CPLX>::T* __restrict__ gT,
                                                             const typename VT<CPLX>::T* __restrict__ c,
                                                             typename VT<CPLX>::T* __restrict__ sigma, int n_vec) {
    using V = VT<CPLX>;
    using T = typename V::T;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const int grp = blockIdx.x % P.ngroups;
    const int jb = blockIdx.x / P.ngroups;
    const Sigma2eBlock blk = P.blocks[jb];
    const Cat& C = S.cats[blk.cat];
    const int deg = C.deg;
    const int nj = blk.count;
    const int tot = nj * deg;
    const int M = S.sp.M;
    const int64_t MM = (int64_t)M * M;
    const int64_t nd = S.sp.ndets;

    // LDS layout
    T* dsh = reinterpret_cast<T*>(smem);                                   // [tot][NV]
    int64_t* tgt = reinterpret_cast<int64_t*>(dsh + (size_t)P.max_tot * NV);  // [tot]
    int32_t* pr = reinterpret_cast<int32_t*>(tgt + P.max_tot);             // [tot] pair<<1 | neg
    int32_t* rows = pr + P.max_tot;                                        // [tot] (jj << 16) | slot
    int32_t* coff = rows + P.max_tot;                                      // [tot] pair * M^2
    Det* dets = reinterpret_cast<Det*>(coff + P.max_tot);                  // [nj]
    __shared__ int scan[S2_THREADS];
    __shared__ uint8_t ygrp[MMAX];

    if (tid < M) ygrp[tid] = (uint8_t)P.ygroup[tid];
    for (int jj = tid; jj < nj; jj += S2_THREADS) decode(S, C, blk.j0 + jj, dets[jj]);
    __syncthreads();

    // Phase 1: moves and gathers; each thread a contiguous chunk of (jj, slot)
    const int chunk = (tot + S2_THREADS - 1) / S2_THREADS;
    const int i0 = tid * chunk;
    const int i1 = min(tot, i0 + chunk);
    int cnt = 0;
    for (int i = i0; i < i1; ++i) {
        const int jj = i / deg;
        const int slot = i - jj * deg;
        const Det& d = dets[jj];
        int cls, xs, ys, lx, ly, sg;
        slot_move(S, C, d, slot, cls, xs, ys, lx, ly);
        const int64_t t = apply_move(S, C, cls, xs, ys, lx, ly, d, sg);
        const int x = S.sp.sub_off[xs] + lx, y = S.sp.sub_off[ys] + ly;
        tgt[i] = t;
        pr[i] = ((y * M + x) << 1) | (sg < 0 ? 1 : 0);
        coff[i] = (y * M + x) * (int32_t)MM;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T val = (v < n_vec) ? c[(int64_t)v * nd + t] : V::zero();
            dsh[(size_t)i * NV + v] = (sg < 0) ? V::scale(val, -1.0) : val;
        }
        cnt += (ygrp[y] == grp) ? 1 : 0;
    }
    // block-wide exclusive scan of the row counts
    scan[tid] = cnt;
    __syncthreads();
    for (int off = 1; off < S2_THREADS; off <<= 1) {
        int add = (tid >= off) ? scan[tid - off] : 0;
        __syncthreads();
        scan[tid] += add;
        __syncthreads();
    }
    const int nrows = scan[S2_THREADS - 1];
    int w = scan[tid] - cnt;
    for (int i = i0; i < i1; ++i) {
        const int y = (pr[i] >> 1) / M;
        if (ygrp[y] == grp) {
            const int jj = i / deg;
            rows[w++] = (jj << 16) | (i - jj * deg);
        }
    }
    __syncthreads();

    // Phase 2: one row per thread.  Offsets are 32-bit element offsets into gT
    // (M <= 64 keeps them below 2^31 bytes), so each load is a base register
    // plus one 32-bit add; the column offsets of four moves come in one LDS read.
    for (int r = tid; r < nrows; r += S2_THREADS) {
        const int jj = rows[r] >> 16;
        const int slot = rows[r] & 0xffff;
        const int base = jj * deg;
        const int32_t prow = pr[base + slot] >> 1;
        T acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = V::zero();
        const int32_t* cj = coff + base;
        const T* dj = dsh + (size_t)base * NV;
        int col = 0;
        for (; col + 4 <= deg; col += 4) {
            const int32_t o0 = cj[col] + prow, o1 = cj[col + 1] + prow;
            const int32_t o2 = cj[col + 2] + prow, o3 = cj[col + 3] + prow;
            const T g0 = gT[o0], g1 = gT[o1], g2 = gT[o2], g3 = gT[o3];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                acc[v] = V::mad(g0, dj[(col + 0) * NV + v], acc[v]);
                acc[v] = V::mad(g1, dj[(col + 1) * NV + v], acc[v]);
                acc[v] = V::mad(g2, dj[(col + 2) * NV + v], acc[v]);
                acc[v] = V::mad(g3, dj[(col + 3) * NV + v], acc[v]);
            }
        }
        for (; col < deg; ++col) {
            const T g0 = gT[cj[col] + prow];
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] = V::mad(g0, dj[col * NV + v], acc[v]);
        }
        const double s = (pr[base + slot] & 1) ? -0.5 : 0.5;
        const int64_t t = tgt[base + slot];
#pragma unroll
        for (int v = 0; v < NV; ++v)
            if (v < n_vec) V::atomic_add(&sigma[(int64_t)v * nd + t], V::scale(acc[v], s));
    }
}

size_t sigma2e_tiled_lds(const Sigma2eSched& P, int nv, bool cplx) {
    size_t sb = cplx ? 16 : 8;
    return (size_t)P.max_tot * (nv * sb + 8 + 4 + 4 + 4) + (size_t)P.max_nj * sizeof(Det);
}

hipError_t launch_sigma2e_tiled(const DevSpace& S, const Sigma2eSched& P, bool cplx, const void* gT, const void* c,
                                void* sigma, int n_vec, hipStream_t st) {
    const int nd_blocks = P.nblocks * P.ngroups;
    for (int v0 = 0; v0 < n_vec; v0 += 2) {
        const int nv = (n_vec - v0 >= 2) ? 2 : 1;
        const size_t lds = sigma2e_tiled_lds(P, nv, cplx);
        const int64_t off = (int64_t)v0 * S.sp.ndets;
        if (cplx) {
            const cd* cc = (const cd*)c + off;
            cd* ss = (cd*)sigma + off;
            if (nv == 2)
                hipLaunchKernelGGL((k_sigma2e_tiled<true, 2>), dim3(nd_blocks), dim3(S2_THREADS), lds, st, S, P,
                                   (const cd*)gT, cc, ss, 2);
            else
                hipLaunchKernelGGL((k_sigma2e_tiled<true, 1>), dim3(nd_blocks), dim3(S2_THREADS), lds, st, S, P,
                                   (const cd*)gT, cc, ss, 1);
        } else {
            const double* cc = (const double*)c + off;
            double* ss = (double*)sigma + off;
            if (nv == 2)
                hipLaunchKernelGGL((k_sigma2e_tiled<false, 2>), dim3(nd_blocks), dim3(S2_THREADS), lds, st, S, P,
                                   (const double*)gT, cc, ss, 2);
            else
                hipLaunchKernelGGL((k_sigma2e_tiled<false, 1>), dim3(nd_blocks), dim3(S2_THREADS), lds, st, S, P,
                                   (const double*)gT, cc, ss, 1);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace stp
