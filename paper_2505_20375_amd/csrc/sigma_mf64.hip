// FP64 matrix-core form of the pair-resolved sigma build.
//
// Per pair intermediate K' (one wavefront, as in k_sigma_pair) the product
// e = A_K' d is computed as a real product with four right-hand columns,
//   B = [Re d_0, Re d_1, Im d_0, Im d_1]    (two vectors; one vector: [Re d, Im d, 0, 0]),
//   C1 = Re(A_K') B,  C2 = Im(A_K') B,
//   Re e_v = C1[., v] - C2[., 2 + v],   Im e_v = C1[., 2 + v] + C2[., v],
// on v_mfma_f64_4x4x4f64 (4 blocks of 4 x 4 x 4; the four blocks take 16
// consecutive rows of A_K' and share one B).  Lane layouts (checked on the
// device with an in-bounds probe): A lane 16k + 4 blk + r holds row
// 4 blk + r, step k; B lane 16k + 4 blk + c holds B[k][c]; output lane
// 16 r + 4 blk + c holds row 4 blk + r, column c.  With 16 consecutive slots
// per instruction and a step of 4 columns, one load instruction reads four
// runs of 16 adjacent table entries, instead of 64 scattered lines.  Every
// table entry of A_K' is read once per K' (both triangles); the Hermitian
// pairing of the vector-ALU kernel is not used.
//
// Slice per wavefront: header, targets, row words (pair << 1 | sign), and B
// as [slot][4] doubles; rows and steps padded to 32 slots (padding slots have
// d = 0, pair 0 and are not scattered); the table entries of the next 10
// steps (5 groups of 2) are in flight while a step's products run, which at
// 3 wavefronts per SIMD keeps about 30 loads in flight per SIMD.  Phase 3 writes each complex entry as two FP64 halves from the
// two lanes that hold them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"
#include "pair_arith.hpp"
#include "stp_device.hpp"

namespace stp {

struct Mf64Layout {
    size_t tgt_off, rinf_off, b_off, hdr_off, bytes;
    __host__ __device__ explicit Mf64Layout(int deg_cap) {
        const size_t cap = (size_t)((deg_cap + 31) & ~31);
        tgt_off = 0;
        rinf_off = tgt_off + cap * 8;
        b_off = (rinf_off + cap * 4 + 15) & ~(size_t)15;
        hdr_off = b_off + cap * 32;
        bytes = hdr_off + sizeof(PairHdr);
    }
};

size_t pair_mf64_slice_bytes(int deg_max) { return Mf64Layout(deg_max).bytes; }

template <bool CPLX, int NV, bool STORE>
__device__ __forceinline__ void mf64_det(const DevSpace& S, const typename VT<CPLX>::T* __restrict__ A,
                                         const typename VT<CPLX>::T* __restrict__ c,
                                         typename VT<CPLX>::T* __restrict__ sigma,
                                         typename VT<CPLX>::T* __restrict__ E, int nq, int n_vec, int deg_cap,
                                         unsigned char* base, int lane, int64_t J) {
    using V64 = VT<CPLX>;
    using TE = typename V64::T;
    const Mf64Layout L(deg_cap);
    int64_t* tgt = reinterpret_cast<int64_t*>(base + L.tgt_off);
    int32_t* rinf = reinterpret_cast<int32_t*>(base + L.rinf_off);
    double* bsh = reinterpret_cast<double*>(base + L.b_off);   // [slot][4]
    PairHdr* hd = reinterpret_cast<PairHdr*>(base + L.hdr_off);
    const int64_t nd = S.sp.ndets;
    const int w = find_segment(S.pwork_begin, S.sp.npcat, J);
    const PairCat& P = S.pcats[w];
    const int64_t jloc = J - S.pwork_begin[w];
    const int deg = P.deg;
    const int cap = (deg + 31) & ~31;

    // ---- phase 1: header, then per slot the target, row word and B row
    if (lane < S.sp.K) pair_hdr_sub(S, P, jloc, lane, hd);
    wave_lds_sync();
    if (lane < S.sp.M) pair_hdr_orb(S, P, lane, hd);
    if (lane < P.ncls) pair_hdr_cls(S, P, lane, hd);
    if (lane == 63) pair_hdr_bits(S, hd);
    wave_lds_sync();
    bool nz = false;
    for (int slot = lane; slot < cap; slot += 64) {
        double b4[4] = {0.0, 0.0, 0.0, 0.0};
        if (slot >= deg) {
            rinf[slot] = 0;
        } else {
            int64_t addr;
            int pi, q;
            const bool neg = pair_slot(S, P, hd, slot, addr, pi, q);
            tgt[slot] = STORE ? addr * nq + q : addr;
            rinf[slot] = (pi << 1) | (neg ? 1 : 0);
            const double sg = neg ? -1.0 : 1.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                if (v >= n_vec) break;
                const TE x = c[(int64_t)v * nd + addr];
                nz = nz || V64::abs2(x) != 0.0;
                if constexpr (CPLX) {
                    // two vectors: [Re0, Re1, Im0, Im1]; one vector: [Re, Im, 0, 0]
                    b4[NV == 2 ? v : 0] = sg * x.x;
                    b4[NV == 2 ? 2 + v : 1] = sg * x.y;
                } else {
                    b4[v] = sg * x;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) bsh[slot * 4 + j] = b4[j];
    }
    wave_lds_sync();
    const bool live = __ballot(nz) != 0;

    // ---- phases 2 and 3: 16-row tiles of A_K' on the matrix cores
    const int NP = S.sp.npairs;
    const int kq = lane >> 4;    // A and B lanes: step within the 4-column group
    const int col = lane & 3;    // B and output lanes: column
    // output lane: row 4 blk + r with blk = (lane >> 2) & 3, r = lane >> 4
    const int orow = (((lane >> 2) & 3) << 2) + (lane >> 4);
    const int nks = cap >> 2;
    for (int rt = 0; live && rt < cap; rt += 16) {   // (cap is a multiple of 32: nks of 8)
        const int prow = rinf[rt + (lane & 15)] >> 1;   // this A lane's row pair
        const TE* arow = A + prow;
        double c1a = 0.0, c2a = 0.0, c1b = 0.0, c2b = 0.0;   // two chains per product
        constexpr int G = 2;   // steps per group
        constexpr int RG = 6;   // groups in flight
        const int ngrp = nks / G;
        TE ab[RG][G];
        double bb[RG][G];
        auto ldgrp = [&](int g, TE (&a)[G], double (&b)[G]) {
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const int ks4 = ((g * G + j) << 2) + kq;
                a[j] = arow[(int64_t)(rinf[ks4] >> 1) * NP];
                b[j] = bsh[ks4 * 4 + col];
            }
        };
        auto mfgrp = [&](const TE (&a)[G], const double (&b)[G]) {
#pragma unroll
            for (int j = 0; j < G; j += 2) {
                if constexpr (CPLX) {
                    c1a = __builtin_amdgcn_mfma_f64_4x4x4f64(a[j].x, b[j], c1a, 0, 0, 0);
                    c2a = __builtin_amdgcn_mfma_f64_4x4x4f64(a[j].y, b[j], c2a, 0, 0, 0);
                    c1b = __builtin_amdgcn_mfma_f64_4x4x4f64(a[j + 1].x, b[j + 1], c1b, 0, 0, 0);
                    c2b = __builtin_amdgcn_mfma_f64_4x4x4f64(a[j + 1].y, b[j + 1], c2b, 0, 0, 0);
                } else {
                    c1a = __builtin_amdgcn_mfma_f64_4x4x4f64(a[j], b[j], c1a, 0, 0, 0);
                    c1b = __builtin_amdgcn_mfma_f64_4x4x4f64(a[j + 1], b[j + 1], c1b, 0, 0, 0);
                }
            }
        };
#pragma unroll
        for (int u = 0; u < RG - 1; ++u)
            if (u < ngrp) ldgrp(u, ab[u], bb[u]);
        for (int g = 0; g < ngrp; g += RG) {
#pragma unroll
            for (int u = 0; u < RG; ++u) {
                if (g + u >= ngrp) break;
                if (g + u + RG - 1 < ngrp) ldgrp(g + u + RG - 1, ab[(u + RG - 1) % RG], bb[(u + RG - 1) % RG]);
                mfgrp(ab[u], bb[u]);
            }
        }
        const double c1 = c1a + c1b;
        // this lane's result: component comp of vector v of row orow
        double val;
        int v, comp;
        bool use;
        if constexpr (CPLX) {
            const double c2 = c2a + c2b;
            if (NV == 2) {
                const double p = __shfl_xor(c2, 2, 64);   // column c ^ 2 of Im(A) B
                val = (col < 2) ? c1 - p : c1 + p;
                v = col & 1;
                comp = col >> 1;
                use = true;
            } else {
                const double p = __shfl_xor(c2, 1, 64);   // column c ^ 1
                val = (col == 0) ? c1 - p : c1 + p;
                v = 0;
                comp = col;
                use = col < 2;
            }
        } else {
            val = c1;
            v = col;
            comp = 0;
            use = col < NV;
        }
        const int slot = rt + orow;
        if (use && slot < deg && v < n_vec) {
            const int32_t ri = rinf[slot];
            const double x = (ri & 1) ? -val : val;
            const int64_t t = tgt[slot];
            if (STORE)
                reinterpret_cast<double*>(E + t * NV + v)[comp] = x;
            else
                unsafeAtomicAdd(reinterpret_cast<double*>(sigma + (int64_t)v * nd + t) + comp, x);
        }
    }
    if (STORE && !live) {
        // no product: zeros for this K''s entries of the contribution workspace
        for (int slot = lane; slot < deg; slot += 64)
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < n_vec) E[tgt[slot] * NV + v] = V64::zero();
    }
    wave_lds_sync();   // the next K' reuses this wavefront's slice
}

template <bool CPLX, int NV, bool STORE>
__global__ __launch_bounds__(256) void k_sigma_pair_mf64(DevSpace S, const typename VT<CPLX>::T* __restrict__ A,
                                                        const typename VT<CPLX>::T* __restrict__ c,
                                                        typename VT<CPLX>::T* __restrict__ sigma,
                                                        typename VT<CPLX>::T* __restrict__ E, int nq, int n_vec,
                                                        int deg_cap) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    unsigned char* base = smem + (size_t)wid * Mf64Layout(deg_cap).bytes;
    const int64_t total = S.sp.npwork_dets;
    const int64_t nw = (int64_t)gridDim.x * wpb;
    for (int64_t J = (int64_t)blockIdx.x * wpb + wid; J < total; J += nw)
        mf64_det<CPLX, NV, STORE>(S, A, c, sigma, E, nq, n_vec, deg_cap, base, lane, J);
}

bool pair_mf64_supported(int n_elec, int deg_max) {
    return n_elec >= 2 && deg_max > 0 && pair_mf64_slice_bytes(deg_max) <= 64 * 1024;
}

template <bool CPLX, int NV, bool STORE>
static hipError_t launch_mf64_nv(const DevSpace& S, int deg_max, const void* A, const void* c, void* sigma, void* E,
                                 int nq, int nv, hipStream_t st) {
    using T64 = typename VT<CPLX>::T;
    const size_t per_wave = pair_mf64_slice_bytes(deg_max);
    const int wpb = waves_per_group(per_wave);
    const size_t lds = per_wave * wpb;
    int64_t blocks = (S.sp.npwork_dets + wpb - 1) / wpb;
    blocks = std::max<int64_t>(1, std::min<int64_t>(blocks, 256 * 64));
    hipLaunchKernelGGL((k_sigma_pair_mf64<CPLX, NV, STORE>), dim3((unsigned)blocks), dim3(64 * wpb), lds, st, S,
                       (const T64*)A, (const T64*)c, (T64*)sigma, (T64*)E, nq, nv, deg_max);
    return hipGetLastError();
}

template <bool CPLX>
static hipError_t launch_mf64_all(const DevSpace& S, int deg_max, const void* A, const void* c, void* sigma, void* E,
                                  int n_vec, double e_core, const LaunchMarks* mk, hipStream_t st) {
    using T64 = typename VT<CPLX>::T;
    hipError_t e;
    const int nq = S.sp.N * (S.sp.N - 1) / 2;
    if (!E) {
        e = launch_fill_init(CPLX, sigma, c, e_core, S.sp.ndets * n_vec, st);
        if (e != hipSuccess) return e;
    }
    for (int v0 = 0; v0 < n_vec; v0 += 2) {
        const int nv = (n_vec - v0 >= 2) ? 2 : 1;
        const int64_t off = (int64_t)v0 * S.sp.ndets;
        const T64* cc = (const T64*)c + off;
        T64* ss = (T64*)sigma + off;
        if (mk) mk->fn(mk->user, 0, true);
        if (E)
            e = (nv == 2) ? launch_mf64_nv<CPLX, 2, true>(S, deg_max, A, cc, ss, E, nq, 2, st)
                          : launch_mf64_nv<CPLX, 1, true>(S, deg_max, A, cc, ss, E, nq, 1, st);
        else
            e = (nv == 2) ? launch_mf64_nv<CPLX, 2, false>(S, deg_max, A, cc, ss, nullptr, 0, 2, st)
                          : launch_mf64_nv<CPLX, 1, false>(S, deg_max, A, cc, ss, nullptr, 0, 1, st);
        if (mk) mk->fn(mk->user, 0, false);
        if (e != hipSuccess) return e;
        if (E) {
            if (mk) mk->fn(mk->user, 1, true);
            e = launch_pair_reduce(S, CPLX, nv, ss, cc, E, nv, e_core, st);
            if (mk) mk->fn(mk->user, 1, false);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_sigma_pair_mf64(const DevSpace& S, int deg_max, bool cplx, const void* A, const void* c,
                                  void* sigma, void* E, int n_vec, double e_core, const LaunchMarks* mk,
                                  hipStream_t st) {
    return cplx ? launch_mf64_all<true>(S, deg_max, A, c, sigma, E, n_vec, e_core, mk, st)
                : launch_mf64_all<false>(S, deg_max, A, c, sigma, E, n_vec, e_core, mk, st);
}

}  // namespace stp
