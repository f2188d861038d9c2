// BF16 matrix-core form of the pair-resolved sigma build (precision form).
//
// The pair form computes, for every (N-2)-electron intermediate K',
// e = A_K' d with d[Q] = sgn(a+_q a+_s |K'>) c[K' + {q, s}] and scatters
// e[P] to K' + {p, r}.  A_K' is the pair-pair table restricted to the pairs
// that lead from K' into the space.  Here a batch of K' is contracted at once
// as a dense product over all pairs,
//   E[P, col] = sum_Q A[P, Q] D[Q, col],   col = (K' of the batch, vector),
// with D[Q, col] = d[Q] of that K' where Q leads into the space and 0
// elsewhere, so that one pass of A serves 16 columns and the product runs on
// the matrix cores (v_mfma_f32_16x16x32_bf16: bfloat16 operands, FP32
// accumulation).  A complex product takes four real ones:
//   Re E = Ar Dr + (-Ai) Di,  Im E = Ar Di + Ai Dr.
// The padding (pairs a K' cannot create) adds multiply-adds with zeros only;
// the executed matrix-core flops are reported apart from the useful ones.
//
// Per workgroup and batch of BK = 16 / NV intermediates: phase 1 (one
// wavefront per K', as in the FP64 kernel) decodes K', computes each slot's
// target, sign and pair index, and writes d in bfloat16 into the column of
// D (LDS, [column][pair]) and the slot into a pair -> slot map; phase 2 (each
// wavefront a set of 16-row tiles of E) runs the MFMA chain over the pair
// index with A fragments read from the table (L2-resident) and D fragments
// from LDS; phase 3 scatters the E entries whose pair is a slot of their K'
// (store-and-reduce into the per-target contribution array, else device
// atomics), straight from the accumulators.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"
#include "pair_arith.hpp"
#include "stp_device.hpp"

namespace stp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MF_COLS = 16;   // product columns per batch (intermediates x vectors)
constexpr int MF_PAD = 8;     // bfloat16 padding of a D column (LDS bank spread)

int pair_mfma_npp(int npairs) { return (npairs + 31) & ~31; }

// bfloat16 bits of a finite float, rounded to nearest even.
__device__ __forceinline__ uint16_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// LDS layout of one workgroup: BK headers, per-K' targets and row words,
// the pair -> slot maps, and D (real, then imaginary part).
struct MfmaLayout {
    size_t hdr_off, tgt_off, rinf_off, map_off, dr_off, di_off, bytes;
    __host__ __device__ MfmaLayout(int bk, int deg_cap, int npp, bool cplx) {
        auto al = [](size_t x) { return (x + 15) & ~(size_t)15; };
        hdr_off = 0;
        tgt_off = al(hdr_off + (size_t)bk * sizeof(PairHdr));
        rinf_off = al(tgt_off + (size_t)bk * deg_cap * 8);
        map_off = al(rinf_off + (size_t)bk * deg_cap * 4);
        dr_off = al(map_off + (size_t)bk * npp * 2);
        const size_t dcol = (size_t)MF_COLS * (npp + MF_PAD) * 2;
        di_off = dr_off + dcol;
        bytes = di_off + (cplx ? dcol : 0);
    }
};

template <bool CPLX>
__device__ __forceinline__ double im_part(typename VT<CPLX>::T x) {
    if constexpr (CPLX) return x.y;
    else return 0.0;
}

template <bool CPLX>
__device__ __forceinline__ typename VT<CPLX>::T make_scalar(double re, double im) {
    if constexpr (CPLX) return cd{re, im};
    else return re;
}

template <bool CPLX, int NV, bool STORE>
__global__ __launch_bounds__(512) void k_sigma_pair_mfma(DevSpace S, const uint16_t* __restrict__ Ab, int npp,
                                                        const typename VT<CPLX>::T* __restrict__ c,
                                                        typename VT<CPLX>::T* __restrict__ sigma,
                                                        typename VT<CPLX>::T* __restrict__ E, int nq, int n_vec,
                                                        int deg_cap) {
    using V64 = VT<CPLX>;
    using TE = typename V64::T;
    constexpr int BK = MF_COLS / NV;
    extern __shared__ __align__(16) unsigned char smem[];
    const MfmaLayout L(BK, deg_cap, npp, CPLX);
    PairHdr* hdr = reinterpret_cast<PairHdr*>(smem + L.hdr_off);
    int64_t* tgt = reinterpret_cast<int64_t*>(smem + L.tgt_off);     // [BK][deg_cap]
    int32_t* rinf = reinterpret_cast<int32_t*>(smem + L.rinf_off);   // [BK][deg_cap] pair << 1 | negative
    int16_t* pmap = reinterpret_cast<int16_t*>(smem + L.map_off);    // [BK][npp] slot of a pair, or -1
    uint16_t* Dr = reinterpret_cast<uint16_t*>(smem + L.dr_off);     // [MF_COLS][npp + MF_PAD]
    uint16_t* Di = reinterpret_cast<uint16_t*>(smem + L.di_off);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nwv = blockDim.x >> 6;
    const int64_t total = S.sp.npwork_dets;
    const int64_t nd = S.sp.ndets;
    const int ldd = npp + MF_PAD;
    const size_t msz = (size_t)npp * npp;
    const int64_t nbatch = (total + BK - 1) / BK;
    const int nrt = npp / 16, nks = npp / 32;
    const int cl = lane & 15, kq = lane >> 4;   // matrix-core lane roles

    for (int64_t bt = blockIdx.x; bt < nbatch; bt += gridDim.x) {
        const int64_t j0 = bt * BK;
        // maps to -1, D to zero
        {
            uint4* z = reinterpret_cast<uint4*>(smem + L.map_off);
            const int nm = (int)((L.dr_off - L.map_off) / 16);
            const int nz = (int)((L.bytes - L.map_off) / 16);
            for (int i = tid; i < nz; i += blockDim.x)
                z[i] = (i < nm) ? make_uint4(0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu)
                                : make_uint4(0u, 0u, 0u, 0u);
        }
        __syncthreads();

        // ---- phase 1: one wavefront per K' of the batch
        int nz = 0;   // a nonzero coefficient among this lane's gathers
        for (int b = wid; b < BK; b += nwv) {
            const int64_t J = j0 + b;
            if (J >= total) break;
            const int w = find_segment(S.pwork_begin, S.sp.npcat, J);
            const PairCat& P = S.pcats[w];
            const int64_t jloc = J - S.pwork_begin[w];
            PairHdr* hd = hdr + b;
            if (lane < S.sp.K) pair_hdr_sub(S, P, jloc, lane, hd);
            wave_lds_sync();
            if (lane < S.sp.M) pair_hdr_orb(S, P, lane, hd);
            if (lane < P.ncls) pair_hdr_cls(S, P, lane, hd);
            if (lane == 63) pair_hdr_bits(S, hd);
            wave_lds_sync();
            for (int slot = lane; slot < P.deg; slot += 64) {
                int64_t addr;
                int pi, q;
                const bool neg = pair_slot(S, P, hd, slot, addr, pi, q);
                tgt[b * deg_cap + slot] = STORE ? addr * nq + q : addr;
                rinf[b * deg_cap + slot] = (pi << 1) | (neg ? 1 : 0);
                pmap[b * npp + pi] = (int16_t)slot;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    if (v >= n_vec) break;
                    const TE x = c[(int64_t)v * nd + addr];
                    nz |= V64::abs2(x) != 0.0;
                    const float sg = neg ? -1.0f : 1.0f;
                    const int col = b * NV + v;
                    Dr[col * ldd + pi] = bf16_bits(sg * (float)V64::re(x));
                    if (CPLX) Di[col * ldd + pi] = bf16_bits(sg * (float)im_part<CPLX>(x));
                }
            }
        }
        // a batch whose gathered coefficients are all zero contributes nothing
        // (zero blocks skipped, here per batch of intermediates): no product,
        // and in store mode zeros for its entries
        if (!__syncthreads_or(nz)) {
            if (STORE)
                for (int b = wid; b < BK; b += nwv) {
                    const int64_t J = j0 + b;
                    if (J >= total) break;
                    const int deg = S.pcats[find_segment(S.pwork_begin, S.sp.npcat, J)].deg;
                    for (int slot = lane; slot < deg; slot += 64)
#pragma unroll
                        for (int v = 0; v < NV; ++v)
                            if (v < n_vec) E[tgt[b * deg_cap + slot] * NV + v] = V64::zero();
                }
            __syncthreads();   // the next batch rewrites the slice
            continue;
        }

        // ---- phases 2 and 3: 16-row tiles of E over the wavefronts
        const int bcol = cl / NV, vcol = cl % NV;   // this lane's output column
        const bool live = (j0 + bcol < total) && (vcol < n_vec);
        for (int rt = wid; rt < nrt; rt += nwv) {
            f32x4 er = {0.f, 0.f, 0.f, 0.f}, er2 = er, ei = er, ei2 = er;
            const uint16_t* ap = Ab + (size_t)(rt * 16 + cl) * npp + kq * 8;
            const uint16_t* dpr = Dr + cl * ldd + kq * 8;
            const uint16_t* dpi = Di + cl * ldd + kq * 8;
            bf16x8 a0 = *reinterpret_cast<const bf16x8*>(ap);
            bf16x8 a1, a2;
            if (CPLX) {
                a1 = *reinterpret_cast<const bf16x8*>(ap + msz);
                a2 = *reinterpret_cast<const bf16x8*>(ap + 2 * msz);
            }
            for (int ks = 0; ks < nks; ++ks) {
                // fragments of this step; the next step's A fragments are
                // requested before the products (the last step rereads its own)
                const int kn = (ks + 1 < nks) ? ks + 1 : ks;
                const bf16x8 br = *reinterpret_cast<const bf16x8*>(dpr + ks * 32);
                const bf16x8 c0 = a0;
                a0 = *reinterpret_cast<const bf16x8*>(ap + kn * 32);
                er = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c0, br, er, 0, 0, 0);
                if (CPLX) {
                    const bf16x8 bi = *reinterpret_cast<const bf16x8*>(dpi + ks * 32);
                    const bf16x8 c1 = a1, c2 = a2;
                    a1 = *reinterpret_cast<const bf16x8*>(ap + msz + kn * 32);
                    a2 = *reinterpret_cast<const bf16x8*>(ap + 2 * msz + kn * 32);
                    ei = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c0, bi, ei, 0, 0, 0);
                    er2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c2, bi, er2, 0, 0, 0);
                    ei2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c1, br, ei2, 0, 0, 0);
                }
            }
            if (!live) continue;
            // this lane holds rows rt * 16 + 4 kq + i of column cl
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int pr = rt * 16 + kq * 4 + i;
                const int slot = pmap[bcol * npp + pr];
                if (slot < 0) continue;
                const double sg = (rinf[bcol * deg_cap + slot] & 1) ? -1.0 : 1.0;
                const TE val = make_scalar<CPLX>(sg * ((double)er[i] + (double)er2[i]),
                                                 sg * ((double)ei[i] + (double)ei2[i]));
                const int64_t t = tgt[bcol * deg_cap + slot];
                if (STORE)
                    E[t * NV + vcol] = val;
                else
                    V64::atomic_add(&sigma[(int64_t)vcol * nd + t], val);
            }
        }
        __syncthreads();   // the next batch rewrites the slice
    }
}

static size_t mfma_lds_bytes(int nv, int deg_max, int npp, bool cplx) {
    return MfmaLayout(MF_COLS / nv, deg_max, npp, cplx).bytes;
}

constexpr size_t MF_LDS_MAX = 160 * 1024;

// Single vectors use the 16-intermediate batch where its slice fits, else
// the 8-intermediate batch of the two-vector kernel with the second column
// of each intermediate left zero.
static bool single_fits(int deg_max, int npp, bool cplx) { return mfma_lds_bytes(1, deg_max, npp, cplx) <= MF_LDS_MAX; }

bool pair_mfma_supported(const DevSpace& S, int deg_max, bool cplx) {
    const int npp = pair_mfma_npp(S.sp.npairs);
    return S.sp.N >= 2 && deg_max > 0 && deg_max < 32768 && mfma_lds_bytes(2, deg_max, npp, cplx) <= MF_LDS_MAX;
}

template <bool CPLX, int NV, bool STORE>
static hipError_t launch_mfma_nv(const DevSpace& S, int deg_max, const void* Ab, const void* c, void* sigma,
                                 void* E, int n_vec, hipStream_t st) {
    using T64 = typename VT<CPLX>::T;
    const int npp = pair_mfma_npp(S.sp.npairs);
    const size_t lds = mfma_lds_bytes(NV, deg_max, npp, CPLX);
    const int nq = S.sp.N * (S.sp.N - 1) / 2;
    const int64_t nbatch = (S.sp.npwork_dets + MF_COLS / NV - 1) / (MF_COLS / NV);
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(nbatch, 256 * 8));
    hipLaunchKernelGGL((k_sigma_pair_mfma<CPLX, NV, STORE>), dim3((unsigned)blocks), dim3(512), lds, st, S,
                       (const uint16_t*)Ab, npp, (const T64*)c, (T64*)sigma, (T64*)E, nq, n_vec, deg_max);
    return hipGetLastError();
}

template <bool CPLX>
static hipError_t launch_mfma_all(const DevSpace& S, int deg_max, const void* Ab, const void* c, void* sigma,
                                  void* E, int n_vec, double e_core, const LaunchMarks* mk, hipStream_t st) {
    using T64 = typename VT<CPLX>::T;
    hipError_t e;
    if (!E) {
        e = launch_fill_init(CPLX, sigma, c, e_core, S.sp.ndets * n_vec, st);
        if (e != hipSuccess) return e;
    }
    const bool one = single_fits(deg_max, pair_mfma_npp(S.sp.npairs), CPLX);
    for (int v0 = 0; v0 < n_vec; v0 += 2) {
        const int nv = (n_vec - v0 >= 2) ? 2 : 1;
        const int kv = (nv == 1 && one) ? 1 : 2;   // vector width of the kernel (and of E)
        const int64_t off = (int64_t)v0 * S.sp.ndets;
        const T64* cc = (const T64*)c + off;
        T64* ss = (T64*)sigma + off;
        if (mk) mk->fn(mk->user, 0, true);
        if (E)
            e = (kv == 2) ? launch_mfma_nv<CPLX, 2, true>(S, deg_max, Ab, cc, ss, E, nv, st)
                          : launch_mfma_nv<CPLX, 1, true>(S, deg_max, Ab, cc, ss, E, 1, st);
        else
            e = (kv == 2) ? launch_mfma_nv<CPLX, 2, false>(S, deg_max, Ab, cc, ss, nullptr, nv, st)
                          : launch_mfma_nv<CPLX, 1, false>(S, deg_max, Ab, cc, ss, nullptr, 1, st);
        if (mk) mk->fn(mk->user, 0, false);
        if (e != hipSuccess) return e;
        if (E) {
            if (mk) mk->fn(mk->user, 1, true);
            e = launch_pair_reduce(S, CPLX, kv, ss, cc, E, nv, e_core, st);
            if (mk) mk->fn(mk->user, 1, false);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_sigma_pair_mfma(const DevSpace& S, int deg_max, bool cplx, const void* Ab, const void* c,
                                  void* sigma, void* E, int n_vec, double e_core, const LaunchMarks* mk,
                                  hipStream_t st) {
    return cplx ? launch_mfma_all<true>(S, deg_max, Ab, c, sigma, E, n_vec, e_core, mk, st)
                : launch_mfma_all<false>(S, deg_max, Ab, c, sigma, E, n_vec, e_core, mk, st);
}

}  // namespace stp
