// Pair-resolved sigma build (the library's default for N >= 2).
//
// The Hamiltonian restricted to N electrons is written as one two-body
// operator, H - e_core = sum_{p<r, q<s} A[(p,r),(q,s)] a+_p a+_r a_s a_q with
//   A[(p,r),(q,s)] = g'_pqrs - g'_psrq,
//   g'_pqrs = (pq|rs) + (h_pq d_rs + d_pq h_rs) / (N - 1),
// (the one-electron part folded into the two-electron integrals, which is
// exact on the N-electron sector).  A is Hermitian in the pair indices.
// Inserting the identity over (N-2)-electron determinants K' between the
// creation and annihilation pairs (the resolution of Eq. sigmaL2e taken two
// electrons down):
//   d[Q]  = sgn(a+_q a+_s |K'>) c[K' + {q, s}]         (gather)
//   e     = A_K' d,   A_K'[P, Q] = A[pair P, pair Q]    (Hermitian tiles)
//   sigma[K' + {p, r}] += sgn(a+_p a+_r |K'>) e[P]      (scatter)
// over the pairs P, Q that lead from K' into the space.  The K' are grouped
// into occupation categories of the same subspaces (STP-DAS); targets are
// addressed through the per-subspace string tables, as in the one-move form.
// One wavefront handles one K' with its LDS slice.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"
#include "pair_arith.hpp"
#include "stp_device.hpp"
#include "symtile.hpp"

namespace stp {

// LDS layout of one wavefront's slice: d (contraction type) and e (FP64),
// targets, row pair indices, header.
__host__ __device__ inline SliceLayout pair_layout(int deg_max, int nv, bool cplx, bool f32) {
    const int se = cplx ? 16 : 8;
    const int sb = f32 ? se / 2 : se;
    return SliceLayout(deg_max, nv, sb, se, sizeof(PairHdr));
}

size_t pair_slice_bytes(int deg_max, int nv, bool cplx, bool f32) { return pair_layout(deg_max, nv, cplx, f32).bytes; }

bool pair_supported(int n_elec, int deg_max, bool cplx) {
    return n_elec >= 2 && deg_max > 0 && pair_slice_bytes(deg_max, 2, cplx, false) <= 64 * 1024;
}

// STORE: e[P] goes to E[(target * nq + q) * NV + v] (each entry written by
// exactly one K'; k_pair_reduce sums them), else it is added to sigma with
// device atomics.
template <bool CPLX, bool F32, int NV, bool STORE>
__device__ __forceinline__ void pair_det(const DevSpace& S, const typename PT<CPLX, F32>::T* __restrict__ A,
                                         const typename VT<CPLX>::T* __restrict__ c,
                                         typename VT<CPLX>::T* __restrict__ sigma, typename VT<CPLX>::T* __restrict__ E,
                                         int nq, int n_vec, int deg_cap, unsigned char* base, int lane, int64_t J) {
    using V = PT<CPLX, F32>;
    using V64 = VT<CPLX>;
    using T = typename V::T;
    using TE = typename V64::T;
    constexpr int SB = sizeof(T);
    constexpr int SE = sizeof(TE);
    const SliceLayout L(deg_cap, NV, SB, SE, sizeof(PairHdr));
    T* dsh = reinterpret_cast<T*>(base + L.d_off);                 // padded [slot][NV]
    TE* esh = reinterpret_cast<TE*>(base + L.e_off);               // padded [slot][NV], FP64
    int64_t* tgt = reinterpret_cast<int64_t*>(base + L.tgt_off);   // target address
    int32_t* rinf = reinterpret_cast<int32_t*>(base + L.i0_off);   // pair(P) << 1 | negative sign
    PairHdr* hd = reinterpret_cast<PairHdr*>(base + L.x_off);
    const int K = S.sp.K;
    const int64_t nd = S.sp.ndets;
    const int w = find_segment(S.pwork_begin, S.sp.npcat, J);
    const PairCat& P = S.pcats[w];
    const int64_t jloc = J - S.pwork_begin[w];
    const int deg = P.deg;

    // ---- phase 1: strings of K', its empty orbitals and class bases, then
    // per pair slot the target, sign and gathered coefficients
    if (lane < K) pair_hdr_sub(S, P, jloc, lane, hd);
    wave_lds_sync();
    if (lane < S.sp.M) pair_hdr_orb(S, P, lane, hd);
    if (lane < P.ncls) pair_hdr_cls(S, P, lane, hd);
    if (lane == 63) pair_hdr_bits(S, hd);
    wave_lds_sync();
    const int NP = S.sp.npairs;
    bool nz = false;   // a nonzero coefficient among this lane's slots
    for (int slot = lane; slot < ((deg + 3) & ~3); slot += 64) {
        if (slot >= deg) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                dsh[st_idx<NV, SB>(slot, v)] = V::zero();
                esh[st_idx<NV, SE>(slot, v)] = V64::zero();
            }
            rinf[slot] = 0;
            continue;
        }
        int64_t addr;
        int pi, q;
        const bool neg = pair_slot(S, P, hd, slot, addr, pi, q);
        tgt[slot] = STORE ? addr * nq + q : addr;
        rinf[slot] = (pi << 1) | (neg ? 1 : 0);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const TE x = (v < n_vec) ? c[(int64_t)v * nd + addr] : V64::zero();
            nz = nz || V64::abs2(x) != 0.0;
            T val = V::from64(x);
            if (neg) val = V::scale(val, -1.0);
            dsh[st_idx<NV, SB>(slot, v)] = val;
            esh[st_idx<NV, SE>(slot, v)] = V64::zero();
        }
    }
    wave_lds_sync();
    // an intermediate whose gathered coefficients are all zero contributes
    // nothing (the categorical skipping of zero blocks, here per
    // intermediate): no contraction, and in store mode zeros for its entries
    const bool live = __ballot(nz) != 0;

    // ---- phase 2: e = A_K' d
    if (live) tile_contract<CPLX, F32, NV>(A, NP, dsh, esh, rinf, deg, lane);
    wave_lds_sync();

    // ---- phase 3: sigma[K' + P] += sgn(P) e[P]
    for (int slot = lane; slot < ((STORE || live) ? deg : 0); slot += 64) {
        const double sg = (rinf[slot] & 1) ? -1.0 : 1.0;
        const int64_t t = tgt[slot];
        if (STORE) {
#pragma unroll
            for (int v = 0; v < NV; ++v) E[t * NV + v] = V64::scale(esh[st_idx<NV, SE>(slot, v)], sg);
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < n_vec)
                    V64::atomic_add(&sigma[(int64_t)v * nd + t], V64::scale(esh[st_idx<NV, SE>(slot, v)], sg));
        }
    }
    wave_lds_sync();  // the next K' reuses this wavefront's LDS slice
}

template <bool CPLX, bool F32, int NV, bool STORE>
__global__ __launch_bounds__(256) void k_sigma_pair(DevSpace S, const typename PT<CPLX, F32>::T* __restrict__ A,
                                                   const typename VT<CPLX>::T* __restrict__ c,
                                                   typename VT<CPLX>::T* __restrict__ sigma,
                                                   typename VT<CPLX>::T* __restrict__ E, int nq, int n_vec,
                                                   int deg_cap) {
    using T = typename PT<CPLX, F32>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    unsigned char* base = smem + (size_t)wid * pair_layout(deg_cap, NV, CPLX, F32).bytes;
    const int64_t total = S.sp.npwork_dets;
    const int64_t nw = (int64_t)gridDim.x * wpb;
    for (int64_t J = (int64_t)blockIdx.x * wpb + wid; J < total; J += nw)
        pair_det<CPLX, F32, NV, STORE>(S, A, c, sigma, E, nq, n_vec, deg_cap, base, lane, J);
}

// sigma[v][L] = e_core c[v][L] + sum_q E[(L * nq + q) * NV + v]: the pair
// contributions of every target, summed in a fixed order.  Eight lanes share
// a target: lane g adds entries g, g + 8, ... of its nq * NV contiguous
// entries (so every read instruction covers 128 contiguous bytes per complex
// target), then the lanes holding the same vector (g mod NV) are combined by
// a fixed butterfly.
constexpr int PR_LANES = 8;
template <bool CPLX, int NV>
__global__ __launch_bounds__(256) void k_pair_reduce(typename VT<CPLX>::T* __restrict__ sigma,
                                                    const typename VT<CPLX>::T* __restrict__ c,
                                                    const typename VT<CPLX>::T* __restrict__ E, double e_core,
                                                    int64_t nd, int nq, int n_vec) {
    static_assert(PR_LANES % NV == 0, "each lane must hold one vector");
    using V64 = VT<CPLX>;
    using TE = typename V64::T;
    const int g = threadIdx.x & (PR_LANES - 1);
    const int per = nq * NV;
    const int64_t step = (int64_t)gridDim.x * (blockDim.x / PR_LANES);
    // L is equal on the eight lanes of a group, so groups enter and leave the
    // loop together and the shuffles stay inside active groups
    for (int64_t L = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / PR_LANES; L < nd; L += step) {
        TE acc = V64::zero();
        const TE* e = E + L * per;
        // eight reads in flight per lane, added in the same order as one by one
        constexpr int PR_BATCH = 8;
        for (int f = g; f < per; f += PR_BATCH * PR_LANES) {
            TE x[PR_BATCH];
#pragma unroll
            for (int k = 0; k < PR_BATCH; ++k)
                if (f + k * PR_LANES < per) x[k] = e[f + k * PR_LANES];
#pragma unroll
            for (int k = 0; k < PR_BATCH; ++k)
                if (f + k * PR_LANES < per) acc = V64::add(acc, x[k]);
        }
        for (int m = NV; m < PR_LANES; m <<= 1) acc = V64::add(acc, V64::shfl_xor(acc, m));
        if (g < NV && g < n_vec) {
            // e_core = 0 (the usual case) skips the read of c
            const TE base = e_core != 0.0 ? V64::scale(c[(int64_t)g * nd + L], e_core) : V64::zero();
            sigma[(int64_t)g * nd + L] = V64::add(base, acc);
        }
    }
}

template <bool CPLX, bool F32, int NV, bool STORE>
static hipError_t launch_pair_nv(const DevSpace& S, int deg_max, const void* A, const void* c, void* sigma, void* E,
                                 int nq, int nv, double e_core, const LaunchMarks* mk, hipStream_t st) {
    using T = typename PT<CPLX, F32>::T;
    using T64 = typename VT<CPLX>::T;
    const size_t per_wave = pair_slice_bytes(deg_max, NV, CPLX, F32);
    const int wpb = waves_per_group(per_wave);
    const size_t lds = per_wave * wpb;
    int64_t blocks = (S.sp.npwork_dets + wpb - 1) / wpb;
    blocks = std::max<int64_t>(1, std::min<int64_t>(blocks, 256 * 64));
    if (mk) mk->fn(mk->user, 0, true);
    hipLaunchKernelGGL((k_sigma_pair<CPLX, F32, NV, STORE>), dim3((unsigned)blocks), dim3(64 * wpb), lds, st, S,
                       (const T*)A, (const T64*)c, (T64*)sigma, (T64*)E, nq, nv, deg_max);
    if (mk) mk->fn(mk->user, 0, false);
    if (STORE) {
        const int64_t nd = S.sp.ndets;
        const int g = (int)std::max<int64_t>(1, std::min<int64_t>(16384, (nd * PR_LANES + 255) / 256));
        if (mk) mk->fn(mk->user, 1, true);
        hipLaunchKernelGGL((k_pair_reduce<CPLX, NV>), dim3(g), dim3(256), 0, st, (T64*)sigma, (const T64*)c,
                           (const T64*)E, e_core, nd, nq, nv);
        if (mk) mk->fn(mk->user, 1, false);
    }
    return hipGetLastError();
}

template <bool CPLX, bool F32>
static hipError_t launch_pair_all(const DevSpace& S, int deg_max, const void* A, const void* c, void* sigma,
                                  void* E, int n_vec, double e_core, const LaunchMarks* mk, hipStream_t st) {
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
        if (E)
            e = (nv == 2) ? launch_pair_nv<CPLX, F32, 2, true>(S, deg_max, A, cc, ss, E, nq, 2, e_core, mk, st)
                          : launch_pair_nv<CPLX, F32, 1, true>(S, deg_max, A, cc, ss, E, nq, 1, e_core, mk, st);
        else
            e = (nv == 2) ? launch_pair_nv<CPLX, F32, 2, false>(S, deg_max, A, cc, ss, nullptr, 0, 2, 0.0, mk, st)
                          : launch_pair_nv<CPLX, F32, 1, false>(S, deg_max, A, cc, ss, nullptr, 0, 1, 0.0, mk, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// sigma = e_core c + sum_q E for nv (1 or 2) vectors stored with stride nv.
hipError_t launch_pair_reduce(const DevSpace& S, bool cplx, int nv, void* sigma, const void* c, const void* E,
                              int n_vec, double e_core, hipStream_t st) {
    const int64_t nd = S.sp.ndets;
    const int nq = S.sp.N * (S.sp.N - 1) / 2;
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>(16384, (nd * PR_LANES + 255) / 256));
    if (cplx) {
        using T = VT<true>::T;
        if (nv == 2)
            hipLaunchKernelGGL((k_pair_reduce<true, 2>), dim3(g), dim3(256), 0, st, (T*)sigma, (const T*)c,
                               (const T*)E, e_core, nd, nq, n_vec);
        else
            hipLaunchKernelGGL((k_pair_reduce<true, 1>), dim3(g), dim3(256), 0, st, (T*)sigma, (const T*)c,
                               (const T*)E, e_core, nd, nq, n_vec);
    } else {
        if (nv == 2)
            hipLaunchKernelGGL((k_pair_reduce<false, 2>), dim3(g), dim3(256), 0, st, (double*)sigma,
                               (const double*)c, (const double*)E, e_core, nd, nq, n_vec);
        else
            hipLaunchKernelGGL((k_pair_reduce<false, 1>), dim3(g), dim3(256), 0, st, (double*)sigma,
                               (const double*)c, (const double*)E, e_core, nd, nq, n_vec);
    }
    return hipGetLastError();
}

size_t pair_store_bytes(const DevSpace& S, bool cplx) {
    return (size_t)S.sp.ndets * (size_t)(S.sp.N * (S.sp.N - 1) / 2) * 2 * (cplx ? 16 : 8);
}

hipError_t launch_sigma_pair(const DevSpace& S, int deg_max, bool cplx, bool f32, const void* A, const void* c,
                             void* sigma, void* E, int n_vec, double e_core, const LaunchMarks* mk, hipStream_t st) {
    if (cplx)
        return f32 ? launch_pair_all<true, true>(S, deg_max, A, c, sigma, E, n_vec, e_core, mk, st)
                   : launch_pair_all<true, false>(S, deg_max, A, c, sigma, E, n_vec, e_core, mk, st);
    return f32 ? launch_pair_all<false, true>(S, deg_max, A, c, sigma, E, n_vec, e_core, mk, st)
               : launch_pair_all<false, false>(S, deg_max, A, c, sigma, E, n_vec, e_core, mk, st);
}

// Host check of the pair arithmetic above (the same functions, run on the
// host tables): for up to max_dets_per_cat K' of every pair category, every
// slot's target must be K' + {p, r} in the space, with the sign of
// a+_p a+_r |K'> from the global occupation bits and the pair index of p < r.
int64_t check_pairs_host(const DevSpace& S, int64_t max_dets_per_cat, int64_t* n_checked,
                         bool (*to_bits)(const void*, int64_t, uint64_t*), const void* user) {
    int64_t bad = 0, checked = 0;
    const int K = S.sp.K;
    for (int w = 0; w < S.sp.npcat; ++w) {
        const PairCat& P = S.pcats[w];
        const int64_t step = P.size <= max_dets_per_cat ? 1 : P.size / max_dets_per_cat;
        for (int64_t j = 0; j < P.size; j += step) {
            PairHdr hd;
            for (int k = 0; k < K; ++k) pair_hdr_sub(S, P, j, k, &hd);
            for (int g = 0; g < S.sp.M; ++g) pair_hdr_orb(S, P, g, &hd);
            for (int c = 0; c < P.ncls; ++c) pair_hdr_cls(S, P, c, &hd);
            pair_hdr_bits(S, &hd);
            uint64_t Kb = 0;
            for (int k = 0; k < K; ++k) Kb |= (uint64_t)hd.str[k] << S.sp.sub_off[k];
            for (int slot = 0; slot < P.deg; ++slot) {
                int64_t t;
                int pi, q;
                const bool neg = pair_slot(S, P, &hd, slot, t, pi, q);
                ++checked;
                // recover p < r from the pair index
                int r = 1;
                while ((r + 1) * r / 2 <= pi) ++r;
                const int p = pi - r * (r - 1) / 2;
                const bool free_pr = p < r && !((Kb >> p) & 1ULL) && !((Kb >> r) & 1ULL);
                const uint64_t want = Kb | (1ULL << p) | (1ULL << r);
                const int par = __builtin_popcountll(Kb & ((1ULL << r) - 1ULL)) +
                                __builtin_popcountll(Kb & ((1ULL << p) - 1ULL));
                // q: index of {p, r} in the list of the target's occupied pairs (i < j)
                int occ[64], no = 0, qw = -1;
                for (int x = 0; x < S.sp.M; ++x)
                    if ((want >> x) & 1ULL) occ[no++] = x;
                for (int jj = 1, n = 0; jj < no && qw < 0; ++jj)
                    for (int ii = 0; ii < jj; ++ii, ++n)
                        if (occ[ii] == p && occ[jj] == r) qw = n;
                uint64_t got = 0;
                if (!free_pr || t < 0 || t >= S.sp.ndets || !to_bits(user, t, &got) || got != want ||
                    neg != ((par & 1) != 0) || q != qw)
                    ++bad;
            }
        }
    }
    if (n_checked) *n_checked = checked;
    return bad;
}

}  // namespace stp
