// Categorical compression of CI vectors and the compression-compatible sigma
// build (Results, categorical compression; Methods, Alg. sigmaBuild).
//
// A compressed vector keeps, per space category B, the nonzero coefficients
// V^B and their local addresses A^B (position inside the category's dense
// block), ascending: the CSC pair (V, A) of the paper.  Here the categories'
// entries are stored one after the other, with cat_ptr[B] .. cat_ptr[B + 1]
// the entries of category B (an empty category has none and is skipped as a
// whole).
//
// sigma from a compressed vector follows the pair resolution of the dense
// kernels (H on the N-electron sector as one two-body operator with the
// pair-pair table A, identity over (N-2)-electron intermediates K'):
//   1. only intermediates reached from a nonzero coefficient contribute: each
//      nonzero K marks the K' = K - {q, s} of its occupied pairs;
//   2. per marked K' (one wavefront), its pair list Q leads to source
//      determinants K' + Q; the list of one pair class is the sorted
//      excitation list of Alg. sigmaBuild, and each of its addresses is
//      intersected with A^B by the exponential search of that algorithm
//      (galloping from the start of the category's entries, then a binary
//      search), giving d[Q] = sgn V[j] on a match and 0 otherwise;
//   3. e = A_K' d over the matched Q only, and sigma[K' + P] += sgn e[P].
// The work is proportional to the marked intermediates, i.e. to the
// nonzeros, not to the size of the space.  sigma is returned dense (FP64,
// device atomics), e_core c included.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "kernels.hpp"
#include "pair_arith.hpp"
#include "space.hpp"
#include "stp_device.hpp"

namespace stp {

// ---- exponential search (Alg. sigmaBuild, subroutine exponentialSearch) ----
//
// The lowest index j >= i with A[j] >= x, or n if there is none, A ascending
// on [i, n).  Reading of the printed subroutine (whose j is not initialised):
// j starts at i and is returned at once when A[i] >= x; otherwise j advances
// by 1, 2, 4, ... while A[j] < x, and the answer lies after the last probe
// below x and at or before min(j, n), found by a binary search there.
__host__ __device__ inline int64_t csc_exp_search(const uint32_t* A, int64_t n, int64_t i, uint32_t x) {
    int64_t j = i;
    if (j >= n || A[j] >= x) return j;
    int64_t d = 1;
    while (j < n && A[j] < x) {
        j += d;
        d <<= 1;
    }
    int64_t lo = j - d / 2 + 1;          // just after the last probe known to be below x
    int64_t hi = j < n ? j : n;          // A[hi] >= x, or hi = n
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (A[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// ---- compression: dense -> (cat_ptr, A, V) --------------------------------

constexpr int CSC_BLK = 1024;   // elements per counting block (256 threads x 4)

template <bool CPLX>
__device__ __forceinline__ bool csc_keep(const typename VT<CPLX>::T& x, double t2) {
    const double a = VT<CPLX>::abs2(x);
    return a != 0.0 && a >= t2;
}

// cnt[b] = kept entries of block b.
template <bool CPLX>
__global__ __launch_bounds__(256) void k_csc_count(const typename VT<CPLX>::T* __restrict__ x, int64_t n, double t2,
                                                   int64_t* __restrict__ cnt) {
    __shared__ int part[4];
    const int64_t b0 = (int64_t)blockIdx.x * CSC_BLK;
    int c = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = b0 + u * 256 + threadIdx.x;
        if (i < n && csc_keep<CPLX>(x[i], t2)) ++c;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// In-place exclusive prefix sum of cnt[0..nb) by one workgroup (nb up to a
// few million blocks: a few milliseconds), total in cnt[nb].
__global__ __launch_bounds__(1024) void k_csc_scan(int64_t* __restrict__ cnt, int64_t nb) {
    __shared__ int64_t sh[1024];
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = (i < nb) ? cnt[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t t = (threadIdx.x >= o) ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) cnt[i] = carry + sh[threadIdx.x] - v;
        const int64_t tot = sh[1023];
        __syncthreads();
        carry += tot;
    }
    if (threadIdx.x == 0) cnt[nb] = carry;
}

// Kept entries written in address order: each block's entries from its
// prefix, in order within the block (a wavefront ballot per 64 elements).
template <bool CPLX>
__global__ __launch_bounds__(256) void k_csc_write(const typename VT<CPLX>::T* __restrict__ x, int64_t n, double t2,
                                                   const int64_t* __restrict__ pre, const int64_t* __restrict__ cat_off,
                                                   int ncat, uint32_t* __restrict__ A,
                                                   typename VT<CPLX>::T* __restrict__ V, int64_t cap) {
    __shared__ int wcnt[16];
    const int64_t b0 = (int64_t)blockIdx.x * CSC_BLK;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // sub-blocks of 64 in address order: u * 4 + wid
    bool keep[4];
    int c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = b0 + (u * 4 + wid) * 64 + lane;
        keep[u] = i < n && csc_keep<CPLX>(x[i], t2);
        const uint64_t m = __ballot(keep[u]);
        c[u] = __popcll(m);
        if (lane == 0) wcnt[u * 4 + wid] = c[u];
        const uint64_t below = (lane == 0) ? 0ull : (m & ((1ull << lane) - 1ull));
        c[u] = __popcll(below);   // rank of this lane's entry in its sub-block
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (!keep[u]) continue;
        const int sb = u * 4 + wid;
        int64_t pos = pre[blockIdx.x];
        for (int t = 0; t < sb; ++t) pos += wcnt[t];
        pos += c[u];
        if (pos >= cap) continue;
        const int64_t i = b0 + sb * 64 + lane;
        const int cat = find_segment(cat_off, ncat, i);
        A[pos] = (uint32_t)(i - cat_off[cat]);
        V[pos] = x[i];
    }
}

// cat_ptr[c] = kept entries before the category's first element.
template <bool CPLX>
__global__ void k_csc_catptr(const typename VT<CPLX>::T* __restrict__ x, int64_t n, double t2,
                             const int64_t* __restrict__ pre, const int64_t* __restrict__ cat_off, int ncat,
                             int64_t* __restrict__ cat_ptr) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > ncat) return;
    const int64_t off = (c == ncat) ? n : cat_off[c];
    const int64_t b = off / CSC_BLK;
    int64_t p = pre[b];
    for (int64_t i = b * CSC_BLK; i < off; ++i)
        if (csc_keep<CPLX>(x[i], t2)) ++p;
    cat_ptr[c] = p;
}

template <bool CPLX>
__global__ void k_csc_expand(const int64_t* __restrict__ cat_ptr, const int64_t* __restrict__ cat_off, int ncat,
                             const uint32_t* __restrict__ A, const typename VT<CPLX>::T* __restrict__ V,
                             typename VT<CPLX>::T* __restrict__ x) {
    const int64_t nnz = cat_ptr[ncat];
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nnz; t += (int64_t)gridDim.x * blockDim.x) {
        const int c = find_segment(cat_ptr, ncat, t);
        x[cat_off[c] + A[t]] = V[t];
    }
}

// ---- sigma from a compressed vector ---------------------------------------

// Colex rank of a local string (binomials C(n, k) at binom[n * 33 + k]).
__device__ __forceinline__ int64_t csc_rank(uint32_t m, const int32_t* binom) {
    int64_t r = 0;
    for (int i = 0; m; m &= m - 1u, ++i) r += binom[__builtin_ctz(m) * 33 + i + 1];
    return r;
}

// Pair intermediates of the nonzeros: K' = K - {q, s} for the occupied pairs
// of every nonzero K, marked in a bitmap over the pair-intermediate index;
// and sigma = e_core c on the nonzeros (sigma zero elsewhere beforehand).
template <bool CPLX>
__global__ __launch_bounds__(256) void k_csc_mark(DevSpace S, const int64_t* __restrict__ cat_ptr,
                                                  const uint32_t* __restrict__ A,
                                                  const typename VT<CPLX>::T* __restrict__ V,
                                                  const int32_t* __restrict__ pcat_of, double e_core,
                                                  typename VT<CPLX>::T* __restrict__ sigma,
                                                  uint32_t* __restrict__ bitmap) {
    __shared__ int32_t binom[32 * 33];
    for (int t = threadIdx.x; t < 32 * 33; t += blockDim.x) {
        const int n = t / 33, k = t % 33;
        int64_t b = (k <= n) ? 1 : 0;
        for (int x = 1; x <= k && k <= n; ++x) b = b * (n - k + x) / x;
        binom[t] = (int32_t)b;
    }
    __syncthreads();
    const int K = S.sp.K, ns = S.sp.nspace;
    const int64_t nnz = cat_ptr[ns];
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nnz; t += (int64_t)gridDim.x * blockDim.x) {
        const int c = find_segment(cat_ptr, ns, t);
        const Cat& C = S.cats[c];
        const int64_t j = A[t];
        sigma[C.offset + j] = VT<CPLX>::scale(V[t], e_core);
        Det d;
        decode(S, C, j, d);
        for (int a = 0; a < K; ++a) {
            for (int b = a; b < K; ++b) {
                const int w = pcat_of[(c * KMAX + a) * KMAX + b];
                if (w < 0) continue;
                const PairCat& P = S.pcats[w];
                // every occupied q in subspace a and s in subspace b (q < s
                // when a == b): remove both, locate K' in its category
                for (uint32_t ma = d.s[a]; ma; ma &= ma - 1u) {
                    const uint32_t qa = ma & (0u - ma);   // lowest remaining bit: q
                    uint32_t mb = d.s[b];
                    if (a == b) mb &= ~((qa << 1) - 1u);  // s above q
                    const int64_t ra = (a == b) ? 0 : csc_rank(d.s[a] & ~qa, binom);
                    for (; mb; mb &= mb - 1u) {
                        const uint32_t sb = mb & (0u - mb);
                        const int64_t rb = (a == b) ? csc_rank(d.s[a] & ~qa & ~sb, binom)
                                                    : csc_rank(d.s[b] & ~sb, binom);
                        int64_t jl = 0;
                        for (int k = 0; k < K; ++k) {
                            const int64_t rk = (k == b) ? rb : (k == a ? ra : d.r[k]);
                            jl += rk * P.stride[k];
                        }
                        const int64_t J = S.pwork_begin[w] + jl;
                        atomicOr(&bitmap[J >> 5], 1u << (J & 31));
                    }
                }
            }
        }
    }
}

// Marked intermediates as a list (any order).
__global__ __launch_bounds__(256) void k_csc_collect(const uint32_t* __restrict__ bitmap, int64_t nwords,
                                                     int64_t* __restrict__ list, unsigned long long* __restrict__ count,
                                                     int64_t cap) {
    for (int64_t wd = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; wd < nwords;
         wd += (int64_t)gridDim.x * blockDim.x) {
        uint32_t m = bitmap[wd];
        if (!m) continue;
        int64_t pos = (int64_t)atomicAdd(count, (unsigned long long)__popc(m));
        for (; m; m &= m - 1u, ++pos)
            if (pos < cap) list[pos] = wd * 32 + __builtin_ctz(m);
    }
}

// LDS slice of one wavefront.
struct CscLayout {
    size_t d_off, e_off, t_off, i_off, nz_off, h_off, bytes;
    __host__ __device__ CscLayout(int deg, int se) {
        const int dp = (deg + 63) & ~63;
        d_off = 0;
        e_off = d_off + (size_t)dp * se;
        t_off = e_off + (size_t)dp * se;
        i_off = t_off + (size_t)dp * 8;
        nz_off = i_off + (size_t)dp * 4;
        h_off = (nz_off + (size_t)dp * 4 + 15) & ~(size_t)15;
        bytes = (h_off + sizeof(PairHdr) + 15) & ~(size_t)15;
    }
};

constexpr int CSC_WAVES = 4;

template <bool CPLX>
__global__ __launch_bounds__(CSC_WAVES * 64) void k_csc_contract(DevSpace S, const int64_t* __restrict__ cat_ptr,
                                                                 const uint32_t* __restrict__ A,
                                                                 const typename VT<CPLX>::T* __restrict__ V,
                                                                 const typename VT<CPLX>::T* __restrict__ pA,
                                                                 const int64_t* __restrict__ list,
                                                                 const unsigned long long* __restrict__ count,
                                                                 int64_t cap, int deg_cap,
                                                                 typename VT<CPLX>::T* __restrict__ sigma) {
    using V64 = VT<CPLX>;
    using TE = typename V64::T;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const CscLayout L(deg_cap, sizeof(TE));
    unsigned char* base = smem + (size_t)wid * L.bytes;
    TE* dsh = reinterpret_cast<TE*>(base + L.d_off);
    TE* esh = reinterpret_cast<TE*>(base + L.e_off);
    int64_t* tgt = reinterpret_cast<int64_t*>(base + L.t_off);
    int32_t* rinf = reinterpret_cast<int32_t*>(base + L.i_off);   // pair << 1 | negative sign
    int32_t* nzq = reinterpret_cast<int32_t*>(base + L.nz_off);
    PairHdr* hd = reinterpret_cast<PairHdr*>(base + L.h_off);
    const int K = S.sp.K, NP = S.sp.npairs;
    const int64_t nact = min((int64_t)*count, cap);
    for (int64_t it = (int64_t)blockIdx.x * CSC_WAVES + wid; it < nact; it += (int64_t)gridDim.x * CSC_WAVES) {
        const int64_t J = list[it];
        const int w = find_segment(S.pwork_begin, S.sp.npcat, J);
        const PairCat& P = S.pcats[w];
        const int64_t jloc = J - S.pwork_begin[w];
        const int deg = P.deg;
        if (lane < K) pair_hdr_sub(S, P, jloc, lane, hd);
        wave_lds_sync();
        if (lane < S.sp.M) pair_hdr_orb(S, P, lane, hd);
        if (lane < P.ncls) pair_hdr_cls(S, P, lane, hd);
        if (lane == 63) pair_hdr_bits(S, hd);
        wave_lds_sync();
        // pair list of K': target / source address, sign; the source's
        // coefficient from the compressed category by exponential search
        int nnz_w = 0;
        for (int s0 = 0; s0 < deg; s0 += 64) {
            const int slot = s0 + lane;
            bool hit = false;
            if (slot < deg) {
                int64_t addr;
                int pi, q;
                const bool neg = pair_slot(S, P, hd, slot, addr, pi, q);
                const uint32_t info = S.pslot[P.slot_off + slot];
                const int cat = P.cls_target[info & 255u];
                const int64_t lo = cat_ptr[cat], hi = cat_ptr[cat + 1];
                const uint32_t la = (uint32_t)(addr - S.cats[cat].offset);
                TE x = V64::zero();
                if (lo < hi) {
                    const int64_t jj = csc_exp_search(A, hi, lo, la);
                    if (jj < hi && A[jj] == la) {
                        x = V[jj];
                        hit = true;
                    }
                }
                tgt[slot] = addr;
                rinf[slot] = (pi << 1) | (neg ? 1 : 0);
                dsh[slot] = neg ? V64::scale(x, -1.0) : x;
                esh[slot] = V64::zero();
            }
            // compact the matched slots of this round into nzq
            const uint64_t m = __ballot(hit);
            if (hit) nzq[nnz_w + __popcll(m & ((1ull << lane) - 1ull))] = slot;
            nnz_w += __popcll(m);
        }
        wave_lds_sync();
        if (nnz_w == 0) continue;   // no nonzero source: nothing to add
        // e[P] = sum over the matched Q of A[P, Q] d[Q] (pA[pair Q * NP + pair P])
        for (int u = 0; u < nnz_w; ++u) {
            const int qs = nzq[u];
            const TE dq = dsh[qs];
            const int64_t rowq = (int64_t)(rinf[qs] >> 1) * NP;
            for (int slot = lane; slot < deg; slot += 64) {
                const TE a = pA[rowq + (rinf[slot] >> 1)];
                esh[slot] = V64::mad(a, dq, esh[slot]);
            }
        }
        wave_lds_sync();
        for (int slot = lane; slot < deg; slot += 64) {
            const double sg = (rinf[slot] & 1) ? -1.0 : 1.0;
            V64::atomic_add(&sigma[tgt[slot]], V64::scale(esh[slot], sg));
        }
        wave_lds_sync();
    }
}

// ---- host side ------------------------------------------------------------

void build_csc_pcat_of(const HostSpace& H, std::vector<int32_t>& out) {
    const Space& sp = H.sp;
    out.assign((size_t)sp.nspace * KMAX * KMAX, -1);
    for (int c = 0; c < sp.nspace; ++c) {
        const Cat& C = H.cats[c];
        for (int a = 0; a < sp.K; ++a)
            for (int b = a; b < sp.K; ++b) {
                int occ[KMAX];
                for (int k = 0; k < sp.K; ++k) occ[k] = C.occ[k];
                --occ[a];
                --occ[b];
                bool ok = true;
                for (int k = 0; k < sp.K; ++k) ok = ok && occ[k] >= 0;
                if (!ok) continue;
                for (int w = 0; w < sp.npcat; ++w) {
                    bool eq = true;
                    for (int k = 0; k < sp.K; ++k) eq = eq && H.pcats[w].occ[k] == occ[k];
                    if (eq) {
                        out[((size_t)c * KMAX + a) * KMAX + b] = w;
                        break;
                    }
                }
            }
    }
}

size_t csc_slice_bytes(int deg_max, bool cplx) { return CscLayout(deg_max, cplx ? 16 : 8).bytes; }

hipError_t launch_csc_compress(const DevSpace& S, bool cplx, const void* x, double thresh, const int64_t* cat_off,
                               int64_t* cnt, int64_t* cat_ptr, uint32_t* A, void* V, int64_t cap, hipStream_t st) {
    const int64_t n = S.sp.ndets;
    const int64_t nb = (n + CSC_BLK - 1) / CSC_BLK;
    const double t2 = thresh * thresh;
    const int ncat = S.sp.nspace;
    if (cplx) {
        using T = VT<true>::T;
        hipLaunchKernelGGL(k_csc_count<true>, dim3((unsigned)nb), dim3(256), 0, st, (const T*)x, n, t2, cnt);
        hipLaunchKernelGGL(k_csc_scan, dim3(1), dim3(1024), 0, st, cnt, nb);
        hipLaunchKernelGGL(k_csc_catptr<true>, dim3((ncat + 1 + 63) / 64), dim3(64), 0, st, (const T*)x, n, t2, cnt,
                           cat_off, ncat, cat_ptr);
        hipLaunchKernelGGL(k_csc_write<true>, dim3((unsigned)nb), dim3(256), 0, st, (const T*)x, n, t2, cnt, cat_off,
                           ncat, A, (T*)V, cap);
    } else {
        using T = VT<false>::T;
        hipLaunchKernelGGL(k_csc_count<false>, dim3((unsigned)nb), dim3(256), 0, st, (const T*)x, n, t2, cnt);
        hipLaunchKernelGGL(k_csc_scan, dim3(1), dim3(1024), 0, st, cnt, nb);
        hipLaunchKernelGGL(k_csc_catptr<false>, dim3((ncat + 1 + 63) / 64), dim3(64), 0, st, (const T*)x, n, t2, cnt,
                           cat_off, ncat, cat_ptr);
        hipLaunchKernelGGL(k_csc_write<false>, dim3((unsigned)nb), dim3(256), 0, st, (const T*)x, n, t2, cnt, cat_off,
                           ncat, A, (T*)V, cap);
    }
    return hipGetLastError();
}

hipError_t launch_csc_expand(const DevSpace& S, bool cplx, const int64_t* cat_ptr, const int64_t* cat_off,
                             const uint32_t* A, const void* V, void* x, hipStream_t st) {
    const int ncat = S.sp.nspace;
    if (cplx)
        hipLaunchKernelGGL(k_csc_expand<true>, dim3(2048), dim3(256), 0, st, cat_ptr, cat_off, ncat, A,
                           (const VT<true>::T*)V, (VT<true>::T*)x);
    else
        hipLaunchKernelGGL(k_csc_expand<false>, dim3(2048), dim3(256), 0, st, cat_ptr, cat_off, ncat, A,
                           (const VT<false>::T*)V, (VT<false>::T*)x);
    return hipGetLastError();
}

hipError_t launch_csc_sigma(const DevSpace& S, bool cplx, const int64_t* cat_ptr, const uint32_t* A, const void* V,
                            const void* pA, const int32_t* pcat_of, double e_core, int deg_max, uint32_t* bitmap,
                            int64_t nwords, int64_t* list, unsigned long long* count, int64_t cap, void* sigma,
                            hipStream_t st) {
    const size_t lds = (size_t)CSC_WAVES * CscLayout(deg_max, cplx ? 16 : 8).bytes;
    if (cplx) {
        using T = VT<true>::T;
        hipLaunchKernelGGL(k_csc_mark<true>, dim3(2048), dim3(256), 0, st, S, cat_ptr, A, (const T*)V, pcat_of,
                           e_core, (T*)sigma, bitmap);
        hipLaunchKernelGGL(k_csc_collect, dim3(2048), dim3(256), 0, st, bitmap, nwords, list, count, cap);
        hipLaunchKernelGGL(k_csc_contract<true>, dim3(2048), dim3(CSC_WAVES * 64), lds, st, S, cat_ptr, A,
                           (const T*)V, (const T*)pA, list, count, cap, deg_max, (T*)sigma);
    } else {
        using T = VT<false>::T;
        hipLaunchKernelGGL(k_csc_mark<false>, dim3(2048), dim3(256), 0, st, S, cat_ptr, A, (const T*)V, pcat_of,
                           e_core, (T*)sigma, bitmap);
        hipLaunchKernelGGL(k_csc_collect, dim3(2048), dim3(256), 0, st, bitmap, nwords, list, count, cap);
        hipLaunchKernelGGL(k_csc_contract<false>, dim3(2048), dim3(CSC_WAVES * 64), lds, st, S, cat_ptr, A,
                           (const T*)V, (const T*)pA, list, count, cap, deg_max, (T*)sigma);
    }
    return hipGetLastError();
}

__global__ void k_csc_search_test(const uint32_t* __restrict__ A, int64_t n, const int64_t* __restrict__ starts,
                                  const uint32_t* __restrict__ xs, int64_t* __restrict__ out, int64_t m) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) out[t] = csc_exp_search(A, n, starts[t], xs[t]);
}

hipError_t launch_csc_search_test(const uint32_t* A, int64_t n, const int64_t* starts, const uint32_t* xs,
                                  int64_t* out, int64_t m, hipStream_t st) {
    if (m > 0)
        hipLaunchKernelGGL(k_csc_search_test, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, A, n, starts, xs,
                           out, m);
    return hipGetLastError();
}

int64_t csc_exp_search_host(const uint32_t* A, int64_t n, int64_t i, uint32_t x) {
    return csc_exp_search(A, n, i, x);
}

}  // namespace stp
