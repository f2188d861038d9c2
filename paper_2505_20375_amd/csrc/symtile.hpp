// Hermitian-tile contraction shared by the sigma kernels: e = G d for one
// intermediate determinant, where G is a Hermitian submatrix of a global
// integral table selected by the intermediate's move (or pair) list.
//
// The list of d slots is cut into blocks of 4; the upper triangle of 4x4
// block pairs (b <= b') is split evenly over the 64 lanes of the wavefront.
// A lane loads one 16-element tile (rows: 4 slots, whose table indices are
// usually adjacent in memory) and uses every element for all vectors and, off
// the diagonal, twice:
//   e[rows b]  += G[b, b'] d[b']          (kept in registers while b repeats)
//   e[cols b'] += G[b, b']^H d[b]         (added to LDS with LDS atomics).
// Element (row slot s, column slot t) is table[coff[t] + (rinf[s] >> 1)].
#pragma once
#include "stp_device.hpp"

namespace stp {

constexpr int ST_TILE = 4;

// LDS index of (slot, vector): blocks of 4 slots are padded by 16 bytes so
// that the lanes of a wavefront, which read blocks at a stride of one block,
// start on different banks.
template <int NV, int SB>
__device__ __forceinline__ int st_idx(int slot, int v) {
    constexpr int blk = ST_TILE * NV + 16 / SB;  // elements per padded block
    return (slot >> 2) * blk + (slot & 3) * NV + v;
}

template <int NV, int SB>
__host__ __device__ constexpr int st_elems(int deg_cap) {
    return ((deg_cap + 3) >> 2) * (ST_TILE * NV + 16 / SB);
}

// Requires: slots [deg, (deg + 3) & ~3) hold d = e = 0 and in-range rinf/coff.
template <bool CPLX, bool F32, int NV>
__device__ __forceinline__ void tile_contract(const typename PT<CPLX, F32>::T* __restrict__ gT,
                                              const typename PT<CPLX, F32>::T* dsh, typename PT<CPLX, F32>::T* esh,
                                              const int32_t* rinf, const int32_t* coff, int deg, int lane) {
    using V = PT<CPLX, F32>;
    using T = typename V::T;
    constexpr int SB = sizeof(T);
    const int nb = (deg + ST_TILE - 1) / ST_TILE;
    const int np = nb * (nb + 1) / 2;
    const int p0 = (int)(((int64_t)lane * np) >> 6);
    const int p1 = (int)(((int64_t)(lane + 1) * np) >> 6);
    int b = 0, start = 0;
    while (b < nb && start + (nb - b) <= p0) {
        start += nb - b;
        ++b;
    }
    int bp = b + (p0 - start);
    int cur = -1;
    int prow[ST_TILE];
    T drow[ST_TILE][NV], erow[ST_TILE][NV];
    for (int p = p0; p < p1; ++p) {
        if (b != cur) {
            if (cur >= 0) {
#pragma unroll
                for (int r = 0; r < ST_TILE; ++r)
#pragma unroll
                    for (int v = 0; v < NV; ++v) V::lds_add(&esh[st_idx<NV, SB>(cur * ST_TILE + r, v)], erow[r][v]);
            }
            cur = b;
#pragma unroll
            for (int r = 0; r < ST_TILE; ++r) {
                const int s = b * ST_TILE + r;
                prow[r] = rinf[s] >> 1;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    drow[r][v] = dsh[st_idx<NV, SB>(s, v)];
                    erow[r][v] = V::zero();
                }
            }
        }
        const bool offdiag = (bp != b);
#pragma unroll
        for (int k = 0; k < ST_TILE; ++k) {
            const int s = bp * ST_TILE + k;
            if (s >= deg) break;
            const int co = coff[s];
            T dcol[NV], ecol[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                dcol[v] = dsh[st_idx<NV, SB>(s, v)];
                ecol[v] = V::zero();
            }
            T g[ST_TILE];
#pragma unroll
            for (int r = 0; r < ST_TILE; ++r) g[r] = gT[co + prow[r]];
#pragma unroll
            for (int r = 0; r < ST_TILE; ++r)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    erow[r][v] = V::mad(g[r], dcol[v], erow[r][v]);
                    ecol[v] = V::cmad(g[r], drow[r][v], ecol[v]);
                }
            if (offdiag) {
#pragma unroll
                for (int v = 0; v < NV; ++v) V::lds_add(&esh[st_idx<NV, SB>(s, v)], ecol[v]);
            }
        }
        if (++bp == nb) {
            ++b;
            bp = b;
        }
    }
    if (cur >= 0) {
#pragma unroll
        for (int r = 0; r < ST_TILE; ++r)
#pragma unroll
            for (int v = 0; v < NV; ++v) V::lds_add(&esh[st_idx<NV, SB>(cur * ST_TILE + r, v)], erow[r][v]);
    }
}

// sigma <- e_core * c (or 0), n elements of each described problem; used before
// the accumulating sigma kernels.
template <bool CPLX>
__device__ __forceinline__ void fill_init(typename VT<CPLX>::T* __restrict__ sigma,
                                          const typename VT<CPLX>::T* __restrict__ c, double e_core, int64_t n,
                                          int64_t first, int64_t step) {
    if (e_core == 0.0) {
        for (int64_t e = first; e < n; e += step) sigma[e] = VT<CPLX>::zero();
    } else {
        for (int64_t e = first; e < n; e += step) sigma[e] = VT<CPLX>::scale(c[e], e_core);
    }
}

}  // namespace stp
