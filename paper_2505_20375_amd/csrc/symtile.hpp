// Hermitian-tile contraction shared by the sigma kernels: e = G d for one
// intermediate determinant, where G is a Hermitian submatrix of a global
// integral table selected by the intermediate's move (or pair) list.
//
// The list of d slots is cut into blocks of 4; the upper triangle of 4x4
// block pairs (b <= b') is split evenly over the 64 lanes.  A lane loads one
// 16-element tile (rows: 4 slots, whose table indices are usually adjacent in
// memory) and uses every element for all vectors and, off the diagonal, twice:
//   e[rows b]  += G[b, b'] d[b']          (kept in registers while b repeats)
//   e[cols b'] += G[b, b']^H d[b]         (added to LDS with FP64 LDS atomics).
// Element (row slot s, column slot t) is table[row(t) * stride + row(s)],
// row(s) = rinf[s] >> 1.  The tiles of a lane are software-pipelined by half
// tiles: the 8 loads of the next half tile are issued before the current half
// is contracted.
// Partial sums are kept in the contraction type T (FP32 for the FP32 form);
// the LDS accumulators e are FP64 in both forms.
#pragma once
#include "stp_device.hpp"

namespace stp {

constexpr int ST_TILE = 4;

// LDS index of (slot, vector): blocks of 4 slots are padded by 16 bytes so
// that lanes reading blocks at a stride of one block start on different banks.
template <int NV, int SB>
__host__ __device__ __forceinline__ int st_idx(int slot, int v) {
    constexpr int blk = ST_TILE * NV + 16 / SB;  // elements per padded block
    return (slot >> 2) * blk + (slot & 3) * NV + v;
}

template <int NV, int SB>
__host__ __device__ constexpr int st_elems(int deg_cap) {
    return ((deg_cap + 3) >> 2) * (ST_TILE * NV + 16 / SB);
}

// Per-wavefront LDS slice: d [padded slots][NV] in the contraction type (sb
// bytes), e [padded slots][NV] FP64 (se bytes), then per slot an int64 target
// and an int32 word (rinf), then `extra` bytes.  All offsets are multiples of
// 16 bytes; every per-slot array covers the padded slot count.
struct SliceLayout {
    size_t d_off, e_off, tgt_off, i0_off, x_off, bytes;
    __host__ __device__ SliceLayout(int deg_cap, int nv, int sb, int se, size_t extra) {
        const int cap4 = (deg_cap + 3) & ~3;
        const size_t blocks = (size_t)((deg_cap + 3) >> 2);
        d_off = 0;
        e_off = blocks * (size_t)(ST_TILE * nv * sb + 16);
        tgt_off = e_off + blocks * (size_t)(ST_TILE * nv * se + 16);
        i0_off = tgt_off + (size_t)cap4 * 8;
        x_off = i0_off + (size_t)((cap4 * 4 + 15) & ~15);
        bytes = x_off + extra;
    }
};

template <bool CPLX, bool F32, int NV>
struct TileIO {
    using V = PT<CPLX, F32>;
    using T = typename V::T;
    using V64 = VT<CPLX>;
    using TE = typename V64::T;
    static constexpr int SB = sizeof(T);
    static constexpr int SE = sizeof(TE);
    static __device__ __forceinline__ void add_e(TE* esh, int s, int v, T x) {
        V64::lds_add(&esh[st_idx<NV, SE>(s, v)], V::to64(x));
    }
};

// Upper-triangle tile walk of one lane: tile index p -> block pair (b, bp).
struct TileWalk {
    int nb, b, bp;
    __device__ __forceinline__ void start(int p) {
        b = 0;
        int start = 0;
        while (b < nb && start + (nb - b) <= p) {
            start += nb - b;
            ++b;
        }
        bp = b + (p - start);
    }
    __device__ __forceinline__ void next() {
        if (++bp == nb) {
            ++b;
            bp = b;
        }
    }
};

// Requires: slots [deg, (deg + 3) & ~3) hold d = 0 and in-range rinf.
template <bool CPLX, bool F32, int NV>
__device__ __forceinline__ void tile_contract(const typename PT<CPLX, F32>::T* __restrict__ tab, int stride,
                                              const typename PT<CPLX, F32>::T* dsh, typename VT<CPLX>::T* esh,
                                              const int32_t* rinf, int deg, int lane) {
    using IO = TileIO<CPLX, F32, NV>;
    using V = typename IO::V;
    using T = typename IO::T;
    constexpr int SB = IO::SB;
    const int nb = (deg + ST_TILE - 1) / ST_TILE;
    const int np = nb * (nb + 1) / 2;
    const int p0 = (int)(((int64_t)lane * np) >> 6);
    const int p1 = (int)(((int64_t)(lane + 1) * np) >> 6);
    if (p0 >= p1) return;

    // table offsets: rows of block b (reread when b changes), columns of one
    // half tile (2 columns) of block bp
    // (byte offsets from the table base, 32-bit: the table is below 4 GB)
    constexpr int H = ST_TILE / 2;
    const char* tb = reinterpret_cast<const char*>(tab);
    uint32_t ro[ST_TILE], co[H];
    int lrb = -1;
    auto offsets = [&](const TileWalk& w, int half) {
        if (w.b != lrb) {
            lrb = w.b;
#pragma unroll
            for (int r = 0; r < ST_TILE; ++r) ro[r] = (uint32_t)(rinf[w.b * ST_TILE + r] >> 1) * (uint32_t)sizeof(T);
        }
#pragma unroll
        for (int k = 0; k < H; ++k)
            co[k] = (uint32_t)(rinf[w.bp * ST_TILE + half * H + k] >> 1) * (uint32_t)(stride * (int)sizeof(T));
    };
    auto load = [&](T (&g)[H][ST_TILE]) {
#pragma unroll
        for (int k = 0; k < H; ++k)
#pragma unroll
            for (int r = 0; r < ST_TILE; ++r) g[k][r] = *reinterpret_cast<const T*>(tb + (co[k] + ro[r]));
    };

    TileWalk cw{nb, 0, 0};   // tile being contracted
    cw.start(p0);
    TileWalk lw = cw;        // tile whose first half is loaded ahead
    T gA[H][ST_TILE], gB[H][ST_TILE];
    offsets(lw, 0);
    load(gA);

    int cur = -1;
    T drow[ST_TILE][NV], erow[ST_TILE][NV];
    auto flush_rows = [&]() {
#pragma unroll
        for (int r = 0; r < ST_TILE; ++r)
#pragma unroll
            for (int v = 0; v < NV; ++v) IO::add_e(esh, cur * ST_TILE + r, v, erow[r][v]);
    };
    // columns half*H .. half*H + H - 1 of the current tile
    auto contract = [&](const T (&g)[H][ST_TILE], int half) {
        if (cw.b != cur) {
            if (cur >= 0) flush_rows();
            cur = cw.b;
#pragma unroll
            for (int r = 0; r < ST_TILE; ++r)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    drow[r][v] = dsh[st_idx<NV, SB>(cur * ST_TILE + r, v)];
                    erow[r][v] = V::zero();
                }
        }
        // diagonal tiles add their full 4 x 4 block through the rows only
        const double cscale = (cw.bp != cw.b) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const int s = cw.bp * ST_TILE + half * H + k;
            T dcol[NV], ecol[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                dcol[v] = dsh[st_idx<NV, SB>(s, v)];
                ecol[v] = V::zero();
            }
#pragma unroll
            for (int r = 0; r < ST_TILE; ++r)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    erow[r][v] = V::mad(g[k][r], dcol[v], erow[r][v]);
                    ecol[v] = V::cmad(g[k][r], drow[r][v], ecol[v]);
                }
#pragma unroll
            for (int v = 0; v < NV; ++v) IO::add_e(esh, s, v, V::scale(ecol[v], cscale));
        }
    };

    // one tile per trip: the second half is loaded while the first is
    // contracted, the next tile's first half while the second is; after the
    // lane's last tile the first half of that tile is reloaded (in range,
    // unused) so that every trip issues the same loads
    for (int p = p0; p < p1; ++p) {
        offsets(cw, 1);
        load(gB);
        contract(gA, 0);
        if (p + 1 < p1) lw.next();
        offsets(lw, 0);
        load(gA);
        contract(gB, 1);
        cw.next();
    }
    if (cur >= 0) flush_rows();
}

// sigma <- e_core * c (or 0), n elements; used before the accumulating sigma kernels.
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
