// Fused sigma build, one wavefront per intermediate determinant, Hermitian
// 4x4 tiles (the kernel the library uses by default).
//
// For an intermediate determinant J with moves m = (x created, y annihilated)
// into the space (Eq. sigmaL2e resolved over J):
//   d[m]       = sign(m) C[target(m)]
//   G_J[m', m] = (x' y' | y x)            Hermitian in (m', m)
//   e          = G_J d,   sigma[target(m')] += 1/2 sign(m') e[m'].
// When J lies in the space the same d also yields the one-electron term of
// Eq. sigmaL1e for L = J: sigma_J += sum_m h'_{y x} d[m].
//
// The moves of J are cut into blocks of 4 consecutive slots; the upper
// triangle of 4x4 block pairs (b <= b') is split evenly over the 64 lanes.
// A lane loads one 16-element tile of G_J (rows: 4 consecutive x' of one
// annihilated orbital, so each column's 4 elements are adjacent in memory)
// and uses every element for both vectors and, off the diagonal, twice:
//   e[rows b]  += G[b, b'] d[b']          (kept in registers while b repeats)
//   e[cols b'] += G[b, b']^H d[b]         (added to LDS with FP64 atomics).
// Each integral element feeds 4 complex multiply-adds per vector pair, the
// LDS traffic for d is one 4-vector per tile side, and all partial sums meet
// in the wavefront's LDS slice before one atomic update of sigma per move.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"
#include "stp_device.hpp"
#include "symtile.hpp"

namespace stp {

// LDS layout of one wavefront's slice: d (contraction type), e (FP64),
// targets, row move indices.
__host__ __device__ inline SliceLayout symtile_layout(int deg_max, int nv, bool cplx, bool f32) {
    const int se = cplx ? 16 : 8;
    return SliceLayout(deg_max, nv, f32 ? se / 2 : se, se, 0);
}

// Sigma contribution of one intermediate determinant J (index over the
// work categories of S), computed by one wavefront with its LDS slice.
template <bool CPLX, bool F32, int NV>
__device__ __forceinline__ void symtile_det(const DevSpace& S, const typename PT<CPLX, F32>::T* __restrict__ gT,
                                            const typename PT<CPLX, F32>::T* __restrict__ hp,
                                            const typename VT<CPLX>::T* __restrict__ c,
                                            typename VT<CPLX>::T* __restrict__ sigma, int n_vec, int deg_cap,
                                            unsigned char* base, int lane, int64_t J) {
    using V = PT<CPLX, F32>;     // contraction arithmetic
    using V64 = VT<CPLX>;        // vector storage and sigma accumulation
    using T = typename V::T;
    using TE = typename V64::T;
    constexpr int SB = sizeof(T);
    constexpr int SE = sizeof(TE);
    const SliceLayout L(deg_cap, NV, SB, SE, 0);
    T* dsh = reinterpret_cast<T*>(base + L.d_off);                 // padded [slot][NV]
    TE* esh = reinterpret_cast<TE*>(base + L.e_off);               // padded [slot][NV], FP64
    int64_t* tgt = reinterpret_cast<int64_t*>(base + L.tgt_off);   // target address
    int32_t* rinf = reinterpret_cast<int32_t*>(base + L.i0_off);   // pair(m) << 1 | negative sign
    const int M = S.sp.M;
    const int MM = M * M;
    const int64_t nd = S.sp.ndets;
    const int w = find_segment(S.work_begin, S.sp.nwork, J);
    const Cat& C = S.cats[S.work_cat[w]];
    const int64_t jloc = J - S.work_begin[w];
    Det dt;
    decode(S, C, jloc, dt);
    const int deg = C.deg;

    // ---- phase 1: moves, gathers, one-electron term
    T one[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) one[v] = V::zero();
    for (int slot = lane; slot < ((deg + 3) & ~3); slot += 64) {
        if (slot >= deg) {  // padding slots of the last block: d = e = 0, in-range indices
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                dsh[st_idx<NV, SB>(slot, v)] = V::zero();
                esh[st_idx<NV, SE>(slot, v)] = V64::zero();
            }
            rinf[slot] = 0;
            continue;
        }
        int cls, xs, ys, lx, ly, sg;
        slot_move(S, C, dt, slot, cls, xs, ys, lx, ly);
        const int64_t t = apply_move(S, C, cls, xs, ys, lx, ly, dt, sg);
        const int x = S.sp.sub_off[xs] + lx, y = S.sp.sub_off[ys] + ly;
        const int pair = y * M + x;
        tgt[slot] = t;
        rinf[slot] = (pair << 1) | (sg < 0 ? 1 : 0);
        const T hv = hp[y * M + x];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T val = (v < n_vec) ? V::from64(c[(int64_t)v * nd + t]) : V::zero();
            if (sg < 0) val = V::scale(val, -1.0);
            dsh[st_idx<NV, SB>(slot, v)] = val;
            esh[st_idx<NV, SE>(slot, v)] = V64::zero();
            one[v] = V::mad(hv, val, one[v]);
        }
    }
    if (C.in_space) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const typename V64::T s = wave_sum<CPLX>(V::to64(one[v]));
            if (lane == 0 && v < n_vec) V64::atomic_add(&sigma[(int64_t)v * nd + C.offset + jloc], s);
        }
    }
    wave_lds_sync();

    // ---- phase 2: e = G_J d over the upper-triangle tiles
    tile_contract<CPLX, F32, NV>(gT, MM, dsh, esh, rinf, deg, lane);
    wave_lds_sync();

    // ---- phase 3: one atomic update of sigma per move and vector
    for (int slot = lane; slot < deg; slot += 64) {
        const double s = (rinf[slot] & 1) ? -0.5 : 0.5;
        const int64_t t = tgt[slot];
#pragma unroll
        for (int v = 0; v < NV; ++v)
            if (v < n_vec)
                V64::atomic_add(&sigma[(int64_t)v * nd + t], V64::scale(esh[st_idx<NV, SE>(slot, v)], s));
    }
    wave_lds_sync();  // the next determinant reuses this wavefront's LDS slice
}

template <bool CPLX, bool F32, int NV>
__global__ __launch_bounds__(256) void k_sigma_symtile(DevSpace S, const typename PT<CPLX, F32>::T* __restrict__ gT,
                                                      const typename PT<CPLX, F32>::T* __restrict__ hp,
                                                      const typename VT<CPLX>::T* __restrict__ c,
                                                      typename VT<CPLX>::T* __restrict__ sigma, int n_vec,
                                                      int deg_cap) {
    using T = typename PT<CPLX, F32>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    unsigned char* base = smem + (size_t)wid * symtile_layout(deg_cap, NV, CPLX, F32).bytes;
    const int64_t total = S.sp.nwork_dets;
    const int64_t nw = (int64_t)gridDim.x * wpb;
    for (int64_t J = (int64_t)blockIdx.x * wpb + wid; J < total; J += nw)
        symtile_det<CPLX, F32, NV>(S, gT, hp, c, sigma, n_vec, deg_cap, base, lane, J);
}

template <bool CPLX>
__global__ __launch_bounds__(256) void k_fill_init(typename VT<CPLX>::T* __restrict__ sigma,
                                                  const typename VT<CPLX>::T* __restrict__ c, double e_core,
                                                  int64_t n) {
    fill_init<CPLX>(sigma, c, e_core, n, blockIdx.x * (int64_t)blockDim.x + threadIdx.x,
                    (int64_t)gridDim.x * blockDim.x);
}

hipError_t launch_fill_init(bool cplx, void* sigma, const void* c, double e_core, int64_t n, hipStream_t st) {
    const int zg = (int)std::max<int64_t>(1, std::min<int64_t>(8192, (n + 255) / 256));
    if (cplx)
        hipLaunchKernelGGL(k_fill_init<true>, dim3(zg), dim3(256), 0, st, (cd*)sigma, (const cd*)c, e_core, n);
    else
        hipLaunchKernelGGL(k_fill_init<false>, dim3(zg), dim3(256), 0, st, (double*)sigma, (const double*)c, e_core,
                           n);
    return hipGetLastError();
}

size_t symtile_slice_bytes(int deg_max, int nv, bool cplx, bool f32) {
    return symtile_layout(deg_max, nv, cplx, f32).bytes;
}

bool symtile_supported(int deg_max, bool cplx) { return symtile_slice_bytes(deg_max, 2, cplx, false) <= 64 * 1024; }

// Waves per workgroup for a per-wave LDS slice: at most 4 and 48 KB per group.
int waves_per_group(size_t per_wave) {
    int wpb = 4;
    while (wpb > 1 && per_wave * wpb > 48 * 1024) wpb >>= 1;
    return wpb;
}

template <bool CPLX, bool F32, int NV>
static hipError_t launch_sym_nv(const DevSpace& S, int deg_max, const void* gT, const void* hp, const void* c,
                                void* sigma, int nv, hipStream_t st) {
    using T = typename PT<CPLX, F32>::T;
    using T64 = typename VT<CPLX>::T;
    const size_t per_wave = symtile_slice_bytes(deg_max, NV, CPLX, F32);
    const int wpb = waves_per_group(per_wave);
    const size_t lds = per_wave * wpb;
    int64_t blocks = (S.sp.nwork_dets + wpb - 1) / wpb;
    blocks = std::max<int64_t>(1, std::min<int64_t>(blocks, 256 * 64));
    hipLaunchKernelGGL((k_sigma_symtile<CPLX, F32, NV>), dim3((unsigned)blocks), dim3(64 * wpb), lds, st, S,
                       (const T*)gT, (const T*)hp, (const T64*)c, (T64*)sigma, nv, deg_max);
    return hipGetLastError();
}

template <bool CPLX, bool F32>
static hipError_t launch_sym_all(const DevSpace& S, int deg_max, const void* gT, const void* hp, const void* c,
                                 void* sigma, int n_vec, double e_core, hipStream_t st) {
    using T64 = typename VT<CPLX>::T;
    hipError_t e = launch_fill_init(CPLX, sigma, c, e_core, S.sp.ndets * n_vec, st);
    if (e != hipSuccess) return e;
    for (int v0 = 0; v0 < n_vec; v0 += 2) {
        const int nv = (n_vec - v0 >= 2) ? 2 : 1;
        const int64_t off = (int64_t)v0 * S.sp.ndets;
        const T64* cc = (const T64*)c + off;
        T64* ss = (T64*)sigma + off;
        e = (nv == 2) ? launch_sym_nv<CPLX, F32, 2>(S, deg_max, gT, hp, cc, ss, 2, st)
                      : launch_sym_nv<CPLX, F32, 1>(S, deg_max, gT, hp, cc, ss, 1, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_sigma_symtile(const DevSpace& S, int deg_max, bool cplx, bool f32, const void* gT, const void* hp,
                                const void* c, void* sigma, int n_vec, double e_core, hipStream_t st) {
    if (cplx)
        return f32 ? launch_sym_all<true, true>(S, deg_max, gT, hp, c, sigma, n_vec, e_core, st)
                   : launch_sym_all<true, false>(S, deg_max, gT, hp, c, sigma, n_vec, e_core, st);
    return f32 ? launch_sym_all<false, true>(S, deg_max, gT, hp, c, sigma, n_vec, e_core, st)
               : launch_sym_all<false, false>(S, deg_max, gT, hp, c, sigma, n_vec, e_core, st);
}

}  // namespace stp
