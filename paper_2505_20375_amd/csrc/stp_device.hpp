// Device-side helpers shared by the HIP kernels: scalar traits (real and
// complex FP64) and the string / move machinery of the categorical space.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "stp_internal.hpp"

namespace stp {

struct alignas(16) cd {
    double x, y;
};

template <bool CPLX>
struct VT;
template <>
struct VT<false> {
    using T = double;
    static __device__ __forceinline__ T zero() { return 0.0; }
    static __device__ __forceinline__ T mad(T a, T b, T c) { return fma(a, b, c); }
    static __device__ __forceinline__ T scale(T a, double s) { return a * s; }
    static __device__ __forceinline__ T add(T a, T b) { return a + b; }
    static __device__ __forceinline__ T sub(T a, T b) { return a - b; }
    static __device__ __forceinline__ T conjmul(T a, T b) { return a * b; }
    // conj(a) * b + c
    static __device__ __forceinline__ T cmad(T a, T b, T c) { return fma(a, b, c); }
    static __device__ __forceinline__ void atomic_add(T* p, T v) { unsafeAtomicAdd(p, v); }
    static __device__ __forceinline__ void lds_add(T* p, T v) { atomicAdd(p, v); }
    static __device__ __forceinline__ double re(T a) { return a; }
    static __device__ __forceinline__ double abs2(T a) { return a * a; }
    static __device__ __forceinline__ T shfl_xor(T a, int m) { return __shfl_xor(a, m, 64); }
};
template <>
struct VT<true> {
    using T = cd;
    static __device__ __forceinline__ T zero() { return cd{0.0, 0.0}; }
    static __device__ __forceinline__ T mad(T a, T b, T c) {
        c.x = fma(a.x, b.x, c.x);
        c.x = fma(-a.y, b.y, c.x);
        c.y = fma(a.x, b.y, c.y);
        c.y = fma(a.y, b.x, c.y);
        return c;
    }
    static __device__ __forceinline__ T scale(T a, double s) { return cd{a.x * s, a.y * s}; }
    static __device__ __forceinline__ T add(T a, T b) { return cd{a.x + b.x, a.y + b.y}; }
    static __device__ __forceinline__ T sub(T a, T b) { return cd{a.x - b.x, a.y - b.y}; }
    // conj(a) * b
    static __device__ __forceinline__ T conjmul(T a, T b) {
        return cd{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
    }
    static __device__ __forceinline__ T cmad(T a, T b, T c) {
        c.x = fma(a.x, b.x, c.x);
        c.x = fma(a.y, b.y, c.x);
        c.y = fma(a.x, b.y, c.y);
        c.y = fma(-a.y, b.x, c.y);
        return c;
    }
    static __device__ __forceinline__ void atomic_add(T* p, T v) {
        unsafeAtomicAdd(&p->x, v.x);
        unsafeAtomicAdd(&p->y, v.y);
    }
    static __device__ __forceinline__ void lds_add(T* p, T v) {
        atomicAdd(&p->x, v.x);
        atomicAdd(&p->y, v.y);
    }
    static __device__ __forceinline__ double re(T a) { return a.x; }
    static __device__ __forceinline__ double abs2(T a) { return a.x * a.x + a.y * a.y; }
    static __device__ __forceinline__ T shfl_xor(T a, int m) { return cd{__shfl_xor(a.x, m, 64), __shfl_xor(a.y, m, 64)}; }
};

struct alignas(8) cf {
    float x, y;
};

// Compute-precision traits of the sigma contraction: T is the arithmetic type
// of the integrals, gathered coefficients and partial sums; T64 the storage
// type of the CI vectors (always FP64).
template <bool CPLX, bool F32>
struct PT;
template <bool CPLX>
struct PT<CPLX, false> : VT<CPLX> {
    using T64 = typename VT<CPLX>::T;
    static __device__ __forceinline__ typename VT<CPLX>::T from64(T64 a) { return a; }
    static __device__ __forceinline__ T64 to64(typename VT<CPLX>::T a) { return a; }
};
template <>
struct PT<false, true> {
    using T = float;
    using T64 = double;
    static __device__ __forceinline__ T zero() { return 0.0f; }
    static __device__ __forceinline__ T mad(T a, T b, T c) { return fmaf(a, b, c); }
    static __device__ __forceinline__ T cmad(T a, T b, T c) { return fmaf(a, b, c); }
    static __device__ __forceinline__ T scale(T a, double s) { return a * (float)s; }
    static __device__ __forceinline__ void lds_add(T* p, T v) { atomicAdd(p, v); }
    static __device__ __forceinline__ T from64(T64 a) { return (float)a; }
    static __device__ __forceinline__ T64 to64(T a) { return (double)a; }
};
template <>
struct PT<true, true> {
    using T = cf;
    using T64 = cd;
    static __device__ __forceinline__ T zero() { return cf{0.0f, 0.0f}; }
    static __device__ __forceinline__ T mad(T a, T b, T c) {
        c.x = fmaf(a.x, b.x, c.x);
        c.x = fmaf(-a.y, b.y, c.x);
        c.y = fmaf(a.x, b.y, c.y);
        c.y = fmaf(a.y, b.x, c.y);
        return c;
    }
    static __device__ __forceinline__ T cmad(T a, T b, T c) {
        c.x = fmaf(a.x, b.x, c.x);
        c.x = fmaf(a.y, b.y, c.x);
        c.y = fmaf(a.x, b.y, c.y);
        c.y = fmaf(-a.y, b.x, c.y);
        return c;
    }
    static __device__ __forceinline__ T scale(T a, double s) { return cf{a.x * (float)s, a.y * (float)s}; }
    static __device__ __forceinline__ void lds_add(T* p, T v) {
        atomicAdd(&p->x, v.x);
        atomicAdd(&p->y, v.y);
    }
    static __device__ __forceinline__ T from64(T64 a) { return cf{(float)a.x, (float)a.y}; }
    static __device__ __forceinline__ T64 to64(T a) { return cd{(double)a.x, (double)a.y}; }
};

// ---------------------------------------------------------------------------
// string / move machinery
// ---------------------------------------------------------------------------
struct Det {
    int64_t r[KMAX];   // local ranks
    uint32_t s[KMAX];  // local occupation masks
};
static_assert(sizeof(Det) == DET_BYTES, "decoded determinant size");

__host__ __device__ __forceinline__ void decode(const DevSpace& S, const Cat& C, int64_t j, Det& d) {
    const int K = S.sp.K;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        if (k < K) {
            int64_t r = (j / C.stride[k]) % C.count[k];
            d.r[k] = r;
            d.s[k] = S.bits[S.tabs[C.tab[k]].bits_off + r];
        }
    }
}

__host__ __device__ __forceinline__ int nth_set(uint32_t v, int i) {
    for (int t = 0; t < i; ++t) v &= v - 1u;
    return __builtin_ctz(v);
}

__host__ __device__ __forceinline__ uint32_t lowmask(int m) { return (m >= 32) ? 0xffffffffu : ((1u << m) - 1u); }
__host__ __device__ __forceinline__ int popc32(uint32_t v) { return __builtin_popcount(v); }
__host__ __device__ __forceinline__ int popc64(uint64_t v) { return __builtin_popcountll(v); }

// Apply the move of class `cls` (local orbitals lx in xs, ly in ys) to d.
// Returns the vector address of the target and its sign.
__host__ __device__ __forceinline__ int64_t apply_move(const DevSpace& S, const Cat& C, int cls, int xs, int ys, int lx,
                                              int ly, const Det& d, int& sign) {
    const int K = S.sp.K;
    const Cat& T = S.cats[C.cls_target[cls]];
    int sg = 1;
    int64_t rx = d.r[xs], ry = d.r[ys];
    if (xs == ys) {
        if (lx != ly) {
            const StrTab& t0 = S.tabs[C.tab[ys]];
            int32_t a = S.ann[t0.ann_off + d.r[ys] * t0.m + ly];
            int64_t r1 = (a < 0 ? -a : a) - 1;
            if (a < 0) sg = -sg;
            const StrTab& t1 = S.tabs[t0.tab_dn];
            int32_t b = S.cre[t1.cre_off + r1 * t1.m + lx];
            rx = (b < 0 ? -b : b) - 1;
            if (b < 0) sg = -sg;
            ry = rx;
        }
    } else {
        const StrTab& ty = S.tabs[C.tab[ys]];
        int32_t a = S.ann[ty.ann_off + d.r[ys] * ty.m + ly];
        ry = (a < 0 ? -a : a) - 1;
        if (a < 0) sg = -sg;
        const StrTab& tx = S.tabs[C.tab[xs]];
        int32_t b = S.cre[tx.cre_off + d.r[xs] * tx.m + lx];
        rx = (b < 0 ? -b : b) - 1;
        if (b < 0) sg = -sg;
        if (C.cls_phase[cls]) sg = -sg;
    }
    int64_t addr = T.offset;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        if (k < K) {
            int64_t r = (k == xs) ? rx : ((k == ys) ? ry : d.r[k]);
            addr += r * T.stride[k];
        }
    }
    sign = sg;
    return addr;
}

// Move of slot `slot` of category C for determinant d.
__host__ __device__ __forceinline__ void slot_move(const DevSpace& S, const Cat& C, const Det& d, int slot, int& cls,
                                          int& xs, int& ys, int& lx, int& ly) {
    const int K = S.sp.K;
    int c = 0;
    while (C.cls_begin[c + 1] <= slot) ++c;
    cls = c;
    int code = C.cls_code[c];
    xs = code / K;
    ys = code - xs * K;
    int t = slot - C.cls_begin[c];
    int w = C.cls_width[c];
    int i = t / w, jx = t - i * w;
    ly = nth_set(d.s[ys], i);
    int mx = S.sp.sub_m[xs];
    int nvirt = mx - C.occ[xs];
    lx = (jx < nvirt) ? nth_set(~d.s[xs] & lowmask(mx), jx) : ly;
}

__host__ __device__ __forceinline__ int find_segment(const int64_t* begin, int n, int64_t x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Sum over the 64 lanes of a wavefront (every lane gets the result).
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
template <bool CPLX>
__device__ __forceinline__ typename VT<CPLX>::T wave_sum(typename VT<CPLX>::T v);
template <>
__device__ __forceinline__ double wave_sum<false>(double v) { return wave_sum_d(v); }
template <>
__device__ __forceinline__ cd wave_sum<true>(cd v) { return cd{wave_sum_d(v.x), wave_sum_d(v.y)}; }

// Make the LDS writes of all lanes of this wavefront visible to all its lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace stp
