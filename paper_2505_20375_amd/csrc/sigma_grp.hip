// Grouped matrix-core form of the pair-resolved sigma build, for spaces of
// one subspace (every determinant of N electrons in M spin-orbitals).
//
// There every (N-2)-electron intermediate K' couples to all pairs of its empty
// orbitals, and its pair-pair block A_K' is A restricted to those pairs.  The
// intermediates K'_u = K'' + o_u that share a core K'' (N-3 electrons) have
// blocks inside one block A_K'' over the pairs of the core's empty orbitals
// (the pairs of K'_u are the core pairs without o_u).  One workgroup of four
// wavefronts takes an item of U such intermediates (U = 8, or 4 where the
// slice of 8 would not fit): the core pairs index the rows and columns of
// A_K'', intermediate u owns CW consecutive columns of the right-hand side B,
//   complex: [Re d_0, Re d_1, Im d_0, Im d_1] (one vector: [Re d, Im d]), real: [d_0, d_1] (one vector: [d]),
// at each core pair (0 where the pair holds o_u), the row of B padded to whole
// 16-column groups, and each 16 x 4 piece of A_K'' read from the table feeds
// one v_mfma_f64_16x16x4f64 per column group and real or imaginary part of
// the table.  With two complex vectors that is 32 right-hand columns per table
// read (4 in the one-intermediate kernel), at 80 % useful entries for 24
// spin-orbitals and 8 electrons (the core has one more empty orbital).  Lane
// layouts (checked on the device with in-bounds probes): A lane l holds row
// l % 16, step l / 16; B lane l holds step l / 16, column l % 16; output
// register i of lane l holds row l / 16 + 4 i, column l % 16 (FP64) or row
// 4 (l / 16) + i (v_mfma_f32_16x16x4f32 of the FP32 form).  The complex
// combination and the scatter of each intermediate's rows follow the
// one-intermediate kernel.
//
// The slot arithmetic is plain bit arithmetic here: the target K'_u + {p, r}
// is addressed by its colex rank (binomial table in LDS), the sign of
// a+_p a+_r |K'_u> counts the electrons of K'_u below r and below p, so each
// core pair costs one gather of c and no table chains.
//
// Items come from the host: cores in colex order take their intermediates
// not yet placed U at a time; the rest go by the core without their lowest
// electron.  Each intermediate is in exactly one item.  Each XCD works through
// a contiguous eighth of the items.  For 24 spin-orbitals the FP64 slice of
// eight is 52 KB of LDS: three workgroups share a compute unit, and launch
// bounds of three let the accumulators live in VGPRs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cstdint>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"
#include "space.hpp"
#include "stp_device.hpp"

namespace stp {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// One 16 x 16 x 4 matrix-core step, FP64 or FP32 (FP32 accumulation).
__device__ __forceinline__ f64x4 grp_mfma(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 grp_mfma(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}


// Workgroup slice: core pairs (global pair index; p | r << 8), B as
// [row][16] doubles, targets [intermediate][row] (target << 1 | sign, -1:
// none), binomial coefficients C(n, k) (n < M, k <= N; row stride N + 1) for
// colex ranks, flags.
struct GrpLayout {
    size_t rinf_off, prs_off, b_off, tgt_off, bin_off, flag_off, bytes;
    __host__ __device__ GrpLayout(int cap, int M, int N, int bsz, int U, int bw) {
        rinf_off = 0;
        prs_off = (size_t)cap * 4;
        b_off = (prs_off + (size_t)cap * 4 + 15) & ~(size_t)15;
        tgt_off = b_off + (size_t)cap * bw * bsz;
        bin_off = tgt_off + (size_t)U * cap * 4;
        flag_off = (bin_off + (size_t)M * (N + 1) * 4 + 15) & ~(size_t)15;
        bytes = flag_off + 16;
    }
};

static int grp_core_pairs(const Space& sp) {
    const int e = sp.M - (sp.N - 3);   // empty orbitals of a core
    return e * (e - 1) / 2;
}

static int grp_cap(const Space& sp) { return (grp_core_pairs(sp) + 15) & ~15; }

// Intermediates per item: 8 where the FP64 workgroup slice fits 54 KB of LDS
// (three workgroups per compute unit; each table read feeds 32 right-hand
// columns), else 4 within 64 KB; 0: unsupported.
int pair_grp_unit(const Space& sp) {
    if (!(sp.K == 1 && sp.N >= 3 && sp.M <= 32 && sp.npcat == 1)) return 0;
    if (GrpLayout(grp_cap(sp), sp.M, sp.N, 8, 8, 32).bytes <= 54 * 1024) return 8;
    if (GrpLayout(grp_cap(sp), sp.M, sp.N, 8, 4, 16).bytes <= 64 * 1024) return 4;
    return 0;
}

bool pair_grp_supported(const Space& sp) { return pair_grp_unit(sp) > 0; }

// Items of the grouped kernel (see the file comment); false when the space is
// not one subspace or too large for the host pass.
bool build_pair_groups(const HostSpace& H, std::vector<GrpItem>& items) {
    items.clear();
    const Space& sp = H.sp;
    const int U = pair_grp_unit(sp);
    if (U == 0) return false;
    const PairCat& P = H.pcats[0];
    const int64_t cnt = P.count[0];
    const int M = sp.M, nc = sp.N - 3;
    double ncores = 1.0;
    for (int i = 0; i < nc; ++i) ncores = ncores * (M - i) / (i + 1);
    if (cnt <= 0 || cnt > (1 << 24) || ncores > (double)(1 << 24)) return false;
    const StrTab& T = H.tabs[P.tab[0]];
    std::unordered_map<uint32_t, int32_t> rank;
    rank.reserve((size_t)cnt * 2);
    for (int64_t r = 0; r < cnt; ++r) rank.emplace(H.bits[T.bits_off + r], (int32_t)r);
    std::vector<char> placed((size_t)cnt, 0);
    int64_t n_placed = 0;
    auto emit = [&](uint32_t core, const int32_t* j, int n) {
        GrpItem it{};
        it.core = core;
        it.n = n;
        for (int u = 0; u < GRP_U; ++u) it.j[u] = u < n ? j[u] : -1;
        items.push_back(it);
        n_placed += n;
    };
    // cores in colex order (next subset of the same size)
    const uint64_t lim = 1ull << M;
    uint64_t x = (1ull << nc) - 1;
    while (x < lim) {
        const uint32_t core = (uint32_t)x;
        int32_t mem[32];
        int n = 0;
        for (int o = 0; o < M; ++o) {
            if ((core >> o) & 1u) continue;
            const auto f = rank.find(core | (1u << o));
            if (f == rank.end() || placed[f->second]) continue;
            mem[n++] = f->second;
        }
        for (int a = 0; a + U <= n; a += U) {
            for (int u = 0; u < U; ++u) placed[mem[a + u]] = 1;
            emit(core, mem + a, U);
        }
        if (nc == 0) break;
        const uint64_t cbit = x & (~x + 1), r = x + cbit;
        x = (((r ^ x) >> 2) / cbit) | r;
    }
    // the rest: by the core without the lowest electron
    std::unordered_map<uint32_t, std::vector<int32_t>> rest;
    for (int64_t r = 0; r < cnt; ++r)
        if (!placed[r]) {
            const uint32_t s = H.bits[T.bits_off + r];
            rest[s & (s - 1)].push_back((int32_t)r);
        }
    for (auto& kv : rest)
        for (size_t a = 0; a < kv.second.size(); a += U)
            emit(kv.first, kv.second.data() + a, (int)std::min<size_t>(U, kv.second.size() - a));
    return n_placed == cnt;
}

size_t pair_grp_slice_bytes(const Space& sp) {
    const int U = pair_grp_unit(sp);
    return GrpLayout(grp_cap(sp), sp.M, sp.N, 8, U, 4 * U).bytes;
}

// Right-hand columns per intermediate: complex [Re d_0, Re d_1, Im d_0, Im d_1]
// (one vector: [Re d, Im d]), real [d_0, d_1] (one vector: [d]); the row of B
// is padded to whole 16-column groups.
__host__ __device__ constexpr int grp_cw(bool cplx, int nv) { return cplx ? 2 * nv : nv; }
__host__ __device__ constexpr int grp_bw(bool cplx, int nv, int U) { return (U * grp_cw(cplx, nv) + 15) / 16 * 16; }

// Value of x in lane (lane ^ X) of the same quad, X = 1 or 2 (DPP quad permutation).
template <int X>
__device__ __forceinline__ double grp_quad_xor(double x) {
    constexpr int ctrl = (X == 2) ? 0x4E : 0xB1;   // quad_perm [2,3,0,1] or [1,0,3,2]
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Position of the k-th set bit of m (k < popcount(m)).
__device__ __forceinline__ int grp_nth_bit(uint64_t m, int k) {
    for (int i = 0; i < k; ++i) m &= m - 1;
    return __ffsll((unsigned long long)m) - 1;
}

// F32: table, right-hand side and accumulation in FP32, sums of the
// contributions in FP64 as in the FP64 form.
template <bool CPLX, bool F32, int NV, bool STORE, int U>
__global__ __launch_bounds__(256, 3) void k_sigma_pair_grp(DevSpace S, const GrpItem* __restrict__ items, int nitems,
                                                       const typename PT<CPLX, F32>::T* __restrict__ A,
                                                       const typename VT<CPLX>::T* __restrict__ c,
                                                       typename VT<CPLX>::T* __restrict__ sigma,
                                                       typename VT<CPLX>::T* __restrict__ E, int nq, int n_vec,
                                                       int cap) {
    using V64 = VT<CPLX>;
    using TE = typename V64::T;                        // coefficients (FP64)
    using TA = typename PT<CPLX, F32>::T;              // table entries
    using BT = typename std::conditional<F32, float, double>::type;
    using ACC = typename std::conditional<F32, f32x4, f64x4>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int CW = grp_cw(CPLX, NV);   // right-hand columns per intermediate
    constexpr int BW = grp_bw(CPLX, NV, U);   // B row width
    constexpr int NG = BW / 16;            // 16-column groups of the right-hand side
    // core pairs per lane taken together in phase 1 (FP64: as many as the
    // registers of the products allow at no cost in occupancy)
    constexpr int PB = F32 ? 2 : 4;
    const GrpLayout L(cap, S.sp.M, S.sp.N, (int)sizeof(BT), U, BW);
    const int BN = S.sp.N + 1;   // row stride of the binomial table
    int32_t* rinf = reinterpret_cast<int32_t*>(smem + L.rinf_off);
    BT* bsh = reinterpret_cast<BT*>(smem + L.b_off);
    int32_t* tgt = reinterpret_cast<int32_t*>(smem + L.tgt_off);   // target << 1 | sign (below 2^31)
    int32_t* prs = reinterpret_cast<int32_t*>(smem + L.prs_off);
    int32_t* binom = reinterpret_cast<int32_t*>(smem + L.bin_off);
    int* flags = reinterpret_cast<int*>(smem + L.flag_off);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const PairCat& P = S.pcats[0];
    const int M = S.sp.M, NP = S.sp.npairs;
    const int64_t kbits_off = S.tabs[P.tab[0]].bits_off;   // strings of K' by rank
    const int64_t base = S.cats[P.cls_target[0]].offset;    // address of colex rank 0
    const int ncp = (M - S.sp.N + 3) * (M - S.sp.N + 2) / 2;   // core pairs
    const int64_t nd = S.sp.ndets;
    const uint64_t full = (M == 64) ? ~0ull : ((1ull << M) - 1ull);
    const int nT = cap >> 4, nks = cap >> 2;
    const int kq = lane >> 4;     // A and B lanes: step within the 4-column group
    const int c16 = lane & 15;    // A lanes: row; B and output lanes: column
    const int col = c16 % CW;     // column within the intermediate's CW
    int v, comp;
    if constexpr (CPLX) {
        v = (NV == 2) ? (col & 1) : 0;
        comp = (NV == 2) ? (col >> 1) : col;
    } else {
        v = col;
        comp = 0;
    }
    // lane's value of the complex product from C1 = Re(A) B and C2 = Im(A) B
    // (the partner column, Im for Re and Re for Im, is lane ^ 2 or lane ^ 1)
    auto combine = [&](double c1, double c2) -> double {
        if constexpr (CPLX) {
            const double p = grp_quad_xor<NV == 2 ? 2 : 1>(c2);
            return (col < NV) ? c1 - p : c1 + p;
        } else {
            (void)c2;
            return c1;
        }
    };

    for (int t = threadIdx.x; t < S.sp.M * BN; t += blockDim.x) {
        const int nn = t / BN, kk = t % BN;
        int64_t b = (kk <= nn) ? 1 : 0;
        for (int i = 1; i <= kk && kk <= nn; ++i) b = b * (nn - kk + i) / i;
        binom[t] = (int32_t)b;
    }
    // padding columns of B (past U CW) are written by no item: zero them once
    if constexpr (BW > U * CW) {
        constexpr int PW = BW - U * CW;
        for (int t = threadIdx.x; t < cap * PW; t += blockDim.x) bsh[(t / PW) * BW + U * CW + t % PW] = (BT)0;
    }
    __syncthreads();
    // XCD-aware item order: workgroups are dealt round-robin to the 8 XCDs, so
    // workgroup b runs on XCD b % 8; each XCD takes one contiguous eighth of
    // the items (neighbouring cores, whose targets share most occupied
    // orbitals and hence nearby addresses), so that its L2 holds the
    // coefficients it gathers and the workspace lines it writes.
    const int xcd = blockIdx.x & 7, nloc = gridDim.x >> 3;
    const int chunk = (nitems + 7) >> 3;
    const int it_end = min(nitems, (xcd + 1) * chunk);
    int turn = (int)(blockIdx.x >> 3);   // rotation of the row tiles over the wavefronts
    for (int it = xcd * chunk + (int)(blockIdx.x >> 3); it < it_end; it += nloc, ++turn) {
        const uint32_t core = items[it].core;
        const int n = items[it].n;
        const uint64_t emp = ~(uint64_t)core & full;
        // ---- phase 1: core pairs (all threads), then per wavefront its
        // intermediates K'_u = core + o: B columns and target of every core
        // pair {p, r} (zero and none where the pair holds o).  The target
        // K'_u + {p, r} is addressed by its colex rank, a+_p a+_r |K'_u> has
        // the sign of the electrons of K'_u below r and below p, and q is the
        // position of {p, r} among the target's occupied pairs.
        for (int l = threadIdx.x; l < cap; l += blockDim.x) {
            int pi = 0, pr = 0;
            if (l < ncp) {
                int t = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)l)) * 0.5f);   // C(t,2) <= l < C(t+1,2)
                while (t * (t - 1) / 2 > l) --t;
                while ((t + 1) * t / 2 <= l) ++t;
                const int r = grp_nth_bit(emp, t), p = grp_nth_bit(emp, l - t * (t - 1) / 2);
                pi = r * (r - 1) / 2 + p;
                pr = p | (r << 8);
            }
            rinf[l] = pi;
            prs[l] = pr;
        }
        __syncthreads();
        bool nz = false;
        for (int u = wid; u < U; u += 4) {   // this wavefront's intermediates of the item
            const bool have = u < n;
            const uint32_t kb = have ? S.bits[kbits_off + items[it].j[u]] : 0u;
            const int o = have ? __builtin_ctz(kb & ~core) : -1;
            for (int l0 = 0; l0 < cap; l0 += 64 * PB) {
                int64_t addr[PB];
                int qq[PB];
                bool ok[PB], ng[PB];
#pragma unroll
                for (int i = 0; i < PB; ++i) {
                    const int l = l0 + 64 * i + lane;
                    const int pr = (l < cap) ? prs[l] : 0;
                    const int p = pr & 255, r = pr >> 8;
                    ok[i] = have && l < ncp && p != o && r != o;
                    const uint32_t T = kb | (1u << p) | (1u << r);
                    int64_t rk = 0;
                    uint32_t m = T;
                    for (int e = 1; m; ++e) {
                        rk += binom[__builtin_ctz(m) * BN + e];
                        m &= m - 1;
                    }
                    addr[i] = ok[i] ? base + rk : 0;
                    const uint32_t below_p = (1u << p) - 1u, below_r = (1u << r) - 1u;
                    ng[i] = ((__builtin_popcount(kb & below_r) + __builtin_popcount(kb & below_p)) & 1) != 0;
                    const int ip = __builtin_popcount(T & below_p), ir = __builtin_popcount(T & below_r);
                    qq[i] = ir * (ir - 1) / 2 + ip;
                }
                TE x[PB][NV];
#pragma unroll
                for (int i = 0; i < PB; ++i)
#pragma unroll
                    for (int vv = 0; vv < NV; ++vv) x[i][vv] = c[(int64_t)(vv < n_vec ? vv : 0) * nd + addr[i]];
#pragma unroll
                for (int i = 0; i < PB; ++i) {
                    const int l = l0 + 64 * i + lane;
                    if (l >= cap) break;
                    const double sg = ng[i] ? -1.0 : 1.0;
                    double bc[CW];
#pragma unroll
                    for (int j = 0; j < CW; ++j) bc[j] = 0.0;
                    if (ok[i]) {
#pragma unroll
                        for (int vv = 0; vv < NV; ++vv) {
                            if (vv >= n_vec) break;
                            nz = nz || V64::abs2(x[i][vv]) != 0.0;
                            if constexpr (CPLX) {
                                bc[vv] = sg * x[i][vv].x;
                                bc[NV + vv] = sg * x[i][vv].y;
                            } else {
                                bc[vv] = sg * x[i][vv];
                            }
                        }
                    }
#pragma unroll
                    for (int j = 0; j < CW; ++j) bsh[l * BW + CW * u + j] = (BT)bc[j];
                    const int64_t t = STORE ? addr[i] * nq + qq[i] : addr[i];
                    tgt[u * cap + l] = ok[i] ? (int32_t)((t << 1) | (ng[i] ? 1 : 0)) : -1;
                }
            }
        }
        const bool live = __ballot(nz) != 0;
        if (lane == 0) flags[wid] = live ? 1 : 0;
        __syncthreads();
        const bool any = (flags[0] | flags[1] | flags[2] | flags[3]) != 0;

        // ---- phases 2 and 3: 16-row tiles of A_K'' split over the wavefronts;
        // the first tile of a wavefront turns with the item, so that the short
        // shares (nT not a multiple of 4) fall on each SIMD in turn
        for (int R = (wid + turn) & 3; R < nT; R += 4) {
            // one accumulator per real product: consecutive steps alternate between
            // the two, which keeps a dependent pair two instructions apart
            ACC c1[NG], c2[NG];
#pragma unroll
            for (int h = 0; h < NG; ++h) c1[h] = c2[h] = ACC{0, 0, 0, 0};
            if (any) {
                const TA* arow = A + rinf[R * 16 + c16];   // this A lane's row pair
                constexpr int G = 2;    // steps per group
                constexpr int RG = 4;   // groups in flight
                const int ngrp = nks / G;
                TA ab[RG][G];
                auto ldgrp = [&](int g, TA (&a)[G]) {
#pragma unroll
                    for (int j = 0; j < G; ++j) a[j] = arow[(int64_t)rinf[((g * G + j) << 2) + kq] * NP];
                };
                // right-hand fragments of a group, read from LDS one group ahead
                // of their products (two buffers alternate; RG is even)
                BT bb[2][G][NG];
                auto ldb = [&](int g, BT (&b)[G][NG]) {
#pragma unroll
                    for (int j = 0; j < G; ++j)
#pragma unroll
                        for (int h = 0; h < NG; ++h) b[j][h] = bsh[(((g * G + j) << 2) + kq) * BW + c16 + 16 * h];
                };
                auto mfgrp = [&](const TA (&a)[G], const BT (&b)[G][NG]) {
#pragma unroll
                    for (int j = 0; j < G; ++j)
#pragma unroll
                        for (int h = 0; h < NG; ++h) {
                            if constexpr (CPLX) {
                                c1[h] = grp_mfma(a[j].x, b[j][h], c1[h]);
                                c2[h] = grp_mfma(a[j].y, b[j][h], c2[h]);
                            } else {
                                c1[h] = grp_mfma(a[j], b[j][h], c1[h]);
                            }
                        }
                };
                static_assert(RG % 2 == 0, "the two fragment buffers alternate over the ring");
                // the loads are unconditional (past the last group: the last group
                // again, in range, unused), so that every group keeps the same
                // number of reads in flight
#pragma unroll
                for (int u = 0; u < RG - 1; ++u) {
                    ldgrp(u < ngrp ? u : ngrp - 1, ab[u]);
                    __builtin_amdgcn_sched_barrier(0);   // requested in group order, as in the loop
                }
                ldb(0, bb[0]);
                // whole rounds of RG groups without conditions (so that every
                // read stays ahead of its use), then the last partial round
                const int nfull = ngrp - ngrp % RG;
                auto round = [&](int g, bool tail) {
#pragma unroll
                    for (int u = 0; u < RG; ++u) {
                        const int gl = g + u + RG - 1, gb = g + u + 1;
                        ldgrp(gl < ngrp ? gl : ngrp - 1, ab[(u + RG - 1) % RG]);
                        ldb(gb < ngrp ? gb : ngrp - 1, bb[(u + 1) & 1]);
                        if (!tail || g + u < ngrp) mfgrp(ab[u], bb[u & 1]);
                    }
                };
                for (int g = 0; g < nfull; g += RG) round(g, false);
                if (nfull < ngrp) round(nfull, true);
            }
            // output register i: row R * 16 + kq + 4 i (FP32: R * 16 + 4 kq + i),
            // column 16 h + c16 (intermediate (16 h + c16) / CW; padding columns
            // past U CW have none)
#pragma unroll
            for (int h = 0; h < NG; ++h) {
                const int u = (16 * h + c16) / CW;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const double val = combine((double)c1[h][i], (double)c2[h][i]);
                    const int l = R * 16 + (F32 ? 4 * kq + i : kq + 4 * i);
                    if (u < n && v < n_vec && (STORE || any)) {
                        const int32_t tw = tgt[u * cap + l];
                        if (tw >= 0) {
                            const double x = (tw & 1) ? -val : val;
                            const int64_t t = tw >> 1;
                            if (STORE)
                                reinterpret_cast<double*>(E + t * NV + v)[comp] = x;
                            else
                                unsafeAtomicAdd(reinterpret_cast<double*>(sigma + (int64_t)v * nd + t) + comp, x);
                        }
                    }
                }
            }
        }
        __syncthreads();   // the next item reuses the slice
    }
}

template <bool CPLX, bool F32, int NV, bool STORE>
static hipError_t launch_grp_nv(const DevSpace& S, const GrpItem* items, int nitems, const void* A, const void* c,
                                void* sigma, void* E, int nq, int nv, hipStream_t st) {
    using T64 = typename VT<CPLX>::T;
    using TA = typename PT<CPLX, F32>::T;
    const int cap = grp_cap(S.sp);
    const int U = pair_grp_unit(S.sp);
    const size_t lds = GrpLayout(cap, S.sp.M, S.sp.N, F32 ? 4 : 8, U, grp_bw(CPLX, NV, U)).bytes;
    // a multiple of 8 workgroups (one share per XCD), at most 16 per compute unit
    const int blocks = std::min(((nitems + 7) >> 3) << 3, 256 * 16);
    if (U == 8)
        hipLaunchKernelGGL((k_sigma_pair_grp<CPLX, F32, NV, STORE, 8>), dim3((unsigned)blocks), dim3(256), lds, st, S,
                           items, nitems, (const TA*)A, (const T64*)c, (T64*)sigma, (T64*)E, nq, nv, cap);
    else
        hipLaunchKernelGGL((k_sigma_pair_grp<CPLX, F32, NV, STORE, 4>), dim3((unsigned)blocks), dim3(256), lds, st, S,
                           items, nitems, (const TA*)A, (const T64*)c, (T64*)sigma, (T64*)E, nq, nv, cap);
    return hipGetLastError();
}

template <bool CPLX, bool F32>
static hipError_t launch_grp_all(const DevSpace& S, const GrpItem* items, int nitems, const void* A, const void* c,
                                 void* sigma, void* E, int n_vec, double e_core, const LaunchMarks* mk,
                                 hipStream_t st) {
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
            e = (nv == 2) ? launch_grp_nv<CPLX, F32, 2, true>(S, items, nitems, A, cc, ss, E, nq, 2, st)
                          : launch_grp_nv<CPLX, F32, 1, true>(S, items, nitems, A, cc, ss, E, nq, 1, st);
        else
            e = (nv == 2) ? launch_grp_nv<CPLX, F32, 2, false>(S, items, nitems, A, cc, ss, nullptr, 0, 2, st)
                          : launch_grp_nv<CPLX, F32, 1, false>(S, items, nitems, A, cc, ss, nullptr, 0, 1, st);
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

hipError_t launch_sigma_pair_grp(const DevSpace& S, const GrpItem* items_dev, int nitems, bool cplx, bool f32,
                                 const void* A, const void* c, void* sigma, void* E, int n_vec, double e_core,
                                 const LaunchMarks* mk, hipStream_t st) {
    if (!pair_grp_supported(S.sp) || nitems <= 0) return hipErrorInvalidValue;
    if (f32)
        return cplx ? launch_grp_all<true, true>(S, items_dev, nitems, A, c, sigma, E, n_vec, e_core, mk, st)
                    : launch_grp_all<false, true>(S, items_dev, nitems, A, c, sigma, E, n_vec, e_core, mk, st);
    return cplx ? launch_grp_all<true, false>(S, items_dev, nitems, A, c, sigma, E, n_vec, e_core, mk, st)
                : launch_grp_all<false, false>(S, items_dev, nitems, A, c, sigma, E, n_vec, e_core, mk, st);
}

}  // namespace stp
