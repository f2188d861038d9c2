// Spectator-batched matrix-core form of the pair-resolved sigma build, for
// spaces of several subspaces (distributed active spaces, K >= 2).
//
// The pair resolution (H on the N-electron sector as one two-body operator
// with the pair-pair table A, inserted identity over (N-2)-electron
// intermediates K', the resolution of Eq. sigmaL2e taken two electrons down)
// gives per K' the product e = A_K' d over the pairs that lead from K' into
// the space.  In STP-DAS the intermediates of one pair category that agree on
// the strings of the leading subspaces 1..K-1 differ only in subspace L = K:
// the operator strings of Eq. sigmaL2e act on them with the same integrals,
// the last subspace being the spectator (or, for pairs reaching into L, the
// subspace whose occupations select which rows apply).  Such a group is
// contracted as ONE product E = A_G B: rows and columns of A_G are the
// group's padded pair list (every orbital of subspace L, the empty orbitals
// of the others), B holds one column per member and vector component with
// the signed gathered coefficients (zero where a pair meets an orbital
// occupied in that member), and E is scattered back with the same
// arithmetic.  Consecutive members are consecutive strings of subspace L,
// the fastest index of every block, so the gathers and the scatter of the
// pairs that do not touch L walk contiguous addresses.
//
// Kernel shape (gfx950): one workgroup of eight wavefronts per compute unit
// (two per SIMD), persistent over the items; each XCD works through a
// contiguous eighth of them.  An item's right-hand side is at most four
// 16-column groups (64 columns); each wavefront owns one 16-row tile of E
// per pass (in a pass of at most four tiles, two or four wavefronts share a
// tile, each taking part of every chunk's steps and adding its part of E to
// sigma) and accumulates all column groups with v_mfma_f64_16x16x4f64
// (complex: one product with the real and one with the imaginary part of
// the table, combined by a lane exchange).  B is built 64 rows at a time
// into LDS (double buffered, the gathers of the next chunk in flight during
// the products of the current one; every entry formed without branches; the
// last chunk's products stop at its last group of 16 rows that holds rows of
// the list); each table fragment (one 16-byte read per lane) feeds one
// product per column group and table part.  E is added to sigma with device atomics
// (sigma is not bitwise deterministic).  The FP32 form of the precision
// option runs the same kernel with the FP32 table, B rounded to FP32 in LDS
// and v_mfma_f32_16x16x4f32 (FP32 accumulation of a product; its output rows
// lie at 4 (lane / 16) + i instead of lane / 16 + 4 i); E is added to the
// FP64 sigma.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "space.hpp"
#include "stp_device.hpp"

namespace stp {

typedef double sb_f64x4 __attribute__((ext_vector_type(4)));
typedef float sb_f32x4 __attribute__((ext_vector_type(4)));

constexpr int SB_WAVES = 8;                  // wavefronts per workgroup
constexpr int SB_NG = 4;                     // 16-column groups per item (accumulators: 64 VGPRs)
constexpr int SB_SGP = SB_NG / 2;            // column groups staged at a time for the scatter
constexpr int SB_TK = 64;                    // rows of B per chunk (steps of 4 rows)
constexpr int SB_NQ = SB_TK / 16;             // groups of four steps per chunk
constexpr int SB_BSTR = SB_NG * 16 + 16;     // B row stride (elements): rows alternate bank halves
constexpr int SB_BK = 33;                    // binomial table: C(n, k), n < 32, k <= 32
constexpr int SB_KMAX = SB_NG * 16;          // members per item at one column each
static_assert(SB_WAVES * 16 * SB_SGP * 16 <= 2 * SB_TK * SB_BSTR, "scatter staging must fit the B buffers");
constexpr uint32_t SB_PADROW = 0xffffffffu;  // row past the padded list
constexpr int SB_ROWS_MAX = 2048;            // padded rows (LDS row arrays)

__device__ __forceinline__ sb_f64x4 sb_mfma(double a, double b, sb_f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ sb_f32x4 sb_mfma(float a, float b, sb_f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---- arithmetic shared by the kernel and the host check ------------------

// colex rank of a local mask: sum over its set bits (ascending, e-th bit at
// position b) of C(b, e)
__host__ __device__ __forceinline__ int64_t sb_rank(uint32_t m, const int32_t* binom) {
    int64_t r = 0;
    for (int e = 1; m; ++e) {
        r += binom[__builtin_ctz(m) * SB_BK + e];
        m &= m - 1u;
    }
    return r;
}

__host__ __device__ __forceinline__ int sb_nth_zero(uint32_t s, int m, int i) {
    uint32_t z = ~s & lowmask(m);
    for (int t = 0; t < i; ++t) z &= z - 1u;
    return __builtin_ctz(z);
}

// Leading-subspace strings of an item's group (first member at local index jloc0).
struct SbHdr {
    uint64_t fbits;          // occupation bits of subspaces 1..K-1
    int64_t rank[KMAX];
    uint32_t str[KMAX];
};

__host__ __device__ inline void sb_hdr_sub(const DevSpace& S, const PairCat& P, int64_t jloc0, int k, SbHdr* h) {
    const int64_t r = (jloc0 / P.stride[k]) % P.count[k];
    h->rank[k] = r;
    h->str[k] = S.bits[S.tabs[P.tab[k]].bits_off + r];
}

__host__ __device__ inline void sb_hdr_bits(const DevSpace& S, SbHdr* h) {
    uint64_t b = 0;
    for (int k = 0; k + 1 < S.sp.K; ++k) b |= (uint64_t)h->str[k] << S.sp.sub_off[k];
    h->fbits = b;
}

// Row of the padded pair list: pair p < r (global orbitals), its pair index,
// and the part of the target address and sign fixed by the leading
// subspaces.  inf = pi | mode << 12 | sgnF << 14 | sL << 16 | qL << 21, mode 0:
// p, r in subspaces 1..K-1; 1: r in L; 2: p, r in L (sL, qL: local orbitals
// of r and p in L).
__host__ __device__ inline void sb_row(const DevSpace& S, const PairCat& P, const SbHdr* h, uint32_t slot,
                                       const int32_t* binom, int64_t* base_out, uint32_t* inf_out) {
    const int K = S.sp.K, L = K - 1;
    const int cl = (int)(slot & 255u), i = (int)((slot >> 8) & 255u), j = (int)(slot >> 16);
    const int a = P.cls_a[cl], b = P.cls_b[cl];
    int pl, rl;   // local orbitals
    if (a == L) {
        pl = i;
        rl = j;
    } else {
        pl = sb_nth_zero(h->str[a], S.sp.sub_m[a], i);
        rl = (b == L) ? j : sb_nth_zero(h->str[b], S.sp.sub_m[b], j);
    }
    const int p = S.sp.sub_off[a] + pl, r = S.sp.sub_off[b] + rl;
    const Cat& T = S.cats[P.cls_target[cl]];
    int64_t base = T.offset;
    for (int k = 0; k < L; ++k) {
        uint32_t s = h->str[k];
        int64_t rk;
        if (k == a || k == b) {
            if (k == a) s |= 1u << pl;
            if (k == b) s |= 1u << rl;
            rk = sb_rank(s, binom);
        } else {
            rk = h->rank[k];
        }
        base += rk * T.stride[k];
    }
    const int mode = (a == L) ? 2 : (b == L ? 1 : 0);
    const uint64_t f = h->fbits;
    const int par = popc64(f & ((1ull << r) - 1ull)) + popc64(f & ((1ull << p) - 1ull));
    uint32_t inf = (uint32_t)(r * (r - 1) / 2 + p) | (uint32_t)mode << 12 | (uint32_t)(par & 1) << 14;
    if (mode >= 1) inf |= (uint32_t)rl << 16;
    if (mode == 2) inf |= (uint32_t)pl << 21;
    *base_out = base;
    *inf_out = inf;
}

// Member table: for a member string t of subspace L with set bits
// t_0 < ... < t_{n-1}, the prefix sums P_x[k] = sum_{i<k} C(t_i, i + 1 + x)
// for x = 0, 1, 2 and k = 0..n, stored as pre[x * (n + 1) + k].  Creating
// one or two electrons in L moves the bits above them up by one or two
// places of the colex sum, so the rank of the result takes three prefix
// values and two binomials, with no loop over the string.
__host__ __device__ inline void sb_member(uint32_t t, int n, const int32_t* binom, int32_t* pre) {
    const int ps = n + 1;
    int32_t a0 = 0, a1 = 0, a2 = 0;
    pre[0] = pre[ps] = pre[2 * ps] = 0;
    int i = 0;
    for (uint32_t m = t; m; m &= m - 1u, ++i) {
        const int b = __builtin_ctz(m);
        a0 += binom[b * SB_BK + i + 1];
        a1 += (i + 2 < SB_BK) ? binom[b * SB_BK + i + 2] : 0;
        a2 += (i + 3 < SB_BK) ? binom[b * SB_BK + i + 3] : 0;
        pre[i + 1] = a0;
        pre[ps + i + 1] = a1;
        pre[2 * ps + i + 1] = a2;
    }
}

// Entry (row, member with subspace-L string tL of n electrons, rank jL, table
// pre): 0 when the pair meets an orbital occupied in the member, else +-1
// with the target address.  Mode 1 creates s in L (a = electrons of tL below
// s): rank = P_0[a] + C(s, a + 1) + P_1[n] - P_1[a]; mode 2 creates q < s in L
// (a below q, b below s): rank = P_0[a] + C(q, a + 1) + P_1[b] - P_1[a] +
// C(s, b + 2) + P_2[n] - P_2[b]; the sign adds the electrons of tL below each
// created orbital.  Written without branches (every table value is read and
// the result selected by the mode), so that the entries of a thread issue
// their LDS reads together; inf must be a row of the list (mode <= 2, local
// orbitals below 31), every index then stays inside the tables.
__host__ __device__ __forceinline__ int sb_entry(uint32_t inf, int64_t base, uint32_t tL, int n, const int32_t* pre,
                                                 int64_t jL, const int32_t* binom, int64_t* addr) {
    const int mode = (int)((inf >> 12) & 3u);
    const int sl = (int)((inf >> 16) & 31u);   // 0 in mode 0
    const int ql = (int)((inf >> 21) & 31u);   // 0 in modes 0 and 1
    const int ps = n + 1;
    const int b = popc32(tL & ((1u << sl) - 1u));
    const int a = popc32(tL & ((1u << ql) - 1u));
    const int64_t p1n = pre[ps + n], p1b = pre[ps + b];
    const int64_t r1 = (int64_t)pre[b] + binom[sl * SB_BK + b + 1] + p1n - p1b;
    const int64_t r2 = (int64_t)pre[a] + binom[ql * SB_BK + a + 1] + p1b - pre[ps + a] + binom[sl * SB_BK + b + 2] +
                       pre[2 * ps + n] - pre[2 * ps + b];
    const bool hit = (mode >= 1 && ((tL >> sl) & 1u)) || (mode == 2 && ((tL >> ql) & 1u));
    const int neg = (int)((inf >> 14) & 1u) ^ (mode == 0 ? 0 : mode == 1 ? (b & 1) : ((a + b) & 1));
    *addr = base + (mode == 0 ? jL : mode == 1 ? r1 : r2);
    return hit ? 0 : (neg ? -1 : 1);
}

// ---- plan (host) ----------------------------------------------------------

// Column chunks of a group of count_L members at cw columns each: the
// 16-column groups split as evenly as possible into chunks of at most SB_NG.
__host__ __device__ inline int sb_nchunk(int count_L, int cw) {
    const int ncg = (count_L * cw + 15) / 16;
    return (ncg + SB_NG - 1) / SB_NG;
}
__host__ __device__ inline void sb_chunk_span(int count_L, int cw, int nch, int ch, int* cg0, int* cg1) {
    const int ncg = (count_L * cw + 15) / 16;
    *cg0 = ch * ncg / nch;
    *cg1 = (ch + 1) * ncg / nch;
}

bool build_sb_plan(const HostSpace& H, SbHostPlan& plan) {
    plan = SbHostPlan{};
    const Space& sp = H.sp;
    const int K = sp.K, L = K - 1;
    if (K < 2 || sp.N < 2 || sp.sub_m[L] > 31) return false;
    int maxpad = 0, maxn = 0;
    for (int w = 0; w < sp.npcat; ++w) {
        const PairCat& P = H.pcats[w];
        SbCat c{};
        c.w = w;
        c.row_off = (int32_t)plan.rows.size();
        for (int cl = 0; cl < P.ncls; ++cl) {
            const int a = P.cls_a[cl], b = P.cls_b[cl];
            const int ea = (a == L) ? sp.sub_m[a] : sp.sub_m[a] - P.occ[a];
            const int eb = (b == L) ? sp.sub_m[b] : sp.sub_m[b] - P.occ[b];
            if (a == b) {
                for (int j = 1; j < eb; ++j)
                    for (int i = 0; i < j; ++i)
                        plan.rows.push_back((uint32_t)cl | (uint32_t)i << 8 | (uint32_t)j << 16);
            } else {
                for (int j = 0; j < eb; ++j)
                    for (int i = 0; i < ea; ++i)
                        plan.rows.push_back((uint32_t)cl | (uint32_t)i << 8 | (uint32_t)j << 16);
            }
        }
        c.npad = (int32_t)plan.rows.size() - c.row_off;
        if (c.npad > SB_ROWS_MAX) return false;
        maxpad = std::max(maxpad, c.npad);
        maxn = std::max(maxn, P.occ[L]);
        c.count_L = (int32_t)P.count[L];
        c.ngroups = P.size / P.count[L];
        plan.cats.push_back(c);
    }
    if (plan.cats.empty()) return false;
    // streams grouped by (log2(CW), column groups of the chunk)
    for (int x = 0; x < 3; ++x) {
        const int cw = 1 << x;
        for (int g = 1; g <= 8; ++g) {
            plan.sbegin[x][g - 1] = (int32_t)plan.streams.size();
            int64_t items = 0;
            if (g <= SB_NG)
                for (int ci = 0; ci < (int)plan.cats.size(); ++ci) {
                    const SbCat& c = plan.cats[ci];
                    const int nch = sb_nchunk(c.count_L, cw);
                    for (int ch = 0; ch < nch; ++ch) {
                        int cg0, cg1;
                        sb_chunk_span(c.count_L, cw, nch, ch, &cg0, &cg1);
                        if (cg1 - cg0 != g) continue;
                        plan.streams.push_back(SbStream{ci, ch, items});
                        items += c.ngroups;
                    }
                }
            plan.nitems[x][g - 1] = items;
        }
        plan.sbegin[x][8] = (int32_t)plan.streams.size();
    }
    plan.cap = (maxpad + SB_TK - 1) / SB_TK * SB_TK;   // whole chunks of rows
    plan.nlmax = maxn;
    return true;
}

// Matrix-core flops and items of one launch sequence (one pass of at most
// two vectors): per item, (npad rounded to 16) / 16 row tiles x (npad
// rounded to 16) / 4 steps (the last chunk's products stop at its last
// group of 16 rows that holds rows of the list) x its column groups x 2048
// flop per v_mfma_f64_16x16x4f64, twice for complex (the real and the
// imaginary part of the table).
void sb_plan_counts(const SbHostPlan& plan, bool cplx, int nv, double* flops, int64_t* items) {
    const int cw = cplx ? 2 * nv : nv;
    const int x = (cw == 1) ? 0 : (cw == 2 ? 1 : 2);
    double f = 0;
    int64_t it = 0;
    for (int g = 1; g <= SB_NG; ++g)
        for (int q = plan.sbegin[x][g - 1]; q < plan.sbegin[x][g]; ++q) {
            const SbCat& c = plan.cats[plan.streams[q].cat];
            const double nrt = (c.npad + 15) / 16, nks = ((c.npad + 15) / 16) * 4;
            f += (double)c.ngroups * nrt * nks * g * 2048.0 * (cplx ? 2 : 1);
            it += c.ngroups;
        }
    *flops = f;
    *items = it;
}

bool pair_sb_supported(const Space& sp) {
    return sp.K >= 2 && sp.N >= 2 && sp.sub_m[sp.K - 1] <= 31 && sp.M <= 64;
}

// LDS layout of a workgroup: rows (target base, info), members (strings and
// prefix tables), binomials, chunk flags, header, two B buffers.
struct SbLayout {
    size_t base_off, inf_off, col_off, pre_off, bin_off, flag_off, hdr_off, b_off, bytes;
    __host__ __device__ SbLayout(int cap, int nlmax, int bsz) {
        base_off = 0;
        inf_off = base_off + (size_t)cap * 8;
        col_off = inf_off + (size_t)cap * 4;
        pre_off = col_off + (size_t)SB_KMAX * 4;
        bin_off = pre_off + (size_t)SB_KMAX * 3 * (nlmax + 1) * 4;
        flag_off = bin_off + (size_t)32 * SB_BK * 4;
        hdr_off = (flag_off + (size_t)(SB_ROWS_MAX / SB_TK + 4) * 4 + 15) & ~(size_t)15;
        b_off = (hdr_off + sizeof(SbHdr) + 15) & ~(size_t)15;
        bytes = b_off + (size_t)2 * SB_TK * SB_BSTR * bsz;
    }
};

size_t pair_sb_lds_bytes(int cap, int nlmax) { return SbLayout(cap, nlmax, 8).bytes; }

// Value of x in lane (lane ^ X) of the same quad (DPP quad permutation).
template <int X>
__device__ __forceinline__ double sb_quad_xor(double x) {
    constexpr int ctrl = (X == 2) ? 0x4E : 0xB1;   // quad_perm [2,3,0,1] or [1,0,3,2]
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int X>
__device__ __forceinline__ float sb_quad_xor(float x) {
    constexpr int ctrl = (X == 2) ? 0x4E : 0xB1;
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), ctrl, 0xF, 0xF, false));
}

// f(integral_constant<int, I>) ... f(integral_constant<int, N - 1>), unrolled.
template <int I, int N, class F>
__device__ __forceinline__ void sb_static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        sb_static_for<I + 1, N>(f);
    }
}

// The products of a group of four steps of a B chunk (steps K0..K0+3 of 4
// rows each) for NGU column groups with the table fragments af of those
// steps, the B fragments read one step ahead.
template <int NGU, int K0, bool CPLX, typename TA, typename BT, typename ACC>
__device__ __forceinline__ void sb_mma(const BT* __restrict__ B, int kq, int c16, const TA (&af)[4],
                                       ACC (&c1)[NGU], ACC (&c2)[NGU]) {
    BT bf[2][NGU];
#pragma unroll
    for (int h = 0; h < NGU; ++h) bf[0][h] = B[(K0 * 4 + kq) * SB_BSTR + c16 + 16 * h];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        if (ks + 1 < 4) {
#pragma unroll
            for (int h = 0; h < NGU; ++h)
                bf[(ks + 1) & 1][h] = B[((K0 + ks + 1) * 4 + kq) * SB_BSTR + c16 + 16 * h];
        }
#pragma unroll
        for (int h = 0; h < NGU; ++h) {
            if constexpr (CPLX) {
                c1[h] = sb_mfma(af[ks].x, bf[ks & 1][h], c1[h]);
                c2[h] = sb_mfma(af[ks].y, bf[ks & 1][h], c2[h]);
            } else {
                c1[h] = sb_mfma(af[ks], bf[ks & 1][h], c1[h]);
            }
        }
    }
}

// Table fragments of a group of four steps: lane (kq, c16) holds A[row pair, pair of
// chunk row 4 (K0 + ks) + kq] for ks < 4 (rows past the list: pair 0).
template <int K0, typename TA>
__device__ __forceinline__ void sb_afrag(const uint32_t* __restrict__ rinf, const TA* __restrict__ arow, int NP,
                                         int kq, TA (&af)[4]) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        const uint32_t qi = rinf[(K0 + ks) * 4 + kq];
        af[ks] = arow[(int64_t)((qi == SB_PADROW) ? 0u : (qi & 0xfffu)) * NP];
    }
}

// ---- kernel -----------------------------------------------------------------

// State of one item shared by its passes (LDS arrays and item scalars).
struct SbItem {
    const int64_t* rbase;
    const uint32_t* rinf;
    const uint32_t* colstr;
    const int32_t* pre;
    const int32_t* binom;
    int* flags;
    int nk, j0, nL, ps3, nkc, nRT, npad;
};

// Passes over the row tiles of one item with NGU column groups: wavefront
// wid owns row tile pass * 8 + wid; B is rebuilt chunk by chunk in every
// pass (the gathers of the next chunk in flight during the products of the
// current one); the row tile is then scattered through an LDS staging area
// with device atomics.
template <bool CPLX, int NV, int NGU, bool F32, typename TA, typename BT>
__device__ __forceinline__ void sb_item(const SbItem& I, const TA* __restrict__ A, int NP,
                                        const typename VT<CPLX>::T* __restrict__ c,
                                        typename VT<CPLX>::T* __restrict__ sigma, int64_t nd, int n_vec, BT* bsh,
                                        int tid) {
    using V64 = VT<CPLX>;
    using TE = typename V64::T;
    using ACC = std::conditional_t<F32, sb_f32x4, sb_f64x4>;
    constexpr int CW = CPLX ? 2 * NV : NV;   // columns per member
    constexpr int KPG = 16 / CW;             // members per column group
    constexpr int NT = SB_WAVES * 64;
    constexpr int KSPAN = NGU * KPG;         // member slots of the item
    constexpr int EPT = (SB_TK * NV * KSPAN + NT - 1) / NT;   // B entries per thread per chunk
    const int lane = tid & 63, wid = tid >> 6;
    const int kq = lane >> 4, c16 = lane & 15;
    const int col = c16 % CW;
    const int nkc = I.nkc;

    // B entries of this thread: the addresses and signs are formed first and
    // every gather issued without a branch (an entry that vanishes reads
    // element 0 and is replaced by zero afterwards), so that a chunk's
    // gathers are in flight together while the products of the previous
    // chunk run
    TE gx[EPT];
    int gsg[EPT];    // +-1, or 0 for a vanishing entry
    int gcol[EPT];   // LDS position (row * SB_BSTR + first column) or -1
    auto gen_issue = [&](int kc) {
        int64_t ga[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int ent = tid + e * NT;
            const int jj = ent % KSPAN;
            const int rest = ent / KSPAN;
            const int v = rest % NV, q = rest / NV;
            gcol[e] = (q < SB_TK) ? q * SB_BSTR + jj * CW + v : -1;
            const int R = kc * SB_TK + min(q, SB_TK - 1);
            const uint32_t inf0 = I.rinf[R];
            const bool ok = q < SB_TK && inf0 != SB_PADROW && jj < I.nk && v < n_vec;
            int64_t addr;
            const int s0 = sb_entry(ok ? inf0 : 0u, I.rbase[R], I.colstr[jj], I.nL, I.pre + jj * I.ps3, I.j0 + jj,
                                    I.binom, &addr);
            const int sg = ok ? s0 : 0;
            gsg[e] = sg;
            ga[e] = (sg != 0) ? (int64_t)v * nd + addr : 0;
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) gx[e] = c[ga[e]];
    };
    auto gen_commit = [&](int kc, int buf) {
        BT* B = bsh + (size_t)buf * SB_TK * SB_BSTR;
        bool nz = false;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const double sgd = (double)gsg[e];
            if constexpr (CPLX) {
                const BT xr = (BT)(gsg[e] ? sgd * gx[e].x : 0.0), xi = (BT)(gsg[e] ? sgd * gx[e].y : 0.0);
                if (gcol[e] >= 0) {
                    B[gcol[e]] = xr;
                    B[gcol[e] + NV] = xi;
                }
                nz = nz || xr != (BT)0 || xi != (BT)0;
            } else {
                const BT xr = (BT)(gsg[e] ? sgd * gx[e] : 0.0);
                if (gcol[e] >= 0) B[gcol[e]] = xr;
                nz = nz || xr != (BT)0;
            }
        }
        if (__ballot(nz) != 0 && lane == 0) atomicOr(&I.flags[kc], 1);
    };

    const int npass = (I.nRT + SB_WAVES - 1) / SB_WAVES;
    for (int pass = 0; pass < npass; ++pass) {
        // the pass's row tiles; when it holds at most half (a quarter) as
        // many tiles as wavefronts, the wavefronts of a tile share its
        // products, each taking two groups (one group) of four steps of
        // every chunk, and each adds its part of E to sigma
        const int r = min(SB_WAVES, I.nRT - pass * SB_WAVES);
        const int split = (r <= SB_WAVES / 4) ? 4 : (r <= SB_WAVES / 2) ? 2 : 1;
        const int RT = pass * SB_WAVES + wid % r;
        const int kpart = wid / r;   // this wavefront's share of the groups of four steps
        const bool own = kpart < split;
        auto mine = [&](int G) { return (G * split) / SB_NQ == kpart; };
        ACC c1[NGU], c2[NGU];
#pragma unroll
        for (int h = 0; h < NGU; ++h) c1[h] = c2[h] = ACC{0, 0, 0, 0};
        // this A lane's row pair (rows past the list: pair 0, outputs dropped)
        const uint32_t pinf = own ? I.rinf[RT * 16 + c16] : SB_PADROW;
        const TA* arow = A + ((pinf == SB_PADROW) ? 0u : (pinf & 0xfffu));
        // table fragments of the chunk in use, in groups of four steps:
        // each group of the next chunk is requested as soon as the products
        // of the same group of the current chunk are issued (the last after
        // the chunk build, which must not wait for it: loads complete in
        // order)
        TA af[SB_NQ][4];
        if (own) sb_static_for<0, SB_NQ>([&](auto G) {
            if (mine(G)) sb_afrag<4 * G>(I.rinf, arow, NP, kq, af[G]);
        });
        gen_issue(0);
        gen_commit(0, 0);
        __syncthreads();
        for (int kc = 0; kc < nkc; ++kc) {
            const int buf = kc & 1;
            const bool more = kc + 1 < nkc;
            const BT* B = bsh + (size_t)buf * SB_TK * SB_BSTR;
            const uint32_t* rnext = I.rinf + (kc + 1) * SB_TK;
            // the table fragments of this chunk (requested during the
            // previous one) are in: stating it here keeps the compiler from
            // waiting inside the products below for the gathers issued next
            // (its count of outstanding loads cannot tell them apart across
            // the loop edge)
            __builtin_amdgcn_s_waitcnt(0);
            if (more) gen_issue(kc + 1);
            const bool mm = own && I.flags[kc];
            // groups of 16 rows of this chunk that hold rows of the list (the
            // rest of the last chunk is padding: its products add zeros)
            const int ngv = min(SB_NQ, (I.npad - kc * SB_TK + 15) >> 4);
            sb_static_for<0, SB_NQ>([&](auto G) {
                if (mm && G < ngv && mine(G)) sb_mma<NGU, 4 * G, CPLX>(B, kq, c16, af[G], c1, c2);
                if constexpr (G + 1 < SB_NQ) {
                    if (own && more && mine(G)) sb_afrag<4 * G>(rnext, arow, NP, kq, af[G]);
                }
            });
            if (more) gen_commit(kc + 1, buf ^ 1);
            if (own && more && mine(SB_NQ - 1)) sb_afrag<4 * (SB_NQ - 1)>(rnext, arow, NP, kq, af[SB_NQ - 1]);
            __syncthreads();
        }
        // ---- scatter of this wavefront's row tile, staged through LDS (the
        // B buffers are free after the last chunk): SB_SGP column groups at a
        // time, register i of column group h holding row kq + 4 i and column
        // 16 h + c16 of the tile; then each lane adds the values of one (row,
        // member) pair, consecutive lanes taking consecutive members
        // (consecutive addresses for the pairs that leave subspace L alone)
        bool any = false;
        for (int kc = 0; kc < nkc; ++kc) any = any || I.flags[kc] != 0;
        constexpr int SC = SB_SGP * 16;   // staged columns
        constexpr int MH = SC / CW;       // members per part
        BT* stage = bsh + (size_t)wid * 16 * SC;
#pragma unroll
        for (int part = 0; part * SB_SGP < NGU; ++part) {
            if (!own || !any) break;
#pragma unroll
            for (int hh = 0; hh < SB_SGP; ++hh) {
                const int h = SB_SGP * part + hh;
                if (h >= NGU) break;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    BT val;
                    if constexpr (CPLX) {
                        const BT pv = sb_quad_xor<NV == 2 ? 2 : 1>((BT)c2[h][i]);
                        val = (col < NV) ? c1[h][i] - pv : c1[h][i] + pv;
                    } else {
                        val = c1[h][i];
                    }
                    stage[(F32 ? 4 * kq + i : kq + 4 * i) * SC + 16 * hh + c16] = val;
                }
            }
            wave_lds_sync();
            const int jbase = part * MH;
            for (int e = lane; e < 16 * MH; e += 64) {
                const int jl = e % MH, row = e / MH;
                const int jj = jbase + jl;
                const int R = RT * 16 + row;
                const uint32_t inf = I.rinf[R];
                if (inf == SB_PADROW || jj >= I.nk) continue;
                int64_t addr;
                const int sg = sb_entry(inf, I.rbase[R], I.colstr[jj], I.nL, I.pre + jj * I.ps3, I.j0 + jj, I.binom,
                                        &addr);
                if (sg == 0) continue;
                const double sgd = sg < 0 ? -1.0 : 1.0;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    if (v >= n_vec) break;
                    double* dst = reinterpret_cast<double*>(sigma + (int64_t)v * nd + addr);
                    if constexpr (CPLX) {
                        unsafeAtomicAdd(dst, sgd * (double)stage[row * SC + jl * CW + v]);
                        unsafeAtomicAdd(dst + 1, sgd * (double)stage[row * SC + jl * CW + NV + v]);
                    } else {
                        unsafeAtomicAdd(dst, sgd * (double)stage[row * SC + jl * CW + v]);
                    }
                }
            }
            wave_lds_sync();
        }
        __syncthreads();   // the next pass rebuilds B where the tiles were staged
    }
}

// One launch per item shape: items of NGU column groups (the streams of
// (log2(CW), NGU)), persistent over the items, each XCD a contiguous share.
template <bool CPLX, int NV, int NGU, bool F32>
__global__ __launch_bounds__(SB_WAVES * 64, 1) void k_sigma_pair_sb(DevSpace S, SbPlan plan,
                                                                    const typename PT<CPLX, F32>::T* __restrict__ A,
                                                                    const typename VT<CPLX>::T* __restrict__ c,
                                                                    typename VT<CPLX>::T* __restrict__ sigma,
                                                                    int n_vec) {
    using BT = std::conditional_t<F32, float, double>;
    constexpr int CW = CPLX ? 2 * NV : NV;   // columns per member
    constexpr int CWI = (CW == 1) ? 0 : (CW == 2 ? 1 : 2);
    constexpr int KPG = 16 / CW;             // members per column group
    constexpr int NT = SB_WAVES * 64;
    extern __shared__ __align__(16) unsigned char smem[];
    const SbLayout LY(plan.cap, plan.nlmax, (int)sizeof(BT));
    int64_t* rbase = reinterpret_cast<int64_t*>(smem + LY.base_off);
    uint32_t* rinf = reinterpret_cast<uint32_t*>(smem + LY.inf_off);
    uint32_t* colstr = reinterpret_cast<uint32_t*>(smem + LY.col_off);
    int32_t* pre = reinterpret_cast<int32_t*>(smem + LY.pre_off);
    int32_t* binom = reinterpret_cast<int32_t*>(smem + LY.bin_off);
    int* flags = reinterpret_cast<int*>(smem + LY.flag_off);
    SbHdr* hd = reinterpret_cast<SbHdr*>(smem + LY.hdr_off);
    BT* bsh = reinterpret_cast<BT*>(smem + LY.b_off);
    const int tid = threadIdx.x;
    const int K = S.sp.K, L = K - 1;
    const int NP = S.sp.npairs;
    const int64_t nd = S.sp.ndets;

    for (int t = tid; t < 32 * SB_BK; t += NT) {
        const int n = t / SB_BK, k = t % SB_BK;
        int64_t b = (k <= n) ? 1 : 0;
        for (int x = 1; x <= k && k <= n; ++x) b = b * (n - k + x) / x;
        binom[t] = (int32_t)b;
    }

    const int s0 = plan.sbegin[CWI][NGU - 1], s1 = plan.sbegin[CWI][NGU];
    const int64_t total = plan.nitems[CWI][NGU - 1];
    const int xcd = blockIdx.x & 7, nloc = gridDim.x >> 3;
    const int64_t share = (total + 7) >> 3;
    const int64_t it_end = min(total, (int64_t)(xcd + 1) * share);
    for (int64_t it = (int64_t)xcd * share + (blockIdx.x >> 3); it < it_end; it += nloc) {
        // ---- item: stream (category, column chunk), group
        int lo = s0, hi = s1 - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (plan.streams[mid].item_begin <= it) lo = mid; else hi = mid - 1;
        }
        const SbStream& st = plan.streams[lo];
        const SbCat& sc = plan.cats[st.cat];
        const PairCat& P = S.pcats[sc.w];
        const int64_t grp = it - st.item_begin;
        int cg0, cg1;
        sb_chunk_span(sc.count_L, CW, sb_nchunk(sc.count_L, CW), st.chunk, &cg0, &cg1);
        SbItem I;
        I.j0 = cg0 * KPG;                                   // first member (rank in subspace L)
        I.nk = min(sc.count_L, cg1 * KPG) - I.j0;           // members of this item
        const int64_t jloc0 = grp * (int64_t)sc.count_L;
        const int npad = sc.npad;
        I.nL = P.occ[L];
        I.ps3 = 3 * (I.nL + 1);
        I.nkc = (npad + SB_TK - 1) / SB_TK;                 // chunks of B rows
        I.npad = npad;
        I.nRT = (npad + 15) >> 4;                           // 16-row tiles
        I.rbase = rbase;
        I.rinf = rinf;
        I.colstr = colstr;
        I.pre = pre;
        I.binom = binom;
        I.flags = flags;
        __syncthreads();   // the previous item's readers of the LDS arrays are done
        if (tid < L) sb_hdr_sub(S, P, jloc0, tid, hd);
        const int64_t lbits = S.tabs[P.tab[L]].bits_off + I.j0;
        for (int t = tid; t < I.nk; t += NT) {
            const uint32_t tl = S.bits[lbits + t];
            colstr[t] = tl;
            sb_member(tl, I.nL, binom, pre + t * I.ps3);
        }
        for (int t = tid; t < I.nkc; t += NT) flags[t] = 0;
        __syncthreads();
        if (tid == 0) sb_hdr_bits(S, hd);
        __syncthreads();
        for (int r = tid; r < I.nkc * SB_TK; r += NT) {
            int64_t b = 0;
            uint32_t inf = SB_PADROW;
            if (r < npad) sb_row(S, P, hd, plan.rows[sc.row_off + r], binom, &b, &inf);
            rbase[r] = b;
            rinf[r] = inf;
        }
        __syncthreads();
        sb_item<CPLX, NV, NGU, F32>(I, A, NP, c, sigma, nd, n_vec, bsh, tid);
    }
}

template <bool CPLX, int NV, int NGU, bool F32>
static hipError_t launch_sb_g(const DevSpace& S, const SbPlan& plan, const void* A, const void* c, void* sigma,
                              int nv, hipStream_t st) {
    using T64 = typename VT<CPLX>::T;
    using TA = typename PT<CPLX, F32>::T;
    constexpr int CW = CPLX ? 2 * NV : NV;
    constexpr int CWI = (CW == 1) ? 0 : (CW == 2 ? 1 : 2);
    if (plan.nitems[CWI][NGU - 1] == 0) return hipSuccess;
    const size_t lds = SbLayout(plan.cap, plan.nlmax, F32 ? 4 : 8).bytes;
    hipLaunchKernelGGL((k_sigma_pair_sb<CPLX, NV, NGU, F32>), dim3(256), dim3(SB_WAVES * 64), lds, st, S, plan,
                       (const TA*)A, (const T64*)c, (T64*)sigma, nv);
    return hipGetLastError();
}

// One launch per column-group count, SB_NG down to 1.
template <bool CPLX, int NV, bool F32, int NGU = SB_NG>
static hipError_t launch_sb_nv(const DevSpace& S, const SbPlan& plan, const void* A, const void* c, void* sigma,
                               int nv, hipStream_t st) {
    static_assert(NGU >= 1 && NGU <= SB_NG, "column-group count");
    const hipError_t e = launch_sb_g<CPLX, NV, NGU, F32>(S, plan, A, c, sigma, nv, st);
    if constexpr (NGU > 1) {
        if (e == hipSuccess) return launch_sb_nv<CPLX, NV, F32, NGU - 1>(S, plan, A, c, sigma, nv, st);
    }
    return e;
}

template <bool CPLX, bool F32>
static hipError_t launch_sb_all(const DevSpace& S, const SbPlan& plan, const void* A, const void* c, void* sigma,
                                int n_vec, double e_core, const LaunchMarks* mk, hipStream_t st) {
    using T64 = typename VT<CPLX>::T;
    hipError_t e = launch_fill_init(CPLX, sigma, c, e_core, S.sp.ndets * n_vec, st);
    if (e != hipSuccess) return e;
    for (int v0 = 0; v0 < n_vec; v0 += 2) {
        const int nv = (n_vec - v0 >= 2) ? 2 : 1;
        const int64_t off = (int64_t)v0 * S.sp.ndets;
        const T64* cc = (const T64*)c + off;
        T64* ss = (T64*)sigma + off;
        if (mk) mk->fn(mk->user, 0, true);
        e = (nv == 2) ? launch_sb_nv<CPLX, 2, F32>(S, plan, A, cc, ss, 2, st)
                      : launch_sb_nv<CPLX, 1, F32>(S, plan, A, cc, ss, 1, st);
        if (mk) mk->fn(mk->user, 0, false);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_sigma_pair_sb(const DevSpace& S, const SbPlan& plan, bool cplx, bool f32, const void* A,
                                const void* c, void* sigma, int n_vec, double e_core, const LaunchMarks* mk,
                                hipStream_t st) {
    if (plan.ncat <= 0 || plan.cap <= 0 || plan.cap > SB_ROWS_MAX ||
        SbLayout(plan.cap, plan.nlmax, f32 ? 4 : 8).bytes > 160 * 1024)
        return hipErrorInvalidValue;
    if (f32)
        return cplx ? launch_sb_all<true, true>(S, plan, A, c, sigma, n_vec, e_core, mk, st)
                    : launch_sb_all<false, true>(S, plan, A, c, sigma, n_vec, e_core, mk, st);
    return cplx ? launch_sb_all<true, false>(S, plan, A, c, sigma, n_vec, e_core, mk, st)
                : launch_sb_all<false, false>(S, plan, A, c, sigma, n_vec, e_core, mk, st);
}

// Host check of the arithmetic above (the same functions on the host
// tables): for up to max_groups groups of every pair category, every padded
// row and every member, the entry must be zero exactly when the pair meets an
// orbital occupied in the member, and otherwise give the address of
// K' + {p, r} in the space and the sign of a+_p a+_r |K'> from the global
// occupation bits; every pair of K' that leads into the space must appear
// in its category's padded list exactly once.
int64_t check_sb_host(const DevSpace& S, const SbHostPlan& plan, int64_t max_groups, int64_t* n_checked,
                      bool (*to_bits)(const void*, int64_t, uint64_t*), const void* user) {
    const std::vector<SbCat>& cats = plan.cats;
    const std::vector<uint32_t>& rows = plan.rows;
    int64_t bad = 0, checked = 0;
    const int K = S.sp.K, L = K - 1;
    std::vector<int32_t> binom(32 * SB_BK);
    for (int n = 0; n < 32; ++n)
        for (int k = 0; k < SB_BK; ++k) {
            int64_t b = (k <= n) ? 1 : 0;
            for (int x = 1; x <= k && k <= n; ++x) b = b * (n - k + x) / x;
            binom[n * SB_BK + k] = (int32_t)b;
        }
    std::vector<int32_t> pre(3 * 33);
    for (const SbCat& sc : cats) {
        const PairCat& P = S.pcats[sc.w];
        const int64_t step = sc.ngroups <= max_groups ? 1 : sc.ngroups / max_groups;
        const StrTab& tl = S.tabs[P.tab[L]];
        const int nL = P.occ[L];
        for (int64_t g = 0; g < sc.ngroups; g += step) {
            SbHdr hd{};
            const int64_t jloc0 = g * sc.count_L;
            for (int k = 0; k < L; ++k) sb_hdr_sub(S, P, jloc0, k, &hd);
            sb_hdr_bits(S, &hd);
            for (int64_t jL = 0; jL < sc.count_L; ++jL) {
                const uint32_t tL = S.bits[tl.bits_off + jL];
                sb_member(tL, nL, binom.data(), pre.data());
                const uint64_t Kb = hd.fbits | (uint64_t)tL << S.sp.sub_off[L];
                int hits = 0;
                for (int r = 0; r < sc.npad; ++r) {
                    int64_t base;
                    uint32_t inf;
                    sb_row(S, P, &hd, rows[sc.row_off + r], binom.data(), &base, &inf);
                    int64_t addr = -1;
                    const int sg = sb_entry(inf, base, tL, nL, pre.data(), jL, binom.data(), &addr);
                    ++checked;
                    const int pi = (int)(inf & 0xfffu);
                    int rr = 1;
                    while ((rr + 1) * rr / 2 <= pi) ++rr;
                    const int p = pi - rr * (rr - 1) / 2;
                    const bool free_pr = p < rr && !((Kb >> p) & 1ULL) && !((Kb >> rr) & 1ULL);
                    if (!free_pr) {
                        bad += (sg != 0);
                        continue;
                    }
                    ++hits;
                    const uint64_t want = Kb | (1ULL << p) | (1ULL << rr);
                    const int par = popc64(Kb & ((1ULL << rr) - 1ULL)) + popc64(Kb & ((1ULL << p) - 1ULL));
                    uint64_t got = 0;
                    if (sg == 0 || addr < 0 || addr >= S.sp.ndets || !to_bits(user, addr, &got) || got != want ||
                        (sg < 0) != ((par & 1) != 0))
                        ++bad;
                }
                bad += (hits != P.deg);
            }
        }
    }
    // every (category, chunk) in exactly one stream, the chunks of a
    // category covering its members exactly once, streams counted right
    for (int x = 0; x < 3; ++x) {
        const int cw = 1 << x;
        std::vector<std::vector<int>> seen(cats.size());
        for (size_t ci = 0; ci < cats.size(); ++ci) seen[ci].assign(sb_nchunk(cats[ci].count_L, cw), 0);
        for (int g = 1; g <= 8; ++g) {
            int64_t items = 0;
            for (int q = plan.sbegin[x][g - 1]; q < plan.sbegin[x][g]; ++q) {
                const SbStream& st = plan.streams[q];
                const SbCat& c = cats[st.cat];
                int cg0, cg1;
                sb_chunk_span(c.count_L, cw, sb_nchunk(c.count_L, cw), st.chunk, &cg0, &cg1);
                bad += (cg1 - cg0 != g) || (st.item_begin != items);
                ++seen[st.cat][st.chunk];
                items += c.ngroups;
            }
            bad += (items != plan.nitems[x][g - 1]);
        }
        for (size_t ci = 0; ci < cats.size(); ++ci) {
            const int nch = (int)seen[ci].size();
            int covered = 0;
            for (int ch = 0; ch < nch; ++ch) {
                bad += (seen[ci][ch] != 1);
                int cg0, cg1;
                sb_chunk_span(cats[ci].count_L, cw, nch, ch, &cg0, &cg1);
                bad += (cg0 != covered) || (cg1 - cg0 > SB_NG) || (cg1 <= cg0);
                covered = cg1;
            }
            bad += (covered * (16 / cw) < cats[ci].count_L);
        }
    }
    if (n_checked) *n_checked = checked;
    return bad;
}

}  // namespace stp
