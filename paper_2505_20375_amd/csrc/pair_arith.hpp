// Pair arithmetic of the pair-resolved sigma build, shared by its kernels
// (one lane per item) and by the host check (loops over items): the header
// of a pair intermediate K' (its strings, empty orbitals, creation ranks and
// class bases) and, per pair slot, the target address, pair index, target
// pair position and sign.
#pragma once
#include "stp_device.hpp"

namespace stp {

// Per-wave header after the slot arrays (bytes, 16-aligned).
struct PairHdr {
    int64_t rank[KMAX];      // local string ranks of K'
    int64_t cbase[NPCLS];    // class: target offset + untouched subspaces' rank * stride
    int64_t cstra[NPCLS];    // class: target stride of subspace a
    int64_t cstrb[NPCLS];    // class: target stride of subspace b
    uint32_t str[KMAX];      // local strings of K'
    int32_t voff[KMAX];      // first empty-orbital position of subspace k
    int32_t vcre[MMAX];      // creation of the empty orbital at position v on K' (sign * (rank + 1))
    uint8_t vglob[MMAX];     // global index of the empty orbital at position v
    uint64_t kbits;          // global occupation bits of K'
    uint64_t pad_;
};
static_assert(sizeof(PairHdr) % 16 == 0, "pair header alignment");

// ---- the pair arithmetic, shared by the kernel (one lane per item) and the
// host check (loops over items)

// Subspace k of K' (local index jloc in its category): rank, string, first
// empty-orbital position.
__host__ __device__ inline void pair_hdr_sub(const DevSpace& S, const PairCat& P, int64_t jloc, int k, PairHdr* hd) {
    const int64_t r = (jloc / P.stride[k]) % P.count[k];
    hd->rank[k] = r;
    hd->str[k] = S.bits[S.tabs[P.tab[k]].bits_off + r];
    int vo = 0;
    for (int q = 0; q < k; ++q) vo += S.sp.sub_m[q] - P.occ[q];
    hd->voff[k] = vo;
}

// Global orbital g: when empty in K', its position among the empties, and the
// creation a+_g on its subspace string.  Needs pair_hdr_sub of every subspace.
__host__ __device__ inline void pair_hdr_orb(const DevSpace& S, const PairCat& P, int g, PairHdr* hd) {
    const int K = S.sp.K;
    int k = 0;
    while (k + 1 < K && g >= S.sp.sub_off[k + 1]) ++k;
    const int l = g - S.sp.sub_off[k];
    const uint32_t s = hd->str[k];
    if ((s >> l) & 1u) return;
    const int v = hd->voff[k] + popc32(~s & lowmask(l));
    const StrTab& t = S.tabs[P.tab[k]];
    hd->vglob[v] = (uint8_t)g;
    hd->vcre[v] = (t.cre_off >= 0) ? S.cre[t.cre_off + hd->rank[k] * t.m + l] : 0;
}

// Pair class c: target offset plus the untouched subspaces' rank * stride,
// and the target strides of the two created subspaces.
__host__ __device__ inline void pair_hdr_cls(const DevSpace& S, const PairCat& P, int c, PairHdr* hd) {
    const int a = P.cls_a[c], b = P.cls_b[c];
    const Cat& T2 = S.cats[P.cls_target[c]];
    int64_t bs = T2.offset;
    for (int k = 0; k < S.sp.K; ++k)
        if (k != a && k != b) bs += hd->rank[k] * T2.stride[k];
    hd->cbase[c] = bs;
    hd->cstra[c] = T2.stride[a];
    hd->cstrb[c] = T2.stride[b];
}

// Global occupation bits of K' (after pair_hdr_sub of every subspace).
__host__ __device__ inline void pair_hdr_bits(const DevSpace& S, PairHdr* hd) {
    uint64_t b = 0;
    for (int k = 0; k < S.sp.K; ++k) b |= (uint64_t)hd->str[k] << S.sp.sub_off[k];
    hd->kbits = b;
}

// Slot `slot` < deg of K': target address, pair index r (r - 1) / 2 + p of the
// created pair p < r, the position q of {p, r} among the occupied pairs of the
// target (q = i_r (i_r - 1) / 2 + i_p, i_x = occupied orbitals of the target
// below x), and the sign of a+_p a+_r |K'> (true: negative).
__host__ __device__ inline bool pair_slot(const DevSpace& S, const PairCat& P, const PairHdr* hd, int slot,
                                          int64_t& addr, int& pi, int& q) {
    const uint32_t info = S.pslot[P.slot_off + slot];
    const int cl = (int)(info & 255u), i = (int)((info >> 8) & 255u), j = (int)(info >> 16);
    const int a = P.cls_a[cl], b = P.cls_b[cl];
    const int va = hd->voff[a] + i, vb = hd->voff[b] + j;
    const int gp = hd->vglob[va], gr = hd->vglob[vb];
    bool neg;
    if (a != b) {
        const int ca = hd->vcre[va], cb = hd->vcre[vb];
        const int64_t ra = (ca < 0 ? -ca : ca) - 1, rb = (cb < 0 ? -cb : cb) - 1;
        neg = ((ca < 0) != (cb < 0)) != (P.cls_phase[cl] != 0);
        addr = hd->cbase[cl] + ra * hd->cstra[cl] + rb * hd->cstrb[cl];
    } else {
        // a+_r first on the K' string, then a+_p (p < r) on the result
        const int c1 = hd->vcre[vb];
        const int64_t r1 = (c1 < 0 ? -c1 : c1) - 1;
        const StrTab& t1 = S.tabs[S.tabs[P.tab[a]].tab_up];
        const int c2 = S.cre[t1.cre_off + r1 * t1.m + (gp - S.sp.sub_off[a])];
        const int64_t r2 = (c2 < 0 ? -c2 : c2) - 1;
        neg = (c1 < 0) != (c2 < 0);
        addr = hd->cbase[cl] + r2 * hd->cstra[cl];
    }
    pi = gr * (gr - 1) / 2 + gp;
    const int ip = popc64(hd->kbits & ((1ULL << gp) - 1ULL));
    const int ir = popc64(hd->kbits & ((1ULL << gr) - 1ULL)) + 1;
    q = ir * (ir - 1) / 2 + ip;
    return neg;
}

}  // namespace stp
