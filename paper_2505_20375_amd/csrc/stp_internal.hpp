// Internal data layout shared by the host tables (space.cpp) and the HIP
// kernels (kernels.hip).  Plain structs only; no HIP types.
#pragma once
#include <cstdint>

namespace stp {

constexpr int KMAX = 8;          // subspaces (distributed active spaces)
constexpr int MMAX = 64;         // spin-orbitals in total
constexpr int MSUB = 32;         // spin-orbitals per subspace (local strings are uint32 masks)
constexpr int NCLS = KMAX * KMAX;
constexpr int DET_BYTES = 96;   // sizeof of the device-side decoded determinant (ranks + masks)
constexpr int NPCLS = KMAX * (KMAX + 1) / 2;   // pair classes (a <= b)

// A local string table: all strings of n electrons in an m-orbital subspace,
// ranked in colexicographic order (= ascending value of the bit mask).
// ann[rank*m + l]: a_l applied to the string, packed as sign*(rank'+1) in the
// table `tab_dn` (n-1 electrons), 0 if l is empty.  cre[rank*m + l]: a+_l,
// packed into table `tab_up` (n+1 electrons), 0 if l is occupied.  The sign is
// (-1)^(number of occupied local orbitals below l).
struct StrTab {
    int32_t m, n;
    int64_t count;
    int64_t bits_off;   // into bits[]
    int64_t ann_off;    // into ann[] (count*m entries) or -1
    int64_t cre_off;    // into cre[] (count*m entries) or -1
    int32_t tab_dn;     // table index of (m, n-1) or -1
    int32_t tab_up;     // table index of (m, n+1) or -1
};

// One category: an occupation tuple (n_1..n_K).  Categories inside the space
// own a dense block of the CI vector (row-major over the local ranks, subspace
// 1 slowest); categories outside the space appear only as intermediates of
// the two-electron resolution.
//
// Move classes: a move creates x in subspace xs and annihilates y in subspace
// ys (x == y allowed when xs == ys).  Class c = xs*K + ys is usable when the
// category reached, cat + e_xs - e_ys, lies in the space; its slots are
// enumerated y-major: slot = i*width + j with y = i-th occupied orbital of
// the ys string and x = j-th empty orbital of the xs string, or x = y for the
// last j when xs == ys.
struct Cat {
    int32_t occ[KMAX];
    int32_t tab[KMAX];          // string table of (subspace k, occ[k])
    int64_t count[KMAX];        // strings per subspace
    int64_t stride[KMAX];       // row-major strides over local ranks
    int64_t size;               // number of determinants
    int64_t offset;             // vector offset (space categories) or -1
    int64_t jbegin;             // first index in the intermediate enumeration, -1 if none
    int32_t in_space;
    int32_t deg;                // moves into the space from one determinant
    int32_t ncls;
    int32_t cls_code[NCLS];     // xs*K + ys
    int32_t cls_width[NCLS];    // (m_xs - n_xs) + (xs == ys)
    int32_t cls_begin[NCLS + 1];
    int32_t cls_target[NCLS];   // category index reached
    int32_t cls_phase[NCLS];    // 0/1: parity of electrons passed between subspaces
};

// One pair-intermediate category: an (N-2)-electron occupation tuple
// (n'_1..n'_K), any 0 <= n'_k <= m_k, from which creating a pair of electrons
// p < r reaches the space.  Pair class c creates p in subspace cls_a[c] and r
// in subspace cls_b[c] >= cls_a[c]; its slots are listed in pslot[slot_off ..
// slot_off + deg) as cls | i << 8 | j << 16 with p = i-th and r = j-th empty
// orbital of their subspaces (i < j inside one subspace), p fastest.
struct PairCat {
    int32_t occ[KMAX];
    int32_t tab[KMAX];          // string table of (subspace k, occ[k])
    int64_t count[KMAX];
    int64_t stride[KMAX];
    int64_t size;
    int32_t deg;                // pair creations into the space
    int32_t ncls;
    int32_t slot_off;           // into pslot[]
    int32_t pad_;
    int32_t cls_a[NPCLS];
    int32_t cls_b[NPCLS];
    int32_t cls_begin[NPCLS + 1];
    int32_t cls_target[NPCLS];  // space category reached
    int32_t cls_phase[NPCLS];   // 0/1: parity of the electrons of subspaces a..b-1 (a < b)
};

struct Space {
    int32_t K, M, N;
    int32_t sub_off[KMAX];
    int32_t sub_m[KMAX];
    int32_t ncat;               // all categories (space first, then intermediates)
    int32_t nspace;             // number of space categories
    int32_t nwork;              // categories with deg > 0 (intermediates of the 2e sum)
    int64_t ndets;              // determinants in the space
    int64_t nwork_dets;         // determinants over all work categories
    int32_t npcat;              // pair-intermediate categories (N >= 2)
    int32_t npairs;             // M (M - 1) / 2 ordered orbital pairs p < r
    int64_t npwork_dets;        // determinants over all pair-intermediate categories
};

// One item of the grouped pair kernel (spaces of one subspace): up to GRP_U
// intermediates K' (ranks j, -1 past n) that each add one electron to the
// (N-3)-electron core.
constexpr int GRP_U = 8;
struct GrpItem {
    uint32_t core;   // occupation bits of the core
    int32_t n;
    int32_t j[GRP_U];
};

// Spectator-batched pair kernel (spaces of several subspaces): the pair
// intermediates K' of one pair category that share their strings on the
// leading subspaces 1..K-1 form a group; they differ only in the string of
// the last subspace L = K (the fastest index of every block, so consecutive
// members reach consecutive target addresses through the same pair).  The
// rows of a group's product are its padded pair list: per usable pair class,
// the pairs of empty orbitals of the leading subspaces and of every orbital
// of subspace L (a pair holding an orbital occupied in a member contributes
// zero for that member).  sbrow[] holds the padded list of each pair
// category as cls | i << 8 | j << 16, i (j) the index of p (r) among the
// empties of its subspace, or the local orbital when the subspace is L.
// An item is one group and a span of its members (column chunk); CW =
// columns per member (1, 2 or 4) selects the chunking, index log2(CW).
struct SbCat {
    int32_t w;             // pair category
    int32_t npad;          // padded rows
    int32_t row_off;       // first entry in sbrow[]
    int32_t count_L;       // members per group (strings of subspace L)
    int64_t ngroups;
};

// A stream: the items of one column chunk of every group of one pair
// category (ngroups items, the chunk's column-group count fixed).  The
// streams of one (log2(CW), column-group count) pair are listed together,
// so that one launch handles items of one shape.
struct SbStream {
    int32_t cat;           // index into the SbCat array
    int32_t chunk;         // column chunk of the groups
    int64_t item_begin;    // first item of the stream within its list
};

struct SbPlan {
    const SbCat* cats;
    const uint32_t* rows;
    const SbStream* streams;
    int32_t ncat;
    int32_t cap;           // largest padded row count rounded up to 32
    int32_t nlmax;         // largest electron count of subspace L over the pair categories
    int32_t pad_;
    int32_t sbegin[3][9];  // streams of (log2(CW), column groups g = 1..8): [sbegin[x][g-1], sbegin[x][g])
    int64_t nitems[3][8];  // items of (log2(CW), column groups g = 1..8) at [x][g-1]
};

// Device view passed by value to kernels.
struct DevSpace {
    Space sp;
    const Cat* cats;
    const StrTab* tabs;
    const uint32_t* bits;
    const int32_t* ann;
    const int32_t* cre;
    const int32_t* work_cat;     // [nwork] category index
    const int64_t* work_begin;   // [nwork + 1] prefix over sizes
    const int64_t* space_begin;  // [nspace + 1] vector offsets
    const PairCat* pcats;        // [npcat]
    const int64_t* pwork_begin;  // [npcat + 1] prefix over sizes
    const uint32_t* pslot;       // slot tables of the pair categories
};

// Schedule of the tiled two-electron kernel: blocks of consecutive
// determinants of one intermediate category, times groups of annihilated
// orbitals y' (ygroup[orbital] = group id).
struct Sigma2eBlock {
    int32_t cat;
    int32_t count;
    int64_t j0;
};

struct Sigma2eSched {
    const Sigma2eBlock* blocks;
    const int32_t* ygroup;
    int32_t nblocks;
    int32_t ngroups;
    int32_t max_tot;   // largest count * deg over the blocks
    int32_t max_nj;    // largest count
};

}  // namespace stp
