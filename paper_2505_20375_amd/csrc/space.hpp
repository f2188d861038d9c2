// Host side of the categorical space: distributed active spaces (contiguous
// orbital subspaces), occupation categories, local string tables and the
// algorithmic work counts.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "stp_internal.hpp"

namespace stp {

struct HostSpace {
    Space sp{};
    std::vector<int> lo, hi;
    std::vector<Cat> cats;
    std::vector<StrTab> tabs;
    std::vector<uint32_t> bits;
    std::vector<int32_t> ann, cre;
    std::vector<int32_t> work_cat;
    std::vector<int64_t> work_begin;
    std::vector<int64_t> space_begin;
    // pair intermediates (N - 2 electrons) of the pair-resolved two-electron term
    std::vector<PairCat> pcats;
    std::vector<int64_t> pwork_begin;
    std::vector<uint32_t> pslot;
    // tab_of[m][n] -> table index (-1 if not built)
    std::vector<std::vector<int>> tab_of;
    // algorithmic counts (complex or real multiply-adds, couplings)
    double W1 = 0, W2 = 0, nnz = 0, sum_deg = 0;
    int max_deg = 0;
    // pair resolution: Wp = sum |K'| deg(K')^2 complex multiply-adds
    double Wp = 0, sum_pdeg = 0;
    int pmax_deg = 0;

    bool build(int n_elec, int n_sub, const int* sub_size, const int* win_lo, const int* win_hi,
               std::string& err);
    // global occupation bits of a space determinant
    bool address_to_det(int64_t addr, uint64_t* bits_out) const;
    // address of a determinant given as global occupation bits (-1 if outside)
    int64_t det_to_address(uint64_t b) const;
    int find_cat(const int* occ) const;
};

// colexicographic rank of a local mask among masks of equal popcount
int64_t colex_rank(uint32_t mask);

}  // namespace stp
