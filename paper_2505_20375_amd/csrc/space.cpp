// Categorical STP-DAS space: partition into distributed active spaces,
// occupation categories (Results section, Fig. 2A, categorical vector
// C = (+)_B C^B), local string ranks and the factorised one-electron
// excitation tables (the "categorical one-electron excitation lists" of the
// sigma equations), plus the algorithmic work counts used for reporting.
#include "space.hpp"

#include <algorithm>
#include <map>
#include <sstream>

namespace stp {

static int64_t binom(int n, int k) {
    if (k < 0 || k > n) return 0;
    int64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// C(n, k) for 0 <= n <= 32, 0 <= k <= 34 (0 for k > n).
struct BinomTable {
    int64_t v[33][35];
    BinomTable() {
        for (int n = 0; n <= 32; ++n)
            for (int k = 0; k <= 34; ++k) v[n][k] = binom(n, k);
    }
};
static const BinomTable kBinom;

int64_t colex_rank(uint32_t mask) {
    int64_t r = 0;
    int i = 0;
    while (mask) {
        int b = __builtin_ctz(mask);
        r += kBinom.v[b][i + 1];
        ++i;
        mask &= mask - 1;
    }
    return r;
}

int HostSpace::find_cat(const int* occ) const {
    for (size_t c = 0; c < cats.size(); ++c) {
        bool eq = true;
        for (int k = 0; k < sp.K; ++k)
            if (cats[c].occ[k] != occ[k]) { eq = false; break; }
        if (eq) return (int)c;
    }
    return -1;
}

static void enum_tuples(int K, const int* m, const int* lo, const int* hi, int N,
                        std::vector<std::vector<int>>& out) {
    std::vector<int> cur(K, 0);
    std::function<void(int, int)> rec;
    rec = [&](int k, int left) {
        if (k == K) {
            if (left == 0) out.push_back(cur);
            return;
        }
        int a = std::max(lo[k], 0), b = std::min(std::min(hi[k], m[k]), left);
        for (int n = a; n <= b; ++n) {
            cur[k] = n;
            rec(k + 1, left - n);
        }
    };
    rec(0, N);
}

bool HostSpace::build(int n_elec, int n_sub, const int* sub_size, const int* win_lo,
                      const int* win_hi, std::string& err) {
    std::ostringstream es;
    if (n_sub < 1 || n_sub > KMAX) { es << "n_sub must be in [1," << KMAX << "]"; err = es.str(); return false; }
    int M = 0;
    for (int k = 0; k < n_sub; ++k) {
        if (sub_size[k] < 1 || sub_size[k] > MSUB) {
            es << "subspace " << k << " size must be in [1," << MSUB << "]"; err = es.str(); return false;
        }
        if (win_lo[k] > win_hi[k]) { es << "empty window in subspace " << k; err = es.str(); return false; }
        M += sub_size[k];
    }
    if (M > MMAX) { es << "at most " << MMAX << " spin-orbitals"; err = es.str(); return false; }
    if (n_elec < 1 || n_elec > M) { es << "n_elec must be in [1," << M << "]"; err = es.str(); return false; }
    sp = Space{};
    sp.K = n_sub; sp.M = M; sp.N = n_elec;
    lo.assign(win_lo, win_lo + n_sub);
    hi.assign(win_hi, win_hi + n_sub);
    int off = 0;
    for (int k = 0; k < n_sub; ++k) { sp.sub_off[k] = off; sp.sub_m[k] = sub_size[k]; off += sub_size[k]; }
    const int K = n_sub;

    // space categories (lexicographic) and their one-move neighbours
    std::vector<std::vector<int>> space_t, all_t;
    enum_tuples(K, sub_size, win_lo, win_hi, n_elec, space_t);
    if (space_t.empty()) { err = "no occupation pattern satisfies the windows"; return false; }
    std::vector<int> zlo(K, 0), zhi(sub_size, sub_size + K);
    enum_tuples(K, sub_size, zlo.data(), zhi.data(), n_elec, all_t);
    auto in_space = [&](const std::vector<int>& t) {
        for (int k = 0; k < K; ++k) if (t[k] < win_lo[k] || t[k] > win_hi[k]) return false;
        return true;
    };
    std::vector<std::vector<int>> inter_t;
    for (auto& t : all_t) {
        if (in_space(t)) continue;
        bool reach = false;
        for (int xs = 0; xs < K && !reach; ++xs)
            for (int ys = 0; ys < K && !reach; ++ys) {
                if (xs == ys) continue;
                // t = B + e_xs - e_ys  <=>  B = t - e_xs + e_ys
                std::vector<int> b = t;
                b[xs] -= 1; b[ys] += 1;
                if (b[xs] < 0 || b[ys] > sub_size[ys]) continue;
                if (in_space(b)) reach = true;
            }
        if (reach) inter_t.push_back(t);
    }

    cats.clear();
    auto make_cat = [&](const std::vector<int>& t, bool insp) {
        Cat c{};
        for (int k = 0; k < KMAX; ++k) { c.occ[k] = 0; c.tab[k] = -1; c.count[k] = 1; c.stride[k] = 0; }
        int64_t s = 1;
        for (int k = K - 1; k >= 0; --k) {
            c.occ[k] = t[k];
            c.count[k] = binom(sub_size[k], t[k]);
            c.stride[k] = s;
            s *= c.count[k];
        }
        c.size = s;
        c.in_space = insp ? 1 : 0;
        c.offset = -1;
        c.jbegin = -1;
        return c;
    };
    for (auto& t : space_t) cats.push_back(make_cat(t, true));
    for (auto& t : inter_t) cats.push_back(make_cat(t, false));
    sp.ncat = (int)cats.size();
    sp.nspace = (int)space_t.size();
    int64_t o = 0;
    space_begin.assign(1, 0);
    for (int c = 0; c < sp.nspace; ++c) { cats[c].offset = o; o += cats[c].size; space_begin.push_back(o); }
    sp.ndets = o;

    // move classes
    std::map<std::vector<int>, int> idx;
    for (int c = 0; c < sp.ncat; ++c) idx[std::vector<int>(cats[c].occ, cats[c].occ + K)] = c;
    max_deg = 0;
    for (int c = 0; c < sp.ncat; ++c) {
        Cat& C = cats[c];
        C.ncls = 0;
        int begin = 0;
        for (int xs = 0; xs < K; ++xs)
            for (int ys = 0; ys < K; ++ys) {
                std::vector<int> t(C.occ, C.occ + K);
                int ny = t[ys];
                int width = (sub_size[xs] - t[xs]) + (xs == ys ? 1 : 0);
                if (ny < 1 || width < 1) continue;
                if (xs != ys) {
                    if (t[xs] >= sub_size[xs]) continue;
                    t[xs] += 1; t[ys] -= 1;
                }
                if (!in_space(t)) continue;
                auto it = idx.find(t);
                if (it == idx.end()) continue;  // cannot happen: space categories are all listed
                int j = C.ncls++;
                C.cls_code[j] = xs * K + ys;
                C.cls_width[j] = width;
                C.cls_begin[j] = begin;
                C.cls_target[j] = it->second;
                // parity of electrons passed: sum_{k<ys} n_k(C) + sum_{k<xs} n_k(C - e_ys)
                int par = 0;
                if (xs != ys) {
                    for (int k = 0; k < ys; ++k) par += C.occ[k];
                    for (int k = 0; k < xs; ++k) par += C.occ[k] - (k == ys ? 1 : 0);
                }
                C.cls_phase[j] = par & 1;
                begin += ny * width;
            }
        C.cls_begin[C.ncls] = begin;
        C.deg = begin;
        max_deg = std::max(max_deg, begin);
    }

    // work categories (intermediates of the two-electron resolution)
    work_cat.clear();
    work_begin.assign(1, 0);
    int64_t w = 0;
    for (int c = 0; c < sp.ncat; ++c) {
        if (cats[c].deg <= 0) continue;
        cats[c].jbegin = w;
        work_cat.push_back(c);
        w += cats[c].size;
        work_begin.push_back(w);
    }
    sp.nwork = (int)work_cat.size();
    sp.nwork_dets = w;

    // pair intermediates: every (N-2)-electron tuple from which a pair
    // creation p < r (both in subspace a = b, or p in a < r in b) reaches the
    // space; windows do not apply to the intermediates themselves
    pcats.clear();
    pwork_begin.assign(1, 0);
    pslot.clear();
    Wp = sum_pdeg = 0;
    pmax_deg = 0;
    if (n_elec >= 2) {
        std::vector<std::vector<int>> pt;
        enum_tuples(K, sub_size, zlo.data(), zhi.data(), n_elec - 2, pt);
        int64_t pw = 0;
        for (auto& t : pt) {
            PairCat P{};
            for (int k = 0; k < KMAX; ++k) { P.occ[k] = 0; P.tab[k] = -1; P.count[k] = 1; P.stride[k] = 0; }
            int64_t sz = 1;
            for (int k = K - 1; k >= 0; --k) {
                P.occ[k] = t[k];
                P.count[k] = binom(sub_size[k], t[k]);
                P.stride[k] = sz;
                sz *= P.count[k];
            }
            P.size = sz;
            int begin = 0;
            P.ncls = 0;
            for (int a = 0; a < K; ++a)
                for (int b = a; b < K; ++b) {
                    const int va = sub_size[a] - t[a], vb = sub_size[b] - t[b];
                    const int cnt = (a == b) ? va * (va - 1) / 2 : va * vb;
                    if (cnt <= 0) continue;
                    std::vector<int> u = t;
                    u[a] += 1;
                    u[b] += 1;
                    if (!in_space(u)) continue;
                    auto it = idx.find(u);
                    if (it == idx.end()) continue;
                    const int c = P.ncls++;
                    P.cls_a[c] = a;
                    P.cls_b[c] = b;
                    P.cls_begin[c] = begin;
                    P.cls_target[c] = it->second;
                    int par = 0;
                    for (int k = a; k < b; ++k) par += t[k];
                    P.cls_phase[c] = par & 1;
                    begin += cnt;
                }
            P.cls_begin[P.ncls] = begin;
            P.deg = begin;
            if (begin == 0) continue;
            P.slot_off = (int32_t)pslot.size();
            for (int c = 0; c < P.ncls; ++c) {
                const int a = P.cls_a[c], b = P.cls_b[c];
                const int va = sub_size[a] - t[a], vb = sub_size[b] - t[b];
                if (a == b) {
                    for (int j = 1; j < va; ++j)
                        for (int i = 0; i < j; ++i) pslot.push_back((uint32_t)c | (uint32_t)i << 8 | (uint32_t)j << 16);
                } else {
                    for (int j = 0; j < vb; ++j)
                        for (int i = 0; i < va; ++i) pslot.push_back((uint32_t)c | (uint32_t)i << 8 | (uint32_t)j << 16);
                }
            }
            pcats.push_back(P);
            pw += sz;
            pwork_begin.push_back(pw);
            Wp += (double)sz * begin * begin;
            sum_pdeg += (double)sz * begin;
            pmax_deg = std::max(pmax_deg, begin);
        }
        sp.npwork_dets = pw;
    }
    sp.npcat = (int)pcats.size();
    sp.npairs = M * (M - 1) / 2;

    // string tables: which (m, n) need bits, ann, cre
    std::map<std::pair<int, int>, int> need;  // bit0 bits, bit1 ann, bit2 cre
    for (const PairCat& P : pcats) {
        for (int k = 0; k < K; ++k) {
            need[{sub_size[k], P.occ[k]}] |= 1 | 4;
            if (P.occ[k] < sub_size[k]) need[{sub_size[k], P.occ[k] + 1}] |= 1;
        }
        for (int c = 0; c < P.ncls; ++c) {
            const int a = P.cls_a[c];
            need[{sub_size[a], P.occ[a] + 1}] |= 1 | ((a == P.cls_b[c]) ? 4 : 0);
            if (a == P.cls_b[c]) need[{sub_size[a], P.occ[a] + 2}] |= 1;
            need[{sub_size[P.cls_b[c]], P.occ[P.cls_b[c]] + 1}] |= 1;
        }
    }
    for (int c = 0; c < sp.ncat; ++c) {
        const Cat& C = cats[c];
        for (int k = 0; k < K; ++k) need[{sub_size[k], C.occ[k]}] |= 1;
        for (int j = 0; j < C.ncls; ++j) {
            int xs = C.cls_code[j] / K, ys = C.cls_code[j] % K;
            need[{sub_size[ys], C.occ[ys]}] |= 2;
            need[{sub_size[ys], C.occ[ys] - 1}] |= 1;
            int nx = (xs == ys) ? C.occ[xs] - 1 : C.occ[xs];
            need[{sub_size[xs], nx}] |= 4 | 1;
            need[{sub_size[xs], nx + 1}] |= 1;
        }
    }
    int mmax = 0;
    for (int k = 0; k < K; ++k) mmax = std::max(mmax, sub_size[k]);
    tab_of.assign(mmax + 1, std::vector<int>(mmax + 2, -1));
    tabs.clear(); bits.clear(); ann.clear(); cre.clear();
    for (auto& kv : need) {
        int m = kv.first.first, n = kv.first.second;
        if (n < 0 || n > m) continue;
        StrTab T{};
        T.m = m; T.n = n; T.count = binom(m, n);
        T.bits_off = (int64_t)bits.size();
        T.ann_off = -1; T.cre_off = -1; T.tab_dn = -1; T.tab_up = -1;
        // masks with popcount n in ascending order (colex order)
        if (n == 0) {
            bits.push_back(0u);
        } else {
            uint32_t v = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
            for (int64_t r = 0; r < T.count; ++r) {
                bits.push_back(v);
                if (r + 1 < T.count) {  // next mask with the same popcount (Gosper's hack)
                    uint32_t t = v | (v - 1);
                    v = (t + 1) | (((~t & -~t) - 1) >> (__builtin_ctz(v) + 1));
                }
            }
        }
        tab_of[m][n] = (int)tabs.size();
        tabs.push_back(T);
    }
    for (auto& kv : need) {
        int m = kv.first.first, n = kv.first.second;
        if (n < 0 || n > m) continue;
        StrTab& T = tabs[tab_of[m][n]];
        if (n >= 1 && tab_of[m][n - 1] >= 0) T.tab_dn = tab_of[m][n - 1];
        if (n + 1 <= m && tab_of[m][n + 1] >= 0) T.tab_up = tab_of[m][n + 1];
        // ranks after removing or adding one electron from the colex sum
        // rank(s) = sum_i C(p_i, i + 1) over the set bits p_0 < p_1 < ...:
        // removing bit j leaves the bits below in place and moves those above
        // down one index; adding a bit at l with j bits below it moves the
        // bits from j on up one index (prefix and suffix sums per string)
        if ((kv.second & 2) && T.tab_dn >= 0) {
            T.ann_off = (int64_t)ann.size();
            ann.resize(ann.size() + (size_t)T.count * m, 0);
            int pos[32];
            int64_t pre[33], suf[33];
            for (int64_t r = 0; r < T.count; ++r) {
                const uint32_t s = bits[T.bits_off + r];
                int nb = 0;
                for (uint32_t t = s; t; t &= t - 1u) pos[nb++] = __builtin_ctz(t);
                pre[0] = 0;
                for (int i = 0; i < nb; ++i) pre[i + 1] = pre[i] + kBinom.v[pos[i]][i + 1];
                suf[nb] = 0;
                for (int i = nb - 1; i >= 0; --i) suf[i] = suf[i + 1] + kBinom.v[pos[i]][i];   // index i - 1 after removal
                for (int j = 0; j < nb; ++j) {
                    const int l = pos[j];
                    const int64_t r2 = pre[j] + suf[j + 1];
                    ann[T.ann_off + r * m + l] = (int32_t)((j & 1) ? -(r2 + 1) : (r2 + 1));
                }
            }
        }
        if ((kv.second & 4) && T.tab_up >= 0) {
            T.cre_off = (int64_t)cre.size();
            cre.resize(cre.size() + (size_t)T.count * m, 0);
            int pos[32];
            int64_t pre[33], suf[33];
            for (int64_t r = 0; r < T.count; ++r) {
                const uint32_t s = bits[T.bits_off + r];
                int nb = 0;
                for (uint32_t t = s; t; t &= t - 1u) pos[nb++] = __builtin_ctz(t);
                pre[0] = 0;
                for (int i = 0; i < nb; ++i) pre[i + 1] = pre[i] + kBinom.v[pos[i]][i + 1];
                suf[nb] = 0;
                for (int i = nb - 1; i >= 0; --i) suf[i] = suf[i + 1] + kBinom.v[pos[i]][i + 2];   // index i + 1 after insertion
                int j = 0;   // set bits below l
                for (int l = 0; l < m; ++l) {
                    if ((s >> l) & 1u) {
                        ++j;
                        continue;
                    }
                    const int64_t r2 = pre[j] + kBinom.v[l][j + 1] + suf[j];
                    cre[T.cre_off + r * m + l] = (int32_t)((j & 1) ? -(r2 + 1) : (r2 + 1));
                }
            }
        }
    }
    for (auto& C : cats)
        for (int k = 0; k < K; ++k) C.tab[k] = tab_of[sub_size[k]][C.occ[k]];
    for (auto& P : pcats)
        for (int k = 0; k < K; ++k) P.tab[k] = tab_of[sub_size[k]][P.occ[k]];

    // work counts
    W1 = W2 = nnz = sum_deg = 0;
    for (int c = 0; c < sp.ncat; ++c) {
        const Cat& C = cats[c];
        if (C.in_space) W1 += (double)C.size * C.deg;
        if (C.deg > 0) { W2 += (double)C.size * C.deg * C.deg; sum_deg += (double)C.size * C.deg; }
    }
    // nonzero couplings per row: 1 + singles + doubles landing in the space
    for (int c = 0; c < sp.nspace; ++c) {
        const Cat& A = cats[c];
        double singles = A.deg - sp.N;
        double doubles = 0;
        std::vector<int> t(A.occ, A.occ + K);
        for (int a = 0; a < K; ++a)
            for (int b = a; b < K; ++b) {
                double wy = (a == b) ? (double)t[a] * (t[a] - 1) / 2 : (double)t[a] * t[b];
                if (wy <= 0) continue;
                for (int cc = 0; cc < K; ++cc)
                    for (int d = cc; d < K; ++d) {
                        int vc = sub_size[cc] - t[cc], vd = sub_size[d] - t[d];
                        double wx = (cc == d) ? (double)vc * (vc - 1) / 2 : (double)vc * vd;
                        if (wx <= 0) continue;
                        std::vector<int> u = t;
                        u[a]--; u[b]--; u[cc]++; u[d]++;
                        bool ok = true;
                        for (int k = 0; k < K; ++k) if (u[k] < 0 || u[k] > sub_size[k]) ok = false;
                        if (!ok || !in_space(u)) continue;
                        doubles += wy * wx;
                    }
            }
        nnz += (double)A.size * (1.0 + singles + doubles);
    }
    return true;
}

bool HostSpace::address_to_det(int64_t addr, uint64_t* out) const {
    if (addr < 0 || addr >= sp.ndets) return false;
    int c = (int)(std::upper_bound(space_begin.begin(), space_begin.end(), addr) - space_begin.begin()) - 1;
    const Cat& C = cats[c];
    int64_t j = addr - C.offset;
    uint64_t b = 0;
    for (int k = 0; k < sp.K; ++k) {
        int64_t r = (j / C.stride[k]) % C.count[k];
        const StrTab& T = tabs[C.tab[k]];
        b |= (uint64_t)bits[T.bits_off + r] << sp.sub_off[k];
    }
    *out = b;
    return true;
}

int64_t HostSpace::det_to_address(uint64_t b) const {
    int occ[KMAX];
    uint32_t loc[KMAX];
    for (int k = 0; k < sp.K; ++k) {
        uint64_t mk = (sp.sub_m[k] >= 64) ? ~0ULL : ((1ULL << sp.sub_m[k]) - 1ULL);
        loc[k] = (uint32_t)((b >> sp.sub_off[k]) & mk);
        occ[k] = __builtin_popcount(loc[k]);
    }
    int c = find_cat(occ);
    if (c < 0 || !cats[c].in_space) return -1;
    const Cat& C = cats[c];
    int64_t a = C.offset;
    for (int k = 0; k < sp.K; ++k) a += colex_rank(loc[k]) * C.stride[k];
    return a;
}

}  // namespace stp
