// C ABI of libstpci: context, integrals, space, sigma, diagonal, profiling.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <new>
#include <sstream>

#include "ctx.hpp"
#include "kernels.hpp"

using namespace stp;

stpci_ctx::~stpci_ctx() {
    if (!host_only) {
        (void)hipSetDevice(device);
        if (pin) (void)hipHostFree(pin);
        for (auto& e : events) {
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
        for (DevBuf* b : {&d_E, &d_csc_cnt, &d_csc_pcat, &d_csc_bitmap, &d_csc_list, &d_csc_count, &d_sbcats, &d_sbrows, &d_sbstreams, &d_grp, &d_pcats, &d_pwork, &d_pslot, &d_pA, &d_pA32, &d_pAbf, &d_gT32, &d_hp32, &d_s2blocks, &d_ygroup, &d_cats, &d_tabs, &d_bits, &d_ann, &d_cre, &d_work_cat, &d_work_begin, &d_space_begin,
                          &d_hp, &d_gT, &d_hd, &d_JK, &d_V, &d_W, &d_X, &d_T, &d_partial, &d_small, &d_topv,
                          &d_topi})
            b->free_();
    }
}

namespace stp {

stpci_status set_err(stpci_ctx* c, stpci_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

stpci_status hip_check(stpci_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return STPCI_OK;
    std::ostringstream o;
    o << what << ": " << hipGetErrorString(e);
    return set_err(c, e == hipErrorOutOfMemory ? STPCI_ENOMEM : STPCI_EHIP, o.str());
}

size_t scalar_bytes(const stpci_ctx* c) { return c->cplx ? 16 : 8; }

stpci_status ensure(stpci_ctx* c, DevBuf& b, size_t bytes, const char* what) {
    if (b.bytes >= bytes && b.p) return STPCI_OK;
    b.free_();
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        std::ostringstream o;
        o << "device allocation of " << bytes << " bytes for " << what << " failed";
        return set_err(c, STPCI_ENOMEM, o.str());
    }
    b.bytes = bytes;
    return STPCI_OK;
}

template <class T>
static stpci_status upload(stpci_ctx* c, DevBuf& b, const std::vector<T>& v, const char* what) {
    size_t bytes = v.size() * sizeof(T);
    stpci_status s = ensure(c, b, bytes, what);
    if (s) return s;
    if (bytes) return hip_check(c, hipMemcpy(b.p, v.data(), bytes, hipMemcpyHostToDevice), what);
    return STPCI_OK;
}

// Pair-pair table of the pair kernel: A[(p,r),(q,s)] = g'_pqrs - g'_psrq for
// p < r, q < s, g'_pqrs = (pq|rs) + (h_pq d_rs + d_pq h_rs) / (N - 1), stored
// as pA[pair(q,s) * npairs + pair(p,r)], pair(p,r) = r (r - 1) / 2 + p.
static void build_pair_table(stpci_ctx* c) {
    const int M = c->M, N = c->hs.sp.N;
    const int w = c->cplx ? 2 : 1;
    const size_t NP = (size_t)M * (M - 1) / 2;
    const double f = 1.0 / (double)(N - 1);
    auto gp = [&](int p, int q, int r, int s, int k) {
        double v = c->g[((((size_t)p * M + q) * M + r) * M + s) * w + k];
        if (r == s) v += f * c->h[((size_t)p * M + q) * w + k];
        if (p == q) v += f * c->h[((size_t)r * M + s) * w + k];
        return v;
    };
    c->pA.assign(NP * NP * w, 0.0);
    for (int r = 1; r < M; ++r)
        for (int p = 0; p < r; ++p) {
            const size_t P = (size_t)r * (r - 1) / 2 + p;
            for (int s = 1; s < M; ++s)
                for (int q = 0; q < s; ++q) {
                    const size_t Q = (size_t)s * (s - 1) / 2 + q;
                    for (int k = 0; k < w; ++k) c->pA[(Q * NP + P) * w + k] = gp(p, q, r, s, k) - gp(p, s, r, q, k);
                }
        }
    c->pA32.assign(c->pA.begin(), c->pA.end());
    // bfloat16 copy for the matrix-core form: row-major [P][Q] = A[P, Q]
    // (= pA[Q * NP + P]) padded to npp columns and rows; complex tables hold
    // the real part, the imaginary part and its negation
    const size_t npp = (size_t)pair_mfma_npp((int)NP);
    const int nm = c->cplx ? 3 : 1;
    c->pAbf.assign(nm * npp * npp, 0);
    auto bf = [](double x) {
        const float f = (float)x;
        uint32_t u;
        std::memcpy(&u, &f, 4);
        u += 0x7fffu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    };
    for (size_t P = 0; P < NP; ++P)
        for (size_t Q = 0; Q < NP; ++Q) {
            const double* a = &c->pA[(Q * NP + P) * w];
            c->pAbf[P * npp + Q] = bf(a[0]);
            if (c->cplx) {
                c->pAbf[npp * npp + P * npp + Q] = bf(a[1]);
                c->pAbf[2 * npp * npp + P * npp + Q] = bf(-a[1]);
            }
        }
}

// Sigma kernel prepare() selects for this context.
int select_kernel(const stpci_ctx* c) {
    const HostSpace& H = c->hs;
    // 1: the row-tiled one-move kernel (any degree), 3: the Hermitian-tile
    // one-move kernel, 4: the pair form (0 and 2 are unused numbers)
    const bool ok[5] = {false, true, false, symtile_supported(H.max_deg, c->cplx),
                        pair_supported(H.sp.N, H.pmax_deg, c->cplx)};
    if (c->kernel_req >= 0) {
        // 4..9: the pair form (automatic unit; with device atomics; on the FP64
        // matrix cores; on the vector ALUs; grouped intermediates on the FP64
        // matrix cores; spectator-batched groups on the FP64 matrix cores)
        const int k = (c->kernel_req >= 4) ? 4 : c->kernel_req;
        if (c->kernel_req == 6 && !pair_mf64_supported(H.sp.N, H.pmax_deg)) return -1;
        if (c->kernel_req == 8 && !(ok[4] && pair_grp_supported(H.sp))) return -1;
        if (c->kernel_req == 9 && !(H.sp.N >= 2 && pair_sb_supported(H.sp))) return -1;
        if (c->kernel_req == 9) return 4;
        return ok[k] ? k : -1;
    }
    return ok[4] ? 4 : (ok[3] ? 3 : 1);
}

// Device bytes of the tables and integrals prepare() (and, for FP32, ensure32())
// uploads; mirrors the uploads below.
int64_t device_table_bytes(const stpci_ctx* c, bool f32) {
    const HostSpace& H = c->hs;
    const int k = select_kernel(c);
    const int64_t sb = (int64_t)scalar_bytes(c);
    int64_t b = (int64_t)(H.cats.size() * sizeof(Cat) + H.tabs.size() * sizeof(StrTab));
    b += (int64_t)(H.bits.size() + H.ann.size() + H.cre.size() + H.work_cat.size()) * 4;
    b += (int64_t)(H.work_begin.size() + H.space_begin.size()) * 8;
    b += (int64_t)(c->hd.size() + c->JK.size()) * 8;
    const int64_t M = c->M, NP = M * (M - 1) / 2;
    if (k == 4) {
        b += (int64_t)(H.pcats.size() * sizeof(PairCat) + H.pwork_begin.size() * 8 + H.pslot.size() * 4);
        b += NP * NP * sb * (f32 ? 3 : 2) / 2;
    } else {
        b += (M * M + M * M * M * M) * sb * (f32 ? 3 : 2) / 2;
        if (k == 1) b += H.sp.nwork_dets * 16 + M * 4;  // row-tile schedule (upper bound)
    }
    return b;
}

stpci_status prepare(stpci_ctx* c) {
    if (c->host_only) return set_err(c, STPCI_ESTATE, "host-only context has no device");
    if (!c->have_ints) return set_err(c, STPCI_ESTATE, "integrals not set");
    if (!c->have_space) return set_err(c, STPCI_ESTATE, "space not set");
    if (c->prepared) return STPCI_OK;
    if (c->hs.sp.M != c->M) {
        std::ostringstream o;
        o << "space covers " << c->hs.sp.M << " spin-orbitals but the integrals have " << c->M;
        return set_err(c, STPCI_EINVAL, o.str());
    }
    stpci_status s;
    if ((s = hip_check(c, hipSetDevice(c->device), "hipSetDevice"))) return s;
    HostSpace& H = c->hs;
    if ((s = upload(c, c->d_cats, H.cats, "categories"))) return s;
    if ((s = upload(c, c->d_tabs, H.tabs, "string tables"))) return s;
    if ((s = upload(c, c->d_bits, H.bits, "string masks"))) return s;
    if ((s = upload(c, c->d_ann, H.ann, "annihilation table"))) return s;
    if ((s = upload(c, c->d_cre, H.cre, "creation table"))) return s;
    if ((s = upload(c, c->d_work_cat, H.work_cat, "work categories"))) return s;
    if ((s = upload(c, c->d_work_begin, H.work_begin, "work offsets"))) return s;
    if ((s = upload(c, c->d_space_begin, H.space_begin, "space offsets"))) return s;
    if ((s = upload(c, c->d_hd, c->hd, "diagonal integrals"))) return s;
    if ((s = upload(c, c->d_JK, c->JK, "Coulomb-exchange integrals"))) return s;
    // sigma kernel: the requested one, else pair intermediates where they apply
    {
        const int k = select_kernel(c);
        if (k < 0) return set_err(c, STPCI_EINVAL, "the requested sigma kernel does not support this space");
        c->s2_kernel = k;
    }
    if (c->s2_kernel == 4) {
        // scatter: store-and-reduce when its workspace fits a quarter of the
        // free device memory (or 1 GB), device atomics otherwise
        size_t fr = 0, tot = 0;
        (void)hipMemGetInfo(&fr, &tot);
        DevSpace tmp{};
        tmp.sp = H.sp;
        const size_t eb = pair_store_bytes(tmp, c->cplx);
        c->pair_store = c->kernel_req != 5 && (eb <= ((size_t)1 << 30) || eb <= fr / 4);
        // FP64 products on the matrix cores where the pair table stays in one
        // XCD's L2 (they read both triangles of each tile); the vector-ALU
        // kernel reads one triangle and wins when the table spills to the MALL
        const size_t table = (size_t)H.sp.npairs * H.sp.npairs * scalar_bytes(c);
        const bool auto_unit = c->kernel_req < 0 || c->kernel_req == 4 || c->kernel_req == 5;
        c->pair_mf64 = pair_mf64_supported(H.sp.N, H.pmax_deg) &&
                       (c->kernel_req == 6 || (auto_unit && table <= ((size_t)4 << 20)));
        // spaces of one subspace: eight (or four) intermediates per table read
        c->pair_grp = false;
        c->grp_items.clear();
        // (the grouped kernel keeps targets as 32-bit words: target << 1 | sign)
        const int64_t nq = (int64_t)H.sp.N * (H.sp.N - 1) / 2;
        const bool grp_fits = (c->pair_store ? H.sp.ndets * nq : H.sp.ndets) < ((int64_t)1 << 30);
        if (c->kernel_req == 8 || (auto_unit && grp_fits && pair_grp_supported(H.sp))) {
            c->pair_grp = grp_fits && build_pair_groups(H, c->grp_items);
            if (!c->pair_grp && c->kernel_req == 8)
                return set_err(c, STPCI_EINVAL, "the grouped pair kernel does not support this space");
            if (c->pair_grp && (s = upload(c, c->d_grp, c->grp_items, "pair groups"))) return s;
        }
        // spaces of several subspaces: the members of a group (pair
        // intermediates sharing the strings of subspaces 1..K-1) contracted
        // as one product, where the table does not fit the L2 of an XCD
        c->pair_sb = false;
        if (c->kernel_req == 9 || (auto_unit && !c->pair_grp && !c->pair_mf64 && pair_sb_supported(H.sp))) {
            SbHostPlan pl;
            c->pair_sb = build_sb_plan(H, pl) && pair_sb_lds_bytes(pl.cap, pl.nlmax) <= 160 * 1024;
            if (!c->pair_sb && c->kernel_req == 9)
                return set_err(c, STPCI_EINVAL, "the spectator-batched pair kernel does not support this space");
            if (c->pair_sb) {
                if ((s = upload(c, c->d_sbcats, pl.cats, "batched pair categories"))) return s;
                if ((s = upload(c, c->d_sbrows, pl.rows, "batched pair rows"))) return s;
                if ((s = upload(c, c->d_sbstreams, pl.streams, "batched pair streams"))) return s;
                SbPlan& P = c->sb_plan;
                P.cats = (const SbCat*)c->d_sbcats.p;
                P.rows = (const uint32_t*)c->d_sbrows.p;
                P.streams = (const SbStream*)c->d_sbstreams.p;
                P.ncat = (int32_t)pl.cats.size();
                P.cap = pl.cap;
                P.nlmax = pl.nlmax;
                std::memcpy(P.sbegin, pl.sbegin, sizeof(P.sbegin));
                std::memcpy(P.nitems, pl.nitems, sizeof(P.nitems));
                c->pair_store = false;   // contributions go to sigma with device atomics
            }
        }
        build_pair_table(c);
        if ((s = upload(c, c->d_pcats, H.pcats, "pair categories"))) return s;
        if ((s = upload(c, c->d_pwork, H.pwork_begin, "pair offsets"))) return s;
        if ((s = upload(c, c->d_pslot, H.pslot, "pair slots"))) return s;
        if ((s = upload(c, c->d_pA, c->pA, "pair-pair integrals"))) return s;
    } else {
        if ((s = upload(c, c->d_hp, c->hprime, "h'"))) return s;
        if ((s = upload(c, c->d_gT, c->gT, "two-electron integrals"))) return s;
    }
    if (c->s2_kernel == 1) {
        int ngroups = 0;
        if (const char* g = getenv("STPCI_S2_GROUPS")) ngroups = atoi(g);
        if (ngroups <= 0) {
            // integrals touched by one group of rows should fit a quarter of an XCD's L2 (4 MB)
            double gbytes = (double)H.sp.M * H.sp.M * H.sp.M * H.sp.M * scalar_bytes(c);
            ngroups = 1;
            while (ngroups < 8 && gbytes / ngroups > 1.5e6) ngroups *= 2;
        }
        ngroups = std::max(1, std::min(ngroups, H.sp.M));
        size_t budget = 60 * 1024;  // dynamic LDS per workgroup (the kernel adds ~1.3 KB static)
        if (const char* b = getenv("STPCI_S2_LDS_KB")) budget = (size_t)atoi(b) * 1024;
        const size_t per_move = 2 * scalar_bytes(c) + 8 + 4 + 4 + 4;
        std::vector<Sigma2eBlock> blocks;
        int max_tot = 0, max_nj = 0;
        for (int w = 0; w < H.sp.nwork; ++w) {
            const Cat& C = H.cats[H.work_cat[w]];
            int nj = (int)std::max<int64_t>(1, (int64_t)(budget / (per_move * C.deg + DET_BYTES)));
            nj = std::min(nj, 4096);
            for (int64_t j0 = 0; j0 < C.size; j0 += nj) {
                int cnt = (int)std::min<int64_t>(nj, C.size - j0);
                blocks.push_back(Sigma2eBlock{H.work_cat[w], cnt, j0});
                max_tot = std::max(max_tot, cnt * C.deg);
                max_nj = std::max(max_nj, cnt);
            }
        }
        std::vector<int32_t> yg(H.sp.M);
        for (int o = 0; o < H.sp.M; ++o) yg[o] = (int32_t)((int64_t)o * ngroups / H.sp.M);
        if ((s = upload(c, c->d_s2blocks, blocks, "sigma2e schedule"))) return s;
        if ((s = upload(c, c->d_ygroup, yg, "row groups"))) return s;
        c->s2.blocks = (const Sigma2eBlock*)c->d_s2blocks.p;
        c->s2.ygroup = (const int32_t*)c->d_ygroup.p;
        c->s2.nblocks = (int32_t)blocks.size();
        c->s2.ngroups = ngroups;
        c->s2.max_tot = max_tot;
        c->s2.max_nj = max_nj;
    }
    DevSpace& D = c->dev;
    D.sp = H.sp;
    D.cats = (const Cat*)c->d_cats.p;
    D.tabs = (const StrTab*)c->d_tabs.p;
    D.bits = (const uint32_t*)c->d_bits.p;
    D.ann = (const int32_t*)c->d_ann.p;
    D.cre = (const int32_t*)c->d_cre.p;
    D.work_cat = (const int32_t*)c->d_work_cat.p;
    D.work_begin = (const int64_t*)c->d_work_begin.p;
    D.space_begin = (const int64_t*)c->d_space_begin.p;
    D.pcats = (const PairCat*)c->d_pcats.p;
    D.pwork_begin = (const int64_t*)c->d_pwork.p;
    D.pslot = (const uint32_t*)c->d_pslot.p;
    c->have32 = false;   // the reduced-precision copies follow the tables rebuilt above
    c->have_bf = false;
    c->prepared = true;
    return STPCI_OK;
}

static void record(stpci_ctx* c, int kind, bool start) {
    if (!c->profile) return;
    if (start) {
        KernelEvent e{kind, nullptr, nullptr};
        (void)hipEventCreate(&e.a);
        (void)hipEventCreate(&e.b);
        (void)hipEventRecord(e.a, c->stream);
        c->events.push_back(e);
    } else {
        (void)hipEventRecord(c->events.back().b, c->stream);
    }
}

stpci_status ensure_bf16(stpci_ctx* c) {
    if (c->have_bf) return STPCI_OK;
    stpci_status s = upload(c, c->d_pAbf, c->pAbf, "bfloat16 pair-pair integrals");
    if (s) return s;
    c->have_bf = true;
    return STPCI_OK;
}

stpci_status ensure32(stpci_ctx* c) {
    if (c->have32) return STPCI_OK;
    stpci_status s;
    if (c->s2_kernel == 4) {
        if ((s = upload(c, c->d_pA32, c->pA32, "FP32 pair-pair integrals"))) return s;
    } else {
        if ((s = upload(c, c->d_gT32, c->gT32, "FP32 two-electron integrals"))) return s;
        if ((s = upload(c, c->d_hp32, c->hp32, "FP32 h'"))) return s;
    }
    c->have32 = true;
    return STPCI_OK;
}

stpci_status sigma_impl(stpci_ctx* c, const void* cin, void* sout, int n_vec, stpci_precision prec, void* ws) {
    if (prec != STPCI_FP64 && prec != STPCI_FP32 && prec != STPCI_BF16)
        return set_err(c, STPCI_EINVAL, "unsupported sigma precision");
    const bool f32 = prec == STPCI_FP32;
    hipError_t e;
    if (prec == STPCI_BF16) {
        // pair products on the matrix cores (bfloat16 operands, FP32 accumulation)
        if (c->s2_kernel != 4 || !pair_mfma_supported(c->dev, c->hs.pmax_deg, c->cplx))
            return set_err(c, STPCI_EINVAL, "the BF16 contraction needs the pair kernel within its LDS limits");
        stpci_status s = ensure_bf16(c);
        if (s) return s;
        struct Mark {
            stpci_ctx* c;
            static void fn(void* u, int what, bool start) {
                Mark* m = static_cast<Mark*>(u);
                record(m->c, what == 0 ? 4 : 3, start);
            }
        } mark{c};
        const LaunchMarks mk{&Mark::fn, &mark};
        void* E = ws;
        if (c->pair_store && !ws) {
            if ((s = ensure(c, c->d_E, pair_store_bytes(c->dev, c->cplx), "pair contribution workspace"))) return s;
            E = c->d_E.p;
        }
        if (!c->pair_store) E = nullptr;
        e = launch_sigma_pair_mfma(c->dev, c->hs.pmax_deg, c->cplx, c->d_pAbf.p, cin, sout, E, n_vec, c->e_core,
                                   c->profile ? &mk : nullptr, c->stream);
        return e == hipSuccess ? STPCI_OK : hip_check(c, e, "sigma launch");
    }
    if (f32) {
        // category-block contraction in FP32 (FP32 accumulation); sigma accumulated in FP64
        if (c->s2_kernel < 3) return set_err(c, STPCI_EINVAL, "the FP32 contraction needs a tile kernel");
        stpci_status s = ensure32(c);
        if (s) return s;
    }
    const int kind = f32 ? 2 : 1;
    if (c->s2_kernel == 4) {
        // events bracket the pair kernel (kind 1 or 2) and the reduce (kind 3) separately
        struct Mark {
            stpci_ctx* c;
            int kind;
            static void fn(void* u, int what, bool start) {
                Mark* m = static_cast<Mark*>(u);
                record(m->c, what == 0 ? m->kind : 3, start);
            }
        } mark{c, kind};
        const LaunchMarks mk{&Mark::fn, &mark};
        void* E = ws;
        if (c->pair_store && !ws) {
            stpci_status s = ensure(c, c->d_E, pair_store_bytes(c->dev, c->cplx), "pair contribution workspace");
            if (s) return s;
            E = c->d_E.p;
        }
        if (!c->pair_store) E = nullptr;
        if (c->pair_sb)
            e = launch_sigma_pair_sb(c->dev, c->sb_plan, c->cplx, f32, f32 ? c->d_pA32.p : c->d_pA.p, cin, sout,
                                     n_vec, c->e_core, c->profile ? &mk : nullptr, c->stream);
        else if (c->pair_grp)
            e = launch_sigma_pair_grp(c->dev, (const GrpItem*)c->d_grp.p, (int)c->grp_items.size(), c->cplx, f32,
                                      f32 ? c->d_pA32.p : c->d_pA.p, cin, sout, E, n_vec, c->e_core,
                                      c->profile ? &mk : nullptr, c->stream);
        else if (c->pair_mf64 && !f32)
            e = launch_sigma_pair_mf64(c->dev, c->hs.pmax_deg, c->cplx, c->d_pA.p, cin, sout, E, n_vec, c->e_core,
                                       c->profile ? &mk : nullptr, c->stream);
        else
            e = launch_sigma_pair(c->dev, c->hs.pmax_deg, c->cplx, f32, f32 ? c->d_pA32.p : c->d_pA.p, cin, sout,
                                  E, n_vec, c->e_core, c->profile ? &mk : nullptr, c->stream);
        return e == hipSuccess ? STPCI_OK : hip_check(c, e, "sigma launch");
    }
    if (c->s2_kernel == 3) {
        record(c, kind, true);
        e = launch_sigma_symtile(c->dev, c->hs.max_deg, c->cplx, f32, f32 ? c->d_gT32.p : c->d_gT.p,
                                 f32 ? c->d_hp32.p : c->d_hp.p, cin, sout, n_vec, c->e_core, c->stream);
        record(c, kind, false);
        return e == hipSuccess ? STPCI_OK : hip_check(c, e, "sigma launch");
    }
    // the row-tiled one-move kernel: one-electron part, then two-electron part
    record(c, 0, true);
    e = launch_sigma1e(c->dev, c->cplx, c->d_hp.p, cin, sout, n_vec, c->stream);
    record(c, 0, false);
    if (e != hipSuccess) return hip_check(c, e, "sigma1e launch");
    record(c, 1, true);
    e = launch_sigma2e_tiled(c->dev, c->s2, c->cplx, c->d_gT.p, cin, sout, n_vec, c->stream);
    record(c, 1, false);
    if (e != hipSuccess) return hip_check(c, e, "sigma launch");
    if (c->e_core != 0.0) {
        e = launch_axpy_core(c->cplx, sout, cin, c->e_core, c->hs.sp.ndets * n_vec, c->stream);
        if (e != hipSuccess) return hip_check(c, e, "e_core term");
    }
    return STPCI_OK;
}

}  // namespace stp

// ---------------------------------------------------------------------------
extern "C" {

stpci_status stpci_create(stpci_ctx** out, int hip_device, void* hip_stream) {
    if (!out) return STPCI_EINVAL;
    *out = nullptr;
    stpci_ctx* c = new (std::nothrow) stpci_ctx();
    if (!c) return STPCI_ENOMEM;
    if (hip_device >= 0) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess || hip_device >= n) {
            (void)hipGetLastError();
            delete c;
            return STPCI_EHIP;
        }
        if (hipSetDevice(hip_device) != hipSuccess) {
            delete c;
            return STPCI_EHIP;
        }
        // the no-allocation sigma's workspace: this device's address of the
        // library's static scratch array, resolved once per device
        if (scratch_setup(hip_device) != hipSuccess) {
            delete c;
            return STPCI_EHIP;
        }
        c->device = hip_device;
        c->host_only = false;
        c->stream = (hipStream_t)hip_stream;
    }
    *out = c;
    return STPCI_OK;
}

void stpci_destroy(stpci_ctx* ctx) { delete ctx; }

const char* stpci_last_error(const stpci_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

stpci_status stpci_set_integrals(stpci_ctx* c, int n_orb, stpci_scalar scalar, int spin_free, const void* h,
                                 const void* g, double e_core) {
    if (!c) return STPCI_EINVAL;
    if (!h || !g) return set_err(c, STPCI_EINVAL, "h and g must be non-NULL");
    if (scalar != STPCI_REAL64 && scalar != STPCI_COMPLEX128) return set_err(c, STPCI_EINVAL, "unknown scalar type");
    const int M = spin_free ? 2 * n_orb : n_orb;
    if (n_orb < 1 || M > MMAX) return set_err(c, STPCI_EINVAL, "n_orb out of range");
    const bool cplx = scalar == STPCI_COMPLEX128;
    const int n = n_orb;
    auto hin = [&](int p, int q, double& re, double& im) {
        const double* a = (const double*)h;
        if (cplx) { re = a[2 * (p * n + q)]; im = a[2 * (p * n + q) + 1]; }
        else { re = a[p * n + q]; im = 0.0; }
    };
    auto gin = [&](int p, int q, int r, int s, double& re, double& im) {
        const double* a = (const double*)g;
        size_t i = (((size_t)p * n + q) * n + r) * n + s;
        if (cplx) { re = a[2 * i]; im = a[2 * i + 1]; }
        else { re = a[i]; im = 0.0; }
    };
    // validation on the given (spatial or spin-orbital) arrays
    double hmax = 0, gmax = 0, hbad = 0, gbad = 0;
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) {
            double a, b, x, y;
            hin(p, q, a, b);
            hin(q, p, x, y);
            hmax = std::max(hmax, std::hypot(a, b));
            hbad = std::max(hbad, std::hypot(a - x, b + y));
        }
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r)
                for (int s = 0; s < n; ++s) {
                    double a, b, x, y, u, v;
                    gin(p, q, r, s, a, b);
                    gin(r, s, p, q, x, y);
                    gin(q, p, s, r, u, v);
                    gmax = std::max(gmax, std::hypot(a, b));
                    gbad = std::max(gbad, std::hypot(a - x, b - y));
                    gbad = std::max(gbad, std::hypot(a - u, b + v));
                }
    if (!(std::isfinite(hmax) && std::isfinite(gmax)))
        return set_err(c, STPCI_EINVAL, "integrals contain non-finite values");
    if (hbad > 1e-12 * std::max(1.0, hmax)) return set_err(c, STPCI_EINVAL, "h is not Hermitian");
    if (gbad > 1e-12 * std::max(1.0, gmax))
        return set_err(c, STPCI_EINVAL, "g violates (pq|rs) = (rs|pq) or (pq|rs) = conj((qp|sr))");

    // spin-orbital arrays (interleaved when complex)
    const int w = cplx ? 2 : 1;
    std::vector<double> H((size_t)M * M * w, 0.0), G((size_t)M * M * M * M * w, 0.0);
    auto spat = [&](int P, int& p, int& sp) { sp = spin_free ? P / n : 0; p = spin_free ? P % n : P; };
    for (int P = 0; P < M; ++P)
        for (int Q = 0; Q < M; ++Q) {
            int p, q, sp, sq;
            spat(P, p, sp);
            spat(Q, q, sq);
            if (sp != sq) continue;
            double a, b;
            hin(p, q, a, b);
            H[((size_t)P * M + Q) * w] = a;
            if (cplx) H[((size_t)P * M + Q) * w + 1] = b;
        }
    for (int P = 0; P < M; ++P)
        for (int Q = 0; Q < M; ++Q)
            for (int R = 0; R < M; ++R)
                for (int S = 0; S < M; ++S) {
                    int p, q, r, s, sp, sq, sr, ss;
                    spat(P, p, sp); spat(Q, q, sq); spat(R, r, sr); spat(S, s, ss);
                    if (sp != sq || sr != ss) continue;
                    double a, b;
                    gin(p, q, r, s, a, b);
                    size_t i = ((((size_t)P * M + Q) * M + R) * M + S) * w;
                    G[i] = a;
                    if (cplx) G[i + 1] = b;
                }
    c->M = M;
    c->cplx = cplx;
    c->e_core = e_core;
    c->h.swap(H);
    c->g.swap(G);
    // derived arrays
    const size_t MM = (size_t)M * M;
    c->hprime.assign(MM * w, 0.0);
    for (int p = 0; p < M; ++p)
        for (int q = 0; q < M; ++q)
            for (int k = 0; k < w; ++k) {
                double v = c->h[((size_t)p * M + q) * w + k];
                for (int r = 0; r < M; ++r) v -= 0.5 * c->g[((((size_t)p * M + r) * M + r) * M + q) * w + k];
                c->hprime[((size_t)p * M + q) * w + k] = v;
            }
    c->gT.assign(MM * MM * w, 0.0);
    for (int xp = 0; xp < M; ++xp)
        for (int yp = 0; yp < M; ++yp)
            for (int y = 0; y < M; ++y)
                for (int x = 0; x < M; ++x) {
                    size_t src = ((((size_t)xp * M + yp) * M + y) * M + x) * w;
                    size_t dst = (((size_t)y * M + x) * MM + ((size_t)yp * M + xp)) * w;
                    for (int k = 0; k < w; ++k) c->gT[dst + k] = c->g[src + k];
                }
    c->hd.assign(M, 0.0);
    c->JK.assign(MM, 0.0);
    for (int i = 0; i < M; ++i) {
        c->hd[i] = c->h[((size_t)i * M + i) * w];
        for (int j = 0; j < M; ++j) {
            double J = c->g[((((size_t)i * M + i) * M + j) * M + j) * w];
            double Kx = c->g[((((size_t)i * M + j) * M + j) * M + i) * w];
            c->JK[(size_t)i * M + j] = J - Kx;
        }
    }
    c->gT32.assign(c->gT.begin(), c->gT.end());
    c->hp32.assign(c->hprime.begin(), c->hprime.end());
    c->have32 = false;
    c->have_bf = false;
    c->have_ints = true;
    c->prepared = false;
    return STPCI_OK;
}

stpci_status stpci_set_space(stpci_ctx* c, int n_elec, int n_sub, const int* sub_size, const int* win_lo,
                             const int* win_hi) {
    if (!c) return STPCI_EINVAL;
    if (!sub_size || !win_lo || !win_hi) return set_err(c, STPCI_EINVAL, "NULL partition array");
    std::string err;
    stp::HostSpace hs;
    try {
        if (!hs.build(n_elec, n_sub, sub_size, win_lo, win_hi, err)) return set_err(c, STPCI_EINVAL, err);
    } catch (const std::bad_alloc&) {
        return set_err(c, STPCI_ENOMEM, "host memory exhausted while building string tables");
    }
    c->hs = std::move(hs);
    c->have_space = true;
    c->prepared = false;
    c->csc_pcat_ready = false;
    return STPCI_OK;
}

stpci_status stpci_space_info(const stpci_ctx* c, int64_t* n_dets, int* n_cat, int64_t* bytes_per_vec,
                              double* w_sigma_macs, double* nnz_h) {
    if (!c) return STPCI_EINVAL;
    if (!c->have_space) return set_err(const_cast<stpci_ctx*>(c), STPCI_ESTATE, "space not set");
    const HostSpace& H = c->hs;
    if (n_dets) *n_dets = H.sp.ndets;
    if (n_cat) *n_cat = H.sp.nspace;
    if (bytes_per_vec) *bytes_per_vec = H.sp.ndets * (int64_t)(c->have_ints ? scalar_bytes(c) : 16);
    if (w_sigma_macs) *w_sigma_macs = H.W1 + H.W2;
    if (nnz_h) *nnz_h = H.nnz;
    return STPCI_OK;
}

stpci_status stpci_work_counts(const stpci_ctx* c, double* w1, double* w2, int64_t* n_inter, int* max_deg) {
    if (!c) return STPCI_EINVAL;
    if (!c->have_space) return set_err(const_cast<stpci_ctx*>(c), STPCI_ESTATE, "space not set");
    if (w1) *w1 = c->hs.W1;
    if (w2) *w2 = c->hs.W2;
    if (n_inter) *n_inter = c->hs.sp.nwork_dets;
    if (max_deg) *max_deg = c->hs.max_deg;
    return STPCI_OK;
}

static bool host_to_bits(const void* u, int64_t a, uint64_t* b) {
    return static_cast<const HostSpace*>(u)->address_to_det(a, b);
}

stpci_status stpci_test_moves(const stpci_ctx* c, int64_t max_dets_per_cat, int64_t* n_checked, int64_t* n_bad) {
    if (!c || !n_checked || !n_bad) return STPCI_EINVAL;
    if (!c->have_space) return set_err(const_cast<stpci_ctx*>(c), STPCI_ESTATE, "space not set");
    const HostSpace& H = c->hs;
    DevSpace D{};
    D.sp = H.sp;
    D.cats = H.cats.data();
    D.tabs = H.tabs.data();
    D.bits = H.bits.data();
    D.ann = H.ann.data();
    D.cre = H.cre.data();
    D.work_cat = H.work_cat.data();
    D.work_begin = H.work_begin.data();
    D.space_begin = H.space_begin.data();
    *n_bad = check_moves_host(D, max_dets_per_cat, n_checked, host_to_bits, &H);
    return STPCI_OK;
}

stpci_status stpci_test_pairs(const stpci_ctx* c, int64_t max_dets_per_cat, int64_t* n_checked, int64_t* n_bad) {
    if (!c || !n_checked || !n_bad) return STPCI_EINVAL;
    if (!c->have_space) return set_err(const_cast<stpci_ctx*>(c), STPCI_ESTATE, "space not set");
    const HostSpace& H = c->hs;
    DevSpace D{};
    D.sp = H.sp;
    D.cats = H.cats.data();
    D.tabs = H.tabs.data();
    D.bits = H.bits.data();
    D.ann = H.ann.data();
    D.cre = H.cre.data();
    D.space_begin = H.space_begin.data();
    D.pcats = H.pcats.data();
    D.pwork_begin = H.pwork_begin.data();
    D.pslot = H.pslot.data();
    *n_bad = check_pairs_host(D, max_dets_per_cat, n_checked, host_to_bits, &H);
    return STPCI_OK;
}

stpci_status stpci_test_sb(const stpci_ctx* c, int64_t max_groups, int64_t* n_checked, int64_t* n_bad) {
    if (!c || !n_checked || !n_bad) return STPCI_EINVAL;
    if (!c->have_space) return set_err(const_cast<stpci_ctx*>(c), STPCI_ESTATE, "space not set");
    const HostSpace& H = c->hs;
    SbHostPlan pl;
    if (!build_sb_plan(H, pl))
        return set_err(const_cast<stpci_ctx*>(c), STPCI_EINVAL,
                       "the spectator-batched pair kernel does not support this space");
    DevSpace D{};
    D.sp = H.sp;
    D.cats = H.cats.data();
    D.tabs = H.tabs.data();
    D.bits = H.bits.data();
    D.ann = H.ann.data();
    D.cre = H.cre.data();
    D.space_begin = H.space_begin.data();
    D.pcats = H.pcats.data();
    D.pwork_begin = H.pwork_begin.data();
    D.pslot = H.pslot.data();
    *n_bad = check_sb_host(D, pl, max_groups, n_checked, host_to_bits, &H);
    return STPCI_OK;
}

stpci_status stpci_sb_counts(const stpci_ctx* c, int n_vec, double* mfma_flops, int64_t* items) {
    if (!c || n_vec < 1) return STPCI_EINVAL;
    if (!c->have_space) return set_err(const_cast<stpci_ctx*>(c), STPCI_ESTATE, "space not set");
    SbHostPlan pl;
    if (!build_sb_plan(c->hs, pl))
        return set_err(const_cast<stpci_ctx*>(c), STPCI_EINVAL,
                       "the spectator-batched pair kernel does not support this space");
    double f = 0;
    int64_t it = 0;
    for (int v0 = 0; v0 < n_vec; v0 += 2) {
        double ff;
        int64_t ii;
        sb_plan_counts(pl, c->have_ints ? c->cplx : true, (n_vec - v0 >= 2) ? 2 : 1, &ff, &ii);
        f += ff;
        it += ii;
    }
    if (mfma_flops) *mfma_flops = f;
    if (items) *items = it;
    return STPCI_OK;
}

stpci_status stpci_test_pair_groups(const stpci_ctx* c, int64_t* n_items, int64_t* n_bad, int* unit) {
    if (!c || !n_items || !n_bad || !unit) return STPCI_EINVAL;
    if (!c->have_space) return set_err(const_cast<stpci_ctx*>(c), STPCI_ESTATE, "space not set");
    const HostSpace& H = c->hs;
    std::vector<GrpItem> items;
    if (!build_pair_groups(H, items))
        return set_err(const_cast<stpci_ctx*>(c), STPCI_EINVAL, "the grouped pair kernel does not support this space");
    const PairCat& P = H.pcats[0];
    const StrTab& T = H.tabs[P.tab[0]];
    const int64_t cnt = P.count[0];
    std::vector<int> seen((size_t)cnt, 0);
    int64_t bad = 0;
    for (const GrpItem& it : items) {
        if (it.n < 1 || it.n > pair_grp_unit(H.sp)) {
            ++bad;
            continue;
        }
        for (int u = 0; u < GRP_U; ++u) {
            const int64_t j = it.j[u];
            if (u >= it.n) {
                bad += (j != -1);
                continue;
            }
            if (j < 0 || j >= cnt) {
                ++bad;
                continue;
            }
            ++seen[(size_t)j];
            const uint32_t s = H.bits[T.bits_off + j];
            if ((s & it.core) != it.core || __builtin_popcount(s ^ it.core) != 1) ++bad;
        }
    }
    for (int x : seen) bad += (x != 1);
    *n_items = (int64_t)items.size();
    *n_bad = bad;
    *unit = pair_grp_unit(H.sp);
    return STPCI_OK;
}

stpci_status stpci_category(const stpci_ctx* c, int cat, int* occ, int64_t* offset, int64_t* n_dets) {
    if (!c) return STPCI_EINVAL;
    if (!c->have_space) return set_err(const_cast<stpci_ctx*>(c), STPCI_ESTATE, "space not set");
    if (cat < 0 || cat >= c->hs.sp.nspace) return set_err(const_cast<stpci_ctx*>(c), STPCI_EINVAL, "bad category");
    const Cat& C = c->hs.cats[cat];
    if (occ)
        for (int k = 0; k < c->hs.sp.K; ++k) occ[k] = C.occ[k];
    if (offset) *offset = C.offset;
    if (n_dets) *n_dets = C.size;
    return STPCI_OK;
}

stpci_status stpci_address_to_det(const stpci_ctx* c, int64_t addr, uint64_t* bits) {
    if (!c || !bits) return STPCI_EINVAL;
    if (!c->have_space) return set_err(const_cast<stpci_ctx*>(c), STPCI_ESTATE, "space not set");
    if (!c->hs.address_to_det(addr, bits)) return set_err(const_cast<stpci_ctx*>(c), STPCI_EINVAL, "bad address");
    return STPCI_OK;
}

stpci_status stpci_sigma(stpci_ctx* c, const void* c_dev, void* sigma_dev, int n_vec, stpci_precision prec) {
    if (!c) return STPCI_EINVAL;
    if (!c_dev || !sigma_dev || n_vec < 1) return set_err(c, STPCI_EINVAL, "bad sigma arguments");
    stpci_status s = prepare(c);
    if (s) return s;
    if ((s = hip_check(c, hipSetDevice(c->device), "hipSetDevice"))) return s;
    size_t bytes = (size_t)c->hs.sp.ndets * scalar_bytes(c) * n_vec;
    const char* a = (const char*)c_dev;
    const char* b = (const char*)sigma_dev;
    if (a < b + bytes && b < a + bytes) return set_err(c, STPCI_EINVAL, "c_dev and sigma_dev overlap");
    return sigma_impl(c, c_dev, sigma_dev, n_vec, prec);
}

stpci_status stpci_diagonal(stpci_ctx* c, double* diag_dev) {
    if (!c) return STPCI_EINVAL;
    if (!diag_dev) return set_err(c, STPCI_EINVAL, "NULL diag_dev");
    stpci_status s = prepare(c);
    if (s) return s;
    return hip_check(c, launch_diag(c->dev, (const double*)c->d_hd.p, (const double*)c->d_JK.p, c->e_core,
                                    diag_dev, c->stream),
                     "diag launch");
}

stpci_status stpci_profile(stpci_ctx* c, int enable) {
    if (!c) return STPCI_EINVAL;
    if (c->host_only) return set_err(c, STPCI_ESTATE, "host-only context");
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto& e : c->events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    c->events.clear();
    c->profile = enable != 0;
    return STPCI_OK;
}

stpci_status stpci_kernel_time(stpci_ctx* c, const char* name, int64_t* launches, double* total_ms) {
    if (!c || !name) return STPCI_EINVAL;
    int kind = -1;
    if (!std::strcmp(name, "sigma1e")) kind = 0;
    if (!std::strcmp(name, "sigma2e") || !std::strcmp(name, "sigma")) kind = 1;
    if (!std::strcmp(name, "sigma_fp32")) kind = 2;
    if (!std::strcmp(name, "sigma_reduce")) kind = 3;
    if (!std::strcmp(name, "sigma_bf16")) kind = 4;
    if (kind < 0) return set_err(c, STPCI_EINVAL, "unknown kernel name");
    if (c->host_only) return set_err(c, STPCI_ESTATE, "host-only context");
    stpci_status s = hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
    if (s) return s;
    int64_t n = 0;
    double t = 0;
    for (auto& e : c->events) {
        if (e.kind != kind) continue;
        float ms = 0;
        if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
            t += ms;
            ++n;
        }
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = t;
    return STPCI_OK;
}

stpci_status stpci_pair_counts(const stpci_ctx* c, double* w_pair, int64_t* n_pair_inter, int* max_pair_deg) {
    if (!c) return STPCI_EINVAL;
    if (!c->have_space) return set_err(const_cast<stpci_ctx*>(c), STPCI_ESTATE, "space not set");
    if (w_pair) *w_pair = c->hs.Wp;
    if (n_pair_inter) *n_pair_inter = c->hs.sp.npwork_dets;
    if (max_pair_deg) *max_pair_deg = c->hs.pmax_deg;
    return STPCI_OK;
}

stpci_status stpci_set_sigma_kernel(stpci_ctx* c, const char* name) {
    if (!c || !name) return STPCI_EINVAL;
    // request numbers 1 and 3..9 (0 and 2 are unused)
    static const char* names[10] = {nullptr,       "rowtile",   nullptr,     "tile",     "pair",
                                    "pair_atomic", "pair_mf64", "pair_valu", "pair_grp", "pair_sb"};
    int k = -1;
    if (!std::strcmp(name, "auto")) k = -2;
    for (int i = 0; i < 10; ++i)
        if (names[i] && !std::strcmp(name, names[i])) k = i;
    if (k == -1) return set_err(c, STPCI_EINVAL, "unknown sigma kernel name");
    c->kernel_req = (k == -2) ? -1 : k;
    // device copies depend on the kernel: rebuild them on the next device call
    for (DevBuf* b : {&c->d_E, &c->d_grp, &c->d_sbcats, &c->d_sbrows, &c->d_sbstreams, &c->d_pcats, &c->d_pwork, &c->d_pslot, &c->d_pA, &c->d_pA32, &c->d_pAbf, &c->d_gT32, &c->d_hp32,
                      &c->d_s2blocks, &c->d_ygroup, &c->d_hp, &c->d_gT})
        if (!c->host_only) b->free_();
    c->have32 = false;
    c->have_bf = false;
    c->prepared = false;
    return STPCI_OK;
}

stpci_status stpci_sigma_kernel(const stpci_ctx* c, const char** name) {
    if (!c || !name) return STPCI_EINVAL;
    static const char* names[5] = {"", "rowtile", "", "tile", "pair"};
    if (!c->prepared) return set_err(const_cast<stpci_ctx*>(c), STPCI_ESTATE, "no device call made yet");
    if (c->s2_kernel == 4 && c->pair_sb)
        *name = "pair_sb";
    else if (c->s2_kernel == 4 && c->pair_grp)
        *name = c->pair_store ? "pair_grp" : "pair_grp_atomic";
    else if (c->s2_kernel == 4)
        *name = c->pair_mf64 ? (c->pair_store ? "pair_mf64" : "pair_mf64_atomic")
                             : (c->pair_store ? "pair_valu" : "pair_valu_atomic");
    else
        *name = names[c->s2_kernel];
    return STPCI_OK;
}

}  // extern "C"
