// Davidson eigensolver driver (Results: Rayleigh-Ritz with the residual
// r = HC - EC appended after preconditioning, convergence on ||r||;
// preconditioner of Eq. sparsePreconditioner with the 1e-12 guard).
// Vectors stay on the device; only the small projected problem (at most 64 x
// 64) is solved on the host (Householder tridiagonalisation and implicit QL).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <limits>
#include <numeric>
#include <sstream>

#include "ctx.hpp"
#include "kernels.hpp"

using namespace stp;
using cplx = std::complex<double>;

namespace stp {

// Eigen-decomposition of a Hermitian n x n matrix A (row-major), eigenvalues
// ascending in w, eigenvectors as columns of V (row-major n x n).
// Householder reduction to tridiagonal form, A = Q T Q^H, a diagonal phase
// change D that makes the off-diagonal of T real and non-negative, then the
// implicit QL iteration with Wilkinson shifts on the real symmetric
// tridiagonal matrix, T = D Z L Z^T D^H, so that V = Q D Z.
void herm_eig(int n, std::vector<cplx> A, std::vector<double>& w, std::vector<cplx>& V) {
    auto a = [&](int i, int j) -> cplx& { return A[(size_t)i * n + j]; };
    std::vector<cplx> Q((size_t)n * n, cplx(0, 0));
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    std::vector<cplx> v(n), p(n);
    // ---- Householder: zero column k below its subdiagonal entry
    for (int k = 0; k + 2 < n; ++k) {
        const int m0 = k + 1;
        double xn2 = 0;
        for (int i = m0; i < n; ++i) xn2 += std::norm(a(i, k));
        const double xn = std::sqrt(xn2);
        if (xn == 0.0) continue;
        const cplx x0 = a(m0, k);
        const cplx ph = (std::abs(x0) > 0) ? x0 / std::abs(x0) : cplx(1, 0);
        const cplx alpha = -ph * xn;
        double vn2 = 0;
        for (int i = m0; i < n; ++i) {
            v[i] = a(i, k);
            if (i == m0) v[i] -= alpha;
            vn2 += std::norm(v[i]);
        }
        if (vn2 == 0.0) continue;
        const double tau = 2.0 / vn2;
        // p = tau * A_sub v over the trailing block, q = p - (tau/2)(v^H p) v
        for (int i = m0; i < n; ++i) {
            cplx t = 0;
            for (int j = m0; j < n; ++j) t += a(i, j) * v[j];
            p[i] = tau * t;
        }
        cplx vp = 0;
        for (int i = m0; i < n; ++i) vp += std::conj(v[i]) * p[i];
        for (int i = m0; i < n; ++i) p[i] -= 0.5 * tau * vp * v[i];
        for (int i = m0; i < n; ++i)
            for (int j = m0; j < n; ++j) a(i, j) -= v[i] * std::conj(p[j]) + p[i] * std::conj(v[j]);
        a(m0, k) = alpha;
        a(k, m0) = std::conj(alpha);
        for (int i = m0 + 1; i < n; ++i) a(i, k) = a(k, i) = 0;
        // Q <- Q H, H = I - tau v v^H
        for (int r = 0; r < n; ++r) {
            cplx t = 0;
            for (int j = m0; j < n; ++j) t += Q[(size_t)r * n + j] * v[j];
            t *= tau;
            for (int j = m0; j < n; ++j) Q[(size_t)r * n + j] -= t * std::conj(v[j]);
        }
    }
    // ---- real tridiagonal: d (diagonal), e[i] = |T[i+1][i]|, phases D
    std::vector<double> d(n), e(n, 0.0);
    std::vector<cplx> D(n, cplx(1, 0));
    for (int i = 0; i < n; ++i) d[i] = a(i, i).real();
    for (int i = 0; i + 1 < n; ++i) {
        const cplx t = a(i + 1, i);
        e[i] = std::abs(t);
        D[i + 1] = (e[i] > 0) ? D[i] * (t / e[i]) : D[i];
    }
    // ---- implicit QL with Wilkinson shifts, rotations accumulated in Z
    std::vector<double> Z((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    const double eps = std::numeric_limits<double>::epsilon();
    for (int l = 0; l < n; ++l) {
        for (int iter = 0; iter < 100; ++iter) {
            int m = l;
            for (; m + 1 < n; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= eps * dd) break;
            }
            if (m == l) break;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            double sn = 1.0, cs = 1.0, pp = 0.0;
            int i = m - 1;
            bool early = false;
            for (; i >= l; --i) {
                const double f = sn * e[i], b = cs * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {  // split: deflate and restart
                    d[i + 1] -= pp;
                    e[m] = 0.0;
                    early = true;
                    break;
                }
                sn = f / r;
                cs = g / r;
                g = d[i + 1] - pp;
                r = (d[i] - g) * sn + 2.0 * cs * b;
                pp = sn * r;
                d[i + 1] = g + pp;
                g = cs * r - b;
                for (int k = 0; k < n; ++k) {
                    double& z0 = Z[(size_t)k * n + i];
                    double& z1 = Z[(size_t)k * n + i + 1];
                    const double fz = z1;
                    z1 = sn * z0 + cs * fz;
                    z0 = cs * z0 - sn * fz;
                }
            }
            if (early) continue;
            d[l] -= pp;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    // ---- V = Q D Z, eigenvalues ascending
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x] < d[y]; });
    w.resize(n);
    V.assign((size_t)n * n, cplx(0, 0));
    for (int jj = 0; jj < n; ++jj) {
        const int j = ord[jj];
        w[jj] = d[j];
        for (int r = 0; r < n; ++r) {
            cplx t = 0;
            for (int k = 0; k < n; ++k) t += Q[(size_t)r * n + k] * D[k] * Z[(size_t)k * n + j];
            V[(size_t)r * n + jj] = t;
        }
    }
}

}  // namespace stp

namespace {

// layout of the small device workspace
constexpr size_t kYOff = 0;                         // coefficient matrices, up to 64 x 32 complex
constexpr size_t kZOff = kYOff + 64 * 32 * 16;      // Ritz coefficient changes, up to 64 x 16 complex
constexpr size_t kThetaOff = kZOff + 64 * 16 * 16;  // Ritz values, 64 doubles
constexpr size_t kRitzOff = kThetaOff + 64 * 8;     // per root ||r||^2, ||t||^2, max |x - ph x_prev|^2 (ritz_slot)
constexpr size_t kNrmOff = kRitzOff + 16 * 3 * 8;   // norms of the corrections after the eps drop (32 slots)
constexpr size_t kGramOff = kNrmOff + 32 * 16;      // Gram matrix of the corrections (after the norms: one fetch)
constexpr size_t kGramBytes = 16 * 16 * 16;
constexpr size_t kDotsOff = kGramOff + 16 * 16 * 16;   // dot products
constexpr int kDotsMax = 64 * 16;                   // dot products queued at once
constexpr size_t kCoefOff = kDotsOff + (size_t)kDotsMax * 16;
constexpr size_t kSmallBytes = kCoefOff + 64 * 16;
static_assert(kDotsOff == kGramOff + kGramBytes, "workspace layout");

// where the Ritz pass leaves ||r_j||^2 (q = 0), ||t_j||^2 (1) and the largest
// |x_j - ph_j x_j(previous)|^2 (2), in doubles from kRitzOff
static int ritz_slot(int j, int q) { return 12 * (j / 4) + 4 * q + j % 4; }

// bytes of the partial-sum area the vector kernels share
static size_t partial_bytes(int64_t N, int k) {
    return std::max({(size_t)dots_blocks(N) * kDotsMax * 16, (size_t)ritz_blocks(N, k) * 12 * 8,
                     (size_t)comb_gram_blocks(N) * 32 * 8});
}

struct Dav {
    stpci_ctx* c;
    int64_t N;
    size_t sb;     // scalar bytes
    bool cx;
    hipStream_t st;

    char* vec(DevBuf& b, int i) { return (char*)b.p + (size_t)i * N * sb; }
    char* small(size_t off) { return (char*)c->d_small.p + off; }

    stpci_status hip(hipError_t e, const char* w) { return hip_check(c, e, w); }

    // a region of the pinned staging buffer for `bytes` (the buffer is
    // reused from its start after a stream synchronisation; when full, the
    // stream is synchronised first); NULL when there is no pinned buffer
    double* stage(size_t bytes) {
        if (!c->pin) return nullptr;
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes > c->pin_bytes) return nullptr;
        if (c->pin_off + bytes > c->pin_bytes) {
            if (hipStreamSynchronize(st) != hipSuccess) return nullptr;
            c->pin_off = 0;
        }
        double* p = (double*)((char*)c->pin + c->pin_off);
        c->pin_off += bytes;
        return p;
    }
    stpci_status synced(hipError_t e) {
        if (e == hipSuccess) c->pin_off = 0;   // every staged copy has completed
        return hip(e, "sync");
    }

    // upload n doubles to d_small + byte_off (through the pinned buffer)
    stpci_status put_doubles(const double* src, size_t n, size_t byte_off) {
        double* p = stage(n * 8);
        if (p) {
            std::memcpy(p, src, n * 8);
            return hip(hipMemcpyAsync(small(byte_off), p, n * 8, hipMemcpyHostToDevice, st), "small upload");
        }
        return hip(hipMemcpyAsync(small(byte_off), src, n * 8, hipMemcpyHostToDevice, st), "small upload");
    }

    // n doubles from d_small + byte_off (one round trip)
    stpci_status get_doubles(size_t byte_off, size_t n, std::vector<double>& out) {
        out.resize(n);
        double* p = stage(n * 8);
        stpci_status s = hip(hipMemcpyAsync(p ? p : out.data(), small(byte_off), n * 8, hipMemcpyDeviceToHost, st),
                             "small copy");
        if (s) return s;
        if ((s = synced(hipStreamSynchronize(st)))) return s;
        if (p) std::memcpy(out.data(), p, n * 8);
        return STPCI_OK;
    }

    // count scalars from d_small + byte_off
    stpci_status get_scalars(size_t byte_off, int count, std::vector<cplx>& out) {
        std::vector<double> raw;
        stpci_status s = get_doubles(byte_off, (size_t)count * (cx ? 2 : 1), raw);
        if (s) return s;
        out.resize(count);
        for (int i = 0; i < count; ++i) out[i] = cx ? cplx(raw[2 * i], raw[2 * i + 1]) : cplx(raw[i], 0.0);
        return STPCI_OK;
    }

    // out[i] = <A_i | w> for i < m  (host result)
    stpci_status dots(const void* A, int m, const void* w, std::vector<cplx>& out) {
        stpci_status s = issue_dots(A, m, w, 1, 0);
        if (s) return s;
        return get_scalars(kDotsOff, m, out);
    }

    // upload a small coefficient matrix Y (row-major) into d_small + off
    stpci_status put_small(const std::vector<cplx>& Y, size_t byte_off) {
        std::vector<double> buf(Y.size() * (cx ? 2 : 1));
        for (size_t i = 0; i < Y.size(); ++i) {
            if (cx) { buf[2 * i] = Y[i].real(); buf[2 * i + 1] = Y[i].imag(); }
            else buf[i] = Y[i].real();
        }
        return put_doubles(buf.data(), buf.size(), byte_off);
    }

    // queue out[off + t m + i] = <A_i | W_t>, i < m, t < nw, in the area at
    // area_off (the dot products by default; no sync); A and W are
    // consecutive vectors of N scalars
    stpci_status issue_dots(const void* A, int m, const void* W, int nw, int off, size_t area_off = kDotsOff) {
        char* out = small(area_off) + (size_t)off * (cx ? 16 : 8);
        return hip(launch_dots(cx, A, N, m, W, nw, N, c->d_partial.p, out, st), "dots");
    }

    // <A_j | W_j> for j < n (A, W: n consecutive vectors each), two roots per
    // launch: the launch for j0, j0 + 1 queues the 2 x 2 block of products at
    // off + 2 j0, whose diagonal holds the two wanted values; pair_slots(n)
    // slots in all
    static int pair_slots(int n) { return 4 * (n / 2) + (n & 1); }
    static int pair_slot(int j, int n) {
        const int j0 = j & ~1, c = std::min(2, n - j0);
        return 2 * j0 + (j - j0) * (c + 1);
    }
    stpci_status issue_pair_dots(char* A, char* W, int n, int off, size_t area_off = kDotsOff) {
        for (int j0 = 0; j0 < n; j0 += 2) {
            const int cnt = std::min(2, n - j0);
            const size_t at = (size_t)j0 * N * sb;
            stpci_status s = issue_dots(A + at, cnt, W + at, cnt, off + 2 * j0, area_off);
            if (s) return s;
        }
        return STPCI_OK;
    }

    stpci_status norm(const void* x, double& n) {
        std::vector<cplx> d;
        stpci_status s = dots(x, 1, x, d);
        n = std::sqrt(std::max(0.0, d[0].real()));
        return s;
    }

    // x <- x - A coef  (coef: m entries)
    stpci_status subtract(const void* A, int m, const std::vector<cplx>& coef, void* x) {
        stpci_status s = put_small(coef, kCoefOff);
        if (s) return s;
        return hip(launch_combine(cx, A, nullptr, N, m, small(kCoefOff), 1, nullptr, x, nullptr, N, 2, st), "cgs");
    }

    // T_q = Eq. sparsePreconditioner applied to R_root[q] with theta[q]:
    // s = r / (theta - H_ii) (0 where |theta - H_ii| < 1e-12), then, with
    // eps > 0, entries below eps ||s_q|| dropped (||s_q||^2 computed on the
    // device and read there by the drop kernel, without a round trip)
    stpci_status precondition(const void* R, void* T, int nt, const int* roots, const double* thetas, double eps) {
        stpci_status s = hip(launch_precond(c->dev, cx, (const double*)c->d_hd.p, (const double*)c->d_JK.p,
                                            c->e_core, R, T, N, nt, roots, thetas, 1e-12, st),
                             "precond");
        if (s || !(eps > 0.0) || nt < 1) return s;
        if ((s = issue_pair_dots((char*)T, (char*)T, nt, 0))) return s;
        int slot[PRE_MAX];
        for (int q = 0; q < nt; ++q) slot[q] = pair_slot(q, nt);
        return hip(launch_eps_drop(cx, T, N, N, nt, slot, (const double*)small(kDotsOff), cx ? 2 : 1, eps, st),
                   "eps drop");
    }

    // X_t -= sum_i A_i <A_i | X_t> for t < nx, the products queued by
    // issue_dots(A, m, X, nx, 0) and read where they lie (no round trip)
    stpci_status subtract_queued(const void* A, int m, int nx, void* X) {
        return hip(launch_combine(cx, A, nullptr, N, m, small(kDotsOff), nx, nullptr, X, nullptr, N, 3, st), "cgs");
    }
};

}  // namespace

// Test hook: the Davidson corrections of n residuals (consecutive vectors of
// r_dev) with Ritz values theta (host), written to t_dev, with the eps drop.
extern "C" stpci_status stpci_test_precond(stpci_ctx* c, const void* r_dev, void* t_dev, int n, const double* theta,
                                           double eps) {
    if (!c || !r_dev || !t_dev || !theta || n < 1 || n > PRE_MAX) return STPCI_EINVAL;
    if (!(eps >= 0.0 && eps < 1.0)) return set_err(c, STPCI_EINVAL, "eps must lie in [0, 1)");
    stpci_status s = prepare(c);
    if (s) return s;
    if ((s = hip_check(c, hipSetDevice(c->device), "hipSetDevice"))) return s;
    const int64_t N = c->hs.sp.ndets;
    if ((s = ensure(c, c->d_partial, partial_bytes(N, n), "dot partials"))) return s;
    if ((s = ensure(c, c->d_small, kSmallBytes, "small workspace"))) return s;
    Dav d{c, N, scalar_bytes(c), c->cplx, c->stream};
    std::vector<int> roots(n);
    for (int q = 0; q < n; ++q) roots[q] = q;
    if ((s = d.precondition(r_dev, t_dev, n, roots.data(), theta, eps))) return s;
    return hip_check(c, hipStreamSynchronize(c->stream), "sync");
}

extern "C" stpci_status stpci_test_dav_cgs_passes(const stpci_ctx* c, int* passes) {
    if (!c || !passes) return STPCI_EINVAL;
    *passes = c->dav.cgs_passes;
    return STPCI_OK;
}

// Test hook: the fused Rayleigh-Ritz pass of the solver on given vectors.
extern "C" stpci_status stpci_test_ritz(stpci_ctx* c, const void* v_dev, const void* w_dev, int m, const double* y,
                                        const double* z, int k, const double* theta, void* x_dev, void* t_dev,
                                        double* red) {
    if (!c || !v_dev || !w_dev || !y || !theta || !x_dev || !t_dev || !red || m < 1 || m > 64 || k < 1 ||
        k > PRE_MAX)
        return STPCI_EINVAL;
    stpci_status s = prepare(c);
    if (s) return s;
    if ((s = hip_check(c, hipSetDevice(c->device), "hipSetDevice"))) return s;
    const int64_t N = c->hs.sp.ndets;
    if ((s = ensure(c, c->d_partial, partial_bytes(N, k), "dot partials"))) return s;
    if ((s = ensure(c, c->d_small, kSmallBytes, "small workspace"))) return s;
    Dav d{c, N, scalar_bytes(c), c->cplx, c->stream};
    const size_t w = d.cx ? 2 : 1;
    if ((s = d.put_doubles(y, (size_t)m * k * w, kYOff))) return s;
    if (z && (s = d.put_doubles(z, (size_t)m * k * w, kZOff))) return s;
    if ((s = d.put_doubles(theta, (size_t)k, kThetaOff))) return s;
    if ((s = d.hip(launch_ritz(c->dev, d.cx, (const double*)c->d_hd.p, (const double*)c->d_JK.p, c->e_core, v_dev,
                               w_dev, N, m, d.small(kYOff), z ? d.small(kZOff) : nullptr, k,
                               (const double*)d.small(kThetaOff), 1e-12, x_dev, t_dev, N, (double*)c->d_partial.p,
                               (double*)d.small(kRitzOff), c->stream),
                   "ritz")))
        return s;
    std::vector<double> raw;
    if ((s = d.get_doubles(kRitzOff, (size_t)12 * ((k + 3) / 4), raw))) return s;
    for (int j = 0; j < k; ++j)
        for (int q = 0; q < 3; ++q) red[3 * j + q] = raw[ritz_slot(j, q)];
    return STPCI_OK;
}

extern "C" stpci_status stpci_test_heev(int n, const double* A, double* w, double* V) {
    if (n < 1 || !A || !w || !V) return STPCI_EINVAL;
    std::vector<cplx> M((size_t)n * n);
    for (size_t i = 0; i < M.size(); ++i) M[i] = cplx(A[2 * i], A[2 * i + 1]);
    std::vector<double> ww;
    std::vector<cplx> VV;
    herm_eig(n, M, ww, VV);
    for (int i = 0; i < n; ++i) w[i] = ww[i];
    for (size_t i = 0; i < VV.size(); ++i) { V[2 * i] = VV[i].real(); V[2 * i + 1] = VV[i].imag(); }
    return STPCI_OK;
}

// ---------------------------------------------------------------------------
// Davidson as a state machine.  A run alternates two steps:
//   pending  -> the sigma products the iteration needs next: W[m..m+nv) = H V[m..m+nv)
//   advance  -> after those products: extend G = V^H W, Rayleigh-Ritz,
//               residuals, convergence test, preconditioned corrections,
//               CGS2, restart, which leaves the next pending products.
// stpci_davidson drives it with its own sigma calls; the request server
// drives many contexts at once and performs their sigma products in one
// grouped launch.
// ---------------------------------------------------------------------------
static int subspace_request(const stpci_dav_opts& o) {
    return o.max_subspace > 0 ? o.max_subspace : std::max(8 * o.k, 32);
}

// Expansion-space size for a request of mmax vectors (at most 64, at most N,
// at least 2k where the space allows it).
static int subspace_cap(int mmax, int k, int64_t N) {
    mmax = (int)std::min<int64_t>(std::min(mmax, 64), N);
    if (mmax < 2 * k && N >= 2 * k) mmax = 2 * k;
    return std::max(mmax, k);
}

namespace stp {
// Upper bound of the device bytes a Davidson run allocates (the expansion
// space is only ever reduced below this when device memory is short).
int64_t dav_device_bytes(const stpci_ctx* c, const stpci_dav_opts& o) {
    const int64_t N = c->hs.sp.ndets;
    const int64_t vb = N * (int64_t)scalar_bytes(c);
    const bool extra = o.certify || (o.refine_tol_energy > 0.0 && o.precision != STPCI_FP64);
    const int k = o.k + ((extra && o.k < 16 && o.k < N) ? 1 : 0);
    stpci_dav_opts run = o;   // the options of the run, with the extra root of certify
    run.k = k;
    const int mmax = subspace_cap(subspace_request(run), k, N);
    int64_t b = vb * (2LL * mmax + 2LL * k);
    b += (int64_t)partial_bytes(N, k) + (int64_t)kSmallBytes;
    if (!o.guess_dev) b += 1024LL * k * 16;  // top-k partials: at most 1024 blocks
    return b;
}
}  // namespace stp

static stpci_status dav_start(stpci_ctx* c, stpci_precision prec, const void* guess_dev, double tol) {
    DavState& D = c->dav;
    const stpci_dav_opts& o = D.opts;
    stpci_status s;
    const int64_t N = c->hs.sp.ndets;
    const int k = o.k;
    D.prec = prec;
    D.tol = tol;
    D.pidx = (prec == STPCI_FP32) ? 1 : (prec == STPCI_BF16) ? 2 : 0;
    D.best_rn = -1.0;
    D.stall = 0;
    const size_t vb = (size_t)N * scalar_bytes(c);
    D.kr_max = std::min(2 * k, 32);
    int mmax = subspace_request(o);
    {
        // expansion space bounded by the device memory left for V and W
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess && vb > 0) {
            const size_t have = c->d_V.bytes + c->d_W.bytes + c->d_X.bytes + c->d_T.bytes;
            const double budget = 0.85 * (double)(fr + have) / (double)vb - 2.0 * k;
            if (budget / 2.0 < mmax) mmax = (int)std::max(budget / 2.0, (double)(2 * k));
        }
    }
    D.mmax = subspace_cap(mmax, k, N);
    D.max_iter = o.max_iter > 0 ? o.max_iter : 100;
    if ((s = ensure(c, c->d_V, vb * D.mmax, "Davidson V"))) return s;
    if ((s = ensure(c, c->d_W, vb * D.mmax, "Davidson W"))) return s;
    if ((s = ensure(c, c->d_X, vb * k, "Ritz vectors"))) return s;
    if ((s = ensure(c, c->d_T, vb * k, "corrections"))) return s;
    if ((s = ensure(c, c->d_partial, partial_bytes(N, k), "dot partials"))) return s;
    if ((s = ensure(c, c->d_small, kSmallBytes, "small workspace"))) return s;
    if (!c->pin) {
        // 1 MB of pinned staging for the small transfers of the iteration
        if (hipHostMalloc(&c->pin, (size_t)1 << 20, hipHostMallocDefault) == hipSuccess) {
            c->pin_bytes = (size_t)1 << 20;
        } else {
            c->pin = nullptr;
            (void)hipGetLastError();
        }
    }
    if ((s = hip_check(c, hipStreamSynchronize(c->stream), "sync"))) return s;   // no staged copy in flight
    c->pin_off = 0;
    Dav d{c, N, scalar_bytes(c), c->cplx, c->stream};
    if (guess_dev) {
        if ((s = d.hip(hipMemcpyAsync(c->d_V.p, guess_dev, vb * k, hipMemcpyDeviceToDevice, c->stream), "guess")))
            return s;
        for (int i = 0; i < k; ++i) {  // orthonormalise the guess (CGS2)
            for (int pass = 0; pass < 2 && i > 0; ++pass) {
                std::vector<cplx> coef;
                if ((s = d.dots(c->d_V.p, i, d.vec(c->d_V, i), coef))) return s;
                if ((s = d.subtract(c->d_V.p, i, coef, d.vec(c->d_V, i)))) return s;
            }
            double nr;
            if ((s = d.norm(d.vec(c->d_V, i), nr))) return s;
            if (nr < 1e-14) return set_err(c, STPCI_EINVAL, "guess vectors are linearly dependent");
            if ((s = d.hip(launch_scale(d.cx, d.vec(c->d_V, i), 1.0 / nr, N, c->stream), "scale"))) return s;
        }
    } else {
        int nb = topk_blocks(c->dev);
        if ((s = ensure(c, c->d_topv, (size_t)nb * k * 8, "top-k values"))) return s;
        if ((s = ensure(c, c->d_topi, (size_t)nb * k * 8, "top-k indices"))) return s;
        if ((s = d.hip(launch_diag_topk(c->dev, (const double*)c->d_hd.p, (const double*)c->d_JK.p, c->e_core, k,
                                        (double*)c->d_topv.p, (int64_t*)c->d_topi.p, c->stream),
                       "top-k")))
            return s;
        std::vector<double> tv((size_t)nb * k);
        std::vector<int64_t> ti((size_t)nb * k);
        (void)hipMemcpyAsync(tv.data(), c->d_topv.p, tv.size() * 8, hipMemcpyDeviceToHost, c->stream);
        (void)hipMemcpyAsync(ti.data(), c->d_topi.p, ti.size() * 8, hipMemcpyDeviceToHost, c->stream);
        if ((s = d.hip(hipStreamSynchronize(c->stream), "sync"))) return s;
        std::vector<int> ord(tv.size());
        std::iota(ord.begin(), ord.end(), 0);
        std::sort(ord.begin(), ord.end(), [&](int a, int b) {
            return tv[a] < tv[b] || (tv[a] == tv[b] && ti[a] < ti[b]);
        });
        for (int i = 0; i < k; ++i)
            if ((s = d.hip(launch_unit(d.cx, d.vec(c->d_V, i), N, ti[ord[i]], c->stream), "unit"))) return s;
    }
    D.G.assign((size_t)64 * 64, cplx(0, 0));
    D.prev_coef.clear();
    D.prev_rows = 0;
    D.theta.assign(k, 0.0);
    D.theta_prev.clear();
    D.energy_stop = false;
    D.rn.assign(k, 0.0);
    D.m = 0;
    D.nv = k;  // pending: W[0..k) = H V[0..k)
    D.it = 0;
    D.converged = false;
    D.done = false;
    D.active = true;
    return STPCI_OK;
}

// After the pending sigma products: one Rayleigh-Ritz iteration.  Sets D.done
// when converged, at max_iter, or when no new direction survives CGS2.
//
// Vector passes of an iteration (k roots, m basis vectors): the new columns
// of G = V^H W (one dot-product pass); one fused Rayleigh-Ritz pass that
// forms the Ritz vectors, the residuals' preconditioned corrections and the
// reductions the host needs (residual norms, correction norms, the largest
// coefficient change) without storing the residuals; the optional eps drop;
// CGS2 of the corrections against V (two dot-product passes and two
// subtractions, the second with the corrections' Gram matrix); Cholesky QR
// into V (with the Gram matrix of the result) and its second pass in place.
// The restart transforms V and W in place.
static stpci_status dav_advance(stpci_ctx* c) {
    DavState& D = c->dav;
    stpci_status s;
    const int64_t N = c->hs.sp.ndets;
    const int k = D.opts.k;
    Dav d{c, N, scalar_bytes(c), c->cplx, c->stream};
    auto Gat = [&](int i, int j) -> cplx& { return D.G[(size_t)i * 64 + j]; };
    c->nsigma[D.pidx] += D.nv;
    // new columns (and rows) of G = V^H W, one round trip
    {
        const int mt = D.m + D.nv;
        if ((s = d.issue_dots(c->d_V.p, mt, d.vec(c->d_W, D.m), D.nv, 0))) return s;
        std::vector<cplx> cols;
        if ((s = d.get_scalars(kDotsOff, D.nv * mt, cols))) return s;
        for (int j = D.m; j < mt; ++j)
            for (int i = 0; i < mt; ++i) {
                Gat(i, j) = cols[(size_t)(j - D.m) * mt + i];
                Gat(j, i) = std::conj(cols[(size_t)(j - D.m) * mt + i]);
            }
    }
    D.m += D.nv;
    D.nv = 0;
    const int m = D.m;
    D.it += 1;
    std::vector<cplx> A((size_t)m * m);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) A[(size_t)i * m + j] = 0.5 * (Gat(i, j) + std::conj(Gat(j, i)));
    std::vector<double> w;
    std::vector<cplx> Y;
    herm_eig(m, A, w, Y);
    std::vector<cplx> Yk((size_t)m * k);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < k; ++j) Yk[(size_t)i * k + j] = Y[(size_t)i * m + j];
    for (int j = 0; j < k; ++j) D.theta[j] = w[j];
    // the change of each Ritz vector since the previous iteration, x_j - ph_j
    // x_j(previous) = V z_j with z_j = y_j - ph_j yp_j (yp_j: the previous Ritz
    // vector's coordinates in this basis, ph_j = <x_prev|x>/|<x_prev|x>| from
    // the coordinates: V has orthonormal columns); its largest entry is
    // reported beside E and ||r|| (Results)
    const bool have_prev = D.prev_rows > 0;
    if (have_prev) {
        std::vector<cplx> Z((size_t)m * k);
        const int pr = std::min(D.prev_rows, m);
        for (int j = 0; j < k; ++j) {
            cplx o(0, 0);
            for (int i = 0; i < pr; ++i) o += std::conj(D.prev_coef[(size_t)i * k + j]) * Yk[(size_t)i * k + j];
            const double a = std::abs(o);
            const cplx ph = a > 0 ? o / a : cplx(1.0, 0.0);
            for (int i = 0; i < m; ++i) {
                const cplx yp = i < pr ? D.prev_coef[(size_t)i * k + j] : cplx(0, 0);
                Z[(size_t)i * k + j] = Yk[(size_t)i * k + j] - ph * yp;
            }
        }
        if ((s = d.put_small(Z, kZOff))) return s;
    }
    if ((s = d.put_small(Yk, kYOff))) return s;
    if ((s = d.put_doubles(D.theta.data(), (size_t)k, kThetaOff))) return s;
    if ((s = d.hip(launch_ritz(c->dev, d.cx, (const double*)c->d_hd.p, (const double*)c->d_JK.p, c->e_core, c->d_V.p,
                               c->d_W.p, N, m, d.small(kYOff), have_prev ? d.small(kZOff) : nullptr, k,
                               (const double*)d.small(kThetaOff), 1e-12, c->d_X.p, c->d_T.p, N,
                               (double*)c->d_partial.p, (double*)d.small(kRitzOff), c->stream),
                   "ritz")))
        return s;
    std::vector<double> red;
    if ((s = d.get_doubles(kRitzOff, (size_t)12 * ((k + 3) / 4), red))) return s;
    std::vector<double> dc(k, std::nan("")), tn2(k);
    for (int j = 0; j < k; ++j) {
        D.rn[j] = std::sqrt(std::max(0.0, red[ritz_slot(j, 0)]));
        tn2[j] = red[ritz_slot(j, 1)];
        if (have_prev) dc[j] = std::sqrt(std::max(0.0, red[ritz_slot(j, 2)]));
    }
    c->history.push_back(DavRecord{D.theta, D.rn, dc, D.pidx});
    bool conv = true;
    for (int j = 0; j < k; ++j) conv = conv && D.rn[j] <= D.tol;
    // FP64 refinement after a reduced-precision phase: with refine_tol_energy
    // > 0 it also ends once the gap-theorem bound ||r_j||^2 / gamma_j^- of
    // every requested root (gamma_j^- from the neighbouring Ritz pairs, the
    // run carrying one root more) is below refine_tol_energy
    const double rte = D.opts.refine_tol_energy;
    const int kq = D.k_req > 0 ? D.k_req : k;
    if (!conv && D.prec == STPCI_FP64 && D.it_prev > 0 && rte > 0.0 && kq < k) {
        bool small = true;
        for (int j = 0; j < kq; ++j) {
            double g = (D.theta[j + 1] - D.rn[j + 1]) - D.theta[j];
            if (j > 0) g = std::min(g, D.theta[j] - (D.theta[j - 1] + D.rn[j - 1]));
            small = small && g > 0 && D.rn[j] * D.rn[j] / g < rte;
        }
        conv = small;
        D.energy_stop = small;
    }
    D.theta_prev = D.theta;
    D.converged = conv;
    if (D.prec == STPCI_BF16 && !conv) {
        // the BF16 phase also ends when its largest residual has not dropped
        // by 10 % over 8 iterations (the bfloat16 rounding floor of sigma)
        const double r = *std::max_element(D.rn.begin(), D.rn.end());
        if (D.best_rn < 0 || r < 0.9 * D.best_rn) {
            D.best_rn = r;
            D.stall = 0;
        } else if (++D.stall >= 8) {
            D.done = true;
            return STPCI_OK;
        }
    }
    if (conv || D.it >= D.max_iter) {
        D.done = true;
        return STPCI_OK;
    }
    // corrections for the unconverged roots (Eq. sparsePreconditioner: the
    // Ritz pass formed t_j for every root; with eps > 0 the entries below
    // eps ||t_j|| are dropped, ||t_j||^2 read where the Ritz pass left it)
    std::vector<char> corr(k, 0);
    int nt = 0;
    for (int j = 0; j < k; ++j)
        if (D.rn[j] > D.tol) {
            corr[j] = 1;
            ++nt;
        }
    const double eps = D.opts.eps_drop;
    if (eps > 0.0) {
        int slot[PRE_MAX];
        for (int q = 0; q < k; ++q) slot[q] = ritz_slot(q, 1);
        if ((s = d.hip(launch_eps_drop(d.cx, c->d_T.p, N, N, k, slot, (const double*)d.small(kRitzOff), 1, eps,
                                       c->stream),
                       "eps drop")))
            return s;
        // the norms after the drop, fetched with the first Gram matrix
        if ((s = d.issue_pair_dots((char*)c->d_T.p, (char*)c->d_T.p, k, 0, kNrmOff))) return s;
    }
    int mm = m;
    // restart when the space would overflow (thick restart with the
    // previous Ritz vectors, "GD+k"): the new basis is V Q, Q = the k lowest
    // Ritz vectors' coefficients Y_k, then the previous iteration's Ritz
    // vectors (coefficients in this basis) orthogonalised against them, then
    // further Ritz vectors while room is left; W <- W Q, G <- Q^H A Q.  Both
    // kinds lie in the basis, so no sigma is repeated; keeping the previous
    // iterate is what lets a small basis (a space where only a few vectors
    // fit the device) converge as a locally optimal iteration.
    std::vector<cplx> Pc;   // coefficients of this iteration's Ritz vectors in the basis after this step
    int Pc_rows = 0;
    if (mm + nt > D.mmax) {
        const int room = std::max(k, std::min(D.kr_max, D.mmax - nt));
        std::vector<std::vector<cplx>> cols;
        auto ortho_push = [&](std::vector<cplx> v) {
            for (int pass = 0; pass < 2; ++pass)
                for (const auto& q : cols) {
                    cplx dot(0, 0);
                    for (int i = 0; i < mm; ++i) dot += std::conj(q[i]) * v[i];
                    for (int i = 0; i < mm; ++i) v[i] -= dot * q[i];
                }
            double nrm = 0;
            for (int i = 0; i < mm; ++i) nrm += std::norm(v[i]);
            nrm = std::sqrt(nrm);
            if (nrm < 1e-8) return false;
            for (int i = 0; i < mm; ++i) v[i] /= nrm;
            cols.push_back(std::move(v));
            return true;
        };
        for (int j = 0; j < k; ++j) {
            std::vector<cplx> v(mm);
            for (int i = 0; i < mm; ++i) v[i] = Y[(size_t)i * mm + j];
            cols.push_back(std::move(v));
        }
        // where room is short of 2k, the previous iterates of the unconverged
        // roots go first, largest residual first (a converged root gains
        // nothing from its own)
        std::vector<int> porder(k);
        std::iota(porder.begin(), porder.end(), 0);
        if (room < 2 * k)
            std::stable_sort(porder.begin(), porder.end(), [&](int a, int b) {
                if (corr[a] != corr[b]) return corr[a] > corr[b];
                return corr[a] && D.rn[a] > D.rn[b];
            });
        for (int jj = 0; jj < k && (int)cols.size() < room && D.prev_rows > 0; ++jj) {
            const int j = porder[jj];
            std::vector<cplx> v(mm, cplx(0, 0));
            for (int i = 0; i < std::min(D.prev_rows, mm); ++i) v[i] = D.prev_coef[(size_t)i * k + j];
            ortho_push(std::move(v));
        }
        for (int j = k; j < mm && (int)cols.size() < room; ++j) {
            std::vector<cplx> v(mm);
            for (int i = 0; i < mm; ++i) v[i] = Y[(size_t)i * mm + j];
            ortho_push(std::move(v));
        }
        const int kr = (int)cols.size();
        std::vector<cplx> Yr((size_t)mm * kr);
        for (int i = 0; i < mm; ++i)
            for (int j = 0; j < kr; ++j) Yr[(size_t)i * kr + j] = cols[j][i];
        // G' = Q^H A Q on the host
        std::vector<cplx> AQ((size_t)mm * kr, cplx(0, 0));
        for (int i = 0; i < mm; ++i)
            for (int l = 0; l < mm; ++l) {
                const cplx a = A[(size_t)i * mm + l];
                for (int j = 0; j < kr; ++j) AQ[(size_t)i * kr + j] += a * Yr[(size_t)l * kr + j];
            }
        std::vector<cplx> Gn((size_t)kr * kr, cplx(0, 0));
        for (int a2 = 0; a2 < kr; ++a2)
            for (int b2 = 0; b2 < kr; ++b2) {
                cplx v(0, 0);
                for (int i = 0; i < mm; ++i) v += std::conj(Yr[(size_t)i * kr + a2]) * AQ[(size_t)i * kr + b2];
                Gn[(size_t)a2 * kr + b2] = v;
            }
        if ((s = d.put_small(Yr, kYOff))) return s;
        if ((s = d.hip(launch_combine_inplace(d.cx, c->d_V.p, N, mm, d.small(kYOff), kr, N, c->stream),
                       "restart V")))
            return s;
        if ((s = d.hip(launch_combine_inplace(d.cx, c->d_W.p, N, mm, d.small(kYOff), kr, N, c->stream),
                       "restart W")))
            return s;
        std::fill(D.G.begin(), D.G.end(), cplx(0, 0));
        for (int a2 = 0; a2 < kr; ++a2)
            for (int b2 = 0; b2 < kr; ++b2) Gat(a2, b2) = Gn[(size_t)a2 * kr + b2];
        mm = kr;
        D.m = kr;
        // this iteration's Ritz vectors are the first k new basis vectors
        Pc.assign((size_t)kr * k, cplx(0, 0));
        for (int j = 0; j < k; ++j) Pc[(size_t)j * k + j] = cplx(1, 0);
        Pc_rows = kr;
    } else {
        Pc = Yk;
        Pc_rows = mm;
    }
    D.prev_coef = std::move(Pc);
    D.prev_rows = Pc_rows;
    // block orthonormalisation of the corrections: two classical Gram-Schmidt
    // passes against V, then two Cholesky QR passes among themselves; a
    // direction that keeps less than 1e-8 of its norm lies in the span
    // (linear dependence) and is dropped.  The passes run over all k
    // corrections (those of converged roots are left out of the Cholesky
    // factor), so that the columns stay where the Ritz pass wrote them.
    const bool fuse = k <= 4;   // the Gram matrices come with the passes that form the vectors
    // the Gram matrix Gm[t * ns + i] = <src_i | src_t> of ns vectors (a fused
    // pass leaves it as a 4 x 4 block of complex slots, a dot-product pass
    // compact), with the corrections' squared norms before orthogonalisation
    // (after the eps drop, queued beside it; else from the Ritz pass)
    auto read_gram = [&](int ns, bool padded, std::vector<cplx>& Gm, std::vector<double>* ref) -> stpci_status {
        const bool norms = ref && eps > 0.0;
        const size_t from = norms ? kNrmOff : kGramOff;
        const size_t gd = padded ? 32 : (size_t)ns * ns * (d.cx ? 2 : 1);
        std::vector<double> raw;
        stpci_status st2 = d.get_doubles(from, (kGramOff - from) / 8 + gd, raw);
        if (st2) return st2;
        const double* gr = raw.data() + (kGramOff - from) / 8;
        Gm.assign((size_t)ns * ns, cplx(0, 0));
        for (int t = 0; t < ns; ++t)
            for (int i = 0; i < ns; ++i) {
                const size_t at = padded ? (size_t)2 * (4 * t + i) : (size_t)(t * ns + i) * (d.cx ? 2 : 1);
                Gm[(size_t)t * ns + i] = cplx(gr[at], (padded || d.cx) ? gr[at + 1] : 0.0);
            }
        if (ref) {
            ref->assign(ns, 1.0);
            for (int t = 0; t < ns; ++t)
                (*ref)[t] = norms ? raw[(size_t)Dav::pair_slot(t, k) * (d.cx ? 2 : 1)] : tn2[t];
        }
        return STPCI_OK;
    };
    // classical Gram-Schmidt against V; the second pass only where the first
    // removed more than half of a correction's squared norm (the criterion
    // of Daniel, Gragg, Kaufman and Stewart, 1976, with 1/sqrt(2)), read from
    // the Gram matrix of the fused first pass (without it: always two passes)
    std::vector<cplx> Gm0;
    std::vector<double> ref0;
    if ((s = d.issue_dots(c->d_V.p, mm, c->d_T.p, k, 0))) return s;
    if (fuse) {
        if ((s = d.hip(launch_comb_gram(d.cx, c->d_V.p, N, mm, d.small(kDotsOff), c->d_T.p, k, N, 3,
                                        (double*)c->d_partial.p, (double*)d.small(kGramOff), c->stream),
                       "cgs")))
            return s;
        if ((s = read_gram(k, true, Gm0, &ref0))) return s;
    } else if ((s = d.subtract_queued(c->d_V.p, mm, k, c->d_T.p))) {
        return s;
    }
    bool second = !fuse;
    for (int t = 0; t < k && fuse; ++t)
        if (corr[t] && Gm0[(size_t)t * k + t].real() < 0.5 * ref0[t]) second = true;
    if (second) {
        if ((s = d.issue_dots(c->d_V.p, mm, c->d_T.p, k, 0))) return s;
        if (fuse) {
            if ((s = d.hip(launch_comb_gram(d.cx, c->d_V.p, N, mm, d.small(kDotsOff), c->d_T.p, k, N, 3,
                                            (double*)c->d_partial.p, (double*)d.small(kGramOff), c->stream),
                           "cgs")))
                return s;
        } else {
            if ((s = d.subtract_queued(c->d_V.p, mm, k, c->d_T.p))) return s;
            if ((s = d.issue_dots(c->d_T.p, k, c->d_T.p, k, 0, kGramOff))) return s;
        }
        if ((s = read_gram(k, fuse, Gm0, &ref0))) return s;
    }
    D.cgs_passes += second ? 2 : 1;
    // Cholesky QR: T_keep = Q R, Q = T R^-1 written to V[mm..] (first pass)
    // and re-orthonormalised in place (second pass)
    const int room = D.mmax - mm;
    std::vector<int> keep;
    for (int qr = 0; qr < 2; ++qr) {
        const int ns = (qr == 0) ? k : (int)keep.size();
        if (ns == 0) break;
        std::vector<cplx> Gm;
        std::vector<double> ref(ns, 1.0);
        if (qr == 0) {
            Gm = Gm0;
            ref = ref0;
        } else if ((s = read_gram(ns, ns <= 4, Gm, nullptr))) {
            return s;
        }
        std::vector<cplx> R((size_t)ns * ns, cplx(0, 0));
        std::vector<int> kept;
        for (int t = 0; t < ns; ++t) {
            if (qr == 0 && !corr[t]) continue;
            double r2 = Gm[(size_t)t * ns + t].real();
            for (int i : kept) {
                cplx v = Gm[(size_t)t * ns + i];
                for (int j : kept) {
                    if (j >= i) break;
                    v -= std::conj(R[(size_t)j * ns + i]) * R[(size_t)j * ns + t];
                }
                R[(size_t)i * ns + t] = v / R[(size_t)i * ns + i];
                r2 -= std::norm(R[(size_t)i * ns + t]);
            }
            if (r2 <= 1e-16 * ref[t] || (int)kept.size() >= room) continue;
            R[(size_t)t * ns + t] = std::sqrt(r2);
            kept.push_back(t);
        }
        // Y = R^-1 on the kept columns (upper triangular), ns x kept
        const int nk = (int)kept.size();
        std::vector<cplx> Yq((size_t)ns * std::max(nk, 1), cplx(0, 0));
        for (int jj = 0; jj < nk; ++jj) {
            // solve R[kept, kept] y = e_jj by back substitution over kept indices
            std::vector<cplx> y(nk, cplx(0, 0));
            for (int ii = jj; ii >= 0; --ii) {
                cplx v = (ii == jj) ? cplx(1, 0) : cplx(0, 0);
                for (int ll = ii + 1; ll <= jj; ++ll) v -= R[(size_t)kept[ii] * ns + kept[ll]] * y[ll];
                y[ii] = v / R[(size_t)kept[ii] * ns + kept[ii]];
            }
            for (int ii = 0; ii <= jj; ++ii) Yq[(size_t)kept[ii] * nk + jj] = y[ii];
        }
        if (qr == 0) {
            keep = kept;
            if (nk == 0) break;
            if ((s = d.put_small(Yq, kYOff))) return s;
            // a second pass only where the first can lose orthogonality: it
            // leaves the directions orthonormal to about kappa eps, kappa the
            // condition number of their Gram matrix (at most 100 here: one
            // pass is enough)
            {
                std::vector<cplx> Gk((size_t)nk * nk);
                for (int a = 0; a < nk; ++a)
                    for (int b = 0; b < nk; ++b) Gk[(size_t)a * nk + b] = Gm[(size_t)kept[b] * ns + kept[a]];
                std::vector<double> ev;
                std::vector<cplx> evec;
                herm_eig(nk, Gk, ev, evec);
                if (ev[0] > 0.0 && ev[nk - 1] <= 100.0 * ev[0]) {
                    if ((s = d.hip(launch_combine(d.cx, c->d_T.p, nullptr, N, ns, d.small(kYOff), nk, nullptr,
                                                  d.vec(c->d_V, mm), nullptr, N, 0, c->stream),
                                   "cholqr")))
                        return s;
                    break;
                }
            }
            if (nk <= 4) {
                if ((s = d.hip(launch_comb_gram(d.cx, c->d_T.p, N, ns, d.small(kYOff), d.vec(c->d_V, mm), nk, N, 0,
                                                (double*)c->d_partial.p, (double*)d.small(kGramOff), c->stream),
                               "cholqr")))
                    return s;
            } else {
                if ((s = d.hip(launch_combine(d.cx, c->d_T.p, nullptr, N, ns, d.small(kYOff), nk, nullptr,
                                              d.vec(c->d_V, mm), nullptr, N, 0, c->stream),
                               "cholqr")))
                    return s;
                if ((s = d.issue_dots(d.vec(c->d_V, mm), nk, d.vec(c->d_V, mm), nk, 0, kGramOff))) return s;
            }
        } else {
            if (nk < ns) break;   // the second pass dropped a direction: keep the first pass' result
            if ((s = d.put_small(Yq, kYOff))) return s;
            if ((s = d.hip(launch_combine_inplace(d.cx, d.vec(c->d_V, mm), N, ns, d.small(kYOff), nk, N, c->stream),
                           "cholqr2")))
                return s;
        }
    }
    const int added = (int)keep.size();
    if (added == 0) {  // no new direction: stagnation
        D.done = true;
        return STPCI_OK;
    }
    D.nv = added;
    return STPCI_OK;
}

namespace stp {

stpci_status dav_begin(stpci_ctx* c, const stpci_dav_opts* o) {
    stpci_status s = prepare(c);
    if (s) return s;
    if ((s = hip_check(c, hipSetDevice(c->device), "hipSetDevice"))) return s;
    const int64_t N = c->hs.sp.ndets;
    if (o->k < 1 || o->k > 16 || o->k > N) return set_err(c, STPCI_EINVAL, "k must be in [1, min(16, n_dets)]");
    if (o->certify != 0 && o->certify != 1) return set_err(c, STPCI_EINVAL, "certify must be 0 or 1");
    // with certify, one root more than requested is converged internally, so
    // that the last requested root also has an upper neighbour for its gap
    const bool extra = o->certify || (o->refine_tol_energy > 0.0 && o->precision != STPCI_FP64);
    const int k_run = (extra && o->k < 16 && o->k < N) ? o->k + 1 : o->k;
    if (o->precision != STPCI_FP64 && o->precision != STPCI_FP32 && o->precision != STPCI_BF16)
        return set_err(c, STPCI_EINVAL, "unknown precision");
    if (!(o->eps_drop >= 0.0 && o->eps_drop < 1.0))
        return set_err(c, STPCI_EINVAL, "eps_drop must lie in [0, 1)");
    if (!(o->refine_tol_energy >= 0.0) || !std::isfinite(o->refine_tol_energy))
        return set_err(c, STPCI_EINVAL, "refine_tol_energy must be finite and >= 0");
    c->dav = DavState{};
    c->dav.opts = *o;
    c->dav.opts.k = k_run;
    c->dav.k_req = o->k;
    c->dav.final_tol = o->tol_residual > 0 ? o->tol_residual : 1e-8;
    c->history.clear();
    c->hist_k = k_run;
    c->nsigma[0] = c->nsigma[1] = c->nsigma[2] = 0;
    // phase A: reduced-precision contractions to a residual their products
    // resolve (FP32 about 1e-7 relative, BF16 about 2^-9)
    if (o->precision == STPCI_FP32)
        return dav_start(c, STPCI_FP32, o->guess_dev, std::max(c->dav.final_tol, 1e-4));
    if (o->precision == STPCI_BF16)
        return dav_start(c, STPCI_BF16, o->guess_dev, std::max(c->dav.final_tol, 2e-2));
    return dav_start(c, STPCI_FP64, o->guess_dev, c->dav.final_tol);
}

// The pending sigma work of the run: n vectors from V[m] into W[m].
bool dav_pending(stpci_ctx* c, const void** in, void** out, int* n, stpci_precision* prec) {
    DavState& D = c->dav;
    if (!D.active || D.done || D.nv == 0) return false;
    const size_t vb = (size_t)c->hs.sp.ndets * scalar_bytes(c);
    *in = (const char*)c->d_V.p + (size_t)D.m * vb;
    *out = (char*)c->d_W.p + (size_t)D.m * vb;
    *n = D.nv;
    *prec = D.prec;
    return true;
}

// Advance after the pending products; moves from a reduced-precision phase to
// FP64 refinement (guess = its Ritz vectors) when the former ends.
stpci_status dav_step_after_sigma(stpci_ctx* c, int* finished) {
    DavState& D = c->dav;
    D.products_ready = false;
    stpci_status s = dav_advance(c);
    if (s) return s;
    if (D.done && D.prec != STPCI_FP64) {
        D.it_prev += D.it;
        const int keep = D.it_prev;
        if ((s = dav_start(c, STPCI_FP64, c->d_X.p, D.final_tol))) return s;
        D.it_prev = keep;
    }
    *finished = D.done ? 1 : 0;
    if (D.done) D.active = false;
    return STPCI_OK;
}

// Error bounds of the converged roots (Methods, Eigenvalue Bound Analysis):
// the gap theorem |dE_j| <= ||r_j||^2 / gamma_j with the lower bound of the gap
// from the neighbouring Ritz pairs, gamma_0^- = (E_1 - ||r_1||) - E_0 (Eq.
// gammaLowerBound) and, for j > 0, also E_j - (E_{j-1} + ||r_{j-1}||) (the
// neighbour below can lie at most its residual norm above its Ritz value).
// Valid when no eigenvalue lies between the Ritz values (none missed);
// gamma_j <= 0 gives no bound (infinity).  The last root run has no
// neighbour above: NaN.
static void certificate(const DavState& D, std::vector<double>& gam, std::vector<double>& bnd) {
    const int kr = D.opts.k;
    gam.assign(kr, std::nan(""));
    bnd.assign(kr, std::nan(""));
    for (int j = 0; j + 1 < kr; ++j) {
        double g = (D.theta[j + 1] - D.rn[j + 1]) - D.theta[j];
        if (j > 0) g = std::min(g, D.theta[j] - (D.theta[j - 1] + D.rn[j - 1]));
        gam[j] = g;
        bnd[j] = g > 0 ? D.rn[j] * D.rn[j] / g : std::numeric_limits<double>::infinity();
    }
}

stpci_status dav_collect(stpci_ctx* c, double* energies, double* resid, void* vecs_dev, int* n_iter) {
    DavState& D = c->dav;
    const int k = D.k_req > 0 ? D.k_req : D.opts.k;
    for (int j = 0; j < k; ++j) {
        energies[j] = D.theta[j];
        resid[j] = D.rn[j];
    }
    certificate(D, c->cert_gamma, c->cert_bound);
    c->cert_k = k;
    if (n_iter) *n_iter = D.it_prev + D.it;
    if (vecs_dev) {
        const size_t vb = (size_t)c->hs.sp.ndets * scalar_bytes(c) * k;
        stpci_status s = hip_check(c, hipMemcpyAsync(vecs_dev, c->d_X.p, vb, hipMemcpyDeviceToDevice, c->stream),
                                   "vecs out");
        if (s) return s;
    }
    stpci_status s = hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (s) return s;
    return D.converged ? STPCI_OK : set_err(c, STPCI_ENOCONV, "Davidson did not converge");
}

}  // namespace stp

extern "C" stpci_status stpci_davidson(stpci_ctx* c, const stpci_dav_opts* o, double* energies, double* resid,
                                       void* vecs_dev, int* n_iter) {
    if (!c || !o || !energies || !resid) return STPCI_EINVAL;
    stpci_status s = dav_begin(c, o);
    if (s) return s;
    for (;;) {
        const void* in;
        void* out;
        int n;
        stpci_precision prec;
        if (!dav_pending(c, &in, &out, &n, &prec)) break;
        if ((s = sigma_impl(c, in, out, n, prec))) return s;
        int fin = 0;
        if ((s = dav_step_after_sigma(c, &fin))) return s;
        if (fin) break;
    }
    return dav_collect(c, energies, resid, vecs_dev, n_iter);
}

extern "C" stpci_status stpci_dav_certificate(const stpci_ctx* c, double* gamma_lower, double* bound) {
    if (!c) return STPCI_EINVAL;
    if (c->cert_k <= 0) return set_err(const_cast<stpci_ctx*>(c), STPCI_ESTATE, "no Davidson run to certify");
    for (int j = 0; j < c->cert_k; ++j) {
        if (gamma_lower) gamma_lower[j] = c->cert_gamma[j];
        if (bound) bound[j] = c->cert_bound[j];
    }
    return STPCI_OK;
}

extern "C" stpci_status stpci_dav_stats(const stpci_ctx* c, int* sigma_fp64, int* sigma_fp32) {
    if (!c) return STPCI_EINVAL;
    if (sigma_fp64) *sigma_fp64 = c->nsigma[0];
    if (sigma_fp32) *sigma_fp32 = c->nsigma[1] + c->nsigma[2];
    return STPCI_OK;
}

extern "C" stpci_status stpci_dav_sigma_count(const stpci_ctx* c, stpci_precision prec, int* n_vectors) {
    if (!c || !n_vectors || prec < STPCI_FP64 || prec > STPCI_BF16) return STPCI_EINVAL;
    *n_vectors = c->nsigma[(int)prec];
    return STPCI_OK;
}

extern "C" stpci_status stpci_dav_history_dc(const stpci_ctx* c, int cap, double* dc) {
    if (!c || !dc || cap < 0) return STPCI_EINVAL;
    const int n = (int)c->history.size(), k = c->hist_k;
    for (int i = 0; i < std::min(n, cap); ++i)
        for (int j = 0; j < k; ++j) dc[i * k + j] = c->history[i].dc[j];
    return STPCI_OK;
}

extern "C" stpci_status stpci_dav_history(const stpci_ctx* c, int* n_iter, int cap, double* energies,
                                          double* resid) {
    if (!c) return STPCI_EINVAL;
    int n = (int)c->history.size();
    if (n_iter) *n_iter = n;
    int k = c->hist_k;
    for (int i = 0; i < std::min(n, cap); ++i)
        for (int j = 0; j < k; ++j) {
            if (energies) energies[i * k + j] = c->history[i].e[j];
            if (resid) resid[i * k + j] = c->history[i].r[j];
        }
    return STPCI_OK;
}
