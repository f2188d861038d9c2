"""Python binding of libstpci (MI355X categorical STP-DAS CI: sigma build and Davidson).

Argument marshalling only: every step of the sigma build and of the Davidson
iteration runs in the library's HIP kernels and its C++ driver.  PyTorch
supplies device memory (tensor data pointers) and the stream.  Importing this
package fails loudly when the compiled library is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstpci.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libstpci.so is not built; run `python paper_2505_20375_amd/build.py` "
                      "(or __graft_entry__.build()) first")

# PyTorch bundles its own HIP runtime (SONAME libamdhip64.so.7).  Loading
# torch first makes libstpci's dependency resolve to that same runtime, so the
# process holds exactly one HIP runtime shared by torch's allocations, streams
# and this library's kernels.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EHIP, ENOCONV, ESTATE = 0, -1, -2, -3, -4, -5
REAL64, COMPLEX128 = 0, 1
FP64, FP32, BF16 = 0, 1, 2
_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EHIP: "EHIP", ENOCONV: "ENOCONV", ESTATE: "ESTATE"}


class DavOpts(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("max_iter", ctypes.c_int), ("max_subspace", ctypes.c_int),
                ("tol_residual", ctypes.c_double), ("eps_drop", ctypes.c_double), ("precision", ctypes.c_int),
                ("refine_tol_energy", ctypes.c_double), ("guess_dev", ctypes.c_void_p), ("certify", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("n_orb", ctypes.c_int), ("scalar", ctypes.c_int), ("spin_free", ctypes.c_int),
                ("h", ctypes.c_void_p), ("g", ctypes.c_void_p), ("e_core", ctypes.c_double),
                ("n_elec", ctypes.c_int), ("n_sub", ctypes.c_int), ("sub_size", ctypes.POINTER(ctypes.c_int)),
                ("win_lo", ctypes.POINTER(ctypes.c_int)), ("win_hi", ctypes.POINTER(ctypes.c_int)),
                ("opts", ctypes.POINTER(DavOpts))]


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_D = ctypes.c_double
_IP = ctypes.POINTER(ctypes.c_int)
_I64P = ctypes.POINTER(ctypes.c_int64)
_DP = ctypes.POINTER(ctypes.c_double)
_SIGS = {
    "stpci_create": ([ctypes.POINTER(_P), _I, _P], _I),
    "stpci_destroy": ([_P], None),
    "stpci_last_error": ([_P], ctypes.c_char_p),
    "stpci_set_integrals": ([_P, _I, _I, _I, _P, _P, _D], _I),
    "stpci_set_space": ([_P, _I, _I, _IP, _IP, _IP], _I),
    "stpci_space_info": ([_P, _I64P, _IP, _I64P, _DP, _DP], _I),
    "stpci_category": ([_P, _I, _IP, _I64P, _I64P], _I),
    "stpci_work_counts": ([_P, _DP, _DP, _I64P, _IP], _I),
    "stpci_address_to_det": ([_P, _I64, ctypes.POINTER(ctypes.c_uint64)], _I),
    "stpci_sigma": ([_P, _P, _P, _I, _I], _I),
    "stpci_sigma_noalloc": ([_P, _P, _P, _I, _I], _I),
    "stpci_csc_compress": ([_P, _P, ctypes.c_double, _P, _P, _P, _I64, _I64P], _I),
    "stpci_csc_expand": ([_P, _P, _P, _P, _P], _I),
    "stpci_sigma_csc": ([_P, _P, _P, _P, _P], _I),
    "stpci_test_exp_search": ([_P, _I64, _I64, ctypes.c_uint32], _I64),
    "stpci_test_exp_search_dev": ([_P, _I64, _P, _P, _P, _I64, _P], _I),
    "stpci_sigma_noalloc_max_bytes": ([], _I64),
    "stpci_diagonal": ([_P, _P], _I),
    "stpci_davidson": ([_P, ctypes.POINTER(DavOpts), _DP, _DP, _P, _IP], _I),
    "stpci_dav_history": ([_P, _IP, _I, _DP, _DP], _I),
    "stpci_dav_stats": ([_P, _IP, _IP], _I),
    "stpci_dav_certificate": ([_P, _DP, _DP], _I),
    "stpci_footprint_bytes": ([_P, ctypes.POINTER(DavOpts)], _I64),
    "stpci_dav_begin": ([_P, ctypes.POINTER(DavOpts)], _I),
    "stpci_dav_sigma_batched": ([ctypes.POINTER(ctypes.c_void_p), _I], _I),
    "stpci_dav_finish_step": ([_P, _IP], _I),
    "stpci_dav_result": ([_P, _DP, _DP, _P, _IP], _I),
    "stpci_dav_sigma_count": ([_P, _I, _IP], _I),
    "stpci_dav_history_dc": ([_P, _I, _DP], _I),
    "stpci_profile": ([_P, _I], _I),
    "stpci_kernel_time": ([_P, ctypes.c_char_p, _I64P, _DP], _I),
    "stpci_test_heev": ([_I, _P, _P, _P], _I),
    "stpci_test_moves": ([_P, _I64, _I64P, _I64P], _I),
    "stpci_test_pairs": ([_P, _I64, _I64P, _I64P], _I),
    "stpci_test_pair_groups": ([_P, _I64P, _I64P, _IP], _I),
    "stpci_test_sb": ([_P, _I64, _I64P, _I64P], _I),
    "stpci_sb_counts": ([_P, _I, _DP, _I64P], _I),
    "stpci_test_precond": ([_P, _P, _P, _I, _DP, _D], _I),
    "stpci_test_ritz": ([_P, _P, _P, _I, _DP, _DP, _I, _DP, _P, _P, _DP], _I),
    "stpci_test_dav_cgs_passes": ([_P, _IP], _I),
    "stpci_pair_counts": ([_P, _DP, _I64P, _IP], _I),
    "stpci_set_sigma_kernel": ([_P, ctypes.c_char_p], _I),
    "stpci_sigma_kernel": ([_P, ctypes.POINTER(ctypes.c_char_p)], _I),
    "stpci_server_create": ([ctypes.POINTER(_P), _I, _P, _I64, _I], _I),
    "stpci_server_phase_times": ([_P, _DP, _DP, _DP], _I),
    "stpci_server_destroy": ([_P], None),
    "stpci_server_last_error": ([_P], ctypes.c_char_p),
    "stpci_server_submit": ([_P, ctypes.POINTER(Request), _IP], _I),
    "stpci_server_cancel": ([_P, _I], _I),
    "stpci_server_tick": ([_P, _IP, _IP], _I),
    "stpci_server_result": ([_P, _I, _IP, _DP, _DP, _IP, _DP, _DP, _DP], _I),
    "stpci_server_request_info": ([_P, _I, _I64P, _DP, _I64P, _IP], _I),
    "stpci_server_stats": ([_P, _I64P, _I64P, _IP, _I64P, _I64P], _I),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def dav_sigma_batched(ctxs):
    """stpci_dav_sigma_batched: the pending sigma products of several
    step-wise Davidson runs (Context objects on one device), each on its own
    stream, launched back to back."""
    arr = (ctypes.c_void_p * len(ctxs))(*[c._h.value for c in ctxs])
    st = _lib.stpci_dav_sigma_batched(arr, len(ctxs))
    if st != OK:
        msg = "stpci_dav_sigma_batched failed"
        for c in ctxs:
            m = _lib.stpci_last_error(c._h).decode()
            if m:
                msg += ": " + m
                break
        raise StpciError(st, msg)


def test_exp_search(a, i, x):
    """The exponential search of the compressed sigma build on the host:
    lowest j >= i with a[j] >= x, or len(a)."""
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return int(_lib.stpci_test_exp_search(a.ctypes.data_as(ctypes.c_void_p), len(a), int(i), int(x)))


def test_exp_search_dev(a, starts, xs, out, stream=None):
    """The same search on the device for every (start, x) pair (torch tensors:
    a int32 holding uint32 values, starts int64, xs int32, out int64)."""
    st = _lib.stpci_test_exp_search_dev(_ptr(a), a.numel(), _ptr(starts), _ptr(xs), _ptr(out), xs.numel(),
                                        _P(stream) if stream else None)
    if st != OK:
        raise StpciError(st, "stpci_test_exp_search_dev failed")


def sigma_noalloc_max_bytes():
    """Size of the static scratch array of stpci_sigma_noalloc (bytes)."""
    return int(_lib.stpci_sigma_noalloc_max_bytes())


class StpciError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_NAMES.get(status, status), msg))
        self.status = status


def _iarr(xs):
    a = (ctypes.c_int * len(xs))(*[int(x) for x in xs])
    return a


def _ptr(t):
    """Device pointer of a torch tensor (or an int)."""
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class SpaceInfo:
    n_dets: int
    n_cat: int
    bytes_per_vec: int
    w_sigma_macs: float
    nnz_h: float


class Context:
    """One CI problem on one device (device=-1: host-only, no GPU calls)."""

    def __init__(self, device: int = 0, stream=None):
        h = _P()
        if device >= 0 and stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        st = _lib.stpci_create(ctypes.byref(h), int(device), _P(stream) if stream else None)
        if st != OK:
            raise StpciError(st, "stpci_create failed (device %d)" % device)
        self._h = h
        self.device = device
        self.cplx = True

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.stpci_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def _check(self, st):
        if st != OK:
            raise StpciError(st, _lib.stpci_last_error(self._h).decode())
        return st

    # -- problem definition -------------------------------------------------
    def set_integrals(self, h, g, spin_free=False, e_core=0.0):
        cplx = np.iscomplexobj(h) or np.iscomplexobj(g)
        dt = np.complex128 if cplx else np.float64
        h = np.ascontiguousarray(h, dtype=dt)
        g = np.ascontiguousarray(g, dtype=dt)
        n = h.shape[0]
        self._check(_lib.stpci_set_integrals(self._h, n, COMPLEX128 if cplx else REAL64, int(bool(spin_free)),
                                             h.ctypes.data_as(_P), g.ctypes.data_as(_P), float(e_core)))
        self.cplx = bool(cplx)

    def set_space(self, n_elec, sub, lo=None, hi=None):
        lo = list(lo) if lo is not None else [0] * len(sub)
        hi = list(hi) if hi is not None else list(sub)
        self._check(_lib.stpci_set_space(self._h, int(n_elec), len(sub), _iarr(sub), _iarr(lo), _iarr(hi)))
        self.n_sub = len(sub)

    def space_info(self) -> SpaceInfo:
        nd, nb = ctypes.c_int64(), ctypes.c_int64()
        nc = ctypes.c_int()
        w, z = ctypes.c_double(), ctypes.c_double()
        self._check(_lib.stpci_space_info(self._h, ctypes.byref(nd), ctypes.byref(nc), ctypes.byref(nb),
                                          ctypes.byref(w), ctypes.byref(z)))
        return SpaceInfo(nd.value, nc.value, nb.value, w.value, z.value)

    def work_counts(self):
        """(w1, w2, intermediate determinants, max moves per determinant)."""
        w1, w2 = ctypes.c_double(), ctypes.c_double()
        ni, md = ctypes.c_int64(), ctypes.c_int()
        self._check(_lib.stpci_work_counts(self._h, ctypes.byref(w1), ctypes.byref(w2), ctypes.byref(ni),
                                           ctypes.byref(md)))
        return w1.value, w2.value, ni.value, md.value

    def category(self, i):
        occ = (ctypes.c_int * 8)()
        off, n = ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.stpci_category(self._h, int(i), occ, ctypes.byref(off), ctypes.byref(n)))
        return tuple(occ[:self.n_sub]), off.value, n.value

    def address_to_det(self, addr) -> int:
        b = ctypes.c_uint64()
        self._check(_lib.stpci_address_to_det(self._h, int(addr), ctypes.byref(b)))
        return b.value

    # -- device work ----------------------------------------------------------
    def sigma(self, c, out, n_vec=1, precision=FP64):
        self._check(_lib.stpci_sigma(self._h, _ptr(c), _ptr(out), int(n_vec), int(precision)))

    def sigma_noalloc(self, c, out, n_vec=1, precision=FP64):
        """stpci_sigma_noalloc: the same sigma without device allocation
        (workspace from the library's static scratch array)."""
        self._check(_lib.stpci_sigma_noalloc(self._h, _ptr(c), _ptr(out), int(n_vec), int(precision)))

    def diagonal(self, out):
        self._check(_lib.stpci_diagonal(self._h, _ptr(out)))

    # -- categorical compression (stpci_csc_*) --------------------------------
    def csc_compress(self, x, thresh=0.0):
        """(cat_ptr, a, v) device tensors of the compressed form of the dense
        vector x: per category the entries with |x_i| >= thresh, ascending
        local addresses (uint32 stored in int32 tensors)."""
        import torch
        info = self.space_info()
        cat_ptr = torch.empty(info.n_cat + 1, dtype=torch.int64, device=x.device)
        nnz = ctypes.c_int64()
        st = _lib.stpci_csc_compress(self._h, _ptr(x), float(thresh), _ptr(cat_ptr), None, None, 0,
                                     ctypes.byref(nnz))
        if st not in (OK, ENOMEM):
            self._check(st)
        n = max(int(nnz.value), 1)
        a = torch.empty(n, dtype=torch.int32, device=x.device)
        v = torch.empty(n, dtype=x.dtype, device=x.device)
        self._check(_lib.stpci_csc_compress(self._h, _ptr(x), float(thresh), _ptr(cat_ptr), _ptr(a), _ptr(v), n,
                                            ctypes.byref(nnz)))
        return cat_ptr, a[:nnz.value], v[:nnz.value]

    def csc_expand(self, cat_ptr, a, v, out):
        self._check(_lib.stpci_csc_expand(self._h, _ptr(cat_ptr), _ptr(a), _ptr(v), _ptr(out)))

    def sigma_csc(self, cat_ptr, a, v, out):
        """out = H c for c given compressed (stpci_sigma_csc)."""
        self._check(_lib.stpci_sigma_csc(self._h, _ptr(cat_ptr), _ptr(a), _ptr(v), _ptr(out)))

    def davidson(self, k=1, tol=1e-8, max_iter=100, max_subspace=0, eps_drop=0.0, precision=FP64,
                 refine_tol_energy=0.0, guess=None, vecs=None, allow_noconv=False, certify=False):
        o = DavOpts(int(k), int(max_iter), int(max_subspace), float(tol), float(eps_drop), int(precision),
                    float(refine_tol_energy), _ptr(guess).value if guess is not None else None, int(bool(certify)))
        e = (ctypes.c_double * k)()
        r = (ctypes.c_double * k)()
        it = ctypes.c_int()
        self._last_k = self._run_k(k, precision, refine_tol_energy, certify)
        self._cert_k = int(k)
        st = _lib.stpci_davidson(self._h, ctypes.byref(o), e, r, _ptr(vecs) if vecs is not None else None,
                                 ctypes.byref(it))
        if st != OK and not (allow_noconv and st == ENOCONV):
            self._check(st)
        return np.array(e[:]), np.array(r[:]), it.value, st

    def _run_k(self, k, precision, refine_tol_energy, certify):
        """Roots a run carries (one more than k with certify, or with the
        energy stop of a reduced-precision run), as the history records them."""
        extra = bool(certify) or (refine_tol_energy > 0 and int(precision) != FP64)
        return int(k) + (1 if extra and k < 16 and k < self.space_info().n_dets else 0)

    # -- step-wise Davidson (stpci_dav_begin ... stpci_dav_result) -----------
    @staticmethod
    def _opts(k, tol, max_iter, max_subspace, eps_drop, precision, refine_tol_energy, certify):
        return DavOpts(int(k), int(max_iter), int(max_subspace), float(tol), float(eps_drop), int(precision),
                       float(refine_tol_energy), None, int(bool(certify)))

    def footprint_bytes(self, k=1, tol=1e-8, max_iter=100, max_subspace=0, eps_drop=0.0, precision=FP64,
                        refine_tol_energy=0.0, certify=False):
        o = self._opts(k, tol, max_iter, max_subspace, eps_drop, precision, refine_tol_energy, certify)
        return int(_lib.stpci_footprint_bytes(self._h, ctypes.byref(o)))

    def dav_begin(self, k=1, tol=1e-8, max_iter=100, max_subspace=0, eps_drop=0.0, precision=FP64,
                  refine_tol_energy=0.0, certify=False):
        o = self._opts(k, tol, max_iter, max_subspace, eps_drop, precision, refine_tol_energy, certify)
        self._step_k = int(k)
        self._cert_k = int(k)
        self._last_k = self._run_k(k, precision, refine_tol_energy, certify)
        self._check(_lib.stpci_dav_begin(self._h, ctypes.byref(o)))

    def dav_finish_step(self):
        """One Davidson iteration after the pending products; True when done."""
        d = ctypes.c_int()
        self._check(_lib.stpci_dav_finish_step(self._h, ctypes.byref(d)))
        return bool(d.value)

    def dav_result(self, vecs=None, allow_noconv=False):
        k = getattr(self, "_step_k", 1)
        e = (ctypes.c_double * k)()
        r = (ctypes.c_double * k)()
        it = ctypes.c_int()
        st = _lib.stpci_dav_result(self._h, e, r, _ptr(vecs) if vecs is not None else None, ctypes.byref(it))
        if st != OK and not (allow_noconv and st == ENOCONV):
            self._check(st)
        return np.array(e[:]), np.array(r[:]), it.value, st

    def certificate(self):
        """(gamma_lower, bound) of the last Davidson run: lower bounds of the
        gaps and gap-theorem bounds ||r_j||^2 / gamma_j of |E_j - exact|."""
        k = self._cert_k
        g = np.zeros(k)
        b = np.zeros(k)
        self._check(_lib.stpci_dav_certificate(self._h, g.ctypes.data_as(_DP), b.ctypes.data_as(_DP)))
        return g, b

    def history(self, full=False):
        """Iterations of the last Davidson run; with full=True, a dict of
        [iterations][k] arrays: energies, residual norms and the largest
        coefficient change of each Ritz vector ("dc", NaN on the first
        iteration of each phase)."""
        n = ctypes.c_int()
        self._check(_lib.stpci_dav_history(self._h, ctypes.byref(n), 0, None, None))
        if not full:
            return n.value
        k = self._last_k
        e = np.zeros(n.value * k)
        r = np.zeros(n.value * k)
        dc = np.zeros(n.value * k)
        self._check(_lib.stpci_dav_history(self._h, ctypes.byref(n), n.value, e.ctypes.data_as(_DP), r.ctypes.data_as(_DP)))
        self._check(_lib.stpci_dav_history_dc(self._h, n.value, dc.ctypes.data_as(_DP)))
        return {"energies": e.reshape(-1, k), "resid": r.reshape(-1, k), "dc": dc.reshape(-1, k)}

    def test_moves(self, max_dets_per_cat=1 << 40):
        """Host check of the kernels' move arithmetic: (moves checked, moves wrong)."""
        n, b = ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.stpci_test_moves(self._h, int(max_dets_per_cat), ctypes.byref(n), ctypes.byref(b)))
        return n.value, b.value

    def test_pairs(self, max_dets_per_cat=1 << 40):
        """Host check of the pair kernel's slot arithmetic: (slots checked, slots wrong)."""
        n, b = ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.stpci_test_pairs(self._h, int(max_dets_per_cat), ctypes.byref(n), ctypes.byref(b)))
        return n.value, b.value

    def test_pair_groups(self):
        """Host check of the grouped pair kernel's items: (items, violations,
        intermediates per item)."""
        n, b, u = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
        self._check(_lib.stpci_test_pair_groups(self._h, ctypes.byref(n), ctypes.byref(b), ctypes.byref(u)))
        return n.value, b.value, u.value

    def test_precond(self, r, t, theta, eps=0.0):
        """The solver's corrections of n residuals (r, t: device [n][n_dets]),
        Eq. sparsePreconditioner with the given eps."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        self._check(_lib.stpci_test_precond(self._h, _ptr(r), _ptr(t), len(th), th.ctypes.data_as(_DP),
                                            float(eps)))

    def test_cgs_passes(self):
        """Gram-Schmidt passes against the basis over the last Davidson run."""
        n = ctypes.c_int()
        self._check(_lib.stpci_test_dav_cgs_passes(self._h, ctypes.byref(n)))
        return n.value

    def test_ritz(self, v, w, m, y, z, theta, x, t):
        """The solver's fused Rayleigh-Ritz pass: v, w device [m][n_dets]; y,
        z (or None) host m x k arrays; theta host k values; x, t device
        [k][n_dets] outputs.  Returns (k, 3): ||r_j||^2, ||t_j||^2,
        max |(V z_j)_i|^2."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        k = len(th)

        def flat(a):
            a = np.asarray(a).reshape(m, k)
            if self.cplx:
                return np.ascontiguousarray(a, dtype=np.complex128).view(np.float64).ravel()
            return np.ascontiguousarray(a, dtype=np.float64).ravel()
        yf = flat(y)
        zf = flat(z) if z is not None else None
        red = np.zeros(3 * k)
        self._check(_lib.stpci_test_ritz(self._h, _ptr(v), _ptr(w), int(m), yf.ctypes.data_as(_DP),
                                         zf.ctypes.data_as(_DP) if zf is not None else None, k,
                                         th.ctypes.data_as(_DP), _ptr(x), _ptr(t), red.ctypes.data_as(_DP)))
        return red.reshape(k, 3)

    def sb_counts(self, n_vec=1):
        """(matrix-core flops executed, items) of the spectator-batched kernel
        for an n_vec-vector sigma."""
        f, n = ctypes.c_double(), ctypes.c_int64()
        self._check(_lib.stpci_sb_counts(self._h, int(n_vec), ctypes.byref(f), ctypes.byref(n)))
        return f.value, n.value

    def test_sb(self, max_groups=1 << 40):
        """Host check of the spectator-batched pair kernel's row and entry
        arithmetic: (entries checked, entries wrong)."""
        n, b = ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.stpci_test_sb(self._h, int(max_groups), ctypes.byref(n), ctypes.byref(b)))
        return n.value, b.value

    def pair_counts(self):
        """(sum deg^2 over pair intermediates, number of pair intermediates, largest pair degree)."""
        w, n, d = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int()
        self._check(_lib.stpci_pair_counts(self._h, ctypes.byref(w), ctypes.byref(n), ctypes.byref(d)))
        return w.value, n.value, d.value

    def set_sigma_kernel(self, name):
        """Select the sigma kernel ("pair", "pair_atomic", "pair_mf64", "pair_valu", "pair_grp", "pair_sb", "tile", "rowtile" or "auto")."""
        self._check(_lib.stpci_set_sigma_kernel(self._h, name.encode()))

    def sigma_kernel(self):
        """Name of the sigma kernel in use (after the first device call)."""
        p = ctypes.c_char_p()
        self._check(_lib.stpci_sigma_kernel(self._h, ctypes.byref(p)))
        return p.value.decode()

    def dav_stats(self):
        """(FP64 sigma vectors, reduced-precision sigma vectors) spent by the
        last Davidson run."""
        a, b = ctypes.c_int(), ctypes.c_int()
        self._check(_lib.stpci_dav_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def dav_sigma_count(self, precision):
        """Sigma vectors of one contraction precision spent by the last run."""
        n = ctypes.c_int()
        self._check(_lib.stpci_dav_sigma_count(self._h, int(precision), ctypes.byref(n)))
        return n.value

    def profile(self, enable=True):
        self._check(_lib.stpci_profile(self._h, int(bool(enable))))

    def kernel_time(self, name):
        n, t = ctypes.c_int64(), ctypes.c_double()
        self._check(_lib.stpci_kernel_time(self._h, name.encode(), ctypes.byref(n), ctypes.byref(t)))
        return n.value, t.value


QUEUED, ACTIVE, DONE, FAILED, CANCELLED = 0, 1, 2, 3, 4


@dataclass
class RequestResult:
    state: int
    energies: np.ndarray
    resid: np.ndarray
    n_iter: int
    t_submit: float
    t_admit: float
    t_done: float
    status: int


class Server:
    """Continuous-batching CI solve server on one device (see stpci_serve.h)."""

    def __init__(self, device: int = 0, mem_budget_bytes: int = 64 << 30, max_active: int = 32, stream=None):
        h = _P()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        st = _lib.stpci_server_create(ctypes.byref(h), int(device), _P(stream) if stream else None,
                                      int(mem_budget_bytes), int(max_active))
        if st != OK:
            raise StpciError(st, "stpci_server_create failed (device %d)" % device)
        self._h = h
        self._k = {}

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.stpci_server_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def _check(self, st):
        if st != OK:
            raise StpciError(st, _lib.stpci_server_last_error(self._h).decode())
        return st

    def submit(self, h, g, n_elec, sub, lo=None, hi=None, k=1, tol=1e-8, max_iter=100, max_subspace=0,
               precision=FP64, spin_free=False, e_core=0.0) -> int:
        cplx = np.iscomplexobj(h) or np.iscomplexobj(g)
        dt = np.complex128 if cplx else np.float64
        h = np.ascontiguousarray(h, dtype=dt)
        g = np.ascontiguousarray(g, dtype=dt)
        lo = list(lo) if lo is not None else [0] * len(sub)
        hi = list(hi) if hi is not None else list(sub)
        o = DavOpts(int(k), int(max_iter), int(max_subspace), float(tol), 0.0, int(precision), 0.0, None, 0)
        r = Request(h.shape[0], COMPLEX128 if cplx else REAL64, int(bool(spin_free)), h.ctypes.data_as(_P),
                    g.ctypes.data_as(_P), float(e_core), int(n_elec), len(sub), _iarr(sub), _iarr(lo), _iarr(hi),
                    ctypes.pointer(o))
        rid = ctypes.c_int()
        self._check(_lib.stpci_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)))
        self._k[rid.value] = int(k)
        return rid.value

    def cancel(self, rid):
        self._check(_lib.stpci_server_cancel(self._h, int(rid)))

    def tick(self):
        """One scheduling step; returns (requests still pending, requests retired now)."""
        a, f = ctypes.c_int(), ctypes.c_int()
        self._check(_lib.stpci_server_tick(self._h, ctypes.byref(a), ctypes.byref(f)))
        return a.value, f.value

    def result(self, rid) -> RequestResult:
        k = self._k[rid]
        e = (ctypes.c_double * k)()
        r = (ctypes.c_double * k)()
        state, it = ctypes.c_int(), ctypes.c_int()
        ts, ta, td = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        st = _lib.stpci_server_result(self._h, int(rid), ctypes.byref(state), e, r, ctypes.byref(it),
                                      ctypes.byref(ts), ctypes.byref(ta), ctypes.byref(td))
        return RequestResult(state.value, np.array(e[:]), np.array(r[:]), it.value, ts.value, ta.value, td.value, st)

    def request_info(self, rid):
        """(n_dets, nnz(H), footprint bytes, sigma vectors used)."""
        n, nz, fp, sv = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64(), ctypes.c_int()
        self._check(_lib.stpci_server_request_info(self._h, int(rid), ctypes.byref(n), ctypes.byref(nz),
                                                   ctypes.byref(fp), ctypes.byref(sv)))
        return n.value, nz.value, fp.value, sv.value

    def stats(self):
        """dict(used, peak, peak_active, ticks, sigma_launches, admit_s, sigma_s, step_s)."""
        u, p, t, gl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        pa = ctypes.c_int()
        self._check(_lib.stpci_server_stats(self._h, ctypes.byref(u), ctypes.byref(p), ctypes.byref(pa),
                                            ctypes.byref(t), ctypes.byref(gl)))
        a, sg, stp = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(_lib.stpci_server_phase_times(self._h, ctypes.byref(a), ctypes.byref(sg), ctypes.byref(stp)))
        return dict(used=u.value, peak=p.value, peak_active=pa.value, ticks=t.value, sigma_launches=gl.value,
                    admit_s=a.value, sigma_s=sg.value, step_s=stp.value)


def heev(A):
    """Host Hermitian eigensolver used by the Davidson driver (exposed for tests)."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    n = A.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n), dtype=np.complex128)
    st = _lib.stpci_test_heev(n, A.ctypes.data_as(_P), w.ctypes.data_as(_P), V.ctypes.data_as(_P))
    if st != OK:
        raise StpciError(st, "heev failed")
    return w, V


EXPORTED = sorted(_SIGS)
