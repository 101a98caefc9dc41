"""ctypes binding of libpawfe (the C ABI in include/pawfe.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch supplies device memory (tensors) and the stream
(``torch.cuda.current_stream()``).  There is no fallback: if the shared
library is missing or fails to load, ``load()`` raises.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpawfe.so")

PAWFE_OK, PAWFE_EINVAL, PAWFE_ENOMEM, PAWFE_EHIP, PAWFE_ENOTSPD, PAWFE_ENONFINITE, PAWFE_EUNSUPPORTED = range(7)
FP64, FP32, BF16X3 = 0, 1, 2
SINV_EXACT_G, SINV_PP = 0, 1
_PREC = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, FP64: FP64, FP32: FP32, BF16X3: BF16X3}
_STATUS = {1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "ENOTSPD", 5: "ENONFINITE", 6: "EUNSUPPORTED"}

# every symbol include/pawfe.h declares
EXPORTS = [
    "pawfe_build_operator", "pawfe_destroy_operator", "pawfe_query", "pawfe_get_dofmap", "pawfe_get_first_visit",
    "pawfe_set_veff", "pawfe_set_vgga", "pawfe_set_dH", "pawfe_apply_H", "pawfe_apply_S", "pawfe_apply_Sinv",
    "pawfe_apply_local",
    "pawfe_cheb_step_local",
    "pawfe_cheb_filter_workspace", "pawfe_cheb_filter", "pawfe_cheb_filter_res", "pawfe_rayleigh_ritz_workspace",
    "pawfe_rayleigh_ritz", "pawfe_rayleigh_ritz_res", "pawfe_band_energy_grad", "pawfe_lanczos_bounds", "pawfe_last_error",
    "pawfe_chfsi_solve_workspace", "pawfe_chfsi_solve",
    "pawfe_batch_create", "pawfe_batch_run", "pawfe_batch_query", "pawfe_batch_destroy",
    "pawfe_apply_H_noalloc", "pawfe_halo_pack_bf16", "pawfe_halo_unpack_bf16",
    "pawfe_batch_tuning_runs", "pawfe_tune_cache_load", "pawfe_tune_cache_save", "pawfe_tune_cache_clear",
    "pawfe_tune_cache_size",
]


class FilterJob(C.Structure):
    """One problem of a batch (pawfe_filter_job)."""
    _fields_ = [
        ("op", C.c_void_p), ("Xin", C.c_void_p), ("ldx", C.c_int64), ("Xout", C.c_void_p),
        ("ldo", C.c_int64), ("nvec", C.c_int64), ("block", C.c_int32), ("lambda_in", C.c_void_p),
        ("degree", C.c_int32), ("b0", C.c_double), ("bW", C.c_double), ("bU", C.c_double),
    ]


class PawfeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pawfe error {_STATUS.get(code, code)}: {msg}")
        self.code = code


class Desc(C.Structure):
    _fields_ = [
        ("ncell", C.c_int32 * 3), ("box", C.c_double * 3), ("degree", C.c_int32),
        ("nq1d", C.c_int32), ("kpoint", C.c_double * 3), ("is_complex", C.c_int32),
        ("veff_q", C.POINTER(C.c_double)), ("natoms", C.c_int32), ("pos", C.POINTER(C.c_double)),
        ("rcut", C.POINTER(C.c_double)), ("nproj", C.POINTER(C.c_int32)),
        ("proj_l", C.POINTER(C.c_int32)), ("proj_m", C.POINTER(C.c_int32)),
        ("proj_sigma", C.POINTER(C.c_double)), ("dH", C.POINTER(C.c_double)),
        ("dS", C.POINTER(C.c_double)), ("sinv_mode", C.c_int32),
        ("xgrid", C.POINTER(C.c_double)), ("vgga_q", C.POINTER(C.c_double)),
    ]


_lib = None


def load(path=LIB_PATH):
    """Load libpawfe.so (raises if it is missing: there is no other path)."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch (when present) loads its own HIP runtime; loading it first makes
    # the library bind to that one instead of bringing a second runtime into
    # the process (the binding takes streams and device memory from PyTorch)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing; build it with `python -m paper_2604_26037_amd.build`")
    lib = C.CDLL(path)
    vp, i32, i64, dbl, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    P = C.POINTER
    sig = {
        "pawfe_build_operator": [P(Desc), vp, P(vp)],
        "pawfe_destroy_operator": [vp],
        "pawfe_query": [vp, P(i64), P(i64), P(i32), P(i32), P(i64), P(i64)],
        "pawfe_get_dofmap": [vp, vp, vp, vp, vp, vp, vp],
        "pawfe_get_first_visit": [vp, vp],
        "pawfe_set_veff": [vp, P(dbl), vp],
        "pawfe_set_vgga": [vp, P(dbl), vp],
        "pawfe_set_dH": [vp, P(dbl), vp],
        "pawfe_apply_H": [vp, vp, i64, vp, i64, i64, i32, vp],
        "pawfe_apply_H_noalloc": [vp, vp, i64, vp, i64, i64, i32, vp],
        "pawfe_halo_pack_bf16": [vp, vp, i64, i64, i32, i32, vp, vp],
        "pawfe_halo_unpack_bf16": [vp, vp, i64, i32, i32, vp, i64, vp],
        "pawfe_apply_S": [vp, vp, i64, vp, i64, i64, i32, vp],
        "pawfe_apply_Sinv": [vp, vp, i64, vp, i64, i64, i32, vp],
        "pawfe_apply_local": [vp, i32, vp, i64, vp, i64, i64, dbl, i32, vp],
        "pawfe_cheb_step_local": [vp, vp, vp, i64, vp, i64, vp, dbl, dbl, dbl, i64, i32, vp],
        "pawfe_cheb_filter_workspace": [vp, i64, i32, i32, P(sz)],
        "pawfe_cheb_filter": [vp, vp, i64, vp, i64, i64, i32, vp, i32, dbl, dbl, dbl, i32, vp, sz, vp],
        "pawfe_cheb_filter_res": [vp, vp, i64, vp, i64, vp, i64, i64, i32, vp, i32, dbl, dbl, dbl, i32, vp, sz, vp],
        "pawfe_rayleigh_ritz_workspace": [vp, i64, P(sz)],
        "pawfe_rayleigh_ritz": [vp, vp, i64, i64, vp, vp, i32, vp, sz, vp],
        "pawfe_rayleigh_ritz_res": [vp, vp, i64, i64, vp, vp, vp, i64, i32, vp, sz, vp],
        "pawfe_band_energy_grad": [vp, vp, i64, i64, vp, vp, vp, vp, vp],
        "pawfe_lanczos_bounds": [vp, i32, C.c_uint64, P(dbl), P(dbl), P(dbl), vp],
        "pawfe_chfsi_solve_workspace": [vp, i64, i32, i32, P(sz)],
        "pawfe_chfsi_solve": [vp, vp, i64, i64, i64, i32, i32, i32, dbl, i32, dbl, i32, vp, vp, P(i32), vp, sz, vp],
        "pawfe_batch_create": [P(FilterJob), i32, i32, i32, i32, vp, P(vp)],
        "pawfe_batch_run": [vp, vp],
        "pawfe_batch_query": [vp, P(i32), P(i32), P(i32), P(i32)],
        "pawfe_batch_tuning_runs": [vp, P(i32)],
        "pawfe_tune_cache_load": [C.c_char_p],
        "pawfe_tune_cache_save": [C.c_char_p],
        "pawfe_tune_cache_clear": [],
        "pawfe_tune_cache_size": [P(C.c_int64)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = i32
    lib.pawfe_batch_destroy.argtypes = [vp]
    lib.pawfe_batch_destroy.restype = None
    lib.pawfe_last_error.argtypes = []
    lib.pawfe_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(code):
    if code != PAWFE_OK:
        msg = _lib.pawfe_last_error().decode(errors="replace")
        raise PawfeError(code, msg)


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _tptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Operator:
    """Device-resident FE-PAW operator (H, S, Sinv_hat) of one system."""

    def __init__(self, system, sinv_mode="exact_g", stream=None):
        lib = load()
        s = system
        self.system = s
        self._keep = dict(
            veff=np.ascontiguousarray(s.veff_q, dtype=np.float64).ravel(),
            pos=np.ascontiguousarray(s.pos, dtype=np.float64).ravel(),
            rcut=np.ascontiguousarray(s.rcut, dtype=np.float64),
            nproj=np.ascontiguousarray(s.nproj, dtype=np.int32),
            l=np.ascontiguousarray(s.proj_l, dtype=np.int32),
            m=np.ascontiguousarray(s.proj_m, dtype=np.int32),
            sig=np.ascontiguousarray(s.proj_sigma, dtype=np.float64),
            dH=np.ascontiguousarray(s.dH, dtype=np.float64),
            dS=np.ascontiguousarray(s.dS, dtype=np.float64),
        )
        xg = getattr(s, "xgrid", None)
        vg = getattr(s, "vgga_q", None)
        if xg is not None:
            self._keep["xgrid"] = np.ascontiguousarray(np.concatenate([np.asarray(b, dtype=np.float64) for b in xg]))
        if vg is not None:
            self._keep["vgga"] = np.ascontiguousarray(vg, dtype=np.float64).ravel()
        k = self._keep
        d = Desc()
        d.ncell[:] = [int(n) for n in s.ncell]
        d.box[:] = [float(b) for b in s.box]
        d.degree = int(s.degree)
        d.nq1d = int(s.nq)
        d.kpoint[:] = [float(x) for x in np.asarray(s.kpoint, dtype=np.float64)]
        d.is_complex = int(bool(s.is_complex))
        d.veff_q = _dptr(k["veff"])
        d.natoms = len(k["rcut"])
        d.pos = _dptr(k["pos"])
        d.rcut = _dptr(k["rcut"])
        d.nproj = _iptr(k["nproj"])
        d.proj_l = _iptr(k["l"])
        d.proj_m = _iptr(k["m"])
        d.proj_sigma = _dptr(k["sig"])
        d.dH = _dptr(k["dH"])
        d.dS = _dptr(k["dS"])
        d.sinv_mode = {"exact_g": SINV_EXACT_G, "pp": SINV_PP}[sinv_mode]
        d.xgrid = _dptr(k["xgrid"]) if "xgrid" in k else None
        d.vgga_q = _dptr(k["vgga"]) if "vgga" in k else None
        self._desc = d
        h = C.c_void_p()
        _check(lib.pawfe_build_operator(C.byref(d), _stream(stream), C.byref(h)))
        self._h = h
        a = [C.c_int64(), C.c_int64(), C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64()]
        _check(lib.pawfe_query(h, *[C.byref(x) for x in a]))
        (self.ndof, self.nquad, self.ncolour, self.nproj_total, self.nsupp_cells,
         self.nsupp_nodes) = [x.value for x in a]
        self.ncells = int(np.prod(s.ncell))
        self.ncell = tuple(int(v) for v in s.ncell)
        self.degree = int(s.degree)
        self.nloc = (int(s.degree) + 1) ** 3
        # complex (k-point) operators take complex tensors (leading dimensions
        # in complex elements)
        self.complex = bool(s.is_complex)

    def close(self):
        if getattr(self, "_h", None):
            _lib.pawfe_destroy_operator(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- integer outputs --------------------------------------------------
    def dofmap(self):
        na = len(self._keep["rcut"])
        cd = np.empty((self.ncells, self.nloc), dtype=np.int32)
        col = np.empty(self.ncells, dtype=np.int32)
        sco = np.empty(na + 1, dtype=np.int64)
        sc = np.empty(max(self.nsupp_cells, 1), dtype=np.int64)
        sno = np.empty(na + 1, dtype=np.int64)
        sn = np.empty(max(self.nsupp_nodes, 1), dtype=np.int64)
        _check(_lib.pawfe_get_dofmap(self._h, cd.ctypes.data, col.ctypes.data, sco.ctypes.data,
                                     sc.ctypes.data, sno.ctypes.data, sn.ctypes.data))
        return cd, col, sco, sc[:self.nsupp_cells], sno, sn[:self.nsupp_nodes]

    def first_visit(self):
        """[E] uint32: bit ca + 3 cb + 9 cc set when the cell makes the first
        visit of its local nodes of that position class in the colour order."""
        out = np.empty(self.ncells, dtype=np.uint32)
        _check(_lib.pawfe_get_first_visit(self._h, out.ctypes.data))
        return out

    def set_veff(self, veff_q, stream=None):
        v = np.ascontiguousarray(veff_q, dtype=np.float64).ravel()
        _check(_lib.pawfe_set_veff(self._h, _dptr(v), _stream(stream)))
        self._keep["veff"] = v

    def set_vgga(self, vgga_q, stream=None):
        v = np.ascontiguousarray(vgga_q, dtype=np.float64).ravel()
        _check(_lib.pawfe_set_vgga(self._h, _dptr(v), _stream(stream)))
        self._keep["vgga"] = v

    def set_dH(self, dH, stream=None):
        v = np.ascontiguousarray(dH, dtype=np.float64).ravel()
        _check(_lib.pawfe_set_dH(self._h, _dptr(v), _stream(stream)))
        self._keep["dH"] = v

    # -- applies ------------------------------------------------------------
    def _dtype(self, prec):
        import torch
        if _PREC[prec] == FP64:
            return torch.complex128 if self.complex else torch.float64
        return torch.complex64 if self.complex else torch.float32

    def _apply(self, fn, X, out, prec, stream):
        import torch
        assert X.is_cuda and X.dim() == 2 and X.shape[0] == self.ndof and X.stride(1) == 1
        dt = self._dtype(prec)
        assert X.dtype == dt, f"X must be {dt}"
        if out is None:
            out = torch.empty((X.shape[0], X.shape[1]), dtype=dt, device=X.device)
        _check(fn(self._h, _tptr(X), X.stride(0), _tptr(out), out.stride(0), X.shape[1],
                  _PREC[prec], _stream(stream)))
        return out

    def apply_H(self, X, out=None, prec=FP64, stream=None):
        return self._apply(_lib.pawfe_apply_H, X, out, prec, stream)

    def apply_H_noalloc(self, X, out, prec=FP64, stream=None):
        """H X through the allocation-free entry point (out must be given)."""
        assert out is not None
        return self._apply(_lib.pawfe_apply_H_noalloc, X, out, prec, stream)

    def halo_pack_bf16(self, Y, kz0, kz1, buf=None, stream=None):
        """BF16 bits of the FP32 block Y on the slab's two shared node planes:
        a device int16 tensor [2][Gx*Gy][ncols] (the bits of each BF16)."""
        import torch
        assert Y.is_cuda and Y.dtype == (torch.complex64 if self.complex else torch.float32) and Y.stride(1) == 1
        nc = Y.shape[1] * (2 if self.complex else 1)
        prow = (self.ncell[0] * self.degree) * (self.ncell[1] * self.degree)
        if buf is None:
            buf = torch.empty((2, prow, nc), dtype=torch.int16, device=Y.device)
        _check(_lib.pawfe_halo_pack_bf16(self._h, _tptr(Y), Y.stride(0), Y.shape[1], int(kz0), int(kz1),
                                         _tptr(buf), _stream(stream)))
        return buf

    def halo_unpack_bf16(self, buf, Y, kz0, kz1, stream=None):
        """Y += the BF16 planes of buf (cast to FP32), in place."""
        _check(_lib.pawfe_halo_unpack_bf16(self._h, _tptr(buf), Y.shape[1], int(kz0), int(kz1), _tptr(Y),
                                           Y.stride(0), _stream(stream)))
        return Y

    def apply_S(self, X, out=None, prec=FP64, stream=None):
        return self._apply(_lib.pawfe_apply_S, X, out, prec, stream)

    def apply_Sinv(self, X, out=None, prec=FP64, stream=None):
        return self._apply(_lib.pawfe_apply_Sinv, X, out, prec, stream)

    def apply_local(self, X, Y, which=0, alpha=1.0, prec=FP64, stream=None):
        """Y += alpha * A_loc X (cell part only); Y must be preallocated."""
        _check(_lib.pawfe_apply_local(self._h, int(which), _tptr(X), X.stride(0), _tptr(Y), Y.stride(0),
                                      X.shape[1], float(alpha), _PREC[prec], _stream(stream)))
        return Y

    def cheb_step_local(self, RY, RX, Y, lamY, a, ac, zz, prec=FP64, stream=None):
        """RX <- (-ac RY - zz RX) + a lamY Y + a H_loc M_D^{-1} RY (local part of a
        filter step, real columns; complex operators: (re, im) pairs); RX in place."""
        assert RY.stride(1) == 1 and RX.stride(1) == 1 and Y.stride(1) == 1
        assert RY.stride(0) == RX.stride(0) and RY.shape == RX.shape
        _check(_lib.pawfe_cheb_step_local(self._h, _tptr(RY), _tptr(RX), RX.stride(0), _tptr(Y), Y.stride(0),
                                          _tptr(lamY), float(a), float(ac), float(zz), RX.shape[1], _PREC[prec],
                                          _stream(stream)))
        return RX

    # -- filter / RR ------------------------------------------------------------
    def cheb_filter_workspace(self, nvec, block, prec=FP64):
        b = C.c_size_t()
        _check(_lib.pawfe_cheb_filter_workspace(self._h, nvec, block, _PREC[prec], C.byref(b)))
        return b.value

    def workspace(self, nbytes, device="cuda"):
        import torch
        return torch.empty(nbytes, dtype=torch.uint8, device=device)

    def cheb_filter(self, X, lam, degree, b0, bW, bU, block=None, prec=FP64, out=None, ws=None,
                    stream=None, R=None):
        """R: the residual H X - S X diag(lam) of the input pairs, as
        rayleigh_ritz(..., R=...) leaves it (pawfe_cheb_filter_res), or None
        to form it here."""
        assert X.is_cuda and X.dtype == self._dtype(FP64) and X.stride(1) == 1
        import torch
        n = X.shape[1]
        block = n if block is None else int(block)
        if out is None:
            out = torch.empty_like(X)
        if ws is None:
            ws = self.workspace(self.cheb_filter_workspace(n, block, prec), X.device)
        lam = lam.to(device=X.device, dtype=torch.float64).contiguous()
        if R is None:
            _check(_lib.pawfe_cheb_filter(self._h, _tptr(X), X.stride(0), _tptr(out), out.stride(0), n, block,
                                          _tptr(lam), int(degree), float(b0), float(bW), float(bU),
                                          _PREC[prec], _tptr(ws), ws.numel(), _stream(stream)))
        else:
            assert R.is_cuda and R.dtype == X.dtype and R.stride(1) == 1 and R.shape == X.shape
            _check(_lib.pawfe_cheb_filter_res(self._h, _tptr(X), X.stride(0), _tptr(R), R.stride(0), _tptr(out),
                                              out.stride(0), n, block, _tptr(lam), int(degree), float(b0),
                                              float(bW), float(bU), _PREC[prec], _tptr(ws), ws.numel(),
                                              _stream(stream)))
        return out

    def rayleigh_ritz_workspace(self, nvec):
        b = C.c_size_t()
        _check(_lib.pawfe_rayleigh_ritz_workspace(self._h, nvec, C.byref(b)))
        return b.value

    def rayleigh_ritz(self, X, ws=None, stream=None, sr_prec=FP64, R=None):
        """In place on X; returns (lambda, resnorm) as device tensors.
        sr_prec=FP32: mixed-precision subspace rotation.  R (same shape and
        type as X): receives the residual H X - S X diag(lambda) of the
        rotated pairs (pawfe_rayleigh_ritz_res), for cheb_filter(..., R=R)."""
        import torch
        assert X.is_cuda and X.dtype == self._dtype(FP64) and X.stride(1) == 1
        n = X.shape[1]
        lam = torch.empty(n, dtype=torch.float64, device=X.device)
        res = torch.empty(n, dtype=torch.float64, device=X.device)
        if ws is None:
            ws = self.workspace(self.rayleigh_ritz_workspace(n), X.device)
        if R is None:
            _check(_lib.pawfe_rayleigh_ritz(self._h, _tptr(X), X.stride(0), n, _tptr(lam), _tptr(res),
                                            _PREC[sr_prec], _tptr(ws), ws.numel(), _stream(stream)))
        else:
            assert R.is_cuda and R.dtype == X.dtype and R.stride(1) == 1 and R.shape == X.shape
            _check(_lib.pawfe_rayleigh_ritz_res(self._h, _tptr(X), X.stride(0), n, _tptr(lam), _tptr(res),
                                                _tptr(R), R.stride(0), _PREC[sr_prec], _tptr(ws), ws.numel(),
                                                _stream(stream)))
        return lam, res

    def band_energy_grad(self, X, occ=None, want_E=True, want_dV=True, want_dH=True, stream=None):
        import torch
        assert X.is_cuda and X.dtype == self._dtype(FP64) and X.stride(1) == 1
        dev = X.device
        E = torch.zeros(1, dtype=torch.float64, device=dev) if want_E else None
        dV = torch.empty(self.nquad, dtype=torch.float64, device=dev) if want_dV else None
        ndh = int(len(self._keep["dH"]))
        dD = torch.empty(max(ndh, 1), dtype=torch.float64, device=dev) if want_dH else None
        occ_t = None if occ is None else occ.to(device=dev, dtype=torch.float64).contiguous()
        _check(_lib.pawfe_band_energy_grad(self._h, _tptr(X), X.stride(0), X.shape[1], _tptr(occ_t),
                                           _tptr(E), _tptr(dV), _tptr(dD), _stream(stream)))
        return E, dV, (dD[:ndh] if dD is not None else None)

    def lanczos_bounds(self, k=20, seed=1234, stream=None):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        _check(_lib.pawfe_lanczos_bounds(self._h, int(k), C.c_uint64(seed), C.byref(a), C.byref(b),
                                         C.byref(c), _stream(stream)))
        return a.value, b.value, c.value

    def chfsi_solve(self, X, degree, tol, max_iter, nwanted=None, block=None, prec=FP64, bU=None,
                    lanczos_k=20, ws=None, stream=None):
        """Filter + Rayleigh-Ritz in place on X until the lowest nwanted
        residual norms are <= tol (pawfe_chfsi_solve).  Returns (lambda,
        resnorm, iterations); lambda and resnorm are device tensors."""
        import torch
        assert X.is_cuda and X.dtype == self._dtype(FP64) and X.stride(1) == 1
        n = X.shape[1]
        block = n if block is None else int(block)
        lam = torch.empty(n, dtype=torch.float64, device=X.device)
        res = torch.empty(n, dtype=torch.float64, device=X.device)
        if ws is None:
            b = C.c_size_t()
            _check(_lib.pawfe_chfsi_solve_workspace(self._h, n, block, _PREC[prec], C.byref(b)))
            ws = self.workspace(b.value, X.device)
        it = C.c_int32()
        _check(_lib.pawfe_chfsi_solve(self._h, _tptr(X), X.stride(0), n, 0 if nwanted is None else int(nwanted),
                                      int(degree), block, _PREC[prec], 0.0 if bU is None else float(bU),
                                      int(lanczos_k), float(tol), int(max_iter), _tptr(lam), _tptr(res),
                                      C.byref(it), _tptr(ws), ws.numel(), _stream(stream)))
        return lam, res, it.value


def band_energy_function():
    """torch.autograd.Function for E = sum_n occ_n x_n^T H[V, Delta_H] x_n.

    Forward and backward both call pawfe_band_energy_grad; nothing is cached
    between them except the inputs themselves.  For real operators the
    gradient with respect to X is 2 H X diag(occ) (H is symmetric), one
    pawfe_apply_H; for complex operators X must not require a gradient.
    """
    import torch

    class BandEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, X, veff_q, dH, op, occ=None):
            if X.requires_grad and op.complex:
                raise NotImplementedError("dE/dX is provided for real operators only; detach X")
            op.set_veff(veff_q.detach().cpu().numpy())
            op.set_dH(dH.detach().cpu().numpy())
            E, _, _ = op.band_energy_grad(X, occ, want_E=True, want_dV=False, want_dH=False)
            ctx.op = op
            ctx.occ = occ
            ctx.vshape = tuple(veff_q.shape)
            ctx.vdev = veff_q.device
            ctx.ddev = dH.device
            ctx.save_for_backward(X)
            return E[0].clone()

        @staticmethod
        def backward(ctx, g):
            (X,) = ctx.saved_tensors
            _, dV, dD = ctx.op.band_energy_grad(X, ctx.occ, want_E=False, want_dV=True, want_dH=True)
            gv = (g * dV).view(ctx.vshape).to(ctx.vdev)
            gd = (g * dD).to(ctx.ddev)
            gx = None
            if ctx.needs_input_grad[0]:
                Xc = X.detach().contiguous()
                HX = ctx.op.apply_H(Xc)
                w = 2.0 * g if ctx.occ is None else 2.0 * g * ctx.occ.to(device=HX.device, dtype=HX.dtype)
                gx = HX * w
            return gx, gv, gd, None, None

    return BandEnergy


def tune_cache_load(path):
    """Merge a tuning cache written by tune_cache_save into the process table."""
    _check(load().pawfe_tune_cache_load(os.fsencode(path)))


def tune_cache_save(path):
    """Write the process-wide tuning cache of the batch autotuner to `path`."""
    _check(load().pawfe_tune_cache_save(os.fsencode(path)))


def tune_cache_clear():
    _check(load().pawfe_tune_cache_clear())


def tune_cache_size():
    n = C.c_int64()
    _check(load().pawfe_tune_cache_size(C.byref(n)))
    return n.value


class Batch:
    """Filters of several independent problems captured into one HIP graph.

    jobs: list of dicts with keys op (Operator), X (device FP64 [ndof][n]),
    out (same shape, may be X), lam (device FP64 [n]), degree, b0, bW, bU and
    optionally block (default: autotuned).  nstreams=None lets the library
    pick 1, 2 or 4 streams by timing.  max_graph_launches bounds the kernel
    launches of each captured graph (None: the library's default).  The
    tensors are kept alive by the batch; run() replays the graphs on the
    current stream.
    """

    def __init__(self, jobs, prec=FP64, nstreams=None, stream=None, max_graph_launches=None):
        import torch
        lib = load()
        self._jobs = []
        arr = (FilterJob * len(jobs))()
        for i, j in enumerate(jobs):
            X, out, lam = j["X"], j.get("out", j["X"]), j["lam"]
            xdt = j["op"]._dtype(FP64)   # complex128 for complex (k-point) operators
            for t in (X, out):
                assert t.is_cuda and t.dtype == xdt
            assert lam.is_cuda and lam.dtype == torch.float64
            assert X.stride(1) == 1 and out.stride(1) == 1 and lam.is_contiguous()
            self._jobs.append((j["op"], X, out, lam))
            arr[i] = FilterJob(j["op"]._h.value,
                               X.data_ptr(), X.stride(0), out.data_ptr(), out.stride(0), X.shape[1],
                               int(j.get("block", 0) or 0), lam.data_ptr(), int(j["degree"]),
                               float(j["b0"]), float(j["bW"]), float(j["bU"]))
        h = C.c_void_p()
        _check(lib.pawfe_batch_create(arr, len(jobs), _PREC[prec], 0 if nstreams is None else int(nstreams),
                                      0 if max_graph_launches is None else int(max_graph_launches),
                                      _stream(stream), C.byref(h)))
        self._h = h
        self.njobs = len(jobs)

    def run(self, stream=None):
        _check(_lib.pawfe_batch_run(self._h, _stream(stream)))

    def schedule(self):
        ns = C.c_int32()
        blocks = np.zeros(self.njobs, dtype=np.int32)
        sof = np.zeros(self.njobs, dtype=np.int32)
        _check(_lib.pawfe_batch_query(self._h, C.byref(ns), _iptr(blocks), _iptr(sof), None))
        return ns.value, blocks, sof

    @property
    def tuning_runs(self):
        """Timed tuning runs spent when the batch was created (0: all cached)."""
        n = C.c_int32()
        _check(_lib.pawfe_batch_tuning_runs(self._h, C.byref(n)))
        return n.value

    @property
    def ngraphs(self):
        n = C.c_int32()
        _check(_lib.pawfe_batch_query(self._h, None, None, None, C.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pawfe_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
