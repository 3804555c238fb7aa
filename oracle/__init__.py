"""FP64 CPU oracle for the DMK point code (arXiv 2308.00292).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark use it; the product library never imports it.  The
arithmetic lives in the C sources next to this file (``liboracle.so``); this
module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")


def build() -> None:
    """Compile liboracle.so with the Makefile beside this file."""
    subprocess.run(["make", "-s", "-B", "-C", _HERE, "liboracle.so"], check=True)


class Params(C.Structure):
    _fields_ = [("tol", C.c_double), ("c", C.c_double), ("nf", C.c_int), ("p", C.c_int),
                ("nw", C.c_int), ("hw", C.c_double)]


_MAXTERM = 96
_GLEXT = 256


class Pswf(C.Structure):
    _fields_ = [("c", C.c_double), ("nterm", C.c_int), ("coef", C.c_double * _MAXTERM),
                ("chi", C.c_double), ("psi0", C.c_double), ("lambda0", C.c_double),
                ("c0", C.c_double), ("c2", C.c_double),
                ("glx", C.c_double * _GLEXT), ("glw", C.c_double * _GLEXT),
                ("glpsi", C.c_double * _GLEXT)]


_P = C.POINTER
_i64p = _P(C.c_int64)
_u64p = _P(C.c_uint64)
_f64p = _P(C.c_double)
_i32p = _P(C.c_int32)
_u8p = _P(C.c_uint8)


class _Tree(C.Structure):
    _fields_ = [("dim", C.c_int), ("bits", C.c_int), ("ns", C.c_int), ("maxdepth", C.c_int),
                ("n", C.c_int64), ("center", C.c_double * 3), ("side", C.c_double),
                ("perm", _i64p), ("key", _u64p), ("xs", _f64p), ("nlevels", C.c_int),
                ("level_start", _i64p), ("nbox", C.c_int64), ("level", _i32p), ("bkey", _u64p),
                ("parent", _i64p), ("child0", _i64p), ("pstart", _i64p), ("pcount", _i64p),
                ("leaf", _u8p), ("fout", _u8p), ("fin", _u8p), ("terminal", _u8p),
                ("colleague", _i64p), ("ncoarse", _i32p), ("coarse", _i64p), ("tlevel", _i32p)]


class _Result(C.Structure):
    _fields_ = [("n", C.c_int64), ("u", _f64p), ("ufar", _f64p), ("ures", _f64p),
                ("p", C.c_int), ("nf", C.c_int), ("proxy", _P(_f64p)), ("local", _P(_f64p))]


class _Split2(C.Structure):
    _fields_ = [("kern", C.c_int), ("lam", C.c_double), ("nlev", C.c_int), ("deg", C.c_int),
                ("coef", _f64p), ("self", _f64p)]


class _Split3(C.Structure):
    _fields_ = [("lam", C.c_double), ("nlev", C.c_int), ("deg", C.c_int), ("coef", _P(C.c_double)),
                ("self", _P(C.c_double))]


class _Pow2(C.Structure):
    _fields_ = [("ps", C.c_void_p), ("c1", C.c_double), ("coef", C.c_double * 48)]


class VParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("q", C.c_int), ("sigma0", C.c_double), ("p", C.c_int), ("nf", C.c_int),
                ("nw", C.c_int), ("hw", C.c_double), ("nleg", C.c_int), ("tau_a", C.c_double),
                ("tpan_gl", C.c_int), ("tpan_w", C.c_double), ("split", C.c_int), ("c", C.c_double),
                ("theta1", C.c_double), ("nfit", C.c_int), ("fit_t", C.c_double * 32), ("fit_w", C.c_double * 32),
                ("fit_err", C.c_double)]


class _VTree(C.Structure):
    _fields_ = [("q", C.c_int), ("nleaf", C.c_int64), ("level", _i32p), ("ijk", _i32p)]


class _VResult(C.Structure):
    _fields_ = [("n", C.c_int64), ("u", _f64p), ("ufar", _f64p), ("unear", _f64p), ("utail", _f64p)]


DENSITY_FN = C.CFUNCTYPE(None, C.c_int64, _f64p, _f64p, C.c_void_p)

LOG2, YUK2 = 0, 1  # 2-D kernels: -log(r)/(2 pi) and K_0(lambda r)
LAP3, YUK3, POW3 = 0, 1, 2  # 3-D kernels: 1/(4 pi r), exp(-lambda r)/(4 pi r), 1/r^2

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            build()
        L = C.CDLL(_LIBPATH)
        L.orc_params_for.argtypes = [C.c_double, _P(Params)]
        L.orc_params_set.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, _P(Params)]
        L.orc_pswf_init.argtypes = [C.c_double, _P(Pswf)]
        for f in ("orc_pswf_eval", "orc_pswf_eval_ext", "orc_pswf_phi"):
            getattr(L, f).argtypes = [_P(Pswf), C.c_double]
            getattr(L, f).restype = C.c_double
        L.orc_split_w0.argtypes = [_P(Pswf), C.c_double]
        L.orc_split_w0.restype = C.c_double
        for f in ("orc_split_d", "orc_split_r", "orc_dhat"):
            getattr(L, f).argtypes = [_P(Pswf), C.c_int, C.c_double]
            getattr(L, f).restype = C.c_double
        L.orc_split_m0.argtypes = [_P(Pswf), C.c_int]
        L.orc_split_m0.restype = C.c_double
        L.orc_w0hat.argtypes = [_P(Pswf), C.c_double]
        L.orc_w0hat.restype = C.c_double
        L.orc_split_d_pw.argtypes = [_P(Pswf), _P(Params), C.c_int, _f64p]
        L.orc_split_d_pw.restype = C.c_double
        L.orc_split_w0_pw.argtypes = [_P(Pswf), _P(Params), _f64p]
        L.orc_split_w0_pw.restype = C.c_double
        L.orc_gauss_legendre.argtypes = [C.c_int, _f64p, _f64p]
        L.orc_tree_build.argtypes = [C.c_int, C.c_int64, _f64p, C.c_int, C.c_int, _P(_Tree)]
        L.orc_tree_free.argtypes = [_P(_Tree)]
        L.orc_dmk_eval.argtypes = [_P(_Tree), _P(Params), _P(Pswf), _f64p, C.c_int, _P(_Result)]
        L.orc_dmk_result_free.argtypes = [_P(_Tree), _P(_Result)]
        L.orc_direct.argtypes = [C.c_int64, _f64p, _f64p, C.c_int64, _i64p, _f64p]
        L.orc_dmk_run.argtypes = [C.c_int64, _f64p, _f64p, C.c_double, C.c_int, C.c_int, _f64p,
                                  _f64p]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = C.c_int
        # 2-D
        for f in ("orc_bessel_k0", "orc_bessel_k1"):
            getattr(L, f).argtypes = [C.c_double]
            getattr(L, f).restype = C.c_double
        L.orc2_kernel.argtypes = [C.c_int, C.c_double, C.c_double]
        L.orc2_kernel.restype = C.c_double
        L.orc_params2_for.argtypes = [C.c_double, _P(Params)]
        L.orc2_dhat.argtypes = [_P(Pswf), C.c_int, C.c_double, C.c_int, C.c_double]
        L.orc2_dhat.restype = C.c_double
        L.orc2_w0hat.argtypes = [_P(Pswf), C.c_int, C.c_double, C.c_double]
        L.orc2_w0hat.restype = C.c_double
        L.orc2_smooth_quad.argtypes = [_P(Pswf), C.c_int, C.c_double, C.c_double]
        L.orc2_smooth_quad.restype = C.c_double
        L.orc2_split_init.argtypes = [_P(Pswf), C.c_int, C.c_double, C.c_int, _P(_Split2)]
        L.orc2_split_free.argtypes = [_P(_Split2)]
        L.orc2_smooth.argtypes = [_P(_Split2), C.c_int, C.c_double]
        L.orc2_smooth.restype = C.c_double
        L.orc2_residual.argtypes = [_P(_Split2), C.c_int, C.c_double]
        L.orc2_residual.restype = C.c_double
        L.orc2_d_pw.argtypes = [_P(Pswf), _P(Params), C.c_int, C.c_double, C.c_int, _f64p]
        L.orc2_d_pw.restype = C.c_double
        L.orc2_w0_pw.argtypes = [_P(Pswf), _P(Params), C.c_int, C.c_double, _f64p]
        L.orc2_w0_pw.restype = C.c_double
        L.orc_dmk2_eval.argtypes = [_P(_Tree), _P(Params), _P(Pswf), C.c_int, C.c_double, _f64p, C.c_int,
                                    _P(_Result)]
        L.orc_direct2.argtypes = [C.c_int, C.c_double, C.c_int64, _f64p, _f64p, C.c_int64, _i64p, _f64p]
        # 3-D Yukawa
        L.orc_dmk_eval_k.argtypes = [_P(_Tree), _P(Params), _P(Pswf), C.c_int, C.c_double, _f64p, C.c_int,
                                     _P(_Result)]
        L.orc_y3_dhat.argtypes = [_P(Pswf), C.c_double, C.c_int, C.c_double]
        L.orc_y3_that.argtypes = [C.c_double, C.c_double]
        L.orc_y3_w0hat.argtypes = [_P(Pswf), C.c_double, C.c_double]
        L.orc_y3_smooth_quad.argtypes = [_P(Pswf), C.c_double, C.c_double]
        for f in ("orc_y3_dhat", "orc_y3_that", "orc_y3_w0hat", "orc_y3_smooth_quad", "orc_y3_smooth",
                  "orc_y3_residual", "orc_y3_d_pw", "orc_y3_w0_pw"):
            getattr(L, f).restype = C.c_double
        L.orc_y3_split_init.argtypes = [_P(Pswf), C.c_double, C.c_int, _P(_Split3)]
        L.orc_y3_split_free.argtypes = [_P(_Split3)]
        L.orc_y3_smooth.argtypes = [_P(_Split3), C.c_int, C.c_double]
        L.orc_y3_residual.argtypes = [_P(_Split3), C.c_int, C.c_double]
        L.orc_y3_d_pw.argtypes = [_P(Pswf), _P(Params), C.c_double, C.c_int, _f64p]
        L.orc_y3_w0_pw.argtypes = [_P(Pswf), _P(Params), C.c_double, _f64p]
        L.orc_direct_yuk3.argtypes = [C.c_double, C.c_int64, _f64p, _f64p, C.c_int64, _i64p, _f64p]
        # 3-D 1/r^2
        L.orc_p2_c1.argtypes = [_P(Pswf)]
        L.orc_p2_phi_quad.argtypes = [_P(Pswf), C.c_double]
        L.orc_p2_init.argtypes = [_P(Pswf), _P(_Pow2)]
        for f in ("orc_p2_phi", "orc_p2_w0", "orc_p2_w0hat"):
            getattr(L, f).argtypes = [_P(_Pow2), C.c_double]
        L.orc_p2_m0.argtypes = [_P(_Pow2), C.c_int]
        for f in ("orc_p2_d", "orc_p2_r", "orc_p2_dhat"):
            getattr(L, f).argtypes = [_P(_Pow2), C.c_int, C.c_double]
        L.orc_p2_d_pw.argtypes = [_P(_Pow2), _P(Params), C.c_int, _f64p]
        L.orc_p2_w0_pw.argtypes = [_P(_Pow2), _P(Params), _f64p]
        for f in ("orc_p2_c1", "orc_p2_phi_quad", "orc_p2_phi", "orc_p2_w0", "orc_p2_w0hat", "orc_p2_m0",
                  "orc_p2_d", "orc_p2_r", "orc_p2_dhat", "orc_p2_d_pw", "orc_p2_w0_pw"):
            getattr(L, f).restype = C.c_double
        L.orc_direct_pow2.argtypes = [C.c_int64, _f64p, _f64p, C.c_int64, _i64p, _f64p]
        # volume
        L.orc_vparams_for.argtypes = [C.c_double, C.c_int, _P(VParams)]
        for f in ("orc_gsplit_m", "orc_gsplit_d", "orc_gsplit_r", "orc_gdhat"):
            getattr(L, f).argtypes = [_P(VParams), C.c_int, C.c_double]
            getattr(L, f).restype = C.c_double
        L.orc_gw0hat.argtypes = [_P(VParams), C.c_double]
        L.orc_gw0hat.restype = C.c_double
        L.orc_gsplit_d_pw.argtypes = [_P(VParams), C.c_int, _f64p]
        L.orc_gsplit_d_pw.restype = C.c_double
        L.orc_gsplit_w0_pw.argtypes = [_P(VParams), _f64p]
        L.orc_gsplit_w0_pw.restype = C.c_double
        L.orc_vsog.argtypes = [_P(VParams), C.c_double, C.c_double, _f64p, _f64p]
        L.orc_vsog_count.argtypes = [_P(VParams), C.c_double, C.c_double]
        L.orc_vfit_target.argtypes = [_P(VParams), C.c_double]
        L.orc_vfit_target.restype = C.c_double
        L.orc_vtree_build.argtypes = [_P(VParams), C.c_double, C.c_int, C.c_int, C.c_int, _f64p, DENSITY_FN,
                                      C.c_void_p, _P(_VTree)]
        L.orc_vtree_free.argtypes = [_P(_VTree)]
        L.orc_vol_nodes.argtypes = [_P(_VTree), _f64p]
        L.orc_vol_eval.argtypes = [_P(_VTree), _P(VParams), _f64p, _P(_VResult)]
        L.orc_vol_result_free.argtypes = [_P(_VResult)]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_f64p)


def params_for(tol: float) -> Params:
    pr = Params()
    if lib().orc_params_for(tol, C.byref(pr)) != 0:
        raise ValueError(f"unsupported tolerance {tol}")
    return pr


def params_set(tol: float, c: float, nf: int, p: int, dim: int = 3) -> Params:
    """Params for any (c, nf, p), root window spacing by the oracle's reading."""
    pr = Params()
    if lib().orc_params_set(float(tol), float(c), int(nf), int(p), int(dim), C.byref(pr)) != 0:
        raise ValueError("bad parameters")
    return pr


class PSWF:
    """psi_0^c with its constants (c_0, c_2, lambda_0, psi(0))."""

    def __init__(self, c: float):
        self.s = Pswf()
        lib().orc_pswf_init(c, C.byref(self.s))

    def __getattr__(self, k):
        if k in ("c", "nterm", "chi", "psi0", "lambda0", "c0", "c2"):
            return getattr(self.s, k)
        raise AttributeError(k)

    def psi(self, x):
        return lib().orc_pswf_eval_ext(C.byref(self.s), float(x))

    def psi_series(self, x):
        return lib().orc_pswf_eval(C.byref(self.s), float(x))

    def phi(self, x):
        return lib().orc_pswf_phi(C.byref(self.s), float(x))

    def w0(self, r):
        return lib().orc_split_w0(C.byref(self.s), float(r))

    def d(self, l, r):
        return lib().orc_split_d(C.byref(self.s), int(l), float(r))

    def r(self, L, r):
        return lib().orc_split_r(C.byref(self.s), int(L), float(r))

    def m0(self, L):
        return lib().orc_split_m0(C.byref(self.s), int(L))

    def dhat(self, l, k):
        return lib().orc_dhat(C.byref(self.s), int(l), float(k))

    def w0hat(self, k):
        return lib().orc_w0hat(C.byref(self.s), float(k))

    def d_pw(self, params: Params, l, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().orc_split_d_pw(C.byref(self.s), C.byref(params), int(l), _dp(x))

    def w0_pw(self, params: Params, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().orc_split_w0_pw(C.byref(self.s), C.byref(params), _dp(x))


    # ---- 2-D split (kern: LOG2 or YUK2; lam: scaled Yukawa parameter)
    def d2hat(self, kern, lam, l, k):
        return lib().orc2_dhat(C.byref(self.s), int(kern), float(lam), int(l), float(k))

    def w02hat(self, kern, lam, k):
        return lib().orc2_w0hat(C.byref(self.s), int(kern), float(lam), float(k))

    def smooth_quad(self, kern, mu, x):
        return lib().orc2_smooth_quad(C.byref(self.s), int(kern), float(mu), float(x))

    def d2_pw(self, params: Params, kern, lam, l, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().orc2_d_pw(C.byref(self.s), C.byref(params), int(kern), float(lam), int(l), _dp(x))

    def w02_pw(self, params: Params, kern, lam, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().orc2_w0_pw(C.byref(self.s), C.byref(params), int(kern), float(lam), _dp(x))


class Yuk3:
    """The 3-D Yukawa split e^{-lam r}/r (root-box units): transforms,
    mollified kernel by quadrature, per-level tables, plane-wave sums."""

    def __init__(self, pswf: "PSWF", lam: float, nlev: int = 0):
        self.ps, self.lam = pswf, float(lam)
        self._s = None
        if nlev:
            self._s = _Split3()
            lib().orc_y3_split_init(C.byref(pswf.s), self.lam, int(nlev), C.byref(self._s))
            self.self_ = np.ctypeslib.as_array(self._s.self, shape=(nlev,)).copy()

    def dhat(self, l, k):
        return lib().orc_y3_dhat(C.byref(self.ps.s), self.lam, int(l), float(k))

    def that(self, k):
        return lib().orc_y3_that(self.lam, float(k))

    def w0hat(self, k):
        return lib().orc_y3_w0hat(C.byref(self.ps.s), self.lam, float(k))

    def smooth_quad(self, mu, x):
        return lib().orc_y3_smooth_quad(C.byref(self.ps.s), float(mu), float(x))

    def smooth(self, l, x):
        return lib().orc_y3_smooth(C.byref(self._s), int(l), float(x))

    def residual(self, l, r):
        return lib().orc_y3_residual(C.byref(self._s), int(l), float(r))

    def d_pw(self, params: "Params", l, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().orc_y3_d_pw(C.byref(self.ps.s), C.byref(params), self.lam, int(l), _dp(x))

    def w0_pw(self, params: "Params", x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().orc_y3_w0_pw(C.byref(self.ps.s), C.byref(params), self.lam, _dp(x))

    def __del__(self):
        try:
            if self._s is not None:
                lib().orc_y3_split_free(C.byref(self._s))
        except Exception:
            pass


def direct_yuk3(lam, pts, charges, tidx=None):
    """u_i = sum_{j != i, r > 0} q_j exp(-lam r_ij)/(4 pi r_ij) (lam in input units)."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    q = np.ascontiguousarray(charges, dtype=np.float64)
    n = pts.shape[0]
    if tidx is None:
        tidx = np.arange(n, dtype=np.int64)
    tidx = np.ascontiguousarray(tidx, dtype=np.int64)
    out = np.zeros(len(tidx))
    lib().orc_direct_yuk3(float(lam), n, _dp(pts), _dp(q), len(tidx), tidx.ctypes.data_as(_i64p), _dp(out))
    return out


class Pow2:
    """The 3-D 1/r^2 split (PSWF power function, root-box units)."""

    def __init__(self, pswf: "PSWF"):
        self.ps = pswf
        self._t = _Pow2()
        lib().orc_p2_init(C.byref(pswf.s), C.byref(self._t))
        self.c1 = self._t.c1

    def phi_quad(self, x):
        return lib().orc_p2_phi_quad(C.byref(self.ps.s), float(x))

    def phi(self, x):
        return lib().orc_p2_phi(C.byref(self._t), float(x))

    def m0(self, L):
        return lib().orc_p2_m0(C.byref(self._t), int(L))

    def d(self, l, r):
        return lib().orc_p2_d(C.byref(self._t), int(l), float(r))

    def r(self, L, r):
        return lib().orc_p2_r(C.byref(self._t), int(L), float(r))

    def w0(self, r):
        return lib().orc_p2_w0(C.byref(self._t), float(r))

    def dhat(self, l, k):
        return lib().orc_p2_dhat(C.byref(self._t), int(l), float(k))

    def w0hat(self, k):
        return lib().orc_p2_w0hat(C.byref(self._t), float(k))

    def d_pw(self, params: "Params", l, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().orc_p2_d_pw(C.byref(self._t), C.byref(params), int(l), _dp(x))

    def w0_pw(self, params: "Params", x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().orc_p2_w0_pw(C.byref(self._t), C.byref(params), _dp(x))


def direct_pow2(pts, charges, tidx=None):
    """u_i = sum_{j != i, r > 0} q_j / r_ij^2."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    q = np.ascontiguousarray(charges, dtype=np.float64)
    n = pts.shape[0]
    if tidx is None:
        tidx = np.arange(n, dtype=np.int64)
    tidx = np.ascontiguousarray(tidx, dtype=np.int64)
    out = np.zeros(len(tidx))
    lib().orc_direct_pow2(n, _dp(pts), _dp(q), len(tidx), tidx.ctypes.data_as(_i64p), _dp(out))
    return out


class Split2:
    """Per-level residual tables of the 2-D split (smooth part and M_l(0))."""

    def __init__(self, pswf: PSWF, kern: int, lam: float, nlev: int):
        self._s = _Split2()
        lib().orc2_split_init(C.byref(pswf.s), int(kern), float(lam), int(nlev), C.byref(self._s))
        self.nlev, self.deg = nlev, self._s.deg
        self.coef = np.ctypeslib.as_array(self._s.coef, shape=(nlev * (self.deg + 1),)).reshape(
            nlev, self.deg + 1).copy()
        self.self_ = np.ctypeslib.as_array(self._s.self, shape=(nlev,)).copy()

    def smooth(self, l, x):
        return lib().orc2_smooth(C.byref(self._s), int(l), float(x))

    def residual(self, l, r):
        return lib().orc2_residual(C.byref(self._s), int(l), float(r))

    def __del__(self):
        try:
            lib().orc2_split_free(C.byref(self._s))
        except Exception:
            pass


def params2_for(tol: float) -> Params:
    pr = Params()
    if lib().orc_params2_for(tol, C.byref(pr)) != 0:
        raise ValueError(f"unsupported tolerance {tol}")
    return pr


def bessel_k0(x):
    return lib().orc_bessel_k0(float(x))


def bessel_k1(x):
    return lib().orc_bessel_k1(float(x))


def kernel2(kern, lam, r):
    return lib().orc2_kernel(int(kern), float(lam), float(r))


def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().orc_gauss_legendre(n, _dp(x), _dp(w))
    return x, w


class Tree:
    """Level-restricted adaptive tree (copied out of the C structure)."""

    def __init__(self, pts: np.ndarray, ns: int, maxdepth: int = 0):
        pts = np.ascontiguousarray(pts, dtype=np.float64)
        n, dim = pts.shape
        self._t = _Tree()
        rc = lib().orc_tree_build(dim, n, _dp(pts), ns, maxdepth, C.byref(self._t))
        if rc != 0:
            raise RuntimeError("orc_tree_build failed")
        t = self._t
        nb = t.nbox
        ncol = 3 ** dim
        nco = 2 ** dim - 1

        def arr(ptr, cnt, dt):
            if cnt == 0:
                return np.zeros(0, dtype=dt)
            return np.ctypeslib.as_array(ptr, shape=(cnt,)).astype(dt, copy=True)

        self.dim, self.n, self.ns, self.maxdepth = dim, n, ns, t.maxdepth
        self.center = np.array(t.center[:dim])
        self.side = t.side
        self.perm = arr(t.perm, n, np.int64)
        self.key = arr(t.key, n, np.uint64)
        self.xs = arr(t.xs, n * dim, np.float64).reshape(n, dim)
        self.nlevels = t.nlevels
        self.level_start = arr(t.level_start, t.nlevels + 1, np.int64)
        self.nbox = nb
        self.level = arr(t.level, nb, np.int32)
        self.bkey = arr(t.bkey, nb, np.uint64)
        self.parent = arr(t.parent, nb, np.int64)
        self.child0 = arr(t.child0, nb, np.int64)
        self.pstart = arr(t.pstart, nb, np.int64)
        self.pcount = arr(t.pcount, nb, np.int64)
        self.leaf = arr(t.leaf, nb, np.uint8)
        self.fout = arr(t.fout, nb, np.uint8)
        self.fin = arr(t.fin, nb, np.uint8)
        self.terminal = arr(t.terminal, nb, np.uint8)
        self.colleague = arr(t.colleague, nb * ncol, np.int64).reshape(nb, ncol)
        self.ncoarse = arr(t.ncoarse, nb, np.int32)
        self.coarse = arr(t.coarse, nb * nco, np.int64).reshape(nb, nco)
        self.tlevel = arr(t.tlevel, n, np.int32)

    def __del__(self):
        try:
            lib().orc_tree_free(C.byref(self._t))
        except Exception:
            pass


def dmk_eval(tree: Tree, params: Params, pswf: PSWF, charges: np.ndarray, keep: bool = False,
             kern: int = LOG2, lam: float = 0.0):
    """Run Steps 2-5 on a built tree.  Returns a dict with the potential in
    input order (u) and, in sorted order and normalised units, the far and
    residual parts; with keep=True also the per-box proxies and local values.
    kern and lam (input units): 2-D trees LOG2 / YUK2; 3-D trees LAP3 / YUK3."""
    q = np.ascontiguousarray(charges, dtype=np.float64)
    res = _Result()
    if tree.dim == 2:
        rc = lib().orc_dmk2_eval(C.byref(tree._t), C.byref(params), C.byref(pswf.s), int(kern), float(lam),
                                 _dp(q), 1 if keep else 0, C.byref(res))
    else:  # kern 0: 1/(4 pi r); kern 1: exp(-lam r)/(4 pi r); kern 2: 1/r^2
        rc = lib().orc_dmk_eval_k(C.byref(tree._t), C.byref(params), C.byref(pswf.s), int(kern), float(lam),
                                  _dp(q), 1 if keep else 0, C.byref(res))
    if rc != 0:
        raise RuntimeError("orc_dmk_eval failed")
    n = tree.n
    out = {}
    if n:
        out["u"] = np.ctypeslib.as_array(res.u, shape=(n,)).copy()
        out["ufar"] = np.ctypeslib.as_array(res.ufar, shape=(n,)).copy()
        out["ures"] = np.ctypeslib.as_array(res.ures, shape=(n,)).copy()
    else:
        out["u"] = np.zeros(0)
        out["ufar"] = np.zeros(0)
        out["ures"] = np.zeros(0)
    if keep and n:
        p3 = params.p ** tree.dim
        prox, loc = {}, {}
        for b in range(tree.nbox):
            if res.proxy[b]:
                prox[b] = np.ctypeslib.as_array(res.proxy[b], shape=(p3,)).copy()
            if res.local[b]:
                loc[b] = np.ctypeslib.as_array(res.local[b], shape=(p3,)).copy()
        out["proxy"] = prox
        out["local"] = loc
    lib().orc_dmk_result_free(C.byref(tree._t), C.byref(res))
    return out


def dmk(pts, charges, tol=1e-6, ns=50, maxdepth=0):
    pr = params_for(tol)
    ps = PSWF(pr.c)
    tr = Tree(pts, ns, maxdepth)
    return dmk_eval(tr, pr, ps, charges)["u"]


def dmk_run(pts, charges, tol, ns, maxdepth=0):
    """Whole pipeline in C; returns (u, plan_seconds, eval_seconds)."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    q = np.ascontiguousarray(charges, dtype=np.float64)
    n = pts.shape[0]
    u = np.zeros(n)
    tm = np.zeros(2)
    rc = lib().orc_dmk_run(n, _dp(pts), _dp(q), tol, ns, maxdepth, _dp(u), _dp(tm))
    if rc != 0:
        raise RuntimeError(f"orc_dmk_run failed ({rc})")
    return u, tm[0], tm[1]


def union_targets(src, q, tgt):
    """Separate target sets as one point set: the sources followed by the
    targets, which carry zero charge (they add nothing to any potential).
    Returns (union points, union charges, indices of the targets)."""
    src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3)
    tgt = np.ascontiguousarray(tgt, dtype=np.float64).reshape(-1, 3)
    pts = np.ascontiguousarray(np.concatenate([src, tgt]))
    qq = np.concatenate([np.asarray(q, dtype=np.float64), np.zeros(len(tgt))])
    return pts, qq, np.arange(len(src), len(src) + len(tgt), dtype=np.int64)


def direct(pts, charges, tidx=None):
    """u_i = sum_{j != i, r > 0} q_j / (4 pi r_ij) at the listed targets."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    q = np.ascontiguousarray(charges, dtype=np.float64)
    n = pts.shape[0]
    if tidx is None:
        tidx = np.arange(n, dtype=np.int64)
    tidx = np.ascontiguousarray(tidx, dtype=np.int64)
    out = np.zeros(len(tidx))
    lib().orc_direct(n, _dp(pts), _dp(q), len(tidx), tidx.ctypes.data_as(_i64p), _dp(out))
    return out


def direct2(kern, lam, pts, charges, tidx=None):
    """u_i = sum_{j != i, r > 0} K(r_ij) q_j, K = -log(r)/(2 pi) or K_0(lam r)."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    q = np.ascontiguousarray(charges, dtype=np.float64)
    n = pts.shape[0]
    if tidx is None:
        tidx = np.arange(n, dtype=np.int64)
    tidx = np.ascontiguousarray(tidx, dtype=np.int64)
    out = np.zeros(len(tidx))
    lib().orc_direct2(int(kern), float(lam), n, _dp(pts), _dp(q), len(tidx), tidx.ctypes.data_as(_i64p),
                      _dp(out))
    return out


def num_threads() -> int:
    return lib().orc_num_threads()


def set_threads(n: int) -> int:
    """threads of the oracle's parallel loops from now on; returns the previous count"""
    return int(lib().orc_set_threads(int(n)))


# ---------------------------------------------------------------- volume
def vparams_for(tol: float = 1e-3, q: int = 8) -> VParams:
    vp = VParams()
    if lib().orc_vparams_for(tol, q, C.byref(vp)) != 0:
        raise ValueError(f"unsupported volume parameters tol={tol} q={q}")
    return vp


def vfit(vp: VParams):
    """PSWF split (tol 1e-6): the fitted Gaussians (t s_L, w s_L) and the
    function they stand for, h(x) = (erf(theta1 x) - Phi(x)) / x."""
    n = vp.nfit
    t = np.array(vp.fit_t[:n])
    w = np.array(vp.fit_w[:n])
    return t, w, np.vectorize(lambda x: lib().orc_vfit_target(C.byref(vp), float(x)))


class GSplit:
    """Gaussian multilevel split of 1/r (unscaled, root box side 1)."""

    def __init__(self, vp: VParams):
        self.vp = vp

    def m(self, l, r):
        return lib().orc_gsplit_m(C.byref(self.vp), int(l), float(r))

    def d(self, l, r):
        return lib().orc_gsplit_d(C.byref(self.vp), int(l), float(r))

    def r(self, l, r):
        return lib().orc_gsplit_r(C.byref(self.vp), int(l), float(r))

    def dhat(self, l, k):
        return lib().orc_gdhat(C.byref(self.vp), int(l), float(k))

    def w0hat(self, k):
        return lib().orc_gw0hat(C.byref(self.vp), float(k))

    def d_pw(self, l, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().orc_gsplit_d_pw(C.byref(self.vp), int(l), _dp(x))

    def w0_pw(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return lib().orc_gsplit_w0_pw(C.byref(self.vp), _dp(x))

    def sog(self, t_lo, t_hi):
        n = lib().orc_vsog_count(C.byref(self.vp), float(t_lo), float(t_hi))
        t = np.zeros(max(n, 1))
        w = np.zeros(max(n, 1))
        lib().orc_vsog(C.byref(self.vp), float(t_lo), float(t_hi), _dp(t), _dp(w))
        return t[:n], w[:n]


def density_callback(f):
    """Wrap f(xyz[n,3]) -> rho[n] as the C density callback."""
    def cb(n, xyz, out, ctx):
        x = np.ctypeslib.as_array(xyz, shape=(n * 3,)).reshape(n, 3)
        o = np.ctypeslib.as_array(out, shape=(n,))
        o[:] = f(x)
    return DENSITY_FN(cb)


class VTree:
    """Leaves (level, cell) of the volume tree, in Morton order."""

    def __init__(self, vp: VParams, density, rho_scale: float, min_level: int = 0, max_level: int = 12,
                 features=None):
        self.vp = vp
        self._t = _VTree()
        self._cb = density_callback(density)
        feat = np.ascontiguousarray(np.zeros((0, 4)) if features is None else features, dtype=np.float64)
        self._feat = feat
        rc = lib().orc_vtree_build(C.byref(vp), float(rho_scale), int(min_level), int(max_level), len(feat),
                                   _dp(feat), self._cb, None, C.byref(self._t))
        if rc != 0:
            raise RuntimeError("orc_vtree_build failed")
        n = self._t.nleaf
        self.q, self.nleaf = vp.q, n
        self.level = np.ctypeslib.as_array(self._t.level, shape=(n,)).copy()
        self.ijk = np.ctypeslib.as_array(self._t.ijk, shape=(n * 3,)).reshape(n, 3).copy()

    def nodes(self):
        q3 = self.q ** 3
        xyz = np.zeros((self.nleaf * q3, 3))
        lib().orc_vol_nodes(C.byref(self._t), _dp(xyz))
        return xyz

    def eval(self, rho):
        """Potential at the leaf nodes; returns dict u, ufar, unear, utail."""
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        if rho.shape != (self.nleaf * self.q ** 3,):
            raise ValueError("rho must hold nleaf*q^3 node values")
        res = _VResult()
        if lib().orc_vol_eval(C.byref(self._t), C.byref(self.vp), _dp(rho), C.byref(res)) != 0:
            raise RuntimeError("orc_vol_eval failed")
        n = res.n
        out = {k: np.ctypeslib.as_array(getattr(res, k), shape=(n,)).copy() for k in ("u", "ufar", "unear", "utail")}
        lib().orc_vol_result_free(C.byref(res))
        return out

    def __del__(self):
        try:
            lib().orc_vtree_free(C.byref(self._t))
        except Exception:
            pass
