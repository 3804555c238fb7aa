"""MI355X (gfx950) DMK point code: Python binding of the C ABI in include/dmk.h.

Argument marshalling only: every stage of the computation runs in the HIP
kernels of ``libdmk.so``.  PyTorch supplies device memory and streams.  There
is no fallback: if the library is missing, importing a binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libdmk.so")

DMK_FP64, DMK_MIXED = 0, 1
DMK_LAPLACE, DMK_YUKAWA, DMK_POWER2 = 0, 1, 2
DMK_FLAG_BATCHED = 2
DMK_FLAG_NO_WORKSPACE = 4
DMK_FLAG_LEVEL_LAUNCHES = 8
DMK_FLAG_QUEUE_LAUNCHES = 16
NOALLOC_MAX_BYTES = 128 << 20

# exported symbols, in the order of include/dmk.h
SYMBOLS = ["dmk_plan", "dmk_plan_targets", "dmk_plan_batched", "dmk_tune_leaf", "dmk_tune", "dmk_problem_info", "dmk_eval", "dmk_eval_noalloc", "dmk_eval_parts",
           "dmk_plan_info", "dmk_export_tree", "dmk_export_near_lists", "dmk_copy_box_data", "dmk_precompute_probe",
           "dmk_stage_timing", "dmk_stage_times", "dmk_stage_work",
           "dmk_vol_plan", "dmk_vol_info", "dmk_vol_leaves", "dmk_vol_nodes", "dmk_vol_eval",
           "dmk_plan_destroy", "dmk_last_error"]

# density callback of dmk_vol_plan: (n, xyz[3n], out[n], ctx), host arrays
DENSITY_FN = C.CFUNCTYPE(None, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p)

STAGES = ["gather", "upward", "root", "proxy2pw", "local", "pwshift", "pw2grid", "leaf",
          "residual", "finalize"]


class Opts(C.Structure):
    _fields_ = [("leaf_max", C.c_int32), ("max_depth", C.c_int32), ("precision", C.c_int32),
                ("reserved0", C.c_int32), ("flags", C.c_uint64), ("lambda_", C.c_double),
                ("p", C.c_int32), ("n_f", C.c_int32), ("pswf_c", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("nbox", C.c_int64), ("nlevels", C.c_int32), ("p", C.c_int32),
                ("nf", C.c_int32), ("nw", C.c_int32), ("c", C.c_double), ("tol", C.c_double),
                ("leaf_max", C.c_int32), ("precision", C.c_int32), ("nleaf", C.c_int64),
                ("nfout", C.c_int64), ("nfin", C.c_int64), ("npairs", C.c_int64),
                ("device_bytes", C.c_int64), ("center", C.c_double * 3), ("side", C.c_double),
                ("dim", C.c_int32), ("nprob", C.c_int32), ("nsrc", C.c_int64), ("ntgt", C.c_int64),
                ("queue_timeouts", C.c_int32), ("reserved1", C.c_int32)]


class DmkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"DMK status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """The loaded libdmk.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} is missing: build it with paper_2308_00292_amd/build.py")
        L = C.CDLL(LIBPATH)
        vp, i64, f64p = C.c_void_p, C.c_int64, C.POINTER(C.c_double)
        L.dmk_plan.argtypes = [C.c_int, C.c_int, C.c_double, i64, vp, C.POINTER(Opts), vp, C.POINTER(vp)]
        L.dmk_plan_targets.argtypes = [C.c_int, C.c_int, C.c_double, i64, vp, i64, vp, C.POINTER(Opts), vp,
                                       C.POINTER(vp)]
        L.dmk_plan_batched.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int32, vp, vp, C.POINTER(Opts), vp,
                                       C.POINTER(vp)]
        L.dmk_problem_info.argtypes = [vp, C.c_int32, f64p, f64p]
        L.dmk_tune_leaf.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int32, vp, vp, vp, C.POINTER(Opts), vp,
                                    C.c_int32, C.c_int32, vp, vp, vp]
        L.dmk_tune.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int32, vp, vp, vp, C.POINTER(Opts), vp,
                               C.c_int32, C.c_int32, vp, C.POINTER(Opts), vp, vp]
        L.dmk_eval.argtypes = [vp, vp, vp, vp]
        L.dmk_eval_noalloc.argtypes = [vp, vp, vp, vp]
        L.dmk_eval_parts.argtypes = [vp, vp, vp, vp, vp]
        L.dmk_plan_info.argtypes = [vp, C.POINTER(Stats)]
        L.dmk_export_tree.argtypes = [vp] + [vp] * 11
        L.dmk_export_near_lists.argtypes = [vp, vp, vp, vp]
        L.dmk_copy_box_data.argtypes = [vp, C.c_int, i64, f64p]
        L.dmk_precompute_probe.argtypes = [C.c_double, C.c_int, i64, vp, vp]
        L.dmk_stage_timing.argtypes = [vp, C.c_int]
        L.dmk_stage_times.argtypes = [vp, vp, vp, C.c_int]
        L.dmk_stage_work.argtypes = [vp, vp, vp, C.c_int]
        L.dmk_vol_plan.argtypes = [C.c_double, C.c_int32, C.c_double, C.c_int32, C.c_int32, C.c_int32, vp,
                                   DENSITY_FN, vp, C.POINTER(Opts), vp, C.POINTER(vp)]
        L.dmk_vol_info.argtypes = [vp, vp, vp]
        L.dmk_vol_leaves.argtypes = [vp, vp, vp]
        L.dmk_vol_nodes.argtypes = [vp, vp, vp]
        L.dmk_vol_eval.argtypes = [vp, vp, vp, vp, vp, vp]
        L.dmk_plan_destroy.argtypes = [vp]
        L.dmk_plan_destroy.restype = None
        L.dmk_last_error.restype = C.c_char_p
        for f in SYMBOLS[:-2]:
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise DmkError(rc, lib().dmk_last_error().decode())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def tune_leaf(pts, charges, candidates, tol=1e-6, precision=DMK_FP64, flags=0, reps=3, kernel=DMK_LAPLACE,
              lam=0.0, offsets=None, stream=None):
    """dmk_tune_leaf: (best leaf capacity, {candidate: mean eval ms})."""
    pts = pts.contiguous()
    q = charges.contiguous()
    n, dim = int(pts.shape[0]), int(pts.shape[1])
    off = np.ascontiguousarray([0, n] if offsets is None else offsets, dtype=np.int64)
    cand = np.ascontiguousarray(candidates, dtype=np.int32)
    ms = np.zeros(len(cand))
    best = np.zeros(1, dtype=np.int32)
    o = Opts(0, 0, precision, 0, flags, float(lam))
    _check(lib().dmk_tune_leaf(dim, int(kernel), float(tol), len(off) - 1, _np_ptr(off), _ptr(pts), _ptr(q),
                               C.byref(o), _np_ptr(cand), len(cand), int(reps), _stream_handle(stream),
                               _np_ptr(best), _np_ptr(ms)))
    return int(best[0]), dict(zip(cand.tolist(), ms.tolist()))


def tune(pts, charges, candidates, tol=1e-6, precision=DMK_FP64, flags=0, reps=3, kernel=DMK_LAPLACE, lam=0.0,
         offsets=None, p=0, n_f=0, stream=None):
    """dmk_tune: (best options as a dict, {candidate: mean eval ms}, sampled error)."""
    pts = pts.contiguous()
    q = charges.contiguous()
    n, dim = int(pts.shape[0]), int(pts.shape[1])
    off = np.ascontiguousarray([0, n] if offsets is None else offsets, dtype=np.int64)
    cand = np.ascontiguousarray(candidates, dtype=np.int32)
    ms = np.zeros(len(cand))
    err = np.zeros(1)
    o = Opts(0, 0, precision, 0, flags, float(lam), int(p), int(n_f), 0.0)
    best = Opts()
    _check(lib().dmk_tune(dim, int(kernel), float(tol), len(off) - 1, _np_ptr(off), _ptr(pts), _ptr(q),
                          C.byref(o), _np_ptr(cand), len(cand), int(reps), _stream_handle(stream), C.byref(best),
                          _np_ptr(ms), _np_ptr(err)))
    b = dict(leaf_max=best.leaf_max, p=best.p, n_f=best.n_f, pswf_c=best.pswf_c)
    return b, dict(zip(cand.tolist(), ms.tolist())), float(err[0])


def precompute_probe(tol, what, x=None, n=None):
    """Host-only view of the precomputed tables (see dmk_precompute_probe)."""
    if x is not None:
        x = np.ascontiguousarray(x, dtype=np.float64)
        n = len(x)
    out = np.zeros(n)
    _check(lib().dmk_precompute_probe(float(tol), int(what), int(n), _np_ptr(x), _np_ptr(out)))
    return out


class Plan:
    """dmk_plan on device points [n, dim] (dim 2 or 3); with offsets (host
    int64 [nprob+1]) dmk_plan_batched over the concatenated problems.
    eval() applies dmk_eval to charge vectors."""

    def __init__(self, pts, tol=1e-6, leaf_max=64, max_depth=0, precision=DMK_FP64, flags=0,
                 stream=None, kernel=DMK_LAPLACE, lam=0.0, offsets=None, p=0, n_f=0, pswf_c=0.0, targets=None):
        import torch
        if not (isinstance(pts, torch.Tensor) and pts.is_cuda and pts.dtype == torch.float64
                and pts.dim() == 2 and pts.shape[1] in (2, 3)):
            raise TypeError("pts must be a float64 CUDA tensor of shape [n, 2] or [n, 3]")
        pts = pts.contiguous()
        self.n = int(pts.shape[0])
        self.dim = int(pts.shape[1])
        o = Opts(leaf_max, max_depth, precision, 0, flags, float(lam), int(p), int(n_f), float(pswf_c))
        h = C.c_void_p()
        self.nsrc = self.ntgt = self.n
        if targets is not None:
            if not (isinstance(targets, torch.Tensor) and targets.is_cuda and targets.dtype == torch.float64
                    and targets.dim() == 2 and targets.shape[1] == self.dim):
                raise TypeError("targets must be a float64 CUDA tensor of shape [m, dim]")
            targets = targets.contiguous()
            self.ntgt = int(targets.shape[0])
            _check(lib().dmk_plan_targets(self.dim, int(kernel), float(tol), self.n, _ptr(pts), self.ntgt,
                                          _ptr(targets), C.byref(o), _stream_handle(stream), C.byref(h)))
        elif offsets is None:
            _check(lib().dmk_plan(self.dim, int(kernel), float(tol), self.n, _ptr(pts), C.byref(o),
                                  _stream_handle(stream), C.byref(h)))
        else:
            off = np.ascontiguousarray(offsets, dtype=np.int64)
            if off[-1] != self.n:
                raise ValueError("offsets[-1] must equal the number of points")
            _check(lib().dmk_plan_batched(self.dim, int(kernel), float(tol), len(off) - 1, _np_ptr(off),
                                          _ptr(pts), C.byref(o), _stream_handle(stream), C.byref(h)))
        self._h = h
        self.device = pts.device

    def close(self):
        if getattr(self, "_h", None):
            lib().dmk_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def eval(self, charges, out=None, stream=None):
        import torch
        q = charges.contiguous()
        if q.dtype != torch.float64 or not q.is_cuda or q.numel() != self.nsrc:
            raise TypeError("charges must be a float64 CUDA tensor with one entry per source")
        if out is None:
            out = torch.empty(self.ntgt, dtype=torch.float64, device=q.device)
        _check(lib().dmk_eval(self._h, _ptr(q), _ptr(out), _stream_handle(stream)))
        return out

    def eval_noalloc(self, charges, out, stream=None):
        """dmk_eval_noalloc: the workspace comes from the library's static
        scratch; ``out`` (float64 CUDA [n]) is required, nothing is allocated."""
        import torch
        if charges.dtype != torch.float64 or not charges.is_cuda or charges.numel() != self.nsrc \
                or not charges.is_contiguous():
            raise TypeError("charges must be a contiguous float64 CUDA tensor with one entry per source")
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() != self.ntgt or not out.is_contiguous():
            raise TypeError("out must be a contiguous float64 CUDA tensor with one entry per target")
        _check(lib().dmk_eval_noalloc(self._h, _ptr(charges), _ptr(out), _stream_handle(stream)))
        return out

    def eval_parts(self, charges, stream=None):
        import torch
        q = charges.contiguous()
        far = torch.empty(self.ntgt, dtype=torch.float64, device=q.device)
        near = torch.empty(self.ntgt, dtype=torch.float64, device=q.device)
        _check(lib().dmk_eval_parts(self._h, _ptr(q), _ptr(far), _ptr(near), _stream_handle(stream)))
        return far, near

    def info(self):
        st = Stats()
        _check(lib().dmk_plan_info(self._h, C.byref(st)))
        d = {k: getattr(st, k) for k, _ in Stats._fields_}
        d["center"] = list(st.center)
        return d

    def problem_info(self, b):
        c = np.zeros(3)
        sd = np.zeros(1)
        _check(lib().dmk_problem_info(self._h, int(b), c.ctypes.data_as(C.POINTER(C.c_double)),
                                      sd.ctypes.data_as(C.POINTER(C.c_double))))
        return c[: self.dim], float(sd[0])

    def export_tree(self):
        inf = self.info()
        n, nb = inf["n"], inf["nbox"]
        ncol, nco = 3 ** self.dim, 2 ** self.dim - 1
        out = dict(perm=np.zeros(n, np.int64), level=np.zeros(nb, np.int32),
                   bkey=np.zeros(nb, np.uint64), parent=np.zeros(nb, np.int64),
                   child0=np.zeros(nb, np.int64), pstart=np.zeros(nb, np.int64),
                   pcount=np.zeros(nb, np.int64), flags=np.zeros(nb, np.uint8),
                   colleague=np.zeros((nb, ncol), np.int64), ncoarse=np.zeros(nb, np.int32),
                   coarse=np.zeros((nb, nco), np.int64))
        keys = ["perm", "level", "bkey", "parent", "child0", "pstart", "pcount", "flags",
                "colleague", "ncoarse", "coarse"]
        _check(lib().dmk_export_tree(self._h, *[_np_ptr(out[k]) for k in keys]))
        return out

    def export_near_lists(self):
        inf = self.info()
        nl = inf["nleaf"]
        leaf = np.zeros(max(nl, 1), np.int64)
        off = np.zeros(nl + 1, np.int64)
        _check(lib().dmk_export_near_lists(self._h, _np_ptr(leaf), _np_ptr(off), None))
        src = np.zeros(max(int(off[-1]), 1), np.int64)
        _check(lib().dmk_export_near_lists(self._h, _np_ptr(leaf), _np_ptr(off), _np_ptr(src)))
        return leaf[:nl], off, src[: int(off[-1])]

    def stage_timing(self, enable=True):
        _check(lib().dmk_stage_timing(self._h, 1 if enable else 0))

    def stage_times(self):
        ms = np.zeros(len(STAGES))
        cnt = np.zeros(len(STAGES), np.int64)
        _check(lib().dmk_stage_times(self._h, _np_ptr(ms), _np_ptr(cnt), len(STAGES)))
        return dict(zip(STAGES, ms)), dict(zip(STAGES, cnt))

    def stage_work(self):
        fl = np.zeros(len(STAGES))
        by = np.zeros(len(STAGES))
        _check(lib().dmk_stage_work(self._h, _np_ptr(fl), _np_ptr(by), len(STAGES)))
        return dict(zip(STAGES, fl)), dict(zip(STAGES, by))

    def box_data(self, what, box):
        p = self.info()["p"]
        out = np.zeros(p ** self.dim)
        _check(lib().dmk_copy_box_data(self._h, int(what), int(box),
                                       out.ctypes.data_as(C.POINTER(C.c_double))))
        return out


class VolPlan:
    """dmk_vol_plan: volume potential of a density on the unit cube.
    ``density`` maps host coordinates [n, 3] (numpy) to values [n]; it is
    called while the tree is built.  eval(rho) maps node values (CUDA float64
    [npoints]) to potentials at the same nodes."""

    def __init__(self, density, tol=1e-3, q=8, rho_scale=1.0, min_level=1, max_level=12, features=None,
                 precision=DMK_FP64, flags=0, stream=None):
        def cb(n, xyz, out, ctx):
            x = np.ctypeslib.as_array(xyz, shape=(n * 3,)).reshape(n, 3)
            o = np.ctypeslib.as_array(out, shape=(n,))
            o[:] = density(x)
        self._cb = DENSITY_FN(cb)
        o = Opts(0, 0, precision, 0, int(flags), 0.0)
        h = C.c_void_p()
        feat = np.ascontiguousarray(np.zeros((0, 4)) if features is None else features, dtype=np.float64)
        _check(lib().dmk_vol_plan(float(tol), int(q), float(rho_scale), int(min_level), int(max_level), len(feat),
                                  _np_ptr(feat) if len(feat) else None, self._cb, None, C.byref(o),
                                  _stream_handle(stream), C.byref(h)))
        self._h = h
        nl = np.zeros(1, np.int64)
        npt = np.zeros(1, np.int64)
        _check(lib().dmk_vol_info(self._h, _np_ptr(nl), _np_ptr(npt)))
        self.nleaf, self.n, self.q = int(nl[0]), int(npt[0]), int(q)

    def close(self):
        if getattr(self, "_h", None):
            lib().dmk_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        return Plan.info(self)

    def leaves(self):
        lev = np.zeros(self.nleaf, np.int32)
        ijk = np.zeros((self.nleaf, 3), np.int32)
        _check(lib().dmk_vol_leaves(self._h, _np_ptr(lev), _np_ptr(ijk)))
        return lev, ijk

    def nodes(self, stream=None):
        import torch
        xyz = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
        _check(lib().dmk_vol_nodes(self._h, _ptr(xyz), _stream_handle(stream)))
        return xyz

    def eval(self, rho, out=None, parts=False, stream=None):
        """u at the nodes; with parts=True returns (u, far, near)."""
        import torch
        r = rho.contiguous()
        if r.dtype != torch.float64 or not r.is_cuda or r.numel() != self.n:
            raise TypeError("rho must be a float64 CUDA tensor with one value per node")
        if out is None:
            out = torch.empty_like(r)
        far = torch.empty_like(r) if parts else None
        near = torch.empty_like(r) if parts else None
        _check(lib().dmk_vol_eval(self._h, _ptr(r), _ptr(out), _ptr(far), _ptr(near), _stream_handle(stream)))
        return (out, far, near) if parts else out

    def stage_timing(self, enable=True):
        _check(lib().dmk_stage_timing(self._h, 1 if enable else 0))

    def stage_times(self):
        ms = np.zeros(len(STAGES))
        cnt = np.zeros(len(STAGES), np.int64)
        _check(lib().dmk_stage_times(self._h, _np_ptr(ms), _np_ptr(cnt), len(STAGES)))
        return dict(zip(STAGES, ms)), dict(zip(STAGES, cnt))

    def stage_work(self):
        fl = np.zeros(len(STAGES))
        by = np.zeros(len(STAGES))
        _check(lib().dmk_stage_work(self._h, _np_ptr(fl), _np_ptr(by), len(STAGES)))
        return dict(zip(STAGES, fl)), dict(zip(STAGES, by))
