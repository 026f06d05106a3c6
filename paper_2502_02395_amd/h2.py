"""Python binding of the HIP H^2-ULV library (include/h2.h), argument
marshalling only: every step of build, factor, solve and matvec runs in the
library's kernels.  PyTorch provides device memory and the current stream.

Matrices cross the ABI column-major: an (n x nrhs) right-hand side is held
here as a torch tensor of shape (nrhs, n) (row-major storage of the transpose).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libh2.so")

OK, ERR_ARG, ERR_ALLOC, ERR_HIP, ERR_NOT_SPD, ERR_STATE, ERR_NOCONV, ERR_UNSUPPORTED = range(8)
PREC_FP64, PREC_FP32, PREC_BF16, PREC_BF16X3 = 0, 1, 2, 3
SYMBOLS = ["h2_build", "h2_build_batched", "h2_build_fixed", "h2_factor", "h2_solve",
           "h2_solve_noalloc", "h2_matvec",
           "h2_stats", "h2_get_counts", "h2_get_structure", "h2_get_pairs", "h2_get_basis",
           "h2_get_root", "h2_mlp_forward", "h2_mlp_train_step", "h2_box_features",
           "h2_destroy", "h2_status_str"]


class H2Error(RuntimeError):
    def __init__(self, status: int, what: str, where: dict | None = None):
        msg = f"{what}: {_status_str(status)} ({status})"
        if where:
            msg += " at level {fail_level}, box {fail_box}, instance {fail_inst}".format(**where)
        super().__init__(msg)
        self.status = status
        self.where = where


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    """h2_allocator: the device memory callbacks of a handle."""
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


class TorchAllocator:
    """PyTorch's caching allocator (on the current stream) behind h2_allocator.
    ``fail_at`` (1-based) makes that allocation call fail, to exercise the
    library's H2_ERR_ALLOC path; ``live`` counts outstanding allocations."""

    def __init__(self, fail_at: int = 0):
        self.fail_at = fail_at
        self.calls = 0
        self.live = 0
        self._alloc = _ALLOC_FN(self._do_alloc)
        self._free = _FREE_FN(self._do_free)
        self.struct = Allocator(self._alloc, self._free, None)

    def _do_alloc(self, nbytes, user):
        import torch
        self.calls += 1
        if self.fail_at and self.calls == self.fail_at:
            return None
        try:
            p = torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:  # out of memory: the library reports H2_ERR_ALLOC
            return None
        self.live += 1
        return p

    def _do_free(self, ptr, user):
        try:
            import torch
            torch.cuda.caching_allocator_delete(ptr)
            self.live -= 1
        except Exception:  # interpreter shutdown
            pass


_default_allocator = None


def default_allocator() -> TorchAllocator:
    global _default_allocator
    if _default_allocator is None:
        _default_allocator = TorchAllocator()
    return _default_allocator


class Kernel(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int32), ("delta", ctypes.c_double), ("kappa", ctypes.c_double),
                ("ell", ctypes.c_double), ("nugget", ctypes.c_double), ("beta", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("leaf", ctypes.c_int32), ("eta", ctypes.c_double),
                ("eps", ctypes.c_double), ("max_rank", ctypes.c_int32), ("s_far", ctypes.c_int32),
                ("s_near", ctypes.c_int32), ("gemm_prec", ctypes.c_int32),
                ("ir_max_iter", ctypes.c_int32), ("ir_tol", ctypes.c_double),
                ("use_pcg", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("rank_model", ctypes.c_void_p), ("rank_margin", ctypes.c_double),
                ("timing", ctypes.c_int32), ("no_autotune", ctypes.c_int32),
                ("solve_prec", ctypes.c_int32), ("gs_sweeps", ctypes.c_int32),
                ("allocator", ctypes.c_void_p), ("matvec_prec", ctypes.c_int32),
                ("factor_lu", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_inst", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("n_boxes", ctypes.c_int64), ("near_pairs", ctypes.c_int64),
                ("far_pairs", ctypes.c_int64), ("leaf_near_blocks", ctypes.c_int64),
                ("max_rank_seen", ctypes.c_int32), ("max_m_seen", ctypes.c_int32),
                ("root_n", ctypes.c_int32), ("flops_factor", ctypes.c_double),
                ("flops_solve", ctypes.c_double), ("bytes_factors", ctypes.c_double),
                ("t_build", ctypes.c_double), ("t_factor", ctypes.c_double),
                ("t_solve", ctypes.c_double), ("ir_iters", ctypes.c_int32),
                ("ir_residual", ctypes.c_double), ("fail_level", ctypes.c_int32),
                ("fail_box", ctypes.c_int32), ("fail_inst", ctypes.c_int32),
                ("rank_fallbacks", ctypes.c_int32), ("t_pair_gemm", ctypes.c_double),
                ("flops_pair_gemm", ctypes.c_double), ("pair_launches", ctypes.c_int32),
                ("bytes_basis", ctypes.c_double), ("tuned_lists", ctypes.c_int32),
                ("tuned_cfg_hist", ctypes.c_int32 * 4),
                ("t_gather", ctypes.c_double * 3), ("bytes_gather", ctypes.c_double * 3),
                ("gather_launches", ctypes.c_int32 * 3),
                ("t_factor_phase", ctypes.c_double * 9), ("gather_partials", ctypes.c_int64),
                ("flops_factor_phase", ctypes.c_double * 9), ("flops_schur", ctypes.c_double),
                ("t_build_id", ctypes.c_double), ("flops_prefactor", ctypes.c_double),
                ("ir_fp64_matvecs", ctypes.c_int32), ("t_gather_mv32", ctypes.c_double),
                ("bytes_gather_mv32", ctypes.c_double), ("gather_launches_mv32", ctypes.c_int32),
                ("lu_variant", ctypes.c_int32)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["tuned_cfg_hist"] = list(self.tuned_cfg_hist)
        for f in ("t_gather", "bytes_gather", "gather_launches", "t_factor_phase",
                  "flops_factor_phase"):
            d[f] = list(getattr(self, f))
        return d



_lib = None


def load() -> ctypes.CDLL:
    """Load libh2.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2502_02395_amd.build_lib`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.h2_status_str.restype = ctypes.c_char_p
    L.h2_status_str.argtypes = [ctypes.c_int]
    L.h2_build.argtypes = [vp, i64, P(Kernel), P(Params), vp, vp, P(vp)]
    L.h2_build_batched.argtypes = [i32, vp, vp, P(Kernel), P(Params), vp, vp, P(vp)]
    L.h2_build_fixed.argtypes = [vp, i64, P(Kernel), P(Params), vp, vp, vp, vp, P(vp)]
    L.h2_factor.argtypes = [vp, vp]
    L.h2_solve.argtypes = [vp, vp, vp, i64, i64, vp]
    L.h2_solve_noalloc.argtypes = [vp, vp, vp, i64, i64, vp]
    L.h2_matvec.argtypes = [vp, vp, vp, i64, i64, vp]
    L.h2_stats.argtypes = [vp, P(Stats)]
    L.h2_get_counts.argtypes = [vp, P(i64), P(i64)]
    L.h2_get_structure.argtypes = [vp, vp, vp, vp, vp]
    L.h2_get_pairs.argtypes = [vp, i32, i32, vp, P(i64)]
    L.h2_get_basis.argtypes = [vp, i32, i32, i32, vp, P(i32), P(i32)]
    L.h2_get_root.argtypes = [vp, i32, vp, P(i64)]
    L.h2_mlp_forward.argtypes = [vp, vp, vp, i64, vp]
    L.h2_mlp_train_step.argtypes = [vp, vp, vp, vp, vp, vp, i64, i32, ctypes.c_float, vp, vp]
    L.h2_box_features.argtypes = [vp, vp, vp]
    L.h2_destroy.argtypes = [vp]
    L.h2_destroy.restype = None
    for name in SYMBOLS:
        if name not in ("h2_status_str", "h2_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _status_str(s: int) -> str:
    try:
        return load().h2_status_str(s).decode()
    except Exception:  # library unavailable while formatting an error
        return "status"


def _check(s: int, what: str):
    if s != OK:
        raise H2Error(s, what)


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_kernel(k) -> Kernel:
    return Kernel(int(k.id), float(k.delta), float(k.kappa), float(k.ell), float(k.nugget),
                  float(getattr(k, "beta", 0.0)))


def make_params(dim: int, leaf: int, eta: float, eps: float, s_far: int = -1, s_near: int = -1,
                max_rank: int = 0, gemm_prec: int = PREC_FP64, ir_max_iter: int = 0,
                ir_tol: float = 1e-10, use_pcg: bool = False, use_graph: bool = False,
                timing: bool = False, rank_model=None, rank_margin: float = 0.25,
                autotune: bool = True, solve_prec: int = PREC_FP64, gs_sweeps: int = 0,
                allocator=None, matvec_prec: int = PREC_FP64, factor_lu: bool = False) -> Params:
    """rank_model: numpy float32 array of the 4801 predictor weights (kept alive
    by the caller for the duration of the build call).  allocator: a
    TorchAllocator (or None: the library's hipMalloc); it must outlive the
    handle."""
    ptr = None
    if rank_model is not None:
        assert rank_model.dtype == np.float32 and rank_model.size == 4801
        assert rank_model.flags["C_CONTIGUOUS"]
        ptr = rank_model.ctypes.data
    aptr = None if allocator is None else ctypes.addressof(allocator.struct)
    return Params(dim, leaf, eta, eps, max_rank, s_far, s_near, gemm_prec, ir_max_iter, ir_tol,
                  int(use_pcg), int(use_graph), ptr, rank_margin, int(timing), int(not autotune),
                  int(solve_prec), int(gs_sweeps), aptr, int(matvec_prec), int(factor_lu))


def _as_cols(t, n):
    """(n,) or (n, nrhs) tensor -> contiguous (nrhs, n) float64 on the device."""
    import torch
    if t.dim() == 1:
        t = t[:, None]
    assert t.shape[0] == n
    return t.to(dtype=torch.float64).t().contiguous()


class Handle:
    """An H^2 matrix built on the device (one instance or a batch)."""

    def __init__(self, ptr: ctypes.c_void_p, n: int, allocator=None):
        self._h = ptr
        self.n = n
        self._allocator = allocator  # its callbacks must outlive the handle

    def close(self):
        if self._h:
            load().h2_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def factor(self, stream=None):
        _check(load().h2_factor(self._h, _stream(stream)), "h2_factor")

    def solve(self, b, stream=None):
        """b: device tensor (n,) or (n, nrhs); returns x of the same shape."""
        import torch
        cols = _as_cols(b, self.n)
        x = torch.empty_like(cols)
        s = load().h2_solve(self._h, ctypes.c_void_p(cols.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                            cols.shape[0], self.n, _stream(stream))
        if s not in (OK, ERR_NOCONV):
            _check(s, "h2_solve")
        self.last_solve_status = s
        out = x.t()
        return out[:, 0] if b.dim() == 1 else out

    def solve_into(self, cols_b, cols_x, stream=None) -> int:
        """Raw form: (nrhs, n) contiguous tensors, no copies; returns the status."""
        return load().h2_solve(self._h, ctypes.c_void_p(cols_b.data_ptr()),
                               ctypes.c_void_p(cols_x.data_ptr()), cols_b.shape[0], self.n,
                               _stream(stream))

    def solve_noalloc_into(self, cols_b, cols_x, stream=None) -> int:
        """h2_solve_noalloc on (nrhs, n) contiguous tensors; returns the status."""
        return load().h2_solve_noalloc(self._h, ctypes.c_void_p(cols_b.data_ptr()),
                                       ctypes.c_void_p(cols_x.data_ptr()), cols_b.shape[0],
                                       self.n, _stream(stream))

    def matvec(self, x, stream=None):
        import torch
        cols = _as_cols(x, self.n)
        y = torch.empty_like(cols)
        _check(load().h2_matvec(self._h, ctypes.c_void_p(cols.data_ptr()),
                                ctypes.c_void_p(y.data_ptr()), cols.shape[0], self.n,
                                _stream(stream)), "h2_matvec")
        out = y.t()
        return out[:, 0] if x.dim() == 1 else out

    def stats(self) -> dict:
        s = Stats()
        _check(load().h2_stats(self._h, ctypes.byref(s)), "h2_stats")
        return s.as_dict()

    def structure(self):
        """(perm, ranks, ms, skeleton ids) as numpy arrays, boxes in levels L..1."""
        L = load()
        nb, nsk = ctypes.c_int64(), ctypes.c_int64()
        _check(L.h2_get_counts(self._h, ctypes.byref(nb), ctypes.byref(nsk)), "h2_get_counts")
        perm = np.zeros(self.n, dtype=np.int64)
        ranks = np.zeros(nb.value, dtype=np.int32)
        ms = np.zeros(nb.value, dtype=np.int32)
        skel = np.zeros(nsk.value, dtype=np.int64)
        _check(L.h2_get_structure(self._h, perm.ctypes.data, ranks.ctypes.data, ms.ctypes.data,
                                  skel.ctypes.data), "h2_get_structure")
        return perm, ranks, ms, skel

    def pairs(self, level: int, far: bool) -> list:
        L = load()
        cnt = ctypes.c_int64()
        _check(L.h2_get_pairs(self._h, level, int(far), None, ctypes.byref(cnt)), "h2_get_pairs")
        buf = np.zeros(2 * cnt.value, dtype=np.int32)
        _check(L.h2_get_pairs(self._h, level, int(far), buf.ctypes.data, ctypes.byref(cnt)),
               "h2_get_pairs")
        return [(int(buf[2 * q]), int(buf[2 * q + 1])) for q in range(cnt.value)]

    def basis(self, level: int, box: int, inst: int = 0):
        """(P, k): the two-sided basis [Q^S | Q^R L(r)^{-T}] (m x m) of a box
        after factor, and its rank."""
        L = load()
        m, k = ctypes.c_int32(), ctypes.c_int32()
        _check(L.h2_get_basis(self._h, inst, level, box, None, ctypes.byref(m), ctypes.byref(k)),
               "h2_get_basis")
        a = np.zeros((m.value, m.value))
        _check(L.h2_get_basis(self._h, inst, level, box, a.ctypes.data, ctypes.byref(m),
                              ctypes.byref(k)), "h2_get_basis")
        return a.T.copy(), k.value  # column-major -> row-major

    def root(self, inst: int = 0) -> np.ndarray:
        L = load()
        n0 = ctypes.c_int64()
        _check(L.h2_get_root(self._h, inst, None, ctypes.byref(n0)), "h2_get_root")
        a = np.zeros((n0.value, n0.value))
        _check(L.h2_get_root(self._h, inst, a.ctypes.data, ctypes.byref(n0)), "h2_get_root")
        return a.T.copy()  # column-major -> row-major

    def box_features(self):
        import torch
        nb = ctypes.c_int64()
        _check(load().h2_get_counts(self._h, ctypes.byref(nb), None), "h2_get_counts")
        f = torch.empty((nb.value, 8), dtype=torch.float32, device="cuda")
        _check(load().h2_box_features(self._h, ctypes.c_void_p(f.data_ptr()), _stream(None)),
               "h2_box_features")
        return f


def _built(status: int, out: ctypes.c_void_p, what: str, n: int, alloc) -> Handle:
    """A successful build's handle; otherwise raise (a breakdown's failed-state
    handle is read for the location, then destroyed)."""
    if status == OK:
        return Handle(out, n, alloc)
    where = None
    if status == ERR_NOT_SPD and out.value:
        s = Stats()
        if load().h2_stats(out, ctypes.byref(s)) == OK:
            where = {"fail_level": s.fail_level, "fail_box": s.fail_box,
                     "fail_inst": s.fail_inst}
        load().h2_destroy(out)
    raise H2Error(status, what, where)


def _alloc_kw(kw: dict):
    """The allocator a build uses: PyTorch's caching allocator unless the
    caller passes one (allocator=None selects the library's hipMalloc)."""
    if "allocator" not in kw:
        kw["allocator"] = default_allocator()
    return kw["allocator"]


def build(points: np.ndarray, kernel, leaf: int, eta: float, eps: float, perm=None,
          s_far: int = -1, s_near: int = -1, stream=None, **kw) -> Handle:
    L = load()
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n, dim = pts.shape
    alloc = _alloc_kw(kw)
    prm = make_params(dim, leaf, eta, eps, s_far, s_near, **kw)
    k = make_kernel(kernel)
    pp = None if perm is None else np.ascontiguousarray(perm, dtype=np.int64)
    out = ctypes.c_void_p()
    s = L.h2_build(pts.ctypes.data, n, ctypes.byref(k), ctypes.byref(prm),
                   None if pp is None else pp.ctypes.data, _stream(stream), ctypes.byref(out))
    return _built(s, out, "h2_build", n, alloc)


def build_fixed(points: np.ndarray, kernel, leaf: int, eta: float, eps: float, perm, ranks,
                skel, s_far: int = -1, s_near: int = -1, stream=None, **kw) -> Handle:
    """Build with a prescribed skeleton selection (ranks per box in levels
    L..1 order, skeleton positions concatenated)."""
    L = load()
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n, dim = pts.shape
    alloc = _alloc_kw(kw)
    prm = make_params(dim, leaf, eta, eps, s_far, s_near, **kw)
    k = make_kernel(kernel)
    pp = np.ascontiguousarray(perm, dtype=np.int64)
    rk = np.ascontiguousarray(ranks, dtype=np.int32)
    sk = np.ascontiguousarray(skel, dtype=np.int32)
    out = ctypes.c_void_p()
    s = L.h2_build_fixed(pts.ctypes.data, n, ctypes.byref(k), ctypes.byref(prm), pp.ctypes.data,
                         rk.ctypes.data, sk.ctypes.data, _stream(stream), ctypes.byref(out))
    return _built(s, out, "h2_build_fixed", n, alloc)


def build_batched(point_sets, kernels, leaf: int, eta: float, eps: float, perms=None,
                  s_far: int = -1, s_near: int = -1, stream=None, **kw) -> Handle:
    L = load()
    pts = [np.ascontiguousarray(p, dtype=np.float64) for p in point_sets]
    ns = np.array([p.shape[0] for p in pts], dtype=np.int64)
    dim = pts[0].shape[1]
    alloc = _alloc_kw(kw)
    prm = make_params(dim, leaf, eta, eps, s_far, s_near, **kw)
    ks = (Kernel * len(pts))(*[make_kernel(k) for k in kernels])
    pptr = (ctypes.c_void_p * len(pts))(*[p.ctypes.data for p in pts])
    if perms is not None:
        perms = [np.ascontiguousarray(q, dtype=np.int64) for q in perms]
        qptr = (ctypes.c_void_p * len(pts))(*[q.ctypes.data for q in perms])
    else:
        qptr = None
    out = ctypes.c_void_p()
    s = L.h2_build_batched(len(pts), pptr, ns.ctypes.data, ks, ctypes.byref(prm), qptr,
                           _stream(stream), ctypes.byref(out))
    h = _built(s, out, "h2_build_batched", int(ns.sum()), alloc)
    h._keep = (pts, perms)
    return h


def mlp_forward(w, x, stream=None):
    import torch
    y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    _check(load().h2_mlp_forward(ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                 ctypes.c_void_p(y.data_ptr()), x.shape[0], _stream(stream)),
           "h2_mlp_forward")
    return y


def mlp_train_step(w, m, v, g, x, t, step: int, lr: float, loss, stream=None):
    _check(load().h2_mlp_train_step(*(ctypes.c_void_p(a.data_ptr()) for a in (w, m, v, g, x, t)),
                                    x.shape[0], step, lr, ctypes.c_void_p(loss.data_ptr()),
                                    _stream(stream)), "h2_mlp_train_step")

