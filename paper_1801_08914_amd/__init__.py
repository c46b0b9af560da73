"""MI355X hybridization library: thin Python binding over libhyb.so.

Every step of the path runs in the library's HIP kernels; this module only
marshals arguments (numpy arrays for the host-side mesh, torch tensors for
device buffers and the current HIP stream).  There is no CPU fallback: if
``libhyb.so`` is missing, every entry point raises.

Usage::

    plan = Plan(xyz, e2v, k)            # host topology (no GPU needed)
    plan.bind()                          # device buffers on cuda:0
    plan.setup(alpha, beta, f)           # M_T, Cholesky, H_T -> H, r
    lam, info = plan.pcg(1e-12, 2000)    # Jacobi-PCG on H
    u = plan.recover(lam)                # broken flux, ne x n
    lam, u, info = plan.solve(f2)        # rhs + PCG + recovery for a new load
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _abi

__all__ = ["Plan", "Batch", "HybError", "load_library", "LIB_PATH"]

LIB_PATH = _abi.LIB_PATH
HybError = _abi.HybError
load_library = _abi.load_library


def _dptr(t):
    return ctypes.c_void_p(0 if t is None else int(t.data_ptr()))


class Plan:
    """One hybridization problem: mesh + order, its topology and device buffers."""

    def __init__(self, xyz: np.ndarray, e2v: np.ndarray, k: int, stream=None, generic: bool = False,
                 pcg_reduce: int = 0, precision: str = "fp64", sweeps: int | None = None,
                 system: str = "hybrid", weighted_c: bool = False, ess=None, quad_q: int = 0):
        lib = load_library()
        self._lib = lib
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.e2v = np.ascontiguousarray(e2v, dtype=np.int32)
        self.k = int(k)
        # ess (ne, 6): 0 marks a natural boundary face (None: all essential)
        self.ess = None if ess is None else np.ascontiguousarray(ess, dtype=np.uint8).reshape(-1, 6)
        if self.ess is not None and self.ess.shape[0] != self.e2v.shape[0]:
            raise ValueError("ess must have one row of 6 flags per element")
        mesh = _abi.HybMesh(self.xyz.shape[0], self.e2v.shape[0],
                            self.xyz.ctypes.data_as(ctypes.c_void_p),
                            self.e2v.ctypes.data_as(ctypes.c_void_p),
                            None if self.ess is None else self.ess.ctypes.data_as(ctypes.c_void_p))
        self._stream_obj = stream
        if precision not in ("fp64", "mixed"):
            raise ValueError(f"precision must be 'fp64' or 'mixed', not {precision!r}")
        if system not in ("hybrid", "static"):
            raise ValueError(f"system must be 'hybrid' or 'static', not {system!r}")
        self.precision, self.system = precision, system
        opts = _abi.HybOpts(_abi.HYB_MIXED if precision == "mixed" else _abi.HYB_FP64,
                            ctypes.c_void_p(self._stream_handle()), 1 if generic else 0,
                            -1 if sweeps is None else int(sweeps), int(pcg_reduce),
                            _abi.HYB_STATIC if system == "static" else _abi.HYB_HYBRID, 1 if weighted_c else 0,
                            int(quad_q))
        self._plan = ctypes.c_void_p()
        sz = _abi.HybSizes()
        rc = lib.hyb_plan_create(ctypes.byref(mesh), self.k, ctypes.byref(opts), ctypes.byref(self._plan),
                                 ctypes.byref(sz))
        _abi.check(lib, rc)
        self.sizes = sz
        self.ne, self.n, self.m, self.nnz = sz.ne, sz.n_local, sz.m, sz.nnz
        self.bufs = None

    def _stream_handle(self) -> int:
        if self._stream_obj is None:
            return 0                     # the null stream (torch's default stream)
        return int(self._stream_obj.cuda_stream)

    def set_stream(self, stream):
        """Run the plan's later work on ``stream`` (a torch.cuda.Stream or None)."""
        self._stream_obj = stream
        _abi.check(self._lib, self._lib.hyb_set_stream(self._plan, ctypes.c_void_p(self._stream_handle())))

    def __del__(self):
        try:
            if getattr(self, "_plan", None) and self._plan.value:
                self._lib.hyb_destroy(self._plan)
                self._plan = ctypes.c_void_p()
        except Exception:
            pass

    # ---------------------------------------------------------------- host
    def topology(self):
        """Host copies: elem_face (ne,6), elem_pi (ne,6), face_owner (F,2),
        face_nbr (F,2), row_ptr (m+1,), col (nnz,)."""
        s = self.sizes
        ef = np.empty((s.ne, 6), np.int32)
        ep = np.empty((s.ne, 6), np.uint8)
        fo = np.empty((s.n_faces, 2), np.int32)
        fn = np.empty((s.n_faces, 2), np.int32)
        rp = np.empty(s.m + 1, np.int64)
        ci = np.empty(s.nnz, np.int32)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _abi.check(self._lib, self._lib.hyb_plan_topology(self._plan, p(ef), p(ep), p(fo), p(fn), p(rp), p(ci)))
        return dict(elem_face=ef, elem_pi=ep, face_owner=fo, face_nbr=fn, row_ptr=rp, col=ci)

    # -------------------------------------------------------------- device
    def bind(self, device="cuda:0"):
        """Allocate every device buffer with torch on ``device`` and attach it."""
        import torch
        s = self.sizes
        dev = torch.device(device)
        u8 = lambda nbytes: torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=dev)  # noqa: E731
        f64 = lambda n: torch.empty(max(int(n), 1), dtype=torch.float64, device=dev)  # noqa: E731
        b = dict(
            maps=u8(s.bytes_maps),
            factor=f64(s.bytes_factor // 8),
            y=f64(s.bytes_y // 8),
            row_ptr=torch.empty(s.m + 1, dtype=torch.int64, device=dev),
            col=torch.empty(max(s.nnz, 1), dtype=torch.int32, device=dev),
            val=f64(s.nnz),
            r=f64(s.m),
            work=f64(s.bytes_work // 8 + 1),
            status=torch.zeros(4, dtype=torch.int32, device=dev),
        )
        hb = _abi.HybBuffers(*[_dptr(b[name]) for name in _abi.BUFFER_FIELDS])
        self.device = dev
        self.bufs = b
        _abi.check(self._lib, self._lib.hyb_bind(self._plan, ctypes.byref(hb)))
        return self

    def _dev(self, x, shape):
        import torch
        if x is None:
            return None
        t = torch.as_tensor(x, dtype=torch.float64, device=self.device).reshape(shape).contiguous()
        return t

    def setup(self, alpha, beta, f=None, g=None):
        """Local assembly + Cholesky + H_T scatter (and the rhs when f is given)."""
        ne = self.ne
        self._alpha = self._dev(alpha, (ne,))
        self._beta = self._dev(beta, (ne,))
        self._f = self._dev(f, (ne, 3))
        self._g = self._dev(g, (ne, 6 * (self.k + 1) ** 2))
        rc = self._lib.hyb_setup(self._plan, _dptr(self._alpha), _dptr(self._beta), _dptr(self._f), _dptr(self._g))
        _abi.check(self._lib, rc)

    def rhs(self, f, g=None):
        ne = self.ne
        self._f = self._dev(f, (ne, 3))
        self._g = self._dev(g, (ne, 6 * (self.k + 1) ** 2))
        _abi.check(self._lib, self._lib.hyb_rhs(self._plan, _dptr(self._f), _dptr(self._g)))

    def pcg(self, rtol=1e-12, maxit=10000, lam=None, noalloc=False):
        """Jacobi-PCG on H lambda = r (hyb_pcg, or hyb_pcg_noalloc with its
        work in the library's fixed device array): (lambda, info)."""
        import torch
        if lam is None:
            lam = torch.empty(max(self.m, 1), dtype=torch.float64, device=self.device)
        info = _abi.HybSolveInfo()
        fn = self._lib.hyb_pcg_noalloc if noalloc else self._lib.hyb_pcg
        rc = fn(self._plan, ctypes.c_double(rtol), int(maxit), _dptr(lam), ctypes.byref(info))
        if rc not in (0, _abi.HYB_E_NOCONV):
            _abi.check(self._lib, rc)
        return lam[: self.m], dict(iters=info.iters, converged=bool(info.converged), rel_res=info.rel_res)

    def solve(self, f, g=None, rtol=1e-12, maxit=10000, lam=None, u=None):
        """The whole solve for a load on the current factors (hyb_solve: rhs,
        PCG, recovery): (lambda, u, info)."""
        import torch
        ne = self.ne
        self._f = self._dev(f, (ne, 3))
        self._g = self._dev(g, (ne, 6 * (self.k + 1) ** 2))
        if lam is None:
            lam = torch.empty(max(self.m, 1), dtype=torch.float64, device=self.device)
        if u is None:
            u = torch.empty((ne, self.n), dtype=torch.float64, device=self.device)
        info = _abi.HybSolveInfo()
        rc = self._lib.hyb_solve(self._plan, _dptr(self._f), _dptr(self._g), ctypes.c_double(rtol), int(maxit),
                                 _dptr(lam), _dptr(u), ctypes.byref(info))
        if rc not in (0, _abi.HYB_E_NOCONV):
            _abi.check(self._lib, rc)
        return lam[: self.m], u, dict(iters=info.iters, converged=bool(info.converged), rel_res=info.rel_res)

    def recover(self, lam, u=None):
        import torch
        lam = self._dev(lam, (self.m,)) if not isinstance(lam, torch.Tensor) else lam.contiguous()
        if u is None:
            u = torch.empty((self.ne, self.n), dtype=torch.float64, device=self.device)
        _abi.check(self._lib, self._lib.hyb_recover(self._plan, _dptr(lam), _dptr(u)))
        return u

    def fallback_count(self) -> int:
        """Elements the last setup or rhs of a mixed plan solved in FP64."""
        c = ctypes.c_int64()
        _abi.check(self._lib, self._lib.hyb_fallback_count(self._plan, ctypes.byref(c)))
        return c.value

    def status(self):
        """Synchronise and return (code, element) of the first device error."""
        d = ctypes.c_int64()
        rc = self._lib.hyb_status(self._plan, ctypes.byref(d))
        return rc, d.value

    def timing(self, on: bool = True):
        """Start (or stop) HIP-event timing of the setup and recovery kernels."""
        _abi.check(self._lib, self._lib.hyb_timing_enable(self._plan, 1 if on else 0))

    def timing_read(self):
        """Summed kernel milliseconds since timing(True): dict with
        setup_ms, setup_n, recover_ms, recover_n (then cleared)."""
        ms_s, ms_r = ctypes.c_double(), ctypes.c_double()
        n_s, n_r = ctypes.c_int(), ctypes.c_int()
        _abi.check(self._lib, self._lib.hyb_timing_read(self._plan, ctypes.byref(ms_s), ctypes.byref(n_s),
                                                         ctypes.byref(ms_r), ctypes.byref(n_r)))
        return dict(setup_ms=ms_s.value, setup_n=n_s.value, recover_ms=ms_r.value, recover_n=n_r.value)

    def csr_pointers(self):
        """hyb_get_csr: device addresses of row_ptr, col, val and m, nnz."""
        rp, ci, va = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        m, nnz = ctypes.c_int64(), ctypes.c_int64()
        _abi.check(self._lib, self._lib.hyb_get_csr(self._plan, ctypes.byref(rp), ctypes.byref(ci), ctypes.byref(va),
                                                     ctypes.byref(m), ctypes.byref(nnz)))
        return dict(row_ptr=rp.value or 0, col=ci.value or 0, val=va.value or 0, m=m.value, nnz=nnz.value)

    def csr(self):
        """Device CSR arrays (row_ptr, col, val) of H: the bound buffers that
        hyb_get_csr points into."""
        b = self.bufs
        return b["row_ptr"], b["col"][: self.nnz], b["val"][: self.nnz]

    def r(self):
        return self.bufs["r"][: self.m]

    def y_raw(self):
        """The cached L^{-1} f_hat buffer in the library's internal layout."""
        return self.bufs["y"]


class Batch:
    """Independent problems of mixed order and mesh (bound Plans): setup and
    recovery of all of them in one persistent launch each, optionally
    replayed as hipGraphs, with tiles from the library's autotuner."""

    def __init__(self, plans):
        self.plans = list(plans)
        lib = self.plans[0]._lib
        self._lib = lib
        arr = (ctypes.c_void_p * len(self.plans))(*[p._plan.value for p in self.plans])
        self._arr = arr
        self._b = ctypes.c_void_p()
        _abi.check(lib, lib.hyb_batch_create(arr, len(self.plans), ctypes.byref(self._b)))
        self._keep = {}

    def __del__(self):
        try:
            if getattr(self, "_b", None) and self._b.value:
                self._lib.hyb_batch_destroy(self._b)
                self._b = ctypes.c_void_p()
        except Exception:
            pass

    def set(self, p: int, alpha, beta, f=None, g=None, lam=None, u=None):
        """Device inputs of problem p (torch tensors or arrays, copied to the
        plan's device); u (ne x n) is allocated when not given."""
        import torch
        pl = self.plans[p]
        ne = pl.ne
        a = pl._dev(alpha, (ne,))
        b = pl._dev(beta, (ne,))
        ff = pl._dev(f, (ne, 3))
        gg = pl._dev(g, (ne, 6 * (pl.k + 1) ** 2))
        lm = pl._dev(lam, (max(pl.m, 1),))
        if u is None:
            u = torch.empty((ne, pl.n), dtype=torch.float64, device=pl.device)
        self._keep[p] = (a, b, ff, gg, lm, u)
        _abi.check(self._lib, self._lib.hyb_batch_set(self._b, int(p), _dptr(a), _dptr(b), _dptr(ff), _dptr(gg),
                                                      _dptr(lm), _dptr(u)))

    def set_lambda(self, p: int, lam):
        a, b, ff, gg, _, u = self._keep[p]
        self.set(p, a, b, ff, gg, lam, u)

    def u(self, p: int):
        return self._keep[p][5]

    def setup(self):
        _abi.check(self._lib, self._lib.hyb_batch_setup(self._b))

    def recover(self):
        _abi.check(self._lib, self._lib.hyb_batch_recover(self._b))

    def graph(self, on: bool = True):
        _abi.check(self._lib, self._lib.hyb_batch_graph(self._b, 1 if on else 0))

    def tiles(self, blocks_per_cu: int | None = None, items_per_block: int | None = None):
        t = _abi.HybBatchTiles()
        if blocks_per_cu is not None or items_per_block is not None:
            t.blocks_per_cu = int(blocks_per_cu or 0)
            t.items_per_block = int(items_per_block or 0)
            _abi.check(self._lib, self._lib.hyb_batch_set_tiles(self._b, ctypes.byref(t)))
        _abi.check(self._lib, self._lib.hyb_batch_get_tiles(self._b, ctypes.byref(t)))
        return (t.blocks_per_cu, t.items_per_block)

    def timing(self, on: bool = True):
        """Start (or stop) HIP-event timing of the setup and recovery phases."""
        _abi.check(self._lib, self._lib.hyb_batch_timing_enable(self._b, 1 if on else 0))

    def timing_read(self):
        """Summed phase milliseconds since timing(True): dict with setup_ms,
        setup_n, recover_ms, recover_n (then cleared)."""
        ms_s, ms_r = ctypes.c_double(), ctypes.c_double()
        n_s, n_r = ctypes.c_int(), ctypes.c_int()
        _abi.check(self._lib, self._lib.hyb_batch_timing_read(self._b, ctypes.byref(ms_s), ctypes.byref(n_s),
                                                               ctypes.byref(ms_r), ctypes.byref(n_r)))
        return dict(setup_ms=ms_s.value, setup_n=n_s.value, recover_ms=ms_r.value, recover_n=n_r.value)

    def autotune(self, reps: int = 3):
        t = _abi.HybBatchTiles()
        _abi.check(self._lib, self._lib.hyb_batch_autotune(self._b, int(reps), ctypes.byref(t)))
        return (t.blocks_per_cu, t.items_per_block)
